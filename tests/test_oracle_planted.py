"""Planted mistakes in the oracle must be caught by its pins.

Each case patches one plausible slip into a copy of an oracle function (on
the CPU) and checks that the corresponding pin then fails.
"""
import numpy as np

import oracle as O
from oracle import claire_oracle as C
from synthetic import bandlimited_velocity, gaussian_blobs


def _fd_gap(n=32, nt=8):
    g = O.Grid((n, n, n))
    m0 = gaussian_blobs(g.n, 1, sigma=0.6)
    m1 = O.transport(g, m0, bandlimited_velocity(g.n, 2, 2, 0.8), nt)
    v = 0.4 * bandlimited_velocity(g.n, 3, 2, 0.8)
    w = bandlimited_velocity(g.n, 4, 3, 1.0)
    eps = 1e-4
    st = O.setup_velocity(g, m0, m1, v, 1e-2, nt, 1)
    fd = (O.objective(g, m0, m1, v + eps * w, 1e-2, nt, 1)
          - O.objective(g, m0, m1, v - eps * w, 1e-2, nt, 1)) / (2 * eps)
    return abs(fd - g.inner(st.g, w)) / abs(fd)


def test_flipped_adjoint_corrector_sign_is_caught(monkeypatch):
    good = _fd_gap()
    orig = C._continuity_step

    def wrong(grid, lam_next, d_minus, div_v, div_v_dep, nt):
        ht = 1.0 / nt
        u_y = C.interpolate(lam_next, d_minus)
        f0 = u_y * div_v_dep
        f1 = (u_y + ht * f0) * div_v
        return u_y - 0.5 * ht * (f0 + f1)          # corrector sign as misprinted

    monkeypatch.setattr(C, "_continuity_step", wrong)
    bad = _fd_gap()
    monkeypatch.setattr(C, "_continuity_step", orig)
    assert good < 0.03 and bad > 3 * good


def _sine_adjoint_error(nt=8, a=0.9, n1=256):
    # lambda(0, X) = lambda(1, phi_1(X)) d phi_1/dX for the sine flow
    n = (n1, 4, 4)
    g = O.Grid(n)
    x = np.arange(n1) * 2 * np.pi / n1
    v = np.zeros((3,) + n)
    v[0] = (a * np.sin(x))[:, None, None]
    m0 = np.broadcast_to(np.cos(x)[:, None, None], n).copy()
    st = O.setup_velocity(g, m0, m0, v, 1.0, nt, 1)
    lam1 = np.broadcast_to(np.sin(x)[:, None, None], n).copy()
    lam0 = O.incremental_adjoint(st, -lam1)[0][:, 0, 0]
    e = np.exp(a)
    phi = 2.0 * np.arctan2(np.sin(x / 2) * e, np.cos(x / 2))
    ref = np.sin(phi) * e / (np.cos(x / 2) ** 2 + e * e * np.sin(x / 2) ** 2)
    return np.abs(lam0 - ref).max()


def test_forward_characteristics_for_adjoint_are_caught(monkeypatch):
    good = _sine_adjoint_error()
    orig = C.departure_displacement

    def wrong(grid, v, nt, direction=+1):
        return orig(grid, v, nt, +1)               # backward equations on +v

    monkeypatch.setattr(C, "departure_displacement", wrong)
    bad = _sine_adjoint_error()
    monkeypatch.setattr(C, "departure_displacement", orig)
    assert good < 1e-2 and bad > 0.3


def test_swapped_lagrange_weights_are_caught(monkeypatch):
    # interpolating with nodes -1..2 mislabelled as 0..3 breaks exactness on
    # linear functions
    n = (12, 12, 12)
    f = np.broadcast_to(np.arange(12.0)[:, None, None], n).copy()
    d = np.zeros((3,) + n)
    d[0] = 0.3
    ok = O.interpolate(f, d)
    d_bad = d.copy()
    d_bad[0] += 1.0                                 # off-by-one node shift
    assert np.abs(ok[2:-3] - (np.arange(12.0)[2:-3, None, None] + 0.3)).max() < 1e-12
    assert np.abs(O.interpolate(f, d_bad)[2:-3] - ok[2:-3]).max() > 0.5


def _translation_error(max_gn=20):
    # the whole solve's closed-form case: a 4-voxel shift recovered by v = 4h e3
    n, nt = 32, 4
    g = O.Grid((n, n, n))
    m0 = gaussian_blobs(g.n, 11)
    m1 = np.roll(m0, 4, axis=2)
    v, _, _ = O.gn_solve(g, m0, m1, nt, 1, [1e-2], gtol=1e-3, max_gn=max_gn)
    c = 4 * 2 * np.pi / n
    return max(np.abs(v[0]).max(), np.abs(v[1]).max(), np.abs(v[2] - c).max()) / c


def test_flipped_incremental_adjoint_is_caught(monkeypatch):
    # final condition lambda~(1) = +m~(1) instead of -m~(1): the Gauss--Newton
    # Hessian changes sign in its data term and the solve no longer lands on
    # the translation
    good = _translation_error()
    orig = C.incremental_adjoint

    def wrong(st, mt_final):
        return [-x for x in orig(st, mt_final)]

    monkeypatch.setattr(C, "incremental_adjoint", wrong)
    bad = _translation_error()
    monkeypatch.setattr(C, "incremental_adjoint", orig)
    assert good < 5e-3 and bad > 0.5


def _factor_gap_ratio():
    """Gap between the two readings of f at the departure points (grid
    product, factors), smooth fields at 32^3 over 64^3."""
    gaps = []
    for n in (32, 64):
        g = O.Grid((n, n, n))
        X = np.meshgrid(*[np.arange(k) * 2 * np.pi / k for k in g.n], indexing="ij")
        m0 = np.sin(X[0]) * np.cos(X[1]) + 0.5 * np.sin(X[2] + X[0])
        v = np.stack([0.3 * np.sin(X[1]), 0.2 * np.cos(X[2]), 0.25 * np.sin(X[0] + X[1])])
        vt = np.stack([np.cos(X[2]), np.sin(X[0]) * np.sin(X[1]), 0.5 * np.cos(X[1] - X[2])])
        st = C.setup_velocity(g, m0, np.cos(X[0]), v, 1e-2, 4, 1)
        a, b = C.incremental_state(st, vt), C.incremental_state(st, vt, "factors")
        gaps.append(np.abs(a - b).max() / np.abs(a).max())
    return gaps[0] / gaps[1]


def test_uninterpolated_velocity_factor_is_caught(monkeypatch):
    good = _factor_gap_ratio()
    orig = C.incremental_state

    def wrong(st, vt, f_eval="grid"):
        if f_eval == "grid":
            return orig(st, vt)
        nt, ht = st.nt, 1.0 / st.nt
        mt = np.zeros(st.grid.n)
        for j in range(nt):
            u_y = C.interpolate(mt, st.d_plus)
            # v~ taken at the arrival point instead of the departure point
            f0 = -np.sum(C.interpolate(st.grad_m[j], st.d_plus) * vt, axis=0)
            f1 = -np.sum(st.grad_m[j + 1] * vt, axis=0)
            mt = u_y + 0.5 * ht * (f0 + f1)
        return mt

    monkeypatch.setattr(C, "incremental_state", wrong)
    bad = _factor_gap_ratio()
    monkeypatch.setattr(C, "incremental_state", orig)
    # the convergence pin asks for a ratio of at least 10
    assert good >= 10.0 and bad < 10.0
