"""Pins of the oracle's near-incompressible model (appendix, "(Near-)
Incompressible Diffeomorphisms"): reduced gradient
g = alpha L v + b - grad M Delta^{-1} div b, b = int lambda grad m dt,
M = (alpha (beta (-Delta^{-1} + id))^{-1} + id)^{-1}, and its Hessian.

The projection K = I - grad M Delta^{-1} div and the penalty
beta/2 <div v, (-Delta^{-1} + id) div v> are coded separately (different
operators, different functions). They are tied together by the identity
K grad J~ = g: with no data term (the inverse-crime point, lambda = 0) the
directional derivative of J~ along K w equals <g, w> exactly for Nyquist-free
v, w, and only for the printed M. Further pins: the beta -> infinity (Leray
projection) and beta -> 0 limits, divergence-free data passing unchanged, the
closed form on a single gradient mode, and finite-difference consistency of
the Hessian.
"""
import numpy as np
import pytest

import oracle as O
from synthetic import bandlimited_velocity, gaussian_blobs

ALPHA, BETA = 1e-2, 1e-2


def trig_field(grid, seed, kmax):
    return bandlimited_velocity(grid.n, seed, kmax, 1.0)


def inverse_crime(n=16, nt=4, seed=1):
    g = O.Grid((n, n, n))
    m0 = gaussian_blobs(g.n, seed, sigma=0.6)
    vs = bandlimited_velocity(g.n, seed + 1, 2, 0.8)
    m1 = O.transport(g, m0, vs, nt)
    return g, m0, m1, vs


def _pairing_gap(g, m0, m1, vs, nt, alpha, beta, w):
    st = O.setup_velocity(g, m0, m1, vs, alpha, nt, 1, beta=beta)
    assert np.abs(st.data).max() == 0.0          # lambda = 0 at the inverse-crime point
    kw = O.ni_project(g, w, alpha, beta)
    eps = 1e-4
    fd = (O.objective(g, m0, m1, vs + eps * kw, alpha, nt, 1, beta)
          - O.objective(g, m0, m1, vs - eps * kw, alpha, nt, 1, beta)) / (2 * eps)
    return abs(fd - g.inner(st.g, w)) / abs(g.inner(st.g, w))


@pytest.mark.parametrize("alpha,beta", [(1e-2, 1e-2), (1e-3, 1e-4), (1e-2, 1.0)])
def test_projected_gradient_pairs_with_the_penalised_objective(alpha, beta):
    g, m0, m1, vs = inverse_crime()
    w = trig_field(g, 7, 3)
    gap = _pairing_gap(g, m0, m1, vs, 4, alpha, beta, w)
    # J_dist is O(eps^2) along the line: its odd (cubic) term leaves O(eps^2)
    # in the central difference
    assert gap < 1e-6, gap


def test_pairing_fails_for_a_wrong_M(monkeypatch):
    """Negative control: drop the '+ id' inside M (M = beta a / alpha); the
    same pairing then misses by O(1)."""
    g, m0, m1, vs = inverse_crime()
    w = trig_field(g, 7, 3)

    def wrong_M(grid, u, alpha, beta):
        kk = O.laplacian_power_symbol(grid, 1)
        pen = beta * (np.where(kk == 0.0, 0.0, 1.0 / np.where(kk == 0.0, 1.0, kk)) + 1.0)
        return O.claire_oracle._ifft(O.claire_oracle._fft(u) * pen / alpha, grid.n)

    monkeypatch.setattr(O.claire_oracle, "ni_operator_M", wrong_M)
    assert _pairing_gap(g, m0, m1, vs, 4, ALPHA, BETA, w) > 1e-2


def test_limits():
    g = O.Grid((16, 16, 16))
    b = trig_field(g, 3, 5)
    # beta -> infinity: the Leray projection, divergence-free output
    out = O.ni_project(g, b, ALPHA, 1e12)
    assert np.abs(O.spectral_divergence(g, out)).max() <= 1e-9 * np.abs(
        O.spectral_divergence(g, b)).max()
    # beta -> 0: the plain model
    out = O.ni_project(g, b, ALPHA, 1e-14)
    assert np.abs(out - b).max() <= 1e-10 * np.abs(b).max()


def test_divergence_free_data_unchanged():
    g = O.Grid((16, 8, 32))
    psi = trig_field(g, 4, 3)
    # curl of a smooth field
    d = [O.spectral_gradient(g, psi[a]) for a in range(3)]
    b = np.stack([d[2][1] - d[1][2], d[0][2] - d[2][0], d[1][0] - d[0][1]])
    assert np.abs(O.ni_project(g, b, ALPHA, BETA) - b).max() <= 1e-12 * np.abs(b).max()


def test_single_gradient_mode_closed_form():
    """b = grad phi, phi = cos(k . x + 0.3): Delta^{-1} div b = phi, so the
    projection subtracts M(|k|) b with M(|k|) = 1 / (alpha / (beta (1/|k|^2 + 1)) + 1)."""
    g = O.Grid((16, 16, 16))
    x = np.meshgrid(*[np.arange(n) * 2 * np.pi / n for n in g.n], indexing="ij")
    for k in [(1, 2, -3), (0, 0, 1), (4, -1, 0)]:
        phase = k[0] * x[0] + k[1] * x[1] + k[2] * x[2] + 0.3
        b = np.stack([-k[a] * np.sin(phase) for a in range(3)])
        kk = float(k[0] ** 2 + k[1] ** 2 + k[2] ** 2)
        m = 1.0 / (ALPHA / (BETA * (1.0 / kk + 1.0)) + 1.0)
        assert np.abs(O.ni_project(g, b, ALPHA, BETA) - (1 - m) * b).max() <= 1e-12


def _hess_gap(n, nt):
    g, m0, m1, vs = inverse_crime(n, nt)
    w = trig_field(g, 4, 3)
    eps = 1e-4
    st = O.setup_velocity(g, m0, m1, vs, ALPHA, nt, 1, beta=BETA)
    gp = O.setup_velocity(g, m0, m1, vs + eps * w, ALPHA, nt, 1, beta=BETA).g
    gm = O.setup_velocity(g, m0, m1, vs - eps * w, ALPHA, nt, 1, beta=BETA).g
    hv = O.hessian_matvec(st, w)
    return np.abs((gp - gm) / (2 * eps) - hv).max() / np.abs(hv).max()


def test_hessian_finite_difference_converges():
    # at lambda = 0 the Gauss--Newton Hessian is the full Hessian; discrete g
    # and H agree up to discretisation error that shrinks under refinement
    h1, h2 = _hess_gap(16, 4), _hess_gap(32, 8)
    assert h2 < 0.03 and h1 / h2 > 3, (h1, h2)


def test_solve_lowers_divergence_and_objective():
    g = O.Grid((16, 16, 16))
    m0 = gaussian_blobs(g.n, 11, sigma=0.6)
    vs = bandlimited_velocity(g.n, 12, 2, 0.8)
    m1 = O.transport(g, m0, vs, 4)
    v0, _, s0 = O.gn_solve(g, m0, m1, 4, 1, [ALPHA])
    v1, st1, s1 = O.gn_solve(g, m0, m1, 4, 1, [ALPHA], beta=BETA)
    assert not s1.warnings and s1.rel_grad <= 5e-2
    Js = [h["J"] for h in s1.history]
    assert all(b < a for a, b in zip(Js, Js[1:]))
    div0 = np.linalg.norm(O.spectral_divergence(g, v0))
    div1 = np.linalg.norm(O.spectral_divergence(g, v1))
    assert div1 < 0.9 * div0, (div0, div1)
    with pytest.raises(ValueError):
        O.gn_solve(g, m0, m1, 4, 1, [ALPHA], beta=BETA, precond="twolevel")
