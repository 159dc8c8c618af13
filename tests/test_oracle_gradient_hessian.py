"""Pins of the oracle's reduced gradient (eq. e:rgrad), Gauss--Newton Hessian
matvec (eq. e:matvec with eqs. e:incstate, e:incadj), PCG (Algorithm 2) and
Gauss--Newton solve (Algorithm 1).

Exact cases: v = 0 (the zero-velocity Hessian of Section 2.5.6 is then the
GN Hessian exactly), constant images, the inverse-crime point (m1 = m0
transported by v*, where lambda = 0 and g = alpha L v*), whole-voxel
translations (every SL step is a shift, so H is exactly symmetric).
Convergence: finite differences of J and of g. Because the method is
optimize-then-discretize, discrete g and H are consistent with the discrete J
only up to discretisation error (Section 2.3); the gap must shrink under
refinement of n and n_t.
Brute force: the 8^3 Hessian assembled column by column.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle as O
from helpers import blob_problem
from synthetic import bandlimited_velocity, gaussian_blobs


def _problem(n, nt, seed=1, sigma=0.6):
    g = O.Grid((n, n, n))
    m0 = gaussian_blobs(g.n, seed, sigma=sigma)
    vs = bandlimited_velocity(g.n, seed + 1, 2, 0.8)
    m1 = O.transport(g, m0, vs, nt)
    return g, m0, m1, vs


def test_zero_velocity_closed_forms():
    g, m0, m1, _ = _problem(16, 4)
    alpha, nt = 1e-2, 4
    st = O.setup_velocity(g, m0, m1, np.zeros((3,) + g.n), alpha, nt, 1)
    gm0 = O.spectral_gradient(g, m0)
    # g = -(m0 - m1) grad m0 (Section 2.5.6, zero velocity approximation)
    assert np.abs(st.g - (-(m0 - m1) * gm0)).max() <= 1e-13 * np.abs(st.g).max()
    vt = bandlimited_velocity(g.n, 9, 3, 1.0)
    # m~(1) = -grad m0 . v~ and H v~ = alpha L v~ + (grad m0 (x) grad m0) v~
    mt = O.incremental_state(st, vt)
    ref_mt = -np.sum(gm0 * vt, axis=0)
    assert np.abs(mt - ref_mt).max() <= 1e-13 * np.abs(ref_mt).max()
    hv = O.hessian_matvec(st, vt)
    ref = O.regularization_operator(g, vt, alpha, 1) + np.sum(gm0 * vt, axis=0) * gm0
    assert np.abs(hv - ref).max() <= 1e-12 * np.abs(ref).max()


def test_inverse_crime_point():
    g, m0, m1, vs = _problem(16, 4)
    for p in (1, 2):
        st = O.setup_velocity(g, m0, m1, vs, 3e-2, 4, p)
        assert np.abs(st.m[-1] - m1).max() == 0.0
        assert all(np.abs(l).max() == 0.0 for l in st.lam)
        assert np.array_equal(st.g, O.regularization_operator(g, vs, 3e-2, p))
        assert st.J_dist == 0.0


def test_constant_image():
    n = (16, 16, 16)
    g = O.Grid(n)
    m = np.full(n, 0.4)
    v = bandlimited_velocity(n, 5, 3, 1.0)
    st = O.setup_velocity(g, m, m, v, 1e-2, 4, 2)
    assert np.abs(st.g - O.regularization_operator(g, v, 1e-2, 2)).max() < 1e-12
    vt = bandlimited_velocity(n, 6, 3, 1.0)
    ref = O.regularization_operator(g, vt, 1e-2, 2)
    assert np.abs(O.hessian_matvec(st, vt) - ref).max() < 1e-12 * np.abs(ref).max()


def _fd_gaps(n, nt):
    g, m0, m1, vs = _problem(n, nt)
    alpha = 1e-2
    v = 0.4 * bandlimited_velocity(g.n, 3, 2, 0.8)
    w = bandlimited_velocity(g.n, 4, 3, 1.0)
    eps = 1e-4
    st = O.setup_velocity(g, m0, m1, v, alpha, nt, 1)
    jp = O.objective(g, m0, m1, v + eps * w, alpha, nt, 1)
    jm = O.objective(g, m0, m1, v - eps * w, alpha, nt, 1)
    fd = (jp - jm) / (2 * eps)
    grad_gap = abs(fd - g.inner(st.g, w)) / abs(fd)
    st_star = O.setup_velocity(g, m0, m1, vs, alpha, nt, 1)
    gp = O.setup_velocity(g, m0, m1, vs + eps * w, alpha, nt, 1).g
    gm = O.setup_velocity(g, m0, m1, vs - eps * w, alpha, nt, 1).g
    hv = O.hessian_matvec(st_star, w)
    hess_gap = np.abs((gp - gm) / (2 * eps) - hv).max() / np.abs(hv).max()
    return grad_gap, hess_gap


def test_finite_difference_consistency_converges():
    g1, h1 = _fd_gaps(16, 4)
    g2, h2 = _fd_gaps(32, 8)
    # a dropped term or a flipped sign leaves an O(1) gap that does not shrink
    assert g2 < 0.03 and g1 / g2 > 4, (g1, g2)
    assert h2 < 0.03 and h1 / h2 > 3, (h1, h2)


def _assemble(op, shape):
    N = int(np.prod(shape))
    M = np.empty((N, N))
    e = np.zeros(N)
    for i in range(N):
        e[:] = 0.0
        e[i] = 1.0
        M[:, i] = op(e.reshape(shape)).ravel()
    return M


def test_brute_force_8cubed_hessian():
    g, m0, m1, vs = _problem(8, 2, sigma=0.9)
    alpha = 1e-2
    st = O.setup_velocity(g, m0, m1, 0.5 * vs, alpha, 2, 1)
    shape = (3,) + g.n
    H = _assemble(lambda e: O.hessian_matvec(st, e), shape)
    R = _assemble(lambda e: O.regularization_operator(g, e, alpha, 1), shape)
    D = H - R
    ev = np.linalg.eigvalsh(0.5 * (D + D.T))
    assert ev.min() >= -1e-4 * ev.max()                     # GN data part is PSD
    assert np.abs(D - D.T).max() <= 0.1 * np.abs(D).max()  # symmetric up to discretisation
    assert np.abs(R - R.T).max() <= 1e-12 * np.abs(R).max()


def test_translation_hessian_exactly_symmetric_and_pcg():
    n, nt = 8, 2
    g = O.Grid((n, n, n))
    m0 = gaussian_blobs(g.n, 3, sigma=0.9)
    shift = np.array([1, 0, -1])
    v = np.stack([np.full(g.n, shift[a] * g.h[a] * nt) for a in range(3)])
    m1 = gaussian_blobs(g.n, 4, sigma=0.9)
    alpha = 1e-2
    st = O.setup_velocity(g, m0, m1, v, alpha, nt, 1)
    shape = (3,) + g.n
    H = _assemble(lambda e: O.hessian_matvec(st, e), shape)
    assert np.abs(H - H.T).max() <= 1e-12 * np.abs(H).max()
    # PCG (Algorithm 2) for 10 iterations against SciPy's preconditioned CG
    Minv = spla.LinearOperator(H.shape, matvec=lambda r: O.precondition(
        g, r.reshape(shape), alpha, 1).ravel())
    Hop = spla.LinearOperator(H.shape, matvec=lambda x: H @ x)
    ref, _ = spla.cg(Hop, -st.g.ravel(), x0=np.zeros(H.shape[0]), rtol=0.0, atol=0.0,
                     maxiter=10, M=Minv)
    vt, its, hist, _ = O.pcg(lambda s: O.hessian_matvec(st, s),
                             lambda r: O.precondition(g, r, alpha, 1),
                             st.g, fixed_iters=10)
    assert its == 10
    assert np.abs(vt.ravel() - ref).max() <= 1e-8 * np.abs(ref).max()
    # and run to convergence: the dense solution
    vt_full, its_full, _, _ = O.pcg(lambda s: O.hessian_matvec(st, s),
                                    lambda r: O.precondition(g, r, alpha, 1),
                                    st.g, fixed_iters=300)
    dense = np.linalg.solve(H, -st.g.ravel())
    assert np.abs(vt_full.ravel() - dense).max() <= 1e-8 * np.abs(dense).max()


def test_forcing_rule():
    assert O.forcing_tolerance(4.0) == 2.0                 # eta = 1/2
    assert abs(O.forcing_tolerance(0.04) - 0.2 * 0.04) < 1e-15
    assert abs(O.forcing_tolerance(0.04, "quadratic") - 0.04 * 0.04) < 1e-15


@pytest.mark.parametrize("p", [1, 2])
def test_gn_solve_invariants(p):
    n, nt = 16, 4
    g, m0, m1, vs = _problem(n, nt)
    alpha = 1e-2 if p == 1 else 1e-3
    v, st, stats = O.gn_solve(g, m0, m1, nt, p, [alpha], gtol=5e-2, max_gn=20)
    hist = [h["J"] for h in stats.history]
    assert all(b < a for a, b in zip(hist, hist[1:]))        # Armijo: monotone
    assert stats.rel_grad <= 5e-2 and not stats.warnings
    assert stats.J < stats.J0 and stats.rel_mismatch < 0.5
    assert O.deformation_determinant(g, v, nt).min() > 0
    assert stats.pde_solves == 2 + 2 * stats.gn_iters + 2 * stats.matvecs + stats.ls_trials


def test_gn_solve_recovers_a_translation():
    """Closed-form solution of the whole solve (Alg. 1): m1 is m0 shifted by 4
    voxels along x3. The constant velocity v = 4h e3 moves m0 onto m1 exactly
    (semi-Lagrangian steps of one whole voxel interpolate exactly) and the H1
    seminorm does not penalise constants, so it is the global minimiser with
    J = 0. Solved to gtol 1e-3 from v = 0 the oracle lands on it; a wrong sign
    or term in the gradient, the Hessian or the line search would not."""
    n, nt = 32, 4
    g = O.Grid((n, n, n))
    m0 = gaussian_blobs(g.n, 11)
    m1 = np.roll(m0, 4, axis=2)
    v, st, stats = O.gn_solve(g, m0, m1, nt, 1, [1e-2], gtol=1e-3)
    c = 4 * 2 * np.pi / n
    err = max(np.abs(v[0]).max(), np.abs(v[1]).max(), np.abs(v[2] - c).max()) / c
    assert stats.rel_grad <= 1e-3 and not stats.warnings
    assert err <= 5e-3                          # observed 1.4e-3
    assert stats.J <= 1e-5 * stats.J0           # observed 2.3e-6 J0


def test_pcg_stops_on_nonpositive_curvature():
    """Truncated CG: <s, Hs> <= 0 stops PCG with the current iterate; on the
    first direction the preconditioned steepest-descent direction is taken."""
    rng = np.random.default_rng(8)
    g = rng.standard_normal((3, 4, 4, 4))
    ident = lambda r: r.copy()          # noqa: E731
    # negative definite: the first curvature is negative
    vt, its, _, hit = O.pcg(lambda s: -2.0 * s, ident, g)
    assert its == 1 and O.pcg.neg_curv and not hit
    assert np.array_equal(vt, -g)
    # indefinite diagonal: positive curvature first, negative later
    d = np.where(rng.random(g.shape) < 0.5, 1.0, -3.0)
    d[0, 0, 0, 0] = 50.0
    g2 = np.where(d > 0, 1.0, 1e-3) * rng.standard_normal(g.shape)
    vt, its, _, _ = O.pcg(lambda s: d * s, ident, g2, fixed_iters=40)
    assert O.pcg.neg_curv and 2 <= its < 40
    vt_prev, _, _, _ = O.pcg(lambda s: d * s, ident, g2, fixed_iters=its - 1)
    assert np.array_equal(vt, vt_prev)
    # positive definite: unaffected
    O.pcg(lambda s: 2.0 * s, ident, g)
    assert not O.pcg.neg_curv


def test_memory_lean_setup_matches_stored():
    # grad m^j recomputed on access (the 512^3 setting) gives bit-identical
    # gradient and Hessian matvec to the stored gradients
    grid, m0, m1, vstar = blob_problem()
    v = 0.5 * vstar
    vt = bandlimited_velocity(grid.n, 91, 4, 0.5)
    for deriv in ("spectral", "fd8"):
        st = O.setup_velocity(grid, m0, m1, v, 1e-2, 4, 1, deriv)
        lean = O.setup_velocity(grid, m0, m1, v, 1e-2, 4, 1, deriv, store_grad=False)
        assert isinstance(lean.grad_m, O.RecomputedGradients) and lean.lam is None
        assert np.array_equal(st.g, lean.g) and st.J == lean.J
        assert np.array_equal(O.hessian_matvec(st, vt), O.hessian_matvec(lean, vt))


def _smooth_problem(n, nt=4):
    """Images and velocities made of a few fixed Fourier modes: the same
    functions at every n, so discretisation gaps can be followed under
    refinement."""
    g = O.Grid((n, n, n))
    X = np.meshgrid(*[np.arange(k) * 2 * np.pi / k for k in g.n], indexing="ij")
    m0 = np.sin(X[0]) * np.cos(X[1]) + 0.5 * np.sin(X[2] + X[0])
    m1 = np.cos(X[0] + 0.3) * np.sin(X[1])
    v = np.stack([0.3 * np.sin(X[1]), 0.2 * np.cos(X[2]), 0.25 * np.sin(X[0] + X[1])])
    vt = np.stack([np.cos(X[2]), np.sin(X[0]) * np.sin(X[1]), 0.5 * np.cos(X[1] - X[2])])
    return O.setup_velocity(g, m0, m1, v, 1e-2, nt, 1), vt


def _f_eval_gap(st, vt):
    a, b = O.incremental_state(st, vt), O.incremental_state(st, vt, "factors")
    ha, hb = O.hessian_matvec(st, vt), O.hessian_matvec(st, vt, "factors")
    return (np.abs(a - b).max() / np.abs(a).max(), np.abs(ha - hb).max() / np.abs(ha).max())


def test_departure_f_variants_agree_on_whole_voxel_shifts():
    # every departure point is a grid point: interpolation is a shift, and the
    # shifted product equals the product of the shifted factors
    n, nt = 8, 2
    g = O.Grid((n, n, n))
    shift = np.array([1, -1, 2])
    v = np.stack([np.full(g.n, shift[a] * g.h[a] * nt) for a in range(3)])
    st = O.setup_velocity(g, gaussian_blobs(g.n, 3, sigma=0.9), gaussian_blobs(g.n, 4, sigma=0.9),
                          v, 1e-2, nt, 1)
    vt = bandlimited_velocity(g.n, 5, 3, 1.0)
    gap_mt, gap_hv = _f_eval_gap(st, vt)
    assert gap_mt <= 1e-13 and gap_hv <= 1e-13
    with pytest.raises(ValueError):
        O.incremental_state(st, vt, "both")


def test_departure_f_variants_gap_converges():
    # Section 2.5.2 leaves open whether f is interpolated as a grid product or
    # factor by factor; for smooth fields the two differ by the tricubic
    # interpolation error, O(h^4): the gap must fall by well over 2^3 per
    # halving of h (a variant that skipped interpolating a factor, or took
    # the wrong time level, would not converge at all)
    g32 = _f_eval_gap(*_smooth_problem(32))
    g64 = _f_eval_gap(*_smooth_problem(64))
    for coarse, fine in zip(g32, g64):
        assert coarse / fine >= 10.0
    assert max(g64) <= 2e-5
