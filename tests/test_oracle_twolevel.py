"""Pins of the two-level zero-velocity preconditioner in the oracle
(Section 2.5.6): spectral restriction and prolongation against trigonometric
polynomials, (alpha L)^{-1/2} against the regularisation preconditioner, the
preconditioner's closed forms on high-frequency input and for a constant
image, and its symmetry when the coarse system is solved exactly."""
import numpy as np

import oracle as O
from helpers import blob_problem


def trig(grid, terms):
    x = [np.arange(k) * 2 * np.pi / k for k in grid.n]
    X = np.meshgrid(*x, indexing="ij")
    return sum(a * np.cos(k1 * X[0] + k2 * X[1] + k3 * X[2] + ph)
               for a, k1, k2, k3, ph in terms)


LOW = [(1.0, 1, 2, 3, 0.3), (0.5, -3, 1, 0, 1.1), (0.2, 0, -2, 3, -0.7)]   # |k_a| < 4
HIGH = [(1.0, 5, 0, 1, 0.2), (0.7, 1, 6, -2, 0.9), (0.3, 0, 1, 7, 0.4)]   # some |k_a| >= 4


def test_restrict_and_prolong_trig_polynomials():
    g, gc = O.Grid((16, 16, 16)), O.Grid((8, 8, 8))
    u = trig(g, LOW)
    assert np.allclose(O.spectral_restrict(g, u, gc), trig(gc, LOW), atol=1e-12)
    assert np.allclose(O.spectral_prolong(gc, trig(gc, LOW), g), u, atol=1e-12)
    # the cut-off removes modes at or above the coarse Nyquist
    assert np.allclose(O.spectral_restrict(g, trig(g, HIGH), gc), 0.0, atol=1e-12)
    w = trig(g, LOW + HIGH)
    low = O.spectral_prolong(gc, O.spectral_restrict(g, w, gc), g)
    assert np.allclose(low, u, atol=1e-12)


def test_inverse_square_root_squares_to_the_preconditioner():
    g = O.Grid((8, 12, 16))
    rng = np.random.default_rng(1)
    r = rng.standard_normal((3,) + g.n)
    for p in (1, 2):
        twice = O.reg_inverse_sqrt(g, O.reg_inverse_sqrt(g, r, 1e-2, p), 1e-2, p)
        assert np.allclose(twice, O.precondition(g, r, 1e-2, p), rtol=1e-11, atol=1e-12)


def make(st_alpha=1e-2, const=False, rtol=1e-12):
    grid, m0, m1, vstar = blob_problem(n=(16, 16, 16))
    if const:
        m0 = np.full(grid.n, 0.4)
        m1 = np.full(grid.n, 0.6)
    st = O.setup_velocity(grid, m0, m1, np.zeros((3,) + grid.n), st_alpha, 2, 1)
    return grid, st, O.TwoLevelPreconditioner(st, inner_rtol=rtol)


def test_high_frequency_input_is_regularisation_preconditioned():
    grid, st, P = make()
    r = np.stack([trig(grid, HIGH), 0.5 * trig(grid, HIGH[1:]), trig(grid, HIGH[:1])])
    assert np.allclose(P(r), O.precondition(grid, r, st.alpha, st.p), rtol=1e-10, atol=1e-12)


def test_constant_image_low_modes():
    # grad m = 0: the coarse operator is I - mean, so zero-mean low-frequency
    # input is preconditioned by (alpha L)^{-1} exactly
    grid, st, P = make(const=True)
    r = np.stack([trig(grid, LOW), trig(grid, LOW[1:]), 2 * trig(grid, LOW[:1])])
    assert np.allclose(P(r), O.precondition(grid, r, st.alpha, st.p), rtol=1e-9, atol=1e-11)


def test_symmetric_with_exact_coarse_solve():
    grid, st, P = make(rtol=1e-13)
    rng = np.random.default_rng(2)
    a = rng.standard_normal((3,) + grid.n)
    b = rng.standard_normal((3,) + grid.n)
    lhs, rhs = float(np.sum(P(a) * b)), float(np.sum(a * P(b)))
    assert abs(lhs - rhs) <= 1e-9 * abs(lhs)
    assert float(np.sum(P(a) * a)) > 0


def test_coarse_operator_is_the_coarse_hessian_at_zero_velocity():
    """At v = 0 every characteristic stays at its grid point, m(t) = m0, the
    incremental state is m~(1) = -grad m0 . v~ and the incremental adjoint is
    constant in time, so the Gauss--Newton Hessian is exactly
    H0 = alpha L + grad m0 (grad m0)^T (the zero-velocity Hessian). The coarse
    operator of the preconditioner, scaled back by R_c^{1/2} on both sides,
    must therefore equal the full Hessian matvec (semi-Lagrangian transport,
    incremental state and adjoint) on the coarse grid with the restricted
    template: R_c^{1/2} K0_c R_c^{1/2} w = H_c w."""
    grid, m0, m1, _ = blob_problem(n=(16, 32, 16), kmax=3)
    gc = O.Grid((8, 16, 8))
    for p in (1, 2):
        alpha = 1e-2
        st = O.setup_velocity(grid, m0, m1, np.zeros((3,) + grid.n), alpha, 4, p)
        P = O.TwoLevelPreconditioner(st, inner_rtol=1e-8)
        m0c = O.spectral_restrict(grid, m0, gc)
        m1c = O.spectral_restrict(grid, m1, gc)
        stc = O.setup_velocity(gc, m0c, m1c, np.zeros((3,) + gc.n), alpha, 4, p)
        rng = np.random.default_rng(3 + p)
        w = rng.standard_normal((3,) + gc.n)

        def R_half(u):   # R^{1/2} u = R^{-1/2} (alpha L u + mean u)
            mean = u.mean(axis=(1, 2, 3), keepdims=True)
            return O.reg_inverse_sqrt(gc, O.regularization_operator(gc, u, alpha, p) + mean,
                                      alpha, p)

        lhs = R_half(P.coarse_operator(R_half(w)))
        rhs = O.hessian_matvec(stc, w)
        assert np.abs(lhs - rhs).max() <= 1e-10 * np.abs(rhs).max()
