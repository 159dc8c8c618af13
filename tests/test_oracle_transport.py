"""Pins of the oracle's semi-Lagrangian solvers (Section 2.5.2): backtrace,
state, adjoint (continuity equation) and deformation gradient.

Exact cases: zero velocity, constant images, whole-voxel translations.
Closed form: the 1D sine flow v = (a sin x1, 0, 0), whose flow map is
phi_t(X) = 2 atan2(sin(X/2) e^{at}, cos(X/2)) with
d phi_t / dX = e^{at} / (cos^2(X/2) + e^{2at} sin^2(X/2)).
The RK2 schemes must converge to it at second order in h_t, which pins the
backtrace formula, the sign of the RK2 corrector and the direction and sign
of the backward-in-time (adjoint) equations.
"""
import numpy as np

import oracle as O
from synthetic import bandlimited_velocity, gaussian_blobs

A = 0.9


def _phi(X, t):
    return 2.0 * np.arctan2(np.sin(X / 2) * np.exp(A * t), np.cos(X / 2))


def _dphi(X, t):
    e = np.exp(A * t)
    return e / (np.cos(X / 2) ** 2 + e * e * np.sin(X / 2) ** 2)


def _sine_setup(n1, nt, m0fun, m1=None):
    n = (n1, 4, 4)
    g = O.Grid(n)
    x = np.arange(n1) * 2 * np.pi / n1
    v = np.zeros((3,) + n)
    v[0] = (A * np.sin(x))[:, None, None]
    m0 = np.broadcast_to(m0fun(x)[:, None, None], n).copy()
    return g, x, v, m0


def test_zero_velocity_identity():
    n = (16, 16, 16)
    g = O.Grid(n)
    m0 = gaussian_blobs(n, 7)
    v = np.zeros((3,) + n)
    assert np.array_equal(O.departure_displacement(g, v, 4, +1), np.zeros((3,) + n))
    assert np.array_equal(O.transport(g, m0, v, 4), m0)
    F = O.deformation_gradient(g, v, 4)
    assert np.abs(F - np.eye(3)[:, :, None, None, None]).max() == 0.0


def test_constant_image_stays_constant():
    n = (16, 16, 16)
    g = O.Grid(n)
    v = bandlimited_velocity(n, 8, 3, 1.5)
    m = O.transport(g, np.full(n, 0.6), v, 4)
    assert np.abs(m - 0.6).max() < 1e-14


def test_whole_voxel_translation_is_exact():
    n = (16, 16, 16)
    g = O.Grid(n)
    nt = 4
    shift = np.array([2, -1, 3])                 # voxels per time step
    v = np.stack([np.full(n, shift[a] * g.h[a] * nt) for a in range(3)])
    d = O.departure_displacement(g, v, nt, +1)
    assert np.allclose(d, -shift[:, None, None, None], atol=1e-14, rtol=0)
    m0 = gaussian_blobs(n, 9)
    m1 = O.transport(g, m0, v, nt)
    ref = np.roll(m0, tuple(nt * shift), axis=(0, 1, 2))
    assert np.abs(m1 - ref).max() < 1e-13
    # F stays the identity: grad v = 0
    F = O.deformation_gradient(g, v, nt)
    assert np.abs(F - np.eye(3)[:, :, None, None, None]).max() < 1e-14


def test_backtrace_third_order_local_error_on_sine_flow():
    errs = []
    for nt in (4, 8, 16):
        g, x, v, _ = _sine_setup(256, nt, np.cos)
        d = O.departure_displacement(g, v, nt, +1)[0, :, 0, 0]
        y = x + d * g.h[0]
        y_exact = _phi(x, -1.0 / nt)
        err = np.abs(np.angle(np.exp(1j * (y - y_exact)))).max()
        errs.append(err)
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 2.7, (errs, rates)
    # and the backward characteristics use -v
    g, x, v, _ = _sine_setup(256, 8, np.cos)
    dm = O.departure_displacement(g, v, 8, -1)[0, :, 0, 0]
    err_minus = np.abs(x + dm * g.h[0] - _phi(x, 1.0 / 8)).max()
    assert err_minus < 1.5 * errs[1]            # same RK2 error as the +v case


def test_state_converges_second_order_on_sine_flow():
    m0fun = lambda x: np.exp(np.cos(x))  # noqa: E731
    errs = []
    for nt in (4, 8, 16):
        g, x, v, m0 = _sine_setup(512, nt, m0fun)
        m1 = O.transport(g, m0, v, nt)[:, 0, 0]
        ref = m0fun(_phi(x, -1.0))          # m(1, x) = m0(phi_1^{-1}(x))
        errs.append(np.abs(m1 - ref).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 1.8, (errs, rates)


def test_adjoint_continuity_equation_on_sine_flow():
    # lambda(0, X) = lambda(1, phi_1(X)) * d phi_1/dX for
    # d_t lambda + div(lambda v) = 0; run the oracle's backward solver with
    # final value lam1 (passed as -m~(1) to the GN incremental adjoint, which
    # is the same continuity equation).
    lam1fun = lambda x: np.sin(x) + 0.5 * np.cos(2 * x)  # noqa: E731
    errs = []
    for nt in (4, 8, 16):
        g, x, v, m0 = _sine_setup(512, nt, np.cos)
        st = O.setup_velocity(g, m0, m0, v, 1.0, nt, 1)
        lam1 = np.broadcast_to(lam1fun(x)[:, None, None], g.n).copy()
        lam0 = O.incremental_adjoint(st, -lam1)[0][:, 0, 0]
        ref = lam1fun(_phi(x, 1.0)) * _dphi(x, 1.0)
        errs.append(np.abs(lam0 - ref).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 1.8, (errs, rates)


def test_deformation_gradient_on_sine_flow():
    errs = []
    for nt in (4, 8, 16):
        g, x, v, _ = _sine_setup(512, nt, np.cos)
        F = O.deformation_gradient(g, v, nt)
        ref = _dphi(_phi(x, -1.0), 1.0)          # d phi_1/dX at X = phi_1^{-1}(x)
        errs.append(np.abs(F[0, 0, :, 0, 0] - ref).max())
        assert np.abs(F[1, 1] - 1).max() < 1e-12 and np.abs(F[2, 2] - 1).max() < 1e-12
        assert np.abs(F[0, 1]).max() < 1e-12 and np.abs(F[1, 0]).max() < 1e-12
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 1.8, (errs, rates)
    det = O.det3(F)
    assert det.min() > 0


def test_det3_against_numpy():
    rng = np.random.default_rng(12)
    F = rng.standard_normal((3, 3, 5, 4, 3))
    ref = np.linalg.det(np.moveaxis(F, (0, 1), (-2, -1)))
    assert np.abs(O.det3(F) - ref).max() < 1e-12
