"""Pins of the oracle's pseudo-spectral operators (Section 2.5.3; L of
Section 2.2; (alpha L)^{-1} of Sections 2.5.5-2.5.6) against closed forms.

Trigonometric polynomials below Nyquist are differentiated exactly by the
Fourier method, so gradient, divergence, L and the inverse are compared with
their analytic values; a wrong sign, axis, normalisation or power fails.
"""
import numpy as np
import pytest

import oracle as O
from synthetic import grid_coordinates, trig_field


def _phase(n, k):
    x = grid_coordinates(n)
    return (k[0] * x[0])[:, None, None] + (k[1] * x[1])[None, :, None] \
        + (k[2] * x[2])[None, None, :]


def _exact_partial(n, terms, axis):
    out = np.zeros(n)
    for k, a, b in terms:
        ph = _phase(n, k)
        out += k[axis] * (-a * np.sin(ph) + b * np.cos(ph))
    return out


def _exact_power(n, terms, p):
    out = np.zeros(n)
    for k, a, b in terms:
        ph = _phase(n, k)
        out += float(np.dot(k, k)) ** p * (a * np.cos(ph) + b * np.sin(ph))
    return out


SHAPES = [(16, 16, 16), (8, 16, 32), (32, 8, 16)]


@pytest.mark.parametrize("n", SHAPES)
def test_gradient_exact_on_trig_polynomials(n):
    g = O.Grid(n)
    u, terms = trig_field(n, seed=11, terms=7, kfrac=1.0)
    gu = O.spectral_gradient(g, u)
    for a in range(3):
        ref = _exact_partial(n, terms, a)
        assert np.abs(gu[a] - ref).max() <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n", SHAPES)
def test_divergence_exact_on_trig_polynomials(n):
    g = O.Grid(n)
    comps, refs = [], []
    for a in range(3):
        u, terms = trig_field(n, seed=20 + a, terms=5, kfrac=1.0)
        comps.append(u)
        refs.append(_exact_partial(n, terms, a))
    dv = O.spectral_divergence(g, np.stack(comps))
    ref = sum(refs)
    assert np.abs(dv - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("n", SHAPES)
def test_L_and_inverse_exact(n, p):
    g = O.Grid(n)
    u, terms = trig_field(n, seed=31, terms=6, kfrac=1.0)
    u = u + 0.75                                   # a mean, which L annihilates
    Lu = O.apply_L(g, u, p)
    ref = _exact_power(n, terms, p)
    assert np.abs(Lu - ref).max() <= 1e-11 * np.abs(ref).max()
    alpha = 3e-2
    back = O.apply_alphaL_inverse(g, alpha * Lu, alpha, p)
    # (alpha L)^{-1} alpha L u = u - mean(u): the k = 0 mode is the identity
    assert np.abs(back - (u - u.mean())).max() <= 1e-11 * np.abs(u).max()
    # the mean passes through (alpha L)^{-1} unchanged
    assert abs(O.apply_alphaL_inverse(g, np.full(n, 2.5), alpha, p).mean() - 2.5) < 1e-13


def test_laplacian_sign_and_h1_seminorm():
    # L = -Laplacian: <L u, u> = ||grad u||^2 >= 0 (Section 2.2, H1 seminorm)
    n = (16, 16, 16)
    g = O.Grid(n)
    u, _ = trig_field(n, seed=5, terms=5, kfrac=1.0)
    lhs = g.inner(O.apply_L(g, u, 1), u)
    gu = O.spectral_gradient(g, u)
    rhs = sum(g.inner(gu[a], gu[a]) for a in range(3))
    assert lhs > 0 and abs(lhs - rhs) <= 1e-12 * rhs


def test_nyquist_mode_reading():
    # Odd derivatives drop the Nyquist mode; even symbols keep (n/2)^2.
    n = (8, 8, 8)
    g = O.Grid(n)
    x = grid_coordinates(n)[0]
    u = np.broadcast_to(np.cos(4 * x)[:, None, None], n).copy()
    assert np.abs(O.spectral_gradient(g, u)).max() < 1e-13
    assert np.abs(O.apply_L(g, u, 1) - 16.0 * u).max() < 1e-12


def test_fft_convention_matches_brute_force_dft():
    # The oracle's transforms are the standard DFT sum_l u_l exp(-i k x_l):
    # check the spectral derivative against an explicit DFT built from the
    # definition at n = 4 x 4 x 8.
    n = (4, 4, 8)
    rng = np.random.default_rng(3)
    u = rng.standard_normal(n)
    g = O.Grid(n)
    x = grid_coordinates(n)
    # brute-force derivative along x3 of the trigonometric interpolant
    k3 = np.fft.fftfreq(n[2], 1.0 / n[2])
    k3[np.abs(k3) == n[2] // 2] = 0.0
    E = np.exp(-1j * np.outer(k3, x[2]))             # forward DFT matrix
    uh = np.einsum("kz,abz->abk", E, u)
    du = np.einsum("zk,abk->abz", np.conj(E).T, 1j * k3 * uh).real / n[2]
    assert np.abs(O.spectral_gradient(g, u)[2] - du).max() < 1e-12


# ---------------------------------------------------------------- FD8
def test_fd8_exact_on_polynomials_up_to_degree_8():
    """The 8th-order central stencil differentiates polynomials of degree <= 8
    exactly (away from the periodic wrap); at degree 9 it is off by its
    leading truncation term."""
    n = 32
    g = O.Grid((n, n, n))
    x = np.arange(n, dtype=np.float64) * g.h[0]
    X1, X2, X3 = np.meshgrid(x, x, x, indexing="ij")
    inner = (slice(5, n - 5),) * 3
    c = 1.3
    for deg in range(1, 9):
        u = (X2 - c) ** deg
        du = O.fd8_derivative(g, u, 1)
        exact = deg * (X2 - c) ** (deg - 1)
        scale = np.abs(exact[inner]).max()
        assert np.abs(du[inner] - exact[inner]).max() <= 1e-10 * scale, deg
    # degree 9: the error is the leading truncation term -h^8 f^(9) / 630
    u = (X3 - c) ** 9
    du = O.fd8_derivative(g, u, 2)
    exact = 9 * (X3 - c) ** 8
    lead = -(g.h[2] ** 8) * 362880.0 / 630.0
    assert np.allclose(du[inner] - exact[inner], lead, rtol=1e-5, atol=0)


def test_fd8_modified_wavenumber():
    """On exp(i k x) the stencil acts as i s(k h) / h with
    s(t) = (1344 sin t - 336 sin 2t + 64 sin 3t - 6 sin 4t) / 840."""
    n = (16, 24, 32)
    g = O.Grid(n)
    x = np.arange(n[2]) * g.h[2]
    for k in (1, 3, 7, 15):
        u = np.broadcast_to(np.sin(k * x), n).copy()
        t = k * g.h[2]
        s = (1344 * np.sin(t) - 336 * np.sin(2 * t) + 64 * np.sin(3 * t) - 6 * np.sin(4 * t)) / 840
        expect = (s / g.h[2]) * np.broadcast_to(np.cos(k * x), n)
        assert np.allclose(O.fd8_derivative(g, u, 2), expect, atol=1e-12)


def test_fd8_eighth_order_convergence():
    errs = []
    for n in (16, 32):
        g = O.Grid((n, n, n))
        x = np.arange(n) * g.h[0]
        X1 = np.meshgrid(x, x, x, indexing="ij")[0]
        errs.append(np.abs(O.fd8_derivative(g, np.sin(2 * X1), 0) - 2 * np.cos(2 * X1)).max())
    assert 200 < errs[0] / errs[1] < 300       # 2^8 = 256


def test_fd8_divergence_is_minus_adjoint_of_gradient():
    rng = np.random.default_rng(4)
    g = O.Grid((8, 12, 16))
    u = rng.standard_normal(g.n)
    v = rng.standard_normal((3,) + g.n)
    lhs = g.inner(O.fd8_divergence(g, v), u)
    rhs = -sum(g.inner(v[a], O.fd8_gradient(g, u)[a]) for a in range(3))
    assert np.isclose(lhs, rhs, rtol=1e-12)
    # dispatch
    assert np.array_equal(O.gradient(g, u, "fd8"), O.fd8_gradient(g, u))
    assert np.array_equal(O.divergence(g, v, "spectral"), O.spectral_divergence(g, v))
