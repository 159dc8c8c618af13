"""Seeded synthetic images and velocity fields on the periodic grid [0, 2*pi)^3.

The paper's measurements use clinical T1 brain MRI of about 256^3 voxels with
intensities in [0, 1] (Section 3). Those scans are not available here; the
generators below produce inputs of the same size class, intensity range and
smoothness:

* ``gaussian_blobs``: a sum of periodised Gaussians (small smoke workloads);
* ``ellipsoid_phantom``: nested ellipsoids with piecewise-constant
  intensities, blurred periodically (a head-like phantom with sharp tissue
  boundaries softened to about one voxel);
* ``bandlimited_velocity``: a stationary velocity with random Fourier
  coefficients up to a Euclidean wavenumber radius, scaled to a given maximum
  pointwise speed.

Every array is float64 in C order [n1][n2][n3] (x3 fastest); vector fields are
structure-of-arrays [3][n1][n2][n3]. Grid point i along axis a sits at
x_a = i * 2*pi / n_a.
"""

from __future__ import annotations

import numpy as np

TWO_PI = 2.0 * np.pi

# Workload recipes (sizes, time steps, regulariser, weights, random seeds).
# "reg_order" 1 = H1 seminorm (symbol |k|^2), 2 = H2 seminorm (|k|^4).
WORKLOADS = {
    "blobs32": dict(
        n=(32, 32, 32), nt=4, reg_order=1, alphas=(1e-2,), phantom="blobs",
        kmax=4, vmax=0.5, noise=0.0, seed=1001, pcg_fixed=10,
    ),
    "ellipsoids128": dict(
        n=(128, 128, 128), nt=4, reg_order=2, alphas=(1e-1, 1e-2, 1e-3, 1e-4),
        phantom="ellipsoids", kmax=8, vmax=1.0, noise=0.01, seed=1002, gtol=5e-2,
    ),
    "ellipsoids256": dict(
        n=(256, 256, 256), nt=4, reg_order=1, alphas=(1e-3,), phantom="ellipsoids",
        kmax=8, vmax=1.0, noise=0.01, seed=1003, gtol=5e-2,
    ),
    "ellipsoids512": dict(
        n=(512, 512, 512), nt=8, reg_order=1, alphas=(1e-3,), phantom="ellipsoids",
        kmax=16, vmax=1.0, noise=0.01, seed=1005, gtol=5e-2,
    ),
    # the grid of the paper's NIREP brain images (256 x 300 x 256), same phantom recipe
    "ellipsoids_nirep": dict(
        n=(256, 300, 256), nt=4, reg_order=1, alphas=(1e-3,), phantom="ellipsoids",
        kmax=8, vmax=1.0, noise=0.01, seed=1006, gtol=5e-2,
    ),
}


def grid_coordinates(n):
    """1D node coordinates x_a = i * 2*pi / n_a, one array per axis."""
    return [np.arange(k, dtype=np.float64) * (TWO_PI / k) for k in n]


def _min_image(d):
    """Periodic (minimum-image) difference on a 2*pi-periodic axis."""
    return d - TWO_PI * np.round(d / TWO_PI)


def gaussian_blobs(n, seed, count=8, sigma=0.3, amp_range=(0.5, 1.0)):
    """Sum of ``count`` periodised Gaussians of width ``sigma`` (physical units).

    Centres are uniform on [0, 2*pi)^3 and amplitudes uniform on ``amp_range``.
    """
    rng = np.random.default_rng(seed)
    centres = rng.uniform(0.0, TWO_PI, size=(count, 3))
    amps = rng.uniform(amp_range[0], amp_range[1], size=count)
    x1, x2, x3 = grid_coordinates(n)
    out = np.zeros(tuple(n), dtype=np.float64)
    for c, a in zip(centres, amps):
        d1 = _min_image(x1 - c[0])[:, None, None]
        d2 = _min_image(x2 - c[1])[None, :, None]
        d3 = _min_image(x3 - c[2])[None, None, :]
        out += a * np.exp(-(d1 * d1 + d2 * d2 + d3 * d3) / (2.0 * sigma * sigma))
    return out


def _periodic_blur(u, sigma_vox):
    """Periodic Gaussian blur of width ``sigma_vox`` voxels (FFT multiplier)."""
    n = u.shape
    f1 = np.fft.fftfreq(n[0])[:, None, None]
    f2 = np.fft.fftfreq(n[1])[None, :, None]
    f3 = np.fft.rfftfreq(n[2])[None, None, :]
    mult = np.exp(-2.0 * np.pi**2 * sigma_vox**2 * (f1 * f1 + f2 * f2 + f3 * f3))
    return np.fft.irfftn(np.fft.rfftn(u) * mult, s=n)


def ellipsoid_phantom(n, seed, levels=(0.2, 0.4, 0.6, 0.8, 1.0),
                      scales=(1.0, 0.8, 0.6, 0.4, 0.2), blur_vox=1.0):
    """Nested axis-aligned ellipsoids, intensities rising inwards, then blurred.

    Centre 2*pi*U[0.45, 0.55]^3; outer full axes 2*pi*U[0.3, 0.8] per axis;
    the k-th ellipsoid has the outer axes times ``scales[k]`` and intensity
    ``levels[k]``. The piecewise-constant image is blurred periodically with a
    Gaussian of ``blur_vox`` voxels.
    """
    rng = np.random.default_rng(seed)
    centre = TWO_PI * rng.uniform(0.45, 0.55, size=3)
    full_axes = TWO_PI * rng.uniform(0.3, 0.8, size=3)
    x1, x2, x3 = grid_coordinates(n)
    d1 = _min_image(x1 - centre[0])[:, None, None]
    d2 = _min_image(x2 - centre[1])[None, :, None]
    d3 = _min_image(x3 - centre[2])[None, None, :]
    img = np.zeros(tuple(n), dtype=np.float64)
    for lev, sc in zip(levels, scales):
        a = 0.5 * sc * full_axes
        inside = (d1 / a[0]) ** 2 + (d2 / a[1]) ** 2 + (d3 / a[2]) ** 2 <= 1.0
        img[inside] = lev
    if blur_vox > 0:
        img = _periodic_blur(img, blur_vox)
    return img


def _lowpass_real_field(coef, kmax, n):
    """Re sum_k coef[k] exp(i k.x) over the integer cube |k_a| <= kmax (separable)."""
    ks = np.arange(-kmax, kmax + 1, dtype=np.float64)
    xs = grid_coordinates(n)
    e = [np.exp(1j * np.outer(ks, x)) for x in xs]  # [2K+1, n_a]
    t = np.einsum("abc,cz->abz", coef, e[2])        # [2K+1, 2K+1, n3]
    t = np.einsum("abz,by->ayz", t, e[1])           # [2K+1, n2, n3]
    # Real part of sum_a e1[a, x] * t[a, y, z], without forming the complex cube.
    re = np.tensordot(e[0].real.T, t.real, axes=(1, 0))
    re -= np.tensordot(e[0].imag.T, t.imag, axes=(1, 0))
    return re


def bandlimited_velocity(n, seed, kmax, vmax):
    """Stationary velocity [3][n1][n2][n3] with Fourier support 1 <= |k|_2 <= kmax.

    Each component takes independent N(0,1) real and imaginary coefficients on
    the integer wavenumbers inside the ball; the real part of the Fourier sum
    is the field (equivalent to Hermitian symmetrisation). The field is then
    scaled so that the pointwise Euclidean speed peaks at ``vmax``.
    """
    if any(2 * kmax >= k for k in n):
        raise ValueError("kmax must stay below the Nyquist wavenumber on every axis")
    rng = np.random.default_rng(seed)
    ks = np.arange(-kmax, kmax + 1)
    kk = ks[:, None, None] ** 2 + ks[None, :, None] ** 2 + ks[None, None, :] ** 2
    mask = (kk >= 1) & (kk <= kmax * kmax)
    side = 2 * kmax + 1
    v = np.empty((3,) + tuple(n), dtype=np.float64)
    for a in range(3):
        re = rng.standard_normal((side, side, side))
        im = rng.standard_normal((side, side, side))
        coef = np.where(mask, re + 1j * im, 0.0)
        v[a] = _lowpass_real_field(coef, kmax, n)
    speed = np.sqrt(np.sum(v * v, axis=0)).max()
    return v * (vmax / speed)


def noise(n, seed, std):
    """Independent N(0, std^2) voxel noise."""
    return np.random.default_rng(seed).normal(0.0, std, size=tuple(n))


def trig_field(n, seed, terms=6, kfrac=0.5):
    """Random real trigonometric polynomial and its terms.

    Returns (u, terms) with u(x) = sum_t a_t cos(k_t.x) + b_t sin(k_t.x),
    integer wavenumbers |k_t,a| < kfrac * n_a / 2 (strictly below Nyquist).
    """
    rng = np.random.default_rng(seed)
    xs = grid_coordinates(n)
    lim = [max(1, int(kfrac * k / 2) - 1) for k in n]
    u = np.zeros(tuple(n), dtype=np.float64)
    out = []
    for _ in range(terms):
        k = np.array([rng.integers(-l, l + 1) for l in lim])
        a, b = rng.standard_normal(2)
        phase = (k[0] * xs[0])[:, None, None] + (k[1] * xs[1])[None, :, None] \
            + (k[2] * xs[2])[None, None, :]
        u += a * np.cos(phase) + b * np.sin(phase)
        out.append((k, a, b))
    return u, out
