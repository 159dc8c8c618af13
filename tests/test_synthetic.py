"""The seeded input generators: deterministic, correctly shaped and scaled."""
import numpy as np

from synthetic import (WORKLOADS, bandlimited_velocity, ellipsoid_phantom,
                       gaussian_blobs, noise)


def test_blobs_deterministic_and_periodic():
    a = gaussian_blobs((16, 16, 16), 3)
    b = gaussian_blobs((16, 16, 16), 3)
    assert np.array_equal(a, b) and a.min() >= 0 and 0.4 < a.max() < 8.0


def test_velocity_bandlimit_and_scale():
    n = (32, 32, 32)
    v = bandlimited_velocity(n, 7, 4, 0.5)
    assert v.shape == (3,) + n
    assert abs(np.sqrt((v * v).sum(0)).max() - 0.5) < 1e-12
    vh = np.fft.fftn(v[1])
    k = np.fft.fftfreq(32, 1 / 32)
    kk = k[:, None, None] ** 2 + k[None, :, None] ** 2 + k[None, None, :] ** 2
    assert np.abs(vh[kk > 16]).max() < 1e-9 * np.abs(vh).max()
    assert abs(vh[0, 0, 0]) < 1e-9 * np.abs(vh).max()
    assert np.array_equal(v, bandlimited_velocity(n, 7, 4, 0.5))


def test_ellipsoid_phantom_range():
    m = ellipsoid_phantom((32, 32, 32), 5)
    assert -0.05 < m.min() and m.max() < 1.05 and m.max() > 0.8
    assert np.array_equal(m, ellipsoid_phantom((32, 32, 32), 5))


def test_noise_and_workloads():
    z = noise((8, 8, 8), 1, 0.01)
    assert abs(z.std() - 0.01) < 0.003
    assert WORKLOADS["ellipsoids256"]["n"] == (256, 256, 256)
