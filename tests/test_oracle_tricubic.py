"""Pins of the oracle's tricubic Lagrange interpolation (Section 2.5.4, p = 3).

Cubic Lagrange interpolation through four nodes reproduces every polynomial of
degree <= 3 per axis, and this determines the four weights uniquely; the tests
check that on all 64 tensor monomials, plus grid-point identity, periodic wrap
(against numpy.roll), partition of unity and fourth-order convergence.
"""
import numpy as np
import pytest

import oracle as O

N = (16, 12, 20)


def _tensor_cubic(coef, q1, q2, q3):
    out = 0.0
    for p in range(4):
        for r in range(4):
            for s in range(4):
                out = out + coef[p, r, s] * q1**p * q2**r * q3**s
    return out


def test_exact_on_tensor_cubics_points():
    rng = np.random.default_rng(1)
    coef = rng.standard_normal((4, 4, 4))
    i1, i2, i3 = np.meshgrid(*[np.arange(k, dtype=float) for k in N], indexing="ij")
    f = _tensor_cubic(coef, i1 / 8, i2 / 8, i3 / 8)
    # interior points: the 4-node stencil must not cross the periodic wrap
    q = np.stack([rng.uniform(1.0, k - 3.0, 400) for k in N], axis=1)
    got = O.interpolate_points(f, q)
    ref = _tensor_cubic(coef, q[:, 0] / 8, q[:, 1] / 8, q[:, 2] / 8)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


def test_exact_on_tensor_cubics_grid_displacements():
    rng = np.random.default_rng(2)
    coef = rng.standard_normal((4, 4, 4))
    ii = np.meshgrid(*[np.arange(k, dtype=float) for k in N], indexing="ij")
    f = _tensor_cubic(coef, ii[0] / 8, ii[1] / 8, ii[2] / 8)
    d = np.stack([rng.uniform(-0.99, 0.99, N) for _ in range(3)])
    got = O.interpolate(f, d)
    q = [ii[a] + d[a] for a in range(3)]
    inner = np.ones(N, dtype=bool)
    for a in range(3):
        inner &= (np.floor(q[a]) >= 1) & (np.floor(q[a]) <= N[a] - 3)
    ref = _tensor_cubic(coef, q[0] / 8, q[1] / 8, q[2] / 8)
    assert inner.sum() > 1000
    assert np.abs(got - ref)[inner].max() <= 1e-12 * np.abs(ref).max()


def test_each_monomial_separately():
    # a transposed node or weight would break one of these 1D pins
    rng = np.random.default_rng(3)
    for p in range(4):
        f = np.broadcast_to((np.arange(N[0], dtype=float)[:, None, None] / 4) ** p, N).copy()
        q = np.stack([rng.uniform(1, N[0] - 3, 50), rng.uniform(0, N[1], 50),
                      rng.uniform(0, N[2], 50)], axis=1)
        got = O.interpolate_points(f, q)
        assert np.abs(got - (q[:, 0] / 4) ** p).max() <= 1e-12 * max(1, (N[0] / 4) ** p)


def test_zero_and_integer_displacement_is_exact_roll():
    rng = np.random.default_rng(4)
    f = rng.standard_normal(N)
    assert np.array_equal(O.interpolate(f, np.zeros((3,) + N)), f)
    shift = (3, -5, 27)            # crosses the periodic boundary, |27| > n3
    d = np.stack([np.full(N, float(s)) for s in shift])
    ref = np.roll(f, tuple(-s for s in shift), axis=(0, 1, 2))
    assert np.array_equal(O.interpolate(f, d), ref)


def test_partition_of_unity_and_stacked_fields():
    rng = np.random.default_rng(5)
    d = np.stack([rng.uniform(-7, 7, N) for _ in range(3)])
    c = O.interpolate(np.full(N, 3.25), d)
    assert np.abs(c - 3.25).max() < 1e-13
    f = rng.standard_normal((2,) + N)
    both = O.interpolate(f, d)
    assert np.array_equal(both[1], O.interpolate(f[1], d))


def test_grid_and_point_forms_agree_across_wrap():
    rng = np.random.default_rng(6)
    f = rng.standard_normal(N)
    d = np.stack([rng.uniform(-9, 9, N) for _ in range(3)])
    ii = np.meshgrid(*[np.arange(k, dtype=float) for k in N], indexing="ij")
    q = np.stack([(ii[a] + d[a]).ravel() for a in range(3)], axis=1)
    got = O.interpolate_points(f, q).reshape(N)
    assert np.abs(got - O.interpolate(f, d)).max() < 1e-12


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_fourth_order_convergence_periodic(axis):
    # smooth periodic function; the same fractional offset (2.5 voxels) at
    # each resolution, so the error constant is the same and only h changes
    errs = []
    for n in (16, 32, 64):
        shape = [4, 4, 4]
        shape[axis] = n
        x = np.arange(n) * 2 * np.pi / n
        prof = np.exp(np.sin(x))
        f = np.broadcast_to(prof.reshape([-1 if a == axis else 1 for a in range(3)]),
                            shape).copy()
        delta = 2.5 * (2 * np.pi / n)                  # physical offset
        d = np.zeros((3,) + tuple(shape))
        d[axis] = 2.5
        got = O.interpolate(f, d)
        ref = np.exp(np.sin(x + delta)).reshape([-1 if a == axis else 1 for a in range(3)])
        errs.append(np.abs(got - ref).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates.min() > 3.5, (errs, rates)
