"""Pins of the warm-start network oracle (CPU only).

Each check is independent of the formula it pins: the convolution against a
circular correlation computed with FFTs, the backward pass against adjoint
identities and finite differences of the loss, pooling and upsampling against
closed forms, Adam's first step against its closed form, the grid transfer
against polynomial exactness and block means by brute force, and the
bfloat16 rounding against a bit-level implementation.
"""
import numpy as np
import pytest
import scipy.fft as sfft

from oracle import warmstart_oracle as W

rng = np.random.default_rng(20240131)


def test_bf16_rounding_matches_bit_level_rounding():
    x = rng.standard_normal(20000).astype(np.float32) * np.float32(10.0) ** rng.integers(
        -5, 5, 20000).astype(np.float32)
    bits = x.view(np.uint32).astype(np.uint64)
    lsb = (bits >> 16) & 1
    rounded = ((bits + 0x7FFF + lsb) & 0xFFFF0000).astype(np.uint32).view(np.float32)
    assert np.array_equal(W.bf16(x.astype(np.float64)), rounded.astype(np.float64))
    # ties to even at 1 + 2^-8 (between 1 and 1 + 2^-7) and at 1 + 3 * 2^-8
    assert W.bf16(1 + 2.0 ** -8) == 1.0
    assert W.bf16(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6
    assert W.bf16(0.0) == 0.0 and W.bf16(-1.0) == -1.0


def test_conv_is_fft_circular_correlation():
    B, n, ci, co = 2, (6, 4, 8), 3, 2
    x = rng.standard_normal((B, *n, ci))
    w = rng.standard_normal((co, 27, ci))
    b = rng.standard_normal(co)
    y = W.conv3d(x, w, b)
    for bb in range(B):
        for o in range(co):
            acc = np.zeros(n, dtype=complex)
            for c in range(ci):
                k = np.zeros(n)
                for t, off in enumerate(W.TAPS):
                    k[off[0] % n[0], off[1] % n[1], off[2] % n[2]] += w[o, t, c]
                # sum_o k(o) x(i + o)  <=>  X(f) conj(K(f))
                acc += sfft.fftn(x[bb, ..., c]) * np.conj(sfft.fftn(k))
            ref = sfft.ifftn(acc).real + b[o]
            assert np.allclose(y[bb, ..., o], ref, atol=1e-12)


def test_conv_tap_order_and_direction():
    # a single tap (o1, o2, o3) = (1, 0, -1) reads x(i1 + 1, i2, i3 - 1)
    x = rng.standard_normal((1, 4, 4, 4, 1))
    w = np.zeros((1, 27, 1))
    t = 9 * 2 + 3 * 1 + 0
    w[0, t, 0] = 1.0
    y = W.conv3d(x, w)
    assert np.array_equal(y[0, 1, 2, 3, 0], x[0, 2, 2, 2, 0])
    assert np.array_equal(y[0, 3, 0, 0, 0], x[0, 0, 0, 3, 0])


def test_conv_backward_adjoint_identities():
    B, n, ci, co = 2, (4, 8, 4), 5, 3
    x = rng.standard_normal((B, *n, ci))
    w = rng.standard_normal((co, 27, ci))
    dz = rng.standard_normal((B, *n, co))
    dx, dw, db = W.conv3d_backward(x, w, dz)
    # <conv(x), dz> = <x, dx>  (linear in x)
    assert np.isclose(np.sum(W.conv3d(x, w) * dz), np.sum(x * dx), rtol=1e-12)
    # <conv_{w2}(x), dz> = <w2, dw>  (linear in w)
    w2 = rng.standard_normal(w.shape)
    assert np.isclose(np.sum(W.conv3d(x, w2) * dz), np.sum(w2 * dw), rtol=1e-12)
    # bias: d/db sum(dz * (conv + b)) = sum over voxels of dz
    b2 = rng.standard_normal(co)
    lhs = np.sum((W.conv3d(x, w, b2) - W.conv3d(x, w)) * dz)
    assert np.isclose(lhs, np.sum(b2 * db), rtol=1e-12)


def test_pool_and_upsample():
    x = rng.standard_normal((2, 4, 8, 6, 3))
    # brute-force block mean
    p = W.pool2(x)
    ref = np.zeros_like(p)
    for i in range(2):
        for j in range(2):
            for k in range(2):
                ref += x[:, i::2, j::2, k::2, :] / 8
    assert np.allclose(p, ref, atol=1e-14)
    assert np.allclose(W.pool2(W.up2(p)), p, rtol=0, atol=1e-15)
    d = rng.standard_normal(p.shape)
    e = rng.standard_normal(x.shape)
    assert np.isclose(np.sum(W.pool2(e) * d), np.sum(e * W.pool2_adjoint(d)), rtol=1e-12)
    assert np.isclose(np.sum(W.up2(d) * e), np.sum(d * W.up2_adjoint(e)), rtol=1e-12)


def test_leaky_slope_from_output():
    z = rng.standard_normal(1000)
    y = W.leaky(z)
    h = 1e-7
    fd = (W.leaky(z + h) - W.leaky(z - h)) / (2 * h)
    keep = np.abs(z) > 1e-5
    assert np.allclose(W.leaky_slope(y)[keep], fd[keep], atol=1e-6)


SMALL = W.NetSpec(channels=(2, 3, 2, 4))


def small_problem(R=8, B=2, seed=5):
    r = np.random.default_rng(seed)
    params = {}
    for name, ci, co in SMALL.layers():
        params[name] = (r.standard_normal((co, 27, ci)) * np.sqrt(2.0 / (27 * ci)),
                        0.1 * r.standard_normal(co))
    m0 = r.random((B, R, R, R))
    m1 = r.random((B, R, R, R))
    target = r.standard_normal((B, R, R, R, 3))
    return params, W.input_features(m0, m1), target


def test_network_gradient_finite_differences():
    params, x, target = small_problem()
    loss, grads, _ = W.loss_and_grads(SMALL, params, x, target)
    flat = SMALL.flatten(params)
    g = SMALL.flatten(grads)
    r = np.random.default_rng(11)
    for trial in range(4):
        d = r.standard_normal(flat.size)
        h = 1e-7   # below the distance of every pre-activation from the kink
        lp, _, _ = W.loss_and_grads(SMALL, SMALL.unflatten(flat + h * d), x, target)
        lm, _, _ = W.loss_and_grads(SMALL, SMALL.unflatten(flat - h * d), x, target)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g @ d) <= 1e-6 * max(1.0, abs(fd)), (trial, fd, g @ d)
    # single parameters in the first, a middle and the last layer
    for name in ("enc1a", "dec3a", "head"):
        k0 = 0
        for nm, ci, co in SMALL.layers():
            if nm == name:
                break
            k0 += co * 27 * ci + co
        for k in (k0, k0 + 7):
            e = np.zeros(flat.size)
            e[k] = 1.0
            h = 1e-7   # below the distance of every pre-activation from the kink
            lp, _, _ = W.loss_and_grads(SMALL, SMALL.unflatten(flat + h * e), x, target)
            lm, _, _ = W.loss_and_grads(SMALL, SMALL.unflatten(flat - h * e), x, target)
            assert abs((lp - lm) / (2 * h) - g[k]) <= 1e-7 + 1e-5 * abs(g[k]), (name, k)


def test_network_shapes_and_flatten_roundtrip():
    params, x, target = small_problem(R=16, B=1)
    v, _ = W.forward(SMALL, params, x)
    assert v.shape == (1, 16, 16, 16, 3)
    flat = SMALL.flatten(params)
    assert flat.size == SMALL.param_count()
    back = SMALL.unflatten(flat)
    for name in params:
        assert np.array_equal(back[name][0], params[name][0])
        assert np.array_equal(back[name][1], params[name][1])


def test_network_is_translation_equivariant():
    # periodic convolutions, 2x pooling and upsampling commute with shifts by
    # multiples of 8 voxels (the coarsest level's spacing)
    params, x, _ = small_problem(R=16, B=1)
    v, _ = W.forward(SMALL, params, x)
    vs, _ = W.forward(SMALL, params, np.roll(x, (8, 0, 8), axis=(1, 2, 3)))
    assert np.allclose(np.roll(v, (8, 0, 8), axis=(1, 2, 3)), vs, atol=1e-12)


def test_bf16_storage_changes_little():
    params, x, target = small_problem()
    l64, g64, _ = W.loss_and_grads(SMALL, params, x, target)
    lq, gq, _ = W.loss_and_grads(SMALL, params, x, target, store=W.bf16)
    assert abs(lq - l64) <= 2e-2 * l64
    a, b = SMALL.flatten(g64), SMALL.flatten(gq)
    assert np.linalg.norm(a - b) <= 5e-2 * np.linalg.norm(a)


def test_adam_first_step_closed_form():
    p = rng.standard_normal(100)
    g = rng.standard_normal(100)
    opt = W.Adam(lr=1e-2)
    p1 = opt.step(p, g)
    assert np.allclose(p1, p - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # a constant gradient keeps the bias-corrected moments at g and g^2
    p2 = opt.step(p1, g)
    assert np.allclose(p2, p1 - 1e-2 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-14)


def test_restrict_block_mean_brute_force():
    f = rng.standard_normal((2, 4, 6, 8))
    r = W.restrict2(f)
    for a in range(2):
        for i in range(2):
            for j in range(3):
                for k in range(4):
                    blk = f[a, 2 * i:2 * i + 2, 2 * j:2 * j + 2, 2 * k:2 * k + 2]
                    assert np.isclose(r[a, i, j, k], blk.mean(), rtol=0, atol=1e-15)


def test_prolong_interpolatory_and_cubic_exact():
    f = rng.standard_normal((3, 8, 8, 8))
    p = W.prolong2(f)
    assert np.array_equal(p[:, ::2, ::2, ::2], f)
    # exact on a cubic polynomial away from the periodic wrap
    n = 16
    i = np.arange(n, dtype=np.float64)
    c1, c2, c3 = np.meshgrid(i, i, i, indexing="ij")
    poly = lambda a, b, c: 0.3 * a ** 3 - a * b * c + 2 * b ** 2 - c ** 3 / 7 + a * c ** 2 + 1
    fine = W.prolong2(poly(c1, c2, c3)[None])[0]
    h = np.arange(2 * n) / 2.0
    f1, f2, f3 = np.meshgrid(h, h, h, indexing="ij")
    inner = (slice(4, 2 * n - 6),) * 3
    assert np.allclose(fine[inner], poly(f1, f2, f3)[inner], rtol=0, atol=1e-9)


def test_prolong_fourth_order_on_trig_field():
    errs = []
    for n in (16, 32):
        x = np.arange(n) * 2 * np.pi / n
        c1, c2, c3 = np.meshgrid(x, x, x, indexing="ij")
        f = np.sin(c1) * np.cos(2 * c2) + np.cos(c3)
        xf = np.arange(2 * n) * np.pi / n
        g1, g2, g3 = np.meshgrid(xf, xf, xf, indexing="ij")
        exact = np.sin(g1) * np.cos(2 * g2) + np.cos(g3)
        errs.append(np.abs(W.prolong2(f[None])[0] - exact).max())
    assert 12 < errs[0] / errs[1] < 20      # 2^4 = 16


def test_resample_round_trip_of_bandlimited_field():
    n = 32
    x = np.arange(n) * 2 * np.pi / n
    c1, c2, c3 = np.meshgrid(x, x, x, indexing="ij")
    f = np.cos(c1 + c2) + 0.5 * np.sin(2 * c3)
    # restriction of a trig mode multiplies it by cos(k h / 2) per axis
    r = W.restrict2(f[None])[0]
    h = 2 * np.pi / n
    xc = np.arange(n // 2) * 2 * h + h / 2
    d1, d2, d3 = np.meshgrid(xc, xc, xc, indexing="ij")
    ref = np.cos(h / 2) ** 2 * np.cos(d1 + d2) + 0.5 * np.cos(h) * np.sin(2 * d3)
    assert np.allclose(r, ref, atol=1e-12)
