"""Learned warm start on the GPU against the FP64 oracle
(oracle/warmstart_oracle.py): single layers (forward, backward data, weight
and bias gradients), the grid transfer, the whole network's output and
parameter gradient, Adam, the warm-start pipeline, and a short training run.

Tolerances. A single layer multiplies bfloat16 operands exactly in float32
and accumulates K = 27 cin products in float32: the max-norm error relative
to the largest output stays below ~K 2^-24, well under the 2e-5 bar. For the
whole network, bfloat16 storage of every activation is noise of relative size
~2^-9 per element that the layers propagate: where float32 and float64 sums
round to different bfloat16 neighbours the difference is one ulp, which
perturbs the next layer's pre-activations by about an ulp and so flips further
roundings, so no emulation tracks the GPU element by element. The bar is
therefore the noise ball itself: the oracle's bfloat16 emulation against the
plain float64 network measures it, and the GPU result must lie within twice
that distance of the float64 network (output in relative L2; each layer's
weight and bias gradient within 3x the emulation's own distance).
"""
import numpy as np
import pytest

from oracle import warmstart_oracle as W

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def WS():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_17493_amd import warmstart
    return warmstart


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


# (1, 16, 24, 3), (2, 16, 16, 16) and (1, 16, 48, 16) take the narrow-layer
# kernel (at most 16 output columns, 4x4x16 bricks), the others the 4^3-brick
# or the unstaged kernel
@pytest.mark.parametrize("B,R,cin,cout", [(2, 8, 8, 16), (1, 16, 24, 3), (2, 4, 48, 40),
                                          (1, 2, 16, 8), (2, 16, 16, 16), (1, 16, 48, 16)])
@pytest.mark.parametrize("act", [0, 1])
def test_conv3d_forward(WS, B, R, cin, cout, act):
    r = np.random.default_rng(100 + R + cin + cout)
    x = f32(r.standard_normal((B, R, R, R, cin)))
    w = f32(r.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin))
    b = f32(r.standard_normal(cout))
    y = host(WS.conv3d(dev(x), dev(w), dev(b), act=bool(act)))
    ref = W.conv3d(W.bf16(x), W.bf16(w), b)
    if act:
        ref = W.leaky(ref)
    err = rel(y, ref)
    print("conv3d B%d R%d %d->%d act%d: %.2e" % (B, R, cin, cout, act, err))
    assert err <= 2e-5


# (1, 16, 24, 8), (2, 16, 16, 16) and (2, 16, 32, 16) take the brick-staged
# weight gradient (at most 16 outputs, x3 extent >= 16) with one partly
# filled, one and two 16-channel tiles
@pytest.mark.parametrize("B,R,cin,cout", [(2, 8, 8, 16), (1, 16, 24, 8), (2, 4, 48, 40),
                                          (1, 2, 16, 8), (2, 16, 16, 16), (2, 16, 32, 16)])
def test_conv3d_backward(WS, B, R, cin, cout):
    r = np.random.default_rng(200 + R + cin + cout)
    x = f32(r.standard_normal((B, R, R, R, cin)))
    w = f32(r.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin))
    dz = f32(r.standard_normal((B, R, R, R, cout)))
    dx, dw, db = (host(t) for t in WS.conv3d_backward(dev(x), dev(w), dev(dz)))
    rdx, rdw, rdb = W.conv3d_backward(W.bf16(x), W.bf16(w), W.bf16(dz))
    errs = rel(dx, rdx), rel(dw, rdw), rel(db, rdb)
    print("conv3d backward B%d R%d %d->%d: dx %.2e dw %.2e db %.2e" % ((B, R, cin, cout) + errs))
    assert max(errs) <= 2e-5


# The widths of the shipped network (channels 16, 32, 64, 128): 128 -> 128
# (bottleneck), the decoder concatenations 192 -> 64 and 96 -> 32, whose
# output columns span two or more 64-wide blocks and whose backward-data
# GEMM has more than 64 rows; and the weight gradient at B = 4, R = 64, where
# the voxel reduction is split 1024 ways (the cap). At R = 8 and 4 the
# convolutions have too few 64 x 64 tiles to fill the chip and split their
# reduction (k_conv_halo, and k_conv for the 192-channel input).
PRODUCTION = [(1, 8, 128, 128), (1, 8, 192, 64), (2, 8, 96, 32), (1, 4, 48, 16)]


@pytest.mark.parametrize("B,R,cin,cout", PRODUCTION)
def test_conv3d_production_widths(WS, B, R, cin, cout):
    r = np.random.default_rng(400 + R + cin + cout)
    x = f32(r.standard_normal((B, R, R, R, cin)))
    w = f32(r.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin))
    b = f32(r.standard_normal(cout))
    dz = f32(r.standard_normal((B, R, R, R, cout)))
    y = host(WS.conv3d(dev(x), dev(w), dev(b), act=True))
    ref = W.leaky(W.conv3d(W.bf16(x), W.bf16(w), b))
    dx, dw, db = (host(t) for t in WS.conv3d_backward(dev(x), dev(w), dev(dz)))
    rdx, rdw, rdb = W.conv3d_backward(W.bf16(x), W.bf16(w), W.bf16(dz))
    errs = rel(y, ref), rel(dx, rdx), rel(dw, rdw), rel(db, rdb)
    print("conv3d B%d R%d %d->%d: y %.2e dx %.2e dw %.2e db %.2e" % ((B, R, cin, cout) + errs))
    assert max(errs) <= 2e-5


# Two to six 16-column groups in the narrow-layer kernel (at least 256
# bricks of 4x4x16 voxels: B R^3 >= 65536): forward 16 -> 48, 32 -> 32,
# 16 -> 64, 32 -> 96, and the data gradients of 48 -> 16 and 96 -> 32 (48
# and 96 output columns), the shapes of the two finest decoder layers'
# backward passes.
@pytest.mark.parametrize("B,R,cin,cout", [(2, 32, 16, 48), (2, 32, 32, 32), (2, 32, 16, 64),
                                          (2, 32, 48, 16), (2, 32, 32, 96), (2, 32, 96, 32)])
def test_conv3d_column_groups(WS, B, R, cin, cout):
    r = np.random.default_rng(600 + cin + cout)
    x = f32(r.standard_normal((B, R, R, R, cin)))
    w = f32(r.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin))
    b = f32(r.standard_normal(cout))
    dz = f32(r.standard_normal((B, R, R, R, cout)))
    y = host(WS.conv3d(dev(x), dev(w), dev(b), act=True))
    ref = W.leaky(W.conv3d(W.bf16(x), W.bf16(w), b))
    dx, dw, db = (host(t) for t in WS.conv3d_backward(dev(x), dev(w), dev(dz)))
    rdx, rdw, rdb = W.conv3d_backward(W.bf16(x), W.bf16(w), W.bf16(dz))
    errs = rel(y, ref), rel(dx, rdx), rel(dw, rdw), rel(db, rdb)
    print("conv3d B%d R%d %d->%d: y %.2e dx %.2e dw %.2e db %.2e" % ((B, R, cin, cout) + errs))
    assert max(errs) <= 2e-5


# Weight gradients of wide inputs on 16^3 bricks: the input's 16-channel
# tiles are dealt to 2 or 4 workgroup groups of at most three (64 -> 64,
# 96 -> 32, 192 -> 64), with 2 and 4 tiles of 16 output rows.
@pytest.mark.parametrize("B,R,cin,cout", [(4, 16, 64, 64), (2, 16, 96, 32), (2, 16, 192, 64)])
def test_conv3d_backward_channel_groups(WS, B, R, cin, cout):
    r = np.random.default_rng(700 + cin + cout)
    x = f32(r.standard_normal((B, R, R, R, cin)))
    w = f32(r.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin))
    dz = f32(r.standard_normal((B, R, R, R, cout)))
    dx, dw, db = (host(t) for t in WS.conv3d_backward(dev(x), dev(w), dev(dz)))
    rdx, rdw, rdb = W.conv3d_backward(W.bf16(x), W.bf16(w), W.bf16(dz))
    errs = rel(dx, rdx), rel(dw, rdw), rel(db, rdb)
    print("conv3d backward B%d R%d %d->%d: dx %.2e dw %.2e db %.2e" % ((B, R, cin, cout) + errs))
    assert max(errs) <= 2e-5


def test_wgrad_split_cap(WS):
    # B R^3 = 4 * 64^3 voxels: 2048 chunks of 512 would be needed, the split
    # count is capped at 1024 (chunks of 1024 voxels)
    B, R, cin, cout = 4, 64, 8, 16
    r = np.random.default_rng(500)
    x = f32(r.standard_normal((B, R, R, R, cin)))
    w = f32(r.standard_normal((cout, 27, cin)) / np.sqrt(27 * cin))
    dz = f32(r.standard_normal((B, R, R, R, cout)))
    dx, dw, db = (host(t) for t in WS.conv3d_backward(dev(x), dev(w), dev(dz)))
    rdx, rdw, rdb = W.conv3d_backward(W.bf16(x), W.bf16(w), W.bf16(dz))
    errs = rel(dx, rdx), rel(dw, rdw), rel(db, rdb)
    print("conv3d backward B%d R%d %d->%d: dx %.2e dw %.2e db %.2e" % ((B, R, cin, cout) + errs))
    assert max(errs) <= 2e-5


@pytest.mark.parametrize("n_src,n_dst,c", [(32, 8, 1), (8, 32, 3), (16, 64, 3), (64, 16, 2),
                                           (16, 16, 1)])
def test_resample(WS, n_src, n_dst, c):
    r = np.random.default_rng(300 + n_src + n_dst)
    f = f32(r.standard_normal((c, n_src, n_src, n_src)))
    out = host(WS.resample(dev(f), n_dst))
    ref = W.resample(f, n_dst)
    err = rel(out, ref)
    print("resample %d -> %d (c %d): %.2e" % (n_src, n_dst, c, err))
    assert err <= 2e-6


SPEC = W.NetSpec(channels=(8, 16, 16, 24))


def random_params(spec, seed):
    r = np.random.default_rng(seed)
    params = {}
    for name, ci, co in spec.layers():
        scale = np.sqrt(2.0 / (27 * ci)) * (0.3 if name == "head" else 1.0)
        params[name] = (f32(r.standard_normal((co, 27, ci)) * scale),
                        f32(0.05 * r.standard_normal(co)))
    return params


def smooth_images(B, R, seed):
    r = np.random.default_rng(seed)
    x = np.arange(R) * 2 * np.pi / R
    c1, c2, c3 = np.meshgrid(x, x, x, indexing="ij")
    out = []
    for b in range(B):
        a = r.uniform(0.5, 1.5, 6)
        p = r.uniform(0, 2 * np.pi, 6)
        out.append(0.5 + 0.2 * (np.sin(a[0] * c1 + p[0]) * np.cos(c2 + p[1]) +
                                np.cos(c3 + p[2]) * np.sin(2 * c1 + p[3]) +
                                0.5 * np.sin(c2 + c3 + p[4])))
    return f32(np.array(out))


def l2rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


def test_network_forward_and_gradient(WS):
    B, R = 2, 16
    params = random_params(SPEC, 7)
    m0 = smooth_images(B, R, 1)
    m1 = smooth_images(B, R, 2)
    target = f32(np.random.default_rng(3).standard_normal((B, 3, R, R, R)) * 0.3)
    flat = f32(SPEC.flatten(params))
    with WS.Net(R, SPEC.channels, max_batch=B) as net:
        assert net.nparam == SPEC.param_count()
        net.set_params(dev(flat))
        assert np.array_equal(host(net.get_params()), flat)
        loss, v = net.loss_grad(dev(m0), dev(m1), dev(target), want_v=True)
        g = host(net.get_grads())
        v = host(v)
        v2 = host(net.forward(dev(m0), dev(m1)))
    assert np.array_equal(v, v2)          # deterministic
    x = W.input_features(m0, m1)
    t_cl = np.moveaxis(target, 1, -1)
    lq, gq, vq = W.loss_and_grads(SPEC, params, x, t_cl, store=W.bf16)
    l64, g64, v64 = W.loss_and_grads(SPEC, params, x, t_cl)
    vq = np.moveaxis(vq, -1, 1)
    v64 = np.moveaxis(v64, -1, 1)
    noise = l2rel(vq, v64)                 # what bfloat16 storage costs (oracle vs oracle)
    print("net v (rel L2): gpu-emulated %.2e, gpu-float64 %.2e, emulated-float64 %.2e; "
          "max-norm gpu-float64 %.2e; loss %.6e / %.6e / %.6e" % (
              l2rel(v, vq), l2rel(v, v64), noise, rel(v, v64), loss, lq, l64))
    gd, gqd, g64d = SPEC.unflatten(g), SPEC.unflatten(SPEC.flatten(gq)), \
        SPEC.unflatten(SPEC.flatten(g64))
    worst = 0.0
    for name, _, _ in SPEC.layers():
        for k, what in ((0, "w"), (1, "b")):
            e_gpu = l2rel(gd[name][k], g64d[name][k])
            e_q = l2rel(gqd[name][k], g64d[name][k])
            print("  grad %-5s %s: gpu-float64 %.2e, emulated-float64 %.2e, gpu-emulated %.2e" % (
                name, what, e_gpu, e_q, l2rel(gd[name][k], gqd[name][k])))
            worst = max(worst, e_gpu / max(e_q, 1e-3))
    # the GPU network sits inside the bfloat16 noise ball that the oracle's own
    # bfloat16 emulation measures against the float64 network
    assert l2rel(v, v64) <= 2 * noise + 1e-3
    assert abs(loss - l64) <= 1e-2 * l64
    assert worst <= 3.0, worst


def test_production_network_forward_and_gradient(WS):
    # the shipped network's widths (16, 32, 64, 128) at R = 32, within the
    # same bfloat16 noise ball as above
    from paper_2401_17493_amd.warmstart import DEFAULT_CHANNELS
    spec = W.NetSpec(channels=tuple(DEFAULT_CHANNELS))
    B, R = 1, 32
    params = random_params(spec, 17)
    m0 = smooth_images(B, R, 41)
    m1 = smooth_images(B, R, 42)
    target = f32(np.random.default_rng(43).standard_normal((B, 3, R, R, R)) * 0.3)
    with WS.Net(R, spec.channels, max_batch=B) as net:
        net.set_params(dev(f32(spec.flatten(params))))
        loss, v = net.loss_grad(dev(m0), dev(m1), dev(target), want_v=True)
        g = host(net.get_grads())
        v = host(v)
    x = W.input_features(m0, m1)
    t_cl = np.moveaxis(target, 1, -1)
    lq, gq, vq = W.loss_and_grads(spec, params, x, t_cl, store=W.bf16)
    l64, g64, v64 = W.loss_and_grads(spec, params, x, t_cl)
    vq = np.moveaxis(vq, -1, 1)
    v64 = np.moveaxis(v64, -1, 1)
    noise = l2rel(vq, v64)
    print("production net v (rel L2): gpu-float64 %.2e, emulated-float64 %.2e; loss %.6e / %.6e"
          % (l2rel(v, v64), noise, loss, l64))
    gd, gqd, g64d = spec.unflatten(g), spec.unflatten(spec.flatten(gq)), \
        spec.unflatten(spec.flatten(g64))
    worst = 0.0
    for name, _, _ in spec.layers():
        for k, what in ((0, "w"), (1, "b")):
            e_gpu = l2rel(gd[name][k], g64d[name][k])
            e_q = l2rel(gqd[name][k], g64d[name][k])
            print("  grad %-5s %s: gpu-float64 %.2e, emulated-float64 %.2e" % (
                name, what, e_gpu, e_q))
            worst = max(worst, e_gpu / max(e_q, 1e-3))
    assert l2rel(v, v64) <= 2 * noise + 1e-3
    assert abs(loss - l64) <= 1e-2 * l64
    assert worst <= 3.0, worst


def test_adam_steps(WS):
    B, R = 1, 8
    spec = W.NetSpec(channels=(8, 8, 8, 8))
    params = random_params(spec, 11)
    flat = f32(spec.flatten(params))
    r = np.random.default_rng(12)
    g1 = f32(r.standard_normal(flat.size))
    g2 = f32(r.standard_normal(flat.size))
    opt = W.Adam(lr=3e-3)
    ref = opt.step(opt.step(flat, g1), g2)
    with WS.Net(R, spec.channels, max_batch=B) as net:
        net.set_params(dev(flat))
        net.set_grads(dev(g1))
        net.adam_step(3e-3)
        net.set_grads(dev(g2))
        net.adam_step(3e-3)
        p = host(net.get_params())
    err = np.abs(p - ref).max()
    print("adam two steps: max |dp| error %.2e (step size 3e-3)" % err)
    assert err <= 1e-6


def test_warm_start_pipeline(WS):
    R, n = 16, 64
    params = random_params(SPEC, 21)
    flat = f32(SPEC.flatten(params))
    m0 = smooth_images(1, n, 5)[0]
    m1 = smooth_images(1, n, 6)[0]
    with WS.Net(R, SPEC.channels, max_batch=1) as net:
        net.set_params(dev(flat))
        v0 = host(net.warm_start(dev(m0), dev(m1)))
    ref = W.warm_start(SPEC, params, m0, m1, R, store=W.bf16)
    ref64 = W.warm_start(SPEC, params, m0, m1, R)
    err, noise = l2rel(v0, ref64), l2rel(ref, ref64)
    print("warm start %d^3 via %d^3 (rel L2): gpu-float64 %.2e, emulated-float64 %.2e" % (
        n, R, err, noise))
    assert v0.shape == (3, n, n, n)
    assert err <= 2 * noise + 1e-3


def test_training_fits_a_batch(WS):
    # the whole training step (forward, backward, Adam) lowers the loss on a
    # fixed batch by a large factor
    B, R = 2, 16
    m0 = smooth_images(B, R, 31)
    m1 = smooth_images(B, R, 32)
    x = np.arange(R) * 2 * np.pi / R
    c1, c2, c3 = np.meshgrid(x, x, x, indexing="ij")
    target = f32(np.stack([np.stack([0.3 * np.sin(c2 + b), 0.2 * np.cos(c3 - b),
                                     0.1 * np.sin(c1 + c3)]) for b in range(B)]))
    with WS.Net(R, (8, 16, 16, 24), max_batch=B, seed=3) as net:
        a, b, t = dev(m0), dev(m1), dev(target)
        first = net.train_step(a, b, t, 1e-3)
        for _ in range(150):
            last = net.train_step(a, b, t, 1e-3)
    print("training: loss %.4e -> %.4e" % (first, last))
    assert np.isfinite(last) and last < 0.1 * first
