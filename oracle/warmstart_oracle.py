"""FP64 CPU oracle of the learned warm start: a periodic 3D conv
encoder--decoder that maps (m0, m1) to an initial velocity for the
Gauss--Newton--Krylov solve.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library. It shares no code with
the HIP path.

The network is not part of the paper; it plugs into the solver's warm-start
hook (the initial velocity of Alg. 1, which the paper's parameter
continuation in Section 2.6 also uses: each level starts from the previous
level's solution). Its definition, written out here and implemented
independently in HIP:

* input: 8 channels at a working resolution R^3 (periodic):
  (m0, m1, m1 - m0, 0, 0, 0, 0, 0), channels last, batch first;
* 3x3x3 convolutions with periodic wrap (cross-correlation):
  y(i, co) = b(co) + sum_t sum_ci w(co, t, ci) x(i + o_t, ci), tap
  t = 9 (o1 + 1) + 3 (o2 + 1) + (o3 + 1) for offsets o in {-1, 0, 1}^3;
* LeakyReLU with slope 0.1 after every convolution except the last;
* encoder: two convolutions per level at R, R/2, R/4, R/8 with c1..c4
  channels, 2x2x2 average pooling between levels;
* decoder: nearest-neighbour 2x upsampling, concatenation
  [upsampled, encoder skip] (channels in that order), two convolutions per
  level; a last convolution to 3 channels gives v (channels last);
* loss: mean squared error over all outputs; optimiser: Adam.

Mixed precision (the network's storage format): every convolution operand,
i.e. input features, stored activations, the gradients w.r.t.
pre-activations and the weights, is rounded to bfloat16 (round to nearest
even); all other arithmetic and storage is float32 on the GPU, float64 here.
``store`` arguments take the rounding function (``bf16``) to reproduce those
storage points exactly, or ``None`` for the plain float64 network.

Restriction (2x2x2 block mean) and prolongation (periodic cubic Lagrange
midpoint rule, separable) move fields between the registration grid and the
network's working resolution.

Pins: tests/test_oracle_warmstart.py (FFT circular correlation, adjoint
identities, closed forms, finite differences, Adam's first step).
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np

LEAK = 0.1
IN_CHANNELS = 8
OUT_CHANNELS = 3
TAPS = [(o1, o2, o3) for o1 in (-1, 0, 1) for o2 in (-1, 0, 1) for o3 in (-1, 0, 1)]


def bf16(x):
    """Round to the nearest bfloat16 value (8 significant bits, ties to even),
    returned in float64."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                      # x = m 2^e, 0.5 <= |m| < 1
    return np.ldexp(np.round(m * 256.0), e - 8)


def _keep(x):
    return x


# ------------------------------------------------------------------ layers
def conv3d(x, w, b=None):
    """Periodic 3x3x3 cross-correlation. x: (B, n1, n2, n3, Cin), w: (Cout,
    27, Cin), b: (Cout,) or None -> (B, n1, n2, n3, Cout)."""
    y = 0.0
    for t, o in enumerate(TAPS):
        xs = np.roll(x, shift=(-o[0], -o[1], -o[2]), axis=(1, 2, 3))      # xs(i) = x(i + o)
        y = y + np.tensordot(xs, w[:, t, :], axes=([4], [1]))
    if b is not None:
        y = y + b
    return y


def conv3d_backward(x, w, dz):
    """Gradients of sum(dz * conv3d(x, w, b)) w.r.t. x, w and b."""
    dx = 0.0
    dw = np.zeros_like(w)
    for t, o in enumerate(TAPS):
        xs = np.roll(x, shift=(-o[0], -o[1], -o[2]), axis=(1, 2, 3))
        dw[:, t, :] = np.tensordot(dz, xs, axes=([0, 1, 2, 3], [0, 1, 2, 3]))
        # d/dx(j) of dz(i) w x(i + o) with j = i + o: dz(j - o) w
        dx = dx + np.roll(np.tensordot(dz, w[:, t, :], axes=([4], [0])),
                          shift=(o[0], o[1], o[2]), axis=(1, 2, 3))
    db = dz.sum(axis=(0, 1, 2, 3))
    return dx, dw, db


def leaky(z):
    return np.where(z > 0, z, LEAK * z)


def leaky_slope(y):
    """Derivative of LeakyReLU from its output (same sign as its input)."""
    return np.where(y > 0, 1.0, LEAK)


def pool2(x):
    """2x2x2 block mean of (B, n1, n2, n3, C)."""
    B, n1, n2, n3, C = x.shape
    return x.reshape(B, n1 // 2, 2, n2 // 2, 2, n3 // 2, 2, C).mean(axis=(2, 4, 6))


def pool2_adjoint(d):
    return up2(d) / 8.0


def up2(x):
    """Nearest-neighbour 2x upsampling of (B, n1, n2, n3, C)."""
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def up2_adjoint(d):
    B, n1, n2, n3, C = d.shape
    return d.reshape(B, n1 // 2, 2, n2 // 2, 2, n3 // 2, 2, C).sum(axis=(2, 4, 6))


# ----------------------------------------------------------------- network
@dataclass(frozen=True)
class NetSpec:
    channels: tuple = (16, 32, 64, 128)

    def layers(self):
        """(name, cin, cout) in forward order."""
        c1, c2, c3, c4 = self.channels
        return [
            ("enc1a", IN_CHANNELS, c1), ("enc1b", c1, c1),
            ("enc2a", c1, c2), ("enc2b", c2, c2),
            ("enc3a", c2, c3), ("enc3b", c3, c3),
            ("bota", c3, c4), ("botb", c4, c4),
            ("dec3a", c4 + c3, c3), ("dec3b", c3, c3),
            ("dec2a", c3 + c2, c2), ("dec2b", c2, c2),
            ("dec1a", c2 + c1, c1), ("dec1b", c1, c1),
            ("head", c1, OUT_CHANNELS),
        ]

    def param_count(self):
        return sum(co * 27 * ci + co for _, ci, co in self.layers())

    def unflatten(self, flat):
        """Flat parameter vector (per layer: w as (Cout, 27, Cin) in C order,
        then b) -> dict name -> (w, b)."""
        flat = np.asarray(flat, dtype=np.float64)
        out, k = {}, 0
        for name, ci, co in self.layers():
            nw = co * 27 * ci
            out[name] = (flat[k:k + nw].reshape(co, 27, ci), flat[k + nw:k + nw + co])
            k += nw + co
        assert k == flat.size
        return out

    def flatten(self, params):
        return np.concatenate([np.concatenate([params[name][0].ravel(), params[name][1]])
                               for name, _, _ in self.layers()])


def input_features(m0, m1):
    """(B, R, R, R) images -> (B, R, R, R, 8) network input."""
    m0 = np.asarray(m0, dtype=np.float64)
    m1 = np.asarray(m1, dtype=np.float64)
    x = np.zeros(m0.shape + (IN_CHANNELS,))
    x[..., 0] = m0
    x[..., 1] = m1
    x[..., 2] = m1 - m0
    return x


def forward(spec, params, x, store=None):
    """Network output v (B, R, R, R, 3) and the cache for ``backward``."""
    q = store or _keep
    W = {name: (q(w), b) for name, (w, b) in params.items()}
    cache = {}

    def layer(name, inp):
        y = q(leaky(conv3d(inp, *W[name])))
        cache[name] = (inp, y)
        return y

    x0 = q(x)
    s1 = layer("enc1b", layer("enc1a", x0))
    s2 = layer("enc2b", layer("enc2a", q(pool2(s1))))
    s3 = layer("enc3b", layer("enc3a", q(pool2(s2))))
    bt = layer("botb", layer("bota", q(pool2(s3))))
    d3 = layer("dec3b", layer("dec3a", np.concatenate([up2(bt), s3], axis=4)))
    d2 = layer("dec2b", layer("dec2a", np.concatenate([up2(d3), s2], axis=4)))
    d1 = layer("dec1b", layer("dec1a", np.concatenate([up2(d2), s1], axis=4)))
    v = conv3d(d1, *W["head"])
    cache["head"] = (d1, v)
    cache["skips"] = (s1, s2, s3)
    cache["W"] = W
    return v, cache


def backward(spec, cache, dv, store=None):
    """Parameter gradients (dict name -> (dw, db)) of sum(dv * v)."""
    q = store or _keep
    W = cache["W"]
    s1, s2, s3 = cache["skips"]
    grads = {}

    def conv_grads(name, dz):
        inp = cache[name][0]
        dx, dw, db = conv3d_backward(inp, W[name][0], dz)
        grads[name] = (dw, db)
        return dx

    def through(name, dx):
        """dz of layer `name` from the gradient w.r.t. its output."""
        return q(dx * leaky_slope(cache[name][1]))

    c1, c2, c3, _ = spec.channels
    dx = conv_grads("head", q(dv))
    dx = conv_grads("dec1b", through("dec1b", dx))
    dx = conv_grads("dec1a", through("dec1a", dx))
    dskip1 = dx[..., c2:]
    dx = conv_grads("dec2b", through("dec2b", up2_adjoint(dx[..., :c2])))
    dx = conv_grads("dec2a", through("dec2a", dx))
    dskip2 = dx[..., c3:]
    dx = conv_grads("dec3b", through("dec3b", up2_adjoint(dx[..., :c3])))
    dx = conv_grads("dec3a", through("dec3a", dx))
    dskip3 = dx[..., spec.channels[3]:]
    dx = conv_grads("botb", through("botb", up2_adjoint(dx[..., :spec.channels[3]])))
    dx = conv_grads("bota", through("bota", dx))
    dx = conv_grads("enc3b", through("enc3b", pool2_adjoint(dx) + dskip3))
    dx = conv_grads("enc3a", through("enc3a", dx))
    dx = conv_grads("enc2b", through("enc2b", pool2_adjoint(dx) + dskip2))
    dx = conv_grads("enc2a", through("enc2a", dx))
    dx = conv_grads("enc1b", through("enc1b", pool2_adjoint(dx) + dskip1))
    conv_grads("enc1a", through("enc1a", dx))
    return grads


def mse(v, target):
    """Loss and its gradient w.r.t. v."""
    d = np.asarray(v, dtype=np.float64) - np.asarray(target, dtype=np.float64)
    return float(np.mean(d * d)), 2.0 * d / d.size


def loss_and_grads(spec, params, x, target, store=None):
    v, cache = forward(spec, params, x, store)
    loss, dv = mse(v, target)
    return loss, backward(spec, cache, dv, store), v


@dataclass
class Adam:
    """Adam with bias correction (first and second moment decay b1, b2)."""
    lr: float = 1e-3
    b1: float = 0.9
    b2: float = 0.999
    eps: float = 1e-8
    t: int = 0
    m: np.ndarray = None
    v: np.ndarray = None

    def step(self, p, g):
        p = np.asarray(p, dtype=np.float64)
        g = np.asarray(g, dtype=np.float64)
        if self.m is None:
            self.m = np.zeros_like(p)
            self.v = np.zeros_like(p)
        self.t += 1
        self.m = self.b1 * self.m + (1 - self.b1) * g
        self.v = self.b2 * self.v + (1 - self.b2) * g * g
        mh = self.m / (1 - self.b1 ** self.t)
        vh = self.v / (1 - self.b2 ** self.t)
        return p - self.lr * mh / (np.sqrt(vh) + self.eps)


# ------------------------------------------- grid transfer (channels first)
def restrict2(f):
    """2x2x2 block mean over the last three axes."""
    f = np.asarray(f, dtype=np.float64)
    *lead, n1, n2, n3 = f.shape
    g = f.reshape(*lead, n1 // 2, 2, n2 // 2, 2, n3 // 2, 2)
    return g.mean(axis=(-5, -3, -1))


def _prolong_axis(f, axis):
    """Periodic cubic Lagrange 2x refinement along one axis: even points keep
    the values, midpoints take (-f(i-1) + 9 f(i) + 9 f(i+1) - f(i+2)) / 16."""
    fm1 = np.roll(f, 1, axis=axis)
    fp1 = np.roll(f, -1, axis=axis)
    fp2 = np.roll(f, -2, axis=axis)
    mid = (-fm1 + 9.0 * f + 9.0 * fp1 - fp2) / 16.0
    shape = list(f.shape)
    shape[axis] *= 2
    out = np.empty(shape)
    sl_even = [slice(None)] * f.ndim
    sl_odd = [slice(None)] * f.ndim
    sl_even[axis] = slice(0, None, 2)
    sl_odd[axis] = slice(1, None, 2)
    out[tuple(sl_even)] = f
    out[tuple(sl_odd)] = mid
    return out


def prolong2(f):
    """Separable periodic cubic 2x refinement over the last three axes."""
    f = np.asarray(f, dtype=np.float64)
    for axis in (-3, -2, -1):
        f = _prolong_axis(f, f.ndim + axis)
    return f


def resample(f, n_to):
    """Restrict (block means) or prolong (cubic) by powers of two to n_to per
    axis (cubic grids)."""
    f = np.asarray(f, dtype=np.float64)
    while f.shape[-1] > n_to:
        f = restrict2(f)
    while f.shape[-1] < n_to:
        f = prolong2(f)
    return f


def warm_start(spec, params, m0, m1, res, store=None):
    """Initial velocity [3][n1][n2][n3] for images on an n^3 grid: restrict to
    the working resolution, run the network, prolong back."""
    n = np.asarray(m0).shape[-1]
    a = resample(m0, res)[None]
    b = resample(m1, res)[None]
    v, _ = forward(spec, params, input_features(a, b), store)
    v = np.moveaxis(v[0], -1, 0)          # (3, R, R, R)
    return resample(v, n)
