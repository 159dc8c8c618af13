"""Python binding of the learned warm start (argument marshalling only).

The network, its training step and the grid transfer run in the HIP kernels
of ``libclaire_gfx950.so`` (include/claire_net.h). Images are float32 GPU
tensors [n, n, n] or batches [B, R, R, R]; velocities [3, n, n, n] or
[B, 3, R, R, R]. Parameters travel as one flat float32 tensor in the
layer order of the C header.
"""
from __future__ import annotations

import ctypes
import json
from typing import Optional, Sequence

import numpy as np
import torch

from . import _lib as L
from .claire import _check, _ptr, _stream

DEFAULT_CHANNELS = (16, 32, 64, 128)


class Net:
    """Periodic 3D conv encoder--decoder at working resolution ``res``^3."""

    def __init__(self, res: int = 64, channels: Sequence[int] = DEFAULT_CHANNELS,
                 max_batch: int = 4, seed: int = 0):
        self.lib = L.load()
        self.res = int(res)
        self.channels = tuple(int(c) for c in channels)
        self.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        ch = (ctypes.c_int * 4)(*self.channels)
        _check(self.lib.claire_net_create(ctypes.byref(h), self.res, ch, self.max_batch,
                                          ctypes.c_ulonglong(int(seed)), _stream()))
        self._h = h
        self.nparam = int(self.lib.claire_net_param_count(self._h))

    def close(self):
        if getattr(self, "_h", None):
            self.lib.claire_net_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # --------------------------------------------------------------- params
    def set_params(self, p: torch.Tensor):
        _check(self.lib.claire_net_set_params(self._h, _ptr(p, (self.nparam,), "params")))

    def get_params(self) -> torch.Tensor:
        p = torch.empty(self.nparam, dtype=torch.float32, device="cuda")
        _check(self.lib.claire_net_get_params(self._h, _ptr(p, (self.nparam,), "params")))
        return p

    def get_grads(self) -> torch.Tensor:
        g = torch.empty(self.nparam, dtype=torch.float32, device="cuda")
        _check(self.lib.claire_net_get_grads(self._h, _ptr(g, (self.nparam,), "grads")))
        return g

    def set_grads(self, g: torch.Tensor):
        _check(self.lib.claire_net_set_grads(self._h, _ptr(g, (self.nparam,), "grads")))

    def save(self, path: str):
        p = self.get_params()
        torch.cuda.synchronize()
        np.savez(path, params=p.cpu().numpy(),
                 meta=np.frombuffer(json.dumps({"res": self.res, "channels": self.channels})
                                    .encode(), dtype=np.uint8))

    @classmethod
    def load(cls, path: str, max_batch: int = 1) -> "Net":
        with np.load(path) as z:             # plain arrays, no pickled objects
            meta = json.loads(bytes(z["meta"]).decode())
            params = z["params"].astype(np.float32)
        net = cls(meta["res"], meta["channels"], max_batch=max_batch)
        net.set_params(torch.from_numpy(params).cuda())
        return net

    # ------------------------------------------------------------- compute
    def _batch(self, m: torch.Tensor, name: str):
        if m.dim() == 3:
            m = m.unsqueeze(0)
        return m, int(m.shape[0])

    def forward(self, m0: torch.Tensor, m1: torch.Tensor) -> torch.Tensor:
        m0, B = self._batch(m0, "m0")
        m1, _ = self._batch(m1, "m1")
        R = self.res
        v = torch.empty((B, 3, R, R, R), dtype=torch.float32, device="cuda")
        _check(self.lib.claire_net_forward(self._h, _ptr(m0, (B, R, R, R), "m0"),
                                           _ptr(m1, (B, R, R, R), "m1"), B,
                                           _ptr(v, (B, 3, R, R, R), "v")))
        return v

    def loss_grad(self, m0, m1, target, want_v: bool = False):
        m0, B = self._batch(m0, "m0")
        m1, _ = self._batch(m1, "m1")
        R = self.res
        loss = ctypes.c_double()
        v = torch.empty((B, 3, R, R, R), dtype=torch.float32, device="cuda") if want_v else None
        _check(self.lib.claire_net_loss_grad(
            self._h, _ptr(m0, (B, R, R, R), "m0"), _ptr(m1, (B, R, R, R), "m1"),
            _ptr(target, (B, 3, R, R, R), "target"), B, ctypes.byref(loss),
            _ptr(v, (B, 3, R, R, R), "v") if want_v else None))
        return (loss.value, v) if want_v else loss.value

    def adam_step(self, lr: float):
        _check(self.lib.claire_net_adam_step(self._h, float(lr)))

    def train_step(self, m0, m1, target, lr: float) -> float:
        m0, B = self._batch(m0, "m0")
        m1, _ = self._batch(m1, "m1")
        R = self.res
        loss = ctypes.c_double()
        _check(self.lib.claire_net_train_step(
            self._h, _ptr(m0, (B, R, R, R), "m0"), _ptr(m1, (B, R, R, R), "m1"),
            _ptr(target, (B, 3, R, R, R), "target"), B, float(lr), ctypes.byref(loss)))
        return loss.value

    def warm_start(self, m0: torch.Tensor, m1: torch.Tensor) -> torch.Tensor:
        n = int(m0.shape[0])
        v0 = torch.empty((3, n, n, n), dtype=torch.float32, device="cuda")
        _check(self.lib.claire_net_warm_start(self._h, _ptr(m0, (n, n, n), "m0"),
                                              _ptr(m1, (n, n, n), "m1"), n,
                                              _ptr(v0, (3, n, n, n), "v0")))
        return v0


def resample(src: torch.Tensor, n_dst: int) -> torch.Tensor:
    """Block-mean restriction / cubic prolongation of [n]^3 or [c, n, n, n]."""
    single = src.dim() == 3
    f = src.unsqueeze(0) if single else src
    c, n = int(f.shape[0]), int(f.shape[-1])
    out = torch.empty((c, n_dst, n_dst, n_dst), dtype=torch.float32, device="cuda")
    _check(L.load().claire_resample(_ptr(f, (c, n, n, n), "src"), n, _ptr(out, out.shape, "dst"),
                                    int(n_dst), c, _stream()))
    return out[0] if single else out


def conv3d(x: torch.Tensor, w: torch.Tensor, b: Optional[torch.Tensor], act: bool = False):
    """One network layer on [B, R, R, R, cin] (bfloat16 operands, float32 out)."""
    B, R, cin = int(x.shape[0]), int(x.shape[1]), int(x.shape[-1])
    cout = int(w.shape[0])
    y = torch.empty((B, R, R, R, cout), dtype=torch.float32, device="cuda")
    _check(L.load().claire_conv3d(_ptr(x, (B, R, R, R, cin), "x"), _ptr(w, (cout, 27, cin), "w"),
                                  _ptr(b, (cout,), "b") if b is not None else None, B, R, cin,
                                  cout, 1 if act else 0, _ptr(y, y.shape, "y"), _stream()))
    return y


def conv3d_backward(x: torch.Tensor, w: torch.Tensor, dz: torch.Tensor):
    """(dx, dw, db) of sum(dz * conv3d(x, w)) (bfloat16 operands)."""
    B, R, cin = int(x.shape[0]), int(x.shape[1]), int(x.shape[-1])
    cout = int(w.shape[0])
    dx = torch.empty_like(x)
    dw = torch.empty_like(w)
    db = torch.empty(cout, dtype=torch.float32, device="cuda")
    _check(L.load().claire_conv3d_backward(
        _ptr(x, (B, R, R, R, cin), "x"), _ptr(w, (cout, 27, cin), "w"),
        _ptr(dz, (B, R, R, R, cout), "dz"), B, R, cin, cout, _ptr(dx, dx.shape, "dx"),
        _ptr(dw, dw.shape, "dw"), _ptr(db, (cout,), "db"), _stream()))
    return dx, dw, db
