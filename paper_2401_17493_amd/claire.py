"""Python binding of the gfx950 registration engine (argument marshalling only).

Every computation runs in the HIP kernels of ``libclaire_gfx950.so``; this
module checks tensors (CUDA/HIP device, float32, contiguous, shape, 16-byte
alignment), passes raw device pointers and torch's current stream, and turns
status codes into exceptions. Names follow the C ABI in include/claire.h.

Fields are float32 tensors on the GPU: images [n1, n2, n3], vector fields
[3, n1, n2, n3] (structure of arrays), on the periodic grid x_i = 2*pi*i/n.
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import torch

from . import _lib as L

OP_GRAD, OP_DIV, OP_REG, OP_REG_INV, OP_FD8_GRAD, OP_FD8_DIV = 0, 1, 2, 3, 4, 5
OP_NI_PROJECT, OP_NI_PENALTY = 6, 7
DERIV_SPECTRAL, DERIV_FD8 = 0, 1
PRECOND_REG, PRECOND_TWOLEVEL = 0, 1
(KERNEL_INC_STATE_STEP, KERNEL_ADJOINT_STEP, KERNEL_ASSEMBLE, KERNEL_COPY, KERNEL_BACKTRACE,
 KERNEL_INC_STATE_STEP_MIXED) = range(6)
FIELD_DISP_PLUS, FIELD_DISP_MINUS, FIELD_STATE, FIELD_GRAD_STATE, FIELD_ADJOINT, FIELD_DIVV = range(6)

WARNINGS = {1: "gauss-newton max iterations", 2: "line search failed",
            3: "pcg max iterations", 4: "det F <= 0", 5: "pcg nonpositive curvature"}


class ClaireError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("claire error %d: %s" % (code, msg))
        self.code = code


def _check(rc: int) -> int:
    if rc < 0:
        msg = L.load().claire_last_error()
        raise ClaireError(rc, msg.decode() if msg else "")
    return rc


def _stream(stream=None) -> ctypes.c_void_p:
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t: torch.Tensor, shape, name: str) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if t.device.type != "cuda":
        raise ValueError("%s must live on the GPU" % name)
    if t.dtype != torch.float32:
        raise ValueError("%s must be float32" % name)
    if tuple(t.shape) != tuple(shape):
        raise ValueError("%s has shape %s, expected %s" % (name, tuple(t.shape), tuple(shape)))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    if t.data_ptr() % 16:
        raise ValueError("%s must be 16-byte aligned" % name)
    return ctypes.c_void_p(t.data_ptr())


def _nx(n: Sequence[int]):
    return (ctypes.c_int * 3)(*[int(k) for k in n])


def default_opts(**kw) -> L.ClaireOpts:
    """claire_opts with the library defaults, overridden by keyword arguments.
    ``alpha_levels`` may be a sequence of floats."""
    lib = L.load()
    o = L.ClaireOpts()
    lib.claire_opts_default(ctypes.byref(o))
    levels = kw.pop("alpha_levels", None)
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    if levels:
        arr = (ctypes.c_double * len(levels))(*[float(a) for a in levels])
        o.alpha_levels = ctypes.cast(arr, L.c_double_p)
        o.n_levels = len(levels)
        o._levels_keepalive = arr
    return o


class Context:
    """A registration context (claire_ctx) bound to a grid, n_t, alpha and L."""

    def __init__(self, n: Sequence[int], nt: int, alpha: float, reg_order: int = 1,
                 stream=None):
        self.lib = L.load()
        self.n = tuple(int(k) for k in n)
        self.nt = int(nt)
        self.alpha = float(alpha)
        self.reg_order = int(reg_order)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        self._h = ctypes.c_void_p()
        _check(self.lib.claire_ctx_create(ctypes.byref(self._h), _nx(self.n), self.nt,
                                          self.alpha, self.reg_order,
                                          ctypes.c_void_p(self.stream.cuda_stream)))
        self.vshape = (3,) + self.n

    def close(self):
        if self._h:
            self.lib.claire_ctx_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def _new(self, shape, dtype=torch.float32):
        return torch.empty(shape, dtype=dtype, device="cuda")

    def set_alpha(self, alpha: float):
        _check(self.lib.claire_ctx_set_alpha(self._h, float(alpha)))
        self.alpha = float(alpha)

    def set_precision(self, precision: int):
        """0: float32 matvec storage; 1: float16 storage in the Hessian matvec."""
        _check(self.lib.claire_ctx_set_precision(self._h, int(precision)))

    def set_beta(self, beta: float):
        """Near-incompressible model weight (0: plain model) for later setups."""
        _check(self.lib.claire_ctx_set_beta(self._h, float(beta)))

    def set_derivative(self, derivative: int):
        """DERIV_SPECTRAL or DERIV_FD8 for grad m^j, div v (and grad v in detdefgrad)."""
        _check(self.lib.claire_ctx_set_derivative(self._h, int(derivative)))

    def set_images(self, m0: torch.Tensor, m1: torch.Tensor):
        _check(self.lib.claire_ctx_set_images(self._h, _ptr(m0, self.n, "m0"),
                                              _ptr(m1, self.n, "m1")))

    def set_velocity(self, v: torch.Tensor):
        _check(self.lib.claire_ctx_set_velocity(self._h, _ptr(v, self.vshape, "v")))

    def gradient(self):
        g = self._new(self.vshape)
        J = ctypes.c_double()
        _check(self.lib.claire_ctx_gradient(self._h, _ptr(g, self.vshape, "g"), ctypes.byref(J)))
        return g, J.value

    def objective(self, v: torch.Tensor) -> float:
        J = ctypes.c_double()
        _check(self.lib.claire_ctx_objective(self._h, _ptr(v, self.vshape, "v"), ctypes.byref(J)))
        return J.value

    def hessian_matvec(self, vt: torch.Tensor, out: Optional[torch.Tensor] = None):
        out = self._new(self.vshape) if out is None else out
        _check(self.lib.claire_ctx_hessian_matvec(self._h, _ptr(vt, self.vshape, "vt"),
                                                  _ptr(out, self.vshape, "Hvt")))
        return out

    def precond(self, r: torch.Tensor, out: Optional[torch.Tensor] = None):
        out = self._new(self.vshape) if out is None else out
        _check(self.lib.claire_ctx_precond(self._h, _ptr(r, self.vshape, "r"),
                                           _ptr(out, self.vshape, "z")))
        return out

    def precond_twolevel(self, r: torch.Tensor, inner_rtol: float, max_inner: int = 200,
                         out: Optional[torch.Tensor] = None):
        """Two-level zero-velocity preconditioner z = P r at the last
        set_velocity's state; returns (z, inner CG iterations)."""
        out = self._new(self.vshape) if out is None else out
        its = ctypes.c_int(0)
        _check(self.lib.claire_ctx_precond_twolevel(
            self._h, _ptr(r, self.vshape, "r"), _ptr(out, self.vshape, "z"), float(inner_rtol),
            int(max_inner), ctypes.byref(its)))
        return out, its.value

    def solve(self, v0: Optional[torch.Tensor] = None, **opts):
        o = default_opts(reg_order=self.reg_order, **opts)
        v = torch.zeros(self.vshape, dtype=torch.float32, device="cuda") if v0 is None \
            else v0.clone()
        st = L.ClaireStats()
        rc = _check(self.lib.claire_ctx_solve(self._h, ctypes.byref(o),
                                              _ptr(v, self.vshape, "v_inout"), ctypes.byref(st)))
        d = st.as_dict()
        d["status"] = rc
        d["warning"] = WARNINGS.get(rc)
        return v, d

    def solve_trace(self):
        """Per-iterate records and PCG residual histories of the last solve."""
        counts = (ctypes.c_int * 2)()
        _check(self.lib.claire_ctx_solve_trace(self._h, None, 0, None, 0, counts))
        ni, nr = counts[0], counts[1]
        it = (ctypes.c_double * max(1, 8 * ni))()
        res = (ctypes.c_double * max(1, nr))()
        _check(self.lib.claire_ctx_solve_trace(self._h, it, ni, res, nr, counts))
        recs = []
        pos = 0
        for q in range(ni):
            r = it[8 * q:8 * q + 8]
            rec = dict(level=int(r[0]), k=int(r[1]), J=r[2], gnorm=r[3],
                       pcg_its=int(r[4]), gamma=r[5], ls=int(r[6]))
            m = int(r[7])
            if m:
                rec["pcg_res"] = list(res[pos:pos + m])
                pos += m
            recs.append(rec)
        return recs

    def detdefgrad(self, want_field: bool = False):
        det = self._new(self.n, torch.float64) if want_field else None
        stats = (ctypes.c_double * 4)()
        rc = _check(self.lib.claire_ctx_detdefgrad(
            self._h, ctypes.c_void_p(det.data_ptr()) if det is not None else None, stats))
        return det, dict(min=stats[0], mean=stats[1], max=stats[2],
                         nonpositive=int(stats[3]), status=rc)

    def spectral(self, op: int, x: torch.Tensor) -> torch.Tensor:
        shapes = {OP_GRAD: (self.n, self.vshape), OP_DIV: (self.vshape, self.n),
                  OP_REG: (self.vshape, self.vshape), OP_REG_INV: (self.vshape, self.vshape),
                  OP_FD8_GRAD: (self.n, self.vshape), OP_FD8_DIV: (self.vshape, self.n),
                  OP_NI_PROJECT: (self.vshape, self.vshape),
                  OP_NI_PENALTY: (self.vshape, self.vshape)}
        sin, sout = shapes[op]
        out = self._new(sout)
        _check(self.lib.claire_ctx_spectral(self._h, int(op), _ptr(x, sin, "in"),
                                            _ptr(out, sout, "out")))
        return out

    def interpolate(self, f: torch.Tensor, disp: torch.Tensor) -> torch.Tensor:
        nf = 1 if f.dim() == 3 else int(f.shape[0])
        shape = self.n if f.dim() == 3 else (nf,) + self.n
        out = self._new(shape)
        _check(self.lib.claire_ctx_interpolate(self._h, _ptr(f, shape, "f"), nf,
                                               _ptr(disp, self.vshape, "disp"),
                                               _ptr(out, shape, "out")))
        return out

    def get_field(self, which: int, index: int = 0) -> torch.Tensor:
        vec = which in (FIELD_DISP_PLUS, FIELD_DISP_MINUS, FIELD_GRAD_STATE)
        shape = self.vshape if vec else self.n
        out = self._new(shape)
        _check(self.lib.claire_ctx_get_field(self._h, int(which), int(index),
                                             _ptr(out, shape, "out")))
        return out

    def time_kernel(self, kernel: int, reps: int = 20) -> float:
        """Average milliseconds per launch of one hot-path kernel (HIP events)."""
        ms = ctypes.c_double()
        _check(self.lib.claire_ctx_time_kernel(self._h, int(kernel), int(reps), ctypes.byref(ms)))
        return ms.value


# ------------------------------------------------------ stateless functions
def transport(m0: torch.Tensor, v: torch.Tensor, nt: int) -> torch.Tensor:
    n = tuple(m0.shape)
    out = torch.empty_like(m0)
    _check(L.load().claire_transport(_ptr(m0, n, "m0"), _ptr(v, (3,) + n, "v"), _nx(n), int(nt),
                                     _ptr(out, n, "m1_out"), _stream()))
    return out


def transport_noalloc(m0: torch.Tensor, v: torch.Tensor, nt: int, out: torch.Tensor) -> torch.Tensor:
    """claire_transport_noalloc: the caller provides the output; the library
    allocates nothing (its scratch is a fixed per-GPU device array)."""
    n = tuple(m0.shape)
    _check(L.load().claire_transport_noalloc(_ptr(m0, n, "m0"), _ptr(v, (3,) + n, "v"), _nx(n),
                                             int(nt), _ptr(out, n, "m1_out"), _stream()))
    return out


def transport_noalloc_max_voxels() -> int:
    return int(L.load().claire_transport_noalloc_max_voxels())


def gradient(m0, m1, v, alpha: float, nt: int, reg_order: int = 1):
    n = tuple(m0.shape)
    g = torch.empty((3,) + n, dtype=torch.float32, device="cuda")
    J = ctypes.c_double()
    _check(L.load().claire_gradient(_ptr(m0, n, "m0"), _ptr(m1, n, "m1"), _ptr(v, (3,) + n, "v"),
                                    _nx(n), float(alpha), int(nt), int(reg_order),
                                    _ptr(g, (3,) + n, "g"), ctypes.byref(J), _stream()))
    return g, J.value


def hessian_matvec(m0, m1, v, vt, alpha: float, nt: int, reg_order: int = 1):
    n = tuple(m0.shape)
    out = torch.empty((3,) + n, dtype=torch.float32, device="cuda")
    _check(L.load().claire_hessian_matvec(_ptr(m0, n, "m0"), _ptr(m1, n, "m1"),
                                          _ptr(v, (3,) + n, "v"), _ptr(vt, (3,) + n, "vt"),
                                          _nx(n), float(alpha), int(nt), int(reg_order),
                                          _ptr(out, (3,) + n, "Hvt"), _stream()))
    return out


def solve(m0, m1, alpha: float, nt: int, v0=None, **opts):
    n = tuple(m0.shape)
    o = default_opts(**opts)
    v = torch.zeros((3,) + n, dtype=torch.float32, device="cuda") if v0 is None else v0.clone()
    st = L.ClaireStats()
    rc = _check(L.load().claire_solve(_ptr(m0, n, "m0"), _ptr(m1, n, "m1"), _nx(n), float(alpha),
                                      int(nt), ctypes.byref(o), _ptr(v, (3,) + n, "v_inout"),
                                      ctypes.byref(st), _stream()))
    d = st.as_dict()
    d["status"] = rc
    d["warning"] = WARNINGS.get(rc)
    return v, d
