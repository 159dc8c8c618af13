"""ctypes view of ``libclaire_gfx950.so`` (the C ABI declared in include/claire.h and
include/claire_net.h).

Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libclaire_gfx950.so")

c_int = ctypes.c_int
c_double = ctypes.c_double
c_void_p = ctypes.c_void_p
c_int_p = ctypes.POINTER(ctypes.c_int)
c_double_p = ctypes.POINTER(ctypes.c_double)


class ClaireOpts(ctypes.Structure):
    _fields_ = [
        ("reg_order", c_int),
        ("precision", c_int),
        ("gtol", c_double),
        ("gabs", c_double),
        ("forcing", c_int),
        ("max_gn", c_int),
        ("max_pcg", c_int),
        ("fixed_pcg_iters", c_int),
        ("max_linesearch", c_int),
        ("armijo_c1", c_double),
        ("alpha_levels", c_double_p),
        ("n_levels", c_int),
        ("compute_det", c_int),
        ("tol_from_zero", c_int),
        ("derivative", c_int),
        ("precond", c_int),
        ("beta", c_double),
    ]


class ClaireStats(ctypes.Structure):
    _fields_ = [
        ("gn_iters", c_int),
        ("matvecs", c_int),
        ("pde_solves", c_int),
        ("linesearch_trials", c_int),
        ("pcg_max_hits", c_int),
        ("J0", c_double),
        ("J", c_double),
        ("rel_mismatch", c_double),
        ("rel_grad", c_double),
        ("det_min", c_double),
        ("det_mean", c_double),
        ("det_max", c_double),
        ("det_nonpositive", ctypes.c_longlong),
        ("seconds", c_double),
        ("inner_iters", c_int),
        ("initial_rejected", c_int),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# name -> (restype, argtypes)
SIGNATURES = {
    "claire_opts_default": (None, [ctypes.POINTER(ClaireOpts)]),
    "claire_last_error": (ctypes.c_char_p, []),
    "claire_ctx_create": (c_int, [ctypes.POINTER(c_void_p), c_int_p, c_int, c_double, c_int, c_void_p]),
    "claire_ctx_destroy": (c_int, [c_void_p]),
    "claire_ctx_set_alpha": (c_int, [c_void_p, c_double]),
    "claire_ctx_set_images": (c_int, [c_void_p, c_void_p, c_void_p]),
    "claire_ctx_set_velocity": (c_int, [c_void_p, c_void_p]),
    "claire_ctx_gradient": (c_int, [c_void_p, c_void_p, c_double_p]),
    "claire_ctx_objective": (c_int, [c_void_p, c_void_p, c_double_p]),
    "claire_ctx_hessian_matvec": (c_int, [c_void_p, c_void_p, c_void_p]),
    "claire_ctx_precond": (c_int, [c_void_p, c_void_p, c_void_p]),
    "claire_ctx_precond_twolevel": (c_int, [c_void_p, c_void_p, c_void_p, c_double, c_int,
                                            c_void_p]),
    "claire_ctx_set_precision": (c_int, [c_void_p, c_int]),
    "claire_ctx_set_derivative": (c_int, [c_void_p, c_int]),
    "claire_ctx_set_beta": (c_int, [c_void_p, c_double]),
    "claire_ctx_solve": (c_int, [c_void_p, ctypes.POINTER(ClaireOpts), c_void_p,
                                 ctypes.POINTER(ClaireStats)]),
    "claire_ctx_detdefgrad": (c_int, [c_void_p, c_void_p, c_double_p]),
    "claire_ctx_solve_trace": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_int, c_int_p]),
    "claire_ctx_spectral": (c_int, [c_void_p, c_int, c_void_p, c_void_p]),
    "claire_ctx_interpolate": (c_int, [c_void_p, c_void_p, c_int, c_void_p, c_void_p]),
    "claire_ctx_get_field": (c_int, [c_void_p, c_int, c_int, c_void_p]),
    "claire_ctx_time_kernel": (c_int, [c_void_p, c_int, c_int, c_double_p]),
    "claire_transport": (c_int, [c_void_p, c_void_p, c_int_p, c_int, c_void_p, c_void_p]),
    "claire_transport_noalloc": (c_int, [c_void_p, c_void_p, c_int_p, c_int, c_void_p,
                                         c_void_p]),
    "claire_transport_noalloc_max_voxels": (ctypes.c_longlong, []),
    "claire_gradient": (c_int, [c_void_p, c_void_p, c_void_p, c_int_p, c_double, c_int, c_int,
                                c_void_p, c_double_p, c_void_p]),
    "claire_hessian_matvec": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int_p, c_double,
                                      c_int, c_int, c_void_p, c_void_p]),
    "claire_solve": (c_int, [c_void_p, c_void_p, c_int_p, c_double, c_int,
                             ctypes.POINTER(ClaireOpts), c_void_p, ctypes.POINTER(ClaireStats),
                             c_void_p]),
    # learned warm start (include/claire_net.h)
    "claire_net_create": (c_int, [ctypes.POINTER(c_void_p), c_int, c_int_p, c_int,
                                  ctypes.c_ulonglong, c_void_p]),
    "claire_net_destroy": (c_int, [c_void_p]),
    "claire_net_param_count": (ctypes.c_longlong, [c_void_p]),
    "claire_net_set_params": (c_int, [c_void_p, c_void_p]),
    "claire_net_get_params": (c_int, [c_void_p, c_void_p]),
    "claire_net_get_grads": (c_int, [c_void_p, c_void_p]),
    "claire_net_set_grads": (c_int, [c_void_p, c_void_p]),
    "claire_net_forward": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    "claire_net_loss_grad": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_double_p,
                                     c_void_p]),
    "claire_net_adam_step": (c_int, [c_void_p, c_double]),
    "claire_net_train_step": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_int, c_double,
                                      c_double_p]),
    "claire_net_warm_start": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_void_p]),
    "claire_resample": (c_int, [c_void_p, c_int, c_void_p, c_int, c_int, c_void_p]),
    "claire_conv3d": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int, c_int,
                              c_void_p, c_void_p]),
    "claire_conv3d_backward": (c_int, [c_void_p, c_void_p, c_void_p, c_int, c_int, c_int, c_int,
                                       c_void_p, c_void_p, c_void_p, c_void_p]),
}

_lib = None


def load():
    """Load the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            "libclaire_gfx950.so is not built: run `python -c 'import __graft_entry__ as g; "
            "g.build()'` (or `python -m paper_2401_17493_amd.build`) first")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
