"""claire_transport_noalloc (the allocation-free transport) against
claire_transport, through the C ABI.

Both run the same kernels (backtrace, brick boxes, nt gathers), so the
outputs must be identical bit for bit. Two calls in a row on one GPU, the
first at the largest grid the scratch array serves and the second smaller,
check that a call leaves nothing behind that changes the next one; a grid over
the limit is refused on the host before anything is launched.
"""
import ctypes

import numpy as np
import pytest

from helpers import f32

pytestmark = pytest.mark.gpu


def _inputs(n, seed, vmax):
    from synthetic import bandlimited_velocity, gaussian_blobs
    m0 = f32(gaussian_blobs(n, seed))
    v = f32(bandlimited_velocity(n, seed + 1000, min(4, min(n) // 2 - 1), vmax))
    return m0, v


def _run_both(n, nt, seed, vmax):
    import torch

    from paper_2401_17493_amd import _lib as L
    lib = L.load()
    m0, v = _inputs(n, seed, vmax)
    dm0 = torch.from_numpy(m0.astype(np.float32)).cuda()
    dv = torch.from_numpy(v.astype(np.float32)).cuda()
    ref = torch.full_like(dm0, float("nan"))
    out = torch.full_like(dm0, float("nan"))
    nx = (ctypes.c_int * 3)(*n)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    print("noalloc case n=%s nt=%d seed=%d" % (n, nt, seed), flush=True)
    rc = lib.claire_transport(ctypes.c_void_p(dm0.data_ptr()), ctypes.c_void_p(dv.data_ptr()), nx,
                              nt, ctypes.c_void_p(ref.data_ptr()), stream)
    assert rc == 0, lib.claire_last_error()
    rc = lib.claire_transport_noalloc(ctypes.c_void_p(dm0.data_ptr()),
                                      ctypes.c_void_p(dv.data_ptr()), nx, nt,
                                      ctypes.c_void_p(out.data_ptr()), stream)
    assert rc == 0, lib.claire_last_error()
    torch.cuda.synchronize()
    a, b = out.cpu().numpy(), ref.cpu().numpy()
    assert np.isfinite(a).all()
    diff = float(np.abs(a - b).max())
    print("noalloc vs claire_transport n=%s nt=%d: max |diff| %.3e" % (n, nt, diff), flush=True)
    assert diff == 0.0
    return m0, v, a


def test_noalloc_transport_two_calls():
    from paper_2401_17493_amd import claire as C
    assert C.transport_noalloc_max_voxels() == 128 ** 3
    # first call at the limit, second smaller (general grid, odd nt) on the
    # same scratch array
    _run_both((128, 128, 128), 4, 1101, 1.0)
    m0, v, out = _run_both((24, 20, 16), 3, 1102, 0.5)
    # and the smaller result against the FP64 oracle (same bar as the
    # transport parity tests)
    import oracle as O
    from helpers import rel_err
    ref = O.transport(O.Grid((24, 20, 16)), m0, v, 3)
    e = rel_err(out, ref)
    print("noalloc vs oracle 24x20x16: %.3e" % e, flush=True)
    assert e < 1e-5


def test_noalloc_rejects_oversize():
    import torch

    from paper_2401_17493_amd import _lib as L
    lib = L.load()
    n = (256, 128, 128)   # 2^22 voxels: over the limit, refused before any launch
    m0 = torch.zeros(n, device="cuda")
    v = torch.zeros((3,) + n, device="cuda")
    out = torch.empty(n, device="cuda")
    rc = lib.claire_transport_noalloc(ctypes.c_void_p(m0.data_ptr()),
                                      ctypes.c_void_p(v.data_ptr()), (ctypes.c_int * 3)(*n), 4,
                                      ctypes.c_void_p(out.data_ptr()), None)
    assert rc == -1
    assert b"scratch limit" in lib.claire_last_error()
