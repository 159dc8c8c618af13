"""Parity at the benchmark's full size: 256^3, n_t = 4, H1, alpha = 1e-3, the
nested-ellipsoid workload with its band-limited velocity, in the launch
configuration the benchmark times (same context API, same kernels).

The FP64 oracle computes the whole per-velocity setup and one Hessian matvec
on the host (tens of seconds on the machine's cores); every output is compared
element by element at the 1e-5 max-norm bar. The velocity is half the true
one, so departure points are off-grid everywhere (about 5 voxels per step).
"""
import numpy as np
import pytest

import oracle as O
from helpers import Parity, f32
from synthetic import WORKLOADS, bandlimited_velocity, ellipsoid_phantom, noise

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def C():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_17493_amd import claire
    return claire


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.double().cpu().numpy()


def test_setup_and_matvec_256(C):
    w = WORKLOADS["ellipsoids256"]
    n, nt, seed, alpha, p = w["n"], w["nt"], w["seed"], w["alphas"][-1], w["reg_order"]
    grid = O.Grid(n)
    clean = ellipsoid_phantom(n, seed)
    vstar = f32(bandlimited_velocity(n, seed + 1000, w["kmax"], w["vmax"]))
    m0 = f32(clean + noise(n, seed + 2000, w["noise"]))
    m1 = f32(O.transport(grid, clean, vstar, nt) + noise(n, seed + 3000, w["noise"]))
    v = f32(0.5 * vstar)
    vt = f32(bandlimited_velocity(n, seed + 4000, w["kmax"], 1.0))
    st = O.setup_velocity(grid, m0, m1, v, alpha, nt, p)
    hv_ref = O.hessian_matvec(st, vt)
    P = Parity("ellipsoids256")
    with C.Context(n, nt, alpha, p) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        ctx.set_velocity(dev(v))
        P.rel("disp+", host(ctx.get_field(C.FIELD_DISP_PLUS)), st.d_plus, TOL)
        P.rel("disp-", host(ctx.get_field(C.FIELD_DISP_MINUS)), st.d_minus, TOL)
        P.rel("m^nt", host(ctx.get_field(C.FIELD_STATE, nt)), st.m[nt], TOL)
        P.rel("grad m^nt", host(ctx.get_field(C.FIELD_GRAD_STATE, nt)), st.grad_m[nt], TOL)
        P.rel("lambda^0", host(ctx.get_field(C.FIELD_ADJOINT, 0)), st.lam[0], TOL)
        g, J = ctx.gradient()
        P.rel("g", host(g), st.g, TOL)
        P.value("J", J, st.J, TOL)
        P.rel("Hv", host(ctx.hessian_matvec(dev(vt))), hv_ref, TOL)
        P.rel("(aL)^-1 g", host(ctx.precond(g)), O.precondition(grid, host(g), alpha, p), TOL)
    P.done()
