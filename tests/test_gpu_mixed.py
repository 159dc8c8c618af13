"""Mixed-precision Hessian matvec (float16 storage of grad m^j and of the
incremental-state sources -grad m^j . v~; float32 arithmetic, fields and
FFTs otherwise) against the FP64 oracle.

The bar for the mixed path is a max-norm relative error of 1e-3. float16 has
a unit round-off of 2^-11 = 4.9e-4; each stored operand is rounded once and
enters the result linearly (the per-step fields that are re-rounded at every
step stay float32), so the expected error is a few 1e-4.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from helpers import Parity, blob_problem, f32, phantom_problem
from synthetic import WORKLOADS, bandlimited_velocity, ellipsoid_phantom, noise

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-3


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


@pytest.mark.parametrize("p", [1, 2])
@pytest.mark.parametrize("nt", [1, 4])
def test_mixed_matvec_blobs32(C, p, nt):
    grid, m0, m1, vstar = blob_problem(nt=nt)
    v = f32(0.5 * vstar)
    vt = f32(bandlimited_velocity(grid.n, 77, 4, 0.5))
    st = O.setup_velocity(grid, m0, m1, v, 1e-2, nt, p)
    ref = O.hessian_matvec(st, vt)
    P = Parity("mixed blobs32 p%d nt%d" % (p, nt))
    with C.Context(grid.n, nt, 1e-2, p) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        ctx.set_precision(1)
        ctx.set_velocity(dev(v))
        g, J = ctx.gradient()
        P.rel("g (float32 path)", host(g), st.g, 1e-5)
        hv = ctx.hessian_matvec(dev(vt))
        P.rel("Hv", host(hv), ref, TOL)
        # linear in v~ with no float16 overflow: scale the input by 1e4
        hv_big = ctx.hessian_matvec(dev(1e4 * vt))
        P.rel("H(1e4 v~)/1e4", host(hv_big) / 1e4, ref, TOL)
        # switching back to float32 requires a new setup
        ctx.set_precision(0)
        with pytest.raises(C.ClaireError):
            ctx.hessian_matvec(dev(vt))
        ctx.set_velocity(dev(v))
        P.rel("Hv float32", host(ctx.hessian_matvec(dev(vt))), ref, 1e-5)
    P.done()


def test_mixed_matvec_256(C):
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
    ref = O.hessian_matvec(st, vt)
    P = Parity("mixed ellipsoids256")
    with C.Context(n, nt, alpha, p) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        ctx.set_precision(1)
        ctx.set_velocity(dev(v))
        P.rel("Hv", host(ctx.hessian_matvec(dev(vt))), ref, TOL)
    P.done()


def test_mixed_continuation_solve_128(C):
    ref = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                      "ellipsoids128_h2_solve.json")))
    grid, m0, m1, vstar, w = phantom_problem("ellipsoids128")
    with C.Context(grid.n, w["nt"], w["alphas"][-1], w["reg_order"]) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        v, st = ctx.solve(alpha_levels=list(w["alphas"]), gtol=w["gtol"], precision=1,
                          compute_det=1)
        vh = host(v)
    samples = np.array([[vh[a][tuple(i)] for a in range(3)] for i in ref["sample_idx"]])
    v_err = np.abs(samples - np.array(ref["v_samples"])).max() / max(ref["v_max"])
    J_err = abs(st["J"] - ref["J"]) / ref["J"]
    print("MIXED solve: gn %d (oracle %d), matvecs %d (%d), J rel err %.2e, v rel err %.2e, "
          "rel_grad %.4f" % (st["gn_iters"], ref["gn_iters"], st["matvecs"], ref["matvecs"],
                             J_err, v_err, st["rel_grad"]))
    assert st["status"] == 0 and st["rel_grad"] <= w["gtol"]
    assert J_err <= TOL and v_err <= TOL
    assert abs(st["gn_iters"] - ref["gn_iters"]) <= 2
    assert abs(st["matvecs"] - ref["matvecs"]) <= 0.1 * ref["matvecs"]
    assert st["det_nonpositive"] == 0


def test_time_kernel_mixed_step(C):
    """The mixed incremental-state step can be timed only with the float16
    copy in place (set_precision(1) before set_velocity)."""
    grid, m0, m1, vstar = blob_problem()
    with C.Context(grid.n, 4, 1e-2, 1) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        ctx.set_velocity(dev(f32(0.5 * vstar)))
        with pytest.raises(C.ClaireError) as e:
            ctx.time_kernel(C.KERNEL_INC_STATE_STEP_MIXED, reps=2)
        assert e.value.code == -1
        ctx.set_precision(1)
        ctx.set_velocity(dev(f32(0.5 * vstar)))
        for k in (C.KERNEL_INC_STATE_STEP_MIXED, C.KERNEL_INC_STATE_STEP,
                  C.KERNEL_ADJOINT_STEP, C.KERNEL_COPY):
            assert ctx.time_kernel(k, reps=2) > 0.0
