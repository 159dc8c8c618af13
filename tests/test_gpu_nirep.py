"""The paper's grid, 256 x 300 x 256 (Section 3.1; nested-ellipsoid phantom
standing in for the NIREP images, H1, alpha = 1e-3, n_t = 4), against the
FP64 oracle's run of the same solve (tests/golden/ellipsoids_nirep_h1_solve.json,
written by tests/golden/make_solve_golden.py).

The first three Gauss--Newton steps are compared at the 1e-5 bar: per
iterate J and ||g||_inf, the PCG matvec counts and residual histories, and
the iterate after each step at the record's sample voxels. This exercises
the general-grid path (ragged bricks, mixed-radix 2*3*5^2 column
transforms) at full size against the oracle. The rest of the solve is
compared by its counts and final state, which the oracle decides.

From v = 0 at this alpha (no continuation) the oracle's own solve does not
converge: after a step taken on negative curvature the map folds (det F <= 0
at some voxels), the gradient grows by four orders and the line search
fails. The GPU solve must follow it there: the same outcome, GN and matvec
counts within the bars of the other full solves.
"""
import hashlib
import json
import os

import numpy as np
import pytest

from helpers import Parity, phantom_problem, trace_parity

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "ellipsoids_nirep_h1_solve.json")


@pytest.fixture(scope="module")
def C():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_17493_amd import claire
    return claire


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def samples(v, idx):
    torch.cuda.synchronize()
    t = torch.as_tensor(np.array(idx), device=v.device)
    return v[:, t[:, 0], t[:, 1], t[:, 2]].double().cpu().numpy().T


def test_nirep_grid_first_steps(C):
    if not os.path.exists(GOLDEN):
        pytest.skip("no oracle record of the 256x300x256 solve")
    ref = json.load(open(GOLDEN))
    grid, m0, m1, vstar, w = phantom_problem("ellipsoids_nirep")
    sha = hashlib.sha256(np.ascontiguousarray(m1, dtype=np.float32).tobytes()).hexdigest()
    assert sha == ref["m1_sha256"]
    idx = ref["sample_idx"]
    P = Parity("256x300x256")
    with C.Context(grid.n, w["nt"], w["alphas"][-1], w["reg_order"]) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        ctx.set_velocity(torch.zeros((3,) + grid.n, device="cuda"))
        g0, _ = ctx.gradient()
        P.rel("g(0) samples", samples(g0, idx), np.array(ref["g0_samples"]), 1e-5)
        for k, snap in sorted(ref["snapshots"].items()):
            vk, sk = ctx.solve(gtol=w["gtol"], max_gn=int(k))
            trace = ctx.solve_trace()
            P.rel("v after %s GN steps" % k, samples(vk, idx), np.array(snap["v_samples"]), 1e-5)
            P.value("J after %s GN steps" % k, sk["J"], snap["J"], 1e-5)
        v, st = ctx.solve(gtol=w["gtol"], compute_det=1)
        full = ctx.solve_trace()
    # the stopped solve's last record took no step: compare the records before it
    trace_parity(P, "first steps", trace, ref["history"], 1e-5, steps=len(trace) - 1)
    print("GPU:", {k: st[k] for k in ("status", "gn_iters", "matvecs", "linesearch_trials", "J",
                                      "rel_grad", "det_min", "det_nonpositive")}, flush=True)
    print("ORACLE:", {k: ref[k] for k in ("gn_iters", "matvecs", "ls_trials", "J", "rel_grad",
                                          "det_min", "det_nonpositive", "warnings")}, flush=True)
    print("PCG matvecs per step: GPU %s, oracle %s"
          % ([t["pcg_its"] for t in full], [h.get("pcg_its") for h in ref["history"]]), flush=True)
    P.done()
    # the oracle's verdict on this problem: a non-diffeomorphic map and no convergence
    assert ref["det_nonpositive"] > 0 and ref["rel_grad"] > ref["gtol"]
    assert st["status"] != 0 and st["det_nonpositive"] > 0 and st["rel_grad"] > w["gtol"]
    assert abs(st["gn_iters"] - ref["gn_iters"]) <= 2
    assert abs(st["matvecs"] - ref["matvecs"]) <= 0.1 * ref["matvecs"]


NI_GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                         "ellipsoids_nirep_ni_solve.json")


def test_nirep_grid_ni_first_steps(C):
    """The near-incompressible model (beta = 1e-4, the paper's model for its
    NIREP runs) on the same grid: the oracle's first three Gauss--Newton
    steps (its record stops there) at the 1e-5 bar."""
    if not os.path.exists(NI_GOLDEN):
        pytest.skip("no oracle record of the near-incompressible 256x300x256 solve")
    ref = json.load(open(NI_GOLDEN))
    grid, m0, m1, vstar, w = phantom_problem("ellipsoids_nirep")
    sha = hashlib.sha256(np.ascontiguousarray(m1, dtype=np.float32).tobytes()).hexdigest()
    assert sha == ref["m1_sha256"] and ref["beta"] > 0
    idx = ref["sample_idx"]
    P = Parity("256x300x256 beta %g" % ref["beta"])
    with C.Context(grid.n, w["nt"], w["alphas"][-1], w["reg_order"]) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        ctx.set_beta(ref["beta"])
        ctx.set_velocity(torch.zeros((3,) + grid.n, device="cuda"))
        g0, _ = ctx.gradient()
        P.rel("g(0) samples", samples(g0, idx), np.array(ref["g0_samples"]), 1e-5)
        for k, snap in sorted(ref["snapshots"].items()):
            vk, sk = ctx.solve(gtol=w["gtol"], max_gn=int(k), beta=ref["beta"])
            trace = ctx.solve_trace()
            P.rel("v after %s GN steps" % k, samples(vk, idx), np.array(snap["v_samples"]), 1e-5)
            P.value("J after %s GN steps" % k, sk["J"], snap["J"], 1e-5)
    steps = min(3, ref["max_gn"])
    trace_parity(P, "first steps", trace, ref["history"], 1e-5, steps=steps)
    P.done()
