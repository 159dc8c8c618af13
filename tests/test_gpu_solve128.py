"""Full Gauss--Newton--Krylov solve with parameter continuation on the 128^3
nested-ellipsoid workload (H2 seminorm, alpha 1e-1 -> 1e-4, n_t = 4,
gtol 5e-2) against the FP64 oracle's run stored in
tests/golden/ellipsoids128_h2_solve.json (written by
tests/golden/make_solve_golden.py, which calls only the oracle).

The float32 GPU solve follows the oracle's path: same Gauss--Newton
iterations, PCG matvecs and line-search trials per level, and the objective,
the solution (at 256 stored voxels and in norm) and det F within the 1e-5
relative bar. (A residual within round-off of the PCG forcing tolerance could
in principle end PCG one iteration apart; the GPU path is deterministic, so
the comparison is stable from run to run.)
"""
import json
import os

import numpy as np
import pytest

from helpers import phantom_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "ellipsoids128_h2_solve.json")


@pytest.fixture(scope="module")
def C():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2401_17493_amd import claire
    return claire


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def test_continuation_solve_128_h2(C):
    ref = json.load(open(GOLDEN))
    grid, m0, m1, vstar, w = phantom_problem("ellipsoids128")
    with C.Context(grid.n, w["nt"], w["alphas"][-1], w["reg_order"]) as ctx:
        ctx.set_images(dev(m0), dev(m1))
        v, st = ctx.solve(alpha_levels=list(w["alphas"]), gtol=w["gtol"], compute_det=1)
        torch.cuda.synchronize()
        vh = v.double().cpu().numpy()
    print("GPU:", {k: st[k] for k in ("gn_iters", "matvecs", "linesearch_trials", "J0", "J",
                                      "rel_grad", "rel_mismatch", "det_min", "det_mean",
                                      "det_max")})
    print("ORACLE:", {k: ref[k] for k in ("gn_iters", "matvecs", "ls_trials", "J0", "J",
                                          "rel_grad", "rel_mismatch", "det_min", "det_mean",
                                          "det_max")})
    samples = np.array([[vh[a][tuple(i)] for a in range(3)] for i in ref["sample_idx"]])
    ref_s = np.array(ref["v_samples"])
    vmax = max(ref["v_max"])
    sample_err = np.abs(samples - ref_s).max() / vmax
    l2_err = max(abs(np.sqrt(np.sum(vh[a] ** 2)) - ref["v_l2"][a]) / ref["v_l2"][a]
                 for a in range(3))
    print("v sample err / max|v| %.3e, |v|_2 rel err %.3e" % (sample_err, l2_err))
    tol = 1e-5
    assert st["status"] == 0 and st["rel_grad"] <= w["gtol"]
    assert st["gn_iters"] == ref["gn_iters"] and st["matvecs"] == ref["matvecs"]
    assert st["linesearch_trials"] == ref["ls_trials"]
    assert abs(st["J0"] - ref["J0"]) <= tol * ref["J0"]
    assert abs(st["J"] - ref["J"]) <= tol * ref["J"]
    assert abs(st["rel_mismatch"] - ref["rel_mismatch"]) <= tol * ref["rel_mismatch"]
    # ||g||_inf / ||g_0||_inf: g carries a float32 error of order 1e-5 ||g_0||_inf
    assert abs(st["rel_grad"] - ref["rel_grad"]) <= 5e-5
    assert sample_err <= tol and l2_err <= tol
    assert st["det_nonpositive"] == 0
    for k in ("det_min", "det_mean", "det_max"):
        assert abs(st[k] - ref[k]) <= tol * ref[k]
