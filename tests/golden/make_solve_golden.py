"""Write tests/golden/ellipsoids128_h2_solve.json with the FP64 oracle.

Runs the oracle's Gauss--Newton--Krylov solve (Algorithm 1, H2 seminorm,
alpha continuation 1e-1 -> 1e-4, n_t = 4, gtol 5e-2) on the 128^3
nested-ellipsoid workload and stores its trajectory, final statistics and the
solution at fixed sample voxels. Calls only oracle/ and synthetic/; takes
several minutes on the CPU.

    python tests/golden/make_solve_golden.py
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.dirname(HERE))

import oracle as O  # noqa: E402
from helpers import phantom_problem  # noqa: E402

SAMPLES = 256


def sample_indices(n, count=SAMPLES, seed=7):
    rng = np.random.default_rng(seed)
    return [tuple(int(rng.integers(0, k)) for k in n) for _ in range(count)]


def main():
    grid, m0, m1, vstar, w = phantom_problem("ellipsoids128")
    t0 = time.time()
    v, st, s = O.gn_solve(grid, m0, m1, w["nt"], w["reg_order"], list(w["alphas"]),
                          gtol=w["gtol"])
    idx = sample_indices(grid.n)
    det = O.deformation_determinant(grid, v, w["nt"])
    out = {
        "workload": "ellipsoids128", "n": list(grid.n), "nt": w["nt"],
        "reg_order": w["reg_order"], "alphas": list(w["alphas"]), "gtol": w["gtol"],
        "seconds": time.time() - t0,
        "gn_iters": s.gn_iters, "matvecs": s.matvecs, "ls_trials": s.ls_trials,
        "J0": s.J0, "J": s.J, "rel_grad": s.rel_grad, "rel_mismatch": s.rel_mismatch,
        "warnings": s.warnings, "history": s.history,
        "v_max": [float(np.abs(v[a]).max()) for a in range(3)],
        "v_l2": [float(np.sqrt(np.sum(v[a] ** 2))) for a in range(3)],
        "sample_idx": idx,
        "v_samples": [[float(v[a][i]) for a in range(3)] for i in idx],
        "det_min": float(det.min()), "det_mean": float(det.mean()), "det_max": float(det.max()),
    }
    path = os.path.join(HERE, "ellipsoids128_h2_solve.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path, "in %.0f s" % out["seconds"])


if __name__ == "__main__":
    main()
