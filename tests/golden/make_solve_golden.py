"""Write golden records of whole Gauss--Newton--Krylov solves with the FP64 oracle.

Runs the oracle's solve (Algorithm 1 with PCG, Algorithm 2, and the Armijo
line search; parameter continuation where the workload lists several alpha
levels) on a seeded workload and stores its trajectory (per iterate: J,
||g||_inf, PCG matvecs and residual history, step length, line-search
trials), its final statistics, the solution at fixed sample voxels, snapshots
of the iterate after the first few Gauss--Newton steps and det F(1). Calls
only oracle/ and synthetic/ (through tests/helpers.py).

    python tests/golden/make_solve_golden.py                       # 128^3 H2 continuation
    python tests/golden/make_solve_golden.py ellipsoids256         # 256^3 H1, alpha 1e-3
    python tests/golden/make_solve_golden.py ellipsoids_nirep      # 256x300x256 H1
    python tests/golden/make_solve_golden.py ellipsoids_nirep --beta 1e-4

The 128^3 run takes minutes; the 256^3 and 256x300x256 runs take hours on
eight cores (3.9 h and 2.0 h for the committed records, with two runs
sharing the cores).
"""
import argparse
import hashlib
import json
import os
import platform
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
SNAPSHOTS = (1, 2, 3)


def sample_indices(n, count=SAMPLES, seed=7):
    rng = np.random.default_rng(seed)
    return [tuple(int(rng.integers(0, k)) for k in n) for _ in range(count)]


def digest(a):
    """SHA-256 of the float32 bytes of an input (identifies the problem)."""
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float32).tobytes()).hexdigest()


def host_info():
    model = platform.processor()
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "threads": O.WORKERS}


def golden_name(workload, beta):
    if workload == "ellipsoids128":
        return "ellipsoids128_h2_solve.json"
    return "%s_%s_solve.json" % (workload, "ni" if beta > 0 else "h%d" % 1)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload", nargs="?", default="ellipsoids128")
    ap.add_argument("--beta", type=float, default=0.0,
                    help="near-incompressible weight (0: plain model)")
    ap.add_argument("--max-gn", type=int, default=50)
    args = ap.parse_args()

    grid, m0, m1, vstar, w = phantom_problem(args.workload)
    idx = sample_indices(grid.n)
    snaps = {}

    def record(level, k, v, st):
        if level == 0 and k in SNAPSHOTS:
            snaps[str(k)] = {
                "J": st.J, "gnorm": float(np.abs(st.g).max()),
                "v_samples": [[float(v[a][i]) for a in range(3)] for i in idx],
                "v_max": [float(np.abs(v[a]).max()) for a in range(3)],
            }
        print("level %d step %d: J %.9e  ||g||_inf %.6e  (%.0f s)"
              % (level, k, st.J, float(np.abs(st.g).max()), time.time() - t0), flush=True)

    t0 = time.time()
    st0 = O.setup_velocity(grid, m0, m1, np.zeros((3,) + grid.n), w["alphas"][0], w["nt"],
                           w["reg_order"], beta=args.beta)
    g0_samples = [[float(st0.g[a][i]) for a in range(3)] for i in idx]
    g0_max = float(np.abs(st0.g).max())
    del st0
    t0 = time.time()
    v, st, s = O.gn_solve(grid, m0, m1, w["nt"], w["reg_order"], list(w["alphas"]),
                          gtol=w["gtol"], beta=args.beta, max_gn=args.max_gn,
                          callback=record)
    seconds = time.time() - t0
    det = O.deformation_determinant(grid, v, w["nt"])
    out = {
        "workload": args.workload, "n": list(grid.n), "nt": w["nt"],
        "reg_order": w["reg_order"], "alphas": list(w["alphas"]), "gtol": w["gtol"],
        "beta": args.beta, "max_gn": args.max_gn,
        "m0_sha256": digest(m0), "m1_sha256": digest(m1),
        "seconds": seconds, "host": host_info(),
        "gn_iters": s.gn_iters, "matvecs": s.matvecs, "ls_trials": s.ls_trials,
        "pde_solves": s.pde_solves,
        "J0": s.J0, "J": s.J, "rel_grad": s.rel_grad, "rel_mismatch": s.rel_mismatch,
        "warnings": s.warnings, "history": s.history,
        "g0_max": g0_max,
        "g0_samples": g0_samples,
        "v_max": [float(np.abs(v[a]).max()) for a in range(3)],
        "v_l2": [float(np.sqrt(np.sum(v[a] ** 2))) for a in range(3)],
        "sample_idx": idx,
        "v_samples": [[float(v[a][i]) for a in range(3)] for i in idx],
        "snapshots": snaps,
        "det_min": float(det.min()), "det_mean": float(det.mean()),
        "det_max": float(det.max()), "det_nonpositive": int(np.sum(det <= 0)),
    }
    path = os.path.join(HERE, golden_name(args.workload, args.beta))
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print("wrote", path, "in %.0f s" % seconds)


if __name__ == "__main__":
    main()
