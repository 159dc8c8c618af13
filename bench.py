#!/usr/bin/env python3
"""Benchmark: Gauss--Newton--Krylov time-to-solution + Hessian matvecs/s.

One step = one full registration solve (Algorithm 1 with PCG, Armijo line
search and the final det F check) on the 256^3 nested-ellipsoid workload:
H1 seminorm, alpha = 1e-3, n_t = 4, gradient tolerance 5e-2, from v = 0,
inputs resident in HBM. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                  [--precision mixed|fp32|both] [--warmstart WEIGHTS|none]

``value`` is the time-to-solution (seconds) of the mixed-precision solve
(float16 storage of grad m and the incremental sources in the Hessian matvec,
float32 arithmetic) started from the learned warm start: the timed region
holds the network's inference (restriction to its working resolution,
forward pass, prolongation), the extra state/adjoint solve at v = 0 that
fixes the stopping test at ||g||_inf <= gtol ||g(0)||_inf, and the solve.
The cold mixed and float32 solves (from v = 0, same tolerance) are timed too
and reported beside it, with the differences between the solutions. Without
trained weights (--warmstart none) ``value`` is the cold mixed solve. The line
also carries the Hessian matvec throughput, the HBM roofline of the dominant
kernel (average launch duration measured here with HIP events) and the FP64
CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GN-Krylov time-to-solution at 256^3 (s, gtol 5e-2) + Hessian matvecs/s"
WEIGHTS = os.path.join(ROOT, "paper_2401_17493_amd", "weights", "warmstart_r64.npz")
HBM_PEAK_GBS = 8000.0

# Algorithmic bytes per voxel of one launch of each timed kernel (float32):
#   inc-state step: gather source w^j (4), y+ displacement (12), grad m^{j+1} (12),
#                   v~ (12), output (4);
#   adjoint step:   gather source (4), y- displacement (12), A (4), output (4);
#   assembly:       lambda~^j (4 (nt+1)), grad m^j (12 (nt+1)), alpha L v~ (12), output (12);
#   copy:           3 floats in, 3 floats out.
def kernel_bytes_per_voxel(kernel, nt):
    return {"inc_state_step": 44, "adjoint_step": 24,
            "assemble": 16 * (nt + 1) + 24, "copy": 24}[kernel]


# HIP sources that define each timed kernel (its code and launch)
KERNEL_SOURCES = {"inc_state_step": ["sl.hip", "internal.h"],
                  "adjoint_step": ["sl.hip", "internal.h"],
                  "assemble": ["sl.hip", "internal.h"],
                  "copy": ["blas.hip", "internal.h"]}


def source_digest(kernel):
    """Hash of the kernel's HIP sources: counter data taken for another
    version of the kernel is stale."""
    h = hashlib.sha256()
    d = os.path.join(ROOT, "paper_2401_17493_amd", "csrc")
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(d, f), "rb") as fh:
            h.update(f.encode() + fh.read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter summary, when
    it was taken on the current sources."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_digest") != source_digest(kernel):
        return None
    return rec.get("hbm_bytes_per_launch")


def make_inputs(name, torch, C):
    import numpy as np

    from synthetic import (WORKLOADS, bandlimited_velocity, ellipsoid_phantom, noise)
    w = WORKLOADS[name]
    n, seed = w["n"], w["seed"]
    clean = ellipsoid_phantom(n, seed)
    vstar = bandlimited_velocity(n, seed + 1000, w["kmax"], w["vmax"])
    m0 = clean + noise(n, seed + 2000, w["noise"])
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()  # noqa: E731
    # the reference image: clean template transported by v* (this library's
    # transport), plus independent noise
    m1 = C.transport(dev(clean), dev(vstar), w["nt"]) + dev(noise(n, seed + 3000, w["noise"]))
    torch.cuda.synchronize()
    return w, dev(m0), m1.contiguous(), dev(vstar), (clean, vstar)


def cpu_baseline(name, host_inputs):
    """FP64 oracle on the host: one GN Hessian matvec at v = v*/2 (untimed
    setup first). Returns the cpu_baseline record."""
    import numpy as np

    import oracle as O
    from synthetic import WORKLOADS, bandlimited_velocity, noise
    w = WORKLOADS[name]
    n, seed, nt = w["n"], w["seed"], w["nt"]
    clean, vstar = host_inputs
    grid = O.Grid(n)
    m0 = clean + noise(n, seed + 2000, w["noise"])
    m1 = O.transport(grid, clean, vstar, nt) + noise(n, seed + 3000, w["noise"])
    st = O.setup_velocity(grid, m0, m1, 0.5 * vstar, w["alphas"][-1], nt, w["reg_order"])
    vt = bandlimited_velocity(n, seed + 4000, w["kmax"], 1.0)
    t0 = time.perf_counter()
    O.hessian_matvec(st, vt)
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "Hessian matvecs/s", "cores": O.WORKERS,
            "kind": "oracle", "seconds_per_matvec": dt,
            "sample": "1 FP64 GN Hessian matvec at %dx%dx%d, nt=%d, v=v*/2, after an "
                      "untimed setup (numpy/scipy.fft + C/OpenMP tricubic)" % (n + (nt,))}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ellipsoids256")
    ap.add_argument("--matvecs", type=int, default=40, help="timed Hessian matvecs")
    # the adjoint (continuity) step is the largest kernel by GPU time in the
    # mixed-precision solves (8 of the matvec's gathers are it or the
    # incremental-state step; the adjoint step also runs in every setup)
    ap.add_argument("--roofline-kernel", default="adjoint_step",
                    choices=["inc_state_step", "adjoint_step", "assemble", "copy"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", default="both", choices=["mixed", "fp32", "both"])
    ap.add_argument("--precond", default="reg", choices=["reg", "twolevel"],
                    help="PCG preconditioner: (alpha L)^-1 or the two-level zero-velocity scheme")
    ap.add_argument("--beta", type=float, default=0.0,
                    help="> 0: near-incompressible model with this divergence-penalty weight")
    ap.add_argument("--warmstart", default=WEIGHTS,
                    help="trained warm-start weights (.npz) or 'none'")
    ap.add_argument("--kernels-only", action="store_true",
                    help="set up at v = v*/2 and launch only the roofline kernel and the copy "
                         "kernel (for hardware-counter runs); prints their timings")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this engine has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2401_17493_amd import claire as C

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    w, m0, m1, vstar, host_inputs = make_inputs(args.workload, torch, C)
    n, nt = w["n"], w["nt"]
    alpha = w["alphas"][-1]
    levels = list(w["alphas"]) if len(w["alphas"]) > 1 else None
    opts = dict(gtol=w.get("gtol", 5e-2), compute_det=1,
                precond={"reg": C.PRECOND_REG, "twolevel": C.PRECOND_TWOLEVEL}[args.precond],
                beta=args.beta)
    if levels:
        opts["alpha_levels"] = levels

    ctx = C.Context(n, nt, alpha, w["reg_order"])
    ctx.set_images(m0, m1)
    if args.beta > 0:
        ctx.set_beta(args.beta)   # the matvec timing uses the same model as the solve
    kid = {"inc_state_step": C.KERNEL_INC_STATE_STEP, "adjoint_step": C.KERNEL_ADJOINT_STEP,
           "assemble": C.KERNEL_ASSEMBLE, "copy": C.KERNEL_COPY}[args.roofline_kernel]
    if args.kernels_only:
        ctx.set_velocity((0.5 * vstar).contiguous())
        ms_k = ctx.time_kernel(kid, reps=5)
        ms_c = ctx.time_kernel(C.KERNEL_COPY, reps=5)
        print(json.dumps({"kernel": args.roofline_kernel, "ms_per_launch": ms_k,
                          "copy_ms_per_launch": ms_c, "voxels": n[0] * n[1] * n[2]}))
        ctx.close()
        return
    precisions = {"mixed": [1], "fp32": [0], "both": [1, 0]}[args.precision]
    net = None
    # the warm-start network takes power-of-two grids only
    pow2 = all(k & (k - 1) == 0 for k in n)
    if args.warmstart != "none" and os.path.exists(args.warmstart) and 1 in precisions and pow2:
        from paper_2401_17493_amd.warmstart import Net
        net = Net.load(args.warmstart)
    # (label, precision, warm start)
    modes = ([("mixed+warm", 1, True)] if net is not None else []) + \
        [("mixed" if p else "fp32", p, False) for p in precisions]
    runs = {}
    for label, prec, warm in modes:
        o = dict(opts, precision=prec)
        if warm:
            o["tol_from_zero"] = 1

        def one_solve():
            v0 = net.warm_start(m0, m1) if warm else None
            return ctx.solve(v0, **o)
        for _ in range(args.warmup):
            one_solve()
        torch.cuda.synchronize()
        times, stats, v = [], None, None
        for _ in range(args.steps):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            v, stats = one_solve()
            torch.cuda.synchronize()
            times.append(time.perf_counter() - t0)
            print("step (%s): solve %.3f s, %d GN iterations, %d matvecs, %d inner" %
                  (label, times[-1], stats["gn_iters"], stats["matvecs"], stats["inner_iters"]),
                  file=sys.stderr, flush=True)
        rec = dict(tts=sum(times) / len(times), stats=stats, v=v, prec=prec)
        if not warm:
            # Hessian matvec throughput at the solution, HIP events on the context stream
            ctx.set_precision(prec)
            ctx.set_velocity(v)
            vt = (0.5 * vstar).contiguous()
            hv = torch.empty_like(vt)
            ctx.hessian_matvec(vt, hv)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(ctx.stream)
            for _ in range(args.matvecs):
                ctx.hessian_matvec(vt, hv)
            e1.record(ctx.stream)
            e1.synchronize()
            rec["ms_matvec"] = e0.elapsed_time(e1) / args.matvecs
        runs[label] = rec
    if net is not None:
        net.close()
        runs["mixed+warm"]["ms_matvec"] = runs["mixed"]["ms_matvec"]
    head = runs[modes[0][0]]
    tts, stats, ms_matvec = head["tts"], head["stats"], head["ms_matvec"]
    # roofline of the dominant kernel at v = v*/2, the state the counter runs
    # (--kernels-only) use: algorithmic bytes / live launch duration
    ctx.set_precision(0)
    ctx.set_velocity((0.5 * vstar).contiguous())

    ms_kernel = ctx.time_kernel(kid, reps=50)
    voxels = n[0] * n[1] * n[2]
    alg_bytes = kernel_bytes_per_voxel(args.roofline_kernel, nt) * voxels
    achieved = alg_bytes / (ms_kernel * 1e-3) / 1e9
    ms_copy = ctx.time_kernel(C.KERNEL_COPY, reps=50)
    copy_gbs = 24 * voxels / (ms_copy * 1e-3) / 1e9
    print("kernel %s: %.4f ms/launch, %.0f GB/s algorithmic; copy kernel %.0f GB/s; "
          "matvec %.3f ms" % (args.roofline_kernel, ms_kernel, achieved, copy_gbs, ms_matvec),
          file=sys.stderr, flush=True)
    ctx.close()

    def solve_rec(r):
        st = r["stats"]
        rec = {k: st[k] for k in ("gn_iters", "matvecs", "inner_iters", "pde_solves",
                                  "linesearch_trials",
                                  "rel_grad", "rel_mismatch", "J0", "J", "det_min", "det_max",
                                  "det_nonpositive")}
        rec.update(time_to_solution_s=round(r["tts"], 4),
                   hessian_matvecs_per_s=round(1000.0 / r["ms_matvec"], 2),
                   ms_per_matvec=round(r["ms_matvec"], 4))
        return rec

    out = {
        "metric": METRIC,
        "value": round(tts, 4),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(tts * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded nested-ellipsoid phantom, band-limited v*)",
        "config": {"workload": args.workload, "grid": list(n), "nt": nt,
                   "alpha": alpha if not levels else levels,
                   "regularization": "H%d seminorm" % w["reg_order"] + (
                       "" if args.beta <= 0 else
                       ", near-incompressible (divergence penalty beta = %g)" % args.beta),
                   "gtol": opts["gtol"],
                   "preconditioner": "(alpha L)^-1" if args.precond == "reg" else
                   "two-level zero-velocity H0 (coarse grid n/2, inner CG to 0.1 eta)",
                   "precision": "mixed: float16 grad m and incremental sources in the "
                                "Hessian matvec, float32 arithmetic/FFTs, float64 reductions"
                   if head["prec"] == 1 else "float32 fields and FFTs, float64 reductions",
                   "initial_guess": "learned warm start (%s), stopping test against "
                                    "||g(v=0)||_inf" % os.path.basename(args.warmstart)
                   if modes[0][2] else "v = 0",
                   "parallelism": "single GPU"},
        "hessian_matvecs_per_s": round(1000.0 / ms_matvec, 2),
        "ms_per_matvec": round(ms_matvec, 4),
        "solve": solve_rec(head),
        "roofline": {"kernel": args.roofline_kernel, "bound": "hbm",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic(args.roofline_kernel, args.workload),
                     "ms_per_launch": round(ms_kernel, 5),
                     "algorithmic_bytes_per_launch": alg_bytes,
                     "copy_kernel_GBs": round(copy_gbs, 1)},
    }
    def compare(a, b):
        va, vb = a["v"], b["v"]
        return {"speedup": round(b["tts"] / a["tts"], 3),
                "v_rel_maxnorm": float((va - vb).abs().max() / vb.abs().max()),
                "J_rel": abs(a["stats"]["J"] - b["stats"]["J"]) / b["stats"]["J"],
                "rel_grad": [a["stats"]["rel_grad"], b["stats"]["rel_grad"]]}
    if "mixed+warm" in runs:
        out["mixed_solve"] = solve_rec(runs["mixed"])
        if "fp32" in runs:
            out["warm_vs_fp32"] = compare(runs["mixed+warm"], runs["fp32"])
        out["warm_vs_mixed"] = compare(runs["mixed+warm"], runs["mixed"])
    if "fp32" in runs:
        out["fp32_solve"] = solve_rec(runs["fp32"])
        if "mixed" in runs:
            out["mixed_vs_fp32"] = compare(runs["mixed"], runs["fp32"])
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, host_inputs)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
