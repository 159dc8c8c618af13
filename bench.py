#!/usr/bin/env python3
"""Benchmark: Gauss--Newton--Krylov time-to-solution + Hessian matvecs/s.

One step = one full registration solve (Algorithm 1 with PCG, Armijo line
search and the final det F check) on the 256^3 nested-ellipsoid workload:
H1 seminorm, alpha = 1e-3, n_t = 4, gradient tolerance 5e-2, from v = 0,
inputs resident in HBM. Prints one JSON line.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
                  [--precision mixed|fp32|both] [--warmstart WEIGHTS|none]

``value`` is the time-to-solution (seconds) of the mixed-precision solve
(the Hessian matvec reads grad m^j from a float16 copy; float32 arithmetic
and fields) started from the learned warm start: the timed region
holds the network's inference (restriction to its working resolution,
forward pass, prolongation), the extra state/adjoint solve at v = 0 that
fixes the stopping test at ||g||_inf <= gtol ||g(0)||_inf, and the solve.
The cold mixed and float32 solves (from v = 0, same tolerance) are timed too
and reported beside it, with the differences between the solutions. Without
trained weights (--warmstart none) ``value`` is the cold mixed solve.

The inputs are the FP64 oracle's problem: m1 is the oracle's transport of the
clean phantom (written by tests/golden/make_inputs.py). Each solve is reported
with its status and, when the oracle's record of the same solve exists
(tests/golden/make_solve_golden.py), its relative errors against it in v, J
and the final gradient norm. A solve that ends with a warning or above the
gradient tolerance gets no time-to-solution (and the run exits with status
3). The line also carries the Hessian matvec throughput and its fraction of
the HBM roofline, the roofline of the dominant kernel (average launch
duration measured here with HIP events) and the FP64 CPU oracle timed on a
bounded sample of the same workload.
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
#   backtrace:      v (12), y+ and y- displacements (24).
def kernel_bytes_per_voxel(kernel, nt):
    # inc-state step: w^j 4 + displacement 12 + grad m^{j+1} 12 (float16: 6)
    # + v~ 12 + out 4; adjoint step: lambda~ 4 + displacement 12 + A 4 + out 4
    return {"inc_state_step": 44, "inc_state_step_mixed": 38, "adjoint_step": 24,
            "assemble": 16 * (nt + 1) + 24, "copy": 24, "backtrace": 36}[kernel]


def kernel_table(ctx, C, nt, voxels, reps=20):
    """Average launch time (HIP events on the context stream) and algorithmic
    HBM rate of each hot-path kernel at the context's current velocity."""
    ids = {"inc_state_step": C.KERNEL_INC_STATE_STEP,
           "inc_state_step_mixed": C.KERNEL_INC_STATE_STEP_MIXED,
           "adjoint_step": C.KERNEL_ADJOINT_STEP,
           "assemble": C.KERNEL_ASSEMBLE, "backtrace": C.KERNEL_BACKTRACE,
           "copy": C.KERNEL_COPY}
    out = {}
    for name, k in ids.items():
        ms = ctx.time_kernel(k, reps=reps)
        gbs = kernel_bytes_per_voxel(name, nt) * voxels / (ms * 1e-3) / 1e9
        out[name] = {"ms": round(ms, 4), "bytes_per_voxel": kernel_bytes_per_voxel(name, nt),
                     "GBs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4)}
    return out


# HIP sources that define each timed kernel (its code and launch)
KERNEL_SOURCES = {"inc_state_step": ["sl.hip", "internal.h"],
                  "inc_state_step_mixed": ["sl.hip", "internal.h"],
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


GOLDEN_DIR = os.path.join(ROOT, "tests", "golden")


def load_inputs(name):
    """m0 and m1 (float32 host arrays) of a workload, as the FP64 oracle builds
    them (m1 = oracle transport of the clean phantom by v*, plus noise), from
    the file tests/golden/make_inputs.py writes; the script runs first when
    the file is missing. Also returns v* (seeded generator, rounded to
    float32) and the SHA-256 of m1."""
    import subprocess

    import numpy as np

    from synthetic import WORKLOADS, bandlimited_velocity
    w = WORKLOADS[name]
    n = tuple(w["n"])
    path = os.path.join(GOLDEN_DIR, "inputs", "%s.npz" % name)
    if not os.path.exists(path):
        t0 = time.time()
        subprocess.run([sys.executable, os.path.join(GOLDEN_DIR, "make_inputs.py"), name,
                        "--out", path], check=True)
        print("inputs of %s generated in %.1f s" % (name, time.time() - t0),
              file=sys.stderr, flush=True)
    with np.load(path) as z:
        m0, m1, sha = z["m0"], z["m1"], str(z["m1_sha256"])
    vstar = bandlimited_velocity(n, w["seed"] + 1000, min(w["kmax"], n[0] // 2 - 1), w["vmax"])
    return w, m0, m1, vstar.astype(np.float32), sha


def load_golden(name, w, beta):
    """The FP64 oracle's record of the same solve (tests/golden/make_solve_golden.py)."""
    tag = "ni" if beta > 0 else "h%d" % w["reg_order"]
    path = os.path.join(GOLDEN_DIR, "%s_%s_solve.json" % (name, tag))
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        g = json.load(fh)
    # a record of the first Gauss--Newton steps only is no whole-solve reference
    return g if g.get("max_gn", 50) >= 50 else None


def vs_oracle(v, stats, trace, golden, m1_sha):
    """Relative errors of a GPU solve against the FP64 oracle's solve of the
    same problem: v at the golden's sample voxels (max-norm), the final
    objective and the final gradient norm (the Newton residual), and the
    iteration counts of both."""
    import numpy as np
    if golden is None:
        return None
    if golden.get("m1_sha256") != m1_sha:
        return {"error": "inputs differ from the oracle record's (m1 digest)"}
    idx = np.array(golden["sample_idx"])
    got = v[:, idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy().T
    ref = np.array(golden["v_samples"])
    g_gpu = trace[-1]["gnorm"] if trace else float("nan")
    g_ora = golden["history"][-1]["gnorm"]
    return {"v_rel_maxnorm_samples": float(np.abs(got - ref).max() / np.abs(ref).max()),
            "J_rel": abs(stats["J"] - golden["J"]) / abs(golden["J"]),
            "residual_rel": abs(g_gpu - g_ora) / g_ora,
            "rel_grad": [stats["rel_grad"], golden["rel_grad"]],
            "gn_iters": [stats["gn_iters"], golden["gn_iters"]],
            "matvecs": [stats["matvecs"], golden["matvecs"]],
            "samples": len(ref),
            "oracle_seconds": round(golden["seconds"], 1),
            "oracle_host": golden.get("host")}


def host_info():
    import oracle as O
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu_model": model, "threads": O.WORKERS}


def median_time(fn, runs=3):
    """Median wall time of `runs` calls after one untimed warm-up call."""
    fn()
    ts = []
    for _ in range(runs):
        t0 = time.perf_counter()
        fn()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)[len(ts) // 2]


def cpu_baseline(name, m0, m1, vstar):
    """The FP64 oracle on this host: median of 3 timed runs after a warm-up of
    one GN Hessian matvec at v = v*/2 (setup untimed), of its kernels (one
    spectral gradient = 1 R2C + 3 C2R FFTs, one tricubic gather of a field,
    the RK2 backtrace of one direction) and of the 32^3 one-step solve (10 PCG
    matvecs); the oracle's time-to-solution of the 128^3 and 256^3 solves
    quoted from its golden records (taken on the host named there)."""
    import numpy as np

    import oracle as O
    from synthetic import WORKLOADS, bandlimited_velocity, gaussian_blobs
    w = WORKLOADS[name]
    n, seed, nt = tuple(w["n"]), w["seed"], w["nt"]
    grid = O.Grid(n)
    m0 = m0.astype(np.float64)
    m1 = m1.astype(np.float64)
    v = 0.5 * vstar.astype(np.float64)
    st = O.setup_velocity(grid, m0, m1, v, w["alphas"][-1], nt, w["reg_order"])
    vt = bandlimited_velocity(n, seed + 4000, min(w["kmax"], n[0] // 2 - 1), 1.0)
    t_mv = median_time(lambda: O.hessian_matvec(st, vt))
    kernels = {
        "spectral_gradient_s": median_time(lambda: O.gradient(grid, st.m[-1])),
        "tricubic_gather_s": median_time(lambda: O.interpolate(st.m[-1], st.d_plus)),
        "backtrace_s": median_time(lambda: O.departure_displacement(grid, v, nt, +1)),
    }
    del st
    # config 1: 32^3 blobs, one GN step with exactly 10 PCG matvecs from v = 0
    b = WORKLOADS["blobs32"]
    g32 = O.Grid(b["n"])
    b0 = gaussian_blobs(b["n"], b["seed"]).astype(np.float32).astype(np.float64)
    bv = bandlimited_velocity(b["n"], b["seed"] + 1000, b["kmax"], b["vmax"])
    b1 = O.transport(g32, b0, bv.astype(np.float32).astype(np.float64), b["nt"])
    t_c1 = median_time(lambda: O.gn_solve(g32, b0, b1, b["nt"], b["reg_order"],
                                          list(b["alphas"]), max_gn=1, fixed_pcg=10))
    tts = {"blobs32_one_gn_step_10_matvecs_s": round(t_c1, 3)}
    for wl, tag in (("ellipsoids128", "h2"), ("ellipsoids256", "h1")):
        path = os.path.join(GOLDEN_DIR, "%s_%s_solve.json" % (wl, tag))
        if os.path.exists(path):
            with open(path) as fh:
                gd = json.load(fh)
            tts["%s_solve_s" % wl] = {"seconds": round(gd["seconds"], 1),
                                      "gn_iters": gd["gn_iters"], "matvecs": gd["matvecs"],
                                      "host": gd.get("host"), "source": "golden record"}
    return {"value": 1.0 / t_mv, "unit": "Hessian matvecs/s", "cores": O.WORKERS,
            "kind": "oracle", "seconds_per_matvec": t_mv,
            "host": host_info(),
            "kernels_s": {k: round(v_, 4) for k, v_ in kernels.items()},
            "time_to_solution": tts,
            "sample": "median of 3 FP64 GN Hessian matvecs at %dx%dx%d, nt=%d, v=v*/2, after "
                      "a warm-up and an untimed setup (numpy/scipy.fft + C/OpenMP tricubic); "
                      "kernels and the 32^3 step the same way" % (n + (nt,))}


def net_train_timing(steps, R=64, B=4):
    """Milliseconds per training step of the warm-start network (forward,
    loss, backward, Adam; the library's MFMA kernels) on random inputs, and
    the step's convolution flops: 2 x 27 cin cout per output voxel for the
    forward pass, as much again for the data and the weight gradients (not
    the first layer's data gradient)."""
    import torch

    from paper_2401_17493_amd.warmstart import Net
    ch = (16, 32, 64, 128)
    net = Net(R, ch, max_batch=B, seed=1)
    g = torch.Generator(device="cuda").manual_seed(0)
    x0 = torch.rand((B, R, R, R), device="cuda", generator=g)
    x1 = torch.rand((B, R, R, R), device="cuda", generator=g)
    tg = 0.1 * torch.randn((B, 3, R, R, R), device="cuda", generator=g)
    net.train_step(x0, x1, tg, 1e-3)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        net.train_step(x0, x1, tg, 1e-3)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / steps * 1e3
    net.close()
    c1, c2, c3, c4 = ch
    layers = [(8, c1, 0), (c1, c1, 0), (c1, c2, 1), (c2, c2, 1), (c2, c3, 2), (c3, c3, 2),
              (c3, c4, 3), (c4, c4, 3), (c4 + c3, c3, 2), (c3, c3, 2), (c3 + c2, c2, 1),
              (c2, c2, 1), (c2 + c1, c1, 0), (c1, c1, 0), (c1, 3, 0)]
    fwd = [2.0 * 27 * ci * co * B * (R >> lv) ** 3 for ci, co, lv in layers]
    flops = 3 * sum(fwd) - fwd[0]
    tflops = flops / (ms * 1e-3) / 1e12
    return {"net_train_ms_per_step": round(ms, 3), "gflop_per_step": round(flops / 1e9, 1),
            "tflops": round(tflops, 1), "bf16_peak_tflops": 2500.0,
            "mfma_frac": round(tflops / 2500.0, 4),
            "config": {"resolution": R, "batch": B, "channels": list(ch)}}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="ellipsoids256")
    ap.add_argument("--matvecs", type=int, default=40, help="timed Hessian matvecs")
    # the mixed incremental-state step is the largest kernel by GPU time in the
    # mixed-precision solves (n_t per matvec, 167 us at 256^3), ahead of the
    # adjoint step (n_t per matvec and per setup, 130-150 us)
    ap.add_argument("--roofline-kernel", default="inc_state_step_mixed",
                    choices=["inc_state_step", "inc_state_step_mixed", "adjoint_step",
                             "assemble", "copy"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", default="both", choices=["mixed", "fp32", "both"])
    ap.add_argument("--precond", default="reg", choices=["reg", "twolevel"],
                    help="PCG preconditioner: (alpha L)^-1 or the two-level zero-velocity scheme")
    ap.add_argument("--beta", type=float, default=0.0,
                    help="> 0: near-incompressible model with this divergence-penalty weight")
    ap.add_argument("--warmstart", default=WEIGHTS,
                    help="trained warm-start weights (.npz) or 'none'")
    ap.add_argument("--no-solve", action="store_true",
                    help="matvec throughput and the kernel table only, at v = v*/2 (for "
                         "workloads whose solve has no time-to-solution, e.g. 512^3)")
    ap.add_argument("--kernels-only", action="store_true",
                    help="set up at v = v*/2 and launch only the roofline kernel and the copy "
                         "kernel (for hardware-counter runs); prints their timings")
    ap.add_argument("--net-train-steps", type=int, default=0,
                    help="> 0: only time this many warm-start network training steps (64^3, "
                         "batch 4, channels 16-128, random inputs) after one warm-up step")
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
    if args.net_train_steps > 0:
        print(json.dumps(net_train_timing(args.net_train_steps)), flush=True)
        return
    w, m0_h, m1_h, vstar_h, m1_sha = load_inputs(args.workload)
    golden = load_golden(args.workload, w, args.beta) if args.precond == "reg" else None
    dev = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    m0, m1, vstar = dev(m0_h), dev(m1_h), dev(vstar_h)
    torch.cuda.synchronize()
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
    kid = {"inc_state_step": C.KERNEL_INC_STATE_STEP,
           "inc_state_step_mixed": C.KERNEL_INC_STATE_STEP_MIXED,
           "adjoint_step": C.KERNEL_ADJOINT_STEP,
           "assemble": C.KERNEL_ASSEMBLE, "copy": C.KERNEL_COPY}[args.roofline_kernel]
    if args.kernels_only:
        # the kernels' state at v = v*/2, with the float16 copy for the mixed step
        ctx.set_precision(1)
        ctx.set_velocity((0.5 * vstar).contiguous())
        ms_k = ctx.time_kernel(kid, reps=5)
        ms_c = ctx.time_kernel(C.KERNEL_COPY, reps=5)
        print(json.dumps({"kernel": args.roofline_kernel, "ms_per_launch": ms_k,
                          "copy_ms_per_launch": ms_c, "voxels": n[0] * n[1] * n[2]}))
        ctx.close()
        return
    precisions = {"mixed": [1], "fp32": [0], "both": [1, 0]}[args.precision]
    if args.no_solve:
        voxels = n[0] * n[1] * n[2]
        rec = {"metric": METRIC, "value": None, "unit": "s", "n_gpus": 1, "steps": 0,
               "warmup": 0, "higher_is_better": False, "dtype": "f32",
               "data": "synthetic (seeded nested-ellipsoid phantom, band-limited v*)",
               "config": {"workload": args.workload, "grid": list(n), "nt": nt,
                          "alpha": alpha, "velocity": "v*/2"},
               "note": "matvec throughput and kernel table only, no solve"}
        vt = (0.5 * vstar).contiguous()
        hv = torch.empty_like(vt)
        for prec in precisions:
            ctx.set_precision(prec)
            ctx.set_velocity((0.5 * vstar).contiguous())
            ctx.hessian_matvec(vt, hv)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(ctx.stream)
            for _ in range(args.matvecs):
                ctx.hessian_matvec(vt, hv)
            e1.record(ctx.stream)
            e1.synchronize()
            ms = e0.elapsed_time(e1) / args.matvecs
            fields = 29 + 21 * nt if prec == 0 else 18 * nt + 26
            gbs = 4.0 * fields * voxels / (ms * 1e-3) / 1e9
            rec["fp32" if prec == 0 else "mixed"] = {
                "ms_per_matvec": round(ms, 3), "hessian_matvecs_per_s": round(1000.0 / ms, 2),
                "matvec_roofline": {"fields": fields, "achieved": round(gbs, 1),
                                    "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                    "frac": round(gbs / HBM_PEAK_GBS, 4)}}
        ctx.set_precision(1)
        ctx.set_velocity((0.5 * vstar).contiguous())
        rec["kernels"] = kernel_table(ctx, C, nt, voxels)
        ctx.close()
        print(json.dumps(rec), flush=True)
        return
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
            print("step (%s): solve %.3f s, %d GN iterations, %d matvecs, %d inner, status %d" %
                  (label, times[-1], stats["gn_iters"], stats["matvecs"], stats["inner_iters"],
                   stats["status"]), file=sys.stderr, flush=True)
        rec = dict(tts=sum(times) / len(times), stats=stats, v=v, prec=prec,
                   trace=ctx.solve_trace())
        rec["vs_oracle"] = vs_oracle(v, stats, rec["trace"], golden, m1_sha)
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
    # (--kernels-only) use: algorithmic bytes / live launch duration (the
    # mixed setup also holds the float32 fields the other kernels read)
    ctx.set_precision(1)
    ctx.set_velocity((0.5 * vstar).contiguous())

    ms_kernel = ctx.time_kernel(kid, reps=50)
    voxels = n[0] * n[1] * n[2]
    alg_bytes = kernel_bytes_per_voxel(args.roofline_kernel, nt) * voxels
    achieved = alg_bytes / (ms_kernel * 1e-3) / 1e9
    ms_copy = ctx.time_kernel(C.KERNEL_COPY, reps=50)
    copy_gbs = 24 * voxels / (ms_copy * 1e-3) / 1e9
    ktable = kernel_table(ctx, C, nt, voxels)
    print("kernel %s: %.4f ms/launch, %.0f GB/s algorithmic; copy kernel %.0f GB/s; "
          "matvec %.3f ms" % (args.roofline_kernel, ms_kernel, achieved, copy_gbs, ms_matvec),
          file=sys.stderr, flush=True)
    ctx.close()

    def converged(r):
        # a time-to-solution is only reported for a solve that ended without
        # a warning and met the gradient tolerance
        st = r["stats"]
        return st["status"] == 0 and st["rel_grad"] <= opts["gtol"]

    def matvec_roofline(r):
        # algorithmic fields per matvec: 29 + 21 nt float32 (incremental state
        # 7 + 11 nt, adjoint 6 nt, assembly 4 (nt + 1) + 3, alpha L v~ 15);
        # mixed: each read of a float16 grad m^j component counts half a field:
        # state 5.5 + 9.5 nt, adjoint 6 nt, assembly 2.5 (nt + 1) + 3, alpha
        # L v~ 15 -> 18 nt + 26
        fields = 29 + 21 * nt if r["prec"] == 0 else 18 * nt + 26
        nbytes = 4.0 * fields * n[0] * n[1] * n[2]
        gbs = nbytes / (r["ms_matvec"] * 1e-3) / 1e9
        return {"fields": fields, "algorithmic_bytes": nbytes, "achieved": round(gbs, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(gbs / HBM_PEAK_GBS, 4)}

    def solve_rec(r):
        st = r["stats"]
        rec = {k: st[k] for k in ("status", "warning", "initial_rejected", "gn_iters", "matvecs",
                                  "inner_iters", "pde_solves", "linesearch_trials",
                                  "rel_grad", "rel_mismatch", "J0", "J", "det_min", "det_max",
                                  "det_nonpositive")}
        rec.update(converged=converged(r),
                   time_to_solution_s=round(r["tts"], 4) if converged(r) else None,
                   hessian_matvecs_per_s=round(1000.0 / r["ms_matvec"], 2),
                   ms_per_matvec=round(r["ms_matvec"], 4),
                   matvec_roofline=matvec_roofline(r),
                   vs_oracle=r["vs_oracle"])
        return rec

    ok = converged(head)
    out = {
        "metric": METRIC,
        "value": round(tts, 4) if ok else None,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(tts * 1e3, 2),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if head["prec"] == 0 else "f32 arithmetic, f16 storage (mixed)",
        "data": "synthetic (seeded nested-ellipsoid phantom, band-limited v*)",
        "config": {"workload": args.workload, "grid": list(n), "nt": nt,
                   "alpha": alpha if not levels else levels,
                   "regularization": "H%d seminorm" % w["reg_order"] + (
                       "" if args.beta <= 0 else
                       ", near-incompressible (divergence penalty beta = %g)" % args.beta),
                   "gtol": opts["gtol"],
                   "preconditioner": "(alpha L)^-1" if args.precond == "reg" else
                   "two-level zero-velocity H0 (coarse grid n/2, inner CG to 0.1 eta)",
                   "precision": "mixed: float16 grad m^j read by the "
                                "Hessian matvec, float32 arithmetic/FFTs, float64 reductions"
                   if head["prec"] == 1 else "float32 fields and FFTs, float64 reductions",
                   "initial_guess": "learned warm start (%s), stopping test against "
                                    "||g(v=0)||_inf" % os.path.basename(args.warmstart)
                   if modes[0][2] else "v = 0",
                   "parallelism": "single GPU"},
        "hessian_matvecs_per_s": round(1000.0 / ms_matvec, 2),
        "ms_per_matvec": round(ms_matvec, 4),
        "matvec_roofline": matvec_roofline(head),
        "solve": solve_rec(head),
        "kernels": ktable,
        "inputs": {"m1": "FP64 oracle transport of the clean phantom by v* (+ noise), "
                         "float32", "m1_sha256": m1_sha[:16],
                   "oracle_record": None if golden is None else
                   "tests/golden/%s_%s_solve.json" % (args.workload, "ni" if args.beta > 0
                                                      else "h%d" % w["reg_order"])},
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
    if not ok:
        out["error"] = ("the headline solve did not converge (status %d, rel_grad %.3g): no "
                        "time-to-solution is reported" % (head["stats"]["status"],
                                                          head["stats"]["rel_grad"]))
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(args.workload, m0_h, m1_h, vstar_h)
    print(json.dumps(out), flush=True)
    if not ok:
        sys.exit(3)


if __name__ == "__main__":
    main()
