"""Train the learned warm start on triples (m0, m1, v) produced by the plain
Gauss--Newton--Krylov solver itself.

For each sample: a random nested-ellipsoid phantom m0 (64^3 or 128^3), a
band-limited velocity v* (|k| <= 8, max speed U[0.5, 1]), m1 = m0 transported
by v* (this library's claire_transport) plus noise; the solver registers m0
to m1 (H1, alpha 1e-3, nt 4, gtol 5e-2) and its solution v is the training
target. Images and targets are restricted to the network's working
resolution (block means) and kept on the GPU; training runs the library's
forward/backward/Adam kernels (claire_net_train_step). Held-out samples
measure the relative error of the prediction against the solver's v.

    python -m paper_2401_17493_amd.train_warmstart --samples 2000 \\
        --out paper_2401_17493_amd/weights/warmstart_r64.npz

Phantoms are generated on the host by a process pool (CPU only); every GPU
call happens in the main process.
"""
from __future__ import annotations

import argparse
import json
import math
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from synthetic import bandlimited_velocity, ellipsoid_phantom, noise  # noqa: E402

ALPHA, NT, GTOL, KMAX = 1e-3, 4, 5e-2, 8


def make_inputs(args):
    """Host-side phantom, velocity and noise of one sample (seeded)."""
    n, seed = args
    r = np.random.default_rng(seed)
    vmax = float(r.uniform(0.5, 1.0))
    shape = (n, n, n)
    clean = ellipsoid_phantom(shape, seed).astype(np.float32)
    vstar = bandlimited_velocity(shape, seed + 1, KMAX, vmax).astype(np.float32)
    n0 = noise(shape, seed + 2, 0.01).astype(np.float32)
    n1 = noise(shape, seed + 3, 0.01).astype(np.float32)
    return n, seed, clean, vstar, n0, n1


def log(msg):
    print(msg, flush=True)


def generate(pool, samples, frac128, res, seed0):
    """Solve `samples` registrations; returns GPU tensors at res^3 and stats."""
    import torch
    from paper_2401_17493_amd import claire
    from paper_2401_17493_amd.warmstart import resample
    every = int(round(1.0 / frac128)) if frac128 > 0 else 0      # every k-th sample at 128^3
    jobs = [(128 if every and i % every == 0 else 64, seed0 + 10 * i) for i in range(samples)]
    R = res
    M0 = torch.empty((samples, R, R, R), device="cuda")
    M1 = torch.empty_like(M0)
    V = torch.empty((samples, 3, R, R, R), device="cuda")
    stats = {"gn_iters": [], "matvecs": [], "seconds": [], "n": []}
    t0 = time.time()
    for i, (n, seed, clean, vstar, n0, n1) in enumerate(pool.imap(make_inputs, jobs,
                                                                   chunksize=4)):
        c = torch.from_numpy(clean).cuda()
        m0 = c + torch.from_numpy(n0).cuda()
        m1 = claire.transport(c, torch.from_numpy(vstar).cuda(), NT) + \
            torch.from_numpy(n1).cuda()
        v, st = claire.solve(m0, m1, ALPHA, NT, reg_order=1, gtol=GTOL, precision=1)
        M0[i] = resample(m0, R)
        M1[i] = resample(m1, R)
        V[i] = resample(v, R)
        for k in ("gn_iters", "matvecs", "seconds"):
            stats[k].append(st[k])
        stats["n"].append(n)
        if (i + 1) % 100 == 0 or i + 1 == samples:
            log("[data] %d/%d solved (%.1f s; last: n %d, %d GN, %d matvecs, %.3f s)" % (
                i + 1, samples, time.time() - t0, n, st["gn_iters"], st["matvecs"],
                st["seconds"]))
    torch.cuda.synchronize()
    return M0, M1, V, stats


def train(net, M0, M1, V, idx_train, idx_val, epochs, batch, lr, seed):
    import torch
    rng = np.random.default_rng(seed)
    steps_per_epoch = len(idx_train) // batch
    total = epochs * steps_per_epoch
    history = []
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        perm = rng.permutation(idx_train)
        losses = []
        for s in range(steps_per_epoch):
            b = torch.from_numpy(perm[s * batch:(s + 1) * batch]).cuda()
            # cosine decay from lr to lr / 20
            cur = lr * (0.05 + 0.95 * 0.5 * (1 + math.cos(math.pi * step / max(1, total))))
            losses.append(net.train_step(M0[b].contiguous(), M1[b].contiguous(),
                                         V[b].contiguous(), cur))
            step += 1
        val = evaluate(net, M0, M1, V, idx_val)
        history.append({"epoch": ep + 1, "train_loss": float(np.mean(losses)),
                        "val_rel_err": val, "seconds": time.time() - t0})
        log("[train] epoch %d: loss %.4e, held-out rel. error %.3f (%.1f s)" % (
            ep + 1, np.mean(losses), val, time.time() - t0))
    return history


def evaluate(net, M0, M1, V, idx):
    """Mean over samples of ||v_net - v_solver||_2 / ||v_solver||_2."""
    errs = []
    for i in idx:
        v = net.forward(M0[i].contiguous(), M1[i].contiguous())[0]
        errs.append(float((v - V[i]).norm() / V[i].norm().clamp_min(1e-30)))
    return float(np.mean(errs))


def solve_pair(net, n, seed, precision):
    """Cold (v0 = 0) and warm (v0 from the network) solves of one held-out
    problem at n^3; both stop at ||g||_inf <= gtol ||g(v = 0)||_inf. The warm
    time includes the network's inference (restriction, forward pass,
    prolongation)."""
    import torch
    from paper_2401_17493_amd import claire
    _, _, clean, vstar, n0, n1 = make_inputs((n, seed))
    c = torch.from_numpy(clean).cuda()
    m0 = c + torch.from_numpy(n0).cuda()
    m1 = claire.transport(c, torch.from_numpy(vstar).cuda(), NT) + torch.from_numpy(n1).cuda()
    out = {}
    with claire.Context((n, n, n), NT, ALPHA, 1) as ctx:
        ctx.set_images(m0, m1)
        ctx.solve(None, max_gn=0)        # allocates the solver's buffers (untimed)
        for mode in ("cold", "warm"):
            torch.cuda.synchronize()
            t = time.time()
            v0 = net.warm_start(m0, m1) if mode == "warm" else None
            v, st = ctx.solve(v0, gtol=GTOL, precision=precision,
                              tol_from_zero=1 if mode == "warm" else 0)
            torch.cuda.synchronize()
            out[mode] = {"seconds": time.time() - t, "gn_iters": st["gn_iters"],
                         "matvecs": st["matvecs"], "J0": st["J0"], "J": st["J"],
                         "rel_grad": st["rel_grad"], "rel_mismatch": st["rel_mismatch"],
                         "status": st["status"]}
    return out


def evaluate_solves(net, sizes, seeds, precision=1):
    rows = []
    for n in sizes:
        for sd in seeds:
            r = solve_pair(net, n, sd, precision)
            r["n"], r["seed"] = n, sd
            rows.append(r)
            log("[eval] n %d seed %d: cold %d GN / %d matvecs / %.3f s, warm %d GN / %d matvecs"
                " / %.3f s (J0 %.4f -> %.4f)" % (
                    n, sd, r["cold"]["gn_iters"], r["cold"]["matvecs"], r["cold"]["seconds"],
                    r["warm"]["gn_iters"], r["warm"]["matvecs"], r["warm"]["seconds"],
                    r["cold"]["J0"], r["warm"]["J0"]))
    return rows


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--samples", type=int, default=2000)
    ap.add_argument("--frac128", type=float, default=0.2, help="share of 128^3 samples")
    ap.add_argument("--holdout", type=int, default=64)
    ap.add_argument("--res", type=int, default=64)
    ap.add_argument("--channels", type=str, default="16,32,64,128")
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=9000)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", type=str, required=True)
    ap.add_argument("--log", type=str, default=None)
    ap.add_argument("--eval-sizes", type=str, default="128,256",
                    help="grids of the held-out cold/warm solve comparison ('' to skip)")
    ap.add_argument("--eval-seeds", type=int, default=3)
    a = ap.parse_args(argv)

    # the host worker pool starts before this process touches the GPU
    pool = mp.get_context("spawn").Pool(a.workers)
    import torch
    from paper_2401_17493_amd.warmstart import Net
    if not torch.cuda.is_available():
        raise SystemExit("a GPU is required")
    channels = tuple(int(c) for c in a.channels.split(","))
    log("[setup] %d samples (%.0f%% at 128^3), working resolution %d^3, channels %s" % (
        a.samples, 100 * a.frac128, a.res, channels))
    t0 = time.time()
    M0, M1, V, stats = generate(pool, a.samples, a.frac128, a.res, a.seed)
    pool.close()
    pool.join()
    t_data = time.time() - t0
    idx = np.arange(a.samples)
    idx_val = idx[-a.holdout:]
    idx_train = idx[:-a.holdout]
    net = Net(a.res, channels, max_batch=a.batch, seed=a.seed)
    log("[setup] %d parameters; data %.1f s" % (net.nparam, t_data))
    val0 = evaluate(net, M0, M1, V, idx_val)
    zero_err = 1.0     # v0 = 0 has relative error 1 by definition
    log("[train] untrained held-out rel. error %.3f" % val0)
    t1 = time.time()
    hist = train(net, M0, M1, V, idx_train, idx_val, a.epochs, a.batch, a.lr, a.seed)
    t_train = time.time() - t1
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    net.save(a.out)
    sizes = [int(k) for k in a.eval_sizes.split(",") if k]
    eval_seeds = [a.seed + 10 * (a.samples + 100 + i) for i in range(a.eval_seeds)]
    rows = evaluate_solves(net, sizes, eval_seeds) if sizes else []
    record = {
        "command": "python -m paper_2401_17493_amd.train_warmstart " + " ".join(
            argv if argv is not None else sys.argv[1:]),
        "samples": a.samples, "holdout": a.holdout, "res": a.res, "channels": channels,
        "epochs": a.epochs, "batch": a.batch, "lr": a.lr, "seed": a.seed,
        "solver": {"alpha": ALPHA, "nt": NT, "gtol": GTOL, "reg_order": 1, "precision": "mixed",
                   "mean_gn_iters": float(np.mean(stats["gn_iters"])),
                   "mean_matvecs": float(np.mean(stats["matvecs"])),
                   "mean_seconds": float(np.mean(stats["seconds"])),
                   "n_128": int(sum(1 for n in stats["n"] if n == 128))},
        "data_seconds": t_data, "train_seconds": t_train,
        "val_rel_err_untrained": val0, "val_rel_err_zero": zero_err,
        "val_rel_err": hist[-1]["val_rel_err"], "history": hist,
        "eval_solves": rows,
    }
    log_path = a.log or os.path.splitext(a.out)[0] + ".json"
    with open(log_path, "w") as f:
        json.dump(record, f, indent=1)
    log("[done] held-out rel. error %.3f (untrained %.3f); weights %s" % (
        hist[-1]["val_rel_err"], val0, a.out))
    net.close()


if __name__ == "__main__":
    main()
