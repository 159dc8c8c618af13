"""Write the FP64 oracle's values at sampled voxels of the 512^3 workload
(n_t = 8, H1, alpha = 1e-3): one transport and one Gauss--Newton Hessian
matvec, for element-wise comparison with the GPU at full size.

* transport: m(1) of the float32-rounded clean phantom by v* (the recipe's
  band-limited velocity, |k| <= 16);
* setup at v = v*/2 on the workload's images (m1 = oracle transport of the
  clean phantom plus noise): J, g at the samples;
* H v~ at the samples for v~ = the seeded band-limited field (seed + 4000).

The setup keeps the state m^j but recomputes grad m^j where it is used
(store_grad=False): the stored float64 gradients alone would take 27 GiB.
Calls only oracle/ and synthetic/ (through tests/helpers.py). About 50 GiB
of memory; minutes on a 16-core host, about an hour on eight slower cores.

    python tests/golden/make_512_golden.py [--out PATH]
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
from helpers import f32, phantom_problem  # noqa: E402
from synthetic import WORKLOADS, bandlimited_velocity, ellipsoid_phantom  # noqa: E402

SAMPLES = 2048


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(a, dtype=np.float32).tobytes()).hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(HERE, "ellipsoids512_samples.json"))
    args = ap.parse_args()
    name = "ellipsoids512"
    w = WORKLOADS[name]
    t0 = time.time()
    grid, m0, m1, vstar, _ = phantom_problem(name)
    n, nt = grid.n, w["nt"]
    print("inputs (incl. the reference transport) %.0f s" % (time.time() - t0), flush=True)
    rng = np.random.default_rng(5120)
    idx = np.stack([rng.integers(0, k, SAMPLES) for k in n], axis=1)
    at = lambda a: a[..., idx[:, 0], idx[:, 1], idx[:, 2]]  # noqa: E731

    t1 = time.time()
    clean = f32(ellipsoid_phantom(n, w["seed"]))
    mt = O.transport(grid, clean, vstar, nt)
    t_transport = time.time() - t1
    transport = at(mt).tolist()
    del mt, clean
    print("transport %.0f s" % t_transport, flush=True)

    t1 = time.time()
    v = f32(0.5 * vstar)
    st = O.setup_velocity(grid, m0, m1, v, w["alphas"][-1], nt, w["reg_order"],
                          store_grad=False)
    t_setup = time.time() - t1
    print("setup %.0f s" % t_setup, flush=True)
    vt = f32(bandlimited_velocity(n, w["seed"] + 4000, w["kmax"], 1.0))
    t1 = time.time()
    hv = O.hessian_matvec(st, vt)
    t_matvec = time.time() - t1
    print("matvec %.0f s" % t_matvec, flush=True)
    model = platform.processor()
    try:
        with open("/proc/cpuinfo") as fh:
            model = next(l.split(":", 1)[1].strip() for l in fh if l.startswith("model name"))
    except (OSError, StopIteration):
        pass
    out = {
        "workload": name, "n": list(n), "nt": nt, "alpha": w["alphas"][-1],
        "reg_order": w["reg_order"], "m1_sha256": digest(m1),
        "sample_idx": idx.tolist(),
        "transport_clean_by_vstar": transport,
        "v": "f32(0.5 v*)", "vt": "f32(bandlimited(n, seed + 4000, kmax, 1.0))",
        "J": st.J, "g": at(st.g).T.tolist(), "g_max": float(np.abs(st.g).max()),
        "Hv": at(hv).T.tolist(), "Hv_max": float(np.abs(hv).max()),
        "seconds": {"transport": t_transport, "setup": t_setup, "matvec": t_matvec},
        "host": {"nproc": os.cpu_count(), "cpu_model": model, "threads": O.WORKERS},
    }
    path = args.out
    with open(path, "w") as fh:
        json.dump(out, fh)
    print("wrote", path, "in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
