"""Shared helpers of the tests: seeded workloads, float32 rounding, error norms."""
import numpy as np

import oracle as O
from synthetic import (WORKLOADS, bandlimited_velocity, ellipsoid_phantom, gaussian_blobs,
                       noise)


def f32(a):
    """Round to float32 and back: the oracle sees exactly the GPU's inputs."""
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def rel_err(got, ref):
    """max |got - ref| / max |ref| (max-norm relative error)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.abs(ref).max()
    return float(np.abs(got - ref).max() / (den if den > 0 else 1.0))


def blob_problem(n=(32, 32, 32), nt=4, seed=1001, kmax=4, vmax=0.5, sigma=0.3):
    """Template, reference (oracle transport by v*, inverse crime) and v*."""
    grid = O.Grid(n)
    m0 = f32(gaussian_blobs(n, seed, sigma=sigma))
    vstar = f32(bandlimited_velocity(n, seed + 1000, kmax, vmax))
    m1 = f32(O.transport(grid, m0, vstar, nt))
    return grid, m0, m1, vstar


def phantom_problem(name, n=None, nt=None):
    """Ellipsoid workload of the named recipe, optionally at another size."""
    w = dict(WORKLOADS[name])
    n = tuple(n or w["n"])
    nt = nt or w["nt"]
    grid = O.Grid(n)
    seed = w["seed"]
    clean = ellipsoid_phantom(n, seed)
    vstar = f32(bandlimited_velocity(n, seed + 1000, min(w["kmax"], n[0] // 2 - 1), w["vmax"]))
    m0 = f32(clean + noise(n, seed + 2000, w["noise"]))
    m1 = f32(O.transport(grid, clean, vstar, nt) + noise(n, seed + 3000, w["noise"]))
    return grid, m0, m1, vstar, w


class Parity:
    """Collects (name, error, tolerance) triples, prints them, and fails at
    the end if any error exceeds its tolerance (so one run shows them all)."""

    def __init__(self, label):
        self.label = label
        self.rows = []

    def rel(self, name, got, ref, tol):
        e = rel_err(got, ref)
        self.rows.append((name, e, tol))
        print("PARITY %s %-28s rel_err %.3e  tol %.1e  %s"
              % (self.label, name, e, tol, "ok" if e <= tol else "FAIL"), flush=True)
        return e

    def value(self, name, got, ref, tol):
        e = abs(got - ref) / max(abs(ref), 1e-300)
        self.rows.append((name, e, tol))
        print("PARITY %s %-28s rel_err %.3e  tol %.1e  %s"
              % (self.label, name, e, tol, "ok" if e <= tol else "FAIL"), flush=True)
        return e

    def done(self):
        bad = [(n, e, t) for n, e, t in self.rows if not e <= t]
        assert not bad, bad


def trace_parity(P, label, trace, history, tol, steps=None):
    """Per-iterate J and ||g||_inf, PCG matvec counts and the PCG residual
    histories ||r_l||_inf of a GPU solve against the oracle's record (the
    first ``steps`` records if given, else all and the same count).

    ||g_k||_inf is compared relative to the level's first ||g_0||_inf: g_k is
    alpha L v + the data term, two parts of the size of g_0 that cancel as the
    solve converges, so its float32 error scales with ||g_0||_inf."""
    if steps is None:
        assert len(trace) == len(history), (len(trace), len(history))
    else:
        trace, history = trace[:steps], history[:steps]
        assert len(trace) == len(history) == steps, (len(trace), len(history))
    g0 = {}
    for t, h in zip(trace, history):
        g0.setdefault(h.get("alpha", 0), h["gnorm"])
        P.value("%s J k=%d" % (label, h["k"]), t["J"], h["J"], tol)
        P.value("%s |g|/|g0| k=%d" % (label, h["k"]), 1.0 + (t["gnorm"] - h["gnorm"]) /
                g0[h.get("alpha", 0)], 1.0, tol)
        if "pcg_its" in h:
            assert t["pcg_its"] == h["pcg_its"], (h["k"], t["pcg_its"], h["pcg_its"])
            assert t["ls"] == h["ls"] and t["gamma"] == h["gamma"]
            res, ref = np.array(t["pcg_res"]), np.array(h["pcg_res"])
            assert res.shape == ref.shape
            # each residual relative to the step's initial residual ||g||_inf
            P.value("%s |r_l| k=%d (max over l)" % (label, h["k"]),
                    1.0 + float(np.abs(res - ref).max() / ref[0]), 1.0, tol)
