"""Write the stored oracle results that the large GPU parity tests compare with.

Runs only the CPU oracle (oracle/) on the seeded workloads of
paper_2508_13986_amd.scenarios, which are too large for the oracle to run
inside a test, and stores for each snapshot what pins the whole grid without
storing it: the cell count, a SHA-256 of the sorted cell indices (exact
membership), index-weighted density moments over every cell, the oracle's
smallest threshold margin, and the densities of an evenly spaced sample of
cells.  Usage: python tests/golden/make_golden.py [name ...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SAMPLE = 512


def membership_hash(idx):
    return hashlib.sha256(np.ascontiguousarray(idx, dtype="<i4").tobytes()).hexdigest()


def moments(idx, p):
    """sum P, sum P i_j and sum P i_j^2 per dimension, with the matching sums of
    |P| |i_j|^k that bound their rounding."""
    i = idx.astype(np.float64)
    ap = np.abs(p)
    return {"m0": float(p.sum()), "m1": (p @ i).tolist(), "m2": (p @ (i * i)).tolist(),
            "a0": float(ap.sum()), "a1": (ap @ np.abs(i)).tolist(), "a2": (ap @ (i * i)).tolist()}


def snapshot(orc, label):
    idx, p = orc.export()
    st = orc.stats()
    n = len(p)
    pick = np.unique(np.concatenate([np.linspace(0, n - 1, SAMPLE).astype(np.int64), [int(np.argmax(p))]]))
    return {"label": label, "t": st["t"], "steps": st["steps"], "prunes": st["prunes"],
            "cell_updates": st["cell_updates"], "cells": n, "idx_sha256": membership_hash(idx),
            "max_p": float(p.max()), "min_margin": st["min_margin"], "moments": moments(idx, p),
            "sample_idx": idx[pick].tolist(), "sample_p": [float(v) for v in p[pick]]}


def run_l63_corrections():
    """The Lorenz '63 corrections workload as specified (h = 0.25, cov 2 I,
    thr 1e-6, x1 corrections every 0.25 to t = 2): the grid before the first
    correction and after every correction."""
    from paper_2508_13986_amd import scenarios as S
    import oracle
    cfg = S.l63_corrections()
    o = oracle.Oracle(cfg).init_gaussian()
    snaps = [snapshot(o, "init")]
    for k, m in enumerate(cfg["measurements"]):
        o.step(m[0])
        if k == 0:
            snaps.append(snapshot(o, f"t={m[0]}"))
        o.correct(m[1], m[2], m[3])
        snaps.append(snapshot(o, f"t={m[0]} corrected"))
    return cfg, snaps, None


def run_l96_6d_first_steps():
    """The Lorenz '96 6D benchmark workload at full size (h = 0.25, thr 1e-7,
    1.1e7 initial cells): the initial grid and its first two steps."""
    from paper_2508_13986_amd import scenarios as S
    import oracle
    cfg = S.l96_6d()
    o = oracle.Oracle(cfg).init_gaussian()
    snaps = [snapshot(o, "init")]
    for k in (1, 2):
        o.step(cfg["t_end"], 1)
        snaps.append(snapshot(o, f"step {k}"))
    return cfg, snaps, None


def run_l96_6d_h04():
    """Lorenz '96 6D at h = 0.4, thr 1e-5 (2.3e5 initial cells): 22 steps,
    pruned after step 20."""
    from paper_2508_13986_amd import scenarios as S
    import oracle
    cfg = S.l96_6d(h=0.4, thresh_rel=1e-5)
    o = oracle.Oracle(cfg).init_gaussian()
    snaps = []
    o.step(cfg["t_end"], 20)
    snaps.append(snapshot(o, "step 20 (pruned)"))
    o.step(cfg["t_end"], 2)
    snaps.append(snapshot(o, "step 22"))
    return cfg, snaps, None


def serving_request(k):
    """Request k of the serving stream (scenarios.serving_requests(64), seed 5);
    the Lorenz '96 ones that the pool tests use are cut to a horizon of 0.3
    (with the measurements before it), where their grids stay small enough for
    the oracle."""
    from paper_2508_13986_amd import scenarios as S
    reqs, _ = S.serving_requests(64)
    cfg = dict(reqs[k])
    if cfg["n"] == 6:
        cfg["t_end"] = min(cfg["t_end"], 0.3)
        cfg["measurements"] = [m for m in cfg["measurements"] if m[0] <= cfg["t_end"]]
    return cfg


def run_serving_request(k):
    """Request k of the serving stream (scenarios.serving_requests(64), seed 5),
    propagated as the pool runs it: step to each measurement time, correct, step
    to the horizon; the final grid."""
    import oracle
    cfg = serving_request(k)
    o = oracle.Oracle(cfg).init_gaussian()
    for (t, comp, y, sigma) in sorted(cfg["measurements"]):
        if t <= cfg["t_end"]:
            o.step(t)
            o.correct(comp, y, sigma)
    o.step(cfg["t_end"])
    return cfg, [snapshot(o, "final")], None


# Requests of the serving stream that the pool tests run.
SERVING_TEST_REQUESTS = (1, 2, 4, 8, 9, 12, 14, 15, 41, 52)

RUNS = {"l63_corrections": run_l63_corrections, "l96_6d_first_steps": run_l96_6d_first_steps,
        "l96_6d_h04_22steps": run_l96_6d_h04}


for _k in SERVING_TEST_REQUESTS:
    RUNS[f"serving_req{_k}"] = (lambda k: (lambda: run_serving_request(k)))(_k)
    RUNS[f"serving_req{_k}"].__doc__ = run_serving_request.__doc__.replace("Request k", f"Request {_k}")


def main(names):
    for name in names or list(RUNS):
        t0 = time.time()
        cfg, snaps, _ = RUNS[name]()
        out = {"name": name, "source": "oracle/ (CPU, FP64), written by tests/golden/make_golden.py",
               "doc": RUNS[name].__doc__.strip(), "config": {k: v for k, v in cfg.items() if k != "request"},
               "snapshots": snaps}
        with open(os.path.join(HERE, f"{name}.json"), "w") as fh:
            json.dump(out, fh, indent=0)
        print(name, f"{time.time() - t0:.0f} s", [(s["label"], s["cells"]) for s in snaps], flush=True)


if __name__ == "__main__":
    main(sys.argv[1:])
