"""Comparison of a GPU grid with a stored oracle snapshot (tests/golden/*.json).

A snapshot pins the whole grid without storing it: exact membership through a
SHA-256 of the sorted cell indices, the index-weighted density moments over
every cell, and the densities of an evenly spaced sample of cells (see
tests/golden/make_golden.py, which runs only the oracle).
"""
import hashlib
import json
import os

import numpy as np

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    with open(os.path.join(HERE, f"{name}.json")) as fh:
        return json.load(fh)


def _packed(idx):
    """One int64 per cell (63 // n bits per biased coordinate), ordered like the
    lexicographic order of the rows."""
    idx = np.asarray(idx, dtype=np.int64).reshape(len(idx), -1)
    bits = 63 // idx.shape[1]
    bias = 1 << (bits - 1)
    assert idx.size == 0 or (idx.min() >= -bias and idx.max() < bias), "index outside the packed range"
    key = np.zeros(len(idx), dtype=np.int64)
    for j in range(idx.shape[1]):
        key = (key << bits) + (idx[:, j] + bias)
    return key


def check(gi, gp, gt, snap, thr, tol=1e-12, near=1e-11, label=""):
    """Assert the GPU grid (sorted idx, P, t) matches the snapshot: same time,
    same cells (unless the oracle took a threshold decision within `near` of
    max P, which is reported), sampled densities within tol * max P, and the
    moments sum P i_j^k (k = 0, 1, 2) within the bound that a per-cell error
    of tol * max P allows.  When the cell sets differ after a near-threshold
    decision, sampled densities must agree within 4 thr * max P: a flipped
    decision concerns a cell within rounding of p* = thr * max P, and the
    densities it reroutes stay of that size.  Returns the largest sampled error
    over max P."""
    assert gt == snap["t"], (label, gt, snap["t"])
    scale = snap["max_p"]
    same = hashlib.sha256(np.ascontiguousarray(gi, dtype="<i4").tobytes()).hexdigest() == snap["idx_sha256"]
    print(f"[{label}] cells gpu={len(gi)} oracle={snap['cells']} same_set={same} margin={snap['min_margin']:.3g}",
          flush=True)
    if not same:
        assert snap["min_margin"] < near, f"{label}: membership differs ({len(gi)} vs {snap['cells']} cells)"
    else:
        assert len(gi) == snap["cells"]
    # sampled densities
    keys = _packed(gi)
    sk = _packed(np.asarray(snap["sample_idx"], dtype=np.int64))
    pos = np.searchsorted(keys, sk)
    found = (pos < len(keys)) & (keys[np.minimum(pos, len(keys) - 1)] == sk)
    if same:
        assert found.all(), f"{label}: sampled cells missing"
    got = np.where(found, gp[np.minimum(pos, len(gp) - 1)], 0.0)
    err = np.abs(got - np.asarray(snap["sample_p"])) / scale
    bad = np.flatnonzero(err > (tol if same else 4 * thr))
    assert bad.size == 0, f"{label}: sampled density error {err.max():.3g} at {np.asarray(snap['sample_idx'])[bad[:5]]}"
    if same:
        # moments over every cell
        i = gi.astype(np.float64)
        mo = snap["moments"]
        assert abs(gp.sum() - mo["m0"]) <= tol * scale * len(gi), (label, "m0")
        for k, (gm, om) in enumerate([(gp @ i, mo["m1"]), (gp @ (i * i), mo["m2"])], start=1):
            bound = tol * scale * (np.abs(i) ** k).sum(axis=0)
            assert np.all(np.abs(gm - np.asarray(om)) <= bound), (label, f"m{k}", gm, om)
    return float(err.max()) if err.size else 0.0
