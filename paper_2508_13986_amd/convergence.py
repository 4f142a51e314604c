"""Convergence study of the propagation (Sec. 5.2.2, Eq. 10 and Figs. 7-8 in
their Lorenz '63 form): runs of the GPU path with a scaled time step or cell
width, compared against a reference run with a much smaller one.

Metrics, on the reference run's cells (host-side, from exported grids):

* E(t) = V_ref * sum_i |p(x_i, t) - p0(x_i, t)|, the 1-norm of Eq. 10;
* BC(t) = V_ref * sum_i sqrt(p(x_i, t) p0(x_i, t)), the Bhattacharyya
  coefficient of Eq. 9 with the cell volume the printed formula leaves out.

Readings (the figures and their captions give only the parameter sets):

* the time-step factor eps scales the CFL step: the Courant number C = eps;
* the cell-width factor eta scales every h_j, at C = 0.1 for all runs;
* grids of different cell widths are compared on the reference lattice: a
  coarse density is piecewise constant over its cells, so p(x_i) is the
  density of the coarse cell containing the reference centre x_i; the sum runs
  over reference centres inside a cell of either grid (missing cells are 0);
* both runs take the same measurement updates at the same times, and the
  metrics are evaluated right after each update and at the horizon.

Nothing here changes the propagation: it drives the library through the
binding and post-processes exported grids.
"""
import argparse
import json

import numpy as np

from . import gbees as G
from . import scenarios as S


def base_config(h=0.5, t_end=2.0):
    """Lorenz '63 with corrections every 0.25 (the study's scenario): the
    corrections workload at cell width h."""
    return S.with_(S.workload("l63_corrections"), h=[float(h)] * 3, t_end=float(t_end))


def snapshots(cfg, max_cells=64 * 200_000):
    """Run cfg; return [(t, idx, P)] after every measurement update and at t_end."""
    g = G.Grid.gaussian(cfg, max_cells)
    out = []
    try:
        for (t, comp, y, sigma) in sorted(cfg.get("measurements", [])):
            if t <= cfg["t_end"]:
                g.step(t)
                g.correct(comp, y, sigma)
                idx, P, tt = g.export()
                out.append((tt, idx, P))
        g.step(cfg["t_end"])
        idx, P, tt = g.export()
        if not out or out[-1][0] != tt:
            out.append((tt, idx, P))
    finally:
        g.close()
    return out


_BIAS = 1 << 20


def _keys(idx):
    """One int64 per multi-index (|i_j| < 2^20, 21 bits per dimension)."""
    idx = np.asarray(idx, dtype=np.int64)
    k = np.zeros(idx.shape[0], dtype=np.int64)
    for j in range(idx.shape[1]):
        k = (k << 21) | (idx[:, j] + _BIAS)
    return k


def _lookup(keys_sorted, vals_sorted, q):
    """vals at keys q (0 where absent)."""
    pos = np.searchsorted(keys_sorted, q)
    pos = np.minimum(pos, len(keys_sorted) - 1)
    hit = (len(keys_sorted) > 0) & (keys_sorted[pos] == q) if len(keys_sorted) else np.zeros(len(q), bool)
    return np.where(hit, vals_sorted[pos] if len(keys_sorted) else 0.0, 0.0)


def _covered_reference_points(idx, h, h_ref):
    """Reference-lattice indices whose centres lie in the cells idx of width h
    (same origin: centres at mean + i h and mean + i_r h_ref)."""
    idx = np.asarray(idx, dtype=np.int64)
    n = idx.shape[1]
    lo = np.ceil((idx - 0.5) * h / h_ref - 1e-9).astype(np.int64)
    hi = np.ceil((idx + 0.5) * h / h_ref - 1e-9).astype(np.int64) - 1
    span = int((hi - lo).max()) + 1 if idx.size else 0
    pts = []
    for off in np.ndindex(*([span] * n)):
        o = np.asarray(off, dtype=np.int64)
        cand = lo + o
        keep = np.all(cand <= hi, axis=1)
        pts.append(cand[keep])
    return np.concatenate(pts) if pts else np.zeros((0, n), dtype=np.int64)


def compare(run, ref, h, h_ref):
    """E and BC of grid `run` (cell width h) against `ref` (cell width h_ref),
    both given as (idx, P); widths are per-dimension sequences."""
    idx, P = run
    ridx, rP = ref
    h = np.asarray(h, dtype=np.float64)
    h_ref = np.asarray(h_ref, dtype=np.float64)
    vol_ref = float(np.prod(h_ref))
    k_run = _keys(idx)
    o = np.argsort(k_run)
    k_run, P_s = k_run[o], np.asarray(P, dtype=np.float64)[o]
    k_ref = _keys(ridx)
    o = np.argsort(k_ref)
    k_ref, rP_s = k_ref[o], np.asarray(rP, dtype=np.float64)[o]
    if np.array_equal(h, h_ref):
        points = np.unique(np.concatenate([k_run, k_ref]))
        p = _lookup(k_run, P_s, points)
    else:
        pts = np.concatenate([_covered_reference_points(idx, h, h_ref), np.asarray(ridx, dtype=np.int64)])
        pts = np.unique(pts, axis=0)
        points = _keys(pts)
        # the coarse cell holding each reference centre: floor(x / h + 1/2)
        cell = np.floor(pts * h_ref / h + 0.5 + 1e-9).astype(np.int64)
        p = _lookup(k_run, P_s, _keys(cell))
    p0 = _lookup(k_ref, rP_s, points)
    E = vol_ref * float(np.abs(p - p0).sum())
    BC = vol_ref * float(np.sqrt(np.maximum(p, 0.0) * np.maximum(p0, 0.0)).sum())
    return E, BC


def study(kind, factors, ref_factor, h_star=0.5, t_end=2.0, max_cells=64 * 200_000):
    """Temporal (kind 'eps': C = factor) or spatial (kind 'eta': h = factor
    h_star at C = 0.1) study.  Returns {factor: [(t, E, BC), ...]}."""
    def cfg_for(f):
        if kind == "eps":
            return S.with_(base_config(h_star, t_end), cfl=float(f))
        return S.with_(base_config(f * h_star, t_end), cfl=0.1)

    ref_cfg = cfg_for(ref_factor)
    ref = snapshots(ref_cfg, max_cells)
    out = {}
    for f in factors:
        cfg = cfg_for(f)
        snaps = snapshots(cfg, max_cells)
        assert len(snaps) == len(ref)
        rows = []
        for (t, idx, P), (t0, ridx, rP) in zip(snaps, ref):
            assert abs(t - t0) < 1e-12
            E, BC = compare((idx, P), (ridx, rP), cfg["h"], ref_cfg["h"])
            rows.append((t, E, BC))
        out[f] = rows
    return out


def main():
    ap = argparse.ArgumentParser(description="Temporal and spatial convergence of the Lorenz '63 propagation.")
    ap.add_argument("--out", required=True)
    ap.add_argument("--eps", default="1,0.5,0.2,0.1")
    ap.add_argument("--eps-ref", type=float, default=0.01)
    ap.add_argument("--eta", default="1.25,1,0.8,0.6")
    ap.add_argument("--eta-ref", type=float, default=0.5)
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    eps = [float(v) for v in args.eps.split(",")]
    eta = [float(v) for v in args.eta.split(",")]
    res = {"scenario": "Lorenz '63 (10, 28, 8/3), mean (-11.5, -10, 9.5), cov 2 I, thr 1e-6, MC limiter, "
                       "corrections on x1 every 0.25 to t = 2; h* = 0.5",
           "temporal": {"reference_eps": args.eps_ref, "runs": {}},
           "spatial": {"reference_eta": args.eta_ref, "cfl": 0.1, "runs": {}}}
    for f, rows in study("eps", eps, args.eps_ref).items():
        res["temporal"]["runs"][str(f)] = [{"t": t, "E": E, "BC": BC} for t, E, BC in rows]
        print(json.dumps({"eps": f, "E_end": rows[-1][1], "BC_end": rows[-1][2]}), flush=True)
    for f, rows in study("eta", eta, args.eta_ref).items():
        res["spatial"]["runs"][str(f)] = [{"t": t, "E": E, "BC": BC} for t, E, BC in rows]
        print(json.dumps({"eta": f, "E_end": rows[-1][1], "BC_end": rows[-1][2]}), flush=True)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
