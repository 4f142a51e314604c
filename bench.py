"""Benchmark of the GBEES hot path on one MI355X.

One benchmark step is one whole propagation job of the Lorenz '96 6D workload
(n = 6, F = 4, mean (4.5, 4, ..., 4), cov 0.25 I, h = 0.25, thr 1e-7, CFL 0.9,
MC-limited CTU, prune every 20 steps, t in [0, 1] with one x1 correction at
t = 0.5): Gaussian initialisation, grow / CFL / flux / update every step,
prune + renormalisation, the Bayesian correction.  The metric is CTU
cell-updates per second over the whole job (the paper's "cells/s").

Prints one JSON line (metric, value, roofline of the dominant kernel measured
with HIP events on the launch stream, and the CPU oracle on a bounded sample).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E


def flux_b_bytes_per_brick(n, real_size):
    """Algorithmic bytes of one brick (64 cell slots) in the flux-B pass: density
    row read, updated density row written, brick key, mask and 2n axis links,
    and the upwind face layers of the neighbours' corrected states (one layer of
    64/2 values per dimension: across each brick face only the downwind brick
    reads the upwind side's layer).  Neighbour density rows count zero (each is
    some brick's own row, read once with perfect reuse)."""
    return 64 * real_size + 64 * real_size + 8 + 8 + 4 * 2 * n + n * 32 * real_size


def flux_a_bytes_per_brick(n, real_size):
    """Flux-A pass: density row read, key, mask and links, and the face layers
    of Q written for the downwind neighbours (one layer of 64/2 values per
    dimension on average)."""
    return 64 * real_size + 8 + 8 + 4 * 2 * n + n * 32 * real_size


def alg_bytes_per_cell_update(n, real_size):
    """Algorithmic bytes of one cell-update of the flux + update pass (per cell,
    cell state read once and written once, connectivity stored per cell): the
    packed key (8, for the drift), P read and P' written (2 s) and 2n four-byte
    axis-neighbour indices.  72 B in 6-D FP64, 64 B in 6-D FP32, 48 B in 3-D
    FP64."""
    return 8 + 2 * real_size + 4 * 2 * n


# Whole-step bytes per cell-update of the 6-D FP64 method (flux + update, the
# grow check and the prune amortised over 20 steps), the model the end-to-end
# figure is read against.
WHOLE_STEP_BYTES_6D_FP64 = 160.0


def fused_bytes_per_brick(n, real_size):
    """Lower bound for any one-pass form of the whole flux + update: density
    row in, updated row out, key, mask and links."""
    return 2 * 64 * real_size + 8 + 8 + 4 * 2 * n


def pmc_record(workload):
    """Counter averages for one flux-B launch from the committed rocprofv3 --pmc
    runs of this workload, if they were taken on the current kernel source."""
    from paper_2508_13986_amd.profsum import kernel_source_hash
    path = os.path.join(ROOT, "profiles", f"flux_b_{workload}_pmc.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        d = json.load(fh)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d


def measured_traffic(rec, bricks_per_launch):
    """HBM bytes per flux-B launch (counter bytes per brick, scaled to this run)."""
    if rec is None or "fetch_bytes_per_launch" not in rec or "write_bytes_per_launch" not in rec:
        return None
    per_brick = (rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]) / rec["bricks_per_launch"]
    return per_brick * bricks_per_launch


# Capacity (cell slots) per workload: the L96 grids grow about 16-fold over t in [0, 1].
MAX_CELLS = {"l96_6d": 64 * 8_000_000, "l96_6d_fp32": 64 * 30_000_000}


def grid_errors(a, b, cell_volume):
    """L1 = V * sum |Pa - Pb| and max |Pa - Pb| / max Pb over the union of the two
    grids (a missing cell counts as P = 0); a and b are (idx, P) exports."""
    import numpy as np

    def packed(idx):
        bits = 63 // idx.shape[1]
        key = np.zeros(len(idx), dtype=np.int64)
        for j in range(idx.shape[1]):
            key = (key << bits) + (idx[:, j].astype(np.int64) + (1 << (bits - 1)))
        return key

    ka, kb = packed(a[0]), packed(b[0])
    keys = np.union1d(ka, kb)
    diff = np.zeros(len(keys))
    diff[np.searchsorted(keys, ka)] += a[1]
    diff[np.searchsorted(keys, kb)] -= b[1]
    return {"l1": float(cell_volume * np.abs(diff).sum()), "max_rel": float(np.abs(diff).max() / np.abs(b[1]).max()),
            "cells": [len(a[0]), len(b[0])]}


def fp32_accuracy(G, S):
    """Error of the FP32 form on the downsampled L96 grid (h = 0.5, thr 1e-5):
    against the FP64 oracle over the first 0.05 time units (8 steps, what the
    oracle finishes in under a minute), and against the FP64 GPU path over the
    whole horizon with the correction."""
    import oracle
    import numpy as np
    base = S.l96_6d_downsampled()
    c32 = S.with_(base, precision=1)
    V = float(np.prod(base["h"][:base["n"]]))
    out = {"workload": "l96_6d_downsampled: Lorenz-96 n=6, h=0.5, thr=1e-5"}
    g = G.Grid.gaussian(c32, 64 * 200_000)
    g.step(0.05)
    gi, gp, _ = g.export()
    g.close()
    o = oracle.Oracle(base).init_gaussian()
    o.step(0.05)
    oi, op = o.export()[:2]
    out["vs_fp64_oracle_t0.05"] = grid_errors((gi, gp), (oi, op), V)
    ex = []
    for c in (c32, base):
        g = G.run_scenario(c, max_cells=64 * 2_000_000)
        ex.append(g.export()[:2])
        g.close()
    out["vs_fp64_gpu_full_horizon"] = grid_errors(ex[0], ex[1], V)
    return out


def serving_bench(args):
    """The serving stream through the device pool: the same requests one at a
    time on the plain FP64 path (for the mean service time and the baseline),
    then all requests at once (burst), then Poisson arrivals at each offered
    load rho = lambda E[S] of the sweep.  With --serving-precision 1 the pool
    runs the FP32 form and reports its error against the FP64 results alone."""
    import numpy as np
    import torch

    from paper_2508_13986_amd import scenarios as S
    from paper_2508_13986_amd import serving as V

    torch.cuda.set_device(0)
    reqs, gaps = S.serving_requests(args.requests, seed=5)
    V.one_at_a_time(reqs[:1])  # warm-up: module load and first-touch of the kernels
    fp32 = args.serving_precision == 1
    alone = V.one_at_a_time(reqs, results=fp32)
    s_alone = np.array([a["seconds"] for a in alone])
    cu = float(sum(a["cell_updates"] for a in alone))
    pool_bytes = int(args.pool_gib * (1 << 30))
    preqs = [dict(r, precision=1) for r in reqs] if fp32 else reqs
    burst, mk_b = V.serve(preqs, np.zeros(len(reqs)), pool_bytes, args.max_active, group=args.group_size)
    sb = V.summarize(burst, mk_b)
    sweep = []
    for rho in args.loads:
        lam = rho / s_alone.mean()
        pois, mk_p = V.serve(preqs, gaps / lam, pool_bytes, args.max_active, group=args.group_size)
        sweep.append(dict(V.summarize(pois, mk_p), offered_load=rho, rate_per_s=lam))
        print(json.dumps({"offered_load": rho, "p50": sweep[-1]["p50_latency_s"], "p99": sweep[-1]["p99_latency_s"],
                          "cell_updates_per_s": sweep[-1]["cell_updates_per_s"]}), file=sys.stderr, flush=True)
    n3 = sum(1 for r in reqs if r["n"] == 3)
    line = {
        "metric": "serving: aggregate cell-updates/s, mixed Lorenz-63/96 request stream",
        "value": sb["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": mk_b * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64",
        "data": "synthetic (seeded request stream: priors, horizons, truth-trajectory measurements)",
        "config": {"workload": f"serving stream, seed 5: {len(reqs)} requests ({n3} Lorenz-63, {len(reqs) - n3} "
                               f"Lorenz-96 6D), horizons 0.5-2, 0-4 corrections each",
                   "max_active": args.max_active, "group_size": args.group_size or 4, "pool_gib": args.pool_gib, "parallelism": "single GPU"},
        "one_at_a_time": {"seconds": float(s_alone.sum()), "cell_updates_per_s": cu / float(s_alone.sum()),
                          "mean_service_s": float(s_alone.mean()), "p50_service_s": float(np.percentile(s_alone, 50)),
                          "p99_service_s": float(np.percentile(s_alone, 99)), "dtype": "f64"},
        "burst": sb,
        "poisson_sweep": sweep,
        "speedup_vs_one_at_a_time": sb["cell_updates_per_s"] / (cu / float(s_alone.sum())),
    }
    if fp32:
        # Error of each FP32 pool result against the same request's FP64 result
        # alone (an extra, untimed burst that copies every result out).
        with_res, _ = V.serve(preqs, np.zeros(len(reqs)), pool_bytes, args.max_active, results=True,
                              group=args.group_size)
        l1, mx = [], []
        for r, a, b in zip(reqs, with_res, alone):
            e = grid_errors(a["result"], b["result"], float(np.prod(r["h"][: r["n"]])))
            l1.append(e["l1"])
            mx.append(e["max_rel"])
        l1, mx = np.array(l1), np.array(mx)
        line["fp32_error_vs_fp64_alone"] = {
            "l1_percentiles_50_90_99_max": [float(v) for v in np.percentile(l1, [50, 90, 99, 100])],
            "max_rel_percentiles_50_90_99_max": [float(v) for v in np.percentile(mx, [50, 90, 99, 100])],
            "requests_l1_above_1e-3": int((l1 > 1e-3).sum()),
            "worst": [{"request": int(reqs[k]["request"]), "n": reqs[k]["n"], "h": reqs[k]["h"][0],
                       "thresh_rel": reqs[k]["thresh_rel"], "l1": float(l1[k])} for k in np.argsort(l1)[-3:]]}
    print(json.dumps(line), flush=True)


def run_job(G, cfg, max_cells, profile, probe=False):
    grid = G.Grid.gaussian(cfg, max_cells)
    if profile:
        grid.profile(True)
    G.run_scenario(cfg, grid=grid)
    st = grid.stats()
    prof = grid.profile_read() if profile else None
    if probe:  # hashtable probe lengths on the final grid (one sub-millisecond kernel)
        st["probes"] = grid.probe_stats(1 << 20)
    grid.close()
    return st, prof


def host_cpu():
    """The host's CPU model and logical core count (the oracle uses one thread)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "nproc": os.cpu_count()}


def cpu_baseline(budget_s):
    """The oracle, single-threaded, on the downsampled L96 6D grid (h = 0.5, thr
    1e-5): as many whole steps as fit in the time budget."""
    import oracle
    from paper_2508_13986_amd import scenarios as S

    cfg = S.l96_6d_downsampled()
    o = oracle.Oracle(cfg).init_gaussian()
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.step(cfg["t_end"], 1)
    dt = time.perf_counter() - t0
    st = o.stats()
    cpu = host_cpu()
    return {"value": st["cell_updates"] / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"L96 6D h=0.5 thr=1e-5 ({o.count()} cells), first {st['steps']} steps, "
                      f"{dt:.1f} s single-threaded", "host_cpu": cpu["model"], "host_nproc": cpu["nproc"]}


def cpu_baseline_full(c3_steps):
    """The oracle on the Lorenz '63 workload in full and on the first steps of
    the full Lorenz '96 6D benchmark grid (1.1e7 initial cells), single-threaded:
    cell-updates per second of the step loop (initialisation timed apart)."""
    import oracle
    from paper_2508_13986_amd import scenarios as S

    out = {"kind": "oracle", "cores": 1, **host_cpu()}
    for name, cfg, steps in (("l63_small", S.l63_small(), 0), ("l96_6d", S.l96_6d(), c3_steps)):
        t0 = time.perf_counter()
        o = oracle.Oracle(cfg).init_gaussian()
        t1 = time.perf_counter()
        o.step(cfg["t_end"], steps)
        t2 = time.perf_counter()
        st = o.stats()
        out[name] = {"init_s": t1 - t0, "steps": st["steps"], "step_s": t2 - t1, "cell_updates": st["cell_updates"],
                     "cell_updates_per_s": st["cell_updates"] / (t2 - t1), "cells_final": st["cells"],
                     "span": "whole horizon t in [0, 0.5]" if steps == 0 else f"first {steps} steps (per-cell-update rate)"}
        print(name, json.dumps(out[name]), flush=True)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="l96_6d")
    ap.add_argument("--max-cells", type=int, default=0, help="capacity in cell slots (default: per workload)")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the FP32-form error report")
    ap.add_argument("--requests", type=int, default=256, help="serving: requests in the stream")
    ap.add_argument("--loads", type=float, nargs="+", default=[0.5, 1.0, 2.0, 4.0, 8.0],
                    help="serving: offered loads rho = lambda * E[service] of the Poisson sweep")
    ap.add_argument("--serving-precision", type=int, default=0, help="serving: 0 FP64, 1 FP32 form in the pool")
    ap.add_argument("--max-active", type=int, default=96, help="serving: requests running at once")
    ap.add_argument("--pool-gib", type=float, default=160.0, help="serving: arena of the pool")
    ap.add_argument("--group-size", type=int, default=8, help="serving: requests stepped together (0: the pool's 4)")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-baseline-full", type=int, default=0, metavar="STEPS",
                    help="only time the oracle: Lorenz-63 workload in full and the first STEPS steps of the full "
                         "Lorenz-96 grid; prints one JSON line")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run one plain device copy of this many bytes (for counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print("bench.py runs on one GPU only: there is no multi-GPU path (requests or Morton ranges would be sharded; not implemented)",
              file=sys.stderr)
        sys.exit(2)

    if args.cpu_baseline_full:
        print(json.dumps(cpu_baseline_full(args.cpu_baseline_full)), flush=True)
        return

    if args.workload == "serving":
        serving_bench(args)
        return

    import torch

    from paper_2508_13986_amd import gbees as G
    from paper_2508_13986_amd import scenarios as S

    torch.cuda.set_device(0)
    cfg = S.workload(args.workload)
    n = cfg["n"]
    real_size = 4 if cfg.get("precision", 0) == 1 else 8
    if not args.max_cells:
        args.max_cells = MAX_CELLS.get(args.workload, 64 * 8_000_000)

    if args.calibrate_copy:  # a plain copy of known size, to scale the HBM byte counters by
        src = torch.ones(args.calibrate_copy, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        torch.cuda.empty_cache()

    for _ in range(args.warmup):
        run_job(G, cfg, args.max_cells, profile=False)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    totals = {"cell_updates": 0, "brick_updates": 0, "steps": 0, "grow_bricks": 0, "inserted": 0}
    prof_sum = {}
    last = None
    for k in range(args.steps):
        st, prof = run_job(G, cfg, args.max_cells, profile=True, probe=(k == args.steps - 1))
        for k in totals:
            totals[k] += st[k]
        for k, (ms, cnt) in prof.items():
            a = prof_sum.setdefault(k, [0.0, 0])
            a[0] += ms
            a[1] += cnt
        last = st
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    value = totals["cell_updates"] / elapsed
    fb_ms, fb_n = prof_sum["flux_b"]
    fa_ms, fa_n = prof_sum["flux_a"]
    bricks_per_launch = totals["brick_updates"] / max(fb_n, 1)
    avg_b = fb_ms / 1e3 / max(fb_n, 1)
    avg_a = fa_ms / 1e3 / max(fa_n, 1)
    bytes_b = flux_b_bytes_per_brick(n, real_size) * bricks_per_launch
    bytes_a = flux_a_bytes_per_brick(n, real_size) * bricks_per_launch
    rec = pmc_record(args.workload)
    traffic = measured_traffic(rec, bricks_per_launch)
    valu_busy = rec.get("derived", {}).get("valu_busy_pct") if rec else None
    cells_per_step = totals["cell_updates"] / max(totals["steps"], 1)
    # The method's bytes: per cell-update, for the cells one launch updates.
    alg_per_launch = alg_bytes_per_cell_update(n, real_size) * cells_per_step
    achieved = alg_per_launch / avg_b / 1e9
    line = {
        "metric": "CTU cell-updates/s (Lorenz-96 6D)",
        "value": value,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if real_size == 4 else "f64",
        "data": "synthetic (seeded Gaussian initial pdf and seeded truth-trajectory measurement)",
        "config": {
            "workload": f"{args.workload}: Lorenz-96 n={n} F=4, h={cfg['h'][0]}, thr={cfg['thresh_rel']}, "
                        f"CFL {cfg['cfl']}, MC limiter, prune every {cfg['prune_every']}, t in [0,{cfg['t_end']}], "
                        f"{len(cfg['measurements'])} correction(s)",
            "steps_per_job": totals["steps"] // args.steps,
            "cells_per_step_mean": cells_per_step,
            "cells_final": last["cells"],
            "bricks_per_step_mean": bricks_per_launch,
            "brick_occupancy": cells_per_step / (64 * bricks_per_launch),
            "grow_bricks_per_step": totals["grow_bricks"] / max(totals["steps"], 1),
            "cells_inserted_per_step": totals["inserted"] / max(totals["steps"], 1),
            "hash_probes_final_grid": last.get("probes"),
            "parallelism": "single GPU",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": f"k_flux_b<{n},{'float' if real_size == 4 else 'double'}>",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "basis": f"{alg_bytes_per_cell_update(n, real_size)} B per cell-update x cells per launch",
            "valu_busy_pct": valu_busy,
            "avg_launch_us": avg_b * 1e6,
            "algorithmic_bytes_per_launch": alg_per_launch,
        },
        # The whole flux + update step (both passes) against the same bytes.
        "flux_step_roofline": {
            "achieved": alg_per_launch / (avg_a + avg_b) / 1e9,
            "frac": alg_per_launch / (avg_a + avg_b) / 1e9 / HBM_PEAK_GBPS,
            "ms_per_step": (avg_a + avg_b) * 1e3,
        },
        "end_to_end_roofline": {
            "achieved": value * WHOLE_STEP_BYTES_6D_FP64 / 1e9 if (n == 6 and real_size == 8) else None,
            "frac": value * WHOLE_STEP_BYTES_6D_FP64 / 1e9 / HBM_PEAK_GBPS if (n == 6 and real_size == 8) else None,
            "basis": f"{WHOLE_STEP_BYTES_6D_FP64:.0f} B per 6-D FP64 cell-update (flux, grow check, prune every 20)",
        },
        "phases_ms_per_job": {k: v[0] / args.steps for k, v in prof_sum.items()},
        "flux_passes_cell_updates_per_s": cells_per_step / (avg_a + avg_b),
        # Per-kernel diagnostics on the brick-slot basis (every lane of every
        # swept brick, plus the corrected-state face layers of the two-pass form).
        "slot_basis": {
            "flux_b_bytes_per_brick": flux_b_bytes_per_brick(n, real_size),
            "flux_b_gbps": bytes_b / avg_b / 1e9,
            "flux_a_gbps": bytes_a / avg_a / 1e9,
            "fused_bound_bytes_per_brick": fused_bytes_per_brick(n, real_size),
            "fused_bound_frac": fused_bytes_per_brick(n, real_size) * bricks_per_launch / (avg_a + avg_b) / 1e9 / HBM_PEAK_GBPS,
        },
    }
    if real_size == 4 and not args.no_accuracy:
        line["accuracy"] = fp32_accuracy(G, S)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_budget)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
