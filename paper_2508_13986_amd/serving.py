"""Serving driver: a stream of propagation requests through the device pool.

The pool (gbees_pool_* in the C ABI) does the work: it admits requests as
arena memory and slots free up and runs them concurrently on the GPU.  This
module only generates the request stream (``scenarios.serving_requests``),
submits each request at its arrival time, calls ``Pool.progress`` in a loop
and records latencies.  ``one_at_a_time`` runs the same requests through the
plain FP64 path (``Grid``), one after the other, for comparison.
"""
import math
import time

import numpy as np

from . import gbees as G
from . import scenarios as S

# Capacity per request: growth over the initial cells, and a floor (cells).
# Lorenz '96 grids at thr 1e-2 spread along the unstable directions: measured
# growth from 0.4x to 240x over the horizons of the stream, up to 8.3e6 cells.
GROWTH = {3: 16.0, 6: 24.0}
FLOOR = {3: 2.5e5, 6: 8.0e6}


def capacity_for(cfg, factor=1.0):
    """Cell slots for one request, in bricks at 40% occupancy."""
    cells = max(S.initial_cells_estimate(cfg) * GROWTH[cfg["n"]], FLOOR[cfg["n"]]) * factor
    return 64 * int(math.ceil(cells / (64 * 0.4)))


def one_at_a_time(reqs, results=False):
    """Each request alone through the synchronous FP64 path; per-request seconds."""
    import torch

    out = []
    for cfg in reqs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        factor = 1.0
        while True:
            try:
                g = G.run_scenario(cfg, max_cells=capacity_for(cfg, factor))
                break
            except G.GbeesError as e:
                if e.code != G.E_CAPACITY:
                    raise
                factor *= 4.0
        torch.cuda.synchronize()
        st = g.stats()
        rec = {"seconds": time.perf_counter() - t0, "cell_updates": st["cell_updates"], "cells": st["cells"],
               "steps": st["steps"], "retries": int(round(math.log(factor, 4)))}
        if results:
            rec["result"] = g.export()[:2]
        g.close()
        out.append(rec)
    return out


def serve(reqs, arrivals, pool_bytes, max_active=16, results=False, spin=2e-4, group=0):
    """Submit request k at time arrivals[k] (seconds from start) and drive the
    pool until every request has finished.  A request that outgrows its
    capacity continues in a larger arena slice inside the pool; only if no
    such slice is free does it fail, and it is then resubmitted with four
    times the capacity, keeping its arrival time.  group > 0 sets the number
    of requests stepped together by one driver (the pool's default otherwise)."""
    pool = G.Pool(pool_bytes, max_active)
    if group > 0:
        pool.group_size(group)
    order = np.argsort(arrivals, kind="stable")
    t0 = pool.clock()
    nxt, live, done = 0, {}, {}
    factor = {}
    while len(done) < len(reqs):
        now = pool.clock() - t0
        while nxt < len(order) and arrivals[order[nxt]] <= now:
            k = int(order[nxt])
            factor[k] = 1.0
            live[pool.submit(reqs[k], capacity_for(reqs[k]))] = k
            nxt += 1
        pool.progress()
        for rid in list(live):
            inf = pool.info(rid)
            if inf["status"] == 2 or inf["status"] < 0:
                k = live.pop(rid)
                if inf["status"] == G.E_CAPACITY:
                    factor[k] *= 4.0
                    live[pool.submit(reqs[k], capacity_for(reqs[k], factor[k]))] = k
                elif inf["status"] < 0:
                    raise G.GbeesError(inf["status"], f"request {k}")
                else:
                    rec = {"latency": inf["t_done"] - t0 - arrivals[k], "queued": inf["t_admit"] - t0 - arrivals[k],
                           "cell_updates": inf["stats"]["cell_updates"], "cells": inf["cells"],
                           "arena_bytes": inf["arena_bytes"], "retries": int(round(math.log(factor[k], 4))),
                           "resizes": inf["resizes"]}
                    if results:
                        rec["result"] = pool.result(rid)
                    done[k] = rec
                pool.release(rid)
        if spin:
            time.sleep(spin)
    makespan = pool.clock() - t0
    pool.close()
    return [done[k] for k in range(len(reqs))], makespan


def summarize(recs, makespan):
    lat = np.array([r["latency"] for r in recs])
    cu = float(sum(r["cell_updates"] for r in recs))
    return {"requests": len(recs), "makespan_s": makespan, "cell_updates": cu, "cell_updates_per_s": cu / makespan,
            "p50_latency_s": float(np.percentile(lat, 50)), "p99_latency_s": float(np.percentile(lat, 99)),
            "mean_queued_s": float(np.mean([r["queued"] for r in recs])),
            "retries": int(sum(r["retries"] for r in recs)),
            "resized_in_pool": int(sum(1 for r in recs if r.get("resizes", 0) > 0))}
