"""Serving pool (gbees_pool_*): results in the mix equal results alone and the
oracle's (stored oracle runs of the same requests, tests/golden/serving_req*),
admission by arena footprint, growth past a request's capacity, and the error
paths.  Runs on the GPU through the C ABI."""
import numpy as np
import pytest

from paper_2508_13986_amd import scenarios as S

import _golden

pytestmark = pytest.mark.gpu

TOL = 1e-12


def oracle_check(res, info, r, label):
    """An FP64 pool result against the oracle's run of the same request."""
    snap = _golden.load(f"serving_req{r['request']}")["snapshots"][-1]
    idx, P = res
    _golden.check(idx, P, info["stats"]["t"], snap, r["thresh_rel"], label=f"{label} vs oracle")


def oracle_check_fp32(res, r, label):
    """An FP32 pool result against the FP64 oracle: cell count within 2% and
    sampled densities within 1e-2 of max P (single-precision rounding and the
    threshold decisions it moves; the FP64 path meets 1e-12)."""
    snap = _golden.load(f"serving_req{r['request']}")["snapshots"][-1]
    idx, P = res
    assert abs(len(idx) - snap["cells"]) <= 0.02 * snap["cells"], (label, len(idx), snap["cells"])
    keys = _golden._packed(idx)
    sk = _golden._packed(np.asarray(snap["sample_idx"]))
    pos = np.minimum(np.searchsorted(keys, sk), len(keys) - 1)
    got = np.where(keys[pos] == sk, P[pos], 0.0)
    err = np.abs(got - np.asarray(snap["sample_p"])).max() / snap["max_p"]
    print(f"[{label}] fp32 vs fp64 oracle: cells {len(idx)} / {snap['cells']}, sampled max err {err:.3g}", flush=True)
    assert err <= 1e-2, (label, err)


@pytest.fixture(scope="module")
def G():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2508_13986_amd import gbees

    gbees.lib()
    return gbees


# Requests of the serving stream (seed 5) used below, with stored oracle runs
# (tests/golden/make_golden.py): Lorenz-63 ones, and two Lorenz-96 6D ones cut
# to a horizon of 0.3, where their grids stay small enough for the oracle.
MIXED = (1, 41, 2, 52, 4, 8)


def requests(ids):
    reqs, _ = S.serving_requests(64)
    by_id = {r["request"]: r for r in reqs}
    out = []
    for k in ids:
        r = dict(by_id[k])
        if r["n"] == 6:
            r["t_end"] = min(r["t_end"], 0.3)
            r["measurements"] = [m for m in r["measurements"] if m[0] <= r["t_end"]]
        out.append(r)
    return out


def cap(r):
    return 64 * (200_000 if r["n"] == 6 else 8_000)


def alone(G, r):
    g = G.run_scenario(r, max_cells=cap(r))
    res = g.export()[:2]
    g.close()
    return res


def assert_same(a, b, label):
    (ai, ap), (bi, bp) = a, b
    assert len(ai) == len(bi) and np.array_equal(ai, bi), f"{label}: membership differs"
    assert np.abs(ap - bp).max() <= TOL * np.abs(bp).max(), label


def drain(pool, ids, max_seconds=120.0):
    """Drive the pool until every request ended; fetch each finished grid at
    once (which frees its arena slice).  Returns {id: (info, result or None)}."""
    import time

    done = {}
    t0 = time.monotonic()
    while len(done) < len(ids):
        pool.progress()
        for rid in ids:
            if rid not in done:
                inf = pool.info(rid)
                if inf["status"] == 2:
                    done[rid] = (inf, pool.result(rid))
                elif inf["status"] < 0:
                    done[rid] = (inf, None)
        assert time.monotonic() - t0 < max_seconds, "pool did not drain"
    return done


def test_pool_results_equal_alone(G):
    """Six requests of both models in a burst through three slots: each result
    equals the same request run alone through the plain path."""
    reqs = requests(MIXED)
    assert {r["n"] for r in reqs} == {3, 6}
    ref = [alone(G, r) for r in reqs]
    pool = G.Pool(sum(G.arena_bytes(r, cap(r)) for r in reqs) + (1 << 20), max_active=3)
    ids = [pool.submit(r, cap(r)) for r in reqs]
    out = drain(pool, ids)
    running = sorted((i["t_admit"], i["t_done"]) for i, _ in out.values())
    for k, (rid, r) in enumerate(zip(ids, reqs)):
        assert out[rid][0]["status"] == 2
        assert_same(out[rid][1], ref[k], f"request {k}")
        oracle_check(out[rid][1], out[rid][0], r, f"request {r['request']}")
        pool.release(rid)
    # never more than three at once
    for t, _ in running:
        assert sum(1 for a, b in running if a <= t < b) <= 3
    pool.close()


def test_pool_group_of_eight_equal_alone(G):
    """Eight Lorenz-63 requests (different cell sizes, horizons and
    measurements) stepped together by one driver with shared launches (group
    size 8): each result equals the request run alone, and the oracle's."""
    reqs, _ = S.serving_requests(64)
    reqs = [r for r in reqs if r["n"] == 3][:8]
    assert len(reqs) == 8 and len({(r["h"][0], r["t_end"]) for r in reqs}) > 1
    ref = [alone(G, r) for r in reqs]
    pool = G.Pool(sum(G.arena_bytes(r, cap(r)) for r in reqs) + (1 << 20), max_active=8)
    pool.group_size(8)
    ids = [pool.submit(r, cap(r)) for r in reqs]
    out = drain(pool, ids)
    for k, rid in enumerate(ids):
        assert out[rid][0]["status"] == 2
        assert_same(out[rid][1], ref[k], f"request {k}")
        oracle_check(out[rid][1], out[rid][0], reqs[k], f"request {reqs[k]['request']}")
        pool.release(rid)
    pool.close()


def test_pool_request_outgrowing_its_capacity_resumes(G):
    """A request whose grid outgrows its capacity mid-run is rolled back to the
    start of the failing step and continues in a larger arena slice
    (gbees_resize): its result equals the request run alone with ample capacity
    and the oracle's."""
    reqs, _ = S.serving_requests(64)
    r = [q for q in reqs if q["request"] == 2][0]
    probe = G.Grid.gaussian(r, max_cells=cap(r))
    b0 = probe.stats()["bricks"]
    probe.close()
    tight = 64 * (b0 + 4)
    pool = G.Pool(G.arena_bytes(r, tight) + 8 * G.arena_bytes(r, 4 * tight), max_active=2)
    rid = pool.submit(r, tight)
    out = drain(pool, [rid])
    inf, res = out[rid]
    assert inf["status"] == 2 and inf["resizes"] >= 1, inf
    assert_same(res, alone(G, r), "resumed request")
    oracle_check(res, inf, r, "resumed request")
    pool.release(rid)
    pool.close()


def test_pool_fp32_group_equal_alone(G):
    """The FP32 form through shared launches: three Lorenz-63 requests with
    FP32 densities in one group give the FP32 path's result alone."""
    reqs, _ = S.serving_requests(64)
    reqs = [dict(r, precision=1) for r in reqs if r["n"] == 3][:3]
    ref = [alone(G, r) for r in reqs]
    pool = G.Pool(sum(G.arena_bytes(r, cap(r)) for r in reqs) + (1 << 20), max_active=3)
    ids = [pool.submit(r, cap(r)) for r in reqs]
    out = drain(pool, ids)
    for k, rid in enumerate(ids):
        assert out[rid][0]["status"] == 2
        assert_same(out[rid][1], ref[k], f"fp32 request {k}")
        oracle_check_fp32(out[rid][1], reqs[k], f"fp32 request {reqs[k]['request']}")
        pool.release(rid)
    pool.close()


def test_pool_admits_by_footprint(G):
    """An arena that holds one request at a time: requests run one after the
    other even with free slots, and their results are unchanged."""
    reqs = requests((1, 2, 4))
    sizes = [G.arena_bytes(r, cap(r)) for r in reqs]
    assert len(reqs) == 3 and len(set(sizes)) == 1
    pool = G.Pool(sizes[0] + 4096, max_active=4)
    ids = [pool.submit(r, cap(r)) for r in reqs]
    out = drain(pool, ids)
    spans = sorted((out[i][0]["t_admit"], out[i][0]["t_done"]) for i in ids)
    for (a0, b0), (a1, b1) in zip(spans, spans[1:]):
        assert a1 >= b0
    for rid, r in zip(ids, reqs):
        assert_same(out[rid][1], alone(G, r), "serial")
        oracle_check(out[rid][1], out[rid][0], r, f"serial request {r['request']}")
        pool.release(rid)
    pool.close()


def test_pool_group_survives_a_failing_member(G):
    """A group member whose grid does not fit its capacity (here already the
    initial grid) fails alone: the other members of its group finish with the
    results they get alone."""
    reqs, _ = S.serving_requests(64)
    reqs = [r for r in reqs if r["n"] == 3][:3]
    caps = [cap(reqs[0]), 64 * 16, cap(reqs[2])]  # the middle one outgrows 16 bricks
    ref = {0: alone(G, reqs[0]), 2: alone(G, reqs[2])}
    pool = G.Pool(sum(G.arena_bytes(r, c) for r, c in zip(reqs, caps)) + (1 << 20), max_active=3)
    ids = [pool.submit(r, c) for r, c in zip(reqs, caps)]
    out = drain(pool, ids)
    assert out[ids[1]][0]["status"] == G.E_CAPACITY
    for k in (0, 2):
        assert out[ids[k]][0]["status"] == 2
        assert_same(out[ids[k]][1], ref[k], f"request {k}")
        oracle_check(out[ids[k]][1], out[ids[k]][0], reqs[k], f"request {reqs[k]['request']}")
    for rid in ids:
        pool.release(rid)
    pool.close()


def test_pool_error_paths(G):
    r = requests((2,))[0]
    pool = G.Pool(G.arena_bytes(r, cap(r)) + 4096, max_active=2)
    with pytest.raises(G.GbeesError) as e:
        pool.submit(r, cap(r) * 64)  # footprint beyond the whole arena
    assert e.value.code == G.E_CAPACITY
    bad = pool.submit(r, 64 * 16)  # outgrows 16 bricks
    out = drain(pool, [bad])
    assert out[bad][0]["status"] == G.E_CAPACITY
    with pytest.raises(G.GbeesError) as e:
        pool.result(bad)
    assert e.value.code == G.E_CAPACITY
    pool.release(bad)
    ok = pool.submit(r, cap(r))  # the slice came back: the pool still serves
    out = drain(pool, [ok])
    assert out[ok][0]["status"] == 2
    assert_same(out[ok][1], alone(G, r), "after failure")
    oracle_check(out[ok][1], out[ok][0], r, f"request {r['request']} after failure")
    pool.close()
