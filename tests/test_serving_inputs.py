"""The serving request stream (CPU): seeded, and shaped as the serving workload
states: both models, grid sizes from ~1e3 to ~2e6 cells, horizons in [0.5, 2],
0..4 measurements inside the horizon."""
import numpy as np

from paper_2508_13986_amd import scenarios as S


def test_stream_is_seeded_and_shaped():
    a, ta = S.serving_requests(64, seed=5)
    b, tb = S.serving_requests(64, seed=5)
    assert np.array_equal(ta, tb)
    assert [r["measurements"] for r in a] == [r["measurements"] for r in b]
    assert ta[0] == 0.0 and np.all(np.diff(ta) >= 0)
    ns = [r["n"] for r in a]
    assert 20 < ns.count(3) < 44 and ns.count(3) + ns.count(6) == 64
    for r in a:
        T = r["t_end"]
        assert 0.5 <= T <= 2.0
        assert 0 <= len(r["measurements"]) <= 4
        times = [m[0] for m in r["measurements"]]
        assert times == sorted(times) and all(0.0 <= t <= T for t in times)
        assert all(0 <= m[1] < r["n"] for m in r["measurements"])
        assert r["h"][0] in ((0.5, 0.25) if r["n"] == 3 else (0.3, 0.25))
        assert r["thresh_rel"] == (1e-5 if r["n"] == 3 else 1e-2)
        assert 4e2 < S.initial_cells_estimate(r) < 2.2e6


def test_initial_size_estimate_matches_a_lattice_count():
    """The volume estimate against a brute-force count of the init ellipsoid."""
    r = S.l63_small()
    n, h = r["n"], np.asarray(r["h"][:3])
    cov = np.asarray(r["cov"])
    R = int(np.ceil(np.sqrt(2 * np.log(1 / r["thresh_rel"]) * cov.diagonal().max()) / h.min())) + 1
    g = np.stack(np.meshgrid(*([np.arange(-R, R + 1)] * n), indexing="ij"), -1).reshape(-1, n) * h
    q = np.einsum("ij,jk,ik->i", g, np.linalg.inv(cov), g)
    count = int((q <= 2 * np.log(1 / r["thresh_rel"])).sum())
    assert count == 3743
    assert abs(S.initial_cells_estimate(r) / count - 1) < 0.05
