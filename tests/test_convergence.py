"""Convergence study (Sec. 5.2.2, Eq. 10, Figs. 7-8): the E / BC metrics on
known grids (CPU), and convergence of the GPU path as the time step and the
cell width shrink (GPU)."""
import numpy as np
import pytest

from paper_2508_13986_amd import convergence as C
from paper_2508_13986_amd import scenarios as S


def test_metrics_same_lattice():
    idx = np.array([[0, 0, 0], [1, 0, 0], [0, -1, 2]])
    P = np.array([1.0, 2.0, 3.0])
    h = [0.5] * 3
    E, BC = C.compare((idx, P), (idx, P), h, h)
    assert E == 0.0 and BC == pytest.approx(0.125 * 6.0)
    # disjoint supports: E is the sum of both masses, BC is 0
    other = np.array([[5, 5, 5]])
    E, BC = C.compare((idx, P), (other, np.array([4.0])), h, h)
    assert E == pytest.approx(0.125 * 10.0) and BC == 0.0
    # symmetric in its arguments on one lattice
    a = C.compare((idx, P), (idx[:2], np.array([1.5, 1.0])), h, h)
    b = C.compare((idx[:2], np.array([1.5, 1.0])), (idx, P), h, h)
    assert a[0] == pytest.approx(b[0]) and a[1] == pytest.approx(b[1])


def test_metrics_across_lattices():
    """A density constant on coarse cells equals its own refinement (E = 0,
    BC = mass); the coarse cell of width 1 holds the fine centres at -0.5 and
    0 of the 0.5 lattice, not the one at +0.5 (cells are half-open)."""
    pts = C._covered_reference_points(np.array([[0]]), np.array([1.0]), np.array([0.5]))
    assert sorted(pts[:, 0].tolist()) == [-1, 0]
    rng = np.random.default_rng(1)
    coarse = np.array([[i, j] for i in range(-2, 3) for j in range(-1, 2)])
    Pc = rng.uniform(0.1, 1.0, len(coarse))
    fine, Pf = [], []
    for (i, j), p in zip(coarse, Pc):
        for a in (2 * i - 1, 2 * i):
            for b in (2 * j - 1, 2 * j):
                fine.append((a, b))
                Pf.append(p)
    E, BC = C.compare((coarse, Pc), (np.array(fine), np.array(Pf)), [1.0, 1.0], [0.5, 0.5])
    assert E == pytest.approx(0.0, abs=1e-15)
    assert BC == pytest.approx(0.25 * np.sum(Pf))
    # cells 0..2 of width 1.25 span [-0.625, 3.125): fine centres -0.5 .. 3.0
    pts = C._covered_reference_points(np.array([[0], [1], [2]]), np.array([1.25]), np.array([0.5]))
    assert sorted(pts[:, 0].tolist()) == list(range(-1, 7))


@pytest.fixture(scope="module")
def gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2508_13986_amd import gbees

    gbees.lib()
    return True


@pytest.mark.gpu
def test_temporal_convergence(gpu):
    """E shrinks and BC grows toward 1 as the Courant number falls (reference C = 0.05)."""
    res = C.study("eps", [1.0, 0.5, 0.2], 0.05, h_star=0.5, t_end=0.5)
    E = [res[f][-1][1] for f in (1.0, 0.5, 0.2)]
    BC = [res[f][-1][2] for f in (1.0, 0.5, 0.2)]
    assert E[0] > E[1] > E[2] > 0.0
    assert BC[0] < BC[1] < BC[2] <= 1.0 + 1e-12


@pytest.mark.gpu
def test_spatial_convergence(gpu):
    """E shrinks as the cell width falls toward the reference (eta = 0.5 of h* = 0.5, C = 0.1)."""
    res = C.study("eta", [1.25, 1.0, 0.8], 0.5, h_star=0.5, t_end=0.5)
    E = [res[f][-1][1] for f in (1.25, 1.0, 0.8)]
    assert E[0] > E[1] > E[2] > 0.0


@pytest.mark.gpu
def test_study_metrics_match_oracle(gpu):
    """E and BC between two Courant numbers, from GPU runs and from oracle
    runs of the same configurations, agree: the study's numbers are the
    method's, not an artefact of the GPU path."""
    import oracle
    from paper_2508_13986_amd import gbees as G

    base = S.with_(S.workload("l63_small"), t_end=0.05)
    gpu_runs, orc_runs = {}, {}
    for cfl in (0.9, 0.45):
        cfg = S.with_(base, cfl=cfl)
        g = G.Grid.gaussian(cfg, 1 << 20)
        g.step(cfg["t_end"])
        gi, gp, _ = g.export()
        g.close()
        orc = oracle.Oracle(cfg)
        orc.init_gaussian()
        orc.step(cfg["t_end"])
        gpu_runs[cfl] = (gi, gp)
        orc_runs[cfl] = orc.export()
    h = base["h"]
    Eg, BCg = C.compare(gpu_runs[0.9], gpu_runs[0.45], h, h)
    Eo, BCo = C.compare(orc_runs[0.9], orc_runs[0.45], h, h)
    assert Eo > 0.0
    assert Eg == pytest.approx(Eo, rel=1e-6)
    assert BCg == pytest.approx(BCo, rel=1e-9)
