"""Seeded synthetic workloads for the GBEES hot path (inputs only).

This module generates the inputs both the GPU library and the CPU oracle are
run on: model/grid configurations and measurement sequences.  It contains none
of the propagation method's arithmetic; the only dynamics here is a fixed-step
RK4 "truth" trajectory used to synthesise measurement values, as the paper does
with its seeded truth runs (Sec. 5.1.1: a measurement y = x_c + noise at the
correction time).

Every workload is a plain dict with the fields

    n, model, params, h, mean, cov, thresh_rel, cfl, dt_fixed, prune_every,
    limiter, grow_mode, precision, max_cells, t_end, measurements

where ``measurements`` is a list of (t, component, y, sigma) tuples sorted by t.
Model ids: 1 Lorenz '63, 2 Lorenz '96, 3 linear f = A x + b, 4 uniform f = b.
"""
import copy
import math

import numpy as np

L63, L96, LINEAR, UNIFORM = 1, 2, 3, 4


def _base(n, model, params, h, mean, cov, thresh_rel, t_end, **kw):
    d = dict(n=n, model=model, params=list(params), h=[float(h)] * n if np.isscalar(h) else list(h),
             mean=list(mean), cov=np.asarray(cov, dtype=np.float64).reshape(n, n).tolist(),
             thresh_rel=thresh_rel, cfl=0.9, dt_fixed=0.0, prune_every=20, limiter=1,
             grow_mode=0, precision=0, max_cells=0, t_end=t_end, measurements=[])
    d.update(kw)
    return d


def lorenz63(sigma=10.0, rho=28.0, beta=8.0 / 3.0, z_shift=0.0):
    return [sigma, rho, beta, z_shift]


def lorenz96(F=4.0):
    return [F]


# ---------------------------------------------------------------------------
# Named workloads.  Lorenz '63 in standard form with (10, 28, 8/3); Lorenz '96
# with n = 6 and F = 4 (Sec. 5.1.2).  Sizes and thresholds as in the workload
# table of the design notes.
# ---------------------------------------------------------------------------

def l63_small():
    """Lorenz '63, h = 0.5, thr 1e-5, t in [0, 0.5], no measurements (3743 initial cells)."""
    return _base(3, L63, lorenz63(), 0.5, [-11.5, -10.0, 9.5], np.eye(3), 1e-5, 0.5)


def l63_corrections(seed=2):
    """Lorenz '63, h = 0.25, cov 2 I, thr 1e-6, t in [0, 2], corrections on x1 every 0.25."""
    d = _base(3, L63, lorenz63(), 0.25, [-11.5, -10.0, 9.5], 2.0 * np.eye(3), 1e-6, 2.0)
    d["measurements"] = truth_measurements(d, [0.25 * k for k in range(1, 9)], comp=0, sigma=1.0, seed=seed)
    return d


def l96_6d(h=0.25, thresh_rel=1e-7, seed=3, precision=0):
    """Lorenz '96 6D, F = 4, mean (4.5, 4, ..., 4), cov 0.25 I, t in [0, 1], one x1 correction at 0.5."""
    d = _base(6, L96, lorenz96(4.0), h, [4.5, 4.0, 4.0, 4.0, 4.0, 4.0], 0.25 * np.eye(6), thresh_rel, 1.0,
              precision=precision)
    d["measurements"] = truth_measurements(d, [0.5], comp=0, sigma=0.5, seed=seed)
    return d


def l96_6d_fp32(seed=3):
    """The precision form: the same problem at h = 0.2 with FP32 densities."""
    return l96_6d(h=0.2, thresh_rel=1e-7, seed=seed, precision=1)


def l96_6d_downsampled(seed=3):
    """L96 6D at h = 0.5, thr 1e-5: the size the oracle runs over the full horizon."""
    return l96_6d(h=0.5, thresh_rel=1e-5, seed=seed)


def l63_paper(thresh_rel=1e-5):
    """The paper's Lorenz '63 case (Sec. 5.1.1): (sigma, b, r) = (4, 1, 48) in
    its shifted form (standard form with rho = r and z_shift = r), mean
    (-11.5, -10, 9.5), unit variances, h = 0.5, a measurement y = x3 = -8 with
    sigma_y = 1 at t = 1, horizon 2, time step 1.0 x CFL (Table 2).  The
    threshold is not stated (read as 1e-5)."""
    d = _base(3, L63, lorenz63(sigma=4.0, rho=48.0, beta=1.0, z_shift=48.0), 0.5, [-11.5, -10.0, 9.5],
              np.eye(3), thresh_rel, 2.0, cfl=1.0)
    d["measurements"] = [(1.0, 2, -8.0, 1.0)]
    return d


def l96_paper(thresh_rel=1e-4, h=0.1):
    """The paper's Lorenz '96 case (Sec. 5.1.2): n = 6, F = 4, mean
    (F + 0.5, F, ..., F), standard deviation 0.2, h = 0.1 (half the standard
    deviation, Table 2), horizon 1.3, no measurement, time step 1.0 x CFL.  The
    threshold is not stated; 1e-4 gives about the largest grid Table 2 reports
    (about 5e7 cells), where 1e-5 gives several times more."""
    return _base(6, L96, lorenz96(4.0), h, [4.5, 4.0, 4.0, 4.0, 4.0, 4.0], 0.04 * np.eye(6), thresh_rel, 1.3,
                 cfl=1.0)


WORKLOADS = {
    "l63_small": l63_small,
    "l63_corrections": l63_corrections,
    "l96_6d": l96_6d,
    "l96_6d_fp32": l96_6d_fp32,
    "l96_6d_downsampled": l96_6d_downsampled,
    "l63_paper": l63_paper,
    "l96_paper": l96_paper,
}


def workload(name, **overrides):
    d = WORKLOADS[name]()
    d = copy.deepcopy(d)
    d.update(overrides)
    return d


def with_(cfg, **overrides):
    d = copy.deepcopy(cfg)
    d.update(overrides)
    return d


# ---------------------------------------------------------------------------
# Measurement synthesis: x0 = mean + L z (Cholesky L of cov, z ~ N(0, I) from a
# PCG64 generator with the given seed), truth by RK4 with a fixed 1e-4 step,
# y_k = x_comp(t_k) + sigma * eps_k with eps drawn from the same generator.
# ---------------------------------------------------------------------------

def _truth_drift(cfg, x):
    n, p = cfg["n"], cfg["params"]
    if cfg["model"] == L63:
        z = x[2] + p[3]
        return np.array([p[0] * (x[1] - x[0]), x[0] * (p[1] - z) - x[1], x[0] * x[1] - p[2] * z])
    if cfg["model"] == L96:
        return np.array([(x[(j + 1) % n] - x[(j - 2) % n]) * x[(j - 1) % n] - x[j] + p[0] for j in range(n)])
    if cfg["model"] == LINEAR:
        A = np.asarray(p[: n * n]).reshape(n, n)
        return A @ x + np.asarray(p[n * n: n * n + n])
    return np.asarray(p[:n], dtype=np.float64)


def truth_trajectory(cfg, times, seed, dt=1e-4):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = cfg["n"]
    L = np.linalg.cholesky(np.asarray(cfg["cov"], dtype=np.float64))
    x = np.asarray(cfg["mean"], dtype=np.float64) + L @ rng.standard_normal(n)
    out, t = [], 0.0
    for tk in times:
        steps = int(round((tk - t) / dt))
        for _ in range(steps):
            k1 = _truth_drift(cfg, x)
            k2 = _truth_drift(cfg, x + 0.5 * dt * k1)
            k3 = _truth_drift(cfg, x + 0.5 * dt * k2)
            k4 = _truth_drift(cfg, x + dt * k3)
            x = x + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        t = tk
        out.append(x.copy())
    return np.array(out), rng


def truth_measurements(cfg, times, comp, sigma, seed):
    xs, rng = truth_trajectory(cfg, times, seed)
    eps = rng.standard_normal(len(times))
    return [(float(t), int(comp), float(x[comp] + sigma * e), float(sigma)) for t, x, e in zip(times, xs, eps)]


# ---------------------------------------------------------------------------
# Small seeded inputs for tests: random cell sets and densities.
# ---------------------------------------------------------------------------

def random_blob(n, radius, seed, density=0.7):
    """A seeded random set of cells inside a box of the given radius with positive densities."""
    rng = np.random.Generator(np.random.PCG64(seed))
    grid = np.stack(np.meshgrid(*([np.arange(-radius, radius + 1)] * n), indexing="ij"), -1).reshape(-1, n)
    keep = rng.random(len(grid)) < density
    idx = grid[keep].astype(np.int32)
    p = rng.random(len(idx)) + 0.05
    return idx, p


def random_linear(n, seed, scale=1.0, offset=None):
    """A seeded linear drift f = A x + b with a stable A."""
    rng = np.random.Generator(np.random.PCG64(seed))
    A = scale * (rng.standard_normal((n, n)) * 0.5 - np.eye(n))
    b = rng.standard_normal(n) if offset is None else np.asarray(offset, dtype=np.float64)
    return list(A.reshape(-1)) + list(b)


def linear_config(n, A_b, h=1.0, mean=None, thresh_rel=0.0, **kw):
    mean = [0.0] * n if mean is None else mean
    cov = kw.pop("cov", np.eye(n))
    return _base(n, LINEAR, A_b, h, mean, cov, thresh_rel, 1.0, **kw)


def uniform_config(n, u, h=1.0, mean=None, thresh_rel=0.0, **kw):
    mean = [0.0] * n if mean is None else mean
    cov = kw.pop("cov", np.eye(n))
    return _base(n, UNIFORM, list(u), h, mean, cov, thresh_rel, 1.0, **kw)


# ---------------------------------------------------------------------------
# Serving stream: many independent objects of uneven grid size.  Each request
# picks Lorenz '63 or Lorenz '96 (n = 6) with equal odds, a cell width, a mean
# within +-2 of the workload mean, a covariance scale in [0.25, 2], a horizon
# in [0.5, 2] and 0..4 scalar measurements of random components at sorted
# uniform times, drawn from its own seeded truth trajectory (RK4, step 1e-3).
# Thresholds 1e-5 (L63) and 1e-2 (L96) give initial grids of ~1e3 to ~2e6
# cells.  Arrival gaps are unit-rate exponentials; a driver divides them by
# the arrival rate it wants.
# ---------------------------------------------------------------------------

def _serving_truth(cfg, times, comps, sigma, seed, dt=1e-3):
    rng = np.random.Generator(np.random.PCG64(seed))
    n = cfg["n"]
    L = np.linalg.cholesky(np.asarray(cfg["cov"], dtype=np.float64))
    x = np.asarray(cfg["mean"], dtype=np.float64) + L @ rng.standard_normal(n)
    out, t = [], 0.0
    for tk, c in zip(times, comps):
        steps = int(round((tk - t) / dt))
        for _ in range(steps):
            k1 = _truth_drift(cfg, x)
            k2 = _truth_drift(cfg, x + 0.5 * dt * k1)
            k3 = _truth_drift(cfg, x + 0.5 * dt * k2)
            k4 = _truth_drift(cfg, x + dt * k3)
            x = x + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
        t = steps * dt + t
        out.append((float(tk), int(c), float(x[c] + sigma * rng.standard_normal()), float(sigma)))
    return out


def initial_cells_estimate(cfg):
    """Lattice points of the initial ellipsoid, by its volume in cell units."""
    from math import gamma, pi
    n = cfg["n"]
    cov = np.asarray(cfg["cov"], dtype=np.float64)
    r2 = 2.0 * np.log(1.0 / cfg["thresh_rel"])
    vol = pi ** (n / 2) / gamma(n / 2 + 1) * r2 ** (n / 2) * np.sqrt(np.linalg.det(cov)) / np.prod(cfg["h"][:n])
    return float(vol)


def serving_requests(n_req=256, seed=5):
    """(requests, unit-rate arrival offsets) of the serving stream."""
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = []
    for k in range(n_req):
        if rng.random() < 0.5:
            n, model, params = 3, L63, lorenz63()
            h = [0.5, 0.25][int(rng.integers(2))]
            mean = np.array([-11.5, -10.0, 9.5]) + rng.uniform(-2.0, 2.0, 3)
            cov, thr, sigma = rng.uniform(0.25, 2.0) * np.eye(3), 1e-5, 1.0
        else:
            n, model, params = 6, L96, lorenz96(4.0)
            h = [0.3, 0.25][int(rng.integers(2))]
            mean = np.array([4.5, 4.0, 4.0, 4.0, 4.0, 4.0]) + rng.uniform(-2.0, 2.0, 6)
            cov, thr, sigma = rng.uniform(0.25, 2.0) * 0.25 * np.eye(6), 1e-2, 0.5
        T = float(rng.uniform(0.5, 2.0))
        m = int(rng.integers(0, 5))
        times = np.sort(rng.uniform(0.0, T, m))
        comps = rng.integers(0, n, m)
        d = _base(n, model, params, h, mean, cov, thr, T)
        d["measurements"] = _serving_truth(d, times, comps, sigma, seed=seed * 100003 + k)
        d["request"] = k
        reqs.append(d)
    gaps = rng.exponential(1.0, n_req)
    return reqs, np.cumsum(gaps) - gaps[0]
