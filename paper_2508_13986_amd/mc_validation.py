"""Accuracy against Monte Carlo (Sec. 5.2.1, Eq. 9, Table 1, Lorenz '63 case):
the Bhattacharyya coefficient between the propagated grid and a kernel
density estimate of a Monte Carlo ensemble with the same initial Gaussian.

* Ensemble: n_samples draws x0 = mean + L z (Cholesky L, z from PCG64 with
  the given seed), each integrated by RK4 with a fixed step to the time of
  comparison (before the measurement update, which the ensemble cannot take).
* KDE: Gaussian kernels with covariance s^2 * (sample covariance), Scott's
  factor s = n^(-1/(d+4)).  It is evaluated binned on the grid's lattice:
  the samples are histogrammed into the lattice cells and the histogram is
  convolved with the kernel sampled at the lattice offsets (normalised to
  unit sum), then divided by n V.  (Binning moves each sample by at most h/2.)
* BC = V * sum over the grid's cells of sqrt(p(x_i) p_kde(x_i)), Eq. 9 with
  the cell volume V that the printed formula leaves out.

The propagation itself runs through the library; this module only samples,
integrates the ensemble and post-processes.
"""
import argparse
import json

import numpy as np
from scipy.signal import fftconvolve

from . import gbees as G
from . import scenarios as S


def ensemble(cfg, t, n_samples, seed, dt=1e-3):
    """Monte Carlo ensemble at time t: array (n, n_samples)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = cfg["n"]
    L = np.linalg.cholesky(np.asarray(cfg["cov"], dtype=np.float64))
    x = np.asarray(cfg["mean"], dtype=np.float64)[:, None] + L @ rng.standard_normal((n_samples, n)).T
    steps = int(round(t / dt))
    f = lambda y: S._truth_drift(cfg, y)
    for _ in range(steps):
        k1 = f(x)
        k2 = f(x + 0.5 * dt * k1)
        k3 = f(x + 0.5 * dt * k2)
        k4 = f(x + dt * k3)
        x = x + (dt / 6.0) * (k1 + 2 * k2 + 2 * k3 + k4)
    return x


class BinnedKDE:
    """Scott-bandwidth Gaussian KDE of samples (n, N), binned on the lattice
    of cell centres mean + i h."""

    def __init__(self, samples, mean, h, reach=4.0):
        n, N = samples.shape
        self.mean = np.asarray(mean, dtype=np.float64)
        self.h = np.asarray(h, dtype=np.float64)
        s = N ** (-1.0 / (n + 4))
        cov = np.atleast_2d(np.cov(samples)) * s * s
        std = np.sqrt(np.diag(cov))
        half = np.ceil(reach * std / self.h).astype(int)  # kernel half-width in cells
        cells = np.floor((samples - self.mean[:, None]) / self.h[:, None] + 0.5).astype(np.int64)
        self.lo = cells.min(axis=1) - half
        shape = tuple((cells.max(axis=1) + half - self.lo + 1).tolist())
        hist = np.zeros(shape)
        np.add.at(hist, tuple(cells - self.lo[:, None]), 1.0)
        axes = [np.arange(-k, k + 1) * hj for k, hj in zip(half, self.h)]
        offs = np.stack(np.meshgrid(*axes, indexing="ij"), axis=-1)
        inv = np.linalg.inv(cov)
        kern = np.exp(-0.5 * np.einsum("...i,ij,...j->...", offs, inv, offs))
        kern /= kern.sum()
        self.dens = np.maximum(fftconvolve(hist, kern, mode="same"), 0.0) / (N * float(np.prod(self.h)))

    def at(self, idx):
        """Density at the cells idx (count, n); 0 outside the box."""
        k = np.asarray(idx, dtype=np.int64) - self.lo[None, :]
        ok = np.all((k >= 0) & (k < np.asarray(self.dens.shape)[None, :]), axis=1)
        out = np.zeros(len(k))
        out[ok] = self.dens[tuple(k[ok].T)]
        return out


def bhattacharyya(idx, P, kde, h):
    return float(np.prod(h)) * float(np.sqrt(np.maximum(P, 0.0) * kde.at(idx)).sum())


def run(cfg, t, n_samples=100_000, seed=11, max_cells=64 * 200_000):
    """BC at time t (before any measurement at t) of the grid against the ensemble's KDE."""
    g = G.Grid.gaussian(cfg, max_cells)
    try:
        for (tm, comp, y, sigma) in sorted(cfg.get("measurements", [])):
            if tm < t:
                g.step(tm)
                g.correct(comp, y, sigma)
        g.step(t)
        idx, P, _ = g.export()
    finally:
        g.close()
    x = ensemble(cfg, t, n_samples, seed)
    kde = BinnedKDE(x, cfg["mean"], cfg["h"])
    h = np.asarray(cfg["h"], dtype=np.float64)
    bc = bhattacharyya(idx, P, kde, h)
    kmass = float(np.prod(h)) * float(kde.at(idx).sum())
    # samples whose cell is in the grid (support coverage, no KDE involved)
    cells = np.floor((x - np.asarray(cfg["mean"])[:, None]) / h[:, None] + 0.5).astype(np.int64).T
    grid = set(map(tuple, np.asarray(idx, dtype=np.int64).tolist()))
    inside = float(np.mean([tuple(c) in grid for c in cells.tolist()]))
    return {"t": t, "h": float(h[0]), "cells": int(len(idx)), "samples": n_samples, "bc": bc,
            "kde_mass_on_grid": kmass, "bc_kde_renormalised_on_grid": bc / np.sqrt(kmass) if kmass > 0 else 0.0,
            "samples_inside_grid": inside}


def main():
    ap = argparse.ArgumentParser(description="Lorenz '63 grid against a Monte Carlo KDE (Bhattacharyya coefficient).")
    ap.add_argument("--out", required=True)
    ap.add_argument("--samples", type=int, default=100_000)
    args = ap.parse_args()
    import torch

    torch.cuda.set_device(0)
    res = {"scenario": "Lorenz '63, (sigma, b, r) = (4, 1, 48) shifted form, mean (-11.5, -10, 9.5), unit variances, "
                       "thr 1e-5, CFL 0.9, MC limiter; h = 0.5 (the paper's) and 0.25",
           "paper_table_1": {"t": 1.0, "h": 0.5, "bc_gpu": 0.9027}, "runs": []}
    for h in (0.5, 0.25):
        cfg = S.with_(S.workload("l63_paper"), h=[h] * 3)
        for t in (1.0 / 3.0, 2.0 / 3.0, 1.0):
            r = run(cfg, t, args.samples)
            res["runs"].append(r)
            print(json.dumps(r), flush=True)
    with open(args.out, "w") as fh:
        json.dump(res, fh, indent=1)


if __name__ == "__main__":
    main()
