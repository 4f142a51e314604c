"""Independent numpy references used to pin the oracle (test code only).

* ``drift``/``face_velocities``: the model right-hand sides of Sec. 5.1 written
  out in numpy, evaluated at backward-face centres mean_j + (i_j - 1/2) h_j.
* ``dense_ctu_step``: the CTU step on a dense box in the algebraically
  equivalent gather form (per-cell transverse fluctuations T_j, corrected
  states Q_l, upwind face fluxes), derived from Eq. 7 and Algorithm 1; this is
  a different formulation from the oracle's literal scatter form.
* closed forms: binomial / pairwise-operator solutions for constant velocity.
"""
import itertools

import numpy as np

from paper_2508_13986_amd.scenarios import L63, L96, LINEAR, UNIFORM


def drift(cfg, x, j):
    """f_j at points x[..., n]."""
    n, p = cfg["n"], cfg["params"]
    m = cfg["model"]
    if m == L63:
        z = x[..., 2] + p[3]
        return [p[0] * (x[..., 1] - x[..., 0]), x[..., 0] * (p[1] - z) - x[..., 1], x[..., 0] * x[..., 1] - p[2] * z][j]
    if m == L96:
        return (x[..., (j + 1) % n] - x[..., (j - 2) % n]) * x[..., (j - 1) % n] - x[..., j] + p[0]
    if m == LINEAR:
        A = np.asarray(p[: n * n]).reshape(n, n)
        b = np.asarray(p[n * n: n * n + n])
        return x @ A[j] + b[j]
    if m == UNIFORM:
        return np.full(x.shape[:-1], float(p[j]))
    raise ValueError(m)


def centres(cfg, idx):
    idx = np.asarray(idx, dtype=np.float64)
    return np.asarray(cfg["mean"])[: cfg["n"]] + idx * np.asarray(cfg["h"])[: cfg["n"]]


def face_velocity(cfg, idx, j):
    """f_{i - 1/2 e_j, j} for integer indices idx[..., n]."""
    x = centres(cfg, idx)
    x[..., j] = cfg["mean"][j] + (np.asarray(idx, dtype=np.float64)[..., j] - 0.5) * cfg["h"][j]
    return drift(cfg, x, j)


def grid_moments(cfg, idx, p):
    """Mean and covariance of a cell-average density on the grid (mass V * sum P)."""
    x = centres(cfg, idx)
    w = p / p.sum()
    mu = w @ x
    d = x - mu
    return mu, (d * w[:, None]).T @ d


# ---------------------------------------------------------------------------
# Dense-box CTU in gather form.
# ---------------------------------------------------------------------------

def _shift(a, j, s):
    """b[i] = a[i + s e_j] with zero outside the box."""
    b = np.zeros_like(a)
    src = [slice(None)] * a.ndim
    dst = [slice(None)] * a.ndim
    if s > 0:
        src[j] = slice(s, None)
        dst[j] = slice(None, -s)
    else:
        src[j] = slice(None, s)
        dst[j] = slice(-s, None)
    b[tuple(dst)] = a[tuple(src)]
    return b


def dense_ctu_step(cfg, P, lo, dt, limiter):
    """One CTU step on the dense box whose cell (0,...,0) has index lo; returns P'."""
    n = cfg["n"]
    h = cfg["h"]
    shape = P.shape
    grids = np.meshgrid(*[np.arange(shape[j]) + lo[j] for j in range(n)], indexing="ij")
    idx = np.stack(grids, -1)
    U = [face_velocity(cfg, idx, j) for j in range(n)]             # backward faces
    Uf = [face_velocity(cfg, idx + np.eye(n, dtype=int)[j], j) for j in range(n)]  # forward faces
    inbox = np.ones(shape, dtype=bool)
    ex_p = [_shift(inbox, j, +1) for j in range(n)]   # i + e_j in the box
    ex_m = [_shift(inbox, j, -1) for j in range(n)]   # i - e_j in the box
    Pm = [_shift(P, j, -1) for j in range(n)]
    Pp = [_shift(P, j, +1) for j in range(n)]
    pos = lambda v: np.maximum(v, 0.0)
    neg = lambda v: np.minimum(v, 0.0)
    # transverse fluctuation of each cell along j
    T = [pos(U[j]) * (P - Pm[j]) + np.where(ex_p[j], neg(Uf[j]) * (Pp[j] - P), 0.0) for j in range(n)]
    c = [dt / (2.0 * h[j]) for j in range(n)]
    Q = []
    for l in range(n):
        q = P.copy()
        for j in range(n):
            if j != l:
                q = q - c[j] * T[j]
        Q.append(q)
    out = P.copy()
    for l in range(n):
        # flux through the backward l-face of every cell
        F = pos(U[l]) * _shift(Q[l], l, -1) + neg(U[l]) * Q[l]
        if limiter:
            W = P - Pm[l]
            Pmm = _shift(P, l, -2)
            Wup = np.where(U[l] > 0, Pm[l] - Pmm, Pp[l] - P)
            a = np.abs(U[l])
            lim = np.where(W * Wup <= 0, 0.0,
                           np.sign(W) * np.minimum(np.abs(W + Wup) / 2, np.minimum(2 * np.abs(W), 2 * np.abs(Wup))))
            F = F + 0.5 * a * (1 - dt * a / h[l]) * lim
        Ffwd = _shift(F, l, +1)
        out = out + (dt / h[l]) * np.where(ex_m[l], F, 0.0) - (dt / h[l]) * np.where(ex_p[l], Ffwd, 0.0)
    return out


def to_dense(idx, p, lo, shape):
    P = np.zeros(shape)
    loc = np.asarray(idx) - np.asarray(lo)
    P[tuple(loc.T)] = p
    return P


def from_dense(P, lo):
    nz = np.argwhere(P != 0)
    return nz + np.asarray(lo), P[tuple(nz.T)]


# ---------------------------------------------------------------------------
# Closed forms for constant velocity.
# ---------------------------------------------------------------------------

def pairwise_operator_step(P, courant, signs):
    """(1 - sum_j a_j D_j + sum_{j<l} a_j a_l D_j D_l) P with (D_j P)_i = P_i - P_{i - s_j e_j}."""
    n = P.ndim

    def D(j, A):
        return A - _shift(A, j, -signs[j])

    out = P.copy()
    for j in range(n):
        out = out - courant[j] * D(j, P)
    for j, l in itertools.combinations(range(n), 2):
        out = out + courant[j] * courant[l] * D(j, D(l, P))
    return out
