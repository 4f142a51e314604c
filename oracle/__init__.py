"""ctypes wrapper of the CPU oracle (oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by tests/, by the smoke check and by the
benchmark's CPU-baseline leg, never by the product package.  The oracle is a
plain FP64 implementation of the GBEES time step (arXiv 2508.13986, Sec. 2-3,
Eq. 4-8, Algorithms 1 and 3) over a std::unordered_map grid.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_LIB = None


class OracleConfig(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("model", ctypes.c_int32),
        ("params", ctypes.c_double * 48),
        ("h", ctypes.c_double * 6),
        ("mean", ctypes.c_double * 6),
        ("cov", ctypes.c_double * 36),
        ("thresh_rel", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("dt_fixed", ctypes.c_double),
        ("prune_every", ctypes.c_int32),
        ("limiter", ctypes.c_int32),
        ("grow_mode", ctypes.c_int32),
    ]


class OracleStats(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double),
        ("dt_last", ctypes.c_double),
        ("min_margin", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("steps", ctypes.c_int64),
        ("cell_updates", ctypes.c_int64),
        ("cells", ctypes.c_int64),
        ("prunes", ctypes.c_int64),
    ]


def lib():
    """Load liboracle.so, building it first if it is missing or stale."""
    global _LIB
    if _LIB is None:
        # GBEES_ORACLE_LIB points the tests at another build of oracle.cpp (mutation checks).
        path = os.environ.get("GBEES_ORACLE_LIB") or _build.build(force=False)
        L = ctypes.CDLL(path)
        vp = ctypes.c_void_p
        L.oracle_new.restype = vp
        L.oracle_new.argtypes = [ctypes.POINTER(OracleConfig)]
        L.oracle_free.argtypes = [vp]
        L.oracle_init_gaussian.argtypes = [vp]
        L.oracle_init_cells.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double]
        L.oracle_step.argtypes = [vp, ctypes.c_double, ctypes.c_int64]
        L.oracle_grow.restype = ctypes.c_int64
        L.oracle_grow.argtypes = [vp]
        L.oracle_prune.argtypes = [vp]
        L.oracle_normalise.argtypes = [vp]
        L.oracle_smax.restype = ctypes.c_double
        L.oracle_smax.argtypes = [vp]
        L.oracle_correct.argtypes = [vp, ctypes.c_int32, ctypes.c_double, ctypes.c_double]
        L.oracle_count.restype = ctypes.c_int64
        L.oracle_count.argtypes = [vp]
        L.oracle_export.restype = ctypes.c_int64
        L.oracle_export.argtypes = [vp, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.oracle_marginals.restype = ctypes.c_int64
        L.oracle_marginals.argtypes = [vp, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64]
        L.oracle_get_stats.argtypes = [vp, ctypes.POINTER(OracleStats)]
        L.oracle_log.restype = ctypes.c_int64
        L.oracle_log.argtypes = [vp, ctypes.c_void_p, ctypes.c_int64]
        L.oracle_drift.restype = ctypes.c_double
        L.oracle_drift.argtypes = [vp, ctypes.c_void_p, ctypes.c_int32]
        L.oracle_face_vel.restype = ctypes.c_double
        L.oracle_face_vel.argtypes = [vp, ctypes.c_void_p, ctypes.c_int32]
        _LIB = L
    return _LIB


def _fill(arr, values):
    for k, v in enumerate(values):
        arr[k] = float(v)


def make_config(cfg: dict) -> OracleConfig:
    """Marshal a scenario dict (see paper_2508_13986_amd.scenarios) into the oracle struct."""
    c = OracleConfig()
    n = int(cfg["n"])
    c.n = n
    c.model = int(cfg["model"])
    _fill(c.params, cfg.get("params", []))
    _fill(c.h, cfg["h"])
    _fill(c.mean, cfg["mean"])
    _fill(c.cov, np.asarray(cfg["cov"], dtype=np.float64).reshape(-1))
    c.thresh_rel = float(cfg.get("thresh_rel", 0.0))
    c.cfl = float(cfg.get("cfl", 0.9))
    c.dt_fixed = float(cfg.get("dt_fixed", 0.0))
    c.prune_every = int(cfg.get("prune_every", 0))
    c.limiter = int(cfg.get("limiter", 0))
    c.grow_mode = int(cfg.get("grow_mode", 0))
    return c


class Oracle:
    """One oracle grid.  Methods follow the paper's operations one to one."""

    def __init__(self, cfg: dict):
        self.cfg = dict(cfg)
        self.n = int(cfg["n"])
        self._c = make_config(cfg)
        self._L = lib()
        self._h = self._L.oracle_new(ctypes.byref(self._c))
        if not self._h:
            raise ValueError("oracle: bad config")

    def __del__(self):
        h = getattr(self, "_h", None)
        if h:
            self._L.oracle_free(h)
            self._h = None

    def init_gaussian(self):
        if self._L.oracle_init_gaussian(self._h) != 0:
            raise ValueError("oracle: init_gaussian failed")
        return self

    def init_cells(self, idx, p, t0=0.0):
        idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, self.n)
        p = np.ascontiguousarray(p, dtype=np.float64).reshape(-1)
        self._L.oracle_init_cells(self._h, idx.ctypes.data, p.ctypes.data, len(p), float(t0))
        return self

    def step(self, t_stop, max_steps=0):
        self._L.oracle_step(self._h, float(t_stop), int(max_steps))
        return self

    def grow(self):
        return int(self._L.oracle_grow(self._h))

    def prune(self):
        self._L.oracle_prune(self._h)

    def normalise(self):
        self._L.oracle_normalise(self._h)

    def smax(self):
        return float(self._L.oracle_smax(self._h))

    def correct(self, comp, y, sigma):
        if self._L.oracle_correct(self._h, int(comp), float(y), float(sigma)) != 0:
            raise ValueError("oracle: bad correction")
        return self

    def count(self):
        return int(self._L.oracle_count(self._h))

    def export(self):
        """(idx int32[count, n], P float64[count]) sorted lexicographically by index."""
        cnt = self.count()
        idx = np.zeros((max(cnt, 1), self.n), dtype=np.int32)
        p = np.zeros(max(cnt, 1), dtype=np.float64)
        got = self._L.oracle_export(self._h, idx.ctypes.data, p.ctypes.data, cnt)
        assert got == cnt
        return idx[:cnt], p[:cnt]

    def marginals(self, dims):
        mask = 0
        for d in dims:
            mask |= 1 << int(d)
        m = bin(mask).count("1")
        cap = max(self.count(), 1)
        idx = np.zeros((cap, m), dtype=np.int32)
        val = np.zeros(cap, dtype=np.float64)
        got = self._L.oracle_marginals(self._h, mask, idx.ctypes.data, val.ctypes.data, cap)
        assert got >= 0
        return idx[:got], val[:got]

    def stats(self) -> dict:
        s = OracleStats()
        self._L.oracle_get_stats(self._h, ctypes.byref(s))
        return {f: getattr(s, f) for f, _ in OracleStats._fields_}

    def log(self):
        """Per-step rows (t, dt, smax, maxP, step_margin, cells_updated)."""
        rows = -self._L.oracle_log(self._h, None, 0) if self.stats()["steps"] else 0
        out = np.zeros((max(rows, 1), 6), dtype=np.float64)
        got = self._L.oracle_log(self._h, out.ctypes.data, rows)
        return out[:max(got, 0)]

    def drift(self, x, j):
        x = np.zeros(6, dtype=np.float64) + np.pad(np.asarray(x, dtype=np.float64), (0, 6 - self.n))
        return float(self._L.oracle_drift(self._h, x.ctypes.data, int(j)))

    def face_vel(self, idx, j):
        i = np.zeros(6, dtype=np.int32)
        i[: self.n] = np.asarray(idx, dtype=np.int32)
        return float(self._L.oracle_face_vel(self._h, i.ctypes.data, int(j)))
