"""Python binding of libgbees.so (include/gbees.h): argument marshalling only.

Every step of the method runs in the library's HIP kernels.  PyTorch supplies
the device arena (a uint8 tensor on the GPU) and the stream.  Loading fails
loudly if the library has not been built (``python -m paper_2508_13986_amd.build``
or ``__graft_entry__.build()``).
"""
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgbees.so")

OK, E_ARG, E_CAPACITY, E_RANGE, E_DEVICE, E_BUFFER, E_STATE = 0, -1, -2, -3, -4, -5, -6
L63, L96, LINEAR, UNIFORM = 1, 2, 3, 4
PROFILE_KINDS = ("grow", "grow_fix", "flux_a", "flux_b", "prune", "other")


class GbeesConfig(ctypes.Structure):
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
        ("precision", ctypes.c_int32),
        ("max_cells", ctypes.c_int64),
        ("hash_load", ctypes.c_double),
    ]


class GbeesStats(ctypes.Structure):
    _fields_ = [
        ("t", ctypes.c_double),
        ("dt_last", ctypes.c_double),
        ("mass", ctypes.c_double),
        ("max_p", ctypes.c_double),
        ("smax", ctypes.c_double),
        ("steps", ctypes.c_int64),
        ("cell_updates", ctypes.c_int64),
        ("brick_updates", ctypes.c_int64),
        ("cells", ctypes.c_int64),
        ("bricks", ctypes.c_int64),
        ("prunes", ctypes.c_int64),
        ("grow_bricks", ctypes.c_int64),
        ("inserted", ctypes.c_int64),
        ("deferred", ctypes.c_int64),
        ("mass_pruned", ctypes.c_double),
    ]


class GbeesError(RuntimeError):
    def __init__(self, code, where):
        self.code = code
        super().__init__(f"{where}: {lib().gbees_strerror(code).decode()} ({code})")


_LIB = None


def lib():
    """Load libgbees.so (raises if it is missing: there is no fallback path)."""
    global _LIB
    if _LIB is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"libgbees.so not built at {LIB_PATH}; run paper_2508_13986_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        vp, i64, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        cfgp = ctypes.POINTER(GbeesConfig)
        L.gbees_arena_bytes.restype = ctypes.c_size_t
        L.gbees_arena_bytes.argtypes = [cfgp]
        L.gbees_init_gaussian.argtypes = [cfgp, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.gbees_init_cells.argtypes = [cfgp, vp, vp, i64, dbl, vp, ctypes.c_size_t, vp, ctypes.POINTER(vp)]
        L.gbees_step.argtypes = [vp, dbl, i64, ctypes.POINTER(GbeesStats)]
        L.gbees_correct.argtypes = [vp, ctypes.c_int32, dbl, dbl]
        L.gbees_marginals.argtypes = [vp, ctypes.c_uint32, i64, vp, vp, ctypes.POINTER(i64)]
        L.gbees_export.argtypes = [vp, i64, vp, vp, ctypes.POINTER(i64), ctypes.POINTER(dbl)]
        L.gbees_get_stats.argtypes = [vp, ctypes.POINTER(GbeesStats)]
        L.gbees_probe_stats.argtypes = [vp, i64, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(dbl)]
        L.gbees_profile.argtypes = [vp, ctypes.c_int]
        L.gbees_profile_read.argtypes = [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64)]
        L.gbees_destroy.argtypes = [vp]
        L.gbees_resize.argtypes = [vp, i64, vp, ctypes.c_size_t]
        if hasattr(L, "gbees_marginals_noalloc"):
            L.gbees_marginals_noalloc.argtypes = [vp, ctypes.c_uint32, i64, vp, vp, vp]
            L.gbees_marginals_noalloc.restype = ctypes.c_int
        L.gbees_strerror.restype = ctypes.c_char_p
        L.gbees_strerror.argtypes = [ctypes.c_int]
        pp = ctypes.POINTER(ctypes.c_int32)
        L.gbees_pool_create.argtypes = [vp, ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(vp)]
        L.gbees_pool_submit.argtypes = [vp, cfgp, dbl, ctypes.POINTER(GbeesMeas), ctypes.c_int32, ctypes.POINTER(i64)]
        L.gbees_pool_progress.argtypes = [vp, pp, pp]
        L.gbees_pool_info.argtypes = [vp, i64, ctypes.POINTER(GbeesReqInfo)]
        L.gbees_pool_result.argtypes = [vp, i64, i64, vp, vp, ctypes.POINTER(i64)]
        L.gbees_pool_release.argtypes = [vp, i64]
        L.gbees_pool_group_size.argtypes = [vp, ctypes.c_int32]
        L.gbees_pool_clock.argtypes = [vp]
        L.gbees_pool_clock.restype = dbl
        L.gbees_pool_destroy.argtypes = [vp]
        for name in ("gbees_init_gaussian", "gbees_init_cells", "gbees_step", "gbees_correct", "gbees_marginals",
                     "gbees_export", "gbees_get_stats", "gbees_probe_stats", "gbees_profile",
                     "gbees_profile_read", "gbees_destroy", "gbees_resize", "gbees_pool_create", "gbees_pool_submit",
                     "gbees_pool_progress", "gbees_pool_info", "gbees_pool_result", "gbees_pool_release", "gbees_pool_group_size",
                     "gbees_pool_destroy"):
            getattr(L, name).restype = ctypes.c_int
        _LIB = L
    return _LIB

class GbeesMeas(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("component", ctypes.c_int32), ("y", ctypes.c_double), ("sigma", ctypes.c_double)]


class GbeesReqInfo(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int32),
        ("t_submit", ctypes.c_double),
        ("t_admit", ctypes.c_double),
        ("t_done", ctypes.c_double),
        ("arena_bytes", ctypes.c_int64),
        ("cells", ctypes.c_int64),
        ("stats", GbeesStats),
        ("resizes", ctypes.c_int64),
    ]


def _fill(arr, values):
    for k, v in enumerate(values):
        arr[k] = float(v)


def make_config(cfg: dict, max_cells=None) -> GbeesConfig:
    """Marshal a scenario dict (see scenarios.py) into gbees_config."""
    c = GbeesConfig()
    c.n = int(cfg["n"])
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
    c.precision = int(cfg.get("precision", 0))
    mc = max_cells if max_cells is not None else int(cfg.get("max_cells", 0) or 0)
    c.max_cells = int(mc) if mc else 1 << 20
    c.hash_load = float(cfg.get("hash_load", 0.5))
    return c


def arena_bytes(cfg: dict, max_cells=None) -> int:
    c = make_config(cfg, max_cells)
    return int(lib().gbees_arena_bytes(ctypes.byref(c)))


def _check(code, where):
    if code != OK:
        raise GbeesError(code, where)


class Grid:
    """One GBEES grid on the current CUDA/HIP device.

    ``Grid.gaussian(cfg)`` / ``Grid.from_cells(cfg, idx, P)`` create it; methods
    mirror the C ABI: step, correct, marginals, export, stats, probe_stats.
    """

    def __init__(self, cfg: dict, max_cells=None, device=None, stream=None):
        import torch

        self.cfg = dict(cfg)
        self.n = int(cfg["n"])
        self._c = make_config(cfg, max_cells)
        nbytes = int(lib().gbees_arena_bytes(ctypes.byref(self._c)))
        if nbytes == 0:
            raise GbeesError(E_ARG, "gbees_arena_bytes")
        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.arena = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        self._h = ctypes.c_void_p()

    @classmethod
    def gaussian(cls, cfg, max_cells=None, **kw):
        g = cls(cfg, max_cells, **kw)
        code = lib().gbees_init_gaussian(ctypes.byref(g._c), ctypes.c_void_p(g.arena.data_ptr()),
                                         ctypes.c_size_t(g.arena.numel()), ctypes.c_void_p(g.stream.cuda_stream),
                                         ctypes.byref(g._h))
        _check(code, "gbees_init_gaussian")
        return g

    @classmethod
    def from_cells(cls, cfg, idx, p, t0=0.0, max_cells=None, **kw):
        g = cls(cfg, max_cells, **kw)
        idx = np.ascontiguousarray(idx, dtype=np.int32).reshape(-1, g.n)
        p = np.ascontiguousarray(p, dtype=np.float64).reshape(-1)
        code = lib().gbees_init_cells(ctypes.byref(g._c), idx.ctypes.data, p.ctypes.data, len(p), float(t0),
                                      ctypes.c_void_p(g.arena.data_ptr()), ctypes.c_size_t(g.arena.numel()),
                                      ctypes.c_void_p(g.stream.cuda_stream), ctypes.byref(g._h))
        _check(code, "gbees_init_cells")
        return g

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().gbees_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step(self, t_stop, max_steps=0) -> dict:
        s = GbeesStats()
        _check(lib().gbees_step(self._h, float(t_stop), int(max_steps), ctypes.byref(s)), "gbees_step")
        return _stats_dict(s)

    def resize(self, max_cells):
        """Move the grid into a new arena of capacity max_cells (the old one is dropped)."""
        import torch

        c = make_config(self.cfg, max_cells)
        nbytes = int(lib().gbees_arena_bytes(ctypes.byref(c)))
        if nbytes == 0:
            raise GbeesError(E_ARG, "gbees_arena_bytes")
        arena = torch.empty(nbytes, dtype=torch.uint8, device=self.arena.device)
        _check(lib().gbees_resize(self._h, int(max_cells), ctypes.c_void_p(arena.data_ptr()), ctypes.c_size_t(nbytes)),
               "gbees_resize")
        self.arena = arena
        self._c = c

    def correct(self, component, y, sigma):
        _check(lib().gbees_correct(self._h, int(component), float(y), float(sigma)), "gbees_correct")

    def stats(self) -> dict:
        s = GbeesStats()
        _check(lib().gbees_get_stats(self._h, ctypes.byref(s)), "gbees_get_stats")
        return _stats_dict(s)

    def export(self):
        """(idx int32[count, n], P float64[count], t), cells sorted by index."""
        cnt = ctypes.c_int64(0)
        t = ctypes.c_double(0)
        code = lib().gbees_export(self._h, 0, None, None, ctypes.byref(cnt), ctypes.byref(t))
        if code not in (OK, E_BUFFER):
            raise GbeesError(code, "gbees_export")
        n = cnt.value
        idx = np.zeros((max(n, 1), self.n), dtype=np.int32)
        p = np.zeros(max(n, 1), dtype=np.float64)
        _check(lib().gbees_export(self._h, n, idx.ctypes.data, p.ctypes.data, ctypes.byref(cnt), ctypes.byref(t)),
               "gbees_export")
        return idx[: cnt.value], p[: cnt.value], t.value

    def marginals(self, dims):
        mask = 0
        for d in dims:
            mask |= 1 << int(d)
        m = bin(mask).count("1")
        cnt = ctypes.c_int64(0)
        code = lib().gbees_marginals(self._h, mask, 0, None, None, ctypes.byref(cnt))
        if code not in (OK, E_BUFFER):
            raise GbeesError(code, "gbees_marginals")
        n = cnt.value
        idx = np.zeros((max(n, 1), m), dtype=np.int32)
        val = np.zeros(max(n, 1), dtype=np.float64)
        _check(lib().gbees_marginals(self._h, mask, n, idx.ctypes.data, val.ctypes.data, ctypes.byref(cnt)),
               "gbees_marginals")
        return idx[: cnt.value], val[: cnt.value]

    def probe_stats(self, n_miss=1 << 16):
        hit, miss, load = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        _check(lib().gbees_probe_stats(self._h, int(n_miss), ctypes.byref(hit), ctypes.byref(miss),
                                       ctypes.byref(load)), "gbees_probe_stats")
        return {"hit": hit.value, "miss": miss.value, "load": load.value}

    def profile(self, enable=True):
        _check(lib().gbees_profile(self._h, 1 if enable else 0), "gbees_profile")

    def profile_read(self) -> dict:
        ms = (ctypes.c_double * 6)()
        n = (ctypes.c_int64 * 6)()
        _check(lib().gbees_profile_read(self._h, ms, n), "gbees_profile_read")
        return {k: (ms[i], n[i]) for i, k in enumerate(PROFILE_KINDS)}


def _stats_dict(s: GbeesStats) -> dict:
    return {f: getattr(s, f) for f, _ in GbeesStats._fields_}


class Pool:
    """The serving pool (gbees_pool_*): requests share one device arena and run
    concurrently; ``progress()`` advances them without waiting on the device."""

    def __init__(self, arena_bytes: int, max_active: int = 16, device=None):
        import torch

        dev = device if device is not None else torch.device("cuda", torch.cuda.current_device())
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=dev)
        self._h = ctypes.c_void_p()
        _check(lib().gbees_pool_create(ctypes.c_void_p(self.arena.data_ptr()), ctypes.c_size_t(self.arena.numel()),
                                       int(max_active), ctypes.byref(self._h)), "gbees_pool_create")
        self.n = {}

    def submit(self, cfg: dict, max_cells: int, t_end=None, measurements=None) -> int:
        """Queue the scenario ``cfg`` (its t_end and measurements unless given)."""
        c = make_config(cfg, max_cells)
        meas = cfg.get("measurements", []) if measurements is None else measurements
        arr = (GbeesMeas * max(len(meas), 1))()
        for k, (t, comp, y, sig) in enumerate(meas):
            arr[k] = GbeesMeas(float(t), int(comp), float(y), float(sig))
        rid = ctypes.c_int64(0)
        te = float(cfg["t_end"] if t_end is None else t_end)
        _check(lib().gbees_pool_submit(self._h, ctypes.byref(c), te, arr, len(meas), ctypes.byref(rid)),
               "gbees_pool_submit")
        self.n[rid.value] = int(cfg["n"])
        return rid.value

    def progress(self):
        """(running, waiting) after one non-blocking pass."""
        r, w = ctypes.c_int32(0), ctypes.c_int32(0)
        _check(lib().gbees_pool_progress(self._h, ctypes.byref(r), ctypes.byref(w)), "gbees_pool_progress")
        return r.value, w.value

    def info(self, rid: int) -> dict:
        i = GbeesReqInfo()
        _check(lib().gbees_pool_info(self._h, int(rid), ctypes.byref(i)), "gbees_pool_info")
        st = {f: getattr(i.stats, f) for f, _ in GbeesStats._fields_}
        return {"status": i.status, "t_submit": i.t_submit, "t_admit": i.t_admit, "t_done": i.t_done,
                "arena_bytes": i.arena_bytes, "cells": i.cells, "stats": st, "resizes": i.resizes}

    def result(self, rid: int):
        """(idx int32[count, n], P float64[count]) of a finished request."""
        cnt = ctypes.c_int64(0)
        code = lib().gbees_pool_result(self._h, int(rid), 0, None, None, ctypes.byref(cnt))
        if code not in (OK, E_BUFFER):
            raise GbeesError(code, "gbees_pool_result")
        n = self.n[int(rid)]
        idx = np.zeros((cnt.value, n), dtype=np.int32)
        P = np.zeros(cnt.value, dtype=np.float64)
        _check(lib().gbees_pool_result(self._h, int(rid), cnt.value, idx.ctypes.data_as(ctypes.c_void_p),
                                       P.ctypes.data_as(ctypes.c_void_p), ctypes.byref(cnt)), "gbees_pool_result")
        return idx, P

    def group_size(self, k: int):
        _check(lib().gbees_pool_group_size(self._h, int(k)), "gbees_pool_group_size")

    def release(self, rid: int):
        _check(lib().gbees_pool_release(self._h, int(rid)), "gbees_pool_release")

    def clock(self) -> float:
        return float(lib().gbees_pool_clock(self._h))

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().gbees_pool_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_scenario(cfg, max_cells=None, grid=None):
    """Propagate a scenario to t_end applying its measurements in time order."""
    g = grid if grid is not None else Grid.gaussian(cfg, max_cells)
    for (t, comp, y, sigma) in sorted(cfg.get("measurements", [])):
        if t <= cfg["t_end"]:
            g.step(t)
            g.correct(comp, y, sigma)
    g.step(cfg["t_end"])
    return g
