"""Orthant against pairwise grow/prune (Sec. 3.3 and Figs. 2-3 against the
staged axis + 2-D diagonal growth of Sec. 4.4.1): the same propagation with
grow_mode 0 (downwind axis and pairwise-edge cells) and grow_mode 2 (every
combination of downwind steps, up to 2^n - 1 cells), each compared with a
reference run of the pairwise mode at a 1000-fold lower threshold, which
tracks the density 3 decades further into its tails.

Reported per mode and time: cells, cells created by grow, the mass fraction
the prunes removed so far, and E = V sum |p - p_ref| (the 1-norm of Eq. 10)
over the union of the two grids, a cell missing from one grid counting as 0.
Nothing here changes the propagation: it drives the library through the
binding and post-processes exported grids.
"""
import argparse
import json
import time

import numpy as np

from . import gbees as G
from . import scenarios as S


def _packed(idx):
    bits = 63 // idx.shape[1]
    key = np.zeros(len(idx), dtype=np.int64)
    for j in range(idx.shape[1]):
        key = (key << bits) + (idx[:, j].astype(np.int64) + (1 << (bits - 1)))
    return key


def l1_union(a, b, volume):
    """V * sum |Pa - Pb| over the union of two exported grids (idx, P)."""
    ka, kb = _packed(a[0]), _packed(b[0])
    keys = np.union1d(ka, kb)
    pa = np.zeros(len(keys))
    pb = np.zeros(len(keys))
    pa[np.searchsorted(keys, ka)] = a[1]
    pb[np.searchsorted(keys, kb)] = b[1]
    return float(volume * np.abs(pa - pb).sum())


def run(cfg, times, max_cells):
    g = G.Grid.gaussian(cfg, max_cells)
    out = []
    t0 = time.perf_counter()
    for t in times:
        g.step(t)
        st = g.stats()
        idx, P, _ = g.export()
        out.append({"t": t, "idx": idx, "P": P, "cells": st["cells"], "inserted": st["inserted"],
                    "mass_pruned": st["mass_pruned"], "steps": st["steps"], "cell_updates": st["cell_updates"]})
    out[-1]["seconds"] = time.perf_counter() - t0
    g.close()
    return out


CASES = {
    "l63": (lambda: S.l63_small(), [0.1, 0.25, 0.5], 64 * 400_000),
    "l96_6d": (lambda: S.l96_6d_downsampled(), [0.1, 0.25, 0.5], 64 * 4_000_000),
}


def study(names=("l63", "l96_6d")):
    res = {}
    for name in names:
        make, times, cap = CASES[name]
        base = S.with_(make(), measurements=[])
        V = float(np.prod(base["h"][: base["n"]]))
        ref = run(S.with_(base, thresh_rel=base["thresh_rel"] * 1e-3), times, cap)
        rows = {}
        for mode, label in ((0, "pairwise"), (2, "orthant")):
            r = run(S.with_(base, grow_mode=mode), times, cap)
            rows[label] = [{"t": x["t"], "cells": x["cells"], "inserted": x["inserted"],
                            "mass_pruned": x["mass_pruned"], "steps": x["steps"],
                            "E_vs_reference": l1_union((x["idx"], x["P"]), (y["idx"], y["P"]), V)}
                           for x, y in zip(r, ref)]
            rows[label][-1]["seconds"] = r[-1]["seconds"]
            rows[label][-1]["cell_updates"] = r[-1]["cell_updates"]
        rows["reference"] = [{"t": y["t"], "cells": y["cells"], "mass_pruned": y["mass_pruned"]} for y in ref]
        res[name] = {"workload": f"{name}: h={base['h'][0]}, thr={base['thresh_rel']}, CFL {base['cfl']}, "
                                 f"MC limiter, prune every {base['prune_every']}, no measurements",
                     "reference": f"pairwise, thr={base['thresh_rel'] * 1e-3}", "rows": rows}
        print(name, json.dumps({k: v[-1] for k, v in rows.items()}), flush=True)
    return res


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    out = study()
    if args.out:
        with open(args.out, "w") as fh:
            json.dump(out, fh, indent=1)
