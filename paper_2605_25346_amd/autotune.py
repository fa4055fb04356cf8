"""Launch-shape autotuner for the persistent kernels.

For a workload (networks + batch) it times graph replays of each entry point while
sweeping the number of persistent workgroups per CU of that kernel kind (1..max, the
4-bit fields of ``dr_options.tile_cfg``), keeps the fastest per kind (coordinate
descent, kinds are independent launches) and stores the packed configuration in a
JSON cache keyed by precision and network shapes.  ``BoundContext(tile_cfg="auto")``
reads the cache.
"""
from __future__ import annotations

import json
import os
from typing import Dict, Optional

import numpy as np

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tile_cache.json")
KINDS = {"bound_init": 0, "spec_chains": 1, "dual_ascent": 2, "reach_dt": 3}


def key_of(nets, precision: str) -> str:
    return precision + ":" + "|".join("-".join(str(w) for w in n.widths) for n in nets)


def load_cache(path: str = CACHE) -> Dict[str, int]:
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return {k: int(v["tile_cfg"]) if isinstance(v, dict) else int(v) for k, v in json.load(f).items()}


def lookup(nets, precision: str, path: str = CACHE) -> int:
    return load_cache(path).get(key_of(nets, precision), 0)


def _time(torch, fn, reps=5):
    fn(); torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True); e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record(); torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(wl, precision="f32", kinds=("bound_init", "spec_chains", "dual_ascent", "reach_dt"), max_cap=8,
         path: str = CACHE, verbose=True) -> int:
    import torch
    from .api import BoundContext, DeviceBatch
    S = wl.batch.n_sub
    ms = max(int(np.max(np.diff(wl.batch.split_ptr))) if S else 0, 1)
    db = DeviceBatch(wl.batch)
    cfg = 0
    results = {}
    for kind in kinds:
        if kind == "reach_dt" and not wl.horizon:
            continue
        if kind != "reach_dt" and wl.horizon:
            continue
        if kind == "dual_ascent" and not wl.iters:
            continue
        shift = 4 * KINDS[kind]
        best = None
        for cap in range(0, max_cap + 1):
            trial = (cfg & ~(15 << shift)) | (cap << shift)
            ctx = BoundContext(wl.nets, precision=precision, max_sub=S, max_splits=ms, tile_cfg=trial)
            if kind == "reach_dt":
                fn = lambda: ctx.dr_reach_dt(db, wl.horizon)
            else:
                ctx.dr_bound_init(db)
                if kind == "bound_init":
                    fn = lambda: ctx.dr_bound_init(db)
                elif kind == "spec_chains":
                    fn = lambda: ctx.dr_propagate_backward()
                else:
                    alpha, beta = ctx.new_duals()
                    fn = lambda: ctx.dr_optimize_duals(wl.iters, wl.lr, alpha, beta)
            t = _time(torch, fn)
            ctx.close()
            if verbose:
                print(f"autotune {kind} cap={cap}: {t:.3f} ms", flush=True)
            if best is None or t < best[1] * 0.98:
                best = (cap, t)
        cfg = (cfg & ~(15 << shift)) | (best[0] << shift)
        results[kind] = dict(cap=best[0], ms=best[1])
    cache = {}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    cache[key_of(wl.nets, precision)] = dict(tile_cfg=cfg, detail=results)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    return cfg
