"""Launch-shape autotuner for the batched step.

Times a few steps of the actual batch for each candidate workgroup size (cells per
tile) and keeps the fastest.  Results are cached in a JSON file keyed by the
device name, lattice, collision/forcing, storage and the batch's size signature
(box count, total cells, component-count histogram), so a sweep is paid once.
"""
from __future__ import annotations

import json
import os
import time

CANDIDATE_TILES = (64, 128, 256)


def _key(boxes, lattice, collision, forcing, storage):
    import numpy as np
    import torch
    cells = int(sum(int(np.prod(b["shape"])) for b in boxes))
    hist = {}
    for b in boxes:
        nc = len(b["mix"]["a"])
        hist[nc] = hist.get(nc, 0) + 1
    sig = ",".join(f"{k}:{hist[k]}" for k in sorted(hist))
    return f"{torch.cuda.get_device_name(0)}|{lattice}|{collision}|{forcing}|{storage}|{len(boxes)}|{cells}|{sig}"


def tune_batch(boxes, lattice="D2Q9", collision="bgk", forcing="edm", storage="f32", steps=20, warmup=5,
               candidates=CANDIDATE_TILES, cache_path=None, mrt_s=None):
    """Return {"tile": best, "ms_per_step": t, "trials": {tile: ms}} for this batch."""
    import torch

    from . import lbm

    key = _key(boxes, lattice, collision, forcing, storage)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as fh:
            try:
                cache = json.load(fh)
            except ValueError:
                cache = {}
    if key in cache:
        return cache[key]
    trials = {}
    for tile in candidates:
        b = lbm.LbmBatch(boxes, lattice, collision=collision, forcing=forcing, storage=storage, tile=tile,
                         mrt_s=mrt_s)
        b.step(warmup)
        b.check()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        b.check()
        trials[int(tile)] = (time.perf_counter() - t0) * 1e3 / steps
        b.close()
        del b
        torch.cuda.empty_cache()
    best = min(trials, key=trials.get)
    res = {"tile": int(best), "ms_per_step": trials[best], "trials": trials}
    if cache_path:
        cache[key] = res
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return res
