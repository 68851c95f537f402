"""Launch-shape autotuners.

tune_batch: times a few steps of the actual batch for each candidate (workgroup
tile, persistent grid) pair and keeps the fastest.  Results are cached in a JSON
file keyed by the device name, lattice, collision/forcing, storage and the
batch's size signature (box count, total cells, component-count histogram), so a
sweep is paid once per storage format.

tune_single: times the kernel schedules of one box (the two-pass schedule, the
blocked schedule at several slab heights, the overlapped schedule) for a context
factory and keeps the fastest.

Both time with HIP events on the stream the launches go to.
"""
from __future__ import annotations

import json
import os

CANDIDATE_TILES = (64, 128, 256)
# persistent grid: 0 = the resident workgroups of each kernel; larger values
# oversubscribe the device (each workgroup then walks fewer tiles)
CANDIDATE_GRIDS = (0, 4096, 16384)


def _key(boxes, lattice, collision, forcing, storage, fused=False):
    import numpy as np
    import torch
    cells = int(sum(int(np.prod(b["shape"])) for b in boxes))
    hist = {}
    for b in boxes:
        nc = len(b["mix"]["a"])
        hist[nc] = hist.get(nc, 0) + 1
    sig = ",".join(f"{k}:{hist[k]}" for k in sorted(hist))
    step = "|fused" if fused else ""
    return (f"{torch.cuda.get_device_name(0)}|{lattice}|{collision}|{forcing}|{storage}{step}|{len(boxes)}|{cells}|"
            f"{sig}")


def _event_ms(torch, stream, run):
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    run()
    t1.record(stream)
    t1.synchronize()
    return t0.elapsed_time(t1)


def tune_batch(boxes, lattice="D2Q9", collision="bgk", forcing="edm", storage="f32", steps=20, warmup=5,
               tiles=CANDIDATE_TILES, grids=CANDIDATE_GRIDS, cache_path=None, mrt_s=None, fused=False):
    """Return {"tile", "grid", "ms_per_step", "trials": {"tile/grid": ms}} for this
    batch and storage format; fused=True tunes the one-launch step
    (lbm_batch_params.fused) instead of the two launches."""
    import torch

    from . import lbm

    key = _key(boxes, lattice, collision, forcing, storage, fused)
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
    for tile in tiles:
        for grid in grids:
            b = lbm.LbmBatch(boxes, lattice, collision=collision, forcing=forcing, storage=storage, tile=tile,
                             grid=grid, mrt_s=mrt_s, fused=fused)
            b.step(warmup)
            b.check()
            ms = _event_ms(torch, b.stream, lambda: b.step(steps)) / steps
            b.check()
            trials[f"{tile}/{grid}"] = ms
            b.close()
            del b
            torch.cuda.empty_cache()
    best = min(trials, key=trials.get)
    tile, grid = (int(v) for v in best.split("/"))
    res = {"tile": tile, "grid": grid, "ms_per_step": trials[best], "trials": trials, "storage": storage,
           "fused": bool(fused)}
    if cache_path:
        cache[key] = res
        os.makedirs(os.path.dirname(os.path.abspath(cache_path)), exist_ok=True)
        with open(cache_path, "w") as fh:
            json.dump(cache, fh, indent=1)
    return res


def tune_single(make, steps=20, warmup=5, slabs=(16, 32, 64)):
    """make(schedule, slab_planes) -> LbmContext.  Times each schedule candidate and
    returns {"schedule", "slab_planes", "ms_per_step", "trials"}."""
    import torch

    cands = [("two_pass", 0)] + [("blocked", s) for s in slabs] + [("overlap", 0)]
    trials = {}
    for sched, slab in cands:
        c = make(sched, slab)
        c.step(warmup)
        c.check()
        ms = _event_ms(torch, c.stream, lambda: c.step(steps)) / steps
        c.check()
        trials[f"{sched}/{slab}"] = ms
        del c
        torch.cuda.empty_cache()
    best = min(trials, key=trials.get)
    sched, slab = best.split("/")
    return {"schedule": sched, "slab_planes": int(slab), "ms_per_step": trials[best], "trials": trials}
