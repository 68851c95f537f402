#!/usr/bin/env python3
"""Benchmark of the multi-component pseudo-potential LB step on one MI355X.

Workload (default): four-component D3Q19 box of 128^3 cells with a spherical drop
of radius 32 in vapor, MRT collision with exact-difference forcing, one component
supercritical (the seeded four-component configuration of inputs.config_c3), with
populations stored as float16 offsets (float32 collision, float64 EOS / psi).

One step = one lbm_step (densities, EOS, psi, force stencil, split, collision,
streaming); every `--diag-every` steps the conservation totals are reduced on
the device as well.  Inputs are resident in HBM before the timed region.

Prints ONE JSON line.  `value` is MLUPS x components (cells * nc * steps / s / 1e6)
of the whole job.  `roofline` prices the dominant kernel: algorithmic bytes per
cell update (populations read + written once, psi written + read once, the
float32 base of the offset formats) times the cells of one launch, divided by the
kernel's average duration from HIP events over the timed region.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import subprocess
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS×components + HBM GB/s % peak, FP16/FP32 vs FP64 at 1e-4 mole-frac err"
PEAK_HBM_GBS = 8000.0
STORAGE_BYTES = {"f64": 8, "f32": 4, "f16": 2}
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")


def b_alg(nc: int, Q: int, storage: str) -> int:
    """Algorithmic bytes per cell update: 2 nc Q s (populations) + 16 (psi written
    and read once) + 8 nc for the float32 base (read + write) of the offset formats."""
    s = STORAGE_BYTES[storage]
    return 2 * nc * Q * s + 16 + (8 * nc if storage != "f64" else 0)


def b_alg_collide(nc: int, Q: int, storage: str) -> int:
    """Share of b_alg carried by the collide kernel: populations read and written
    once, the float32 base read and written once (offset formats), psi read once
    (the psi write, 8 B, belongs to the density/psi kernel)."""
    return b_alg(nc, Q, storage) - 8


# the sources that define the single-box step kernels and their launches: a change
# to any of them voids the stored counters (host-only code elsewhere does not)
STEP_KERNEL_SOURCES = ("lattice.hpp", "lbm_kernels.hpp", "lbm_dispatch.hpp", "lbm_internal.hpp", "lbm_ctx.hpp",
                       "lbm.hip", "lbm_d2q9.hip", "lbm_d3q19.hip")


def kernel_source_sha() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1909_12390_amd", "csrc")
    for name in STEP_KERNEL_SOURCES:
        with open(os.path.join(csrc, name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_profile(kernel_key: str):
    """The profile record of this kernel (HBM bytes per launch from rocprofv3
    FETCH_SIZE/WRITE_SIZE runs, pipe busy fractions from its counter runs), or {}
    if absent or taken on different kernel sources."""
    try:
        with open(TRAFFIC_FILE) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return {}
    ent = rec.get(kernel_key)
    if not ent or ent.get("source_sha") != kernel_source_sha():
        return {}
    return ent


def phase_mole_fractions(rho_s, M, geometry, shape):
    """Bulk liquid/vapor states with fixed masks: drop liquid = r <= R0/2, vapor =
    r >= min(L)/2 (box corners); mole fractions x_i = sum_mask n_i / sum_mask n and
    the mask-mean molar densities (for the fugacities)."""
    import torch
    dev = rho_s.device
    grids = torch.meshgrid(*[torch.arange(n, dtype=torch.float64, device=dev) for n in shape], indexing="ij")
    r2 = sum((g - n / 2.0) ** 2 for g, n in zip(grids, shape))
    r = torch.sqrt(r2)
    R0 = geometry["R0"]
    liq = r <= R0 / 2.0
    vap = r >= min(shape) / 2.0
    n = rho_s / torch.as_tensor(M, dtype=torch.float64, device=dev).reshape((-1,) + (1,) * len(shape))
    out = {}
    for name, mask in (("liquid", liq), ("vapor", vap)):
        ni = torch.stack([n[i][mask].sum() for i in range(n.shape[0])])
        out[name] = (ni / ni.sum()).cpu().numpy()
        out["n_" + name] = (ni / mask.sum()).cpu().numpy()
    return out


def fugacities(lbm, mix, T, n_l, n_v):
    """Fugacities of the bulk liquid and vapour (Eq. fugacity at each state's own
    p_EOS, no root choice) and the iso-fugacity residual of Eq. (error)."""
    f = lbm.lbm_fugacity(mix, T, np.stack([n_l, n_v]))
    fl, fv = np.asarray(f["fug"][0]), np.asarray(f["fug"][1])
    return fl, fv, float(np.sum((fl / fv - 1.0) ** 2)), 0.5 * float(f["p"][0] + f["p"][1])


def copy_bandwidth(torch, lbm, nbytes=2 << 30, reps=5, grids=(2048, 4096, 8192, 16384, 32768)):
    """Measured HBM ceiling: the library's streaming copy (16-byte non-temporal loads
    and stores, every byte read once and written once) of nbytes, timed with HIP
    events over `reps` copies for each workgroup count; GB/s = 2 nbytes / time.
    Returns the best rate, the per-grid rates and torch's own copy_ for reference."""
    n = nbytes // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    st = torch.cuda.current_stream()
    per = {}
    for g in grids:
        lbm.stream_copy(b, a, nbytes, g, st)
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        t0.record(st)
        for _ in range(reps):
            lbm.stream_copy(b, a, nbytes, g, st)
        t1.record(st)
        t1.synchronize()
        per[g] = 2.0 * nbytes / (t0.elapsed_time(t1) / reps * 1e-3) / 1e9
    if not torch.equal(a, b):
        raise RuntimeError("stream copy produced wrong data")
    b.copy_(a)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(st)
    for _ in range(reps):
        b.copy_(a)
    t1.record(st)
    t1.synchronize()
    torch_copy = 2.0 * nbytes / (t0.elapsed_time(t1) / reps * 1e-3) / 1e9
    del a, b
    best = max(per, key=per.get)
    return {"GBps": per[best], "grid": best, "per_grid": per, "bytes_each_way": nbytes,
            "torch_copy_GBps": torch_copy}


def cpu_baseline_worker(side: int, steps: int):
    """Oracle timing on a bounded sample (runs in a child with one BLAS/OpenMP thread)."""
    from oracle import lattice as olat
    from oracle import lbm as olbm
    from oracle import thermo as oth
    from paper_1909_12390_amd import inputs

    class _Oracle:
        def critical_temperature(self, mix):
            return oth.Mixture(**mix).Tc

        def bubble_pressure(self, mix, T, z):
            return oth.bubble_pressure(oth.Mixture(**mix), T, z)

        def dew_pressure(self, mix, T, z):
            return oth.dew_pressure(oth.Mixture(**mix), T, z)

        def flash(self, mix, T, p, z):
            return oth.flash(oth.Mixture(**mix), T, p, z)

        def pressure(self, mix, T, n):
            import numpy as _np
            m = oth.Mixture(**mix)
            n = _np.atleast_2d(_np.asarray(n, dtype=_np.float64))
            return _np.where((n @ m.b) < 1.0, oth.pressure_molar(n.T, T, m), _np.nan)

    cfg = inputs.config_c3(_Oracle(), shape=(side, side, side), R0=side / 4.0)
    lat = olat.d3q19()
    prm = olbm.StepParams(T=cfg.T, tau=cfg.tau, gamma=cfg.gamma, beta=cfg.beta, collision=cfg.collision,
                          forcing=cfg.forcing, mrt_s=cfg.mrt_s)
    mix = oth.Mixture(**cfg.mix)
    f = olbm.init_populations(cfg.rho0, lat)
    f = olbm.step(f, mix, prm, lat)            # warm-up
    t0 = time.perf_counter()
    for _ in range(steps):
        f = olbm.step(f, mix, prm, lat)
    dt = time.perf_counter() - t0
    cells = side ** 3
    print(json.dumps({"value": cells * cfg.nc * steps / dt / 1e6, "seconds": dt}))


def cpu_baseline(side: int, steps: int):
    env = dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1", MKL_NUM_THREADS="1",
               HIP_VISIBLE_DEVICES="", CUDA_VISIBLE_DEVICES="")
    res = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-worker",
                          "--cpu-side", str(side), "--cpu-steps", str(steps)],
                         capture_output=True, text=True, env=env, timeout=600)
    if res.returncode != 0:
        sys.stderr.write(res.stderr)
        return None
    rec = json.loads(res.stdout.strip().splitlines()[-1])
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": rec["value"], "unit": "MLUPS×components", "cores": 1, "kind": "oracle",
            "sample": f"same four-component D3Q19 MRT+EDM mixture on a {side}^3 periodic box, "
                      f"{steps} steps after 1 warm-up step, float64 NumPy, one thread "
                      f"({rec['seconds']:.1f} s)",
            "cpu_model": model, "host_cpu_count": os.cpu_count()}


def batched_section(args, torch, lbm, inputs):
    """Many independent D2Q9 boxes (sides from {32, 48, 64, 96, 128}, binary or
    ternary, own T and composition), one launch per pass per step, K steps per HIP
    graph, workgroup size from the autotuner.  Reports throughput and, after
    --batch-precision-steps steps, the bulk phase mole-fraction error of the float32
    and float16 storage against the float64 path, box by box."""
    from paper_1909_12390_amd import autotune
    cfgs = inputs.config_c4_boxes(lbm.LibThermo(), nboxes=args.batch_boxes)
    boxes = [{"mix": c.mix, "shape": c.shape, "T": c.T, "tau": c.tau, "beta": c.beta, "gamma": c.gamma,
              "rho0": c.rho0, "R0": c.geometry["R0"]} for c in cfgs]
    cells = sum(c.cells for c in cfgs)
    comp_cells = sum(c.cells * c.nc for c in cfgs)
    tunes = {st: autotune.tune_batch(boxes, "D2Q9", "bgk", "edm", st, steps=20) for st in ("f32", "f16", "f64")}
    res = {"workload": f"{len(boxes)} independent D2Q9 boxes, sides from {{32,48,64,96,128}}, binary or ternary, "
                       f"BGK + exact-difference forcing, own T and composition per box",
           "boxes": len(boxes), "cells": cells, "component_cells": comp_cells, "autotune": tunes}
    graph_steps = 100
    for storage in ("f32", "f16", "f64"):
        tune = tunes[storage]
        b = lbm.LbmBatch(boxes, "D2Q9", collision="bgk", forcing="edm", storage=storage, tile=tune["tile"],
                         grid=tune["grid"], graph_steps=graph_steps)
        b.step(2 * graph_steps)
        b.check()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(b.stream)
        b.step(args.batch_steps)
        stop.record(b.stream)
        stop.synchronize()
        ms = start.elapsed_time(stop) / args.batch_steps
        b.check()
        s = STORAGE_BYTES[storage]
        alg = sum(c.cells * (2 * c.nc * 9 * s + 16 + (8 * c.nc if storage != "f64" else 0)) for c in cfgs)
        res[storage] = {"ms_per_step": ms, "mlups_x_comp": comp_cells / (ms * 1e-3) / 1e6,
                        "alg_GBps": alg / (ms * 1e-3) / 1e9}
        b.close()
        del b
        torch.cuda.empty_cache()
    # the one-launch step (psi of each tile and its neighbours in LDS), at its own
    # tuned launch shape, beside the two launches
    res["fused"] = {"step": "one launch per step, psi of each tile and its neighbours computed into LDS"}
    for storage in ("f32", "f16"):
        tune = autotune.tune_batch(boxes, "D2Q9", "bgk", "edm", storage, steps=20, fused=True)
        b = lbm.LbmBatch(boxes, "D2Q9", collision="bgk", forcing="edm", storage=storage, tile=tune["tile"],
                         grid=tune["grid"], graph_steps=graph_steps, fused=True)
        b.step(2 * graph_steps)
        b.check()
        start = torch.cuda.Event(enable_timing=True)
        stop = torch.cuda.Event(enable_timing=True)
        start.record(b.stream)
        b.step(args.batch_steps)
        stop.record(b.stream)
        stop.synchronize()
        ms = start.elapsed_time(stop) / args.batch_steps
        b.check()
        res["fused"][storage] = {"ms_per_step": ms, "mlups_x_comp": comp_cells / (ms * 1e-3) / 1e6,
                                 "tile": tune["tile"], "grid": tune["grid"],
                                 "time_vs_two_launches": ms / res[storage]["ms_per_step"]}
        b.close()
        del b
        torch.cuda.empty_cache()
    if args.batch_precision_steps > 0:
        fr = {}
        for storage in ("f64", "f32", "f16"):
            b = lbm.LbmBatch(boxes, "D2Q9", collision="bgk", forcing="edm", storage=storage,
                             tile=tunes[storage]["tile"], grid=tunes[storage]["grid"], graph_steps=graph_steps)
            b.step(args.batch_precision_steps)
            bad = b.box_errors()
            if bad.any():
                raise RuntimeError(f"{storage}: boxes {np.nonzero(bad)[0].tolist()} left the EOS domain")
            b.check()
            rho = b.fields()
            fr[storage] = [phase_mole_fractions(r, bx["mix"]["M"], {"R0": bx["R0"]}, bx["shape"])
                           for r, bx in zip(rho, boxes)]
            for ph, bx in zip(fr[storage], boxes):
                try:
                    ph["fl"], ph["fv"], ph["residual"], _ = fugacities(lbm, bx["mix"], bx["T"], ph["n_liquid"],
                                                                       ph["n_vapor"])
                except lbm.LbmError:       # a mask state with p_EOS <= 0: no bulk phase there (e.g. the drop left)
                    ph["fl"] = None
            b.close()
            del b, rho
            torch.cuda.empty_cache()
        for storage in ("f32", "f16"):
            e = np.array([max(float(np.max(np.abs(a[ph] - c[ph]))) for ph in ("liquid", "vapor"))
                          for a, c in zip(fr[storage], fr["f64"])])
            res[f"{storage}_max_abs_molefrac_err_vs_f64"] = float(e.max())
            res[f"{storage}_median_abs_molefrac_err_vs_f64"] = float(np.median(e))
            res[f"{storage}_boxes_over_1e-4"] = int((e > 1e-4).sum())
            res[f"{storage}_worst_box"] = int(np.argmax(e))
            ok = [(a, c) for a, c in zip(fr[storage], fr["f64"]) if a["fl"] is not None and c["fl"] is not None]
            ef = np.array([max(float(np.max(np.abs(a[k] / c[k] - 1.0))) for k in ("fl", "fv")) for a, c in ok])
            res[f"{storage}_max_rel_fugacity_err_vs_f64"] = float(ef.max())
            res[f"{storage}_median_rel_fugacity_err_vs_f64"] = float(np.median(ef))
            res[f"{storage}_max_residual_eq_error"] = float(max(a["residual"] for a, _ in ok))
        good = [a["residual"] for a in fr["f64"] if a["fl"] is not None]
        res["boxes_without_two_bulk_phases"] = len(boxes) - len(good)
        res["f64_max_residual_eq_error"] = float(max(good))
        res["f64_median_residual_eq_error"] = float(np.median(good))
        res["precision_steps"] = args.batch_precision_steps
    return res


def slab_section(args, torch, lbm, inputs):
    """The ternary 256^2 slab (MRT + exact-difference forcing) for its configured
    steps in float64 and float32 storage: bulk phases on fixed masks (liquid
    |y - y_c| <= H/8, vapour |y - y_c| >= 3H/8) against the flash at the LB's bulk
    pressure and overall composition, the Eq. (error) residual of the bulk states,
    and the float32 run's mole-fraction and fugacity errors against float64."""
    th = lbm.LibThermo()
    cfg = inputs.config_c2(th)
    M = np.asarray(cfg.mix["M"], dtype=np.float64)
    ny = cfg.shape[0]
    y = np.arange(ny) - ny / 2.0
    liq, vap = np.abs(y) <= ny / 8.0, np.abs(y) >= 3.0 * ny / 8.0
    res = {"workload": f"ternary D2Q9 {ny}x{cfg.shape[1]} slab of half the height, MRT + exact-difference "
                       f"forcing, beta {cfg.beta}, {cfg.steps} steps", "steps": cfg.steps, "beta": cfg.beta}
    out = {}
    for storage in ("f64", "f32"):
        c = lbm.LbmContext(cfg.mix, cfg.lattice, cfg.shape, cfg.T, cfg.tau, cfg.beta, cfg.gamma, cfg.rho0,
                           collision=cfg.collision, forcing=cfg.forcing, storage=storage, mrt_s=cfg.mrt_s,
                           graph_steps=1000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c.step(cfg.steps)
        c.check()
        ms = (time.perf_counter() - t0) * 1e3
        rho = c.moments(totals=False)["rho_s"].cpu().numpy()
        c.close()
        n = rho / M[:, None, None]
        nl, nv = n[:, liq, :].mean(axis=(1, 2)), n[:, vap, :].mean(axis=(1, 2))
        fl, fv, resid, p_lb = fugacities(lbm, cfg.mix, cfg.T, nl, nv)
        nt = n.reshape(cfg.nc, -1).sum(axis=1)
        out[storage] = {"x": nl / nl.sum(), "y": nv / nv.sum(), "fl": fl, "fv": fv, "residual": resid,
                        "p": p_lb, "z": nt / nt.sum()}
        res[storage] = {"ms_total": ms, "ms_per_step": ms / cfg.steps, "x": (nl / nl.sum()).tolist(),
                        "y": (nv / nv.sum()).tolist(), "residual_eq_error": resid, "p_lb": p_lb}
    r = out["f64"]
    fl = lbm.lbm_flash(cfg.mix, cfg.T, r["p"], r["z"])
    res["flash_at_lb_pressure"] = {"x": list(fl.x), "y": list(fl.y)}
    for storage in ("f64", "f32"):
        o = out[storage]
        res[storage]["max_rel_err_vs_flash"] = float(max(np.max(np.abs(o["x"] - np.asarray(fl.x)) / np.asarray(fl.x)),
                                                         np.max(np.abs(o["y"] - np.asarray(fl.y)) / np.asarray(fl.y))))
    f32 = out["f32"]
    res["f32_max_abs_molefrac_err_vs_f64"] = float(max(np.max(np.abs(f32["x"] - r["x"])),
                                                       np.max(np.abs(f32["y"] - r["y"]))))
    res["f32_max_rel_fugacity_err_vs_f64"] = float(max(np.max(np.abs(f32[k] / r[k] - 1.0)) for k in ("fl", "fv")))
    return res


def adjoint_section(args, torch, lbm, inputs):
    """Gradient of the liquid-composition loss on the ternary D2Q9 128^2 drop:
    wall time of a forward-only run and of the checkpointed forward + reverse
    (lbm_adjoint), float32 and float64 storage, and the float32 gradient's
    relative difference from the float64 one.  The forward steps replay HIP graphs
    of one checkpoint interval (the box is small enough for launches to dominate)."""
    from paper_1909_12390_amd import adjoint as padj
    cfg = inputs.config_c5(lbm.LibThermo())
    mask = inputs.drop_mask(cfg.shape, cfg.geometry["R0"])
    x_tgt = inputs.adjoint_target(cfg)
    res = {"workload": f"ternary D2Q9 {cfg.shape[0]}x{cfg.shape[1]} drop, BGK + exact-difference forcing, "
                       f"{args.adjoint_steps} steps, checkpoint every {args.adjoint_every}, "
                       f"loss = squared liquid mole-fraction mismatch",
           "steps": args.adjoint_steps, "checkpoint_every": args.adjoint_every,
           "graph_steps": args.adjoint_every}
    grads = {}
    for storage in ("f32", "f64"):
        def ctx():
            return lbm.LbmContext(cfg.mix, "D2Q9", cfg.shape, cfg.T, cfg.tau, cfg.beta, cfg.gamma, cfg.rho0,
                                  collision="bgk", forcing="edm", storage=storage, graph_steps=args.adjoint_every)
        c = ctx()
        c.step(2 * args.adjoint_every)            # warm-up, captures both graphs
        c.check()
        t0 = time.perf_counter()
        c.step(args.adjoint_steps)
        c.check()
        fwd = (time.perf_counter() - t0) * 1e3
        c.close()
        c = ctx()
        c.adjoint(20, 10, mask, x_tgt)            # warm-up (workspace, code objects)
        c.close()
        c = ctx()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = c.adjoint(args.adjoint_steps, args.adjoint_every, mask, x_tgt)
        full = (time.perf_counter() - t0) * 1e3
        c.close()
        grads[storage] = padj.pack_gradient(r["d_k"], r["d_a"], r["d_b"])
        res[storage] = {"forward_ms": fwd, "forward_plus_adjoint_ms": full, "ratio": full / fwd,
                        "loss": r["loss"], "x_liq": r["x_liq"].tolist()}
    res["gradient_f64"] = grads["f64"].tolist()
    res["f32_gradient_max_rel_diff_vs_f64"] = float(np.max(np.abs(grads["f32"] - grads["f64"]))
                                                    / np.max(np.abs(grads["f64"])))
    return res


def walls_section(args, torch, lbm, inputs, cfg, make, timed, modes_res):
    """The headline drop inside a synthetic porous medium (random overlapping
    spheres, periodic) with halfway bounce-back walls and psi_w midway between the
    vapour's and the liquid's psi (psi_w at the vapour's repels the liquid cut by
    the spheres out of the EOS domain in the first step, oracle and GPU alike):
    time per step against the same step without walls, float16 and float64
    storage; throughput counted over all cells and over the fluid cells."""
    solid = inputs.porous_spheres(cfg.shape, args.walls_solid, args.walls_radius, seed=0)
    probe = make("f64", "two_pass")
    psi = probe.moments(fields=True, totals=False)["psi"]
    h = cfg.shape[0] // 2
    psi_w = 0.5 * float(psi[0, 0, 0].item() + psi[h, h, h].item())
    del probe, psi
    torch.cuda.empty_cache()
    fluid = int((~solid).sum())
    res = {"workload": f"{cfg.nc}-component D3Q19 {cfg.shape[0]}^3 drop in random overlapping spheres "
                       f"(radius {args.walls_radius}, solid fraction {solid.mean():.3f}), halfway bounce-back, "
                       f"psi_w midway between the phases' psi, two_pass schedule",
           "solid_fraction": float(solid.mean()), "psi_wall": psi_w, "steps": args.walls_steps}
    for m in ("f16", "f64"):
        c = make(m, "two_pass")
        c.set_solid(solid, psi_w)
        m0 = c.moments(fields=False)["mass"]
        w, k = timed(c, args.walls_steps, args.warmup, args.diag_every)
        drift = float(np.max(np.abs(c.moments(fields=False)["mass"] / m0 - 1)))
        ms = w / args.walls_steps
        r = {"ms_per_step": ms, "kernel_ms": [x / args.walls_steps for x in k],
             "mlups_x_comp_all_cells": cfg.cells * cfg.nc / (ms * 1e-3) / 1e6,
             "mlups_x_comp_fluid_cells": fluid * cfg.nc / (ms * 1e-3) / 1e6, "mass_drift_rel": drift}
        ref = modes_res.get(f"{m}/two_pass") if modes_res else None
        if ref is None:
            c0 = make(m, "two_pass")
            w0, _ = timed(c0, args.walls_steps, args.warmup, args.diag_every)
            ref = {"ms_per_step": w0 / args.walls_steps}
            del c0
        r["no_walls_ms_per_step"] = ref["ms_per_step"]
        r["time_ratio_vs_no_walls"] = ms / ref["ms_per_step"]
        res[m] = r
        del c
        torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--storage", default="f16", choices=list(STORAGE_BYTES))
    ap.add_argument("--schedule", default="two_pass", choices=["two_pass", "blocked", "overlap"])
    ap.add_argument("--slab-planes", type=int, default=0, help="blocked schedule: planes per slab (0 = auto)")
    ap.add_argument("--side", type=int, default=128)
    ap.add_argument("--diag-every", type=int, default=100)
    ap.add_argument("--modes", default="f64,f32,f16", help="storage modes also timed (comma list, '' = none)")
    ap.add_argument("--precision-steps", type=int, default=5000,
                    help="steps run per storage mode for the mole-fraction error (0 = skip)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-side", type=int, default=64)
    ap.add_argument("--cpu-steps", type=int, default=60)
    ap.add_argument("--cpu-baseline-worker", action="store_true")
    ap.add_argument("--no-copy", action="store_true")
    ap.add_argument("--no-slab", dest="slab", action="store_false", help="skip the ternary slab section")
    ap.add_argument("--tune-single", action="store_true",
                    help="also time every single-box schedule per storage mode (autotune.tune_single)")
    ap.add_argument("--batch-boxes", type=int, default=512, help="batched section: number of boxes (0 = skip)")
    ap.add_argument("--batch-steps", type=int, default=500)
    ap.add_argument("--batch-precision-steps", type=int, default=10000)
    ap.add_argument("--adjoint-steps", type=int, default=2000, help="adjoint section: steps (0 = skip)")
    ap.add_argument("--adjoint-every", type=int, default=100, help="adjoint section: checkpoint interval")
    ap.add_argument("--walls-steps", type=int, default=200, help="porous-medium walls section: steps (0 = skip)")
    ap.add_argument("--walls-solid", type=float, default=0.3, help="walls section: solid fraction")
    ap.add_argument("--walls-radius", type=float, default=6.0, help="walls section: sphere radius (cells)")
    args = ap.parse_args()

    if args.cpu_baseline_worker:
        cpu_baseline_worker(args.cpu_side, args.cpu_steps)
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the multi-GPU sharding "
              f"(boxes across GPUs, z-slabs with halo exchange) is designed but not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1909_12390_amd import inputs, lbm

    torch.cuda.set_device(0)
    side = args.side
    cfg = inputs.config_c3(lbm.LibThermo(), shape=(side, side, side), R0=side / 4.0)
    nc, Q, cells = cfg.nc, 19, cfg.cells
    rho0 = torch.as_tensor(cfg.rho0, dtype=torch.float64, device="cuda")

    def make(storage, schedule=None, slab=None):
        return lbm.LbmContext(cfg.mix, "D3Q19", cfg.shape, cfg.T, cfg.tau, cfg.beta, cfg.gamma, rho0,
                              collision=cfg.collision, forcing=cfg.forcing, storage=storage,
                              schedule=schedule or args.schedule, mrt_s=cfg.mrt_s,
                              slab_planes=args.slab_planes if slab is None else slab)

    def timed(ctx, steps, warmup, diag_every):
        """Time exactly `steps` steps (HIP events around every kernel; totals every
        diag_every steps).  Returns wall ms, summed kernel ms."""
        ctx.step(warmup)
        ctx.check()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kms = [0.0, 0.0]
        done = 0
        while done < steps:
            n = min(diag_every, steps - done)
            a, b = ctx.step_timed(n)
            kms[0] += a
            kms[1] += b
            done += n
            if done % diag_every == 0:
                ctx.moments(fields=False, totals=True)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        ctx.check()
        return wall, kms

    def plain(ctx, steps, warmup, diag_every):
        """Time exactly `steps` plain lbm_step calls (conservation totals every
        diag_every steps) between two HIP events on the context's stream, bracketed
        by device synchronisation; returns (wall ms, event ms)."""
        ctx.step(warmup)
        ctx.check()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(ctx.stream)
        done = 0
        while done < steps:
            n = min(diag_every, steps - done)
            ctx.step(n)
            done += n
            if done % diag_every == 0:
                ctx.moments(fields=False, totals=True)
        e1.record(ctx.stream)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) * 1e3
        ctx.check()
        return wall, e0.elapsed_time(e1)

    def measure(ctx, steps, warmup, diag_every):
        """Plain-step wall time of `steps` steps, then the per-kernel split from a
        second pass of the same length: (wall ms, [psi ms, collide ms])."""
        w, _ = plain(ctx, steps, warmup, diag_every)
        _, k = timed(ctx, steps, 0, diag_every)
        return w, k

    # the measured copy ceiling first (it also brings the device out of idle)
    copy = None if args.no_copy else copy_bandwidth(torch, lbm)

    # headline: the chosen storage mode, plain steps between two events
    ctx = make(args.storage)
    t_start_mass = ctx.moments(fields=False)["mass"]
    wall_ms, event_ms = plain(ctx, args.steps, args.warmup, args.diag_every)
    mass_drift = float(np.max(np.abs(ctx.moments(fields=False)["mass"] / t_start_mass - 1)))
    ms_per_step = wall_ms / args.steps
    value = cells * nc * args.steps / (wall_ms * 1e-3) / 1e6
    # per-kernel split from a separate pass of the same length with HIP events around
    # every launch on the context's stream
    split_wall, kms = timed(ctx, args.steps, 0, args.diag_every)
    # dominant kernel: the collide pass (it carries all but the psi write of b_alg)
    kname = "k_collide"
    avg_ms = kms[1] / args.steps                      # collide time per step (all slabs)
    bytes_launch = b_alg_collide(nc, Q, args.storage) * cells
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    key = f"{kname}:{args.schedule}:{args.storage}:D3Q19:nc{nc}:{side}^3"
    prof = measured_profile(key)
    traffic = prof.get("bytes_per_launch")
    del ctx
    torch.cuda.empty_cache()

    out = {
        "metric": METRIC, "value": value, "unit": "MLUPS×components", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.storage != "f64" else "f64", "data": "synthetic",
        "config": {"workload": f"four-component D3Q19 {side}^3 drop (R0={side // 4}), MRT + exact-difference "
                               f"forcing, one supercritical component, {args.storage} population storage "
                               f"(float64 EOS/psi), {args.schedule} schedule",
                   "lattice": "D3Q19", "shape": [side] * 3, "nc": nc, "collision": cfg.collision,
                   "forcing": cfg.forcing, "storage": args.storage, "schedule": args.schedule,
                   "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
                     "frac": achieved / PEAK_HBM_GBS,
                     "traffic": None if traffic is None else traffic / (avg_ms * 1e-3) / 1e9,
                     "kernel": kname, "kernel_ms_per_step": avg_ms,
                     "kernel_alg_bytes_per_cell": b_alg_collide(nc, Q, args.storage),
                     "cells_per_step": cells, "traffic_bytes_per_step": traffic,
                     "pipe_busy": prof.get("pipe_busy"),
                     "frac_of_measured_copy": None if copy is None else achieved / copy["GBps"]},
        "event_ms_per_step": event_ms / args.steps,
        "step_alg_GBps": b_alg(nc, Q, args.storage) * cells / (ms_per_step * 1e-3) / 1e9,
        "step_alg_bytes_per_cell": b_alg(nc, Q, args.storage),
        "kernel_ms_per_step": {"psi": kms[0] / args.steps, "collide": kms[1] / args.steps,
                               "split_pass_wall_ms_per_step": split_wall / args.steps},
        "mass_drift_rel": mass_drift,
    }
    if copy is not None:
        out["copy_GBps"] = copy["GBps"]
        out["copy"] = copy

    def progress(what):
        print(f"bench: {what} done", file=sys.stderr, flush=True)

    progress("headline")

    modes = [m for m in args.modes.split(",") if m]
    res = {}
    if modes:
        for m in modes:
            for sched in ("two_pass", "blocked", "overlap"):
                c = make(m, sched)
                w, k = measure(c, args.steps, args.warmup, args.diag_every)
                res[f"{m}/{sched}"] = {
                    "ms_per_step": w / args.steps, "mlups_x_comp": cells * nc * args.steps / (w * 1e-3) / 1e6,
                    "kernel_ms": [x / args.steps for x in k],
                    "alg_GBps_step": b_alg(nc, Q, m) * cells / (w / args.steps * 1e-3) / 1e9}
                del c
                torch.cuda.empty_cache()
        ref = res.get("f64/two_pass")
        if ref:
            for key in res:
                res[key]["speedup_vs_f64_two_pass"] = ref["ms_per_step"] / res[key]["ms_per_step"]
        out["modes"] = res
        progress("modes")

    if args.tune_single:
        from paper_1909_12390_amd import autotune
        out["single_box_autotune"] = {
            m: autotune.tune_single(lambda sched, slab, m=m: make(m, sched, slab), steps=args.steps)
            for m in [x for x in args.modes.split(",") if x]}
        progress("single-box autotune")

    if args.precision_steps > 0:
        prec = {"steps": args.precision_steps}
        fr = {}
        for m in ("f64", "f32", "f16"):
            c = make(m)
            c.step(args.precision_steps)
            mo = c.moments(fields=True, totals=False)
            c.check()
            fr[m] = phase_mole_fractions(mo["rho_s"], cfg.mix["M"], cfg.geometry, cfg.shape)
            fr[m]["fl"], fr[m]["fv"], fr[m]["residual"], _ = fugacities(lbm, cfg.mix, cfg.T, fr[m]["n_liquid"],
                                                                        fr[m]["n_vapor"])
            del c, mo
            torch.cuda.empty_cache()
        for m in ("f32", "f16"):
            prec[f"{m}_max_abs_molefrac_err_vs_f64"] = float(max(
                np.max(np.abs(fr[m][ph] - fr["f64"][ph])) for ph in ("liquid", "vapor")))
            prec[f"{m}_max_rel_fugacity_err_vs_f64"] = float(max(
                np.max(np.abs(fr[m][k] / fr["f64"][k] - 1.0)) for k in ("fl", "fv")))
            prec[f"{m}_residual_eq_error"] = fr[m]["residual"]
        prec["f64_residual_eq_error"] = fr["f64"]["residual"]
        prec["f64_liquid_x"] = fr["f64"]["liquid"].tolist()
        prec["f64_vapor_y"] = fr["f64"]["vapor"].tolist()
        out["precision"] = prec
        progress("precision")

    if args.walls_steps > 0:
        out["walls"] = walls_section(args, torch, lbm, inputs, cfg, make, measure, res)
        progress("walls")

    if args.slab:
        out["slab"] = slab_section(args, torch, lbm, inputs)
        progress("ternary slab")

    if args.batch_boxes > 0:
        out["batched"] = batched_section(args, torch, lbm, inputs)
        progress("batched")

    if args.adjoint_steps > 0:
        out["adjoint"] = adjoint_section(args, torch, lbm, inputs)
        progress("adjoint")

    if not args.no_cpu_baseline:
        cb = cpu_baseline(args.cpu_side, args.cpu_steps)
        if cb and cb.get("value"):
            # GPU over the float64 oracle on the same mixture: at the same precision
            # (the float64 GPU step) and for the headline storage
            cb["gpu_over_oracle"] = {"headline": out["value"] / cb["value"]}
            f64 = out.get("modes", {}).get("f64/two_pass")
            if f64:
                cb["gpu_over_oracle"]["f64"] = f64["mlups_x_comp"] / cb["value"]
        out["cpu_baseline"] = cb
        progress("cpu baseline")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
