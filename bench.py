#!/usr/bin/env python3
"""Throughput of the chunked leapfrog wave stencil on one MI355X.

One bench step = one full run of the headline workload: 1000 leapfrog
steps of the 8192 x 8192 row share (rows [8192, 16384) of a 32768 x 8192
domain, Dirichlet zero outside the share) split into 4 device-local chunks,
halo exchanges included, through ccl_wave_step.  Inputs are resident in HBM
before the timed region; the timed region is bracketed by synchronisation.

The launch config (temporal depth T, rows per tile) is the fastest, as
measured, of the learned cost model's three best candidates when a trained
model is present, else the best of a quick autotuner sweep; ``--depth``
(with ``--tile-rows``, 0 = automatic) overrides both.  Besides the
headline ("tuned") form the line reports the plain form (T = 1), device
energy per step, the 64-grid batched workload run as one graph launch
against per-grid loops, the 768^3 workload (swept vs learned), and the
headline share with float64 and 16-bit fields (roofline fraction on each
type's own bytes).

Prints one JSON line; value = Mcells/s (cell updates per second / 1e6).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, published
MODEL_PATH = os.path.join(ROOT, "paper_2505_06022_amd", "costmodel.json")


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def load_traffic(depth: int, rows: int, path: str | None = None):
    """HBM bytes per stencil launch from the committed rocprofv3 counter
    summary (one section per profiled launch configuration), if one was
    taken on the current kernel source and this config."""
    from paper_2505_06022_amd.profile_run import kernel_source_hash
    path = path or os.path.join(ROOT, "profiles", "traffic_wave2d_8192_share_k4.md")
    try:
        with open(path) as f:
            docs = [json.loads(l[len("traffic-json: "):]) for l in f
                    if l.startswith("traffic-json: ")]
    except (OSError, ValueError):
        return None
    for doc in docs:
        if (doc.get("kernel_hash") == kernel_source_hash() and doc.get("depth") == depth
                and doc.get("tile_rows") == rows):
            return doc.get("bytes_per_launch")
    return None


def host_cpu_model() -> str:
    """The host CPU's model name (from /proc/cpuinfo) and logical CPU count."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{name}, {os.cpu_count()} logical CPUs visible"


def _oracle_rate(u_prev, u_cur, r2, steps, threads, seconds):
    """Mcells/s of the oracle stepping (u_prev, u_cur): `steps` steps when they
    fit in about `seconds`, else as many as fit; repeated while time is left
    (at most 5 runs).  Returns (Mcells/s, steps per run, runs, seconds)."""
    import numpy as np

    import oracle
    oracle.wave(u_prev, u_cur, r2, 2, threads=threads)  # page in, spin up threads
    t0 = time.perf_counter()
    oracle.wave(u_prev, u_cur, r2, 10, threads=threads)
    per_step = max((time.perf_counter() - t0) / 10, 1e-6)
    n = int(max(10, min(steps, seconds / per_step)))
    runs, dt = 0, 0.0
    while runs < 5 and (runs == 0 or dt < seconds):
        t0 = time.perf_counter()
        oracle.wave(u_prev, u_cur, r2, n, threads=threads)
        dt += time.perf_counter() - t0
        runs += 1
    return float(np.prod(u_cur.shape)) * n * runs / dt / 1e6, n, runs, dt


def cpu_baseline(w, seconds: float = 12.0):
    """The oracle on the host cores over bounded samples of the workloads.

    `value`: the float32 oracle on the 8192 x 8192 share (the whole 1000
    steps when they fit in about `seconds`, else as many steps as fit),
    repeated while time is left.  Beside it, shorter samples of the float64
    oracle on the same share, of the float32 oracle on the 768^3 workload,
    and of the float32 oracle on grids of the 64-grid batch."""
    import numpy as np

    import oracle
    import synth
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or oracle.max_threads()
    u0 = synth.gaussian_field(w["shape"], w["sigma"], w["seed"])
    rate, n, runs, dt = _oracle_rate(u0.copy(), u0, w["r2"], w["steps"], threads, seconds)
    what = ("the whole workload" if n == w["steps"] else
            f"{n} of the workload's {w['steps']} steps")
    out = {"value": round(rate, 1), "unit": "Mcells/s", "cores": threads, "kind": "oracle",
           "host_cpu": host_cpu_model(),
           "sample": f"float32 oracle, {w['shape'][0]}x{w['shape'][1]} share, {what} "
                     f"x {runs}, {dt:.1f} s on {threads} host threads"}
    u64 = u0.astype(np.float64)
    rate, n, runs, dt = _oracle_rate(u64.copy(), u64, w["r2"], w["steps"], threads, 4.0)
    out["fp64_share"] = {"mcells": round(rate, 1),
                         "sample": f"float64 oracle, same share, {n} steps x {runs}, "
                                   f"{dt:.1f} s"}
    del u0, u64
    w3 = synth.WORKLOADS["wave3d_768_k8"]
    v0 = synth.gaussian_field(w3["shape"], w3["sigma"], w3["seed"])
    rate, n, runs, dt = _oracle_rate(v0.copy(), v0, w3["r2"], w3["steps"], threads, 4.0)
    out["wave3d_768"] = {"mcells": round(rate, 1),
                         "sample": f"float32 oracle, 768^3, {n} of 200 steps x {runs}, "
                                   f"{dt:.1f} s"}
    del v0
    # the batch: its first 8 grids, each for its own step count when it fits
    cells_steps, t_total = 0.0, 0.0
    for d in synth.batched_grids()[:8]:
        g0 = synth.gaussian_field((d["ny"], d["nx"]), d["sigma"], d["seed"])
        rate, n, runs, dt = _oracle_rate(g0.copy(), g0, 0.25, d["steps"], threads, 0.5)
        cells_steps += d["ny"] * d["nx"] * n * runs
        t_total += dt
    out["batched_64"] = {"mcells": round(cells_steps / t_total / 1e6, 1),
                         "sample": f"float32 oracle, the batch's first 8 grids, "
                                   f"{t_total:.1f} s"}
    return out


def saxpy_calibration(n: int = 1 << 28, reps: int = 10):
    import torch

    import paper_2505_06022_amd as ccl
    x = torch.rand(n, device="cuda")
    y = torch.rand(n, device="cuda")
    z = torch.empty(n, device="cuda")
    ccl.ccl_saxpy(n, 2.0, x.data_ptr(), y.data_ptr(), z.data_ptr())
    torch.cuda.synchronize()
    ccl.ccl_timing_enable(True)
    for _ in range(reps):
        ccl.ccl_saxpy(n, 2.0, x.data_ptr(), y.data_ptr(), z.data_ptr())
    torch.cuda.synchronize()
    launches, ms = ccl.ccl_timing_query(ccl.CCL_KERNEL_SAXPY)
    ccl.ccl_timing_enable(False)
    del x, y, z
    return 12.0 * n / (ms / launches * 1e-3) / 1e9


def average_power(run_once, min_span=2.0, limit=30.0):
    """Mean device power (W) over back-to-back runs, between two updates of
    the device energy counter at least `min_span` s apart by the counter's
    own timestamps (the counter advances in coarse steps, so the window is
    aligned to its updates; an update is a change of the energy value)."""
    import torch

    import paper_2505_06022_amd as ccl
    prev, _ = ccl.ccl_energy_read(0, None)
    first = None
    t0 = time.perf_counter()
    while True:
        run_once()
        torch.cuda.synchronize()
        e, ts = ccl.ccl_energy_read(0, None)
        if e != prev:
            if first is None or e < first[0] or ts <= first[1]:
                first = (e, ts)  # first update seen (or the counter went back)
            elif (ts - first[1]) * 1e-9 >= min_span:
                return (e - first[0]) / ((ts - first[1]) * 1e-9)
        prev = e
        if time.perf_counter() - t0 > limit:
            raise RuntimeError("energy counter did not advance")


def pick_config(w, args):
    """(T, rows, how) for the headline share."""
    if args.depth:
        return args.depth, args.tile_rows, "given"
    from paper_2505_06022_amd import tune
    return tune.launch_config(w["shape"], w["chunks"], w["steps"], w["r2"],
                              model_path=None if args.sweep else MODEL_PATH)


def time_runs(cw, steps, runs):
    import torch
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    a = torch.cuda.Event(enable_timing=True)
    b = torch.cuda.Event(enable_timing=True)
    a.record(stream)
    for _ in range(runs):
        cw.step(steps)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) * 1e-3


def batched_forms(log_energy=False):
    """The 64-grid workload, each form on the same data:
    * batched: one graph launch of the persistent kernel (per-grid depth
      picked by the cost model, else T=4; tile rows sized by the batch);
    * batched_per_grid: one graph launch holding every grid's own
      ccl_wave_step sequence (the cost model's depth and rows per grid);
    * per_grid_learned_loop: a host loop of ordinary ccl_wave_step calls, one
      per grid, with the same per-grid depth and rows and no graph (the same
      work as batched_per_grid, launched one call at a time: the gain of the
      graph launch over it is the gain of batching itself);
    * per_grid_loop: a host loop of plain T=1 ccl_wave_step calls."""
    import torch

    import paper_2505_06022_amd as ccl
    import synth
    from paper_2505_06022_amd import tune
    from paper_2505_06022_amd.fields import BatchedWaves, ChunkedWave
    grids = synth.batched_grids()
    specs, specs_pg, how = tune.batch_specs(grids, MODEL_PATH)
    cell_steps = sum(d["ny"] * d["nx"] * d["steps"] for d in grids)

    def run_batch(sp, flags):
        bw = BatchedWaves(sp, flags=flags)
        for g, d in enumerate(grids):
            u0 = synth.gaussian_field((d["ny"], d["nx"]), d["sigma"], d["seed"])
            bw.scatter(g, u0, u0)
        torch.cuda.synchronize()
        bw.run()
        ccl.ccl_batch_check(bw.handle)
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        reps = 3
        a.record()
        for _ in range(reps):
            bw.run()
        b.record()
        ccl.ccl_batch_check(bw.handle)
        t = a.elapsed_time(b) * 1e-3 / reps
        p = average_power(bw.run) if log_energy else None
        bw.close()
        del bw
        torch.cuda.empty_cache()
        return t, p

    def run_loop(depth_rows):
        """A host loop of one ccl_wave_step call per grid (one chunk each)."""
        cws = []
        for g, d in enumerate(grids):
            T, rows = depth_rows(g)
            cw = ChunkedWave((0, 0), (d["ny"], d["nx"]), 1, 0.25, depth=T, tile_rows=rows)
            u0 = synth.gaussian_field((d["ny"], d["nx"]), d["sigma"], d["seed"])
            cw.scatter(u0, u0)
            cws.append(cw)

        def loop_once():
            for cw, d in zip(cws, grids):
                cw.step(d["steps"])

        loop_once()
        torch.cuda.synchronize()
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        reps = 2
        a.record()
        for _ in range(reps):
            loop_once()
        b.record()
        torch.cuda.synchronize()
        t = a.elapsed_time(b) * 1e-3 / reps
        p = average_power(loop_once) if log_energy else None
        del cws
        torch.cuda.empty_cache()
        return t, p

    t_batched, p_batched = run_batch(specs, 0)
    t_pg, p_pg = run_batch(specs_pg, ccl.CCL_BATCH_PER_GRID)
    t_ll, p_ll = run_loop(lambda g: (specs_pg[g]["depth"], specs_pg[g]["tile_rows"]))
    t_loop, p_loop = run_loop(lambda g: (1, 0))
    nj = lambda p, t: None if p is None else round(p * t / cell_steps * 1e9, 4)
    return {"grids": len(grids), "cell_steps": cell_steps,
            "batched_mcells": round(cell_steps / t_batched / 1e6, 1),
            "batched_ms": round(t_batched * 1e3, 3),
            "batched_nj_per_cell_step": nj(p_batched, t_batched),
            "batched_per_grid_mcells": round(cell_steps / t_pg / 1e6, 1),
            "batched_per_grid_ms": round(t_pg * 1e3, 3),
            "batched_per_grid_nj_per_cell_step": nj(p_pg, t_pg),
            "per_grid_learned_loop_mcells": round(cell_steps / t_ll / 1e6, 1),
            "per_grid_learned_loop_ms": round(t_ll * 1e3, 3),
            "per_grid_learned_loop_nj_per_cell_step": nj(p_ll, t_ll),
            "batching_gain": round(t_ll / min(t_batched, t_pg), 4),
            "per_grid_loop_mcells": round(cell_steps / t_loop / 1e6, 1),
            "per_grid_loop_ms": round(t_loop * 1e3, 3),
            "per_grid_loop_nj_per_cell_step": nj(p_loop, t_loop),
            "configs": how}


def wave3d_forms(with_energy=False):
    """768^3, r2 = 0.1, 8 z-slab chunks, 200 steps: the swept best (depth,
    tile planes) vs the cost model's pick and vs the fastest of the model's
    three best as measured (all among 8-chunk configs), timed with the
    workload's own data through ccl_wave_step, with J/step."""
    import numpy as np
    import torch

    import synth
    from paper_2505_06022_amd import ccl_wave_plan_rows, tune
    from paper_2505_06022_amd.fields import ChunkedWave
    w = synth.WORKLOADS["wave3d_768_k8"]
    shape = w["shape"]
    # every candidate is timed over the workload's own step count, so a
    # depth that does not divide it pays for its shorter last block (the
    # library's sweep, ccl_autotune_sweep)
    cands, res, best = tune.sweep(shape, w["chunks"], w["r2"], steps=w["steps"], reps=3)
    swept = cands[best]
    learned = verified = None
    if os.path.exists(MODEL_PATH):
        m = tune.CostModel.load(MODEL_PATH)
        learned, _ = m.pick(shape, "time", nchunks=w["chunks"])
        # the model's three best candidates, the fastest of them as measured
        # (3 measurements instead of the sweep's len(cands))
        order = m.rank(shape, "time", nchunks=w["chunks"])[:3]
        allc = tune.candidates(shape)
        vres = tune.measure([allc[i] for i in order], w["r2"], reps=3, steps=w["steps"])
        verified = allc[order[int(np.argmin([r["s_per_step"] for r in vres]))]]
        m.close()
    u0 = synth.gaussian_field(shape, w["sigma"], w["seed"])
    out = {"workload": "3D leapfrog 768^3, r2=0.1, 200 steps, 8 z-slab chunks",
           "candidates": len(cands)}
    cells = float(np.prod(shape))
    for name, cfg in (("swept", swept), ("learned", learned), ("learned_top3_measured", verified)):
        if cfg is None:
            continue
        cw = ChunkedWave((0, 0, 0), shape, w["chunks"], w["r2"], depth=cfg.temporal_depth,
                         tile_rows=cfg.tile_rows)
        cw.scatter(u0, u0)
        cw.step(w["steps"])
        t = time_runs(cw, w["steps"], 2) / 2
        entry = {"depth": cfg.temporal_depth, "tile_planes": cfg.tile_rows,
                 "planned_planes": ccl_wave_plan_rows(cfg),
                 "mcells": round(cells * w["steps"] / t / 1e6, 1),
                 "ms_per_run": round(t * 1e3, 3)}
        if with_energy:
            p = average_power(lambda: cw.step(w["steps"]))
            entry["j_per_step"] = round(p * t / w["steps"], 5)
        out[name] = entry
        del cw
        torch.cuda.empty_cache()
    for name in ("learned", "learned_top3_measured"):
        if name in out:
            out[name]["time_over_swept"] = round(out[name]["ms_per_run"] /
                                                 out["swept"]["ms_per_run"], 4)
    return out


def precision_forms(w, u0, depths=(1, 2, 4, 6, 8)):
    """The headline share (8192 x 8192, 1000 steps, 4 chunks) with the
    fields in float64, bfloat16 and binary16 (the last two with float32
    arithmetic), at each temporal depth in `depths` (automatic tile rows);
    per element type the fastest depth, with its roofline fraction on its
    own bytes: 3 elements per cell per launch at T = 1 (in place), 4 at
    T > 1."""
    import numpy as np
    import torch

    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.fields import ChunkedWave
    cells = int(np.prod(w["shape"]))
    out = {}
    for dt in ("f64", "bf16", "f16"):
        esize = ccl.DTYPE_BYTES[ccl.DTYPES[dt]]
        host = u0.astype(np.float64) if dt == "f64" else u0
        rows = []
        for T in depths:
            cw = ChunkedWave(w["share_offset"], w["shape"], w["chunks"], w["r2"], depth=T,
                             buffer_range=w["global_shape"], dtype=dt)
            cw.scatter(host, host)
            cw.step(w["steps"])
            t = time_runs(cw, w["steps"], 2) / 2
            ccl.ccl_timing_enable(True)  # launch durations: a separate run
            time_runs(cw, w["steps"], 1)
            n, ms = ccl.ccl_timing_query(ccl.CCL_KERNEL_STENCIL)
            ccl.ccl_timing_enable(False)
            per_cell = (3 if T == 1 else 4) * esize
            gbs = per_cell * cells / (ms / n * 1e-3) / 1e9
            rows.append({"depth": T, "mcells": round(cells * w["steps"] / t / 1e6, 1),
                         "ms_per_run": round(t * 1e3, 3),
                         "stencil_launch_ms": round(ms / n, 4),
                         "bytes_per_cell_launch": per_cell,
                         "achieved_gbs": round(gbs, 1),
                         "roofline_frac": round(gbs / HBM_PEAK_GBS, 4)})
            del cw
            torch.cuda.empty_cache()
        best = max(rows, key=lambda r: r["mcells"])
        out[dt] = {"best": best, "depths": rows}
        log(f"{dt}: best T={best['depth']} {best['mcells']} Mcells/s, "
            f"frac {best['roofline_frac']}")
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed bench steps (full runs)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--depth", type=int, default=0, help="temporal depth T (0 = pick)")
    ap.add_argument("--tile-rows", type=int, default=0,
                    help="rows per tile with --depth (0 = automatic)")
    ap.add_argument("--sweep", action="store_true", help="pick by autotuner sweep, not model")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip SAXPY, energy, plain and batched forms")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2505_06022_amd as ccl
    import synth
    from paper_2505_06022_amd import tune
    from paper_2505_06022_amd.fields import ChunkedWave

    if not ccl.LIB_PATH.exists():
        import __graft_entry__
        __graft_entry__.build()
    torch.cuda.set_device(0)
    name = "wave2d_8192_share_k4"
    w = synth.WORKLOADS[name]
    depth, rows, how = pick_config(w, args)
    log(f"workload {name}: T={depth}, tile rows={rows} ({how}); generating input")
    u0 = synth.gaussian_field(w["shape"], w["sigma"], w["seed"])
    cw = ChunkedWave(w["share_offset"], w["shape"], w["chunks"], w["r2"], depth=depth,
                     tile_rows=rows, buffer_range=w["global_shape"])
    cw.scatter(u0, u0)
    torch.cuda.synchronize()

    for i in range(args.warmup):
        cw.step(w["steps"])
        torch.cuda.synchronize()
        log(f"warmup {i + 1}/{args.warmup} done")

    elapsed = time_runs(cw, w["steps"], args.steps)
    log(f"timed {args.steps} runs in {elapsed:.3f} s")
    # per-launch durations for the roofline: the same runs again, each
    # launch bracketed by HIP events on its own stream (the event records
    # between launches add gaps, so they stay out of the timed runs above)
    ccl.ccl_timing_enable(True)
    elapsed_ev = time_runs(cw, w["steps"], args.steps)
    n_launch, st_ms = ccl.ccl_timing_query(ccl.CCL_KERNEL_STENCIL)
    h_launch, h_ms = ccl.ccl_timing_query(ccl.CCL_KERNEL_HALO)
    ccl.ccl_timing_enable(False)
    log(f"the same {args.steps} runs with per-launch events: {elapsed_ev:.3f} s")
    sample = cw.gather_points([(w["share_offset"][0] + 4096, 4096)])
    if not np.all(np.isfinite(sample)):
        raise SystemExit("bench: non-finite field")

    cells = int(np.prod(w["shape"]))
    cell_steps = cells * w["steps"] * args.steps
    mcells = cell_steps / elapsed / 1e6
    per_cell = 12 if depth == 1 else 16  # in place: 2 reads + 1 write; else 2 + 2
    bytes_per_launch = per_cell * cells
    avg_s = st_ms / n_launch * 1e-3
    achieved = bytes_per_launch / avg_s / 1e9
    roof_equiv = HBM_PEAK_GBS * 1e9 / 12.0 / 1e6  # Mcells/s at 12 B/cell-step

    out = {
        "metric": "wave-stencil Mcells/s", "value": round(mcells, 1), "unit": "Mcells/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D leapfrog wave, 8192x8192 share of 32768x8192, FP32, "
                               "r2=0.25, 1000 steps, 4 device-local row chunks",
                   "temporal_depth": depth, "tile_rows": rows, "picked_by": how,
                   "cells": cells, "leapfrog_steps": w["steps"], "chunks": w["chunks"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": load_traffic(depth, rows)},
        "hbm_roofline_equiv_pct": round(100.0 * mcells / roof_equiv, 2),
        "ms_per_step_with_launch_events": round(elapsed_ev / args.steps * 1e3, 3),
        "stencil_launch_ms": round(st_ms / n_launch, 4), "stencil_launches": n_launch,
        "halo_launch_ms": round(h_ms / max(h_launch, 1), 4), "halo_launches": h_launch,
    }
    if not args.no_extras:
        log("energy window")
        try:
            power = average_power(lambda: cw.step(w["steps"]))
            out["power_w"] = round(power, 1)
            out["j_per_step"] = round(power * elapsed / (w["steps"] * args.steps), 6)
            out["energy_backend"] = ccl.ccl_energy_backend(0)
        except (ccl.CclError, RuntimeError) as e:
            out["j_per_step"] = None
            out["energy_backend"] = f"unavailable ({e})"
        del cw
        torch.cuda.empty_cache()
        log("plain form (T=1)")
        # the plain form's tile rows as the launcher would choose them: the
        # fastest of the autotuner's T = 1 candidates for this split, measured
        pcands = [c for c in tune.candidates(w["shape"])
                  if c.nchunks == w["chunks"] and c.temporal_depth == 1]
        pres = tune.measure(pcands, w["r2"], reps=3, steps=200)
        prow = pcands[int(np.argmin([r["s_per_step"] for r in pres]))].tile_rows
        out["plain_tile_rows"] = prow
        cp = ChunkedWave(w["share_offset"], w["shape"], w["chunks"], w["r2"], depth=1,
                         tile_rows=prow, buffer_range=w["global_shape"])
        cp.scatter(u0, u0)
        cp.step(w["steps"])
        t_plain = time_runs(cp, w["steps"], 2)
        out["plain_mcells"] = round(cells * w["steps"] * 2 / t_plain / 1e6, 1)
        if out.get("j_per_step") is not None:
            p_plain = average_power(lambda: cp.step(w["steps"]))
            out["plain_j_per_step"] = round(p_plain * t_plain / (2 * w["steps"]), 6)
        del cp
        torch.cuda.empty_cache()
        log("SAXPY calibration")
        out["saxpy_gbs"] = round(saxpy_calibration(), 1)
        log("batched workload")
        out["batched"] = batched_forms(log_energy=out.get("j_per_step") is not None)
        log("3D workload")
        out["wave3d"] = wave3d_forms(with_energy=out.get("j_per_step") is not None)
        log("float64 and 16-bit storage")
        out["precisions"] = precision_forms(w, u0)
    if not args.no_cpu_baseline:
        log("timing the CPU oracle")
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
