#!/usr/bin/env python3
"""Throughput of the chunked leapfrog wave stencil on one MI355X.

One bench step = one full run of the workload: 1000 leapfrog steps of the
8192 x 8192 row share (rows [8192, 16384) of a 32768 x 8192 domain, Dirichlet
zero outside the share) split into 4 device-local chunks, with the halo
exchanges between them, through ccl_wave_step.  Inputs are resident in HBM
before the timed region; the timed region is bracketed by synchronisation.

Prints one JSON line: value = Mcells/s (cell updates per second / 1e6).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in ("wave2d.hip", "wave_step.cpp", "halo.hip"):
        with open(os.path.join(ROOT, "paper_2505_06022_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(depth: int):
    """HBM bytes per stencil launch from the committed rocprofv3 counter
    summary, if it was taken on the current kernel source and depth."""
    path = os.path.join(ROOT, "profiles", "traffic_wave2d_8192_share_k4.json")
    try:
        with open(path) as f:
            doc = json.load(f)
    except (OSError, ValueError):
        return None
    if doc.get("kernel_hash") != kernel_source_hash() or doc.get("depth") != depth:
        return None
    return doc.get("bytes_per_launch")


def cpu_baseline(w, seconds: float = 15.0):
    """The float32 oracle on the host cores over a bounded sample of the
    workload: the full 8192 x 8192 share for as many of its steps as fit in
    about `seconds` (sized from a 5-step probe run)."""
    import numpy as np

    import oracle
    import synth
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or oracle.max_threads()
    u0 = synth.gaussian_field(w["shape"], w["sigma"], w["seed"])
    t0 = time.perf_counter()
    oracle.wave(u0.copy(), u0, w["r2"], 5, threads=threads)
    per_step = max((time.perf_counter() - t0) / 5, 1e-4)
    steps = int(max(5, min(w["steps"], seconds / per_step)))
    t0 = time.perf_counter()
    oracle.wave(u0.copy(), u0, w["r2"], steps, threads=threads)
    dt = time.perf_counter() - t0
    cells = int(np.prod(w["shape"]))
    return {"value": round(cells * steps / dt / 1e6, 1), "unit": "Mcells/s", "cores": threads,
            "kind": "oracle",
            "sample": f"float32 oracle, {w['shape'][0]}x{w['shape'][1]} share, {steps} of the "
                      f"workload's {w['steps']} steps, {dt:.1f} s on {threads} host threads"}


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


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10, help="timed bench steps (full runs)")
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--depth", type=int, default=4, help="temporal depth T")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-saxpy", action="store_true")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2505_06022_amd as ccl
    import synth
    from paper_2505_06022_amd.fields import ChunkedWave

    if not ccl.LIB_PATH.exists():
        import __graft_entry__
        __graft_entry__.build()
    torch.cuda.set_device(0)
    name = "wave2d_8192_share_k4"
    w = synth.WORKLOADS[name]
    print(f"[bench] workload {name}: T={args.depth}, generating input", file=sys.stderr,
          flush=True)
    u0 = synth.gaussian_field(w["shape"], w["sigma"], w["seed"])
    cw = ChunkedWave(w["share_offset"], w["shape"], w["chunks"], w["r2"], depth=args.depth,
                     tile_rows=args.tile_rows, buffer_range=w["global_shape"])
    cw.scatter(u0, u0)
    torch.cuda.synchronize()

    saxpy_gbs = None if args.no_saxpy else saxpy_calibration()

    for i in range(args.warmup):
        cw.step(w["steps"])
        torch.cuda.synchronize()
        print(f"[bench] warmup {i + 1}/{args.warmup} done", file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()
    energy_ok = True
    try:
        e0, _ = ccl.ccl_energy_read(0, stream)
        backend = ccl.ccl_energy_backend(0)
    except ccl.CclError as e:
        energy_ok, backend = False, f"unavailable ({e.message})"
    ccl.ccl_timing_enable(True)
    torch.cuda.synchronize()
    t_start = torch.cuda.Event(enable_timing=True)
    t_stop = torch.cuda.Event(enable_timing=True)
    wall0 = time.perf_counter()
    t_start.record(stream)
    for _ in range(args.steps):
        cw.step(w["steps"])
    t_stop.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    e1 = ccl.ccl_energy_read(0, stream)[0] if energy_ok else None
    elapsed = t_start.elapsed_time(t_stop) * 1e-3
    n_launch, st_ms = ccl.ccl_timing_query(ccl.CCL_KERNEL_STENCIL)
    h_launch, h_ms = ccl.ccl_timing_query(ccl.CCL_KERNEL_HALO)
    ccl.ccl_timing_enable(False)
    print(f"[bench] timed {args.steps} runs in {elapsed:.3f} s (wall {wall:.3f} s)",
          file=sys.stderr, flush=True)

    sample = cw.gather_points([(w["share_offset"][0] + 4096, 4096)])
    if not np.all(np.isfinite(sample)):
        raise SystemExit("bench: non-finite field")

    cells = int(np.prod(w["shape"]))
    cell_steps = cells * w["steps"] * args.steps
    mcells = cell_steps / elapsed / 1e6
    # dominant kernel: the stencil launch; algorithmic bytes per launch
    per_cell = 12 if args.depth == 1 else 16  # in place: 2 reads + 1 write; else 2 + 2
    bytes_per_launch = per_cell * cells
    avg_s = st_ms / n_launch * 1e-3
    achieved = bytes_per_launch / avg_s / 1e9
    roof_equiv = HBM_PEAK_GBS * 1e9 / 12.0 / 1e6  # Mcells/s at 12 B/cell-step
    traffic = load_traffic(args.depth)

    out = {
        "metric": "wave-stencil Mcells/s", "value": round(mcells, 1), "unit": "Mcells/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(elapsed / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "2D leapfrog wave, 8192x8192 share of 32768x8192, FP32, "
                               "r2=0.25, 1000 steps, 4 device-local row chunks",
                   "temporal_depth": args.depth, "cells": cells, "leapfrog_steps": w["steps"],
                   "chunks": w["chunks"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic},
        "hbm_roofline_equiv_pct": round(100.0 * mcells / roof_equiv, 2),
        "stencil_launch_ms": round(st_ms / n_launch, 4), "stencil_launches": n_launch,
        "halo_ms_total": round(h_ms, 3), "halo_launches": h_launch,
        "saxpy_gbs": None if saxpy_gbs is None else round(saxpy_gbs, 1),
        "energy_backend": backend,
        "j_per_step": None if e1 is None else round((e1 - e0) / (w["steps"] * args.steps), 6),
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
