"""Small, fixed workloads for rocprofv3 counter runs, and the parser that
turns their counter output into the HBM-traffic summary under profiles/.

    rocprofv3 --pmc FETCH_SIZE -d OUT -o fetch -- python3 -m paper_2505_06022_amd.profile_run run --depth 8 --rows 128
    rocprofv3 --pmc WRITE_SIZE -d OUT -o write -- python3 -m paper_2505_06022_amd.profile_run run --depth 8 --rows 128
    python3 -m paper_2505_06022_amd.profile_run summarise --fetch OUT/.../fetch_counter_collection.csv \
        --write OUT/.../write_counter_collection.csv --depth 8 --rows 128 --md profiles/traffic_wave2d_8192_share_k4.md

`run` launches, on the headline share (8192 x 8192, 4 chunks), a few blocks
of T steps through ccl_wave_step, then one SAXPY over 2^26 floats whose
algorithmic traffic is known exactly (8 B read and 4 B written per element);
`summarise` scales the stencil's per-dispatch counters by what the same
counters read for that SAXPY and writes the summary bench.py reports.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAXPY_N = 1 << 26


SOURCES = {2: ("prec.h", "wave2d_tile.h", "wave2d.hip", "wave_step.cpp", "halo.hip"),
           3: ("prec.h", "wave3d_cell.h", "wave3d.hip", "wave3d_tb.hip", "wave_step.cpp",
               "halo.hip")}


def kernel_source_hash(dims: int = 2) -> str:
    h = hashlib.sha256()
    for name in SOURCES[dims]:
        with open(os.path.join(ROOT, "paper_2505_06022_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def run(depth: int, rows: int, blocks: int = 6, dims: int = 2):
    sys.path.insert(0, ROOT)
    import torch

    import paper_2505_06022_amd as ccl
    import synth
    from paper_2505_06022_amd.fields import ChunkedWave
    torch.cuda.set_device(0)
    name = "wave2d_8192_share_k4" if dims == 2 else "wave3d_768_k8"
    w = synth.WORKLOADS[name]
    u0 = synth.gaussian_field(w["shape"], w["sigma"], w["seed"])
    cw = ChunkedWave(w.get("share_offset", (0,) * len(w["shape"])), w["shape"], w["chunks"],
                     w["r2"], depth=depth,
                     tile_rows=rows, buffer_range=w.get("global_shape"))
    cw.scatter(u0, u0)
    cw.step(depth * blocks)
    torch.cuda.synchronize()
    x = torch.rand(SAXPY_N, device="cuda")
    y = torch.rand(SAXPY_N, device="cuda")
    z = torch.empty(SAXPY_N, device="cuda")
    ccl.ccl_saxpy(SAXPY_N, 2.0, x.data_ptr(), y.data_ptr(), z.data_ptr())
    torch.cuda.synchronize()
    print(f"profile_run: {name}, {blocks} blocks of T={depth}, rows={rows}; saxpy n={SAXPY_N}",
          flush=True)


def run_batch(specs_out=None):
    """The 64-grid batch (per-grid depth from the cost model) stepped once
    by the persistent kernel and once grid by grid (CCL_BATCH_PER_GRID),
    both launched directly (no graph), then the calibration SAXPY.  The
    launch specs go to `specs_out` (JSON) for the summary."""
    sys.path.insert(0, ROOT)
    import torch

    import paper_2505_06022_amd as ccl
    import synth
    from paper_2505_06022_amd import tune
    from paper_2505_06022_amd.fields import BatchedWaves
    torch.cuda.set_device(0)
    grids = synth.batched_grids()
    specs, specs_pg, how = tune.batch_specs(
        grids, os.path.join(ROOT, "paper_2505_06022_amd", "costmodel.json"))
    if specs_out:
        with open(specs_out, "w") as f:
            json.dump({"persistent": specs, "per_grid": specs_pg, "how": how}, f)
    for sp, flags in ((specs, ccl.CCL_BATCH_NO_GRAPH),
                      (specs_pg, ccl.CCL_BATCH_NO_GRAPH | ccl.CCL_BATCH_PER_GRID)):
        bw = BatchedWaves(sp, flags=flags)
        for g, d in enumerate(grids):
            u0 = synth.gaussian_field((d["ny"], d["nx"]), d["sigma"], d["seed"])
            bw.scatter(g, u0, u0)
        torch.cuda.synchronize()
        bw.run()
        torch.cuda.synchronize()
        ccl.ccl_batch_check(bw.handle)
        bw.close()
        del bw
        torch.cuda.empty_cache()
    x = torch.rand(SAXPY_N, device="cuda")
    y = torch.rand(SAXPY_N, device="cuda")
    z = torch.empty(SAXPY_N, device="cuda")
    ccl.ccl_saxpy(SAXPY_N, 2.0, x.data_ptr(), y.data_ptr(), z.data_ptr())
    torch.cuda.synchronize()
    print(f"profile_run: 64-grid batch, persistent and per-grid; saxpy n={SAXPY_N}", flush=True)


def batch_algorithmic_bytes(specs):
    """Algorithmic bytes of one pass over a batch: per grid and block of T
    steps, 16 B per cell (two levels read, two written), 12 B for a grid
    stepped one step at a time in place."""
    total = 0
    for s in specs:
        T, steps = int(s["depth"]), int(s["steps"])
        blocks = -(-steps // T)
        total += int(s["ny"]) * int(s["nx"]) * blocks * (12 if T == 1 else 16)
    return total


def summarise_batch(fetch_csv, write_csv, specs_json, md_path):
    """HBM bytes of the two batch modes against their algorithmic bytes,
    from counter runs of `run --batch` and the specs it wrote: the
    persistent kernel is one dispatch, the per-grid mode every stencil and
    halo dispatch after it."""
    with open(specs_json) as f:
        sj = json.load(f)
    specs, how = sj["persistent"], sj["how"]
    sums = {}
    for path, counter in ((fetch_csv, "FETCH_SIZE"), (write_csv, "WRITE_SIZE")):
        tot = {"persistent": 0.0, "per_grid": 0.0, "saxpy": 0.0, "launches_per_grid": 0}
        with open(path) as f:
            for row in csv.DictReader(f):
                if row.get("Counter_Name", counter) != counter:
                    continue
                name, val = row.get("Kernel_Name", ""), float(row.get("Counter_Value", "nan"))
                if "batch_kernel" in name:
                    tot["persistent"] += val
                elif "wave2d_kernel" in name or "copy_boxes_kernel" in name:
                    tot["per_grid"] += val
                    tot["launches_per_grid"] += 1
                elif "saxpy_kernel" in name:
                    tot["saxpy"] = val
        sums[counter] = tot
    f_scale = 8.0 * SAXPY_N / 1024.0 / sums["FETCH_SIZE"]["saxpy"]
    w_scale = 4.0 * SAXPY_N / 1024.0 / sums["WRITE_SIZE"]["saxpy"]
    alg = batch_algorithmic_bytes(specs)
    doc = {"workload": "64-grid batch", "configs": how, "fetch_scale": f_scale,
           "write_scale": w_scale, "algorithmic_bytes": alg,
           "launches_per_grid_mode": sums["FETCH_SIZE"]["launches_per_grid"]}
    for mode in ("persistent", "per_grid"):
        fb = sums["FETCH_SIZE"][mode] * f_scale * 1024.0
        wb = sums["WRITE_SIZE"][mode] * w_scale * 1024.0
        doc[mode] = {"fetch_bytes": fb, "write_bytes": wb, "ratio": (fb + wb) / alg}
    lines = [
        "# HBM traffic of the 64-grid batch: persistent kernel against per-grid launches",
        "",
        "Counters from two rocprofv3 runs, one per counter; the batch (per-grid depth "
        f"from the {how}) runs once in each mode, launched directly; FETCH_SIZE and "
        f"WRITE_SIZE are scaled by what they read for a SAXPY of {SAXPY_N} floats in the "
        "same program:",
        "",
        "```",
        "rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch -o p -- python3 -m "
        "paper_2505_06022_amd.profile_run run --batch --specs-out OUT/specs.json",
        "rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write -o p -- python3 -m "
        "paper_2505_06022_amd.profile_run run --batch",
        "python3 -m paper_2505_06022_amd.profile_run summarise-batch --fetch "
        "OUT/fetch/p_counter_collection.csv --write OUT/write/p_counter_collection.csv "
        f"--specs OUT/specs.json --md {os.path.relpath(md_path, ROOT)}",
        "```",
        "",
        f"Algorithmic bytes of one pass (16 B per cell per block of T steps): {alg:,}.",
        "",
        "| mode | fetched (GB) | written (GB) | traffic / algorithmic |",
        "|---|---|---|---|",
    ]
    for mode, label in (("persistent", "persistent kernel (one dispatch)"),
                        ("per_grid", f"per grid ({doc['launches_per_grid_mode']} stencil and "
                                     "halo dispatches)")):
        m = doc[mode]
        lines.append(f"| {label} | {m['fetch_bytes'] / 1e9:.2f} | {m['write_bytes'] / 1e9:.2f} | "
                     f"{m['ratio']:.3f} |")
    lines += ["", "batch-traffic-json: " + json.dumps(doc), ""]
    with open(md_path, "w") as f:
        f.write("\n".join(lines))
    print("\n".join(lines))


def _per_kernel(path, counter):
    """{kernel-name-prefix: [values per dispatch]} from a rocprofv3 counter CSV."""
    out = {}
    with open(path) as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name", counter) != counter:
                continue
            name = row.get("Kernel_Name", "")
            val = float(row.get("Counter_Value", "nan"))
            key = ("wave2d" if "wave2d_kernel" in name else
                   "wave3d" if ("wave3d_kernel" in name or "wave3d_tb_kernel" in name) else
                   "saxpy" if "saxpy_kernel" in name else
                   "halo" if "copy_boxes_kernel" in name else None)
            if key:
                out.setdefault(key, []).append(val)
    return out


def summarise(fetch_csv, write_csv, depth, rows, md_path, dims=2, append=False):
    fetch = _per_kernel(fetch_csv, "FETCH_SIZE")
    write = _per_kernel(write_csv, "WRITE_SIZE")
    kern = "wave2d" if dims == 2 else "wave3d"
    sx_read = 8.0 * SAXPY_N / 1024.0   # KiB, algorithmic
    sx_write = 4.0 * SAXPY_N / 1024.0
    f_scale = sx_read / (sum(fetch["saxpy"]) / len(fetch["saxpy"]))
    w_scale = sx_write / (sum(write["saxpy"]) / len(write["saxpy"]))
    # skip the first stencil dispatch (cold caches after the host scatter)
    fw = fetch[kern][1:] or fetch[kern]
    ww = write[kern][1:] or write[kern]
    f_kib = sum(fw) / len(fw) * f_scale
    w_kib = sum(ww) / len(ww) * w_scale
    cells = 8192 * 8192 if dims == 2 else 768 ** 3
    alg = (12 if depth == 1 else 16) * cells
    wl = "8192x8192 share, 4 chunks" if dims == 2 else "768^3, 8 chunks"
    doc = dict(kernel=f"{kern}_kernel", workload=wl, depth=depth,
               tile_rows=rows, kernel_hash=kernel_source_hash(dims),
               fetch_kib_per_dispatch_raw=sum(fw) / len(fw),
               write_kib_per_dispatch_raw=sum(ww) / len(ww),
               fetch_scale=f_scale, write_scale=w_scale,
               bytes_per_launch=int(round((f_kib + w_kib) * 1024.0)),
               algorithmic_bytes_per_launch=alg, dispatches=len(fw))
    lines = [
        f"# HBM traffic of the {kern} stencil launch — {wl}, T={depth}, "
        f"{rows if rows else 'automatic'} rows per tile",
        "",
        "Counters from two rocprofv3 runs, one per counter, scaled by what the same counters "
        f"read for a SAXPY of {SAXPY_N} floats (8 B read, 4 B written per element) launched "
        "at the end of the same program:",
        "",
        "```",
        f"rocprofv3 --pmc FETCH_SIZE --output-format csv -d OUT/fetch -o p -- python3 -m "
        f"paper_2505_06022_amd.profile_run run --dims {dims} --depth {depth} --rows {rows}",
        f"rocprofv3 --pmc WRITE_SIZE --output-format csv -d OUT/write -o p -- python3 -m "
        f"paper_2505_06022_amd.profile_run run --dims {dims} --depth {depth} --rows {rows}",
        f"python3 -m paper_2505_06022_amd.profile_run summarise --fetch OUT/fetch/.../"
        f"p_counter_collection.csv --write OUT/write/.../p_counter_collection.csv --dims {dims} "
        f"--depth {depth} --rows {rows} --md {os.path.relpath(md_path, ROOT)}"
        + (" --append" if append and os.path.exists(md_path) else ""),
        "```",
        "",
        "The first stencil dispatch (cold caches after the host scatter) is left out of the "
        f"average over the other {len(fw)}.",
        "",
        "| quantity | value |",
        "|---|---|",
        f"| FETCH_SIZE per stencil dispatch (raw, KiB) | {doc['fetch_kib_per_dispatch_raw']:.0f} |",
        f"| WRITE_SIZE per stencil dispatch (raw, KiB) | {doc['write_kib_per_dispatch_raw']:.0f} |",
        f"| SAXPY scale factors (fetch, write) | {f_scale:.4f}, {w_scale:.4f} |",
        f"| HBM bytes per launch (scaled) | {doc['bytes_per_launch']:,} |",
        f"| algorithmic bytes per launch | {alg:,} |",
        f"| traffic / algorithmic | {doc['bytes_per_launch'] / alg:.3f} |",
        "",
        "traffic-json: " + json.dumps(doc),
        "",
    ]
    if append and os.path.exists(md_path):
        # one section per launch configuration in the same file
        lines[0] = "#" + lines[0]
        with open(md_path, "a") as f:
            f.write("\n" + "\n".join(lines))
    else:
        with open(md_path, "w") as f:
            f.write("\n".join(lines))
    print("\n".join(lines))


def _counter_rows(paths):
    """{counter: [per-dispatch values]} of the stencil kernel, plus its
    per-dispatch durations (ns) and register counts, from rocprofv3 counter
    CSVs (one or more passes over the same program)."""
    vals, dur, regs = {}, [], None
    for path in paths:
        seen = set()
        with open(path) as f:
            for row in csv.DictReader(f):
                name = row.get("Kernel_Name", "")
                if not ("wave2d_kernel" in name or "wave3d_kernel" in name or
                        "wave3d_tb_kernel" in name):
                    continue
                vals.setdefault(row["Counter_Name"], []).append(float(row["Counter_Value"]))
                did = row.get("Dispatch_Id")
                if did not in seen and row.get("Start_Timestamp"):
                    seen.add(did)
                    dur.append(float(row["End_Timestamp"]) - float(row["Start_Timestamp"]))
                regs = (row.get("VGPR_Count"), row.get("Accum_VGPR_Count"),
                        row.get("LDS_Block_Size"), row.get("Workgroup_Size"))
    return vals, dur, regs


def counters(paths, depth, rows, md_path, dims=2, title=None, commands=(), append=False,
             kernel_hash=None):
    """Where the stencil launch spends its time, from SQ/GRBM counters: VALU
    instructions per useful cell-step, VALU busy share, waits, occupancy and
    LDS activity.  The first dispatch of each pass (cold caches) is left out.
    rocprofv3 sums each counter over the device's blocks: SQ counters over
    all shader engines (cycle counters in quad-cycles), GRBM_GUI_ACTIVE over
    the 8 XCDs, so one XCD's active cycles are GRBM_GUI_ACTIVE / 8 (the
    `max` that rocprofv3's own VALUBusy and OccupancyPercent divide by)."""
    vals, dur, regs = _counter_rows(paths)
    avg = {k: sum(v[1:] or v) / len(v[1:] or v) for k, v in vals.items()}
    d_ns = sum(dur[1:] or dur) / max(1, len(dur[1:] or dur))
    cells = 8192 * 8192 if dims == 2 else 768 ** 3
    cu_num, xcds = 256, 8
    cell_steps = cells * depth
    out = {"kernel": "wave2d_kernel" if dims == 2 else "wave3d_tb_kernel",
           "depth": depth, "tile_rows": rows,
           "kernel_hash": kernel_hash or kernel_source_hash(dims),
           "dispatch_us": d_ns / 1e3, "rocprof_vgpr_count": regs[0] if regs else None,
           "lds_bytes": regs[2] if regs else None, "workgroup": regs[3] if regs else None,
           "counters": avg}
    g = avg.get("GRBM_GUI_ACTIVE")
    g = g / xcds if g else None  # active cycles of one XCD
    der = {}
    if "SQ_INSTS_VALU" in avg:
        der["valu_lane_ops_per_cell_step"] = avg["SQ_INSTS_VALU"] * 64 / cell_steps
    if g and d_ns:
        der["clock_ghz"] = g / d_ns
    if g and "SQ_ACTIVE_INST_VALU" in avg:
        # quad-cycles of VALU work per CU over the dispatch's cycles: the
        # share of time the SIMDs issue vector instructions
        der["valu_busy_share"] = avg["SQ_ACTIVE_INST_VALU"] / cu_num / g
    if g and "SQ_WAVE_CYCLES" in avg:
        der["waves_per_cu"] = 4 * avg["SQ_WAVE_CYCLES"] / g / cu_num
    if "SQ_WAIT_INST_ANY" in avg and "SQ_WAVE_CYCLES" in avg:
        der["wait_inst_any_share_of_wave_cycles"] = avg["SQ_WAIT_INST_ANY"] / avg["SQ_WAVE_CYCLES"]
    if "SQ_WAIT_ANY" in avg and "SQ_WAVE_CYCLES" in avg:
        der["wait_any_share_of_wave_cycles"] = avg["SQ_WAIT_ANY"] / avg["SQ_WAVE_CYCLES"]
    if "SQ_WAIT_INST_LDS" in avg and "SQ_WAVE_CYCLES" in avg:
        der["wait_inst_lds_share_of_wave_cycles"] = avg["SQ_WAIT_INST_LDS"] / avg["SQ_WAVE_CYCLES"]
    if "SQ_ACTIVE_INST_LDS" in avg and "SQ_WAVE_CYCLES" in avg:
        der["lds_active_share_of_wave_cycles"] = avg["SQ_ACTIVE_INST_LDS"] / avg["SQ_WAVE_CYCLES"]
    if g and "SQ_LDS_BANK_CONFLICT" in avg:
        der["lds_bank_conflict_share"] = avg["SQ_LDS_BANK_CONFLICT"] / g / cu_num
    if "SQ_WAVES" in avg:
        der["valu_insts_per_wave"] = avg.get("SQ_INSTS_VALU", 0) / avg["SQ_WAVES"]
        der["lds_insts_per_wave"] = avg.get("SQ_INSTS_LDS", 0) / avg["SQ_WAVES"]
    out["derived"] = der
    wl = "8192x8192 share, 4 chunks" if dims == 2 else "768^3, 8 chunks"
    lines = [f"# {title or 'Counters of the stencil launch'} — {wl}, T={depth}, "
             f"{rows if rows else 'automatic'} rows per tile", "", "Commands:", "", "```"]
    lines += list(commands) + ["```", "",
                               f"Stencil dispatch: {d_ns / 1e3:.1f} us under counter collection; "
                               f"LDS {out['lds_bytes']} B per work-group of {out['workgroup']}.",
                               "",
                               "| counter (per dispatch) | value |", "|---|---|"]
    for k in sorted(avg):
        lines.append(f"| {k} | {avg[k]:,.0f} |")
    lines += ["", "| derived | value |", "|---|---|"]
    for k, v in der.items():
        lines.append(f"| {k} | {v:.4g} |" if v is not None else f"| {k} | — |")
    lines += ["", "counters-json: " + json.dumps(out), ""]
    if append and os.path.exists(md_path):
        lines[0] = "#" + lines[0]
        with open(md_path, "a") as f:
            f.write("\n" + "\n".join(lines))
    else:
        with open(md_path, "w") as f:
            f.write("\n".join(lines))
    print("\n".join(lines))


def trace_summary(db_path, md_path, title, command, append=False):
    """Per-kernel call counts and durations from a rocprofv3 kernel-trace
    database (its `top_kernels` view), as a markdown table."""
    import sqlite3
    db = sqlite3.connect(db_path)
    rows = db.execute("select name, total_calls, total_duration, average, percentage "
                      "from top_kernels order by total_duration desc").fetchall()
    lines = [f"# {title}", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | total (us) | average (us) | % |", "|---|---|---|---|---|"]
    for name, calls, total, avg, pct in rows[:12]:
        short = name.replace("ccl::(anonymous namespace)::", "").replace("void ", "")
        short = short.split("(")[0][:90]
        lines.append(f"| `{short}` | {calls} | {total:.1f} | {avg:.3f} | {pct:.2f} |")
    lines.append("")
    if append and os.path.exists(md_path):
        # one section per launch configuration in the same file
        lines[0] = "#" + lines[0]
        with open(md_path, "a") as f:
            f.write("\n" + "\n".join(lines))
    else:
        with open(md_path, "w") as f:
            f.write("\n".join(lines))
    print("\n".join(lines))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    r = sub.add_parser("run")
    r.add_argument("--depth", type=int)
    r.add_argument("--rows", type=int)
    r.add_argument("--batch", action="store_true", help="the 64-grid batch in both modes")
    r.add_argument("--specs-out", help="with --batch: where to write the launch specs")
    r.add_argument("--blocks", type=int, default=6)
    r.add_argument("--dims", type=int, default=2)
    s = sub.add_parser("summarise")
    s.add_argument("--fetch", required=True)
    s.add_argument("--write", required=True)
    s.add_argument("--depth", type=int, required=True)
    s.add_argument("--rows", type=int, required=True)
    s.add_argument("--md", required=True)
    s.add_argument("--dims", type=int, default=2)
    s.add_argument("--append", action="store_true",
                   help="add a section for this configuration to an existing summary")
    sb = sub.add_parser("summarise-batch")
    sb.add_argument("--fetch", required=True)
    sb.add_argument("--write", required=True)
    sb.add_argument("--specs", required=True)
    sb.add_argument("--md", required=True)
    t = sub.add_parser("trace-summary")
    t.add_argument("--db", required=True)
    t.add_argument("--md", required=True)
    t.add_argument("--title", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--append", action="store_true")
    c = sub.add_parser("counters")
    c.add_argument("--csv", action="append", required=True)
    c.add_argument("--depth", type=int, required=True)
    c.add_argument("--rows", type=int, required=True)
    c.add_argument("--dims", type=int, default=2)
    c.add_argument("--md", required=True)
    c.add_argument("--title")
    c.add_argument("--command", action="append", default=[])
    c.add_argument("--append", action="store_true")
    c.add_argument("--kernel-hash", help="source hash the counters were taken on, when it "
                                          "is not the current source's")
    a = ap.parse_args(argv)
    if a.cmd == "counters":
        counters(a.csv, a.depth, a.rows, a.md, a.dims, a.title, a.command, a.append,
                 a.kernel_hash)
        return 0
    if a.cmd == "trace-summary":
        trace_summary(a.db, a.md, a.title, a.command, a.append)
        return 0
    if a.cmd == "summarise-batch":
        summarise_batch(a.fetch, a.write, a.specs, a.md)
        return 0
    if a.cmd == "run":
        if a.batch:
            run_batch(a.specs_out)
        elif a.depth is None or a.rows is None:
            ap.error("run needs --depth and --rows, or --batch")
        else:
            run(a.depth, a.rows, a.blocks, a.dims)
    else:
        summarise(a.fetch, a.write, a.depth, a.rows, a.md, a.dims, a.append)
    return 0


if __name__ == "__main__":
    sys.exit(main())
