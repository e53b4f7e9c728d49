"""Learned launch-config selection: collect, train, evaluate.

    python -m paper_2505_06022_amd.learn collect  --out DIR [--shapes 250 --per-shape 16]
    python -m paper_2505_06022_amd.learn train    --data DIR/samples.json --model MODEL.json
    python -m paper_2505_06022_amd.learn evaluate --model MODEL.json --out DIR [--shapes 200]

collect  : seeded training shapes (2D, sides log-uniform on 256..16384), a
           seeded subset of each shape's candidates, each measured by the
           library's autotuner (time; device energy on an energy subset);
train    : the 12-64-64-2 MLP fitted on the GPU by the library's kernels;
evaluate : seeded held-out shapes never seen in training, each swept
           exhaustively (every candidate measured); the model's pick is
           judged by the measured sweep (ratio pick/best, time and energy),
           next to the default config without the model (T=1, 64 rows, K=1)
           and an untrained network's pick.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

TRAIN_SHAPE_SEED = 3
HELD_OUT_SEED = 4
SAMPLE_SEED = 5


def _log(msg):
    print(f"[learn] {msg}", flush=True)


def collect(out_dir, n_shapes=250, per_shape=16, energy_configs=0, energy_window_s=2.5,
            n_shapes_3d=40):
    from . import ccl_costmodel_features, tune
    os.makedirs(out_dir, exist_ok=True)
    shapes, cfgs = tune.sample_space(n_shapes, TRAIN_SHAPE_SEED, per_shape, SAMPLE_SEED,
                                     n_shapes_3d)
    _log(f"{len(cfgs)} configs over {len(shapes)} shapes")
    t0 = time.perf_counter()
    samples = []
    # measure shape by shape so progress is visible
    by_shape = {}
    for c in cfgs:
        by_shape.setdefault(tuple(c.shape[:c.dims]), []).append(c)
    for i, (sh, cs) in enumerate(by_shape.items()):
        samples.extend(tune.measure(cs))
        if (i + 1) % 25 == 0:
            _log(f"  {i + 1}/{len(by_shape)} shapes, {time.perf_counter() - t0:.0f} s")
    if energy_configs:
        rs = np.random.default_rng(SAMPLE_SEED + 1)
        pick = sorted(rs.choice(len(cfgs), size=min(energy_configs, len(cfgs)), replace=False))
        _log(f"energy windows for {len(pick)} configs")
        for j in pick:
            r = tune.measure([cfgs[j]], energy_window_s=energy_window_s)[0]
            samples[j]["j_per_step"] = r["j_per_step"]
            samples[j]["j_per_cell_step"] = r["j_per_cell_step"]
            samples[j]["window_s"] = r["window_s"]
    X = ccl_costmodel_features(cfgs)
    doc = dict(samples=samples, features=X.tolist(),
               meta=dict(shapes=len(shapes), configs=len(cfgs),
                         seconds=time.perf_counter() - t0))
    with open(os.path.join(out_dir, "samples.json"), "w") as f:
        json.dump(doc, f)
    _log(f"collected in {time.perf_counter() - t0:.0f} s")
    return doc


def train(data_path, model_path, epochs=4000, lr=3e-3, seed=0):
    from . import tune
    with open(data_path) as f:
        doc = json.load(f)
    X = np.array(doc["features"], dtype=np.float64)
    Y, W = tune.targets_of(doc["samples"])
    m = tune.CostModel.fit(X, Y, W, epochs=epochs, lr=lr, seed=seed)
    pred = m.predict(X)
    rmse = np.array([np.sqrt(np.sum(W[:, k] * (pred[:, k] - Y[:, k]) ** 2) / max(W[:, k].sum(), 1))
                     for k in range(2)])
    m.meta["train_rmse_log"] = rmse.tolist()
    m.save(model_path)
    _log(f"trained on {len(X)} samples in {m.meta['train_seconds']:.2f} s, "
         f"final loss {m.meta['final_loss']:.4g}, rmse(log t, log E) = {rmse}")
    return m


def evaluate(model_path, out_dir, n_shapes=200, energy_shapes=0, energy_window_s=2.5):
    """Exhaustive sweep of every held-out shape, and the ratio of the
    model's pick to the measured best (time; energy on a subset)."""
    from . import tune
    os.makedirs(out_dir, exist_ok=True)
    import synth
    shapes = synth.cost_model_shapes(n_shapes, HELD_OUT_SEED)
    model = tune.CostModel.load(model_path)
    untrained = tune.CostModel(tune.CostModel.init_params(1), model.xs, model.ys)
    rows = []
    t0 = time.perf_counter()
    for i, sh in enumerate(shapes):
        cfgs, res = tune.sweep(sh)
        t = np.array([r["s_per_step"] for r in res])
        best = int(np.argmin(t))
        pick_cfg, pick = model.pick(sh, "time")
        ucfg, upick = untrained.pick(sh, "time")
        default = next(j for j, c in enumerate(cfgs)
                       if c.nchunks == 1 and c.temporal_depth == 1 and c.tile_rows == 64)
        rows.append(dict(shape=list(sh), best=tune.cfg_key(cfgs[best]),
                         pick=tune.cfg_key(cfgs[pick]), t_best=t[best], t_pick=t[pick],
                         t_default=t[default], t_untrained=t[upick],
                         ratio=t[pick] / t[best], ratio_default=t[default] / t[best],
                         ratio_untrained=t[upick] / t[best]))
        if (i + 1) % 20 == 0:
            _log(f"  {i + 1}/{len(shapes)} shapes swept, {time.perf_counter() - t0:.0f} s")
    ratios = np.array([r["ratio"] for r in rows])
    summary = dict(
        shapes=len(rows),
        geomean_pick_over_best=float(np.exp(np.mean(np.log(ratios)))),
        frac_within_5pct=float(np.mean(ratios <= 1.05)),
        worst=float(ratios.max()),
        geomean_default_over_best=float(np.exp(np.mean(np.log([r["ratio_default"] for r in rows])))),
        geomean_untrained_over_best=float(np.exp(np.mean(np.log([r["ratio_untrained"] for r in rows])))),
        sweep_seconds=time.perf_counter() - t0,
    )
    if energy_shapes:
        erows = []
        for sh in shapes[:energy_shapes]:
            # energy of the measured-best-time config, the model's energy
            # pick and the energy-best among the top time candidates
            cfgs, res = tune.sweep(sh)
            t = np.array([r["s_per_step"] for r in res])
            order = np.argsort(t)[:4]
            pick_cfg, pick = model.pick(sh, "energy")
            idx = sorted(set(order.tolist()) | {pick})
            meas = tune.measure([cfgs[j] for j in idx], energy_window_s=energy_window_s)
            e = {j: m["j_per_step"] for j, m in zip(idx, meas)}
            best_e = min(e.values())
            erows.append(dict(shape=list(sh), e_pick=e[pick], e_best=best_e,
                              ratio=e[pick] / best_e))
        er = np.array([r["ratio"] for r in erows])
        summary["energy"] = dict(shapes=len(erows),
                                 geomean_pick_over_best=float(np.exp(np.mean(np.log(er)))),
                                 frac_within_5pct=float(np.mean(er <= 1.05)), rows=erows)
    with open(os.path.join(out_dir, "evaluation.json"), "w") as f:
        json.dump(dict(summary=summary, rows=rows), f)
    _log(json.dumps(summary))
    model.close()
    untrained.close()
    return summary


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--out", required=True)
    c.add_argument("--shapes", type=int, default=250)
    c.add_argument("--per-shape", type=int, default=16)
    c.add_argument("--energy-configs", type=int, default=0)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True)
    t.add_argument("--model", required=True)
    t.add_argument("--epochs", type=int, default=4000)
    t.add_argument("--lr", type=float, default=3e-3)
    e = sub.add_parser("evaluate")
    e.add_argument("--model", required=True)
    e.add_argument("--out", required=True)
    e.add_argument("--shapes", type=int, default=200)
    e.add_argument("--energy-shapes", type=int, default=0)
    a = ap.parse_args(argv)
    import torch
    torch.cuda.set_device(0)
    if a.cmd == "collect":
        collect(a.out, a.shapes, a.per_shape, a.energy_configs)
    elif a.cmd == "train":
        train(a.data, a.model, a.epochs, a.lr)
    else:
        evaluate(a.model, a.out, a.shapes, a.energy_shapes)
    return 0


if __name__ == "__main__":
    sys.exit(main())
