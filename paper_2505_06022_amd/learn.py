"""Learned launch-config selection: collect, train, evaluate.

    python -m paper_2505_06022_amd.learn collect  --out DIR [--shapes 250 --per-shape 16 --append]
    python -m paper_2505_06022_amd.learn energy   --out DIR [--count 120 --window 1.0]
    python -m paper_2505_06022_amd.learn remeasure --out DIR [--dims 3 --min-depth 2]
    python -m paper_2505_06022_amd.learn train    --data DIR/samples.json --model MODEL.json
    python -m paper_2505_06022_amd.learn evaluate --model MODEL.json --out DIR [--shapes 200]
    python -m paper_2505_06022_amd.learn energy-check --model MODEL.json --out DIR [--count 24]
    python -m paper_2505_06022_amd.learn summarise --out DIR [--model MODEL.json --dims 2]
    python -m paper_2505_06022_amd.learn report --out DIR --md profiles/costmodel_evaluation.md
    python -m paper_2505_06022_amd.learn export --data DIR/samples.json --csv costmodel_samples.csv

collect  : seeded training shapes (2D sides log-uniform on 256..16384, 3D
           sides 64..768), a seeded subset of each shape's candidates, each
           timed by the library's autotuner;
energy   : device energy for a seeded subset of those samples (each needs a
           window spanning two updates of the ~1 Hz energy counter);
remeasure: new time (and energy, where labelled) for the samples of one
           kernel family after that kernel changed, in place;
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
import os
import sys
import time

import numpy as np

TRAIN_SHAPE_SEED = 3
HELD_OUT_SEED = 4
SAMPLE_SEED = 5
TOP_K = (3, 5)


def _log(msg):
    print(f"[learn] {msg}", flush=True)


def _key(k):
    return (tuple(k[0]), int(k[1]), int(k[2]), int(k[3]))


def collect(out_dir, n_shapes=250, per_shape=16, n_shapes_3d=40, append=False, budget_s=1e9,
            n_shapes_3d_large=40):
    """Time samples of the seeded training configs, saved to samples.json.
    With `append`, configs already in samples.json are skipped and the new
    samples are added to it (saved every 10 shapes)."""
    from . import ccl_costmodel_features, tune
    os.makedirs(out_dir, exist_ok=True)
    shapes, cfgs = tune.sample_space(n_shapes, TRAIN_SHAPE_SEED, per_shape, SAMPLE_SEED,
                                     n_shapes_3d, n_shapes_3d_large)
    doc = dict(samples=[], features=[], meta={})
    path = os.path.join(out_dir, "samples.json")
    if append and os.path.exists(path):
        with open(path) as f:
            doc = json.load(f)
        have = {_key(s["key"]) for s in doc["samples"]}
        cfgs = [c for c in cfgs if _key(tune.cfg_key(c)) not in have]
    _log(f"{len(cfgs)} configs to measure over {len(shapes)} shapes")
    t0 = time.perf_counter()
    by_shape = {}
    for c in cfgs:
        by_shape.setdefault(tuple(c.shape[:c.dims]), []).append(c)
    for i, (sh, cs) in enumerate(by_shape.items()):
        doc["samples"].extend(tune.measure(cs))
        doc["features"].extend(ccl_costmodel_features(cs).tolist())
        if (i + 1) % 10 == 0:
            _save(out_dir, doc)
            _log(f"  {i + 1}/{len(by_shape)} shapes, {time.perf_counter() - t0:.0f} s")
        if time.perf_counter() - t0 > budget_s:
            _log("time budget reached")
            break
    doc["meta"] = dict(shapes=len(shapes), configs=len(doc["samples"]),
                       seconds=doc.get("meta", {}).get("seconds", 0.0) + time.perf_counter() - t0)
    _save(out_dir, doc)
    _log(f"{len(doc['samples'])} time samples after {time.perf_counter() - t0:.0f} s")
    return doc


SAMPLE_COLUMNS = ("shape", "chunks", "depth", "tile_rows", "steps", "s_per_step", "j_per_step",
                  "window_s")


def export_samples(doc, csv_path):
    """The time (and, where measured, energy) samples as a CSV table: the
    training set behind the committed model, from which `train` re-derives
    it (features are recomputed from each config)."""
    import csv
    with open(csv_path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(SAMPLE_COLUMNS)
        for smp in doc["samples"]:
            shape, K, T, rows = smp["key"]
            j = smp.get("j_per_step")
            w.writerow(["x".join(str(v) for v in shape), K, T, rows, smp["steps"],
                        f"{smp['s_per_step']:.6e}",
                        "" if j is None or not np.isfinite(j) else f"{j:.6e}",
                        f"{smp.get('window_s', 0.0):.3f}"])


def load_samples(path):
    """Samples from a samples.json (collect / energy output) or from the
    CSV table `export_samples` writes."""
    if not path.endswith(".csv"):
        with open(path) as f:
            return json.load(f)
    import csv
    samples = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            shape = [int(v) for v in r["shape"].split("x")]
            cells = float(np.prod(shape))
            t = float(r["s_per_step"])
            j = float(r["j_per_step"]) if r["j_per_step"] else float("nan")
            samples.append(dict(key=[shape, int(r["chunks"]), int(r["depth"]), int(r["tile_rows"])],
                                steps=int(r["steps"]), s_per_step=t, j_per_step=j,
                                s_per_cell_step=t / cells, j_per_cell_step=j / cells,
                                window_s=float(r["window_s"])))
    return dict(samples=samples, meta={})


def _save(out_dir, doc):
    tmp = os.path.join(out_dir, "samples.json.tmp")
    with open(tmp, "w") as f:
        json.dump(doc, f)
    os.replace(tmp, os.path.join(out_dir, "samples.json"))


def energy(out_dir, count=120, window_s=1.0, budget_s=600.0):
    """Adds device-energy labels to a seeded subset of the collected samples
    (resumable: samples that already have one are skipped)."""
    from . import make_tune_config, tune
    path = os.path.join(out_dir, "samples.json")
    with open(path) as f:
        doc = json.load(f)
    samples = doc["samples"]
    # a seeded permutation: a larger count extends the same subset
    rs = np.random.default_rng(SAMPLE_SEED + 1)
    pick = rs.permutation(len(samples))[:count]
    t0 = time.perf_counter()
    done = 0
    for n, j in enumerate(pick):
        s = samples[int(j)]
        if s.get("j_per_cell_step") is not None and np.isfinite(s["j_per_cell_step"]):
            done += 1
            continue
        shape, K, T, rows = s["key"]
        c = make_tune_config(shape, K, T, rows)
        r = tune.measure([c], energy_window_s=window_s)[0]
        s["j_per_step"], s["j_per_cell_step"] = r["j_per_step"], r["j_per_cell_step"]
        s["window_s"] = r["window_s"]
        done += 1
        if done % 5 == 0:
            _log(f"  energy {done}/{len(pick)}, {time.perf_counter() - t0:.0f} s")
            _save(out_dir, doc)
        if time.perf_counter() - t0 > budget_s:
            break
    _save(out_dir, doc)
    _log(f"energy labels: {done}/{len(pick)} in {time.perf_counter() - t0:.0f} s")


def remeasure(out_dir, dims=3, min_depth=2, window_s=1.0):
    """Re-measures in place the samples of one kernel family (domains of
    `dims` dimensions at depth T >= min_depth), for use after that kernel
    changed: every such sample gets a new time, and those that held an
    energy label a new energy label, so the labelled subset and the order
    of the samples stay as they were."""
    from . import ccl_costmodel_features, make_tune_config, tune
    path = os.path.join(out_dir, "samples.json")
    with open(path) as f:
        doc = json.load(f)
    samples, feats = doc["samples"], doc["features"]
    by_shape = {}
    for j, s in enumerate(samples):
        shape, _, T, _ = s["key"]
        if len(shape) == dims and T >= min_depth:
            by_shape.setdefault(tuple(shape), []).append(j)
    _log(f"{sum(map(len, by_shape.values()))} samples over {len(by_shape)} shapes to re-measure")
    t0 = time.perf_counter()
    relabelled = 0
    for i, (sh, idx) in enumerate(by_shape.items()):
        cfgs = [make_tune_config(*samples[j]["key"]) for j in idx]
        new = tune.measure(cfgs)
        x = ccl_costmodel_features(cfgs).tolist()
        for j, c, r, f in zip(idx, cfgs, new, x):
            old = samples[j]
            had_energy = old.get("j_per_cell_step") is not None and np.isfinite(
                old["j_per_cell_step"])
            if had_energy:
                e = tune.measure([c], energy_window_s=window_s)[0]
                r["j_per_step"], r["j_per_cell_step"] = e["j_per_step"], e["j_per_cell_step"]
                r["window_s"] = e["window_s"]
                relabelled += 1
            samples[j], feats[j] = r, f
        if (i + 1) % 10 == 0:
            _save(out_dir, doc)
            _log(f"  {i + 1}/{len(by_shape)} shapes, {relabelled} energy labels, "
                 f"{time.perf_counter() - t0:.0f} s")
    doc["meta"]["remeasured"] = dict(dims=dims, min_depth=min_depth,
                                     samples=sum(map(len, by_shape.values())),
                                     energy_labels=relabelled,
                                     seconds=time.perf_counter() - t0)
    _save(out_dir, doc)
    _log(f"re-measured {sum(map(len, by_shape.values()))} samples ({relabelled} energy labels) "
         f"in {time.perf_counter() - t0:.0f} s")


def _pick_quality(model, X, Y, groups):
    """Geometric mean over groups (the sampled configs of one shape) of the
    measured time of the model's pick among them over the group's measured
    best: how well the model ranks configs it was not trained on."""
    pred = model.predict(X)
    r = []
    for idx in groups:
        if len(idx) < 2:
            continue
        p = idx[int(np.argmin(pred[idx, 0]))]
        b = idx[int(np.argmin(Y[idx, 0]))]
        r.append(Y[p, 0] - Y[b, 0])
    return float(np.exp(np.mean(r))) if r else float("nan")


def train(data_path, model_path, epochs=4000, lr=3e-3, seed=0, seeds=1, val_frac=0.2):
    """Fits the model to the samples; features are recomputed from each
    sample's config, so they always follow the library's current
    definition (and this device's occupancy).  With seeds > 1 the
    initialisation seed is chosen first: for each of `seeds` seeds a model is
    fitted without a seeded `val_frac` of the training shapes and judged on
    how well it ranks those shapes' sampled configs; the chosen seed is then
    fitted on all samples."""
    from . import ccl_costmodel_features, make_tune_config, tune
    doc = load_samples(data_path)
    keys = [s["key"] for s in doc["samples"]]
    cfgs = [make_tune_config(tuple(k[0]), int(k[1]), int(k[2]), int(k[3])) for k in keys]
    X = ccl_costmodel_features(cfgs).astype(np.float64)
    Y, W = tune.targets_of(doc["samples"])
    selection = None
    if seeds > 1:
        by_shape = {}
        for i, k in enumerate(keys):
            by_shape.setdefault(tuple(k[0]), []).append(i)
        shapes = sorted(by_shape)
        rs = np.random.default_rng(SAMPLE_SEED + 2)
        val = set(tuple(shapes[j]) for j in rs.permutation(len(shapes))[:int(val_frac * len(shapes))])
        tr = np.array([i for i, k in enumerate(keys) if tuple(k[0]) not in val])
        groups = [np.array(by_shape[sh]) for sh in shapes if sh in val]
        scores = {}
        for sd in range(seed, seed + seeds):
            m = tune.CostModel.fit(X[tr], Y[tr], W[tr], epochs=epochs, lr=lr, seed=sd)
            scores[sd] = _pick_quality(m, X, Y, groups)
            m.close()
            _log(f"  seed {sd}: validation pick/best {scores[sd]:.4f}")
        seed = min(scores, key=scores.get)
        selection = dict(val_shapes=len(groups), scores={str(k): v for k, v in scores.items()},
                         chosen=seed)
    m = tune.CostModel.fit(X, Y, W, epochs=epochs, lr=lr, seed=seed)
    pred = m.predict(X)
    rmse = np.array([np.sqrt(np.sum(W[:, k] * (pred[:, k] - Y[:, k]) ** 2) / max(W[:, k].sum(), 1))
                     for k in range(2)])
    m.meta["train_rmse_log"] = rmse.tolist()
    if selection:
        m.meta["seed_selection"] = selection
    m.save(model_path)
    _log(f"trained on {len(X)} samples in {m.meta['train_seconds']:.2f} s (seed {seed}), "
         f"final loss {m.meta['final_loss']:.4g}, rmse(log t, log W) = {rmse}")
    return m


def training_shapes():
    """Every shape the training samples come from (2D and 3D)."""
    from . import tune
    shapes, _ = tune.sample_space(250, TRAIN_SHAPE_SEED, 0, SAMPLE_SEED, 40, 40)
    return set(tuple(s) for s in shapes)


def held_out_shapes(n_shapes, dims=2):
    """Seeded held-out shapes: 2D as the training shapes' distribution, 3D
    with sides 64..768, drawn from seeds that no training set uses; a drawn
    shape that is also a training shape, or was drawn before, is skipped
    and the next one drawn instead, so the n_shapes are distinct and none
    was seen in training."""
    import synth
    train = training_shapes()
    draw = (lambda k: synth.cost_model_shapes(k, HELD_OUT_SEED)) if dims == 2 else \
        (lambda k: synth.cost_model_shapes_3d(k, HELD_OUT_SEED + 100))
    k = n_shapes
    while True:
        out, seen = [], set()
        for sh in draw(k):  # the draws are prefix-stable in k
            if sh in train or sh in seen:
                continue
            seen.add(sh)
            out.append(sh)
            if len(out) == n_shapes:
                return out
        k *= 2


def _tag(dims):
    return "" if dims == 2 else "_3d"


def evaluate(model_path, out_dir, n_shapes=200, start=0, count=None, budget_s=1e9,
             reps=2, target_cell_steps=1.5e9, dims=2):
    """Exhaustive time sweep of held-out shapes [start, start+count): every
    candidate measured; rows written to evaluation[_3d]_part_<start>.json."""
    from . import tune
    os.makedirs(out_dir, exist_ok=True)
    shapes = held_out_shapes(n_shapes, dims)
    count = len(shapes) - start if count is None else count
    model = tune.CostModel.load(model_path)
    untrained = tune.CostModel(tune.CostModel.init_params(1), model.xs, model.ys)
    rows = []
    t0 = time.perf_counter()
    path = os.path.join(out_dir, f"evaluation{_tag(dims)}_part_{start:04d}.json")
    for i, sh in enumerate(shapes[start:start + count]):
        cfgs = tune.candidates(sh)
        res = tune.measure(cfgs, reps=reps,
                           steps=tune.steps_for(sh, target_cell_steps=target_cell_steps))
        t = np.array([r["s_per_step"] for r in res])
        best = int(np.argmin(t))
        keys = [tune.cfg_key(c) for c in cfgs]
        pick_cfg, _ = model.pick(sh, "time")
        ucfg, _ = untrained.pick(sh, "time")
        pick = keys.index(tune.cfg_key(pick_cfg))
        upick = keys.index(tune.cfg_key(ucfg))
        default = keys.index((tuple(sh), 1, 1, 0))
        # the model's k best candidates, of which the measured fastest is
        # taken (k measurements instead of the sweep's len(cfgs))
        order = model.rank(sh, "time")
        topk = {k: min(t[j] for j in order[:k]) for k in TOP_K}
        rows.append(dict(index=start + i, shape=list(sh), best=keys[best], pick=keys[pick],
                         t_best=t[best], t_pick=t[pick], t_default=t[default],
                         t_untrained=t[upick], ratio=t[pick] / t[best],
                         ratio_default=t[default] / t[best],
                         ratio_untrained=t[upick] / t[best],
                         **{f"ratio_top{k}": v / t[best] for k, v in topk.items()},
                         t_all=[float(v) for v in t]))
        _log(f"  shape {start + i} {sh}: pick/best {t[pick] / t[best]:.3f}, "
             f"default/best {t[default] / t[best]:.2f} ({time.perf_counter() - t0:.0f} s)")
        with open(path, "w") as f:
            json.dump(rows, f)
        if time.perf_counter() - t0 > budget_s:
            break
    model.close()
    untrained.close()
    return rows


def energy_check(model_path, out_dir, n_shapes=200, start=0, count=24, window_s=1.0, top=10,
                 repeats=3, budget_s=1e9):
    """For held-out shapes [start, start+count): device energy of the model's
    energy pick, of its time pick and of the `top` fastest configs of the
    time sweep (the energy judge is restricted to those, since a full energy
    sweep would need ~2 s of counter time per candidate).  Each config's
    energy is the median over `repeats` windows with a valid reading: one
    window reads the ~1 Hz counter at two updates only, and now and then a
    window reads a third to two thirds of what the windows around it read;
    the median of three discards one such reading.  Rows are written to
    energy_check_part_<start>.json after every shape."""
    from . import tune
    os.makedirs(out_dir, exist_ok=True)
    shapes = held_out_shapes(n_shapes)[start:start + count]
    model = tune.CostModel.load(model_path)
    out = []
    t0 = time.perf_counter()
    path = os.path.join(out_dir, f"energy_check_part_{start:04d}.json")
    for i, sh in enumerate(shapes):
        cfgs = tune.candidates(sh)
        res = tune.measure(cfgs, reps=2, steps=tune.steps_for(sh, target_cell_steps=1.5e9))
        keys = [tune.cfg_key(c) for c in cfgs]
        order = list(np.argsort([r["s_per_step"] for r in res])[:top])
        pick_cfg, _ = model.pick(sh, "energy")
        pick = keys.index(tune.cfg_key(pick_cfg))
        tpick_cfg, _ = model.pick(sh, "time")
        tpick = keys.index(tune.cfg_key(tpick_cfg))
        # the model's three best by predicted energy, the least of them as
        # measured (as the launcher verifies its time shortlist)
        top3 = [int(j) for j in model.rank(sh, "energy")[:3]]
        idx = sorted(set(int(j) for j in order) | {pick, tpick} | set(top3))
        reads = {j: [] for j in idx}
        for _ in range(repeats):
            meas = tune.measure([cfgs[j] for j in idx], energy_window_s=window_s)
            for j, m in zip(idx, meas):
                v = m["j_per_step"]
                if v is not None and np.isfinite(v) and v > 0:
                    reads[j].append(v)
        e = {j: float(np.median(v)) for j, v in reads.items() if v}
        if pick not in e or tpick not in e:
            _log(f"  energy {sh}: no valid energy window for a pick; shape skipped")
            continue
        # the judge: the least energy among the ten fastest configs of the
        # time sweep and the model's candidates
        best = min(e, key=e.get)
        e3 = min(e[j] for j in top3 if j in e) if any(j in e for j in top3) else float("nan")
        out.append(dict(index=start + i, shape=list(sh), pick=keys[pick], time_pick=keys[tpick],
                        best=keys[best], e_pick=e[pick], e_time_pick=e[tpick], e_best=e[best],
                        ratio=e[pick] / e[best], ratio_time_pick=e[tpick] / e[best],
                        ratio_top3=e3 / e[best],
                        reads={str(keys[j][1:]): v for j, v in reads.items()},
                        time_pick_over_best=res[pick]["s_per_step"] / res[order[0]]["s_per_step"]))
        _log(f"  energy {sh}: pick/best {e[pick] / e[best]:.3f} ({keys[pick][1:]} vs "
             f"{keys[best][1:]}), time pick/best {e[tpick] / e[best]:.3f} "
             f"({time.perf_counter() - t0:.0f} s)")
        with open(path, "w") as f:
            json.dump(out, f)
        if time.perf_counter() - t0 > budget_s:
            break
    model.close()
    return out


def rescore_energy(model_path, out_dir):
    """Re-applies the model's current energy-pick rule to stored energy-check
    rows: the rule only decides whether the energy pick falls back to the
    time pick, and both were measured, so each row's pick and its energy
    are updated from the stored measurements (no new measurement)."""
    import glob
    from . import tune
    model = tune.CostModel.load(model_path)
    changed = 0
    try:
        for p in sorted(glob.glob(os.path.join(out_dir, "energy_check_part_*.json"))):
            with open(p) as f:
                rows = json.load(f)
            for r in rows:
                sh = tuple(r["shape"])
                key = list(tune.cfg_key(model.pick(sh, "energy")[0]))
                key[0] = list(key[0])
                if key == r["time_pick"] and r["pick"] != r["time_pick"]:
                    r["pick"], r["e_pick"], r["ratio"] = r["time_pick"], r["e_time_pick"], \
                        r["ratio_time_pick"]
                    changed += 1
                elif key != r["pick"]:
                    raise RuntimeError(f"{sh}: pick {key} is neither the stored energy pick "
                                       f"{r['pick']} nor the time pick {r['time_pick']}")
            with open(p, "w") as f:
                json.dump(rows, f)
    finally:
        model.close()
    _log(f"rescored energy rows: {changed} picks fall back to the time pick")
    return changed


def summarise(out_dir, model_path=None, dims=2):
    """Merges evaluation parts into evaluation[_3d].json with the summary
    (also stored in the model's metadata when `model_path` is given)."""
    import glob
    rows = []
    for p in sorted(glob.glob(os.path.join(out_dir, f"evaluation{_tag(dims)}_part_*.json"))):
        with open(p) as f:
            rows.extend(json.load(f))
    seen = {}
    for r in rows:
        seen[r["index"]] = r
    rows = [seen[k] for k in sorted(seen)]
    ratios = np.array([r["ratio"] for r in rows])
    gm = lambda a: float(np.exp(np.mean(np.log(a))))
    summary = dict(shapes=len(rows), geomean_pick_over_best=gm(ratios),
                   frac_within_5pct=float(np.mean(ratios <= 1.05)), worst=float(ratios.max()),
                   geomean_default_over_best=gm([r["ratio_default"] for r in rows]),
                   geomean_untrained_over_best=gm([r["ratio_untrained"] for r in rows]))
    for k in TOP_K:
        if all(f"ratio_top{k}" in r for r in rows):
            rk = np.array([r[f"ratio_top{k}"] for r in rows])
            summary[f"top{k}_verified"] = dict(geomean_over_best=gm(rk),
                                               frac_within_5pct=float(np.mean(rk <= 1.05)),
                                               worst=float(rk.max()))
    by_index = {}  # a shape measured in two parts counts once (the later part)
    for p in sorted(glob.glob(os.path.join(out_dir, "energy_check_part_*.json"))):
        with open(p) as f:
            for r in json.load(f):
                by_index[r["index"]] = r
    er = [by_index[i] for i in sorted(by_index)]
    if dims == 2 and er:
        summary["energy"] = dict(
            shapes=len(er), judge="median of 3 windows; the 10 fastest of the time sweep, the "
                                  "energy pick and the time pick",
            geomean_pick_over_best=gm([r["ratio"] for r in er]),
            frac_within_5pct=float(np.mean([r["ratio"] <= 1.05 for r in er])),
            worst=float(max(r["ratio"] for r in er)),
            geomean_time_pick_over_best=gm([r["ratio_time_pick"] for r in er]),
            geomean_top3_verified_over_best=gm([r["ratio_top3"] for r in er
                                                if np.isfinite(r.get("ratio_top3", np.nan))]),
            # the launcher's energy choice: the least measured of the top 3
            # by predicted energy and the time pick
            geomean_verified_choice_over_best=gm([min(r["ratio_top3"], r["ratio_time_pick"])
                                                  for r in er
                                                  if np.isfinite(r.get("ratio_top3", np.nan))]),
            frac_pick_no_worse_than_time_pick=float(np.mean(
                [r["e_pick"] <= r["e_time_pick"] * 1.02 for r in er])))
        with open(os.path.join(out_dir, "energy_check.json"), "w") as f:
            json.dump(er, f)
    with open(os.path.join(out_dir, f"evaluation{_tag(dims)}.json"), "w") as f:
        json.dump(dict(summary=summary, rows=rows), f)
    if model_path:
        with open(model_path) as f:
            doc = json.load(f)
        doc.setdefault("meta", {})[f"evaluation{_tag(dims)}"] = summary
        with open(model_path, "w") as f:
            json.dump(doc, f)
    _log(json.dumps(summary))
    return summary


def report(out_dir, md_path):
    """Per-shape rows of the evaluations (2D, 3D) and of the energy check as
    one markdown file: shape, the sweep's best config, the model's pick and
    the measured ratios."""
    lines = ["# Cost-model evaluation on held-out shapes, per shape", "",
             "Configs are (K chunks, T, tile rows; 0 = automatic). Ratios are measured "
             "time (or energy) over the best of the judge set, on the same kernels.", ""]
    for dims in (2, 3):
        p = os.path.join(out_dir, f"evaluation{_tag(dims)}.json")
        if not os.path.exists(p):
            continue
        with open(p) as f:
            doc = json.load(f)
        sm = doc["summary"]
        lines += [f"## {dims}D time: {sm['shapes']} shapes, every candidate measured", "",
                  "summary-json: " + json.dumps(sm), "",
                  "| # | shape | best | pick | pick/best | top-3/best | default/best |",
                  "|---|---|---|---|---|---|---|"]
        for r in doc["rows"]:
            lines.append(f"| {r['index']} | {'x'.join(map(str, r['shape']))} | "
                         f"{tuple(r['best'][1:])} | {tuple(r['pick'][1:])} | {r['ratio']:.3f} | "
                         f"{r.get('ratio_top3', float('nan')):.3f} | {r['ratio_default']:.2f} |")
        lines.append("")
    p = os.path.join(out_dir, "energy_check.json")
    if os.path.exists(p):
        with open(p) as f:
            er = json.load(f)
        lines += [f"## 2D energy: {len(er)} shapes, median of 3 windows per config", "",
                  "| # | shape | least energy | energy pick | pick/least | time pick/least | "
                  "energy top-3 measured/least | measured choice/least |",
                  "|---|---|---|---|---|---|---|---|"]
        for r in er:
            t3 = r.get('ratio_top3', float('nan'))
            lines.append(f"| {r['index']} | {'x'.join(map(str, r['shape']))} | "
                         f"{tuple(r['best'][1:])} | {tuple(r['pick'][1:])} | {r['ratio']:.3f} | "
                         f"{r['ratio_time_pick']:.3f} | {t3:.3f} | "
                         f"{min(t3, r['ratio_time_pick']):.3f} |")
        lines.append("")
    with open(md_path, "w") as f:
        f.write("\n".join(lines))
    _log(f"wrote {md_path}")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__,
                                 formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    c = sub.add_parser("collect")
    c.add_argument("--out", required=True)
    c.add_argument("--shapes", type=int, default=250)
    c.add_argument("--shapes-3d", type=int, default=40)
    c.add_argument("--shapes-3d-large", type=int, default=40)
    c.add_argument("--per-shape", type=int, default=16)
    c.add_argument("--append", action="store_true")
    c.add_argument("--budget", type=float, default=1e9)
    en = sub.add_parser("energy")
    en.add_argument("--out", required=True)
    en.add_argument("--count", type=int, default=120)
    en.add_argument("--window", type=float, default=1.0)
    en.add_argument("--budget", type=float, default=600.0)
    rm = sub.add_parser("remeasure")
    rm.add_argument("--out", required=True)
    rm.add_argument("--dims", type=int, default=3)
    rm.add_argument("--min-depth", type=int, default=2)
    rm.add_argument("--window", type=float, default=1.0)
    t = sub.add_parser("train")
    t.add_argument("--data", required=True)
    t.add_argument("--model", required=True)
    t.add_argument("--epochs", type=int, default=4000)
    t.add_argument("--lr", type=float, default=3e-3)
    t.add_argument("--seeds", type=int, default=1)
    e = sub.add_parser("evaluate")
    e.add_argument("--model", required=True)
    e.add_argument("--out", required=True)
    e.add_argument("--shapes", type=int, default=200)
    e.add_argument("--start", type=int, default=0)
    e.add_argument("--count", type=int, default=None)
    e.add_argument("--budget", type=float, default=1e9)
    e.add_argument("--dims", type=int, default=2, choices=(2, 3))
    ec = sub.add_parser("energy-check")
    ec.add_argument("--model", required=True)
    ec.add_argument("--out", required=True)
    ec.add_argument("--start", type=int, default=0)
    ec.add_argument("--count", type=int, default=24)
    ec.add_argument("--top", type=int, default=10)
    ec.add_argument("--repeats", type=int, default=3)
    ec.add_argument("--budget", type=float, default=1e9)
    ex = sub.add_parser("export")
    ex.add_argument("--data", required=True)
    ex.add_argument("--csv", required=True)
    rp = sub.add_parser("report")
    rp.add_argument("--out", required=True)
    rp.add_argument("--md", required=True)
    rs = sub.add_parser("rescore-energy")
    rs.add_argument("--model", required=True)
    rs.add_argument("--out", required=True)
    sm = sub.add_parser("summarise")
    sm.add_argument("--out", required=True)
    sm.add_argument("--model", default=None)
    sm.add_argument("--dims", type=int, default=2, choices=(2, 3))
    a = ap.parse_args(argv)
    if a.cmd not in ("summarise", "report", "export"):
        import torch
        torch.cuda.set_device(0)
    if a.cmd == "collect":
        collect(a.out, a.shapes, a.per_shape, a.shapes_3d, a.append, a.budget,
                a.shapes_3d_large)
    elif a.cmd == "energy":
        energy(a.out, a.count, a.window, a.budget)
    elif a.cmd == "remeasure":
        remeasure(a.out, a.dims, a.min_depth, a.window)
    elif a.cmd == "train":
        train(a.data, a.model, a.epochs, a.lr, seeds=a.seeds)
    elif a.cmd == "evaluate":
        evaluate(a.model, a.out, a.shapes, a.start, a.count, a.budget, dims=a.dims)
    elif a.cmd == "energy-check":
        energy_check(a.model, a.out, start=a.start, count=a.count, top=a.top,
                     repeats=a.repeats, budget_s=a.budget)
    elif a.cmd == "rescore-energy":
        rescore_energy(a.model, a.out)
    elif a.cmd == "report":
        report(a.out, a.md)
    elif a.cmd == "export":
        export_samples(load_samples(a.data), a.csv)
    else:
        summarise(a.out, a.model, a.dims)
    return 0


if __name__ == "__main__":
    sys.exit(main())
