"""Autotuner and learned cost model for ccl_wave_step launch configs.

* ``candidates(shape)`` — the discrete config space of one shape, as the
  library enumerates it (ccl_autotune_candidates): chunk counts K in
  {1, 2, 4, 8, 16} (K <= rows), rows per tile in {auto, 16, 32, 64, 128},
  temporal depth T in 1..8 (2D and 3D).
* ``measure(cfgs)`` — time (and device energy) per step of each config,
  measured by the library's autotuner on the GPU (ccl_autotune_measure).
* ``CostModel`` — the 12-64-64-2 MLP, trained on the GPU by the library's
  kernels (ccl_mlp_*) on standardised features (ccl_costmodel_features) and
  standardised targets [log s/cell-step, log W (device power)]; ``pick`` scores
  every candidate of a shape on the GPU (ccl_mlp_pick) and returns the best
  by time, energy or energy-delay product.
* ``sweep`` — the exhaustive measurement of every candidate
  (ccl_autotune_sweep): the fallback when no model is available and the
  judge of a model's picks.

The sample and held-out shape sets are drawn from ``synth`` (seeded).
"""
from __future__ import annotations

import json
import math
import os
import time
from dataclasses import dataclass

import numpy as np

from . import (CCL_MLP_NPARAMS, CCL_MLP_PARAMS, CCL_MLP_LOSS, ccl_autotune_candidates,
               ccl_autotune_measure, ccl_autotune_sweep, ccl_costmodel_features,
               ccl_mlp_create, ccl_mlp_destroy, ccl_mlp_get, ccl_mlp_pick, ccl_mlp_rank,
               ccl_mlp_train, make_tune_config)

# weights on the model's outputs [log s/cell-step, log W]: log energy =
# log time + log power, log (energy x delay) = 2 log time + log power
OBJECTIVES = {"time": (1.0, 0.0), "energy": (1.0, 1.0), "edp": (2.0, 1.0)}


def candidates(shape):
    return ccl_autotune_candidates(tuple(int(v) for v in shape))


def sweep(shape, nchunks=0, r2=0.25, steps=None, reps=3, objective="time",
          energy_window_s=0.0):
    """Every candidate of `shape` (only K == nchunks when nchunks > 0)
    measured by the library (ccl_autotune_sweep); returns (configs, one dict
    per config as measure() gives them, index of the best by `objective`)."""
    st = steps or steps_for(shape)
    cfgs, samples, best = ccl_autotune_sweep(shape, nchunks, r2, st, reps, energy_window_s,
                                             objective)
    cells = float(np.prod(shape))
    res = [dict(key=cfg_key(c), steps=st, s_per_step=o.seconds_per_step,
                j_per_step=o.joules_per_step, s_per_cell_step=o.seconds_per_step / cells,
                j_per_cell_step=o.joules_per_step / cells, window_s=o.window_seconds)
           for c, o in zip(cfgs, samples)]
    return cfgs, res, best


def cfg_key(c):
    return (tuple(c.shape[:c.dims]), c.nchunks, c.temporal_depth, c.tile_rows)


def steps_for(shape, target_cell_steps=3e9):
    cells = float(np.prod(shape))
    s = int(round(target_cell_steps / cells / 24.0)) * 24
    return int(min(960, max(24, s)))


def measure(cfgs, r2=0.25, reps=3, energy_window_s=0.0, steps=None, target_cell_steps=3e9):
    """Measures configs grouped by shape; returns one dict per config."""
    by_shape = {}
    for i, c in enumerate(cfgs):
        by_shape.setdefault(tuple(c.shape[:c.dims]), []).append(i)
    out = [None] * len(cfgs)
    for shape, idx in by_shape.items():
        st = steps or steps_for(shape, target_cell_steps)
        res = ccl_autotune_measure([cfgs[i] for i in idx], r2, st, reps, energy_window_s)
        cells = float(np.prod(shape))
        for i, r in zip(idx, res):
            out[i] = dict(key=cfg_key(cfgs[i]), steps=st, s_per_step=r.seconds_per_step,
                          j_per_step=r.joules_per_step, s_per_cell_step=r.seconds_per_step / cells,
                          j_per_cell_step=r.joules_per_step / cells, window_s=r.window_seconds)
    return out


def targets_of(samples):
    """Targets [log s/cell-step, log W] and weights.  The second output is
    the mean device power while the config runs (J/step / s/step); energy
    per cell-step is then the sum of the two logs.  Power varies far less
    across configs than time does, so the few samples with an energy label
    constrain it well.  Weight 0 where no energy was measured (the target
    slot then holds 0)."""
    t = np.zeros((len(samples), 2))
    w = np.ones((len(samples), 2))
    for i, s in enumerate(samples):
        t[i, 0] = math.log(s["s_per_cell_step"])
        e = s.get("j_per_cell_step")
        if e is not None and np.isfinite(e) and e > 0:
            t[i, 1] = math.log(e / s["s_per_cell_step"])
        else:
            w[i, 1] = 0.0
    return t, w


@dataclass
class Standardiser:
    mean: np.ndarray
    std: np.ndarray

    def apply(self, a):
        return ((a - self.mean) / self.std).astype(np.float32)

    def invert(self, a):
        return a * self.std + self.mean


class CostModel:
    """The MLP plus its feature and target standardisation."""

    def __init__(self, params, xs: Standardiser, ys: Standardiser, meta=None):
        self.params = np.asarray(params, dtype=np.float32).ravel()
        self.xs, self.ys = xs, ys
        self.meta = dict(meta or {})
        self.handle = ccl_mlp_create(self.params)

    @staticmethod
    def init_params(seed: int):
        import synth
        ws, bs = synth.mlp_params((12, 64, 64, 2), seed, dtype=np.float32)
        return pack(ws, bs)

    @classmethod
    def fit(cls, X, Y, W=None, epochs=3000, lr=3e-3, seed=0, stream=None):
        """W (n x 2, optional): 1 where a target was measured, 0 where not."""
        import torch
        W = np.ones_like(Y) if W is None else np.asarray(W, np.float64)
        xs = Standardiser(X.mean(0), np.where(X.std(0) > 1e-9, X.std(0), 1.0))
        ym = np.array([np.sum(W[:, k] * Y[:, k]) / max(W[:, k].sum(), 1) for k in range(2)])
        yv = np.array([np.sum(W[:, k] * (Y[:, k] - ym[k]) ** 2) / max(W[:, k].sum(), 1)
                       for k in range(2)])
        ys = Standardiser(ym, np.where(yv > 1e-18, np.sqrt(yv), 1.0))
        m = cls(cls.init_params(seed), xs, ys, meta=dict(epochs=epochs, lr=lr, seed=seed,
                                                         n=int(len(X)),
                                                         n_energy=int(W[:, 1].sum())))
        xd = torch.from_numpy(xs.apply(X)).cuda()
        yd = torch.from_numpy(np.where(W > 0, ys.apply(Y), 0.0).astype(np.float32)).cuda()
        wd = torch.from_numpy(W.astype(np.float32)).cuda()
        t0 = time.perf_counter()
        ccl_mlp_train(m.handle, len(X), xd.data_ptr(), yd.data_ptr(), epochs, lr, stream,
                      w_ptr=wd.data_ptr())
        torch.cuda.synchronize()
        m.meta["train_seconds"] = time.perf_counter() - t0
        m.meta["final_loss"] = float(ccl_mlp_get(m.handle, CCL_MLP_LOSS)[0])
        m.params = ccl_mlp_get(m.handle, CCL_MLP_PARAMS)
        return m

    def predict(self, X):
        """Predicted [log s/cell-step, log W] (host arrays)."""
        import torch

        from . import ccl_mlp_forward
        xd = torch.from_numpy(self.xs.apply(X)).cuda()
        yd = torch.empty((len(X), 2), dtype=torch.float32, device="cuda")
        ccl_mlp_forward(self.handle, len(X), xd.data_ptr(), yd.data_ptr())
        torch.cuda.synchronize()
        return self.ys.invert(yd.cpu().numpy().astype(np.float64))

    # A predicted energy (or EDP) saving over the time pick smaller than
    # this (log units) is not acted on.  A predicted energy is predicted
    # time times predicted power, and the time head's error on its training
    # samples is about 4.6% (rmse of log t; the power head's about 1%), so
    # smaller predicted savings are within the model's own error.  The rule
    # does not make the raw energy pick reliable: on 24 held-out shapes the
    # pick differed from the time pick on 14 (predicted savings above 5% on
    # all of them) and measured more energy on 11; the launcher's energy
    # choice is therefore measured (pick_verified).
    MIN_SAVING = 0.05

    def pick(self, shape, objective="time", nchunks=None, shortlist=8):
        """Best candidate of `shape` by the model (only those with `nchunks`
        chunks when given); returns (config, index into that list).  The
        argmin runs on the GPU (ccl_mlp_pick).  For energy and EDP the pick
        is made among the `shortlist` candidates predicted fastest: power
        varies by a few percent across configs and is labelled for few of
        them, so a slow config is never chosen for a predicted power saving
        the model cannot back; and the time pick is kept unless the other
        candidate's predicted saving exceeds MIN_SAVING."""
        import torch
        cfgs = candidates(shape)
        if nchunks is not None:
            cfgs = [c for c in cfgs if c.nchunks == nchunks]
        X = ccl_costmodel_features(cfgs)
        base = list(range(len(cfgs)))
        if objective != "time" and shortlist and len(cfgs) > shortlist:
            t = self.predict(X)[:, 0]
            base = sorted(np.argsort(t, kind="stable")[:shortlist].tolist())
            X = X[base]
        w = OBJECTIVES[objective]
        # scores in standardised target units, weighted back to log units
        wt, we = w[0] * float(self.ys.std[0]), w[1] * float(self.ys.std[1])
        xd = torch.from_numpy(self.xs.apply(X)).cuda()
        best = torch.zeros(1, dtype=torch.int32, device="cuda")
        ccl_mlp_pick(self.handle, len(X), xd.data_ptr(), wt, we, 0, best.data_ptr())
        torch.cuda.synchronize()
        i = base[int(best.item())]
        if objective != "time":
            tcfg, ti = self.pick(shape, "time", nchunks)
            y = self.predict(ccl_costmodel_features([cfgs[i], cfgs[ti]]))
            score = w[0] * y[:, 0] + w[1] * y[:, 1]
            if score[1] - score[0] < self.MIN_SAVING:
                return tcfg, ti
        return cfgs[i], i

    def rank(self, shape, objective="time", nchunks=None, k=None):
        """Indices into candidates(shape) (restricted to `nchunks` when
        given) ordered by the model's predicted objective, best first (the
        first k of them when k is given); scored and ordered on the GPU
        (ccl_mlp_rank, the scores ccl_mlp_pick minimises)."""
        import torch
        cfgs = candidates(shape)
        idx = [i for i, c in enumerate(cfgs) if nchunks is None or c.nchunks == nchunks]
        k = len(idx) if k is None else max(1, min(int(k), len(idx)))
        w = OBJECTIVES[objective]
        wt, we = w[0] * float(self.ys.std[0]), w[1] * float(self.ys.std[1])
        X = ccl_costmodel_features([cfgs[i] for i in idx])
        xd = torch.from_numpy(self.xs.apply(X)).cuda()
        order = torch.zeros(k, dtype=torch.int32, device="cuda")
        ccl_mlp_rank(self.handle, len(idx), xd.data_ptr(), wt, we, k, order.data_ptr())
        return [idx[j] for j in order.cpu().tolist()]

    def pick_verified(self, shape, objective="time", k=3, r2=0.25, nchunks=None, repeats=3):
        """The model's k best candidates measured by the autotuner; returns
        the fastest (or least-energy) of them and its measurement.  For
        energy and EDP the model's time pick is measured with them, each
        config as the median of `repeats` counter windows (a single window
        now and then reads far low): the model's energy ranking is not
        reliable enough on its own (on 24 held-out shapes its three best by
        predicted energy measured 1.07 x the least energy, its time pick
        1.06 x, the least of the two sets 1.04 x), so the choice is never
        the model's word against a measured time pick."""
        cfgs = candidates(shape)
        order = self.rank(shape, objective, nchunks)[:k]
        if objective == "time":
            top = [cfgs[i] for i in order]
            res = measure(top, r2)
            j = int(np.argmin([r["s_per_step"] for r in res]))
            return top[j], res[j]
        tcfg, _ = self.pick(shape, "time", nchunks)
        keys = [cfg_key(cfgs[i]) for i in order]
        top = [cfgs[i] for i in order] + ([tcfg] if cfg_key(tcfg) not in keys else [])
        runs = [measure(top, r2, energy_window_s=1.0) for _ in range(max(1, repeats))]
        res = []
        for j in range(len(top)):
            rr = [run[j] for run in runs if run[j]["j_per_step"] is not None and
                  np.isfinite(run[j]["j_per_step"]) and run[j]["j_per_step"] > 0]
            if not rr:
                res.append(dict(runs[0][j], j_per_step=float("inf")))
                continue
            rr.sort(key=lambda r: r["j_per_step"])
            res.append(rr[len(rr) // 2])  # the median window
        score = [r["j_per_step"] if objective == "energy" else r["s_per_step"] * r["j_per_step"]
                 for r in res]
        j = int(np.argmin(score))
        return top[j], res[j]

    def to_json(self):
        return dict(params=self.params.tolist(), x_mean=self.xs.mean.tolist(),
                    x_std=self.xs.std.tolist(), y_mean=self.ys.mean.tolist(),
                    y_std=self.ys.std.tolist(), meta=self.meta)

    @classmethod
    def from_json(cls, d):
        return cls(np.array(d["params"], np.float32),
                   Standardiser(np.array(d["x_mean"]), np.array(d["x_std"])),
                   Standardiser(np.array(d["y_mean"]), np.array(d["y_std"])), d.get("meta"))

    def save(self, path):
        with open(path, "w") as f:
            json.dump(self.to_json(), f)

    @classmethod
    def load(cls, path):
        with open(path) as f:
            return cls.from_json(json.load(f))

    def close(self):
        if self.handle is not None:
            ccl_mlp_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pack(ws, bs):
    parts = []
    for w, b in zip(ws, bs):
        parts.append(np.asarray(w, np.float32).ravel())
        parts.append(np.asarray(b, np.float32).ravel())
    p = np.concatenate(parts)
    assert p.size == CCL_MLP_NPARAMS
    return p


def unpack(p, sizes=(12, 64, 64, 2)):
    p = np.asarray(p)
    ws, bs, o = [], [], 0
    for fi, fo in zip(sizes[:-1], sizes[1:]):
        ws.append(p[o:o + fi * fo].reshape(fo, fi))
        o += fi * fo
        bs.append(p[o:o + fo])
        o += fo
    return ws, bs


def sample_space(n_shapes: int, seed: int, per_shape: int, rng_seed: int, n_shapes_3d: int = 0,
                 n_shapes_3d_large: int = 0):
    """Training configs: `n_shapes` seeded 2D shapes (sides log-uniform on
    256..16384), `n_shapes_3d` 3D shapes (sides 64..768) and
    `n_shapes_3d_large` 3D shapes with sides 384..768 (log-uniform sides
    rarely give large volumes), `per_shape` candidates each drawn without
    replacement.  Each set extends the previous ones: a shape's configs do
    not change when later sets are added."""
    import synth
    shapes = synth.cost_model_shapes(n_shapes, seed)
    if n_shapes_3d:
        shapes = shapes + synth.cost_model_shapes_3d(n_shapes_3d, seed + 100)
    if n_shapes_3d_large:
        shapes = shapes + synth.cost_model_shapes_3d(n_shapes_3d_large, seed + 200, lo=384)
    rs = np.random.default_rng(rng_seed)
    cfgs = []
    for sh in shapes:
        cands = candidates(sh)
        pick = rs.choice(len(cands), size=min(per_shape, len(cands)), replace=False)
        cfgs.extend(cands[i] for i in sorted(pick))
    return shapes, cfgs


MODEL_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "costmodel.json")


def shortlist(shape, nchunks, k=3, model_path=MODEL_PATH):
    """The trained cost model's k best candidates (by predicted time) for a
    shape split into `nchunks` chunks, best first, as (T, tile rows) pairs."""
    m = CostModel.load(model_path)
    try:
        cfgs = candidates(shape)
        return [(cfgs[i].temporal_depth, cfgs[i].tile_rows)
                for i in m.rank(shape, "time", nchunks=nchunks)[:k]]
    finally:
        m.close()


def launch_config(shape, nchunks, steps, r2=0.25, model_path=MODEL_PATH, verify=3):
    """(T, tile rows, how) for `steps` leapfrog steps of a shape split into
    `nchunks` chunks.  With a trained cost model: its `verify` best
    candidates, timed by the autotuner, the fastest of them (verify = 1: the
    model's pick unmeasured).  Without a model: the fastest of an autotuner
    sweep of all candidates with that many chunks.  Candidates are timed over
    the workload's own step count, so a depth whose last block is shorter
    (steps not a multiple of T) is charged for it as the workload will be."""
    if model_path and os.path.exists(model_path):
        top = shortlist(shape, nchunks, max(1, verify), model_path)
        if len(top) == 1:
            return top[0][0], top[0][1], "cost model"
        cfgs = [make_tune_config(shape, nchunks, T, rows) for T, rows in top]
        res = measure(cfgs, r2, reps=3, steps=steps)
        i = int(np.argmin([r["s_per_step"] for r in res]))
        return top[i][0], top[i][1], f"cost model, fastest of its top {len(top)} measured"
    cands, _, i = sweep(shape, nchunks, r2, steps=steps, reps=3)
    return cands[i].temporal_depth, cands[i].tile_rows, "autotuner sweep"


def batch_specs(grids, model_path=MODEL_PATH, r2=0.25):
    """Launch specs of a batch of independent 2D grids (dicts with ny, nx,
    steps as ``synth.batched_grids`` gives them), as the batched forms run
    them.  Returns (persistent, per_grid, how):

    * persistent: specs for the persistent kernel, each grid's depth from
      the cost model's time pick for the grid alone (one chunk), tile rows
      left to the batch (0), which sizes tiles for all grids at once;
    * per_grid: the same depths with the model's own rows, for forms that
      launch each grid alone (CCL_BATCH_PER_GRID, a loop of ccl_wave_step
      calls);
    * how: what chose the configs.

    Without a trained model every grid takes T = 4 with 64 rows."""
    model = CostModel.load(model_path) if model_path and os.path.exists(model_path) else None
    persistent, per_grid = [], []
    try:
        for d in grids:
            depth, rows = 4, 64
            if model is not None:
                c, _ = model.pick((d["ny"], d["nx"]), "time", nchunks=1)
                depth, rows = c.temporal_depth, c.tile_rows
            base = dict(ny=int(d["ny"]), nx=int(d["nx"]), steps=int(d["steps"]), r2=r2,
                        depth=int(depth))
            persistent.append(dict(base, tile_rows=0 if model is not None else rows))
            per_grid.append(dict(base, tile_rows=int(rows)))
    finally:
        if model is not None:
            model.close()
    return persistent, per_grid, ("cost model" if model is not None else "T=4, 64 rows")
