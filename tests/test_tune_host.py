"""Host logic of the autotuner / cost-model driver (CPU only)."""
import numpy as np

import synth
from paper_2505_06022_amd import tune


def test_candidate_space():
    c2 = tune.candidates((1024, 4096))
    assert len(c2) == 5 * 5 * 8
    assert {c.temporal_depth for c in c2} == set(range(1, 9))
    assert len(tune.candidates((8, 4096))) == 4 * 5 * 8  # K = 16 > 8 rows dropped
    c3 = tune.candidates((96, 768, 768))
    assert {c.temporal_depth for c in c3} == set(range(1, 9)) and len(c3) == 5 * 5 * 8


def test_sample_space_seeded():
    a_shapes, a = tune.sample_space(6, 3, 5, 5)
    b_shapes, b = tune.sample_space(6, 3, 5, 5)
    assert a_shapes == b_shapes
    assert [tune.cfg_key(c) for c in a] == [tune.cfg_key(c) for c in b]
    assert len(a) == 30
    for sh in a_shapes:
        assert all(256 <= s <= 16384 and s % 64 == 0 for s in sh)
    held = synth.cost_model_shapes(200, 4)
    train = synth.cost_model_shapes(250, 3)
    assert len(set(held) & set(train)) < 10  # mostly distinct shape sets


def test_pack_unpack_roundtrip():
    ws, bs = synth.mlp_params((12, 64, 64, 2), 0)
    p = tune.pack(ws, bs)
    uw, ub = tune.unpack(p)
    for a, b in zip(ws + bs, uw + ub):
        assert np.array_equal(a.astype(np.float32), b)


def test_targets_mask_missing_energy():
    s = [dict(s_per_cell_step=1e-12, j_per_cell_step=float("nan")),
         dict(s_per_cell_step=2e-12, j_per_cell_step=3e-10)]
    t, w = tune.targets_of(s)
    assert w[0, 1] == 0 and w[1, 1] == 1 and np.all(w[:, 0] == 1)
    # second target: log power = log(J per cell-step / s per cell-step)
    assert np.isclose(t[1, 1], np.log(3e-10 / 2e-12)) and np.isclose(t[0, 0], np.log(1e-12))


def test_steps_for():
    assert tune.steps_for((16384, 16384)) == 24
    assert tune.steps_for((256, 256)) == 960
    assert tune.steps_for((4096, 4096)) % 24 == 0


def test_remeasure_replaces_one_family_in_place(tmp_path, monkeypatch):
    """`learn remeasure` re-times only the chosen kernel family, keeps the
    sample order and re-labels energy exactly where a label was held."""
    import json
    from paper_2505_06022_amd import learn
    nan = float("nan")
    keys = [((512, 512), 1, 4, 0), ((64, 96, 128), 2, 1, 0), ((64, 96, 128), 2, 5, 0),
            ((64, 96, 128), 1, 3, 0), ((96, 64, 64), 4, 8, 0)]
    samples = [dict(key=[list(k[0]), *k[1:]], steps=24, s_per_step=1.0, j_per_step=nan,
                    s_per_cell_step=1.0, j_per_cell_step=nan, window_s=0.0) for k in keys]
    samples[2]["j_per_cell_step"] = samples[2]["j_per_step"] = 5.0
    samples[0]["j_per_cell_step"] = samples[0]["j_per_step"] = 7.0
    doc = dict(samples=samples, features=[[0.0] * 12 for _ in keys], meta={})
    (tmp_path / "samples.json").write_text(json.dumps(doc))
    calls = []

    def fake_measure(cfgs, energy_window_s=0.0, **kw):
        calls.append(([tune.cfg_key(c) for c in cfgs], energy_window_s))
        return [dict(key=tune.cfg_key(c), steps=24, s_per_step=2.0, j_per_step=3.0 if
                     energy_window_s else nan, s_per_cell_step=2.0,
                     j_per_cell_step=3.0 if energy_window_s else nan, window_s=energy_window_s)
                for c in cfgs]

    monkeypatch.setattr(tune, "measure", fake_measure)
    learn.remeasure(str(tmp_path), dims=3, min_depth=2, window_s=0.5)
    out = json.loads((tmp_path / "samples.json").read_text())
    got = [tuple([tuple(s["key"][0]), *s["key"][1:]]) for s in out["samples"]]
    assert got == keys
    t = [s["s_per_step"] for s in out["samples"]]
    assert t == [1.0, 1.0, 2.0, 2.0, 2.0]
    e = [s["j_per_cell_step"] for s in out["samples"]]
    assert e[0] == 7.0 and e[2] == 3.0 and all(np.isnan(e[j]) for j in (1, 3, 4))
    assert [w for _, w in calls].count(0.5) == 1
    assert out["features"][0] == [0.0] * 12 and out["features"][2] != [0.0] * 12
    assert out["meta"]["remeasured"]["samples"] == 3


def test_traffic_summary_sections(tmp_path):
    """Counter summaries of several launch configs share one file; the
    bench finds the section of the config it timed."""
    import csv
    import bench
    from paper_2505_06022_amd import profile_run as pr

    def fake_csv(path, counter, stencil_kib):
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, ["Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for v in stencil_kib:
                w.writerow(dict(Kernel_Name="void ccl::wave2d_kernel<8, false>(W2Args)",
                                Counter_Name=counter, Counter_Value=v))
            # the SAXPY counted at 4 B per element for both counters: half
            # its 8 B read (scale 2), all of its 4 B written (scale 1)
            sx = 4.0 * pr.SAXPY_N / 1024.0
            w.writerow(dict(Kernel_Name="saxpy_kernel", Counter_Name=counter, Counter_Value=sx))

    md = tmp_path / "traffic.md"
    for rows, (fk, wk) in ((0, (1000.0, 2000.0)), (32, (1500.0, 2500.0))):
        fc, wc = tmp_path / f"f{rows}.csv", tmp_path / f"w{rows}.csv"
        fake_csv(fc, "FETCH_SIZE", [9e9, fk, fk])
        fake_csv(wc, "WRITE_SIZE", [9e9, wk, wk])
        pr.summarise(str(fc), str(wc), 8, rows, str(md), dims=2, append=True)
    text = md.read_text()
    assert text.count("traffic-json: ") == 2 and text.startswith("# ")
    assert "\n## HBM traffic" in text
    # fetch doubled by the SAXPY's factor, the first (cold) dispatch left out
    assert bench.load_traffic(8, 0, str(md)) == int(round((2 * 1000.0 + 2000.0) * 1024))
    assert bench.load_traffic(8, 32, str(md)) == int(round((2 * 1500.0 + 2500.0) * 1024))
    assert bench.load_traffic(8, 64, str(md)) is None


def test_counter_summary_derived_values(tmp_path):
    """The limiter summary averages each counter over the stencil's
    dispatches (the first, cold one left out) across passes, and derives
    VALU work per useful cell-step, busy shares and waves per CU from them."""
    import csv
    import json
    from paper_2505_06022_amd import profile_run as pr

    def fake(path, counters):
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                                   "Start_Timestamp", "End_Timestamp", "VGPR_Count",
                                   "Accum_VGPR_Count", "LDS_Block_Size", "Workgroup_Size"])
            w.writeheader()
            for d in range(3):
                for name, vals in counters.items():
                    w.writerow(dict(Dispatch_Id=d, Kernel_Name="wave3d_tb_kernel<P32, 6>",
                                    Counter_Name=name, Counter_Value=vals[d],
                                    Start_Timestamp=1000 * d, End_Timestamp=1000 * d + 500,
                                    VGPR_Count=200, Accum_VGPR_Count=0, LDS_Block_Size=98304,
                                    Workgroup_Size=512))
                w.writerow(dict(Dispatch_Id=d, Kernel_Name="saxpy_kernel", Counter_Name="SQ_WAVES",
                                Counter_Value=1, Start_Timestamp=0, End_Timestamp=1))

    cells = 768 ** 3
    a, b = tmp_path / "a.csv", tmp_path / "b.csv"
    fake(a, {"SQ_INSTS_VALU": [1, 6 * cells / 64 * 10, 6 * cells / 64 * 12],
             "SQ_WAVE_CYCLES": [1, 256e3, 256e3], "SQ_WAIT_INST_ANY": [1, 64e3, 64e3],
             "SQ_ACTIVE_INST_VALU": [1, 128e3, 128e3], "GRBM_GUI_ACTIVE": [1, 2000, 2000]})
    fake(b, {"SQ_WAVES": [1, 1000, 1000], "SQ_INSTS_LDS": [1, 5e5, 5e5]})
    md = tmp_path / "c.md"
    pr.counters([str(a), str(b)], 6, 0, str(md), dims=3, title="t", commands=["cmd"])
    doc = json.loads(md.read_text().split("counters-json: ")[1].splitlines()[0])
    d = doc["derived"]
    assert abs(d["valu_lane_ops_per_cell_step"] - 11.0) < 1e-9
    # GRBM_GUI_ACTIVE is summed over 8 XCDs: one XCD was active 250 cycles
    # of the 500 ns dispatch
    assert abs(d["clock_ghz"] - 0.5) < 1e-12
    assert abs(d["valu_busy_share"] - 128e3 / 256 / 250) < 1e-12
    assert abs(d["waves_per_cu"] - 4 * 256e3 / 250 / 256) < 1e-12
    assert abs(d["wait_inst_any_share_of_wave_cycles"] - 0.25) < 1e-12
    assert abs(d["lds_insts_per_wave"] - 500.0) < 1e-9
    assert abs(doc["dispatch_us"] - 0.5) < 1e-12
    assert doc["counters"]["SQ_WAVES"] == 1000


def test_batch_traffic_summary(tmp_path):
    """The batch summary sums the persistent kernel's dispatch and the
    per-grid mode's stencil and halo dispatches separately, scales them by
    the SAXPY's factors and divides by the batch's algorithmic bytes (16 B
    per cell per block of T steps, 12 B per in-place step)."""
    import csv
    import json
    from paper_2505_06022_amd import profile_run as pr
    specs = [dict(ny=10, nx=20, steps=9, depth=4), dict(ny=8, nx=8, steps=5, depth=1)]
    alg = 10 * 20 * 3 * 16 + 8 * 8 * 5 * 12
    assert pr.batch_algorithmic_bytes(specs) == alg
    sj = tmp_path / "specs.json"
    sj.write_text(json.dumps({"persistent": specs, "per_grid": specs, "how": "test"}))

    def fake(path, counter, persistent_kib, per_grid_kib):
        with open(path, "w", newline="") as f:
            w = csv.DictWriter(f, ["Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            w.writerow(dict(Kernel_Name="ccl::batch_kernel<8>", Counter_Name=counter,
                            Counter_Value=persistent_kib))
            for v in per_grid_kib:
                w.writerow(dict(Kernel_Name="ccl::wave2d_kernel<P32, 4, false>",
                                Counter_Name=counter, Counter_Value=v))
            w.writerow(dict(Kernel_Name="copy_boxes_kernel", Counter_Name=counter,
                            Counter_Value=0.5))
            # the SAXPY counted at 4 B per element for both counters
            w.writerow(dict(Kernel_Name="saxpy_kernel", Counter_Name=counter,
                            Counter_Value=4.0 * pr.SAXPY_N / 1024.0))

    fc, wc = tmp_path / "f.csv", tmp_path / "w.csv"
    fake(fc, "FETCH_SIZE", 10.0, [1.0, 2.0])
    fake(wc, "WRITE_SIZE", 6.0, [1.5, 0.5])
    md = tmp_path / "b.md"
    pr.summarise_batch(str(fc), str(wc), str(sj), str(md))
    doc = json.loads(md.read_text().split("batch-traffic-json: ")[1].splitlines()[0])
    assert doc["launches_per_grid_mode"] == 3
    assert abs(doc["persistent"]["fetch_bytes"] - 2 * 10.0 * 1024) < 1e-6
    assert abs(doc["persistent"]["write_bytes"] - 6.0 * 1024) < 1e-6
    assert abs(doc["per_grid"]["fetch_bytes"] - 2 * 3.5 * 1024) < 1e-6
    assert abs(doc["per_grid"]["ratio"] - (2 * 3.5 + 2.5) * 1024 / alg) < 1e-9


def test_held_out_3d_shapes_are_not_trained_on():
    from paper_2505_06022_amd import learn
    trained, _ = tune.sample_space(250, learn.TRAIN_SHAPE_SEED, 1, 0, 40, 40)
    held = learn.held_out_shapes(40, dims=3)
    assert len(held) == 40 and all(len(s) == 3 for s in held)
    assert len(set(held) & set(trained)) <= 2


def test_launch_config_takes_fastest_of_shortlist(tmp_path, monkeypatch):
    """With a model, the launcher times the model's shortlist over the
    workload's own step count and returns the fastest; verify = 1 returns
    the model's pick without measuring."""
    model = tmp_path / "m.json"
    model.write_text("{}")
    monkeypatch.setattr(tune, "shortlist", lambda shape, K, k, path: [(8, 32), (8, 0), (7, 64)][:k])
    times = {(8, 32): 3.0, (8, 0): 2.0, (7, 64): 2.5}
    seen = []

    def fake_measure(cfgs, r2, reps=3, steps=None, **kw):
        seen.append([(c.temporal_depth, c.tile_rows) for c in cfgs])
        assert steps == 1000
        return [dict(s_per_step=times[(c.temporal_depth, c.tile_rows)]) for c in cfgs]

    monkeypatch.setattr(tune, "measure", fake_measure)
    T, rows, how = tune.launch_config((8192, 8192), 4, 1000, 0.25, str(model))
    assert (T, rows) == (8, 0) and "top 3" in how
    assert seen == [[(8, 32), (8, 0), (7, 64)]]
    T, rows, how = tune.launch_config((8192, 8192), 4, 1000, 0.25, str(model), verify=1)
    assert (T, rows, how) == (8, 32, "cost model") and len(seen) == 1


def test_summarise_3d_parts(tmp_path):
    """The 3D evaluation parts merge into evaluation_3d.json and the model's
    `evaluation_3d` metadata, apart from the 2D summary."""
    import json
    from paper_2505_06022_amd import learn
    rows = [dict(index=i, shape=[64, 64, 64], ratio=r, ratio_default=3.0, ratio_untrained=4.0,
                 ratio_top3=1.0, ratio_top5=1.0) for i, r in enumerate((1.0, 1.21, 1.0, 1.02))]
    (tmp_path / "evaluation_3d_part_0000.json").write_text(json.dumps(rows))
    (tmp_path / "m.json").write_text(json.dumps(dict(meta=dict(evaluation=dict(shapes=200)))))
    s = learn.summarise(str(tmp_path), str(tmp_path / "m.json"), dims=3)
    assert s["shapes"] == 4 and np.isclose(s["frac_within_5pct"], 0.75)
    assert np.isclose(s["geomean_pick_over_best"], (1.21 * 1.02) ** 0.25)
    meta = json.loads((tmp_path / "m.json").read_text())["meta"]
    assert meta["evaluation"] == dict(shapes=200) and meta["evaluation_3d"]["shapes"] == 4
    assert (tmp_path / "evaluation_3d.json").exists() and not (tmp_path / "evaluation.json").exists()


def test_held_out_shapes_disjoint_from_training():
    """The held-out shapes of the cost-model evaluation are distinct and
    none of them is a training shape (2D and 3D)."""
    from paper_2505_06022_amd import learn
    train = learn.training_shapes()
    for dims, n in ((2, 200), (3, 40)):
        h = learn.held_out_shapes(n, dims)
        assert len(h) == n and len(set(h)) == n
        assert not set(h) & train
        assert all(len(s) == dims for s in h)
