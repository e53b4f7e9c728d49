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
