"""What the trained cost model gains over launching without it (GPU).

The committed model (paper_2505_06022_amd/costmodel.json, trained by the
library's own MLP kernels on samples the autotuner measured) picks a launch
configuration for held-out shapes it never saw in training.  Each pick is
timed next to (a) the configuration used without a model (one chunk, T = 1,
automatic tile rows) and (b) the best of the exhaustive sweep of the same
shape, all in one measurement call so that they share the device state.
"""
import os

import numpy as np
import pytest


pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                     "paper_2505_06022_amd", "costmodel.json")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(MODEL):
        pytest.skip("no trained cost model committed")
    torch.cuda.set_device(0)
    import paper_2505_06022_amd as ccl
    ccl.lib()
    yield


def held_out_shapes(n=2, max_cells=3.2e7):
    from paper_2505_06022_amd.learn import held_out_shapes as shapes_of
    return [s for s in shapes_of(200) if s[0] * s[1] <= max_cells][:n]


@pytest.mark.parametrize("shape", held_out_shapes())
def test_learned_pick_gains_over_no_model(shape):
    from paper_2505_06022_amd import tune
    cfgs = tune.candidates(shape)
    keys = [tune.cfg_key(c) for c in cfgs]
    res = tune.measure(cfgs, reps=3)
    t = np.array([r["s_per_step"] for r in res])
    m = tune.CostModel.load(MODEL)
    try:
        pick_cfg, _ = m.pick(shape, "time")
    finally:
        m.close()
    pick = keys.index(tune.cfg_key(pick_cfg))
    default = keys.index((tuple(shape), 1, 1, 0))
    best = int(np.argmin(t))
    gain = t[default] / t[pick]
    ratio = t[pick] / t[best]
    print(f"{shape}: pick {keys[pick][1:]} best {keys[best][1:]}; pick/best {ratio:.3f}, "
          f"no-model/pick {gain:.2f}")
    assert gain >= 1.3, f"the model's pick is only {gain:.2f}x faster than no model"
    assert ratio <= 1.25, f"the model's pick is {ratio:.3f}x the swept best"


def test_energy_choice_no_worse_than_time_pick():
    """The launcher's energy choice (the least measured energy among the
    model's three best by predicted energy and its time pick, each the median
    of three counter windows) uses no more energy than the time pick, on the
    first held-out shape where the model's raw energy and time picks differ:
    both re-measured in fresh windows (median of three each), within the 3%
    window-to-window spread.  The raw energy pick alone is not relied on (on
    held-out shapes it measured worse than the time pick on average)."""
    from paper_2505_06022_amd import learn, tune
    m = tune.CostModel.load(MODEL)
    try:
        chosen = None
        for sh in learn.held_out_shapes(200)[:40]:
            e_cfg, _ = m.pick(sh, "energy")
            t_cfg, _ = m.pick(sh, "time")
            if tune.cfg_key(e_cfg) != tune.cfg_key(t_cfg):
                chosen = sh
                break
        sh = chosen or learn.held_out_shapes(200)[0]
        t_cfg, _ = m.pick(sh, "time")
        v_cfg, _ = m.pick_verified(sh, "energy")
    finally:
        m.close()
    reads = {0: [], 1: []}
    for _ in range(3):
        for k, r in enumerate(tune.measure([v_cfg, t_cfg], energy_window_s=1.0)):
            if r["j_per_step"] is not None and np.isfinite(r["j_per_step"]) and r["j_per_step"] > 0:
                reads[k].append(r["j_per_step"])
    assert reads[0] and reads[1], "the energy counter gave no valid window"
    e_choice, e_time = float(np.median(reads[0])), float(np.median(reads[1]))
    print(f"{sh}: energy choice {tune.cfg_key(v_cfg)[1:]} {e_choice:.5f} J/step, time pick "
          f"{tune.cfg_key(t_cfg)[1:]} {e_time:.5f} J/step")
    assert e_choice <= 1.03 * e_time
