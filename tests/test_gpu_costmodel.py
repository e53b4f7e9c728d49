"""GPU tests of the cost-model kernels and the autotuner, through the C ABI.

* Forward, gradient, loss and one Adam step of the 12-64-64-2 MLP against
  the float64 oracle (relative L2 per tensor <= 1e-4 for gradients).
* Training is deterministic (two runs give identical parameters) and tracks
  the float64 oracle's loss trajectory.
* ccl_mlp_pick returns the argmin of the oracle's scores (ties aside).
* ccl_autotune_measure returns positive times for every config and fails
  cleanly on a bad one.
"""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

SIZES = (12, 64, 64, 2)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2505_06022_amd as ccl
    ccl.lib()
    yield


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-30))


def make(seed, n):
    from paper_2505_06022_amd.tune import pack
    ws, bs = synth.mlp_params(SIZES, seed)
    for b in bs:  # non-zero biases exercise the bias gradients
        b[:] = np.random.default_rng(seed + 1).uniform(-0.1, 0.1, size=b.shape)
    x, t = synth.mlp_batch(n, 12, 2, seed + 2)
    # round inputs to float32 so both sides see the same numbers
    ws = [w.astype(np.float32).astype(np.float64) for w in ws]
    bs = [b.astype(np.float32).astype(np.float64) for b in bs]
    x = x.astype(np.float32).astype(np.float64)
    t = t.astype(np.float32).astype(np.float64)
    return ws, bs, x, t, pack(ws, bs)


@pytest.mark.parametrize("n", [1, 63, 64, 200, 4000])
def test_forward_grad_loss_vs_oracle(n):
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.tune import unpack
    ws, bs, x, t, p = make(3, n)
    h = ccl.ccl_mlp_create(p)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    yd = torch.empty((n, 2), device="cuda")
    ccl.ccl_mlp_forward(h, n, xd.data_ptr(), yd.data_ptr())
    ccl.ccl_mlp_grad(h, n, xd.data_ptr(), td.data_ptr())
    torch.cuda.synchronize()
    acts = omlp.forward(ws, bs, x)
    assert rel_l2(yd.cpu().numpy(), acts[-1]) <= 1e-5
    gw, gb = omlp.backward(ws, bs, acts, t)
    g = ccl.ccl_mlp_get(h, ccl.CCL_MLP_GRADS)
    uw, ub = unpack(g)
    for li in range(3):
        assert rel_l2(uw[li], gw[li]) <= 1e-4, f"dW{li + 1}"
        assert rel_l2(ub[li], gb[li]) <= 1e-4, f"db{li + 1}"
    loss = ccl.ccl_mlp_get(h, ccl.CCL_MLP_LOSS)[0]
    assert abs(loss - omlp.loss(acts[-1], t)) <= 1e-5 * max(1.0, omlp.loss(acts[-1], t))
    ccl.ccl_mlp_destroy(h)


def test_weighted_grad_vs_oracle():
    """Per-output weights (a mask over the second output) against the oracle."""
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.tune import unpack
    n = 333
    ws, bs, x, t, p = make(11, n)
    w = np.ones((n, 2))
    w[::3, 1] = 0.0
    w[5::7, 0] = 0.5
    h = ccl.ccl_mlp_create(p)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    wd = torch.from_numpy(w.astype(np.float32)).cuda()
    ccl.ccl_mlp_grad_weighted(h, n, xd.data_ptr(), td.data_ptr(), wd.data_ptr())
    torch.cuda.synchronize()
    acts = omlp.forward(ws, bs, x)
    gw, gb = omlp.backward(ws, bs, acts, t, w)
    uw, ub = unpack(ccl.ccl_mlp_get(h, ccl.CCL_MLP_GRADS))
    for li in range(3):
        assert rel_l2(uw[li], gw[li]) <= 1e-4 and rel_l2(ub[li], gb[li]) <= 1e-4
    loss = ccl.ccl_mlp_get(h, ccl.CCL_MLP_LOSS)[0]
    want = omlp.loss(acts[-1], t, w)
    assert abs(loss - want) <= 1e-5 * max(1.0, want)
    ccl.ccl_mlp_destroy(h)


def test_adam_steps_vs_oracle():
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.tune import pack, unpack
    ws, bs, x, t, p = make(5, 300)
    h = ccl.ccl_mlp_create(p)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    params = ws + bs
    m = [np.zeros_like(q) for q in params]
    v = [np.zeros_like(q) for q in params]
    for step in range(1, 6):
        ccl.ccl_mlp_grad(h, 300, xd.data_ptr(), td.data_ptr())
        ccl.ccl_mlp_adam(h, 1e-3)
        acts = omlp.forward(ws, bs, x)
        gw, gb = omlp.backward(ws, bs, acts, t)
        omlp.adam_step(params, gw + gb, m, v, step, lr=1e-3)
    torch.cuda.synchronize()
    got = ccl.ccl_mlp_get(h, ccl.CCL_MLP_PARAMS)
    want = pack(ws, bs)
    # parameters moved by ~5e-3; require the GPU's move to match to 1e-3 of it
    assert np.max(np.abs(got - want)) <= 1e-3 * np.max(np.abs(want - p)) + 1e-6
    ccl.ccl_mlp_destroy(h)


def test_training_deterministic_and_tracks_oracle():
    import paper_2505_06022_amd as ccl
    ws, bs, x, t, p = make(7, 1000)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    td = torch.from_numpy(t.astype(np.float32)).cuda()
    outs = []
    for _ in range(2):
        h = ccl.ccl_mlp_create(p)
        ccl.ccl_mlp_train(h, 1000, xd.data_ptr(), td.data_ptr(), 200, 1e-3)
        torch.cuda.synchronize()
        outs.append((ccl.ccl_mlp_get(h, ccl.CCL_MLP_PARAMS), ccl.ccl_mlp_get(h, ccl.CCL_MLP_LOSS)))
        ccl.ccl_mlp_destroy(h)
    assert np.array_equal(outs[0][0], outs[1][0])
    params = ws + bs
    m = [np.zeros_like(q) for q in params]
    v = [np.zeros_like(q) for q in params]
    for step in range(1, 201):
        acts = omlp.forward(ws, bs, x)
        gw, gb = omlp.backward(ws, bs, acts, t)
        last = omlp.loss(acts[-1], t)
        omlp.adam_step(params, gw + gb, m, v, step, lr=1e-3)
    # the GPU reports the loss of its last gradient evaluation (before the
    # last Adam step), as `last` here
    assert abs(outs[0][1][0] - last) <= 1e-3 * last


def test_pick_is_oracle_argmin():
    import paper_2505_06022_amd as ccl
    ws, bs, x, t, p = make(9, 777)
    h = ccl.ccl_mlp_create(p)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    best = torch.zeros(1, dtype=torch.int32, device="cuda")
    scores = torch.empty(777, device="cuda")
    for w0, w1 in ((1.0, 0.0), (0.0, 1.0), (0.7, 0.3)):
        ccl.ccl_mlp_pick(h, 777, xd.data_ptr(), w0, w1, scores.data_ptr(), best.data_ptr())
        torch.cuda.synchronize()
        y = omlp.forward(ws, bs, x)[-1]
        s = w0 * y[:, 0] + w1 * y[:, 1]
        b = int(best.item())
        assert s[b] <= s.min() + 1e-5 * max(1.0, abs(s.min()))
        got_scores = scores.cpu().numpy()
        assert b == int(np.argmin(got_scores))
    ccl.ccl_mlp_destroy(h)


@pytest.mark.parametrize("n,k", [(777, 10), (200, 200), (1, 1), (300, 3)])
def test_rank_orders_the_pick_scores(n, k):
    """ccl_mlp_rank: the k smallest of the scores ccl_mlp_pick writes, in
    ascending order with ties to the lower index; its first entry is the
    pick.  The scores are checked against the oracle's forward pass."""
    import paper_2505_06022_amd as ccl
    ws, bs, x, t, p = make(11, n)
    h = ccl.ccl_mlp_create(p)
    xd = torch.from_numpy(x.astype(np.float32)).cuda()
    best = torch.zeros(1, dtype=torch.int32, device="cuda")
    scores = torch.empty(n, device="cuda")
    order = torch.full((k,), -1, dtype=torch.int32, device="cuda")
    for w0, w1 in ((1.0, 0.0), (1.0, 1.0), (2.0, 1.0)):
        ccl.ccl_mlp_pick(h, n, xd.data_ptr(), w0, w1, scores.data_ptr(), best.data_ptr())
        ccl.ccl_mlp_rank(h, n, xd.data_ptr(), w0, w1, k, order.data_ptr())
        torch.cuda.synchronize()
        sc = scores.cpu().numpy()
        got = order.cpu().numpy().tolist()
        assert got == np.argsort(sc, kind="stable")[:k].tolist()
        assert got[0] == int(best.item())
        y = omlp.forward(ws, bs, x)[-1]
        s = w0 * y[:, 0] + w1 * y[:, 1]
        assert np.allclose(sc, s, rtol=1e-4, atol=1e-4)
    with pytest.raises(ccl.CclError):
        ccl.ccl_mlp_rank(h, n, xd.data_ptr(), 1.0, 0.0, n + 1, order.data_ptr())
    ccl.ccl_mlp_destroy(h)


def test_autotune_sweep():
    """ccl_autotune_sweep measures exactly the library's candidates (K fixed
    here) and returns the index of the fastest it measured."""
    import paper_2505_06022_amd as ccl
    shape = (256, 512)
    cfgs, samples, best = ccl.ccl_autotune_sweep(shape, 2, 0.25, 16, reps=1)
    want = ccl.ccl_autotune_candidates(shape, 2)
    key = lambda c: (c.dims, tuple(c.shape[:c.dims]), c.nchunks, c.temporal_depth, c.tile_rows)
    assert [key(c) for c in cfgs] == [key(c) for c in want] and len(cfgs) == 40
    t = [o.seconds_per_step for o in samples]
    assert all(v > 0 for v in t)
    assert best == int(np.argmin(t))


def test_autotune_measure():
    import paper_2505_06022_amd as ccl
    cfgs = [ccl.make_tune_config((512, 1024), K, T, rows)
            for K, T, rows in ((1, 1, 32), (4, 4, 64), (2, 8, 16), (16, 2, 128))]
    cfgs.append(ccl.make_tune_config((64, 48, 300), 3, 1, 8))
    res = ccl.ccl_autotune_measure(cfgs, 0.25, 24, reps=3)
    for r in res:
        assert r.seconds_per_step > 0 and np.isnan(r.joules_per_step)
    bad = [ccl.make_tune_config((512, 1024), 1, 9, 32)]
    with pytest.raises(ccl.CclError):
        ccl.ccl_autotune_measure(bad, 0.25, 24)


def test_wave_slots_and_features_on_device():
    """The occupancy the planner and the features use: positive, a whole
    number of waves per CU, non-increasing with T for the 2D kernel (its
    register ring grows with T); features finite, fill in (0, 1]."""
    import paper_2505_06022_amd as ccl
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    s2 = [ccl.ccl_wave_slots(2, T) for T in range(1, 9)]
    s3 = [ccl.ccl_wave_slots(3, T) for T in range(1, 9)]
    for s in s2 + s3:
        assert s > 0 and s % cus == 0
    assert all(a >= b for a, b in zip(s2[1:], s2[2:]))
    cfgs = [ccl.make_tune_config((8192, 8192), 4, T, 0) for T in range(1, 9)]
    cfgs += [ccl.make_tune_config((768, 768, 768), 8, T, 0) for T in range(1, 9)]
    x = ccl.ccl_costmodel_features(cfgs)
    assert np.all(np.isfinite(x))
    assert np.all(x[:, 8] > 0) and np.all(x[:, 8] <= 1)
    assert np.all(x[:, 4] > 0)  # tiles always stream more cells than they write
