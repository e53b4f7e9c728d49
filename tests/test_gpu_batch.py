"""GPU tests of the batched persistent launch (many grids, one graph launch).

Every grid must come out bitwise equal to the float32 oracle stepping it
alone (same per-cell expression), whatever its depth, tile rows, step count
or shape; graph replays must repeat the eager result; the dependency wait's
time limit, forced to zero from the host, must end the launch with TIMEOUT
rather than hang, and the batch must recover on the next run."""
import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2505_06022_amd as ccl
    ccl.lib()
    yield


SPECS = [
    dict(ny=97, nx=130, steps=17, r2=0.25, depth=1),
    dict(ny=256, nx=517, steps=40, r2=0.25, depth=4),
    dict(ny=64, nx=64, steps=0, r2=0.25, depth=2),
    dict(ny=300, nx=250, steps=23, r2=0.2, depth=3, tile_rows=3),
    dict(ny=33, nx=900, steps=9, r2=0.25, depth=8, tile_rows=16),
    dict(ny=500, nx=31, steps=1, r2=0.25, depth=2),
    dict(ny=128, nx=256, steps=64, r2=0.25, depth=5),
]


def inputs(i, s):
    up = synth.gaussian_field((s["ny"], s["nx"]), s["ny"] / 8.0, seed=100 + i)
    uc = synth.gaussian_field((s["ny"], s["nx"]), s["ny"] / 7.0, seed=200 + i)
    return up, uc


@pytest.mark.parametrize("flags", [0, 1, 2, 3])
def test_batch_matches_oracle(flags):
    """Persistent kernel (flags 0, 1 = without the graph) and per-grid
    ccl_wave_step sequences (2, 3 = without the graph)."""
    from paper_2505_06022_amd.fields import BatchedWaves
    bw = BatchedWaves(SPECS, flags=flags, fill=float("nan"))
    refs = []
    for i, s in enumerate(SPECS):
        up, uc = inputs(i, s)
        bw.scatter(i, up, uc)
        refs.append(oracle.wave(up, uc, s["r2"], s["steps"]))
    bw.run()
    import paper_2505_06022_amd as ccl
    ccl.ccl_batch_check(bw.handle)
    for i, s in enumerate(SPECS):
        rp, rc = refs[i]
        gc = bw.gather(i, "cur")
        gp = bw.gather(i, "prev")
        assert np.all(np.isfinite(gc)), f"grid {i}: non-finite"
        assert np.array_equal(gc, rc), f"grid {i} ({s}): u^n differs from the oracle"
        assert np.array_equal(gp, rp), f"grid {i}: u^(n-1) differs from the oracle"
    bw.close()


@pytest.mark.parametrize("mode", [0, 2])
def test_graph_replays_repeat(mode):
    """Replays of the captured graph, with eager work in between, each equal
    the eager (no-graph) result."""
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.fields import BatchedWaves
    specs = SPECS[:2] + SPECS[3:5]
    bw = BatchedWaves(specs, flags=mode)
    ref = BatchedWaves(specs, flags=ccl.CCL_BATCH_NO_GRAPH)
    ins = [inputs(i, s) for i, s in enumerate(specs)]
    for i in range(len(specs)):
        ref.scatter(i, *ins[i])
    ref.run()
    ccl.ccl_batch_check(ref.handle)
    want = [ref.gather(i) for i in range(len(specs))]
    junk = torch.rand(1 << 20, device="cuda")
    for rep in range(4):
        for i in range(len(specs)):
            bw.scatter(i, *ins[i])
        junk.mul_(1.5).add_(0.25)  # eager work between replays
        bw.run()
        ccl.ccl_batch_check(bw.handle)
        for i in range(len(specs)):
            assert np.array_equal(bw.gather(i), want[i]), f"replay {rep}, grid {i}"
    bw.close()
    ref.close()


def test_wait_limit_timeout_then_recovery():
    """A single-tile grid with 64 dependent blocks: with a zero wait limit the
    waits give up (TIMEOUT is reported, the launch ends); with the default
    limit restored the next run is correct."""
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.fields import BatchedWaves
    spec = [dict(ny=48, nx=200, steps=64, r2=0.25, depth=1, tile_rows=64)]
    bw = BatchedWaves(spec)
    up, uc = inputs(0, spec[0])
    ccl.ccl_batch_set_wait_limit(bw.handle, 0)
    timeouts = 0
    for _ in range(5):
        bw.scatter(0, up, uc)
        bw.run()
        try:
            ccl.ccl_batch_check(bw.handle)
        except ccl.CclError as e:
            assert e.status == ccl.CCL_E_TIMEOUT
            timeouts += 1
    assert timeouts >= 1
    ccl.ccl_batch_set_wait_limit(bw.handle, 10_000_000)
    bw.scatter(0, up, uc)
    bw.run()
    ccl.ccl_batch_check(bw.handle)
    _, rc = oracle.wave(up, uc, 0.25, 64)
    assert np.array_equal(bw.gather(0), rc)
    bw.close()


def test_batched_workload_sample():
    """The 64-grid workload's shapes (sides 512..4096, 100..500 steps): a
    seeded sample of 6 of its grids in one batch, each bitwise equal to the
    oracle."""
    from paper_2505_06022_amd.fields import BatchedWaves
    grids = synth.batched_grids()
    pick = [0, 5, 17, 33, 48, 63]
    specs = []
    for g in pick:
        d = grids[g]
        specs.append(dict(ny=d["ny"], nx=d["nx"], steps=d["steps"] // 4, r2=0.25, depth=4))
    bw = BatchedWaves(specs)
    ins = []
    for i, g in enumerate(pick):
        d = grids[g]
        u0 = synth.gaussian_field((d["ny"], d["nx"]), d["sigma"], d["seed"])
        bw.scatter(i, u0, u0)
        ins.append(u0)
    bw.run()
    import paper_2505_06022_amd as ccl
    ccl.ccl_batch_check(bw.handle)
    th = oracle.max_threads()
    for i, s in enumerate(specs):
        _, rc = oracle.wave(ins[i].copy(), ins[i], 0.25, s["steps"], threads=th)
        assert np.array_equal(bw.gather(i), rc), f"grid {pick[i]}"
    bw.close()
