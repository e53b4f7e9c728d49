"""The batched persistent run without device allocation (ccl_batch_run_static).

Two calls in a row, the second on a smaller batch (fewer and smaller grids,
other depths), each compared bitwise with the same grids run through
ccl_batch_create + ccl_batch_run (the entry point it is a variant of) and
with the float32 oracle.  The static tables keep the first call's contents,
so the second call also shows that the counters and control words are
cleared and the smaller plan replaces the larger one.  A plan larger than
the static array is refused before anything runs.
"""
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


def make_inputs(specs, seed0):
    ins = []
    for g, s in enumerate(specs):
        u0 = synth.gaussian_field((s["ny"], s["nx"]), min(s["ny"], s["nx"]) / 16.0, seed0 + g)
        ins.append(u0)
    return ins


def run_static(specs, inputs):
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.fields import BatchedWaves
    bw = BatchedWaves(specs, fill=float("nan"), create=False)
    for g, u0 in enumerate(inputs):
        bw.scatter(g, u0, u0)
    print(f"static run: {len(specs)} grids", flush=True)
    roles = ccl.ccl_batch_run_static(bw.grids, check=True)
    out = []
    for g, (p, c) in enumerate(roles):
        nx = specs[g]["nx"]
        out.append((bw.tensors[g][p][:, :nx].cpu().numpy(), bw.tensors[g][c][:, :nx].cpu().numpy()))
    return out


def run_created(specs, inputs):
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.fields import BatchedWaves
    bw = BatchedWaves(specs, flags=ccl.CCL_BATCH_NO_GRAPH, fill=float("nan"))
    for g, u0 in enumerate(inputs):
        bw.scatter(g, u0, u0)
    bw.run()
    ccl.ccl_batch_check(bw.handle)
    out = [(bw.gather(g, "prev"), bw.gather(g, "cur")) for g in range(len(specs))]
    bw.close()
    return out


BIG = [dict(ny=700, nx=1300, steps=37, r2=0.25, depth=8),
       dict(ny=1024, nx=512, steps=40, r2=0.25, depth=4),
       dict(ny=333, nx=901, steps=23, r2=0.25, depth=5, tile_rows=40),
       dict(ny=512, nx=2048, steps=30, r2=0.25, depth=8),
       dict(ny=96, nx=100, steps=11, r2=0.2, depth=1)]
SMALL = [dict(ny=200, nx=260, steps=17, r2=0.25, depth=3),
         dict(ny=64, nx=700, steps=9, r2=0.25, depth=2)]


def check(specs, seed0):
    ins = make_inputs(specs, seed0)
    got = run_static(specs, ins)
    ref = run_created(specs, ins)
    for g, s in enumerate(specs):
        op, oc = oracle.wave(ins[g].copy(), ins[g], s["r2"], s["steps"])
        for (a, b), what in ((got[g], "static"), (ref[g], "created")):
            assert np.all(np.isfinite(a)) and np.all(np.isfinite(b)), f"grid {g} {what}: NaN"
            assert np.array_equal(b, oc), f"grid {g} {what}: u^n differs from the oracle"
            assert np.array_equal(a, op), f"grid {g} {what}: u^(n-1) differs from the oracle"
        assert np.array_equal(got[g][1], ref[g][1]) and np.array_equal(got[g][0], ref[g][0])


def test_static_twice_then_smaller():
    check(BIG, 700)
    check(SMALL, 800)


def test_static_refuses_oversized_plan():
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.fields import BatchedWaves
    # one-row tiles of 16 grids of 4096 x 4096 at T = 1: 17 strips of 248
    # output columns x 4096 segments per grid, one 4-byte counter per tile,
    # more than the static array holds (real buffers all the same, in case
    # the plan were accepted)
    specs = [dict(ny=4096, nx=4096, steps=2, r2=0.25, depth=1, tile_rows=1)] * 16
    counters = 16 * 4096 * -(-4096 // 248)
    assert 4 * counters > ccl.CCL_BATCH_STATIC_BYTES
    bw = BatchedWaves(specs, create=False)
    with pytest.raises(ccl.CclError) as e:
        ccl.ccl_batch_run_static(bw.grids)
    assert e.value.status == ccl.CCL_E_RANGE
    del bw
    torch.cuda.empty_cache()
