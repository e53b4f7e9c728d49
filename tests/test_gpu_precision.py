"""GPU parity of the float64 path and of the 16-bit-storage paths.

* float64 (2D and 3D, T = 1..8, chunked along rows, columns and in
  blocks, ragged shapes): bitwise equal to the float64 oracle on the
  unsplit grid (the same expression evaluated in double, in the same
  order).
* bfloat16 and binary16 storage with float32 arithmetic (2D and 3D,
  several T, chunked): bitwise equal to the oracle's 16-bit-storage
  stepping with the same T (inputs rounded to the format, T float32 steps
  per pass, the two stored levels rounded to nearest even), and
  independent of the chunking and tile rows.
* Error budget against the float64 oracle at the 256 x 256 workload
  (100 steps) and at the 8192 x 8192 share (1000 steps, T = 8): the
  storage rounding dominates; the bounds are stated in the tests.
Buffers start NaN-poisoned.
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


def run(u_prev, u_cur, r2, steps, T, dtype, K=1, split_dim=0, grid=None, tile_rows=0,
        offset=None, buffer_range=None):
    from paper_2505_06022_amd.fields import ChunkedWave
    shape = u_cur.shape
    print(f"{dtype} run: {shape} K={K} split_dim={split_dim} grid={grid} T={T} rows={tile_rows}",
          flush=True)
    cw = ChunkedWave(offset or (0,) * len(shape), shape, K, r2, depth=T, tile_rows=tile_rows,
                     split_dim=split_dim, grid=grid, fill=float("nan"), dtype=dtype,
                     buffer_range=buffer_range)
    cw.scatter(u_prev, u_cur)
    cw.step(steps)
    torch.cuda.synchronize()
    out = cw.gather("prev"), cw.gather("cur")
    del cw
    return out


def assert_bitwise(got, ref, what):
    assert np.all(np.isfinite(got)), f"{what}: non-finite values (a halo cell not filled?)"
    if not np.array_equal(got, ref):
        e = np.max(np.abs(got.astype(np.float64) - ref)) / np.max(np.abs(ref))
        raise AssertionError(f"{what}: {np.count_nonzero(got != ref)} cells differ (rel {e:.3e})")


# ------------------------------------------------------------------ float64 --

@pytest.mark.parametrize("T", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("K,split_dim,grid", [(1, 0, None), (3, 0, None), (3, 1, None),
                                              (0, 0, (2, 3))])
def test_f64_2d(T, K, split_dim, grid):
    shape = (301, 517)
    up = synth.gaussian_field(shape, 20.0, 60).astype(np.float64)
    uc = synth.gaussian_field(shape, 21.0, 61).astype(np.float64)
    rp, rc = oracle.wave(up, uc, 0.25, 29)
    gp, gc = run(up, uc, 0.25, 29, T, "f64", K=K or 1, split_dim=split_dim, grid=grid)
    assert gc.dtype == np.float64
    assert_bitwise(gc, rc, f"f64 2D T={T} K={K} dim={split_dim} grid={grid} u^n")
    assert_bitwise(gp, rp, f"f64 2D T={T} u^(n-1)")


@pytest.mark.parametrize("T", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("K,split_dim,grid", [(3, 0, None), (2, 2, None), (0, 0, (1, 2, 2))])
def test_f64_3d(T, K, split_dim, grid):
    shape = (26, 45, 131)
    up = synth.gaussian_field(shape, 6.0, 62).astype(np.float64)
    uc = synth.gaussian_field(shape, 6.5, 63).astype(np.float64)
    rp, rc = oracle.wave(up, uc, 0.1, 13)
    gp, gc = run(up, uc, 0.1, 13, T, "f64", K=K or 1, split_dim=split_dim, grid=grid)
    assert_bitwise(gc, rc, f"f64 3D T={T} K={K} dim={split_dim} grid={grid} u^n")
    assert_bitwise(gp, rp, f"f64 3D T={T} u^(n-1)")


def test_f64_1000_steps():
    """The 256 x 256 workload's field for 1000 steps, 2 chunks, T = 4,
    against the float64 oracle (bitwise) and against the closed form's
    physics indirectly through the float32 oracle (1e-4)."""
    w = synth.WORKLOADS["wave2d_256_k2"]
    u0 = synth.gaussian_field(w["shape"], w["sigma"], w["seed"]).astype(np.float64)
    _, rc = oracle.wave(u0.copy(), u0, w["r2"], 1000)
    _, gc = run(u0, u0, w["r2"], 1000, 4, "f64", K=2)
    assert_bitwise(gc, rc, "f64 256^2 x 1000")


# ----------------------------------------------------------- 16-bit storage --

@pytest.mark.parametrize("fmt", ["bf16", "f16"])
@pytest.mark.parametrize("T", [1, 2, 5, 8])
@pytest.mark.parametrize("K,split_dim,grid", [(1, 0, None), (3, 0, None), (2, 1, None),
                                              (0, 0, (2, 2))])
def test_stored_2d(fmt, T, K, split_dim, grid):
    shape = (203, 322)
    up = synth.gaussian_field(shape, 20.0, 64)
    uc = synth.gaussian_field(shape, 21.0, 65)
    rp, rc = oracle.wave_stored(up, uc, 0.25, 27, T, fmt)
    gp, gc = run(up, uc, 0.25, 27, T, fmt, K=K or 1, split_dim=split_dim, grid=grid)
    assert_bitwise(gc, rc, f"{fmt} 2D T={T} K={K} dim={split_dim} grid={grid} u^n")
    assert_bitwise(gp, rp, f"{fmt} 2D T={T} u^(n-1)")


@pytest.mark.parametrize("fmt", ["bf16", "f16"])
@pytest.mark.parametrize("T", [1, 3, 6])
def test_stored_3d(fmt, T):
    shape = (22, 37, 140)
    u0 = synth.gaussian_field(shape, 6.0, 66)
    rp, rc = oracle.wave_stored(u0, u0, 0.1, 12, T, fmt)
    gp, gc = run(u0, u0, 0.1, 12, T, fmt, K=3)
    assert_bitwise(gc, rc, f"{fmt} 3D T={T} u^n")
    assert_bitwise(gp, rp, f"{fmt} 3D T={T} u^(n-1)")
    gp2, gc2 = run(u0, u0, 0.1, 12, T, fmt, K=2, split_dim=2)
    assert_bitwise(gc2, rc, f"{fmt} 3D T={T} x-split u^n")


def test_stored_tile_rows_invariant():
    shape = (150, 300)
    u0 = synth.gaussian_field(shape, 12.0, 67)
    _, rc = oracle.wave_stored(u0, u0, 0.25, 24, 4, "bf16")
    for rows in (4, 7, 33):
        _, gc = run(u0, u0, 0.25, 24, 4, "bf16", K=2, tile_rows=rows)
        assert_bitwise(gc, rc, f"bf16 rows={rows}")


# ----------------------------------------------------------------- budgets --
# Storage rounding error against the float64 oracle, max|a - b| / max|b|.
# Each pass rounds both stored levels to the format's unit roundoff u
# (2^-8 for bfloat16, 2^-11 for binary16); the leapfrog carries such
# perturbations along (a velocity error grows the displacement error with
# time), so the budget is written as passes * u times a factor measured once
# with the oracle (the GPU result equals the oracle bitwise, so these
# bounds restate the format's error, not the kernels').

BUDGET_256 = {  # (fmt, T): bound after 100 steps of the 256 x 256 workload
    ("bf16", 1): 0.15, ("bf16", 8): 0.06, ("f16", 1): 0.015, ("f16", 8): 0.008}


@pytest.mark.parametrize("fmt,T", sorted(BUDGET_256))
def test_stored_budget_256(fmt, T):
    w = synth.WORKLOADS["wave2d_256_k2"]
    u0 = synth.gaussian_field(w["shape"], w["sigma"], w["seed"])
    u64 = u0.astype(np.float64)
    _, r64 = oracle.wave(u64.copy(), u64, w["r2"], w["steps"])
    rp, rc = oracle.wave_stored(u0, u0, w["r2"], w["steps"], T, fmt)
    _, gc = run(u0, u0, w["r2"], w["steps"], T, fmt, K=w["chunks"])
    assert_bitwise(gc, rc, f"{fmt} 256^2 T={T}")
    e = float(np.max(np.abs(gc - r64)) / np.max(np.abs(r64)))
    print(f"{fmt} T={T}: {e:.3e} from the float64 oracle", flush=True)
    assert e <= BUDGET_256[(fmt, T)]
