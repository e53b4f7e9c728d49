"""GPU parity of block splits and splits along the inner dimensions.

ccl_wave_step over chunks cut along every dimension (ccl_split_grid: 2 x 2
and 4 x 2 in 2D, 2 x 2 x 2 and 1 x 2 x 2 in 3D) and along a single inner
dimension (columns in 2D; rows or columns in 3D), for several temporal
depths: the halos between chunks then run along columns, so the strided
boxes of the exchange (and, at block corners, the diagonal neighbours)
carry real data.  Every run must be bitwise equal to the float32 oracle on
the unsplit grid.  Buffers start NaN-poisoned, so a read of a cell the
exchange did not fill shows up.  Also: ccl_halo_exchange fills exactly the
regions the block-split chunks need, for the neighbourhood, slice and fixed
mappers.
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


def run(u_prev, u_cur, r2, steps, T, grid=None, K=1, split_dim=0, tile_rows=0):
    from paper_2505_06022_amd.fields import ChunkedWave
    shape = u_cur.shape
    print(f"split run: {shape} grid={grid} K={K} split_dim={split_dim} T={T}", flush=True)
    cw = ChunkedWave((0,) * len(shape), shape, K, r2, depth=T, tile_rows=tile_rows,
                     split_dim=split_dim, fill=float("nan"), grid=grid)
    cw.scatter(u_prev, u_cur)
    cw.step(steps)
    torch.cuda.synchronize()
    return cw.gather("prev"), cw.gather("cur")


def assert_bitwise(got, ref, what):
    assert np.all(np.isfinite(got)), f"{what}: non-finite values (a halo cell not filled?)"
    if not np.array_equal(got, ref):
        e = np.max(np.abs(got.astype(np.float64) - ref)) / np.max(np.abs(ref))
        raise AssertionError(f"{what}: {np.count_nonzero(got != ref)} cells differ (rel {e:.3e})")


@pytest.mark.parametrize("grid", [(2, 2), (4, 2), (3, 5), (1, 4)])
@pytest.mark.parametrize("T", [1, 2, 5, 8])
def test_block_split_2d(grid, T):
    """301 x 517 (columns not a multiple of 4): column chunk edges fall
    inside aligned groups of four, so partial groups are stored."""
    shape = (301, 517)
    up = synth.gaussian_field(shape, 20.0, seed=30)
    uc = synth.gaussian_field(shape, 21.0, seed=31)
    rp, rc = oracle.wave(up, uc, 0.25, 29)
    gp, gc = run(up, uc, 0.25, 29, T, grid=grid)
    assert_bitwise(gc, rc, f"2D grid={grid} T={T} u^n")
    assert_bitwise(gp, rp, f"2D grid={grid} T={T} u^(n-1)")


@pytest.mark.parametrize("K", [2, 3, 7])
@pytest.mark.parametrize("T", [1, 3, 4, 8])
def test_column_split_2d(K, T):
    shape = (150, 700)
    u0 = synth.gaussian_field(shape, 30.0, seed=32)
    rp, rc = oracle.wave(u0.copy(), u0, 0.25, 21)
    gp, gc = run(u0, u0, 0.25, 21, T, K=K, split_dim=1)
    assert_bitwise(gc, rc, f"2D columns K={K} T={T}")
    assert_bitwise(gp, rp, f"2D columns K={K} T={T} u^(n-1)")


@pytest.mark.parametrize("grid", [(2, 2, 2), (1, 2, 2), (1, 1, 3)])
@pytest.mark.parametrize("T", [1, 2, 3, 5, 6, 7, 8])
def test_block_split_3d(grid, T):
    """40 x 70 x 150: x chunks of 50 columns, so chunk edges are not at a
    multiple of 4 from their buffers' first columns for most T."""
    shape = (40, 70, 150)
    up = synth.gaussian_field(shape, 6.0, seed=33)
    uc = synth.gaussian_field(shape, 6.5, seed=34)
    rp, rc = oracle.wave(up, uc, 0.1, 17)
    gp, gc = run(up, uc, 0.1, 17, T, grid=grid)
    assert_bitwise(gc, rc, f"3D grid={grid} T={T} u^n")
    assert_bitwise(gp, rp, f"3D grid={grid} T={T} u^(n-1)")


@pytest.mark.parametrize("split_dim", [1, 2])
@pytest.mark.parametrize("T", [1, 2, 3, 4, 5, 6, 7, 8])
def test_inner_split_3d(split_dim, T):
    shape = (24, 66, 301)
    u0 = synth.gaussian_field(shape, 7.0, seed=35)
    rp, rc = oracle.wave(u0.copy(), u0, 0.1, 13)
    gp, gc = run(u0, u0, 0.1, 13, T, K=3, split_dim=split_dim)
    assert_bitwise(gc, rc, f"3D split_dim={split_dim} T={T}")
    assert_bitwise(gp, rp, f"3D split_dim={split_dim} T={T} u^(n-1)")


def test_block_split_tile_rows():
    shape = (200, 300)
    u0 = synth.gaussian_field(shape, 12.0, seed=36)
    _, rc = oracle.wave(u0.copy(), u0, 0.25, 24)
    for rows in (1, 5, 33):
        for T in (1, 4, 7):
            _, gc = run(u0, u0, 0.25, 24, T, grid=(3, 2), tile_rows=rows)
            assert_bitwise(gc, rc, f"grid 3x2 rows={rows} T={T}")


@pytest.mark.parametrize("dims,shape,grid", [(2, (37, 50), (2, 3)), (2, (64, 257), (4, 2)),
                                             (3, (23, 19, 70), (2, 2, 2)),
                                             (3, (9, 30, 41), (1, 3, 2))])
def test_halo_exchange_block_split(dims, shape, grid):
    """Every chunk buffer sized to its mapper's region; after one exchange
    each region holds the global field there (corner boxes from diagonal
    neighbours included), for neighbourhood, slice and fixed mappers."""
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.fields import alloc_buffer, view_of
    g = synth.uniform_field(shape, 40).astype(np.float32)
    chunks = ccl.ccl_split_grid((0,) * dims, shape, grid)
    mappers = [ccl.make_mapper(ccl.NEIGHBORHOOD, (2,) * dims),
               ccl.make_mapper(ccl.SLICE, dim=dims - 1),
               ccl.make_mapper(ccl.SLICE, dim=0),
               ccl.make_mapper(ccl.FIXED, tuple(n // 2 for n in shape),
                               offset=tuple(n // 4 for n in shape))]
    for m in mappers:
        regs = [ccl.ccl_region_of(c, m, None, shape).box() for c in chunks]
        bufs = (ccl.ccl_chunk_buffer * len(chunks))()
        ts = []
        for k, reg in enumerate(regs):
            # the buffer holds the chunk and its region (a fixed box need not
            # contain the chunk)
            lo = tuple(min(a, b) for a, b in zip(reg[0], chunks[k].box()[0]))
            hi = tuple(max(a + n, b + q) for a, n, b, q in
                       zip(reg[0], reg[1], chunks[k].box()[0], chunks[k].box()[1]))
            hold = (lo, tuple(h - l for h, l in zip(hi, lo)))
            t, b = alloc_buffer(hold, fill=float("nan"))
            bufs[k] = b
            ts.append((t, hold))
            box = chunks[k].box()
            sl = tuple(slice(o, o + n) for o, n in zip(*box))
            view_of(t, hold, box).copy_(torch.from_numpy(np.ascontiguousarray(g[sl])))
        ccl.ccl_halo_exchange(chunks, m, None, bufs)
        torch.cuda.synchronize()
        for k, reg in enumerate(regs):
            if 0 in reg[1]:
                continue
            t, hold = ts[k]
            sl = tuple(slice(o, o + n) for o, n in zip(*reg))
            got = view_of(t, hold, reg).cpu().numpy()
            assert np.array_equal(got, g[sl]), f"mapper {m.kind}, chunk {k}: region differs"
