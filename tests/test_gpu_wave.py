"""GPU parity tests of the chunked wave stencil, through the C ABI.

Bar: the HIP path evaluates the same float32 expression as the float32
oracle in the same order, so results must be bitwise equal (the test also
asserts the looser 1e-5 relative max-abs bound), and within 1e-4 relative of
the float64 oracle after 1000 steps.  Chunking, temporal depth and tiling are
re-orderings only: bitwise equal to the unchunked run.

All buffers start NaN-poisoned (halos, padding, cells outside the domain), so
a read of anything the halo exchange did not fill shows up as a NaN.
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
    ccl.lib()  # raises loudly if the library is missing
    yield


def rel_err(a, b):
    return float(np.max(np.abs(a.astype(np.float64) - b.astype(np.float64))) /
                 max(np.max(np.abs(b)), 1e-300))


def gpu_run(u_prev, u_cur, r2, steps, K, T, tile_rows=0, offset=None, buffer_range=None,
            fill=float("nan")):
    from paper_2505_06022_amd.fields import ChunkedWave
    shape = u_cur.shape
    offset = offset or (0,) * len(shape)
    cw = ChunkedWave(offset, shape, K, r2, depth=T, tile_rows=tile_rows,
                     buffer_range=buffer_range, fill=fill)
    cw.scatter(u_prev, u_cur)
    cw.step(steps)
    torch.cuda.synchronize()
    return cw.gather("prev"), cw.gather("cur")


def assert_bitwise(got, ref, what):
    assert np.all(np.isfinite(got)), f"{what}: non-finite values (stray halo read?)"
    e = rel_err(got, ref)
    assert e <= 1e-5, f"{what}: relative max-abs error {e:.3e} > 1e-5"
    assert np.array_equal(got, ref), f"{what}: within 1e-5 ({e:.3e}) but not bitwise equal"


# ------------------------------------------------------------------- SAXPY --

@pytest.mark.parametrize("n", [0, 1, 3, 4, 5, 1000003])
def test_saxpy_bitwise(n):
    import paper_2505_06022_amd as ccl
    rs = np.random.default_rng(n)
    x = rs.standard_normal(max(n, 1)).astype(np.float32)[:n]
    y = rs.standard_normal(max(n, 1)).astype(np.float32)[:n]
    xd = torch.from_numpy(x).cuda()
    yd = torch.from_numpy(y).cuda()
    zd = torch.full((max(n, 1),), float("nan"), device="cuda")
    ccl.ccl_saxpy(n, 1.75, xd.data_ptr(), yd.data_ptr(), zd.data_ptr())
    torch.cuda.synchronize()
    assert np.array_equal(zd.cpu().numpy()[:n], oracle.saxpy(1.75, x, y))


# -------------------------------------------------------------------- halo --

@pytest.mark.parametrize("dims,shape,K,e", [(2, (37, 50), 4, 2), (2, (64, 257), 3, 1),
                                           (3, (23, 9, 70), 5, 3), (2, (40, 40), 1, 2)])
def test_halo_exchange_fills_regions(dims, shape, K, e):
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.fields import alloc_buffer, view_of
    g = synth.uniform_field(shape, 5).astype(np.float32)
    chunks = ccl.ccl_split_range((0,) * dims, shape, K)
    regs = [ccl.ccl_region_of(c, ccl.NEIGHBORHOOD, (e,) * dims, shape).box() for c in chunks]
    bufs = (ccl.ccl_chunk_buffer * K)()
    ts = []
    for k, reg in enumerate(regs):
        t, b = alloc_buffer(reg, fill=float("nan"))
        bufs[k] = b
        ts.append(t)
        box = chunks[k].box()
        sl = tuple(slice(o, o + n) for o, n in zip(*box))
        view_of(t, reg, box).copy_(torch.from_numpy(np.ascontiguousarray(g[sl])))
    ccl.ccl_halo_exchange(chunks, ccl.NEIGHBORHOOD, (e,) * dims, bufs)
    torch.cuda.synchronize()
    for k, reg in enumerate(regs):
        sl = tuple(slice(o, o + n) for o, n in zip(*reg))
        got = view_of(ts[k], reg, reg).cpu().numpy()
        assert np.array_equal(got, g[sl]), f"chunk {k}: region differs after exchange"


def test_pack_unpack_roundtrip():
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.fields import alloc_buffer, view_of
    shape = (30, 45)
    g = synth.uniform_field(shape, 6).astype(np.float32)
    reg = ((0, 0), shape)
    t, b = alloc_buffer(reg)
    t[:, :shape[1]].copy_(torch.from_numpy(g))
    boxes = [ccl.make_subrange((3, 5), (4, 17)), ccl.make_subrange((0, 44), (30, 1)),
             ccl.make_subrange((29, 0), (1, 45))]
    n = sum(bx.range[0] * bx.range[1] for bx in boxes)
    staging = torch.full((n,), float("nan"), device="cuda")
    srcs = (ccl.ccl_chunk_buffer * 3)(b, b, b)
    ccl.ccl_halo_pack(boxes, srcs, 4, staging.data_ptr())
    torch.cuda.synchronize()
    want = np.concatenate([g[o0:o0 + r0, o1:o1 + r1].ravel() for (o0, o1), (r0, r1) in
                           (bx.box() for bx in boxes)])
    assert np.array_equal(staging.cpu().numpy(), want)
    t2, b2 = alloc_buffer(reg, fill=float("nan"))
    dsts = (ccl.ccl_chunk_buffer * 3)(b2, b2, b2)
    ccl.ccl_halo_unpack(boxes, dsts, 4, staging.data_ptr())
    torch.cuda.synchronize()
    got = view_of(t2, reg, reg).cpu().numpy()
    for (o0, o1), (r0, r1) in (bx.box() for bx in boxes):
        assert np.array_equal(got[o0:o0 + r0, o1:o1 + r1], g[o0:o0 + r0, o1:o1 + r1])


# ---------------------------------------------------------------- 2D wave --

def test_config0_256_k2():
    """256x256, r2 = 0.25, sigma 16, seeded noise, 100 steps, 2 row chunks."""
    w = synth.WORKLOADS["wave2d_256_k2"]
    u0 = synth.gaussian_field(w["shape"], w["sigma"], w["seed"])
    ref_p, ref_c = oracle.wave(u0.copy(), u0, w["r2"], w["steps"])
    u64 = u0.astype(np.float64)
    _, ref64 = oracle.wave(u64.copy(), u64, w["r2"], w["steps"])
    for T in (1, 2, 4, 8):
        gp, gc = gpu_run(u0, u0, w["r2"], w["steps"], w["chunks"], T)
        assert_bitwise(gc, ref_c, f"config0 T={T} u^n")
        assert_bitwise(gp, ref_p, f"config0 T={T} u^(n-1)")
        assert rel_err(gc, ref64) <= 1e-4


@pytest.mark.parametrize("T", [1, 2, 3, 4, 5, 8])
def test_chunked_ragged_all_depths(T):
    """301 x 517 (columns not a multiple of 4), 37 steps (not a multiple of T),
    every chunk count, against the float32 oracle."""
    shape = (301, 517)
    u_prev = synth.gaussian_field(shape, 20.0, seed=7)
    u_cur = synth.gaussian_field(shape, 21.0, seed=8)
    _, ref = oracle.wave(u_prev, u_cur, 0.25, 37)
    for K in (1, 2, 3, 5, 8, 16):
        _, gc = gpu_run(u_prev, u_cur, 0.25, 37, K, T)
        assert_bitwise(gc, ref, f"K={K} T={T}")


@pytest.mark.parametrize("tile_rows", [1, 2, 5, 8, 16, 33, 1000])
def test_tile_rows_invariance(tile_rows):
    """Tiles of every height, down to one row: segments shorter than the
    kernel's three-row loop body and row counts (rows + 2T) that are not a
    multiple of three, so the rows stored after the loop are exercised."""
    shape = (200, 300)
    u0 = synth.gaussian_field(shape, 12.0, seed=9)
    _, ref = oracle.wave(u0.copy(), u0, 0.25, 24)
    for T in (1, 3, 6, 7, 8):
        _, gc = gpu_run(u0, u0, 0.25, 24, 3, T, tile_rows=tile_rows)
        assert_bitwise(gc, ref, f"tile_rows={tile_rows} T={T}")


def test_share_with_offset_and_virtual_buffer():
    """A row share at offset (40, 0) of a taller virtual buffer: cells outside
    the share (inside the buffer) never feed the result (Dirichlet share)."""
    shape = (120, 96)
    u0 = synth.gaussian_field(shape, 10.0, seed=10)
    _, ref = oracle.wave(u0.copy(), u0, 0.25, 30)
    for K, T in ((1, 1), (3, 1), (3, 4), (4, 7)):
        _, gc = gpu_run(u0, u0, 0.25, 30, K, T, offset=(40, 0), buffer_range=(400, 96))
        assert_bitwise(gc, ref, f"share K={K} T={T}")


def test_determinism_and_zero_steps():
    shape = (128, 128)
    u0 = synth.gaussian_field(shape, 10.0, seed=12)
    a = gpu_run(u0, u0, 0.25, 20, 2, 4)[1]
    b = gpu_run(u0, u0, 0.25, 20, 2, 4)[1]
    assert np.array_equal(a, b)
    _, c = gpu_run(u0, u0, 0.25, 0, 2, 4)
    assert np.array_equal(c, u0)


def test_fp64_oracle_after_1000_steps():
    """1024 x 1024, 1000 steps, 4 chunks, T = 4: within 1e-4 of float64."""
    shape = (1024, 1024)
    u0 = synth.gaussian_field(shape, 32.0, seed=13)
    th = oracle.max_threads()
    _, ref32 = oracle.wave(u0.copy(), u0, 0.25, 1000, threads=th)
    u64 = u0.astype(np.float64)
    _, ref64 = oracle.wave(u64.copy(), u64, 0.25, 1000, threads=th)
    _, gc = gpu_run(u0, u0, 0.25, 1000, 4, 4)
    assert_bitwise(gc, ref32, "1024^2 x 1000")
    assert rel_err(gc, ref64) <= 1e-4


# ---------------------------------------------------------------- 3D wave --

@pytest.mark.parametrize("K", [1, 3, 7])
def test_wave3d_ragged(K):
    shape = (40, 36, 300)
    u_prev = synth.gaussian_field(shape, 6.0, seed=14)
    u_cur = synth.gaussian_field(shape, 6.5, seed=15)
    _, ref = oracle.wave(u_prev, u_cur, 0.1, 25)
    gp, gc = gpu_run(u_prev, u_cur, 0.1, 25, K, 1)
    assert_bitwise(gc, ref, f"3D K={K}")


@pytest.mark.parametrize("T", [2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("K", [1, 3])
def test_wave3d_depths(T, K):
    """Temporally blocked 3D kernel: several patches in x (56 or 48 output
    columns) and y, ragged tails, 25 steps = blocks of T plus a shorter one."""
    shape = (21, 70, 150)
    u_prev = synth.gaussian_field(shape, 6.0, seed=17)
    u_cur = synth.gaussian_field(shape, 6.5, seed=18)
    ref_prev, ref = oracle.wave(u_prev, u_cur, 0.1, 25)
    gp, gc = gpu_run(u_prev, u_cur, 0.1, 25, K, T)
    assert_bitwise(gc, ref, f"3D T={T} K={K}")
    assert_bitwise(gp, ref_prev, f"3D T={T} K={K} (u^(n-1))")


def test_wave3d_depth_tile_planes():
    shape = (33, 20, 64)
    u0 = synth.gaussian_field(shape, 5.0, seed=16)
    _, ref = oracle.wave(u0.copy(), u0, 0.1, 12)
    for tp in (1, 5, 64):
        _, gc = gpu_run(u0, u0, 0.1, 12, 2, 4, tile_rows=tp)
        assert_bitwise(gc, ref, f"3D T=4 tile_planes={tp}")


def test_wave3d_tile_planes():
    shape = (33, 20, 64)
    u0 = synth.gaussian_field(shape, 5.0, seed=16)
    _, ref = oracle.wave(u0.copy(), u0, 0.1, 12)
    for tp in (1, 5, 64):
        _, gc = gpu_run(u0, u0, 0.1, 12, 2, 1, tile_rows=tp)
        assert_bitwise(gc, ref, f"3D tile_planes={tp}")


# ------------------------------------------------------------ measurement --

def test_timing_counts_launches():
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.fields import ChunkedWave
    u0 = synth.gaussian_field((256, 256), 16.0, seed=0)
    cw = ChunkedWave((0, 0), (256, 256), 2, 0.25, depth=4)
    cw.scatter(u0, u0)
    torch.cuda.synchronize()
    ccl.ccl_timing_enable(True)
    cw.step(10)  # blocks of 4, 4, 2
    torch.cuda.synchronize()
    n, ms = ccl.ccl_timing_query(ccl.CCL_KERNEL_STENCIL)
    nh, _ = ccl.ccl_timing_query(ccl.CCL_KERNEL_HALO)
    ccl.ccl_timing_enable(False)
    # rows split: one exchange before the first block, the stencil launches
    # store the later halos into the neighbours' buffers themselves
    assert n == 3 and ms > 0 and nh == 1
    # columns split: no pushes, an exchange before every block
    cc = ChunkedWave((0, 0), (256, 256), 2, 0.25, depth=4, split_dim=1)
    cc.scatter(u0, u0)
    torch.cuda.synchronize()
    ccl.ccl_timing_enable(True)
    cc.step(10)
    torch.cuda.synchronize()
    n, _ = ccl.ccl_timing_query(ccl.CCL_KERNEL_STENCIL)
    nh, _ = ccl.ccl_timing_query(ccl.CCL_KERNEL_HALO)
    ccl.ccl_timing_enable(False)
    assert n == 3 and nh == 3
    assert np.array_equal(cc.gather("cur"), cw.gather("cur"))


@pytest.mark.parametrize("shape,K,T", [((1, 300), 1, 1), ((1, 300), 1, 4), ((57, 1), 3, 2),
                                       ((40, 3), 40, 4), ((12, 700), 12, 8), ((5, 5), 5, 6),
                                       ((2, 2), 2, 8)])
def test_degenerate_shapes(shape, K, T):
    """Single-row/column grids, one-row chunks whose halo reaches several
    chunks away, domains narrower than one strip, depth beyond the grid."""
    u_prev = synth.gaussian_field(shape, 3.0, seed=20)
    u_cur = synth.gaussian_field(shape, 2.0, seed=21)
    _, ref = oracle.wave(u_prev, u_cur, 0.25, 13)
    _, gc = gpu_run(u_prev, u_cur, 0.25, 13, K, T)
    assert_bitwise(gc, ref, f"{shape} K={K} T={T}")


@pytest.mark.parametrize("shape,K,T", [((1, 1, 1), 1, 1), ((3, 1, 5), 3, 1), ((7, 9, 1), 2, 1),
                                       ((2, 300, 260), 2, 1), ((1, 1, 1), 1, 2),
                                       ((3, 1, 5), 3, 4), ((7, 9, 1), 2, 8),
                                       ((2, 300, 260), 2, 3), ((9, 2, 70), 9, 6)])
def test_degenerate_shapes_3d(shape, K, T):
    u0 = synth.gaussian_field(shape, 2.0, seed=22)
    _, ref = oracle.wave(u0.copy(), u0, 0.1, 9)
    _, gc = gpu_run(u0, u0, 0.1, 9, K, T)
    assert_bitwise(gc, ref, f"3D {shape} K={K} T={T}")


def test_energy_read():
    """Device energy over a window of at least one second, by the counter's
    own timestamps, while the GPU works: the energy rises (dE > 0) and the
    mean power lies in (0, 1400 W], 1400 W being the MI355X's rated board
    power."""
    import time

    import paper_2505_06022_amd as ccl
    s = torch.cuda.current_stream()
    try:
        e0, t0 = ccl.ccl_energy_read(0, s)
    except ccl.CclError as e:
        assert e.status == ccl.CCL_E_UNSUPPORTED
        pytest.skip(f"no energy backend on this machine: {e.message}")
    x = torch.rand(1 << 26, device="cuda")
    start = time.perf_counter()
    while True:
        for _ in range(50):
            x.mul_(1.0000001)
        e1, t1 = ccl.ccl_energy_read(0, s)
        if (t1 - t0) * 1e-9 >= 1.0 and e1 != e0:
            break
        assert time.perf_counter() - start < 30, "energy counter did not advance in 30 s"
    de, dt = e1 - e0, (t1 - t0) * 1e-9
    print(f"energy backend {ccl.ccl_energy_backend(0)}: {de:.3f} J over {dt:.3f} s "
          f"= {de / dt:.1f} W", flush=True)
    assert de > 0, f"energy did not rise over {dt:.3f} s"
    assert 0 < de / dt <= 1400.0, f"mean power {de / dt:.1f} W outside (0, 1400]"
