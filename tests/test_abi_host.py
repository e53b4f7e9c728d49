"""Host-side tests of libccl (CPU only: no kernel is launched).

* The library loads and exports every function include/ccl.h declares.
* ccl_split_range / ccl_region_of / ccl_transfers agree with the oracle's
  interval arithmetic, exhaustively on small ranges.
* Argument validation returns the documented status codes before any device
  work is enqueued.
* The fake energy backend drives the J/step arithmetic.
"""
import ctypes
import os
import re
import subprocess
import sys

import pytest

import paper_2505_06022_amd as ccl
from oracle import ranges

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    with open(os.path.join(ROOT, "include", "ccl.h")) as f:
        src = f.read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ccl_[a-z_0-9]+)\s*\(", src)))


def test_exports_every_declared_symbol():
    names = declared_functions()
    assert len(names) >= 10
    L = ccl.lib()
    for n in names:
        assert hasattr(L, n), f"libccl.so does not export {n}"
    assert set(names) <= set(ccl._SIGS), "binding lacks a signature for a declared function"


def test_version():
    assert "gfx950" in ccl.ccl_version()


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_split_matches_oracle(dims):
    for n in (1, 2, 5, 17, 64):
        for K in range(1, min(n, 16) + 1):
            for sd in range(dims):
                rng = [4] * dims
                rng[sd] = n
                off = [3, -2, 7][:dims]
                got = [c.box() for c in ccl.ccl_split_range(off, rng, K, sd)]
                want = ranges.split_range(tuple(off), tuple(rng), K, sd)
                assert got == want
                for c in ccl.ccl_split_range(off, rng, K, sd):
                    assert tuple(c.global_offset[:dims]) == tuple(off)
                    assert tuple(c.global_range[:dims]) == tuple(rng)


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_region_matches_oracle(dims):
    import numpy as np
    rs = np.random.default_rng(11)
    for _ in range(300):
        buf = tuple(int(v) for v in rs.integers(1, 40, size=dims))
        rng = tuple(int(rs.integers(1, b + 1)) for b in buf)
        off = tuple(int(rs.integers(0, b - r + 1)) for b, r in zip(buf, rng))
        K = int(rs.integers(1, rng[0] + 1))
        for c in ccl.ccl_split_range(off, rng, K, 0):
            for kind in (ccl.ONE_TO_ONE, ccl.NEIGHBORHOOD, ccl.ALL):
                e = tuple(int(v) for v in rs.integers(0, 6, size=dims))
                got = ccl.ccl_region_of(c, kind, e, buf).box()
                assert got == ranges.region_of(c.box(), kind, e, buf)


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_split_grid_matches_oracle(dims):
    import itertools
    sizes = (1, 3, 8, 17) if dims < 3 else (1, 4, 9)
    for rng in itertools.product(sizes, repeat=dims):
        off = tuple([3, -2, 7][:dims])
        for counts in itertools.product(*[range(1, min(n, 5) + 1) for n in rng]):
            got = [c.box() for c in ccl.ccl_split_grid(off, rng, counts)]
            assert got == ranges.split_grid(off, rng, counts)
    L = ccl.lib()
    out = (ccl.ccl_chunk * 64)()
    r = ccl.make_subrange((0, 0), (4, 4))
    cn = (ctypes.c_int32 * 3)(5, 1, 1)
    assert L.ccl_split_grid(ctypes.byref(r), cn, out) == ccl.CCL_E_RANGE
    cn = (ctypes.c_int32 * 3)(2, 0, 1)
    assert L.ccl_split_grid(ctypes.byref(r), cn, out) == ccl.CCL_E_INVALID
    assert L.ccl_split_grid(None, cn, out) == ccl.CCL_E_INVALID


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_fixed_and_slice_match_oracle(dims):
    import numpy as np
    rs = np.random.default_rng(12)
    for _ in range(200):
        buf = tuple(int(v) for v in rs.integers(1, 30, size=dims))
        counts = tuple(int(rs.integers(1, min(b, 3) + 1)) for b in buf)
        for c in ccl.ccl_split_grid((0,) * dims, buf, counts):
            fo = tuple(int(rs.integers(-5, b + 3)) for b in buf)
            fe = tuple(int(rs.integers(0, 12)) for _ in buf)
            m = ccl.make_mapper(ccl.FIXED, fe, offset=fo)
            assert ccl.ccl_region_of(c, m, None, buf).box() == \
                ranges.region_of(c.box(), ranges.FIXED, fe, buf, offset=fo)
            for d in range(dims):
                m = ccl.make_mapper(ccl.SLICE, dim=d)
                assert ccl.ccl_region_of(c, m, None, buf).box() == \
                    ranges.region_of(c.box(), ranges.SLICE, (0,) * dims, buf, dim=d)
    L = ccl.lib()
    c = ccl.ccl_split_range((0,) * dims, (4,) * dims, 1)[0]
    out = ccl.ccl_subrange()
    br = ccl._i64((4,) * dims)
    bad = ccl.make_mapper(ccl.SLICE, dim=dims)
    assert L.ccl_region_of(ctypes.byref(c), ctypes.byref(bad), br, ctypes.byref(out)) == \
        ccl.CCL_E_INVALID
    bad = ccl.make_mapper(ccl.FIXED, (-1,) * dims)
    assert L.ccl_region_of(ctypes.byref(c), ctypes.byref(bad), br, ctypes.byref(out)) == \
        ccl.CCL_E_INVALID


def test_block_split_transfers_match_oracle():
    """Transfers among the chunks of block splits (corner boxes included)."""
    for dims, shape, counts in ((2, (37, 29), (2, 2)), (2, (37, 29), (4, 2)),
                                (2, (9, 40), (3, 5)), (3, (19, 11, 13), (2, 2, 2)),
                                (3, (19, 11, 13), (1, 2, 3))):
        chunks = ccl.ccl_split_grid((0,) * dims, shape, counts)
        for e in (0, 1, 2, 4):
            got = sorted((t.owner, t.reader, t.box.box()) for t in
                         ccl.ccl_transfers(chunks, ccl.NEIGHBORHOOD, (e,) * dims, shape))
            regs = [ranges.region_of(c.box(), ranges.NEIGHBORHOOD, (e,) * dims, shape)
                    for c in chunks]
            want = sorted(ranges.transfers([c.box() for c in chunks], regs))
            assert got == want
        for d in range(dims):
            m = ccl.make_mapper(ccl.SLICE, dim=d)
            got = sorted((t.owner, t.reader, t.box.box()) for t in
                         ccl.ccl_transfers(chunks, m, None, shape))
            regs = [ranges.region_of(c.box(), ranges.SLICE, (0,) * dims, shape, dim=d)
                    for c in chunks]
            assert got == sorted(ranges.transfers([c.box() for c in chunks], regs))


def test_transfers_match_oracle():
    for dims, shape in ((2, (37, 11)), (3, (19, 5, 6))):
        for K in (1, 2, 3, 7):
            for e in (0, 1, 2, 4):
                chunks = ccl.ccl_split_range((0,) * dims, shape, K, 0)
                got = sorted((t.owner, t.reader, t.box.box()) for t in
                             ccl.ccl_transfers(chunks, ccl.NEIGHBORHOOD, (e,) * dims, shape))
                regs = [ranges.region_of(c.box(), ranges.NEIGHBORHOOD, (e,) * dims, shape)
                        for c in chunks]
                want = sorted(ranges.transfers([c.box() for c in chunks], regs))
                assert got == want


def _status(fn, *args):
    return fn(*args)


def test_split_errors():
    L = ccl.lib()
    out = (ccl.ccl_chunk * 8)()
    r = ccl.make_subrange((0, 0), (4, 4))
    assert L.ccl_split_range(ctypes.byref(r), 0, 0, out) == ccl.CCL_E_INVALID
    assert L.ccl_split_range(ctypes.byref(r), 5, 0, out) == ccl.CCL_E_RANGE
    assert "exceeds" in ccl.ccl_last_error()
    assert L.ccl_split_range(ctypes.byref(r), 2, 2, out) == ccl.CCL_E_INVALID
    assert L.ccl_split_range(None, 2, 0, out) == ccl.CCL_E_INVALID
    bad = ccl.make_subrange((0, 0, 0, 0)[:3], (4, 4, 4))
    bad.dims = 4
    assert L.ccl_split_range(ctypes.byref(bad), 2, 0, out) == ccl.CCL_E_INVALID
    bad.dims = 2
    bad.range[1] = 0
    assert L.ccl_split_range(ctypes.byref(bad), 2, 0, out) == ccl.CCL_E_INVALID


def test_region_errors():
    L = ccl.lib()
    c = ccl.ccl_split_range((0, 0), (8, 8), 2)[0]
    m = ccl.make_mapper(7)
    out = ccl.ccl_subrange()
    br = ccl._i64((8, 8))
    assert L.ccl_region_of(ctypes.byref(c), ctypes.byref(m), br, ctypes.byref(out)) == ccl.CCL_E_INVALID
    m = ccl.make_mapper(ccl.NEIGHBORHOOD, (-1, 0))
    assert L.ccl_region_of(ctypes.byref(c), ctypes.byref(m), br, ctypes.byref(out)) == ccl.CCL_E_INVALID


def _fake_buffers(chunks, regions, base=0x10000000, pitch_align=64):
    arr = (ccl.ccl_chunk_buffer * len(chunks))()
    for k, reg in enumerate(regions):
        off, rng = reg
        b = arr[k]
        b.base = base + k * (1 << 30)
        b.region = ccl.make_subrange(off, rng)
        p = (rng[-1] + pitch_align - 1) // pitch_align * pitch_align
        if len(rng) == 2:
            b.pitch[0], b.pitch[1] = p, 1
        else:
            b.pitch[0], b.pitch[1], b.pitch[2] = p * rng[1], p, 1
    return arr


def test_wave_step_validation_no_launch():
    """Every failure below is detected on the host before any launch (the
    buffer addresses are never dereferenced)."""
    shape = (64, 32)
    chunks = ccl.ccl_split_range((0, 0), shape, 4)
    L = ccl.lib()

    def call(p, u_prev, u_cur, w_prev=None, w_cur=None, n=10, chunks=chunks):
        return L.ccl_wave_step(ctypes.byref(p), len(chunks), chunks, u_prev, u_cur, w_prev,
                               w_cur, n, None)

    regs1 = [ccl.ccl_region_of(c, ccl.NEIGHBORHOOD, (1, 1), shape).box() for c in chunks]
    regs0 = [c.box() for c in chunks]
    good = ccl.make_wave_params(2, 0.25, 1)
    # bad params
    for p in (ccl.make_wave_params(4, 0.25), ccl.make_wave_params(2, -1.0),
              ccl.make_wave_params(2, 0.25, 0), ccl.make_wave_params(2, 0.25, 9),
              ccl.make_wave_params(2, float("nan"))):
        assert call(p, _fake_buffers(chunks, regs1), _fake_buffers(chunks, regs1)) == ccl.CCL_E_INVALID
    assert call(good, _fake_buffers(chunks, regs1), _fake_buffers(chunks, regs1), n=-1) == ccl.CCL_E_INVALID
    # u^n region without its halo
    assert call(good, _fake_buffers(chunks, regs1), _fake_buffers(chunks, regs0)) == ccl.CCL_E_RANGE
    assert "halo" in ccl.ccl_last_error()
    # T=1 rotates u_prev into the u^n role: one_to_one u_prev fails from step 2 on
    assert call(good, _fake_buffers(chunks, regs0), _fake_buffers(chunks, regs1)) == ccl.CCL_E_RANGE
    # T>1 without the second buffer pair
    p4 = ccl.make_wave_params(2, 0.25, 4)
    regs4 = [ccl.ccl_region_of(c, ccl.NEIGHBORHOOD, (4, 4), shape).box() for c in chunks]
    assert call(p4, _fake_buffers(chunks, regs4), _fake_buffers(chunks, regs4)) == ccl.CCL_E_INVALID
    # misaligned base
    bad = _fake_buffers(chunks, regs1)
    bad[0].base = bad[0].base + 4
    assert call(good, bad, _fake_buffers(chunks, regs1)) == ccl.CCL_E_INVALID
    # pitch not a multiple of 4
    bad = _fake_buffers(chunks, regs1)
    bad[1].pitch[0] = 34
    assert call(good, bad, _fake_buffers(chunks, regs1)) == ccl.CCL_E_INVALID
    # element types: unknown dtype; float64 groups are two elements (pitch 34
    # is fine, an 8-byte offset is not); 16-bit groups are 8 bytes
    pbad = ccl.make_wave_params(2, 0.25, 1)
    pbad.dtype = 7
    assert call(pbad, _fake_buffers(chunks, regs1), _fake_buffers(chunks, regs1)) == ccl.CCL_E_INVALID
    p64 = ccl.make_wave_params(2, 0.25, 1, dtype="f64")
    odd = _fake_buffers(chunks, regs1)
    odd[1].pitch[0] = 33
    assert call(p64, odd, _fake_buffers(chunks, regs1)) == ccl.CCL_E_INVALID
    off8 = _fake_buffers(chunks, regs1)
    off8[0].base = off8[0].base + 8
    assert call(p64, off8, _fake_buffers(chunks, regs1)) == ccl.CCL_E_INVALID
    pb = ccl.make_wave_params(2, 0.25, 1, dtype="bf16")
    off4 = _fake_buffers(chunks, regs1)
    off4[0].base = off4[0].base + 4
    assert call(pb, off4, _fake_buffers(chunks, regs1)) == ccl.CCL_E_INVALID
    # r2 that overflows float is refused for the float-arithmetic types only
    assert call(ccl.make_wave_params(2, 1e300, 1), _fake_buffers(chunks, regs1),
                _fake_buffers(chunks, regs1)) == ccl.CCL_E_INVALID
    # overlapping chunks
    ov = ccl.ccl_split_range((0, 0), shape, 4)
    ov[1].offset[0] -= 1
    ov[1].range[0] += 1
    assert call(good, _fake_buffers(chunks, regs1), _fake_buffers(chunks, regs1),
                chunks=ov) == ccl.CCL_E_RANGE
    # 3D with T > 1 also needs the second buffer pair
    c3 = ccl.ccl_split_range((0, 0, 0), (8, 8, 8), 1)
    p3 = ccl.make_wave_params(3, 0.1, 2)
    r3 = [c3[0].box()]
    assert call(p3, _fake_buffers(c3, r3), _fake_buffers(c3, r3), chunks=c3) == ccl.CCL_E_INVALID
    assert "w_prev" in ccl.ccl_last_error()
    # zero steps is a no-op that succeeds without touching memory
    assert call(good, _fake_buffers(chunks, regs1), _fake_buffers(chunks, regs1), n=0) == ccl.CCL_OK


def test_halo_exchange_validation_no_launch():
    shape = (32, 16)
    chunks = ccl.ccl_split_range((0, 0), shape, 2)
    L = ccl.lib()
    m = ccl.make_mapper(ccl.NEIGHBORHOOD, (2, 2))
    small = _fake_buffers(chunks, [c.box() for c in chunks])
    assert L.ccl_halo_exchange(2, chunks, ctypes.byref(m), small, 4, None) == ccl.CCL_E_RANGE
    regs = [ccl.ccl_region_of(c, ccl.NEIGHBORHOOD, (2, 2), shape).box() for c in chunks]
    assert L.ccl_halo_exchange(2, chunks, ctypes.byref(m), _fake_buffers(chunks, regs), 3,
                               None) == ccl.CCL_E_INVALID


def test_saxpy_validation_no_launch():
    L = ccl.lib()
    assert L.ccl_saxpy(-1, 1.0, None, None, None, None) == ccl.CCL_E_INVALID
    assert L.ccl_saxpy(0, 1.0, None, None, None, None) == ccl.CCL_OK
    assert L.ccl_saxpy(16, 1.0, ctypes.c_void_p(0x1004), ctypes.c_void_p(0x2000),
                       ctypes.c_void_p(0x3000), None) == ccl.CCL_E_INVALID


def test_fake_energy_backend():
    code = ("import time, paper_2505_06022_amd as c; a,_=c.ccl_energy_read(0); time.sleep(0.2); "
            "b,_=c.ccl_energy_read(0); print(c.ccl_energy_backend(0), b-a)")
    env = dict(os.environ, CCL_ENERGY_BACKEND="fake", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, env=env,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    name, delta = r.stdout.split()
    assert name == "fake"
    assert 0.2 * 250 * 0.9 <= float(delta) <= 0.2 * 250 * 3  # 250 W scripted


def test_batch_create_validation_no_launch():
    L = ccl.lib()
    h = ctypes.c_void_p()
    g = ccl.ccl_batch_grid()
    g.ny, g.nx, g.pitch, g.steps, g.temporal_depth, g.r2 = 16, 16, 16, 4, 1, 0.25
    for k in range(4):
        g.buf[k] = 0x10000000 + k * 4096
    arr = (ccl.ccl_batch_grid * 1)(g)
    assert L.ccl_batch_create(0, arr, 0, ctypes.byref(h)) == ccl.CCL_E_INVALID
    bad = ccl.ccl_batch_grid.from_buffer_copy(g)
    bad.pitch = 18
    assert L.ccl_batch_create(1, (ccl.ccl_batch_grid * 1)(bad), 0, ctypes.byref(h)) == ccl.CCL_E_INVALID
    bad = ccl.ccl_batch_grid.from_buffer_copy(g)
    bad.temporal_depth = 9
    assert L.ccl_batch_create(1, (ccl.ccl_batch_grid * 1)(bad), 0, ctypes.byref(h)) == ccl.CCL_E_INVALID
    bad = ccl.ccl_batch_grid.from_buffer_copy(g)
    bad.temporal_depth, bad.tile_rows = 4, 2
    assert L.ccl_batch_create(1, (ccl.ccl_batch_grid * 1)(bad), 0, ctypes.byref(h)) == ccl.CCL_E_INVALID
    bad = ccl.ccl_batch_grid.from_buffer_copy(g)
    bad.buf[2] = 0x10000004
    assert L.ccl_batch_create(1, (ccl.ccl_batch_grid * 1)(bad), 0, ctypes.byref(h)) == ccl.CCL_E_INVALID
    assert L.ccl_batch_create(1, arr, 8, ctypes.byref(h)) == ccl.CCL_E_INVALID
    assert L.ccl_batch_destroy(None) == ccl.CCL_OK


def test_costmodel_features_host():
    """Features of three configs written out by hand from the kernels'
    tiling (2D strips of 256 columns, 3D one-step tiles of 256 x 4, 3D
    blocked patches of 64 x 64 cells streamed by 16 waves)."""
    import math
    import numpy as np
    c2 = ccl.make_tune_config((1024, 4096), 4, 8, 64)
    c3 = ccl.make_tune_config((96, 768, 768), 8, 1, 32)
    c3b = ccl.make_tune_config((100, 200, 300), 3, 5, 16)
    x = ccl.ccl_costmodel_features([c2, c3, c3b])

    def fill(waves, slots):
        return waves / (math.ceil(waves / slots) * slots)

    # 2D, T = 8: strips of 256 - 2*8 = 240 output columns, segments of 64 rows
    halo2 = 2 * 3 * 15 * (4 * 4096) * 2 / 8
    waves2 = 4 * math.ceil(256 / 64) * math.ceil(4096 / 240)
    red2 = 4 * math.ceil(256 / 64) * (64 + 16) * math.ceil(4096 / 240) * 256 / (1024 * 4096)
    s2 = ccl.ccl_wave_slots(2, 8)
    want2 = [10, 12, 0, 0, math.log2(red2), 2, 6, 8, fill(waves2, s2), math.log2(1 + halo2), 2.0,
             math.log2(waves2)]
    # 3D, T = 1: 96 planes in 8 chunks of 12, tiles of 32 planes, 256 x 4 cells
    halo3 = 2 * 7 * 1 * (4 * 768 * 768) * 2 / 1
    waves3 = 8 * math.ceil(12 / 32) * math.ceil(768 / 256) * math.ceil(768 / 4)
    red3 = 8 * (32 + 2) * 3 * 256 * 192 * 6 / (96 * 768 * 768)
    s3 = ccl.ccl_wave_slots(3, 1)
    want3 = [math.log2(96), math.log2(768), math.log2(768), 1, math.log2(red3), 3, 5, 1,
             fill(waves3, s3), math.log2(1 + halo3), 12.0, math.log2(waves3)]
    # 3D, T = 5: 16-wave patches of 64 x 64 cells writing 48 x 54; chunks of 33, 33, 34 planes
    segs = [math.ceil(33 / 16), math.ceil(33 / 16), math.ceil(34 / 16)]
    tiles = [s * math.ceil(300 / 48) * math.ceil(200 / 54) for s in segs]
    waves3b = 16 * sum(tiles)
    red3b = sum(t * (16 + 10) * 64 * 64 for t in tiles) / (100 * 200 * 300)
    halo3b = 2 * 2 * 9 * (4 * 200 * 300) * 2 / 5
    s3b = ccl.ccl_wave_slots(3, 5)
    want3b = [math.log2(100), math.log2(200), math.log2(300), 1, math.log2(red3b),
              math.log2(3), 4, 5, fill(waves3b, s3b), math.log2(1 + halo3b), 16 / 5,
              math.log2(waves3b)]
    assert np.allclose(x[0], want2, rtol=1e-6)
    assert np.allclose(x[1], want3, rtol=1e-6)
    assert np.allclose(x[2], want3b, rtol=1e-6)
    L = ccl.lib()
    bad = ccl.make_tune_config((16, 16), 0, 1, 16)
    arr = (ccl.ccl_tune_config * 1)(bad)
    out = (ctypes.c_float * 12)()
    assert L.ccl_costmodel_features(1, arr, out) == ccl.CCL_E_INVALID


def test_parallel_for_validation_no_launch():
    """ccl_parallel_for rejects a bad call on the host before any copy or
    launch (buffers here are fake addresses that are never touched)."""
    shape = (40, 30)
    chunks = ccl.ccl_split_grid((0, 0), shape, (2, 2))
    o2o = ccl.make_mapper(ccl.ONE_TO_ONE)
    nbh = ccl.make_mapper(ccl.NEIGHBORHOOD, (1, 1))
    own = [c.box() for c in chunks]
    fb = lambda regs, base: _fake_buffers(chunks, regs, base=base)
    L = ccl.lib()

    def call(fn, accs, a=1.0, dim=0):
        k = ccl.ccl_kernel_fn()
        k.fn, k.a, k.dim = fn, a, dim
        arr = (ccl.ccl_accessor * len(accs))(*accs)
        return L.ccl_parallel_for(ctypes.byref(k), len(chunks), chunks, len(accs), arr, None)

    R, W = ccl.CCL_ACCESS_READ, ccl.CCL_ACCESS_WRITE
    x = ccl.make_accessor(o2o, R, shape, fb(own, 0x10000000))
    y = ccl.make_accessor(o2o, R, shape, fb(own, 0x20000000))
    z = ccl.make_accessor(o2o, W, shape, fb(own, 0x30000000))
    assert call(ccl.CCL_FN_SAXPY, [x, y]) == ccl.CCL_E_INVALID            # arity
    assert call(7, [x, y, z]) == ccl.CCL_E_INVALID                         # unknown function
    assert call(ccl.CCL_FN_SAXPY, [x, y, ccl.make_accessor(o2o, R, shape, fb(own, 0x30000000))]) \
        == ccl.CCL_E_INVALID                                               # z not writable
    assert call(ccl.CCL_FN_SAXPY, [ccl.make_accessor(o2o, W, shape, fb(own, 0x10000000)), y, z]) \
        == ccl.CCL_E_INVALID                                               # x not readable
    assert call(ccl.CCL_FN_SAXPY, [x, y, ccl.make_accessor(nbh, W, shape, fb(own, 0x30000000))]) \
        == ccl.CCL_E_INVALID                                               # written through nbh
    assert "ONE_TO_ONE" in ccl.ccl_last_error()
    # a read through neighborhood(1) needs buffers holding the grown chunk
    assert call(ccl.CCL_FN_SAXPY, [ccl.make_accessor(nbh, R, shape, fb(own, 0x10000000)), y, z]) \
        == ccl.CCL_E_RANGE
    # the range must lie inside every accessor's buffer range
    assert call(ccl.CCL_FN_SAXPY, [ccl.make_accessor(o2o, R, (40, 20), fb(own, 0x10000000)), y, z]) \
        == ccl.CCL_E_RANGE
    # sum along a dimension: x's mapper must span the whole range there
    out = ccl.make_accessor(o2o, W, shape, fb(own, 0x30000000))
    assert call(ccl.CCL_FN_SUM_ALONG, [x, out], dim=1) == ccl.CCL_E_RANGE
    assert call(ccl.CCL_FN_SUM_ALONG, [x, out], dim=2) == ccl.CCL_E_INVALID
    sl = ccl.make_mapper(ccl.SLICE, dim=0)
    regs = [ccl.ccl_region_of(c, sl, None, shape).box() for c in chunks]
    xs = ccl.make_accessor(sl, R, shape, fb(regs, 0x10000000))
    assert call(ccl.CCL_FN_SUM_ALONG, [xs, out], dim=1) == ccl.CCL_E_RANGE  # slice(0) for dim 1


def test_wave_energy_validates_before_launch():
    """ccl_wave_energy refuses malformed arguments before touching a device
    (no GPU needed): NULL pointers, dims, dtype, empty extents, pitches
    smaller than the rows or planes they hold."""
    L = ccl.lib()
    I64 = ctypes.c_int64 * 3
    dev = ctypes.c_void_p(0x10000)  # never dereferenced: every call below is refused
    shape, pitch = I64(4, 8, 8), I64(64, 8, 0)
    assert L.ccl_wave_energy(3, shape, pitch, ccl.CCL_DTYPE_F32, 0.1, None, dev, dev,
                             None) == ccl.CCL_E_INVALID
    assert L.ccl_wave_energy(3, shape, pitch, ccl.CCL_DTYPE_F32, 0.1, dev, dev, None,
                             None) == ccl.CCL_E_INVALID
    assert L.ccl_wave_energy(4, shape, pitch, ccl.CCL_DTYPE_F32, 0.1, dev, dev, dev,
                             None) == ccl.CCL_E_INVALID
    assert L.ccl_wave_energy(3, shape, pitch, 9, 0.1, dev, dev, dev, None) == ccl.CCL_E_INVALID
    assert L.ccl_wave_energy(3, I64(4, 0, 8), pitch, ccl.CCL_DTYPE_F32, 0.1, dev, dev, dev,
                             None) == ccl.CCL_E_INVALID
    assert L.ccl_wave_energy(3, shape, I64(64, 7, 0), ccl.CCL_DTYPE_F32, 0.1, dev, dev, dev,
                             None) == ccl.CCL_E_INVALID
    assert L.ccl_wave_energy(3, shape, I64(63, 8, 0), ccl.CCL_DTYPE_F32, 0.1, dev, dev, dev,
                             None) == ccl.CCL_E_INVALID
    assert L.ccl_wave_energy(2, I64(8, 8, 0), I64(7, 0, 0), ccl.CCL_DTYPE_F64, 0.1, dev, dev,
                             dev, None) == ccl.CCL_E_INVALID


def test_autotune_candidates_enumeration():
    """The library's candidate set: K in {1, 2, 4, 8, 16} up to the extent
    along dimension 0, tile rows in {0, 16, 32, 64, 128}, T in 1..8, K
    slowest; the nchunks filter; RANGE (with the count) when the room is
    short; argument errors.  The sweep refuses an energy objective without
    an energy window before it measures anything."""
    for shape in [(512, 1024), (3, 700), (20, 40, 70), (1, 5, 5)]:
        want = [(K, rows, T) for K in (1, 2, 4, 8, 16) if K <= shape[0]
                for rows in (0, 16, 32, 64, 128) for T in range(1, 9)]
        got = ccl.ccl_autotune_candidates(shape)
        assert [(c.nchunks, c.tile_rows, c.temporal_depth) for c in got] == want
        assert all(c.dims == len(shape) and tuple(c.shape[:c.dims]) == shape for c in got)
        only4 = ccl.ccl_autotune_candidates(shape, 4)
        assert [(c.nchunks, c.tile_rows, c.temporal_depth) for c in only4] == \
            [w for w in want if w[0] == 4]
    L = ccl.lib()
    sh = (ctypes.c_int64 * 3)(64, 64, 0)
    n = ctypes.c_int32(0)
    out = (ccl.ccl_tune_config * 10)()
    assert L.ccl_autotune_candidates(2, sh, 0, 10, out, ctypes.byref(n)) == ccl.CCL_E_RANGE
    assert n.value == 5 * 5 * 8
    assert L.ccl_autotune_candidates(4, sh, 0, 10, out, ctypes.byref(n)) == ccl.CCL_E_INVALID
    assert L.ccl_autotune_candidates(2, None, 0, 10, out, ctypes.byref(n)) == ccl.CCL_E_INVALID
    assert L.ccl_autotune_candidates(2, (ctypes.c_int64 * 3)(0, 64, 0), 0, 10, out,
                                     ctypes.byref(n)) == ccl.CCL_E_INVALID
    samples = (ccl.ccl_tune_sample * 200)()
    cfgs = (ccl.ccl_tune_config * 200)()
    best = ctypes.c_int32(-1)
    assert L.ccl_autotune_sweep(2, sh, 0, 0.25, 8, 1, 0.0, ccl.CCL_OBJECTIVE_ENERGY, 0, None,
                                200, cfgs, samples, ctypes.byref(n),
                                ctypes.byref(best)) == ccl.CCL_E_INVALID
    assert L.ccl_autotune_sweep(2, sh, 0, 0.25, 8, 1, 0.0, 7, 0, None, 200, cfgs, samples,
                                ctypes.byref(n), ctypes.byref(best)) == ccl.CCL_E_INVALID
