"""GPU parity of the generic chunked parallel_for (ccl_parallel_for).

* The paper's second listing: SAXPY over a range split into chunks, with
  one_to_one accessors x, y (read) and z (write), in 1D, 2D and 3D, block
  splits included, every chunk in its own buffers: bitwise equal to the
  float32 oracle.  Also with buffers larger than the chunks and chunk starts
  off the 16-byte grid (the element-by-element path).
* A reduction along one dimension read through a slice mapper: each chunk's
  buffer holds the whole extent along that dimension, filled by the inferred
  transfers from the other chunks before the launch: bitwise equal to the
  oracle's float32 sum in index order.
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


def chunk_buffers(chunks, regions, fill=float("nan"), data=None):
    """One buffer per chunk holding `regions[k]`; the chunk's own cells take
    `data` (the global array) when given."""
    import paper_2505_06022_amd as ccl
    from paper_2505_06022_amd.fields import alloc_buffer, view_of
    bufs = (ccl.ccl_chunk_buffer * len(chunks))()
    ts = []
    for k, reg in enumerate(regions):
        t, b = alloc_buffer(reg, fill=fill)
        bufs[k] = b
        ts.append((t, reg))
        if data is not None:
            box = chunks[k].box()
            sl = tuple(slice(o, o + n) for o, n in zip(*box))
            view_of(t, reg, box).copy_(torch.from_numpy(np.ascontiguousarray(data[sl])))
    return bufs, ts


def gather(chunks, ts, shape):
    from paper_2505_06022_amd.fields import view_of
    out = np.full(shape, np.nan, dtype=np.float32)
    for k, (t, reg) in enumerate(ts):
        box = chunks[k].box()
        sl = tuple(slice(o, o + n) for o, n in zip(*box))
        out[sl] = view_of(t, reg, box).cpu().numpy()
    return out


@pytest.mark.parametrize("shape,split", [((1 << 20) + 3, 4), ((1000,), 3), ((257, 129), (2, 2)),
                                         ((64, 300), (4, 3)), ((9, 31, 70), (2, 2, 2)),
                                         ((5, 6, 7), 5)])
def test_saxpy_one_to_one(shape, split):
    import paper_2505_06022_amd as ccl
    shape = shape if isinstance(shape, tuple) else (shape,)
    dims = len(shape)
    if isinstance(split, tuple):
        chunks = ccl.ccl_split_grid((0,) * dims, shape, split)
    else:
        chunks = ccl.ccl_split_range((0,) * dims, shape, split)
    x = synth.uniform_field(shape, 50).astype(np.float32)
    y = synth.uniform_field(shape, 51).astype(np.float32)
    regs = [c.box() for c in chunks]  # one_to_one: each buffer holds its chunk
    # the tensors behind every buffer stay referenced until the results are
    # read: a dropped one returns its memory to torch's cache, where the
    # next allocation reuses it
    bx, tx = chunk_buffers(chunks, regs, data=x)
    by, ty = chunk_buffers(chunks, regs, data=y)
    bz, tz = chunk_buffers(chunks, regs)
    o2o = ccl.make_mapper(ccl.ONE_TO_ONE)
    acc = [ccl.make_accessor(o2o, ccl.CCL_ACCESS_READ, shape, bx),
           ccl.make_accessor(o2o, ccl.CCL_ACCESS_READ, shape, by),
           ccl.make_accessor(o2o, ccl.CCL_ACCESS_WRITE, shape, bz)]
    ccl.ccl_parallel_for(ccl.CCL_FN_SAXPY, chunks, acc, a=1.75)
    torch.cuda.synchronize()
    got = gather(chunks, tz, shape)
    assert np.array_equal(got, oracle.saxpy(1.75, x, y))
    del tx, ty


def test_saxpy_unaligned_chunk_starts():
    """Whole-range buffers for every chunk: chunk starts at 333 and 666 are
    off the 16-byte grid, so those chunks take the element-by-element path."""
    import paper_2505_06022_amd as ccl
    shape = (999,)
    chunks = ccl.ccl_split_range((0,), shape, 3)
    x = synth.uniform_field(shape, 52).astype(np.float32)
    y = synth.uniform_field(shape, 53).astype(np.float32)
    whole = [((0,), shape)] * 3
    bx, tx = chunk_buffers(chunks, whole, data=x)
    by, ty = chunk_buffers(chunks, whole, data=y)
    bz, tz = chunk_buffers(chunks, whole)
    o2o = ccl.make_mapper(ccl.ONE_TO_ONE)
    acc = [ccl.make_accessor(o2o, ccl.CCL_ACCESS_READ, shape, bx),
           ccl.make_accessor(o2o, ccl.CCL_ACCESS_READ, shape, by),
           ccl.make_accessor(o2o, ccl.CCL_ACCESS_WRITE, shape, bz)]
    ccl.ccl_parallel_for(ccl.CCL_FN_SAXPY, chunks, acc, a=-0.5)
    torch.cuda.synchronize()
    assert np.array_equal(gather(chunks, tz, shape), oracle.saxpy(-0.5, x, y))
    del tx, ty


@pytest.mark.parametrize("shape,grid,dim", [((37, 50), (2, 3), 1), ((37, 50), (3, 2), 0),
                                            ((64, 257), (4, 2), 1), ((9, 20, 33), (2, 2, 2), 2),
                                            ((9, 20, 33), (1, 3, 2), 1)])
def test_sum_along_slice_mapper(shape, grid, dim):
    """x read through slice(dim): each chunk's x buffer is sized to its
    slice region and holds only its own cells on entry; the inferred
    transfers fill the rest from the other chunks before the launch."""
    import paper_2505_06022_amd as ccl
    dims = len(shape)
    chunks = ccl.ccl_split_grid((0,) * dims, shape, grid)
    x = synth.uniform_field(shape, 54).astype(np.float32)
    sl_map = ccl.make_mapper(ccl.SLICE, dim=dim)
    regs = [ccl.ccl_region_of(c, sl_map, None, shape).box() for c in chunks]
    bx, tx = chunk_buffers(chunks, regs, data=x)
    bo, to = chunk_buffers(chunks, [c.box() for c in chunks])
    acc = [ccl.make_accessor(sl_map, ccl.CCL_ACCESS_READ, shape, bx),
           ccl.make_accessor(ccl.make_mapper(ccl.ONE_TO_ONE), ccl.CCL_ACCESS_WRITE, shape, bo)]
    ccl.ccl_parallel_for(ccl.CCL_FN_SUM_ALONG, chunks, acc, dim=dim)
    torch.cuda.synchronize()
    assert np.array_equal(gather(chunks, to, shape), oracle.sum_along(x, dim))
    del tx
