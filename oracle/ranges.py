"""Oracle for range splitting and range mappers (test infrastructure only).

Follows section 3 of the paper: a kernel's N-D index range is split into
chunks, one per device, and each accessor's range mapper turns a chunk into
the region of the buffer the chunk needs; the regions not owned locally are
what must be transferred before the chunk runs.

Definitions (plain interval arithmetic, one dimension at a time):
  * split: along ``split_dim`` of extent n starting at offset o, chunk k of K
    covers [o + floor(k n / K), o + floor((k+1) n / K)); other dims are whole.
  * block split (split_grid): the same 1D split applied independently along
    every dimension d with counts[d] pieces; the chunks are all products of
    one piece per dimension, numbered with the last dimension fastest.
  * one_to_one: region = the chunk itself (the kernel touches only index i).
  * neighborhood(e): region = chunk grown by e_d on both sides of each dim,
    intersected with the buffer's index range [0, buffer_range_d).
  * all: region = the whole buffer.
  * fixed(box): region = the given box, whatever the chunk, intersected with
    the buffer's index range.
  * slice(d): region = the chunk with dimension d replaced by the buffer's
    whole extent [0, buffer_range_d).
  * halo = region minus chunk; transfers = for every ordered pair of chunks
    (owner, reader), region(reader) intersected with chunk(owner).

Boxes are (offset tuple, range tuple).
"""
from __future__ import annotations

ONE_TO_ONE, NEIGHBORHOOD, ALL, FIXED, SLICE = 0, 1, 2, 3, 4


def split_range(offset, rng, nchunks: int, split_dim: int = 0):
    dims = len(rng)
    if dims not in (1, 2, 3) or len(offset) != dims:
        raise ValueError("dims must be 1, 2 or 3")
    if nchunks < 1 or not (0 <= split_dim < dims):
        raise ValueError("bad nchunks or split_dim")
    n = rng[split_dim]
    if nchunks > n:
        raise ValueError("more chunks than indices along the split dimension")
    out = []
    for k in range(nchunks):
        lo = (k * n) // nchunks
        hi = ((k + 1) * n) // nchunks
        off = list(offset)
        r = list(rng)
        off[split_dim] = offset[split_dim] + lo
        r[split_dim] = hi - lo
        out.append((tuple(off), tuple(r)))
    return out


def split_grid(offset, rng, counts):
    dims = len(rng)
    if dims not in (1, 2, 3) or len(offset) != dims or len(counts) != dims:
        raise ValueError("dims must be 1, 2 or 3, with one count per dimension")
    pieces = []
    for d in range(dims):
        if counts[d] < 1 or counts[d] > rng[d]:
            raise ValueError("a count is below 1 or above the extent")
        n, K = rng[d], counts[d]
        pieces.append([(offset[d] + (k * n) // K, ((k + 1) * n) // K - (k * n) // K)
                       for k in range(K)])
    out = []
    for combo in _product(pieces):  # last dimension fastest
        out.append((tuple(o for o, _ in combo), tuple(r for _, r in combo)))
    return out


def _product(lists):
    if not lists:
        return [()]
    rest = _product(lists[1:])
    return [(x,) + r for x in lists[0] for r in rest]


def region_of(chunk, kind: int, extent, buffer_range, offset=None, dim=0):
    """`extent`: neighborhood's growth per side, or fixed's box extent;
    `offset`: fixed's box origin; `dim`: the dimension slice takes whole."""
    off, rng = chunk
    dims = len(rng)
    if kind == ONE_TO_ONE:
        return (tuple(off), tuple(rng))
    if kind == ALL:
        return (tuple([0] * dims), tuple(buffer_range))
    if kind == FIXED:
        lo, r = [], []
        for d in range(dims):
            a = min(max(0, offset[d]), buffer_range[d])
            b = max(a, min(buffer_range[d], offset[d] + extent[d]))
            lo.append(a)
            r.append(b - a)
        return (tuple(lo), tuple(r))
    if kind == SLICE:
        if not 0 <= dim < dims:
            raise ValueError("slice dimension out of range")
        lo, r = list(off), list(rng)
        lo[dim], r[dim] = 0, buffer_range[dim]
        return (tuple(lo), tuple(r))
    if kind != NEIGHBORHOOD:
        raise ValueError("unknown mapper")
    lo, r = [], []
    for d in range(dims):
        a = max(0, off[d] - extent[d])
        b = min(buffer_range[d], off[d] + rng[d] + extent[d])
        lo.append(a)
        r.append(max(0, b - a))
    return (tuple(lo), tuple(r))


def intersect(a, b):
    (ao, ar), (bo, br) = a, b
    lo, r = [], []
    for d in range(len(ar)):
        x0 = max(ao[d], bo[d])
        x1 = min(ao[d] + ar[d], bo[d] + br[d])
        if x1 <= x0:
            return None
        lo.append(x0)
        r.append(x1 - x0)
    return (tuple(lo), tuple(r))


def transfers(chunks, regions):
    """(owner k, reader j, box) for every box chunk k owns that region j needs."""
    out = []
    for j, reg in enumerate(regions):
        for k, ch in enumerate(chunks):
            if k == j:
                continue
            box = intersect(reg, ch)
            if box is not None:
                out.append((k, j, box))
    return out
