"""Pins of the remaining oracle parts (CPU only).

* ranges: exhaustive brute force for small ranges: chunks are disjoint,
  cover the range, differ in size by at most one; neighborhood(e) equals the
  bounding box of the cells a radius-e box stencil reads, clipped to the
  buffer; transfers cover exactly region minus chunk.
* SAXPY: each output equals the exact a*x+y rounded once to float32 (ties to
  even), computed with Python fractions.
* MLP: analytic gradients vs central finite differences; Adam's first step
  equals lr*g/(|g|+eps) (bias correction); with the hidden layers frozen,
  training the last layer reaches the linear least-squares optimum.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp, ranges


# ------------------------------------------------------------------ ranges --

@pytest.mark.parametrize("dims", [1, 2, 3])
def test_split_exhaustive(dims):
    for n in range(1, 25):
        for K in range(1, min(n, 16) + 1):
            for sd in range(dims):
                rng = [3] * dims
                rng[sd] = n
                off = [5] * dims
                ch = ranges.split_range(tuple(off), tuple(rng), K, sd)
                assert len(ch) == K
                cover = []
                sizes = []
                for o, r in ch:
                    for d in range(dims):
                        if d != sd:
                            assert o[d] == off[d] and r[d] == rng[d]
                    cover.extend(range(o[sd], o[sd] + r[sd]))
                    sizes.append(r[sd])
                assert sorted(cover) == list(range(off[sd], off[sd] + n))  # disjoint + cover
                assert max(sizes) - min(sizes) <= 1 and min(sizes) >= 1


def test_split_rejects():
    with pytest.raises(ValueError):
        ranges.split_range((0,), (4,), 5)
    with pytest.raises(ValueError):
        ranges.split_range((0,), (4,), 0)
    with pytest.raises(ValueError):
        ranges.split_range((0, 0), (4, 4), 2, split_dim=2)


def _bbox_of_reads(chunk, e, buf):
    off, rng = chunk
    dims = len(rng)
    pts = []
    for cell in itertools.product(*[range(off[d], off[d] + rng[d]) for d in range(dims)]):
        for delta in itertools.product(*[range(-e[d], e[d] + 1) for d in range(dims)]):
            q = tuple(cell[d] + delta[d] for d in range(dims))
            if all(0 <= q[d] < buf[d] for d in range(dims)):
                pts.append(q)
    lo = tuple(min(p[d] for p in pts) for d in range(dims))
    hi = tuple(max(p[d] for p in pts) + 1 for d in range(dims))
    return lo, tuple(h - l for h, l in zip(hi, lo))


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_region_brute_force(dims):
    rs = np.random.default_rng(7)
    for _ in range(60):
        buf = tuple(int(v) for v in rs.integers(1, 9 if dims < 3 else 6, size=dims))
        off = tuple(int(rs.integers(0, b)) for b in buf)
        rng = tuple(int(rs.integers(1, b - o + 1)) for o, b in zip(off, buf))
        e = tuple(int(v) for v in rs.integers(0, 4, size=dims))
        chunk = (off, rng)
        assert ranges.region_of(chunk, ranges.NEIGHBORHOOD, e, buf) == _bbox_of_reads(chunk, e, buf)
        assert ranges.region_of(chunk, ranges.ONE_TO_ONE, e, buf) == chunk
        assert ranges.region_of(chunk, ranges.ALL, e, buf) == ((0,) * dims, buf)


def test_transfers_cover_halo():
    buf = (20, 7)
    chunks = ranges.split_range((0, 0), buf, 5, 0)
    for e in range(0, 5):
        regs = [ranges.region_of(c, ranges.NEIGHBORHOOD, (e, e), buf) for c in chunks]
        tr = ranges.transfers(chunks, regs)
        for j, (reg, ch) in enumerate(zip(regs, chunks)):
            need = set(itertools.product(range(reg[0][0], reg[0][0] + reg[1][0]),
                                         range(reg[0][1], reg[0][1] + reg[1][1])))
            own = set(itertools.product(range(ch[0][0], ch[0][0] + ch[1][0]),
                                        range(ch[0][1], ch[0][1] + ch[1][1])))
            got = []
            for k, jj, (o, r) in tr:
                if jj == j:
                    got.extend(itertools.product(range(o[0], o[0] + r[0]), range(o[1], o[1] + r[1])))
            assert sorted(got) == sorted(need - own)  # exact, no duplicates


# ------------------------------------------------------------------- saxpy --

def _round_f32(q: Fraction) -> np.float32:
    c = np.float32(float(q))
    cands = [np.nextafter(c, np.float32(-np.inf)), c, np.nextafter(c, np.float32(np.inf))]
    best = None
    for v in cands:
        d = abs(Fraction(float(v)) - q)
        key = (d, int(np.frombuffer(np.float32(v).tobytes(), np.uint32)[0]) & 1)
        if best is None or key < best[0]:
            best = (key, v)
    return np.float32(best[1])


def test_saxpy_exact_rounding(oracle_lib):
    rs = np.random.default_rng(3)
    x = rs.standard_normal(2000).astype(np.float32)
    y = rs.standard_normal(2000).astype(np.float32)
    y[:10] = -2.5 * x[:10]  # exact cancellation cases
    a = np.float32(2.5)
    z = oracle.saxpy(a, x, y)
    for i in range(x.size):
        q = Fraction(float(a)) * Fraction(float(x[i])) + Fraction(float(y[i]))
        assert z[i] == _round_f32(q), i


# --------------------------------------------------------------------- MLP --

SIZES = (12, 64, 64, 2)


def test_mlp_gradcheck():
    ws, bs = synth.mlp_params(SIZES, seed=1)
    x, t = synth.mlp_batch(16, 12, 2, seed=2)
    acts = mlp.forward(ws, bs, x)
    dws, dbs = mlp.backward(ws, bs, acts, t)
    h = 1e-6
    rs = np.random.default_rng(0)
    for li in range(3):
        for arr, grad in ((ws[li], dws[li]), (bs[li], dbs[li])):
            flat = arr.reshape(-1)
            gflat = grad.reshape(-1)
            for idx in rs.choice(flat.size, size=min(12, flat.size), replace=False):
                old = flat[idx]
                flat[idx] = old + h
                lp = mlp.loss(mlp.forward(ws, bs, x)[-1], t)
                flat[idx] = old - h
                lm = mlp.loss(mlp.forward(ws, bs, x)[-1], t)
                flat[idx] = old
                fd = (lp - lm) / (2 * h)
                assert abs(fd - gflat[idx]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9


def test_mlp_weighted_gradcheck():
    """Weighted loss: finite differences again, with a mask on output 2."""
    ws, bs = synth.mlp_params(SIZES, seed=12)
    x, t = synth.mlp_batch(10, 12, 2, seed=13)
    w = np.ones((10, 2))
    w[::2, 1] = 0.0
    w[3, 0] = 0.25
    acts = mlp.forward(ws, bs, x)
    dws, _ = mlp.backward(ws, bs, acts, t, w)
    h = 1e-6
    for li in range(3):
        flat = ws[li].reshape(-1)
        for idx in (0, flat.size // 2, flat.size - 1):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(mlp.forward(ws, bs, x)[-1], t, w)
            flat[idx] = old - h
            lm = mlp.loss(mlp.forward(ws, bs, x)[-1], t, w)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - dws[li].reshape(-1)[idx]) <= 1e-7 * max(1.0, abs(fd)) + 1e-9


def test_mlp_forward_linear_region():
    """With every pre-activation positive, the net is the affine map
    W3 W2 W1 x + (W3 W2 b1 + W3 b2 + b3)."""
    rs = np.random.default_rng(4)
    ws = [np.abs(rs.standard_normal((o, i))) for i, o in zip(SIZES[:-1], SIZES[1:])]
    bs = [np.abs(rs.standard_normal(o)) for o in SIZES[1:]]
    x = np.abs(rs.standard_normal((5, 12)))
    y = mlp.forward(ws, bs, x)[-1]
    A = ws[2] @ ws[1] @ ws[0]
    c = ws[2] @ (ws[1] @ bs[0] + bs[1]) + bs[2]
    assert np.allclose(y, x @ A.T + c, rtol=1e-12)


def test_adam_first_step():
    p = [np.array([1.0, -2.0, 3.0])]
    g = [np.array([0.5, -1e-3, 0.0])]
    m = [np.zeros(3)]
    v = [np.zeros(3)]
    mlp.adam_step(p, g, m, v, t=1, lr=1e-2)
    expect = np.array([1.0, -2.0, 3.0]) - 1e-2 * g[0] / (np.abs(g[0]) + 1e-8)
    assert np.allclose(p[0], expect, rtol=0, atol=1e-15)


def test_last_layer_reaches_least_squares():
    ws, bs = synth.mlp_params(SIZES, seed=5)
    x, t = synth.mlp_batch(512, 12, 2, seed=6)  # overdetermined: 512 rows, 65 unknowns
    acts = mlp.forward(ws, bs, x)
    H = np.hstack([acts[2], np.ones((512, 1))])
    sol, *_ = np.linalg.lstsq(H, t, rcond=None)
    best = mlp.loss(H @ sol, t)
    params = [ws[2], bs[2]]
    m = [np.zeros_like(q) for q in params]
    v = [np.zeros_like(q) for q in params]
    for step in range(1, 5001):
        a = mlp.forward(ws, bs, x)
        dws, dbs = mlp.backward(ws, bs, a, t)
        lr = 1e-2 if step < 3000 else (1e-3 if step < 4000 else 1e-4)
        mlp.adam_step(params, [dws[2], dbs[2]], m, v, step, lr=lr)
    final = mlp.loss(mlp.forward(ws, bs, x)[-1], t)
    assert best * (1 - 1e-12) <= final <= best * (1 + 1e-8)


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_split_grid_exhaustive(dims):
    """Block split: every cell of the range in exactly one chunk, chunks are
    boxes whose extents along each dimension differ by at most one, chunk
    count = product of the counts, and each dimension's pieces are the 1D
    split along it (a block split with one count above 1 is split_range)."""
    sizes = (1, 2, 5, 7) if dims < 3 else (1, 3, 5)
    for rng in itertools.product(sizes, repeat=dims):
        off = tuple(2 - d for d in range(dims))
        for counts in itertools.product(*[range(1, min(n, 4) + 1) for n in rng]):
            ch = ranges.split_grid(off, rng, counts)
            assert len(ch) == int(np.prod(counts))
            cells = []
            for o, r in ch:
                cells.extend(itertools.product(*[range(o[d], o[d] + r[d]) for d in range(dims)]))
            want = list(itertools.product(*[range(off[d], off[d] + rng[d]) for d in range(dims)]))
            assert sorted(cells) == sorted(want)
            for d in range(dims):
                ext = [r[d] for _, r in ch]
                assert max(ext) - min(ext) <= 1
                pieces = sorted({(o[d], r[d]) for o, r in ch})
                one_d = ranges.split_range((off[d],), (rng[d],), counts[d], 0)
                assert pieces == sorted((o[0], r[0]) for o, r in one_d)
            # numbering: last dimension fastest
            assert ch == sorted(ch, key=lambda c: c[0])
            nz = [i for i, c in enumerate(counts) if c > 1]
            if len(nz) == 1:
                assert ch == ranges.split_range(off, rng, counts[nz[0]], nz[0])


def test_split_grid_rejects():
    with pytest.raises(ValueError):
        ranges.split_grid((0, 0), (4, 4), (5, 1))
    with pytest.raises(ValueError):
        ranges.split_grid((0, 0), (4, 4), (0, 1))
    with pytest.raises(ValueError):
        ranges.split_grid((0, 0), (4, 4), (2,))


def _bbox(pts, dims):
    if not pts:
        return None
    lo = tuple(min(p[d] for p in pts) for d in range(dims))
    hi = tuple(max(p[d] for p in pts) + 1 for d in range(dims))
    return lo, tuple(h - l for h, l in zip(hi, lo))


@pytest.mark.parametrize("dims", [1, 2, 3])
def test_fixed_and_slice_brute_force(dims):
    """fixed(box): the cells of a kernel that reads every cell of the box,
    whatever its own index, kept if inside the buffer; slice(d): the cells a
    kernel reads when index i touches every cell that agrees with i outside
    dimension d (a reduction along d).  Each region is the bounding box of
    those reads."""
    rs = np.random.default_rng(8)
    for _ in range(60):
        buf = tuple(int(v) for v in rs.integers(1, 7 if dims < 3 else 5, size=dims))
        off = tuple(int(rs.integers(0, b)) for b in buf)
        rng = tuple(int(rs.integers(1, b - o + 1)) for o, b in zip(off, buf))
        chunk = (off, rng)
        cells = list(itertools.product(*[range(off[d], off[d] + rng[d]) for d in range(dims)]))
        # fixed: a box that may stick out of the buffer on either side
        fo = tuple(int(rs.integers(-2, b + 1)) for b in buf)
        fe = tuple(int(rs.integers(1, 5)) for _ in buf)
        reads = [q for q in itertools.product(*[range(fo[d], fo[d] + fe[d]) for d in range(dims)])
                 if all(0 <= q[d] < buf[d] for d in range(dims))]
        want = _bbox(reads, dims)
        got = ranges.region_of(chunk, ranges.FIXED, fe, buf, offset=fo)
        if want is None:
            assert 0 in got[1]
        else:
            assert got == want
        for d in range(dims):
            reads = []
            for c in cells:
                for v in range(buf[d]):
                    q = list(c)
                    q[d] = v
                    reads.append(tuple(q))
            assert ranges.region_of(chunk, ranges.SLICE, (0,) * dims, buf, dim=d) == \
                _bbox(reads, dims)


# --------------------------------------------------------------- sum along --

@pytest.mark.parametrize("shape,dim", [((7,), 0), ((5, 9), 0), ((5, 9), 1), ((4, 3, 6), 2),
                                       ((4, 3, 6), 0)])
def test_sum_along_exact_on_integers(shape, dim):
    """Small integers (every partial sum exact in float32): the sum equals
    the exact integer sum, broadcast along the summed dimension."""
    rs = np.random.default_rng(3)
    k = rs.integers(-1000, 1000, size=shape)
    got = oracle.sum_along(k.astype(np.float32), dim)
    want = np.broadcast_to(k.sum(axis=dim, keepdims=True), shape)
    assert np.array_equal(got, want.astype(np.float32))


def test_sum_along_error_bound_and_order():
    """Random reals: within the recursive-summation bound (n-1) u sum|x| of
    the exact sum; and the order is index order: a sum whose float32 result
    depends on the order matches the left-to-right one."""
    rs = np.random.default_rng(4)
    x = rs.uniform(-1, 1, size=(6, 300)).astype(np.float32)
    got = oracle.sum_along(x, 1)[:, 0].astype(np.float64)
    exact = np.array([float(sum(Fraction(float(v)) for v in row)) for row in x])
    bound = 299 * 2.0 ** -24 * np.abs(x.astype(np.float64)).sum(axis=1)
    assert np.all(np.abs(got - exact) <= bound)
    big = np.array([[2.0 ** 24, 1.0, 1.0, -2.0 ** 24]], dtype=np.float32)
    # left to right: 2^24 + 1 -> 2^24 (ties to even), + 1 -> 2^24, - 2^24 -> 0
    assert oracle.sum_along(big, 1)[0, 0] == 0.0
    # right to left: -2^24 + 1 and + 1 are exact, + 2^24 -> 2
    assert oracle.sum_along(big[:, ::-1].copy(), 1)[0, 0] == 2.0
    assert oracle.sum_along(np.array([[1.0, 2.0 ** 24, -2.0 ** 24, 1.0]], np.float32), 1)[0, 0] == 1.0
