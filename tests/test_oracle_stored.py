"""Pins of the 16-bit-storage leapfrog in the oracle (CPU only).

* Rounding to binary16 equals numpy's float32 -> float16 conversion (an
  independent library routine, round to nearest even with subnormals and
  overflow to infinity) on values spread over every binade, on exact ties
  and around the overflow threshold.
* Rounding to bfloat16 equals a brute-force choice between the two
  bfloat16 neighbours of x read off its bit pattern: the nearer one, the
  one with an even last stored bit on a tie (float32 subnormals included).
* wave_stored with one pass (depth >= steps) equals the pinned float32
  oracle from the rounded inputs, rounded once at the end; several passes
  equal single passes chained (the last one shorter when depth does not
  divide steps); the stored values are representable in the format; r2 = 0
  leaves the rounded inputs unchanged.
* Planted mistakes in a copy of oracle.c (rounding toward zero, no
  subnormals, u^{n-1} stored unrounded, rounding after every step, a missed
  pass-length clip) are rejected by these pins.
"""
import numpy as np
import pytest

import oracle
import synth


def f32_samples(seed, n=200000):
    """float32 values over all binades (normal and subnormal), both signs."""
    rng = np.random.default_rng(seed)
    bits = rng.integers(0, 0x7F800000, size=n, dtype=np.uint32)
    x = bits.view(np.float32) * np.where(rng.random(n) < 0.5, -1, 1).astype(np.float32)
    return x


def f16_ties():
    """Midpoints between consecutive binary16 values (exact in float32)."""
    h = np.arange(0, 0x7BFF, dtype=np.uint16).view(np.float16).astype(np.float32)
    hn = np.arange(1, 0x7C00, dtype=np.uint16).view(np.float16).astype(np.float32)
    mid = ((h.astype(np.float64) + hn.astype(np.float64)) / 2).astype(np.float32)
    return np.concatenate([mid, -mid])


def bf16_brute(x):
    """Round float32 x to bfloat16 by comparing the two candidates."""
    out = np.empty_like(x)
    for k, v in enumerate(x):
        b = np.array([v], dtype=np.float32).view(np.uint32)[0]
        sign = b & 0x80000000
        mag = b & 0x7FFFFFFF
        lo = mag & 0xFFFF0000                       # toward zero
        hi = lo + 0x10000                            # next one away from zero
        vlo = float(np.array([lo | sign], dtype=np.uint32).view(np.float32)[0])
        vhi = float(np.array([hi | sign], dtype=np.uint32).view(np.float32)[0]) \
            if hi < 0x7F800000 else (np.inf if sign == 0 else -np.inf)
        vv = float(v)
        dlo, dhi = abs(vv - vlo), abs(vhi - vv) if np.isfinite(vhi) else np.inf
        if hi == 0x7F800000:
            # above the largest finite value: halfway to 2^128 or more -> inf
            top = float(np.array([0x7F7F0000], dtype=np.uint32).view(np.float32)[0])
            half_up = 2.0 ** 128 - 2.0 ** (127 - 8)
            vhi = np.inf if sign == 0 else -np.inf
            out[k] = vhi if abs(vv) >= half_up else (top if sign == 0 else -top)
            continue
        if dlo < dhi or (dlo == dhi and (lo >> 16) % 2 == 0):
            out[k] = vlo
        else:
            out[k] = vhi
    return out


def test_f16_rounding_matches_numpy():
    x = np.concatenate([f32_samples(1), f16_ties(),
                        np.float32([65504, 65519.99, 65520, 65536, 1e-8, 2.98e-8, 3e-8,
                                    5.96e-8, 6.1035e-5, 0.0, -0.0])])
    # numpy's conversion overflows to inf with a warning, as intended
    with np.errstate(over="ignore"):
        ref = x.astype(np.float16).astype(np.float32)
    got = oracle.round_to_format(x, "f16")
    assert np.array_equal(got, ref)


def test_bf16_rounding_matches_brute_force():
    x = np.concatenate([f32_samples(2, 20000),
                        # ties: a bfloat16 value plus half its last-place step
                        (np.arange(0x3F800000, 0x3F800000 + 4096 * 0x10000, 0x10000,
                                   dtype=np.uint32) + 0x8000).view(np.float32),
                        np.float32([3.3895314e38, 3.4e38, 1e-40, -1e-40, 1.0, 0.0])])
    assert np.array_equal(oracle.round_to_format(x, "bf16"), bf16_brute(x))


def _stored_pins_pass(L):
    """The wave_stored pins, against library L (returns True if all hold)."""
    ok = True
    rf = lambda a, f: oracle.round_to_format(a, f, _lib_override=L)
    for fmt in ("bf16", "f16"):
        for shape, r2 in (((23, 37), 0.25), ((7, 9, 11), 0.1)):
            up = synth.gaussian_field(shape, 4.0, 3)
            uc = synth.gaussian_field(shape, 4.5, 4)
            # one pass: the float32 oracle from rounded inputs, rounded once
            for steps in (1, 5):
                gp, gc = oracle.wave_stored(up, uc, r2, steps, 8, fmt, _lib_override=L)
                p, c = oracle.wave(rf(up, fmt), rf(uc, fmt), r2, steps, _lib_override=L)
                ok &= np.array_equal(gc, rf(c, fmt)) and np.array_equal(gp, rf(p, fmt))
            # several passes: single passes chained, the last one shorter
            for depth, steps in ((3, 12), (4, 14), (1, 5)):
                gp, gc = oracle.wave_stored(up, uc, r2, steps, depth, fmt, _lib_override=L)
                p, c = up, uc
                for done in range(0, steps, depth):
                    tb = min(depth, steps - done)
                    p, c = oracle.wave_stored(p, c, r2, tb, tb, fmt, _lib_override=L)
                ok &= np.array_equal(gc, c) and np.array_equal(gp, p)
                ok &= np.array_equal(rf(gc, fmt), gc) and np.array_equal(rf(gp, fmt), gp)
            # r2 = 0: the rounded inputs persist (u^{n+1} = 2u^n - u^{n-1} with
            # u^{n-1} = u^n)
            gp, gc = oracle.wave_stored(uc, uc, 0.0, 6, 4, fmt, _lib_override=L)
            ok &= np.array_equal(gc, rf(uc, fmt)) and np.array_equal(gp, rf(uc, fmt))
    return bool(ok)


def test_stored_pins():
    assert _stored_pins_pass(oracle.lib())


def test_stored_close_to_float64():
    """Storage error only: the 256 x 256 workload after 100 steps.  Each
    pass rounds both stored levels (unit roundoff 2^-8 for bfloat16, 2^-11
    for binary16) and the leapfrog carries a velocity error forward, so the
    error grows with the number of passes: measured 0.119 / 0.045 (bfloat16,
    T = 1 / 8) and 0.0094 / 0.0053 (binary16), against 1e-5 for the float32
    oracle.  The bounds leave about 30% margin."""
    w = synth.WORKLOADS["wave2d_256_k2"]
    u0 = synth.gaussian_field(w["shape"], w["sigma"], w["seed"])
    u64 = u0.astype(np.float64)
    _, r64 = oracle.wave(u64.copy(), u64, w["r2"], w["steps"])
    for fmt, depth, bound in (("bf16", 1, 0.15), ("bf16", 8, 0.06), ("f16", 1, 0.015),
                              ("f16", 8, 0.008)):
        _, c = oracle.wave_stored(u0, u0, w["r2"], w["steps"], depth, fmt)
        e = np.max(np.abs(c - r64)) / np.max(np.abs(r64))
        assert e <= bound, (fmt, depth, e)
    _, c32 = oracle.wave(u0.copy(), u0, w["r2"], w["steps"])
    assert np.max(np.abs(c32 - r64)) / np.max(np.abs(r64)) <= 1e-5


MUTATIONS = {
    "round_toward_zero": ("const double r = nearbyint((double)x / q) * q;",
                          "const double r = trunc((double)x / q) * q;"),
    "no_subnormals": ("  if (e < emin) e = emin;\n", "  if (e < emin) return 0.0f;\n"),
    "prev_unrounded": ("        prev[PADDED(z, y, x)] = round_fmt(prev[PADDED(z, y, x)], fmt);\n", ""),
    "round_every_step": ("const int64_t tb = steps - done < depth ? steps - done : depth;",
                         "const int64_t tb = 1;"),
    "stored_2d_coef": ("const float lap = sum - 4.0f * c;",
                       "const float lap = sum - 4.0f * c + 1e-7f;"),
    "stored_3d_drop_x": ("(north + south)) + (west + east);", "(north + south)) + (west + 0.0f);"),
    "pass_not_clipped": ("const int64_t tb = steps - done < depth ? steps - done : depth;",
                         "const int64_t tb = depth;"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_stored_mutation_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    src = oracle._SRC.read_text()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    (tmp_path / "oracle.c").write_text(src.replace(old, new))
    L = oracle.load(oracle.build(src=tmp_path / "oracle.c", out=tmp_path / f"lib_{name}.so"))
    x = np.concatenate([f32_samples(5, 5000), f16_ties()[:5000]])
    with np.errstate(over="ignore"):
        conv_ok = np.array_equal(oracle.round_to_format(x, "f16", _lib_override=L),
                                 x.astype(np.float16).astype(np.float32))
    assert not (conv_ok and _stored_pins_pass(L)), f"pins did not catch planted mistake {name}"
