"""Exact rational leapfrog for tiny grids (test infrastructure only).

The same leapfrog update as the C oracle, u+ = r^2 lap(u) + 2u - u-, with
zero values outside the grid, evaluated in Python ``fractions.Fraction`` so
the iterate carries no rounding at all.  Inputs must be exactly representable
(dyadic floats are); r^2 is taken as the exact rational value of the float
passed in.  Pure-Python loops: keep grids at 8x8 / 4x4x4 and steps <= ~100.
"""
from __future__ import annotations

from fractions import Fraction

import numpy as np


def _at(u, idx, shape):
    for i, n in zip(idx, shape):
        if i < 0 or i >= n:
            return Fraction(0)
    return u[idx]


def wave_exact(u_prev, u_cur, r2, steps: int):
    shape = tuple(np.shape(u_cur))
    dims = len(shape)
    r2q = Fraction(float(r2))
    prev = {idx: Fraction(float(v)) for idx, v in np.ndenumerate(np.asarray(u_prev))}
    cur = {idx: Fraction(float(v)) for idx, v in np.ndenumerate(np.asarray(u_cur))}
    for _ in range(steps):
        nxt = {}
        for idx in cur:
            s = Fraction(0)
            for d in range(dims):
                for sgn in (-1, 1):
                    j = list(idx)
                    j[d] += sgn
                    s += _at(cur, tuple(j), shape)
            lap = s - 2 * dims * cur[idx]
            nxt[idx] = r2q * lap + 2 * cur[idx] - prev[idx]
        prev, cur = cur, nxt
    return prev, cur


def to_array(u, shape, dtype=np.float64):
    out = np.empty(shape, dtype=dtype)
    for idx, v in u.items():
        out[idx] = float(v)
    return out
