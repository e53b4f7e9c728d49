"""CPU oracle: plain, slow, obviously correct reference implementations.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no
code with the HIP library and never imports it.

Contents
  * ``oracle.c`` (built to ``liboracle.so`` with gcc, no HIP headers): the
    float32 and float64 leapfrog wave steppers in 1D/2D/3D, the discrete
    leapfrog energy, the SAXPY of the paper's first listing (section 2), and
    the leapfrog with bfloat16 / binary16 storage between passes of float32
    steps (with the round-to-nearest-even conversion it stores through).
  * ``ranges``: the split of a kernel's index range into chunks (along one
    dimension, or a block split along several) and the range mappers
    one_to_one / neighborhood / all / fixed / slice (section 3, second
    listing and the paragraph after it), as interval arithmetic.
  * ``sum_along``: the float32 reduction along one dimension that a kernel
    reading through a slice mapper computes.
  * ``exact``: the leapfrog iterated in exact rational arithmetic (tiny grids).
  * ``mlp``: the 12-64-64-2 cost-model MLP in float64: forward, analytic
    backward, mean-squared-error loss and Adam.

Pins (what ties each function to something other than itself) are listed in
the test files that exercise them; functions without one say so there.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from pathlib import Path

import numpy as np

_HERE = Path(__file__).resolve().parent
_SRC = _HERE / "oracle.c"
_LIB_PATH = _HERE / "liboracle.so"

CFLAGS = ["-O3", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
          "-fno-fast-math", "-mavx2", "-mfma"]


def build(verbose: bool = False, src=None, out=None) -> Path:
    """Compile oracle.c with gcc into liboracle.so (always recompiles)."""
    src = Path(src) if src else _SRC
    out = Path(out) if out else _LIB_PATH
    tmp = out.with_suffix(f".so.{os.getpid()}.tmp")  # concurrent builds do not clash
    cmd = ["gcc", *CFLAGS, str(src), "-o", str(tmp), "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


_lib = None

_f32p = ctypes.POINTER(ctypes.c_float)
_f64p = ctypes.POINTER(ctypes.c_double)
_i64 = ctypes.c_int64


def load(path) -> ctypes.CDLL:
    """Load a build of oracle.c from ``path`` and declare its signatures."""
    L = ctypes.CDLL(str(path))
    L.oracle_wave2d_f32.argtypes = [_i64, _i64, ctypes.c_float, _i64, _f32p, _f32p,
                                    _f32p, _f32p, ctypes.c_int]
    L.oracle_wave2d_f64.argtypes = [_i64, _i64, ctypes.c_double, _i64, _f64p, _f64p,
                                    _f64p, _f64p, ctypes.c_int]
    L.oracle_wave3d_f32.argtypes = [_i64, _i64, _i64, ctypes.c_float, _i64, _f32p,
                                    _f32p, _f32p, _f32p, ctypes.c_int]
    L.oracle_wave3d_f64.argtypes = [_i64, _i64, _i64, ctypes.c_double, _i64, _f64p,
                                    _f64p, _f64p, _f64p, ctypes.c_int]
    L.oracle_wave1d_f64.argtypes = [_i64, ctypes.c_double, _i64, _f64p, _f64p, _f64p,
                                    _f64p]
    for name in ("oracle_wave2d_f32", "oracle_wave2d_f64", "oracle_wave3d_f32",
                 "oracle_wave3d_f64", "oracle_wave1d_f64", "oracle_saxpy_f32",
                 "oracle_max_threads"):
        getattr(L, name).restype = ctypes.c_int
    L.oracle_energy1d.argtypes = [_f64p, _f64p, _i64, ctypes.c_double]
    L.oracle_energy2d.argtypes = [_f64p, _f64p, _i64, _i64, ctypes.c_double]
    L.oracle_energy3d.argtypes = [_f64p, _f64p, _i64, _i64, _i64, ctypes.c_double]
    for name in ("oracle_energy1d", "oracle_energy2d", "oracle_energy3d"):
        getattr(L, name).restype = ctypes.c_double
    L.oracle_saxpy_f32.argtypes = [_i64, ctypes.c_float, _f32p, _f32p, _f32p]
    L.oracle_round_to_format.argtypes = [_i64, _f32p, _f32p, ctypes.c_int]
    L.oracle_round_to_format.restype = ctypes.c_int
    L.oracle_wave_stored.argtypes = [_i64, _i64, _i64, ctypes.c_float, _i64, _i64, ctypes.c_int,
                                     _f32p, _f32p, _f32p, _f32p, ctypes.c_int]
    L.oracle_wave_stored.restype = ctypes.c_int
    return L


def lib():
    global _lib
    if _lib is None:
        if not _LIB_PATH.exists():
            build()
        _lib = load(_LIB_PATH)
    return _lib


def _ptr(a, ty):
    return a.ctypes.data_as(ty)


def max_threads() -> int:
    return int(lib().oracle_max_threads())


def wave(u_prev, u_cur, r2: float, steps: int, threads: int = 1, _lib_override=None):
    """Advance (u^{-1}, u^0) by ``steps`` leapfrog steps on a Dirichlet-0 grid.

    The precision is that of the inputs (float32 or float64; both must match).
    Returns (u^{steps-1}, u^{steps}) as new arrays of the input shape.
    """
    u_prev = np.ascontiguousarray(u_prev)
    u_cur = np.ascontiguousarray(u_cur)
    if u_prev.shape != u_cur.shape or u_prev.dtype != u_cur.dtype:
        raise ValueError("u_prev and u_cur must match in shape and dtype")
    dt = u_cur.dtype
    if dt not in (np.float32, np.float64):
        raise TypeError(f"unsupported dtype {dt}")
    f32 = dt == np.float32
    P = _f32p if f32 else _f64p
    out_prev = np.empty_like(u_cur)
    out_cur = np.empty_like(u_cur)
    L = _lib_override or lib()
    shp = u_cur.shape
    if len(shp) == 1:
        if f32:
            raise TypeError("1D oracle is float64 only")
        rc = L.oracle_wave1d_f64(shp[0], float(r2), int(steps), _ptr(u_prev, P),
                                 _ptr(u_cur, P), _ptr(out_prev, P), _ptr(out_cur, P))
    elif len(shp) == 2:
        fn = L.oracle_wave2d_f32 if f32 else L.oracle_wave2d_f64
        r = np.float32(r2) if f32 else float(r2)
        rc = fn(shp[0], shp[1], float(r), int(steps), _ptr(u_prev, P), _ptr(u_cur, P),
                _ptr(out_prev, P), _ptr(out_cur, P), int(threads))
    elif len(shp) == 3:
        fn = L.oracle_wave3d_f32 if f32 else L.oracle_wave3d_f64
        r = np.float32(r2) if f32 else float(r2)
        rc = fn(shp[0], shp[1], shp[2], float(r), int(steps), _ptr(u_prev, P),
                _ptr(u_cur, P), _ptr(out_prev, P), _ptr(out_cur, P), int(threads))
    else:
        raise ValueError(f"unsupported rank {len(shp)}")
    if rc != 0:
        raise RuntimeError(f"oracle wave failed with status {rc}")
    return out_prev, out_cur


FORMATS = {"bf16": 1, "f16": 2}


def round_to_format(x, fmt: str, _lib_override=None):
    """``x`` (float32) rounded to nearest, ties to even, to bfloat16 ("bf16")
    or IEEE binary16 ("f16"), returned as float32 holding the exact values."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    out = np.empty_like(x)
    L = _lib_override or lib()
    rc = L.oracle_round_to_format(x.size, _ptr(x, _f32p), _ptr(out, _f32p), FORMATS[fmt])
    if rc != 0:
        raise RuntimeError(f"oracle rounding failed with status {rc}")
    return out


def wave_stored(u_prev, u_cur, r2: float, steps: int, depth: int, fmt: str, threads: int = 1,
                _lib_override=None):
    """The leapfrog with the fields stored in ``fmt`` ("bf16" or "f16") and
    float32 arithmetic: inputs rounded to the format, then passes of
    min(depth, steps left) float32 steps, each storing its last two levels
    rounded to the format.  2D or 3D float32 inputs; returns (u^{steps-1},
    u^{steps}) as float32 arrays of exactly representable values."""
    u_prev = np.ascontiguousarray(u_prev, dtype=np.float32)
    u_cur = np.ascontiguousarray(u_cur, dtype=np.float32)
    if u_prev.shape != u_cur.shape or u_cur.ndim not in (2, 3):
        raise ValueError("2D or 3D inputs of one shape")
    shp = (0,) + u_cur.shape if u_cur.ndim == 2 else u_cur.shape
    out_prev = np.empty_like(u_cur)
    out_cur = np.empty_like(u_cur)
    L = _lib_override or lib()
    rc = L.oracle_wave_stored(shp[0], shp[1], shp[2], float(np.float32(r2)), int(steps),
                              int(depth), FORMATS[fmt], _ptr(u_prev, _f32p), _ptr(u_cur, _f32p),
                              _ptr(out_prev, _f32p), _ptr(out_cur, _f32p), int(threads))
    if rc != 0:
        raise RuntimeError(f"oracle wave_stored failed with status {rc}")
    return out_prev, out_cur


def energy(u_new, u_old, r2: float, _lib_override=None) -> float:
    """Discrete leapfrog energy E^{n+1/2} of (u^{n+1}, u^n), float64."""
    a = np.ascontiguousarray(u_new, dtype=np.float64)
    b = np.ascontiguousarray(u_old, dtype=np.float64)
    if a.shape != b.shape:
        raise ValueError("shape mismatch")
    L = _lib_override or lib()
    if a.ndim == 1:
        return float(L.oracle_energy1d(_ptr(a, _f64p), _ptr(b, _f64p), a.shape[0], r2))
    if a.ndim == 2:
        return float(L.oracle_energy2d(_ptr(a, _f64p), _ptr(b, _f64p), a.shape[0],
                                       a.shape[1], r2))
    if a.ndim == 3:
        return float(L.oracle_energy3d(_ptr(a, _f64p), _ptr(b, _f64p), a.shape[0],
                                       a.shape[1], a.shape[2], r2))
    raise ValueError("rank must be 1, 2 or 3")


def sum_along(x, dim: int):
    """out[i] = x[i with i_dim = 0] + x[i with i_dim = 1] + ... in float32,
    summed in index order starting from 0 (each addition rounded once), the
    same value at every index along `dim`: the reduction a kernel with a
    slice(dim) range mapper computes (section 3: a mapper naming the whole
    extent along one dimension)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    acc = np.zeros(x.shape[:dim] + x.shape[dim + 1:], dtype=np.float32)
    for v in range(x.shape[dim]):
        acc = acc + np.take(x, v, axis=dim)  # float32 + float32 -> float32, rounded
    return np.ascontiguousarray(np.broadcast_to(np.expand_dims(acc, dim), x.shape))


def saxpy(a: float, x, y):
    """z = fma(a, x, y) in float32 (the paper's first listing, section 2)."""
    x = np.ascontiguousarray(x, dtype=np.float32)
    y = np.ascontiguousarray(y, dtype=np.float32)
    if x.shape != y.shape:
        raise ValueError("shape mismatch")
    z = np.empty_like(x)
    rc = lib().oracle_saxpy_f32(x.size, float(np.float32(a)), _ptr(x, _f32p),
                                _ptr(y, _f32p), _ptr(z, _f32p))
    if rc != 0:
        raise RuntimeError(f"oracle saxpy failed with status {rc}")
    return z
