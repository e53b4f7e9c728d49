"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module only draws and lays out input data: initial wave fields, the
shapes and step counts of batched grids, and points of the launch-config
sample space.  It holds none of the stencil, range-splitting or cost-model
arithmetic; both sides receive what it returns as plain arrays.

Input recipe (the paper has no workload of its own; these stand in for it):

* Initial field u0 = A * prod_d exp(-(i_d - c_d)^2 / (2 sigma^2)) + eta,
  with A = 1, c_d = (n_d - 1) / 2, evaluated in float64 as a product of
  per-axis Gaussians, plus noise eta ~ U(-1e-3, 1e-3) drawn from numpy's
  PCG64 ``default_rng(seed)`` in C order, then rounded once to float32.
* The field before the first step equals u0 (zero initial velocity).
* Dirichlet zero outside the grid.
"""
from __future__ import annotations

import numpy as np

NOISE_AMPLITUDE = 1e-3


def _axis_gauss(n: int, sigma: float) -> np.ndarray:
    c = (n - 1) / 2.0
    i = np.arange(n, dtype=np.float64)
    return np.exp(-((i - c) ** 2) / (2.0 * sigma * sigma))


def gaussian_field(shape, sigma: float, seed: int | None, amp: float = 1.0,
                   noise: float = NOISE_AMPLITUDE, dtype=np.float32,
                   slab: int = 64) -> np.ndarray:
    """Gaussian bump centred on the grid plus seeded uniform noise.

    ``shape`` is (ny, nx) or (nz, ny, nx), slowest axis first.  ``seed=None``
    or ``noise=0`` gives the noise-free bump.  The noise is drawn slab by slab
    along axis 0; PCG64 uniform doubles consume one 64-bit draw each, so the
    result equals a single draw of the whole array.
    """
    shape = tuple(int(s) for s in shape)
    if len(shape) not in (1, 2, 3) or min(shape) < 1:
        raise ValueError(f"bad shape {shape}")
    gs = [_axis_gauss(n, sigma) for n in shape]
    out = np.empty(shape, dtype=dtype)
    rng = None if (seed is None or noise == 0.0) else np.random.default_rng(seed)
    for z0 in range(0, shape[0], slab):
        z1 = min(shape[0], z0 + slab)
        g = gs[0][z0:z1]
        for ga in gs[1:]:
            g = g[..., None] * ga
        g = amp * g
        if rng is not None:
            g = g + rng.uniform(-noise, noise, size=g.shape)
        out[z0:z1] = g.astype(dtype)
    return out


def mode_field(shape, modes, dtype=np.float64) -> np.ndarray:
    """Product of sines sin(pi m_d (i_d+1) / (n_d+1)): a Dirichlet eigenmode."""
    out = None
    for n, m in zip(shape, modes):
        i = np.arange(1, n + 1, dtype=np.float64)
        s = np.sin(np.pi * m * i / (n + 1))
        out = s if out is None else out[..., None] * s
    return out.astype(dtype)


def uniform_field(shape, seed: int, lo=-1.0, hi=1.0, dtype=np.float64):
    return np.random.default_rng(seed).uniform(lo, hi, size=tuple(shape)).astype(dtype)


def dyadic_field(shape, seed: int, bits: int = 8) -> np.ndarray:
    """Random dyadic rationals k / 2^bits in [-1, 1] (exact in float32)."""
    rng = np.random.default_rng(seed)
    k = rng.integers(-(1 << bits), (1 << bits) + 1, size=tuple(shape))
    return (k.astype(np.float64) / float(1 << bits))


# --------------------------------------------------------------------------
# Workloads.  Sizes follow the wave-stencil configurations this library is
# measured on; every random choice is seeded here.
# --------------------------------------------------------------------------

WORKLOADS = {
    "wave2d_256_k2": dict(dims=2, shape=(256, 256), r2=0.25, sigma=16.0, seed=0,
                          steps=100, chunks=2, share_offset=(0, 0)),
    # one GPU's 8192-row share (rows [8192, 16384)) of a 32768 x 8192 domain
    "wave2d_8192_share_k4": dict(dims=2, shape=(8192, 8192), r2=0.25, sigma=256.0,
                                 seed=1, steps=1000, chunks=4,
                                 global_shape=(32768, 8192), share_offset=(8192, 0)),
    "wave3d_768_k8": dict(dims=3, shape=(768, 768, 768), r2=0.1, sigma=48.0, seed=4,
                          steps=200, chunks=8, share_offset=(0, 0, 0)),
}


def batched_grids(count: int = 64, seed: int = 2, lo: int = 512, hi: int = 4096,
                  step: int = 64, steps_lo: int = 100, steps_hi: int = 500):
    """Independent 2D grids: (ny, nx, steps, sigma, seed) per grid.

    ny and nx are drawn independently from {lo, lo+step, ..., hi}; steps are
    uniform integers in [steps_lo, steps_hi]; sigma = min(ny, nx) / 16; the
    noise seed of grid g is 2000 + g.
    """
    rng = np.random.default_rng(seed)
    sides = np.arange(lo, hi + 1, step)
    ny = rng.choice(sides, size=count)
    nx = rng.choice(sides, size=count)
    st = rng.integers(steps_lo, steps_hi + 1, size=count)
    return [dict(ny=int(ny[g]), nx=int(nx[g]), steps=int(st[g]),
                 sigma=float(min(ny[g], nx[g])) / 16.0, seed=2000 + g)
            for g in range(count)]


def cost_model_shapes(count: int, seed: int, lo: int = 256, hi: int = 16384,
                      align: int = 64):
    """2D shapes with each side log-uniform on [lo, hi], rounded to ``align``."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        s = np.exp(rng.uniform(np.log(lo), np.log(hi), size=2))
        s = np.clip((np.round(s / align) * align).astype(int), lo, hi)
        out.append((int(s[0]), int(s[1])))
    return out


def cost_model_shapes_3d(count: int, seed: int, lo: int = 64, hi: int = 768, align: int = 32,
                         max_cells: int = 1 << 29):
    """3D shapes with each side log-uniform on [lo, hi], rounded to ``align``,
    at most ``max_cells`` cells."""
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        s = np.exp(rng.uniform(np.log(lo), np.log(hi), size=3))
        s = np.clip((np.round(s / align) * align).astype(int), lo, hi)
        if int(np.prod(s)) <= max_cells:
            out.append((int(s[0]), int(s[1]), int(s[2])))
    return out


def mlp_params(sizes, seed: int, dtype=np.float64):
    """He-uniform initial weights W_l (out x in) and zero biases."""
    rng = np.random.default_rng(seed)
    ws, bs = [], []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        bound = np.sqrt(6.0 / fan_in)
        ws.append(rng.uniform(-bound, bound, size=(fan_out, fan_in)).astype(dtype))
        bs.append(np.zeros(fan_out, dtype=dtype))
    return ws, bs


def mlp_batch(n: int, n_in: int, n_out: int, seed: int, dtype=np.float64):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, n_in)).astype(dtype)
    t = rng.standard_normal((n, n_out)).astype(dtype)
    return x, t
