"""Pins of the CPU oracle's leapfrog steppers (CPU only).

Each check ties the oracle to something other than its own formula:
  * the discrete standing-wave closed form (Dirichlet eigenmodes of the
    5-/7-/3-point Laplacian; the amplitude recurrence a^{k+1} = 2 cos(theta)
    a^k - a^{k-1} with cos(theta) = 1 - 2 r^2 S), to 1e-10 after 1000 steps;
  * conservation of the discrete leapfrog energy, to 1e-12 relative;
  * exact rational iteration on 8x8 and 4x4x4 grids (stored fixture);
  * special cases: r^2 = 0 is the identity, zero stays zero, a centred
    noise-free bump stays bitwise mirror/transpose symmetric in float32;
  * OpenMP threading leaves results bitwise unchanged.
Non-square grids are used throughout so that a transposed index fails.
"""
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def closed_form(shape, modes, r2, k, start):
    """Exact amplitude of a Dirichlet eigenmode after k leapfrog steps."""
    S = sum(math.sin(math.pi * m / (2.0 * (n + 1))) ** 2 for n, m in zip(shape, modes))
    theta = 2.0 * math.asin(math.sqrt(r2 * S))
    if start == "rest":  # u^{-1} = u^0 = phi
        return math.cos((k + 0.5) * theta) / math.cos(0.5 * theta)
    return math.cos(k * theta)  # u^{-1} = phi cos(theta)


def prev_for(shape, modes, r2, phi, start):
    if start == "rest":
        return phi.copy()
    S = sum(math.sin(math.pi * m / (2.0 * (n + 1))) ** 2 for n, m in zip(shape, modes))
    return phi * (1.0 - 2.0 * r2 * S)


@pytest.mark.parametrize("start", ["rest", "moving"])
@pytest.mark.parametrize("modes", [(1, 1), (3, 2), (29, 19), (15, 1), (7, 13)])
def test_closed_form_2d(oracle_lib, modes, start):
    shape, r2, steps = (30, 20), 0.25, 1000
    phi = synth.mode_field(shape, modes)
    up, uc = oracle.wave(prev_for(shape, modes, r2, phi, start), phi, r2, steps)
    a_cur = closed_form(shape, modes, r2, steps, start)
    a_prev = closed_form(shape, modes, r2, steps - 1, start)
    assert np.max(np.abs(uc - a_cur * phi)) <= 1e-10
    assert np.max(np.abs(up - a_prev * phi)) <= 1e-10


@pytest.mark.parametrize("modes", [(1, 1, 1), (2, 5, 3), (11, 9, 8), (6, 1, 7)])
def test_closed_form_3d(oracle_lib, modes):
    shape, r2, steps = (12, 10, 9), 0.1, 1000
    phi = synth.mode_field(shape, modes)
    _, uc = oracle.wave(phi.copy(), phi, r2, steps)
    assert np.max(np.abs(uc - closed_form(shape, modes, r2, steps, "rest") * phi)) <= 1e-10


@pytest.mark.parametrize("m", [1, 4, 49])
def test_closed_form_1d(oracle_lib, m):
    shape, r2, steps = (50,), 0.81, 1000
    phi = synth.mode_field(shape, (m,))
    _, uc = oracle.wave(phi.copy(), phi, r2, steps)
    assert np.max(np.abs(uc - closed_form(shape, (m,), r2, steps, "rest") * phi)) <= 1e-10


def test_closed_form_fp32_tracks(oracle_lib):
    """The float32 stepper follows the same mode to float32 accuracy."""
    shape, modes, r2, steps = (30, 20), (3, 2), 0.25, 1000
    phi = synth.mode_field(shape, modes)
    p32 = phi.astype(np.float32)
    _, uc = oracle.wave(p32.copy(), p32, r2, steps)
    exact = closed_form(shape, modes, r2, steps, "rest") * phi
    assert np.max(np.abs(uc.astype(np.float64) - exact)) <= 1e-4


def _energy_series(u_prev, u_cur, r2, steps):
    es = [oracle.energy(u_cur, u_prev, r2)]
    for _ in range(steps):
        u_prev, u_cur = oracle.wave(u_prev, u_cur, r2, 1)
        es.append(oracle.energy(u_cur, u_prev, r2))
    return np.array(es)


def test_energy_conserved_2d(oracle_lib):
    shape, r2 = (40, 28), 0.25
    u_prev = synth.uniform_field(shape, 11)
    u_cur = synth.uniform_field(shape, 12)
    es = _energy_series(u_prev, u_cur, r2, 1000)
    assert es[0] > 0
    assert np.max(np.abs(es - es[0])) / es[0] <= 1e-12


def test_energy_conserved_3d(oracle_lib):
    shape, r2 = (9, 8, 7), 0.1
    u_prev = synth.uniform_field(shape, 13)
    u_cur = synth.uniform_field(shape, 14)
    es = _energy_series(u_prev, u_cur, r2, 500)
    assert es[0] > 0
    assert np.max(np.abs(es - es[0])) / es[0] <= 1e-12


def test_energy_conserved_1d(oracle_lib):
    shape, r2 = (64,), 0.64
    es = _energy_series(synth.uniform_field(shape, 15), synth.uniform_field(shape, 16), r2, 500)
    assert np.max(np.abs(es - es[0])) / es[0] <= 1e-12


def test_energy_is_discrete_form(oracle_lib):
    """E on a 2x1 grid written out by hand: two cells, one interior edge and
    four ghost edges (two at each end of the column, one each side in x)."""
    a1, b1, a0, b0, r2 = 0.3, -0.2, 0.1, 0.5, 0.25
    new = np.array([[a1], [b1]])
    old = np.array([[a0], [b0]])
    kin = (a1 - a0) ** 2 + (b1 - b0) ** 2
    pot = (a1 - b1) * (a0 - b0) + a1 * a0 + b1 * b0  # y edges incl. ghosts
    pot += 2 * a1 * a0 + 2 * b1 * b0  # x edges to the ghost columns
    assert oracle.energy(new, old, r2) == pytest.approx(kin + r2 * pot, rel=1e-15)


def test_exact_rational_golden_2d(oracle_lib):
    with open(os.path.join(GOLDEN, "exact_8x8.json")) as f:
        g = json.load(f)
    u0 = np.array(g["u0"], dtype=np.float64)
    up, uc = oracle.wave(u0.copy(), u0, g["r2"], g["steps"])
    exact = np.array(g["u_final"], dtype=np.float64)
    scale = np.max(np.abs(exact))
    assert np.max(np.abs(uc - exact)) <= 1e-13 * scale
    # float32 oracle on the same (float32-exact) inputs stays within float32 rounding
    u32 = u0.astype(np.float32)
    _, uc32 = oracle.wave(u32.copy(), u32, g["r2"], g["steps"])
    assert np.max(np.abs(uc32.astype(np.float64) - exact)) <= 1e-5 * scale


def test_exact_rational_golden_3d(oracle_lib):
    with open(os.path.join(GOLDEN, "exact_4x4x4.json")) as f:
        g = json.load(f)
    u0 = np.array(g["u0"], dtype=np.float64)
    _, uc = oracle.wave(u0.copy(), u0, g["r2"], g["steps"])
    exact = np.array(g["u_final"], dtype=np.float64)
    assert np.max(np.abs(uc - exact)) <= 1e-13 * np.max(np.abs(exact))


def test_exact_rational_live_small(oracle_lib):
    """Exact iteration recomputed here (not from the fixture) on a 5x3 grid."""
    from oracle import exact
    u0 = synth.dyadic_field((5, 3), 21)
    um = synth.dyadic_field((5, 3), 22)
    ep, ec = exact.wave_exact(um, u0, 0.25, 20)
    up, uc = oracle.wave(um, u0, 0.25, 20)
    assert np.array_equal(uc, exact.to_array(ec, (5, 3)))  # dyadic stays exact in fp64
    assert np.array_equal(up, exact.to_array(ep, (5, 3)))


@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_r2_zero_is_identity(oracle_lib, dtype):
    u = synth.gaussian_field((33, 17), 4.0, seed=3).astype(dtype)
    up, uc = oracle.wave(u.copy(), u, 0.0, 57)
    assert np.array_equal(uc, u) and np.array_equal(up, u)


def test_zero_stays_zero(oracle_lib):
    z = np.zeros((16, 9), np.float32)
    up, uc = oracle.wave(z, z, 0.25, 40)
    assert not np.any(uc) and not np.any(up)
    z3 = np.zeros((5, 6, 7), np.float32)
    _, uc3 = oracle.wave(z3, z3, 0.1, 20)
    assert not np.any(uc3)


def test_symmetry_fp32_bitwise(oracle_lib):
    u = synth.gaussian_field((64, 64), 6.0, seed=None)
    up, uc = oracle.wave(u.copy(), u, 0.25, 300)
    assert np.array_equal(uc, uc[::-1, :])
    assert np.array_equal(uc, uc[:, ::-1])
    assert np.array_equal(uc, uc.T)


def test_symmetry_3d_mirror_fp32_bitwise(oracle_lib):
    u = synth.gaussian_field((20, 18, 16), 3.0, seed=None)
    _, uc = oracle.wave(u.copy(), u, 0.1, 60)
    assert np.array_equal(uc, uc[::-1])
    assert np.array_equal(uc, uc[:, ::-1])
    assert np.array_equal(uc, uc[:, :, ::-1])


def test_threads_bitwise(oracle_lib):
    u = synth.gaussian_field((96, 80), 8.0, seed=5)
    a = oracle.wave(u.copy(), u, 0.25, 30, threads=1)[1]
    b = oracle.wave(u.copy(), u, 0.25, 30, threads=4)[1]
    assert np.array_equal(a, b)
    u3 = synth.gaussian_field((12, 10, 8), 3.0, seed=6)
    a3 = oracle.wave(u3.copy(), u3, 0.1, 10, threads=1)[1]
    b3 = oracle.wave(u3.copy(), u3, 0.1, 10, threads=3)[1]
    assert np.array_equal(a3, b3)


def test_fp64_vs_fp32_gap_small(oracle_lib):
    """float32 and float64 steppers from the same float32 start agree to the
    level float32 rounding allows (100 steps, 256x256 workload shape)."""
    u = synth.gaussian_field((256, 256), 16.0, seed=0)
    _, c32 = oracle.wave(u.copy(), u, 0.25, 100)
    u64 = u.astype(np.float64)
    _, c64 = oracle.wave(u64.copy(), u64, 0.25, 100)
    rel = np.max(np.abs(c32 - c64)) / np.max(np.abs(c64))
    assert rel <= 1e-5
