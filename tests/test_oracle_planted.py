"""Plants plausible mistakes in a copy of the oracle's C source and checks
that the pins reject every one of them (CPU only; the copy is compiled into
a temporary folder and never touches the real oracle build)."""

import numpy as np
import pytest

import oracle
import synth
from test_oracle_wave import closed_form

MUTATIONS = {
    # a dropped neighbour term in 2D
    "drop_east": ("(cur[P2(i, j - 1)] + cur[P2(i, j + 1)])", "(cur[P2(i, j - 1)] + 0)"),
    # wrong sign on the previous level
    "sign_prev": ("FMA(r2, lap, TWO * c - prev[P2(i, j)])", "FMA(r2, lap, TWO * c + prev[P2(i, j)])"),
    # wrong centre coefficient
    "coef_four": ("WAVE2D_BODY(double, fma, 4.0, 2.0)", "WAVE2D_BODY(double, fma, 3.9, 2.0)"),
    # transposed read of the input (in bounds, wrong cell)
    "transpose_in": ("cur[P2(i, j)] = u_cur0[i * nx + j];", "cur[P2(i, j)] = u_cur0[j * ny + i];"),
    # index shifted: north neighbour read two rows up
    "shift_north": ("T sum = (cur[P2(i - 1, j)]", "T sum = (cur[P2(i - 1 > -1 ? i - 2 : i - 1, j)]"),
    # 3D: a dropped z neighbour
    "drop_zplus": ("T sum = ((cur[P3(z - 1, y, x)] + cur[P3(z + 1, y, x)]) +",
                   "T sum = ((cur[P3(z - 1, y, x)] + 0) +"),
    # energy: edges to the ghost layer left out
    "energy_no_ghost": ("const int64_t lo[3] = {active[0] ? -1 : 0, active[1] ? -1 : 0, active[2] ? -1 : 0};",
                        "const int64_t lo[3] = {0, 0, 0};"),
    # energy: wrong r^2 weight
    "energy_r2": ("return kin.s + r2 * pot.s;", "return kin.s + pot.s;"),
}


def _pins_pass(L):
    """Runs the closed-form and energy pins against library L."""
    ok = True
    shape, modes, r2 = (30, 20), (3, 2), 0.25
    phi = synth.mode_field(shape, modes)
    _, uc = oracle.wave(phi.copy(), phi, r2, 200, _lib_override=L)
    ok &= np.max(np.abs(uc - closed_form(shape, modes, r2, 200, "rest") * phi)) <= 1e-10
    shp3, m3, r3 = (8, 7, 6), (2, 3, 1), 0.1
    phi3 = synth.mode_field(shp3, m3)
    _, u3 = oracle.wave(phi3.copy(), phi3, r3, 100, _lib_override=L)
    ok &= np.max(np.abs(u3 - closed_form(shp3, m3, r3, 100, "rest") * phi3)) <= 1e-10
    for shape_e, rr in (((12, 9), 0.25), ((5, 4, 6), 0.1)):
        up = synth.uniform_field(shape_e, 1)
        u = synth.uniform_field(shape_e, 2)
        e0 = oracle.energy(u, up, rr, _lib_override=L)
        for _ in range(50):
            up, u = oracle.wave(up, u, rr, 1, _lib_override=L)
        e1 = oracle.energy(u, up, rr, _lib_override=L)
        ok &= abs(e1 - e0) <= 1e-12 * abs(e0) and e0 > 0
    return bool(ok)


def test_unmutated_copy_passes(tmp_path):
    L = oracle.load(oracle.build(out=tmp_path / "liboracle_copy.so"))
    assert _pins_pass(L)


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(tmp_path, name):
    old, new = MUTATIONS[name]
    src = oracle._SRC.read_text()
    assert src.count(old) == 1, f"mutation anchor for {name} not unique"
    (tmp_path / "oracle.c").write_text(src.replace(old, new))
    L = oracle.load(oracle.build(src=tmp_path / "oracle.c", out=tmp_path / f"lib_{name}.so"))
    assert not _pins_pass(L), f"pins did not catch planted mistake {name}"
