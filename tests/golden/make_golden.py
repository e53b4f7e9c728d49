"""Writes the exact-rational fixtures in this folder.

Calls only the oracle's exact rational stepper and the seeded input
generators.  Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import synth  # noqa: E402
from oracle import exact  # noqa: E402


def write(name, shape, seed, r2, steps):
    u0 = synth.dyadic_field(shape, seed)
    _, uc = exact.wave_exact(u0, u0, r2, steps)
    doc = {
        "what": "leapfrog u+ = r2*lap(u) + 2u - u-, Dirichlet-0, u^-1 = u^0, "
                "iterated in exact rationals; u_final = u^steps rounded to float64",
        "input": f"synth.dyadic_field({shape}, seed={seed}) (k/256, exact in float32)",
        "r2": r2, "steps": steps,
        "u0": u0.tolist(),
        "u_final": exact.to_array(uc, shape).tolist(),
    }
    with open(os.path.join(HERE, name), "w") as f:
        json.dump(doc, f, indent=None)
        f.write("\n")


if __name__ == "__main__":
    write("exact_8x8.json", (8, 8), 31, 0.25, 64)
    write("exact_4x4x4.json", (4, 4, 4), 32, 0.1, 30)
