"""Writes tests/golden/exact_energies.json by exact diagonalisation with the oracle only.

Run from the repository root:  python tests/golden/make_golden.py
The values are ground-state energies per site of the full lattice Hamiltonians
(eq. groundstate) that the pins compare bounds against.
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import exact  # noqa: E402

CASES = [
    ("tfi_ring_N8_h1", synth.tfi_terms(1.0, 1.0, 1), (8, 1)),
    ("afh_ring_N8", synth.afh_terms(1), (8, 1)),
    ("afh_ring_N20", synth.afh_terms(1), (20, 1)),
    ("tfi_torus_4x4_h1", synth.tfi_terms(1.0, 1.0, 2), (4, 4)),
    ("tfi_torus_4x4_h2", synth.tfi_terms(2.0, 1.0, 2), (4, 4)),
    ("tfi_torus_4x4_h3", synth.tfi_terms(3.0, 1.0, 2), (4, 4)),
    ("afh_torus_4x4", synth.afh_terms(2), (4, 4)),
    ("xxz_ring_N8_Jz0.5", synth.xxz_terms(0.5, 1), (8, 1)),
]

if __name__ == "__main__":
    out = {}
    for name, terms, extent in CASES:
        E0, _ = exact.ground_state(terms, extent)
        out[name] = {"extent": list(extent), "E0_per_site": E0 / (extent[0] * extent[1])}
        print(name, out[name], flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "exact_energies.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
