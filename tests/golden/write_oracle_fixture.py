"""Writes oracle_water192.json: the FP64 oracle's energy and forces for the
192-atom water box with the 2-layer model (F = 32, K = 8, two species).

The stored values come from the oracle alone (this script imports only the
oracle and the seeded input generators), so a later change to the oracle's
arithmetic shows up as a difference against them.  Run from the repository
root: python tests/golden/write_oracle_fixture.py
"""
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import oracle as O  # noqa: E402
from paper_2506_04055_amd import synth  # noqa: E402


def input_digest(s, w) -> str:
    h = hashlib.sha256()
    for a in (np.asarray(s.pos, np.float32), np.asarray(s.species, np.int32), np.asarray(s.box, np.float64),
              np.asarray(w, np.float32)):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def main():
    s, hdr, w = synth.workload("water192")
    E, F = O.energy_forces(hdr, w, s.pos, s.species, s.box)
    out = {
        "what": "FP64 oracle energy (eV) and forces (eV/A, rows = atoms, F = -dE/dr) of the 192-atom water box",
        "model": "PaiNN-form message passing, T = 2, F = 32, K = 8, rc = 5 A, two species (Methods, "
                 "'Graph Neural Networks' and 'Chosen Architectures'; energy as the sum of per-atom "
                 "energies and forces as its negative gradient, Results, 'Distributed potential computation')",
        "inputs": "synth.workload('water192'): 4^3 water molecules on a jittered 3.105 A lattice, seed 0; "
                  "weights N(0, 1/fan_in), seed 0",
        "input_sha256": input_digest(s, w),
        "written_by": "tests/golden/write_oracle_fixture.py (oracle only)",
        "energy": float(E),
        "forces": [[float(x) for x in row] for row in F],
    }
    with open(os.path.join(HERE, "oracle_water192.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
