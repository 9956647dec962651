"""The oracle against its own stored result (CPU only).

tests/golden/oracle_water192.json holds the FP64 oracle's energy and forces
for the 192-atom water box, written by tests/golden/write_oracle_fixture.py.
The inputs are regenerated from their seeds and must hash to the stored
digest; the oracle must then reproduce the stored values to rounding, so any
later change to its arithmetic (or to the seeded generators) is visible.
"""
import json
import os

import numpy as np

from paper_2506_04055_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_fixture():
    with open(os.path.join(GOLDEN, "oracle_water192.json")) as f:
        return json.load(f)


def test_inputs_regenerate_bit_for_bit():
    import importlib.util
    spec = importlib.util.spec_from_file_location("wof", os.path.join(GOLDEN, "write_oracle_fixture.py"))
    wof = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(wof)
    s, hdr, w = synth.workload("water192")
    assert wof.input_digest(s, w) == load_fixture()["input_sha256"]


def test_oracle_reproduces_stored_result(oracle):
    d = load_fixture()
    s, hdr, w = synth.workload("water192")
    E, F = oracle.energy_forces(hdr, w, s.pos, s.species, s.box)
    Fs = np.array(d["forces"], np.float64)
    assert F.shape == Fs.shape == (s.n_atoms, 3)
    assert abs(E - d["energy"]) <= 1e-12 * abs(d["energy"])
    assert np.abs(F - Fs).max() <= 1e-12 * np.abs(Fs).max()
