"""CPU-side checks of the C-ABI library (no GPU calls) and of the input generators."""
import ctypes
import json
import os
import re

import numpy as np
import pytest

from paper_2506_04055_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mlp.h")
LIB = os.path.join(ROOT, "paper_2506_04055_amd", "libmlp.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mlp_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libmlp.so is not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "mlp_energy_forces" in names and "mlp_build_neighbors" in names and "mlp_submit" in names
    for n in names:
        assert hasattr(lib, n), f"{n} declared in include/mlp.h but not exported"


def _create(lib, header, w):
    lib.mlp_model_create.argtypes = [ctypes.c_char_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int,
                                     ctypes.POINTER(ctypes.c_void_p)]
    lib.mlp_model_create.restype = ctypes.c_int
    lib.mlp_last_error.restype = ctypes.c_char_p
    h = ctypes.c_void_p()
    w = np.ascontiguousarray(w, np.float32)
    rc = lib.mlp_model_create(header.encode(), w.ctypes.data_as(ctypes.c_void_p), w.size, 0, ctypes.byref(h))
    return rc, lib.mlp_last_error().decode()


def test_header_validation_rejects_before_touching_the_device(lib):
    hdr, w = synth.make_weights(32, 8, 2, 2)
    rc, msg = _create(lib, json.dumps(hdr), w[:-3])
    assert rc == -1 and "weight count" in msg
    bad = dict(hdr, basis="gaussian")
    rc, msg = _create(lib, json.dumps(bad), w)
    assert rc == -1 and "basis" in msg
    bad = dict(hdr, F=48)
    rc, msg = _create(lib, json.dumps(bad), w)
    assert rc == -1
    rc, msg = _create(lib, "not json", w)
    assert rc == -1
    missing = {k: v for k, v in hdr.items() if k != "r_c"}
    rc, msg = _create(lib, json.dumps(missing), w)
    assert rc == -1 and "r_c" in msg


def test_generators_are_float32_exact_and_wrapped():
    for s in (synth.water_box(4, 3.105), synth.peptide_like(900, 2), synth.fcc_crystal(3)):
        assert s.pos.dtype == np.float32
        assert np.all(s.box == s.box.astype(np.float32))
        for d in range(3):
            assert np.all(s.pos[:, d] >= 0) and np.all(s.pos[:, d] < np.float32(s.box[d]))


def test_generator_recipes():
    s = synth.water_box(20, 3.105)
    assert s.n_atoms == 24000 and np.isclose(s.box[0], 62.1, atol=1e-5)
    # 1 g/cm^3: 8000 molecules * 18.015 amu in 62.1^3 A^3
    rho = 8000 * 18.015 * 1.66054 / 62.1**3
    assert abs(rho - 1.0) < 0.01
    p = synth.peptide_like(5000, 3)
    assert np.bincount(p.species).tolist() == [3000, 1000, 500, 500]
    assert abs(5000 / p.box[0] ** 3 - synth.PEPTIDE_DENSITY) < 1e-4
    g = synth.fcc_crystal(4, ghost_depth=15.0)
    assert g.n_local == 256 and np.all(g.box == 0) and g.owner.max() < 256
    # each ghost is an image of its owner shifted by a lattice vector of the box
    L = 4 * 4.05
    shift = (g.pos[g.n_local:].astype(np.float64) - g.pos[g.owner].astype(np.float64)) / np.float32(L)
    assert np.abs(shift - np.round(shift)).max() < 1e-5
    sizes, seeds = synth.serving_requests(2000, seed=1)
    assert sizes.min() >= 500 and sizes.max() <= 20000 and len(set(seeds.tolist())) > 1990


def test_weight_layout_matches_header():
    hdr, w = synth.make_weights(128, 20, 3, 2)
    assert w.size == hdr["n_weights"] == 576513
    V = synth.weight_views(hdr, w)
    assert V["l2.A"].shape == (384, 20) and V["W5"].shape == (64, 128)
