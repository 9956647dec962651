"""MACE (two layers, correlation 3, l_max 3) through the C ABI against the
FP64 MACE oracle on identical seeded inputs.

The GPU path evaluates the couplings from its own harmonics and a host
quadrature, contracts expanded product terms per channel, mixes channels on
the matrix cores and runs a hand-written adjoint; the oracle contracts the
coupling tensors of its own harmonics with torch and differentiates by
autograd.  Tolerances and the per-row bound are those of tests/parity.py.
"""
import numpy as np
import pytest

from oracle import mace as MO
from oracle import oracle as O
from paper_2506_04055_amd import synth
from parity import TOL, check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_04055_amd import mlp as M
    M.lib()
    return M


def run(M, h, w, sysm, precision="fp32", skin=0.5, fold=True):
    import torch
    model = M.Model(h, w, precision)
    owner = sysm.owner if (fold and sysm.n_atoms > sysm.n_local) else None
    d = M.System(model, sysm.pos, sysm.species, sysm.box, n_local=sysm.n_local, skin=skin, ghost_owner=owner)
    out = d.compute(atom_energy=True, stats=True)
    torch.cuda.synchronize()
    return {"E": float(out["energy"].item()), "F": out["forces"].t().cpu().numpy().astype(np.float64),
            "U": out["atom_energy"].cpu().numpy().astype(np.float64), "stats": out["stats"], "sys": d,
            "model": model}


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16_node"])
def test_mace_fcc_periodic(mlp, precision):
    h, w = synth.make_mace_weights(1, seed=0, bias_scale=0.1)
    s = synth.fcc_crystal(3, seed=0, sigma=0.1)
    print(f"[case] mace fcc108 {precision}", flush=True)
    E_ref, F_ref, U_ref = MO.energy_forces(h, w, s.pos, s.species, s.box, per_atom=True)
    r = run(mlp, h, w, s, precision)
    check("mace fcc108", precision, r["E"], E_ref, r["F"], F_ref)
    et, _ = TOL[precision]
    du = np.abs(r["U"] - U_ref).max() / np.abs(U_ref).mean()
    print(f"[measured] mace fcc108 {precision}: per-atom energy max |dU|/mean|U| {du:.2e}")
    assert du <= 20 * et


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_mace_water_two_species(mlp, precision):
    h, w = synth.make_mace_weights(2, seed=3, bias_scale=0.2)
    s = synth.water_box(4, 3.105, seed=1)
    print(f"[case] mace water192 {precision}", flush=True)
    E_ref, F_ref = MO.energy_forces(h, w, s.pos, s.species, s.box)
    r = run(mlp, h, w, s, precision, skin=1.0)
    check("mace water192", precision, r["E"], E_ref, r["F"], F_ref)


def test_mace_four_species_and_ragged_size(mlp):
    h, w = synth.make_mace_weights(4, seed=5, bias_scale=0.1)
    s = synth.peptide_like(700, 3)
    print("[case] mace peptide700 fp32", flush=True)
    E_ref, F_ref = MO.energy_forces(h, w, s.pos, s.species, s.box)
    r = run(mlp, h, w, s, "fp32")
    check("mace peptide700 S=4", "fp32", r["E"], E_ref, r["F"], F_ref)


def test_mace_ghost_domain_and_fold(mlp):
    # one domain's share with a ghost shell of depth 2 rc (two layers: two hops)
    h, w = synth.make_mace_weights(1, seed=7, bias_scale=0.1)
    dom = synth.fcc_crystal(4, seed=2, ghost_depth=10.0)
    print(f"[case] mace fcc4 ghost domain {dom.n_local} locals {dom.n_atoms} rows", flush=True)
    E_ref, F_ref = MO.energy_forces(h, w, dom.pos, dom.species, np.zeros(3), n_local=dom.n_local)
    r = run(mlp, h, w, dom, "fp32", fold=False)
    check("mace fcc4 ghost (raw rows)", "fp32", r["E"], E_ref, r["F"], F_ref)
    r2 = run(mlp, h, w, dom, "fp32", fold=True)
    Ff = O.fold_ghost_forces(F_ref, dom.n_local, dom.owner)
    check("mace fcc4 ghost (folded)", "fp32", r2["E"], E_ref, r2["F"], Ff)
    hops = r["stats"]["n_within_hops"]
    assert hops[0] == dom.n_local
    # atoms beyond two hops of the locals carry no force
    assert hops[2] <= dom.n_atoms


def test_mace_larger_box_every_row(mlp):
    # 500 atoms: many workgroups of every kernel and a ragged tail
    h, w = synth.make_mace_weights(1, seed=11, bias_scale=0.1)
    s = synth.fcc_crystal(5, seed=4, sigma=0.1)
    print("[case] mace fcc500 fp32+bf16", flush=True)
    E_ref, F_ref = MO.energy_forces(h, w, s.pos, s.species, s.box)
    for prec in ("fp32", "bf16"):
        r = run(mlp, h, w, s, prec)
        check("mace fcc500", prec, r["E"], E_ref, r["F"], F_ref)


def test_mace_determinism_and_permutation(mlp):
    import torch
    h, w = synth.make_mace_weights(2, seed=2)
    s = synth.water_box(4, 3.105, seed=2)
    r1 = run(mlp, h, w, s, "fp32", skin=1.0)
    r1["sys"].compute()
    torch.cuda.synchronize()
    F_again = r1["sys"].forces.t().cpu().numpy().astype(np.float64)
    assert np.array_equal(F_again, r1["F"])
    perm = np.random.default_rng(0).permutation(s.n_atoms)
    s2 = synth.System(s.pos[perm], s.species[perm], s.box, s.n_atoms)
    r2 = run(mlp, h, w, s2, "fp32", skin=1.0)
    assert abs(r2["E"] - r1["E"]) <= 2e-6 * abs(r1["E"])
    assert np.abs(r2["F"] - r1["F"][perm]).max() <= 1e-5 * np.abs(r1["F"]).max()


def test_mace_header_errors(mlp):
    h, w = synth.make_mace_weights(1, seed=0)
    with pytest.raises(mlp.MLPError):
        mlp.Model(h, w[:-1], "fp32")
    for bad in (dict(h, l_max=2), dict(h, channels=16), dict(h, correlation=2), dict(h, envelope="cosine"),
                dict(h, radial_hidden=[64, 64, 64, 64, 64]), dict(h, readout_hidden=64)):
        with pytest.raises(mlp.MLPError):
            mlp.Model(bad, w, "fp32")
