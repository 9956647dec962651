"""Allegro (single tensor-product layer) through the C ABI against the FP64
Allegro oracle on identical seeded inputs.

The GPU path builds each atom's environment from spherical harmonics and
contracts every edge against it; the oracle sums Legendre polynomials over
pairs of edges.  The two agree only if the harmonics, their normalisation,
the channel layout and the adjoint are right.  Tolerances and the per-row
bound are those of tests/parity.py (the same operand forms as PaiNN's).
"""
import numpy as np
import pytest

from oracle import allegro as AO
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
def test_al_fcc_periodic(mlp, precision):
    h, w = synth.make_allegro_weights(1, seed=0, bias_scale=0.1)
    # sigma = 0.1 A: near a perfect lattice the net forces are small
    # differences of large edge terms, and their relative error measures that
    # cancellation rather than the path (at sigma = 0.05 A the FP32 and split
    # bf16 results both sit at ~1.1e-5, the same float32 geometry floor)
    s = synth.fcc_crystal(3, seed=0, sigma=0.1)
    print(f"[case] allegro fcc108 {precision}", flush=True)
    E_ref, F_ref, U_ref = AO.energy_forces(h, w, s.pos, s.species, s.box, per_atom=True)
    r = run(mlp, h, w, s, precision)
    check("allegro fcc108", precision, r["E"], E_ref, r["F"], F_ref)
    et, _ = TOL[precision]
    du = np.abs(r["U"] - U_ref).max() / np.abs(U_ref).mean()
    print(f"[measured] allegro fcc108 {precision}: per-atom energy max |dU|/mean|U| {du:.2e}")
    assert du <= 20 * et


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_al_water_two_species(mlp, precision):
    h, w = synth.make_allegro_weights(2, seed=3, bias_scale=0.2)
    s = synth.water_box(4, 3.105, seed=1)
    print(f"[case] allegro water192 {precision}", flush=True)
    E_ref, F_ref = AO.energy_forces(h, w, s.pos, s.species, s.box)
    r = run(mlp, h, w, s, precision, skin=1.0)
    check("allegro water192", precision, r["E"], E_ref, r["F"], F_ref)


def test_al_four_species_and_ragged_size(mlp):
    h, w = synth.make_allegro_weights(4, seed=5, bias_scale=0.1)
    s = synth.peptide_like(700, 3)
    print("[case] allegro peptide700 fp32", flush=True)
    E_ref, F_ref = AO.energy_forces(h, w, s.pos, s.species, s.box)
    r = run(mlp, h, w, s, "fp32")
    check("allegro peptide700 S=4", "fp32", r["E"], E_ref, r["F"], F_ref)


def test_al_ghost_domain_and_fold(mlp):
    # one domain's share with a ghost shell of depth rc (strictly local: one hop)
    h, w = synth.make_allegro_weights(1, seed=7, bias_scale=0.1)
    dom = synth.fcc_crystal(4, seed=2, ghost_depth=5.0)
    print(f"[case] allegro fcc4 ghost domain {dom.n_local} locals {dom.n_atoms} rows", flush=True)
    E_ref, F_ref = AO.energy_forces(h, w, dom.pos, dom.species, np.zeros(3), n_local=dom.n_local)
    r = run(mlp, h, w, dom, "fp32", fold=False)
    check("allegro fcc4 ghost (raw rows)", "fp32", r["E"], E_ref, r["F"], F_ref)
    r2 = run(mlp, h, w, dom, "fp32", fold=True)
    Ff = O.fold_ghost_forces(F_ref, dom.n_local, dom.owner)
    check("allegro fcc4 ghost (folded)", "fp32", r2["E"], E_ref, r2["F"], Ff)
    # atoms more than one hop from the locals carry nothing
    assert r["stats"]["n_within_hops"][0] == dom.n_local


def test_al_larger_box_every_row(mlp):
    # 500 atoms: several workgroups of every kernel and a ragged tail
    h, w = synth.make_allegro_weights(1, seed=11, bias_scale=0.1)
    s = synth.fcc_crystal(5, seed=4, sigma=0.1)
    print("[case] allegro fcc500 fp32+bf16", flush=True)
    E_ref, F_ref = AO.energy_forces(h, w, s.pos, s.species, s.box)
    for prec in ("fp32", "bf16"):
        r = run(mlp, h, w, s, prec)
        check("allegro fcc500", prec, r["E"], E_ref, r["F"], F_ref)


def test_al_determinism_and_permutation(mlp):
    import torch
    h, w = synth.make_allegro_weights(2, seed=2)
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


def test_al_header_errors(mlp):
    h, w = synth.make_allegro_weights(1, seed=0)
    with pytest.raises(mlp.MLPError):
        mlp.Model(h, w[:-1], "fp32")
    bad = dict(h, channels=[32, 16, 8, 8, 8])
    with pytest.raises(mlp.MLPError):
        mlp.Model(bad, w, "fp32")
    bad = dict(h, envelope="cosine")
    with pytest.raises(mlp.MLPError):
        mlp.Model(bad, w, "fp32")
