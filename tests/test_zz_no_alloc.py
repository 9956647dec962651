"""The allocation-free entry point (mlp_energy_forces_noalloc) against
mlp_energy_forces, through the C ABI.

Both run the same kernels in the same order on the same inputs, so their
energies, per-atom energies and forces must agree bit for bit; the results
are also held to the oracle's FP32 bar.  Two calls in a row on one GPU, the
second with a smaller system, check that the shared scratch array carries
nothing from one call into the next.
"""
import numpy as np
import pytest

from paper_2506_04055_amd import synth
from parity import check

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def mlp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_04055_amd import mlp as M
    M.lib()
    return M


def _both(M, d, owner=None):
    """(E, F, U) from mlp_energy_forces, then from the allocation-free entry
    point into fresh output buffers, on the same neighbour handle."""
    import torch
    out = d.compute(atom_energy=True)
    torch.cuda.synchronize()
    ref = (out["energy"].clone(), out["forces"].clone(), out["atom_energy"].clone())
    e = torch.full((1,), np.nan, dtype=torch.float64, device="cuda")
    f = torch.full((3, d.n), np.nan, dtype=torch.float32, device="cuda")
    u = torch.full((d.n,), np.nan, dtype=torch.float32, device="cuda")
    M.mlp_energy_forces_noalloc(d.model.handle, d.nbr, d.pos, d.n_local, e, f, owner, u)
    torch.cuda.synchronize()
    return ref, (e, f, u)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_noalloc_equals_entry_point_two_calls(mlp, oracle, precision):
    import torch
    hdr, w = synth.make_weights(128, 20, 3, 2, seed=0)
    model = mlp.Model(hdr, w, precision)
    # first a 648-atom box, then the smaller 192-atom box on the same GPU
    for n_side in (6, 4):
        s = synth.water_box(n_side, 3.105, seed=n_side)
        d = mlp.System(model, s.pos, s.species, s.box, skin=1.0)
        ref, got = _both(mlp, d)
        print(f"[case] noalloc {precision} water n={s.n_atoms}", flush=True)
        for a, b, name in zip(ref, got, ("energy", "forces", "atom energies")):
            assert torch.equal(a, b), f"{name} differ from mlp_energy_forces (n={s.n_atoms})"
        E_ref, F_ref = oracle.energy_forces(hdr, w, s.pos, s.species, s.box)
        check(f"noalloc water{s.n_atoms}", precision, float(got[0].item()), E_ref,
              got[1].t().cpu().numpy().astype(np.float64), F_ref)
        del d


@pytest.mark.parametrize("kind", ["allegro", "mace"])
def test_noalloc_equivariant_models_two_calls(mlp, kind):
    # the Allegro and MACE paths through the allocation-free entry point: a
    # 192-atom water box, then a smaller 108-atom crystal on the same GPU
    import torch
    make = synth.make_allegro_weights if kind == "allegro" else synth.make_mace_weights
    hdr, w = make(2, seed=4, bias_scale=0.1)
    model = mlp.Model(hdr, w, "fp32")
    for s in (synth.water_box(4, 3.105, seed=3), synth.fcc_crystal(3, seed=5, sigma=0.1)):
        d = mlp.System(model, s.pos, s.species, s.box, skin=1.0)
        print(f"[case] noalloc {kind} n={s.n_atoms}", flush=True)
        ref, got = _both(mlp, d)
        for a, b, name in zip(ref, got, ("energy", "forces", "atom energies")):
            assert torch.equal(a, b), f"{kind}: {name} differ from mlp_energy_forces (n={s.n_atoms})"
        del d


def test_noalloc_ghost_domain_fold(mlp, oracle):
    import torch
    hdr, w = synth.make_weights(32, 8, 2, 1, seed=3)
    model = mlp.Model(hdr, w, "fp32")
    dom = synth.fcc_crystal(4, seed=2, ghost_depth=10.0)
    d = mlp.System(model, dom.pos, dom.species, dom.box, n_local=dom.n_local, skin=0.5, ghost_owner=dom.owner)
    print(f"[case] noalloc ghost domain {dom.n_local} locals, {dom.n_atoms} rows", flush=True)
    # the owner map is prepared by the first mlp_energy_forces call (inside _both)
    ref, got = _both(mlp, d, d.ghost_owner)
    for a, b in zip(ref, got):
        assert torch.equal(a, b)
    E_ref, F_ref = oracle.energy_forces(hdr, w, dom.pos, dom.species, np.zeros(3), n_local=dom.n_local)
    F_ref = oracle.fold_ghost_forces(F_ref, dom.n_local, dom.owner)
    check("noalloc fcc4 ghost domain (folded)", "fp32", float(got[0].item()), E_ref,
          got[1].t().cpu().numpy().astype(np.float64), F_ref)
    # another owner array than the one the map was prepared from: refused
    other = d.ghost_owner.clone()
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    f = torch.zeros(3, d.n, dtype=torch.float32, device="cuda")
    with pytest.raises(mlp.MLPError) as ei:
        mlp.mlp_energy_forces_noalloc(model.handle, d.nbr, d.pos, d.n_local, e, f, other)
    assert ei.value.code == -1 and "owner map" in str(ei.value)


def test_noalloc_rejects_a_system_beyond_the_scratch(mlp):
    import torch
    hdr, w = synth.make_weights(128, 20, 3, 1, seed=0)
    model = mlp.Model(hdr, w, "fp32")
    s = synth.fcc_crystal(12, seed=0)      # 6,912 atoms: more than the array holds at F = 128
    d = mlp.System(model, s.pos, s.species, s.box, skin=0.5)
    e = torch.zeros(1, dtype=torch.float64, device="cuda")
    f = torch.zeros(3, d.n, dtype=torch.float32, device="cuda")
    with pytest.raises(mlp.MLPError) as ei:
        mlp.mlp_energy_forces_noalloc(model.handle, d.nbr, d.pos, d.n_local, e, f)
    assert ei.value.code == -3 and "bytes" in str(ei.value)
    # nothing was enqueued: the outputs are untouched, and the handle still works
    assert float(e.item()) == 0.0
    out = d.compute()
    torch.cuda.synchronize()
    assert np.isfinite(float(out["energy"].item()))
