"""GPU path (through the C ABI) against the FP64 oracle on identical seeded inputs.

Tolerances per precision mode and the per-row force bound are stated in
tests/parity.py.  Neighbour sets are compared with the FP64 brute-force set
(pairs within a float32 rounding band of the cutoff may differ and are
counted); hop counts are compared exactly on the device's graph.
"""
import json
import os

import numpy as np
import pytest

from paper_2506_04055_amd import synth
from parity import ROW, TOL, check, check_neighbors_fp64, rel_rms, row_err

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
MODES = ["fp32", "bf16", "bf16_node", "bf16_node_x3", "bf16_fast"]

_ORACLE = {}


def oracle_cached(oracle, key, *args, **kw):
    """Oracle results shared by the tests of this module (same inputs)."""
    if key not in _ORACLE:
        _ORACLE[key] = oracle.energy_forces(*args, **kw)
    return _ORACLE[key]


@pytest.fixture(scope="module")
def mlp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2506_04055_amd import mlp as M
    M.lib()
    return M


def run_gpu(M, sysm, hdr, w, precision="fp32", skin=1.0, stats=False, atom_energy=False, fold=True):
    import torch
    model = M.Model(hdr, w, precision)
    owner = sysm.owner if (fold and sysm.n_atoms > sysm.n_local) else None
    d = M.System(model, sysm.pos, sysm.species, sysm.box, n_local=sysm.n_local, skin=skin, ghost_owner=owner)
    out = d.compute(stats=stats, atom_energy=atom_energy)
    torch.cuda.synchronize()
    res = {"E": float(out["energy"].item()), "F": out["forces"].t().cpu().numpy().astype(np.float64),
           "sys": d, "model": model}
    if stats:
        res["stats"] = out["stats"]
    if atom_energy:
        res["U"] = out["atom_energy"].cpu().numpy().astype(np.float64)
    return res


# ------------------------------------------------------------------ graph

def test_neighbor_graph_fp64(mlp, oracle):
    # skin graph and pruned graph of a periodic water box against the FP64
    # brute-force sets; the float32 pair rule of the header is also checked
    # exactly (a secondary check of the stated formula)
    s = synth.water_box(4, 3.105, seed=0)
    hdr, w = synth.make_weights(32, 8, 2, 2, seed=0)
    model = mlp.Model(hdr, w)
    d = mlp.System(model, s.pos, s.species, s.box, skin=1.0)
    dst, src = mlp.mlp_nbr_edges(d.nbr, 0)
    check_neighbors_fp64(oracle, "water192 rc+skin", dst, src, s.pos, s.box, 6.0, s.box.max())
    od, os_ = oracle.neighbors_f32(s.pos, s.box.astype(np.float32), 5.0, 1.0)
    assert np.array_equal(dst, od) and np.array_equal(src, os_)
    d.compute()
    dst, src = mlp.mlp_nbr_edges(d.nbr, 1)
    check_neighbors_fp64(oracle, "water192 rc", dst, src, s.pos, s.box, 5.0, s.box.max())


def test_neighbor_graph_fp64_open_domain(mlp, oracle):
    # many cells per dimension, open box with explicit ghosts
    s = synth.fcc_crystal(4, seed=2, ghost_depth=6.0)
    hdr, w = synth.make_weights(32, 8, 1, 1, seed=0)
    model = mlp.Model(hdr, w)
    d = mlp.System(model, s.pos, s.species, s.box, n_local=s.n_local, skin=0.5)
    dst, src = mlp.mlp_nbr_edges(d.nbr, 0)
    cmax = float(np.abs(s.pos).max())
    check_neighbors_fp64(oracle, "fcc4 ghost rc+skin", dst, src, s.pos, np.zeros(3), 5.5, cmax)
    d.compute()
    dst, src = mlp.mlp_nbr_edges(d.nbr, 1)
    check_neighbors_fp64(oracle, "fcc4 ghost rc", dst, src, s.pos, np.zeros(3), 5.0, cmax)


def test_neighbor_graph_fp64_24k(mlp, oracle):
    # the benchmark box: the pruned graph of 1.3M edges against FP64
    s, hdr, w = synth.workload("water24k")
    model = mlp.Model(hdr, w)
    d = mlp.System(model, s.pos, s.species, s.box, skin=1.0)
    d.compute()
    dst, src = mlp.mlp_nbr_edges(d.nbr, 1)
    check_neighbors_fp64(oracle, "water24k rc", dst, src, s.pos, s.box, 5.0, s.box.max())


def test_neighbor_counts_on_fcc_shells(mlp):
    # perfect fcc (a = 4.05, 6^3 cells): every atom has the textbook shell
    # counts within rc + skin = 6 A (shells 1-4) and, after pruning, within
    # rc = 5 A (shells 1-3); lattice sites sit exactly on cell boundaries
    with open(os.path.join(GOLDEN, "lattice_shells.json")) as f:
        cnt = json.load(f)["fcc"]["count"]
    s = synth.fcc_crystal(6, sigma=0.0)
    hdr, w = synth.make_weights(32, 8, 1, 1, seed=0)
    model = mlp.Model(hdr, w)
    d = mlp.System(model, s.pos, s.species, s.box, skin=1.0)
    dst, src = mlp.mlp_nbr_edges(d.nbr, 0)
    assert np.all(np.bincount(dst, minlength=s.n_atoms) == sum(cnt[:4]))
    d.compute()
    dst, src = mlp.mlp_nbr_edges(d.nbr, 1)
    assert np.all(np.bincount(dst, minlength=s.n_atoms) == sum(cnt[:3]))


# ------------------------------------------------------------------ small systems

def test_water192_energy_forces(mlp, oracle):
    s, hdr, w = synth.workload("water192")
    E_ref, F_ref = oracle.energy_forces(hdr, w, s.pos, s.species, s.box)
    r = run_gpu(mlp, s, hdr, w)
    check("water192", "fp32", r["E"], E_ref, r["F"], F_ref)


@pytest.mark.parametrize("precision", MODES)
def test_water192_against_stored_oracle(mlp, precision):
    # the oracle's stored result (tests/golden/oracle_water192.json)
    with open(os.path.join(GOLDEN, "oracle_water192.json")) as f:
        ref = json.load(f)
    s, hdr, w = synth.workload("water192")
    r = run_gpu(mlp, s, hdr, w, precision=precision)
    check("water192 (stored oracle)", precision, r["E"], ref["energy"], r["F"], np.array(ref["forces"], np.float64))


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_biases_and_four_species(mlp, oracle, precision):
    # four species and non-zero biases; F = 64 with four species takes the
    # unfactorised first layer (its matrices do not fit the borrowed rows)
    s = synth.peptide_like(700, seed=3)
    hdr, w = synth.make_weights(64, 20, 3, 4, seed=4, bias_scale=0.2)
    E_ref, F_ref = oracle_cached(oracle, "pep700", hdr, w, s.pos, s.species, s.box)
    r = run_gpu(mlp, s, hdr, w, precision=precision, skin=0.7)
    check("peptide700 S=4 F=64", precision, r["E"], E_ref, r["F"], F_ref)


def test_bench_model_ragged_size(mlp, oracle):
    # the benchmark's model (T=3, F=128, K=20) on 648 atoms: several GEMM
    # tiles plus a ragged tail
    s = synth.water_box(6, 3.105, seed=7)
    hdr, w = synth.make_weights(128, 20, 3, 2, seed=7)
    E_ref, F_ref, U_ref = oracle.energy_forces(hdr, w, s.pos, s.species, s.box, per_atom=True)
    r = run_gpu(mlp, s, hdr, w, atom_energy=True)
    check("water648 F=128", "fp32", r["E"], E_ref, r["F"], F_ref)
    assert np.abs(r["U"] - U_ref).max() <= 1e-5 * np.abs(U_ref).max()


# ------------------------------------------------------------------ full-size water, every precision mode

@pytest.mark.parametrize("precision", MODES)
def test_full_size_24k_water(mlp, oracle, precision):
    # the benchmark's workload at full size, every output compared
    s, hdr, w = synth.workload("water24k")
    E_ref, F_ref = oracle_cached(oracle, "water24k", hdr, w, s.pos, s.species, s.box)
    r = run_gpu(mlp, s, hdr, w, precision=precision, stats=True)
    check("water24k", precision, r["E"], E_ref, r["F"], F_ref)


# ------------------------------------------------------------------ ghost domains

def _hops_on_device_graph(mlp, oracle, r, dom, T):
    # hop counts (integer work): the device's hop sets against the oracle's
    # hop count on the same pruned graph, exactly
    dst, src = mlp.mlp_nbr_edges(r["sys"].nbr, 1)
    hops = oracle.hops(dom.n_atoms, dom.n_local, dst, src, T)
    cum = np.cumsum(np.bincount(hops, minlength=T + 2))
    assert r["stats"]["n_within_hops"][: T + 1] == cum[: T + 1].tolist()
    return dst, src


def test_ghost_domain_and_fold(mlp, oracle):
    # one domain's share: locals + a T*rc ghost shell, open boundaries
    hdr, w = synth.make_weights(128, 20, 3, 1, seed=9, bias_scale=0.1)
    dom = synth.fcc_crystal(4, seed=3, ghost_depth=15.0)
    per = synth.fcc_crystal(4, seed=3)
    E_ref, F_ref = oracle.energy_forces(hdr, w, dom.pos, dom.species, np.zeros(3), n_local=dom.n_local)
    r = run_gpu(mlp, dom, hdr, w, skin=0.5, stats=True)
    # ghost rows keep their partial forces; local rows hold the folded sums
    folded_ref = oracle.fold_ghost_forces(F_ref, dom.n_local, dom.owner)
    check("fcc4 ghost domain (folded)", "fp32", r["E"], E_ref, r["F"], folded_ref)
    # folded local forces equal the periodic system's forces (Eq. 2)
    Ep, Fp = oracle.energy_forces(hdr, w, per.pos, per.species, per.box)
    assert rel_rms(r["F"][: dom.n_local], Fp) <= 1e-4   # ghost rows are float32-rounded images
    dst, src = _hops_on_device_graph(mlp, oracle, r, dom, 3)
    check_neighbors_fp64(oracle, "fcc4 ghost15 rc", dst, src, dom.pos, np.zeros(3), 5.0, float(np.abs(dom.pos).max()))


@pytest.fixture(scope="module")
def fcc12_domain(oracle):
    # 12^3 cells (6,912 locals) + the 15 A shell: 31k rows, many workgroups
    # per XCD in every kernel, oracle-feasible on every row
    hdr, w = synth.make_weights(128, 20, 3, 1, seed=21, bias_scale=0.1)
    dom = synth.fcc_crystal(12, seed=5, ghost_depth=15.0)
    E_ref, F_ref, U_ref = oracle.energy_forces(hdr, w, dom.pos, dom.species, np.zeros(3), n_local=dom.n_local,
                                               per_atom=True)
    return dom, hdr, w, E_ref, F_ref, U_ref


@pytest.mark.parametrize("precision", ["fp32", "bf16", "bf16_node"])
def test_ghost_domain_12cells_every_row(mlp, oracle, fcc12_domain, precision):
    dom, hdr, w, E_ref, F_ref, U_ref = fcc12_domain
    r = run_gpu(mlp, dom, hdr, w, precision=precision, skin=0.5, stats=True, atom_energy=True, fold=False)
    print(f"[info] fcc12 domain: {dom.n_local} locals, {dom.n_atoms} rows, {r['stats']['n_edges']} edges, "
          f"hop sets {r['stats']['n_within_hops'][:4]}")
    # raw partial forces on every row (locals and ghosts) and per-atom energies
    check("fcc12 ghost domain (raw rows)", precision, r["E"], E_ref, r["F"], F_ref)
    et, _ = TOL[precision]
    u_scale = np.abs(U_ref[: dom.n_local]).mean()
    du = np.abs(r["U"][: dom.n_local] - U_ref[: dom.n_local]).max() / u_scale
    print(f"[measured] fcc12 {precision}: per-atom energy max |dU|/mean|U| {du:.2e}")
    assert du <= ROW * et
    if precision == "fp32":
        dst, src = _hops_on_device_graph(mlp, oracle, r, dom, 3)
        check_neighbors_fp64(oracle, "fcc12 ghost15 rc", dst, src, dom.pos, np.zeros(3), 5.0,
                             float(np.abs(dom.pos).max()))
    # the fold on the same handle: ghost rows unchanged, local rows folded
    import torch
    d = r["sys"]
    d.ghost_owner = torch.as_tensor(dom.owner).cuda()
    d.compute()
    torch.cuda.synchronize()
    Ff = d.forces.t().cpu().numpy().astype(np.float64)
    assert np.array_equal(Ff[dom.n_local:], r["F"][dom.n_local:])
    check("fcc12 ghost domain (folded)", precision, r["E"], E_ref, Ff,
          oracle.fold_ghost_forces(F_ref, dom.n_local, dom.owner))


def test_bad_ghost_owner_fails_without_stats(mlp):
    import torch
    hdr, w = synth.make_weights(32, 8, 2, 1, seed=0)
    dom = synth.fcc_crystal(4, seed=3, ghost_depth=10.0)
    model = mlp.Model(hdr, w)
    d = mlp.System(model, dom.pos, dom.species, dom.box, n_local=dom.n_local, skin=0.5)
    bad = dom.owner.copy()
    bad[len(bad) // 2] = dom.n_local          # one past the last local atom
    d.ghost_owner = torch.as_tensor(bad).cuda()
    with pytest.raises(mlp.MLPError) as e:
        d.compute(stats=False)
    assert e.value.code == -1
    bad[len(bad) // 2] = -1
    d.ghost_owner = torch.as_tensor(bad).cuda()
    with pytest.raises(mlp.MLPError) as e:
        d.compute(stats=False)
    assert e.value.code == -1
    # a valid owner array on the same handle works afterwards
    d.ghost_owner = torch.as_tensor(dom.owner).cuda()
    d.compute()
    torch.cuda.synchronize()
    assert np.isfinite(d.forces.cpu().numpy()).all()


# ------------------------------------------------------------------ the aluminium MD model

@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_al_model_config(mlp, oracle, precision):
    # the model of the aluminium protocol and the capacity point (F = 64,
    # K = 20, T = 4, one species, factorised first layer, radial filter and
    # readout scaled for MD) on a perturbed 500-atom fcc box with skin 2 A
    _, hdr, w = synth.al_nvt_workload(5)
    s = synth.fcc_crystal(5, a=4.065, sigma=0.05, seed=13)
    E_ref, F_ref = oracle_cached(oracle, "al500", hdr, w, s.pos, s.species, s.box)
    r = run_gpu(mlp, s, hdr, w, precision=precision, skin=2.0)
    check("al500 F=64 T=4", precision, r["E"], E_ref, r["F"], F_ref)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_al_model_ghost_domain(mlp, oracle, precision):
    # the same model on a domain share with a T*rc = 20 A ghost shell, folded
    _, hdr, w = synth.al_nvt_workload(5)
    dom = synth.fcc_crystal(5, a=4.065, sigma=0.05, seed=13, ghost_depth=20.0)
    E_ref, F_ref = oracle_cached(oracle, "al500_ghost", hdr, w, dom.pos, dom.species, np.zeros(3),
                                 n_local=dom.n_local)
    r = run_gpu(mlp, dom, hdr, w, precision=precision, skin=2.0)
    check("al500 ghost20 (folded)", precision, r["E"], E_ref, r["F"],
          oracle.fold_ghost_forces(F_ref, dom.n_local, dom.owner))


# ------------------------------------------------------------------ special cases

def test_isolated_atoms_and_single_atom(mlp, oracle):
    hdr, w = synth.make_weights(32, 8, 2, 3, seed=1, bias_scale=0.3)
    pos = np.array([[1.0, 1.0, 1.0], [10.0, 1.0, 1.0], [1.0, 12.0, 1.0], [15.0, 15.0, 15.0]], np.float32)
    sp = np.array([0, 1, 2, 1], np.int32)
    box = np.array([30.0, 30.0, 30.0])
    s = synth.System(pos, sp, box, 4)
    E_ref, F_ref = oracle.energy_forces(hdr, w, pos, sp, box)
    r = run_gpu(mlp, s, hdr, w)
    assert abs(r["E"] - E_ref) <= TOL["fp32"][0] * abs(E_ref)
    assert np.all(r["F"] == 0.0)
    s1 = synth.System(pos[:1], sp[:1], box, 1)
    E1, _ = oracle.energy_forces(hdr, w, pos[:1], sp[:1], box)
    r1 = run_gpu(mlp, s1, hdr, w)
    assert abs(r1["E"] - E1) <= TOL["fp32"][0] * abs(E1) and np.all(r1["F"] == 0.0)


def test_permutation_and_determinism(mlp):
    s, hdr, w = synth.workload("water192")
    r = run_gpu(mlp, s, hdr, w)
    r2 = run_gpu(mlp, s, hdr, w)
    assert r["E"] == r2["E"] and np.array_equal(r["F"], r2["F"])   # bitwise reproducible
    perm = np.random.default_rng(0).permutation(s.n_atoms)
    sp = synth.System(s.pos[perm], s.species[perm], s.box, s.n_atoms)
    r3 = run_gpu(mlp, sp, hdr, w)
    assert abs(r3["E"] - r["E"]) <= 1e-6 * abs(r["E"])
    assert rel_rms(r3["F"], r["F"][perm]) <= 1e-6 and row_err(r3["F"], r["F"][perm]) <= 2e-5


def test_capacity_growth_on_one_handle(mlp, oracle):
    import torch
    hdr, w = synth.make_weights(32, 8, 2, 2, seed=2)
    model = mlp.Model(hdr, w)
    small = synth.water_box(4, 3.105, seed=1)
    big = synth.water_box(5, 3.105, seed=2)
    d = mlp.System(model, small.pos, small.species, small.box, skin=0.5)
    d.compute()
    # rebuild the same handle with a larger system: buffers grow, results stay exact
    d.n = big.n_atoms
    d.n_local = big.n_atoms
    d.pos = torch.as_tensor(big.pos).t().contiguous().cuda()
    d.species = torch.as_tensor(big.species).cuda()
    d.box = list(big.box)
    d.forces = torch.zeros(3, big.n_atoms, device="cuda")
    d.build()
    out = d.compute(stats=True)
    E_ref, F_ref = oracle.energy_forces(hdr, w, big.pos, big.species, big.box)
    assert out["stats"]["n_grows"] > 0 and out["stats"]["n_builds"] == 2
    check("water375 regrown", "fp32", out["energy"].item(), E_ref,
          out["forces"].t().cpu().numpy().astype(np.float64), F_ref)


def test_invalid_arguments(mlp):
    hdr, w = synth.make_weights(32, 8, 2, 2, seed=0)
    with pytest.raises(mlp.MLPError) as e:
        mlp.Model(hdr, w[:-1])
    assert e.value.code == -1
    with pytest.raises(mlp.MLPError) as e:
        mlp.Model(hdr, w, 9)                  # unknown precision mode
    assert e.value.code == -1
    model = mlp.Model(hdr, w)
    s = synth.water_box(4, 3.105, seed=0)
    bad = s.species.copy()
    bad[3] = 7
    with pytest.raises(mlp.MLPError) as e:
        mlp.System(model, s.pos, bad, s.box)
    assert e.value.code == -1
    with pytest.raises(mlp.MLPError) as e:
        mlp.System(model, s.pos, s.species, s.box, skin=1.5)   # 6.5 >= 12.42 / 2
    assert e.value.code == -4
    d = mlp.System(model, s.pos, s.species, s.box)
    with pytest.raises(mlp.MLPError) as e:
        mlp.mlp_energy_forces(model.handle, d.nbr, d.pos[:, :100].contiguous(), 100, d.energy)
    assert e.value.code == -1


def test_autograd_function(mlp, oracle):
    s, hdr, w = synth.workload("water192")
    model = mlp.Model(hdr, w)
    d = mlp.System(model, s.pos, s.species, s.box)
    x = d.pos.clone().requires_grad_(True)
    E = mlp.MLPEnergy.apply(x, d)
    E.backward()
    E_ref, F_ref = oracle.energy_forces(hdr, w, s.pos, s.species, s.box)
    check("water192 autograd", "fp32", float(E.item()), E_ref, -x.grad.t().cpu().numpy().astype(np.float64), F_ref)


def test_autograd_after_a_move_beyond_half_skin(mlp, oracle):
    # positions moved by more than skin/2 since the build: the function
    # rebuilds the graph first, so pairs that entered rc are seen
    import torch
    s, hdr, w = synth.workload("water192")
    model = mlp.Model(hdr, w)
    d = mlp.System(model, s.pos, s.species, s.box, skin=0.4)
    rng = np.random.default_rng(5)
    moved = s.pos.astype(np.float64) + rng.uniform(-0.35, 0.35, s.pos.shape)
    moved = np.mod(moved, s.box).astype(np.float32)
    assert mlp.mlp_nbr_check_displacement(d.nbr, torch.as_tensor(moved).t().contiguous().cuda())
    x = torch.as_tensor(moved).t().contiguous().cuda().requires_grad_(True)
    E = mlp.MLPEnergy.apply(x, d)
    E.backward()
    E_ref, F_ref = oracle.energy_forces(hdr, w, moved, s.species, s.box)
    check("water192 moved", "fp32", float(E.item()), E_ref, -x.grad.t().cpu().numpy().astype(np.float64), F_ref)
    # and the same positions again: no rebuild is due
    assert not mlp.mlp_nbr_check_displacement(d.nbr, x.detach())
