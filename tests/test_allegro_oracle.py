"""Pins of the single-layer Allegro oracle (oracle/allegro.py) against what
mathematics and the model's structure fix, independent of the oracle's own
arithmetic:

* forces: central finite differences of the energy, per component and along
  random directions; zero net force;
* E(3) invariance: rotations with and without reflection, translation,
  permutation of the atoms;
* periodic replication: a 2x2x2 supercell has 8x the energy and replicated
  forces;
* structure: with the latent MLP switched off, the energy is a sum of pair
  terms, equal to the sum of the energies of the isolated dimers; strict
  locality (moving an atom changes no per-atom energy of atoms farther than
  r_c from it before and after); the envelope vanishes with its first two
  derivatives at r_c, so a pair crossing the cutoff changes the energy
  continuously; atoms without neighbours carry zero energy and force;
* the ghost-domain form (Eq. 1-2): a domain with its ghost shell of depth r_c
  gives the periodic energy, and folded forces give the periodic forces;
* the angular part: the oracle's Legendre polynomials against scipy's, and
  the addition theorem sum_m Y_lm(a) Y_lm(b) = (2l+1) P_l(a.b) that connects
  them with the spherical-harmonic form of the tensor product (scipy's
  complex harmonics turned real).
"""
import math

import numpy as np
import pytest
import torch

from oracle import allegro as A
from oracle import oracle as O
from paper_2506_04055_amd import synth


def _model(S=2, seed=0, bias=0.1):
    return synth.make_allegro_weights(S, seed=seed, bias_scale=bias)


def _cluster(n, extent, S, seed, dmin=1.0):
    """Random open cluster with a minimum distance (float32 positions)."""
    rng = np.random.default_rng(seed)
    pts = []
    while len(pts) < n:
        p = rng.uniform(0, extent, 3)
        if all(np.linalg.norm(p - q) > dmin for q in pts):
            pts.append(p)
    pos = np.array(pts, np.float32)
    return pos, rng.integers(0, S, n).astype(np.int32)


def test_finite_differences_and_net_force():
    h, w = _model(S=2, seed=1)
    pos, Z = _cluster(14, 6.0, 2, seed=3)
    box = np.zeros(3)
    E, F = A.energy_forces(h, w, pos, Z, box)
    p64 = pos.astype(np.float64)
    hstep = 1e-5
    for i in range(0, 14, 3):
        for d in range(3):
            pp, pm = p64.copy(), p64.copy()
            pp[i, d] += hstep
            pm[i, d] -= hstep
            fd = -(A.energy_forces(h, w, pp, Z, box)[0] - A.energy_forces(h, w, pm, Z, box)[0]) / (2 * hstep)
            assert abs(fd - F[i, d]) <= 1e-6 * (1 + abs(F[i, d])), (i, d, fd, F[i, d])
    rng = np.random.default_rng(5)
    for _ in range(3):
        dl = rng.standard_normal(p64.shape)
        fd = (A.energy_forces(h, w, p64 + hstep * dl, Z, box)[0]
              - A.energy_forces(h, w, p64 - hstep * dl, Z, box)[0]) / (2 * hstep)
        assert abs(fd + (F * dl).sum()) <= 1e-6 * (1 + np.abs(F).sum())
    assert np.abs(F.sum(0)).max() <= 1e-10 * np.abs(F).max()


def test_periodic_finite_differences_small_box():
    # a box smaller than 2 r_c: several images of one pair are neighbours
    h, w = _model(S=1, seed=2)
    s = synth.fcc_crystal(2, seed=1, sigma=0.1)
    E, F = A.energy_forces(h, w, s.pos, s.species, s.box)
    p64 = s.pos.astype(np.float64)
    hstep = 1e-5
    rng = np.random.default_rng(1)
    for _ in range(3):
        dl = rng.standard_normal(p64.shape)
        fd = (A.energy_forces(h, w, p64 + hstep * dl, s.species, s.box)[0]
              - A.energy_forces(h, w, p64 - hstep * dl, s.species, s.box)[0]) / (2 * hstep)
        assert abs(fd + (F * dl).sum()) <= 1e-6 * (1 + np.abs(F).sum())


def test_rotation_reflection_translation_permutation():
    h, w = _model(S=3, seed=4)
    pos, Z = _cluster(16, 7.0, 3, seed=8)
    p64 = pos.astype(np.float64)
    box = np.zeros(3)
    E, F = A.energy_forces(h, w, p64, Z, box)
    rng = np.random.default_rng(2)
    for reflect in (False, True):
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        if (np.linalg.det(Q) < 0) != reflect:
            Q[:, 0] *= -1
        q = p64 @ Q.T + np.array([3.0, -1.5, 0.25])
        E2, F2 = A.energy_forces(h, w, q, Z, box)
        assert abs(E2 - E) <= 1e-12 * abs(E)
        assert np.abs(F2 - F @ Q.T).max() <= 1e-11 * np.abs(F).max()
    perm = rng.permutation(16)
    E3, F3 = A.energy_forces(h, w, p64[perm], Z[perm], box)
    assert abs(E3 - E) <= 1e-12 * abs(E)
    assert np.abs(F3 - F[perm]).max() <= 1e-12 * np.abs(F).max()


def test_periodic_replication():
    h, w = _model(S=1, seed=6)
    s1 = synth.fcc_crystal(3, seed=2)
    E1, F1 = A.energy_forces(h, w, s1.pos, s1.species, s1.box)
    # the same crystal repeated twice along each axis
    L = s1.box[0]
    reps = [s1.pos.astype(np.float64) + L * np.array([a, b, c]) for a in range(2) for b in range(2) for c in range(2)]
    p2 = np.concatenate(reps)
    E2, F2 = A.energy_forces(h, w, p2, np.zeros(len(p2), np.int32), 2 * s1.box)
    assert abs(E2 - 8 * E1) <= 1e-11 * abs(E2)
    assert np.abs(F2 - np.tile(F1, (8, 1))).max() <= 1e-10 * np.abs(F1).max()


def _latent_off(h, w):
    w = w.copy()
    o = 0
    for name, shape, _ in synth.allegro_layout(h):
        k = int(np.prod(shape))
        if name.startswith("lat_"):
            w[o:o + k] = 0.0
        o += k
    return w


def test_pair_additivity_without_the_latent_update():
    # with MLP_lat = 0 every edge energy depends on its own pair only, so the
    # cluster energy is the sum over pairs of the isolated dimers' energies
    h, w = _model(S=2, seed=7)
    w0 = _latent_off(h, w)
    pos, Z = _cluster(9, 6.0, 2, seed=11)
    box = np.zeros(3)
    E, _ = A.energy_forces(h, w0, pos, Z, box)
    tot = 0.0
    for i in range(9):
        for j in range(i + 1, 9):
            if np.linalg.norm(pos[i].astype(np.float64) - pos[j]) < h["r_c"]:
                tot += A.energy_forces(h, w0, pos[[i, j]], Z[[i, j]], box)[0]
    assert abs(E - tot) <= 1e-12 * max(1.0, abs(E))
    # with the latent update on, the energy is not pair-additive
    E_on, _ = A.energy_forces(h, w, pos, Z, box)
    tot_on = sum(A.energy_forces(h, w, pos[[i, j]], Z[[i, j]], box)[0]
                 for i in range(9) for j in range(i + 1, 9)
                 if np.linalg.norm(pos[i].astype(np.float64) - pos[j]) < h["r_c"])
    assert abs(E_on - tot_on) > 1e-6 * abs(E_on)


def test_strict_locality():
    h, w = _model(S=2, seed=9)
    pos, Z = _cluster(20, 11.0, 2, seed=12)
    box = np.zeros(3)
    _, _, U = A.energy_forces(h, w, pos, Z, box, per_atom=True)
    p2 = pos.astype(np.float64).copy()
    k = 0
    p2[k] += np.array([0.3, -0.2, 0.1])
    _, _, U2 = A.energy_forces(h, w, p2, Z, box, per_atom=True)
    far = [i for i in range(20) if i != k and np.linalg.norm(pos[i] - pos[k]) > h["r_c"]
           and np.linalg.norm(p2[i] - p2[k]) > h["r_c"]]
    near = [i for i in range(20) if i != k and np.linalg.norm(pos[i] - pos[k]) < h["r_c"] - 0.5]
    assert far and near
    assert np.array_equal(U[far], U2[far])
    assert np.abs(U[near] - U2[near]).max() > 1e-8


def test_envelope_and_cutoff_continuity():
    p = 2
    x = torch.tensor([1.0], dtype=torch.float64, requires_grad=True)
    u = A.envelope(x, p)
    (g,) = torch.autograd.grad(u, x, create_graph=True)
    (g2,) = torch.autograd.grad(g, x)
    assert abs(float(u.detach())) < 1e-15 and abs(float(g.detach())) < 1e-14 and abs(float(g2)) < 1e-13
    assert float(A.envelope(torch.tensor(0.0, dtype=torch.float64), p)) == 1.0
    # a dimer approaching the cutoff from inside: E ~ (r_c - r)^3
    h, w = _model(S=1, seed=3, bias=0.3)
    Z = np.zeros(2, np.int32)
    e = [A.energy_forces(h, w, np.array([[0, 0, 0], [h["r_c"] - dlt, 0, 0]]), Z, np.zeros(3))[0]
         for dlt in (1e-2, 5e-3)]
    assert abs(e[1]) < abs(e[0]) / 6 and abs(e[0]) < 1e-3
    E_out, F_out = A.energy_forces(h, w, np.array([[0, 0, 0], [h["r_c"] + 1e-3, 0, 0]]), Z, np.zeros(3))
    assert E_out == 0.0 and not F_out.any()


def test_ghost_domain_equals_periodic_system():
    h, w = _model(S=1, seed=10)
    s = synth.fcc_crystal(3, seed=4)
    E_p, F_p = A.energy_forces(h, w, s.pos, s.species, s.box)
    dom = synth.fcc_crystal(3, seed=4, ghost_depth=h["r_c"])
    # exact FP64 images (the stored float32 ghost rows are rounded)
    own = s.pos[dom.owner].astype(np.float64)
    shift = np.round((dom.pos[dom.n_local:] - own) / s.box)
    gpos = np.concatenate([s.pos.astype(np.float64), own + shift * s.box])
    E_d, F_d = A.energy_forces(h, w, gpos, dom.species, np.zeros(3), n_local=dom.n_local)
    Ff = O.fold_ghost_forces(F_d, dom.n_local, dom.owner)
    assert abs(E_d - E_p) <= 1e-11 * abs(E_p)
    assert np.abs(Ff[: dom.n_local] - F_p).max() <= 1e-10 * np.abs(F_p).max()


def test_legendre_and_addition_theorem():
    sp = pytest.importorskip("scipy.special")
    t = torch.linspace(-1, 1, 41, dtype=torch.float64)
    for l in range(4):
        assert np.allclose(A.legendre(l, t).numpy(), sp.eval_legendre(l, t.numpy()), atol=1e-14)
    rng = np.random.default_rng(0)
    a, b = rng.standard_normal(3), rng.standard_normal(3)
    a, b = a / np.linalg.norm(a), b / np.linalg.norm(b)

    def real_sh(l, v):
        # component normalisation: sqrt(4 pi) times the orthonormal real harmonics
        th, ph = math.acos(v[2]), math.atan2(v[1], v[0])
        out = []
        for m in range(-l, l + 1):
            # scipy >= 1.15 names it sph_harm_y(l, m, theta, phi); older sph_harm(m, l, phi, theta)
            y = (sp.sph_harm_y(l, abs(m), th, ph) if hasattr(sp, "sph_harm_y") else sp.sph_harm(abs(m), l, ph, th))
            if m < 0:
                val = math.sqrt(2) * (-1) ** m * y.imag
            elif m == 0:
                val = y.real
            else:
                val = math.sqrt(2) * (-1) ** m * y.real
            out.append(math.sqrt(4 * math.pi) * val)
        return np.array(out)

    for l in range(4):
        lhs = float(real_sh(l, a) @ real_sh(l, b))
        rhs = (2 * l + 1) * float(A.legendre(l, torch.tensor(float(a @ b), dtype=torch.float64)))
        assert abs(lhs - rhs) <= 1e-12 * (2 * l + 1)
        assert abs(float(real_sh(l, a) @ real_sh(l, a)) - (2 * l + 1)) <= 1e-12 * (2 * l + 1)


def test_isolated_atoms():
    h, w = _model(S=2, seed=1)
    pos = np.array([[0, 0, 0], [20, 0, 0], [0, 30, 0]], np.float64)
    E, F, U = A.energy_forces(h, w, pos, np.array([0, 1, 0], np.int32), np.zeros(3), per_atom=True)
    assert E == 0.0 and not F.any() and not U.any()
