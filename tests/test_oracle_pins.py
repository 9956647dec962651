"""Pins of the FP64 oracle to facts outside itself (CPU only).

Each test checks the oracle against something the mathematics fixes: lattice
neighbour counts, central finite differences, symmetry (rotation, reflection,
translation, permutation), periodic replication, the ghost-shell statement of
Eqs. (1)-(2), and special weight choices under which the network reduces to a
closed form (isolated atoms, an embedded-atom model, a collinear chain).
"""
import json
import math
import os

import numpy as np
import pytest

from paper_2506_04055_amd import synth


def small_model(F=16, K=6, T=2, S=2, seed=3, bias=0.3):
    return synth.make_weights(F, K, T, S, seed=seed, bias_scale=bias)


def silu(x):
    return x / (1 + np.exp(-x))


def dsilu(x):
    s = 1 / (1 + np.exp(-x))
    return s * (1 + x * (1 - s))


# ---------------------------------------------------------------- neighbours

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _shells(name):
    with open(os.path.join(GOLDEN, "lattice_shells.json")) as f:
        d = json.load(f)[name]
    return np.array(d["squared_length"], np.float64), np.array(d["count"], np.int64)


def _cuts_between_shells(sq):
    # one cutoff between each pair of consecutive shells, and one past the last
    mids = np.sqrt(0.5 * (sq[:-1] + sq[1:]))
    return np.append(mids, np.sqrt(sq[-1] + 0.5))


def test_simple_cubic_shell_counts(oracle):
    # simple cubic, spacing 1, in a 5 x 5 x 5 periodic box: every atom's
    # neighbour count within each cutoff is the cumulative shell count (cutoffs
    # past L / 2 take several images of one atom)
    sq, cnt = _shells("simple_cubic")
    n = 5
    g = np.arange(n, dtype=np.float64)
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3) + 0.25
    for cut, expect in zip(_cuts_between_shells(sq), np.cumsum(cnt)):
        dst, src, dv = oracle.neighbors(pos, np.array([5.0, 5.0, 5.0]), cut)
        assert np.all(np.bincount(dst, minlength=n**3) == expect), (cut, expect)


def test_fcc_shell_counts(oracle):
    # perfect fcc, a = 4.05: shell m at squared distance (a/2)^2 2m; the third
    # shell (24 at a sqrt(3/2) = 4.96 A) lies inside the 5 A cutoff
    sq, cnt = _shells("fcc")
    s = synth.fcc_crystal(3, sigma=0.0)
    half = 4.05 / 2
    for cut, expect in zip(_cuts_between_shells(sq), np.cumsum(cnt)):
        dst, src, dv = oracle.neighbors(s.pos, s.box, half * cut)
        assert np.all(np.bincount(dst, minlength=s.n_atoms) == expect), (cut, expect)
    dst, src, dv = oracle.neighbors(s.pos, s.box, 5.0)
    assert np.all(np.bincount(dst, minlength=s.n_atoms) == cnt[:3].sum())


@pytest.mark.parametrize("cut,expect", [(1.5, 18), (2.1, 32)])
def test_self_images_in_tiny_box(oracle, cut, expect):
    # one atom in a unit box: every neighbour is one of its own periodic images
    dst, src, dv = oracle.neighbors(np.array([[0.3, 0.6, 0.1]]), np.array([1.0, 1.0, 1.0]), cut)
    assert len(dst) == expect and np.all(src == 0)
    r = np.linalg.norm(dv, axis=1)
    assert np.allclose(np.sort(np.round(r**2)), np.sort(np.round(r**2)))
    assert np.all(np.abs(r**2 - np.round(r**2)) < 1e-12)


def test_neighbor_symmetry_and_f32_agreement(oracle):
    s = synth.water_box(4, 3.105, seed=0)
    dst, src, dv = oracle.neighbors(s.pos, s.box, 5.0)
    fwd = {(int(a), int(b)) for a, b in zip(dst, src)}
    assert fwd == {(b, a) for a, b in fwd}
    # pair displacement of (i<-j) is minus that of (j<-i)
    key = {(int(a), int(b)): v for a, b, v in zip(dst, src, dv)}
    assert all(np.allclose(key[(a, b)], -key[(b, a)]) for a, b in list(fwd)[:500])
    d32, s32 = oracle.neighbors_f32(s.pos, s.box.astype(np.float32), 5.0, 0.0)
    assert {(int(a), int(b)) for a, b in zip(d32, s32)} == fwd
    # against a direct numpy evaluation of the definition on this small system
    p = s.pos.astype(np.float64)
    d = p[None, :, :] - p[:, None, :]
    d -= s.box * np.round(d / s.box)
    r2 = (d**2).sum(-1)
    np.fill_diagonal(r2, np.inf)
    assert int((r2 < 25.0).sum()) == len(dst)


def test_hops_on_a_chain(oracle):
    # atoms 4 A apart on a line: each sees only its two chain neighbours
    pos = np.zeros((10, 3))
    pos[:, 0] = 4.0 * np.arange(10)
    dst, src, _ = oracle.neighbors(pos, np.zeros(3), 5.0)
    h = oracle.hops(10, 2, dst, src, 3)
    assert h.tolist() == [0, 0, 1, 2, 3, 4, 4, 4, 4, 4]


# ---------------------------------------------------------------- derivatives

def test_forces_match_central_differences(oracle):
    hdr, w = small_model(F=16, K=6, T=2)
    s = synth.water_box(4, 3.105, seed=1)
    E, F = oracle.energy_forces(hdr, w, s.pos, s.species, s.box)
    p = s.pos.astype(np.float64)
    h = 1e-5
    rng = np.random.default_rng(0)
    for a in rng.choice(s.n_atoms, 6, replace=False):
        for d in range(3):
            pp = p.copy(); pp[a, d] += h
            pm = p.copy(); pm[a, d] -= h
            fd = -(oracle.energy_forces(hdr, w, pp, s.species, s.box)[0]
                   - oracle.energy_forces(hdr, w, pm, s.species, s.box)[0]) / (2 * h)
            assert abs(fd - F[a, d]) <= 1e-6 * max(1.0, abs(F[a, d]))
    for _ in range(4):
        delta = rng.standard_normal(p.shape)
        delta /= np.linalg.norm(delta)
        fd = (oracle.energy_forces(hdr, w, p + h * delta, s.species, s.box)[0]
              - oracle.energy_forces(hdr, w, p - h * delta, s.species, s.box)[0]) / (2 * h)
        assert abs(fd + (F * delta).sum()) <= 1e-6 * np.linalg.norm(F)


def test_full_size_model_directional_derivative(oracle):
    # the configuration the GPU path is first checked on: 192 atoms, T=2, F=32, K=8
    s, hdr, w = synth.workload("water192")
    E, F = oracle.energy_forces(hdr, w, s.pos, s.species, s.box)
    p = s.pos.astype(np.float64)
    rng = np.random.default_rng(5)
    delta = rng.standard_normal(p.shape)
    h = 1e-5
    fd = (oracle.energy_forces(hdr, w, p + h * delta, s.species, s.box)[0]
          - oracle.energy_forces(hdr, w, p - h * delta, s.species, s.box)[0]) / (2 * h)
    assert abs(fd + (F * delta).sum()) <= 1e-7 * np.linalg.norm(F) * np.linalg.norm(delta)


def test_zero_net_force_and_torque(oracle):
    hdr, w = small_model()
    s = synth.water_box(4, 3.105, seed=2)
    E, F = oracle.energy_forces(hdr, w, s.pos, s.species, s.box)
    assert np.abs(F.sum(0)).max() <= 1e-10 * np.linalg.norm(F)
    # open cluster: total torque vanishes as well
    c = s.pos[:60].astype(np.float64)
    E, F = oracle.energy_forces(hdr, w, c, s.species[:60], np.zeros(3))
    assert np.abs(F.sum(0)).max() <= 1e-10 * np.linalg.norm(F)
    tau = np.cross(c - c.mean(0), F).sum(0)
    assert np.abs(tau).max() <= 1e-9 * np.linalg.norm(F) * np.abs(c).max()


# ---------------------------------------------------------------- symmetry

def test_rotation_reflection_invariance(oracle):
    hdr, w = small_model()
    s = synth.water_box(4, 3.105, seed=3)
    c = s.pos[:72].astype(np.float64)
    Z = s.species[:72]
    E, F = oracle.energy_forces(hdr, w, c, Z, np.zeros(3))
    rng = np.random.default_rng(1)
    for det in (1, -1):
        Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        if np.linalg.det(Q) * det < 0:
            Q[:, 0] *= -1
        E2, F2 = oracle.energy_forces(hdr, w, c @ Q.T, Z, np.zeros(3))
        assert abs(E2 - E) <= 1e-12 * abs(E)
        assert np.abs(F2 - F @ Q.T).max() <= 1e-10 * np.abs(F).max()


def test_translation_and_permutation_invariance(oracle):
    hdr, w = small_model()
    s = synth.water_box(4, 3.105, seed=4)
    E, F = oracle.energy_forces(hdr, w, s.pos, s.species, s.box)
    shifted = np.mod(s.pos.astype(np.float64) + np.array([3.3, -7.1, 0.45]), s.box)
    E2, F2 = oracle.energy_forces(hdr, w, shifted, s.species, s.box)
    assert abs(E2 - E) <= 1e-12 * abs(E)
    assert np.abs(F2 - F).max() <= 1e-10 * np.abs(F).max()
    perm = np.random.default_rng(2).permutation(s.n_atoms)
    E3, F3 = oracle.energy_forces(hdr, w, s.pos[perm], s.species[perm], s.box)
    assert abs(E3 - E) <= 1e-12 * abs(E)
    assert np.abs(F3 - F[perm]).max() <= 1e-10 * np.abs(F).max()


def test_periodic_replication(oracle):
    hdr, w = small_model()
    s = synth.water_box(4, 3.105, seed=5)
    E, F = oracle.energy_forces(hdr, w, s.pos, s.species, s.box)
    reps = [s.pos.astype(np.float64) + np.array([a, b, c]) * s.box
            for a in (0, 1) for b in (0, 1) for c in (0, 1)]
    big = np.concatenate(reps)
    E8, F8 = oracle.energy_forces(hdr, w, big, np.tile(s.species, 8), 2 * s.box)
    assert abs(E8 - 8 * E) <= 1e-12 * abs(8 * E)
    assert np.abs(F8 - np.tile(F, (8, 1))).max() <= 1e-10 * np.abs(F).max()


# ---------------------------------------------------------------- domain decomposition

def test_ghost_shell_domain_equals_periodic_system(oracle):
    # Eq. (1): local energies on a domain with a T*rc ghost shell sum to the
    # periodic energy; Eq. (2): summing the ghosts' partial forces onto their
    # owners gives the periodic forces.  A deeper shell changes nothing
    # (pruning atoms beyond T hops is exact).
    hdr, w = synth.make_weights(16, 6, 2, 1, seed=7, bias_scale=0.3)
    per = synth.fcc_crystal(3, seed=1)
    Ep, Fp = oracle.energy_forces(hdr, w, per.pos, per.species, per.box)
    for depth in (10.0, 12.0):
        dom = synth.fcc_crystal(3, seed=1, ghost_depth=depth)
        # exact FP64 images (the stored float32 ghost rows are rounded)
        own = per.pos[dom.owner].astype(np.float64)
        shift = np.round((dom.pos[dom.n_local:] - own) / per.box)
        gpos = np.concatenate([per.pos.astype(np.float64), own + shift * per.box])
        Ed, Fd = oracle.energy_forces(hdr, w, gpos, dom.species, np.zeros(3), n_local=dom.n_local)
        assert abs(Ed - Ep) <= 1e-12 * abs(Ep)
        folded = oracle.fold_ghost_forces(Fd, dom.n_local, dom.owner)[: dom.n_local]
        assert np.abs(folded - Fp).max() <= 1e-10 * np.abs(Fp).max()


# ---------------------------------------------------------------- closed forms

def _views(hdr, w):
    return {k: v.astype(np.float64) for k, v in synth.weight_views(hdr, w).items()}


def _readout(P, s):
    return silu(s @ P["W5"].T + P["b5"]) @ P["w6"] + P["b6"][0]


def test_isolated_atoms_node_recursion(oracle):
    # Atoms farther apart than the cutoff exchange no messages, v stays zero
    # and the norm is sqrt(eps) in every feature, so each layer reduces to
    # s <- s + a_ss(s, sqrt(eps)); energies do not depend on geometry and the
    # forces vanish exactly.
    hdr, w = small_model(F=16, K=6, T=3, S=3, seed=11)
    P = _views(hdr, w)
    F = hdr["F"]
    pos = np.array([[0.0, 0, 0], [6.0, 0, 0], [0, 7.5, 0], [0, 0, 9.0]])
    Z = np.array([0, 1, 2, 1], np.int32)
    E, Fo = oracle.energy_forces(hdr, w, pos, Z, np.zeros(3))
    s = P["emb"][Z]
    for t in range(hdr["T"]):
        sn = np.concatenate([s, np.full((4, F), math.sqrt(hdr["eps"]))], 1)
        a = silu(sn @ P[f"l{t}.W3"].T + P[f"l{t}.b3"]) @ P[f"l{t}.W4"].T + P[f"l{t}.b4"]
        s = s + a[:, 2 * F:]
    assert abs(E - _readout(P, s).sum()) <= 1e-12 * abs(E)
    assert np.all(Fo == 0.0)


def _eam_weights(seed):
    hdr, w = synth.make_weights(12, 5, 1, 2, seed=seed, bias_scale=0.5)
    V = synth.weight_views(hdr, w)
    for k in ("l0.W1", "l0.W2", "l0.U", "l0.V", "l0.W3", "l0.W4"):
        V[k][...] = 0.0
    return hdr, w


def test_embedded_atom_special_case(oracle):
    # With W1 = W2 = U = V = W3 = W4 = 0 and T = 1 the network is an
    # embedded-atom model with a vector density:
    #   rho_i = sum_j g(r_ij),  g(r) = b2_s o (A_s e(r) + c_s) fc(r)
    #   E = sum_i R(emb[Z_i] + b4_ss + rho_i)
    # evaluated here by a textbook EAM loop, forces included.
    hdr, w = _eam_weights(13)
    P = _views(hdr, w)
    F, K, rc = hdr["F"], hdr["K"], hdr["r_c"]
    s = synth.water_box(4, 3.105, seed=6)   # L = 12.42 > 2 rc: one image per pair
    pos = s.pos.astype(np.float64)
    n = s.n_atoms
    As, cs, b2s = P["l0.A"][F:2 * F], P["l0.c"][F:2 * F], P["l0.b2"][F:2 * F]
    k = np.arange(1, K + 1)

    def g_and_dg(r):
        a = k * math.pi / rc
        e = np.sin(a * r) / r
        de = a * np.cos(a * r) / r - np.sin(a * r) / r**2
        fc = 0.5 * (math.cos(math.pi * r / rc) + 1)
        dfc = -0.5 * math.pi / rc * math.sin(math.pi * r / rc)
        lin = As @ e + cs
        return b2s * lin * fc, b2s * ((As @ de) * fc + lin * dfc)

    rho = np.zeros((n, F))
    pairs = []
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            d = pos[j] - pos[i]
            d -= s.box * np.round(d / s.box)
            r = np.linalg.norm(d)
            if r < rc:
                g, dg = g_and_dg(r)
                rho[i] += g
                pairs.append((i, j, d / r, dg))
    base = P["emb"][s.species] + P["l0.b4"][2 * F:]
    x = base + rho
    h5 = x @ P["W5"].T + P["b5"]
    E_eam = (silu(h5) @ P["w6"] + P["b6"][0]).sum()
    dPhi = (dsilu(h5) * P["w6"]) @ P["W5"]          # dR/d rho_i, (n, F)
    F_eam = np.zeros((n, 3))
    for i, j, u, dg in pairs:                       # u: unit vector from i to j
        F_eam[i] += (dPhi[i] @ dg) * u               # d rho_i / d r_i pulls along u
        F_eam[j] -= (dPhi[i] @ dg) * u
    E, Fo = oracle.energy_forces(hdr, w, s.pos, s.species, s.box)
    assert abs(E - E_eam) <= 1e-12 * abs(E_eam)
    assert np.abs(Fo - F_eam).max() <= 1e-10 * np.abs(F_eam).max()


def test_collinear_chain_reduces_to_scalar_model(oracle):
    # Atoms on the x axis: every vector feature is e_x (x) q_i, so the layer
    # reduces to scalars per feature:
    #   dq_i = sum_j q_j o x_vv + sign(x_j - x_i) x_vs
    #   Uv.Vv -> (U q) o (V q),  n = sqrt((V q)^2 + eps)
    # and by symmetry the forces have no y or z component.
    hdr, w = small_model(F=10, K=5, T=2, S=2, seed=17, bias=0.4)
    P = _views(hdr, w)
    F, K, rc, eps = hdr["F"], hdr["K"], hdr["r_c"], hdr["eps"]
    xs = np.array([0.0, 1.3, 2.9, 4.1])
    Z = np.array([0, 1, 1, 0], np.int32)
    pos = np.zeros((4, 3)); pos[:, 0] = xs
    k = np.arange(1, K + 1)

    def energy(x):
        s = P["emb"][Z].copy()
        q = np.zeros((4, F))
        for t in range(hdr["T"]):
            L = lambda nm: P[f"l{t}.{nm}"]
            phi = silu(s @ L("W1").T + L("b1")) @ L("W2").T + L("b2")
            s1, q1 = s.copy(), q.copy()
            for i in range(4):
                for j in range(4):
                    r = abs(x[j] - x[i])
                    if i == j or r >= rc:
                        continue
                    e = np.sin(k * math.pi * r / rc) / r
                    wv = (L("A") @ e + L("c")) * 0.5 * (math.cos(math.pi * r / rc) + 1)
                    xx = phi[j] * wv
                    s1[i] += xx[F:2 * F]
                    q1[i] += q[j] * xx[:F] + np.sign(x[j] - x[i]) * xx[2 * F:]
            Uq, Vq = q1 @ L("U").T, q1 @ L("V").T
            nrm = np.sqrt(Vq**2 + eps)
            a = silu(np.concatenate([s1, nrm], 1) @ L("W3").T + L("b3")) @ L("W4").T + L("b4")
            q = q1 + a[:, :F] * Uq
            s = s1 + a[:, F:2 * F] * Uq * Vq + a[:, 2 * F:]
        return _readout(P, s).sum()

    E, Fo = oracle.energy_forces(hdr, w, pos, Z, np.zeros(3))
    assert abs(E - energy(xs)) <= 1e-12 * abs(E)
    h = 1e-6
    for i in range(4):
        xp, xm = xs.copy(), xs.copy()
        xp[i] += h; xm[i] -= h
        assert abs(-(energy(xp) - energy(xm)) / (2 * h) - Fo[i, 0]) <= 1e-6 * np.abs(Fo).max()
    assert np.abs(Fo[:, 1:]).max() <= 1e-12 * np.abs(Fo).max()


# --------------------------------------------------------------------------
# Nose-Hoover chain (NVT) oracle.
# --------------------------------------------------------------------------
def _md_water192():
    s, hdr, w = synth.workload("water192")
    V = synth.weight_views(hdr, w)
    for t in range(hdr["T"]):
        V[f"l{t}.A"][...] *= np.float32(synth.MD_FILTER_SCALE)
        V[f"l{t}.c"][...] *= np.float32(synth.MD_FILTER_SCALE)
    V["w6"][...] *= np.float32(synth.MD_READOUT_SCALE)
    return s, hdr, w


def test_nhc_with_infinite_damping_is_velocity_verlet(oracle):
    # Q -> infinity: the chain never moves, the scale factor is exactly 1 and
    # the NVT step is the plain velocity-Verlet step
    s, hdr, w = _md_water192()
    v0 = synth.maxwell_velocities(s, 300.0, seed=1)
    st = oracle.nhc_state(3 * s.n_atoms - 3, 300.0, 1e30, 3)
    x1, v1, E1, _, _ = oracle.nhc_velocity_verlet(hdr, w, s.pos, v0, s.species, s.masses, s.box, 0.5, 4, st)
    x2, v2, E2 = oracle.velocity_verlet(hdr, w, s.pos, v0, s.species, s.masses, s.box, 0.5, 4)
    assert np.array_equal(x1, x2) and np.array_equal(v1, v2) and np.array_equal(E1, E2)


def _chain_ode(t, y, nf, kT, Q):
    # y = [ln KE, xi_1..xi_M, v_1..v_M]; free particles (F = 0): the chain
    # equations of motion with p_xi = Q v
    M = len(Q)
    ke = np.exp(y[0])
    v = y[1 + M:]
    dv = np.empty(M)
    for k in range(M):
        base = (2.0 * ke - nf * kT) / Q[0] if k == 0 else (Q[k - 1] * v[k - 1] ** 2 - kT) / Q[k]
        dv[k] = base - (v[k] * v[k + 1] if k + 1 < M else 0.0)
    return np.concatenate([[-2.0 * v[0]], v, dv])


@pytest.mark.parametrize("chain", [1, 3])
def test_nhc_free_particles_follow_the_chain_equations(oracle, chain):
    # With zero forces the NVT flow reduces to a closed ODE for (KE, xi, v);
    # a tight general-purpose solve of that ODE pins the splitting, and the
    # error shrinks as dt^2 (second-order integrator)
    from scipy.integrate import solve_ivp
    n, T0, T_target, tau, t_end = 64, 600.0, 300.0, 40.0, 200.0
    species = np.zeros(n, np.int32)
    masses = np.array([12.0])
    rng = np.random.default_rng(3)
    vel = rng.standard_normal((n, 3)) * np.sqrt(oracle.KB_EV * T0 / 12.0 * oracle.ACC_UNIT)
    pos = rng.uniform(0, 50, (n, 3))
    zero = lambda x: (0.0, np.zeros_like(x))
    nf = 3 * n
    errs = []
    for dt in (2.0, 1.0):
        st = oracle.nhc_state(nf, T_target, tau, chain)
        ke0 = oracle.kinetic_energy(vel, species, masses)
        _, v, _, K, H = oracle.nhc_velocity_verlet(None, None, pos, vel, species, masses, np.zeros(3), dt,
                                                   int(round(t_end / dt)), st, force_fn=zero)
        y0 = np.concatenate([[np.log(ke0)], np.zeros(chain), np.zeros(chain)])
        sol = solve_ivp(_chain_ode, (0.0, t_end), y0, args=(float(nf), st["kT"], st["Q"]), rtol=1e-12,
                        atol=1e-14, method="DOP853")
        y = sol.y[:, -1]
        errs.append(max(abs(K[-1] - np.exp(y[0])) / np.exp(y[0]),
                        np.abs(st["v"] - y[1 + chain:]).max() / np.abs(y[1 + chain:]).max()))
        # the thermostat has moved the kinetic energy substantially
        assert abs(K[-1] - ke0) > 0.1 * ke0
    assert errs[1] < 2e-3
    assert 3.0 < errs[0] / errs[1] < 5.0


def test_nhc_extended_energy_is_conserved(oracle):
    # H = KE + E_pot + thermostat energy is the conserved quantity of the NVT
    # flow; with a strongly coupled thermostat the kinetic energy moves a lot
    # while H stays put to the integrator's O(dt^2)
    s, hdr, w = _md_water192()
    v0 = synth.maxwell_velocities(s, 600.0, seed=2)
    st = oracle.nhc_state(3 * s.n_atoms - 3, 300.0, 25.0, 3)
    _, _, E, K, H = oracle.nhc_velocity_verlet(hdr, w, s.pos, v0, s.species, s.masses, s.box, 0.25, 160, st)
    ext = E + K + H
    assert np.ptp(K) > 0.3 * K[0]
    assert np.ptp(ext) < 2e-3 * np.ptp(K)
