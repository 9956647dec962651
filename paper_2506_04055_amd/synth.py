"""Seeded synthetic inputs: atomic systems, velocities and model weights.

This module holds no arithmetic of the potential itself.  It only draws
positions, species, periodic boxes, ghost shells, velocities and weight arrays
from ``numpy.random.default_rng(seed)`` so that the GPU library and the FP64
CPU oracle are fed byte-identical inputs.

Workload shapes follow the systems the paper simulates (Methods, "Molecular
Dynamics Simulations"; Table 2): a water-like liquid, a water slab between
vacuum regions, a perturbed fcc crystal and a solvated-peptide-like mixture of
H/C/N/O.  The paper's datasets and trained weights are not used; the recipes
below stand in for them.

Conventions shared with both consumers (stated, not computed here):
  * units: Angstrom, eV, amu, fs;
  * positions are float32 values stored as an (N, 3) array, wrapped into
    [0, L) for periodic systems; box lengths are float32-representable;
  * weights are one flat float32 array in the order of ``weight_layout``,
    every matrix stored row-major as [out][in] (y = W x).
"""
from __future__ import annotations

import json
import math
from dataclasses import dataclass, field

import numpy as np

# Standard water geometry (O-H bond, H-O-H angle) and masses.
OH_BOND = 0.96
HOH_ANGLE_DEG = 104.5
MASS = {"H": 1.008, "C": 12.011, "N": 14.007, "O": 15.999}
# Boltzmann constant in eV/K and the unit factor (eV/Angstrom/amu) -> Angstrom/fs^2.
KB_EV = 8.617333262e-5
ACC_UNIT = 9.648533212e-3


@dataclass
class System:
    """One atomic system.  Locals come first; ghosts (if any) follow."""

    pos: np.ndarray          # (N, 3) float32
    species: np.ndarray      # (N,) int32
    box: np.ndarray          # (3,) float64 holding float32-exact lengths; 0 = open
    n_local: int
    owner: np.ndarray | None = None   # (N - n_local,) int32 local index of each ghost
    masses: np.ndarray | None = None  # (n_species,) float64 amu
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_atoms(self) -> int:
        return int(self.pos.shape[0])


def f32(x):
    return np.float32(x)


def _wrap_f32(pos64: np.ndarray, box: np.ndarray) -> np.ndarray:
    """Wrap into [0, L) per periodic dimension and round to float32 so that the
    stored value is itself inside [0, L)."""
    out = pos64.copy()
    for d in range(3):
        L = box[d]
        if L > 0:
            out[:, d] = np.mod(out[:, d], L)
    p32 = out.astype(np.float32)
    for d in range(3):
        L = np.float32(box[d])
        if L > 0:
            bad = p32[:, d] >= L
            p32[bad, d] = np.float32(0.0)
    return p32


def _random_rotations(rng: np.random.Generator, n: int) -> np.ndarray:
    """Uniform random rotations from normalised Gaussian quaternions."""
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    w, x, y, z = q.T
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (y * y + z * z)
    R[:, 0, 1] = 2 * (x * y - z * w)
    R[:, 0, 2] = 2 * (x * z + y * w)
    R[:, 1, 0] = 2 * (x * y + z * w)
    R[:, 1, 1] = 1 - 2 * (x * x + z * z)
    R[:, 1, 2] = 2 * (y * z - x * w)
    R[:, 2, 0] = 2 * (x * z - y * w)
    R[:, 2, 1] = 2 * (y * z + x * w)
    R[:, 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def _water_offsets() -> np.ndarray:
    half = math.radians(HOH_ANGLE_DEG) / 2
    return np.array([
        [0.0, 0.0, 0.0],
        [OH_BOND * math.sin(half), OH_BOND * math.cos(half), 0.0],
        [-OH_BOND * math.sin(half), OH_BOND * math.cos(half), 0.0],
    ])


def _place_waters(rng, centers: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Water molecules (O, H, H) with uniformly random orientations at the
    given oxygen sites.  Species: O = 0, H = 1."""
    n = centers.shape[0]
    R = _random_rotations(rng, n)
    off = _water_offsets()
    atoms = centers[:, None, :] + np.einsum("nij,kj->nki", R, off)
    species = np.tile(np.array([0, 1, 1], dtype=np.int32), n)
    return atoms.reshape(-1, 3), species


def water_box(n_side: int, spacing: float, seed: int = 0, name: str = "") -> System:
    """Cubic water-like liquid: n_side^3 molecules on a jittered simple-cubic
    lattice (uniform jitter of +-0.1 spacing per axis), random orientations.

    n_side=4,  spacing=3.105 -> 192 atoms,    L = fp32(12.42)
    n_side=20, spacing=3.105 -> 24,000 atoms, L = fp32(62.1)   (1.00 g/cm^3)
    """
    rng = np.random.default_rng(seed)
    L = float(f32(n_side * spacing))
    g = (np.arange(n_side) + 0.5) * spacing
    centers = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    centers = centers + rng.uniform(-0.1 * spacing, 0.1 * spacing, centers.shape)
    atoms, species = _place_waters(rng, centers)
    box = np.array([L, L, L])
    pos = _wrap_f32(atoms, box)
    return System(pos, species, box, pos.shape[0],
                  masses=np.array([MASS["O"], MASS["H"]]), name=name or f"water{n_side}",
                  meta={"recipe": "water_box", "n_side": n_side, "spacing": spacing, "seed": seed})


def water_slab(seed: int = 0, n_mol: int = 16000, lateral: float = 109.39, thick: float = 40.0,
               box_z: float = 180.0, vapor_frac: float = 0.005, grid=(36, 36, 13)) -> System:
    """Liquid-vapour slab: a 1 g/cm^3 water slab of the given thickness centred
    in z of a tall periodic box, plus a small fraction of molecules placed at
    random in the vacuum gap (rejecting any closer than 2.5 A to another O)."""
    rng = np.random.default_rng(seed)
    Lx = float(f32(lateral))
    Lz = float(f32(box_z))
    n_vap = int(round(vapor_frac * n_mol))
    n_slab = n_mol - n_vap
    nx, ny, nz = grid
    sx, sy, sz = Lx / nx, Lx / ny, thick / nz
    z0 = 0.5 * (Lz - thick)
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    sites = np.stack([(ii + 0.5) * sx, (jj + 0.5) * sy, z0 + (kk + 0.5) * sz], -1).reshape(-1, 3)
    pick = rng.choice(sites.shape[0], size=n_slab, replace=False)
    centers = sites[np.sort(pick)]
    centers = centers + rng.uniform(-0.1, 0.1, centers.shape) * np.array([sx, sy, sz])
    vap = []
    lo, hi = z0 - 2.0, z0 + thick + 2.0
    while len(vap) < n_vap:
        c = rng.uniform(0, 1, 3) * np.array([Lx, Lx, Lz])
        if lo <= c[2] <= hi:
            continue
        ok = all(np.linalg.norm(c - o) > 2.5 for o in vap)
        if ok:
            vap.append(c)
    centers = np.concatenate([centers, np.array(vap).reshape(-1, 3)], 0)
    atoms, species = _place_waters(rng, centers)
    box = np.array([Lx, Lx, Lz])
    pos = _wrap_f32(atoms, box)
    return System(pos, species, box, pos.shape[0], masses=np.array([MASS["O"], MASS["H"]]),
                  name="water_slab", meta={"recipe": "water_slab", "seed": seed, "n_vapor": n_vap})


def fcc_crystal(n_cells: int, a: float = 4.05, sigma: float = 0.05, seed: int = 0,
                ghost_depth: float = 0.0) -> System:
    """Perturbed fcc crystal of n_cells^3 conventional cells (4 atoms each),
    Gaussian displacement sigma per component, one species.

    With ghost_depth > 0 the system is one domain's share as an MD engine hands
    it over: the periodic images of the local atoms that fall within
    ghost_depth of the box are appended as explicit ghost atoms (Results,
    "Distributed potential computation", Fig. 1d), the box is then open in all
    dimensions (box = 0), and ``owner`` maps each ghost to its local atom."""
    rng = np.random.default_rng(seed)
    L = float(f32(n_cells * a))
    basis = np.array([[0, 0, 0], [0.5, 0.5, 0], [0.5, 0, 0.5], [0, 0.5, 0.5]]) * a
    g = np.arange(n_cells) * a
    cells = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 1, 3)
    atoms = (cells + basis[None]).reshape(-1, 3)
    atoms = atoms + rng.normal(0.0, sigma, atoms.shape)
    box = np.array([L, L, L])
    pos = _wrap_f32(atoms, box)
    n_local = pos.shape[0]
    species = np.zeros(n_local, dtype=np.int32)
    if ghost_depth <= 0:
        return System(pos, species, box, n_local, masses=np.array([26.9815]),
                      name=f"fcc{n_cells}", meta={"recipe": "fcc", "seed": seed})
    p64 = pos.astype(np.float64)
    gpos, gown = [], []
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            for sz in (-1, 0, 1):
                if sx == sy == sz == 0:
                    continue
                q = p64 + np.array([sx, sy, sz]) * L
                inside = np.all((q >= -ghost_depth) & (q < L + ghost_depth), axis=1)
                idx = np.nonzero(inside)[0]
                gpos.append(q[idx])
                gown.append(idx)
    gpos = np.concatenate(gpos).astype(np.float32)
    gown = np.concatenate(gown).astype(np.int32)
    allpos = np.concatenate([pos, gpos], 0)
    allsp = np.zeros(allpos.shape[0], dtype=np.int32)
    return System(allpos, allsp, np.zeros(3), n_local, owner=gown, masses=np.array([26.9815]),
                  name=f"fcc{n_cells}_ghost", meta={"recipe": "fcc+ghost", "seed": seed,
                                                    "ghost_depth": ghost_depth, "box_local": L})


PEPTIDE_SPECIES = ("H", "C", "N", "O")
PEPTIDE_FRACTIONS = (0.6, 0.2, 0.1, 0.1)
PEPTIDE_DENSITY = 0.10024  # atoms / A^3: 1 g/cm^3 at the mean mass of the mixture


def peptide_like(n_atoms: int, seed: int) -> System:
    """Solvated-peptide-like mixture: H/C/N/O at exact 60/20/10/10 % counts,
    shuffled, on a jittered simple-cubic lattice at 1 g/cm^3 (0.10024 atoms/A^3)
    in a cubic periodic box of side (N / 0.10024)^(1/3)."""
    rng = np.random.default_rng(seed)
    L = float(f32((n_atoms / PEPTIDE_DENSITY) ** (1.0 / 3.0)))
    n_side = int(math.ceil(n_atoms ** (1.0 / 3.0) - 1e-9))
    sp = L / n_side
    g = (np.arange(n_side) + 0.5) * sp
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    pick = np.sort(rng.choice(sites.shape[0], size=n_atoms, replace=False))
    atoms = sites[pick] + rng.uniform(-0.1 * sp, 0.1 * sp, (n_atoms, 3))
    counts = [int(round(f * n_atoms)) for f in PEPTIDE_FRACTIONS]
    counts[0] += n_atoms - sum(counts)
    species = np.concatenate([np.full(c, k, dtype=np.int32) for k, c in enumerate(counts)])
    rng.shuffle(species)
    box = np.array([L, L, L])
    pos = _wrap_f32(atoms, box)
    return System(pos, species, box, n_atoms,
                  masses=np.array([MASS[s] for s in PEPTIDE_SPECIES]), name=f"peptide{n_atoms}",
                  meta={"recipe": "peptide_like", "seed": seed})


def serving_requests(n_requests: int = 2000, seed: int = 1, n_min: int = 500, n_max: int = 20000):
    """Request sizes N ~ U{n_min..n_max} and a per-request system seed."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_min, n_max + 1, size=n_requests)
    seeds = rng.integers(0, 2**31 - 1, size=n_requests)
    return sizes.astype(np.int64), seeds.astype(np.int64)


def poisson_arrivals(n: int, rate_per_s: float, seed: int = 1) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed + 7919)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, size=n))


def maxwell_velocities(system: System, temperature: float, seed: int = 0) -> np.ndarray:
    """Maxwell-Boltzmann velocities (A/fs) at the given temperature with the
    centre-of-mass momentum removed.  Returned as (N, 3) float32."""
    rng = np.random.default_rng(seed + 104729)
    m = system.masses[system.species[: system.n_local]]
    sd = np.sqrt(KB_EV * temperature / m * ACC_UNIT)
    v = rng.standard_normal((system.n_local, 3)) * sd[:, None]
    p = (v * m[:, None]).sum(0)
    v -= p / m.sum()
    return v.astype(np.float32)


# --------------------------------------------------------------------------
# Model weights
# --------------------------------------------------------------------------

def weight_layout(F: int, K: int, T: int, n_species: int):
    """Ordered (name, shape, fan_in) of every parameter block.

    fan_in = 0 marks biases (drawn as zeros); the embedding table is drawn
    from N(0, 1).  Split orders inside 3F-wide blocks: the message-function
    output and the filter are [vv | s | vs]; the update-MLP output is
    [vv | sv | ss]."""
    Fh = F // 2
    out = [("emb", (n_species, F), 1)]
    for t in range(T):
        out += [
            (f"l{t}.W1", (F, F), F), (f"l{t}.b1", (F,), 0),
            (f"l{t}.W2", (3 * F, F), F), (f"l{t}.b2", (3 * F,), 0),
            (f"l{t}.A", (3 * F, K), K), (f"l{t}.c", (3 * F,), 0),
            (f"l{t}.U", (F, F), F), (f"l{t}.V", (F, F), F),
            (f"l{t}.W3", (F, 2 * F), 2 * F), (f"l{t}.b3", (F,), 0),
            (f"l{t}.W4", (3 * F, F), F), (f"l{t}.b4", (3 * F,), 0),
        ]
    out += [("W5", (Fh, F), F), ("b5", (Fh,), 0), ("w6", (Fh,), Fh), ("b6", (1,), 0)]
    return out


def model_header(F: int, K: int, T: int, n_species: int, r_c: float = 5.0, eps: float = 1e-8) -> dict:
    layout = weight_layout(F, K, T, n_species)
    return {
        "model": "painn",
        "F": F, "K": K, "T": T, "n_species": n_species,
        "r_c": r_c, "eps": eps,
        "basis": "bessel_sin_over_r", "envelope": "cosine",
        "units": {"length": "angstrom", "energy": "eV"},
        "graph": "full_directed_csr_by_destination",
        "split": {"message": ["vv", "s", "vs"], "update": ["vv", "sv", "ss"]},
        "layout": [[n, list(s)] for n, s, _ in layout],
        "n_weights": int(sum(int(np.prod(s)) for _, s, _ in layout)),
    }


def make_weights(F: int, K: int, T: int, n_species: int, seed: int = 0, r_c: float = 5.0,
                 eps: float = 1e-8, bias_scale: float = 0.0):
    """Flat float32 weights: matrices ~ N(0, 1/fan_in), embedding ~ N(0, 1),
    biases 0 (or N(0, bias_scale^2) when bias_scale > 0, used by tests so that
    every bias path is exercised).  Draw order = layout order, float64 draws
    cast to float32."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape, fan_in in weight_layout(F, K, T, n_species):
        n = int(np.prod(shape))
        if fan_in == 0:
            if bias_scale > 0:
                parts.append(rng.standard_normal(n) * bias_scale)
            else:
                parts.append(np.zeros(n))
        else:
            parts.append(rng.standard_normal(n) / math.sqrt(fan_in))
    w = np.concatenate(parts).astype(np.float32)
    return model_header(F, K, T, n_species, r_c, eps), w


def weight_views(header: dict, w: np.ndarray) -> dict:
    """Named views into a flat weight array (no arithmetic)."""
    out, off = {}, 0
    for name, shape in header["layout"]:
        n = int(np.prod(shape))
        out[name] = w[off: off + n].reshape(shape)
        off += n
    assert off == w.size
    return out


def header_json(header: dict) -> str:
    return json.dumps(header, sort_keys=True)


# Allegro (single tensor-product layer): the widths the paper gives for its
# water and aluminium models (a 5 A cutoff, 8 radial functions, polynomial
# envelope of order 2, l_max = 3, two-body MLP [8, 16, 32] into a 64-wide
# latent, hidden MLP width 64), with per-degree channel counts (32, 16, 8, 8)
# for l = 0..3 and a 32-wide output MLP.
ALLEGRO_DEFAULTS = {"n_basis": 8, "envelope_p": 2, "mlp_2b": [8, 16, 32, 64], "channels": [32, 16, 8, 8],
                    "latent_hidden": 64, "out_hidden": 32}


def allegro_layout(h: dict):
    """Ordered (name, shape, fan_in) of every Allegro parameter block;
    fan_in = 0 marks biases.  Matrices are [out][in] row-major."""
    S, nb = h["n_species"], h["n_basis"]
    d = list(h["mlp_2b"])
    NC, D, L, O = sum(h["channels"]), d[-1], h["latent_hidden"], h["out_hidden"]
    out, prev = [], 2 * S + nb
    for q, w in enumerate(d):
        out += [(f"2b_W{q + 1}", (w, prev), prev), (f"2b_b{q + 1}", (w,), 0)]
        prev = w
    out += [("Wv", (NC, D), D), ("We", (NC, D), D),
            ("lat_W1", (L, D + NC), D + NC), ("lat_b1", (L,), 0), ("lat_W2", (D, L), L), ("lat_b2", (D,), 0),
            ("out_W1", (O, D), D), ("out_b1", (O,), 0), ("out_w2", (O,), O), ("out_b2", (1,), 0)]
    return out


def allegro_header(n_species: int, r_c: float = 5.0, env_scale: float | None = None, **kw) -> dict:
    h = dict(ALLEGRO_DEFAULTS, **kw)
    h.update({"model": "allegro", "n_species": n_species, "r_c": r_c, "l_max": len(h["channels"]) - 1,
              "basis": "bessel", "envelope": "polynomial",
              "units": {"length": "angstrom", "energy": "eV"}, "graph": "full_directed_csr_by_destination"})
    # 1 / sqrt(mean neighbour count) of a liquid or fcc metal at r_c = 5 A
    h["env_scale"] = float(np.float32(1.0 / math.sqrt(40.0) if env_scale is None else env_scale))
    lay = allegro_layout(h)
    h["layout"] = [[n, list(s)] for n, s, _ in lay]
    h["n_weights"] = int(sum(int(np.prod(s)) for _, s, _ in lay))
    return h


def make_allegro_weights(n_species: int, seed: int = 0, bias_scale: float = 0.0, **kw):
    """Flat float32 Allegro weights: matrices ~ N(0, 1/fan_in), biases 0 (or
    N(0, bias_scale^2)); draw order = layout order, float64 draws cast to
    float32."""
    h = allegro_header(n_species, **kw)
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape, fan_in in allegro_layout(h):
        n = int(np.prod(shape))
        if fan_in == 0:
            parts.append(rng.standard_normal(n) * bias_scale if bias_scale > 0 else np.zeros(n))
        else:
            parts.append(rng.standard_normal(n) / math.sqrt(fan_in))
    return h, np.concatenate(parts).astype(np.float32)


# MACE at the paper's settings: two interaction layers, correlation order 3,
# l_max = 3, 32 channels (hidden irreps 32x0e + 32x1o), 8 radial basis
# functions, polynomial envelope of order 6, 5 A cutoff; a 64-wide radial MLP
# (the paper's node embedding width read as the width of the radial network)
# and a 16-wide readout MLP.
MACE_DEFAULTS = {"n_basis": 8, "envelope_p": 6, "l_max": 3, "channels": 32, "correlation": 3,
                 "radial_hidden": [64, 64, 64], "readout_hidden": 16, "avg_neighbors": 40.0}


def _mace_couples(l1, l2, L):
    return abs(l1 - l2) <= L <= l1 + l2 and (l1 + l2 + L) % 2 == 0


def mace_layout(h: dict):
    """Ordered (name, shape, fan_in) of every MACE parameter block (fan_in = 0:
    bias).  Conv paths (l1, l2, L) and contraction paths are enumerated in the
    order the model header documents (see include/mlp.h)."""
    S, K, nb, lmax, corr = h["n_species"], h["channels"], h["n_basis"], h["l_max"], h["correlation"]
    rh = list(h["radial_hidden"])
    lin, lout = ([0], [0, 1]), ([0, 1], [0])
    out = [("W_emb", (K, S), 1)]
    for t in range(2):
        conv = [(l1, l2, L) for l2 in lin[t] for l1 in range(lmax + 1) for L in range(lmax + 1)
                if _mace_couples(l1, l2, L)]
        for l2 in lin[t]:
            out.append((f"l{t}.W_up{l2}", (K, K), K))
        prev = nb
        for q, wdt in enumerate(rh):
            out.append((f"l{t}.rad{q}", (wdt, prev), prev))
            prev = wdt
        out.append((f"l{t}.rad{len(rh)}", (len(conv) * K, prev), prev))
        for L in range(lmax + 1):
            nL = sum(1 for c in conv if c[2] == L)
            if nL:
                out.append((f"l{t}.W_A{L}", (K, nL * K), nL * K))
        for Lo in lout[t]:
            npth = (1 if Lo <= lmax else 0)
            if corr >= 2:
                npth += sum(1 for l1 in range(lmax + 1) for l2 in range(l1, lmax + 1) if _mace_couples(l1, l2, Lo))
            if corr >= 3:
                npth += sum(1 for l1 in range(lmax + 1) for l2 in range(l1, lmax + 1) for lam in range(lmax + 1)
                            if _mace_couples(l1, l2, lam) for l3 in range(lmax + 1) if _mace_couples(lam, l3, Lo))
            out.append((f"l{t}.W_sym{Lo}", (S, K, npth), npth))
        for Lo in lout[t]:
            out.append((f"l{t}.W_out{Lo}", (K, K), K))
        for Lo in lout[t]:
            if Lo in lin[t]:
                out.append((f"l{t}.W_sc{Lo}", (S, K, K), K))
    RH = h["readout_hidden"]
    out += [("w_r1", (K,), K), ("W_r2", (RH, K), K), ("b_r2", (RH,), 0), ("w_r2", (RH,), RH), ("b_r3", (1,), 0)]
    return out


def mace_header(n_species: int, r_c: float = 5.0, **kw) -> dict:
    h = dict(MACE_DEFAULTS, **kw)
    h.update({"model": "mace", "n_species": n_species, "r_c": r_c, "basis": "bessel", "envelope": "polynomial",
              "units": {"length": "angstrom", "energy": "eV"}, "graph": "full_directed_csr_by_destination"})
    lay = mace_layout(h)
    h["layout"] = [[n, list(s)] for n, s, _ in lay]
    h["n_weights"] = int(sum(int(np.prod(s)) for _, s, _ in lay))
    return h


def make_mace_weights(n_species: int, seed: int = 0, bias_scale: float = 0.0, **kw):
    """Flat float32 MACE weights: matrices ~ N(0, 1/fan_in) (the embedding
    ~ N(0, 1)), biases 0 (or N(0, bias_scale^2)); draw order = layout order."""
    h = mace_header(n_species, **kw)
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape, fan_in in mace_layout(h):
        n = int(np.prod(shape))
        if fan_in == 0:
            parts.append(rng.standard_normal(n) * bias_scale if bias_scale > 0 else np.zeros(n))
        else:
            parts.append(rng.standard_normal(n) / math.sqrt(fan_in))
    return h, np.concatenate(parts).astype(np.float32)


MD_FILTER_SCALE = 0.1
MD_READOUT_SCALE = 1e-2


# Named workloads (sizes from the evaluation setups this path is measured on).
def al_nvt_workload(n_cells: int, seed: int = 0) -> tuple[System, dict, np.ndarray]:
    """The aluminium MD setting of the paper's timing runs (Methods,
    "Molecular Dynamics Simulations"): an fcc lattice with a = 4.065 A
    replicated n_cells times along each axis (4 n_cells^3 atoms), for NVT at
    1000 K with a 3 fs step and a 2.0 A skin; PaiNN with T = 4 and F = 64 as
    for the aluminium model (Methods, "Chosen Architectures" and "H2O-PBE0TS
    and ANI-AL Models"), K = 20 (not stated there), rc = 5 A.
    Random weights with the MD scaling of the radial filter and the readout
    (see water24k_md), which keeps the trajectory finite."""
    sysm = fcc_crystal(n_cells, a=4.065, sigma=0.0, seed=seed)
    hdr, w = make_weights(64, 20, 4, 1, seed)
    V = weight_views(hdr, w)
    for t in range(hdr["T"]):
        V[f"l{t}.A"][...] *= np.float32(MD_FILTER_SCALE)
        V[f"l{t}.c"][...] *= np.float32(MD_FILTER_SCALE)
    V["w6"][...] *= np.float32(MD_READOUT_SCALE)
    return sysm, hdr, w


def workload(name: str, seed: int = 0) -> tuple[System, dict, np.ndarray]:
    if name == "water192":
        sysm = water_box(4, 3.105, seed)
        hdr, w = make_weights(32, 8, 2, 2, seed)
    elif name == "water24k":
        sysm = water_box(20, 3.105, seed)
        hdr, w = make_weights(128, 20, 3, 2, seed)
    elif name == "water24k_md":
        # Same system and architecture for a velocity-Verlet run.  With the
        # plain N(0, 1/fan_in) draw a random PaiNN has no short-range
        # repulsion: atoms that approach each other in a 300 K trajectory
        # give radial features that grow layer over layer until float32
        # overflows.  Scaling the radial filter (A, c) by 0.1 keeps features
        # bounded at close contact and scaling the readout by 1e-2 keeps
        # forces small; the trajectory then stays finite with a liquid-like
        # neighbour-list rebuild cadence, and the work per step is unchanged.
        sysm = water_box(20, 3.105, seed)
        hdr, w = make_weights(128, 20, 3, 2, seed)
        V = weight_views(hdr, w)
        for t in range(hdr["T"]):
            V[f"l{t}.A"][...] *= np.float32(MD_FILTER_SCALE)
            V[f"l{t}.c"][...] *= np.float32(MD_FILTER_SCALE)
        V["w6"][...] *= np.float32(MD_READOUT_SCALE)
    elif name == "fcc1m_ghost":
        sysm = fcc_crystal(64, ghost_depth=15.0, seed=seed)
        hdr, w = make_weights(128, 20, 3, 1, seed)
    elif name == "slab48k":
        sysm = water_slab(seed)
        hdr, w = make_weights(128, 20, 3, 2, seed)
    else:
        raise KeyError(name)
    return sysm, hdr, w
