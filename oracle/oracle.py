"""ctypes wrapper around the FP64 CPU oracle (oracle.c) plus the few oracle
steps that are plain array bookkeeping (ghost-force fold, velocity Verlet).

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark import this module.  It imports nothing from the
GPU package, and the GPU package never imports it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc (-O2, OpenMP, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-D_DEFAULT_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_model_size.restype = ctypes.c_int64
        L.orc_model_size.argtypes = [P]
        L.orc_neighbors.restype = ctypes.c_int64
        L.orc_neighbors.argtypes = [P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int64, P, P, P]
        L.orc_neighbors_f32.restype = ctypes.c_int64
        L.orc_neighbors_f32.argtypes = [P, ctypes.c_int, P, ctypes.c_float, ctypes.c_float,
                                        ctypes.c_int64, P, P]
        L.orc_hops.restype = None
        L.orc_hops.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int64, P, P, ctypes.c_int, P]
        L.orc_energy_forces.restype = ctypes.c_double
        L.orc_energy_forces.argtypes = [P, P, P, ctypes.c_int64, P, P, ctypes.c_int, ctypes.c_int,
                                        P, P, P, P]
        L.orc_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def neighbors(pos, box, cutoff: float):
    """Brute-force FP64 neighbour list over periodic images.
    Returns (dst, src, dvec) sorted by (dst, src, image)."""
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    box = np.ascontiguousarray(box, dtype=np.float64)
    n = pos.shape[0]
    E = lib().orc_neighbors(_ptr(pos), n, _ptr(box), float(cutoff), 0, None, None, None)
    dst = np.empty(E, np.int32)
    src = np.empty(E, np.int32)
    dv = np.empty((E, 3), np.float64)
    lib().orc_neighbors(_ptr(pos), n, _ptr(box), float(cutoff), E, _ptr(dst), _ptr(src), _ptr(dv))
    return dst, src, dv


def neighbors_f32(pos, box, rc: float, skin: float):
    """Neighbour pairs decided in float32 by the device's formula (see
    orc_neighbors_f32).  Returns (dst, src) sorted by (dst, src)."""
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    box = np.ascontiguousarray(box, dtype=np.float32)
    n = pos.shape[0]
    E = lib().orc_neighbors_f32(_ptr(pos), n, _ptr(box), np.float32(rc), np.float32(skin), 0, None, None)
    dst = np.empty(E, np.int32)
    src = np.empty(E, np.int32)
    lib().orc_neighbors_f32(_ptr(pos), n, _ptr(box), np.float32(rc), np.float32(skin), E,
                            _ptr(dst), _ptr(src))
    return dst, src


def hops(n: int, n_local: int, dst, src, T: int):
    dst = np.ascontiguousarray(dst, np.int32)
    src = np.ascontiguousarray(src, np.int32)
    out = np.empty(n, np.int8)
    lib().orc_hops(n, n_local, dst.size, _ptr(dst), _ptr(src), T, _ptr(out))
    return out


def energy_forces(header: dict, weights, pos, species, box, n_local: int | None = None,
                  per_atom: bool = False):
    """E = sum_{i < n_local} U_i and F = -dE/dr for every atom (FP64).

    ``weights`` are upcast exactly from their stored float32 values."""
    dims = np.array([header["F"], header["K"], header["T"], header["n_species"]], np.int32)
    rce = np.array([header["r_c"], header["eps"]], np.float64)
    W = np.ascontiguousarray(np.asarray(weights, dtype=np.float32).astype(np.float64))
    if lib().orc_model_size(_ptr(dims)) != W.size:
        raise ValueError("weight count does not match the model dimensions")
    pos = np.ascontiguousarray(np.asarray(pos).astype(np.float64))
    Z = np.ascontiguousarray(species, np.int32)
    box = np.ascontiguousarray(box, np.float64)
    n = pos.shape[0]
    nl = n if n_local is None else int(n_local)
    F = np.zeros((n, 3), np.float64)
    U = np.zeros(n, np.float64)
    ne = np.zeros(1, np.int64)
    E = lib().orc_energy_forces(_ptr(dims), _ptr(rce), _ptr(W), W.size, _ptr(pos), _ptr(Z), n, nl,
                                _ptr(box), _ptr(F), _ptr(U), _ptr(ne))
    if not np.isfinite(E):
        raise ValueError("oracle rejected the model")
    if per_atom:
        return E, F, U
    return E, F


def fold_ghost_forces(forces, n_local: int, owner):
    """Sum each ghost row into its owner's row (the reverse summation of
    partial forces, Eq. 2); ghost rows are returned unchanged."""
    out = np.array(forces, dtype=np.float64, copy=True)
    np.add.at(out, np.asarray(owner, np.int64), out[n_local:])
    return out


ACC_UNIT = 9.648533212e-3  # (eV / Angstrom / amu) -> Angstrom / fs^2


def velocity_verlet(header, weights, pos, vel, species, masses, box, dt: float, n_steps: int):
    """Velocity Verlet in FP64 with positions wrapped into [0, L) after each
    drift.  Returns (pos, vel, energies) after n_steps."""
    x = np.array(pos, np.float64)
    v = np.array(vel, np.float64)
    m = np.asarray(masses, np.float64)[np.asarray(species)]
    inv_m = (ACC_UNIT / m)[:, None]
    E, F = energy_forces(header, weights, x, species, box)
    Es = []
    for _ in range(n_steps):
        v += 0.5 * dt * F * inv_m
        x += dt * v
        for d in range(3):
            if box[d] > 0:
                x[:, d] = np.mod(x[:, d], box[d])
        E, F = energy_forces(header, weights, x, species, box)
        v += 0.5 * dt * F * inv_m
        Es.append(E)
    return x, v, np.array(Es)


KB_EV = 8.617333262e-5     # Boltzmann constant, eV / K
MVV2E = 1.0 / ACC_UNIT     # amu Angstrom^2 / fs^2 -> eV


def nhc_half_step(state: dict, ke: float, h: float) -> tuple[float, float]:
    """Propagate a Nose-Hoover chain over a time h (the thermostat part of the
    NVT splitting; the paper's runs are NVT with a Nose-Hoover thermostat,
    Methods, "Molecular Dynamics Simulations").  The chain equations are
        d xi_k / dt = v_k,
        d v_1 / dt = (2 KE - N_f kT) / Q_1 - v_1 v_2,
        d v_k / dt = (Q_{k-1} v_{k-1}^2 - kT) / Q_k - v_k v_{k+1},  (last: no v_{k+1} term)
    and the particle velocities are scaled by exp(-int v_1 dt).  The update is
    the symmetric Trotter splitting of these flows: chain kicks from the last
    thermostat to the first, each damped by its successor over half the kick
    interval on both sides; one scaling of the particles and one drift of
    every xi over h; the same kicks from the first thermostat to the last.
    state: {"Q": array, "v": array, "xi": array, "nf": float, "kT": float};
    updated in place.  Returns (velocity scale factor, kinetic energy after
    scaling)."""
    Q, v, xi, nf, kT = state["Q"], state["v"], state["xi"], state["nf"], state["kT"]
    M = len(Q)

    def g(k, ke_now):
        if k == 0:
            return (2.0 * ke_now - nf * kT) / Q[0]
        return (Q[k - 1] * v[k - 1] ** 2 - kT) / Q[k]

    quarter = h / 4.0
    v[M - 1] += (h / 2.0) * g(M - 1, ke)
    for k in range(M - 2, -1, -1):
        damp = np.exp(-quarter * v[k + 1])
        v[k] *= damp
        v[k] += (h / 2.0) * g(k, ke)
        v[k] *= damp
    scale = np.exp(-h * v[0])
    ke = ke * scale * scale
    xi += h * v
    for k in range(M - 1):
        damp = np.exp(-quarter * v[k + 1])
        v[k] *= damp
        v[k] += (h / 2.0) * g(k, ke)
        v[k] *= damp
    v[M - 1] += (h / 2.0) * g(M - 1, ke)
    return float(scale), float(ke)


def nhc_state(n_dof: int, temperature: float, tau_fs: float, chain: int) -> dict:
    """Chain of `chain` thermostats at rest, Q_1 = N_f kT tau^2, Q_k = kT tau^2."""
    kT = KB_EV * temperature
    Q = np.array([(n_dof if k == 0 else 1.0) * kT * tau_fs ** 2 for k in range(chain)], np.float64)
    return {"Q": Q, "v": np.zeros(chain), "xi": np.zeros(chain), "nf": float(n_dof), "kT": kT}


def thermostat_energy(state: dict) -> float:
    """sum_k Q_k v_k^2 / 2 + N_f kT xi_1 + kT sum_{k>1} xi_k."""
    Q, v, xi = state["Q"], state["v"], state["xi"]
    return float(0.5 * np.sum(Q * v * v) + state["nf"] * state["kT"] * xi[0] + state["kT"] * np.sum(xi[1:]))


def kinetic_energy(vel, species, masses) -> float:
    m = np.asarray(masses, np.float64)[np.asarray(species)]
    return float(0.5 * MVV2E * np.sum(m[:, None] * np.asarray(vel, np.float64) ** 2))


def nhc_velocity_verlet(header, weights, pos, vel, species, masses, box, dt: float, n_steps: int, state: dict,
                        force_fn=None):
    """NVT steps in FP64: chain over dt/2, velocity Verlet, chain over dt/2.
    force_fn(x) -> (E, F) replaces the PaiNN oracle when given.  Returns
    (pos, vel, potential energies, kinetic energies, thermostat energies)."""
    x = np.array(pos, np.float64)
    v = np.array(vel, np.float64)
    m = np.asarray(masses, np.float64)[np.asarray(species)]
    inv_m = (ACC_UNIT / m)[:, None]
    ef = force_fn or (lambda y: energy_forces(header, weights, y, species, box))
    E, F = ef(x)
    Es, Ks, Hs = [], [], []
    for _ in range(n_steps):
        s, _ = nhc_half_step(state, kinetic_energy(v, species, masses), 0.5 * dt)
        v *= s
        v += 0.5 * dt * F * inv_m
        x += dt * v
        for d in range(3):
            if box[d] > 0:
                x[:, d] = np.mod(x[:, d], box[d])
        E, F = ef(x)
        v += 0.5 * dt * F * inv_m
        s, ke = nhc_half_step(state, kinetic_energy(v, species, masses), 0.5 * dt)
        v *= s
        Es.append(E)
        Ks.append(ke)
        Hs.append(thermostat_energy(state))
    return x, v, np.array(Es), np.array(Ks), np.array(Hs)
