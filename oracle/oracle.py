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
