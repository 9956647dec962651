"""Python binding of libmlp (ctypes).  Argument marshalling only: every step
of the energy/force path runs in the library's HIP kernels.  PyTorch supplies
device memory and streams.

The functions keep the C names (mlp_model_create, mlp_build_neighbors,
mlp_energy_forces, mlp_md_step, mlp_server_create, mlp_submit, mlp_poll);
the classes below wrap handle lifetimes and tensor layouts.
"""
from __future__ import annotations

import ctypes
import json
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmlp.so")

MLP_OK, MLP_PENDING = 0, 1
MLP_FP32, MLP_BF16, MLP_BF16_FAST, MLP_BF16_NODE, MLP_BF16_NODE_X3 = 0, 1, 2, 3, 4
# precision names: operand forms of the node GEMMs / the radial filter
PRECISIONS = {"fp32": MLP_FP32,            # FP32 / FP32
              "bf16": MLP_BF16,            # split bf16 ("bf16x3") / split bf16
              "bf16x3": MLP_BF16,
              "bf16_fast": MLP_BF16_FAST,  # plain bf16 / plain bf16
              "bf16_node": MLP_BF16_NODE,  # plain bf16 / FP32
              "bf16_node_x3": MLP_BF16_NODE_X3}   # plain bf16 / split bf16
_ERRORS = {-1: "INVALID_ARG", -2: "OOM", -3: "CAPACITY", -4: "BOX_TOO_SMALL", -5: "DEVICE", -6: "UNKNOWN_TICKET"}


class MLPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRORS.get(code, code)}: {msg}")
        self.code = code


class Stats(ctypes.Structure):
    _fields_ = [
        ("n_edges_skin", ctypes.c_int64), ("n_edges", ctypes.c_int64),
        ("n_atoms", ctypes.c_int32), ("n_local", ctypes.c_int32),
        ("n_within_hops", ctypes.c_int32 * 8), ("n_cells", ctypes.c_int32 * 3),
        ("max_cell_occupancy", ctypes.c_int32), ("n_builds", ctypes.c_int32),
        ("n_grows", ctypes.c_int32), ("device_bytes", ctypes.c_int64),
        ("n_edges_within_hops", ctypes.c_int64 * 8),
    ]

    def as_dict(self):
        return {
            "n_edges_skin": self.n_edges_skin, "n_edges": self.n_edges, "n_atoms": self.n_atoms,
            "n_local": self.n_local, "n_within_hops": list(self.n_within_hops),
            "n_cells": list(self.n_cells), "max_cell_occupancy": self.max_cell_occupancy,
            "n_builds": self.n_builds, "n_grows": self.n_grows, "device_bytes": self.device_bytes,
            "n_edges_within_hops": list(self.n_edges_within_hops),
        }


class Request(ctypes.Structure):
    _fields_ = [("pos", ctypes.c_void_p), ("species", ctypes.c_void_p), ("n_atoms", ctypes.c_int32),
                ("box", ctypes.c_double * 3)]


class Timing(ctypes.Structure):
    _fields_ = [("latency_us", ctypes.c_double), ("queue_us", ctypes.c_double), ("batch_size", ctypes.c_int32)]


_lib = None


def lib():
    """Load libmlp.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(python -m paper_2506_04055_amd.build)")
    L = ctypes.CDLL(LIB_PATH)
    P, I32, I64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.mlp_last_error.restype = ctypes.c_char_p
    L.mlp_model_create.argtypes = [ctypes.c_char_p, P, ctypes.c_size_t, ctypes.c_int, ctypes.POINTER(P)]
    L.mlp_model_destroy.argtypes = [P]
    L.mlp_build_neighbors.argtypes = [P, P, P, I32, I32, P, ctypes.c_float, P, ctypes.POINTER(P)]
    L.mlp_nbr_destroy.argtypes = [P]
    L.mlp_nbr_edges.argtypes = [P, I32, P, P, I64, ctypes.POINTER(I64), P]
    L.mlp_energy_forces.argtypes = [P, P, P, I32, I32, P, P, P, P, P, ctypes.POINTER(Stats)]
    L.mlp_energy_forces_noalloc.argtypes = [P, P, P, I32, I32, P, P, P, P, P]
    L.mlp_nbr_check_displacement.argtypes = [P, P, I32, P, ctypes.POINTER(I32)]
    L.mlp_md_step.argtypes = [P, P, P, P, P, P, P, I32, P, ctypes.c_float, ctypes.c_float, P, P,
                              ctypes.POINTER(I32)]
    L.mlp_nvt_create.argtypes = [I32, ctypes.c_double, ctypes.c_double, I32, ctypes.POINTER(P)]
    L.mlp_nvt_destroy.argtypes = [P]
    L.mlp_nvt_read.argtypes = [P, P, P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), P]
    L.mlp_md_step_nvt.argtypes = [P, P, P, P, P, P, P, P, I32, P, ctypes.c_float, ctypes.c_float, P, P,
                                  ctypes.POINTER(I32)]
    L.mlp_server_create.argtypes = [P, ctypes.c_size_t, I32, ctypes.POINTER(P)]
    L.mlp_server_destroy.argtypes = [P]
    L.mlp_submit.argtypes = [P, ctypes.POINTER(Request), ctypes.POINTER(ctypes.c_uint64)]
    L.mlp_poll.argtypes = [P, ctypes.c_uint64, P, P, ctypes.POINTER(Timing)]
    L.mlp_profile_enable.argtypes = [I32]
    L.mlp_profile_reset.argtypes = []
    L.mlp_profile_read.argtypes = [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64)]
    for name in ("mlp_profile_enable", "mlp_profile_reset", "mlp_profile_read",
                 "mlp_model_create", "mlp_model_destroy", "mlp_build_neighbors", "mlp_nbr_destroy", "mlp_nbr_edges",
                 "mlp_energy_forces", "mlp_energy_forces_noalloc", "mlp_nbr_check_displacement", "mlp_md_step", "mlp_server_create", "mlp_server_destroy",
                 "mlp_submit", "mlp_poll", "mlp_nvt_create", "mlp_nvt_destroy", "mlp_nvt_read", "mlp_md_step_nvt"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc: int):
    if rc < 0:
        raise MLPError(rc, lib().mlp_last_error().decode(errors="replace"))
    return rc


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _box_arr(box):
    return (ctypes.c_double * 3)(*[float(b) for b in box])


# ---------------------------------------------------------------- C names

def mlp_model_create(header_json: str, weights: np.ndarray, precision: int = MLP_FP32):
    w = np.ascontiguousarray(weights, dtype=np.float32)
    h = ctypes.c_void_p()
    _check(lib().mlp_model_create(header_json.encode(), w.ctypes.data_as(ctypes.c_void_p), w.size,
                                  int(precision), ctypes.byref(h)))
    return h


def mlp_build_neighbors(model, pos_soa: torch.Tensor, species: torch.Tensor, n_local: int, box, skin: float,
                        nbr=None, stream=None):
    h = nbr if nbr is not None else ctypes.c_void_p()
    _check(lib().mlp_build_neighbors(model, _ptr(pos_soa), _ptr(species), int(pos_soa.shape[1]), int(n_local),
                                     _box_arr(box), float(skin), _stream(stream), ctypes.byref(h)))
    return h


def mlp_energy_forces(model, nbr, pos_soa, n_local, energy, forces=None, ghost_owner=None, atom_energy=None,
                      stats: bool = False, stream=None):
    st = Stats() if stats else None
    _check(lib().mlp_energy_forces(model, nbr, _ptr(pos_soa), int(pos_soa.shape[1]), int(n_local),
                                   _ptr(ghost_owner), _stream(stream), _ptr(energy), _ptr(forces),
                                   _ptr(atom_energy), ctypes.byref(st) if st is not None else None))
    return st.as_dict() if st is not None else None


def mlp_energy_forces_noalloc(model, nbr, pos_soa, n_local, energy, forces=None, ghost_owner=None,
                              atom_energy=None, stream=None):
    _check(lib().mlp_energy_forces_noalloc(model, nbr, _ptr(pos_soa), int(pos_soa.shape[1]), int(n_local),
                                           _ptr(ghost_owner), _stream(stream), _ptr(energy), _ptr(forces),
                                           _ptr(atom_energy)))


def mlp_nbr_edges(nbr, which: int = 0, stream=None):
    """Directed edges (dst, src) of the graph in the caller's numbering, as
    int64 numpy arrays sorted by (dst, src)."""
    n = ctypes.c_int64(0)
    rc = lib().mlp_nbr_edges(nbr, int(which), None, None, 0, ctypes.byref(n), _stream(stream))
    if rc < 0 and rc != -3:
        _check(rc)
    E = int(n.value)
    dst = torch.empty(max(E, 1), dtype=torch.int32, device="cuda")
    src = torch.empty(max(E, 1), dtype=torch.int32, device="cuda")
    _check(lib().mlp_nbr_edges(nbr, int(which), _ptr(dst), _ptr(src), E, ctypes.byref(n), _stream(stream)))
    d = dst[:E].cpu().numpy().astype(np.int64)
    s_ = src[:E].cpu().numpy().astype(np.int64)
    order = np.lexsort((s_, d))
    return d[order], s_[order]


def mlp_nbr_check_displacement(nbr, pos_soa, stream=None) -> bool:
    """True when some atom moved more than skin/2 since the last build."""
    ex = ctypes.c_int32(0)
    _check(lib().mlp_nbr_check_displacement(nbr, _ptr(pos_soa), pos_soa.shape[1], _stream(stream),
                                            ctypes.byref(ex)))
    return bool(ex.value)


def mlp_md_step(model, nbr, pos, vel, forces, inv_mass, species, box, skin, dt, energy, stream=None):
    rb = ctypes.c_int32(0)
    _check(lib().mlp_md_step(model, nbr, _ptr(pos), _ptr(vel), _ptr(forces), _ptr(inv_mass), _ptr(species),
                             int(pos.shape[1]), _box_arr(box), float(skin), float(dt), _stream(stream),
                             _ptr(energy), ctypes.byref(rb)))
    return bool(rb.value)


def mlp_md_step_nvt(model, nbr, nvt, pos, vel, forces, inv_mass, species, box, skin, dt, energy, stream=None):
    rb = ctypes.c_int32(0)
    _check(lib().mlp_md_step_nvt(model, nbr, nvt, _ptr(pos), _ptr(vel), _ptr(forces), _ptr(inv_mass),
                                 _ptr(species), int(pos.shape[1]), _box_arr(box), float(skin), float(dt),
                                 _stream(stream), _ptr(energy), ctypes.byref(rb)))
    return bool(rb.value)


class Thermostat:
    """Nose-Hoover chain state on the device (mlp_nvt_*)."""

    def __init__(self, n_dof: int, temperature: float, tau_fs: float, chain: int = 3):
        h = ctypes.c_void_p()
        _check(lib().mlp_nvt_create(int(n_dof), float(temperature), float(tau_fs), int(chain), ctypes.byref(h)))
        self.handle, self.chain = h, int(chain)

    def read(self, stream=None):
        """(xi, vxi, thermostat energy (eV), kinetic energy (eV)) after the last step."""
        xi = np.zeros(self.chain)
        vxi = np.zeros(self.chain)
        eth, ke = ctypes.c_double(), ctypes.c_double()
        _check(lib().mlp_nvt_read(self.handle, xi.ctypes.data, vxi.ctypes.data, ctypes.byref(eth), ctypes.byref(ke),
                                  _stream(stream)))
        return xi, vxi, eth.value, ke.value

    def close(self):
        if self.handle:
            lib().mlp_nvt_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mlp_profile_enable(on: bool = True):
    _check(lib().mlp_profile_enable(1 if on else 0))


def mlp_profile_reset():
    _check(lib().mlp_profile_reset())


def mlp_profile_read(kernel: str):
    """(total_ms, launches) of one named kernel since the last reset."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().mlp_profile_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
    return float(ms.value), int(n.value)


# ---------------------------------------------------------------- objects

class Model:
    """A model on the device (header + flat float32 weights)."""

    def __init__(self, header: dict, weights: np.ndarray, precision: str | int = "fp32"):
        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        self.header = header
        self.precision = precision
        self.handle = mlp_model_create(json.dumps(header, sort_keys=True), weights, precision)

    def __del__(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.mlp_model_destroy(self.handle)
            self.handle = None


class System:
    """One domain on the device: positions (SoA), species, box, neighbour
    handle and output buffers."""

    def __init__(self, model: Model, pos, species, box, n_local=None, skin: float = 1.0, ghost_owner=None,
                 device="cuda"):
        self.model = model
        pos = torch.as_tensor(np.asarray(pos, np.float32))
        self.n = pos.shape[0]
        self.n_local = self.n if n_local is None else int(n_local)
        self.pos = pos.t().contiguous().to(device)            # SoA (3, N)
        self.species = torch.as_tensor(np.asarray(species, np.int32)).to(device)
        self.box = [float(b) for b in box]
        self.skin = float(skin)
        self.ghost_owner = (None if ghost_owner is None
                            else torch.as_tensor(np.asarray(ghost_owner, np.int32)).to(device))
        self.energy = torch.zeros(1, dtype=torch.float64, device=device)
        self.forces = torch.zeros(3, self.n, dtype=torch.float32, device=device)
        self.nbr = None
        self.build()

    def build(self):
        self.nbr = mlp_build_neighbors(self.model.handle, self.pos, self.species, self.n_local, self.box,
                                       self.skin, self.nbr)

    def rebuild_if_needed(self) -> bool:
        """Rebuild the graph when an atom moved more than skin/2 since the
        last build (the graph is exact only below that)."""
        if mlp_nbr_check_displacement(self.nbr, self.pos):
            self.build()
            return True
        return False

    def set_positions(self, pos_aos):
        self.pos.copy_(torch.as_tensor(pos_aos, dtype=torch.float32, device=self.pos.device).t())

    def compute(self, forces: bool = True, stats: bool = False, atom_energy: bool = False):
        ae = torch.zeros(self.n, dtype=torch.float32, device=self.pos.device) if atom_energy else None
        st = mlp_energy_forces(self.model.handle, self.nbr, self.pos, self.n_local, self.energy,
                               self.forces if forces else None, self.ghost_owner, ae, stats)
        out = {"energy": self.energy, "forces": self.forces}
        if ae is not None:
            out["atom_energy"] = ae
        if st is not None:
            out["stats"] = st
        return out

    def __del__(self):
        if getattr(self, "nbr", None) is not None and _lib is not None:
            _lib.mlp_nbr_destroy(self.nbr)
            self.nbr = None


class MLPEnergy(torch.autograd.Function):
    """E(pos) with dE/dpos = -F from the library's adjoint pass.

    forward(pos_soa (3, N) float32 on the device, system) -> energy (float64).
    The graph is rebuilt first when the positions moved more than skin/2 from
    those of the last build, so any displacement gives the exact result.
    First derivatives only: a double backward raises."""

    @staticmethod
    def forward(ctx, pos_soa, system: System):
        system.pos.copy_(pos_soa.detach())
        system.rebuild_if_needed()
        system.compute(forces=True)
        ctx.save_for_backward(system.forces.clone())
        return system.energy.clone()

    @staticmethod
    @torch.autograd.function.once_differentiable
    def backward(ctx, grad_e):
        (F,) = ctx.saved_tensors
        return (-grad_e.to(F.dtype) * F), None


class Server:
    """Continuous-batching request server (mlp_server_create / mlp_submit /
    mlp_poll).  Requests are periodic systems given as host arrays."""

    def __init__(self, model: Model, hbm_budget_bytes: int, max_slots: int = 64):
        self.model = model
        self.handle = ctypes.c_void_p()
        _check(lib().mlp_server_create(model.handle, int(hbm_budget_bytes), int(max_slots),
                                       ctypes.byref(self.handle)))

    def submit(self, pos_aos, species, box) -> int:
        pos = np.ascontiguousarray(np.asarray(pos_aos, np.float32).T)       # SoA (3, N)
        sp = np.ascontiguousarray(species, np.int32)
        req = Request(pos.ctypes.data_as(ctypes.c_void_p), sp.ctypes.data_as(ctypes.c_void_p), pos.shape[1],
                      (ctypes.c_double * 3)(*[float(b) for b in box]))
        t = ctypes.c_uint64(0)
        _check(lib().mlp_submit(self.handle, ctypes.byref(req), ctypes.byref(t)))
        return int(t.value)

    def poll(self, ticket: int, n_atoms: int):
        """None while pending, else (energy, forces (N, 3) float32, timing dict)."""
        e = ctypes.c_double(0.0)
        F = np.empty((3, n_atoms), np.float32)
        tm = Timing()
        rc = lib().mlp_poll(self.handle, ctypes.c_uint64(ticket), ctypes.byref(e),
                            F.ctypes.data_as(ctypes.c_void_p), ctypes.byref(tm))
        if rc == MLP_PENDING:
            return None
        _check(rc)
        return float(e.value), F.T.copy(), {"latency_us": tm.latency_us, "queue_us": tm.queue_us,
                                            "batch_size": tm.batch_size}

    def close(self):
        if getattr(self, "handle", None) is not None and _lib is not None:
            _lib.mlp_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        self.close()
