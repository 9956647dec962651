#!/usr/bin/env python3
"""Throughput of the PaiNN energy/force path on one MI355X.

Headline workload: one GPU's domain share of a perturbed fcc crystal,
1,048,576 local atoms (64^3 cells, a = 4.05 A, Gaussian sigma = 0.05 A) plus
the ghost shell of periodic images within T rc = 15 A of the box (413,527
ghosts, 1,462,103 rows), one species, PaiNN T=3, F=128, K=20, rc = 5 A.  One
step = one energy + force evaluation of the domain as an MD step needs it:
per-step edge pruning of the skin-0.5 A graph, T-hop marks, forward, adjoint
forces, FP64 energy and the fold of ghost forces onto their owners; every
stage runs in the library's HIP kernels with inputs resident in HBM.  The
graph is built once before the timed steps (an MD engine rebuilds it only
when an atom has moved more than skin/2); the time of a build is reported
beside the step.  value = local atoms x steps / time.  The headline
precision is timed and the others are timed beside it.

Also measured in the same run:
  * the 24,000-atom water MD (velocity Verlet, both precisions);
  * the serving workload: seeded Poisson arrivals of solvated-peptide-like
    systems of U{500..20000} atoms (H/C/N/O 60/20/10/10 %, 1 g/cm^3), served
    with continuous batching; closed-loop saturated throughput, then p50/p99
    latency at offered loads of 0.5, 0.8 and 0.95 of it;
  * the slab, the aluminium NVT protocol and the largest system on one GPU;
  * the energy/force error against the FP64 oracle for each precision;
  * the CPU baseline: the FP64 oracle timed on the host's cores on bounded
    samples of the workloads.

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "atom-steps/s (energy+forces) at 1 MI355X, FP32 vs BF16; p50/p99 served latency"
PEAKS = {  # published MI355X figures
    "hbm_GBs": 8000.0,
    "fp32_vector_TFLOPs": 157.3,
    "fp32_mfma_TFLOPs": 157.3,
    "bf16_mfma_TFLOPs": 2500.0,
}
# dtype labels of the precision modes: node GEMM operands / radial filter operands
DTYPE = {"fp32": "f32", "bf16": "bf16x3", "bf16_node": "bf16-node/f32-filter",
         "bf16_node_x3": "bf16-node/bf16x3-filter", "bf16_fast": "bf16"}
NODE_BF16 = {"fp32": False, "bf16": True, "bf16_node": True, "bf16_node_x3": True, "bf16_fast": True}
FILTER_BF16 = {"fp32": False, "bf16": True, "bf16_node": False, "bf16_node_x3": True, "bf16_fast": True}


def per_edge_flops(F: int, K: int):
    """Algorithmic flops per directed edge within rc of the message kernels,
    (first layer, later layers), fma = 2 flops.
    Later layers: forward 6KF + 12F (the filter w, K -> 3F, and the messages:
    x = phi o w and the sums s += x_s, v += v_j x_vv + rhat x_vs); adjoint
    12KF + 28F (w and dw/dr recomputed, the gradients of phi_j, v_j, r and
    rhat).  First layer (v = 0, no gradient into the embedding; used where it
    is not factorised): forward 4KF + 9F (w_s, w_vs and their messages);
    adjoint 6KF + 18F (w_vs, dw_s/dr, dw_vs/dr and the geometric sums)."""
    return {"msg_fwd": (4 * K * F + 9 * F, 6 * K * F + 12 * F),
            "msg_bwd": (6 * K * F + 18 * F, 12 * K * F + 28 * F)}


def per_pass_bytes(F: int):
    """Algorithmic HBM bytes of the message kernels, (per edge, per active
    atom): every per-atom row touched once, every edge record once.
    Forward: per edge the geometry (16 B) and the column (4 B); per atom the
    gathered rows phi_s, phi_vs, u (5F floats, one read each), its own s and
    v (4F) and the outputs s1, v1 (4F), the row offsets and hop mark (8 B).
    Adjoint: per edge geometry, column and the edge sums written (36 B); per
    atom phi and v (6F), the gathered gradient rows (4F), the residual dv1
    (3F), the outputs dv and dphi (6F), offsets and hop mark (8 B)."""
    return {"msg_fwd": (20, 13 * F * 4 + 8), "msg_bwd": (36, 19 * F * 4 + 8)}


def node_flops_per_step(hops: list, F: int, T: int, n_local: int):
    """Algorithmic node-GEMM flops of one evaluation with per-layer active
    sets (Results, "Distributed potential computation": layer t's outputs are
    needed only within T - 1 - t hops of the locals).  Layer t: the message
    MLP (8F^2 per atom) of the source atoms within T - t hops (none in the
    first layer, whose phi depends on the species alone), the update block
    (22F^2) of the atoms within T - 1 - t hops; the adjoint the same again;
    readout (2 x F^2) on the locals.  hops[h] = atoms within <= h hops."""
    f = 0
    for t in range(T):
        if t > 0:
            f += 8 * F * F * hops[T - t]
        f += 22 * F * F * hops[T - 1 - t]
    return 2 * f + 2 * F * F * n_local


def source_hash(kernel_file: str) -> str:
    with open(os.path.join(ROOT, "paper_2506_04055_amd", "csrc", kernel_file), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def load_traffic(kernel: str, precision: str, workload: str = "fcc1m"):
    """HBM bytes per launch from committed PMC counter summaries, used only if
    every source the figure depends on (the kernel's file, and the neighbour
    build that fixes the atom order its gathers follow) is unchanged since the
    counters were taken."""
    p = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}_{precision}.json")
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except (OSError, ValueError):
        return None
    srcs = d.get("source_sha256_16")
    if not isinstance(srcs, dict):
        return None
    try:
        if any(source_hash(f) != h for f, h in srcs.items()):
            return None
    except OSError:
        return None
    return d.get("hbm_bytes_per_launch")


def layer_work(st: dict, T: int, factorised: bool):
    """Active edges and atoms of each message-kernel launch of one
    evaluation, in launch order: forward layer t (t = 0..T-1) reaches the
    destinations within T - 1 - t hops, the adjoint of layer t the sources
    within T - t hops.  The first layer is left out when it is factorised
    (then it has no message-kernel launch)."""
    eh, ah = st["n_edges_within_hops"], st["n_within_hops"]
    t0 = 1 if factorised else 0
    fwd = [(t, eh[T - 1 - t], ah[T - 1 - t]) for t in range(t0, T)]
    bwd = [(t, eh[T - t], ah[T - t]) for t in range(T - 1, t0 - 1, -1)]
    return {"msg_fwd": fwd, "msg_bwd": bwd}


def roofline_entry(kernel: str, work: list, F: int, K: int, avg_s: float, precision: str, workload: str):
    """Roofline of one message kernel: algorithmic flops and bytes per launch
    (averaged over its launches) against the binding roof, the larger of the
    two times bytes / HBM peak and flops / MFMA peak of its operand type."""
    first, later = per_edge_flops(F, K)[kernel]
    eb, ab = per_pass_bytes(F)[kernel]
    flops = sum((first if t == 0 else later) * e for t, e, _ in work) / len(work)
    byts = sum(eb * e + ab * a for _, e, a in work) / len(work)
    mfma_peak = PEAKS["bf16_mfma_TFLOPs" if FILTER_BF16[precision] else "fp32_mfma_TFLOPs"]
    t_hbm = byts / (PEAKS["hbm_GBs"] * 1e9)
    t_mfma = flops / (mfma_peak * 1e12)
    hbm = {"achieved": round(byts / avg_s / 1e9, 1), "peak": PEAKS["hbm_GBs"], "unit": "GB/s",
           "frac": round(byts / avg_s / 1e9 / PEAKS["hbm_GBs"], 4)}
    mf = {"achieved": round(flops / avg_s / 1e12, 3), "peak": mfma_peak, "unit": "TFLOP/s",
          "frac": round(flops / avg_s / 1e12 / mfma_peak, 4)}
    bound = "hbm" if t_hbm >= t_mfma else "mfma"
    r = dict(hbm if bound == "hbm" else mf)
    r.update({"bound": bound, "traffic": load_traffic(kernel, precision, workload), "kernel": kernel,
              "avg_launch_us": round(avg_s * 1e6, 2), "launches_per_step": len(work),
              "alg_bytes_per_launch": int(byts), "alg_flops_per_launch": int(flops),
              "other_roof": mf if bound == "hbm" else hbm,
              "work_per_launch": (f"per active edge {later} flop, {eb} B; per active atom {ab} B; active edges "
                                  f"per launch {[int(e) for _, e, _ in work]}, atoms {[int(a) for _, _, a in work]}")})
    return r


def run_md(mlp, synth, torch, precision: str, steps: int, warmup: int):
    """24,000-atom water, velocity Verlet dt = 0.5 fs from 300 K, skin 1 A:
    kick, drift, wrap, displacement check (rebuild when due), prune, forward,
    adjoint, kick per step."""
    import gc
    s, hdr, w = synth.workload("water24k_md")
    n = s.n_atoms
    skin, dt = 1.0, 0.5
    model = mlp.Model(hdr, w, precision)
    d = mlp.System(model, s.pos, s.species, s.box, skin=skin)
    vel = torch.as_tensor(synth.maxwell_velocities(s, 300.0, seed=0)).t().contiguous().cuda()
    inv_m = torch.as_tensor((1.0 / s.masses[s.species]).astype(np.float32)).cuda()
    d.compute()
    torch.cuda.synchronize()

    def step():
        return mlp.mlp_md_step(model.handle, d.nbr, d.pos, vel, d.forces, inv_m, d.species, d.box, skin, dt,
                               d.energy)

    for _ in range(warmup):
        step()
    rebuilds = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        rebuilds += step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    res = {"atom_steps_per_s": round(n * steps / (t1 - t0), 1), "ms_per_step": round(1e3 * (t1 - t0) / steps, 4),
           "steps": steps, "rebuilds": rebuilds}
    del d, model
    gc.collect()
    torch.cuda.empty_cache()
    return res


def run_domain(mlp, synth, torch, sysm, hdr, w, precision: str, steps: int, warmup: int, profile: bool):
    """The headline: energy + forces (+ fold) of one domain share per step on
    a graph built before the timed steps; with profile, HIP events around the
    message kernels during the timed steps and around the node GEMMs in a
    separate untimed pass."""
    import gc
    model = mlp.Model(hdr, w, precision)
    owner = sysm.owner if sysm.n_atoms > sysm.n_local else None
    torch.cuda.synchronize()
    tb0 = time.perf_counter()
    d = mlp.System(model, sysm.pos, sysm.species, sysm.box, n_local=sysm.n_local, skin=0.5, ghost_owner=owner)
    torch.cuda.synchronize()
    t_build = time.perf_counter() - tb0
    st = d.compute(stats=True)["stats"]
    for _ in range(warmup):
        d.compute()
    torch.cuda.synchronize()
    if profile:
        mlp.mlp_profile_reset()
        mlp.mlp_profile_enable(0b011)          # msg_fwd, msg_bwd
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        d.compute()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = {}
    if profile:
        mlp.mlp_profile_enable(0)
        kt = {k: mlp.mlp_profile_read(k) for k in ("msg_fwd", "msg_bwd")}
        extra = max(1, steps // 5)
        mlp.mlp_profile_reset()
        mlp.mlp_profile_enable(0b100)          # node GEMMs
        for _ in range(extra):
            d.compute()
        torch.cuda.synchronize()
        mlp.mlp_profile_enable(0)
        g_ms, g_n = mlp.mlp_profile_read("node_gemm")
        kt["node_gemm"] = (g_ms * steps / extra, g_n * steps // extra)
    # a rebuild of the graph plus one evaluation, for the build's share
    torch.cuda.synchronize()
    tr0 = time.perf_counter()
    d.build()
    d.compute()
    torch.cuda.synchronize()
    t_rebuild_eval = time.perf_counter() - tr0
    el = (t1 - t0) / steps
    res = {"value": sysm.n_local / el, "ms_per_step": 1e3 * el, "stats": st, "kt": kt,
           "ms_build_first": round(1e3 * t_build, 2), "ms_rebuild_plus_eval": round(1e3 * t_rebuild_eval, 2)}
    del d, model
    gc.collect()
    torch.cuda.empty_cache()
    return res


def domain_roofline(head: dict, hdr: dict, precision: str, steps: int, n_local: int):
    F, K, T = hdr["F"], hdr["K"], hdr["T"]
    kt, st = head["kt"], head["stats"]
    fact = kt["msg_bwd"][1] < (T - 0.5) * steps
    work = layer_work(st, T, fact)
    ent = {}
    for k in ("msg_fwd", "msg_bwd"):
        tot_ms, launches = kt[k]
        avg_s = tot_ms / max(launches, 1) / 1e3
        ent[k] = roofline_entry(k, work[k], F, K, avg_s, precision, "fcc1m")
    dom = max(("msg_fwd", "msg_bwd"), key=lambda k: kt[k][0])
    g_ms, g_n = kt["node_gemm"]
    nf = node_flops_per_step(st["n_within_hops"], F, T, n_local)
    peak = PEAKS["bf16_mfma_TFLOPs" if NODE_BF16[precision] else "fp32_mfma_TFLOPs"]
    tf = nf / (g_ms / steps / 1e3) / 1e12
    node = {"achieved": round(tf, 2), "peak": peak, "unit": "TFLOP/s", "frac": round(tf / peak, 4),
            "ms_per_step": round(g_ms / steps, 3), "launches_per_step": g_n / steps,
            "alg_flops_per_step": int(nf),
            "work": "per layer t: 8F^2 per source atom within T-t hops (t > 0) + 22F^2 per atom within T-1-t "
                    "hops, x2 for the adjoint, + 2F^2 per local atom (readout); node GEMMs run on every row"}
    return ent[dom], ent, node


def serve_bench(mlp, synth, precision: str, n_requests: int, loads=(0.5, 0.8, 0.95)):
    hdr, w = synth.make_weights(128, 20, 3, 4, seed=0)
    model = mlp.Model(hdr, w, precision)
    sizes, seeds = synth.serving_requests(n_requests, seed=1)
    systems = [synth.peptide_like(int(nn), int(sd)) for nn, sd in zip(sizes, seeds)]
    server = mlp.Server(model, hbm_budget_bytes=96 << 30, max_slots=64)

    def run(arrivals):
        t0 = time.perf_counter()
        pending = {}
        lat, batch = [], []
        k = 0
        while k < len(systems) or pending:
            now = time.perf_counter() - t0
            while k < len(systems) and (arrivals is None or arrivals[k] <= now):
                s = systems[k]
                pending[server.submit(s.pos, s.species, s.box)] = s.n_atoms
                k += 1
            done = []
            for t, na in pending.items():
                r = server.poll(t, na)
                if r is not None:
                    lat.append(r[2]["latency_us"])
                    batch.append(r[2]["batch_size"])
                    done.append(t)
            for t in done:
                del pending[t]
            if not done:
                time.sleep(0.0002)
        el = time.perf_counter() - t0
        lat = np.array(lat)
        return {"makespan_s": round(el, 3), "atoms_per_s": round(float(sizes.sum()) / el, 1),
                "requests_per_s": round(len(systems) / el, 2),
                "p50_ms": round(float(np.percentile(lat, 50)) / 1e3, 3),
                "p99_ms": round(float(np.percentile(lat, 99)) / 1e3, 3),
                "mean_batch": round(float(np.mean(batch)), 2)}

    run(None)                                  # warm-up pass (grows every buffer)
    closed = run(None)
    out = {"n_requests": n_requests, "closed_loop": closed, "offered": {}}
    rate = closed["requests_per_s"]
    for f in loads:
        arr = synth.poisson_arrivals(n_requests, f * rate, seed=1)
        out["offered"][str(f)] = run(arr)
    server.close()
    return out


def measure_eval(mlp, synth, torch, name: str, precision: str, reps: int = 5, skin: float = 0.5):
    """Energy + forces (+ ghost fold) of a whole domain per call."""
    import gc
    s, hdr, w = synth.workload(name)
    model = mlp.Model(hdr, w, precision)
    owner = s.owner if s.n_atoms > s.n_local else None
    d = mlp.System(model, s.pos, s.species, s.box, n_local=s.n_local, skin=skin, ghost_owner=owner)
    st = d.compute(stats=True)["stats"]
    d.compute()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        d.compute()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    res = {"n_local": s.n_local, "n_atoms": s.n_atoms, "ms_per_eval": round(1e3 * el, 3),
           "local_atom_evals_per_s": round(s.n_local / el, 1), "n_edges_rc": int(st["n_edges"]),
           "n_within_hops": st["n_within_hops"][: hdr["T"] + 1], "device_GB": round(st["device_bytes"] / 2**30, 2)}
    del d, model
    gc.collect()
    torch.cuda.empty_cache()
    return res


def measure_al_nvt(mlp, synth, torch, precision: str, n_cells: int = 35, equil: int = 100, prod: int = 250):
    """The paper's aluminium MD protocol (Methods, "Molecular Dynamics
    Simulations"): fcc a = 4.065 A replicated n_cells^3 (4 n_cells^3 atoms;
    35 gives 171,500, the most the paper's framework ran for PaiNN on one
    80 GB A100, Table 2), NVT with a Nose-Hoover chain (damping 1.1 ps) at
    1000 K, dt = 3 fs, skin 2.0 A, 100 equilibration then 250 timed
    production steps."""
    import gc
    s, hdr, w = synth.al_nvt_workload(n_cells)
    n = s.n_atoms
    model = mlp.Model(hdr, w, precision)
    d = mlp.System(model, s.pos, s.species, s.box, skin=2.0)
    vel = torch.as_tensor(synth.maxwell_velocities(s, 1000.0, seed=0)).t().contiguous().cuda()
    inv_m = torch.as_tensor((1.0 / s.masses[s.species]).astype(np.float32)).cuda()
    th = mlp.Thermostat(3 * n - 3, 1000.0, 1100.0, 3)
    d.compute()

    def step():
        return mlp.mlp_md_step_nvt(model.handle, d.nbr, th.handle, d.pos, vel, d.forces, inv_m, d.species, d.box,
                                   2.0, 3.0, d.energy)

    for _ in range(equil):
        step()
    torch.cuda.synchronize()
    _, _, eth0, ke0 = th.read()
    e0 = d.energy.item()
    rebuilds, temps = 0, []
    t0 = time.perf_counter()
    for k in range(prod):
        rebuilds += step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    _, _, eth1, ke1 = th.read()
    e1 = d.energy.item()
    kb = 8.617333262e-5
    res = {"atoms": n, "precision": precision, "steps_equil": equil, "steps_prod": prod,
           "atom_steps_per_s": round(n * prod / el, 1), "ms_per_step": round(1e3 * el / prod, 3),
           "T_end_K": round(2 * ke1 / ((3 * n - 3) * kb), 1), "rebuilds_prod": rebuilds,
           "extended_energy_change_per_atom_eV": (e1 + ke1 + eth1 - e0 - ke0 - eth0) / n,
           "finite": bool(np.isfinite(e1) and np.isfinite(ke1))}
    th.close()
    del d, model
    gc.collect()
    torch.cuda.empty_cache()
    return res


def measure_capacity(mlp, synth, torch, n_cells: int = 116):
    """One energy + force evaluation of the largest fcc-Al PaiNN system
    (F = 64, T = 4, skin 2.0 A) that fits one MI355X: the analogue of the
    paper's "maximum atoms on one GPU" (Table 2)."""
    import gc
    s, hdr, w = synth.al_nvt_workload(n_cells)
    try:
        model = mlp.Model(hdr, w, "bf16")
        d = mlp.System(model, s.pos, s.species, s.box, skin=2.0)
        st = d.compute(stats=True)["stats"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d.compute()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res = {"atoms": s.n_atoms, "device_GB": round(st["device_bytes"] / 2**30, 2),
               "ms_per_eval": round(1e3 * el, 1), "n_edges_rc": int(st["n_edges"]),
               "finite": bool(np.isfinite(d.energy.item()))}
        del d, model
    except mlp.MLPError as e:
        res = {"atoms": s.n_atoms, "error": str(e)[:300]}
    gc.collect()
    torch.cuda.empty_cache()
    return res


def measure_capacity_eq(mlp, synth, torch, kind: str, n_cells: int):
    """One energy + force evaluation of a large fcc-Al system with an
    equivariant model at the paper's settings (Allegro: one layer, l_max 3;
    MACE: two layers, correlation 3, l_max 3), split bf16, skin 2.0 A: the
    analogue of the paper's "maximum atoms on one GPU" (Table 2) for these
    models."""
    import gc
    s = synth.fcc_crystal(n_cells, a=4.065, sigma=0.1, seed=0)
    h, w = (synth.make_allegro_weights if kind == "allegro" else synth.make_mace_weights)(1, seed=0)
    try:
        model = mlp.Model(h, w, "bf16")
        d = mlp.System(model, s.pos, s.species, s.box, skin=2.0)
        st = d.compute(stats=True)["stats"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d.compute()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res = {"atoms": s.n_atoms, "device_GB": round(st["device_bytes"] / 2**30, 2),
               "ms_per_eval": round(1e3 * el, 1), "n_edges_rc": int(st["n_edges"]),
               "finite": bool(np.isfinite(d.energy.item()))}
        del d, model
    except mlp.MLPError as e:
        res = {"atoms": s.n_atoms, "error": str(e)[:300]}
    gc.collect()
    torch.cuda.empty_cache()
    return res


def measure_allegro(mlp, synth, torch, precision: str, n_cells: int = 49, reps: int = 5):
    """Allegro with one tensor-product layer (the paper's setting for water and
    aluminium: l_max = 3, 8 radial functions, polynomial envelope p = 2,
    two-body MLP [8, 16, 32] into a 64-wide latent, 5 A cutoff) on a periodic
    fcc aluminium crystal of 4 n_cells^3 atoms (49 gives 470,596, the most
    the paper's framework ran for Allegro aluminium on one 80 GB A100,
    Table 2), a = 4.065 A, sigma = 0.1 A: energy + forces per call on a
    graph built with a 0.5 A skin."""
    import gc
    s = synth.fcc_crystal(n_cells, a=4.065, sigma=0.1, seed=0)
    h, w = synth.make_allegro_weights(1, seed=0)
    model = mlp.Model(h, w, precision)
    d = mlp.System(model, s.pos, s.species, s.box, skin=0.5)
    st = d.compute(stats=True)["stats"]
    d.compute()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        d.compute()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    res = {"atoms": s.n_atoms, "precision": precision, "ms_per_eval": round(1e3 * el, 3),
           "atom_steps_per_s": round(s.n_atoms / el, 1), "n_edges_rc": int(st["n_edges"]),
           "device_GB": round(st["device_bytes"] / 2**30, 2)}
    del d, model
    gc.collect()
    torch.cuda.empty_cache()
    return res


def measure_mace(mlp, synth, torch, precision: str, n_cells: int = 33, reps: int = 5):
    """MACE with two layers (the paper's setting: correlation order 3,
    l_max = 3, 32 scalar and 32 vector channels, 8 radial functions,
    polynomial envelope p = 6, 5 A cutoff) on a periodic fcc aluminium crystal
    of 4 n_cells^3 atoms (33 gives 143,748, the per-GPU load of the paper's
    MACE aluminium weak-scaling runs), a = 4.065 A, sigma = 0.1 A: energy +
    forces per call on a graph built with a 0.5 A skin."""
    import gc
    s = synth.fcc_crystal(n_cells, a=4.065, sigma=0.1, seed=0)
    h, w = synth.make_mace_weights(1, seed=0)
    model = mlp.Model(h, w, precision)
    d = mlp.System(model, s.pos, s.species, s.box, skin=0.5)
    st = d.compute(stats=True)["stats"]
    d.compute()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        d.compute()
    torch.cuda.synchronize()
    el = (time.perf_counter() - t0) / reps
    res = {"atoms": s.n_atoms, "precision": precision, "ms_per_eval": round(1e3 * el, 3),
           "atom_steps_per_s": round(s.n_atoms / el, 1), "n_edges_rc": int(st["n_edges"]),
           "device_GB": round(st["device_bytes"] / 2**30, 2)}
    del d, model
    gc.collect()
    torch.cuda.empty_cache()
    return res


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(synth, reps: int = 3):
    """The FP64 oracle timed on the host cores (median of reps) on bounded
    samples: a 16^3-cell fcc domain share with its 15 A ghost shell (the
    headline workload at 1/64 of its locals), the 192-atom water box, and a
    few serving requests spanning the size range."""
    from oracle import oracle as O
    out = {}

    def med(fn, label=""):
        ts = []
        for _ in range(reps):
            t = time.perf_counter()
            fn()
            ts.append(time.perf_counter() - t)
            print(f"bench: CPU baseline {label} {ts[-1]:.2f} s", file=sys.stderr, flush=True)
        return float(np.median(ts))

    dom = synth.fcc_crystal(16, seed=0, ghost_depth=15.0)
    hdr, w = synth.make_weights(128, 20, 3, 1, seed=0)
    t = med(lambda: O.energy_forces(hdr, w, dom.pos, dom.species, np.zeros(3), n_local=dom.n_local), "fcc16")
    out["fcc_domain_share"] = {"n_local": dom.n_local, "n_atoms": dom.n_atoms, "s_per_eval": round(t, 3),
                               "local_atom_steps_per_s": round(dom.n_local / t, 1)}
    s1, h1, w1 = synth.workload("water192")
    t = med(lambda: O.energy_forces(h1, w1, s1.pos, s1.species, s1.box), "water192")
    out["water192"] = {"s_per_eval": round(t, 4), "atom_steps_per_s": round(s1.n_atoms / t, 1)}
    h5, w5 = synth.make_weights(128, 20, 3, 4, seed=0)
    sizes, seeds = synth.serving_requests(2000, seed=1)
    order = np.argsort(sizes)
    pick = order[np.linspace(0, len(order) - 1, 4).astype(int)]
    tot_atoms, tot_t = 0, 0.0
    for k in pick:
        s = synth.peptide_like(int(sizes[k]), int(seeds[k]))
        tot_t += med(lambda: O.energy_forces(h5, w5, s.pos, s.species, s.box), f"request {s.n_atoms}")
        tot_atoms += s.n_atoms
    out["serving_sample"] = {"requests": [int(sizes[k]) for k in pick], "atoms_per_s": round(tot_atoms / tot_t, 1)}
    return out, O.num_threads()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--precision", default="bf16", choices=sorted(DTYPE),
                    help="headline precision mode; fp32 and bf16_node are timed beside it")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--single", action="store_true", help="time the headline precision only")
    ap.add_argument("--requests", type=int, default=2000)
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the water MD, slab, NVT, capacity and Allegro timings")
    ap.add_argument("--allegro-only", action="store_true", help="time only the Allegro workload (a quick check)")
    ap.add_argument("--mace-only", action="store_true", help="time only the MACE workload (a quick check)")
    ap.add_argument("--water-only", action="store_true",
                    help="time only the 24,000-atom water MD workload (100 velocity-Verlet steps)")
    ap.add_argument("--capacity-only", type=int, default=0, metavar="N",
                    help="evaluate only the 4 N^3-atom fcc-Al system of the capacity point (PaiNN F=64, T=4, or "
                         "the model --capacity-model names)")
    ap.add_argument("--capacity-model", default="painn", choices=["painn", "mace", "allegro"])
    ap.add_argument("--serving-only", action="store_true",
                    help="time only the serving workload (closed loop and offered loads)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="first copy 256 MiB device to device (calibrates the HBM byte counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: this build evaluates one GPU's domain; runs on more than one GPU are not part of "
              "it (the sharding design is described in DESIGN.md).", file=sys.stderr)
        sys.exit(2)
    os.environ.setdefault("OMP_PROC_BIND", "close")   # the oracle's threads (CPU baseline)

    import torch
    from paper_2506_04055_amd import mlp, synth

    if args.copy_probe:
        a = torch.ones(64 << 20, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.allegro_only:
        print(json.dumps({p: measure_allegro(mlp, synth, torch, p) for p in (args.precision, "fp32")}), flush=True)
        return
    if args.capacity_only:
        if args.capacity_model == "painn":
            r = measure_capacity(mlp, synth, torch, args.capacity_only)
        else:
            r = measure_capacity_eq(mlp, synth, torch, args.capacity_model, args.capacity_only)
        print(json.dumps(r), flush=True)
        return
    if args.serving_only:
        print(json.dumps(serve_bench(mlp, synth, args.precision, args.requests)), flush=True)
        return
    if args.mace_only:
        print(json.dumps({p: measure_mace(mlp, synth, torch, p) for p in (args.precision, "fp32")}), flush=True)
        return
    if args.water_only:
        print(json.dumps({args.precision: run_md(mlp, synth, torch, args.precision, 100, 10)}), flush=True)
        return
    dom, hdr, w = synth.workload("fcc1m_ghost")
    print(f"bench: headline fcc domain, {dom.n_local} locals, {dom.n_atoms} rows, {args.precision}", file=sys.stderr,
          flush=True)
    head = run_domain(mlp, synth, torch, dom, hdr, w, args.precision, args.steps, args.warmup, profile=True)
    roof, edge, node = domain_roofline(head, hdr, args.precision, args.steps, dom.n_local)
    st = head["stats"]
    out = {
        "metric": METRIC, "value": round(head["value"], 1), "unit": "atom-steps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic (seeded perturbed fcc crystal, random-init PaiNN weights)",
        "config": {"workload": "one GPU's domain share: perturbed fcc 64^3 cells (1,048,576 local atoms, a=4.05 A, "
                               "sigma=0.05 A) + 15 A ghost shell (413,527 ghosts), PaiNN T=3 F=128 K=20 rc=5 A, "
                               "1 species, skin 0.5 A, ghost forces folded onto owners",
                   "n_local": dom.n_local, "n_atoms": dom.n_atoms, "T": hdr["T"], "F": hdr["F"], "K": hdr["K"],
                   "rc": hdr["r_c"], "precision": args.precision},
        "roofline": roof,
        "edge_passes": edge,
        "node_gemm_mfma": node,
        "kernels": {k: {"ms_per_step": round(v[0] / args.steps, 4), "launches_per_step": v[1] / args.steps}
                    for k, v in head["kt"].items()},
        "graph": {"n_edges_rc": int(st["n_edges"]), "n_edges_skin": int(st["n_edges_skin"]),
                  "n_within_hops": st["n_within_hops"][: hdr["T"] + 1],
                  "n_edges_within_hops": st["n_edges_within_hops"][: hdr["T"] + 1],
                  "device_GB": round(st["device_bytes"] / 2**30, 2),
                  "ms_first_build": head["ms_build_first"], "ms_rebuild_plus_eval": head["ms_rebuild_plus_eval"]},
    }
    others = [] if args.single else [p for p in ("fp32", "bf16_node", "bf16") if p != args.precision]
    out["other_precisions"] = {}
    for p in others:
        o = run_domain(mlp, synth, torch, dom, hdr, w, p, args.steps, args.warmup, profile=False)
        out["other_precisions"][p] = {"dtype": DTYPE[p], "value": round(o["value"], 1),
                                      "ms_per_step": round(o["ms_per_step"], 4)}
    del dom

    if not args.no_extra:
        print("bench: extra workloads", file=sys.stderr, flush=True)
        out["other_workloads"] = {
            "water24k_md": {p: run_md(mlp, synth, torch, p, 100, 10) for p in [args.precision] + others},
            "water_slab_48k": {p: measure_eval(mlp, synth, torch, "slab48k", p, reps=5, skin=1.0)
                               for p in [args.precision] + others},
            "al_fcc_nvt_171500": measure_al_nvt(mlp, synth, torch, args.precision),
            "max_atoms_one_gpu_al_fcc_painn_T4_F64": measure_capacity(mlp, synth, torch),
            # 4 n^3 atoms near the device's capacity at skin 2.0 A (measured
            # footprints: MACE 259.6 KiB, Allegro 323 KiB per atom)
            "max_atoms_one_gpu_al_fcc_mace": measure_capacity_eq(mlp, synth, torch, "mace", 64),
            "max_atoms_one_gpu_al_fcc_allegro": measure_capacity_eq(mlp, synth, torch, "allegro", 59),
            "allegro_al_fcc_470596": {p: measure_allegro(mlp, synth, torch, p) for p in [args.precision, "fp32"]},
            "mace_al_fcc_143748": {p: measure_mace(mlp, synth, torch, p) for p in [args.precision, "fp32"]},
        }

    if not args.no_serving:
        print("bench: serving", file=sys.stderr, flush=True)
        out["serving"] = serve_bench(mlp, synth, args.precision, args.requests)

    if not args.no_cpu_baseline:
        print("bench: CPU baseline", file=sys.stderr, flush=True)
        from oracle import oracle as O
        cb, threads = cpu_baseline(synth)
        out["cpu_baseline"] = {
            "value": cb["fcc_domain_share"]["local_atom_steps_per_s"], "unit": "atom-steps/s", "cores": threads,
            "kind": "oracle",
            "sample": (f"median of 3 FP64 energy+force evaluations of a 16^3-cell fcc domain share with its 15 A "
                       f"ghost shell ({cb['fcc_domain_share']['n_local']} locals, {cb['fcc_domain_share']['n_atoms']} "
                       f"rows; the headline workload at 1/64 of its locals): {cb['fcc_domain_share']['s_per_eval']} s "
                       f"each; OMP_PROC_BIND={os.environ.get('OMP_PROC_BIND')}"),
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "other_samples": cb}
        # error of each precision against the oracle on the 12^3-cell domain share (every row)
        acc = {}
        sm = synth.fcc_crystal(12, seed=0, ghost_depth=15.0)
        E_ref, F_ref = O.energy_forces(hdr, w, sm.pos, sm.species, np.zeros(3), n_local=sm.n_local)
        F_ref = O.fold_ghost_forces(F_ref, sm.n_local, sm.owner)
        for prec in [args.precision] + others:
            model = mlp.Model(hdr, w, prec)
            d = mlp.System(model, sm.pos, sm.species, sm.box, n_local=sm.n_local, skin=0.5, ghost_owner=sm.owner)
            d.compute()
            torch.cuda.synchronize()
            E0 = float(d.energy.item())
            F0 = d.forces.t().cpu().numpy().astype(np.float64)
            acc[prec] = {"force_rel_rms": float(np.linalg.norm(F0 - F_ref) / np.linalg.norm(F_ref)),
                         "force_row_max": float(np.linalg.norm(F0 - F_ref, axis=1).max()
                                                / np.sqrt((F_ref ** 2).sum(1).mean())),
                         "energy_rel": float(abs(E0 - E_ref) / abs(E_ref))}
            del d, model
        out["accuracy_vs_oracle"] = dict(acc, at="12^3-cell fcc domain share + 15 A shell (same model and "
                                                 "generator as the headline), every row, folded")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
