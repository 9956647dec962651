"""Shared tolerances and comparisons of the GPU parity tests.

Tolerances per precision mode (operand forms of the node GEMMs / the radial
filter; every accumulation FP32, energy sums FP64):

* fp32 (FP32 / FP32): forces 1e-5 relative RMS, the target for this path;
  energy 5e-6 relative, half of it.  The energy is summed in FP64, but each
  per-atom energy is the output of the FP32 network and carries the rounding
  of its activations (hundreds of FP32 terms per product, three layers), the
  same rounding that the forces carry: measured 1.2e-6 to 2.1e-6 for the
  128-feature water models, depending on the order of the sums in the
  message kernels.  One dropped edge term moves a 192-atom box's energy by
  about 1e-4, so the bound still sees it.
* bf16 = bf16x3 (split bf16 / split bf16): each operand is hi + lo with
  |x - hi - lo| <= 2^-18 |x| and the dropped lo*lo product is <= 2^-18 of the
  product, so a product carries ~2^-17 (7.6e-6) relative error against
  FP32's 2^-24.  Forces 5e-4 and energy 1e-4 relative: ten times the
  measured errors (4.8e-5 / 1.5e-5 at 24k water), far below the 1e-2 target,
  so a dropped hi*lo product or a broken tile fails.
* bf16_node, bf16_node_x3 (plain bf16 node GEMMs; FP32 or split-bf16
  filter): node-GEMM operands rounded to 2^-9.  With these random-init
  weights the rounding is amplified through the quadratic <Uv, Vv> term and
  the norm: measured 7e-3 to 8e-3 on the fcc domains and the serving
  systems, 1.4e-2 (192 atoms) to 3.4e-2 (24k, slab 2.9e-2) on the water
  boxes, so this form meets the 1e-2 target only on some workloads.  It is
  held to 5e-2 on forces and energy, a regression bound and not the target;
  the split form above is the one that meets 1e-2 everywhere.
* bf16_fast (plain bf16 node GEMMs and filter): errors as bf16_node (the
  node GEMMs dominate), held to the same 5e-2 regression bound.

Per-row bound: max_k |F_k - F_ref,k| / max(|F_ref,k|, rms_k |F_ref,k|) <=
ROW_TOL[mode].  A global relative RMS cannot see one wrong row among 24,000
(its share is ~1/sqrt(N)).  Rounding in a row scales with the size of the
terms that make it, and force magnitudes are heavy tailed (close contacts:
the largest row is ~40x the RMS in the 24k water box and ~90x in the slab),
so each row is measured against its own magnitude, floored at the RMS for
rows whose net force is small.  Rows whose edge terms cancel carry more
relative rounding than the global figure: the worst row of the FP32 slab
result is 3.6e-4 against a global 8.6e-6.  The per-row bound is therefore
100x the global tolerance, capped at 0.2; for the plain-bf16 node modes,
whose worst rows reach 0.53 of their own force at 24k water, it is 0.75.
Every cap is below 1, so a zeroed or sign-flipped row fails in every mode,
and so does, in the FP32 and split modes, any row wrong by more than a few
per cent (a dropped edge, a wrong index).
"""
from __future__ import annotations

import numpy as np

TOL = {  # mode: (energy relative to |E_ref|, force relative RMS)
    "fp32": (5e-6, 1e-5),
    "bf16": (1e-4, 5e-4),
    "bf16x3": (1e-4, 5e-4),
    "bf16_fast": (5e-2, 5e-2),
    "bf16_node": (5e-2, 5e-2),
    "bf16_node_x3": (5e-2, 5e-2),
}
ROW_TOL = {mode: (min(100 * f, 0.2) if f < 1e-2 else 0.75) for mode, (_, f) in TOL.items()}
# per-atom energies, and force rows of a homogeneous crystal (no close
# contacts): the largest of N per-row errors within 20x the global bound
ROW = 20.0


def rel_rms(F, Fref) -> float:
    return float(np.linalg.norm(F - Fref) / np.linalg.norm(Fref))


def row_err(F, Fref, where: bool = False):
    """max_k |F_k - F_ref,k| / max(|F_ref,k|, rms_k |F_ref,k|); with where=True
    also the worst row and its |F_ref,k| / rms."""
    d = np.linalg.norm(np.asarray(F) - np.asarray(Fref), axis=1)
    m = np.linalg.norm(np.asarray(Fref), axis=1)
    rms = np.sqrt((m ** 2).mean())
    r = d / np.maximum(m, rms)
    k = int(np.argmax(r))
    return (float(r[k]), k, float(m[k] / rms)) if where else float(r[k])


def check(label: str, mode: str, E, E_ref, F, F_ref, e_scale: float = 1.0, f_scale: float = 1.0):
    """Assert energy, global and per-row force errors of one result against
    the mode's tolerances (optionally scaled); print the measured values."""
    et, ft = TOL[mode]
    et *= e_scale
    ft *= f_scale
    fe = rel_rms(F, F_ref)
    re_, k, mk = row_err(F, F_ref, where=True)
    ee = abs(E - E_ref) / abs(E_ref)
    rt = min(ROW_TOL[mode] * f_scale, 0.75)
    print(f"[measured] {label} {mode}: force rel RMS {fe:.2e} (tol {ft:.0e}), per-row max {re_:.2e} "
          f"(tol {rt:.0e}; row {k}, |F_ref| = {mk:.1f} rms), energy rel {ee:.2e} (tol {et:.0e})",
          flush=True)
    assert ee <= et, f"{label} {mode}: energy error {ee:.3e} > {et:.1e}"
    assert fe <= ft, f"{label} {mode}: force error {fe:.3e} > {ft:.1e}"
    assert re_ <= rt, f"{label} {mode}: per-row force error {re_:.3e} > {rt:.1e}"
    return fe, re_, ee


def ulp32(x: float) -> float:
    return float(np.spacing(np.float32(abs(x))))


def check_neighbors_fp64(oracle, label: str, dst, src, pos, box, cutoff: float, coord_max: float):
    """GPU directed pairs (dst <- src) against the FP64 brute-force set of
    every pair with 0 < |r_j - r_i| < cutoff (minimum image in periodic
    dimensions; cutoff < L/2 there, so at most one image qualifies).

    The device decides each pair in float32: the coordinate difference is
    rounded once (at most half an ulp of the largest coordinate magnitude in
    play, which the periodic fold can reach) and r^2 by a fused chain (a few
    ulps of cutoff^2).  Pairs whose FP64 distance lies within
    band = 2 ulp(coord_max) + 8 ulp(cutoff) of the cutoff may therefore fall
    either way; every other pair must agree.  Returns the number of pairs in
    the band that differ."""
    p = np.asarray(pos, np.float64)
    bx = np.asarray(box, np.float64)
    rd, rs, _ = oracle.neighbors(p, bx, cutoff)
    n = p.shape[0]
    key_g = np.asarray(dst, np.int64) * n + np.asarray(src, np.int64)
    key_r = rd.astype(np.int64) * n + rs.astype(np.int64)
    assert np.unique(key_r).size == key_r.size, "reference holds a pair twice (cutoff >= L/2?)"
    assert np.unique(key_g).size == key_g.size, f"{label}: GPU graph holds a pair twice"
    only_g = np.setdiff1d(key_g, key_r)
    only_r = np.setdiff1d(key_r, key_g)
    band = 2 * ulp32(coord_max) + 8 * ulp32(cutoff)

    def dist(keys):
        i, j = keys // n, keys % n
        d = p[j] - p[i]
        for k in range(3):
            if bx[k] > 0:
                d[:, k] -= bx[k] * np.round(d[:, k] / bx[k])
        return np.sqrt((d * d).sum(1))

    dg, dr = dist(only_g), dist(only_r)
    print(f"[measured] {label}: {key_r.size} FP64 pairs, {only_g.size} GPU-only and {only_r.size} FP64-only "
          f"pairs, all within {band:.1e} A of the cutoff" if (np.all(np.abs(dg - cutoff) <= band)
                                                              and np.all(np.abs(dr - cutoff) <= band))
          else f"[measured] {label}: pairs outside the band", flush=True)
    assert np.all(dg >= cutoff - band) and np.all(np.abs(dg - cutoff) <= band), \
        f"{label}: GPU pairs beyond the cutoff band: {np.sort(dg)[-5:]}"
    assert np.all(np.abs(dr - cutoff) <= band), f"{label}: FP64 pairs missing on the GPU: {np.sort(dr)[:5]}"
    return int(only_g.size + only_r.size)
