"""FP64 CPU oracle for the single-layer Allegro energy and its forces.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark import this module.  It imports nothing from the
GPU package, and the GPU package never imports it.

The paper deploys Allegro (Methods, "Chosen Architectures": an edge-centric,
strictly local equivariant model whose messages pass only between directed
edges that share their central atom) with one tensor-product layer,
l_max = 3, 8 radial basis functions, a polynomial envelope of order 2 and a
5 A cutoff for water and aluminium ("Training Details"), and gives 64 as the
hidden MLP width and 8, 16, 32 as the embedding widths, read here as a
two-body MLP of widths [8, 16, 32] into a 64-wide latent.  The layer equations are those
of the cited Allegro paper, which the paper does not print; the reading used
here, per directed edge e = (i <- j) with 0 < r = |r_j - r_i| < r_c and
rhat = (r_j - r_i) / r:

  x = r / r_c,  u(r) = 1 - (p+1)(p+2)/2 x^p + p(p+2) x^(p+1) - p(p+1)/2 x^(p+2)
  B_k(r) = sqrt(2 / r_c) sin(k pi r / r_c) / r * u(r),   k = 1..n_basis
  x0 = u(r) * MLP_2b([onehot(Z_i) | onehot(Z_j) | B(r)])          (64 wide)
  w0 = Wv x0,  we = We x0                    (one weight per channel c)
  V_e[c, m]   = w0_e[c] Y_(l_c, m)(rhat_e)   (tensor features of the edge)
  env_i[c, m] = nu sum_(k: edges i <- k) we_(ik)[c] Y_(l_c, m)(rhat_ik)
  S_e[c] = 1/(2 l_c + 1) sum_m V_e[c, m] env_i[c, m]
                                             (the scalar outputs l x l -> 0
                                              of the tensor product)
  x1 = (x0 + u(r) MLP_lat([x0 | S_e])) / sqrt(2)
  E_e = u(r) MLP_out(x1);   U_i = sum_(e = (i <- j)) E_e;   E = sum_(i local) U_i

(the envelope on E_e makes every edge term vanish with its first two
derivatives at r_c also when the MLPs carry biases), with
component-normalised real spherical harmonics (sum_m Y_lm^2 = 2l + 1)
and channel counts n_l per degree l = 0..l_max.  In a single layer the
energy needs only the scalar outputs of the tensor product; its tensor
outputs feed a next layer that does not exist.  By the addition theorem,
sum_m Y_lm(a) Y_lm(b) = (2l + 1) P_l(a . b), so

  S_e[c] = nu w0_e[c] sum_(k: edges i <- k) we_(ik)[c] P_(l_c)(rhat_e . rhat_ik),

the form evaluated here: a plain sum over the pairs of edges sharing their
central atom with Legendre polynomials of the bond angle (no spherical
harmonics appear in this file).  Forces F = -dE/dr come from torch float64
reverse-mode differentiation of this program.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import oracle as _base


def layout(h: dict):
    """(name, shape) of every weight block in storage order; matrices are
    [out][in] row-major."""
    S, nb = h["n_species"], h["n_basis"]
    d = list(h["mlp_2b"])
    NC = sum(h["channels"])
    D, L, O = d[-1], h["latent_hidden"], h["out_hidden"]
    out, prev = [], 2 * S + nb
    for q, w in enumerate(d):
        out += [(f"2b_W{q + 1}", (w, prev)), (f"2b_b{q + 1}", (w,))]
        prev = w
    out += [("Wv", (NC, D)), ("We", (NC, D)),
            ("lat_W1", (L, D + NC)), ("lat_b1", (L,)), ("lat_W2", (D, L)), ("lat_b2", (D,)),
            ("out_W1", (O, D)), ("out_b1", (O,)), ("out_w2", (O,)), ("out_b2", (1,))]
    return out


def n_weights(h: dict) -> int:
    return int(sum(np.prod(s) for _, s in layout(h)))


def _unpack(h: dict, w) -> dict:
    w = torch.as_tensor(np.asarray(w, np.float32).astype(np.float64))
    if w.numel() != n_weights(h):
        raise ValueError("weight count does not match the header")
    out, o = {}, 0
    for name, shape in layout(h):
        k = int(np.prod(shape))
        out[name] = w[o:o + k].reshape(shape)
        o += k
    return out


def envelope(x, p: int):
    """Polynomial envelope of order p on x = r / r_c in [0, 1]."""
    return (1.0 - (p + 1) * (p + 2) / 2.0 * x ** p + p * (p + 2) * x ** (p + 1)
            - p * (p + 1) / 2.0 * x ** (p + 2))


def legendre(l: int, t):
    """Legendre polynomial P_l(t) by Bonnet's recursion."""
    p0, p1 = torch.ones_like(t), t
    if l == 0:
        return p0
    for k in range(1, l):
        p0, p1 = p1, ((2 * k + 1) * t * p1 - k * p0) / (k + 1)
    return p1


def _silu(x):
    return x * torch.sigmoid(x)


def energy_forces(header: dict, weights, pos, species, box, n_local: int | None = None, per_atom: bool = False,
                  edges=None):
    """E = sum_{i < n_local} U_i and F = -dE/dr of every atom (FP64).

    edges: optional (dst, src, dvec) to use instead of the brute-force
    neighbour list of the oracle (dvec = r_src + image shift - r_dst)."""
    h = header
    W = _unpack(h, weights)
    S, nb, p, rc, nu = h["n_species"], h["n_basis"], h["envelope_p"], float(h["r_c"]), float(h["env_scale"])
    ch = list(h["channels"])
    pos64 = np.asarray(pos, np.float64)
    n = pos64.shape[0]
    nl = n if n_local is None else int(n_local)
    Z = torch.as_tensor(np.asarray(species, np.int64))
    if edges is None:
        dst, src, dvec = _base.neighbors(pos64, np.asarray(box, np.float64), rc)
    else:
        dst, src, dvec = edges
    dst = np.asarray(dst, np.int64)
    src = np.asarray(src, np.int64)
    shift = torch.as_tensor(np.asarray(dvec, np.float64) - (pos64[src] - pos64[dst]))
    P = torch.tensor(pos64, requires_grad=True)
    ti, tj = torch.as_tensor(dst), torch.as_tensor(src)
    E_n = len(dst)

    U = torch.zeros(n, dtype=torch.float64)
    if E_n:
        d = P[tj] - P[ti] + shift
        r = torch.sqrt((d * d).sum(1))
        rhat = d / r[:, None]
        u = envelope(r / rc, p)
        k = torch.arange(1, nb + 1, dtype=torch.float64)
        B = math.sqrt(2.0 / rc) * torch.sin(k[None, :] * math.pi * r[:, None] / rc) / r[:, None] * u[:, None]
        oh = torch.eye(S, dtype=torch.float64)
        x = torch.cat([oh[Z[ti]], oh[Z[tj]], B], 1)
        nl2b = len(h["mlp_2b"])
        for q in range(nl2b):
            x = x @ W[f"2b_W{q + 1}"].T + W[f"2b_b{q + 1}"]
            if q < nl2b - 1:
                x = _silu(x)
        x0 = u[:, None] * x
        w0 = x0 @ W["Wv"].T
        we = x0 @ W["We"].T
        # pairs of edges sharing their central atom, as a padded [atom][slot] table
        deg = np.bincount(dst, minlength=n)
        Dm = int(deg.max())
        first = np.concatenate([[0], np.cumsum(deg)[:-1]])
        order = np.argsort(dst, kind="stable")
        slot = np.empty(E_n, np.int64)
        slot[order] = np.arange(E_n) - first[dst[order]]
        tab = torch.full((n, Dm), -1, dtype=torch.int64)
        tab[ti[order], torch.as_tensor(slot[order])] = torch.as_tensor(order)
        valid = (tab >= 0).to(torch.float64)
        idx = tab.clamp(min=0)
        rh_t = rhat[idx] * valid[..., None]                # [n, Dm, 3]
        we_t = we[idx] * valid[..., None]                   # [n, Dm, NC]
        cosg = torch.einsum("iad,ibd->iab", rh_t, rh_t)     # [n, Dm, Dm]
        parts, c0 = [], 0
        for l, nc in enumerate(ch):
            if nc:
                T = torch.einsum("iab,ibc->iac", legendre(l, cosg), we_t[..., c0:c0 + nc])
                parts.append(T)
            c0 += nc
        Tall = torch.cat(parts, 2)                          # [n, Dm, NC]
        Sacc = Tall[ti, torch.as_tensor(slot)]              # the row of each edge's own slot
        Sv = nu * w0 * Sacc
        z = _silu(torch.cat([x0, Sv], 1) @ W["lat_W1"].T + W["lat_b1"])
        m = z @ W["lat_W2"].T + W["lat_b2"]
        x1 = (x0 + u[:, None] * m) / math.sqrt(2.0)
        Ee = u * (_silu(x1 @ W["out_W1"].T + W["out_b1"]) @ W["out_w2"] + W["out_b2"][0])
        U = U.index_add(0, ti, Ee)
    E = U[:nl].sum()
    if E.requires_grad:
        (g,) = torch.autograd.grad(E, P)
        F = -g.numpy()
    else:
        F = np.zeros((n, 3))
    if per_atom:
        return float(E.detach()), F, U.detach().numpy()
    return float(E.detach()), F
