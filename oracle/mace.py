"""FP64 CPU oracle for the MACE energy and its forces.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
baseline leg of the benchmark import this module.  It imports nothing from the
GPU package, and the GPU package never imports it.

The paper deploys MACE (Methods, "Graph Neural Networks" and "Chosen
Architectures": messages built in the ACE formalism, correlating a variable
number of neighbours at once) with two interaction layers, correlation order
3, l_max = 3, hidden irreps 32x0e + 32x1o, 8 radial basis functions, a
polynomial envelope of order 6 and a 5 A cutoff ("Training Details").  The
layer equations are those of the cited MACE paper, which the paper does not
print; the reading used here (K channels, real spherical harmonics Y_lm with
sum_m Y_lm^2 = 2l + 1, every coupling of degrees l1 x l2 -> L restricted to
l1 + l2 + L even so that all features keep the parity (-1)^l of harmonics):

  coupling  G(l1, l2, L)[a, b, c] = (1 / 4 pi) int Y_(l1 a) Y_(l2 b) Y_(L c) dOmega
  h0_i      = W_emb[:, Z_i]                                   (K scalars)
  layer t = 1, 2, with input degrees H (layer 1: {0}; layer 2: {0, 1}) and
  output degrees O (layer 1: {0, 1}; layer 2: {0}):
    hb_j,l2     = W_up[l2] h_j,l2                             (per degree)
    R_e         = MLP_rad(B(r_e))    (8 -> 64 -> 64 -> 64 -> K x P, SiLU)
    A_i,k,p     = 1/n_avg sum_(edges i <- j) R_e[p, k]
                  sum_ab G(l1, l2, L)[a, b, :] Y_(l1 a)(rhat_e) hb_(j, k, l2 b)
                  for the conv paths p = (l1, l2, L), l2 in H, L <= l_max
    A'_i,k,L    = sum_(p: L_p = L) sum_k' W_A[L][k, (p, k')] A_i,k',p
    B (per channel k, from A'_k only), for each output degree L_o and path eta:
      nu = 1: A'_(L_o)
      nu = 2: sum_ab G(l1, l2, L_o)[a, b, :] A'_(l1 a) A'_(l2 b)
      nu = 3: sum_(mu c) G(lam, l3, L_o)[mu, c, :]
              (sum_ab G(l1, l2, lam)[a, b, mu] A'_(l1 a) A'_(l2 b)) A'_(l3 c)
    m_i,k,L_o   = sum_eta W_sym[Z_i][L_o][k, eta] B_(k, eta)
    h_i,L_o     = W_out[L_o] m_i,L_o + [L_o in H] W_sc[Z_i][L_o] h_i,L_o
  E_i = w_r1 . h1_i,0 + w_r2 . silu(W_r2 h2_i,0 + b_r2) + b_r3
  E = sum of E_i over local atoms; F = -dE/dr.

Here B(r) = sqrt(2 / r_c) sin(k pi r / r_c) / r u(r), k = 1..8, with the
polynomial envelope u of order p = 6, and rhat_e = (r_j - r_i) / r.  The
coupling coefficients are computed here by an exact quadrature (Gauss-Legendre
in cos(theta) times a uniform grid in phi, exact for the polynomial degrees
involved) of this file's own harmonics, built by the associated-Legendre
recursion.  Forces come from torch float64 reverse-mode differentiation.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import oracle as _base


# ------------------------------------------------------------------ harmonics

def real_sh(lmax: int, v):
    """Real spherical harmonics of unit vectors v [..., 3] (torch), component
    normalised, as a list over l of tensors [..., 2l + 1] ordered m = -l..l:
    Y_l0 = N_l0 Q_l0(z), Y_l,+m = sqrt(2) N_lm Q_lm(z) Re (x + iy)^m,
    Y_l,-m = sqrt(2) N_lm Q_lm(z) Im (x + iy)^m, with P_l^m = (1 - z^2)^(m/2)
    Q_lm and N_lm = sqrt((2l + 1) (l - m)! / (l + m)!)."""
    x, y, z = v[..., 0], v[..., 1], v[..., 2]
    re, im = [torch.ones_like(x)], [torch.zeros_like(x)]
    for m in range(1, lmax + 1):
        re.append(re[-1] * x - im[-1] * y)
        im.append(re[-2] * y + im[-1] * x)
    Q = {}
    for m in range(lmax + 1):
        dfact = 1.0
        for q in range(1, 2 * m, 2):
            dfact *= q
        Q[(m, m)] = torch.full_like(z, dfact)
        if m + 1 <= lmax:
            Q[(m + 1, m)] = (2 * m + 1) * z * Q[(m, m)]
        for l in range(m + 2, lmax + 1):
            Q[(l, m)] = ((2 * l - 1) * z * Q[(l - 1, m)] - (l + m - 1) * Q[(l - 2, m)]) / (l - m)
    out = []
    for l in range(lmax + 1):
        comps = []
        for m in range(-l, l + 1):
            a = abs(m)
            N = math.sqrt((2 * l + 1) * math.factorial(l - a) / math.factorial(l + a))
            if m == 0:
                comps.append(N * Q[(l, 0)])
            elif m > 0:
                comps.append(math.sqrt(2.0) * N * Q[(l, a)] * re[a])
            else:
                comps.append(math.sqrt(2.0) * N * Q[(l, a)] * im[a])
        out.append(torch.stack(comps, -1))
    return out


_GAUNT = {}


def coupling(l1: int, l2: int, L: int) -> torch.Tensor:
    """G(l1, l2, L)[a, b, c] = (1/4pi) int Y_l1a Y_l2b Y_Lc dOmega by an exact
    quadrature (float64)."""
    key = (l1, l2, L)
    if key not in _GAUNT:
        deg = l1 + l2 + L
        nz = deg // 2 + 2
        nphi = deg + 2
        zn, zw = np.polynomial.legendre.leggauss(nz)
        ph = 2 * np.pi * np.arange(nphi) / nphi
        Z, PH = np.meshgrid(zn, ph, indexing="ij")
        W = np.repeat(zw[:, None], nphi, 1) * (2 * np.pi / nphi)
        s = np.sqrt(1 - Z * Z)
        v = torch.as_tensor(np.stack([s * np.cos(PH), s * np.sin(PH), Z], -1).reshape(-1, 3))
        Y = real_sh(max(l1, l2, L), v)
        w = torch.as_tensor(W.reshape(-1)) / (4 * np.pi)
        _GAUNT[key] = torch.einsum("p,pa,pb,pc->abc", w, Y[l1], Y[l2], Y[L])
    return _GAUNT[key]


def _allowed(l1, l2, L):
    return abs(l1 - l2) <= L <= l1 + l2 and (l1 + l2 + L) % 2 == 0


def conv_paths(h_degrees, lmax):
    """(l1, l2, L) of the conv tensor product, in weight order."""
    return [(l1, l2, L) for l2 in h_degrees for l1 in range(lmax + 1) for L in range(lmax + 1) if _allowed(l1, l2, L)]


def sym_paths(L_out, lmax, corr):
    """Paths of the symmetric contraction onto degree L_out, in weight order:
    (1, (L,)), (2, (l1, l2)) with l1 <= l2, (3, (l1, l2, lam, l3)) with l1 <= l2."""
    out = []
    if L_out <= lmax:
        out.append((1, (L_out,)))
    if corr >= 2:
        for l1 in range(lmax + 1):
            for l2 in range(l1, lmax + 1):
                if _allowed(l1, l2, L_out):
                    out.append((2, (l1, l2)))
    if corr >= 3:
        for l1 in range(lmax + 1):
            for l2 in range(l1, lmax + 1):
                for lam in range(lmax + 1):
                    if not _allowed(l1, l2, lam):
                        continue
                    for l3 in range(lmax + 1):
                        if _allowed(lam, l3, L_out):
                            out.append((3, (l1, l2, lam, l3)))
    return out


LAYER_IN = ([0], [0, 1])     # degrees of the node features entering each layer
LAYER_OUT = ([0, 1], [0])    # degrees each layer produces (the last: scalars)


def layout(h: dict):
    """(name, shape) of every weight block in storage order; matrices are
    [out][in] row-major."""
    S, K, nb, lmax, corr = h["n_species"], h["channels"], h["n_basis"], h["l_max"], h["correlation"]
    rh = list(h["radial_hidden"])
    out = [("W_emb", (K, S))]
    for t in range(2):
        P = conv_paths(LAYER_IN[t], lmax)
        for l2 in LAYER_IN[t]:
            out.append((f"l{t}.W_up{l2}", (K, K)))
        prev = nb
        for q, wdt in enumerate(rh):
            out.append((f"l{t}.rad{q}", (wdt, prev)))
            prev = wdt
        out.append((f"l{t}.rad{len(rh)}", (len(P) * K, prev)))
        for L in range(lmax + 1):
            nL = sum(1 for p in P if p[2] == L)
            if nL:
                out.append((f"l{t}.W_A{L}", (K, nL * K)))
        for Lo in LAYER_OUT[t]:
            out.append((f"l{t}.W_sym{Lo}", (S, K, len(sym_paths(Lo, lmax, corr)))))
        for Lo in LAYER_OUT[t]:
            out.append((f"l{t}.W_out{Lo}", (K, K)))
        for Lo in LAYER_OUT[t]:
            if Lo in LAYER_IN[t]:
                out.append((f"l{t}.W_sc{Lo}", (S, K, K)))
    RH = h["readout_hidden"]
    out += [("w_r1", (K,)), ("W_r2", (RH, K)), ("b_r2", (RH,)), ("w_r2", (RH,)), ("b_r3", (1,))]
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
    return (1.0 - (p + 1) * (p + 2) / 2.0 * x ** p + p * (p + 2) * x ** (p + 1)
            - p * (p + 1) / 2.0 * x ** (p + 2))


def _silu(x):
    return x * torch.sigmoid(x)


def _sym_contract(A, Lo, lmax, corr):
    """The B features of every path onto degree Lo from A (a list over l of
    [n, K, 2l + 1]); returns [n, K, n_paths, 2Lo + 1]."""
    Bs = []
    for nu, ls in sym_paths(Lo, lmax, corr):
        if nu == 1:
            Bs.append(A[ls[0]])
        elif nu == 2:
            l1, l2 = ls
            Bs.append(torch.einsum("abc,nka,nkb->nkc", coupling(l1, l2, Lo), A[l1], A[l2]))
        else:
            l1, l2, lam, l3 = ls
            T = torch.einsum("abm,nka,nkb->nkm", coupling(l1, l2, lam), A[l1], A[l2])
            Bs.append(torch.einsum("mcd,nkm,nkc->nkd", coupling(lam, l3, Lo), T, A[l3]))
    return torch.stack(Bs, 2)


def energy_forces(header: dict, weights, pos, species, box, n_local: int | None = None, per_atom: bool = False,
                  edges=None):
    """E = sum_{i < n_local} E_i and F = -dE/dr of every atom (FP64)."""
    h = header
    W = _unpack(h, weights)
    K, nb, p, rc, lmax, corr = h["channels"], h["n_basis"], h["envelope_p"], float(h["r_c"]), h["l_max"], \
        h["correlation"]
    navg = float(h["avg_neighbors"])
    nrad = len(h["radial_hidden"])
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
    d = P[tj] - P[ti] + shift
    r = torch.sqrt((d * d).sum(1))
    rhat = d / r[:, None]
    u = envelope(r / rc, p)
    kk = torch.arange(1, nb + 1, dtype=torch.float64)
    Bas = math.sqrt(2.0 / rc) * torch.sin(kk[None, :] * math.pi * r[:, None] / rc) / r[:, None] * u[:, None]
    Y = real_sh(lmax, rhat)

    hfeat = {0: W["W_emb"][:, Z].T.reshape(n, K, 1)}       # degree -> [n, K, 2l + 1]
    E_atom = torch.zeros(n, dtype=torch.float64)
    for t in range(2):
        pre = f"l{t}."
        Pth = conv_paths(LAYER_IN[t], lmax)
        hb = {l2: torch.einsum("kq,nqm->nkm", W[pre + f"W_up{l2}"], hfeat[l2]) for l2 in LAYER_IN[t]}
        x = Bas
        for q in range(nrad):
            x = _silu(x @ W[pre + f"rad{q}"].T)
        R = (x @ W[pre + f"rad{nrad}"].T).reshape(-1, len(Pth), K)      # [E, P, K]
        Araw = []
        for pi_, (l1, l2, L) in enumerate(Pth):
            msg = torch.einsum("abc,ea,ekb->ekc", coupling(l1, l2, L), Y[l1], hb[l2][tj]) * R[:, pi_, :, None]
            Araw.append(torch.zeros(n, K, 2 * L + 1, dtype=torch.float64).index_add(0, ti, msg) / navg)
        A = []
        for L in range(lmax + 1):
            idx = [q for q, pth in enumerate(Pth) if pth[2] == L]
            if not idx:
                A.append(torch.zeros(n, K, 2 * L + 1, dtype=torch.float64))
                continue
            stack = torch.cat([Araw[q] for q in idx], 1)                   # [n, nL K, 2L + 1]
            A.append(torch.einsum("kq,nqm->nkm", W[pre + f"W_A{L}"], stack))
        new = {}
        for Lo in LAYER_OUT[t]:
            Bf = _sym_contract(A, Lo, lmax, corr)                          # [n, K, paths, 2Lo + 1]
            m = torch.einsum("nkp,nkpm->nkm", W[pre + f"W_sym{Lo}"][Z], Bf)
            hn = torch.einsum("kq,nqm->nkm", W[pre + f"W_out{Lo}"], m)
            if Lo in LAYER_IN[t]:
                hn = hn + torch.einsum("nkq,nqm->nkm", W[pre + f"W_sc{Lo}"][Z], hfeat[Lo])
            new[Lo] = hn
        hfeat = new
        if t == 0:
            E_atom = E_atom + hfeat[0][:, :, 0] @ W["w_r1"]
        else:
            z = _silu(hfeat[0][:, :, 0] @ W["W_r2"].T + W["b_r2"])
            E_atom = E_atom + z @ W["w_r2"] + W["b_r3"][0]
    E = E_atom[:nl].sum()
    (g,) = torch.autograd.grad(E, P, allow_unused=True)
    F = np.zeros((n, 3)) if g is None else -g.numpy()
    if per_atom:
        return float(E.detach()), F, E_atom.detach().numpy()
    return float(E.detach()), F
