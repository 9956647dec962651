// MACE with two interaction layers: energy and forces on the pruned
// neighbour graph.
//
// The paper deploys MACE (Methods, "Graph Neural Networks" and "Chosen
// Architectures": messages in the atomic-cluster-expansion form, many-body
// features built per atom from a one-particle basis) with two layers,
// correlation order 3, l_max = 3, hidden features of 32 scalars and 32
// vectors, 8 radial functions and a polynomial envelope of order 6
// ("Training Details").  The layer equations are those of the cited MACE
// paper; the reading here, per atom i, channel k, directed edge e = (i <- j)
// with r = |r_j - r_i| < rc and rhat = (r_j - r_i) / r:
//   G(l1, l2, L)[a, b, c] = (1 / 4 pi) int Y_l1a Y_l2b Y_Lc  (only l1 + l2 + L even)
//   hb_j,l2   = W_up[l2] h_j,l2                       (layer 1: h = W_emb onehot(Z))
//   R_e       = MLP_rad(B(r))                          (SiLU, no biases; K per conv path)
//   A_i,p,c   = 1/n_avg sum_e R_e,p sum_ab G(l1, l2, L)[a, b, c] Y_l1a(rhat) hb_j,l2b
//               for the conv paths p = (l1, l2, L), l2 a degree the layer takes
//   A'_i,L    = W_A[L] (the A of every path onto L, channels stacked)
//   B_eta     = the nu-fold products of A' of one channel coupled to degree L_o
//               (nu = 1, 2, 3; the nu = 3 ones through an intermediate lambda)
//   m_i,L_o   = sum_eta W_sym[Z_i][L_o][k, eta] B_eta
//   h_i,L_o   = W_out[L_o] m_i,L_o + W_sc[Z_i][L_o] h_i,L_o  (skip where L_o is an input degree)
//   E_i       = w_r1 . h1_i,0 + w_r2 . silu(W_r2 h2_i,0 + b_r2) + b_r3
// Layer 1 takes degree 0 and gives degrees 0 and 1; layer 2 takes 0 and 1 and
// gives 0.  Y are the component-normalised real harmonics of sh.h; the
// couplings are constant expressions of the same harmonics (gaunt.h), so the
// kernels unroll over the nonzero couplings only.
//
// Layout of the work: the radial MLPs are GEMMs over edges and the W_A
// channel mixes GEMMs over (atom, m) rows, on the matrix cores (gemm.hip).
// The convolution, the symmetric contraction and the small per-atom channel
// mixes (W_out, W_sc, W_up, the readouts) run with one half-wave per atom and
// one lane per channel:
// * the l2 = 1 conv paths accumulate per atom the moments
//   M_p[a][b] = sum_e R_e,p Y_l1a hb_j,1b and couple them once per atom
//   (A_p,c = sum_ab G[a][b][c] M_p[a][b]); the adjoint contracts G with the
//   atom's dE/dA once (X_p[a][b] = sum_c G[a][b][c] dE/dA_p,c) and then works
//   per edge on X;
// * the symmetric contraction is factorised: the pair products
//   P(l1, l2 -> lambda) = sum_ab G A'_l1a A'_l2b of a channel are formed once
//   in registers and serve both the two-body paths and, coupled with one
//   more A', the three-body paths.
// Forces come from a hand-written adjoint: the same kernels reversed, the
// gradient of each source's hb collected from per-edge partials through the
// reverse-edge index (no atomics), per-edge sums over channels by DPP
// exchanges within the half-wave, and per edge G_e = dE/d(r_i - r_j),
// assembled into forces by launch_forces.
#include "internal.h"
#include "gemm.h"
#include "gaunt.h"
#include "sh.h"

#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#define MC_INLINE __attribute__((always_inline))

namespace mlp {

namespace {

constexpr int MK = 32;     // channels: one lane each, a half-wave per atom
constexpr int APB = 8;     // atoms per workgroup (256 threads)

inline int nblk(long n, int t) { return (int)((n + t - 1) / t); }

// Conv paths of the second layer in weight order; the first layer's are the
// first four.  0..3: (l1, 0, l1); 4: (0,1,1) 5: (1,1,0) 6: (1,1,2) 7: (2,1,1)
// 8: (2,1,3) 9: (3,1,2).
__host__ __device__ constexpr int cp_l1(int p) {
    return p < 4 ? p : (p == 4 ? 0 : (p <= 6 ? 1 : (p <= 8 ? 2 : 3)));
}
__host__ __device__ constexpr int cp_L(int p) {
    return p < 4 ? p : (p == 4 ? 1 : (p == 5 ? 0 : (p == 6 ? 2 : (p == 7 ? 1 : (p == 8 ? 3 : 2)))));
}
// first accumulator of path p (its 2L + 1 outputs follow)
__host__ __device__ constexpr int cp_off(int p) {
    int o = 0;
    for (int q = 0; q < p; q++) o += 2 * cp_L(q) + 1;
    return o;
}
// position of path p among the paths onto its L (the W_A column block)
__host__ __device__ constexpr int cp_loc(int p) {
    int c = 0;
    for (int q = 0; q < p; q++) c += cp_L(q) == cp_L(p);
    return c;
}
// number of paths onto L among the first np
__host__ __device__ constexpr int cp_nL(int L, int np) {
    int c = 0;
    for (int q = 0; q < np; q++) c += cp_L(q) == L;
    return c;
}
// first moment M_p[a][b] of an l2 = 1 path ((2 l1 + 1) x 3 per path)
__host__ __device__ constexpr int cp_moff(int p) {
    int o = 0;
    for (int q = 4; q < p; q++) o += 3 * (2 * cp_l1(q) + 1);
    return o;
}
constexpr int NMOM = cp_moff(10);
static_assert(cp_off(4) == 16 && cp_off(10) == 40 && NMOM == 72, "accumulator layout");

// ---- compile-time couplings of the conv paths with l2 = 1 ----
struct CEnt {
    int a, b, c;
    float v;
};
struct ConvTab {
    CEnt e[320] = {};
    int beg[11] = {};   // entries of path p: [beg[p], beg[p + 1]), p = 4..9
};
constexpr ConvTab make_conv() {
    ConvTab t{};
    int n = 0;
    for (int p = 4; p < 10; p++) {
        t.beg[p] = n;
        const int l1 = cp_l1(p), L = cp_L(p);
        for (int a = 0; a < 2 * l1 + 1; a++)
            for (int b = 0; b < 3; b++)
                for (int c = 0; c < 2 * L + 1; c++) {
                    const double v = cg::coupling(l1, a, 1, b, L, c);
                    if (v != 0.0) t.e[n++] = CEnt{a, b, c, (float)v};
                }
    }
    t.beg[10] = n;
    return t;
}
inline constexpr ConvTab kConv = make_conv();

// ---- compile-time structure of the symmetric contraction (l_max 3, correlation 3) ----
// Pair products P(l1 <= l2 -> lambda)[mu] = sum_ab G(l1, l2, lambda)[a][b][mu] A_l1a A_l2b.
struct PEnt {
    int i, j, q;   // A slots l1^2 + a, l2^2 + b; P index
    float v;
};
struct PairTab {
    int nc = 0, l1[16] = {}, l2[16] = {}, lam[16] = {}, off[17] = {};
    PEnt e[400] = {};
    int n = 0;
};
constexpr PairTab make_pairs() {
    PairTab t{};
    int q = 0;
    for (int l1 = 0; l1 <= 3; l1++)
        for (int l2 = l1; l2 <= 3; l2++)
            for (int lam = 0; lam <= 3; lam++) {
                if (!cg::couples(l1, l2, lam)) continue;
                const int c = t.nc++;
                t.l1[c] = l1;
                t.l2[c] = l2;
                t.lam[c] = lam;
                t.off[c] = q;
                for (int a = 0; a < 2 * l1 + 1; a++)
                    for (int b = 0; b < 2 * l2 + 1; b++)
                        for (int mu = 0; mu < 2 * lam + 1; mu++) {
                            const double v = cg::coupling(l1, a, l2, b, lam, mu);
                            if (v != 0.0) t.e[t.n++] = PEnt{l1 * l1 + a, l2 * l2 + b, q + mu, (float)v};
                        }
                q += 2 * lam + 1;
            }
    t.off[t.nc] = q;
    return t;
}
inline constexpr PairTab kPair = make_pairs();
constexpr int NPP = kPair.off[kPair.nc];

constexpr int pair_off(int l1, int l2, int lam) {
    for (int c = 0; c < kPair.nc; c++)
        if (kPair.l1[c] == l1 && kPair.l2[c] == l2 && kPair.lam[c] == lam) return kPair.off[c];
    return -1;
}

// Contraction paths onto degree Lo in weight order: kind 1 (A'_Lo), kind 2
// (a pair product onto Lo, P index q0), kind 3 (a pair product onto lambda
// coupled with A'_l3 to Lo: entries (P index, A slot, output component)).
struct SEnt {
    int q, s, d;
    float v;
};
struct SymTab {
    int np = 0, kind[32] = {}, q0[32] = {}, beg[33] = {};
    SEnt e[400] = {};
    int n = 0;
};
constexpr SymTab make_sym(int Lo) {
    SymTab t{};
    t.kind[t.np] = 1;
    t.beg[t.np] = t.n;
    t.np++;
    for (int l1 = 0; l1 <= 3; l1++)
        for (int l2 = l1; l2 <= 3; l2++)
            if (cg::couples(l1, l2, Lo)) {
                t.kind[t.np] = 2;
                t.q0[t.np] = pair_off(l1, l2, Lo);
                t.beg[t.np] = t.n;
                t.np++;
            }
    for (int l1 = 0; l1 <= 3; l1++)
        for (int l2 = l1; l2 <= 3; l2++)
            for (int lam = 0; lam <= 3; lam++) {
                if (!cg::couples(l1, l2, lam)) continue;
                for (int l3 = 0; l3 <= 3; l3++) {
                    if (!cg::couples(lam, l3, Lo)) continue;
                    const int q0 = pair_off(l1, l2, lam);
                    t.kind[t.np] = 3;
                    t.q0[t.np] = q0;
                    t.beg[t.np] = t.n;
                    for (int mu = 0; mu < 2 * lam + 1; mu++)
                        for (int c = 0; c < 2 * l3 + 1; c++)
                            for (int d = 0; d < 2 * Lo + 1; d++) {
                                const double v = cg::coupling(lam, mu, l3, c, Lo, d);
                                if (v != 0.0) t.e[t.n++] = SEnt{q0 + mu, l3 * l3 + c, d, (float)v};
                            }
                    t.np++;
                }
            }
    t.beg[t.np] = t.n;
    return t;
}
inline constexpr SymTab kSym0 = make_sym(0), kSym1 = make_sym(1);
template <int LO>
constexpr const SymTab &sym_tab() {
    if constexpr (LO == 0) return kSym0;
    else return kSym1;
}
static_assert(kSym0.np == 20 && kSym1.np == 27 && NPP == 59, "contraction paths");

__device__ __forceinline__ float mc_sigmoid(float x) { return 1.0f / (1.0f + __expf(-x)); }
__device__ __forceinline__ float mc_silu(float x) { return x * mc_sigmoid(x); }
__device__ __forceinline__ float mc_dsilu(float x) {
    const float s = mc_sigmoid(x);
    return s * (1.0f + x * (1.0f - s));
}

__device__ __forceinline__ void load16(const float *p, float *v) {
    const float4 *p4 = reinterpret_cast<const float4 *>(p);
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const float4 x = p4[q];
        v[4 * q] = x.x;
        v[4 * q + 1] = x.y;
        v[4 * q + 2] = x.z;
        v[4 * q + 3] = x.w;
    }
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
// One exchange of a reduce-scatter: the lane whose bit is set keeps the
// upper W values and hands its lower W to the partner, which keeps the lower.
template <int W, int CTRL>
__device__ __forceinline__ void rs_stage(float *v, bool up) {
#pragma unroll
    for (int q = 0; q < W; q++) {
        const float send = up ? v[q] : v[q + W], keep = up ? v[q + W] : v[q];
        v[q] = keep + dpp_mov<CTRL>(send);
    }
}
// Sum of 16 values over the 32 lanes of a half-wave; lane k returns the total
// of value k & 15.  Partners within a row of 16 lanes: lane i and 15 - i
// (row mirror, bit 3 differs), i and 7 - i (half-row mirror, bit 2), i ^ 2 and
// i ^ 1 (quad permutations); then the two rows.
__device__ __forceinline__ float halfwave_sum16(float *v, int k) {
    rs_stage<8, 0x140>(v, (k & 8) != 0);
    rs_stage<4, 0x141>(v, (k & 4) != 0);
    rs_stage<2, 0x4E>(v, (k & 2) != 0);
    rs_stage<1, 0xB1>(v, (k & 1) != 0);
    return v[0] + __shfl_xor(v[0], 16, 64);
}

__device__ __forceinline__ float halfwave_sum(float v) {
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// ---- symmetric contraction of one channel (A: 16 slots l^2 + m) ----
__device__ __forceinline__ void pair_fwd(const float *A, float *P) {
#pragma unroll
    for (int q = 0; q < NPP; q++) P[q] = 0.f;
    cg::sfor<kPair.n>([&](auto t) MC_INLINE {
        constexpr PEnt E = kPair.e[decltype(t)::value];
        P[E.q] = fmaf(E.v, A[E.i] * A[E.j], P[E.q]);
    });
}

__device__ __forceinline__ void pair_bwd(const float *A, const float *gP, float *gA) {
    cg::sfor<kPair.n>([&](auto t) MC_INLINE {
        constexpr PEnt E = kPair.e[decltype(t)::value];
        const float g = E.v * gP[E.q];
        gA[E.i] = fmaf(g, A[E.j], gA[E.i]);
        gA[E.j] = fmaf(g, A[E.i], gA[E.j]);
    });
}

// m[d] += sum_eta W[eta] B_eta,d for output degree LO; W: this species' and
// channel's weights, path eta at W[eta * MK]
template <int LO>
__device__ __forceinline__ void sym_fwd(const float *A, const float *P, const float *__restrict__ W, float *m) {
    constexpr int NO = 2 * LO + 1;
    cg::sfor<sym_tab<LO>().np>([&](auto eta) MC_INLINE {
        constexpr int h = decltype(eta)::value;
        constexpr int kind = sym_tab<LO>().kind[h];
        const float w = W[h * MK];
        if constexpr (kind == 1) {
#pragma unroll
            for (int d = 0; d < NO; d++) m[d] = fmaf(w, A[LO * LO + d], m[d]);
        } else if constexpr (kind == 2) {
            constexpr int q0 = sym_tab<LO>().q0[h];
#pragma unroll
            for (int d = 0; d < NO; d++) m[d] = fmaf(w, P[q0 + d], m[d]);
        } else {
            constexpr int e0 = sym_tab<LO>().beg[h], ne = sym_tab<LO>().beg[h + 1] - e0;
            float b[NO];
#pragma unroll
            for (int d = 0; d < NO; d++) b[d] = 0.f;
            cg::sfor<ne>([&](auto t) MC_INLINE {
                constexpr SEnt E = sym_tab<LO>().e[e0 + decltype(t)::value];
                b[E.d] = fmaf(E.v, P[E.q] * A[E.s], b[E.d]);
            });
#pragma unroll
            for (int d = 0; d < NO; d++) m[d] = fmaf(w, b[d], m[d]);
        }
    });
}

// adjoint of sym_fwd: gm = dE/dm; adds dE/dA (direct) into gA and dE/dP into gP
template <int LO>
__device__ __forceinline__ void sym_bwd(const float *A, const float *P, const float *__restrict__ W, const float *gm,
                                        float *gA, float *gP) {
    constexpr int NO = 2 * LO + 1;
    cg::sfor<sym_tab<LO>().np>([&](auto eta) MC_INLINE {
        constexpr int h = decltype(eta)::value;
        constexpr int kind = sym_tab<LO>().kind[h];
        const float w = W[h * MK];
        float gb[NO];
#pragma unroll
        for (int d = 0; d < NO; d++) gb[d] = w * gm[d];
        if constexpr (kind == 1) {
#pragma unroll
            for (int d = 0; d < NO; d++) gA[LO * LO + d] += gb[d];
        } else if constexpr (kind == 2) {
            constexpr int q0 = sym_tab<LO>().q0[h];
#pragma unroll
            for (int d = 0; d < NO; d++) gP[q0 + d] += gb[d];
        } else {
            constexpr int e0 = sym_tab<LO>().beg[h], ne = sym_tab<LO>().beg[h + 1] - e0;
            cg::sfor<ne>([&](auto t) MC_INLINE {
                constexpr SEnt E = sym_tab<LO>().e[e0 + decltype(t)::value];
                const float g = E.v * gb[E.d];
                gP[E.q] = fmaf(g, A[E.s], gP[E.q]);
                gA[E.s] = fmaf(g, P[E.q], gA[E.s]);
            });
        }
    });
}

}  // namespace

// Per-L blocks of an atom array (A before and after the W_A mix, and their gradients).
struct McBlk {
    float *p[4];
};

// ---------------------------------------------------------------------------
// Model
// ---------------------------------------------------------------------------
struct McModel {
    int S = 0, NB = 0, NBP = 0, pe = 0, nrad = 0, rh[4] = {0, 0, 0, 0}, RH = 0;
    float rc = 0.f, navg = 1.f, b_r3 = 0.f;
    float *dev = nullptr;     // weights, transposed copies, tables (device)
    void *pk_dev = nullptr;   // packed GEMM operands
    PackedW radF[2][5], radA[2][5], waF[2][4], waA[2][4];
    EdgeMlp rmlp[2];          // the radial MLPs as fused kernels (when their shape allows)
    bool fused = false;
    const float *zero = nullptr, *hb0tab = nullptr, *skip0tab = nullptr;
    const float *w_r1 = nullptr, *W_r2 = nullptr, *b_r2 = nullptr, *w_r2 = nullptr;
    const float *WoutT[2][2] = {}, *Wout[2][2] = {};   // [layer][output degree index]
    const float *WupT1[2] = {}, *Wup1[2] = {};         // second layer's W_up for l2 = 0, 1
    const float *WscT1 = nullptr, *Wsc1 = nullptr;     // second layer's skip (degree 0), [S][K][K]
    const float *Wsym[2][2] = {};                      // [layer][output degree index]: [S][paths][K]
};

// ---------------------------------------------------------------------------
// Forward, per edge: radial functions with the envelope, and the harmonics.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mc_edge(const int *__restrict__ rowc, int n, const float4 *__restrict__ geom,
                                                 int NB, int NBP, int pe, float rc, float *__restrict__ X0,
                                                 float *__restrict__ Y) {
    const long ne = rowc[n];
    const float c0 = sqrtf(2.0f / rc), th = 3.14159265358979f / rc;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (long)gridDim.x * blockDim.x) {
        const float4 gm = geom[e];
        const float r = gm.w, ir = 1.0f / r;
        float u, du;
        envelope(r / rc, pe, u, du);
        float sn, cs;
        sincosf(th * r, &sn, &cs);
        float *x = X0 + e * NBP;
        float sk = sn, skm = 0.f;
        for (int k = 0; k < NB; k++) {
            x[k] = c0 * sk * ir * u;
            const float nx = 2.f * cs * sk - skm;
            skm = sk;
            sk = nx;
        }
        for (int k = NB; k < NBP; k++) x[k] = 0.f;
        float y[16];
        sh16(gm.x * ir, gm.y * ir, gm.z * ir, y);
        float4 *y4 = reinterpret_cast<float4 *>(Y + e * 16);
#pragma unroll
        for (int q = 0; q < 4; q++) y4[q] = make_float4(y[4 * q], y[4 * q + 1], y[4 * q + 2], y[4 * q + 3]);
    }
}

// ---------------------------------------------------------------------------
// Convolution, one half-wave per destination atom, lane = channel: the A of
// every conv path summed over the atom's edges, scaled by 1 / n_avg, written
// as the rows (i, c) of its L block with the path's position among the paths
// onto L selecting the column block (the W_A GEMM's operand layout).
// ---------------------------------------------------------------------------
template <int LAY>
__global__ void __launch_bounds__(256) k_mc_conv(const int *__restrict__ rowc, const int *__restrict__ colc, int nd,
                                                 const float *__restrict__ Y, const float *__restrict__ R,
                                                 const float *__restrict__ HB, const int *__restrict__ zsp,
                                                 const float *__restrict__ hb0, float scale, McBlk AR) {
    constexpr int NP = LAY == 0 ? 4 : 10, NM = LAY == 0 ? 1 : NMOM;
    const int k = threadIdx.x & 31;
    const int i = blockIdx.x * APB + (threadIdx.x >> 5);
    if (i >= nd) return;
    float acc[16], mom[NM];
#pragma unroll
    for (int q = 0; q < 16; q++) acc[q] = 0.f;
#pragma unroll
    for (int q = 0; q < NM; q++) mom[q] = 0.f;
    const int eend = rowc[i + 1];
    for (int e = rowc[i]; e < eend; e++) {
        const int j = colc[e];
        float h0, h1[3] = {0.f, 0.f, 0.f};
        if constexpr (LAY == 0) {
            h0 = hb0[zsp[j] * MK + k];
        } else {
            const float *hb = HB + (long)j * 4 * MK + k;
            h0 = hb[0];
            h1[0] = hb[MK];
            h1[1] = hb[2 * MK];
            h1[2] = hb[3 * MK];
        }
        float y[16], r[NP];
        load16(Y + (long)e * 16, y);
        const float *rr = R + (long)e * NP * MK + k;
#pragma unroll
        for (int p = 0; p < NP; p++) r[p] = rr[p * MK];
#pragma unroll
        for (int p = 0; p < 4; p++) {
            const float s = r[p] * h0;
#pragma unroll
            for (int c = 0; c < 2 * p + 1; c++) acc[p * p + c] = fmaf(s, y[p * p + c], acc[p * p + c]);
        }
        if constexpr (LAY == 1) {
#pragma unroll
            for (int p = 4; p < NP; p++) {
                const int l1 = cp_l1(p), mo = cp_moff(p);
                const float rb[3] = {r[p] * h1[0], r[p] * h1[1], r[p] * h1[2]};
#pragma unroll
                for (int a = 0; a < 2 * l1 + 1; a++)
#pragma unroll
                    for (int b = 0; b < 3; b++) mom[mo + a * 3 + b] = fmaf(y[l1 * l1 + a], rb[b], mom[mo + a * 3 + b]);
            }
        }
    }
#pragma unroll
    for (int p = 0; p < 4; p++) {
        const int L = p, nc = 2 * L + 1, ld = cp_nL(L, NP) * MK;
        float *o = AR.p[L] + (long)i * nc * ld + cp_loc(p) * MK + k;
#pragma unroll
        for (int c = 0; c < nc; c++) o[(long)c * ld] = acc[p * p + c] * scale;
    }
    if constexpr (LAY == 1) {
        cg::sfor<6>([&](auto pi) MC_INLINE {
            constexpr int p = 4 + decltype(pi)::value, L = cp_L(p), nc = 2 * L + 1, ld = cp_nL(L, 10) * MK,
                          mo = cp_moff(p), e0 = kConv.beg[p];
            float v[nc];
#pragma unroll
            for (int c = 0; c < nc; c++) v[c] = 0.f;
            cg::sfor<kConv.beg[p + 1] - e0>([&](auto t) MC_INLINE {
                constexpr CEnt E = kConv.e[e0 + decltype(t)::value];
                v[E.c] = fmaf(E.v, mom[mo + E.a * 3 + E.b], v[E.c]);
            });
            float *o = AR.p[L] + (long)i * nc * ld + cp_loc(p) * MK + k;
#pragma unroll
            for (int c = 0; c < nc; c++) o[(long)c * ld] = v[c] * scale;
        });
    }
}

// ---------------------------------------------------------------------------
// Per-atom kernels: one half-wave per atom, lane = channel; the lane's A'
// (16 values) and pair products in registers, the channel mixes through a
// per-atom LDS row.  Every thread of a workgroup reaches the barriers (rows
// past nd compute on zeros and write nothing).
// ---------------------------------------------------------------------------
struct McNodeArgs {
    McBlk AP;                      // A' [row][2L + 1][K] per L
    const float *Wsym[2];          // per output degree index: [S][paths][K]
    int np[2];
    const float *WoutT[2];         // [k'][k] per output degree index
    const float *skip0tab;         // first layer: W_sc[Z] h0 per species [S][K]
    const float *WupT1[2];
    const float *WscT1;            // second layer's skip [S][k'][k]
    const float *w_r1, *W_r2, *b_r2, *w_r2;
    float b_r3;
    int RH;
    const float *H1;               // first layer's output [row][4][K]
    float *H1o, *HB1o, *H2;        // outputs
    float *U;                      // per-atom energies (rows past nloc: 0)
    int nloc;                      // rows the second layer covers
};

__device__ __forceinline__ void load_ap(const McBlk &AP, bool act, int i, int k, float *A) {
#pragma unroll
    for (int L = 0; L < 4; L++)
#pragma unroll
        for (int m = 0; m < 2 * L + 1; m++) A[L * L + m] = act ? AP.p[L][((long)i * (2 * L + 1) + m) * MK + k] : 0.f;
}

__device__ __forceinline__ void store_gap(const McBlk &GAP, int i, int k, const float *gA) {
#pragma unroll
    for (int L = 0; L < 4; L++)
#pragma unroll
        for (int m = 0; m < 2 * L + 1; m++) GAP.p[L][((long)i * (2 * L + 1) + m) * MK + k] = gA[L * L + m];
}

// x[c] = sum_k' W[c][k' * K + k] xs[c][k'] for c < NC (W per component, [k'][k])
template <int NC>
__device__ __forceinline__ void mix(const float *const *W, const float *xs, int k, float *x) {
#pragma unroll
    for (int c = 0; c < NC; c++) {
        const float *w = W[c] + k;
        const float *v = xs + c * MK;
        float s = 0.f;
#pragma unroll 8
        for (int q = 0; q < MK; q++) s = fmaf(w[q * MK], v[q], s);
        x[c] = s;
    }
}

template <int LAY>
__global__ void __launch_bounds__(256) k_mc_node(int nd, const int *__restrict__ zsp, McNodeArgs a) {
    __shared__ float sx[APB * 4 * MK];
    const int tid = threadIdx.x, k = tid & 31, ai = tid >> 5;
    const int i = blockIdx.x * APB + ai;
    const bool act = i < nd;
    const int z = act ? zsp[i] : 0;
    float A[16], P[NPP];
    load_ap(a.AP, act, i, k, A);
    pair_fwd(A, P);
    float m[4] = {0.f, 0.f, 0.f, 0.f};
    sym_fwd<0>(A, P, a.Wsym[0] + (long)z * a.np[0] * MK + k, m);
    if constexpr (LAY == 0) sym_fwd<1>(A, P, a.Wsym[1] + (long)z * a.np[1] * MK + k, m + 1);
    float *xs = sx + ai * 4 * MK;
    constexpr int NC = LAY == 0 ? 4 : 1;
#pragma unroll
    for (int c = 0; c < NC; c++) xs[c * MK + k] = m[c];
    __syncthreads();
    float h[4];
    {
        const float *W[4] = {a.WoutT[0], a.WoutT[1], a.WoutT[1], a.WoutT[1]};
        mix<NC>(W, xs, k, h);
    }
    __syncthreads();
    if constexpr (LAY == 0) {
        h[0] += a.skip0tab[z * MK + k];
        if (act)
#pragma unroll
            for (int c = 0; c < 4; c++) a.H1o[((long)i * 4 + c) * MK + k] = h[c];
        const float e = halfwave_sum(a.w_r1[k] * h[0]);
        if (act && k == 0) a.U[i] = i < a.nloc ? e : 0.f;
#pragma unroll
        for (int c = 0; c < 4; c++) xs[c * MK + k] = h[c];
        __syncthreads();
        float hb[4];
        const float *W[4] = {a.WupT1[0], a.WupT1[1], a.WupT1[1], a.WupT1[1]};
        mix<4>(W, xs, k, hb);
        if (act)
#pragma unroll
            for (int c = 0; c < 4; c++) a.HB1o[((long)i * 4 + c) * MK + k] = hb[c];
    } else {
        // skip on degree 0 (species-dependent), then the readout MLP
        xs[k] = act ? a.H1[(long)i * 4 * MK + k] : 0.f;
        __syncthreads();
        {
            const float *w = a.WscT1 + (long)z * MK * MK + k;
            float s = 0.f;
#pragma unroll 8
            for (int q = 0; q < MK; q++) s = fmaf(w[q * MK], xs[q], s);
            h[0] += s;
        }
        __syncthreads();
        if (act) a.H2[(long)i * MK + k] = h[0];
        xs[k] = h[0];
        __syncthreads();
        float e = 0.f;
        if (k < a.RH) {
            const float *w = a.W_r2 + k * MK;
            float zz = a.b_r2[k];
            for (int q = 0; q < MK; q++) zz = fmaf(w[q], xs[q], zz);
            e = a.w_r2[k] * mc_silu(zz);
        }
        e = halfwave_sum(e);
        if (act && k == 0) a.U[i] += e + a.b_r3;
    }
}

// ---------------------------------------------------------------------------
// Adjoint of the per-atom kernels.
// ---------------------------------------------------------------------------
struct McNodeBwdArgs {
    McBlk AP, GAP;                 // A' of the layer and dE/dA' (output)
    const float *Wsym[2];
    int np[2];
    const float *Wout[2];          // [k][k'] per output degree index
    const float *Wup1[2];          // second layer's W_up [k][k'] for l2 = 0, 1
    const float *Wsc1;             // [S][K][K]
    const float *w_r1, *W_r2, *b_r2, *w_r2;
    int RH;
    const float *H2;
    float *GH1S;                   // second layer: dE/dh1 (degree 0) through the skip
    // first layer: dE/dhb1 collected from per-edge partials
    const int *rowc, *colc, *revc;
    const float *MSG;
    int nd1;
    const int *perm;
    int n_local;
};

__global__ void __launch_bounds__(256) k_mc_node1_bwd(int nd, const int *__restrict__ zsp, McNodeBwdArgs a) {
    __shared__ float sx[APB * 4 * MK];
    const int tid = threadIdx.x, k = tid & 31, ai = tid >> 5;
    const int i = blockIdx.x * APB + ai;
    const bool act = i < nd;
    const int z = act ? zsp[i] : 0;
    const float gE = (act && a.perm[i] < a.n_local) ? 1.f : 0.f;
    float *xs = sx + ai * 4 * MK;
    xs[k] = act ? a.H2[(long)i * MK + k] : 0.f;
    __syncthreads();
    float gz = 0.f;
    if (k < a.RH) {
        const float *w = a.W_r2 + k * MK;
        float zz = a.b_r2[k];
        for (int q = 0; q < MK; q++) zz = fmaf(w[q], xs[q], zz);
        gz = gE * a.w_r2[k] * mc_dsilu(zz);
    }
    xs[MK + k] = gz;
    __syncthreads();
    float gh = 0.f;
    for (int q = 0; q < a.RH; q++) gh = fmaf(a.W_r2[q * MK + k], xs[MK + q], gh);
    xs[2 * MK + k] = gh;
    __syncthreads();
    float gm[1] = {0.f}, gs = 0.f;
    {
        const float *wo = a.Wout[0] + k, *ws = a.Wsc1 + (long)z * MK * MK + k;
        const float *v = xs + 2 * MK;
#pragma unroll 8
        for (int q = 0; q < MK; q++) {
            gm[0] = fmaf(wo[q * MK], v[q], gm[0]);
            gs = fmaf(ws[q * MK], v[q], gs);
        }
    }
    if (act) a.GH1S[(long)i * MK + k] = gs;
    float A[16], P[NPP], gA[16], gP[NPP];
    load_ap(a.AP, act, i, k, A);
    pair_fwd(A, P);
#pragma unroll
    for (int q = 0; q < 16; q++) gA[q] = 0.f;
#pragma unroll
    for (int q = 0; q < NPP; q++) gP[q] = 0.f;
    sym_bwd<0>(A, P, a.Wsym[0] + (long)z * a.np[0] * MK + k, gm, gA, gP);
    pair_bwd(A, gP, gA);
    if (act) store_gap(a.GAP, i, k, gA);
}

__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_mc_node0_bwd(int nd, const int *__restrict__ zsp,
                                                                                         McNodeBwdArgs a) {
    __shared__ float sx[APB * 4 * MK];
    const int tid = threadIdx.x, k = tid & 31, ai = tid >> 5;
    const int i = blockIdx.x * APB + ai;
    const bool act = i < nd;
    const int z = act ? zsp[i] : 0;
    const float gE = (act && a.perm[i] < a.n_local) ? 1.f : 0.f;
    // dE/dhb1 of this atom: the partials its out-edges left on their reverse edges
    float gh[4] = {0.f, 0.f, 0.f, 0.f};
    if (act) {
        const int eend = a.rowc[i + 1];
        for (int e = a.rowc[i]; e < eend; e++) {
            if (a.colc[e] >= a.nd1) continue;
            const float *mp = a.MSG + (long)a.revc[e] * 4 * MK + k;
#pragma unroll
            for (int c = 0; c < 4; c++) gh[c] += mp[c * MK];
        }
    }
    float *xs = sx + ai * 4 * MK;
#pragma unroll
    for (int c = 0; c < 4; c++) xs[c * MK + k] = gh[c];
    __syncthreads();
    float g1[4];
    {
        const float *W[4] = {a.Wup1[0], a.Wup1[1], a.Wup1[1], a.Wup1[1]};
        mix<4>(W, xs, k, g1);
    }
    g1[0] += gE * a.w_r1[k] + ((act && i < a.nd1) ? a.GH1S[(long)i * MK + k] : 0.f);
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 4; c++) xs[c * MK + k] = g1[c];
    __syncthreads();
    float gm[4];
    {
        const float *W[4] = {a.Wout[0], a.Wout[1], a.Wout[1], a.Wout[1]};
        mix<4>(W, xs, k, gm);
    }
    float A[16], P[NPP], gA[16], gP[NPP];
    load_ap(a.AP, act, i, k, A);
    pair_fwd(A, P);
#pragma unroll
    for (int q = 0; q < 16; q++) gA[q] = 0.f;
#pragma unroll
    for (int q = 0; q < NPP; q++) gP[q] = 0.f;
    sym_bwd<0>(A, P, a.Wsym[0] + (long)z * a.np[0] * MK + k, gm, gA, gP);
    sym_bwd<1>(A, P, a.Wsym[1] + (long)z * a.np[1] * MK + k, gm + 1, gA, gP);
    pair_bwd(A, gP, gA);
    if (act) store_gap(a.GAP, i, k, gA);
}

// ---------------------------------------------------------------------------
// Adjoint of the second layer's convolution, by destination: dE/dR per edge
// (written over R), dE/dY per edge (sums over the channels), and per edge the
// gradient its source's hb receives (MSG[e][4][K]), collected later by the
// source through the reverse edge.  The l2 = 1 paths work on
// X_p[a][b] = sum_c G_p[a][b][c] dE/dA_p,c, formed once per atom.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mc_conv1_bwd(const int *__restrict__ rowc, const int *__restrict__ colc, int nd,
                                                      const float *__restrict__ Y, float *__restrict__ R,
                                                      const float *__restrict__ HB, float scale, McBlk GAR,
                                                      float *__restrict__ GY, float *__restrict__ MSG) {
    constexpr int NP = 10;
    const int k = threadIdx.x & 31;
    const int i = blockIdx.x * APB + (threadIdx.x >> 5);
    if (i >= nd) return;
    float gA0[16], X[NMOM];
#pragma unroll
    for (int p = 0; p < 4; p++) {
        const int L = p, nc = 2 * L + 1, ld = cp_nL(L, NP) * MK;
        const float *o = GAR.p[L] + (long)i * nc * ld + cp_loc(p) * MK + k;
#pragma unroll
        for (int c = 0; c < nc; c++) gA0[p * p + c] = o[(long)c * ld] * scale;
    }
#pragma unroll
    for (int q = 0; q < NMOM; q++) X[q] = 0.f;
    cg::sfor<6>([&](auto pi) MC_INLINE {
        constexpr int p = 4 + decltype(pi)::value, L = cp_L(p), nc = 2 * L + 1, ld = cp_nL(L, NP) * MK,
                      mo = cp_moff(p), e0 = kConv.beg[p];
        const float *o = GAR.p[L] + (long)i * nc * ld + cp_loc(p) * MK + k;
        float g[nc];
#pragma unroll
        for (int c = 0; c < nc; c++) g[c] = o[(long)c * ld] * scale;
        cg::sfor<kConv.beg[p + 1] - e0>([&](auto t) MC_INLINE {
            constexpr CEnt E = kConv.e[e0 + decltype(t)::value];
            X[mo + E.a * 3 + E.b] = fmaf(E.v, g[E.c], X[mo + E.a * 3 + E.b]);
        });
    });
    const int eend = rowc[i + 1];
    for (int e = rowc[i]; e < eend; e++) {
        const int j = colc[e];
        const float *hb = HB + (long)j * 4 * MK + k;
        const float h0 = hb[0], h1[3] = {hb[MK], hb[2 * MK], hb[3 * MK]};
        float y[16], r[NP];
        load16(Y + (long)e * 16, y);
        float *rr = R + (long)e * NP * MK + k;
#pragma unroll
        for (int p = 0; p < NP; p++) r[p] = rr[p * MK];
        float gy[16], gh[4] = {0.f, 0.f, 0.f, 0.f}, gR[NP];
#pragma unroll
        for (int p = 0; p < 4; p++) {
            float d = 0.f;
#pragma unroll
            for (int c = 0; c < 2 * p + 1; c++) {
                d = fmaf(gA0[p * p + c], y[p * p + c], d);
                gy[p * p + c] = gA0[p * p + c] * (r[p] * h0);
            }
            gR[p] = d * h0;
            gh[0] = fmaf(r[p], d, gh[0]);
        }
#pragma unroll
        for (int p = 4; p < NP; p++) {
            const int l1 = cp_l1(p), mo = cp_moff(p);
            float u[3] = {0.f, 0.f, 0.f};
#pragma unroll
            for (int a = 0; a < 2 * l1 + 1; a++) {
                float wa = 0.f;
#pragma unroll
                for (int b = 0; b < 3; b++) {
                    u[b] = fmaf(X[mo + a * 3 + b], y[l1 * l1 + a], u[b]);
                    wa = fmaf(X[mo + a * 3 + b], h1[b], wa);
                }
                gy[l1 * l1 + a] = fmaf(r[p], wa, gy[l1 * l1 + a]);
            }
            gR[p] = u[0] * h1[0] + u[1] * h1[1] + u[2] * h1[2];
#pragma unroll
            for (int b = 0; b < 3; b++) gh[1 + b] = fmaf(r[p], u[b], gh[1 + b]);
        }
#pragma unroll
        for (int p = 0; p < NP; p++) rr[p * MK] = gR[p];
        float *mp = MSG + (long)e * 4 * MK + k;
#pragma unroll
        for (int c = 0; c < 4; c++) mp[c * MK] = gh[c];
        const float s = halfwave_sum16(gy, k);
        if (k < 16) GY[(long)e * 16 + k] = s;
    }
}

// Adjoint of the first layer's convolution (hb depends on the species only,
// so nothing flows to the sources): dE/dR over R, dE/dY added to the second
// layer's for destinations it covers.
__global__ void __launch_bounds__(256) k_mc_conv0_bwd(const int *__restrict__ rowc, const int *__restrict__ colc, int nd,
                                                      int nd1, const float *__restrict__ Y, float *__restrict__ R,
                                                      const int *__restrict__ zsp, const float *__restrict__ hb0,
                                                      float scale, McBlk GAR, float *__restrict__ GY) {
    const int k = threadIdx.x & 31;
    const int i = blockIdx.x * APB + (threadIdx.x >> 5);
    if (i >= nd) return;
    float gA[16];
#pragma unroll
    for (int L = 0; L < 4; L++)
#pragma unroll
        for (int c = 0; c < 2 * L + 1; c++) gA[L * L + c] = GAR.p[L][((long)i * (2 * L + 1) + c) * MK + k] * scale;
    const bool add = i < nd1;
    const int eend = rowc[i + 1];
    for (int e = rowc[i]; e < eend; e++) {
        const float h0 = hb0[zsp[colc[e]] * MK + k];
        float y[16];
        load16(Y + (long)e * 16, y);
        float *rr = R + (long)e * 4 * MK + k;
        float gy[16];
#pragma unroll
        for (int p = 0; p < 4; p++) {
            const float rp = rr[p * MK];
            float d = 0.f;
#pragma unroll
            for (int c = 0; c < 2 * p + 1; c++) {
                d = fmaf(gA[p * p + c], y[p * p + c], d);
                gy[p * p + c] = gA[p * p + c] * (rp * h0);
            }
            rr[p * MK] = d * h0;
        }
        const float s = halfwave_sum16(gy, k);
        if (k < 16) {
            float *g = GY + (long)e * 16 + k;
            *g = add ? *g + s : s;
        }
    }
}

// Per edge: dE/dr through the radial functions and the envelope, dE/drhat
// from the harmonics, G_e = dE/d(r_i - r_j); edges no layer reaches get 0.
__global__ void k_mc_geom(const int *__restrict__ rowc, int n, const int *__restrict__ e0,
                          const float4 *__restrict__ geom, int NB, int NBP, int pe, float rc,
                          const float *__restrict__ GX, const float *__restrict__ GY, float4 *__restrict__ G) {
    const long ne = rowc[n], ne0 = *e0;
    const float c0 = sqrtf(2.0f / rc), th = 3.14159265358979f / rc;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (long)gridDim.x * blockDim.x) {
        if (e >= ne0) {
            G[e] = make_float4(0.f, 0.f, 0.f, 0.f);
            continue;
        }
        const float4 gm = geom[e];
        const float r = gm.w, ir = 1.0f / r;
        float u, du;
        envelope(r / rc, pe, u, du);
        du *= 1.0f / rc;
        float sn, cs;
        sincosf(th * r, &sn, &cs);
        const float *gb = GX + e * NBP;
        float dEdr = 0.f;
        float sk = sn, skm = 0.f, ck = cs, ckm = 1.f;
        for (int k = 0; k < NB; k++) {
            const float kt = (k + 1) * th;
            const float dB = c0 * ((kt * ck * ir - sk * ir * ir) * u + sk * ir * du);
            dEdr = fmaf(gb[k], dB, dEdr);
            const float ns = 2.f * cs * sk - skm, nc = 2.f * cs * ck - ckm;
            skm = sk;
            sk = ns;
            ckm = ck;
            ck = nc;
        }
        const float x = gm.x * ir, y = gm.y * ir, z = gm.z * ir;
        float gy[16];
        load16(GY + e * 16, gy);
        float hx, hy, hz;
        sh16_grad(x, y, z, gy, hx, hy, hz);
        const float rd = hx * x + hy * y + hz * z;
        const float gx = dEdr * x + (hx - rd * x) * ir, gyy = dEdr * y + (hy - rd * y) * ir,
                    gz = dEdr * z + (hz - rd * z) * ir;
        G[e] = make_float4(-gx, -gyy, -gz, 0.f);
    }
}

__global__ void k_mc_zero(float *__restrict__ p, long n) {
    for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) p[q] = 0.f;
}

// Species tables of the first layer, whose input is the embedding alone:
// hb0[z] = W_up0 W_emb[:, z] and skip0[z] = W_sc0[z] W_emb[:, z].
__global__ void k_mc_species(int S, const float *__restrict__ Wemb, const float *__restrict__ Wup0,
                             const float *__restrict__ Wsc0, float *__restrict__ hb0, float *__restrict__ skip0) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= S * MK) return;
    const int z = t / MK, k = t % MK;
    float a = 0.f, b = 0.f;
    for (int q = 0; q < MK; q++) {
        const float h = Wemb[q * S + z];
        a = fmaf(Wup0[k * MK + q], h, a);
        b = fmaf(Wsc0[((long)z * MK + k) * MK + q], h, b);
    }
    hb0[t] = a;
    skip0[t] = b;
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------
struct McArena {
    long X0, Y, P[2][4], A[2][4], R[2], GY, GX0, MSG, AR[2], AP[2], GAP, H1, HB1, H2, GH1S, U, EP, total;
};

static McArena mc_layout(const McModel &a, long N, long E) {
    McArena L;
    long o = 0;
    auto take = [&](long cnt) {
        const long r = o;
        o += (cnt + 63) / 64 * 64;
        return r;
    };
    L.X0 = take(E * a.NBP);
    L.Y = take(E * 16);
    for (int t = 0; t < 2; t++) {
        for (int q = 0; q < 4; q++) L.P[t][q] = L.A[t][q] = 0;
        if (!a.fused)
            for (int q = 0; q < a.nrad; q++) {
                L.P[t][q] = take(E * a.rh[q]);
                L.A[t][q] = take(E * a.rh[q]);
            }
        L.R[t] = take(E * (t == 0 ? 4 : 10) * MK);
    }
    L.GY = take(E * 16);
    L.GX0 = take(E * a.NBP);
    L.MSG = take(E * 4 * MK);
    L.AR[0] = take(N * 16 * MK);
    L.AR[1] = take(N * 40 * MK);
    L.AP[0] = take(N * 16 * MK);
    L.AP[1] = take(N * 16 * MK);
    L.GAP = take(N * 16 * MK);
    L.H1 = take(N * 4 * MK);
    L.HB1 = take(N * 4 * MK);
    L.H2 = take(N * MK);
    L.GH1S = take(N * MK);
    L.U = take(N + 64);
    L.EP = take(2 * energy_part_doubles(N));   // the energy sums' chunk partials (doubles)
    L.total = o + 4096;
    return L;
}

size_t mace_arena_bytes(const mlp_model *m, long n_atoms, long n_edges) {
    return (size_t)mc_layout(*m->mc, n_atoms, n_edges).total * sizeof(float);
}

int mace_create(mlp_model *m, const McDims &d, const float *w, size_t n_weights) {
    if (d.S < 1 || d.S > 64) return fail(-1, "mace: n_species out of range");
    if (d.NB < 1 || d.NB > 16) return fail(-1, "mace: n_basis must be 1..16");
    if (d.p < 1 || d.p > 8) return fail(-1, "mace: envelope_p must be 1..8");
    if (d.lmax != 3 || d.K != MK || d.corr != 3)
        return fail(-1, "mace: this build takes l_max 3, 32 channels and correlation order 3");
    if (d.nrad < 1 || d.nrad > 4) return fail(-1, "mace: radial_hidden needs 1..4 widths");
    for (int q = 0; q < d.nrad; q++)
        if (d.rh[q] < 4 || d.rh[q] % 4 || d.rh[q] > 256) return fail(-1, "mace: radial widths must be multiples of 4 up to 256");
    if (d.RH < 1 || d.RH > MK) return fail(-1, "mace: readout_hidden must be 1..32");
    if (!(d.rc > 0.f) || !(d.navg > 0.f)) return fail(-1, "mace: r_c and avg_neighbors must be positive");
    const int S = d.S, K = MK, NB = d.NB;
    // contraction paths per layer and output degree (layer 1: degrees 0 and 1; layer 2: degree 0)
    const int npath[2][2] = {{kSym0.np, kSym1.np}, {kSym0.np, 0}}, nout[2] = {2, 1};
    // storage order (matrices [out][in]): W_emb (K x S); per layer: W_up per
    // input degree, radial matrices, W_A per L, W_sym per output degree,
    // W_out per output degree, W_sc for degree 0 (the one output degree both
    // layers also take); then w_r1, W_r2, b_r2, w_r2, b_r3
    size_t off = 0;
    auto take = [&](size_t cnt) {
        const size_t r = off;
        off += cnt;
        return r;
    };
    const size_t oEmb = take((size_t)K * S);
    size_t oUp[2][2], oRad[2][5], oWA[2][4], oSym[2][2], oOut[2][2], oSc[2];
    const int NPt[2] = {4, 10};
    for (int t = 0; t < 2; t++) {
        for (int l2 = 0; l2 <= t; l2++) oUp[t][l2] = take((size_t)K * K);
        int prev = NB;
        for (int q = 0; q < d.nrad; q++) {
            oRad[t][q] = take((size_t)d.rh[q] * prev);
            prev = d.rh[q];
        }
        oRad[t][d.nrad] = take((size_t)NPt[t] * K * prev);
        for (int L = 0; L < 4; L++) oWA[t][L] = take((size_t)K * cp_nL(L, NPt[t]) * K);
        for (int q = 0; q < nout[t]; q++) oSym[t][q] = take((size_t)S * K * npath[t][q]);
        for (int q = 0; q < nout[t]; q++) oOut[t][q] = take((size_t)K * K);
        oSc[t] = take((size_t)S * K * K);
    }
    const size_t oR1 = take(K), oWR2 = take((size_t)d.RH * K), oBR2 = take(d.RH), oWr2 = take(d.RH), oBR3 = take(1);
    if (off != n_weights)
        return fail(-1, "mace: weight count " + std::to_string(n_weights) + " does not match the header (" +
                            std::to_string(off) + ")");

    McModel *a = new McModel();
    a->S = S;
    a->NB = NB;
    a->NBP = (NB + 3) / 4 * 4;
    a->pe = d.p;
    a->nrad = d.nrad;
    for (int q = 0; q < d.nrad; q++) a->rh[q] = d.rh[q];
    a->RH = d.RH;
    a->rc = d.rc;
    a->navg = d.navg;
    a->b_r3 = w[oBR3];

    // device floats: the weights as given, then transposed copies and tables
    std::vector<float> host(w, w + n_weights);
    auto push = [&](const std::vector<float> &v) {
        while (host.size() % 64) host.push_back(0.f);
        const size_t r = host.size();
        host.insert(host.end(), v.begin(), v.end());
        return r;
    };
    auto transpose = [&](size_t o) {   // K x K, [k][k'] -> [k'][k]
        std::vector<float> t((size_t)K * K);
        for (int r = 0; r < K; r++)
            for (int c = 0; c < K; c++) t[(size_t)c * K + r] = w[o + (size_t)r * K + c];
        return t;
    };
    size_t oWoutT[2][2] = {}, oWupT1[2], oWscT1, oSymT[2][2] = {};
    for (int t = 0; t < 2; t++)
        for (int q = 0; q < nout[t]; q++) oWoutT[t][q] = push(transpose(oOut[t][q]));
    for (int l2 = 0; l2 < 2; l2++) oWupT1[l2] = push(transpose(oUp[1][l2]));
    {
        std::vector<float> t((size_t)S * K * K);
        for (int z = 0; z < S; z++)
            for (int r = 0; r < K; r++)
                for (int c = 0; c < K; c++) t[((size_t)z * K + c) * K + r] = w[oSc[1] + ((size_t)z * K + r) * K + c];
        oWscT1 = push(t);
    }
    for (int t = 0; t < 2; t++)
        for (int q = 0; q < nout[t]; q++) {
            const int np = npath[t][q];
            std::vector<float> v((size_t)S * np * K);
            for (int z = 0; z < S; z++)
                for (int k = 0; k < K; k++)
                    for (int e = 0; e < np; e++) v[((size_t)z * np + e) * K + k] = w[oSym[t][q] + ((size_t)z * K + k) * np + e];
            oSymT[t][q] = push(v);
        }
    const size_t oZero = push(std::vector<float>(512, 0.f));
    const size_t oHb0 = push(std::vector<float>((size_t)S * K, 0.f));
    const size_t oSkip0 = push(std::vector<float>((size_t)S * K, 0.f));
    float *dev = nullptr;
    if (hipMalloc(&dev, sizeof(float) * host.size()) != hipSuccess) {
        (void)hipGetLastError();
        delete a;
        return fail(-2, "mace: weight allocation failed");
    }
    if (hipMemcpy(dev, host.data(), sizeof(float) * host.size(), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(dev);
        delete a;
        return fail(-5, "mace: weight copy failed");
    }
    a->dev = dev;
    for (int t = 0; t < 2; t++)
        for (int q = 0; q < nout[t]; q++) {
            a->Wsym[t][q] = dev + oSymT[t][q];
            a->WoutT[t][q] = dev + oWoutT[t][q];
            a->Wout[t][q] = dev + oOut[t][q];
        }
    for (int l2 = 0; l2 < 2; l2++) {
        a->WupT1[l2] = dev + oWupT1[l2];
        a->Wup1[l2] = dev + oUp[1][l2];
    }
    a->WscT1 = dev + oWscT1;
    a->Wsc1 = dev + oSc[1];
    a->zero = dev + oZero;
    a->hb0tab = dev + oHb0;
    a->skip0tab = dev + oSkip0;
    a->w_r1 = dev + oR1;
    a->W_r2 = dev + oWR2;
    a->b_r2 = dev + oBR2;
    a->w_r2 = dev + oWr2;
    k_mc_species<<<nblk((long)S * K, 256), 256>>>(S, dev + oEmb, dev + oUp[0][0], dev + oSc[0], dev + oHb0,
                                                   dev + oSkip0);
    // GEMM operands: radial matrices and W_A, forward and adjoint
    struct Item {
        const float *W;
        int R, C;
        bool tr;
        PackedW *dst;
    };
    std::vector<Item> items;
    for (int t = 0; t < 2; t++) {
        int prev = NB;
        for (int q = 0; q <= d.nrad; q++) {
            const int rows = q < d.nrad ? d.rh[q] : NPt[t] * K;
            items.push_back({dev + oRad[t][q], rows, prev, false, &a->radF[t][q]});
            items.push_back({dev + oRad[t][q], rows, prev, true, &a->radA[t][q]});
            prev = rows;
        }
        for (int L = 0; L < 4; L++) {
            const int cols = cp_nL(L, NPt[t]) * K;
            items.push_back({dev + oWA[t][L], K, cols, false, &a->waF[t][L]});
            items.push_back({dev + oWA[t][L], K, cols, true, &a->waA[t][L]});
        }
    }
    size_t pk = 0;
    for (const Item &it : items) pk += packed_bytes(it.R, it.C, it.tr);
    int rc = hipMalloc(&a->pk_dev, pk) == hipSuccess ? 0 : -2;
    for (size_t q = 0, o = 0; rc == 0 && q < items.size(); q++) {
        if (pack_weight(nullptr, items[q].W, items[q].R, items[q].C, items[q].tr, (char *)a->pk_dev + o, items[q].dst))
            rc = -5;
        o += packed_bytes(items[q].R, items[q].C, items[q].tr);
    }
    if (rc == 0 && (hipGetLastError() != hipSuccess || hipDeviceSynchronize() != hipSuccess)) rc = -5;
    if (rc) {
        (void)hipGetLastError();
        if (a->pk_dev) hipFree(a->pk_dev);
        hipFree(dev);
        delete a;
        return fail(rc, "mace: weight packing failed");
    }
    // the radial MLPs run as one fused kernel each way where the shape allows
    // (three hidden layers of at most 64, at most 32 radial functions)
    a->fused = d.nrad == 3 && NB <= 16;
    for (int q = 0; q < d.nrad; q++) a->fused = a->fused && d.rh[q] <= 64;
    for (int t = 0; t < 2; t++) {
        a->rmlp[t].nh = d.nrad;
        for (int q = 0; q <= d.nrad; q++) {
            a->rmlp[t].f[q] = a->radF[t][q];
            a->rmlp[t].a[q] = a->radA[t][q];
        }
    }
    m->mc = a;
    return 0;
}

void mace_destroy(mlp_model *m) {
    if (!m || !m->mc) return;
    if (m->mc->pk_dev) hipFree(m->mc->pk_dev);
    if (m->mc->dev) hipFree(m->mc->dev);
    delete m->mc;
    m->mc = nullptr;
}

static int mgm(hipStream_t s, int P, int epi, const float *A, int lda, const PackedW &B, float *C, int ldc, long M,
               const int *Mc, const float *bias = nullptr, float *C2 = nullptr, int ldc2 = 0,
               const float *R = nullptr, int ldr = 0) {
    if (M <= 0) return 0;
    ProfScope ps(PK_GEMM, s);
    return node_gemm(s, P, epi, A, lda, B, C, ldc, (int)M, bias, C2, ldc2, R, ldr, Mc) ? fail(-5, "mace GEMM failed")
                                                                                         : 0;
}

int mace_evaluate(mlp_model *m, mlp_nbr *g, hipStream_t s, double *energy, float *forces_user,
                  float *atom_energy_user, int n_seg, const int *seg_dev) {
    const McModel &a = *m->mc;
    const int n = g->n_atoms, P = node_operands(m->precision), T = 2;
    const long E = g->n_edges_skin;
    int rc;
    if ((rc = g->act.ensure(mace_arena_bytes(m, n, E), 1.2, &g->n_grows))) return rc;
    if ((rc = g->G.ensure(sizeof(float4) * (size_t)E + 64, 1.2, &g->n_grows))) return rc;
    const McArena L = mc_layout(a, n, E);
    float *base = g->act.as<float>();
    float *X0 = base + L.X0, *Y = base + L.Y, *GY = base + L.GY, *GX0 = base + L.GX0, *MSG = base + L.MSG,
          *H1 = base + L.H1, *HB1 = base + L.HB1, *H2 = base + L.H2, *GH1S = base + L.GH1S, *U = base + L.U;
    const int *rowc = g->rowc.as<int>(), *colc = g->colc.as<int>(), *revc = g->revc.as<int>(),
              *perm = g->perm.as<int>(), *zsp = g->species.as<int>();
    const float4 *geom = g->geom.as<float4>();
    // rows each layer's node work covers: the first layer the atoms within
    // one hop of the locals, the second the locals (all rows without ghosts)
    const bool ho = g->nhop[0] > 0 && g->nhop[T + 1] == n;
    const int nd0 = ho ? g->nhop[1] : n, nd1 = ho ? g->nhop[0] : n;
    // edge rows of each layer: a prefix of the destination-sorted edges,
    // counted on the device
    const int *e0 = rowc + nd0, *e1 = rowc + nd1;
    const float scale = 1.0f / a.navg;
    const int NPt[2] = {4, 10};
    auto blk = [&](long o, int t) {
        McBlk b;
        long q = o;
        for (int Lq = 0; Lq < 4; Lq++) {
            b.p[Lq] = base + q;
            q += (long)n * (2 * Lq + 1) * (t < 0 ? 1 : cp_nL(Lq, NPt[t])) * MK;
        }
        return b;
    };
    const McBlk AR0 = blk(L.AR[0], 0), AR1 = blk(L.AR[1], 1), AP0 = blk(L.AP[0], -1), AP1 = blk(L.AP[1], -1),
                GAP = blk(L.GAP, -1);
    const int eg = (int)std::max<long>(1, std::min<long>(nblk(E, 256), 16384));

    // forward
    k_mc_zero<<<nblk(n + 64, 256), 256, 0, s>>>(U, n + 64);
    k_mc_edge<<<eg, 256, 0, s>>>(rowc, n, geom, a.NB, a.NBP, a.pe, a.rc, X0, Y);
    for (int t = 0; t < 2; t++) {
        if (a.fused) {
            ProfScope ps(PK_GEMM, s);
            if (edge_mlp_forward(s, P, a.rmlp[t], X0, a.NBP, base + L.R[t], NPt[t] * MK, (int)E, t ? e1 : e0))
                return fail(-5, "mace radial MLP failed");
            continue;
        }
        const float *in = X0;
        int ldin = a.NBP;
        for (int q = 0; q < a.nrad; q++) {
            if ((rc = mgm(s, P, GE_BIAS_SILU, in, ldin, a.radF[t][q], base + L.P[t][q], a.rh[q], E, t ? e1 : e0,
                          a.zero, base + L.A[t][q], a.rh[q])))
                return rc;
            in = base + L.A[t][q];
            ldin = a.rh[q];
        }
        if ((rc = mgm(s, P, GE_STORE, in, ldin, a.radF[t][a.nrad], base + L.R[t], NPt[t] * MK, E, t ? e1 : e0)))
            return rc;
    }
    McNodeArgs na{};
    na.skip0tab = a.skip0tab;
    na.WupT1[0] = a.WupT1[0];
    na.WupT1[1] = a.WupT1[1];
    na.WscT1 = a.WscT1;
    na.w_r1 = a.w_r1;
    na.W_r2 = a.W_r2;
    na.b_r2 = a.b_r2;
    na.w_r2 = a.w_r2;
    na.b_r3 = a.b_r3;
    na.RH = a.RH;
    na.H1 = H1;
    na.H1o = H1;
    na.HB1o = HB1;
    na.H2 = H2;
    na.U = U;
    na.nloc = nd1;
    na.np[0] = kSym0.np;
    na.np[1] = kSym1.np;
    for (int t = 0; t < 2; t++) {
        const int nd = t ? nd1 : nd0;
        if (nd <= 0) continue;
        const McBlk &AR = t ? AR1 : AR0, &AP = t ? AP1 : AP0;
        if (t == 0)
            k_mc_conv<0><<<nblk(nd, APB), 256, 0, s>>>(rowc, colc, nd, Y, base + L.R[0], nullptr, zsp, a.hb0tab, scale,
                                                       AR);
        else
            k_mc_conv<1><<<nblk(nd, APB), 256, 0, s>>>(rowc, colc, nd, Y, base + L.R[1], HB1, zsp, a.hb0tab, scale, AR);
        for (int Lq = 0; Lq < 4; Lq++) {
            const int ld = cp_nL(Lq, NPt[t]) * MK;
            if ((rc = mgm(s, P, GE_STORE, AR.p[Lq], ld, a.waF[t][Lq], AP.p[Lq], MK, (long)nd * (2 * Lq + 1), nullptr)))
                return rc;
        }
        na.AP = AP;
        na.Wsym[0] = a.Wsym[t][0];
        na.Wsym[1] = a.Wsym[t][1];
        na.WoutT[0] = a.WoutT[t][0];
        na.WoutT[1] = a.WoutT[t][1];
        if (t == 0) k_mc_node<0><<<nblk(nd, APB), 256, 0, s>>>(nd, zsp, na);
        else k_mc_node<1><<<nblk(nd, APB), 256, 0, s>>>(nd, zsp, na);
    }
    HIP_TRY(hipGetLastError());
    if ((rc = launch_energy(s, U, perm, n, g->n_local, energy, atom_energy_user, n_seg, seg_dev,
                            reinterpret_cast<double *>(base + L.EP))))
        return rc;
    if (!forces_user) return 0;

    // adjoint
    McNodeBwdArgs nb{};
    nb.Wsc1 = a.Wsc1;
    nb.Wup1[0] = a.Wup1[0];
    nb.Wup1[1] = a.Wup1[1];
    nb.w_r1 = a.w_r1;
    nb.W_r2 = a.W_r2;
    nb.b_r2 = a.b_r2;
    nb.w_r2 = a.w_r2;
    nb.RH = a.RH;
    nb.H2 = H2;
    nb.GH1S = GH1S;
    nb.rowc = rowc;
    nb.colc = colc;
    nb.revc = revc;
    nb.MSG = MSG;
    nb.nd1 = nd1;
    nb.perm = perm;
    nb.n_local = g->n_local;
    nb.GAP = GAP;
    nb.np[0] = kSym0.np;
    nb.np[1] = kSym1.np;
    if (nd1 > 0) {
        nb.AP = AP1;
        nb.Wsym[0] = a.Wsym[1][0];
        nb.Wsym[1] = nullptr;
        nb.Wout[0] = a.Wout[1][0];
        nb.Wout[1] = a.Wout[1][0];
        k_mc_node1_bwd<<<nblk(nd1, APB), 256, 0, s>>>(nd1, zsp, nb);
        // dE/dA (before the W_A mix) over the A blocks
        for (int Lq = 0; Lq < 4; Lq++) {
            const int ld = cp_nL(Lq, 10) * MK;
            if ((rc = mgm(s, P, GE_STORE, GAP.p[Lq], MK, a.waA[1][Lq], AR1.p[Lq], ld, (long)nd1 * (2 * Lq + 1), nullptr)))
                return rc;
        }
        k_mc_conv1_bwd<<<nblk(nd1, APB), 256, 0, s>>>(rowc, colc, nd1, Y, base + L.R[1], HB1, scale, AR1, GY, MSG);
    }
    if (nd0 > 0) {
        nb.AP = AP0;
        nb.Wsym[0] = a.Wsym[0][0];
        nb.Wsym[1] = a.Wsym[0][1];
        nb.Wout[0] = a.Wout[0][0];
        nb.Wout[1] = a.Wout[0][1];
        k_mc_node0_bwd<<<nblk(nd0, APB), 256, 0, s>>>(nd0, zsp, nb);
        for (int Lq = 0; Lq < 4; Lq++)
            if ((rc = mgm(s, P, GE_STORE, GAP.p[Lq], MK, a.waA[0][Lq], AR0.p[Lq], MK, (long)nd0 * (2 * Lq + 1), nullptr)))
                return rc;
        k_mc_conv0_bwd<<<nblk(nd0, APB), 256, 0, s>>>(rowc, colc, nd0, nd1, Y, base + L.R[0], zsp, a.hb0tab, scale,
                                                      AR0, GY);
    }
    // the radial MLPs in reverse (dE/dR in R), the first layer's over all its
    // edges first (stored), then the second layer's added on its prefix
    for (int t = 0; t < 2; t++) {
        const int *cnt = t ? e1 : e0;
        if (a.fused) {
            ProfScope ps(PK_GEMM, s);
            if (edge_mlp_adjoint(s, P, a.rmlp[t], X0, a.NBP, base + L.R[t], NPt[t] * MK, GX0, a.NBP, t != 0, (int)E, cnt))
                return fail(-5, "mace radial MLP adjoint failed");
            continue;
        }
        const float *gin = base + L.R[t];
        int ldg = NPt[t] * MK;
        for (int q = a.nrad - 1; q >= 0; q--) {
            float *dst = base + L.A[t][q];
            if ((rc = mgm(s, P, GE_DSILU, gin, ldg, a.radA[t][q + 1], dst, a.rh[q], E, cnt, nullptr, nullptr, 0,
                          base + L.P[t][q], a.rh[q])))
                return rc;
            gin = dst;
            ldg = a.rh[q];
        }
        if ((rc = mgm(s, P, t ? GE_ADD : GE_STORE, gin, ldg, a.radA[t][0], GX0, a.NBP, E, cnt, nullptr, nullptr, 0,
                      GX0, a.NBP)))
            return rc;
    }
    k_mc_geom<<<eg, 256, 0, s>>>(rowc, n, e0, geom, a.NB, a.NBP, a.pe, a.rc, GX0, GY, g->G.as<float4>());
    HIP_TRY(hipGetLastError());
    return launch_forces(s, rowc, revc, g->G.as<float4>(), perm, n, forces_user);
}

}  // namespace mlp
