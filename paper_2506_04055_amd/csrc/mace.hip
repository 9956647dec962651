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
// couplings are computed once on the host by an exact quadrature of the same
// harmonics, so the kernels and the tables share one basis.
//
// Layout of the work: the radial MLPs are GEMMs over edges and the W_A
// channel mixes GEMMs over (atom, m) rows, on the matrix cores (gemm.hip).
// The convolution, the symmetric contraction and the small per-atom channel
// mixes (W_out, W_sc, W_up, the readouts) run with one half-wave per atom and
// one lane per channel.  The symmetric contraction walks a host-built list of
// expanded product terms (uniform over the wave, read through the scalar
// cache) against the lane's A' held in LDS.  Forces come from a hand-written
// adjoint: the same kernels reversed, the gradient of each source's hb
// collected from per-edge partials through the reverse-edge index (no
// atomics), and per edge G_e = dE/d(r_i - r_j), assembled into forces by
// launch_forces.
#include "internal.h"
#include "gemm.h"
#include "sh.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <tuple>
#include <vector>

namespace mlp {

namespace {

constexpr int MK = 32;     // channels: one lane each, a half-wave per atom
constexpr int NT = 72;     // coupled harmonics per edge of the l2 = 1 paths
constexpr int NGC = 318;   // coupling entries of the l2 = 1 paths
constexpr int ONE = 16;    // the LDS slot holding 1 (lower body orders of the contraction)
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
// offsets of an l2 = 1 path in the per-edge table (3 (2L + 1) entries, [b][c])
// and in the coupling table ((2 l1 + 1) 3 (2L + 1) entries, [a][b][c])
__host__ __device__ constexpr int cp_toff(int p) {
    int o = 0;
    for (int q = 4; q < p; q++) o += 3 * (2 * cp_L(q) + 1);
    return o;
}
__host__ __device__ constexpr int cp_goff(int p) {
    int o = 0;
    for (int q = 4; q < p; q++) o += (2 * cp_l1(q) + 1) * 3 * (2 * cp_L(q) + 1);
    return o;
}
static_assert(cp_off(4) == 16 && cp_off(10) == 40, "accumulator layout");
static_assert(cp_toff(10) == NT && cp_goff(10) == NGC, "coupling tables");

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

// Sum of 16 values over the 32 lanes of a half-wave: lane k ends with the
// total of value k >> 1 (each exchange hands over the half the lane drops).
__device__ __forceinline__ float halfwave_sum16(float *v, int k) {
#pragma unroll
    for (int w = 8, sh = 16; w >= 1; w >>= 1, sh >>= 1) {
        const bool up = (k & sh) != 0;
#pragma unroll
        for (int q = 0; q < w; q++) {
            const float send = up ? v[q] : v[q + w], keep = up ? v[q + w] : v[q];
            v[q] = keep + __shfl_xor(send, sh, 64);
        }
    }
    return v[0] + __shfl_xor(v[0], 1, 64);
}

__device__ __forceinline__ float halfwave_sum(float v) {
#pragma unroll
    for (int off = 16; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// T_p[b][c] = sum_a G_p[a][b][c] Y_l1a for one l2 = 1 path (compile-time shape)
template <int p>
__device__ __forceinline__ void edge_tpath(const float *__restrict__ Gc, const float *y, float *t) {
    constexpr int l1 = cp_l1(p), na = 2 * l1 + 1, nc = 2 * cp_L(p) + 1, to = cp_toff(p), go = cp_goff(p);
#pragma unroll
    for (int b = 0; b < 3; b++)
#pragma unroll
        for (int c = 0; c < nc; c++) {
            float s = 0.f;
#pragma unroll
            for (int a = 0; a < na; a++) s = fmaf(Gc[go + (a * 3 + b) * nc + c], y[l1 * l1 + a], s);
            t[to + b * nc + c] = s;
        }
}

// Adjoint of one l2 = 1 path of the second layer's convolution for one edge
// and channel: dE/dR_p, the source's hb gradient (gh[1..3]) and dE/dY_l1a.
template <int p>
__device__ __forceinline__ void conv1_bwd_path(const float *gA, const float *t, const float *h1,
                                               const float *__restrict__ Gc, float rp, float *gy, float *gh,
                                               float *gR) {
    constexpr int l1 = cp_l1(p), na = 2 * l1 + 1, nc = 2 * cp_L(p) + 1, to = cp_toff(p), go = cp_goff(p),
                  ao = cp_off(p);
    float d = 0.f;
#pragma unroll
    for (int b = 0; b < 3; b++) {
        float tb = 0.f;
#pragma unroll
        for (int c = 0; c < nc; c++) tb = fmaf(gA[ao + c], t[to + b * nc + c], tb);
        d = fmaf(tb, h1[b], d);
        gh[1 + b] = fmaf(rp, tb, gh[1 + b]);
    }
    gR[p] = d;
#pragma unroll
    for (int a = 0; a < na; a++) {
        float s = 0.f;
#pragma unroll
        for (int b = 0; b < 3; b++) {
            float sb = 0.f;
#pragma unroll
            for (int c = 0; c < nc; c++) sb = fmaf(Gc[go + (a * 3 + b) * nc + c], gA[ao + c], sb);
            s = fmaf(sb, h1[b], s);
        }
        gy[l1 * l1 + a] = fmaf(rp, s, gy[l1 * l1 + a]);
    }
}

}  // namespace

// Per-L blocks of an atom array (A before and after the W_A mix, and their gradients).
struct McBlk {
    float *p[4];
};

// One layer's symmetric contraction: segments (path, output component, first
// term, end term) grouped by output degree (segments [sb[q], sb[q + 1]) for
// the q-th output degree), terms (a1 | a2 << 5 | a3 << 10, coefficient bits)
// with a the (l, m) slot l^2 + m of A' or ONE, and W_sym per output degree
// as [species][path][K].
struct McSym {
    const int4 *seg;
    const int2 *term;
    int sb[3];
    const float *W[2];
    int np[2];
};

// ---------------------------------------------------------------------------
// Model
// ---------------------------------------------------------------------------
struct McModel {
    int S = 0, NB = 0, NBP = 0, pe = 0, nrad = 0, rh[4] = {0, 0, 0, 0}, RH = 0;
    float rc = 0.f, navg = 1.f, b_r3 = 0.f;
    float *dev = nullptr;     // weights, transposed copies, tables (device)
    int *sym_dev = nullptr;   // segments and terms of both layers (device)
    void *pk_dev = nullptr;   // packed GEMM operands
    PackedW radF[2][5], radA[2][5], waF[2][4], waA[2][4];
    const float *zero = nullptr, *Gc = nullptr, *hb0tab = nullptr, *skip0tab = nullptr;
    const float *w_r1 = nullptr, *W_r2 = nullptr, *b_r2 = nullptr, *w_r2 = nullptr;
    const float *WoutT[2][2] = {}, *Wout[2][2] = {};   // [layer][output degree index]
    const float *WupT1[2] = {}, *Wup1[2] = {};         // second layer's W_up for l2 = 0, 1
    const float *WscT1 = nullptr, *Wsc1 = nullptr;     // second layer's skip (degree 0), [S][K][K]
    McSym sym[2] = {};
};

// ---------------------------------------------------------------------------
// Forward, per edge: radial functions with the envelope, harmonics, and the
// harmonics coupled to the l2 = 1 paths: T_p[b][c] = sum_a G_p[a][b][c] Y_l1a.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mc_edge(const int *__restrict__ rowc, int n, const float4 *__restrict__ geom,
                                                 int NB, int NBP, int pe, float rc, const int *__restrict__ e1,
                                                 const float *__restrict__ Gc, float *__restrict__ X0,
                                                 float *__restrict__ Y, float *__restrict__ TT) {
    const long ne = rowc[n], ne1 = *e1;
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
        if (e < ne1) {
            float t[NT];
            edge_tpath<4>(Gc, y, t);
            edge_tpath<5>(Gc, y, t);
            edge_tpath<6>(Gc, y, t);
            edge_tpath<7>(Gc, y, t);
            edge_tpath<8>(Gc, y, t);
            edge_tpath<9>(Gc, y, t);
            float4 *t4 = reinterpret_cast<float4 *>(TT + e * NT);
#pragma unroll
            for (int q = 0; q < NT / 4; q++) t4[q] = make_float4(t[4 * q], t[4 * q + 1], t[4 * q + 2], t[4 * q + 3]);
        }
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
                                                 const float *__restrict__ Y, const float *__restrict__ TT,
                                                 const float *__restrict__ R, const float *__restrict__ HB,
                                                 const int *__restrict__ zsp, const float *__restrict__ hb0,
                                                 float scale, McBlk AR) {
    constexpr int NP = LAY == 0 ? 4 : 10, NA = cp_off(NP);
    const int k = threadIdx.x & 31;
    const int i = blockIdx.x * APB + (threadIdx.x >> 5);
    if (i >= nd) return;
    float acc[NA];
#pragma unroll
    for (int q = 0; q < NA; q++) acc[q] = 0.f;
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
        float y[16];
        load16(Y + (long)e * 16, y);
        const float *rr = R + (long)e * NP * MK + k;
        float r[NP];
#pragma unroll
        for (int p = 0; p < NP; p++) r[p] = rr[p * MK];
#pragma unroll
        for (int p = 0; p < 4; p++) {
            const float s = r[p] * h0;
#pragma unroll
            for (int c = 0; c < 2 * p + 1; c++) acc[cp_off(p) + c] = fmaf(s, y[p * p + c], acc[cp_off(p) + c]);
        }
        if constexpr (LAY == 1) {
            float t[NT];
            const float4 *t4 = reinterpret_cast<const float4 *>(TT + (long)e * NT);
#pragma unroll
            for (int q = 0; q < NT / 4; q++) {
                const float4 x = t4[q];
                t[4 * q] = x.x;
                t[4 * q + 1] = x.y;
                t[4 * q + 2] = x.z;
                t[4 * q + 3] = x.w;
            }
#pragma unroll
            for (int p = 4; p < NP; p++) {
                const int nc = 2 * cp_L(p) + 1, to = cp_toff(p);
#pragma unroll
                for (int c = 0; c < nc; c++) {
                    const float v = t[to + c] * h1[0] + t[to + nc + c] * h1[1] + t[to + 2 * nc + c] * h1[2];
                    acc[cp_off(p) + c] = fmaf(r[p], v, acc[cp_off(p) + c]);
                }
            }
        }
    }
#pragma unroll
    for (int p = 0; p < NP; p++) {
        const int L = cp_L(p), nc = 2 * L + 1, ld = cp_nL(L, NP) * MK;
        float *o = AR.p[L] + (long)i * nc * ld + cp_loc(p) * MK + k;
#pragma unroll
        for (int c = 0; c < nc; c++) o[(long)c * ld] = acc[cp_off(p) + c] * scale;
    }
}

// ---------------------------------------------------------------------------
// Per-atom kernels: one half-wave per atom, lane = channel; the lane's A'
// (16 values and the constant 1) in an LDS column of its own, the channel
// mixes through a per-atom LDS row.  Every thread of a workgroup reaches the
// barriers (rows past nd compute on zeros and write nothing).
// ---------------------------------------------------------------------------
struct McNodeArgs {
    McBlk AP;                      // A' [row][2L + 1][K] per L
    McSym sym;
    const float *WoutT[2];         // [k'][k] per output degree index
    const float *Wout[2];          // [k][k'] (adjoint)
    const float *skip0tab;         // first layer: W_sc[Z] h0 per species [S][K]
    const float *WupT1[2], *Wup1[2];
    const float *WscT1, *Wsc1;     // second layer's skip [S][K][K] (transposed / as stored)
    const float *w_r1, *W_r2, *b_r2, *w_r2;
    float b_r3;
    int RH;
    const float *H1;               // first layer's output [row][4][K]
    float *H1o, *HB1o, *H2;        // outputs
    float *U;                      // per-atom energies (rows past nloc: 0)
    int nloc;                      // rows the second layer covers
};

__device__ __forceinline__ void sym_forward(const McSym &sy, int q, const float *sA, int tid, int z, int k, float *m) {
    const float *W = sy.W[q] + (long)z * sy.np[q] * MK + k;
    for (int sg = sy.sb[q]; sg < sy.sb[q + 1]; sg++) {
        const int4 S = sy.seg[sg];
        float s = 0.f;
        for (int t = S.z; t < S.w; t++) {
            const int2 T = sy.term[t];
            const float p = sA[(T.x & 31) * 256 + tid] * sA[((T.x >> 5) & 31) * 256 + tid] * sA[(T.x >> 10) * 256 + tid];
            s = fmaf(__int_as_float(T.y), p, s);
        }
        const float v = W[S.x * MK] * s;
        if (q == 0) m[0] += v;
        else if (S.y == 0) m[1] += v;
        else if (S.y == 1) m[2] += v;
        else m[3] += v;
    }
}

__device__ __forceinline__ void sym_adjoint(const McSym &sy, int q, const float *sA, float *sG, int tid, int z, int k,
                                            const float *gm) {
    const float *W = sy.W[q] + (long)z * sy.np[q] * MK + k;
    for (int sg = sy.sb[q]; sg < sy.sb[q + 1]; sg++) {
        const int4 S = sy.seg[sg];
        const float g = W[S.x * MK] * (q == 0 ? gm[0] : (S.y == 0 ? gm[1] : (S.y == 1 ? gm[2] : gm[3])));
        for (int t = S.z; t < S.w; t++) {
            const int2 T = sy.term[t];
            const int a1 = (T.x & 31) * 256 + tid, a2 = ((T.x >> 5) & 31) * 256 + tid, a3 = (T.x >> 10) * 256 + tid;
            const float c = __int_as_float(T.y) * g;
            const float p1 = sA[a1], p2 = sA[a2], p3 = sA[a3];
            sG[a1] += c * p2 * p3;
            sG[a2] += c * p1 * p3;
            sG[a3] += c * p1 * p2;
        }
    }
}

__device__ __forceinline__ void load_ap(const McBlk &AP, bool act, int i, int k, int tid, float *sA) {
#pragma unroll
    for (int L = 0; L < 4; L++)
#pragma unroll
        for (int m = 0; m < 2 * L + 1; m++)
            sA[(L * L + m) * 256 + tid] = act ? AP.p[L][((long)i * (2 * L + 1) + m) * MK + k] : 0.f;
    sA[ONE * 256 + tid] = 1.f;
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
    __shared__ float sA[17 * 256];
    __shared__ float sx[APB * 4 * MK];
    const int tid = threadIdx.x, k = tid & 31, ai = tid >> 5;
    const int i = blockIdx.x * APB + ai;
    const bool act = i < nd;
    const int z = act ? zsp[i] : 0;
    load_ap(a.AP, act, i, k, tid, sA);
    float m[4] = {0.f, 0.f, 0.f, 0.f};
    sym_forward(a.sym, 0, sA, tid, z, k, m);
    if constexpr (LAY == 0) sym_forward(a.sym, 1, sA, tid, z, k, m);
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
    McSym sym;
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
    __shared__ float sA[17 * 256];
    __shared__ float sG[17 * 256];
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
    float gm[4] = {0.f, 0.f, 0.f, 0.f}, gs = 0.f;
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
    load_ap(a.AP, act, i, k, tid, sA);
#pragma unroll
    for (int q = 0; q < 17; q++) sG[q * 256 + tid] = 0.f;
    sym_adjoint(a.sym, 0, sA, sG, tid, z, k, gm);
    if (act)
#pragma unroll
        for (int L = 0; L < 4; L++)
#pragma unroll
            for (int m = 0; m < 2 * L + 1; m++)
                a.GAP.p[L][((long)i * (2 * L + 1) + m) * MK + k] = sG[(L * L + m) * 256 + tid];
}

__global__ void __launch_bounds__(256) k_mc_node0_bwd(int nd, const int *__restrict__ zsp, McNodeBwdArgs a) {
    __shared__ float sA[17 * 256];
    __shared__ float sG[17 * 256];
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
    load_ap(a.AP, act, i, k, tid, sA);
#pragma unroll
    for (int q = 0; q < 17; q++) sG[q * 256 + tid] = 0.f;
    sym_adjoint(a.sym, 0, sA, sG, tid, z, k, gm);
    sym_adjoint(a.sym, 1, sA, sG, tid, z, k, gm);
    if (act)
#pragma unroll
        for (int L = 0; L < 4; L++)
#pragma unroll
            for (int m = 0; m < 2 * L + 1; m++)
                a.GAP.p[L][((long)i * (2 * L + 1) + m) * MK + k] = sG[(L * L + m) * 256 + tid];
}

// ---------------------------------------------------------------------------
// Adjoint of the second layer's convolution, by destination: dE/dR per edge
// (written over R), dE/dY per edge (half-wave sums), and per edge the
// gradient its source's hb receives (MSG[e][4][K]), collected later by the
// source through the reverse edge.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mc_conv1_bwd(const int *__restrict__ rowc, const int *__restrict__ colc, int nd,
                                                      const float *__restrict__ Y, const float *__restrict__ TT,
                                                      float *__restrict__ R, const float *__restrict__ HB,
                                                      const float *__restrict__ Gc, float scale, McBlk GAR,
                                                      float *__restrict__ GY, float *__restrict__ MSG) {
    constexpr int NP = 10, NA = 40;
    const int k = threadIdx.x & 31;
    const int i = blockIdx.x * APB + (threadIdx.x >> 5);
    if (i >= nd) return;
    float gA[NA];
#pragma unroll
    for (int p = 0; p < NP; p++) {
        const int L = cp_L(p), nc = 2 * L + 1, ld = cp_nL(L, NP) * MK;
        const float *o = GAR.p[L] + (long)i * nc * ld + cp_loc(p) * MK + k;
#pragma unroll
        for (int c = 0; c < nc; c++) gA[cp_off(p) + c] = o[(long)c * ld] * scale;
    }
    const int eend = rowc[i + 1];
    for (int e = rowc[i]; e < eend; e++) {
        const int j = colc[e];
        const float *hb = HB + (long)j * 4 * MK + k;
        const float h0 = hb[0], h1[3] = {hb[MK], hb[2 * MK], hb[3 * MK]};
        float y[16], t[NT], r[NP];
        load16(Y + (long)e * 16, y);
        const float4 *t4 = reinterpret_cast<const float4 *>(TT + (long)e * NT);
#pragma unroll
        for (int q = 0; q < NT / 4; q++) {
            const float4 x = t4[q];
            t[4 * q] = x.x;
            t[4 * q + 1] = x.y;
            t[4 * q + 2] = x.z;
            t[4 * q + 3] = x.w;
        }
        float *rr = R + (long)e * NP * MK + k;
#pragma unroll
        for (int p = 0; p < NP; p++) r[p] = rr[p * MK];
        float gy[16], gh[4] = {0.f, 0.f, 0.f, 0.f}, gR[NP];
#pragma unroll
        for (int q = 0; q < 16; q++) gy[q] = 0.f;
#pragma unroll
        for (int p = 0; p < 4; p++) {
            float d = 0.f;
#pragma unroll
            for (int c = 0; c < 2 * p + 1; c++) {
                d = fmaf(gA[p * p + c], y[p * p + c], d);
                gy[p * p + c] = fmaf(gA[p * p + c], r[p] * h0, gy[p * p + c]);
            }
            gR[p] = d * h0;
            gh[0] = fmaf(r[p], d, gh[0]);
        }
        conv1_bwd_path<4>(gA, t, h1, Gc, r[4], gy, gh, gR);
        conv1_bwd_path<5>(gA, t, h1, Gc, r[5], gy, gh, gR);
        conv1_bwd_path<6>(gA, t, h1, Gc, r[6], gy, gh, gR);
        conv1_bwd_path<7>(gA, t, h1, Gc, r[7], gy, gh, gR);
        conv1_bwd_path<8>(gA, t, h1, Gc, r[8], gy, gh, gR);
        conv1_bwd_path<9>(gA, t, h1, Gc, r[9], gy, gh, gR);
#pragma unroll
        for (int p = 0; p < NP; p++) rr[p * MK] = gR[p];
        float *mp = MSG + (long)e * 4 * MK + k;
#pragma unroll
        for (int c = 0; c < 4; c++) mp[c * MK] = gh[c];
        const float s = halfwave_sum16(gy, k);
        if ((k & 1) == 0) GY[(long)e * 16 + (k >> 1)] = s;
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
                gy[p * p + c] = gA[p * p + c] * rp * h0;
            }
            rr[p * MK] = d * h0;
        }
        const float s = halfwave_sum16(gy, k);
        if ((k & 1) == 0) {
            float *g = GY + (long)e * 16 + (k >> 1);
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
// Host side: couplings, expanded contraction terms, weights
// ---------------------------------------------------------------------------
namespace {

constexpr double kPi = 3.14159265358979323846;

bool couples(int l1, int l2, int L) { return std::abs(l1 - l2) <= L && L <= l1 + l2 && (l1 + l2 + L) % 2 == 0; }

// Gauss-Legendre nodes and weights on [-1, 1] (Newton iteration on P_n).
void gauss_legendre(int n, std::vector<double> &x, std::vector<double> &w) {
    x.resize(n);
    w.resize(n);
    for (int i = 0; i < n; i++) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        for (int it = 0; it < 100; it++) {
            double p1 = 1.0, p2 = 0.0;
            for (int j = 1; j <= n; j++) {
                const double p3 = p2;
                p2 = p1;
                p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
            }
            const double pp = n * (z * p1 - p2) / (z * z - 1.0), dz = p1 / pp;
            z -= dz;
            if (std::fabs(dz) < 1e-15) break;
        }
        double p1 = 1.0, p2 = 0.0;
        for (int j = 1; j <= n; j++) {
            const double p3 = p2;
            p2 = p1;
            p1 = ((2.0 * j - 1.0) * z * p2 - (j - 1.0) * p3) / j;
        }
        const double pp = n * (z * p1 - p2) / (z * z - 1.0);
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * pp * pp);
    }
}

// G(l1, l2, L)[a][b][c] = (1 / 4 pi) int Y_l1a Y_l2b Y_Lc over the sphere, by a
// product rule (Gauss-Legendre in z, uniform in phi) exact for the degrees
// involved (at most 9).
struct Gaunt {
    std::map<std::tuple<int, int, int>, std::vector<double>> cache;
    std::vector<std::vector<double>> Yq;   // harmonics at the nodes
    std::vector<double> wq;
    Gaunt() {
        const int nz = 8, nphi = 16;
        std::vector<double> zx, zw;
        gauss_legendre(nz, zx, zw);
        for (int a = 0; a < nz; a++)
            for (int b = 0; b < nphi; b++) {
                const double ph = 2.0 * kPi * b / nphi, s = std::sqrt(std::max(0.0, 1.0 - zx[a] * zx[a]));
                std::vector<double> y(16);
                sh16<double>(s * std::cos(ph), s * std::sin(ph), zx[a], y.data());
                Yq.push_back(y);
                wq.push_back(zw[a] / (2.0 * nphi));   // (2 pi / nphi) / (4 pi)
            }
    }
    const std::vector<double> &get(int l1, int l2, int L) {
        auto key = std::make_tuple(l1, l2, L);
        auto it = cache.find(key);
        if (it != cache.end()) return it->second;
        const int n1 = 2 * l1 + 1, n2 = 2 * l2 + 1, n3 = 2 * L + 1;
        std::vector<double> g((size_t)n1 * n2 * n3, 0.0);
        for (size_t q = 0; q < wq.size(); q++)
            for (int a = 0; a < n1; a++)
                for (int b = 0; b < n2; b++)
                    for (int c = 0; c < n3; c++)
                        g[((size_t)a * n2 + b) * n3 + c] += wq[q] * Yq[q][l1 * l1 + a] * Yq[q][l2 * l2 + b] * Yq[q][L * L + c];
        return cache[key] = g;
    }
};

struct Term {
    int c, a1, a2, a3;
    double coef;
};

// Contraction paths onto degree Lo (l_max 3, correlation 3) in weight order,
// each expanded into product terms of A' slots per output component.
std::vector<std::vector<Term>> contraction_paths(Gaunt &G, int Lo) {
    std::vector<std::vector<Term>> paths;
    const int lmax = 3;
    const double tol = 1e-12;
    {
        std::vector<Term> t;
        for (int c = 0; c < 2 * Lo + 1; c++) t.push_back({c, Lo * Lo + c, ONE, ONE, 1.0});
        paths.push_back(t);
    }
    for (int l1 = 0; l1 <= lmax; l1++)
        for (int l2 = l1; l2 <= lmax; l2++) {
            if (!couples(l1, l2, Lo)) continue;
            const auto &g = G.get(l1, l2, Lo);
            const int n2 = 2 * l2 + 1, n3 = 2 * Lo + 1;
            std::vector<Term> t;
            for (int c = 0; c < n3; c++)
                for (int a = 0; a < 2 * l1 + 1; a++)
                    for (int b = 0; b < n2; b++) {
                        const double v = g[((size_t)a * n2 + b) * n3 + c];
                        if (std::fabs(v) > tol) t.push_back({c, l1 * l1 + a, l2 * l2 + b, ONE, v});
                    }
            paths.push_back(t);
        }
    for (int l1 = 0; l1 <= lmax; l1++)
        for (int l2 = l1; l2 <= lmax; l2++)
            for (int lam = 0; lam <= lmax; lam++) {
                if (!couples(l1, l2, lam)) continue;
                for (int l3 = 0; l3 <= lmax; l3++) {
                    if (!couples(lam, l3, Lo)) continue;
                    const auto &g1 = G.get(l1, l2, lam), &g2 = G.get(lam, l3, Lo);
                    const int n1 = 2 * l1 + 1, n2 = 2 * l2 + 1, nl = 2 * lam + 1, n3 = 2 * l3 + 1, no = 2 * Lo + 1;
                    std::vector<Term> t;
                    for (int d = 0; d < no; d++)
                        for (int a = 0; a < n1; a++)
                            for (int b = 0; b < n2; b++)
                                for (int c = 0; c < n3; c++) {
                                    double v = 0.0;
                                    for (int mu = 0; mu < nl; mu++)
                                        v += g1[((size_t)a * n2 + b) * nl + mu] * g2[((size_t)mu * n3 + c) * no + d];
                                    if (std::fabs(v) > tol) t.push_back({d, l1 * l1 + a, l2 * l2 + b, l3 * l3 + c, v});
                                }
                    paths.push_back(t);
                }
            }
    return paths;
}

}  // namespace

struct McArena {
    long X0, Y, TT, P[2][4], A[2][4], R[2], GY, GX0, MSG, AR[2], AP[2], GAP, H1, HB1, H2, GH1S, U, total;
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
    L.TT = take(E * NT);
    for (int t = 0; t < 2; t++) {
        for (int q = 0; q < 4; q++) L.P[t][q] = L.A[t][q] = 0;
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
    // host-side contraction terms and the weight layout they fix
    Gaunt gnt;
    std::vector<std::vector<std::vector<Term>>> paths[2];   // [layer][output degree index][path]
    const int LOUT[2][2] = {{0, 1}, {0, -1}};
    for (int t = 0; t < 2; t++)
        for (int q = 0; q < 2; q++)
            if (LOUT[t][q] >= 0) paths[t].push_back(contraction_paths(gnt, LOUT[t][q]));
    // storage order (matrices [out][in]): W_emb (K x S); per layer: W_up per
    // input degree, radial matrices, W_A per L, W_sym per output degree,
    // W_out per output degree, W_sc per output degree that is an input
    // degree; then w_r1, W_r2, b_r2, w_r2, b_r3
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
        for (size_t q = 0; q < paths[t].size(); q++) oSym[t][q] = take((size_t)S * K * paths[t][q].size());
        for (size_t q = 0; q < paths[t].size(); q++) oOut[t][q] = take((size_t)K * K);
        oSc[t] = take((size_t)S * K * K);   // degree 0 is the one output degree both layers also take
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

    // device floats: the weights as given, then transposed copies, tables
    std::vector<float> host(w, w + n_weights);
    auto push = [&](const std::vector<float> &v) {
        const size_t r = host.size();
        host.insert(host.end(), v.begin(), v.end());
        while (host.size() % 64) host.push_back(0.f);
        return r;
    };
    auto transpose = [&](size_t o) {   // K x K, [k][k'] -> [k'][k]
        std::vector<float> t((size_t)K * K);
        for (int r = 0; r < K; r++)
            for (int c = 0; c < K; c++) t[(size_t)c * K + r] = w[o + (size_t)r * K + c];
        return t;
    };
    size_t oWoutT[2][2], oWupT1[2], oWscT1, oSymT[2][2];
    for (int t = 0; t < 2; t++)
        for (size_t q = 0; q < paths[t].size(); q++) oWoutT[t][q] = push(transpose(oOut[t][q]));
    for (int l2 = 0; l2 < 2; l2++) oWupT1[l2] = push(transpose(oUp[1][l2]));
    {
        std::vector<float> t((size_t)S * K * K);
        for (int z = 0; z < S; z++)
            for (int r = 0; r < K; r++)
                for (int c = 0; c < K; c++) t[((size_t)z * K + c) * K + r] = w[oSc[1] + ((size_t)z * K + r) * K + c];
        oWscT1 = push(t);
    }
    for (int t = 0; t < 2; t++)
        for (size_t q = 0; q < paths[t].size(); q++) {
            const size_t np = paths[t][q].size();
            std::vector<float> v((size_t)S * np * K);
            for (int z = 0; z < S; z++)
                for (int k = 0; k < K; k++)
                    for (size_t e = 0; e < np; e++) v[((size_t)z * np + e) * K + k] = w[oSym[t][q] + ((size_t)z * K + k) * np + e];
            oSymT[t][q] = push(v);
        }
    std::vector<float> gc(NGC);
    for (int p = 4; p < 10; p++) {
        const auto &g = gnt.get(cp_l1(p), 1, cp_L(p));
        for (size_t q = 0; q < g.size(); q++) gc[cp_goff(p) + q] = (float)g[q];
    }
    const size_t oGc = push(gc);
    const size_t oZero = push(std::vector<float>(512, 0.f));
    const size_t oHb0 = push(std::vector<float>((size_t)S * K, 0.f));
    const size_t oSkip0 = push(std::vector<float>((size_t)S * K, 0.f));
    // segments and terms
    std::vector<int> ints;
    int segoff[2] = {0, 0}, termoff[2] = {0, 0};
    std::vector<int4> segs[2];
    std::vector<int2> terms[2];
    for (int t = 0; t < 2; t++) {
        a->sym[t].sb[0] = 0;
        for (size_t q = 0; q < paths[t].size(); q++) {
            const int Lo = LOUT[t][q];
            for (size_t e = 0; e < paths[t][q].size(); e++)
                for (int c = 0; c < 2 * Lo + 1; c++) {
                    const int tb = (int)terms[t].size();
                    for (const Term &x : paths[t][q][e])
                        if (x.c == c) {
                            float cf = (float)x.coef;
                            int bits;
                            std::memcpy(&bits, &cf, 4);
                            terms[t].push_back(make_int2(x.a1 | (x.a2 << 5) | (x.a3 << 10), bits));
                        }
                    if ((int)terms[t].size() > tb) segs[t].push_back(make_int4((int)e, c, tb, (int)terms[t].size()));
                }
            a->sym[t].sb[q + 1] = (int)segs[t].size();
            a->sym[t].np[q] = (int)paths[t][q].size();
        }
        if (paths[t].size() < 2) a->sym[t].sb[2] = a->sym[t].sb[1];
    }
    for (int t = 0; t < 2; t++) {
        segoff[t] = (int)ints.size();
        for (const int4 &s : segs[t]) {
            ints.push_back(s.x);
            ints.push_back(s.y);
            ints.push_back(s.z);
            ints.push_back(s.w);
        }
        while (ints.size() % 64) ints.push_back(0);
        termoff[t] = (int)ints.size();
        for (const int2 &x : terms[t]) {
            ints.push_back(x.x);
            ints.push_back(x.y);
        }
        while (ints.size() % 64) ints.push_back(0);
    }
    float *dev = nullptr;
    int *idev = nullptr;
    if (hipMalloc(&dev, sizeof(float) * host.size()) != hipSuccess ||
        hipMalloc(&idev, sizeof(int) * ints.size()) != hipSuccess) {
        (void)hipGetLastError();
        if (dev) hipFree(dev);
        delete a;
        return fail(-2, "mace: weight allocation failed");
    }
    if (hipMemcpy(dev, host.data(), sizeof(float) * host.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(idev, ints.data(), sizeof(int) * ints.size(), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(dev);
        hipFree(idev);
        delete a;
        return fail(-5, "mace: weight copy failed");
    }
    a->dev = dev;
    a->sym_dev = idev;
    for (int t = 0; t < 2; t++) {
        a->sym[t].seg = reinterpret_cast<const int4 *>(idev + segoff[t]);
        a->sym[t].term = reinterpret_cast<const int2 *>(idev + termoff[t]);
        for (size_t q = 0; q < paths[t].size(); q++) {
            a->sym[t].W[q] = dev + oSymT[t][q];
            a->WoutT[t][q] = dev + oWoutT[t][q];
            a->Wout[t][q] = dev + oOut[t][q];
        }
    }
    for (int l2 = 0; l2 < 2; l2++) {
        a->WupT1[l2] = dev + oWupT1[l2];
        a->Wup1[l2] = dev + oUp[1][l2];
    }
    a->WscT1 = dev + oWscT1;
    a->Wsc1 = dev + oSc[1];
    a->zero = dev + oZero;
    a->Gc = dev + oGc;
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
        hipFree(idev);
        delete a;
        return fail(rc, "mace: weight packing failed");
    }
    m->mc = a;
    return 0;
}

void mace_destroy(mlp_model *m) {
    if (!m || !m->mc) return;
    if (m->mc->pk_dev) hipFree(m->mc->pk_dev);
    if (m->mc->sym_dev) hipFree(m->mc->sym_dev);
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
    float *X0 = base + L.X0, *Y = base + L.Y, *TT = base + L.TT, *GY = base + L.GY, *GX0 = base + L.GX0,
          *MSG = base + L.MSG, *H1 = base + L.H1, *HB1 = base + L.HB1, *H2 = base + L.H2, *GH1S = base + L.GH1S,
          *U = base + L.U;
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
    k_mc_edge<<<eg, 256, 0, s>>>(rowc, n, geom, a.NB, a.NBP, a.pe, a.rc, e1, a.Gc, X0, Y, TT);
    for (int t = 0; t < 2; t++) {
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
    na.Wup1[0] = a.Wup1[0];
    na.Wup1[1] = a.Wup1[1];
    na.WscT1 = a.WscT1;
    na.Wsc1 = a.Wsc1;
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
    for (int t = 0; t < 2; t++) {
        const int nd = t ? nd1 : nd0;
        if (nd <= 0) continue;
        const McBlk &AR = t ? AR1 : AR0, &AP = t ? AP1 : AP0;
        if (t == 0)
            k_mc_conv<0><<<nblk(nd, APB), 256, 0, s>>>(rowc, colc, nd, Y, TT, base + L.R[0], nullptr, zsp, a.hb0tab,
                                                       scale, AR);
        else
            k_mc_conv<1><<<nblk(nd, APB), 256, 0, s>>>(rowc, colc, nd, Y, TT, base + L.R[1], HB1, zsp, a.hb0tab,
                                                       scale, AR);
        for (int Lq = 0; Lq < 4; Lq++) {
            const int ld = cp_nL(Lq, NPt[t]) * MK;
            if ((rc = mgm(s, P, GE_STORE, AR.p[Lq], ld, a.waF[t][Lq], AP.p[Lq], MK, (long)nd * (2 * Lq + 1), nullptr)))
                return rc;
        }
        na.AP = AP;
        na.sym = a.sym[t];
        na.WoutT[0] = a.WoutT[t][0];
        na.WoutT[1] = a.WoutT[t][1];
        na.Wout[0] = a.Wout[t][0];
        na.Wout[1] = a.Wout[t][1];
        if (t == 0) k_mc_node<0><<<nblk(nd, APB), 256, 0, s>>>(nd, zsp, na);
        else k_mc_node<1><<<nblk(nd, APB), 256, 0, s>>>(nd, zsp, na);
    }
    HIP_TRY(hipGetLastError());
    if ((rc = launch_energy(s, U, perm, n, g->n_local, energy, atom_energy_user, n_seg, seg_dev))) return rc;
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
    if (nd1 > 0) {
        nb.AP = AP1;
        nb.sym = a.sym[1];
        nb.Wout[0] = a.Wout[1][0];
        nb.Wout[1] = a.Wout[1][0];
        k_mc_node1_bwd<<<nblk(nd1, APB), 256, 0, s>>>(nd1, zsp, nb);
        // dE/dA (before the W_A mix) over the A blocks
        for (int Lq = 0; Lq < 4; Lq++) {
            const int ld = cp_nL(Lq, 10) * MK;
            if ((rc = mgm(s, P, GE_STORE, GAP.p[Lq], MK, a.waA[1][Lq], AR1.p[Lq], ld, (long)nd1 * (2 * Lq + 1), nullptr)))
                return rc;
        }
        k_mc_conv1_bwd<<<nblk(nd1, APB), 256, 0, s>>>(rowc, colc, nd1, Y, TT, base + L.R[1], HB1, a.Gc, scale, AR1,
                                                      GY, MSG);
    }
    if (nd0 > 0) {
        nb.AP = AP0;
        nb.sym = a.sym[0];
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
