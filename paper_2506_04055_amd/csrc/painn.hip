// PaiNN energy and forces on the pruned neighbour graph.
//
// Per layer (Methods, "Graph Neural Networks": messages aggregated from the
// neighbours, then a node update; "Chosen Architectures": PaiNN), with the
// layer equations of the PaiNN paper the method cites:
//   phi_j = W2 silu(W1 s_j + b1) + b2
//   w_ij  = (A e(r_ij) + c) fc(r_ij),  e_k = sin(k pi r / rc) / r,
//           fc = (cos(pi r / rc) + 1) / 2
//   s_i  += sum_j (phi_j o w_ij)_s
//   v_i  += sum_j v_j o (phi_j o w_ij)_vv + rhat_ij (x) (phi_j o w_ij)_vs
//   Uv = U v, Vv = V v, n = sqrt(sum_d Vv_d^2 + eps)
//   a = W4 silu(W3 [s; n] + b3) + b4
//   v += a_vv o Uv,  s += a_sv o <Uv, Vv> + a_ss
// Readout U_i = w6 . silu(W5 s_i + b5) + b6; E = sum over local atoms in
// FP64 (Eq. 1).  Forces (Eq. 2) come from a hand-written adjoint: node
// gradients through transposed GEMMs, and per edge the geometric gradient
// G_e = dE/d(r_src - r_dst) with radial filters recomputed (never stored);
// F_k = sum_{e into k} G_e - sum_{e out of k} G_e, assembled by gathering
// through the reverse-edge index, so no floating-point atomics are used and
// results are bitwise reproducible.
#include "internal.h"
#include "gemm.h"
#include "msg.h"

#include <cmath>

namespace mlp {

static inline int nblk(long n, int t) { return (int)((n + t - 1) / t); }

__device__ __forceinline__ float sigmoidf_(float x) { return 1.0f / (1.0f + __expf(-x)); }
__device__ __forceinline__ float siluf_(float x) { return x * sigmoidf_(x); }
__device__ __forceinline__ float dsiluf_(float x) {
    float s = sigmoidf_(x);
    return s * (1.0f + x * (1.0f - s));
}

// ---------------------------------------------------------------------------
// Node GEMMs run on the matrix cores (gemm.hip).
// ---------------------------------------------------------------------------
enum { E_STORE = GE_STORE, E_BIAS = GE_BIAS, E_BIAS_SILU = GE_BIAS_SILU, E_DSILU = GE_DSILU, E_ADD = GE_ADD };

template <int EPI>
static void gemm(hipStream_t s, int prec, const float *A, int lda, const PackedW &B, float *C, int ldc, int M,
                 const float *bias = nullptr, float *C2 = nullptr, int ldc2 = 0, const float *R = nullptr,
                 int ldr = 0) {
    if (M <= 0) return;
    ProfScope ps(PK_GEMM, s);
    node_gemm(s, prec, EPI, A, lda, B, C, ldc, M, bias, C2, ldc2, R, ldr);
}

// A two-layer MLP (or its adjoint) as one chained GEMM kernel.
static void gemm2(hipStream_t s, int prec, const GemmChain &c) {
    if (c.M <= 0) return;
    ProfScope ps(PK_GEMM, s);
    node_gemm_chain(s, prec, c);
}

// phi = W2 silu(W1 s + b1) + b2 and a = W4 silu(W3 [s1; n] + b3) + b4, with
// the pre-activation h kept for the adjoint
static GemmChain mlp_fwd(const float *A, int lda, const PackedW &B1, float *h, int F, const float *b1,
                         const PackedW &B2, float *out, int ldo, const float *b2, int n) {
    GemmChain c;
    c.e1 = GE_BIAS_SILU;
    c.e2 = GE_BIAS;
    c.A = A;
    c.lda = lda;
    c.M = n;
    c.B1 = &B1;
    c.C1 = h;
    c.ldc1 = F;
    c.bias1 = b1;
    c.B2 = &B2;
    c.C2 = out;
    c.ldc2 = ldo;
    c.bias2 = b2;
    return c;
}

// the adjoint of such an MLP: dx = (silu'(h) * (dout W_out)) W_in (+ R2)
static GemmChain mlp_bwd(const float *gout, int ldg, const PackedW &B1, const float *h, int F, const PackedW &B2,
                         float *gx, int ldx, const float *R2, int n) {
    GemmChain c;
    c.e1 = GE_DSILU;
    c.e2 = R2 ? GE_ADD : GE_STORE;
    c.A = gout;
    c.lda = ldg;
    c.M = n;
    c.B1 = &B1;
    c.R1 = h;
    c.ldr1 = F;
    c.B2 = &B2;
    c.C2 = gx;
    c.ldc2 = ldx;
    c.R2 = R2;
    c.ldr2 = ldx;
    return c;
}

// ---------------------------------------------------------------------------
// Elementwise node kernels
// ---------------------------------------------------------------------------

// p[0 .. count) = 0.
__global__ void k_fill_zero(float *__restrict__ p, long count) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < count) p[t] = 0.f;
}

static void fill_zero(hipStream_t s, float *p, long count) {
    if (count > 0) k_fill_zero<<<nblk(count, 256), 256, 0, s>>>(p, count);
}

// UV holds rows [Uv | Vv] of 2F for each (atom, direction): Uv(i, d, f) at
// UV[(3 i + d) 2F + f], Vv(i, d, f) at UV[(3 i + d) 2F + F + f]; gUV likewise.
__global__ void k_norm(const float *__restrict__ UV, int n, int F, float eps, float *__restrict__ sn) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * F) return;
    long i = idx / F;
    int f = idx % F;
    const float *q = UV + i * 6 * F + F;
    float x = eps;
    for (int d = 0; d < 3; d++) x = fmaf(q[d * 2 * F + f], q[d * 2 * F + f], x);
    sn[i * 2 * F + F + f] = sqrtf(x);
}

__global__ void k_update_out(const float *__restrict__ sn, const float *__restrict__ v1,
                             const float *__restrict__ UV, const float *__restrict__ a, int n, int F,
                             float *__restrict__ s2, float *__restrict__ v2) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * F) return;
    long i = idx / F;
    int f = idx % F;
    const long b3 = i * 3 * F, u6 = i * 6 * F;
    float sp = 0.f;
    float avv = a[b3 + f], asv = a[b3 + F + f], ass = a[b3 + 2 * F + f];
    for (int d = 0; d < 3; d++) {
        float u = UV[u6 + d * 2 * F + f];
        sp = fmaf(u, UV[u6 + d * 2 * F + F + f], sp);
        v2[b3 + d * F + f] = fmaf(avv, u, v1[b3 + d * F + f]);
    }
    s2[idx] = fmaf(asv, sp, sn[i * 2 * F + f] + ass);
}

// Adjoint of the gated update (first part): da, dUv and the direct part of dVv.
// gv2 == nullptr stands for dE/dv2 = 0 (the last layer: the readout sees s only).
__global__ void k_update_bwd1(const float *__restrict__ gs2, const float *__restrict__ gv2,
                              const float *__restrict__ UV, const float *__restrict__ a, int n, int F,
                              float *__restrict__ ga, float *__restrict__ gUV) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * F) return;
    long i = idx / F;
    int f = idx % F;
    const long b3 = i * 3 * F, u6 = i * 6 * F;
    float g = gs2[idx];
    float avv = a[b3 + f], asv = a[b3 + F + f];
    float sp = 0.f, gavv = 0.f;
    for (int d = 0; d < 3; d++) {
        float u = UV[u6 + d * 2 * F + f], w = UV[u6 + d * 2 * F + F + f], gv = gv2 ? gv2[b3 + d * F + f] : 0.f;
        sp = fmaf(u, w, sp);
        gavv = fmaf(gv, u, gavv);
        gUV[u6 + d * 2 * F + f] = gv * avv + g * asv * w;
        gUV[u6 + d * 2 * F + F + f] = g * asv * u;
    }
    ga[b3 + f] = gavv;
    ga[b3 + F + f] = g * sp;
    ga[b3 + 2 * F + f] = g;
}

// Adjoint of the gated update (second part): the norm's share of dVv and the
// residual into ds1.
__global__ void k_update_bwd2(const float *__restrict__ gsn, const float *__restrict__ sn,
                              const float *__restrict__ UV, const float *__restrict__ gs2, int n, int F,
                              float *__restrict__ gUV, float *__restrict__ gs1) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * F) return;
    long i = idx / F;
    int f = idx % F;
    const long u6 = i * 6 * F + F;
    float gn = gsn[i * 2 * F + F + f] / sn[i * 2 * F + F + f];
    for (int d = 0; d < 3; d++)
        gUV[u6 + d * 2 * F + f] = fmaf(gn, UV[u6 + d * 2 * F + f], gUV[u6 + d * 2 * F + f]);
    gs1[idx] = gs2[idx] + gsn[i * 2 * F + f];
}

// Readout: U_i, and the gradient seed dE/dh5 = w6 o silu'(h5) on local atoms.
// Sum over the 16 lanes of a DPP row.
__device__ __forceinline__ float row16_sum(float x) {
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x128, 0xF, 0xF, false));   // row_ror:8
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x124, 0xF, 0xF, false));   // row_ror:4
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0x4E, 0xF, 0xF, false));    // quad [2,3,0,1]
    x += __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), 0xB1, 0xF, 0xF, false));    // quad [1,0,3,2]
    return x;
}

// Readout U_i = b6 + sum_h w6[h] silu(h5[i][h]) and its gradient
// g5 = w6 * silu'(h5) (zero for ghost rows), sixteen lanes per atom: lane q
// takes features 4q .. 4q+3 (+ 64 per round) and the row sum gives U_i.
__global__ void k_readout(const float *__restrict__ h5, int n, int Fh, const float *__restrict__ w6,
                          const float *__restrict__ b6, const int *__restrict__ perm, int n_local,
                          float *__restrict__ U, float *__restrict__ g5) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int i = (int)(t >> 4), q = (int)(t & 15);
    float u = 0.f;
    if (i < n) {
        const bool local = perm[i] < n_local;
        for (int h = 4 * q; h < Fh; h += 64) {
            const float4 x = *reinterpret_cast<const float4 *>(h5 + (long)i * Fh + h);
            const float4 w = *reinterpret_cast<const float4 *>(w6 + h);
            u = fmaf(w.x, siluf_(x.x), fmaf(w.y, siluf_(x.y), fmaf(w.z, siluf_(x.z), fmaf(w.w, siluf_(x.w), u))));
            float4 gg = make_float4(0.f, 0.f, 0.f, 0.f);
            if (local) gg = make_float4(w.x * dsiluf_(x.x), w.y * dsiluf_(x.y), w.z * dsiluf_(x.z), w.w * dsiluf_(x.w));
            *reinterpret_cast<float4 *>(g5 + (long)i * Fh + h) = gg;
        }
    }
    u = row16_sum(u);
    if (q == 0 && i < n) U[i] = u + b6[0];
}

constexpr int ERED = 512;      // threads per block of the energy sums
constexpr int ECH = 16384;     // rows per chunk of a segment

// E_b = sum of U_i over the local atoms of segment b (internal rows
// [seg[b], seg[b+1]), or [0, n) without segments), in FP64 with a fixed
// order that depends on the segment alone: the segment is cut into chunks of
// ECH rows from its first row; block (b, c) sums chunk c (strided partial
// sums, a butterfly within each wave, then the wave totals in order) into
// part[o_b + c], o_b = b + seg[b] / ECH (disjoint: segment b has
// ceil(len / ECH) <= 1 + len / ECH chunks); k_energy_total adds the chunk
// sums of each segment in order.  A segment's energy is therefore the same
// whether it is evaluated alone or packed into a batch.
__global__ void __launch_bounds__(ERED) k_energy_chunk(const float *__restrict__ U, const int *__restrict__ perm,
                                                       const int *__restrict__ seg, int n, int n_local,
                                                       double *__restrict__ part) {
    __shared__ double sh[ERED / 64];
    const int b = blockIdx.x, c = blockIdx.y;
    const int a = seg ? seg[b] : 0, e = seg ? seg[b + 1] : n;
    const int ca = a + c * ECH;
    if (ca >= e && !(c == 0 && a == e)) return;   // past the segment (an empty one keeps chunk 0)
    const int ce = min(ca + ECH, e);
    // eight interleaved partial sums per thread; the row's energy and its
    // local flag are loaded together, so eight pairs of loads are in flight
    double acc[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i0 = ca + threadIdx.x; i0 < ce; i0 += 8 * ERED) {
        float u[8];
        int pm[8];
#pragma unroll
        for (int q = 0; q < 8; q++) {
            const int i = i0 + q * ERED;
            u[q] = i < ce ? U[i] : 0.f;
            pm[q] = i < ce ? perm[i] : n_local;
        }
#pragma unroll
        for (int q = 0; q < 8; q++)
            if (pm[q] < n_local) acc[q] += (double)u[q];
    }
    double x = ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
    // butterfly within each wave, then the waves' totals in wave order
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < ERED / 64; w++) t += sh[w];
        part[b + a / ECH + c] = t;
    }
}
__global__ void k_energy_total(const int *__restrict__ seg, int n, int n_seg, const double *__restrict__ part,
                               double *__restrict__ E) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_seg) return;
    const int a = seg ? seg[b] : 0, e = seg ? seg[b + 1] : n;
    const int nc = e > a ? (e - a + ECH - 1) / ECH : 1;
    const double *p = part + b + a / ECH;
    double t = 0.0;
    for (int c = 0; c < nc; c++) t += p[c];
    E[b] = t;
}

// F_k = sum over in-edges e of (G at rev(e)) - (G at e), scattered to the
// caller's atom order (SoA).
// Sixteen lanes per atom (one DPP row): lane q takes the atom's edges
// q, q + 16, ..., and the row sum gives the force.
__global__ void k_forces(const int *__restrict__ rowc, const int *__restrict__ revc,
                         const float4 *__restrict__ Gout, const int *__restrict__ perm, int n,
                         float *__restrict__ F) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int k = (int)(t >> 4), q = (int)(t & 15);
    float fx = 0.f, fy = 0.f, fz = 0.f;
    if (k < n) {
        for (int e = rowc[k] + q; e < rowc[k + 1]; e += 16) {
            const int re = revc[e];
            if (re < 0) continue;  // cannot happen for a symmetric graph; never index with it
            const float4 a = Gout[re], b = Gout[e];
            fx += a.x - b.x;
            fy += a.y - b.y;
            fz += a.z - b.z;
        }
    }
    // every lane of the wave takes part in the row sums (n need not fill the grid)
    fx = row16_sum(fx);
    fy = row16_sum(fy);
    fz = row16_sum(fz);
    if (k < n && q == 0) {
        const int u = perm[k];
        F[u] = fx;
        F[(long)n + u] = fy;
        F[2 * (long)n + u] = fz;
    }
}

__global__ void k_scatter_energy(const float *__restrict__ U, const int *__restrict__ perm, int n,
                                 float *__restrict__ out) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) out[perm[k]] = U[k];
}

// ---------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------
struct Act {
    float *s[MLP_MAX_LAYERS + 1], *v[MLP_MAX_LAYERS + 1];
    float *h1[MLP_MAX_LAYERS], *phi[MLP_MAX_LAYERS], *sn[MLP_MAX_LAYERS], *v1[MLP_MAX_LAYERS],
        *UV[MLP_MAX_LAYERS], *h3[MLP_MAX_LAYERS], *a[MLP_MAX_LAYERS];
    float *gs, *gv, *gs1, *gv1, *gphi, *ga, *gsn, *gUV, *h5, *g5, *U;
    float *u;   // v * phi_vv of the current forward layer (shares gUV: the adjoint starts after the forward)
    double *epart;
    int *queue;   // the message launches' atom counters, MSG_QUEUE_INTS per launch
};
constexpr long QUEUE_INTS = 2L * MLP_MAX_LAYERS * MSG_QUEUE_INTS;

// The update and the norm (and their adjoint) are fused into the chained
// GEMMs for these widths; other widths take the elementwise kernels, whose
// work arrays (da, d[s1 | n]) the fused path does not need.
static bool update_fused(int F) { return F == 64 || F == 128; }

// Columns of the saved gate a of a layer: [a_vv | a_sv] when the update is
// fused (a_ss is consumed in the epilogue that forms it), else all three.
static int a_cols(int F) { return update_fused(F) ? 2 * F : 3 * F; }

int layer_work_per_feature(int F) {
    // s 1, v 3, h1 1, phi 3, [s1 | n] 2, v1 3, [Uv | Vv] 6, h3 1, a
    return 20 + a_cols(F) / F;
}

int adjoint_work_per_feature(int F) {
    // gs 1, gv 3, gs1 1, gv1 3, gphi 3, gUV 6, h5 + g5 1; da 3 and
    // d[s1 | n] 2 for the elementwise update adjoint
    return 18 + (update_fused(F) ? 0 : 5);
}

static size_t act_floats(long N, int F, int T) {
    long per_layer = (long)N * F * layer_work_per_feature(F);
    long io = (long)N * F * 4;  // s, v of the final layer
    long bwd = (long)N * F * adjoint_work_per_feature(F);
    return (size_t)(T * per_layer + io + bwd + N + 64 * (12 * T + 32) + 4096 + QUEUE_INTS +
                    2 * energy_part_doubles(N));
}

static void carve(float *base, long N, int F, int T, Act &A) {
    float *p = base;
    auto take = [&](long cnt) {
        float *r = p;
        p += (cnt + 63) & ~63L;
        return r;
    };
    const long NF = N * F;
    for (int t = 0; t <= T; t++) {
        A.s[t] = take(NF);
        A.v[t] = take(3 * NF);
        if (t == T) break;
        A.h1[t] = take(NF);
        A.phi[t] = take(3 * NF);
        A.sn[t] = take(2 * NF);
        A.v1[t] = take(3 * NF);
        A.UV[t] = take(6 * NF);
        A.h3[t] = take(NF);
        A.a[t] = take((long)a_cols(F) * N);
    }
    A.gs = take(NF);
    A.gv = take(3 * NF);
    A.gs1 = take(NF);
    A.gv1 = take(3 * NF);
    A.gphi = take(3 * NF);
    A.ga = update_fused(F) ? nullptr : take(3 * NF);
    A.gsn = update_fused(F) ? nullptr : take(2 * NF);
    A.gUV = take(6 * NF);
    A.u = A.gUV;
    A.h5 = take(NF / 2 + 64);
    A.g5 = take(NF / 2 + 64);
    A.U = take(N + 64);
    A.epart = reinterpret_cast<double *>(take(2 * energy_part_doubles(N)));
    A.queue = reinterpret_cast<int *>(take(QUEUE_INTS));
}

static MsgArgs msg_args(mlp_nbr *g, mlp_model *m, const LayerW &L, int hop_max) {
    MsgArgs a = {};
    a.rowc = g->rowc.as<int>();
    a.colc = g->colc.as<int>();
    a.geom = g->geom.as<float4>();
    a.n = g->n_atoms;
    a.A = L.A;
    a.c = L.c;
    a.rc = m->rc;
    a.hop = g->hop.as<int8_t>();
    a.hop_max = hop_max;
    a.S = g->Gs.as<float4>();
    a.s_stride = g->n_edges_skin;
    a.species = g->species.as<int>();
    return a;
}

struct L0Layout {
    int ldp, ldr, ldq;
};
static L0Layout l0_layout(int F, int K, int S) {
    const int CS = S * l0_block(K);
    L0Layout l;
    l.ldp = (CS + S + 3) / 4 * 4;
    l.ldr = CS;
    l.ldq = CS;
    (void)F;
    return l;
}

static L0Args l0_args(mlp_nbr *g, mlp_model *m, int hop_max) {
    L0Args a = {};
    a.rowc = g->rowc.as<int>();
    a.colc = g->colc.as<int>();
    a.revc = g->revc.as<int>();
    a.geom = g->geom.as<float4>();
    a.n = g->n_atoms;
    a.rc = m->rc;
    a.hop = g->hop.as<int8_t>();
    a.hop_max = hop_max;
    a.species = g->species.as<int>();
    return a;
}

int first_layer_table(mlp_model *m, hipStream_t s, float *tmp) {
    const int F = m->F, S = m->S;
    const int P = node_operands(m->precision);
    const LayerW L = m->layer(0);
    // the same GEMMs as the later layers' node MLPs, on the S embedding rows
    node_gemm(s, P, GE_BIAS_SILU, m->at(m->off_emb), F, m->pk[0][WP_W1], tmp, F, S, L.b1, tmp + (long)S * F, F);
    node_gemm(s, P, GE_BIAS, tmp + (long)S * F, F, m->pk[0][WP_W2], m->phi0_dev, 3 * F, S, L.b2);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

// Species-scaled first-layer filter weights (CS = S SB columns of basis
// slots, one block of SB = l0_block(K) per species, zero past slot K):
// Wfs[f][z SB + k] = phi_s(z)_f A'_s[f][k] followed by the embedding columns
// Wfs[f][CS + z] = emb[z][f]; Wbs the same without the embedding;
// Wv[f][z SB + k] = phi_vs(z)_f A'_vs[f][k]; A'[.][0] = c.
__global__ void k_l0_weights(const float *__restrict__ A, const float *__restrict__ c,
                             const float *__restrict__ phi0, const float *__restrict__ emb, int F, int K, int S,
                             float *__restrict__ Wfs, float *__restrict__ Wbs, float *__restrict__ Wv) {
    const int SB = l0_block(K), CS = S * SB;
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < (long)F * CS) {
        const int f = (int)(idx / CS), col = (int)(idx % CS), z = col / SB, k = col % SB;
        float ws = 0.f, wv = 0.f;
        if (k <= K) {
            const float as = k == 0 ? c[F + f] : A[(long)(F + f) * K + k - 1];
            const float av = k == 0 ? c[2 * F + f] : A[(long)(2 * F + f) * K + k - 1];
            ws = phi0[(long)z * 3 * F + F + f] * as;
            wv = phi0[(long)z * 3 * F + 2 * F + f] * av;
        }
        Wfs[(long)f * (CS + S) + col] = ws;
        Wbs[(long)f * CS + col] = ws;
        Wv[(long)f * CS + col] = wv;
    } else if (idx < (long)F * CS + (long)F * S) {
        const long r = idx - (long)F * CS;
        const int f = (int)(r / S), z = (int)(r % S);
        Wfs[(long)f * (CS + S) + CS + z] = emb[(long)z * F + f];
    }
}

int first_layer_factor(mlp_model *m) {
    m->l0f = false;
    const int F = m->F, K = m->K, S = m->S, CS = S * l0_block(K);
    if (!l0_factorised(K, S)) return 0;
    // P and R (forward), Q_s and Q_v (adjoint) must fit the 6 F floats per
    // atom of the dUV rows they borrow
    const L0Layout l0 = l0_layout(F, K, S);
    if (l0.ldp + 3 * l0.ldr > 6 * F || 4 * l0.ldq > 6 * F) return 0;
    const LayerW L = m->layer(0);
    float *src = nullptr;
    const size_t nfs = (size_t)F * (CS + S), nb = (size_t)F * CS;
    if (hipMalloc(&src, sizeof(float) * (nfs + 2 * nb)) != hipSuccess) {
        (void)hipGetLastError();
        return fail(-2, "first-layer weight allocation failed");
    }
    float *Wfs = src, *Wbs = src + nfs, *Wv = Wbs + nb;
    const long tot = (long)F * CS + (long)F * S;
    k_l0_weights<<<nblk(tot, 256), 256>>>(L.A, L.c, m->phi0_dev, m->at(m->off_emb), F, K, S, Wfs, Wbs, Wv);
    const float *Ws[4] = {Wfs, Wv, Wbs, Wv};
    const int C[4] = {CS + S, CS, CS, CS};
    const bool tr[4] = {false, false, true, true};
    size_t bytes = 0;
    for (int q = 0; q < 4; q++) bytes += packed_bytes(F, C[q], tr[q]);
    int rc = hipMalloc(&m->pk_l0_dev, bytes) == hipSuccess ? 0 : -2;
    for (size_t q = 0, o = 0; rc == 0 && q < 4; q++) {
        if (pack_weight(nullptr, Ws[q], F, C[q], tr[q], (char *)m->pk_l0_dev + o, &m->pk_l0[q])) rc = -5;
        o += packed_bytes(F, C[q], tr[q]);
    }
    if (hipDeviceSynchronize() != hipSuccess && rc == 0) rc = -5;
    hipFree(src);
    if (rc) {
        (void)hipGetLastError();
        if (m->pk_l0_dev) hipFree(m->pk_l0_dev);
        m->pk_l0_dev = nullptr;
        return fail(rc, "first-layer weight packing failed");
    }
    m->l0f = true;
    return 0;
}

void eval_model_needs(const mlp_model *m, const mlp_nbr *g, size_t *act, size_t *G, size_t *Gs) {
    const size_t ne = (size_t)g->n_edges_skin;
    if (m->al || m->mc) {
        *act = m->al ? allegro_arena_bytes(m, g->n_atoms, (long)ne) : mace_arena_bytes(m, g->n_atoms, (long)ne);
        *G = sizeof(float4) * ne + 64;
        *Gs = 64;
        return;
    }
    *act = act_floats(g->n_atoms, m->F, m->T) * sizeof(float);
    *G = sizeof(float4) * ne + 64;
    *Gs = sizeof(float4) * ne * (size_t)msg_slots(m->F, m->T, m->l0f) + 64;
}

int launch_energy(hipStream_t s, const float *U, const int *perm, int n, int n_local, double *energy,
                  float *atom_energy_user, int n_seg, const int *seg_dev, double *part) {
    const int ns = std::max(1, n_seg);
    const dim3 grid((unsigned)ns, (unsigned)std::max(1, (n + ECH - 1) / ECH));
    k_energy_chunk<<<grid, ERED, 0, s>>>(U, perm, seg_dev, n, n_local, part);
    k_energy_total<<<(unsigned)((ns + 63) / 64), 64, 0, s>>>(seg_dev, n, ns, part, energy);
    if (atom_energy_user) k_scatter_energy<<<nblk(n, 256), 256, 0, s>>>(U, perm, n, atom_energy_user);
    HIP_TRY(hipGetLastError());
    return 0;
}

int launch_forces(hipStream_t s, const int *rowc, const int *revc, const float4 *G, const int *perm, int n,
                  float *forces_user) {
    k_forces<<<nblk(16L * n, 256), 256, 0, s>>>(rowc, revc, G, perm, n, forces_user);
    HIP_TRY(hipGetLastError());
    return 0;
}

int evaluate(mlp_model *m, mlp_nbr *g, hipStream_t s, double *energy, float *forces_user,
             float *atom_energy_user, int n_seg, const int *seg_dev) {
    if (m->al) return allegro_evaluate(m, g, s, energy, forces_user, atom_energy_user, n_seg, seg_dev);
    if (m->mc) return mace_evaluate(m, g, s, energy, forces_user, atom_energy_user, n_seg, seg_dev);
    const int n = g->n_atoms, F = m->F, K = m->K, T = m->T, F3 = 3 * F, Fh = F / 2;
    // MFMA operand forms of the mode for the node GEMMs (P) and for the
    // radial filter (PF): 0 FP32, 1 plain bfloat16, 2 split bfloat16 (hi + lo)
    const int P = node_operands(m->precision);
    const int PF = filter_operands(m->precision);
    int *Gr = &g->n_grows;
    int rc;
    size_t need_act, need_G, need_Gs;
    eval_model_needs(m, g, &need_act, &need_G, &need_Gs);
    if ((rc = g->act.ensure(need_act, 1.2, Gr))) return rc;
    const long ne = g->n_edges_skin;
    if ((rc = g->G.ensure(need_G, 1.2, Gr))) return rc;
    if ((rc = g->Gs.ensure(need_Gs, 1.2, Gr))) return rc;
    Act A;
    carve(g->act.as<float>(), n, F, T, A);
    // every message launch takes its own zeroed atom counters
    fill_zero(s, reinterpret_cast<float *>(A.queue), QUEUE_INTS);
    int nq = 0;
    auto next_queue = [&]() { return A.queue + (long)(nq++) * MSG_QUEUE_INTS; };
    const int *perm = g->perm.as<int>();
    // edge-sum slots: layers 1 .. T-1 take one each, from slot 0; the first
    // layer's come last (one when it is factorised, else one per pass)
    const int slot0 = T - 1, nslot = msg_slots(F, T, m->l0f);
    // factorised first layer: its matrices live in the adjoint's dUV rows
    // (free in the first layer's forward, and again once dv1 is formed)
    const L0Layout l0 = l0_layout(F, K, m->S);

    // Per-layer active sets (Results, "Distributed potential computation",
    // pruning): layer t's outputs are needed within T - 1 - t hops of the
    // locals and its message MLP within T - t hops.  With ghosts the internal
    // order is hop-major (the neighbour build), so those sets are the row
    // prefixes NH(h) and every node kernel runs on its prefix; the message
    // kernels skip atoms by the exact hop marks of this evaluation, which the
    // prefixes contain.  Rows past a prefix hold values that no needed row
    // reads, except the gradients a message adjoint gathers from its
    // destinations: those rows are zeroed (their gradient is zero).
    const bool ho = g->nhop[0] > 0 && g->nhop[std::min(T + 1, MLP_MAX_LAYERS + 1)] == n;
    auto NH = [&](int h) { return ho ? g->nhop[std::max(0, std::min(h, T + 1))] : n; };

    // forward
    for (int t = 0; t < T; t++) {
        LayerW L = m->layer(t);
        const int hop_dst = T - 1 - t;
        const int nsrc = NH(T - t), ndst = NH(T - 1 - t);
        if (t > 0) {
            // phi, and u = v * phi_vv in the same epilogue: the rows the
            // message pass gathers together with phi_s and phi_vs
            GemmChain c = mlp_fwd(A.s[t], F, m->pk[t][WP_W1], A.h1[t], F, L.b1, m->pk[t][WP_W2], A.phi[t], F3, L.b2,
                                  nsrc);
            c.e2 = GE_BIAS_VPROD;
            c.F = F;
            c.v1 = A.v[t];
            c.v2 = A.u;
            gemm2(s, P, c);
        }
        if (t == 0 && m->l0f) {
            // factorised first layer: basis sums per atom and species, then
            // s1 = [P | one-hot] Wfs^T (s0 included) and v1 = R Wv^T
            L0Args la = l0_args(g, m, hop_dst);
            la.P = A.gUV;
            la.R = A.gUV + (long)n * l0.ldp;
            la.ldp = l0.ldp;
            la.ldr = l0.ldr;
            if ((rc = msg_l0_basis_sums(s, K, m->S, la))) return fail(rc, "first-layer kernel launch failed");
            gemm<E_STORE>(s, P, la.P, l0.ldp, m->pk_l0[0], A.sn[0], 2 * F, ndst);
            gemm<E_STORE>(s, P, la.R, l0.ldr, m->pk_l0[1], A.v1[0], F, 3 * ndst);
        } else {
            MsgArgs ma = msg_args(g, m, L, hop_dst);
            ma.layer0 = t == 0;
            // the first layer reads phi and s from the per-species tables
            ma.phi = t == 0 ? m->phi0_dev : A.phi[t];
            ma.u = A.u;
            ma.s = t == 0 ? m->at(m->off_emb) : A.s[t];
            ma.v = A.v[t];
            ma.sn = A.sn[t];
            ma.v1 = A.v1[t];
            ma.queue = next_queue();
            ProfScope ps(PK_MSG_FWD, s);
            if ((rc = msg_forward(s, PF, F, K, ma))) return fail(rc, "message kernel launch failed");
        }
        gemm<E_STORE>(s, P, A.v1[t], F, m->pk[t][WP_UV], A.UV[t], 2 * F, 3 * ndst);
        // n = sqrt(eps + sum_d Vv_d^2): formed where it is used when F is 64
        // or 128 (the update's operand load and the adjoint's epilogue)
        const bool nfused = update_fused(F);
        if (!nfused) k_norm<<<nblk((long)ndst * F, 256), 256, 0, s>>>(A.UV[t], ndst, F, m->eps, A.sn[t]);
        {
            GemmChain c = mlp_fwd(A.sn[t], 2 * F, m->pk[t][WP_W3], A.h3[t], F, L.b3, m->pk[t][WP_W4], A.a[t],
                                  a_cols(F), L.b4, ndst);
            if (F >= 64) {
                // the gated update in the second product's epilogue (the last
                // layer's v is not needed: the readout takes s only)
                c.e2 = nfused ? GE_UPDATE_N : GE_UPDATE;
                c.eps = m->eps;
                c.F = F;
                c.sn = A.sn[t];
                c.v1 = A.v1[t];
                c.UV = A.UV[t];
                c.s2 = A.s[t + 1];
                c.v2 = t == T - 1 ? nullptr : A.v[t + 1];
                gemm2(s, P, c);
            } else {
                gemm2(s, P, c);
                k_update_out<<<nblk((long)ndst * F, 256), 256, 0, s>>>(A.sn[t], A.v1[t], A.UV[t], A.a[t], ndst, F,
                                                                        A.s[t + 1], A.v[t + 1]);
            }
        }
    }
    // readout and energy (the locals are the prefix NH(0); U of the other
    // rows, reported to the caller as per-atom energies, is zero)
    const int nloc = NH(0);
    gemm<E_BIAS>(s, P, A.s[T], F, m->pk_W5, A.h5, Fh, nloc, m->at(m->off_b5));
    k_readout<<<nblk(16L * nloc, 256), 256, 0, s>>>(A.h5, nloc, Fh, m->at(m->off_w6), m->at(m->off_b6), perm,
                                                    g->n_local, A.U, A.g5);
    fill_zero(s, A.U + nloc, (long)(n - nloc));
    if ((rc = launch_energy(s, A.U, perm, n, g->n_local, energy, nullptr, n_seg, seg_dev, A.epart))) return rc;
    if (atom_energy_user) k_scatter_energy<<<nblk(n, 256), 256, 0, s>>>(A.U, perm, n, atom_energy_user);
    if (!forces_user) return 0;

    // adjoint
    gemm<E_STORE>(s, P, A.g5, Fh, m->pk_W5t, A.gs, F, nloc);
    for (int t = T - 1; t >= 0; t--) {
        LayerW L = m->layer(t);
        const int hop_src = T - t;
        const bool last = t == T - 1;   // dE/dv of the last layer's output is zero
        const int ndst = NH(T - 1 - t), nsrc = NH(T - t), nfar = NH(T - t + 1);
        if (update_fused(F)) {
            // one kernel: da (and dUv) formed from ds2, dv2, UV and a as the
            // first product's operand is loaded, then d[s1 | n] -> ds1 = ds2 +
            // d s1 and dVv in the epilogue
            GemmChain c = mlp_bwd(A.a[t], a_cols(F), m->pk[t][WP_W4TP], A.h3[t], F, m->pk[t][WP_W3T], A.gs1, F, A.gs,
                                  ndst);
            c.e2 = GE_UPDATE_ADJ;
            c.F = F;
            c.sn = A.sn[t];
            c.UV = A.UV[t];
            c.gUV = A.gUV;
            c.gv = last ? nullptr : A.gv;
            c.eps = m->eps;
            gemm2(s, P, c);
        } else {
            k_update_bwd1<<<nblk((long)ndst * F, 256), 256, 0, s>>>(A.gs, last ? nullptr : A.gv, A.UV[t], A.a[t],
                                                                    ndst, F, A.ga, A.gUV);
            gemm2(s, P, mlp_bwd(A.ga, F3, m->pk[t][WP_W4T], A.h3[t], F, m->pk[t][WP_W3T], A.gsn, 2 * F, nullptr,
                                ndst));
            k_update_bwd2<<<nblk((long)ndst * F, 256), 256, 0, s>>>(A.gsn, A.sn[t], A.UV[t], A.gs, ndst, F, A.gUV,
                                                                    A.gs1);
        }
        // dv1 = [dUv | dVv] [U; V] + dv2 (the residual)
        if (last) gemm<E_STORE>(s, P, A.gUV, 2 * F, m->pk[t][WP_UVT], A.gv1, F, 3 * ndst);
        else gemm<E_ADD>(s, P, A.gUV, 2 * F, m->pk[t][WP_UVT], A.gv1, F, 3 * ndst, nullptr, nullptr, 0, A.gv, F);
        // destinations past this layer's set carry no gradient; the message
        // adjoint gathers them up to one hop beyond its sources
        fill_zero(s, A.gs1 + (long)ndst * F, (long)(nfar - ndst) * F);
        fill_zero(s, A.gv1 + 3L * ndst * F, 3L * (nfar - ndst) * F);
        if (t == 0 && m->l0f) {
            // factorised first layer: Q_s = gs1 Wbs, Q_v = gv1 Wv, then the
            // edge sums from Q in one slot.  The edge kernel reads Q of every
            // destination of a live source (one hop past the sources), so Q
            // covers the rows through nfar (zero past ndst, as gs1 and gv1).
            L0Args la = l0_args(g, m, hop_src);
            float *Qs = A.gUV, *Qv = A.gUV + (long)n * l0.ldq;
            gemm<E_STORE>(s, P, A.gs1, F, m->pk_l0[2], Qs, l0.ldq, nfar);
            gemm<E_STORE>(s, P, A.gv1, F, m->pk_l0[3], Qv, l0.ldq, 3 * nfar);
            la.Qs = Qs;
            la.Qv = Qv;
            la.ldq = l0.ldq;
            la.S = g->Gs.as<float4>() + (size_t)slot0 * ne;
            if ((rc = msg_l0_edge_sums(s, K, m->S, la))) return fail(rc, "first-layer adjoint kernel launch failed");
        } else {
            MsgArgs ma = msg_args(g, m, L, hop_src);
            ma.phi = t == 0 ? m->phi0_dev : A.phi[t];
            ma.v = A.v[t];
            ma.gs1 = A.gs1;
            ma.gv1 = A.gv1;
            ma.gv_in = A.gv;
            ma.gphi = A.gphi;
            ma.S = g->Gs.as<float4>() + (size_t)(t == 0 ? slot0 : t - 1) * ne;
            ma.layer0 = t == 0;
            ma.queue = next_queue();
            ProfScope ps(PK_MSG_BWD, s);
            if ((rc = msg_adjoint(s, PF, F, K, ma))) return fail(rc, "adjoint message kernel launch failed");
        }
        if (t == 0) break;   // the embedding carries no gradient
        gemm2(s, P, mlp_bwd(A.gphi, F3, m->pk[t][WP_W2T], A.h1[t], F, m->pk[t][WP_W1T], A.gs, F, A.gs1, nsrc));
    }
    if ((rc = msg_assemble_G(s, g->rowc.as<int>(), n, ne, g->geom.as<float4>(), g->Gs.as<float4>(), ne, nslot,
                             g->G.as<float4>())))
        return fail(rc, "edge-gradient kernel launch failed");
    k_forces<<<nblk(16L * n, 256), 256, 0, s>>>(g->rowc.as<int>(), g->revc.as<int>(), g->G.as<float4>(), perm, n,
                                                forces_user);
    HIP_TRY(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------------------------
// Velocity Verlet (SoA, A/fs, amu, eV/A)
// ---------------------------------------------------------------------------
constexpr float ACC = 9.648533212e-3f;  // (eV / A / amu) -> A / fs^2

__global__ void k_kick_drift(float *__restrict__ x, float *__restrict__ v, const float *__restrict__ f,
                             const float *__restrict__ im, int n, float L0, float L1, float L2, float dt) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 3L * n) return;
    int d = idx / n;
    long u = idx % n;
    float vv = fmaf(0.5f * dt * ACC * im[u], f[idx], v[idx]);
    v[idx] = vv;
    float L = d == 0 ? L0 : (d == 1 ? L1 : L2);
    float p = fmaf(dt, vv, x[idx]);
    if (L > 0.f) {
        p = p - L * floorf(p / L);
        if (p >= L) p -= L;
        if (p < 0.f) p += L;
    }
    x[idx] = p;
}

__global__ void k_kick(float *__restrict__ v, const float *__restrict__ f, const float *__restrict__ im, int n,
                       float dt) {
    long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= 3L * n) return;
    long u = idx % n;
    v[idx] = fmaf(0.5f * dt * ACC * im[u], f[idx], v[idx]);
}

int verlet_kick_drift(float *pos, float *vel, const float *forces, const float *inv_mass, int n,
                      const double box[3], float dt, hipStream_t s) {
    k_kick_drift<<<nblk(3L * n, 256), 256, 0, s>>>(pos, vel, forces, inv_mass, n, (float)box[0], (float)box[1],
                                                   (float)box[2], dt);
    HIP_TRY(hipGetLastError());
    return 0;
}

int verlet_kick(float *vel, const float *forces, const float *inv_mass, int n, float dt, hipStream_t s) {
    k_kick<<<nblk(3L * n, 256), 256, 0, s>>>(vel, forces, inv_mass, n, dt);
    HIP_TRY(hipGetLastError());
    return 0;
}

}  // namespace mlp
