// Message pass and its adjoint with the radial-filter contraction on MFMA.
//
// Per directed edge (i <- j) the filter is w = A' e~(r), a dense K+1 -> 3F
// contraction with A' = [c | A] and e~ = [fc, e_1 fc, ..., e_K fc],
// e_k = sin(k pi r / rc) / r.  A wave owns one atom; its edges are taken 16
// at a time and each 16 x 16 MFMA tile computes w for 16 features x 16 edges:
//   A operand = A' rows of 16 features (staged in LDS once per workgroup),
//   B operand = e~ of the 16 edges (each lane evaluates the basis slots it
//               holds; padding slots of a short last chunk are zero, so they
//               contribute nothing),
//   D         = lane l holds features 4g..4g+3 (g = l/16) of edge l%16.
// Products with the gathered neighbour features and the sums over edges run
// on the vector ALUs; the sum over the 16 edge slots of a tile row is a fixed
// reduce-scatter across the 16 lanes of the row, so results are bitwise
// reproducible.  Precision P = 0: FP32 operands (v_mfma_f32_16x16x4_f32);
// P = 1: bfloat16 operands (v_mfma_f32_16x16x32_bf16); accumulation FP32.
//
// The adjoint is organised by source atom j over its in-edges (j <- i), the
// reverses of the edges (i <- j) that carried j's messages; it gathers the
// destination gradients, accumulates dE/dphi_j and dE/dv_j, and for every
// edge computes G = dE/d(x_j - x_i) = (dE/dr) rhat + (I - rhat rhat^T) gr / r
// with dE/dr = sum_f dE/dw_f dw_f/dr, dw/dr = A' de~/dr (a second MFMA).
#include "internal.h"
#include "msg.h"

namespace mlp {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

template <int P, int K>
struct Basis {
    static constexpr int KP = P == 1 ? 32 : ((K + 1 + 3) / 4) * 4;   // padded basis length
    static constexpr int NS = P == 1 ? 1 : KP / 4;                    // MFMA k-steps
    static constexpr int SLOTS = P == 1 ? 8 : NS;                     // basis values held per lane
};

// Basis values (and optionally their r-derivatives) for the slots a lane holds.
// bf16: slots k = 8g + q (q = 0..7); f32: slots k = g + 4s (s = 0..NS-1).
template <int P, int K, bool DERIV>
__device__ __forceinline__ void basis_slots(float r, float rc, bool valid, int g, float *eb, float *db) {
    constexpr int SL = Basis<P, K>::SLOTS;
    const float pi = 3.14159265358979f;
    if (!valid) {
#pragma unroll
        for (int q = 0; q < SL; q++) {
            eb[q] = 0.f;
            if (DERIV) db[q] = 0.f;
        }
        return;
    }
    const float ir = 1.0f / r;
    const float th = pi * r / rc;
    float s1, c1;
    sincosf(th, &s1, &c1);
    const float fc = 0.5f * (c1 + 1.0f);
    const float dfc = -0.5f * (pi / rc) * s1;
    const int k0 = P == 1 ? 8 * g : g;
    const int kstep = P == 1 ? 1 : 4;
    float sk, ck, ss, cs;
    sincosf((float)k0 * th, &sk, &ck);
    if (kstep == 1) {
        ss = s1;
        cs = c1;
    } else {
        sincosf(4.0f * th, &ss, &cs);
    }
#pragma unroll
    for (int q = 0; q < SL; q++) {
        const int k = k0 + kstep * q;
        float e, de;
        if (k == 0) {
            e = fc;
            de = dfc;
        } else if (k <= K) {
            const float ek = sk * ir;
            e = ek * fc;
            de = ((float)k * (pi / rc) * ck * ir - ek * ir) * fc + ek * dfc;
        } else {
            e = 0.f;
            de = 0.f;
        }
        eb[q] = e;
        if (DERIV) db[q] = de;
        const float sn = fmaf(sk, cs, ck * ss);
        const float cn = fmaf(ck, cs, -sk * ss);
        sk = sn;
        ck = cn;
    }
}

// The B operand of one chunk as the MFMA consumes it: 8 packed bfloat16
// values (bf16) or NS floats (f32).
template <int P, int K>
struct BOp {
    float v[Basis<P, K>::NS];
    __device__ __forceinline__ void set(const float *eb) {
#pragma unroll
        for (int q = 0; q < Basis<P, K>::NS; q++) v[q] = eb[q];
    }
};
template <int K>
struct BOp<1, K> {
    v8bf v;
    __device__ __forceinline__ void set(const float *eb) {
#pragma unroll
        for (int q = 0; q < 8; q++) v[q] = (__bf16)eb[q];
    }
};

// Stage A' = [c | A] (3F x (K+1)) into LDS in the layout the A operand reads.
template <int P, int F, int K>
struct WStage {
    static constexpr int KP = Basis<P, K>::KP;
    static constexpr int LD = P == 1 ? KP + 8 : KP + 1;   // padded row stride (elements)
    static constexpr int ELEMS = 3 * F * LD;
};

template <int P, int F, int K>
__device__ __forceinline__ void stage_weights(const float *__restrict__ A, const float *__restrict__ c, void *lds) {
    using WS = WStage<P, F, K>;
    for (int idx = threadIdx.x; idx < 3 * F * WS::KP; idx += blockDim.x) {
        const int f = idx / WS::KP, k = idx % WS::KP;
        float v = 0.f;
        if (k == 0) v = c[f];
        else if (k <= K) v = A[(long)f * K + (k - 1)];
        if (P == 1) reinterpret_cast<__bf16 *>(lds)[f * WS::LD + k] = (__bf16)v;
        else reinterpret_cast<float *>(lds)[f * WS::LD + k] = v;
    }
    __syncthreads();
}

// w (4 features x this lane's edge) of 16-feature tile t from the basis operand.
template <int P, int F, int K>
__device__ __forceinline__ v4f filter_tile(const void *lds, int t, const BOp<P, K> &b, int lane) {
    using WS = WStage<P, F, K>;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    const int row = 16 * t + (lane & 15), g = lane >> 4;
    if constexpr (P == 1) {
        const v8bf a = *reinterpret_cast<const v8bf *>(reinterpret_cast<const __bf16 *>(lds) + row * WS::LD + 8 * g);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b.v, acc, 0, 0, 0);
    } else {
        const float *w = reinterpret_cast<const float *>(lds) + row * WS::LD;
#pragma unroll
        for (int s = 0; s < Basis<P, K>::NS; s++)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w[4 * s + g], b.v[s], acc, 0, 0, 0);
    }
    return acc;
}

// Sum over the 16 lanes of each 16-lane row, scattering the Q results so that
// the lane at row position p receives entries [p*Q/16, (p+1)*Q/16).
template <int Q>
__device__ __forceinline__ void row_reduce_scatter(float *a, int lane) {
    int n = Q;
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) {
        const bool hi = (lane & m) != 0;
        const int h = n / 2;
#pragma unroll
        for (int q = 0; q < Q / 2; q++) {
            if (q < h) {
                const float keep = hi ? a[q + h] : a[q];
                const float send = hi ? a[q] : a[q + h];
                a[q] = keep + __shfl_xor(send, m, 64);
            }
        }
        n = h;
    }
}

constexpr int CMAX = 5;   // chunks of 16 edges held in registers per batch

// ---------------------------------------------------------------------------
// Forward message pass.
// ---------------------------------------------------------------------------
template <int P, int F, int K>
__global__ void __launch_bounds__(256) k_msg_fwd_mfma(const int *__restrict__ rowc, const int *__restrict__ colc,
                                                      const float4 *__restrict__ geom, int n,
                                                      const float *__restrict__ phi, const float *__restrict__ s,
                                                      const float *__restrict__ v, const float *__restrict__ Aw,
                                                      const float *__restrict__ cw, float rc,
                                                      const int8_t *__restrict__ hop, int hop_max,
                                                      float *__restrict__ sn, float *__restrict__ v1) {
    using WS = WStage<P, F, K>;
    constexpr int NG = F / 16, F3 = 3 * F, SL = Basis<P, K>::SLOTS;
    __shared__ __attribute__((aligned(16))) char lds[WS::ELEMS * (P == 1 ? 2 : 4)];
    stage_weights<P, F, K>(Aw, cw, lds);
    const int lane = threadIdx.x & 63, g = lane >> 4, el = lane & 15;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6), nwaves = gridDim.x * 4;
    for (int i = wave; i < n; i += nwaves) {
        const int e0 = rowc[i], e1 = rowc[i + 1];
        const bool active = hop[i] <= hop_max;
        const int deg = active ? e1 - e0 : 0;
        for (int cb = 0; cb < deg || cb == 0; cb += 16 * CMAX) {
            int jj[CMAX];
            float rh[CMAX][3];
            BOp<P, K> eb[CMAX];
            const int nch = min(CMAX, (deg - cb + 15) / 16);
#pragma unroll
            for (int c = 0; c < CMAX; c++) {
                const int e = e0 + cb + 16 * c + el;
                const bool valid = c < nch && (cb + 16 * c + el) < deg;
                float4 gm = valid ? geom[e] : make_float4(0.f, 0.f, 0.f, rc);
                jj[c] = valid ? colc[e] : i;
                const float ir = 1.0f / gm.w;
                rh[c][0] = gm.x * ir;
                rh[c][1] = gm.y * ir;
                rh[c][2] = gm.z * ir;
                float tmp[SL];
                basis_slots<P, K, false>(gm.w, rc, valid, g, tmp, nullptr);
                eb[c].set(tmp);
            }
#pragma unroll 1
            for (int gi = 0; gi < NG; gi++) {
                const int fb = 16 * gi + 4 * g;
                float acc[16];
#pragma unroll
                for (int q = 0; q < 16; q++) acc[q] = 0.f;
#pragma unroll
                for (int c = 0; c < CMAX; c++) {
                    if (c < nch) {
                        const v4f wvv = filter_tile<P, F, K>(lds, gi, eb[c], lane);
                        const v4f ws = filter_tile<P, F, K>(lds, NG + gi, eb[c], lane);
                        const v4f wvs = filter_tile<P, F, K>(lds, 2 * NG + gi, eb[c], lane);
                        const float *pj = phi + (long)jj[c] * F3 + fb;
                        const float *vj = v + (long)jj[c] * F3 + fb;
                        const float4 pvv = *reinterpret_cast<const float4 *>(pj);
                        const float4 pss = *reinterpret_cast<const float4 *>(pj + F);
                        const float4 pvs = *reinterpret_cast<const float4 *>(pj + 2 * F);
                        const float4 v0 = *reinterpret_cast<const float4 *>(vj);
                        const float4 v1_ = *reinterpret_cast<const float4 *>(vj + F);
                        const float4 v2 = *reinterpret_cast<const float4 *>(vj + 2 * F);
                        const float a_vv[4] = {pvv.x, pvv.y, pvv.z, pvv.w};
                        const float a_s[4] = {pss.x, pss.y, pss.z, pss.w};
                        const float a_vs[4] = {pvs.x, pvs.y, pvs.z, pvs.w};
                        const float b0[4] = {v0.x, v0.y, v0.z, v0.w};
                        const float b1[4] = {v1_.x, v1_.y, v1_.z, v1_.w};
                        const float b2[4] = {v2.x, v2.y, v2.z, v2.w};
#pragma unroll
                        for (int r = 0; r < 4; r++) {
                            const float xvv = a_vv[r] * wvv[r];
                            const float xvs = a_vs[r] * wvs[r];
                            acc[r] = fmaf(a_s[r], ws[r], acc[r]);
                            acc[4 + r] = fmaf(b0[r], xvv, fmaf(rh[c][0], xvs, acc[4 + r]));
                            acc[8 + r] = fmaf(b1[r], xvv, fmaf(rh[c][1], xvs, acc[8 + r]));
                            acc[12 + r] = fmaf(b2[r], xvv, fmaf(rh[c][2], xvs, acc[12 + r]));
                        }
                    }
                }
                row_reduce_scatter<16>(acc, lane);
                // lane at row position el holds entry el: component el/4, feature fb + el%4
                const int comp = el >> 2, f = fb + (el & 3);
                float *dst = comp == 0 ? sn + (long)i * 2 * F + f : v1 + (long)i * F3 + (comp - 1) * F + f;
                const float base = cb == 0 ? (comp == 0 ? s[(long)i * F + f] : v[(long)i * F3 + (comp - 1) * F + f])
                                           : *dst;
                *dst = base + acc[0];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint of the message pass.
// ---------------------------------------------------------------------------
template <int P, int F, int K>
__global__ void __launch_bounds__(256) k_msg_bwd_mfma(const int *__restrict__ rowc, const int *__restrict__ colc,
                                                      const float4 *__restrict__ geom, int n,
                                                      const float *__restrict__ phi, const float *__restrict__ v,
                                                      const float *__restrict__ gs1, const float *__restrict__ gv1,
                                                      const float *__restrict__ Aw, const float *__restrict__ cw,
                                                      float rc, const int8_t *__restrict__ hop, int hop_max,
                                                      float *__restrict__ gv_in, float *__restrict__ gphi,
                                                      float4 *__restrict__ Gout) {
    using WS = WStage<P, F, K>;
    constexpr int NG = F / 16, F3 = 3 * F, SL = Basis<P, K>::SLOTS;
    __shared__ __attribute__((aligned(16))) char lds[WS::ELEMS * (P == 1 ? 2 : 4)];
    stage_weights<P, F, K>(Aw, cw, lds);
    const int lane = threadIdx.x & 63, g = lane >> 4, el = lane & 15;
    const int wave = blockIdx.x * 4 + (threadIdx.x >> 6), nwaves = gridDim.x * 4;
    for (int j = wave; j < n; j += nwaves) {
        const int e0 = rowc[j], e1 = rowc[j + 1];
        const bool active = hop[j] <= hop_max;
        const int deg = active ? e1 - e0 : 0;
        for (int cb = 0; cb < deg || cb == 0; cb += 16 * CMAX) {
            int ii[CMAX];
            float rh[CMAX][3], rr[CMAX];
            BOp<P, K> eb[CMAX], db[CMAX];
            float grh[CMAX][3], gr[CMAX];
            const int nch = min(CMAX, (deg - cb + 15) / 16);
#pragma unroll
            for (int c = 0; c < CMAX; c++) {
                const int e = e0 + cb + 16 * c + el;
                const bool valid = c < nch && (cb + 16 * c + el) < deg;
                float4 gm = valid ? geom[e] : make_float4(0.f, 0.f, 0.f, rc);
                ii[c] = valid ? colc[e] : j;
                const float ir = 1.0f / gm.w;
                rr[c] = gm.w;
                rh[c][0] = -gm.x * ir;   // direction of the message edge (i <- j): x_j - x_i
                rh[c][1] = -gm.y * ir;
                rh[c][2] = -gm.z * ir;
                float te[SL], td[SL];
                basis_slots<P, K, true>(gm.w, rc, valid, g, te, td);
                eb[c].set(te);
                db[c].set(td);
                grh[c][0] = grh[c][1] = grh[c][2] = 0.f;
                gr[c] = 0.f;
            }
#pragma unroll 1
            for (int gi = 0; gi < NG; gi++) {
                const int fb = 16 * gi + 4 * g;
                const float *pj = phi + (long)j * F3 + fb;
                const float *vjp = v + (long)j * F3 + fb;
                float ph[3][4], vj[3][4];
#pragma unroll
                for (int p = 0; p < 3; p++) {
                    const float4 a = *reinterpret_cast<const float4 *>(pj + p * F);
                    const float4 b = *reinterpret_cast<const float4 *>(vjp + p * F);
                    ph[p][0] = a.x; ph[p][1] = a.y; ph[p][2] = a.z; ph[p][3] = a.w;
                    vj[p][0] = b.x; vj[p][1] = b.y; vj[p][2] = b.z; vj[p][3] = b.w;
                }
                float acc[32];   // [0,12): dE/dphi_j (vv, s, vs) x 4; [12,24): dE/dv_j (d) x 4; rest pad
#pragma unroll
                for (int q = 0; q < 32; q++) acc[q] = 0.f;
#pragma unroll
                for (int c = 0; c < CMAX; c++) {
                    if (c < nch) {
                        const v4f w0 = filter_tile<P, F, K>(lds, gi, eb[c], lane);
                        const v4f w1 = filter_tile<P, F, K>(lds, NG + gi, eb[c], lane);
                        const v4f w2 = filter_tile<P, F, K>(lds, 2 * NG + gi, eb[c], lane);
                        const v4f d0 = filter_tile<P, F, K>(lds, gi, db[c], lane);
                        const v4f d1 = filter_tile<P, F, K>(lds, NG + gi, db[c], lane);
                        const v4f d2 = filter_tile<P, F, K>(lds, 2 * NG + gi, db[c], lane);
                        const float *gsi = gs1 + (long)ii[c] * F + fb;
                        const float *gvi = gv1 + (long)ii[c] * F3 + fb;
                        const float4 gsv = *reinterpret_cast<const float4 *>(gsi);
                        const float4 ga0 = *reinterpret_cast<const float4 *>(gvi);
                        const float4 ga1 = *reinterpret_cast<const float4 *>(gvi + F);
                        const float4 ga2 = *reinterpret_cast<const float4 *>(gvi + 2 * F);
                        const float gs_[4] = {gsv.x, gsv.y, gsv.z, gsv.w};
                        const float g0[4] = {ga0.x, ga0.y, ga0.z, ga0.w};
                        const float g1[4] = {ga1.x, ga1.y, ga1.z, ga1.w};
                        const float g2[4] = {ga2.x, ga2.y, ga2.z, ga2.w};
#pragma unroll
                        for (int r = 0; r < 4; r++) {
                            const float gxvv = fmaf(g0[r], vj[0][r], fmaf(g1[r], vj[1][r], g2[r] * vj[2][r]));
                            const float gxvs = fmaf(g0[r], rh[c][0], fmaf(g1[r], rh[c][1], g2[r] * rh[c][2]));
                            const float gxs = gs_[r];
                            const float xvv = ph[0][r] * w0[r];
                            const float xvs = ph[2][r] * w2[r];
                            acc[r] = fmaf(gxvv, w0[r], acc[r]);
                            acc[4 + r] = fmaf(gxs, w1[r], acc[4 + r]);
                            acc[8 + r] = fmaf(gxvs, w2[r], acc[8 + r]);
                            acc[12 + r] = fmaf(g0[r], xvv, acc[12 + r]);
                            acc[16 + r] = fmaf(g1[r], xvv, acc[16 + r]);
                            acc[20 + r] = fmaf(g2[r], xvv, acc[20 + r]);
                            grh[c][0] = fmaf(g0[r], xvs, grh[c][0]);
                            grh[c][1] = fmaf(g1[r], xvs, grh[c][1]);
                            grh[c][2] = fmaf(g2[r], xvs, grh[c][2]);
                            gr[c] = fmaf(gxvv * ph[0][r], d0[r],
                                         fmaf(gxs * ph[1][r], d1[r], fmaf(gxvs * ph[2][r], d2[r], gr[c])));
                        }
                    }
                }
                row_reduce_scatter<32>(acc, lane);
                // lane at row position el holds entries 2el, 2el+1: component el/2, features fb + 2(el%2) + {0,1}
                const int comp = el >> 1;
                if (comp < 6) {
#pragma unroll
                    for (int u = 0; u < 2; u++) {
                        const int f = fb + 2 * (el & 1) + u;
                        if (comp < 3) {
                            float *dst = gphi + (long)j * F3 + comp * F + f;
                            *dst = (cb == 0 ? 0.f : *dst) + acc[u];
                        } else {
                            float *dst = gv_in + (long)j * F3 + (comp - 3) * F + f;
                            *dst = (cb == 0 ? gv1[(long)j * F3 + (comp - 3) * F + f] : *dst) + acc[u];
                        }
                    }
                }
            }
            // per edge: finish the sums over features (the four lane rows) and write G
#pragma unroll
            for (int c = 0; c < CMAX; c++) {
                if (c < nch) {
                    float a0 = grh[c][0], a1 = grh[c][1], a2 = grh[c][2], a3 = gr[c];
#pragma unroll
                    for (int m = 16; m <= 32; m <<= 1) {
                        a0 += __shfl_xor(a0, m, 64);
                        a1 += __shfl_xor(a1, m, 64);
                        a2 += __shfl_xor(a2, m, 64);
                        a3 += __shfl_xor(a3, m, 64);
                    }
                    const int e = e0 + cb + 16 * c + el;
                    const bool valid = (cb + 16 * c + el) < deg;
                    if (g == 0 && valid) {
                        const float ir = 1.0f / rr[c];
                        const float rd = a0 * rh[c][0] + a1 * rh[c][1] + a2 * rh[c][2];
                        float4 G = Gout[e];
                        G.x += a3 * rh[c][0] + (a0 - rd * rh[c][0]) * ir;
                        G.y += a3 * rh[c][1] + (a1 - rd * rh[c][1]) * ir;
                        G.z += a3 * rh[c][2] + (a2 - rd * rh[c][2]) * ir;
                        Gout[e] = G;
                    }
                }
            }
        }
    }
}

template <int P, int F, int K>
static int launch_fwd(hipStream_t st, const MsgArgs &a) {
    const int blocks = std::max(1, std::min((a.n + 3) / 4, 2048));
    k_msg_fwd_mfma<P, F, K><<<blocks, 256, 0, st>>>(a.rowc, a.colc, a.geom, a.n, a.phi, a.s, a.v, a.A, a.c, a.rc,
                                                   a.hop, a.hop_max, a.sn, a.v1);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

template <int P, int F, int K>
static int launch_bwd(hipStream_t st, const MsgArgs &a) {
    const int blocks = std::max(1, std::min((a.n + 3) / 4, 2048));
    k_msg_bwd_mfma<P, F, K><<<blocks, 256, 0, st>>>(a.rowc, a.colc, a.geom, a.n, a.phi, a.v, a.gs1, a.gv1, a.A, a.c,
                                                   a.rc, a.hop, a.hop_max, a.gv_in, a.gphi, a.G);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

#define MSG_DISPATCH(FN, P_)                                                     \
    do {                                                                         \
        if (F == 128 && K == 20) return FN<P_, 128, 20>(st, a);                   \
        if (F == 128 && K == 8) return FN<P_, 128, 8>(st, a);                     \
        if (F == 64 && K == 20) return FN<P_, 64, 20>(st, a);                     \
        if (F == 64 && K == 8) return FN<P_, 64, 8>(st, a);                       \
        if (F == 32 && K == 20) return FN<P_, 32, 20>(st, a);                     \
        if (F == 32 && K == 8) return FN<P_, 32, 8>(st, a);                       \
        if (F == 16 && K == 6) return FN<P_, 16, 6>(st, a);                       \
    } while (0)

int msg_forward(hipStream_t st, int precision, int F, int K, const MsgArgs &a) {
    if (precision == 0) MSG_DISPATCH(launch_fwd, 0);
    else MSG_DISPATCH(launch_fwd, 1);
    return -1;
}

int msg_adjoint(hipStream_t st, int precision, int F, int K, const MsgArgs &a) {
    if (precision == 0) MSG_DISPATCH(launch_bwd, 0);
    else MSG_DISPATCH(launch_bwd, 1);
    return -1;
}

}  // namespace mlp
