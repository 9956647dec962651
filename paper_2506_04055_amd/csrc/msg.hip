// Message pass and its adjoint with the radial-filter contraction on MFMA.
//
// Per directed edge (i <- j) the filter is w = A' e~(r), a dense K+1 -> 3F
// contraction with A' = [c | A] and e~ = [fc, e_1 fc, ..., e_K fc],
// e_k = sin(k pi r / rc) / r.  A wave owns one atom; its edges are taken 16
// at a time.  For each chunk the filter is computed as 16 x 16 MFMA tiles
// (16 features x 16 edges):
//   A operand = 16 rows of A' (staged in LDS once per workgroup),
//   B operand = e~ of the 16 edges (each lane evaluates the basis slots it
//               holds; padding slots of a short last chunk are zero, so they
//               contribute nothing),
// and written to a per-wave LDS buffer.  A vector phase then runs with lane =
// (edge parity, feature): it gathers 128-byte segments of the neighbour rows,
// forms the products and accumulates per feature in registers, so sums over
// edges need no cross-lane traffic except one final pairing.  Precision P = 0:
// FP32 operands (v_mfma_f32_16x16x4_f32); P = 1: bfloat16 operands
// (v_mfma_f32_16x16x32_bf16); P = 2: split bfloat16 operands x = hi + lo
// (hi = bf16(x), lo = bf16(x - hi)) with the three products lo*hi + hi*lo +
// hi*hi; accumulation FP32 in all.  Every sum has a fixed order, so results
// are bitwise reproducible.
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
    static constexpr int KP = P >= 1 ? 32 : ((K + 1 + 3) / 4) * 4;   // padded basis length
    static constexpr int NS = P >= 1 ? 1 : KP / 4;                    // MFMA k-steps
    static constexpr int SLOTS = P >= 1 ? 8 : NS;                     // basis values held per lane
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
    const int k0 = P >= 1 ? 8 * g : g;
    const int kstep = P >= 1 ? 1 : 4;
    // (sin, cos) of 2, 4, 8, 16 and 24 theta by angle doubling and addition
    // from the one small-argument sincos, so no large-argument reduction runs
    const float s2 = 2.0f * s1 * c1, c2 = fmaf(-2.0f * s1, s1, 1.0f);
    const float s4 = 2.0f * s2 * c2, c4 = fmaf(-2.0f * s2, s2, 1.0f);
    float sk, ck, ss, cs;
    if (kstep == 1) {
        const float s8 = 2.0f * s4 * c4, c8 = fmaf(-2.0f * s4, s4, 1.0f);
        const float s16 = 2.0f * s8 * c8, c16 = fmaf(-2.0f * s8, s8, 1.0f);
        const float s24 = fmaf(s16, c8, c16 * s8), c24 = fmaf(c16, c8, -s16 * s8);
        sk = g == 0 ? 0.f : (g == 1 ? s8 : (g == 2 ? s16 : s24));
        ck = g == 0 ? 1.f : (g == 1 ? c8 : (g == 2 ? c16 : c24));
        ss = s1;
        cs = c1;
    } else {
        const float s3 = fmaf(s2, c1, c2 * s1), c3 = fmaf(c2, c1, -s2 * s1);
        sk = g == 0 ? 0.f : (g == 1 ? s1 : (g == 2 ? s2 : s3));
        ck = g == 0 ? 1.f : (g == 1 ? c1 : (g == 2 ? c2 : c3));
        ss = s4;
        cs = c4;
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
template <int K>
struct BOp<2, K> {
    v8bf v, lo;
    __device__ __forceinline__ void set(const float *eb) {
#pragma unroll
        for (int q = 0; q < 8; q++) {
            v[q] = (__bf16)eb[q];
            lo[q] = (__bf16)(eb[q] - (float)v[q]);
        }
    }
};

// Stage A' = [c | A] (3F x (K+1)) into LDS in the layout the A operand reads.
template <int P, int F, int K>
struct WStage {
    static constexpr int KP = Basis<P, K>::KP;
    static constexpr int LD = P >= 1 ? KP + 8 : KP + 1;   // padded row stride (elements)
    static constexpr int ELEMS = 3 * F * LD * (P == 2 ? 2 : 1);   // split mode: hi table, then lo table
    static constexpr int BYTES = ELEMS * (P >= 1 ? 2 : 4);
};

template <int P, int F, int K>
__device__ __forceinline__ void stage_weights(const float *__restrict__ A, const float *__restrict__ c, void *lds) {
    using WS = WStage<P, F, K>;
    for (int idx = threadIdx.x; idx < 3 * F * WS::KP; idx += blockDim.x) {
        const int f = idx / WS::KP, k = idx % WS::KP;
        float v = 0.f;
        if (k == 0) v = c[f];
        else if (k <= K) v = A[(long)f * K + (k - 1)];
        if (P >= 1) {
            const __bf16 h = (__bf16)v;
            reinterpret_cast<__bf16 *>(lds)[f * WS::LD + k] = h;
            if (P == 2) reinterpret_cast<__bf16 *>(lds)[3 * F * WS::LD + f * WS::LD + k] = (__bf16)(v - (float)h);
        } else {
            reinterpret_cast<float *>(lds)[f * WS::LD + k] = v;
        }
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
    } else if constexpr (P == 2) {
        const __bf16 *t0 = reinterpret_cast<const __bf16 *>(lds) + row * WS::LD + 8 * g;
        const v8bf a = *reinterpret_cast<const v8bf *>(t0);
        const v8bf al = *reinterpret_cast<const v8bf *>(t0 + 3 * F * WS::LD);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b.v, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b.lo, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b.v, acc, 0, 0, 0);
    } else {
        const float *w = reinterpret_cast<const float *>(lds) + row * WS::LD;
#pragma unroll
        for (int s = 0; s < Basis<P, K>::NS; s++)
            acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w[4 * s + g], b.v[s], acc, 0, 0, 0);
    }
    return acc;
}

// Sum over the L lanes of each aligned group of L lanes (L = 2 * M0), leaving
// the lane at position p in its group with entries [p*Q/L, (p+1)*Q/L).
// Fixed pairings, so the summation order never changes.
template <int H>
__device__ __forceinline__ void rs_stage(float *a, int lane, int m) {
    // Both halves are exchanged and summed, then each lane keeps the half its
    // position selects.  Selecting between two computed sums (not between two
    // array slots) keeps every array index a compile-time constant.
    const bool hi = (lane & m) != 0;
#pragma unroll
    for (int q = 0; q < H; q++) {
        const float lo_sum = a[q] + __shfl_xor(a[q], m, 64);
        const float hi_sum = a[q + H] + __shfl_xor(a[q + H], m, 64);
        a[q] = hi ? hi_sum : lo_sum;
    }
}

template <int Q, int M0>
__device__ __forceinline__ void reduce_scatter(float *a, int lane) {
    if constexpr (M0 >= 1 && Q >= 2) {
        rs_stage<Q / 2>(a, lane, M0);
        reduce_scatter<Q / 2, M0 / 2>(a, lane);
    }
}

// LDS written by some lanes of a wave and read by others: make the writes
// visible within the wave (waves of a workgroup work on different atoms and
// never wait for each other).
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int WAVES = 8;   // waves per workgroup
constexpr int PW = 32;     // features per pass of the vector phase

// Atoms handled by this wave.  Workgroups are dispatched round-robin over the
// XCDs, each with its own L2; XCD x gets the contiguous slice
// [x n / nx, (x+1) n / nx) of the cell-sorted atoms, and the waves of its
// workgroups interleave over that slice, so neighbour rows gathered by one
// XCD stay in its L2.  The slices partition [0, n) whatever the grid size.
struct XcdRange {
    int first, end, stride;
    __device__ __forceinline__ explicit XcdRange(int n) {
        const int nx = gridDim.x < 8 ? (int)gridDim.x : 8;
        const int x = blockIdx.x % nx, b = blockIdx.x / nx;
        const int nb = ((int)gridDim.x - x + nx - 1) / nx;   // workgroups with blockIdx % nx == x
        const int lo = (int)((long)n * x / nx), hi = (int)((long)n * (x + 1) / nx);
        const int wpb = blockDim.x >> 6;
        first = lo + b * wpb + (int)(threadIdx.x >> 6);
        end = hi;
        stride = nb * wpb;
    }
};

// Per-wave LDS: filter values of one pass for the 16 edges of a chunk,
// [edge][part][feature in pass], and the chunk's edge records (8 floats each).
template <int P, int F, int K>
struct MsgLds {
    static constexpr int WBUF = 16 * 3 * PW;
    static constexpr int PER_WAVE = WBUF + 16 * 8;
    static constexpr int BYTES = WStage<P, F, K>::BYTES + WAVES * PER_WAVE * 4;
};

// Filter tiles of pass p (features [p*PW, p*PW + FP) of each part) for the
// current chunk, written to the wave's LDS buffer as [edge][part][feature].
template <int P, int F, int K>
__device__ __forceinline__ void filter_pass_to_lds(const void *lds, const BOp<P, K> &b, int p, int lane,
                                                   float *wbuf) {
    constexpr int NG = F / 16, FP = F < PW ? F : PW;
    const int g = lane >> 4, el = lane & 15;
#pragma unroll
    for (int q = 0; q < 3; q++)
#pragma unroll
        for (int u = 0; u < FP / 16; u++) {
            const int t = q * NG + (p * PW) / 16 + u;
            const v4f d = filter_tile<P, F, K>(lds, t, b, lane);
            *reinterpret_cast<float4 *>(&wbuf[(el * 3 + q) * PW + 16 * u + 4 * g]) = make_float4(d[0], d[1], d[2], d[3]);
        }
}

// ---------------------------------------------------------------------------
// Forward message pass.  Per chunk of 16 edges: the filter tiles on MFMA, then
// a vector phase with lane = (edge parity, feature) that gathers 128-byte row
// segments of the source atoms and accumulates in registers.
// ---------------------------------------------------------------------------
template <int P, int F, int K>
__global__ void __launch_bounds__(64 * WAVES) k_msg_fwd_mfma(const int *__restrict__ rowc,
                                                            const int *__restrict__ colc,
                                                            const float4 *__restrict__ geom, int n,
                                                            const float *__restrict__ phi,
                                                            const float *__restrict__ s,
                                                            const float *__restrict__ v,
                                                            const float *__restrict__ Aw,
                                                            const float *__restrict__ cw, float rc,
                                                            const int8_t *__restrict__ hop, int hop_max,
                                                            float *__restrict__ sn, float *__restrict__ v1) {
    using LS = MsgLds<P, F, K>;
    constexpr int F3 = 3 * F, SL = Basis<P, K>::SLOTS;
    constexpr int FP = F < PW ? F : PW, NP = F / FP;
    __shared__ __attribute__((aligned(16))) char lds[LS::BYTES];
    stage_weights<P, F, K>(Aw, cw, lds);
    const int lane = threadIdx.x & 63, g = lane >> 4, el = lane & 15;
    const int eh = lane >> 5, fi = lane & 31;
    float *wbuf = reinterpret_cast<float *>(lds + WStage<P, F, K>::BYTES) + (threadIdx.x >> 6) * LS::PER_WAVE;
    float *erec = wbuf + LS::WBUF;
    const XcdRange xr(n);
    for (int i = xr.first; i < xr.end; i += xr.stride) {
        const int e0 = rowc[i], e1 = rowc[i + 1];
        const int deg = hop[i] <= hop_max ? e1 - e0 : 0;
        float acc[NP][4];
#pragma unroll
        for (int p = 0; p < NP; p++) acc[p][0] = acc[p][1] = acc[p][2] = acc[p][3] = 0.f;
        for (int cb = 0; cb < deg; cb += 16) {
            const bool valid = cb + el < deg;
            float4 gm = make_float4(0.f, 0.f, 0.f, rc);
            int jj = i;
            if (valid) {
                gm = geom[e0 + cb + el];
                jj = colc[e0 + cb + el];
            }
            float eb[SL];
            basis_slots<P, K, false>(gm.w, rc, valid, g, eb, nullptr);
            BOp<P, K> bop;
            bop.set(eb);
            if (g == 0) {
                const float ir = 1.0f / gm.w;
                *reinterpret_cast<float4 *>(&erec[el * 8]) = make_float4(__int_as_float(jj), gm.x * ir, gm.y * ir, gm.z * ir);
            }
#pragma unroll
            for (int p = 0; p < NP; p++) {
                filter_pass_to_lds<P, F, K>(lds, bop, p, lane, wbuf);
                wave_lds_sync();
                if (fi < FP) {
                    const int f = p * PW + fi;
#pragma unroll 4
                    for (int st = 0; st < 8; st++) {
                        const int ed = 2 * st + eh;
                        const float4 rec = *reinterpret_cast<const float4 *>(&erec[ed * 8]);
                        const int j = __float_as_int(rec.x);
                        const float wvv = wbuf[(ed * 3 + 0) * PW + fi];
                        const float ws = wbuf[(ed * 3 + 1) * PW + fi];
                        const float wvs = wbuf[(ed * 3 + 2) * PW + fi];
                        const float *pj = phi + (long)j * F3 + f;
                        const float *vj = v + (long)j * F3 + f;
                        const float xvv = pj[0] * wvv, xvs = pj[2 * F] * wvs;
                        acc[p][0] = fmaf(pj[F], ws, acc[p][0]);
                        acc[p][1] = fmaf(vj[0], xvv, fmaf(rec.y, xvs, acc[p][1]));
                        acc[p][2] = fmaf(vj[F], xvv, fmaf(rec.z, xvs, acc[p][2]));
                        acc[p][3] = fmaf(vj[2 * F], xvv, fmaf(rec.w, xvs, acc[p][3]));
                    }
                }
                wave_lds_sync();
            }
        }
        // the two edge parities hold partial sums of the same feature
#pragma unroll
        for (int p = 0; p < NP; p++)
#pragma unroll
            for (int c = 0; c < 4; c++) acc[p][c] += __shfl_xor(acc[p][c], 32, 64);
        if (eh == 0 && fi < FP) {
#pragma unroll
            for (int p = 0; p < NP; p++) {
                const int f = p * PW + fi;
                sn[(long)i * 2 * F + f] = s[(long)i * F + f] + acc[p][0];
#pragma unroll
                for (int d = 0; d < 3; d++)
                    v1[(long)i * F3 + d * F + f] = v[(long)i * F3 + d * F + f] + acc[p][1 + d];
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint of the message pass.  Per chunk of 16 in-edges (j <- i) of the
// source atom j: per pass, the filter tiles (then their radial derivatives)
// on MFMA, and a vector phase over (edge parity, feature) lanes that gathers
// the destinations' gradients.  dE/dphi_j and dE/dv_j accumulate in registers;
// the per-edge sums over features (dE/dr and dE/drhat) are reduced across the
// 32 feature lanes once per chunk and give G of edge (i <- j), added at the
// position of (j <- i).
// ---------------------------------------------------------------------------
template <int P, int F, int K>
__global__ void __launch_bounds__(64 * WAVES) k_msg_bwd_mfma(const int *__restrict__ rowc,
                                                            const int *__restrict__ colc,
                                                            const float4 *__restrict__ geom, int n,
                                                            const float *__restrict__ phi,
                                                            const float *__restrict__ v,
                                                            const float *__restrict__ gs1,
                                                            const float *__restrict__ gv1,
                                                            const float *__restrict__ Aw,
                                                            const float *__restrict__ cw, float rc,
                                                            const int8_t *__restrict__ hop, int hop_max,
                                                            float *__restrict__ gv_in, float *__restrict__ gphi,
                                                            float4 *__restrict__ Gout) {
    using LS = MsgLds<P, F, K>;
    constexpr int F3 = 3 * F, SL = Basis<P, K>::SLOTS;
    constexpr int FP = F < PW ? F : PW, NP = F / FP;
    __shared__ __attribute__((aligned(16))) char lds[LS::BYTES];
    stage_weights<P, F, K>(Aw, cw, lds);
    const int lane = threadIdx.x & 63, g = lane >> 4, el = lane & 15;
    const int eh = lane >> 5, fi = lane & 31;
    float *wbuf = reinterpret_cast<float *>(lds + WStage<P, F, K>::BYTES) + (threadIdx.x >> 6) * LS::PER_WAVE;
    float *erec = wbuf + LS::WBUF;
    const XcdRange xr(n);
    for (int j = xr.first; j < xr.end; j += xr.stride) {
        const int e0 = rowc[j], e1 = rowc[j + 1];
        const int deg = hop[j] <= hop_max ? e1 - e0 : 0;
        // One pass per block of FP features.  G is linear in (dE/dr, dE/drhat),
        // so each pass adds the share of its features to G directly.
#pragma unroll 1
        for (int p = 0; p < NP; p++) {
            const int f = p * PW + (fi < FP ? fi : 0);
            float ph[3], vj[3];
#pragma unroll
            for (int q = 0; q < 3; q++) {
                ph[q] = phi[(long)j * F3 + q * F + f];
                vj[q] = v[(long)j * F3 + q * F + f];
            }
            float agp0 = 0.f, agp1 = 0.f, agp2 = 0.f, agv0 = 0.f, agv1 = 0.f, agv2 = 0.f;
#pragma unroll 1
            for (int cb = 0; cb < deg; cb += 16) {
                const bool valid = cb + el < deg;
                float4 gm = make_float4(0.f, 0.f, 0.f, rc);
                int ii = j;
                if (valid) {
                    gm = geom[e0 + cb + el];
                    ii = colc[e0 + cb + el];
                }
                float eb[SL], db[SL];
                basis_slots<P, K, true>(gm.w, rc, valid, g, eb, db);
                BOp<P, K> bop, dop;
                bop.set(eb);
                dop.set(db);
                if (g == 0) {
                    const float ir = 1.0f / gm.w;
                    // direction of the message edge (i <- j) is x_j - x_i = -(x_i - x_j)
                    *reinterpret_cast<float4 *>(&erec[el * 8]) =
                        make_float4(__int_as_float(ii), -gm.x * ir, -gm.y * ir, -gm.z * ir);
                    erec[el * 8 + 4] = gm.w;
                }
                float part[8][4];   // per step: dE/dr, dE/drhat (x, y, z) over this lane's features
                float keep[8][4];   // gathered dE/ds1_i, dE/dv1_i reused by the derivative phase
                filter_pass_to_lds<P, F, K>(lds, bop, p, lane, wbuf);
                wave_lds_sync();
#pragma unroll
                for (int st = 0; st < 8; st++) {
                    const int ed = 2 * st + eh;
                    const float4 rec = *reinterpret_cast<const float4 *>(&erec[ed * 8]);
                    const int i = __float_as_int(rec.x);
                    const float w0 = wbuf[(ed * 3 + 0) * PW + fi];
                    const float w1 = wbuf[(ed * 3 + 1) * PW + fi];
                    const float w2 = wbuf[(ed * 3 + 2) * PW + fi];
                    const float gs = gs1[(long)i * F + f];
                    const float ga = gv1[(long)i * F3 + f];
                    const float gb = gv1[(long)i * F3 + F + f];
                    const float gc = gv1[(long)i * F3 + 2 * F + f];
                    keep[st][0] = gs;
                    keep[st][1] = ga;
                    keep[st][2] = gb;
                    keep[st][3] = gc;
                    const float gxvv = fmaf(ga, vj[0], fmaf(gb, vj[1], gc * vj[2]));
                    const float gxvs = fmaf(ga, rec.y, fmaf(gb, rec.z, gc * rec.w));
                    const float xvv = ph[0] * w0, xvs = ph[2] * w2;
                    agv0 = fmaf(ga, xvv, agv0);
                    agv1 = fmaf(gb, xvv, agv1);
                    agv2 = fmaf(gc, xvv, agv2);
                    agp0 = fmaf(gxvv, w0, agp0);
                    agp1 = fmaf(gs, w1, agp1);
                    agp2 = fmaf(gxvs, w2, agp2);
                    part[st][1] = ga * xvs;
                    part[st][2] = gb * xvs;
                    part[st][3] = gc * xvs;
                }
                wave_lds_sync();
                filter_pass_to_lds<P, F, K>(lds, dop, p, lane, wbuf);
                wave_lds_sync();
#pragma unroll
                for (int st = 0; st < 8; st++) {
                    const int ed = 2 * st + eh;
                    const float4 rec = *reinterpret_cast<const float4 *>(&erec[ed * 8]);
                    const float d0 = wbuf[(ed * 3 + 0) * PW + fi];
                    const float d1 = wbuf[(ed * 3 + 1) * PW + fi];
                    const float d2 = wbuf[(ed * 3 + 2) * PW + fi];
                    const float gxvv = fmaf(keep[st][1], vj[0], fmaf(keep[st][2], vj[1], keep[st][3] * vj[2]));
                    const float gxvs = fmaf(keep[st][1], rec.y, fmaf(keep[st][2], rec.z, keep[st][3] * rec.w));
                    part[st][0] = fmaf(gxvv * ph[0], d0, fmaf(keep[st][0] * ph[1], d1, gxvs * ph[2] * d2));
                }
                if (fi >= FP) {
#pragma unroll
                    for (int st = 0; st < 8; st++) part[st][0] = part[st][1] = part[st][2] = part[st][3] = 0.f;
                }
                // sum over the 32 feature lanes of each edge parity; lane fi
                // then holds entry fi = 4 * step + component
                float flat[32];
#pragma unroll
                for (int st = 0; st < 8; st++)
#pragma unroll
                    for (int c = 0; c < 4; c++) flat[4 * st + c] = part[st][c];
                reduce_scatter<32, 16>(flat, lane);
                const float c1 = __shfl_down(flat[0], 1, 64);
                const float c2 = __shfl_down(flat[0], 2, 64);
                const float c3 = __shfl_down(flat[0], 3, 64);
                const int ed = 2 * (fi >> 2) + eh;
                if ((fi & 3) == 0 && cb + ed < deg) {
                    const float4 rec = *reinterpret_cast<const float4 *>(&erec[ed * 8]);
                    const float ir = 1.0f / erec[ed * 8 + 4];
                    const float gr = flat[0];
                    const float rd = c1 * rec.y + c2 * rec.z + c3 * rec.w;
                    float4 G = Gout[e0 + cb + ed];
                    G.x += gr * rec.y + (c1 - rd * rec.y) * ir;
                    G.y += gr * rec.z + (c2 - rd * rec.z) * ir;
                    G.z += gr * rec.w + (c3 - rd * rec.w) * ir;
                    Gout[e0 + cb + ed] = G;
                }
                wave_lds_sync();
            }
            // the two edge parities hold partial sums of the same feature
            agp0 += __shfl_xor(agp0, 32, 64);
            agp1 += __shfl_xor(agp1, 32, 64);
            agp2 += __shfl_xor(agp2, 32, 64);
            agv0 += __shfl_xor(agv0, 32, 64);
            agv1 += __shfl_xor(agv1, 32, 64);
            agv2 += __shfl_xor(agv2, 32, 64);
            if (eh == 0 && fi < FP) {
                const long b = (long)j * F3 + f;
                gphi[b] = agp0;
                gphi[b + F] = agp1;
                gphi[b + 2 * F] = agp2;
                gv_in[b] = gv1[b] + agv0;
                gv_in[b + F] = gv1[b + F] + agv1;
                gv_in[b + 2 * F] = gv1[b + 2 * F] + agv2;
            }
        }
    }
}

template <int P, int F, int K>
static int launch_fwd(hipStream_t st, const MsgArgs &a) {
    const int blocks = std::max(1, std::min((a.n + WAVES - 1) / WAVES, 2048));
    k_msg_fwd_mfma<P, F, K><<<blocks, 64 * WAVES, 0, st>>>(a.rowc, a.colc, a.geom, a.n, a.phi, a.s, a.v, a.A, a.c,
                                                          a.rc, a.hop, a.hop_max, a.sn, a.v1);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

template <int P, int F, int K>
static int launch_bwd(hipStream_t st, const MsgArgs &a) {
    const int blocks = std::max(1, std::min((a.n + WAVES - 1) / WAVES, 2048));
    k_msg_bwd_mfma<P, F, K><<<blocks, 64 * WAVES, 0, st>>>(a.rowc, a.colc, a.geom, a.n, a.phi, a.v, a.gs1, a.gv1,
                                                          a.A, a.c, a.rc, a.hop, a.hop_max, a.gv_in, a.gphi, a.G);
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
    else if (precision == 1) MSG_DISPATCH(launch_fwd, 1);
    else MSG_DISPATCH(launch_fwd, 2);
    return -1;
}

int msg_adjoint(hipStream_t st, int precision, int F, int K, const MsgArgs &a) {
    if (precision == 0) MSG_DISPATCH(launch_bwd, 0);
    else if (precision == 1) MSG_DISPATCH(launch_bwd, 1);
    else MSG_DISPATCH(launch_bwd, 2);
    return -1;
}

}  // namespace mlp
