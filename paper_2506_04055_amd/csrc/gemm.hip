// Node-feature GEMMs on the matrix cores (MFMA), with fused epilogues.
//
//   C[m][n] = epilogue( sum_k A[m][k] B(k, n) )
//
// A is an FP32 activation matrix (rows = atoms, or atoms x 3 for vector
// features); B is a weight matrix packed once per model (pack_weight) as
// [n][k] with the reduction index contiguous, in FP32 and as bfloat16 hi / lo
// parts, zero-padded so that no load of B needs a bound check.
//
// Each wave owns 16 rows of C and one chunk of 128 columns (eight 16 x 16
// MFMA tiles; the chunk is blockIdx.y, and grid.x is padded to a multiple of
// 8 so the chunks of a row block share one XCD's L2).  The wave first loads
// its whole 16 x K slice of A (K <= 384) into registers, already in MFMA
// operand form, so all of its HBM reads are in flight at once and A is never
// read twice by one wave.  A workgroup of four waves (64 rows) stages B in
// LDS in chunks of KC k-columns, each thread loading a fixed share of the next
// chunk into registers while the current one is multiplied:
//   bf16 (v_mfma_f32_16x16x32_bf16): lane l = 16 g + c holds
//        A[row c][k0 + 8g .. k0 + 8g + 7] and B[k0 + 8g .. +7][col c];
//   f32  (v_mfma_f32_16x16x4_f32): lane l holds A[row c][k0 + 4g + j] and
//        B[k0 + 4g + j][col c] in MFMA step j = 0..3 (one 16-byte load each;
//        the k order inside a 16-block is permuted alike on both sides, which
//        the sum does not see);
//   D:   lane l holds rows 4g .. 4g+3 of column c.
// Split-bf16 mode (P = 2) rounds A on the fly to x = hi + lo with
// hi = bf16(x), lo = bf16(x - hi), and accumulates lo*hi + hi*lo + hi*hi
// (the lo*lo term is below FP32 rounding of the leading part): ~16
// significant bits per operand at the bf16 instruction rate.  The epilogue's
// second operand (residual or pre-activation) is fetched at the start too.
#include "gemm.h"

#include <algorithm>

namespace mlp {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

constexpr int GW = 4;          // waves per workgroup
constexpr int NCH = 128;       // output columns per chunk
constexpr int CT = NCH / 16;   // MFMA tiles per chunk

static inline int round_up(int x, int m) { return (x + m - 1) / m * m; }

__device__ __forceinline__ float g_sigmoid(float x) { return 1.0f / (1.0f + __expf(-x)); }
__device__ __forceinline__ v4f gld4(const float *p) { return *reinterpret_cast<const v4f *>(p); }

// Layout of one packed matrix in its arena: f32 [Np][Kp], then hi, then lo.
struct PackLayout {
    int N, K, Np, Kp;
    size_t cnt, off_hi, off_lo, bytes;
    PackLayout(int R, int C, bool tr) {
        N = tr ? C : R;
        K = tr ? R : C;
        Np = round_up(N, NCH);
        Kp = round_up(K, 32);
        cnt = (size_t)Np * Kp;
        off_hi = (cnt * sizeof(float) + 255) & ~size_t(255);
        off_lo = off_hi + ((cnt * sizeof(__bf16) + 255) & ~size_t(255));
        bytes = off_lo + ((cnt * sizeof(__bf16) + 255) & ~size_t(255));
    }
};

size_t packed_bytes(int R, int C, bool transpose) { return PackLayout(R, C, transpose).bytes; }

__global__ void k_pack(const float *__restrict__ W, int C, bool tr, int N, int K, int Np, int Kp, bool parts3,
                       float *__restrict__ f, __bf16 *__restrict__ hi, __bf16 *__restrict__ lo) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)Np * Kp) return;
    const int n = (int)(idx / Kp), kp = (int)(idx % Kp);
    // parts3: block 3 b + p of the packed k is block b of part p (K / 3 wide)
    const int k = parts3 && kp < K ? (kp / 32) % 3 * (K / 3) + (kp / 96) * 32 + kp % 32 : kp;
    float v = 0.f;
    if (n < N && k < K) v = tr ? W[(long)k * C + n] : W[(long)n * C + k];
    f[idx] = v;
    const __bf16 h = (__bf16)v;
    hi[idx] = h;
    lo[idx] = (__bf16)(v - (float)h);
}

int pack_weight(hipStream_t s, const float *W, int R, int C, bool transpose, void *arena, PackedW *out,
                bool parts3) {
    const PackLayout L(R, C, transpose);
    if (parts3 && (L.K % 96 || L.Kp != L.K)) return -1;
    char *b = reinterpret_cast<char *>(arena);
    float *f = reinterpret_cast<float *>(b);
    __bf16 *hi = reinterpret_cast<__bf16 *>(b + L.off_hi);
    __bf16 *lo = reinterpret_cast<__bf16 *>(b + L.off_lo);
    k_pack<<<(unsigned)((L.cnt + 255) / 256), 256, 0, s>>>(W, C, transpose, L.N, L.K, L.Np, L.Kp, parts3, f, hi,
                                                           lo);
    if (hipGetLastError() != hipSuccess) return -5;
    PackedW p;
    p.N = L.N;
    p.K = L.K;
    p.Np = L.Np;
    p.Kp = L.Kp;
    p.f32 = f;
    p.hi = hi;
    p.lo = lo;
    *out = p;
    return 0;
}

// LDS image of one (128-column x KC) stage of B: bf16 hi rows then lo rows
// (P >= 1), or FP32 rows (P = 0); rows padded to spread the banks.
template <int P>
struct Stage {
    static constexpr int KC = 64;                   // k-columns per stage
    static constexpr int LDH = KC + 8;              // bf16 elements per LDS row
    static constexpr int LDF = KC + 4;              // floats per LDS row
};
constexpr int LDC = NCH + 4;  // floats per row of the output tile parked in LDS
template <int P>
struct GemmLds {
    static constexpr int B_BYTES =
        P == 0 ? NCH * Stage<P>::LDF * 4 : NCH * Stage<P>::LDH * 2 * (P == 2 ? 2 : 1);
    static constexpr int C_BYTES = GW * 16 * LDC * 4;
    static constexpr int BYTES = B_BYTES > C_BYTES ? B_BYTES : C_BYTES;
};

// Waves per SIMD the register budget is sized for: the A slice held in
// registers grows with K.  FP32 slices take twice the registers of bf16
// hi + lo, so FP32 GEMMs with K > 128 leave the epilogue operand to the
// epilogue instead of prefetching it.
template <int P, int KS>
struct GemmWaves {
    static constexpr int N = KS <= 4 ? 3 : 2;
    static constexpr bool RPRE = !(P == 0 && KS > 4);
};
// ---------------------------------------------------------------------------
// Building blocks shared by the single GEMM and the two-GEMM chain.
// ---------------------------------------------------------------------------

// The wave's 16 x (32 KS) slice of an A operand in MFMA operand form: block s
// covers k = 32 s .. 32 s + 31 (bf16 forms: lane (c, g) holds k = 32 s + 8 g
// .. +7 as hi and lo; FP32: k = 32 s + 16 h + 4 g .. +3 for h = 0, 1).
template <int P, int KS>
struct AOp {
    v8bf hi[KS], lo[KS];
    v4f f[KS][2];
    // get4(k): the four values of this lane's row at k .. k+3 (zeros past K)
    template <class Get4>
    __device__ __forceinline__ void load(int g, Get4 get4) {
#pragma unroll
        for (int s = 0; s < KS; s++) {
            if constexpr (P >= 1) {
                const v4f x = get4(32 * s + 8 * g), y = get4(32 * s + 8 * g + 4);
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const float a = q < 4 ? x[q] : y[q - 4];
                    hi[s][q] = (__bf16)a;
                    if (P == 2) lo[s][q] = (__bf16)(a - (float)hi[s][q]);
                }
            } else {
#pragma unroll
                for (int h = 0; h < 2; h++) f[s][h] = get4(32 * s + 16 * h + 4 * g);
            }
        }
    }
    // this lane's row of a row-major operand with K columns (zeros past K and
    // on rows past the end).  With K a multiple of 4 each piece is one
    // 16-byte load, its address clamped in bounds and its value selected
    // away past K, so no branch separates the loads and they are all in
    // flight together.
    __device__ __forceinline__ void load_row(int g, const float *Ar, int K, bool rowok) {
        if ((K & 3) == 0) {
            load(g, [&](int k) {
                const v4f x = *reinterpret_cast<const v4f *>(Ar + min(k, K - 4));
                return (rowok && k < K) ? x : v4f{0.f, 0.f, 0.f, 0.f};
            });
        } else {
            load(g, [&](int k) {
                if (rowok && k + 4 <= K) return *reinterpret_cast<const v4f *>(Ar + k);
                v4f z;
#pragma unroll
                for (int q = 0; q < 4; q++) z[q] = (rowok && k + q < K) ? Ar[k + q] : 0.f;
                return z;
            });
        }
    }
    // block s from the lane's two 4-value pieces: k = 32 s + koff(g, 0) and
    // 32 s + koff(g, 1)
    static __device__ __forceinline__ int koff(int g, int h) { return P >= 1 ? 8 * g + 4 * h : 16 * h + 4 * g; }
    __device__ __forceinline__ void put(int s, v4f x, v4f y) {
        if constexpr (P >= 1) {
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const float a = q < 4 ? x[q] : y[q - 4];
                hi[s][q] = (__bf16)a;
                if (P == 2) lo[s][q] = (__bf16)(a - (float)hi[s][q]);
            }
        } else {
            f[s][0] = x;
            f[s][1] = y;
        }
    }
};

// acc[t] (columns n0 + 16 t .. n0 + 16 t + 15) += A[16 rows][0 .. K) B[0 .. K)[n0 .. n0 + 127].
// B moves through LDS in stages of KC k-columns: the registers of the next
// stage are loaded from L2 while the current stage is multiplied.  Each
// thread takes a fixed, unrolled share, so all loads of a stage are in
// flight together.  Starts with a workgroup barrier (LDS may still be read).
// NT: the number of 16-column tiles computed (the leading ones; a product
// whose B has at most 16 NT columns needs no more).
template <int P, int KS, int NT = CT, int G = GW>
__device__ __forceinline__ void mma_pass(char *lds, const PackedW &B, int n0, int K, const AOp<P, KS> &a,
                                         v4f *acc, int k0 = 0) {
    constexpr int KC = Stage<P>::KC, LDH = Stage<P>::LDH, LDF = Stage<P>::LDF;
    constexpr int VR = P >= 1 ? KC / 8 : KC / 4;   // 16-byte vectors per row of a stage
    constexpr int IT = NCH * VR / (64 * G);
    static_assert(IT * 64 * G == NCH * VR, "stage split");
    constexpr int EV = P >= 1 ? 8 : 4;             // k-elements per vector
    const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
    v8bf sh[IT], sl[IT];
    v4f sf[IT];
    // (k0: the operand's k = 0 is B's row k0)
    auto fetch = [&](int kc) {
        const int kcl = min(KC, B.Kp - k0 - kc);
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int idx = threadIdx.x + 64 * G * it, n = idx / VR, q = idx % VR;
            if (EV * q < kcl) {
                const long go = (long)(n0 + n) * B.Kp + k0 + kc + EV * q;
                if constexpr (P >= 1) {
                    sh[it] = *reinterpret_cast<const v8bf *>(B.hi + go);
                    if (P == 2) sl[it] = *reinterpret_cast<const v8bf *>(B.lo + go);
                } else {
                    sf[it] = gld4(B.f32 + go);
                }
            }
        }
    };
    auto park = [&](int kc) {
        const int kcl = min(KC, B.Kp - k0 - kc);
#pragma unroll
        for (int it = 0; it < IT; it++) {
            const int idx = threadIdx.x + 64 * G * it, n = idx / VR, q = idx % VR;
            if (EV * q < kcl) {
                if constexpr (P >= 1) {
                    __bf16 *h = reinterpret_cast<__bf16 *>(lds) + n * LDH + 8 * q;
                    *reinterpret_cast<v8bf *>(h) = sh[it];
                    if (P == 2) *reinterpret_cast<v8bf *>(h + NCH * LDH) = sl[it];
                } else {
                    *reinterpret_cast<v4f *>(reinterpret_cast<float *>(lds) + n * LDF + 4 * q) = sf[it];
                }
            }
        }
    };
    fetch(0);
#pragma unroll
    for (int kc = 0; kc < KS * 32; kc += KC) {
        if (kc >= K) break;
        __syncthreads();   // every wave is done with the previous use of LDS
        park(kc);
        __syncthreads();
        if (kc + KC < K) fetch(kc + KC);
#pragma unroll
        for (int j = 0; j < KC / 32; j++) {
            const int s = kc / 32 + j;
            if (s >= KS || 32 * s >= K) break;
            if constexpr (P >= 1) {
                const __bf16 *bb = reinterpret_cast<const __bf16 *>(lds) + c16 * LDH + 32 * j + 8 * g;
#pragma unroll
                for (int t = 0; t < NT; t++) {
                    const v8bf bh = *reinterpret_cast<const v8bf *>(bb + 16 * t * LDH);
                    if constexpr (P == 2) {
                        const v8bf bl = *reinterpret_cast<const v8bf *>(bb + 16 * t * LDH + NCH * LDH);
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.lo[s], bh, acc[t], 0, 0, 0);
                        acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi[s], bl, acc[t], 0, 0, 0);
                    }
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a.hi[s], bh, acc[t], 0, 0, 0);
                }
            } else {
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    const float *bb = reinterpret_cast<const float *>(lds) + c16 * LDF + 32 * j + 16 * h + 4 * g;
#pragma unroll
                    for (int t = 0; t < NT; t++) {
                        const v4f b = *reinterpret_cast<const v4f *>(bb + 16 * t * LDF);
#pragma unroll
                        for (int q = 0; q < 4; q++)
                            acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(a.f[s][h][q], b[q], acc[t], 0, 0, 0);
                    }
                }
            }
        }
    }
}

// Parks the wave's 16 x 128 accumulator tile in LDS (row-major, stride LDC)
// and returns it.  The epilogue then reads it back by rows, so C (and its
// second operand) move as whole rows in 16-byte vectors: lane + 64 it covers
// row (lane + 64 it) / 32, columns 4 ((lane + 64 it) % 32) .. +3.
template <int NT = CT>
__device__ __forceinline__ float *park_tile(char *lds, const v4f *acc) {
    const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
    __syncthreads();   // every wave is done with the B stages in LDS
    float *ct = reinterpret_cast<float *>(lds) + (threadIdx.x >> 6) * 16 * LDC;
#pragma unroll
    for (int t = 0; t < NT; t++)
#pragma unroll
        for (int r = 0; r < 4; r++) ct[(4 * g + r) * LDC + 16 * t + c16] = acc[t][r];
    __syncthreads();
    return ct;
}
constexpr int EIT = 16 * NCH / 4 / 64;   // epilogue vectors per lane

// n = sqrt(eps + sum_d x_d^2) per component, the products added in d order
// by fused multiply-adds
__device__ __forceinline__ v4f norm4(v4f x0, v4f x1, v4f x2, float eps) {
    v4f o;
#pragma unroll
    for (int q = 0; q < 4; q++)
        o[q] = sqrtf(__builtin_fmaf(x2[q], x2[q], __builtin_fmaf(x1[q], x1[q], __builtin_fmaf(x0[q], x0[q], eps))));
    return o;
}

__device__ __forceinline__ v4f silu4(v4f h) {
    v4f o;
#pragma unroll
    for (int q = 0; q < 4; q++) o[q] = h[q] * g_sigmoid(h[q]);
    return o;
}
__device__ __forceinline__ v4f dsilu4(v4f x, v4f h) {
    v4f o;
#pragma unroll
    for (int q = 0; q < 4; q++) {
        const float sg = g_sigmoid(h[q]);
        o[q] = x[q] * (sg * (1.0f + h[q] * (1.0f - sg)));
    }
    return o;
}

// The epilogue's second operand of this wave's rows m0 .. m0+15 and columns
// n0 .. n0 + ncols - 1, in the epilogue's row layout.
__device__ __forceinline__ void fetch_rows(const float *R, int ldr, long m0, int n0, int ncols, int M, v4f *rr) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int it = 0; it < EIT; it++) {
        const int idx = lane + 64 * it, row = idx / (NCH / 4), c4 = 4 * (idx % (NCH / 4));
        const long m = m0 + row;
        if (m < M && c4 < ncols) rr[it] = gld4(R + m * ldr + n0 + c4);
    }
}

// ---------------------------------------------------------------------------
// C = epilogue(A B), one 128-column chunk (blockIdx.y) per workgroup.
// ---------------------------------------------------------------------------
template <int P, int EPI, int KS>
__global__ void __launch_bounds__(64 * GW) __attribute__((amdgpu_waves_per_eu(GemmWaves<P, KS>::N))) k_gemm(const float *__restrict__ A, int lda, PackedW B, float *C, int ldc,
                                                  int M, const float *__restrict__ bias, float *__restrict__ C2,
                                                  int ldc2, const float *R, int ldr, const int *Mc) {
    __shared__ __attribute__((aligned(16))) char lds[GemmLds<P>::BYTES];
    // a row count on the device (Mc) bounds M: the grid is sized for M
    if (Mc) M = min(M, *Mc);
    // grid.x is padded to a multiple of 8 (the column chunks of one row block
    // then run on one XCD and share its L2): padding workgroups leave at once
    if ((long)blockIdx.x * GW * 16 >= M) return;
    const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
    const long m0 = ((long)blockIdx.x * GW + (threadIdx.x >> 6)) * 16;
    const int n0 = blockIdx.y * NCH;
    const long arow = m0 + c16;
    const bool rowok = arow < M;
    const float *Ar = A + (rowok ? arow : 0) * (long)lda;
    const int K = B.K;
    // the wave's 16 x K slice of A, loaded at once (all loads in flight together)
    AOp<P, KS> a;
    a.load_row(g, Ar, K, rowok);
    // the epilogue's second operand (R) is fetched now, so its latency
    // overlaps the products
    const int ncols = min(NCH, B.N - n0);   // a multiple of 4
    constexpr bool RPRE = GemmWaves<P, KS>::RPRE && (EPI == GE_DSILU || EPI == GE_ADD);
    v4f rr[EIT];
    if constexpr (RPRE) fetch_rows(R, ldr, m0, n0, ncols, M, rr);
    v4f acc[CT];
#pragma unroll
    for (int t = 0; t < CT; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    mma_pass<P, KS>(lds, B, n0, K, a, acc);
    const float *ct = park_tile(lds, acc);
#pragma unroll
    for (int it = 0; it < EIT; it++) {
        const int idx = lane + 64 * it, row = idx / (NCH / 4), c4 = 4 * (idx % (NCH / 4));
        const long m = m0 + row;
        if (m >= M || c4 >= ncols) continue;
        const int n = n0 + c4;
        const v4f x = *reinterpret_cast<const v4f *>(ct + row * LDC + c4);
        v4f o;
        if constexpr (EPI == GE_STORE) {
            o = x;
        } else if constexpr (EPI == GE_BIAS || EPI == GE_BIAS_SILU) {
#pragma unroll
            for (int q = 0; q < 4; q++) o[q] = x[q] + bias[n + q];
            if constexpr (EPI == GE_BIAS_SILU) *reinterpret_cast<v4f *>(C2 + m * ldc2 + n) = silu4(o);
        } else if constexpr (EPI == GE_DSILU) {
            o = dsilu4(x, RPRE ? rr[it] : gld4(R + m * ldr + n));
        } else {
            o = (RPRE ? rr[it] : gld4(R + m * ldr + n)) + x;
        }
        *reinterpret_cast<v4f *>(C + m * ldc + n) = o;
    }
}

// ---------------------------------------------------------------------------
// Two chained products, C2 = epi2(act(A B1) B2), with act the bias + SiLU
// (E1 = GE_BIAS_SILU; the pre-activation also goes to C1) or the SiLU'
// gate with the saved pre-activation R1 (E1 = GE_DSILU).  The intermediate
// (at most 128 columns) stays in the workgroup's LDS tile and becomes the
// second product's A operand; all column chunks of B2 run in the workgroup.
// ---------------------------------------------------------------------------
template <int P, int E1, int E2, int KS>
__global__ void __launch_bounds__(64 * GW) __attribute__((amdgpu_waves_per_eu(2)))
k_gemm_chain(const float *__restrict__ A, int lda, PackedW B1, float *__restrict__ C1, int ldc1,
             const float *__restrict__ bias1, const float *__restrict__ R1, int ldr1, PackedW B2,
             float *__restrict__ C2, int ldc2, const float *__restrict__ bias2, const float *__restrict__ R2, int ldr2,
             int M, int Fu, const float *__restrict__ sn, const float *__restrict__ v1,
             const float *__restrict__ UV, float *__restrict__ s2, float *__restrict__ v2, float *__restrict__ gUV,
             const float *__restrict__ gv, float eps, const int *Mc) {
    __shared__ __attribute__((aligned(16))) char lds[GemmLds<P>::BYTES];
    if (Mc) M = min(M, *Mc);
    if ((long)blockIdx.x * GW * 16 >= M) return;   // the whole workgroup leaves
    const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
    const long m0 = ((long)blockIdx.x * GW + (threadIdx.x >> 6)) * 16;
    const long arow = m0 + c16;
    const bool rowok = arow < M;
    const float *Ar = A + (rowok ? arow : 0) * (long)lda;
    const int K1 = B1.K, N1 = B1.N;
    float *ct;
    {
        v4f rr[EIT];
        v4f acc[CT];
#pragma unroll
        for (int t = 0; t < CT; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
        if constexpr (E2 == GE_UPDATE_ADJ) {
            // da of the gated update (K1 = 3F = 32 KS), in pieces of two
            // 32-feature blocks, each formed just before it is multiplied: B1
            // is packed with the parts of a feature block adjacent (block
            // 3 b + p = part p of features 32 b .. 32 b + 31), so a piece is
            // six consecutive blocks of k.  All three parts of four features
            // come from one set of loads, and dUv of those features is written
            // on the way.
            constexpr int SP = KS / 3;   // feature blocks: 2 (F = 64) or 4 (F = 128)
            static_assert(3 * SP == KS && SP % 2 == 0, "pieces of two feature blocks");
            const v4f z = v4f{0.f, 0.f, 0.f, 0.f};
            // dv2 = 0 (gv null) reads UV (in bounds) scaled by zero, so no
            // branch separates the loads
            const float gsc = gv ? 1.f : 0.f;
            const float *gvp = gv ? gv : UV;
#pragma unroll
            for (int pc = 0; pc < SP / 2; pc++) {
                AOp<P, 6> a;
                if (!rowok) {
#pragma unroll
                    for (int b = 0; b < 6; b++) a.put(b, z, z);
                } else {
#pragma unroll
                    for (int i = 0; i < 2; i++) {
                        v4f p0[2], p1[2], p2[2];
#pragma unroll
                        for (int h = 0; h < 2; h++) {
                            const int f = 32 * (2 * pc + i) + AOp<P, 6>::koff(g, h);
                            const v4f gs = gld4(R2 + arow * ldr2 + f);
                            const v4f avv = gld4(Ar + f), gasv = gs * gld4(Ar + Fu + f);
                            const float *uv = UV + arow * 6 * Fu + f;   // rows (3 m + d) of [Uv | Vv]
                            v4f gavv = z, dot = z;
#pragma unroll
                            for (int d = 0; d < 3; d++) {
                                const v4f u = gld4(uv + d * 2 * Fu), w = gld4(uv + d * 2 * Fu + Fu);
                                const v4f gvd = gld4(gvp + (3 * arow + d) * Fu + f) * gsc;
                                gavv += gvd * u;   // dE/da_vv = sum_d dv2_d o Uv_d
                                dot += u * w;
                                // dUv_d = dv2_d o a_vv + ds2 a_sv Vv_d
                                *reinterpret_cast<v4f *>(gUV + (3 * arow + d) * 2 * Fu + f) = gvd * avv + gasv * w;
                            }
                            p0[h] = gavv;
                            p1[h] = gs * dot;   // dE/da_sv = ds2 <Uv, Vv>
                            p2[h] = gs;         // dE/da_ss = ds2
                        }
                        a.put(3 * i, p0[0], p0[1]);
                        a.put(3 * i + 1, p1[0], p1[1]);
                        a.put(3 * i + 2, p2[0], p2[1]);
                    }
                }
                mma_pass<P, 6>(lds, B1, 0, 192, a, acc, 192 * pc);
            }
            fetch_rows(R1, ldr1, m0, 0, N1, M, rr);
        } else if constexpr (E2 == GE_UPDATE_N) {
            // [s1 | n] (K1 = 2F = 32 KS): s1 from A, n from the Vv rows
            constexpr int SP = KS / 2;
            static_assert(2 * SP == KS, "two parts of whole blocks");
            AOp<P, KS> a;
            const v4f z = v4f{0.f, 0.f, 0.f, 0.f};
            if (!rowok) {
#pragma unroll
                for (int b = 0; b < KS; b++) a.put(b, z, z);
            } else {
#pragma unroll
                for (int b = 0; b < KS; b++) {
                    v4f x[2];
#pragma unroll
                    for (int h = 0; h < 2; h++) {
                        const int f = 32 * (b % SP) + AOp<P, KS>::koff(g, h);
                        if (b < SP) {
                            x[h] = gld4(Ar + f);
                        } else {
                            const float *vv = UV + arow * 6 * Fu + Fu + f;   // Vv of rows 3 m + d
                            x[h] = norm4(gld4(vv), gld4(vv + 2 * Fu), gld4(vv + 4 * Fu), eps);
                        }
                    }
                    a.put(b, x[0], x[1]);
                }
            }
            mma_pass<P, KS>(lds, B1, 0, K1, a, acc);
        } else {
            AOp<P, KS> a;
            a.load_row(g, Ar, K1, rowok);
            if constexpr (E1 == GE_DSILU) fetch_rows(R1, ldr1, m0, 0, N1, M, rr);
            mma_pass<P, KS>(lds, B1, 0, K1, a, acc);
        }
        ct = park_tile(lds, acc);
        // the activation, written back into the tile (zeros outside the valid
        // rows and columns, which the second product then reads as padding)
#pragma unroll
        for (int it = 0; it < EIT; it++) {
            const int idx = lane + 64 * it, row = idx / (NCH / 4), c4 = 4 * (idx % (NCH / 4));
            const long m = m0 + row;
            v4f y = v4f{0.f, 0.f, 0.f, 0.f};
            if (m < M && c4 < N1) {
                const v4f x = *reinterpret_cast<const v4f *>(ct + row * LDC + c4);
                if constexpr (E1 == GE_BIAS_SILU) {
                    v4f h;
#pragma unroll
                    for (int q = 0; q < 4; q++) h[q] = x[q] + bias1[c4 + q];
                    *reinterpret_cast<v4f *>(C1 + m * ldc1 + c4) = h;
                    y = silu4(h);
                } else {
                    y = dsilu4(x, rr[it]);
                }
            }
            *reinterpret_cast<v4f *>(ct + row * LDC + c4) = y;
        }
        __builtin_amdgcn_wave_barrier();   // each wave reads back only its own tile
    }
    AOp<P, 4> a2;   // K2 = N1 <= 128
    a2.load(g, [&](int k) { return *reinterpret_cast<const v4f *>(ct + c16 * LDC + k); });
    const int K2 = B2.K;
    for (int n0 = 0; n0 < B2.N; n0 += NCH) {
        const int ncols = min(NCH, B2.N - n0);
        v4f rr[EIT];
        if constexpr (E2 == GE_ADD) fetch_rows(R2, ldr2, m0, n0, ncols, M, rr);
        v4f acc[CT];
#pragma unroll
        for (int t = 0; t < CT; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
        mma_pass<P, 4>(lds, B2, n0, K2, a2, acc);
        const float *ct2 = park_tile(lds, acc);
        if constexpr (E2 == GE_UPDATE || E2 == GE_UPDATE_N || E2 == GE_UPDATE_ADJ) {
            // the update epilogues load several operands per vector: a short
            // unroll keeps them from being hoisted all at once
            constexpr int UPD_UNROLL = 2;
#pragma unroll UPD_UNROLL
            for (int it = 0; it < EIT; it++) {
                const int idx = lane + 64 * it, row = idx / (NCH / 4), c4 = 4 * (idx % (NCH / 4));
                const long m = m0 + row;
                if (m >= M || c4 >= ncols) continue;
                const int n = n0 + c4;
                v4f o = *reinterpret_cast<const v4f *>(ct2 + row * LDC + c4);
                // part of the output: F columns each, features f .. f+3
                const int part = n / Fu, f = n - part * Fu;
                if constexpr (E2 == GE_UPDATE || E2 == GE_UPDATE_N) {
                    // part 0: a_vv, part 1: a_sv, part 2: a_ss
#pragma unroll
                    for (int q = 0; q < 4; q++) o[q] += bias2[n + q];
                    const float *uv = UV + m * 6 * Fu + f;   // rows (3m + d) of [Uv | Vv]
                    if (part == 0) {
                        *reinterpret_cast<v4f *>(C2 + m * ldc2 + n) = o;
                        if (v2)
#pragma unroll
                            for (int d = 0; d < 3; d++) {
                                const long b = m * 3 * Fu + d * Fu + f;
                                *reinterpret_cast<v4f *>(v2 + b) = gld4(v1 + b) + o * gld4(uv + d * 2 * Fu);
                            }
                    } else if (part == 1) {
                        *reinterpret_cast<v4f *>(C2 + m * ldc2 + n) = o;
                        v4f dot = gld4(uv) * gld4(uv + Fu);
#pragma unroll
                        for (int d = 1; d < 3; d++) dot += gld4(uv + d * 2 * Fu) * gld4(uv + d * 2 * Fu + Fu);
                        *reinterpret_cast<v4f *>(s2 + m * Fu + f) = gld4(sn + m * 2 * Fu + f) + o * dot;
                    } else {
                        // part 1 of these features was written in an earlier chunk
                        // (by a thread of this workgroup, before the barrier)
                        float *sp = s2 + m * Fu + f;
                        *reinterpret_cast<v4f *>(sp) = gld4(sp) + o;
                    }
                } else {
                    // part 0: ds1, part 1: dn
                    if (part == 0) {
                        *reinterpret_cast<v4f *>(C2 + m * ldc2 + n) = gld4(R2 + m * ldr2 + n) + o;
                    } else {
                        // dVv_d = ds2 a_sv Uv_d + (dn / n) Vv_d
                        const float *uv = UV + m * 6 * Fu + f;   // rows (3 m + d) of [Uv | Vv]
                        const v4f vv[3] = {gld4(uv + Fu), gld4(uv + 3 * Fu), gld4(uv + 5 * Fu)};
                        const v4f gn = o / norm4(vv[0], vv[1], vv[2], eps);
                        const v4f gasv = gld4(R2 + m * ldr2 + f) * gld4(A + m * lda + Fu + f);
#pragma unroll
                        for (int d = 0; d < 3; d++) {
                            const v4f gvu = gasv * gld4(uv + d * 2 * Fu);
                            *reinterpret_cast<v4f *>(gUV + (3 * m + d) * 2 * Fu + Fu + f) = gvu + gn * vv[d];
                        }
                    }
                }
            }
        } else {
            // (three more loads per vector with the v o phi_vv rows: a shorter unroll)
            constexpr int GEN_UNROLL = E2 == GE_BIAS_VPROD ? 4 : EIT;
#pragma unroll GEN_UNROLL
            for (int it = 0; it < EIT; it++) {
                const int idx = lane + 64 * it, row = idx / (NCH / 4), c4 = 4 * (idx % (NCH / 4));
                const long m = m0 + row;
                if (m >= M || c4 >= ncols) continue;
                const int n = n0 + c4;
                v4f o = *reinterpret_cast<const v4f *>(ct2 + row * LDC + c4);
                if constexpr (E2 == GE_BIAS || E2 == GE_BIAS_VPROD) {
#pragma unroll
                    for (int q = 0; q < 4; q++) o[q] += bias2[n + q];
                } else if constexpr (E2 == GE_ADD) {
                    o += rr[it];
                }
                *reinterpret_cast<v4f *>(C2 + m * ldc2 + n) = o;
                if constexpr (E2 == GE_BIAS_VPROD) {
                    if (n < Fu)
#pragma unroll
                        for (int d = 0; d < 3; d++) {
                            const long b = (3 * m + d) * Fu + n;
                            *reinterpret_cast<v4f *>(v2 + b) = gld4(v1 + b) * o;
                        }
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// A bias-free SiLU MLP over rows with every hidden layer kept on chip:
//   forward  C = h_n Wo^T,  h_q = silu(h_(q-1) W_q^T),  h_0 = X
//   adjoint  dE/dX from dE/dC, the hidden layers recomputed per tile and
//            their pre-activations held in registers (in the MFMA output
//            layout, so the SiLU' gates are elementwise on the accumulators)
// Hidden widths are at most 16 HT (HT tiles, HT / 2 32-wide k-blocks; this
// build instantiates HT = 4, widths up to 64), the input at most 32 wide.  Each wave owns 16 rows; the tile parked in LDS
// between layers becomes the next product's A operand.
// ---------------------------------------------------------------------------
#ifndef MLP_GW
#define MLP_GW 4
#endif
constexpr int MG = MLP_GW;   // waves per workgroup of the fused MLP kernels (rows 16 MG per workgroup;
                             // eight measured slower than four on MACE's radial MLPs)
template <int P>
struct MlpLds {
    static constexpr int C_BYTES = MG * 16 * LDC * 4;
    static constexpr int BYTES = GemmLds<P>::B_BYTES > C_BYTES ? GemmLds<P>::B_BYTES : C_BYTES;
};

template <int P, int HT>
__device__ __forceinline__ void silu_tile(float *ct, int N) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int it = 0; it < EIT; it++) {
        const int idx = lane + 64 * it, row = idx / (NCH / 4), c4 = 4 * (idx % (NCH / 4));
        if (c4 >= 16 * HT) continue;
        v4f *p = reinterpret_cast<v4f *>(ct + row * LDC + c4);
        *p = c4 < N ? silu4(*p) : v4f{0.f, 0.f, 0.f, 0.f};
    }
    __builtin_amdgcn_wave_barrier();   // each wave reads back only its own tile
}

template <int P, int NH, int HT>
__global__ void __launch_bounds__(64 * MG) __attribute__((amdgpu_waves_per_eu(2)))
k_mlp_fwd(const float *__restrict__ X, int ldx, EdgeMlp W, float *__restrict__ C, int ldc, int M, const int *Mc) {
    __shared__ __attribute__((aligned(16))) char lds[MlpLds<P>::BYTES];
    if (Mc) M = min(M, *Mc);
    if ((long)blockIdx.x * MG * 16 >= M) return;   // the whole workgroup leaves
    const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
    const long m0 = ((long)blockIdx.x * MG + (threadIdx.x >> 6)) * 16;
    const long arow = m0 + c16;
    const bool rowok = arow < M;
    const float *Xr = X + (rowok ? arow : 0) * (long)ldx;
    constexpr int KH = HT / 2;
    AOp<P, KH> a;
    {
        const int K0 = W.f[0].K;
        AOp<P, 1> x;
        x.load(g, [&](int k) {
            v4f z;
#pragma unroll
            for (int q = 0; q < 4; q++) z[q] = (rowok && k + q < K0) ? Xr[k + q] : 0.f;
            return z;
        });
        v4f acc[HT];
#pragma unroll
        for (int t = 0; t < HT; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
        mma_pass<P, 1, HT, MG>(lds, W.f[0], 0, K0, x, acc);
        float *ct = park_tile<HT>(lds, acc);
        silu_tile<P, HT>(ct, W.f[0].N);
        a.load(g, [&](int k) { return *reinterpret_cast<const v4f *>(ct + c16 * LDC + k); });
    }
#pragma unroll
    for (int q = 1; q < NH; q++) {
        v4f acc[HT];
#pragma unroll
        for (int t = 0; t < HT; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
        mma_pass<P, KH, HT, MG>(lds, W.f[q], 0, W.f[q].K, a, acc);
        float *ct = park_tile<HT>(lds, acc);
        silu_tile<P, HT>(ct, W.f[q].N);
        a.load(g, [&](int k) { return *reinterpret_cast<const v4f *>(ct + c16 * LDC + k); });
    }
    const PackedW &Wo = W.f[NH];
    for (int n0 = 0; n0 < Wo.N; n0 += NCH) {
        const int ncols = min(NCH, Wo.N - n0);
        v4f acc[CT];
#pragma unroll
        for (int t = 0; t < CT; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
        mma_pass<P, KH, CT, MG>(lds, Wo, n0, Wo.K, a, acc);
        const float *ct = park_tile(lds, acc);
#pragma unroll
        for (int it = 0; it < EIT; it++) {
            const int idx = lane + 64 * it, row = idx / (NCH / 4), c4 = 4 * (idx % (NCH / 4));
            const long m = m0 + row;
            if (m >= M || c4 >= ncols) continue;
            *reinterpret_cast<v4f *>(C + m * ldc + n0 + c4) = *reinterpret_cast<const v4f *>(ct + row * LDC + c4);
        }
    }
}

// acc *= SiLU'(pre), elementwise in the MFMA output layout
template <int HT>
__device__ __forceinline__ void dsilu_acc(v4f *acc, const v4f *pre) {
#pragma unroll
    for (int t = 0; t < HT; t++) acc[t] = dsilu4(acc[t], pre[t]);
}

template <int P, int NH, int HT, int KSG>
__global__ void __launch_bounds__(64 * MG) __attribute__((amdgpu_waves_per_eu(2)))
k_mlp_bwd(const float *__restrict__ X, int ldx, EdgeMlp W, const float *__restrict__ GC, int ldgc, float *GX,
          int ldgx, int add, int M, const int *Mc) {
    __shared__ __attribute__((aligned(16))) char lds[MlpLds<P>::BYTES];
    if (Mc) M = min(M, *Mc);
    if ((long)blockIdx.x * MG * 16 >= M) return;
    const int lane = threadIdx.x & 63, c16 = lane & 15, g = lane >> 4;
    const long m0 = ((long)blockIdx.x * MG + (threadIdx.x >> 6)) * 16;
    const long arow = m0 + c16;
    const bool rowok = arow < M;
    constexpr int KH = HT / 2;
    // dE/dC of the wave's rows, loaded first so that its latency overlaps the recompute
    AOp<P, KSG> ga;
    {
        const float *Gr = GC + (rowok ? arow : 0) * (long)ldgc;
        const int NO = W.f[NH].N;
        ga.load_row(g, Gr, NO, rowok);
    }
    // forward recompute: pre-activations of every hidden layer
    v4f pre[NH][HT];
    AOp<P, KH> a;
    {
        const float *Xr = X + (rowok ? arow : 0) * (long)ldx;
        const int K0 = W.f[0].K;
        AOp<P, 1> x;
        x.load(g, [&](int k) {
            v4f z;
#pragma unroll
            for (int q = 0; q < 4; q++) z[q] = (rowok && k + q < K0) ? Xr[k + q] : 0.f;
            return z;
        });
#pragma unroll
        for (int t = 0; t < HT; t++) pre[0][t] = v4f{0.f, 0.f, 0.f, 0.f};
        mma_pass<P, 1, HT, MG>(lds, W.f[0], 0, K0, x, pre[0]);
    }
#pragma unroll
    for (int q = 1; q < NH; q++) {
        float *ct = park_tile<HT>(lds, pre[q - 1]);
        silu_tile<P, HT>(ct, W.f[q - 1].N);
        a.load(g, [&](int k) { return *reinterpret_cast<const v4f *>(ct + c16 * LDC + k); });
#pragma unroll
        for (int t = 0; t < HT; t++) pre[q][t] = v4f{0.f, 0.f, 0.f, 0.f};
        mma_pass<P, KH, HT, MG>(lds, W.f[q], 0, W.f[q].K, a, pre[q]);
    }
    // dE/dh of the last hidden layer through the output matrix, then down
    v4f acc[HT];
#pragma unroll
    for (int t = 0; t < HT; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
    mma_pass<P, KSG, HT, MG>(lds, W.a[NH], 0, W.a[NH].K, ga, acc);
    dsilu_acc<HT>(acc, pre[NH - 1]);
#pragma unroll
    for (int q = NH - 1; q >= 1; q--) {
        float *ct = park_tile<HT>(lds, acc);
        __builtin_amdgcn_wave_barrier();
        a.load(g, [&](int k) { return *reinterpret_cast<const v4f *>(ct + c16 * LDC + k); });
#pragma unroll
        for (int t = 0; t < HT; t++) acc[t] = v4f{0.f, 0.f, 0.f, 0.f};
        mma_pass<P, KH, HT, MG>(lds, W.a[q], 0, W.a[q].K, a, acc);
        dsilu_acc<HT>(acc, pre[q - 1]);
    }
    // dE/dX = dE/dP_0 W_0 (at most 16 columns)
    float *ct = park_tile<HT>(lds, acc);
    __builtin_amdgcn_wave_barrier();
    a.load(g, [&](int k) { return *reinterpret_cast<const v4f *>(ct + c16 * LDC + k); });
    v4f gx[1] = {v4f{0.f, 0.f, 0.f, 0.f}};
    mma_pass<P, KH, 1, MG>(lds, W.a[0], 0, W.a[0].K, a, gx);
    const float *cx = park_tile<1>(lds, gx);
    const int NX = W.a[0].N;
    // 16 rows x 16 columns: lane (row, 4-column group) = (lane / 4, lane % 4)
    const int row = lane >> 2, c4 = 4 * (lane & 3);
    const long m = m0 + row;
    if (m < M && c4 < NX) {
        v4f o = *reinterpret_cast<const v4f *>(cx + row * LDC + c4);
        float *d = GX + m * ldgx + c4;
        if (add) o += gld4(d);
        *reinterpret_cast<v4f *>(d) = o;
    }
}

template <int P, int NH, int HT>
static int mlp_fwd_launch(hipStream_t s, const EdgeMlp &W, const float *X, int ldx, float *C, int ldc, int M,
                          const int *Mc) {
    const unsigned bx = (unsigned)((M + 16 * MG - 1) / (16 * MG));
    k_mlp_fwd<P, NH, HT><<<bx, 64 * MG, 0, s>>>(X, ldx, W, C, ldc, M, Mc);
    return 0;
}

template <int P, int NH, int HT, int KSG>
static int mlp_bwd_launch(hipStream_t s, const EdgeMlp &W, const float *X, int ldx, const float *GC, int ldgc,
                          float *GX, int ldgx, bool add, int M, const int *Mc) {
    const unsigned bx = (unsigned)((M + 16 * MG - 1) / (16 * MG));
    k_mlp_bwd<P, NH, HT, KSG><<<bx, 64 * MG, 0, s>>>(X, ldx, W, GC, ldgc, GX, ldgx, add ? 1 : 0, M, Mc);
    return 0;
}

static bool mlp_shape_ok(const EdgeMlp &W, int *HT) {
    if (W.nh != 3 || W.f[0].K > 32 || W.a[0].N > 16) return false;
    for (int q = 0; q < W.nh; q++)
        if (W.f[q].N > 64) return false;
    *HT = 4;
    return W.f[W.nh].N <= 384;
}

int edge_mlp_forward(hipStream_t s, int precision, const EdgeMlp &W, const float *X, int ldx, float *C, int ldc,
                     int M, const int *Mc) {
    int HT;
    if (M <= 0) return 0;
    if (!mlp_shape_ok(W, &HT)) return -1;
#define MF(P_) mlp_fwd_launch<P_, 3, 4>(s, W, X, ldx, C, ldc, M, Mc)
    if (precision == 0) MF(0);
    else if (precision == 1) MF(1);
    else MF(2);
#undef MF
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

int edge_mlp_adjoint(hipStream_t s, int precision, const EdgeMlp &W, const float *X, int ldx, const float *GC,
                     int ldgc, float *GX, int ldgx, bool add, int M, const int *Mc) {
    int HT;
    if (M <= 0) return 0;
    if (!mlp_shape_ok(W, &HT)) return -1;
    const int NO = W.f[W.nh].N;
#define MB2(P_, HT_)                                                                                          \
    (NO <= 128 ? mlp_bwd_launch<P_, 3, HT_, 4>(s, W, X, ldx, GC, ldgc, GX, ldgx, add, M, Mc)                    \
               : (NO <= 256 ? mlp_bwd_launch<P_, 3, HT_, 8>(s, W, X, ldx, GC, ldgc, GX, ldgx, add, M, Mc)       \
                            : mlp_bwd_launch<P_, 3, HT_, 12>(s, W, X, ldx, GC, ldgc, GX, ldgx, add, M, Mc)))
#define MB(P_) MB2(P_, 4)
    if (precision == 0) MB(0);
    else if (precision == 1) MB(1);
    else MB(2);
#undef MB
#undef MB2
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

template <int P, int EPI, int KS>
static void launch(hipStream_t s, const float *A, int lda, const PackedW &B, float *C, int ldc, int M,
                   const float *bias, float *C2, int ldc2, const float *R, int ldr, const int *Mc) {
    unsigned bx = (unsigned)((M + 16 * GW - 1) / (16 * GW));
    const unsigned by = (unsigned)(B.Np / NCH);
    if (by > 1) bx = (bx + 7) / 8 * 8;
    k_gemm<P, EPI, KS><<<dim3(bx, by), 64 * GW, 0, s>>>(A, lda, B, C, ldc, M, bias, C2, ldc2, R, ldr, Mc);
}

template <int P, int EPI>
static int launch_k(hipStream_t s, const float *A, int lda, const PackedW &B, float *C, int ldc, int M,
                    const float *bias, float *C2, int ldc2, const float *R, int ldr, const int *Mc) {
    if (B.K <= 128) launch<P, EPI, 4>(s, A, lda, B, C, ldc, M, bias, C2, ldc2, R, ldr, Mc);
    else if (B.K <= 256) launch<P, EPI, 8>(s, A, lda, B, C, ldc, M, bias, C2, ldc2, R, ldr, Mc);
    else if (B.K <= 384) launch<P, EPI, 12>(s, A, lda, B, C, ldc, M, bias, C2, ldc2, R, ldr, Mc);
    else return -1;
    return 0;
}

int node_gemm(hipStream_t s, int precision, int epi, const float *A, int lda, const PackedW &B, float *C, int ldc,
              int M, const float *bias, float *C2, int ldc2, const float *R, int ldr, const int *Mc) {
    if (M <= 0 || B.N <= 0 || B.K <= 0) return 0;
    int rc = 0;
#define GL(P_, E_) rc = launch_k<P_, E_>(s, A, lda, B, C, ldc, M, bias, C2, ldc2, R, ldr, Mc)
#define GE(P_)                                   \
    switch (epi) {                               \
        case GE_STORE: GL(P_, GE_STORE); break;   \
        case GE_BIAS: GL(P_, GE_BIAS); break;     \
        case GE_BIAS_SILU: GL(P_, GE_BIAS_SILU); break; \
        case GE_DSILU: GL(P_, GE_DSILU); break;   \
        default: GL(P_, GE_ADD); break;           \
    }
    if (precision == 0) {
        GE(0)
    } else if (precision == 1) {
        GE(1)
    } else {
        GE(2)
    }
#undef GE
#undef GL
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

template <int P, int E1, int E2, int KS>
static void launch_chain(hipStream_t s, const GemmChain &c) {
    const unsigned bx = (unsigned)((c.M + 16 * GW - 1) / (16 * GW));
    k_gemm_chain<P, E1, E2, KS><<<bx, 64 * GW, 0, s>>>(c.A, c.lda, *c.B1, c.C1, c.ldc1, c.bias1, c.R1, c.ldr1, *c.B2,
                                                        c.C2, c.ldc2, c.bias2, c.R2, c.ldr2, c.M, c.F, c.sn, c.v1,
                                                        c.UV, c.s2, c.v2, c.gUV, c.gv, c.eps, c.Mc);
}

template <int P>
static int chain_p(hipStream_t s, const GemmChain &c) {
    const int K = c.B1->K;
    const int ks = K <= 128 ? 4 : (K <= 256 ? 8 : (K <= 384 ? 12 : 0));
#define CL(E1_, E2_)                                                   \
    do {                                                               \
        if (ks == 4) launch_chain<P, E1_, E2_, 4>(s, c);               \
        else if (ks == 8) launch_chain<P, E1_, E2_, 8>(s, c);          \
        else launch_chain<P, E1_, E2_, 12>(s, c);                      \
        return 0;                                                      \
    } while (0)
    if (ks == 0) return -1;
    if (c.e1 == GE_BIAS_SILU && c.e2 == GE_BIAS) CL(GE_BIAS_SILU, GE_BIAS);
    if (c.e1 == GE_BIAS_SILU && c.e2 == GE_BIAS_VPROD) CL(GE_BIAS_SILU, GE_BIAS_VPROD);
    if (c.e1 == GE_BIAS_SILU && c.e2 == GE_UPDATE) CL(GE_BIAS_SILU, GE_UPDATE);
    if (c.e1 == GE_BIAS_SILU && c.e2 == GE_UPDATE_N) {
        // K = 2F in whole blocks: F = 64 or 128
        if (K == 128) launch_chain<P, GE_BIAS_SILU, GE_UPDATE_N, 4>(s, c);
        else if (K == 256) launch_chain<P, GE_BIAS_SILU, GE_UPDATE_N, 8>(s, c);
        else return -1;
        return 0;
    }
    if (c.e1 == GE_DSILU && c.e2 == GE_STORE) CL(GE_DSILU, GE_STORE);
    if (c.e1 == GE_DSILU && c.e2 == GE_ADD) CL(GE_DSILU, GE_ADD);
    if (c.e1 == GE_DSILU && c.e2 == GE_UPDATE_ADJ) {
        // K = 3F in whole blocks: F = 64 or 128
        if (K == 192) launch_chain<P, GE_DSILU, GE_UPDATE_ADJ, 6>(s, c);
        else if (K == 384) launch_chain<P, GE_DSILU, GE_UPDATE_ADJ, 12>(s, c);
        else return -1;
        return 0;
    }
#undef CL
    return -1;
}

int node_gemm_chain(hipStream_t s, int precision, const GemmChain &c) {
    if (c.M <= 0) return 0;
    if (c.B1->N > NCH || c.B2->K != c.B1->N) return -1;
    if ((c.e2 == GE_UPDATE || c.e2 == GE_UPDATE_N || c.e2 == GE_UPDATE_ADJ) &&
        (c.F < 64 || c.F % 4 || c.B2->N % c.F))
        return -1;
    if (c.e2 == GE_UPDATE_N && c.B1->K != 2 * c.F) return -1;
    if (c.e2 == GE_BIAS_VPROD && (c.F <= 0 || c.F % 4 || c.B2->N < c.F)) return -1;
    if (c.e2 == GE_UPDATE_ADJ && (c.B1->K != 3 * c.F || c.lda < 2 * c.F || c.ldr2 < c.F)) return -1;
    const int rc = precision == 0 ? chain_p<0>(s, c) : (precision == 1 ? chain_p<1>(s, c) : chain_p<2>(s, c));
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // namespace mlp
