// Node-feature GEMMs on the matrix cores (MFMA), with fused epilogues.
//
//   C[m][n] = sum_r A[m][r] B(r, n)
//   NT: B(r, n) = W[n][r]   (forward: W stored [out][in])
//   NN: B(r, n) = W[r][n]   (adjoint: multiply by W^T on the right)
//
// 64 x 64 output tile per 256-thread workgroup; the four waves own 32 x 32
// quadrants (2 x 2 MFMA tiles of 16 x 16).  A and B tiles are staged in LDS
// with the reduction index contiguous.  FP32 mode uses
// v_mfma_f32_16x16x4_f32; BF16 mode rounds both operands to bfloat16 when
// staging and uses v_mfma_f32_16x16x32_bf16; accumulation is FP32 in both.
// Operand lane layout (16 x 16 output tile, lane l, g = l / 16):
//   f32:  A[l%16][k0 + g],           B[k0 + g][l%16]
//   bf16: A[l%16][8g .. 8g+7],       B[8g .. 8g+7][l%16]
//   D:    rows 4g .. 4g+3, column l%16 (4 accumulator registers)
// Split-bf16 mode (P = 2) stages each operand as x = hi + lo with
// hi = bf16(x), lo = bf16(x - hi), and accumulates the three products
// lo*hi + hi*lo + hi*hi on the bf16 matrix cores (the lo*lo term is below
// FP32 rounding of the sum's leading part): ~16 significant bits per operand
// at the bf16 instruction rate.
#include "gemm.h"

namespace mlp {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));

__device__ __forceinline__ float g_sigmoid(float x) { return 1.0f / (1.0f + __expf(-x)); }

constexpr int TBM = 64, TBN = 64, TBK = 32;
constexpr int LDF = TBK + 4;   // f32 LDS row stride (floats)
constexpr int LDH = TBK + 8;   // bf16 LDS row stride (elements)

template <int P, bool NT, int EPI>
__global__ void __launch_bounds__(256) k_gemm_mfma(const float *__restrict__ A, int lda,
                                                   const float *__restrict__ B, int ldb, float *C, int ldc,
                                                   int M, int N, int K, const float *__restrict__ bias,
                                                   float *__restrict__ C2, int ldc2, const float *R, int ldr) {
    __shared__ __attribute__((aligned(16))) float smf[P == 0 ? 2 * TBM * LDF : 1];
    __shared__ __attribute__((aligned(16))) __bf16 smh[P >= 1 ? 2 * TBM * LDH : 1];
    __shared__ __attribute__((aligned(16))) __bf16 sml[P == 2 ? 2 * TBM * LDH : 1];
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    const int wm = wave >> 1, wn = wave & 1;
    const int g = lane >> 4, c16 = lane & 15;
    const long m0 = (long)blockIdx.x * TBM;
    const int n0 = blockIdx.y * TBN;
    v4f acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; a++)
#pragma unroll
        for (int b = 0; b < 2; b++) acc[a][b] = v4f{0.f, 0.f, 0.f, 0.f};

    for (int k0 = 0; k0 < K; k0 += TBK) {
        // stage A: 64 rows x 32 k, 8 consecutive k per thread
        {
            const int r = tid >> 2, kq = (tid & 3) * 8;
            const long m = m0 + r;
            float v[8];
#pragma unroll
            for (int q = 0; q < 8; q++) {
                int k = k0 + kq + q;
                v[q] = (m < M && k < K) ? A[m * lda + k] : 0.f;
            }
            if (P == 0) {
#pragma unroll
                for (int q = 0; q < 8; q++) smf[r * LDF + kq + q] = v[q];
            } else {
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const __bf16 h = (__bf16)v[q];
                    smh[r * LDH + kq + q] = h;
                    if (P == 2) sml[r * LDH + kq + q] = (__bf16)(v[q] - (float)h);
                }
            }
        }
        // stage B as [n][k]
        {
            float v[8];
            int nn, kq;
            if (NT) {
                nn = tid >> 2;
                kq = (tid & 3) * 8;
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    int n = n0 + nn, k = k0 + kq + q;
                    v[q] = (n < N && k < K) ? B[(long)n * ldb + k] : 0.f;
                }
            } else {
                nn = tid & 63;
                kq = (tid >> 6) * 8;
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    int n = n0 + nn, k = k0 + kq + q;
                    v[q] = (n < N && k < K) ? B[(long)k * ldb + n] : 0.f;
                }
            }
            if (P == 0) {
#pragma unroll
                for (int q = 0; q < 8; q++) smf[TBM * LDF + nn * LDF + kq + q] = v[q];
            } else {
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    const __bf16 h = (__bf16)v[q];
                    smh[TBM * LDH + nn * LDH + kq + q] = h;
                    if (P == 2) sml[TBM * LDH + nn * LDH + kq + q] = (__bf16)(v[q] - (float)h);
                }
            }
        }
        __syncthreads();
        if (P == 0) {
#pragma unroll
            for (int kk = 0; kk < TBK; kk += 4) {
                float a[2], b[2];
#pragma unroll
                for (int t = 0; t < 2; t++) {
                    a[t] = smf[(wm * 32 + t * 16 + c16) * LDF + kk + g];
                    b[t] = smf[TBM * LDF + (wn * 32 + t * 16 + c16) * LDF + kk + g];
                }
#pragma unroll
                for (int ta = 0; ta < 2; ta++)
#pragma unroll
                    for (int tb = 0; tb < 2; tb++)
                        acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[ta], b[tb], acc[ta][tb], 0, 0, 0);
            }
        } else {
            v8bf a[2], b[2];
#pragma unroll
            for (int t = 0; t < 2; t++) {
                a[t] = *reinterpret_cast<const v8bf *>(&smh[(wm * 32 + t * 16 + c16) * LDH + 8 * g]);
                b[t] = *reinterpret_cast<const v8bf *>(&smh[TBM * LDH + (wn * 32 + t * 16 + c16) * LDH + 8 * g]);
            }
            if (P == 2) {
                v8bf al[2], bl[2];
#pragma unroll
                for (int t = 0; t < 2; t++) {
                    al[t] = *reinterpret_cast<const v8bf *>(&sml[(wm * 32 + t * 16 + c16) * LDH + 8 * g]);
                    bl[t] = *reinterpret_cast<const v8bf *>(&sml[TBM * LDH + (wn * 32 + t * 16 + c16) * LDH + 8 * g]);
                }
#pragma unroll
                for (int ta = 0; ta < 2; ta++)
#pragma unroll
                    for (int tb = 0; tb < 2; tb++) {
                        acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[ta], b[tb], acc[ta][tb], 0, 0, 0);
                        acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ta], bl[tb], acc[ta][tb], 0, 0, 0);
                    }
            }
#pragma unroll
            for (int ta = 0; ta < 2; ta++)
#pragma unroll
                for (int tb = 0; tb < 2; tb++)
                    acc[ta][tb] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ta], b[tb], acc[ta][tb], 0, 0, 0);
        }
        __syncthreads();
    }
    // epilogue
#pragma unroll
    for (int ta = 0; ta < 2; ta++)
#pragma unroll
        for (int tb = 0; tb < 2; tb++) {
            const int n = n0 + wn * 32 + tb * 16 + c16;
            if (n >= N) continue;
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const long m = m0 + wm * 32 + ta * 16 + 4 * g + r;
                if (m >= M) continue;
                float x = acc[ta][tb][r];
                if (EPI == GE_STORE) {
                    C[m * ldc + n] = x;
                } else if (EPI == GE_BIAS) {
                    C[m * ldc + n] = x + bias[n];
                } else if (EPI == GE_BIAS_SILU) {
                    float h = x + bias[n];
                    C[m * ldc + n] = h;
                    C2[m * ldc2 + n] = h * g_sigmoid(h);
                } else if (EPI == GE_DSILU) {
                    float h = R[m * ldr + n];
                    float sg = g_sigmoid(h);
                    C[m * ldc + n] = x * (sg * (1.0f + h * (1.0f - sg)));
                } else {
                    C[m * ldc + n] = R[m * ldr + n] + x;
                }
            }
        }
}

template <int P, bool NT, int EPI>
static void launch(hipStream_t s, const float *A, int lda, const float *B, int ldb, float *C, int ldc, int M, int N,
                   int K, const float *bias, float *C2, int ldc2, const float *R, int ldr) {
    dim3 grid((unsigned)((M + TBM - 1) / TBM), (unsigned)((N + TBN - 1) / TBN));
    k_gemm_mfma<P, NT, EPI><<<grid, 256, 0, s>>>(A, lda, B, ldb, C, ldc, M, N, K, bias, C2, ldc2, R, ldr);
}

int node_gemm(hipStream_t s, int precision, bool nt, int epi, const float *A, int lda, const float *B, int ldb,
              float *C, int ldc, int M, int N, int K, const float *bias, float *C2, int ldc2, const float *R,
              int ldr) {
    if (M <= 0 || N <= 0 || K <= 0) return 0;
#define GL(P_, NT_, E_) launch<P_, NT_, E_>(s, A, lda, B, ldb, C, ldc, M, N, K, bias, C2, ldc2, R, ldr)
#define GE(P_, NT_)                                 \
    switch (epi) {                                  \
        case GE_STORE: GL(P_, NT_, GE_STORE); break; \
        case GE_BIAS: GL(P_, NT_, GE_BIAS); break;   \
        case GE_BIAS_SILU: GL(P_, NT_, GE_BIAS_SILU); break; \
        case GE_DSILU: GL(P_, NT_, GE_DSILU); break; \
        default: GL(P_, NT_, GE_ADD); break;         \
    }
    if (precision == 0) {
        if (nt) { GE(0, true) } else { GE(0, false) }
    } else if (precision == 1) {
        if (nt) { GE(1, true) } else { GE(1, false) }
    } else {
        if (nt) { GE(2, true) } else { GE(2, false) }
    }
#undef GE
#undef GL
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

}  // namespace mlp
