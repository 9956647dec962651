// Node-feature GEMM entry (MFMA).  See gemm.hip.
#pragma once
#include <hip/hip_runtime.h>

namespace mlp {

enum { GE_STORE = 0, GE_BIAS = 1, GE_BIAS_SILU = 2, GE_DSILU = 3, GE_ADD = 4, GE_UPDATE = 5, GE_UPDATE_ADJ = 6,
       GE_UPDATE_N = 7, GE_BIAS_VPROD = 8 };

// One weight matrix packed as the B operand of C = A B: element (k, n) of B
// at [n][k] (reduction index contiguous), zero-padded to Np x Kp
// (Np a multiple of 128, Kp a multiple of 32).  f32 holds it in FP32, hi the
// bfloat16 rounding and lo the bfloat16 rounding of the remainder.
struct PackedW {
    const float *f32 = nullptr;
    const __bf16 *hi = nullptr, *lo = nullptr;
    int N = 0, K = 0, Np = 0, Kp = 0;
};

// Bytes of device memory (a multiple of 256) that pack_weight needs for an
// R x C matrix in the given orientation (all three forms).
size_t packed_bytes(int R, int C, bool transpose);
// Pack W (row-major R x C, FP32, device) into `arena` (device, 256-byte
// aligned, packed_bytes long): transpose = false gives B = W^T (forward, W
// stored [out][in]), transpose = true gives B = W (adjoint).  parts3: the
// reduction index (K = 3P, P a multiple of 32) taken in the order of the
// GE_UPDATE_ADJ operand, block 3 b + p of 32 = rows p P + 32 b .. +31 of
// part p.  Returns 0, -1 (parts3 with another K) or -5.
int pack_weight(hipStream_t s, const float *W, int R, int C, bool transpose, void *arena, PackedW *out,
                bool parts3 = false);

// C = epilogue(A B) for A (M x K, row stride lda, FP32).  Mc (device, may be
// null): a row count known only on the device; rows at or past it are not
// computed (the grid is sized for M, its workgroups past the count leave).
// precision: 0 = FP32 operands, 1 = bfloat16 operands, 2 = split bfloat16
// operands (hi + lo, three products); FP32 accumulation in all.
// Returns 0 or -5 (launch error).
int node_gemm(hipStream_t s, int precision, int epi, const float *A, int lda, const PackedW &B, float *C, int ldc,
              int M, const float *bias = nullptr, float *C2 = nullptr, int ldc2 = 0, const float *R = nullptr,
              int ldr = 0, const int *Mc = nullptr);

// Two chained products C2 = e2(act(A B1) B2) in one kernel, the intermediate
// kept on chip.  e1 = GE_BIAS_SILU: act = SiLU(x + bias1), the pre-activation
// x + bias1 also stored to C1; e1 = GE_DSILU: act = x * SiLU'(R1).  e2 =
// GE_BIAS (+ bias2), GE_STORE or GE_ADD (+ R2), or GE_BIAS_VPROD: GE_BIAS,
// and of the first F output columns (phi_vv of a PaiNN message MLP) also
// v2[(3 m + d) F + f] = v1[(3 m + d) F + f] C2[m][f] for d = 0, 1, 2 (the
// rows a message pass gathers).  B1 has at most 128 columns and
// B2 as many rows.  Returns 0, -1 (unsupported shape or combination) or -5.
// Two further second-stage epilogues apply the gated update of a PaiNN layer
// (F >= 64, so that the three F-column parts of the output fall in
// different 128-column chunks, processed in order):
//   GE_UPDATE (after bias2; the output is a = [a_vv | a_sv | a_ss]):
//     C2 = a_vv, a_sv (a_ss is not stored), v2 = v1 + a_vv o Uv (if v2),
//     s2 = s1 + a_sv o <Uv, Vv> + a_ss, with s1 = sn[:, :F];
//   GE_UPDATE_N: the same, with the first product's operand [s1 | n] formed
//     as it is loaded (F = 64 or 128): s1 = A[:, :F], n = sqrt(eps + sum_d
//     Vv_d^2) from UV (n is then not stored);
//   GE_UPDATE_ADJ (with e1 = GE_DSILU; the whole adjoint of the update and
//     of the norm; F = 64 or 128): the first product's A operand, da =
//     [dE/da_vv | dE/da_sv | dE/da_ss] (K1 = 3F, B1 packed with parts3), is
//     formed as it is needed from ds2 = R2, dv2 = gv (null: zero), UV and
//     a = A (rows of lda floats, [a_vv | a_sv | ...]), and dUv = dv2 o a_vv +
//     ds2 a_sv Vv goes to gUV on the way; the output is [ds1 | dn]: C2 =
//     R2 + ds1, and dVv = ds2 a_sv Uv + (dn / n) o Vv to gUV, with
//     n = sqrt(eps + sum_d Vv_d^2) formed again from UV.
// UV and gUV hold rows [Uv | Vv] of 2F per (atom, direction), v1, v2 and gv
// rows of F per (atom, direction).
struct GemmChain {
    int e1 = GE_BIAS_SILU, e2 = GE_BIAS;
    const float *A = nullptr;
    int lda = 0, M = 0;
    const PackedW *B1 = nullptr, *B2 = nullptr;
    float *C1 = nullptr;
    int ldc1 = 0;
    const float *bias1 = nullptr, *R1 = nullptr;
    int ldr1 = 0;
    float *C2 = nullptr;
    int ldc2 = 0;
    const float *bias2 = nullptr, *R2 = nullptr;
    int ldr2 = 0;
    int F = 0;                                    // feature width of the update epilogues
    const float *sn = nullptr, *v1 = nullptr, *UV = nullptr;
    float *s2 = nullptr, *v2 = nullptr, *gUV = nullptr;
    const float *gv = nullptr;
    float eps = 0.f;                              // the norm's epsilon (GE_UPDATE_N, GE_UPDATE_ADJ)
    const int *Mc = nullptr;                      // device row count bounding M (may be null)
};
int node_gemm_chain(hipStream_t s, int precision, const GemmChain &c);

// A bias-free SiLU MLP over rows (edges) with every hidden layer kept on
// chip: f[q] (B = W_q^T) and a[q] (B = W_q) for the hidden matrices
// q < nh and the output matrix q = nh.  This build takes nh = 3, an input
// of at most 32 columns, hidden widths of at most 64, an output of at most
// 384 columns and (adjoint) an input gradient of at most 16 columns.
struct EdgeMlp {
    int nh = 0;
    PackedW f[5], a[5];
};
// C = h_nh Wo^T with h_q = silu(h_(q-1) W_q^T), h_0 = X (rows bounded by the
// device count Mc when given).  Returns 0, -1 (unsupported shape) or -5.
int edge_mlp_forward(hipStream_t s, int precision, const EdgeMlp &W, const float *X, int ldx, float *C, int ldc,
                     int M, const int *Mc = nullptr);
// GX (+)= dE/dX given GC = dE/dC, recomputing the hidden layers.  Returns
// 0, -1 or -5.
int edge_mlp_adjoint(hipStream_t s, int precision, const EdgeMlp &W, const float *X, int ldx, const float *GC,
                     int ldgc, float *GX, int ldgx, bool add, int M, const int *Mc = nullptr);

}  // namespace mlp
