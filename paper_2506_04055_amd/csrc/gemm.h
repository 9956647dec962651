// Node-feature GEMM entry (MFMA).  See gemm.hip.
#pragma once
#include <hip/hip_runtime.h>

namespace mlp {

enum { GE_STORE = 0, GE_BIAS = 1, GE_BIAS_SILU = 2, GE_DSILU = 3, GE_ADD = 4 };

// precision: 0 = FP32 operands, 1 = bfloat16 operands, 2 = split bfloat16
// operands (hi + lo, three products); FP32 accumulation in all.
// Returns 0 or -5 (launch error).
int node_gemm(hipStream_t s, int precision, bool nt, int epi, const float *A, int lda, const float *B, int ldb,
              float *C, int ldc, int M, int N, int K, const float *bias = nullptr, float *C2 = nullptr,
              int ldc2 = 0, const float *R = nullptr, int ldr = 0);

}  // namespace mlp
