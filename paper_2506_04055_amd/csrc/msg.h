// Message pass and adjoint kernels with the radial filter on MFMA (msg.hip).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlp {

struct MsgArgs {
    const int *rowc, *colc;
    const float4 *geom;       // (dx, dy, dz, r) of each pruned edge, d = x_src - x_dst
    int n;
    const float *phi, *s, *v; // layer inputs (phi of the message MLP)
    const float *A, *c;       // filter weights [3F][K], [3F]
    float rc;
    const int8_t *hop;
    int hop_max;
    float *sn, *v1;           // forward outputs (s1 inside [s1 | n] rows of 2F)
    const float *gs1, *gv1;   // adjoint inputs
    float *gv_in, *gphi;      // adjoint outputs
    float4 *G;                // per-edge geometric gradient accumulator
};

// Return 0, -1 (unsupported F, K) or -5 (launch error).
int msg_forward(hipStream_t st, int precision, int F, int K, const MsgArgs &a);
int msg_adjoint(hipStream_t st, int precision, int F, int K, const MsgArgs &a);

}  // namespace mlp
