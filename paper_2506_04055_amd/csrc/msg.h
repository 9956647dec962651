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
    const float *u;           // v * phi_vv, rows [x | y | z] of 3F (forward gathers)
    const float *A, *c;       // filter weights [3F][K], [3F]
    float rc;
    const int8_t *hop;
    int hop_max;
    float *sn, *v1;           // forward outputs (s1 inside [s1 | n] rows of 2F)
    const float *gs1, *gv1;   // adjoint inputs
    float *gv_in, *gphi;      // adjoint outputs
    float4 *S;                // this layer's edge sums (dE/dr, dE/drhat), pass p at S + p * s_stride
    long s_stride;
    // First layer: v = 0 on input (the forward neither reads v nor u) and the
    // inputs s, v need no gradient (the adjoint writes S only, not gphi or gv_in).
    // There phi and s point to per-species tables ([S][3F], [S][F]) whose rows
    // are picked by species (device int32 per atom).
    bool layer0;
    const int *species;
    // MSG_QUEUE_INTS device ints, zero on entry, used by this launch alone:
    // the counters from which the waves take their atoms
    int *queue;
};
constexpr int MSG_QUEUE_INTS = 2048;

// Return 0, -1 (unsupported F, K) or -5 (launch error).
int msg_forward(hipStream_t st, int precision, int F, int K, const MsgArgs &a);
int msg_adjoint(hipStream_t st, int precision, int F, int K, const MsgArgs &a);

// The factorised first layer (msg.hip): per-atom, per-species sums of the
// radial basis (forward) and the edge sums of the adjoint from the per-atom
// vectors Q.  Each species has a block of l0_block(K) columns, basis slot k
// of species Z at column Z l0_block(K) + k (slots past K meet zero weights).
// Layouts: P rows i of ldp floats, the S blocks then the species one-hot at
// column S l0_block(K) + Z; R, Q_v rows 3 i + d; Q_s rows i.  All leading
// dimensions are multiples of 4.
struct L0Args {
    const int *rowc, *colc, *revc;
    const float4 *geom;
    int n;
    float rc;
    const int8_t *hop;
    int hop_max;
    const int *species;
    float *P, *R;             // forward outputs
    int ldp, ldr;
    const float *Qs, *Qv;     // adjoint inputs
    int ldq;
    float4 *S;                // adjoint output: the layer's single edge-sum slot
};
// Whether this build has the factorised first layer for (K, n_species).
bool l0_factorised(int K, int S);
__host__ __device__ constexpr int l0_block(int K) { return (K + 1 + 7) / 8 * 8; }
// Return 0, -1 (unsupported K, S) or -5 (launch error).
int msg_l0_basis_sums(hipStream_t st, int K, int S, const L0Args &a);
int msg_l0_edge_sums(hipStream_t st, int K, int S, const L0Args &a);

// Feature passes of the adjoint.
int msg_passes(int F);
// Edge-sum slots of one evaluation: one per layer after the first (its
// passes are summed in the kernel), then the first layer's (one when it is
// factorised, else one per pass); slot q at S + q * s_stride.
int msg_slots(int F, int T, bool l0_factorised);
// G[e] over the pruned edges (count rowc[n], at most ne_max), assembled from
// the nslot slots of S (slot q at S + q * s_stride).
int msg_assemble_G(hipStream_t st, const int *rowc, int n, long ne_max, const float4 *geom, const float4 *S,
                   long s_stride, int nslot, float4 *G);

}  // namespace mlp
