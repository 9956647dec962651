// Allegro with a single tensor-product layer: energy and forces on the
// pruned neighbour graph.
//
// The paper deploys Allegro (Methods, "Chosen Architectures": edge-centric
// and strictly local; messages pass only between directed edges that share
// their central atom) with one tensor-product layer, l_max = 3, 8 radial
// functions and a polynomial envelope of order 2 for water and aluminium
// ("Training Details").  Per directed edge e = (i <- j), r = |r_j - r_i| < rc,
// rhat = (r_j - r_i) / r, with the layer equations of the cited Allegro
// paper in this reading:
//   u(r)  = 1 - (p+1)(p+2)/2 x^p + p(p+2) x^(p+1) - p(p+1)/2 x^(p+2),  x = r / rc
//   B_k   = sqrt(2 / rc) sin(k pi r / rc) / r u(r)
//   x0    = u(r) MLP_2b([onehot(Z_i) | onehot(Z_j) | B])
//   w0 = Wv x0,  we = We x0                     (one weight per channel c)
//   env_i[c, m] = nu sum_(edges i <- k) we_ik[c] Y_(l_c m)(rhat_ik)
//   S_e[c] = w0_e[c] / (2 l_c + 1) sum_m Y_(l_c m)(rhat_e) env_i[c, m]
//                                 (the l x l -> 0 outputs of the tensor
//                                  product of V_e = w0_e Y(rhat_e) with env_i)
//   x1  = (x0 + u(r) MLP_lat([x0 | S_e])) / sqrt(2)
//   E_e = u(r) MLP_out(x1),  U_i = sum_(edges i <- j) E_e,  E = sum_(i local) U_i
// Y are component-normalised real spherical harmonics (sum_m Y_lm^2 = 2l+1)
// in Cartesian form.  The environment is built once per atom and the scalar
// outputs contracted against it per edge, so the per-edge angular work is
// O(l_max^2) instead of a sum over pairs of edges.  The MLPs are GEMMs over
// edges on the matrix cores (gemm.hip); the angular and geometric steps are
// edge and atom kernels here.  Forces come from a hand-written adjoint: the
// GEMMs transposed, the tensor-product contraction reversed per atom (a
// gradient of the environment accumulated over the atom's edges, then sent
// back to each edge), and per edge G_e = dE/d(r_i - r_j), assembled into
// forces by gathering through the reverse-edge index (no atomics).
#include "internal.h"
#include "gemm.h"
#include "sh.h"

#include <cmath>
#include <vector>

namespace mlp {

static inline int nblk(long n, int t) { return (int)((n + t - 1) / t); }
static inline int up4(int x) { return (x + 3) / 4 * 4; }

__device__ __forceinline__ float al_sigmoid(float x) { return 1.0f / (1.0f + __expf(-x)); }
__device__ __forceinline__ float al_dsilu(float x) {
    const float s = al_sigmoid(x);
    return s * (1.0f + x * (1.0f - s));
}

struct AlModel {
    AlDims d;
    int KIN = 0;     // columns of the two-body input, internal order [B | onehot_i | onehot_j | 0]
    int NBP = 0;     // radial functions padded to a multiple of 4
    float *vec = nullptr;                       // biases and the output vector on the device
    const float *b2b[6] = {}, *lat_b1 = nullptr, *lat_b2 = nullptr, *out_b1 = nullptr, *out_w2 = nullptr,
                *out_b2 = nullptr;
    float out_b2_host = 0.f;
    // B operands: forward (B = W^T) and adjoint (B = W); a2b[0] is the radial
    // block of the first two-body matrix only
    PackedW f2b[6], fVE, fL1, fL2, fO1;
    PackedW a2b[6], aVE, aL1, aL2, aO1;
    void *pk_dev = nullptr;
};

// ---------------------------------------------------------------------------
// Forward, per edge: envelope, radial functions, harmonics, two-body input.
// One wave per destination atom, lanes over its edges.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_al_edge_in(const int *__restrict__ rowc, const int *__restrict__ colc,
                                                    const float4 *__restrict__ geom, const int *__restrict__ zsp,
                                                    const int *__restrict__ perm, int n, int n_local, int S, int NB,
                                                    int p, int KIN, float rc, float *__restrict__ H0,
                                                    float *__restrict__ U, float *__restrict__ Y,
                                                    float *__restrict__ GL) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const int zi = zsp[i];
    const float loc = perm[i] < n_local ? 1.f : 0.f;   // dE/dE_e: the edge's atom is local
    const float c0 = sqrtf(2.0f / rc), th = 3.14159265358979f / rc;
    for (int e = rowc[i] + lane; e < rowc[i + 1]; e += 64) {
        const float4 gm = geom[e];
        const float r = gm.w, ir = 1.0f / r;
        float u, du;
        envelope(r / rc, p, u, du);
        float sn, cs;
        sincosf(th * r, &sn, &cs);
        float *h = H0 + (long)e * KIN;
        float sk = sn, skm = 0.f;
        for (int k = 0; k < NB; k++) {
            h[k] = c0 * sk * ir * u;
            const float nx = 2.f * cs * sk - skm;
            skm = sk;
            sk = nx;
        }
        const int zj = zsp[colc[e]];
        for (int q = NB; q < KIN; q++) h[q] = 0.f;
        h[NB + zi] = 1.f;
        h[NB + S + zj] = 1.f;
        U[e] = u;
        GL[e] = loc;
        float Ye[16];
        sh16(gm.x * ir, gm.y * ir, gm.z * ir, Ye);
        float4 *y4 = reinterpret_cast<float4 *>(Y + (long)e * 16);
#pragma unroll
        for (int q = 0; q < 4; q++) y4[q] = make_float4(Ye[4 * q], Ye[4 * q + 1], Ye[4 * q + 2], Ye[4 * q + 3]);
    }
}

// out[e][0..D) = u[e] * in[e][0..D) (row strides ldo, ldi), four per thread.
__global__ void k_al_scale_rows(const float *__restrict__ in, int ldi, const float *__restrict__ u,
                                const int *__restrict__ cnt, int D, float *__restrict__ out, int ldo) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int D4 = D / 4;
    const long e = t / D4;
    if (e >= *cnt) return;
    const int f = 4 * (int)(t % D4);
    const float s = u[e];
    const float4 x = *reinterpret_cast<const float4 *>(in + e * ldi + f);
    *reinterpret_cast<float4 *>(out + e * ldo + f) = make_float4(s * x.x, s * x.y, s * x.z, s * x.w);
}

// Channel layout of a lane (= channel c): its degree, first harmonic and the
// 1 / (2 l + 1) of the scalar path.
struct AlChan {
    int l, m0, nm;
    float inv;
    __device__ AlChan(int c, const AlDims &d) {
        int off = 0;
        l = 0;
        for (int q = 0; q <= d.lmax; q++) {
            if (c >= off && c < off + d.ch[q]) l = q;
            off += d.ch[q];
        }
        m0 = l * l;
        nm = 2 * l + 1;
        inv = 1.0f / (float)nm;
    }
};

// The edge's 16 harmonics (the same address in every lane of the wave, so
// they come through the scalar cache) and the lane's own components
// ym[m] = Y_(l, m) for m < 2l + 1, zero above.
__device__ __forceinline__ void al_lane_harm(const float *__restrict__ ye, int l, float *ym) {
    float y[16];
#pragma unroll
    for (int q = 0; q < 16; q++) y[q] = ye[q];
#pragma unroll
    for (int m = 0; m < 7; m++) {
        const float a = m < 1 ? y[m] : 0.f, b = m < 3 ? y[1 + m] : 0.f, c = m < 5 ? y[4 + m] : 0.f, dd = y[9 + m];
        ym[m] = l == 0 ? a : (l == 1 ? b : (l == 2 ? c : dd));
    }
}

// The environment of each atom and the scalar outputs of its edges.  One
// wave per atom (its index made wave-uniform, so the edge loop and the
// harmonic loads are scalar), lane = channel: pass 1 sums env[c][m] over the
// atom's edges, pass 2 contracts each edge's harmonics against it.
__global__ void __launch_bounds__(256) k_al_tp(const int *__restrict__ rowc, int n, AlDims d,
                                               const float *__restrict__ Y, const float *__restrict__ WV,
                                               float *__restrict__ ENV, float *__restrict__ LIN) {
    const int lane = threadIdx.x & 63;
    const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + (threadIdx.x >> 6));
    if (i >= n) return;
    const int NC = d.NC, ldwv = 2 * d.NC, ldl = d.D + d.NC;
    if (lane >= NC) return;
    const AlChan ch(lane, d);
    const int e0 = rowc[i], e1 = rowc[i + 1];
    float env[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    // unrolled so that several edges' loads are in flight together
#pragma unroll 4
    for (int e = e0; e < e1; e++) {
        const float we = WV[(long)e * ldwv + NC + lane];
        float ym[7];
        al_lane_harm(Y + (long)e * 16, ch.l, ym);
#pragma unroll
        for (int m = 0; m < 7; m++) env[m] = fmaf(we, ym[m], env[m]);
    }
    float *en = ENV + ((long)i * NC + lane) * 8;
#pragma unroll
    for (int m = 0; m < 7; m++) {
        env[m] *= d.nu;
        en[m] = env[m];
    }
#pragma unroll 4
    for (int e = e0; e < e1; e++) {
        float ym[7];
        al_lane_harm(Y + (long)e * 16, ch.l, ym);
        float dot = 0.f;
#pragma unroll
        for (int m = 0; m < 7; m++) dot = fmaf(ym[m], env[m], dot);
        LIN[(long)e * ldl + d.D + lane] = WV[(long)e * ldwv + lane] * ch.inv * dot;
    }
}

// x1 = (x0 + u m) / sqrt(2), x0 in the first D columns of LIN.
__global__ void k_al_x1(const float *__restrict__ LIN, int ldl, const float *__restrict__ u,
                        const float *__restrict__ M, const int *__restrict__ cnt, int D, float *__restrict__ X1) {
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int D4 = D / 4;
    const long e = t / D4;
    if (e >= *cnt) return;
    const int f = 4 * (int)(t % D4);
    const float s = u[e], r2 = 0.70710678118654752f;
    const float4 x = *reinterpret_cast<const float4 *>(LIN + e * ldl + f);
    const float4 m = *reinterpret_cast<const float4 *>(M + e * D + f);
    *reinterpret_cast<float4 *>(X1 + e * D + f) =
        make_float4(r2 * fmaf(s, m.x, x.x), r2 * fmaf(s, m.y, x.y), r2 * fmaf(s, m.z, x.z), r2 * fmaf(s, m.w, x.w));
}

// E_e = u (w2 . HO_e + b2) summed over each atom's edges.  One wave per atom:
// eight lane groups take the edges q, q + 8, ..., the eight lanes of a group
// the row's features four at a time (a row is read as whole 16-byte pieces);
// the sums run in a fixed order (group totals, then a butterfly).
__global__ void __launch_bounds__(256) k_al_energy(const int *__restrict__ rowc, int n, int OH,
                                                   const float *__restrict__ HO, const float *__restrict__ u,
                                                   const float *__restrict__ w2, float b2, float *__restrict__ Uat) {
    const int lane = threadIdx.x & 63, q = lane & 7, grp = lane >> 3;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const int e1 = rowc[i + 1];
    float acc = 0.f;
    for (int eb = rowc[i]; eb < e1; eb += 8) {
        const int e = eb + grp;
        float dot = 0.f;
        if (e < e1)
            for (int f = 4 * q; f < OH; f += 32) {
                const float4 h = *reinterpret_cast<const float4 *>(HO + (long)e * OH + f);
                dot += h.x * w2[f] + h.y * w2[f + 1] + h.z * w2[f + 2] + h.w * w2[f + 3];
            }
        dot += __shfl_xor(dot, 1, 64);
        dot += __shfl_xor(dot, 2, 64);
        dot += __shfl_xor(dot, 4, 64);
        if (e < e1 && q == 0) acc = fmaf(u[e], dot + b2, acc);
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) Uat[i] = acc;
}

// ---------------------------------------------------------------------------
// Adjoint
// ---------------------------------------------------------------------------

// dE/dE_e = GL[e] (1 for edges into a local atom, 0 otherwise).  Through
// E_e = u (w2 . silu(PO) + b2): GU[e] = dE/du (first part) and the gradient of
// the output layer's pre-activation, written over HO.  Eight lanes per edge,
// four features each.
__global__ void k_al_out_bwd(const int *__restrict__ cnt, int OH, const float *__restrict__ PO,
                             float *__restrict__ HO, const float *__restrict__ u, const float *__restrict__ GL,
                             const float *__restrict__ w2, float b2, float *__restrict__ GU) {
    const long ne = *cnt;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long e = t >> 3;
    const int q = (int)(t & 7);
    float dot = 0.f;
    if (e < ne) {
        const float gE = GL[e], s = gE * u[e];
        for (int f = 4 * q; f < OH; f += 32) {
            float4 *hp = reinterpret_cast<float4 *>(HO + e * OH + f);
            const float4 h = *hp, pp = *reinterpret_cast<const float4 *>(PO + e * OH + f);
            dot += h.x * w2[f] + h.y * w2[f + 1] + h.z * w2[f + 2] + h.w * w2[f + 3];
            *hp = make_float4(s * w2[f] * al_dsilu(pp.x), s * w2[f + 1] * al_dsilu(pp.y),
                              s * w2[f + 2] * al_dsilu(pp.z), s * w2[f + 3] * al_dsilu(pp.w));
        }
    }
    dot += __shfl_xor(dot, 1, 8);
    dot += __shfl_xor(dot, 2, 8);
    dot += __shfl_xor(dot, 4, 8);
    if (e < ne && q == 0) GU[e] = GL[e] * (dot + b2);
}

// Through x1 = (x0 + u m) / sqrt(2): with GX = dE/dx1 (in X), GU += GX . m / sqrt(2),
// M <- dE/dm = u GX / sqrt(2), X <- dE/dx0 (this path) = GX / sqrt(2).
// Sixteen lanes per edge, four features per lane per step.
__global__ void k_al_x1_bwd(const int *__restrict__ cnt, int D, const float *__restrict__ u, float *__restrict__ X,
                            float *__restrict__ M, float *__restrict__ GU) {
    const long ne = *cnt;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long e = t >> 4;
    const int q = (int)(t & 15);
    const float r2 = 0.70710678118654752f;
    float part = 0.f;
    if (e < ne) {
        const float s = u[e] * r2;
        for (int f = 4 * q; f < D; f += 64) {
            float4 *xp = reinterpret_cast<float4 *>(X + e * D + f);
            float4 *mp = reinterpret_cast<float4 *>(M + e * D + f);
            const float4 gx = *xp, m = *mp;
            part += gx.x * m.x + gx.y * m.y + gx.z * m.z + gx.w * m.w;
            *mp = make_float4(s * gx.x, s * gx.y, s * gx.z, s * gx.w);
            *xp = make_float4(r2 * gx.x, r2 * gx.y, r2 * gx.z, r2 * gx.w);
        }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) part += __shfl_xor(part, off, 16);
    if (e < ne && q == 0) GU[e] += r2 * part;
}

template <int CTRL>
__device__ __forceinline__ float al_dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// The sums over the channels of each degree of q[m] (m < 2l + 1), stored as
// GY[slot l^2 + m] (add: accumulate).  STD: the channel layout (32, 16, 8, 8)
// of degrees 0..3 over the 64 lanes, summed by DPP exchanges (8-lane groups
// by quad permutations and the half-row mirror, 16-lane rows by a row
// rotation, the two rows of degree 0 by one cross-row exchange); otherwise
// through the wave's LDS rows.
template <bool STD>
__device__ __forceinline__ void al_channel_sums(const float *q, int lane, int ny, int kc0, int kc1, int km,
                                                float (*red)[8], float *__restrict__ gy, bool add) {
    if constexpr (STD) {
        float v8[7], v16[3], v32 = 0.f;
#pragma unroll
        for (int m = 0; m < 7; m++) {
            float v = q[m];
            v += al_dpp<0xB1>(v);    // quad_perm [1,0,3,2]
            v += al_dpp<0x4E>(v);    // quad_perm [2,3,0,1]
            v += al_dpp<0x141>(v);   // row_half_mirror: the other quad of the 8
            v8[m] = v;
        }
#pragma unroll
        for (int m = 0; m < 3; m++) v16[m] = v8[m] + al_dpp<0x128>(v8[m]);   // row_ror:8
        v32 = v16[0] + __shfl_xor(v16[0], 16, 64);
        if (lane == 0) gy[0] = add ? gy[0] + v32 : v32;
        if (lane == 32)
#pragma unroll
            for (int m = 0; m < 3; m++) gy[1 + m] = add ? gy[1 + m] + v16[m] : v16[m];
        if (lane == 48)
#pragma unroll
            for (int m = 0; m < 5; m++) gy[4 + m] = add ? gy[4 + m] + v8[m] : v8[m];
        if (lane == 56)
#pragma unroll
            for (int m = 0; m < 7; m++) gy[9 + m] = add ? gy[9 + m] + v8[m] : v8[m];
    } else {
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int m = 0; m < 7; m++) red[lane][m] = q[m];
        __builtin_amdgcn_wave_barrier();
        if (lane < ny) {
            float s = 0.f;
            for (int c = kc0; c < kc1; c++) s += red[c][km];
            gy[lane] = add ? gy[lane] + s : s;
        }
    }
}

// Adjoint of k_al_tp, one wave per atom, lane = channel.  With t = dE/dS_e:
//   pass 1: dE/dw0_e[c] = t Y_e . env[c],  genv[c] += t w0_e[c] Y_e,
//           dE/dY_e[m] += sum_c t w0_e[c] env[c][m];   also X <- X + GLIN[:, :D]
//   pass 2 (genv scaled by nu): dE/dwe_e[c] = genv[c] . Y_e,
//           dE/dY_e[m] += sum_c genv[c][m] we_e[c]
template <bool STD>
__global__ void __launch_bounds__(256) k_al_tp_bwd(const int *__restrict__ rowc, int n, AlDims d,
                                                   const float *__restrict__ Y, const float *__restrict__ WV,
                                                   const float *__restrict__ ENV, const float *__restrict__ GLIN,
                                                   float *__restrict__ X, float *__restrict__ GWV,
                                                   float *__restrict__ GY) {
    __shared__ float red[4][64][8];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = __builtin_amdgcn_readfirstlane(blockIdx.x * 4 + w);
    if (i >= n) return;
    const int NC = d.NC, ldwv = 2 * d.NC, ldl = d.D + d.NC, D = d.D;
    const bool act = lane < NC;
    const AlChan ch(act ? lane : 0, d);
    // the harmonic a lane sums in the LDS reductions (lanes 0..15): degree,
    // order, and the channel range of that degree
    int kl = 0, kc0 = 0, kc1 = 0;
    {
        int off = 0;
        for (int q = 0; q <= d.lmax; q++) {
            if (lane >= q * q && lane < (q + 1) * (q + 1)) {
                kl = q;
                kc0 = off;
                kc1 = off + d.ch[q];
            }
            off += d.ch[q];
        }
    }
    const int ny = (d.lmax + 1) * (d.lmax + 1);
    const int km = lane - kl * kl;
    float env[7], genv[7];
#pragma unroll
    for (int m = 0; m < 7; m++) {
        env[m] = act ? ENV[((long)i * NC + lane) * 8 + m] : 0.f;
        genv[m] = 0.f;
    }
    const int e0 = rowc[i], e1 = rowc[i + 1];
#pragma unroll 2
    for (int e = e0; e < e1; e++) {
        float q[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float ym[7];
        al_lane_harm(Y + (long)e * 16, ch.l, ym);
        if (act) {
            const float t = GLIN[(long)e * ldl + D + lane] * ch.inv;
            const float w0 = WV[(long)e * ldwv + lane];
            float dot = 0.f;
#pragma unroll
            for (int m = 0; m < 7; m++) {
                dot = fmaf(ym[m], env[m], dot);
                genv[m] = fmaf(t * w0, ym[m], genv[m]);
                q[m] = t * w0 * env[m];
            }
            GWV[(long)e * ldwv + lane] = t * dot;
        }
        for (int f = lane; f < D; f += 64) X[(long)e * D + f] += GLIN[(long)e * ldl + f];
        al_channel_sums<STD>(q, lane, ny, kc0, kc1, km, red[w], GY + (long)e * 16, false);
    }
#pragma unroll
    for (int m = 0; m < 7; m++) genv[m] *= d.nu;
#pragma unroll 2
    for (int e = e0; e < e1; e++) {
        float q[7] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        float ym[7];
        al_lane_harm(Y + (long)e * 16, ch.l, ym);
        if (act) {
            const float we = WV[(long)e * ldwv + NC + lane];
            float dot = 0.f;
#pragma unroll
            for (int m = 0; m < 7; m++) {
                dot = fmaf(genv[m], ym[m], dot);
                q[m] = genv[m] * we;
            }
            GWV[(long)e * ldwv + NC + lane] = dot;
        }
        al_channel_sums<STD>(q, lane, ny, kc0, kc1, km, red[w], GY + (long)e * 16, true);
    }
}

// Through x0 = u y: GU += GX0 . y, and Yo <- dE/dy = u GX0.
__global__ void k_al_x0_bwd(const int *__restrict__ cnt, int D, const float *__restrict__ u,
                            const float *__restrict__ GX0, float *__restrict__ Yo, float *__restrict__ GU) {
    const long ne = *cnt;
    const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const long e = t >> 4;
    const int q = (int)(t & 15);
    float part = 0.f;
    if (e < ne) {
        const float s = u[e];
        for (int f = 4 * q; f < D; f += 64) {
            const float4 g = *reinterpret_cast<const float4 *>(GX0 + e * D + f);
            float4 *yp = reinterpret_cast<float4 *>(Yo + e * D + f);
            const float4 y = *yp;
            part += g.x * y.x + g.y * y.y + g.z * y.z + g.w * y.w;
            *yp = make_float4(s * g.x, s * g.y, s * g.z, s * g.w);
        }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) part += __shfl_xor(part, off, 16);
    if (e < ne && q == 0) GU[e] += part;
}

// Per edge: dE/dr from the radial functions and the envelope, dE/drhat from
// the harmonics, G_e = dE/d(r_i - r_j) = -(dE/dr rhat + (I - rhat rhat^T) dE/drhat / r).
__global__ void k_al_geom_bwd(const int *__restrict__ rowc, int n, const float4 *__restrict__ geom, int NB,
                              int NBP, int p, float rc, const float *__restrict__ GB, const float *__restrict__ GU,
                              const float *__restrict__ GY, float4 *__restrict__ G) {
    const long ne = rowc[n];
    const float c0 = sqrtf(2.0f / rc), th = 3.14159265358979f / rc;
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (long)gridDim.x * blockDim.x) {
        const float4 gm = geom[e];
        const float r = gm.w, ir = 1.0f / r;
        float u, du;
        envelope(r / rc, p, u, du);
        du *= 1.0f / rc;
        float sn, cs;
        sincosf(th * r, &sn, &cs);
        const float *gb = GB + e * NBP;
        float dEdr = GU[e] * du;
        float sk = sn, skm = 0.f, ck = cs, ckm = 1.f;
        for (int k = 0; k < NB; k++) {
            const float kt = (k + 1) * th;
            // d/dr [c0 sin(k th r) / r u] = c0 [(k th cos / r - sin / r^2) u + sin / r u']
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
        const float4 *g4 = reinterpret_cast<const float4 *>(GY + e * 16);
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float4 v = g4[q];
            gy[4 * q] = v.x;
            gy[4 * q + 1] = v.y;
            gy[4 * q + 2] = v.z;
            gy[4 * q + 3] = v.w;
        }
        float hx, hy, hz;
        sh16_grad(x, y, z, gy, hx, hy, hz);
        const float rd = hx * x + hy * y + hz * z;
        const float gx = dEdr * x + (hx - rd * x) * ir, gyy = dEdr * y + (hy - rd * y) * ir,
                    gz = dEdr * z + (hz - rd * z) * ir;
        G[e] = make_float4(-gx, -gyy, -gz, 0.f);
    }
}

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

// Offsets (floats) of the per-evaluation arrays in the arena.
struct AlArena {
    long H0, u, GL, Y, P[6], A[6], Yo, LIN, WV, PL, M, X1, PO, HO, GU, GWV, GY, GB, ENV, Uat, EP, total;
};

static AlArena al_layout(const AlModel &a, long N, long E) {
    const AlDims &d = a.d;
    AlArena L;
    long o = 0;
    auto take = [&](long cnt) {
        const long r = o;
        o += (cnt + 63) / 64 * 64;
        return r;
    };
    L.H0 = take(E * a.KIN);
    L.u = take(E);
    L.GL = take(E);
    L.Y = take(E * 16);
    for (int q = 0; q < 6; q++) L.P[q] = L.A[q] = 0;
    for (int q = 0; q + 1 < d.n2b; q++) {
        L.P[q] = take(E * d.d2b[q]);
        L.A[q] = take(E * d.d2b[q]);
    }
    L.Yo = take(E * d.D);
    L.LIN = take(E * (d.D + d.NC));
    L.WV = take(E * 2 * d.NC);
    L.PL = take(E * d.LH);
    L.M = take(E * d.D);
    L.X1 = take(E * d.D);
    L.PO = take(E * d.OH);
    L.HO = take(E * d.OH);
    L.GU = take(E);
    L.GWV = take(E * 2 * d.NC);
    L.GY = take(E * 16);
    L.GB = take(E * a.NBP);
    L.ENV = take(N * d.NC * 8);
    L.Uat = take(N + 64);
    L.EP = take(2 * energy_part_doubles(N));   // the energy sums' chunk partials (doubles)
    L.total = o + 4096;
    return L;
}

size_t allegro_arena_bytes(const mlp_model *m, long n_atoms, long n_edges) {
    return (size_t)al_layout(*m->al, n_atoms, n_edges).total * sizeof(float);
}

static int check_dims(const AlDims &d) {
    if (d.S < 1 || d.S > 64) return fail(-1, "allegro: n_species out of range");
    if (d.NB < 1 || d.NB > 16) return fail(-1, "allegro: n_basis must be 1..16");
    if (d.p < 1 || d.p > 8) return fail(-1, "allegro: envelope_p must be 1..8");
    if (d.n2b < 1 || d.n2b > 6) return fail(-1, "allegro: mlp_2b needs 1..6 widths");
    if (d.lmax < 0 || d.lmax > 3) return fail(-1, "allegro: l_max must be 0..3");
    if (d.NC < 1 || d.NC > 64) return fail(-1, "allegro: the channels must total 1..64");
    for (int q = 0; q < d.n2b; q++)
        if (d.d2b[q] < 4 || d.d2b[q] % 4 || d.d2b[q] > 256) return fail(-1, "allegro: two-body widths must be multiples of 4 up to 256");
    if (d.D > 64) return fail(-1, "allegro: the latent width must be at most 64");
    if (d.LH < 4 || d.LH % 4 || d.LH > 128 || d.OH < 4 || d.OH % 4 || d.OH > 128)
        return fail(-1, "allegro: latent_hidden and out_hidden must be multiples of 4 up to 128");
    if (d.NC % 4) return fail(-1, "allegro: the channel total must be a multiple of 4");
    if (!(d.rc > 0.f) || !(d.nu > 0.f)) return fail(-1, "allegro: r_c and env_scale must be positive");
    return 0;
}

int allegro_create(mlp_model *m, const AlDims &d, const float *w, size_t n_weights) {
    if (int rc = check_dims(d)) return rc;
    const int S = d.S, NB = d.NB, NC = d.NC, D = d.D, LH = d.LH, OH = d.OH;
    // storage order (matrices [out][in]): 2b_W1 b1 .. 2b_Wn bn, Wv, We,
    // lat_W1 lat_b1 lat_W2 lat_b2, out_W1 out_b1 out_w2 out_b2
    size_t off = 0;
    std::vector<size_t> oW(d.n2b), ob(d.n2b);
    int prev = 2 * S + NB;
    for (int q = 0; q < d.n2b; q++) {
        oW[q] = off;
        off += (size_t)d.d2b[q] * prev;
        ob[q] = off;
        off += d.d2b[q];
        prev = d.d2b[q];
    }
    const size_t oWv = off;
    off += (size_t)NC * D;
    const size_t oWe = off;
    off += (size_t)NC * D;
    const size_t oL1 = off;
    off += (size_t)LH * (D + NC);
    const size_t oLb1 = off;
    off += LH;
    const size_t oL2 = off;
    off += (size_t)D * LH;
    const size_t oLb2 = off;
    off += D;
    const size_t oO1 = off;
    off += (size_t)OH * D;
    const size_t oOb1 = off;
    off += OH;
    const size_t oOw2 = off;
    off += OH;
    const size_t oOb2 = off;
    off += 1;
    if (off != n_weights)
        return fail(-1, "allegro: weight count " + std::to_string(n_weights) + " does not match the header (" +
                            std::to_string(off) + ")");
    AlModel *a = new AlModel();
    a->d = d;
    a->KIN = up4(NB + 2 * S);
    a->NBP = up4(NB);
    // host-side matrices in the orientations the GEMMs take: the first
    // two-body matrix with its columns in the internal input order
    // [B | onehot_i | onehot_j | 0], its radial block alone, and [Wv; We]
    std::vector<float> W1p((size_t)d.d2b[0] * a->KIN, 0.f), W1B((size_t)d.d2b[0] * NB);
    for (int o = 0; o < d.d2b[0]; o++) {
        const float *row = w + oW[0] + (size_t)o * (2 * S + NB);
        for (int k = 0; k < NB; k++) W1p[(size_t)o * a->KIN + k] = W1B[(size_t)o * NB + k] = row[2 * S + k];
        for (int z = 0; z < 2 * S; z++) W1p[(size_t)o * a->KIN + NB + z] = row[z];
    }
    // device copies: the permuted W1, W1's radial block, and every block of w
    const size_t nW = n_weights;
    std::vector<float> host(nW + W1p.size() + W1B.size());
    std::copy(w, w + nW, host.begin());
    std::copy(W1p.begin(), W1p.end(), host.begin() + nW);
    std::copy(W1B.begin(), W1B.end(), host.begin() + nW + W1p.size());
    float *dev = nullptr;
    if (hipMalloc(&dev, sizeof(float) * host.size()) != hipSuccess) {
        (void)hipGetLastError();
        delete a;
        return fail(-2, "allegro: weight allocation failed");
    }
    if (hipMemcpy(dev, host.data(), sizeof(float) * host.size(), hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(dev);
        delete a;
        return fail(-5, "allegro: weight copy failed");
    }
    a->vec = dev;
    for (int q = 0; q < d.n2b; q++) a->b2b[q] = dev + ob[q];
    a->lat_b1 = dev + oLb1;
    a->lat_b2 = dev + oLb2;
    a->out_b1 = dev + oOb1;
    a->out_w2 = dev + oOw2;
    a->out_b2 = dev + oOb2;
    a->out_b2_host = w[oOb2];
    const float *dW1p = dev + nW, *dW1B = dev + nW + W1p.size();
    struct Item {
        const float *W;
        int R, C;
        bool tr;
        PackedW *dst;
    };
    std::vector<Item> items;
    items.push_back({dW1p, d.d2b[0], a->KIN, false, &a->f2b[0]});
    items.push_back({dW1B, d.d2b[0], NB, true, &a->a2b[0]});
    prev = d.d2b[0];
    for (int q = 1; q < d.n2b; q++) {
        items.push_back({dev + oW[q], d.d2b[q], prev, false, &a->f2b[q]});
        items.push_back({dev + oW[q], d.d2b[q], prev, true, &a->a2b[q]});
        prev = d.d2b[q];
    }
    // Wv and We are adjacent: [Wv; We] is one 2NC x D matrix
    items.push_back({dev + oWv, 2 * NC, D, false, &a->fVE});
    items.push_back({dev + oWv, 2 * NC, D, true, &a->aVE});
    items.push_back({dev + oL1, LH, D + NC, false, &a->fL1});
    items.push_back({dev + oL1, LH, D + NC, true, &a->aL1});
    items.push_back({dev + oL2, D, LH, false, &a->fL2});
    items.push_back({dev + oL2, D, LH, true, &a->aL2});
    items.push_back({dev + oO1, OH, D, false, &a->fO1});
    items.push_back({dev + oO1, OH, D, true, &a->aO1});
    (void)oWe;
    size_t pk = 0;
    for (const Item &it : items) pk += packed_bytes(it.R, it.C, it.tr);
    int rc = hipMalloc(&a->pk_dev, pk) == hipSuccess ? 0 : -2;
    for (size_t q = 0, o = 0; rc == 0 && q < items.size(); q++) {
        if (pack_weight(nullptr, items[q].W, items[q].R, items[q].C, items[q].tr, (char *)a->pk_dev + o, items[q].dst))
            rc = -5;
        o += packed_bytes(items[q].R, items[q].C, items[q].tr);
    }
    if (rc == 0 && hipDeviceSynchronize() != hipSuccess) rc = -5;
    if (rc) {
        (void)hipGetLastError();
        if (a->pk_dev) hipFree(a->pk_dev);
        hipFree(dev);
        delete a;
        return fail(rc, "allegro: weight packing failed");
    }
    m->al = a;
    return 0;
}

void allegro_destroy(mlp_model *m) {
    if (!m || !m->al) return;
    if (m->al->pk_dev) hipFree(m->al->pk_dev);
    if (m->al->vec) hipFree(m->al->vec);
    delete m->al;
    m->al = nullptr;
}

// A GEMM over the edge rows: grid sized for the skin graph's edges, rows
// bounded by the pruned count on the device (Mc)
static int gm(hipStream_t s, int P, int epi, const float *A, int lda, const PackedW &B, float *C, int ldc, long M,
              const int *Mc, const float *bias = nullptr, float *C2 = nullptr, int ldc2 = 0, const float *R = nullptr,
              int ldr = 0) {
    if (M <= 0) return 0;
    ProfScope ps(PK_GEMM, s);
    return node_gemm(s, P, epi, A, lda, B, C, ldc, (int)M, bias, C2, ldc2, R, ldr, Mc) ? fail(-5, "allegro GEMM failed")
                                                                                       : 0;
}

int allegro_evaluate(mlp_model *m, mlp_nbr *g, hipStream_t s, double *energy, float *forces_user,
                     float *atom_energy_user, int n_seg, const int *seg_dev) {
    const AlModel &a = *m->al;
    const AlDims &d = a.d;
    const int n = g->n_atoms, P = node_operands(m->precision);
    // rows of every edge array: the skin graph's edge count bounds the pruned one
    const long E = g->n_edges_skin;
    int rc;
    if ((rc = g->act.ensure(allegro_arena_bytes(m, n, E), 1.2, &g->n_grows))) return rc;
    if ((rc = g->G.ensure(sizeof(float4) * (size_t)E + 64, 1.2, &g->n_grows))) return rc;
    const AlArena L = al_layout(a, n, E);
    float *base = g->act.as<float>();
    float *H0 = base + L.H0, *u = base + L.u, *GLc = base + L.GL, *Y = base + L.Y, *Yo = base + L.Yo, *LIN = base + L.LIN,
          *WV = base + L.WV, *PL = base + L.PL, *M = base + L.M, *X1 = base + L.X1, *PO = base + L.PO,
          *HO = base + L.HO, *GU = base + L.GU, *GWV = base + L.GWV, *GY = base + L.GY, *GB = base + L.GB,
          *ENV = base + L.ENV, *Uat = base + L.Uat;
    const int *rowc = g->rowc.as<int>(), *colc = g->colc.as<int>(), *perm = g->perm.as<int>();
    const float4 *geom = g->geom.as<float4>();
    const int ldl = d.D + d.NC, D = d.D;
    // edge kernels and GEMMs are sized for E rows and stop at the pruned
    // count, which lives on the device (rowc[n])
    const long ne = E;
    const int *cnt = rowc + n;

    // forward
    k_al_edge_in<<<nblk(n, 4), 256, 0, s>>>(rowc, colc, geom, g->species.as<int>(), perm, n, g->n_local, d.S, d.NB,
                                            d.p, a.KIN, d.rc, H0, u, Y, GLc);
    const float *in = H0;
    int ldin = a.KIN;
    for (int q = 0; q + 1 < d.n2b; q++) {
        float *Pq = base + L.P[q], *Aq = base + L.A[q];
        if ((rc = gm(s, P, GE_BIAS_SILU, in, ldin, a.f2b[q], Pq, d.d2b[q], ne, cnt, a.b2b[q], Aq, d.d2b[q]))) return rc;
        in = Aq;
        ldin = d.d2b[q];
    }
    if ((rc = gm(s, P, GE_BIAS, in, ldin, a.f2b[d.n2b - 1], Yo, D, ne, cnt, a.b2b[d.n2b - 1]))) return rc;
    k_al_scale_rows<<<nblk(ne * (D / 4), 256), 256, 0, s>>>(Yo, D, u, cnt, D, LIN, ldl);
    if ((rc = gm(s, P, GE_STORE, LIN, ldl, a.fVE, WV, 2 * d.NC, ne, cnt))) return rc;
    k_al_tp<<<nblk(n, 4), 256, 0, s>>>(rowc, n, d, Y, WV, ENV, LIN);
    {
        GemmChain c;
        c.e1 = GE_BIAS_SILU;
        c.e2 = GE_BIAS;
        c.A = LIN;
        c.lda = ldl;
        c.M = (int)ne;
        c.B1 = &a.fL1;
        c.C1 = PL;
        c.ldc1 = d.LH;
        c.bias1 = a.lat_b1;
        c.B2 = &a.fL2;
        c.C2 = M;
        c.ldc2 = D;
        c.bias2 = a.lat_b2;
        c.Mc = cnt;
        ProfScope ps(PK_GEMM, s);
        if (node_gemm_chain(s, P, c)) return fail(-5, "allegro latent GEMM failed");
    }
    k_al_x1<<<nblk(ne * (D / 4), 256), 256, 0, s>>>(LIN, ldl, u, M, cnt, D, X1);
    if ((rc = gm(s, P, GE_BIAS_SILU, X1, D, a.fO1, PO, d.OH, ne, cnt, a.out_b1, HO, d.OH))) return rc;
    k_al_energy<<<nblk(n, 4), 256, 0, s>>>(rowc, n, d.OH, HO, u, a.out_w2, a.out_b2_host, Uat);
    if ((rc = launch_energy(s, Uat, perm, n, g->n_local, energy, atom_energy_user, n_seg, seg_dev,
                            reinterpret_cast<double *>(base + L.EP))))
        return rc;
    if (!forces_user) return 0;

    // adjoint
    k_al_out_bwd<<<nblk(ne * 8, 256), 256, 0, s>>>(cnt, d.OH, PO, HO, u, GLc, a.out_w2, a.out_b2_host, GU);
    if ((rc = gm(s, P, GE_STORE, HO, d.OH, a.aO1, X1, D, ne, cnt))) return rc;
    k_al_x1_bwd<<<nblk(ne * 16, 256), 256, 0, s>>>(cnt, D, u, X1, M, GU);
    {
        GemmChain c;
        c.e1 = GE_DSILU;
        c.e2 = GE_STORE;
        c.A = M;
        c.lda = D;
        c.M = (int)ne;
        c.B1 = &a.aL2;
        c.R1 = PL;
        c.ldr1 = d.LH;
        c.B2 = &a.aL1;
        c.C2 = LIN;
        c.ldc2 = ldl;
        c.Mc = cnt;
        ProfScope ps(PK_GEMM, s);
        if (node_gemm_chain(s, P, c)) return fail(-5, "allegro latent adjoint GEMM failed");
    }
    const bool std_layout = d.lmax == 3 && d.ch[0] == 32 && d.ch[1] == 16 && d.ch[2] == 8 && d.ch[3] == 8;
    if (std_layout) k_al_tp_bwd<true><<<nblk(n, 4), 256, 0, s>>>(rowc, n, d, Y, WV, ENV, LIN, X1, GWV, GY);
    else k_al_tp_bwd<false><<<nblk(n, 4), 256, 0, s>>>(rowc, n, d, Y, WV, ENV, LIN, X1, GWV, GY);
    if ((rc = gm(s, P, GE_ADD, GWV, 2 * d.NC, a.aVE, X1, D, ne, cnt, nullptr, nullptr, 0, X1, D))) return rc;
    k_al_x0_bwd<<<nblk(ne * 16, 256), 256, 0, s>>>(cnt, D, u, X1, Yo, GU);
    // the two-body MLP in reverse: dE/dy in Yo, pre-activation gradients over the activations
    const float *gin = Yo;
    int ldg = D;
    for (int q = d.n2b - 1; q >= 1; q--) {
        float *Aq = base + L.A[q - 1], *Pq = base + L.P[q - 1];
        if ((rc = gm(s, P, GE_DSILU, gin, ldg, a.a2b[q], Aq, d.d2b[q - 1], ne, cnt, nullptr, nullptr, 0, Pq, d.d2b[q - 1])))
            return rc;
        gin = Aq;
        ldg = d.d2b[q - 1];
    }
    if ((rc = gm(s, P, GE_STORE, gin, ldg, a.a2b[0], GB, a.NBP, ne, cnt))) return rc;
    k_al_geom_bwd<<<(int)std::max<long>(1, std::min<long>(nblk(E, 256), 16384)), 256, 0, s>>>(
        rowc, n, geom, d.NB, a.NBP, d.p, d.rc, GB, GU, GY, g->G.as<float4>());
    HIP_TRY(hipGetLastError());
    return launch_forces(s, rowc, g->revc.as<int>(), g->G.as<float4>(), perm, n, forces_user);
}

}  // namespace mlp
