// Message pass and its adjoint with the radial-filter contraction on MFMA.
//
// Per directed edge (i <- j) the filter is w = A' e~(r), a dense K+1 -> 3F
// contraction with A' = [c | A] and e~ = [fc, e_1 fc, ..., e_K fc],
// e_k = sin(k pi r / rc) / r.  A wave owns one atom and takes its edges 16 at
// a time.  The filter of a chunk is computed as 16 x 16 MFMA tiles (16
// features x 16 edges) from two operands: 16 rows of A' (staged in LDS once
// per workgroup) and e~ of the 16 edges (each lane evaluates the basis slots
// it holds; the slots of padding edges are zero, so they contribute nothing).
// The vector phase works in the accumulator layout of the tiles; no LDS round
// trip sits between the matrix cores and the vector ALUs.  Features are
// processed in passes of W = min(F, 32).  Two arrangements:
//
// * One pass per workgroup (k_msg_fwd, k_msg_bwd: the first layer when it is
//   not factorised, and models with a single pass).  blockIdx.y is the pass;
//   A' is the first MFMA operand, so lane l = 16 g + e holds features
//   4g .. 4g+3 of the tile for edge e: it gathers the matching 16-byte pieces
//   of its edge's neighbour rows (quarter-contiguously, then moved through
//   LDS), sums over the features of an edge stay inside the lane (plus one
//   exchange across the four lane rows), sums over the edges of the atom stay
//   inside the lane over the chunks (plus one 16-lane DPP row reduction per
//   atom).  The basis is evaluated per pass.
// * All passes in the wave (k_msg_fwd_pw, k_msg_bwd_pw: the layers after the
//   first with more than one pass).  The weight images of every pass are in
//   LDS; the basis of a chunk, in MFMA operand form, is evaluated in the first
//   pass and kept in the wave's LDS for the later ones.  e~ is the first MFMA
//   operand, so the tile comes out transposed: lane (f, g) holds feature f of
//   the tile for the edges 4g .. 4g+3.  It gathers 16 consecutive features of
//   a row per quarter-wave (no exchange), adds its four edges in registers,
//   and the sums over an atom's edges reduce over the four lane rows once per
//   atom and pass; the adjoint's sums over the features of an edge go through
//   a reduce-scatter over the 16 lanes of a row.
//
// Precision P = 0: FP32 operands (v_mfma_f32_16x16x4_f32); P = 1: bfloat16
// operands (v_mfma_f32_16x16x32_bf16); P = 2: split bfloat16 operands
// x = hi + lo (hi = bf16(x), lo = bf16(x - hi)) with the three products
// lo*hi + hi*lo + hi*hi; accumulation FP32 in all.  Every sum has a fixed
// order, so results are bitwise reproducible.
//
// The adjoint is organised by source atom j over its in-edges (j <- i), the
// reverses of the edges (i <- j) that carried j's messages; it gathers the
// destination gradients and accumulates dE/dphi_j and dE/dv_j.  For every edge
// it also forms S = (dE/dr, dE/drhat) summed over the features (dE/dr through
// dw/dr = A' de~/dr, a second MFMA): one slot per layer (the all-pass kernel
// adds the passes up in the wave) or per layer and pass (one pass per
// workgroup), each written by one lane only.  The edge gradient
// G = dE/d(x_j - x_i) = (dE/dr) rhat + (I - rhat rhat^T) dE/drhat / r is linear
// in S and is assembled once after the last layer.
#include "internal.h"
#include "msg.h"

namespace mlp {

typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef float v2f __attribute__((ext_vector_type(2)));
typedef __bf16 v2bf __attribute__((ext_vector_type(2)));
typedef unsigned v4u __attribute__((ext_vector_type(4)));

template <int P, int K>
struct Basis {
    static constexpr int KP = P >= 1 ? 32 : ((K + 1 + 3) / 4) * 4;   // padded basis length
    static constexpr int NS = P >= 1 ? 1 : KP / 4;                    // MFMA k-steps
    static constexpr int SLOTS = P >= 1 ? 8 : NS;                     // basis values held per lane
};

// sin and cos of th in [0, pi] without range reduction: with x = th - pi/2 in
// [-pi/2, pi/2], sin th = cos x and cos th = -sin x, both from their Taylor
// series (through x^13 and x^14; truncation below 1e-9 on this interval).
__device__ __forceinline__ void sincos_0pi(float th, float &s, float &c) {
    const float x = th - 1.57079632679489662f, x2 = x * x;
    float p = 1.0f / 6227020800.0f;
    p = fmaf(p, x2, -1.0f / 39916800.0f);
    p = fmaf(p, x2, 1.0f / 362880.0f);
    p = fmaf(p, x2, -1.0f / 5040.0f);
    p = fmaf(p, x2, 1.0f / 120.0f);
    p = fmaf(p, x2, -1.0f / 6.0f);
    p = fmaf(p, x2, 1.0f);
    float q = -1.0f / 87178291200.0f;
    q = fmaf(q, x2, 1.0f / 479001600.0f);
    q = fmaf(q, x2, -1.0f / 3628800.0f);
    q = fmaf(q, x2, 1.0f / 40320.0f);
    q = fmaf(q, x2, -1.0f / 720.0f);
    q = fmaf(q, x2, 1.0f / 24.0f);
    q = fmaf(q, x2, -0.5f);
    q = fmaf(q, x2, 1.0f);
    s = q;
    c = -x * p;
}

// Basis values (and optionally their r-derivatives) for the slots a lane
// holds: bf16 slots k = 8g + q (q = 0..7), f32 slots k = g + 4q (q = 0..NS-1).
// r < rc for every valid edge, so th = pi r / rc lies in [0, pi).  The lane's
// first angle k0 th comes from angle doubling, the rest from the Chebyshev
// recurrences sin((k+d) th) = 2 cos(d th) sin(k th) - sin((k-d) th) (and the
// same for cos).  Slots k > K meet zero weight columns, so their values do not
// matter as long as they are finite.  Padding edges (valid = false, ir = 0)
// get exact zeros.
template <int P, int K, bool DERIV>
__device__ __forceinline__ void basis_slots(float r, float ir, float pirc, bool valid, int g, float *eb, float *db) {
    constexpr int SL = Basis<P, K>::SLOTS;
    float s1, c1;
    sincos_0pi(r * pirc, s1, c1);
    const float fc = valid ? 0.5f * (c1 + 1.0f) : 0.f;
    const float dfc = valid ? -0.5f * pirc * s1 : 0.f;
    const float es = ir * fc;                    // e_k = sin(k th) es
    const float da = pirc * es, dbb = ir * (dfc - es);   // de_k = cos(k th) k da + sin(k th) dbb
    const float s2 = 2.0f * s1 * c1, c2 = fmaf(-2.0f * s1, s1, 1.0f);
    const float s4 = 2.0f * s2 * c2, c4 = fmaf(-2.0f * s2, s2, 1.0f);
    float sk, ck, sm, cm, tc;
    int k0, step;
    if constexpr (P >= 1) {
        const float s8 = 2.0f * s4 * c4, c8 = fmaf(-2.0f * s4, s4, 1.0f);
        const float s16 = 2.0f * s8 * c8, c16 = fmaf(-2.0f * s8, s8, 1.0f);
        const float s24 = fmaf(s16, c8, c16 * s8), c24 = fmaf(c16, c8, -s16 * s8);
        sk = g == 0 ? 0.f : (g == 1 ? s8 : (g == 2 ? s16 : s24));
        ck = g == 0 ? 1.f : (g == 1 ? c8 : (g == 2 ? c16 : c24));
        sm = fmaf(sk, c1, -ck * s1);   // sin((k0 - 1) th)
        cm = fmaf(ck, c1, sk * s1);
        tc = 2.0f * c1;
        k0 = 8 * g;
        step = 1;
    } else {
        const float s3 = fmaf(s2, c1, c2 * s1), c3 = fmaf(c2, c1, -s2 * s1);
        sk = g == 0 ? 0.f : (g == 1 ? s1 : (g == 2 ? s2 : s3));
        ck = g == 0 ? 1.f : (g == 1 ? c1 : (g == 2 ? c2 : c3));
        sm = fmaf(sk, c4, -ck * s4);   // sin((k0 - 4) th)
        cm = fmaf(ck, c4, sk * s4);
        tc = 2.0f * c4;
        k0 = g;
        step = 4;
    }
#pragma unroll
    for (int q = 0; q < SL; q++) {
        float e = sk * es, de = 0.f;
        if (DERIV) de = fmaf(ck, (float)(k0 + step * q) * da, sk * dbb);
        if (q == 0 && g == 0) {   // k = 0: the envelope itself
            e = fc;
            de = dfc;
        }
        eb[q] = e;
        if (DERIV) db[q] = de;
        const float sn = fmaf(tc, sk, -sm);
        sm = sk;
        sk = sn;
        if (DERIV) {
            const float cn = fmaf(tc, ck, -cm);
            cm = ck;
            ck = cn;
        }
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
    // pairs go through the packed conversion, and hi is widened back from
    // the packed word, so each value costs one conversion half, one shift or
    // mask and one subtraction
    __device__ __forceinline__ void set(const float *eb) {
        v4u hv, lv;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            // element 2q is the low half of word q, element 2q + 1 the high half
            const unsigned hw = __builtin_bit_cast(unsigned, __builtin_convertvector((v2f){eb[2 * q], eb[2 * q + 1]}, v2bf));
            const float h0 = __uint_as_float(hw << 16), h1 = __uint_as_float(hw & 0xffff0000u);
            hv[q] = hw;
            lv[q] = __builtin_bit_cast(unsigned, __builtin_convertvector((v2f){eb[2 * q] - h0, eb[2 * q + 1] - h1}, v2bf));
        }
        v = __builtin_bit_cast(v8bf, hv);
        lo = __builtin_bit_cast(v8bf, lv);
    }
};

// Features per pass (at most WM) and the pass count.
template <int F, int WM>
struct Pass {
    static constexpr int W = F < WM ? F : WM;   // features per pass
    static constexpr int N = F / W;             // passes
    static constexpr int TU = W / 16;           // 16-feature tiles per part and pass
};

// LDS image of the pass's rows of A' = [c | A]: local row q W + f holds the
// global row q F + p W + f (part q = 0, 1, 2), in the layout the A operand
// reads (reduction index contiguous).  Rows are padded against bank
// conflicts (8 bf16 or one float), or, with SW (bf16 only), unpadded and
// swizzled: a 64-byte row is four 16-byte pieces of 8 slots, and piece h of
// row r sits at position h ^ wswz(r), which puts the 16 rows that one
// A-operand read touches (same piece, rows 16 t .. 16 t + 15) on distinct
// 16-byte bank groups for 32 or 64 banks, in 20 % less LDS.
template <int P, int F, int K, int WM, bool SW = false>
struct WStage {
    static constexpr bool SWZ = SW && P >= 1;
    static constexpr int KP = Basis<P, K>::KP;
    static constexpr int ROWS = 3 * Pass<F, WM>::W;
    static constexpr int LD = SWZ ? KP : (P >= 1 ? KP + 8 : KP + 1);   // row stride (elements)
    static constexpr int ELEMS = ROWS * LD * (P == 2 ? 2 : 1);         // split mode: hi table, then lo table
    static constexpr int BYTES = ELEMS * (P >= 1 ? 2 : 4);
};
__device__ __forceinline__ int wswz(int r) { return (((r >> 2) & 1) << 1) | (((r >> 1) ^ (r >> 3)) & 1); }

template <int P, int F, int K, int WM, bool SW = false>
__device__ __forceinline__ void stage_pass(const float *__restrict__ A, const float *__restrict__ c, int p,
                                           void *lds) {
    using WS = WStage<P, F, K, WM, SW>;
    constexpr int W = Pass<F, WM>::W;
    for (int idx = threadIdx.x; idx < WS::ROWS * WS::KP; idx += blockDim.x) {
        const int lr = idx / WS::KP, k = idx % WS::KP;
        const int f = (lr / W) * F + p * W + lr % W;
        float v = 0.f;
        if (k == 0) v = c[f];
        else if (k <= K) v = A[(long)f * K + (k - 1)];
        if (P >= 1) {
            const __bf16 h = (__bf16)v;
            const int at = lr * WS::LD + (WS::SWZ ? ((((k >> 3) ^ wswz(lr)) << 3) | (k & 7)) : k);
            reinterpret_cast<__bf16 *>(lds)[at] = h;
            if (P == 2) reinterpret_cast<__bf16 *>(lds)[WS::ROWS * WS::LD + at] = (__bf16)(v - (float)h);
        } else {
            reinterpret_cast<float *>(lds)[lr * WS::LD + k] = v;
        }
    }
    __syncthreads();
}

// Filter values of local tile t (rows 16t .. 16t+15): lane (e, g) receives
// features 4g .. 4g+3 of the tile for its edge e; with TR (the operands
// swapped, the same products) lane (f, g) receives feature f of the tile for
// the edges 4g .. 4g+3.
template <int P, int F, int K, int WM, bool SW = false, bool TR = false>
__device__ __forceinline__ v4f filter_tile(const void *lds, int t, const BOp<P, K> &b, int lane) {
    using WS = WStage<P, F, K, WM, SW>;
    v4f acc = {0.f, 0.f, 0.f, 0.f};
    const int row = 16 * t + (lane & 15), g = lane >> 4;
    // the swizzled piece position depends on the lane only (16 t leaves bits
    // 1-3 of the row alone)
    const int col = 8 * (WS::SWZ ? g ^ wswz(lane & 15) : g);
    if constexpr (P == 1) {
        const v8bf a = *reinterpret_cast<const v8bf *>(reinterpret_cast<const __bf16 *>(lds) + row * WS::LD + col);
        if constexpr (TR) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b.v, a, acc, 0, 0, 0);
        else acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b.v, acc, 0, 0, 0);
    } else if constexpr (P == 2) {
        const __bf16 *t0 = reinterpret_cast<const __bf16 *>(lds) + row * WS::LD + col;
        const v8bf a = *reinterpret_cast<const v8bf *>(t0);
        const v8bf al = *reinterpret_cast<const v8bf *>(t0 + WS::ROWS * WS::LD);
        if constexpr (TR) {
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b.v, al, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b.lo, a, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(b.v, a, acc, 0, 0, 0);
        } else {
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, b.v, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b.lo, acc, 0, 0, 0);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b.v, acc, 0, 0, 0);
        }
    } else {
        const float *w = reinterpret_cast<const float *>(lds) + row * WS::LD;
#pragma unroll
        for (int s = 0; s < Basis<P, K>::NS; s++) {
            if constexpr (TR) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(b.v[s], w[4 * s + g], acc, 0, 0, 0);
            else acc = __builtin_amdgcn_mfma_f32_16x16x4f32(w[4 * s + g], b.v[s], acc, 0, 0, 0);
        }
    }
    return acc;
}

// DPP move inside rows of 16 lanes.
template <int CTRL>
__device__ __forceinline__ float dpp(float x) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xF, 0xF, false));
}

// Sum over the 16 lanes of each row (lanes 16g .. 16g+15), by rotations of the
// row and quad permutations; every lane of the row receives the total.
__device__ __forceinline__ float row_sum16(float x) {
    x += dpp<0x128>(x);   // row_ror:8
    x += dpp<0x124>(x);   // row_ror:4
    x += dpp<0x4E>(x);    // quad_perm [2,3,0,1]
    x += dpp<0xB1>(x);    // quad_perm [1,0,3,2]
    // materialise the total here: otherwise the last add sinks into the
    // lane-0 store branch, where it cannot take the DPP operand and costs a
    // zeroed register, a DPP move and a plain add per value
    asm volatile("" : "+v"(x));
    return x;
}

// The weight image, at an offset the compiler cannot see through, so the A
// operands are re-read from LDS in every chunk instead of being held in 48
// registers across the chunk loop (which would cost occupancy).
__device__ __forceinline__ const char *lds_chunk(const char *lds) {
    int z = 0;
    asm volatile("" : "+s"(z));
    return lds + z;
}

__device__ __forceinline__ v4f ld4(const float *p) { return *reinterpret_cast<const v4f *>(p); }
__device__ __forceinline__ void st4(float *p, v4f x) { *reinterpret_cast<v4f *>(p) = x; }

// Neighbour rows are gathered quarter-contiguously and then moved to the
// accumulator layout through LDS.  In the accumulator layout lane (g, e) =
// 16 g + e needs features 4g .. 4g+3 (of a 16-feature tile) of edge e, so
// the 16 lanes of a quarter-wave would touch 16 different rows, 16 bytes
// each: the L1 then serves one 16-byte piece per access.  Instead lane
// (g, e) loads features 4(e % 4) .. +3 of the row of edge 4g + e/4 (each
// quarter reads four whole 64-byte pieces) and stores them in LDS at the
// slot of the lane that needs them, 16(e % 4) + 4g + e/4, from where every
// lane reads its own slot.  Slot D sits at index swz(D): its bits 2-3 are
// XOR-ed with its quarter, which keeps the writes and the reads of a
// quarter-wave on 16 distinct 16-byte bank groups.
struct Xch {
    int src;   // lane holding the edge whose row this lane gathers
    int fo;    // feature offset of the gathered piece inside a 16-feature tile
    int wr;    // LDS slot this lane writes
    int rd;    // LDS slot this lane reads
    __device__ static int swz(int d) { return (d & 0x33) | ((((d >> 2) & 3) ^ (d >> 4)) << 2); }
    __device__ Xch(int g, int e) {
        src = 4 * g + (e >> 2);
        fo = 4 * (e & 3);
        wr = swz(16 * (e & 3) + 4 * g + (e >> 2));
        rd = swz(16 * g + e);
    }
    // one 64-lane, 16-byte-per-lane exchange through the wave's buffer slot
    __device__ v4f move(v4f *buf, v4f x) const {
        buf[wr] = x;
        __builtin_amdgcn_wave_barrier();   // the read sees the whole wave's writes
        return buf[rd];
    }
};

#ifndef MSG_MW
#define MSG_MW 4
#endif
constexpr int MW = MSG_MW;   // waves per workgroup
// features per pass of the forward and the adjoint (16 or 32)
#ifndef FWD_W
#define FWD_W 32
#endif
#ifndef BWD_W
#define BWD_W 32
#endif
#ifndef FWD_WAVES
#define FWD_WAVES 4
#endif
#ifndef FWD_WAVES0
#define FWD_WAVES0 5
#endif
#ifndef BWD_WAVES0
#define BWD_WAVES0 4
#endif
#ifndef BWD_WAVES
#define BWD_WAVES 2
#endif

// Atoms for each wave, from a work queue per XCD slice.  Workgroups are
// dispatched round-robin over the XCDs, each with its own L2; with gridDim.x
// a multiple of 8, XCD x runs the workgroups with blockIdx.x % 8 == x and
// works on the contiguous slice [x n / 8, (x+1) n / 8) of the cell-sorted
// atoms.  The waves of a slice take its atoms in order, MSG_QB at a time, from
// one counter, so the atoms in flight on an XCD are always a compact window of
// the slice, whose neighbour rows the XCD's L2 holds (with a fixed
// interleaving the waves drift apart over the slice and the rows in use
// outgrow the L2).  Each counter has its own 128-byte line and starts at
// zero.  The slices partition [0, n) whatever the grid size; every wave leaves
// its loop once its slice's counter has passed the end.
#ifndef MSG_QB
#define MSG_QB 1
#endif
struct AtomQueue {
    int lo, hi;
    int *ctr;
    __device__ __forceinline__ AtomQueue(int n, int *queue, int pass) {
        const int nx = gridDim.x < 8 ? (int)gridDim.x : 8;
        const int x = blockIdx.x % nx;
        lo = (int)((long)n * x / nx);
        hi = (int)((long)n * (x + 1) / nx);
        ctr = queue + (pass * 8 + x) * 32;
    }
    // a ticket: the counter's old value in lane 0 (issue), and the first atom
    // of the wave's batch it names (wave-uniform; >= hi once the slice is
    // drained), read only when needed (resolve), so the atomic's latency can
    // pass under other work
    __device__ __forceinline__ int issue() const {
        int t = 0;
        if ((threadIdx.x & 63) == 0)
            t = __hip_atomic_fetch_add(ctr, MSG_QB, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        return t;
    }
    __device__ __forceinline__ int resolve(int t) const { return lo + __builtin_amdgcn_readfirstlane(t); }
    __device__ __forceinline__ int take() const { return resolve(issue()); }
};
// for (each atom I of the wave, in queue order)
#if MSG_QB == 1
#define MSG_ATOMS(Q, I) for (int I = (Q).take(); I < (Q).hi; I = (Q).take())
// The same with the next ticket issued when an atom starts and resolved when
// it ends, so the atomic's latency passes under the atom's work (the last
// one is not used).  Each wave then holds two tickets, which doubles the
// window of atoms in flight: worth it in the adjoint (2 waves per SIMD), not
// in the forward, whose L2 then holds its window's rows less well.
#define MSG_ATOMS_AHEAD(Q, I)                                                \
    for (int I = (Q).take(), I##_t = (Q).issue(); I < (Q).hi; I = (Q).resolve(I##_t), I##_t = (Q).issue())
#else
#define MSG_ATOMS(Q, I)                                           \
    for (int I##_b = (Q).take(); I##_b < (Q).hi; I##_b = (Q).take()) \
        for (int I = I##_b; I < I##_b + MSG_QB && I < (Q).hi; I++)
#define MSG_ATOMS_AHEAD(Q, I) MSG_ATOMS(Q, I)
#endif

// A chunk's B operand kept in LDS between passes: 16-byte words per lane
// (FP32 mode: 4-byte words), stored lane-contiguously so that the writes
// and reads are conflict-free.  Each lane reads back only what it wrote
// itself, so no barrier is needed.
template <int P, int K>
struct BOpStore {
    static constexpr int WBYTES = P >= 1 ? 16 : 4;                            // bytes per word
    static constexpr int WORDS = P == 2 ? 2 : (P == 1 ? 1 : Basis<P, K>::NS); // words per lane
    static constexpr int BYTES = WORDS * WBYTES * 64;                         // per operand and wave
};
template <int P, int K>
__device__ __forceinline__ void bop_put(char *slot, int lane, const BOp<P, K> &b) {
    if constexpr (P >= 1) {
        v4f *q = reinterpret_cast<v4f *>(slot) + lane;
        q[0] = __builtin_bit_cast(v4f, b.v);
        if constexpr (P == 2) q[64] = __builtin_bit_cast(v4f, b.lo);
    } else {
        float *q = reinterpret_cast<float *>(slot) + lane;
#pragma unroll
        for (int s = 0; s < Basis<P, K>::NS; s++) q[64 * s] = b.v[s];
    }
}
template <int P, int K>
__device__ __forceinline__ void bop_get(const char *slot, int lane, BOp<P, K> &b) {
    if constexpr (P >= 1) {
        const v4f *q = reinterpret_cast<const v4f *>(slot) + lane;
        b.v = __builtin_bit_cast(v8bf, q[0]);
        if constexpr (P == 2) b.lo = __builtin_bit_cast(v8bf, q[64]);
    } else {
        const float *q = reinterpret_cast<const float *>(slot) + lane;
#pragma unroll
        for (int s = 0; s < Basis<P, K>::NS; s++) b.v[s] = q[64 * s];
    }
}

// ---------------------------------------------------------------------------
// Forward message pass, one feature pass (blockIdx.y) per workgroup: the
// first layer, and models with a single pass.
// ---------------------------------------------------------------------------
template <int P, int F, int K, bool V0>
__global__ void __launch_bounds__(64 * MW) __attribute__((amdgpu_waves_per_eu(V0 ? FWD_WAVES0 : FWD_WAVES))) k_msg_fwd(const int *__restrict__ rowc, const int *__restrict__ colc,
                                                     const float4 *__restrict__ geom, int n,
                                                     const float *__restrict__ phi, const float *__restrict__ uvp,
                                                     const float *__restrict__ s, const float *__restrict__ v,
                                                     const float *__restrict__ Aw,
                                                     const float *__restrict__ cw, float rc,
                                                     const int8_t *__restrict__ hop, int hop_max,
                                                     const int *__restrict__ zsp, int *__restrict__ queue,
                                                     float *__restrict__ sn, float *__restrict__ v1) {
    constexpr int WM = FWD_W;
    constexpr int F3 = 3 * F, SL = Basis<P, K>::SLOTS, W = Pass<F, WM>::W, TU = Pass<F, WM>::TU;
    __shared__ __attribute__((aligned(16))) char lds[WStage<P, F, K, WM>::BYTES];
    // first layer: phi and s are per-species tables (rows by zsp), a few rows
    // that every gather hits in L1, read directly in the accumulator layout
    __shared__ v4f xch[MW][V0 ? 1 : 5][64];
    const int p = blockIdx.y;
    stage_pass<P, F, K, WM>(Aw, cw, p, lds);
    const int lane = threadIdx.x & 63, e = lane & 15, g = lane >> 4;
    const int fo = p * W + 4 * g;   // first feature of this lane (tile u adds 16 u)
    const Xch xc(g, e);
    v4f(*xw)[64] = xch[threadIdx.x >> 6];
    const AtomQueue aq(n, queue, p);
    const float pirc = 3.14159265358979f / rc;
    MSG_ATOMS(aq, i) {
        const int e0 = rowc[i], e1 = rowc[i + 1];
        const int deg = hop[i] <= hop_max ? e1 - e0 : 0;
        v4f as[TU], av[3][TU];
#pragma unroll
        for (int u = 0; u < TU; u++) {
            as[u] = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int d = 0; d < 3; d++) av[d][u] = v4f{0.f, 0.f, 0.f, 0.f};
        }
        // edge records of the next chunk are loaded one chunk ahead
        float4 gm_n = make_float4(0.f, 0.f, 0.f, rc);
        int j_n = i;
        if (e < deg) {
            gm_n = geom[e0 + e];
            j_n = colc[e0 + e];
        }
        for (int cb = 0; cb < deg; cb += 16) {
            const char *wl = lds_chunk(lds);
            const bool valid = cb + e < deg;
            const float4 gm = gm_n;
            const int j = j_n;
            gm_n = make_float4(0.f, 0.f, 0.f, rc);
            j_n = i;
            if (cb + 16 + e < deg) {
                gm_n = geom[e0 + cb + 16 + e];
                j_n = colc[e0 + cb + 16 + e];
            }
            // gathered: phi_s, phi_vs and (after the first layer) u = v * phi_vv
            // of the source (5 row slices, quarter-contiguously, then moved to
            // the accumulator layout; the first layer's 2 from the table)
            v4f ph[2][TU], uu[3][TU];
            if constexpr (V0) {
                const float *pj = phi + (long)zsp[j] * F3 + fo;
#pragma unroll
                for (int u = 0; u < TU; u++) {
                    ph[0][u] = ld4(pj + F + 16 * u);
                    ph[1][u] = ld4(pj + 2 * F + 16 * u);
                }
            } else {
                const int jq = __shfl(j, xc.src, 64);
                const float *pj = phi + (long)jq * F3 + p * W + xc.fo;
                const float *uj = uvp + (long)jq * F3 + p * W + xc.fo;
#pragma unroll
                for (int u = 0; u < TU; u++) {
                    ph[0][u] = ld4(pj + F + 16 * u);
                    ph[1][u] = ld4(pj + 2 * F + 16 * u);
#pragma unroll
                    for (int d = 0; d < 3; d++) uu[d][u] = ld4(uj + d * F + 16 * u);
                }
#pragma unroll
                for (int u = 0; u < TU; u++) {
                    ph[0][u] = xc.move(xw[0], ph[0][u]);
                    ph[1][u] = xc.move(xw[1], ph[1][u]);
#pragma unroll
                    for (int d = 0; d < 3; d++) uu[d][u] = xc.move(xw[2 + d], uu[d][u]);
                }
            }
            const float ir = valid ? __builtin_amdgcn_rcpf(gm.w) : 0.f;
            float eb[SL];
            basis_slots<P, K, false>(gm.w, ir, pirc, valid, g, eb, nullptr);
            BOp<P, K> bop;
            bop.set(eb);
            const float rx = gm.x * ir, ry = gm.y * ir, rz = gm.z * ir;
#pragma unroll
            for (int u = 0; u < TU; u++) {
                v4f wvv;
                if constexpr (!V0) wvv = filter_tile<P, F, K, WM>(wl, u, bop, lane);
                const v4f ws = filter_tile<P, F, K, WM>(wl, TU + u, bop, lane);
                const v4f wvs = filter_tile<P, F, K, WM>(wl, 2 * TU + u, bop, lane);
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const float xvs = ph[1][u][r] * wvs[r];
                    as[u][r] = fmaf(ph[0][u][r], ws[r], as[u][r]);
                    if constexpr (V0) {
                        av[0][u][r] = fmaf(rx, xvs, av[0][u][r]);
                        av[1][u][r] = fmaf(ry, xvs, av[1][u][r]);
                        av[2][u][r] = fmaf(rz, xvs, av[2][u][r]);
                    } else {
                        av[0][u][r] = fmaf(uu[0][u][r], wvv[r], fmaf(rx, xvs, av[0][u][r]));
                        av[1][u][r] = fmaf(uu[1][u][r], wvv[r], fmaf(ry, xvs, av[1][u][r]));
                        av[2][u][r] = fmaf(uu[2][u][r], wvv[r], fmaf(rz, xvs, av[2][u][r]));
                    }
                }
            }
        }
        // sum over the 16 edge lanes of each row
#pragma unroll
        for (int u = 0; u < TU; u++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                as[u][r] = row_sum16(as[u][r]);
#pragma unroll
                for (int d = 0; d < 3; d++) av[d][u][r] = row_sum16(av[d][u][r]);
            }
        if (e == 0) {
#pragma unroll
            for (int u = 0; u < TU; u++) {
                const int f = fo + 16 * u;
                const long si = V0 ? (long)zsp[i] : (long)i;
                st4(sn + (long)i * 2 * F + f, ld4(s + si * F + f) + as[u]);
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    if constexpr (V0) st4(v1 + (long)i * F3 + d * F + f, av[d][u]);
                    else st4(v1 + (long)i * F3 + d * F + f, ld4(v + (long)i * F3 + d * F + f) + av[d][u]);
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Forward message pass of the layers after the first with more than one
// feature pass: every wave runs all passes of its atom, with the weight
// images of every pass in LDS, and the radial basis of a chunk, in MFMA
// operand form, is evaluated in the first pass and kept in the wave's LDS for
// the later ones (the first FWD_CACHE chunks of the atom).  The filter tiles
// come out transposed (filter_tile with TR): lane (f, g) holds feature f of
// the tile for the edges 4g .. 4g+3, so it gathers 16 consecutive features
// of one source row per quarter-wave and register (no exchange), adds its
// four edges in registers, and the sums over the atom's edges need only a
// sum over the four lane rows at the end.  The basis is evaluated in the
// layout the MFMA operand takes (lane (e, g): slots of edge e); the source
// index and direction of the edges 4g + r move to the vector layout by lane
// shuffles.
// ---------------------------------------------------------------------------
#ifndef FWD_PIW_WAVES
#define FWD_PIW_WAVES 16
#endif
#ifndef FWD_CACHE
#define FWD_CACHE 3
#endif
template <int P, int F, int K>
__global__ void __launch_bounds__(64 * FWD_PIW_WAVES) __attribute__((amdgpu_waves_per_eu(FWD_WAVES))) k_msg_fwd_pw(const int *__restrict__ rowc, const int *__restrict__ colc,
                                                     const float4 *__restrict__ geom, int n,
                                                     const float *__restrict__ phi, const float *__restrict__ uvp,
                                                     const float *__restrict__ s, const float *__restrict__ v,
                                                     const float *__restrict__ Aw,
                                                     const float *__restrict__ cw, float rc,
                                                     const int8_t *__restrict__ hop, int hop_max,
                                                     int *__restrict__ queue,
                                                     float *__restrict__ sn, float *__restrict__ v1) {
    constexpr int WM = FWD_W;
    constexpr int F3 = 3 * F, SL = Basis<P, K>::SLOTS, W = Pass<F, WM>::W, TU = Pass<F, WM>::TU;
    constexpr int NP = Pass<F, WM>::N, NC = FWD_CACHE;
    constexpr int WB = WStage<P, F, K, WM, true>::BYTES;
    constexpr int CB = BOpStore<P, K>::BYTES;
    __shared__ __attribute__((aligned(16))) char lds[NP * WB];
    __shared__ __attribute__((aligned(16))) char bcache[FWD_PIW_WAVES * NC * CB];
#pragma unroll 1
    for (int q = 0; q < NP; q++) stage_pass<P, F, K, WM, true>(Aw, cw, q, lds + q * WB);
    const int lane = threadIdx.x & 63, e = lane & 15, g = lane >> 4;
    char *bc = bcache + (threadIdx.x >> 6) * NC * CB;
    const AtomQueue aq(n, queue, 0);
    const float pirc = 3.14159265358979f / rc;
    MSG_ATOMS(aq, i) {
        const int e0 = rowc[i], e1 = rowc[i + 1];
        const int deg = hop[i] <= hop_max ? e1 - e0 : 0;
#pragma unroll 1
        for (int p = 0; p < NP; p++) {
            const int fl = p * W + e;   // this lane's feature (tile u adds 16 u)
            float as[TU], av[3][TU];
#pragma unroll
            for (int u = 0; u < TU; u++) {
                as[u] = 0.f;
#pragma unroll
                for (int d = 0; d < 3; d++) av[d][u] = 0.f;
            }
            // edge records (edge e of the chunk) are loaded one chunk ahead
            float4 gm_n = make_float4(0.f, 0.f, 0.f, rc);
            int j_n = i;
            if (e < deg) {
                gm_n = geom[e0 + e];
                j_n = colc[e0 + e];
            }
            for (int cb = 0; cb < deg; cb += 16) {
                const char *wl = lds_chunk(lds + p * WB);
                const bool valid = cb + e < deg;
                const float4 gm = gm_n;
                const int j = j_n;
                gm_n = make_float4(0.f, 0.f, 0.f, rc);
                j_n = i;
                if (cb + 16 + e < deg) {
                    gm_n = geom[e0 + cb + 16 + e];
                    j_n = colc[e0 + cb + 16 + e];
                }
                const float ir = valid ? __builtin_amdgcn_rcpf(gm.w) : 0.f;
                const float rx = gm.x * ir, ry = gm.y * ir, rz = gm.z * ir;
                // source rows and directions of this lane's edges 4g + r (padding
                // edges: the atom's own row and a zero direction; their filter is 0)
                int jr[4];
                float hx[4], hy[4], hz[4];
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int src = 4 * g + r;
                    jr[r] = __shfl(j, src, 64);
                    hx[r] = __shfl(rx, src, 64);
                    hy[r] = __shfl(ry, src, 64);
                    hz[r] = __shfl(rz, src, 64);
                }
                float ps[TU][4], pv[TU][4], uu[3][TU][4];
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const float *pj = phi + (long)jr[r] * F3 + fl;
                    const float *uj = uvp + (long)jr[r] * F3 + fl;
#pragma unroll
                    for (int u = 0; u < TU; u++) {
                        ps[u][r] = pj[F + 16 * u];
                        pv[u][r] = pj[2 * F + 16 * u];
#pragma unroll
                        for (int d = 0; d < 3; d++) uu[d][u][r] = uj[d * F + 16 * u];
                    }
                }
                BOp<P, K> bop;
                const int c = cb >> 4;
                if (p > 0 && c < NC) {
                    bop_get<P, K>(bc + c * CB, lane, bop);
                } else {
                    float eb[SL];
                    basis_slots<P, K, false>(gm.w, ir, pirc, valid, g, eb, nullptr);
                    bop.set(eb);
                    if (p == 0 && c < NC) bop_put<P, K>(bc + c * CB, lane, bop);
                }
#pragma unroll
                for (int u = 0; u < TU; u++) {
                    const v4f wvv = filter_tile<P, F, K, WM, true, true>(wl, u, bop, lane);
                    const v4f ws = filter_tile<P, F, K, WM, true, true>(wl, TU + u, bop, lane);
                    const v4f wvs = filter_tile<P, F, K, WM, true, true>(wl, 2 * TU + u, bop, lane);
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const float xvs = pv[u][r] * wvs[r];
                        as[u] = fmaf(ps[u][r], ws[r], as[u]);
                        av[0][u] = fmaf(uu[0][u][r], wvv[r], fmaf(hx[r], xvs, av[0][u]));
                        av[1][u] = fmaf(uu[1][u][r], wvv[r], fmaf(hy[r], xvs, av[1][u]));
                        av[2][u] = fmaf(uu[2][u][r], wvv[r], fmaf(hz[r], xvs, av[2][u]));
                    }
                }
            }
            // sum over the four lane rows (edges 4g .. 4g+3 of every chunk)
#pragma unroll
            for (int u = 0; u < TU; u++) {
                as[u] += __shfl_xor(as[u], 16, 64);
                as[u] += __shfl_xor(as[u], 32, 64);
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    av[d][u] += __shfl_xor(av[d][u], 16, 64);
                    av[d][u] += __shfl_xor(av[d][u], 32, 64);
                }
            }
            if (g == 0) {
#pragma unroll
                for (int u = 0; u < TU; u++) {
                    const int f = fl + 16 * u;
                    sn[(long)i * 2 * F + f] = s[(long)i * F + f] + as[u];
#pragma unroll
                    for (int d = 0; d < 3; d++)
                        v1[(long)i * F3 + d * F + f] = v[(long)i * F3 + d * F + f] + av[d][u];
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint of the message pass, one feature pass (blockIdx.y) per workgroup:
// the first layer, and models with a single pass.
// Per chunk of 16 in-edges (j <- i) of the source atom j: the filter tiles and
// their radial derivatives on MFMA, the destinations' gradient pieces
// gathered per lane, dE/dphi_j and dE/dv_j accumulated in registers, and the
// edge sums S = (dE/dr, dE/drhat) of the pass stored in the pass's slot.
// ---------------------------------------------------------------------------
template <int P, int F, int K, bool V0>
__global__ void __launch_bounds__(64 * MW) __attribute__((amdgpu_waves_per_eu(V0 ? BWD_WAVES0 : BWD_WAVES))) k_msg_bwd(const int *__restrict__ rowc, const int *__restrict__ colc,
                                                     const float4 *__restrict__ geom, int n,
                                                     const float *__restrict__ phi, const float *__restrict__ v,
                                                     const float *__restrict__ gs1, const float *__restrict__ gv1,
                                                     const float *__restrict__ Aw, const float *__restrict__ cw,
                                                     float rc, const int8_t *__restrict__ hop, int hop_max,
                                                     const int *__restrict__ zsp, int *__restrict__ queue,
                                                     float *__restrict__ gv_in, float *__restrict__ gphi,
                                                     float4 *__restrict__ S, long s_stride) {
    constexpr int WM = BWD_W;
    constexpr int F3 = 3 * F, SL = Basis<P, K>::SLOTS, W = Pass<F, WM>::W, TU = Pass<F, WM>::TU;
    __shared__ __attribute__((aligned(16))) char lds[WStage<P, F, K, WM>::BYTES];
    __shared__ v4f xch[MW][4][64];
    const int p = blockIdx.y;
    stage_pass<P, F, K, WM>(Aw, cw, p, lds);
    float4 *Sp = S + (long)p * s_stride;
    const int lane = threadIdx.x & 63, e = lane & 15, g = lane >> 4;
    const int fo = p * W + 4 * g;
    const Xch xc(g, e);
    v4f(*xw)[64] = xch[threadIdx.x >> 6];
    const AtomQueue aq(n, queue, p);
    const float pirc = 3.14159265358979f / rc;
    MSG_ATOMS(aq, j) {
        const int e0 = rowc[j], e1 = rowc[j + 1];
        const int deg = hop[j] <= hop_max ? e1 - e0 : 0;
        // first layer: v_j = 0 and no node gradient, so phi_vv, v_j, dE/dphi_j
        // and dE/dv_j drop out and only the edge sums remain.
        // Later layers accumulate Y_d = sum_e dE/dv1_d(i) w_vv (from which both
        // dE/dv_j = phi_vv Y_d and dE/dphi_vv = sum_d v_jd Y_d follow once per
        // atom), dE/dphi_s and dE/dphi_vs; the v_j term of dE/dr enters through
        // c_d = v_jd phi_vv.
        v4f ph[3][TU], cv[3][TU], Y[3][TU], ap[2][TU];
#pragma unroll
        for (int u = 0; u < TU; u++) {
#pragma unroll
            for (int q = V0 ? 1 : 0; q < 3; q++) ph[q][u] = ld4(phi + (V0 ? (long)zsp[j] : (long)j) * F3 + q * F + fo + 16 * u);
            if constexpr (!V0) {
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    cv[d][u] = ld4(v + (long)j * F3 + d * F + fo + 16 * u) * ph[0][u];
                    Y[d][u] = v4f{0.f, 0.f, 0.f, 0.f};
                }
                ap[0][u] = v4f{0.f, 0.f, 0.f, 0.f};
                ap[1][u] = v4f{0.f, 0.f, 0.f, 0.f};
            }
        }
        // edges of an atom beyond the hop range carry no gradient in this layer
        if (hop[j] > hop_max)
            for (int q = e0 + lane; q < e1; q += 64) Sp[q] = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 gm_n = make_float4(0.f, 0.f, 0.f, rc);
        int i_n = j;
        if (e < deg) {
            gm_n = geom[e0 + e];
            i_n = colc[e0 + e];
        }
        for (int cb = 0; cb < deg; cb += 16) {
            const char *wl = lds_chunk(lds);
            const bool valid = cb + e < deg;
            const float4 gm = gm_n;
            const int i = i_n;
            gm_n = make_float4(0.f, 0.f, 0.f, rc);
            i_n = j;
            if (cb + 16 + e < deg) {
                gm_n = geom[e0 + cb + 16 + e];
                i_n = colc[e0 + cb + 16 + e];
            }
            // the destinations' gradient rows, gathered quarter-contiguously and
            // moved to the accumulator layout
            const int iq = __shfl(i, xc.src, 64);
            v4f gs[TU], gv[3][TU];
#pragma unroll
            for (int u = 0; u < TU; u++) {
                gs[u] = ld4(gs1 + (long)iq * F + p * W + xc.fo + 16 * u);
#pragma unroll
                for (int d = 0; d < 3; d++) gv[d][u] = ld4(gv1 + (long)iq * F3 + d * F + p * W + xc.fo + 16 * u);
            }
#pragma unroll
            for (int u = 0; u < TU; u++) {
                gs[u] = xc.move(xw[0], gs[u]);
#pragma unroll
                for (int d = 0; d < 3; d++) gv[d][u] = xc.move(xw[1 + d], gv[d][u]);
            }
            const float ir = valid ? __builtin_amdgcn_rcpf(gm.w) : 0.f;
            float eb[SL], db[SL];
            basis_slots<P, K, true>(gm.w, ir, pirc, valid, g, eb, db);
            BOp<P, K> bop, dop;
            bop.set(eb);
            dop.set(db);
            // direction of the message edge (i <- j) is x_j - x_i = -(x_i - x_j)
            const float rx = -gm.x * ir, ry = -gm.y * ir, rz = -gm.z * ir;
            float sr = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
#pragma unroll
            for (int u = 0; u < TU; u++) {
                v4f w0, w1, d0;
                if constexpr (!V0) {
                    w0 = filter_tile<P, F, K, WM>(wl, u, bop, lane);
                    w1 = filter_tile<P, F, K, WM>(wl, TU + u, bop, lane);
                }
                const v4f w2 = filter_tile<P, F, K, WM>(wl, 2 * TU + u, bop, lane);
                if constexpr (!V0) d0 = filter_tile<P, F, K, WM>(wl, u, dop, lane);
                const v4f d1 = filter_tile<P, F, K, WM>(wl, TU + u, dop, lane);
                const v4f d2 = filter_tile<P, F, K, WM>(wl, 2 * TU + u, dop, lane);
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const float ga = gv[0][u][r], gb = gv[1][u][r], gc = gv[2][u][r], gsr = gs[u][r];
                    const float gxvs = fmaf(ga, rx, fmaf(gb, ry, gc * rz));
                    const float xvs = ph[2][u][r] * w2[r];
                    sx = fmaf(ga, xvs, sx);
                    sy = fmaf(gb, xvs, sy);
                    sz = fmaf(gc, xvs, sz);
                    if constexpr (V0) {
                        sr = fmaf(gsr * ph[1][u][r], d1[r], fmaf(gxvs * ph[2][u][r], d2[r], sr));
                        continue;
                    }
                    const float gc0 = fmaf(ga, cv[0][u][r], fmaf(gb, cv[1][u][r], gc * cv[2][u][r]));
                    Y[0][u][r] = fmaf(ga, w0[r], Y[0][u][r]);
                    Y[1][u][r] = fmaf(gb, w0[r], Y[1][u][r]);
                    Y[2][u][r] = fmaf(gc, w0[r], Y[2][u][r]);
                    ap[0][u][r] = fmaf(gsr, w1[r], ap[0][u][r]);
                    ap[1][u][r] = fmaf(gxvs, w2[r], ap[1][u][r]);
                    sr = fmaf(gc0, d0[r], fmaf(gsr * ph[1][u][r], d1[r], fmaf(gxvs * ph[2][u][r], d2[r], sr)));
                }
            }
            // sum over the four lane rows (all features of the pass)
            sr += __shfl_xor(sr, 16, 64);
            sx += __shfl_xor(sx, 16, 64);
            sy += __shfl_xor(sy, 16, 64);
            sz += __shfl_xor(sz, 16, 64);
            sr += __shfl_xor(sr, 32, 64);
            sx += __shfl_xor(sx, 32, 64);
            sy += __shfl_xor(sy, 32, 64);
            sz += __shfl_xor(sz, 32, 64);
            if (g == 0 && valid) Sp[e0 + cb + e] = make_float4(sr, sx, sy, sz);
        }
        if constexpr (V0) continue;
        // sum over the 16 edge lanes of each row
#pragma unroll
        for (int u = 0; u < TU; u++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
#pragma unroll
                for (int d = 0; d < 3; d++) Y[d][u][r] = row_sum16(Y[d][u][r]);
                ap[0][u][r] = row_sum16(ap[0][u][r]);
                ap[1][u][r] = row_sum16(ap[1][u][r]);
            }
        if (e == 0) {
#pragma unroll
            for (int u = 0; u < TU; u++) {
                const long b = (long)j * F3 + fo + 16 * u;
                const v4f pvv = ld4(phi + b);
                v4f gvv = v4f{0.f, 0.f, 0.f, 0.f};
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    gvv += ld4(v + b + d * F) * Y[d][u];
                    st4(gv_in + b + d * F, ld4(gv1 + b + d * F) + pvv * Y[d][u]);
                }
                st4(gphi + b, gvv);
                st4(gphi + b + F, ap[0][u]);
                st4(gphi + b + 2 * F, ap[1][u]);
            }
        }
    }
}

// One stage of a reduce-scatter over the 16 lanes of a row: lane e keeps the
// half of x[0 .. 2H) its bit selects (U) and adds the partner's copy of it,
// which the DPP pattern CTRL brings (the partner's bit is the opposite one).
template <int CTRL, int H>
__device__ __forceinline__ void rs_half(float *x, bool U) {
#pragma unroll
    for (int k = 0; k < H; k++) {
        const float send = U ? x[k] : x[k + H], keep = U ? x[k + H] : x[k];
        x[k] = keep + dpp<CTRL>(send);
    }
}
// Sums of x[0 .. 16) over the 16 lanes of each row; lane e of the row
// receives the sum of x[e].
__device__ __forceinline__ float row_reduce_scatter16(float *x, int e) {
    rs_half<0x140, 8>(x, e & 8);   // row_mirror: e <-> 15 - e
    rs_half<0x141, 4>(x, e & 4);   // row_half_mirror: e <-> 7 - e inside each half
    rs_half<0x1B, 2>(x, e & 2);    // quad_perm [3,2,1,0]: e <-> e ^ 3
    rs_half<0xB1, 1>(x, e & 1);    // quad_perm [1,0,3,2]: e <-> e ^ 1
    return x[0];
}

// ---------------------------------------------------------------------------
// Adjoint of the message pass of the layers after the first with more than
// one feature pass, organised like k_msg_fwd_pw: every wave runs all passes
// of its source atom j with the weight images of every pass in LDS; the
// radial basis and its derivative of a chunk, in MFMA operand form, are
// evaluated in the first pass and kept in the wave's LDS for the later ones
// (the first BWD_CACHE chunks); the filter tiles come out transposed, so
// lane (f, g) works on feature f of the tile for the in-edges 4g .. 4g+3:
// it gathers the destinations' gradient rows 16 consecutive features per
// quarter-wave, accumulates dE/dphi_j and dE/dv_j over its edges in
// registers (summed over the four lane rows once per atom and pass), and
// holds per-edge partial sums over its feature, which a reduce-scatter over
// the 16 lanes of the row turns into the 16 values (4 edges x (dE/dr,
// dE/drhat)) that the row stores as 64 contiguous bytes.  The edge sums of
// the passes are added up in the wave, in pass order (in LDS for the cached
// chunks, in the slot itself for the others: the lane that adds is the lane
// that stored), so the layer has one slot.
// ---------------------------------------------------------------------------
#ifndef BWD_PIW_WAVES
#define BWD_PIW_WAVES 8
#endif
#ifndef BWD_PIW_EU
#define BWD_PIW_EU 2
#endif
#ifndef BWD_CACHE
#define BWD_CACHE 3
#endif
template <int P, int F, int K>
__global__ void __launch_bounds__(64 * BWD_PIW_WAVES) __attribute__((amdgpu_waves_per_eu(BWD_PIW_EU))) k_msg_bwd_pw(const int *__restrict__ rowc, const int *__restrict__ colc,
                                                     const float4 *__restrict__ geom, int n,
                                                     const float *__restrict__ phi, const float *__restrict__ v,
                                                     const float *__restrict__ gs1, const float *__restrict__ gv1,
                                                     const float *__restrict__ Aw, const float *__restrict__ cw,
                                                     float rc, const int8_t *__restrict__ hop, int hop_max,
                                                     int *__restrict__ queue,
                                                     float *__restrict__ gv_in, float *__restrict__ gphi,
                                                     float4 *__restrict__ S) {
    constexpr int WM = BWD_W;
    constexpr int F3 = 3 * F, SL = Basis<P, K>::SLOTS, W = Pass<F, WM>::W, TU = Pass<F, WM>::TU;
    constexpr int NP = Pass<F, WM>::N, NC = BWD_CACHE;
    constexpr int WB = WStage<P, F, K, WM, true>::BYTES;
    constexpr int CB = 2 * BOpStore<P, K>::BYTES;       // basis and derivative of a chunk
    __shared__ __attribute__((aligned(16))) char lds[NP * WB];
    __shared__ __attribute__((aligned(16))) char bcache[BWD_PIW_WAVES * NC * CB];
    __shared__ float sacc[BWD_PIW_WAVES][NC][64];       // edge sums of the cached chunks
#pragma unroll 1
    for (int q = 0; q < NP; q++) stage_pass<P, F, K, WM, true>(Aw, cw, q, lds + q * WB);
    const int lane = threadIdx.x & 63, e = lane & 15, g = lane >> 4;
    char *bc = bcache + (threadIdx.x >> 6) * NC * CB;
    float *Sf = reinterpret_cast<float *>(S);
    const AtomQueue aq(n, queue, 0);
    const float pirc = 3.14159265358979f / rc;
    MSG_ATOMS_AHEAD(aq, j) {
        const int e0 = rowc[j], e1 = rowc[j + 1];
        const int deg = hop[j] <= hop_max ? e1 - e0 : 0;
        // edges of an atom beyond the hop range carry no gradient in this layer
        if (hop[j] > hop_max)
            for (int t = e0 + lane; t < e1; t += 64) S[t] = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll 1
        for (int p = 0; p < NP; p++) {
            const int fl = p * W + e;   // this lane's feature (tile u adds 16 u)
            // Y_d = sum_e dE/dv1_d(i) w_vv (dE/dv_j = phi_vv Y_d and dE/dphi_vv =
            // sum_d v_jd Y_d follow once per atom), dE/dphi_s, dE/dphi_vs; the v_j
            // term of dE/dr enters through c_d = v_jd phi_vv
            float ph[3][TU], cv[3][TU], Y[3][TU], ap[2][TU];
#pragma unroll
            for (int u = 0; u < TU; u++) {
#pragma unroll
                for (int q = 0; q < 3; q++) ph[q][u] = phi[(long)j * F3 + q * F + fl + 16 * u];
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    cv[d][u] = v[(long)j * F3 + d * F + fl + 16 * u] * ph[0][u];
                    Y[d][u] = 0.f;
                }
                ap[0][u] = 0.f;
                ap[1][u] = 0.f;
            }
            float4 gm_n = make_float4(0.f, 0.f, 0.f, rc);
            int i_n = j;
            if (e < deg) {
                gm_n = geom[e0 + e];
                i_n = colc[e0 + e];
            }
            for (int cb = 0; cb < deg; cb += 16) {
                const char *wl = lds_chunk(lds + p * WB);
                const bool valid = cb + e < deg;
                const float4 gm = gm_n;
                const int i = i_n;
                gm_n = make_float4(0.f, 0.f, 0.f, rc);
                i_n = j;
                if (cb + 16 + e < deg) {
                    gm_n = geom[e0 + cb + 16 + e];
                    i_n = colc[e0 + cb + 16 + e];
                }
                const float ir = valid ? __builtin_amdgcn_rcpf(gm.w) : 0.f;
                // direction of the message edge (i <- j) is x_j - x_i = -(x_i - x_j)
                const float rx = -gm.x * ir, ry = -gm.y * ir, rz = -gm.z * ir;
                // destinations and directions of this lane's edges 4g + r (padding
                // edges: the atom itself and a zero direction; their filter is 0)
                int ir_[4];
                float hx[4], hy[4], hz[4];
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const int src = 4 * g + r;
                    ir_[r] = __shfl(i, src, 64);
                    hx[r] = __shfl(rx, src, 64);
                    hy[r] = __shfl(ry, src, 64);
                    hz[r] = __shfl(rz, src, 64);
                }
                float gs[TU][4], gv[3][TU][4];
#pragma unroll
                for (int r = 0; r < 4; r++) {
                    const float *gsi = gs1 + (long)ir_[r] * F + fl;
                    const float *gvi = gv1 + (long)ir_[r] * F3 + fl;
#pragma unroll
                    for (int u = 0; u < TU; u++) {
                        gs[u][r] = gsi[16 * u];
#pragma unroll
                        for (int d = 0; d < 3; d++) gv[d][u][r] = gvi[d * F + 16 * u];
                    }
                }
                BOp<P, K> bop, dop;
                const int c = cb >> 4;
                if (p > 0 && c < NC) {
                    bop_get<P, K>(bc + c * CB, lane, bop);
                    bop_get<P, K>(bc + c * CB + CB / 2, lane, dop);
                } else {
                    float eb[SL], db[SL];
                    basis_slots<P, K, true>(gm.w, ir, pirc, valid, g, eb, db);
                    bop.set(eb);
                    dop.set(db);
                    if (p == 0 && c < NC) {
                        bop_put<P, K>(bc + c * CB, lane, bop);
                        bop_put<P, K>(bc + c * CB + CB / 2, lane, dop);
                    }
                }
                // per edge r: (dE/dr, dE/drhat_x, _y, _z) of this lane's feature
                float es[16];
#pragma unroll
                for (int k = 0; k < 16; k++) es[k] = 0.f;
#pragma unroll
                for (int u = 0; u < TU; u++) {
                    const v4f w0 = filter_tile<P, F, K, WM, true, true>(wl, u, bop, lane);
                    const v4f w1 = filter_tile<P, F, K, WM, true, true>(wl, TU + u, bop, lane);
                    const v4f w2 = filter_tile<P, F, K, WM, true, true>(wl, 2 * TU + u, bop, lane);
                    const v4f d0 = filter_tile<P, F, K, WM, true, true>(wl, u, dop, lane);
                    const v4f d1 = filter_tile<P, F, K, WM, true, true>(wl, TU + u, dop, lane);
                    const v4f d2 = filter_tile<P, F, K, WM, true, true>(wl, 2 * TU + u, dop, lane);
#pragma unroll
                    for (int r = 0; r < 4; r++) {
                        const float ga = gv[0][u][r], gb = gv[1][u][r], gc = gv[2][u][r], gsr = gs[u][r];
                        const float gxvs = fmaf(ga, hx[r], fmaf(gb, hy[r], gc * hz[r]));
                        const float xvs = ph[2][u] * w2[r];
                        es[4 * r + 1] = fmaf(ga, xvs, es[4 * r + 1]);
                        es[4 * r + 2] = fmaf(gb, xvs, es[4 * r + 2]);
                        es[4 * r + 3] = fmaf(gc, xvs, es[4 * r + 3]);
                        const float gc0 = fmaf(ga, cv[0][u], fmaf(gb, cv[1][u], gc * cv[2][u]));
                        Y[0][u] = fmaf(ga, w0[r], Y[0][u]);
                        Y[1][u] = fmaf(gb, w0[r], Y[1][u]);
                        Y[2][u] = fmaf(gc, w0[r], Y[2][u]);
                        ap[0][u] = fmaf(gsr, w1[r], ap[0][u]);
                        ap[1][u] = fmaf(gxvs, w2[r], ap[1][u]);
                        es[4 * r] = fmaf(gc0, d0[r], fmaf(gsr * ph[1][u], d1[r], fmaf(gxvs * ph[2][u], d2[r], es[4 * r])));
                    }
                }
                // lane e of row g receives component e & 3 of edge 4g + (e >> 2),
                // summed over the pass's features
                float o = row_reduce_scatter16(es, e);
                const int ke = cb + 4 * g + (e >> 2);   // the edge this lane stores
                if (ke < deg) {
                    float *acc = c < NC ? &sacc[threadIdx.x >> 6][c][lane] : Sf + 4L * (e0 + cb + 4 * g) + e;
                    if (p > 0) o += *acc;
                    if (c < NC && p + 1 < NP) *acc = o;
                    else Sf[4L * (e0 + cb + 4 * g) + e] = o;
                }
            }
            // sum over the four lane rows
#pragma unroll
            for (int u = 0; u < TU; u++) {
#pragma unroll
                for (int d = 0; d < 3; d++) {
                    Y[d][u] += __shfl_xor(Y[d][u], 16, 64);
                    Y[d][u] += __shfl_xor(Y[d][u], 32, 64);
                }
                ap[0][u] += __shfl_xor(ap[0][u], 16, 64);
                ap[0][u] += __shfl_xor(ap[0][u], 32, 64);
                ap[1][u] += __shfl_xor(ap[1][u], 16, 64);
                ap[1][u] += __shfl_xor(ap[1][u], 32, 64);
            }
            if (g == 0) {
#pragma unroll
                for (int u = 0; u < TU; u++) {
                    const long b = (long)j * F3 + fl + 16 * u;
                    float gvv = 0.f;
#pragma unroll
                    for (int d = 0; d < 3; d++) {
                        gvv = fmaf(v[b + d * F], Y[d][u], gvv);
                        gv_in[b + d * F] = fmaf(ph[0][u], Y[d][u], gv1[b + d * F]);
                    }
                    gphi[b] = gvv;
                    gphi[b + F] = ap[0][u];
                    gphi[b + 2 * F] = ap[1][u];
                }
            }
        }
    }
}

// G of each pruned edge from its edge-sum slots: G = dE/dr rhat + (g - (g . rhat) rhat) / r,
// with rhat the direction of the message edge, the reverse of the stored one.
// The pruned edge count is rowc[n], read on the device.
__global__ void k_assemble_G(const int *__restrict__ rowc, int n, const float4 *__restrict__ geom,
                             const float4 *__restrict__ S, long s_stride, int npass, float4 *__restrict__ G) {
    const long ne = rowc[n];
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (long)gridDim.x * blockDim.x) {
        float4 a = S[e];
        for (int p = 1; p < npass; p++) {
            const float4 b = S[(long)p * s_stride + e];
            a.x += b.x;
            a.y += b.y;
            a.z += b.z;
            a.w += b.w;
        }
        const float4 gm = geom[e];
        const float ir = 1.0f / gm.w;
        const float rx = -gm.x * ir, ry = -gm.y * ir, rz = -gm.z * ir;
        const float rd = a.y * rx + a.z * ry + a.w * rz;
        G[e] = make_float4(a.x * rx + (a.y - rd * rx) * ir, a.x * ry + (a.z - rd * ry) * ir,
                           a.x * rz + (a.w - rd * rz) * ir, 0.f);
    }
}

// ---------------------------------------------------------------------------
// First layer, factorised.  There v = 0 and phi_j = phi(Z_j) depends on the
// species alone, while the messages are linear in the radial basis e~, so the
// sums over neighbours collapse to per-atom, per-species basis sums:
//   s1_i = s0(Z_i) + sum_Z phi_s(Z) o (A'_s P_i^Z),    P_i^Z   = sum_{j: Z_j = Z} e~(r_ij),
//   v1_i = sum_Z phi_vs(Z) o (A'_vs R_i^{Z,d}),        R_i^{Z,d} = sum_{j: Z_j = Z} rhat_ij,d e~(r_ij),
// and the adjoint's edge sums of the message edge (i <- j) need only the
// per-atom vectors Q_s[i][Z] = A'_s^T (gs1_i o phi_s(Z)) and
// Q_d[i][Z] = A'_vs^T (gv1_i,d o phi_vs(Z)):
//   dE/dr = de~ . (Q_s + sum_d rhat_d Q_d),   dE/drhat_d = e~ . Q_d.
// The products with the species-scaled filter weights (phi(Z) o A') are node
// GEMMs; the two kernels below do the O(K) work per edge.  Each species has
// a block of SB = l0_block(K) columns (slot k at Z SB + k; slots past K meet
// zero weights).  Rows of P: the S SB basis sums, then the species one-hot
// (column S SB + Z), which picks s0(Z_i) out of the same GEMM; rows 3 i + d
// of R and of Q_v, rows i of Q_s: the S SB slot columns.  Lane (g, e) = 16 g + e
// holds basis slots k = 8 g .. 8 g + 7 of edge e, as in the kernels above.
// ---------------------------------------------------------------------------
template <int K, int SS>
__global__ void __launch_bounds__(256) k_l0_basis_sums(const int *__restrict__ rowc, const int *__restrict__ colc,
                                                       const float4 *__restrict__ geom, int n, float rc,
                                                       const int8_t *__restrict__ hop, int hop_max,
                                                       const int *__restrict__ zsp, float *__restrict__ P, int ldp,
                                                       float *__restrict__ R, int ldr) {
    constexpr int SB = l0_block(K);
    const int lane = threadIdx.x & 63, e = lane & 15, g = lane >> 4;
    const float pirc = 3.14159265358979f / rc;
    const int nw = (int)(gridDim.x * (blockDim.x >> 6));
    for (int i = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); i < n; i += nw) {
        const int e0 = rowc[i], e1 = rowc[i + 1];
        const int deg = hop[i] <= hop_max ? e1 - e0 : 0;
        float acc[SS][4][8];
#pragma unroll
        for (int z = 0; z < SS; z++)
#pragma unroll
            for (int t = 0; t < 4; t++)
#pragma unroll
                for (int q = 0; q < 8; q++) acc[z][t][q] = 0.f;
        for (int cb = 0; cb < deg; cb += 16) {
            const bool valid = cb + e < deg;
            float4 gm = make_float4(0.f, 0.f, 0.f, rc);
            int z = 0;
            if (valid) {
                gm = geom[e0 + cb + e];
                z = zsp[colc[e0 + cb + e]];
            }
            const float ir = valid ? __builtin_amdgcn_rcpf(gm.w) : 0.f;
            float eb[8];
            basis_slots<1, K, false>(gm.w, ir, pirc, valid, g, eb, nullptr);
            const float wt[4] = {1.f, gm.x * ir, gm.y * ir, gm.z * ir};
#pragma unroll
            for (int zz = 0; zz < SS; zz++) {
                const bool on = z == zz;
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    const float w = on ? wt[t] : 0.f;
#pragma unroll
                    for (int q = 0; q < 8; q++) acc[zz][t][q] = fmaf(w, eb[q], acc[zz][t][q]);
                }
            }
        }
#pragma unroll
        for (int zz = 0; zz < SS; zz++)
#pragma unroll
            for (int t = 0; t < 4; t++)
#pragma unroll
                for (int q = 0; q < 8; q++) acc[zz][t][q] = row_sum16(acc[zz][t][q]);
        // lane row g holds the totals of slots 8 g .. 8 g + 7 (rows past the
        // species block are not stored; slots past K meet zero weights)
        if (e == 0 && 8 * g < SB) {
#pragma unroll
            for (int zz = 0; zz < SS; zz++)
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    float *dst = t == 0 ? P + (long)i * ldp : R + (3L * i + t - 1) * ldr;
                    dst += zz * SB + 8 * g;
                    st4(dst, v4f{acc[zz][t][0], acc[zz][t][1], acc[zz][t][2], acc[zz][t][3]});
                    st4(dst + 4, v4f{acc[zz][t][4], acc[zz][t][5], acc[zz][t][6], acc[zz][t][7]});
                }
        }
        if (lane < SS) P[(long)i * ldp + SS * SB + lane] = zsp[i] == lane ? 1.f : 0.f;
    }
}

template <int K, int SS>
__global__ void __launch_bounds__(256) k_l0_edge_sums(const int *__restrict__ rowc, const int *__restrict__ colc,
                                                      const int *__restrict__ revc, const float4 *__restrict__ geom,
                                                      int n, float rc, const int8_t *__restrict__ hop, int hop_max,
                                                      const int *__restrict__ zsp, const float *__restrict__ Qs,
                                                      const float *__restrict__ Qv, int ldq, float4 *__restrict__ S) {
    constexpr int SB = l0_block(K);
    const int lane = threadIdx.x & 63, e = lane & 15, g = lane >> 4;
    const float pirc = 3.14159265358979f / rc;
    const int nw = (int)(gridDim.x * (blockDim.x >> 6));
    const bool inb = 8 * g < SB;   // this lane row's slots lie inside a species block
    for (int i = (int)(blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6)); i < n; i += nw) {
        const int e0 = rowc[i], deg = rowc[i + 1] - e0;
        if (deg == 0) continue;
        // one or two species: this lane's slots of Q_i for every species, held
        // in registers (Q is zero past K); more species: read per edge below
        constexpr bool REG = SS <= 2;
        float qs[REG ? SS : 1][8], qv[REG ? SS : 1][3][8];
#pragma unroll
        for (int zz = 0; zz < (REG ? SS : 0); zz++)
#pragma unroll
            for (int t = 0; t < 4; t++) {
                const float *src = (t == 0 ? Qs + (long)i * ldq : Qv + (3L * i + t - 1) * ldq) + zz * SB + 8 * g;
                v4f lo = v4f{0.f, 0.f, 0.f, 0.f}, hi = lo;
                if (inb) {
                    lo = ld4(src);
                    hi = ld4(src + 4);
                }
#pragma unroll
                for (int q = 0; q < 4; q++) {
                    float *row = t == 0 ? qs[zz] : qv[zz][t > 0 ? t - 1 : 0];
                    row[q] = lo[q];
                    row[q + 4] = hi[q];
                }
            }
        for (int cb = 0; cb < deg; cb += 16) {
            const bool valid = cb + e < deg;
            float4 gm = make_float4(0.f, 0.f, 0.f, rc);
            int j = i;
            if (valid) {
                gm = geom[e0 + cb + e];
                j = colc[e0 + cb + e];
            }
            const int z = zsp[j];
            const bool live = valid && hop[j] <= hop_max;
            const float ir = valid ? __builtin_amdgcn_rcpf(gm.w) : 0.f;
            float eb[8], db[8];
            basis_slots<1, K, true>(gm.w, ir, pirc, valid, g, eb, db);
            // direction of the message edge (i <- j): x_j - x_i
            const float rx = gm.x * ir, ry = gm.y * ir, rz = gm.z * ir;
            float sr = 0.f, sx = 0.f, sy = 0.f, sz = 0.f;
            float ql[4][8];   // this edge's species: slots of Q_s, Q_x, Q_y, Q_z
            if constexpr (REG) {
                const bool z1 = SS == 2 && z == 1;   // plain selects: no indexing by z
#pragma unroll
                for (int q = 0; q < 8; q++) {
                    ql[0][q] = z1 ? qs[REG ? SS - 1 : 0][q] : qs[0][q];
#pragma unroll
                    for (int d = 0; d < 3; d++) ql[1 + d][q] = z1 ? qv[REG ? SS - 1 : 0][d][q] : qv[0][d][q];
                }
            } else {
                // the atom's Q rows stay in L1 across its chunks
#pragma unroll
                for (int t = 0; t < 4; t++) {
                    const float *src = (t == 0 ? Qs + (long)i * ldq : Qv + (3L * i + t - 1) * ldq) + z * SB + 8 * g;
                    v4f lo = v4f{0.f, 0.f, 0.f, 0.f}, hi = lo;
                    if (inb) {
                        lo = ld4(src);
                        hi = ld4(src + 4);
                    }
#pragma unroll
                    for (int q = 0; q < 4; q++) {
                        ql[t][q] = lo[q];
                        ql[t][q + 4] = hi[q];
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 8; q++) {
                const float a = ql[0][q], bx = ql[1][q], by = ql[2][q], bz = ql[3][q];
                sr = fmaf(db[q], fmaf(rx, bx, fmaf(ry, by, fmaf(rz, bz, a))), sr);
                sx = fmaf(eb[q], bx, sx);
                sy = fmaf(eb[q], by, sy);
                sz = fmaf(eb[q], bz, sz);
            }
            // sum over the four lane rows (all basis slots)
            sr += __shfl_xor(sr, 16, 64);
            sx += __shfl_xor(sx, 16, 64);
            sy += __shfl_xor(sy, 16, 64);
            sz += __shfl_xor(sz, 16, 64);
            sr += __shfl_xor(sr, 32, 64);
            sx += __shfl_xor(sx, 32, 64);
            sy += __shfl_xor(sy, 32, 64);
            sz += __shfl_xor(sz, 32, 64);
            // the sums of edge (i <- j) go to the slot of its reverse (j <- i),
            // where the adjoint of the later layers keeps them
            if (g == 0 && valid)
                S[revc[e0 + cb + e]] = live ? make_float4(sr, sx, sy, sz) : make_float4(0.f, 0.f, 0.f, 0.f);
        }
    }
}

static int grid_x(int n) {
    int b = std::min((n + MW - 1) / MW, 2048);
    if (b >= 8) b -= b % 8;   // keeps blockIdx.x % 8 the XCD in every pass row
    return std::max(1, b);
}

// Workgroups of kern (with the given block size) that the current device
// holds at once: compute units times the workgroups per compute unit.
template <class KERN>
static int resident_grid(KERN kern, int block) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kern, block, 0) != hipSuccess || per <= 0) per = 1;
    return cus * per;
}

template <int P, int F, int K>
static int launch_fwd(hipStream_t st, const MsgArgs &a) {
    constexpr bool piw = Pass<F, FWD_W>::N > 1;
    if constexpr (piw) {
        if (!a.layer0) {
            auto kern = k_msg_fwd_pw<P, F, K>;
            constexpr int block = 64 * FWD_PIW_WAVES;
            static const int resident = resident_grid(kern, block);   // per process: one device type
            int b = std::min(resident, (a.n + FWD_PIW_WAVES - 1) / FWD_PIW_WAVES);
            if (b >= 8) b -= b % 8;
            kern<<<dim3((unsigned)std::max(1, b)), block, 0, st>>>(a.rowc, a.colc, a.geom, a.n, a.phi, a.u, a.s, a.v,
                                                                   a.A, a.c, a.rc, a.hop, a.hop_max, a.queue, a.sn,
                                                                   a.v1);
            return hipGetLastError() == hipSuccess ? 0 : -5;
        }
    }
    dim3 grid((unsigned)grid_x(a.n), (unsigned)Pass<F, FWD_W>::N);
    auto kern = a.layer0 ? k_msg_fwd<P, F, K, true> : k_msg_fwd<P, F, K, false>;
    kern<<<grid, 64 * MW, 0, st>>>(a.rowc, a.colc, a.geom, a.n, a.phi, a.u, a.s, a.v, a.A, a.c, a.rc, a.hop,
                                   a.hop_max, a.species, a.queue, a.sn, a.v1);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

template <int P, int F, int K>
static int launch_bwd(hipStream_t st, const MsgArgs &a) {
    constexpr bool piw = Pass<F, BWD_W>::N > 1;
    if constexpr (piw) {
        if (!a.layer0) {
            auto kern = k_msg_bwd_pw<P, F, K>;
            constexpr int block = 64 * BWD_PIW_WAVES;
            static const int resident = resident_grid(kern, block);   // per process: one device type
            int b = std::min(resident, (a.n + BWD_PIW_WAVES - 1) / BWD_PIW_WAVES);
            if (b >= 8) b -= b % 8;
            kern<<<dim3((unsigned)std::max(1, b)), block, 0, st>>>(a.rowc, a.colc, a.geom, a.n, a.phi, a.v, a.gs1,
                                                                   a.gv1, a.A, a.c, a.rc, a.hop, a.hop_max, a.queue,
                                                                   a.gv_in, a.gphi, a.S);
            return hipGetLastError() == hipSuccess ? 0 : -5;
        }
    }
    dim3 grid((unsigned)grid_x(a.n), (unsigned)Pass<F, BWD_W>::N);
    auto kern = a.layer0 ? k_msg_bwd<P, F, K, true> : k_msg_bwd<P, F, K, false>;
    kern<<<grid, 64 * MW, 0, st>>>(a.rowc, a.colc, a.geom, a.n, a.phi, a.v, a.gs1, a.gv1, a.A, a.c, a.rc, a.hop,
                                   a.hop_max, a.species, a.queue, a.gv_in, a.gphi, a.S, a.s_stride);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

static unsigned l0_blocks(int n) { return (unsigned)std::max(1, std::min((n + 3) / 4, 8192)); }

template <int K, int SS>
static int l0_sums(hipStream_t st, const L0Args &a) {
    k_l0_basis_sums<K, SS><<<l0_blocks(a.n), 256, 0, st>>>(a.rowc, a.colc, a.geom, a.n, a.rc, a.hop, a.hop_max,
                                                           a.species, a.P, a.ldp, a.R, a.ldr);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

template <int K, int SS>
static int l0_edges(hipStream_t st, const L0Args &a) {
    k_l0_edge_sums<K, SS><<<l0_blocks(a.n), 256, 0, st>>>(a.rowc, a.colc, a.revc, a.geom, a.n, a.rc, a.hop,
                                                          a.hop_max, a.species, a.Qs, a.Qv, a.ldq, a.S);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

#define L0_DISPATCH_K(FN, K_)                                      \
    do {                                                           \
        if (S == 1) return FN<K_, 1>(st, a);                       \
        if (S == 2) return FN<K_, 2>(st, a);                       \
        if (S == 3) return FN<K_, 3>(st, a);                       \
        if (S == 4) return FN<K_, 4>(st, a);                       \
    } while (0)
#define L0_DISPATCH(FN)                                            \
    do {                                                           \
        if (K == 20) L0_DISPATCH_K(FN, 20);                        \
        if (K == 8) L0_DISPATCH_K(FN, 8);                          \
        if (K == 6) L0_DISPATCH_K(FN, 6);                          \
    } while (0)

bool l0_factorised(int K, int S) { return (K == 20 || K == 8 || K == 6) && S >= 1 && S <= 4; }

int msg_l0_basis_sums(hipStream_t st, int K, int S, const L0Args &a) {
    const int CS = S * l0_block(K);
    if (a.ldp < CS + S || a.ldr < CS || a.ldp % 4 || a.ldr % 4) return -1;
    L0_DISPATCH(l0_sums);
    return -1;
}

int msg_l0_edge_sums(hipStream_t st, int K, int S, const L0Args &a) {
    if (a.ldq < S * l0_block(K) || a.ldq % 4) return -1;
    L0_DISPATCH(l0_edges);
    return -1;
}

int msg_passes(int F) { return F < BWD_W ? 1 : F / BWD_W; }

int msg_slots(int F, int T, bool l0_factorised) { return T - 1 + (l0_factorised ? 1 : msg_passes(F)); }

static unsigned edge_blocks(long ne_max) { return (unsigned)std::max(1L, std::min((ne_max + 255) / 256, 8192L)); }

int msg_assemble_G(hipStream_t st, const int *rowc, int n, long ne_max, const float4 *geom, const float4 *S,
                   long s_stride, int npass, float4 *G) {
    k_assemble_G<<<edge_blocks(ne_max), 256, 0, st>>>(rowc, n, geom, S, s_stride, npass, G);
    return hipGetLastError() == hipSuccess ? 0 : -5;
}

#define MSG_DISPATCH(FN, P_)                                     \
    do {                                                         \
        if (F == 128 && K == 20) return FN<P_, 128, 20>(st, a);  \
        if (F == 128 && K == 8) return FN<P_, 128, 8>(st, a);    \
        if (F == 64 && K == 20) return FN<P_, 64, 20>(st, a);    \
        if (F == 64 && K == 8) return FN<P_, 64, 8>(st, a);      \
        if (F == 32 && K == 20) return FN<P_, 32, 20>(st, a);    \
        if (F == 32 && K == 8) return FN<P_, 32, 8>(st, a);      \
        if (F == 16 && K == 6) return FN<P_, 16, 6>(st, a);      \
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
