// Neighbour graph on the device: cell binning, deterministic cell-sorted atom
// order, full directed CSR by destination within rc + skin, reverse-edge
// index, per-evaluation pruning to r < rc with compaction, T-hop marks from
// the local atoms, and the owner -> ghost map for the ghost-force fold.
//
// The graph and pruning steps follow Results, "Distributed potential
// computation" (edges between atoms closer than the cutoff; lists built with
// a skin; edges longer than the cutoff removed at every step; atoms reached by
// T rounds of pseudo-messages from the local atoms kept).
#include "internal.h"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

namespace mlp {

static thread_local Error g_err{0, ""};

void set_error(int code, const std::string &msg) { g_err = Error{code, msg}; }
int fail(int code, const std::string &msg) {
    set_error(code, msg);
    return code;
}
const char *last_error_cstr() { return g_err.msg.c_str(); }

int DevBuf::ensure(size_t need, double headroom, int *n_grows) {
    if (p && need <= bytes) return 0;
    if (borrowed)
        return fail(-3, "scratch slice of " + std::to_string(bytes) + " bytes is below the " + std::to_string(need) +
                            " bytes needed");
    size_t nb = (size_t)((double)(need ? need : 1) * headroom) + 256;
    nb = (nb + 255) & ~(size_t)255;
    if (p) {
        hipFree(p);
        p = nullptr;
        bytes = 0;
        if (n_grows) (*n_grows)++;
    }
    hipError_t e = hipMalloc(&p, nb);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        bytes = 0;
        return fail(-2, "device allocation of " + std::to_string(nb) + " bytes failed");
    }
    bytes = nb;
    return 0;
}

void DevBuf::release() {
    if (p && !borrowed) hipFree(p);
    borrowed = false;
    p = nullptr;
    bytes = 0;
}

// ---------------------------------------------------------------------------
// Exclusive scan of int32: out[i] = sum_{k<i} in[k], out[n] = total.
// ---------------------------------------------------------------------------
constexpr int SCAN_T = 256, SCAN_PER = 4, SCAN_B = SCAN_T * SCAN_PER;

__global__ void __launch_bounds__(SCAN_T) k_scan_local(const int *__restrict__ in, int *__restrict__ out,
                                                       int *__restrict__ bsum, int n) {
    __shared__ int sh[SCAN_T];
    const int t = threadIdx.x;
    const long base = (long)blockIdx.x * SCAN_B + t * SCAN_PER;
    int v[SCAN_PER], sum = 0;
#pragma unroll
    for (int q = 0; q < SCAN_PER; q++) {
        v[q] = (base + q < n) ? in[base + q] : 0;
        sum += v[q];
    }
    sh[t] = sum;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int x = (t >= off) ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += x;
        __syncthreads();
    }
    int run = sh[t] - sum;
#pragma unroll
    for (int q = 0; q < SCAN_PER; q++) {
        if (base + q < n) out[base + q] = run;
        run += v[q];
    }
    if (t == SCAN_T - 1) bsum[blockIdx.x] = sh[t];
}

__global__ void __launch_bounds__(1024) k_scan_sums(int *__restrict__ bsum, int nb, int *__restrict__ total) {
    __shared__ int sh[1024];
    __shared__ int carry;
    const int t = threadIdx.x;
    if (t == 0) carry = 0;
    __syncthreads();
    for (int c0 = 0; c0 < nb; c0 += 1024) {
        int i = c0 + t;
        int v = (i < nb) ? bsum[i] : 0;
        sh[t] = v;
        __syncthreads();
        for (int off = 1; off < 1024; off <<= 1) {
            int x = (t >= off) ? sh[t - off] : 0;
            __syncthreads();
            sh[t] += x;
            __syncthreads();
        }
        int excl = sh[t] - v + carry;
        if (i < nb) bsum[i] = excl;
        __syncthreads();
        if (t == 1023) carry += sh[1023];
        __syncthreads();
    }
    if (t == 0) *total = carry;
}

__global__ void k_scan_add(int *__restrict__ out, const int *__restrict__ bsum, int n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] += bsum[i / SCAN_B];
}

static size_t scan_tmp_bytes(int n) {
    int nb = (n + SCAN_B - 1) / SCAN_B;
    if (nb < 1) nb = 1;
    return sizeof(int) * (size_t)(nb + 1);
}

int scan_exclusive(const int *in, int *out, int n, DevBuf &tmp, int *n_grows, hipStream_t s) {
    int nb = (n + SCAN_B - 1) / SCAN_B;
    if (nb < 1) nb = 1;
    if (int rc = tmp.ensure(scan_tmp_bytes(n), 1.5, n_grows)) return rc;
    int *bs = tmp.as<int>();
    if (n == 0) {
        HIP_TRY(hipMemsetAsync(out, 0, sizeof(int), s));
        return 0;
    }
    k_scan_local<<<nb, SCAN_T, 0, s>>>(in, out, bs, n);
    k_scan_sums<<<1, 1024, 0, s>>>(bs, nb, out + n);
    k_scan_add<<<(n + 255) / 256, 256, 0, s>>>(out, bs, n);
    HIP_TRY(hipGetLastError());
    return 0;
}

// ---------------------------------------------------------------------------
// Binning
// ---------------------------------------------------------------------------
struct Grid {
    int nc[3];
    int bits[3];                  // bits of each cell coordinate in the cell key
    float lo[3], inv_w[3], L[3];  // L[d] > 0: periodic dimension
};

// Cell key: the bits of (cx, cy, cz) interleaved from the least significant
// one (a Morton order; a coordinate whose bits are used up drops out).
// Cells close in space get close keys, so the atoms sorted by key, and the
// contiguous slices of them one XCD's workgroups take, are compact regions
// whose neighbours' rows stay in that XCD's L2; a row-major order would
// place the atoms of the adjacent plane a whole plane of cells away.
__host__ __device__ inline int cell_key(const Grid &g, int cx, int cy, int cz) {
    int key = 0, o = 0;
    for (int b = 0; b < 10; b++) {
        if (b < g.bits[0]) key |= ((cx >> b) & 1) << o++;
        if (b < g.bits[1]) key |= ((cy >> b) & 1) << o++;
        if (b < g.bits[2]) key |= ((cz >> b) & 1) << o++;
    }
    return key;
}

__device__ __forceinline__ void cell_coords(const Grid &g, int key, int &cx, int &cy, int &cz) {
    cx = cy = cz = 0;
    int o = 0;
    for (int b = 0; b < 10; b++) {
        if (b < g.bits[0]) cx |= ((key >> o++) & 1) << b;
        if (b < g.bits[1]) cy |= ((key >> o++) & 1) << b;
        if (b < g.bits[2]) cz |= ((key >> o++) & 1) << b;
    }
}

static int bits_for(int n) {
    int b = 0;
    while ((1 << b) < n) b++;
    return b;
}

__device__ __forceinline__ float wrap_coord(float x, float L) {
    // x - L floor(x / L), then one fold into [0, L); the identity on [0, L).
    float y = x - L * floorf(x / L);
    if (y >= L) y -= L;
    if (y < 0.f) y += L;
    return y;
}

__global__ void k_bbox(const float *__restrict__ pos, int n, float *__restrict__ part) {
    __shared__ float sh[6][256];
    float mn[3] = {INFINITY, INFINITY, INFINITY}, mx[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
        for (int d = 0; d < 3; d++) {
            float x = pos[(long)d * n + i];
            if (isfinite(x)) {
                mn[d] = fminf(mn[d], x);
                mx[d] = fmaxf(mx[d], x);
            }
        }
    }
    for (int d = 0; d < 3; d++) {
        sh[d][threadIdx.x] = mn[d];
        sh[3 + d][threadIdx.x] = mx[d];
    }
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int d = 0; d < 3; d++) {
                sh[d][threadIdx.x] = fminf(sh[d][threadIdx.x], sh[d][threadIdx.x + off]);
                sh[3 + d][threadIdx.x] = fmaxf(sh[3 + d][threadIdx.x], sh[3 + d][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ void k_bin(const float *__restrict__ pos, int n, Grid g, float4 *__restrict__ posw,
                      int *__restrict__ cell_of, int *__restrict__ cell_cnt, int *__restrict__ flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float p[3];
    int c[3];
    for (int d = 0; d < 3; d++) {
        float x = pos[(long)d * n + i];
        if (!isfinite(x)) {
            atomicOr(flag, 1);
            x = 0.f;
        }
        if (g.L[d] > 0.f) x = wrap_coord(x, g.L[d]);
        p[d] = x;
        int ci = (int)((x - g.lo[d]) * g.inv_w[d]);
        c[d] = min(max(ci, 0), g.nc[d] - 1);
    }
    posw[i] = make_float4(p[0], p[1], p[2], 0.f);
    int cell = cell_key(g, c[0], c[1], c[2]);
    cell_of[i] = cell;
    atomicAdd(&cell_cnt[cell], 1);
}

__global__ void k_cell_fill(const int *__restrict__ cell_of, int n, const int *__restrict__ cell_start,
                            int *__restrict__ cell_fill, int *__restrict__ tmp_idx) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = cell_of[i];
    int slot = atomicAdd(&cell_fill[c], 1);
    tmp_idx[cell_start[c] + slot] = i;
}

// Ascending user index inside each cell: makes the internal order, and hence
// every result, independent of atomic scheduling.
// One wave per cell: lane l holds the cell's l-th entry and moves it to its
// rank among the entries (user indices are distinct); a cell of more than
// 64 atoms falls back to an insertion sort by its first lane.
__global__ void __launch_bounds__(256) k_cell_sort(const int *__restrict__ cell_start, int ncell,
                                                   int *__restrict__ idx, int *__restrict__ max_occ) {
    const int lane = threadIdx.x & 63;
    const int c = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (c >= ncell) return;
    const int a = cell_start[c], b = cell_start[c + 1], occ = b - a;
    if (occ <= 64) {
        const int v = lane < occ ? idx[a + lane] : 0x7fffffff;
        int rank = 0;
        for (int p = 0; p < occ; p++) rank += __builtin_amdgcn_readlane(v, p) < v;
        if (lane < occ) idx[a + rank] = v;
    } else if (lane == 0) {
        for (int i = a + 1; i < b; i++) {
            int key = idx[i];
            int j = i - 1;
            while (j >= a && idx[j] > key) {
                idx[j + 1] = idx[j];
                j--;
            }
            idx[j + 1] = key;
        }
    }
    // the largest occupancy; the plain read (never above the true maximum)
    // skips most of the atomics on the one shared word
    if (lane == 0 && occ > 0 && occ > *(volatile int *)max_occ) atomicMax(max_occ, occ);
}

__global__ void k_gather_build(const int *__restrict__ perm, int n, const float4 *__restrict__ posw,
                               const int *__restrict__ species_user, int n_species,
                               const int *__restrict__ cell_of_user, float4 *__restrict__ pos_build,
                               int *__restrict__ species, int *__restrict__ cell_int,
                               int *__restrict__ iperm, int *__restrict__ flag) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int u = perm[k];
    pos_build[k] = posw[u];
    int z = species_user[u];
    if (z < 0 || z >= n_species) {
        atomicOr(flag, 2);
        z = 0;
    }
    species[k] = z;
    cell_int[k] = cell_of_user[u];
    iperm[u] = k;
}

// ---------------------------------------------------------------------------
// Stencil search.  The pair decision is the documented float32 formula.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int stencil_list(int c, int nc, bool periodic, int *out) {
    if (nc < 3) {
        for (int q = 0; q < nc; q++) out[q] = q;
        return nc;
    }
    int m = 0;
    for (int q = -1; q <= 1; q++) {
        int x = c + q;
        if (periodic) {
            x = (x + nc) % nc;
        } else if (x < 0 || x >= nc) {
            continue;
        }
        out[m++] = x;
    }
    // ascending (at most 3 entries)
    for (int a = 1; a < m; a++) {
        int key = out[a], b = a - 1;
        while (b >= 0 && out[b] > key) {
            out[b + 1] = out[b];
            b--;
        }
        out[b + 1] = key;
    }
    return m;
}

__device__ __forceinline__ float fold_once(float d, float L) {
    if (L > 0.f) {
        float h = 0.5f * L;
        if (d > h) d = d - L;
        else if (d < -h) d = d + L;
    }
    return d;
}

// Neighbours within rc + skin of row i, one wave per row.  Lane q (< 27)
// computes the key of stencil cell q and its rank among the stencil keys
// (distinct cells have distinct keys); lane r then holds the r-th cell in
// ascending key order, its row range in the cell-sorted order and the
// exclusive prefix of the range lengths.  The candidates of all ranges are
// tested as one concatenated sequence, 64 at a time (lane l takes candidate
// cb + l, found in the few ranges that overlap the chunk); a ballot and a
// prefix popcount place the hits, so the columns of a row come out
// ascending, as from a sequential scan of the cells in key order.
template <bool FILL>
__global__ void __launch_bounds__(256) k_nbr(const float4 *__restrict__ pb, const int *__restrict__ cell_int,
                                             const int *__restrict__ cell_start, int n, Grid g, float cut2,
                                             int *__restrict__ cnt, const int *__restrict__ row,
                                             int *__restrict__ col) {
    __shared__ int skey[4][32];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = blockIdx.x * 4 + w;
    if (i >= n) return;   // wave-local LDS only: no workgroup barrier below
    const float4 pi = pb[i];
    int cx, cy, cz;
    cell_coords(g, cell_int[i], cx, cy, cz);
    int lx[3], ly[3], lz[3];
    const int nx = stencil_list(cx, g.nc[0], g.L[0] > 0.f, lx);
    const int ny = stencil_list(cy, g.nc[1], g.L[1] > 0.f, ly);
    const int nz = stencil_list(cz, g.nc[2], g.L[2] > 0.f, lz);
    const int nk = nx * ny * nz;
    int kq = 0x7fffffff;
    if (lane < nk) {
        const int a = lane / (ny * nz), b = (lane / nz) % ny, q = lane % nz;
        const int x = a == 0 ? lx[0] : (a == 1 ? lx[1] : lx[2]);
        const int y = b == 0 ? ly[0] : (b == 1 ? ly[1] : ly[2]);
        const int z = q == 0 ? lz[0] : (q == 1 ? lz[1] : lz[2]);
        kq = cell_key(g, x, y, z);
    }
    int rank = 0;
    for (int p = 0; p < nk; p++) rank += __builtin_amdgcn_readlane(kq, p) < kq;
    if (lane < nk) skey[w][rank] = kq;
    __builtin_amdgcn_wave_barrier();   // the reads below see the whole wave's writes
    int rb = 0, len = 0;
    if (lane < nk) {
        const int k = skey[w][lane];
        rb = cell_start[k];
        len = cell_start[k + 1] - rb;
    }
    // exclusive prefix of the range lengths over the lanes
    int pre = len;
#pragma unroll
    for (int d = 1; d < 32; d <<= 1) {
        const int v = __shfl_up(pre, d, 64);
        if (lane >= d) pre += v;
    }
    const int total = __builtin_amdgcn_readlane(pre, nk - 1);
    pre -= len;
    int c = 0;
    const int o = FILL ? row[i] : 0;
    const unsigned long long below = (1ull << lane) - 1ull;
    int r0 = 0;   // first range that can still hold candidates (uniform)
    for (int cb = 0; cb < total; cb += 64) {
        while (r0 < nk && __builtin_amdgcn_readlane(pre, r0) + __builtin_amdgcn_readlane(len, r0) <= cb) r0++;
        const int t = cb + lane;
        int j = 0;
        for (int r = r0; r < nk; r++) {
            const int pr = __builtin_amdgcn_readlane(pre, r);
            if (pr >= cb + 64) break;
            if (t >= pr) j = __builtin_amdgcn_readlane(rb, r) + (t - pr);
        }
        bool hit = false;
        if (t < total && j != i) {
            const float4 pj = pb[j];
            const float dx = fold_once(pj.x - pi.x, g.L[0]);
            const float dy = fold_once(pj.y - pi.y, g.L[1]);
            const float dz = fold_once(pj.z - pi.z, g.L[2]);
            hit = fmaf(dz, dz, fmaf(dy, dy, dx * dx)) < cut2;
        }
        const unsigned long long m = __ballot(hit);
        if (FILL && hit) col[o + c + __popcll(m & below)] = j;
        c += __popcll(m);
    }
    if (!FILL && lane == 0) cnt[i] = c;
}

__device__ __forceinline__ int find_sorted(const int *__restrict__ a, int lo, int hi, int key) {
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Reverse-edge index, one wave per row (lanes take the row's edges): the
// position of i in the (ascending) row of j.
__global__ void __launch_bounds__(256) k_rev(const int *__restrict__ row, const int *__restrict__ col, int n,
                                             int *__restrict__ rev, int *__restrict__ flag) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const int e1 = row[i + 1];
    for (int e = row[i] + lane; e < e1; e += 64) {
        const int j = col[e];
        const int a = row[j], b = row[j + 1];
        int p = find_sorted(col, a, b, i);
        if (p >= b || col[p] != i) {
            atomicOr(flag, 4);
            p = e;
        }
        rev[e] = p;
    }
}

// ---------------------------------------------------------------------------
// Per-evaluation pruning (r < rc at the current positions), one wave per row.
// Displacements use the minimum image x - L rint(x / L) in periodic dims;
// it is odd in x, so an edge and its reverse are kept or dropped together.
// ---------------------------------------------------------------------------
__global__ void k_gather_pos(const float *__restrict__ pos, const int *__restrict__ perm, int n,
                             float4 *__restrict__ pos4) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int u = perm[k];
    pos4[k] = make_float4(pos[u], pos[(long)n + u], pos[2 * (long)n + u], 0.f);
}

__device__ __forceinline__ float min_image(float d, float L) {
    if (L > 0.f) d = d - L * rintf(d / L);
    return d;
}

template <bool FILL>
__global__ void __launch_bounds__(256) k_prune(const float4 *__restrict__ p4, const int *__restrict__ row,
                                               const int *__restrict__ col, int n, float L0, float L1,
                                               float L2, float rc2, int *__restrict__ cnt,
                                               const int *__restrict__ rowc, int *__restrict__ colc,
                                               float4 *__restrict__ geom, int *__restrict__ map,
                                               int *__restrict__ oldidx) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    float4 pi = p4[i];
    int a = row[i], b = row[i + 1];
    int base = FILL ? rowc[i] : 0;
    int c = 0;
    for (int e0 = a; e0 < b; e0 += 64) {
        int e = e0 + lane;
        bool keep = false;
        float dx = 0, dy = 0, dz = 0, r2 = 0;
        int j = 0;
        if (e < b) {
            j = col[e];
            float4 pj = p4[j];
            dx = min_image(pj.x - pi.x, L0);
            dy = min_image(pj.y - pi.y, L1);
            dz = min_image(pj.z - pi.z, L2);
            r2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
            keep = r2 < rc2;
        }
        unsigned long long m = __ballot(keep);
        if (FILL) {
            int pre = __popcll(m & ((1ull << lane) - 1ull));
            if (e < b) {
                if (keep) {
                    int o = base + c + pre;
                    colc[o] = j;
                    geom[o] = make_float4(dx, dy, dz, sqrtf(r2));
                    oldidx[o] = e;
                    map[e] = o;
                } else {
                    map[e] = -1;
                }
            }
        }
        c += __popcll(m);
    }
    if (!FILL && lane == 0) cnt[i] = c;
}

// One thread per pruned edge (count rowc[n], read on the device).
__global__ void k_prune_rev(const int *__restrict__ rowc, int n, const int *__restrict__ oldidx,
                            const int *__restrict__ rev, const int *__restrict__ map, int *__restrict__ revc) {
    const long ne = rowc[n];
    for (long e = (long)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (long)gridDim.x * blockDim.x)
        revc[e] = map[rev[oldidx[e]]];
}

// ---------------------------------------------------------------------------
// Hop marks: hop = 0 for locals; T rounds, each marking (with t) every atom
// that has a neighbour marked t - 1; unreached atoms keep T + 1.
// ---------------------------------------------------------------------------
__global__ void k_hop_init(const int *__restrict__ perm, int n, int n_local, int T, int8_t *__restrict__ hop) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) hop[k] = (int8_t)(perm[k] < n_local ? 0 : T + 1);
}

__global__ void k_hop_round(const int *__restrict__ rowc, const int *__restrict__ colc, int n, int t,
                            int T, int8_t *__restrict__ hop) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n || hop[i] != T + 1) return;
    for (int e = rowc[i]; e < rowc[i + 1]; e++) {
        if (hop[colc[e]] == t - 1) {
            hop[i] = (int8_t)t;
            return;
        }
    }
}

// ---------------------------------------------------------------------------
// Hop-major internal order (domains with ghosts).  Hop levels over the
// rc + skin graph bound those over any pruned graph of the same build from
// below (more edges, fewer hops), so the rows within h hops of the locals at
// any evaluation before the next build lie in the prefix of level <= h.
// Atoms are stably partitioned by level (cell order kept inside a level),
// the CSR relabelled and each row's columns emitted level by level, which
// keeps them ascending.
// ---------------------------------------------------------------------------
__global__ void k_level_flag(const int8_t *__restrict__ hop, int n, int L, int *__restrict__ flag) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) flag[k] = hop[k] == L ? 1 : 0;
}

// newpos of the level-L atoms: base[L] + their rank among level L; base[L + 1]
// = base[L] + the level's count (rank[n], the scan total).
__global__ void k_level_assign(const int8_t *__restrict__ hop, int n, int L, const int *__restrict__ rank,
                               int *__restrict__ base, int *__restrict__ newpos) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    const int b = base[L];
    if (k < n && hop[k] == L) newpos[k] = b + rank[k];
    if (k == 0) base[L + 1] = b + rank[n];
}

__global__ void k_reorder_atoms(const int *__restrict__ newpos, int n, const int *__restrict__ perm,
                                const float4 *__restrict__ pos, const int *__restrict__ spec,
                                const int *__restrict__ row, int *__restrict__ perm2, float4 *__restrict__ pos2,
                                int *__restrict__ spec2, int *__restrict__ cnt2, int *__restrict__ iperm) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const int q = newpos[k];
    perm2[q] = perm[k];
    pos2[q] = pos[k];
    spec2[q] = spec[k];
    cnt2[q] = row[k + 1] - row[k];
    iperm[perm[k]] = q;
}

// One wave per old row: its columns relabelled, level by level (ballot
// compaction keeps the old, ascending order inside a level).
__global__ void __launch_bounds__(256) k_relabel_rows(const int *__restrict__ row, const int *__restrict__ col,
                                                      const int8_t *__restrict__ hop, const int *__restrict__ newpos,
                                                      const int *__restrict__ row2, int n, int nlev,
                                                      int *__restrict__ col2) {
    const int lane = threadIdx.x & 63;
    const int k = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (k >= n) return;
    const int a = row[k], b = row[k + 1];
    int o = row2[newpos[k]];
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int L = 0; L < nlev; L++)
        for (int e0 = a; e0 < b; e0 += 64) {
            const int e = e0 + lane;
            int j = 0;
            bool hit = false;
            if (e < b) {
                j = col[e];
                hit = hop[j] == L;
            }
            const unsigned long long m = __ballot(hit);
            if (hit) col2[o + __popcll(m & below)] = newpos[j];
            o += __popcll(m);
        }
}

__global__ void k_hop_hist(const int8_t *__restrict__ hop, const int *__restrict__ rowc, int n,
                           int *__restrict__ hist, unsigned long long *__restrict__ ehist) {
    // per-workgroup counts of atoms and of their pruned in-edges per hop
    // distance in LDS, then one global add per bin and workgroup
    __shared__ int h[MLP_MAX_LAYERS + 2];
    __shared__ unsigned long long eh[MLP_MAX_LAYERS + 2];
    if (threadIdx.x < MLP_MAX_LAYERS + 2) {
        h[threadIdx.x] = 0;
        eh[threadIdx.x] = 0ull;
    }
    __syncthreads();
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        atomicAdd(&h[hop[i]], 1);
        atomicAdd(&eh[hop[i]], (unsigned long long)(rowc[i + 1] - rowc[i]));
    }
    __syncthreads();
    if (threadIdx.x < MLP_MAX_LAYERS + 2 && h[threadIdx.x]) {
        atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
        atomicAdd(&ehist[threadIdx.x], eh[threadIdx.x]);
    }
}

// ---------------------------------------------------------------------------
// Ghost fold (reverse summation of partial forces, Eq. 2), gather form.
// ---------------------------------------------------------------------------
__global__ void k_owner_count(const int *__restrict__ owner, int ng, int n_local, int *__restrict__ cnt,
                              int *__restrict__ flag) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    int o = owner[g];
    if (o < 0 || o >= n_local) {
        atomicOr(flag, 8);
        return;
    }
    atomicAdd(&cnt[o], 1);
}

__global__ void k_owner_fill(const int *__restrict__ owner, int ng, int n_local, const int *__restrict__ ptr,
                             int *__restrict__ fill, int *__restrict__ list) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= ng) return;
    int o = owner[g];
    if (o < 0 || o >= n_local) return;
    int slot = atomicAdd(&fill[o], 1);
    list[ptr[o] + slot] = n_local + g;
}

// Each owner's ghosts in ascending index (a fixed summation order for the
// fold), sorted once per map.
__global__ void k_owner_sort(const int *__restrict__ ptr, int *__restrict__ list, int n_local) {
    int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_local) return;
    int a = ptr[u], b = ptr[u + 1];
    for (int i = a + 1; i < b; i++) {
        int key = list[i], j = i - 1;
        while (j >= a && list[j] > key) {
            list[j + 1] = list[j];
            j--;
        }
        list[j + 1] = key;
    }
}

__global__ void k_fold(const int *__restrict__ ptr, const int *__restrict__ list, int n_local, int n,
                       float *__restrict__ F) {
    int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n_local) return;
    int a = ptr[u], b = ptr[u + 1];
    for (int d = 0; d < 3; d++) {
        float acc = F[(long)d * n + u];
        for (int q = a; q < b; q++) acc += F[(long)d * n + list[q]];
        F[(long)d * n + u] = acc;
    }
}

// ---------------------------------------------------------------------------
// Largest displacement since the build (MD rebuild criterion).
// ---------------------------------------------------------------------------
__global__ void k_maxdisp(const float *__restrict__ pos, const int *__restrict__ iperm,
                          const float4 *__restrict__ pb, int n, float L0, float L1, float L2, float lim2,
                          int epoch, int *__restrict__ flag) {
    int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= n) return;
    float4 q = pb[iperm[u]];
    float dx = min_image(pos[u] - q.x, L0);
    float dy = min_image(pos[(long)n + u] - q.y, L1);
    float dz = min_image(pos[2 * (long)n + u] - q.z, L2);
    // every atom that moved too far writes this check's tag (no reset needed)
    if (!(dx * dx + dy * dy + dz * dz <= lim2)) *flag = epoch;
}

// ---------------------------------------------------------------------------
// Host orchestration
// ---------------------------------------------------------------------------
static inline int nblk(long n, int t) { return (int)((n + t - 1) / t); }

int build_graph(mlp_model *m, mlp_nbr *g, const float *pos, const int32_t *species, int n, int n_local,
                const double box[3], float skin, hipStream_t s) {
    if (n <= 0 || n_local <= 0 || n_local > n) return fail(-1, "need 0 < n_local <= n_atoms");
    if (!(skin >= 0.f) || !std::isfinite(skin)) return fail(-1, "skin must be finite and >= 0");
    const bool ghosts = n > n_local;
    const float cut = m->rc + skin;
    const float cut2 = cut * cut;
    Grid gr;
    float L[3];
    bool any_open = false;
    for (int d = 0; d < 3; d++) {
        L[d] = ghosts ? 0.f : (float)box[d];
        if (!(L[d] >= 0.f) || !std::isfinite(L[d])) return fail(-1, "box lengths must be finite and >= 0");
        if (L[d] == 0.f) any_open = true;
        if (L[d] > 0.f && !(cut < 0.5f * L[d]))
            return fail(-4, "rc + skin must be below half the periodic box length");
        gr.L[d] = L[d];
    }
    int ng = 0;
    auto &err_grows = g->n_grows;
    // status words: 0 build errors, 1 ghost owners, 2 displacement tag,
    // 8 cell sort, 16..31 hop histogram, 32..63 per-hop edge counts (64-bit)
    if (int rc = g->flags.ensure(256, 1.0, &err_grows)) return rc;
    int *flag = g->flags.as<int>();
    float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    if (any_open) {
        const int nb = std::min(nblk(n, 256), 1024);
        if (int rc = g->red.ensure(sizeof(float) * 6 * nb, 1.0, &err_grows)) return rc;
        k_bbox<<<nb, 256, 0, s>>>(pos, n, g->red.as<float>());
        std::vector<float> part(6 * nb);
        HIP_TRY(hipMemcpyAsync(part.data(), g->red.p, sizeof(float) * 6 * nb, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        for (int d = 0; d < 3; d++) {
            lo[d] = INFINITY;
            hi[d] = -INFINITY;
            for (int b = 0; b < nb; b++) {
                lo[d] = std::min(lo[d], part[b * 6 + d]);
                hi[d] = std::max(hi[d], part[b * 6 + 3 + d]);
            }
            if (!std::isfinite(lo[d]) || !std::isfinite(hi[d])) return fail(-1, "non-finite positions");
        }
    }
    const float margin = cut * (1.0f + 1e-5f);
    // the cell arrays are indexed by cell key, whose range is 2^(bits of the
    // three coordinates): at most 8x the cell count
    auto key_space = [&]() {
        long t = 1;
        for (int d = 0; d < 3; d++) {
            gr.bits[d] = bits_for(gr.nc[d]);
            t <<= gr.bits[d];
        }
        return t;
    };
    for (int d = 0; d < 3; d++) {
        float ext = L[d] > 0.f ? L[d] : (hi[d] - lo[d]) * (1.0f + 1e-6f) + 1e-3f;
        int ncd = std::max(1, (int)std::floor(ext / margin));
        ncd = std::min(ncd, 1024);
        gr.nc[d] = ncd;
        gr.lo[d] = L[d] > 0.f ? 0.f : lo[d];
        gr.inv_w[d] = (float)ncd / ext;
    }
    long ncell = key_space();
    // keep the grid modest: coarsen if the key range is extreme (cells stay >= cut)
    while (ncell > (1L << 24)) {
        for (int d = 0; d < 3; d++) {
            float ext = L[d] > 0.f ? L[d] : (hi[d] - lo[d]) * (1.0f + 1e-6f) + 1e-3f;
            gr.nc[d] = std::max(1, gr.nc[d] / 2);
            gr.inv_w[d] = (float)gr.nc[d] / ext;
        }
        ncell = key_space();
    }
    const int nc = (int)ncell;
    int *G = &err_grows;
    int rc;
    if ((rc = g->perm.ensure(sizeof(int) * n, 1.2, G)) || (rc = g->iperm.ensure(sizeof(int) * n, 1.2, G)) ||
        (rc = g->cell_of.ensure(sizeof(int) * 2 * n, 1.2, G)) ||
        (rc = g->cell_start.ensure(sizeof(int) * (nc + 1), 1.2, G)) ||
        (rc = g->cell_cnt.ensure(sizeof(int) * (nc + 1), 1.2, G)) ||
        (rc = g->cell_fill.ensure(sizeof(int) * (nc + 1), 1.2, G)) ||
        (rc = g->tmp_idx.ensure(sizeof(float4) * n, 1.2, G)) ||
        (rc = g->pos_build.ensure(sizeof(float4) * n, 1.2, G)) ||
        (rc = g->species.ensure(sizeof(int) * n, 1.2, G)) || (rc = g->row.ensure(sizeof(int) * (n + 1), 1.2, G)) ||
        (rc = g->cnt.ensure(sizeof(int) * (n + 1), 1.2, G)))
        return rc;
    float4 *posw = g->tmp_idx.as<float4>();  // user-order wrapped positions (scratch)
    int *cell_user = g->cell_of.as<int>();
    int *cell_int = cell_user + n;
    HIP_TRY(hipMemsetAsync(flag, 0, 64, s));
    HIP_TRY(hipMemsetAsync(g->cell_cnt.p, 0, sizeof(int) * (nc + 1), s));
    HIP_TRY(hipMemsetAsync(g->cell_fill.p, 0, sizeof(int) * (nc + 1), s));
    k_bin<<<nblk(n, 256), 256, 0, s>>>(pos, n, gr, posw, cell_user, g->cell_cnt.as<int>(), flag);
    if ((rc = scan_exclusive(g->cell_cnt.as<int>(), g->cell_start.as<int>(), nc, g->scan_tmp, G, s))) return rc;
    // perm is filled through iperm's storage as scratch, then sorted in place
    int *perm = g->perm.as<int>();
    k_cell_fill<<<nblk(n, 256), 256, 0, s>>>(cell_user, n, g->cell_start.as<int>(), g->cell_fill.as<int>(), perm);
    k_cell_sort<<<nblk(nc, 4), 256, 0, s>>>(g->cell_start.as<int>(), nc, perm, flag + 8);
    k_gather_build<<<nblk(n, 256), 256, 0, s>>>(perm, n, posw, species, m->S, cell_user,
                                                  g->pos_build.as<float4>(), g->species.as<int>(), cell_int,
                                                  g->iperm.as<int>(), flag);
    {
    ProfScope ps(PK_NBR, s);
    k_nbr<false><<<nblk(n, 4), 256, 0, s>>>(g->pos_build.as<float4>(), cell_int, g->cell_start.as<int>(), n, gr,
                                              cut2, g->cnt.as<int>(), nullptr, nullptr);
    }
    if ((rc = scan_exclusive(g->cnt.as<int>(), g->row.as<int>(), n, g->scan_tmp, G, s))) return rc;
    int hostv[16];
    int E = 0;
    HIP_TRY(hipMemcpyAsync(&E, g->row.as<int>() + n, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(hostv, flag, sizeof(int) * 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hostv[0] & 1) return fail(-1, "non-finite positions");
    if (hostv[0] & 2) return fail(-1, "species index out of range");
    if (E < 0) return fail(-3, "edge count overflow");
    if ((rc = g->col.ensure(sizeof(int) * (size_t)E + 4, 1.2, G)) ||
        (rc = g->rev.ensure(sizeof(int) * (size_t)E + 4, 1.2, G)))
        return rc;
    k_nbr<true><<<nblk(n, 4), 256, 0, s>>>(g->pos_build.as<float4>(), cell_int, g->cell_start.as<int>(), n, gr,
                                             cut2, nullptr, g->row.as<int>(), g->col.as<int>());
    k_rev<<<nblk(n, 4), 256, 0, s>>>(g->row.as<int>(), g->col.as<int>(), n, g->rev.as<int>(), flag);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(hostv, flag, sizeof(int) * 16, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (hostv[0] & 4) return fail(-5, "neighbour graph is not symmetric");
    const int T = m->T;
    for (int h = 0; h < MLP_MAX_LAYERS + 2; h++) g->nhop[h] = n;
    if (ghosts) {
        // hop levels over the rc + skin graph, then the hop-major order
        const int nlev = T + 2;
        if ((rc = g->hop.ensure(n + 16, 1.2, G)) || (rc = g->ro_perm.ensure(sizeof(int) * n, 1.2, G)) ||
            (rc = g->ro_pos.ensure(sizeof(float4) * n, 1.2, G)) || (rc = g->ro_spec.ensure(sizeof(int) * n, 1.2, G)) ||
            (rc = g->ro_row.ensure(sizeof(int) * (n + 1), 1.2, G)) ||
            (rc = g->ro_col.ensure(sizeof(int) * (size_t)E + 4, 1.2, G)) ||
            (rc = g->ro_newpos.ensure(sizeof(int) * n, 1.2, G)) ||
            (rc = g->ro_rank.ensure(sizeof(int) * (n + 1) * 2, 1.2, G)) ||
            (rc = g->ro_base.ensure(sizeof(int) * (nlev + 2), 1.0, G)))
            return rc;
        int8_t *hop = g->hop.as<int8_t>();
        int *flg = g->ro_rank.as<int>(), *rank = flg + n + 1, *base = g->ro_base.as<int>();
        k_hop_init<<<nblk(n, 256), 256, 0, s>>>(g->perm.as<int>(), n, n_local, T, hop);
        for (int t = 1; t <= T; t++)
            k_hop_round<<<nblk(n, 256), 256, 0, s>>>(g->row.as<int>(), g->col.as<int>(), n, t, T, hop);
        HIP_TRY(hipMemsetAsync(base, 0, sizeof(int), s));
        for (int L = 0; L < nlev; L++) {
            k_level_flag<<<nblk(n, 256), 256, 0, s>>>(hop, n, L, flg);
            if ((rc = scan_exclusive(flg, rank, n, g->scan_tmp, G, s))) return rc;
            k_level_assign<<<nblk(n, 256), 256, 0, s>>>(hop, n, L, rank, base, g->ro_newpos.as<int>());
        }
        int *cnt2 = g->cnt.as<int>();
        k_reorder_atoms<<<nblk(n, 256), 256, 0, s>>>(g->ro_newpos.as<int>(), n, g->perm.as<int>(),
                                                       g->pos_build.as<float4>(), g->species.as<int>(),
                                                       g->row.as<int>(), g->ro_perm.as<int>(), g->ro_pos.as<float4>(),
                                                       g->ro_spec.as<int>(), cnt2, g->iperm.as<int>());
        if ((rc = scan_exclusive(cnt2, g->ro_row.as<int>(), n, g->scan_tmp, G, s))) return rc;
        k_relabel_rows<<<nblk(n, 4), 256, 0, s>>>(g->row.as<int>(), g->col.as<int>(), hop, g->ro_newpos.as<int>(),
                                                  g->ro_row.as<int>(), n, nlev, g->ro_col.as<int>());
        std::swap(g->perm, g->ro_perm);
        std::swap(g->pos_build, g->ro_pos);
        std::swap(g->species, g->ro_spec);
        std::swap(g->row, g->ro_row);
        std::swap(g->col, g->ro_col);
        HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), s));
        k_rev<<<nblk(n, 4), 256, 0, s>>>(g->row.as<int>(), g->col.as<int>(), n, g->rev.as<int>(), flag);
        HIP_TRY(hipGetLastError());
        int lev[MLP_MAX_LAYERS + 4];
        HIP_TRY(hipMemcpyAsync(lev, base, sizeof(int) * (nlev + 1), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipMemcpyAsync(hostv, flag, sizeof(int) * 16, hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (hostv[0] & 4) return fail(-5, "reordered neighbour graph is not symmetric");
        if (lev[nlev] != n) return fail(-5, "hop-level partition lost atoms");
        for (int h = 0; h < MLP_MAX_LAYERS + 2; h++) g->nhop[h] = lev[std::min(h + 1, nlev)];
    }
    g->n_atoms = n;
    g->n_local = n_local;
    g->open = ghosts;
    for (int d = 0; d < 3; d++) {
        g->box[d] = L[d];
        g->nc[d] = gr.nc[d];
        g->lo[d] = gr.lo[d];
        g->inv_w[d] = gr.inv_w[d];
    }
    g->skin = skin;
    g->n_edges_skin = E;
    g->max_occ = hostv[8];
    g->n_builds++;
    (void)ng;
    return 0;
}

void eval_graph_needs(const mlp_nbr *g, size_t need[EN_GRAPH_COUNT]) {
    const size_t n = (size_t)g->n_atoms, E = (size_t)g->n_edges_skin;
    need[EN_POS4] = sizeof(float4) * n;
    need[EN_ROWC] = sizeof(int) * (n + 1);
    need[EN_COLC] = sizeof(int) * E + 4;
    need[EN_REVC] = sizeof(int) * E + 4;
    need[EN_GEOM] = sizeof(float4) * E + 16;
    need[EN_MAP] = sizeof(int) * E + 4;
    need[EN_OLDIDX] = sizeof(int) * E + 4;
    need[EN_HOP] = n + 16;
    need[EN_SCAN] = scan_tmp_bytes((int)n);
}

int prune_graph(mlp_model *m, mlp_nbr *g, const float *pos, hipStream_t s) {
    const int n = g->n_atoms;
    int *G = &g->n_grows;
    int rc;
    size_t nd[EN_GRAPH_COUNT];
    eval_graph_needs(g, nd);
    if ((rc = g->pos4.ensure(nd[EN_POS4], 1.2, G)) || (rc = g->rowc.ensure(nd[EN_ROWC], 1.2, G)) ||
        (rc = g->colc.ensure(nd[EN_COLC], 1.2, G)) || (rc = g->revc.ensure(nd[EN_REVC], 1.2, G)) ||
        (rc = g->geom.ensure(nd[EN_GEOM], 1.2, G)) || (rc = g->map.ensure(nd[EN_MAP], 1.2, G)) ||
        (rc = g->oldidx.ensure(nd[EN_OLDIDX], 1.2, G)) || (rc = g->hop.ensure(nd[EN_HOP], 1.2, G)))
        return rc;
    const float rcut = m->rc;
    const float rc2 = rcut * rcut;
    k_gather_pos<<<nblk(n, 256), 256, 0, s>>>(pos, g->perm.as<int>(), n, g->pos4.as<float4>());
    ProfScope ps(PK_PRUNE, s);
    k_prune<false><<<nblk(n, 4), 256, 0, s>>>(g->pos4.as<float4>(), g->row.as<int>(), g->col.as<int>(), n,
                                             g->box[0], g->box[1], g->box[2], rc2, g->cnt.as<int>(), nullptr,
                                             nullptr, nullptr, nullptr, nullptr);
    if ((rc = scan_exclusive(g->cnt.as<int>(), g->rowc.as<int>(), n, g->scan_tmp, G, s))) return rc;
    k_prune<true><<<nblk(n, 4), 256, 0, s>>>(g->pos4.as<float4>(), g->row.as<int>(), g->col.as<int>(), n,
                                            g->box[0], g->box[1], g->box[2], rc2, nullptr, g->rowc.as<int>(),
                                            g->colc.as<int>(), g->geom.as<float4>(), g->map.as<int>(),
                                            g->oldidx.as<int>());
    k_prune_rev<<<(int)std::max<int64_t>(1, std::min<int64_t>((g->n_edges_skin + 255) / 256, 8192)), 256, 0, s>>>(
        g->rowc.as<int>(), n, g->oldidx.as<int>(), g->rev.as<int>(), g->map.as<int>(), g->revc.as<int>());
    HIP_TRY(hipGetLastError());
    return 0;
}

int compute_hops(mlp_model *m, mlp_nbr *g, hipStream_t s) {
    const int n = g->n_atoms;
    k_hop_init<<<nblk(n, 256), 256, 0, s>>>(g->perm.as<int>(), n, g->n_local, m->T, g->hop.as<int8_t>());
    if (g->n_atoms > g->n_local)
        for (int t = 1; t <= m->T; t++)
            k_hop_round<<<nblk(n, 256), 256, 0, s>>>(g->rowc.as<int>(), g->colc.as<int>(), n, t, m->T,
                                                     g->hop.as<int8_t>());
    HIP_TRY(hipGetLastError());
    return 0;
}

int hop_histogram(mlp_model *m, mlp_nbr *g, hipStream_t s, int *hist_host /* T+2 */,
                  int64_t *ehist_host /* T+2 */) {
    // flags words 16..31 hold the atom counts, 32..63 the edge counts (64-bit)
    int *flag = g->flags.as<int>();
    unsigned long long *eh = reinterpret_cast<unsigned long long *>(flag + 32);
    HIP_TRY(hipMemsetAsync(flag + 16, 0, sizeof(int) * 48, s));
    k_hop_hist<<<std::max(1, std::min(nblk(g->n_atoms, 256), 1024)), 256, 0, s>>>(
        g->hop.as<int8_t>(), g->rowc.as<int>(), g->n_atoms, flag + 16, eh);
    HIP_TRY(hipMemcpyAsync(hist_host, flag + 16, sizeof(int) * (m->T + 2), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(ehist_host, eh, sizeof(int64_t) * (m->T + 2), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return 0;
}

int prepare_owner_map(mlp_nbr *g, const int32_t *owner, hipStream_t s) {
    const int n = g->n_atoms, nl = g->n_local, ng = n - nl;
    if (ng <= 0) return 0;
    if (g->owner_key == owner && g->owner_build == g->n_builds) return 0;
    g->owner_build = -1;
    int *G = &g->n_grows;
    int rc;
    if ((rc = g->ghost_ptr.ensure(sizeof(int) * (nl + 1), 1.2, G)) ||
        (rc = g->ghost_cnt.ensure(sizeof(int) * (nl + 1) * 2, 1.2, G)) ||
        (rc = g->ghost_list.ensure(sizeof(int) * ng + 4, 1.2, G)))
        return rc;
    if (!g->h_flag) {
        if (hipHostMalloc((void **)&g->h_flag, sizeof(int)) != hipSuccess) {
            (void)hipGetLastError();
            g->h_flag = nullptr;
            return fail(-2, "pinned host allocation failed");
        }
    }
    int *cnt = g->ghost_cnt.as<int>(), *fill = cnt + nl + 1;
    int *flag = g->flags.as<int>() + 1;
    HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int) * (nl + 1) * 2, s));
    HIP_TRY(hipMemsetAsync(flag, 0, sizeof(int), s));
    k_owner_count<<<nblk(ng, 256), 256, 0, s>>>(owner, ng, nl, cnt, flag);
    if ((rc = scan_exclusive(cnt, g->ghost_ptr.as<int>(), nl, g->scan_tmp, G, s))) return rc;
    k_owner_fill<<<nblk(ng, 256), 256, 0, s>>>(owner, ng, nl, g->ghost_ptr.as<int>(), fill, g->ghost_list.as<int>());
    k_owner_sort<<<nblk(nl, 256), 256, 0, s>>>(g->ghost_ptr.as<int>(), g->ghost_list.as<int>(), nl);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(g->h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (*g->h_flag) return fail(-1, "ghost owner index out of range [0, n_local)");
    g->owner_key = owner;
    g->owner_build = g->n_builds;
    return 0;
}

int fold_ghosts(mlp_nbr *g, float *forces, hipStream_t s) {
    const int n = g->n_atoms, nl = g->n_local;
    if (n <= nl) return 0;
    if (g->owner_build != g->n_builds) return fail(-1, "ghost owner map missing");
    k_fold<<<nblk(nl, 256), 256, 0, s>>>(g->ghost_ptr.as<int>(), g->ghost_list.as<int>(), nl, n, forces);
    HIP_TRY(hipGetLastError());
    return 0;
}

__global__ void k_export_edges(const int *__restrict__ row, const int *__restrict__ col,
                               const int *__restrict__ perm, int n, int32_t *__restrict__ dst,
                               int32_t *__restrict__ src) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int u = perm[i];
    for (int e = row[i]; e < row[i + 1]; e++) {
        dst[e] = u;
        src[e] = perm[col[e]];
    }
}

int export_edges(mlp_nbr *g, const int *row, const int *col, int32_t *dst, int32_t *src, hipStream_t s) {
    k_export_edges<<<nblk(g->n_atoms, 256), 256, 0, s>>>(row, col, g->perm.as<int>(), g->n_atoms, dst, src);
    HIP_TRY(hipGetLastError());
    return 0;
}

int max_displacement_exceeds(mlp_nbr *g, const float *pos, float limit, hipStream_t s, bool *exceeds) {
    const int n = g->n_atoms;
    int *flag = g->flags.as<int>();
    if (!g->h_flag) {
        if (hipHostMalloc((void **)&g->h_flag, sizeof(int)) != hipSuccess) {
            (void)hipGetLastError();
            g->h_flag = nullptr;
            return fail(-2, "pinned host allocation failed");
        }
    }
    // tags 1, 2, ...: the word holds the tag of the last check that fired
    // (the build clears it), so it never needs a reset on the stream
    g->disp_epoch = g->disp_epoch == 0x7fffffff ? 1 : g->disp_epoch + 1;
    const int epoch = g->disp_epoch;
    k_maxdisp<<<nblk(n, 256), 256, 0, s>>>(pos, g->iperm.as<int>(), g->pos_build.as<float4>(), n, g->box[0],
                                           g->box[1], g->box[2], limit * limit, epoch, flag + 2);
    HIP_TRY(hipMemcpyAsync(g->h_flag, flag + 2, sizeof(int), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *exceeds = *g->h_flag == epoch;
    return 0;
}

}  // namespace mlp
