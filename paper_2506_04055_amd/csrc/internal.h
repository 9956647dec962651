// Internal declarations shared by the libmlp translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <stdint.h>
#include <stddef.h>
#include <string>

#include "gemm.h"

#define MLP_MAX_LAYERS 7
#define MLP_MAX_K 32
// precision modes (values of the C ABI's MLP_FP32 / MLP_BF16 / MLP_BF16_FAST /
// MLP_BF16_NODE / MLP_BF16_NODE_X3)
#define MLP_PREC_FP32 0
#define MLP_PREC_BF16 1
#define MLP_PREC_BF16_FAST 2
#define MLP_PREC_BF16_NODE 3
#define MLP_PREC_BF16_NODE_X3 4

namespace mlp {

// MFMA operand forms: 0 FP32, 1 plain bfloat16, 2 split bfloat16 (hi + lo,
// three products).  A precision mode fixes one form for the node-feature
// GEMMs and one for the radial-filter contraction of the message kernels.
inline int node_operands(int precision) {
    return precision == MLP_PREC_FP32 ? 0 : (precision == MLP_PREC_BF16 ? 2 : 1);
}
inline int filter_operands(int precision) {
    switch (precision) {
    case MLP_PREC_BF16: return 2;
    case MLP_PREC_BF16_FAST: return 1;
    case MLP_PREC_BF16_NODE_X3: return 2;
    default: return 0;   // FP32 and MLP_PREC_BF16_NODE
    }
}

// Status carried through host code; converted to the C return codes at the boundary.
struct Error {
    int code;
    std::string msg;
};

void set_error(int code, const std::string &msg);
int fail(int code, const std::string &msg);

#define HIP_TRY(expr)                                                                   \
    do {                                                                                \
        hipError_t _e = (expr);                                                         \
        if (_e != hipSuccess)                                                           \
            return ::mlp::fail(-5, std::string(#expr) + ": " + hipGetErrorString(_e)); \
    } while (0)

// Grow-only device buffer.  A borrowed buffer is a view of memory the
// library does not own (a slice of the static scratch array): it is never
// grown or freed, and ensure() on one that is too small fails with CAPACITY.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool borrowed = false;
    // Ensure at least `need` bytes; grows to need * headroom.  Returns 0 or error code.
    int ensure(size_t need, double headroom, int *n_grows);
    void release();
    template <class T> T *as() const { return reinterpret_cast<T *>(p); }
};

// Device-side view of one layer's weights (float32 and optional bf16 copies).
struct LayerW {
    const float *W1, *b1, *W2, *b2, *A, *c, *U, *V, *W3, *b3, *W4, *b4;
};

// Indices into mlp_model::pk[t]: forward (B = W^T) then adjoint (B = W);
// UV is the stacked [U; V] (2F x F, adjacent in the weight layout).  WP_W4TP
// is W4's adjoint operand with its reduction index in the order of the fused
// update adjoint (F = 64 or 128 only).
enum { WP_W1 = 0, WP_W2, WP_UV, WP_W3, WP_W4, WP_W1T, WP_W2T, WP_UVT, WP_W3T, WP_W4T, WP_W4TP, WP_COUNT };

// Dimensions of a single-layer Allegro model (allegro.hip): species, radial
// functions, envelope order, the two-body MLP widths, channel counts per
// degree l = 0..lmax (NC in all), latent width D (= the last two-body
// width), latent hidden width LH, output hidden width OH; cutoff and the
// environment normalisation nu.
struct AlDims {
    int S = 0, NB = 0, p = 0, n2b = 0, d2b[6] = {0, 0, 0, 0, 0, 0}, lmax = 0, ch[4] = {0, 0, 0, 0}, NC = 0, D = 0,
        LH = 0, OH = 0;
    float rc = 0.f, nu = 0.f;
};
struct AlModel;

// Dimensions of a two-layer MACE model (mace.hip): species, radial
// functions, envelope order, l_max, channels, correlation order, the radial
// MLP's hidden widths, the readout MLP's hidden width; cutoff and the
// average neighbour count that normalises the convolution.
struct McDims {
    int S = 0, NB = 0, p = 0, lmax = 0, K = 0, corr = 0, nrad = 0, rh[4] = {0, 0, 0, 0}, RH = 0;
    float rc = 0.f, navg = 0.f;
};
struct McModel;

}  // namespace mlp

struct mlp_model {
    int F, K, T, S, precision;
    mlp::AlModel *al = nullptr;          // set for an Allegro model (then T = 1; F, K unused)
    mlp::McModel *mc = nullptr;          // set for a MACE model (then T = 2; F, K unused)
    float rc, eps;
    size_t n_weights;
    float *w_dev = nullptr;              // flat weights on the device
    __hip_bfloat16 *wb_dev = nullptr;    // bf16 copy (same offsets)
    size_t off_emb;
    size_t off_layer[MLP_MAX_LAYERS][12];
    size_t off_W5, off_b5, off_w6, off_b6;
    // weight matrices packed as GEMM B operands (gemm.h): per layer
    // W1 W2 [U; V] W3 W4 for the forward, then the same five for the adjoint
    mlp::PackedW pk[MLP_MAX_LAYERS][mlp::WP_COUNT];
    mlp::PackedW pk_W5, pk_W5t;
    void *pk_dev = nullptr;
    // phi of the first layer per species ([S][3F]): s = emb[species] there, so
    // the first message MLP depends on the species alone
    float *phi0_dev = nullptr;
    // factorised first layer (up to four species): the species-scaled filter
    // weights packed as B operands: [0] forward s (with the embedding rows),
    // [1] forward v, [2] adjoint s, [3] adjoint v
    bool l0f = false;
    mlp::PackedW pk_l0[4];
    void *pk_l0_dev = nullptr;
    mlp::LayerW layer(int t) const;
    const float *at(size_t off) const { return w_dev + off; }
    const __hip_bfloat16 *atb(size_t off) const { return wb_dev + off; }
};

struct mlp_nbr {
    int n_atoms = 0, n_local = 0;
    bool open = false;
    float box[3] = {0, 0, 0};
    float skin = 0;
    int nc[3] = {1, 1, 1};
    float lo[3] = {0, 0, 0};
    float inv_w[3] = {1, 1, 1};
    int64_t n_edges_skin = 0;
    int n_builds = 0, n_grows = 0, max_occ = 0;
    // graph (internal atom order: cell-sorted)
    mlp::DevBuf perm, iperm, cell_of, cell_start, cell_cnt, cell_fill, tmp_idx;
    mlp::DevBuf pos_build;     // float4 positions at build time (internal order)
    mlp::DevBuf species;       // int32 internal order
    mlp::DevBuf row, col, rev; // skin graph CSR
    mlp::DevBuf rowc, colc, revc, geom, map, oldidx, cnt;  // pruned graph
    mlp::DevBuf hop;           // int8 hop distance (capped T+1)
    // With ghosts the internal order is hop-major: atoms within h hops of the
    // locals (over the rc + skin graph) are rows [0, nhop[h]), so a layer's
    // node work runs on a prefix (nhop[T + 1] = n_atoms).  Without ghosts
    // every nhop[h] = n_atoms.
    int nhop[MLP_MAX_LAYERS + 2] = {0};
    mlp::DevBuf ro_perm, ro_pos, ro_spec, ro_row, ro_col, ro_newpos, ro_rank, ro_base;  // reorder scratch
    mlp::DevBuf pos4;          // float4 positions at evaluation (internal order)
    mlp::DevBuf scan_tmp, flags, red;
    mlp::DevBuf ghost_ptr, ghost_list, ghost_cnt;  // owner -> ghosts (user indices)
    const int32_t *owner_key = nullptr;   // ghost_owner array the map was built from
    int owner_build = -1;      // n_builds when it was built (-1: no valid map)
    // model activations
    mlp::DevBuf act;           // one arena for per-layer activations
    size_t act_bytes = 0;
    int act_N = 0, act_F = 0, act_T = 0;
    mlp::DevBuf G, Gs, Fint, Uatom;   // Gs: per-pass edge sums of the adjoint
    int *h_flag = nullptr;     // pinned host word for the per-step displacement check
    int disp_epoch = 0;        // tag of the last displacement check
};

namespace mlp {

// ---- kernel timing (prof.hip) ----
enum ProfKernel { PK_MSG_FWD = 0, PK_MSG_BWD = 1, PK_GEMM = 2, PK_PRUNE = 3, PK_NBR = 4, PK_COUNT = 5 };
extern bool g_prof_on;
void prof_begin(int k, hipStream_t s);
void prof_end(int k, hipStream_t s);
struct ProfScope {
    int k;
    hipStream_t s;
    ProfScope(int k_, hipStream_t s_) : k(k_), s(s_) { if (g_prof_on) prof_begin(k, s); }
    ~ProfScope() { if (g_prof_on) prof_end(k, s); }
};

// ---- scan / utility (nbr.hip) ----
int scan_exclusive(const int *in, int *out, int n, DevBuf &tmp, int *n_grows, hipStream_t s);

// ---- graph (nbr.hip) ----
int build_graph(mlp_model *m, mlp_nbr *g, const float *pos, const int32_t *species, int n, int n_local,
                const double box[3], float skin, hipStream_t s);
int prune_graph(mlp_model *m, mlp_nbr *g, const float *pos, hipStream_t s);
// Bytes each per-evaluation graph buffer needs (the sizes prune_graph and
// compute_hops ensure), in the order pos4, rowc, colc, revc, geom, map,
// oldidx, hop, scan_tmp.
enum { EN_POS4 = 0, EN_ROWC, EN_COLC, EN_REVC, EN_GEOM, EN_MAP, EN_OLDIDX, EN_HOP, EN_SCAN, EN_GRAPH_COUNT };
void eval_graph_needs(const mlp_nbr *g, size_t need[EN_GRAPH_COUNT]);
int compute_hops(mlp_model *m, mlp_nbr *g, hipStream_t s);
// Build and validate the owner -> ghosts map unless the one from the same
// owner array since the last neighbour build is at hand (one stream
// synchronisation when it is built); INVALID_ARG for an owner out of range.
int prepare_owner_map(mlp_nbr *g, const int32_t *owner, hipStream_t s);
// Add each ghost row of forces into its owner's row (after prepare_owner_map).
int fold_ghosts(mlp_nbr *g, float *forces, hipStream_t s);
int max_displacement_exceeds(mlp_nbr *g, const float *pos, float limit, hipStream_t s, bool *exceeds);

// ---- model (painn.hip) ----
// Floats per atom and feature of a PaiNN evaluation's saved layer arrays
// (per layer) and of its adjoint work arrays.
int layer_work_per_feature(int F);
int adjoint_work_per_feature(int F);
// Energy of each of n_seg segments (seg_dev: device [n_seg + 1] internal row
// offsets, or nullptr for one segment covering all rows), forces of all rows.
int evaluate(mlp_model *m, mlp_nbr *g, hipStream_t s, double *energy, float *forces_user,
             float *atom_energy_user, int n_seg = 1, const int *seg_dev = nullptr);
// Bytes of the buffers evaluate() ensures: the activation arena, the edge
// gradients G and the adjoint's edge-sum slots Gs.
void eval_model_needs(const mlp_model *m, const mlp_nbr *g, size_t *act, size_t *G, size_t *Gs);
// Energy of each segment (FP64, fixed order) from per-atom energies U in
// internal order, and U scattered to the caller's order if atom_energy_user.
// part: device scratch of at least energy_part_doubles(n) doubles (n_seg <= n).
int launch_energy(hipStream_t s, const float *U, const int *perm, int n, int n_local, double *energy,
                  float *atom_energy_user, int n_seg, const int *seg_dev, double *part);
inline long energy_part_doubles(long n) { return n + 1024; }
// F_k = sum over in-edges e of (G at rev(e)) - (G at e), G_e = dE/d(x_dst - x_src),
// written to the caller's order (SoA).
int launch_forces(hipStream_t s, const int *rowc, const int *revc, const float4 *G, const int *perm, int n,
                  float *forces_user);

// ---- Allegro (allegro.hip) ----
// Validates the dimensions and the weight count, copies and packs the weights
// (host array in the layout of the model header); sets m->al.
int allegro_create(mlp_model *m, const AlDims &d, const float *weights, size_t n_weights);
void allegro_destroy(mlp_model *m);
int allegro_evaluate(mlp_model *m, mlp_nbr *g, hipStream_t s, double *energy, float *forces_user,
                     float *atom_energy_user, int n_seg, const int *seg_dev);
// Bytes of the per-evaluation arena (per-edge and per-atom activations).
size_t allegro_arena_bytes(const mlp_model *m, long n_atoms, long n_edges);

// ---- MACE (mace.hip) ----
// Validates the dimensions and the weight count, builds the coupling and
// contraction tables, copies, transposes and packs the weights; sets m->mc.
int mace_create(mlp_model *m, const McDims &d, const float *weights, size_t n_weights);
void mace_destroy(mlp_model *m);
int mace_evaluate(mlp_model *m, mlp_nbr *g, hipStream_t s, double *energy, float *forces_user,
                  float *atom_energy_user, int n_seg, const int *seg_dev);
size_t mace_arena_bytes(const mlp_model *m, long n_atoms, long n_edges);
// Fill m->phi0_dev (device, S x 3F) from the embedding and the first layer's
// message MLP, in the model's precision; tmp: device scratch of 2 S F floats.
int first_layer_table(mlp_model *m, hipStream_t s, float *tmp);
// Pack m->pk_l0 from the first layer's filter, phi0 and the embedding (after
// first_layer_table); sets m->l0f.  Leaves m->l0f false where the build has
// no factorised first layer for the model's (F, K, n_species).
int first_layer_factor(mlp_model *m);
int verlet_kick_drift(float *pos, float *vel, const float *forces, const float *inv_mass, int n,
                      const double box[3], float dt, hipStream_t s);
int verlet_kick(float *vel, const float *forces, const float *inv_mass, int n, float dt, hipStream_t s);

}  // namespace mlp
