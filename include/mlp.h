/*
 * libmlp — PaiNN-form machine-learning potential: energy and forces on one
 * MI355X (gfx950).  C ABI; no C++ or torch types cross this boundary.
 *
 * Method (arXiv 2506.04055, Results "Distributed potential computation"):
 *   the total energy of a domain is the sum of semi-local per-atom energies
 *   U_i of the local atoms (Eq. 1); the forces are the partial derivatives of
 *   that sum with respect to every atom of the domain, local and ghost, whose
 *   ghost rows are summed onto their owners (Eq. 2).  Neighbour graphs are
 *   built with a skin and edges longer than the model cutoff are pruned at
 *   every evaluation; atoms farther than T hops from any local atom are
 *   pruned as well (same paragraph, pruning).  Buffers are sized to
 *   capacities that only grow (Results, "Runtime optimizations and
 *   buffering").  The per-atom energy is PaiNN (Methods, "Chosen
 *   Architectures"), with T message/update layers, F features, K radial
 *   Bessel functions sin(k pi r / rc) / r and a cosine cutoff envelope.
 *
 * Units: Angstrom, eV, eV/Angstrom, amu, fs.
 *
 * Conventions for every call
 *   - Return value: MLP_OK (0), MLP_PENDING (1) or a negative MLP_ERR_*.
 *     After an error, mlp_last_error() returns a message (thread-local).
 *   - Device pointers are HIP device memory owned by the caller; the library
 *     never frees or retains them beyond the call.  Host pointers are read
 *     during the call only (mlp_submit copies what it needs).
 *   - Positions and forces are structure-of-arrays: 3 rows of N floats
 *     (x[0..N), then y[0..N), then z[0..N)).
 *   - Work is enqueued on the caller's stream (hipStream_t passed as void*;
 *     NULL is the default stream).  Calls that return sizes or statistics
 *     synchronise that stream; mlp_energy_forces without stats does not.
 *   - Handles (mlp_model, mlp_nbr, mlp_server) are owned by the library and
 *     released with their *_destroy call.  A handle may be used from one
 *     thread at a time.
 */
#ifndef MLP_H
#define MLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    MLP_OK = 0,
    MLP_PENDING = 1,
    MLP_ERR_INVALID_ARG = -1,   /* bad shape, species out of range, bad header */
    MLP_ERR_OOM = -2,           /* device allocation failed */
    MLP_ERR_CAPACITY = -3,      /* a buffer overflowed and could not be grown */
    MLP_ERR_BOX_TOO_SMALL = -4, /* rc + skin >= L/2 in a periodic dimension */
    MLP_ERR_DEVICE = -5,        /* a HIP runtime call failed */
    MLP_ERR_UNKNOWN_TICKET = -6
};

enum { MLP_FP32 = 0, MLP_BF16 = 1, MLP_BF16_FAST = 2, MLP_BF16_NODE = 3, MLP_BF16_NODE_X3 = 4 };

typedef struct mlp_model mlp_model;
typedef struct mlp_nbr mlp_nbr;
typedef struct mlp_server mlp_server;
typedef struct mlp_nvt mlp_nvt;

/* Statistics of one evaluation (the library "returns statistics of the
 * computation", Results, "Runtime optimizations and buffering"). */
typedef struct {
    int64_t n_edges_skin;      /* directed edges within rc + skin            */
    int64_t n_edges;           /* directed edges within rc (used)            */
    int32_t n_atoms;           /* atoms of the domain (local + ghost)        */
    int32_t n_local;
    int32_t n_within_hops[8];  /* atoms within <= t hops of a local atom     */
    int32_t n_cells[3];        /* cell grid of the last neighbour build      */
    int32_t max_cell_occupancy;
    int32_t n_builds;          /* neighbour builds so far on this handle     */
    int32_t n_grows;           /* capacity growths so far on this handle     */
    int64_t device_bytes;      /* device memory held by the nbr handle       */
    int64_t n_edges_within_hops[8]; /* pruned edges whose destination atom is
                                       within <= t hops of a local atom      */
} mlp_stats;

/* Message describing the last error of the calling thread. */
const char *mlp_last_error(void);

/* ---------------------------------------------------------------------------
 * Model
 * header_json: the export properties of the model (Results, "Structure":
 *   units, maximal edge length, graph format) plus the architecture:
 *   {"model":"painn","F":..,"K":..,"T":..,"n_species":..,"r_c":..,"eps":..,
 *    "basis":"bessel_sin_over_r","envelope":"cosine",...}.
 *   Supported: (F, K) in {(128,20), (128,8), (64,20), (64,8), (32,20), (32,8),
 *   (16,6)}, 1 <= T <= 7, n_species >= 1.
 * weights: host float32 array of n_weights values in the stated layout
 *   (emb [S][F]; per layer W1 [F][F] b1 [F] W2 [3F][F] b2 [3F] A [3F][K]
 *   c [3F] U [F][F] V [F][F] W3 [F][2F] b3 [F] W4 [3F][F] b4 [3F]; then
 *   W5 [F/2][F] b5 [F/2] w6 [F/2] b6 [1]); matrices are [out][in] row-major;
 *   3F blocks are split [vv | s | vs] (message) and [vv | sv | ss] (update).
 *   Copied to the device; the caller keeps ownership of its array.
 * header_json may instead describe an Allegro model with one tensor-product
 *   layer (Methods, "Chosen Architectures" and "Training Details": the
 *   strictly local, edge-centric model, one layer, l_max = 3, 8 radial
 *   functions, polynomial envelope of order 2):
 *   {"model":"allegro","n_species":..,"r_c":..,"n_basis":..,"envelope_p":..,
 *    "mlp_2b":[..],"channels":[n_0,..,n_lmax],"latent_hidden":..,
 *    "out_hidden":..,"env_scale":..,"basis":"bessel","envelope":"polynomial"}
 *   with l_max <= 3, channels totalling at most 64 (a multiple of 4), the
 *   last two-body width (the latent width D) at most 64, every width a
 *   multiple of 4.  Weights (matrices [out][in]): for each two-body layer q
 *   W_q [d_q][d_(q-1)] b_q [d_q] (d_0's input: onehot(Z_i) | onehot(Z_j) |
 *   radial functions); Wv [NC][D]; We [NC][D]; lat_W1 [LH][D + NC]
 *   lat_b1 [LH] lat_W2 [D][LH] lat_b2 [D]; out_W1 [OH][D] out_b1 [OH]
 *   out_w2 [OH] out_b2 [1].  An Allegro model is strictly local: its graph
 *   needs ghosts within rc only, and the serving calls do not take it.
 * header_json may instead describe a MACE model with two interaction layers
 *   (Methods, "Chosen Architectures" and "Training Details": correlation
 *   order 3, l_max = 3, 32 scalar and 32 vector channels, 8 radial functions,
 *   polynomial envelope of order 6):
 *   {"model":"mace","n_species":..,"r_c":..,"n_basis":..,"envelope_p":..,
 *    "l_max":3,"channels":32,"correlation":3,"radial_hidden":[..],
 *    "readout_hidden":..,"avg_neighbors":..,"basis":"bessel",
 *    "envelope":"polynomial"}
 *   with 1..4 radial widths (multiples of 4, at most 256) and a readout
 *   width of at most 32.  Layer 1 takes degree 0 and produces degrees 0
 *   and 1, layer 2 takes 0 and 1 and produces 0; a coupling l1 x l2 -> L is
 *   used only where |l1 - l2| <= L <= l1 + l2 and l1 + l2 + L is even.
 *   Conv paths (l1, l2, L) of a layer in order: l2 over its input degrees,
 *   then l1 = 0..3, then L = 0..3.  Contraction paths onto an output
 *   degree L_o in order: (A_Lo); the pairs (l1 <= l2) coupled to L_o; the
 *   triples (l1 <= l2, lambda, l3) with l1 x l2 -> lambda and
 *   lambda x l3 -> L_o, looped l1, l2, lambda, l3.  Weights (K = 32,
 *   matrices [out][in]): W_emb [K][S]; per layer: W_up [K][K] per input
 *   degree; the radial matrices [r_1][n_basis], [r_q][r_(q-1)], and
 *   [P K][r_last] (P conv paths, output column p K + k); W_A [K][n_L K] for
 *   L = 0..3 (n_L paths onto L, columns in path order); W_sym [S][K][paths]
 *   per output degree; W_out [K][K] per output degree; W_sc [S][K][K] for
 *   degree 0; then w_r1 [K], W_r2 [RH][K], b_r2 [RH], w_r2 [RH], b_r3 [1].
 *   Its graph needs ghosts within 2 rc; the serving calls do not take it.
 * precision: the operand forms of the two matrix-core contractions, the
 *   node-feature GEMMs (node) and the radial filter of the message kernels
 *   (filter):
 *   MLP_FP32         node FP32, filter FP32 (v_mfma_f32_16x16x4_f32);
 *   MLP_BF16         node and filter split bfloat16 ("bf16x3"): x = hi + lo,
 *                    three bf16 products per tile (v_mfma_f32_16x16x32_bf16),
 *                    about 16 significant bits per operand;
 *   MLP_BF16_FAST    node and filter plain bfloat16 (one product; bfloat16
 *                    rounding of activations, weights and basis);
 *   MLP_BF16_NODE    node plain bfloat16, filter FP32: bfloat16 node GEMMs with
 *                    FP32 accumulation, everything else FP32;
 *   MLP_BF16_NODE_X3 node plain bfloat16, filter split bfloat16.
 *   Accumulation is FP32 in every mode; geometry, cutoff envelope, message
 *   and force accumulation stay FP32; the energy sum is FP64.
 * Errors: INVALID_ARG (header or weight count), OOM, DEVICE.
 * ------------------------------------------------------------------------- */
int mlp_model_create(const char *header_json, const float *weights, size_t n_weights,
                     int precision, mlp_model **out);
int mlp_model_destroy(mlp_model *model);

/* ---------------------------------------------------------------------------
 * mlp_build_neighbors — cell-list neighbour graph of all atoms within
 * rc + skin (Results, "Distributed potential computation": the MD engine
 * builds lists with a skin so they need not be rebuilt every step).
 * pos: device, SoA 3 x n_atoms float32.  Periodic dimensions (box[d] > 0)
 *   require 0 <= x < box[d]; box lengths should be float32-representable.
 *   Locals are rows [0, n_local); ghosts follow.  With ghosts
 *   (n_atoms > n_local) the domain is open in every dimension: ghost atoms
 *   are explicit copies and no minimum image is applied; box is then ignored.
 * species: device int32 [n_atoms], each in [0, n_species).
 * skin >= 0.  A pair (i, j) is a neighbour iff, in float32,
 *   dx = x_j - x_i, folded once by +-L when |dx| > L/2 (periodic dims),
 *   fma(dz, dz, fma(dy, dy, dx*dx)) < (rc + skin)^2.
 * *inout: NULL to create a handle, or an existing handle to refresh (its
 *   buffers are reused and grown when too small, never shrunk).
 * Synchronises the stream (edge counts size the buffers).
 * Errors: INVALID_ARG (sizes, species, positions outside the box),
 *   BOX_TOO_SMALL (rc + skin >= L/2), OOM, DEVICE.
 * ------------------------------------------------------------------------- */
int mlp_build_neighbors(mlp_model *model, const float *pos, const int32_t *species,
                        int32_t n_atoms, int32_t n_local, const double box[3], float skin,
                        void *stream, mlp_nbr **inout);
int mlp_nbr_destroy(mlp_nbr *nbr);

/* ---------------------------------------------------------------------------
 * mlp_nbr_edges — the directed edges of a neighbour handle in the caller's
 * atom numbering: which = 0 for the rc + skin graph of the last build,
 * which = 1 for the rc graph of the last mlp_energy_forces call.
 * dst, src: device int32 arrays of capacity cap; edge e is (dst[e] <- src[e]).
 * Edges are grouped by destination in the library's internal (cell-sorted)
 * order; callers that need a canonical order sort them.
 * *n_edges (host) receives the count; when it exceeds cap nothing is written
 * and CAPACITY is returned.  Synchronises the stream.
 * ------------------------------------------------------------------------- */
int mlp_nbr_edges(mlp_nbr *nbr, int32_t which, int32_t *dst, int32_t *src, int64_t cap, int64_t *n_edges,
                  void *stream);

/* ---------------------------------------------------------------------------
 * mlp_energy_forces — E = sum_{i < n_local} U_i (Eq. 1) and F = -dE/dr for
 * every row (Eq. 2), on the graph of the last mlp_build_neighbors call with
 * edges pruned to r < rc at the current positions, and atoms farther than
 * T hops from the locals pruned.
 * pos: device SoA 3 x n_atoms (same atom order, count and n_local as the
 *   build; displacements since the build must stay below skin/2 for the
 *   result to be exact).
 * ghost_owner: NULL, or device int32 [n_atoms - n_local] with the local
 *   index each ghost copies; then each ghost row's force is also added into
 *   its owner's row (the reverse summation of partial forces) while ghost
 *   rows keep their own partial forces.  The owner -> ghosts map is built and
 *   validated at the first call after each neighbour build (or when a
 *   different ghost_owner pointer is passed), with one synchronisation of the
 *   stream; an owner outside [0, n_local) then fails with INVALID_ARG before
 *   anything is computed.  Later calls reuse the map, so the array's contents
 *   must not change between neighbour builds.
 * energy: device double [1] (written on the stream).
 * forces: device SoA 3 x n_atoms float32 (written on the stream).
 * atom_energy: NULL or device float [n_atoms] receiving U_i (ghost rows too).
 * stats: NULL, or host struct filled after a stream synchronisation.
 * Errors: INVALID_ARG, CAPACITY, DEVICE.
 * ------------------------------------------------------------------------- */
int mlp_energy_forces(mlp_model *model, mlp_nbr *nbr, const float *pos, int32_t n_atoms,
                      int32_t n_local, const int32_t *ghost_owner, void *stream, double *energy,
                      float *forces, float *atom_energy, mlp_stats *stats);

/* ---------------------------------------------------------------------------
 * mlp_energy_forces_noalloc — mlp_energy_forces for callers that cannot
 * allocate device memory while they run (code under HIP graph capture,
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, result
 * and kernels as mlp_energy_forces without stats; it calls no hipMalloc,
 * hipFree or allocating library routine.  Every per-evaluation buffer (the
 * pruned graph, hop marks, activations, edge gradients and edge sums) is a
 * slice of one static device array of MLP_NOALLOC_SCRATCH_BYTES (256 MiB),
 * which each GPU the library runs on holds until the process ends.
 * Limits: the buffers of the system must fit that array (roughly 3,000
 * atoms at F = 128, T = 3, fewer with a larger skin); a larger system fails
 * with CAPACITY, naming the bytes it needs, before anything is enqueued.
 * The neighbour handle must have been built (mlp_build_neighbors allocates;
 * call it outside the allocation-free region).  With ghost_owner, the
 * owner map must already be prepared for this build and this array (one
 * mlp_energy_forces call with it after the build), else INVALID_ARG.
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other threads, other handles) race and must be
 * serialised by the caller; results are complete once the stream has
 * reached the end of the call's work.  The array keeps the last call's
 * contents; nothing in it is assumed to start at zero.
 * mlp_nbr_edges(which = 1) keeps describing the last mlp_energy_forces call.
 * Errors: INVALID_ARG, CAPACITY, DEVICE.
 * ------------------------------------------------------------------------- */
#define MLP_NOALLOC_SCRATCH_BYTES (256ull << 20)
int mlp_energy_forces_noalloc(mlp_model *model, mlp_nbr *nbr, const float *pos, int32_t n_atoms,
                              int32_t n_local, const int32_t *ghost_owner, void *stream, double *energy,
                              float *forces, float *atom_energy);

/* ---------------------------------------------------------------------------
 * mlp_nbr_check_displacement — whether the graph of the last build is still
 * exact at the given positions: *exceeds (host) is set to 1 when some atom
 * has moved more than skin/2 from its position at the last build (then a
 * pair may have entered rc unseen and mlp_build_neighbors must run before
 * mlp_energy_forces), else 0.  The list-with-skin scheme of Results,
 * "Distributed potential computation".
 * pos: device SoA 3 x n_atoms, same atoms and order as the build; periodic
 *   displacements are taken under the minimum image.
 * Synchronises the stream.  Errors: INVALID_ARG, DEVICE, OOM (pinned word).
 * ------------------------------------------------------------------------- */
int mlp_nbr_check_displacement(mlp_nbr *nbr, const float *pos, int32_t n_atoms, void *stream,
                               int32_t *exceeds);

/* ---------------------------------------------------------------------------
 * mlp_md_step — one velocity-Verlet step (kick, drift, wrap into [0, L),
 * rebuild the neighbour graph when the largest displacement since the last
 * build exceeds skin/2, evaluate, kick) for a periodic system without ghosts,
 * the protocol the paper runs its timing simulations with (Methods,
 * "Molecular Dynamics Simulations", thermostat aside).
 * pos, vel: device SoA 3 x n float32, updated in place (vel in A/fs).
 * forces: device SoA 3 x n float32: on entry the forces at pos, on exit the
 *   forces at the new positions.  inv_mass: device float [n] (1/amu).
 * energy: device double [1], potential energy at the new positions.
 * *rebuilt (host, may be NULL) is set to 1 when the graph was rebuilt.
 * Synchronises the stream once (the displacement check).
 * ------------------------------------------------------------------------- */
int mlp_md_step(mlp_model *model, mlp_nbr *nbr, float *pos, float *vel, float *forces,
                const float *inv_mass, const int32_t *species, int32_t n, const double box[3],
                float skin, float dt, void *stream, double *energy, int32_t *rebuilt);

/* ---------------------------------------------------------------------------
 * NVT thermostat (Methods, "Molecular Dynamics Simulations": the production
 * and timing runs are NVT with a Nose-Hoover thermostat of a given damping
 * time).  A chain of `chain` Nose-Hoover thermostats with masses
 * Q_1 = n_dof kB T tau^2 and Q_k = kB T tau^2 (k > 1), positions and
 * velocities starting at zero, state kept in FP64 on the device.
 * mlp_nvt_create: n_dof >= 1 (3N - 3 when the centre-of-mass momentum is
 *   removed), temperature in K (> 0), tau in fs (> 0), 1 <= chain <= 8.
 *   Allocates device memory; synchronous.  Errors: INVALID_ARG, OOM, DEVICE.
 * mlp_nvt_destroy: frees the handle (NULL is accepted).
 * mlp_nvt_read: host copies of the chain positions xi[chain] and velocities
 *   vxi[chain] (1/fs) (each may be NULL), the thermostat energy
 *   sum_k Q_k vxi_k^2 / 2 + n_dof kB T xi_1 + kB T sum_{k>1} xi_k (eV) and
 *   the kinetic energy (eV) after the last step.  The extended energy
 *   kinetic + potential + thermostat energy is the step's conserved quantity.
 *   Synchronises the stream.  Errors: INVALID_ARG, DEVICE.
 * ------------------------------------------------------------------------- */
int mlp_nvt_create(int32_t n_dof, double temperature, double tau_fs, int32_t chain, mlp_nvt **out);
int mlp_nvt_destroy(mlp_nvt *nvt);
int mlp_nvt_read(mlp_nvt *nvt, double *xi, double *vxi, double *thermostat_energy, double *kinetic,
                 void *stream);

/* ---------------------------------------------------------------------------
 * mlp_md_step_nvt — one NVT step: the thermostat chain propagated over dt/2
 * (velocities scaled on the device), the mlp_md_step velocity-Verlet step
 * (same arguments, same rebuild rule, same single synchronisation), and the
 * chain propagated over dt/2 again.  inv_mass must be the same array the
 * kinetic energy is meant for (m = 1 / inv_mass, amu).
 * Errors: those of mlp_md_step, and INVALID_ARG for a NULL thermostat.
 * ------------------------------------------------------------------------- */
int mlp_md_step_nvt(mlp_model *model, mlp_nbr *nbr, mlp_nvt *nvt, float *pos, float *vel, float *forces,
                    const float *inv_mass, const int32_t *species, int32_t n, const double box[3], float skin,
                    float dt, void *stream, double *energy, int32_t *rebuilt);

/* ---------------------------------------------------------------------------
 * Kernel timing (tracing aid; the library's "statistics of the computation").
 * mlp_profile_enable(1) makes every later launch of the named kernels record a
 * pair of HIP events on the stream it is launched on; 0 stops recording; any
 * other value is a bit mask selecting kernels in the order of the names below
 * (bit 0 "msg_fwd", bit 1 "msg_bwd", ...).
 * mlp_profile_read waits for the recorded events of one kernel name and
 * returns the summed duration (ms) and the number of launches since the last
 * mlp_profile_reset.  Names: "msg_fwd", "msg_bwd", "node_gemm", "prune",
 * "neighbors".  Unknown name: INVALID_ARG.  Process-wide, not thread-safe.
 * ------------------------------------------------------------------------- */
int mlp_profile_enable(int32_t enable);
int mlp_profile_reset(void);
int mlp_profile_read(const char *kernel, double *total_ms, int64_t *launches);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of independent periodic systems.
 * The paper's runtime keeps device buffers of fixed shape and reuses them
 * across calls, growing them (with headroom) only when a system no longer
 * fits, and reports the statistics that decide it (Results, "Runtime
 * optimizations and buffering").  The server applies the same rule to a
 * stream of requests: each slot's buffers only grow, requests are admitted
 * by their device footprint against a fixed budget, and the admitted systems
 * of one wave are evaluated together as one ragged batch (one energy segment
 * per system, the per-system sum of Eq. 1).
 * mlp_server_create starts a scheduler thread and a few preparation threads,
 *   each with its own stream.
 *   hbm_budget_bytes bounds the device memory of admitted requests; a
 *   request whose estimated footprint exceeds the budget on its own is
 *   rejected with INVALID_ARG at submit.  max_slots bounds the number of
 *   requests resident on the device at once.
 * mlp_submit copies the request's host arrays (pos SoA 3 x n float32,
 *   species int32 [n], box) into library-owned host memory, queues it and
 *   returns a ticket without waiting for the GPU (the copies to and from the
 *   device go through pinned buffers the server keeps per slot).
 * mlp_poll returns MLP_PENDING while the request runs, MLP_OK once energy
 *   (host double) and forces (host SoA 3 x n float32) have been copied out
 *   (the ticket is then retired), or an error.  timing (nullable) receives
 *   the request's submit->done latency in microseconds and its queueing part.
 * ------------------------------------------------------------------------- */
typedef struct {
    const float *pos;        /* host SoA 3 x n_atoms */
    const int32_t *species;  /* host [n_atoms] */
    int32_t n_atoms;
    double box[3];
} mlp_request;

typedef struct {
    double latency_us;       /* submit -> results ready */
    double queue_us;         /* submit -> admitted to the device */
    int32_t batch_size;      /* requests in the launch wave that ran it */
} mlp_timing;

int mlp_server_create(mlp_model *model, size_t hbm_budget_bytes, int32_t max_slots,
                      mlp_server **out);
int mlp_server_destroy(mlp_server *server);
int mlp_submit(mlp_server *server, const mlp_request *req, uint64_t *ticket);
int mlp_poll(mlp_server *server, uint64_t ticket, double *energy, float *forces,
             mlp_timing *timing);

#ifdef __cplusplus
}
#endif
#endif /* MLP_H */
