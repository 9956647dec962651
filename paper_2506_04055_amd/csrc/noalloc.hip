// mlp_energy_forces_noalloc: the evaluation of mlp_energy_forces with every
// per-evaluation buffer (the pruned graph, hop marks, scan partials, the
// activation arena, the edge gradients and the adjoint's edge-sum slots)
// carved from one static device array instead of library allocations, for
// callers that cannot allocate device memory while they run (code under HIP
// graph capture, tight serving loops).  The kernels are those of
// mlp_energy_forces; only where their buffers live differs.
#include "../../include/mlp.h"
#include "internal.h"

#include <mutex>
#include <string>

namespace {

// The scratch array: one copy per device, held until the process ends.
static __device__ __align__(256) unsigned char scratch[MLP_NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's scratch array, looked up once per
// device (in host code the array's name is only a host-side stand-in).
int scratch_address(void **out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) {
        (void)hipGetLastError();
        return mlp::fail(MLP_ERR_DEVICE, "no current HIP device for the scratch array");
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return mlp::fail(MLP_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") +
                                                 hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return 0;
}

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

}  // namespace

extern "C" int mlp_energy_forces_noalloc(mlp_model *m, mlp_nbr *g, const float *pos, int32_t n_atoms,
                                         int32_t n_local, const int32_t *ghost_owner, void *stream, double *energy,
                                         float *forces, float *atom_energy) {
    using namespace mlp;
    if (!m || !g || !pos || !energy) return fail(MLP_ERR_INVALID_ARG, "null argument");
    if (g->n_builds == 0) return fail(MLP_ERR_INVALID_ARG, "neighbour handle was never built");
    if (n_atoms != g->n_atoms || n_local != g->n_local)
        return fail(MLP_ERR_INVALID_ARG, "atom counts differ from the last neighbour build");
    const bool fold = forces && ghost_owner && n_atoms > n_local;
    // the owner map lives in the neighbour handle; building it allocates, so
    // it must already be at hand for this build and this owner array
    if (fold && !(g->owner_key == ghost_owner && g->owner_build == g->n_builds))
        return fail(MLP_ERR_INVALID_ARG,
                    "ghost owner map not prepared for this neighbour build: call mlp_energy_forces once with this "
                    "ghost_owner array after the build");
    if (g->scan_tmp.p == nullptr || g->flags.p == nullptr || g->cnt.p == nullptr)
        return fail(MLP_ERR_INVALID_ARG, "neighbour handle has no build buffers");

    // slices of the scratch array, in the sizes the evaluation ensures
    size_t need[EN_GRAPH_COUNT + 3];
    eval_graph_needs(g, need);
    eval_model_needs(m, g, &need[EN_GRAPH_COUNT], &need[EN_GRAPH_COUNT + 1], &need[EN_GRAPH_COUNT + 2]);
    DevBuf *bufs[EN_GRAPH_COUNT + 3] = {&g->pos4, &g->rowc, &g->colc, &g->revc, &g->geom, &g->map,
                                        &g->oldidx, &g->hop, &g->scan_tmp, &g->act, &g->G, &g->Gs};
    size_t total = 0;
    for (size_t b : need) total += align256(b);
    if (total > (size_t)MLP_NOALLOC_SCRATCH_BYTES)
        return fail(MLP_ERR_CAPACITY, "system needs " + std::to_string(total) + " bytes of scratch; the static "
                                      "array holds " + std::to_string((size_t)MLP_NOALLOC_SCRATCH_BYTES));
    void *base = nullptr;
    if (int rc = scratch_address(&base)) return rc;

    // borrow: the handle's own buffers are set aside and restored afterwards
    DevBuf saved[EN_GRAPH_COUNT + 3];
    size_t off = 0;
    for (int q = 0; q < EN_GRAPH_COUNT + 3; q++) {
        saved[q] = *bufs[q];
        bufs[q]->p = static_cast<char *>(base) + off;
        bufs[q]->bytes = need[q];
        bufs[q]->borrowed = true;
        off += align256(need[q]);
    }
    const int grows0 = g->n_grows;
    hipStream_t s = (hipStream_t)stream;
    int rc = prune_graph(m, g, pos, s);
    if (!rc) rc = compute_hops(m, g, s);
    if (!rc) rc = evaluate(m, g, s, energy, forces, atom_energy);
    if (!rc && fold) rc = fold_ghosts(g, forces, s);
    for (int q = 0; q < EN_GRAPH_COUNT + 3; q++) *bufs[q] = saved[q];
    g->n_grows = grows0;
    return rc;
}
