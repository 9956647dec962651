// Kernel timing with HIP events around named launches (off by default).
#include "../../include/mlp.h"
#include "internal.h"

#include <cstring>
#include <vector>

namespace mlp {

bool g_prof_on = false;
unsigned g_prof_mask = 0;

namespace {
struct Rec {
    hipEvent_t a, b;
};
std::vector<Rec> g_recs[PK_COUNT];
std::vector<Rec> g_pool;
Rec g_open[PK_COUNT];
bool g_is_open[PK_COUNT] = {};
const char *g_names[PK_COUNT] = {"msg_fwd", "msg_bwd", "node_gemm", "prune", "neighbors"};

bool get_rec(Rec &r) {
    if (!g_pool.empty()) {
        r = g_pool.back();
        g_pool.pop_back();
        return true;
    }
    if (hipEventCreate(&r.a) != hipSuccess) return false;
    if (hipEventCreate(&r.b) != hipSuccess) {
        hipEventDestroy(r.a);
        return false;
    }
    return true;
}
}  // namespace

void prof_begin(int k, hipStream_t s) {
    if (!((g_prof_mask >> k) & 1u)) return;
    Rec r;
    if (!get_rec(r)) return;
    hipEventRecord(r.a, s);
    g_open[k] = r;
    g_is_open[k] = true;
}

void prof_end(int k, hipStream_t s) {
    if (!g_is_open[k]) return;
    hipEventRecord(g_open[k].b, s);
    g_recs[k].push_back(g_open[k]);
    g_is_open[k] = false;
}

}  // namespace mlp

using namespace mlp;

extern "C" {

int mlp_profile_enable(int32_t enable) {
    g_prof_on = enable != 0;
    g_prof_mask = enable == 1 ? 0xffffffffu : (unsigned)enable;
    return MLP_OK;
}

int mlp_profile_reset(void) {
    for (int k = 0; k < PK_COUNT; k++) {
        for (auto &r : g_recs[k]) g_pool.push_back(r);
        g_recs[k].clear();
    }
    return MLP_OK;
}

int mlp_profile_read(const char *kernel, double *total_ms, int64_t *launches) {
    if (!kernel || !total_ms || !launches) return fail(MLP_ERR_INVALID_ARG, "null argument");
    int k = -1;
    for (int q = 0; q < PK_COUNT; q++)
        if (!std::strcmp(kernel, g_names[q])) k = q;
    if (k < 0) return fail(MLP_ERR_INVALID_ARG, std::string("unknown kernel name ") + kernel);
    double tot = 0.0;
    for (auto &r : g_recs[k]) {
        if (hipEventSynchronize(r.b) != hipSuccess) return fail(MLP_ERR_DEVICE, "event wait failed");
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, r.a, r.b) != hipSuccess) return fail(MLP_ERR_DEVICE, "event timing failed");
        tot += ms;
    }
    *total_ms = tot;
    *launches = (int64_t)g_recs[k].size();
    return MLP_OK;
}

}  // extern "C"
