// Continuous batching of independent periodic systems (mlp_server_*,
// mlp_submit, mlp_poll).
//
// A scheduler thread owns two streams.  Requests are admitted in arrival
// order while a slot is free and the admitted footprint stays within the HBM
// budget; each admitted request is copied to the device, gets its cell-list
// graph built and pruned on the prep stream, and waits as "ready".  Whenever
// no launch wave is running, every ready request is packed into one ragged
// batch (concatenated pruned CSR with atom and edge offsets, one energy
// segment per system) and evaluated by a single pass of the kernels on the
// compute stream, while the next arrivals are copied and built on the prep
// stream.  A wave's energies and forces come back in one copy each into
// pinned memory; when a wave completes, the next one is launched before
// the completed one's rows are handed to its requests, so the device does
// not wait on that host work.  mlp_poll hands the results over.  The fixed-shape buffering of the paper (Results, "Runtime
// optimizations and buffering") becomes grow-only device buffers here: the
// batch arena and the slots only grow.
#include "../../include/mlp.h"
#include "internal.h"
#include "msg.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

namespace mlp {

using clk = std::chrono::steady_clock;
constexpr int PREP_WORKERS = 4;   // preparation threads (and streams) per server

struct Req {
    uint64_t ticket = 0;
    int n = 0;
    double box[3] = {0, 0, 0};
    std::vector<float> pos;      // SoA 3 x n, copied at submit
    std::vector<int> species;
    std::vector<float> forces;   // SoA 3 x n, filled when the wave completes
    double energy = 0.0;
    int state = 0;               // 0 queued, 1 admitted, 2 ready, 3 running, 4 done, < 0 error
    int err = 0;
    std::string errmsg;
    int slot = -1;
    int64_t n_edges = 0;
    size_t bytes = 0;
    clk::time_point t_submit, t_admit, t_done;
    int batch_size = 0;
};

// A slot holds one admitted request: its graph, its device inputs and
// pinned staging for the upload (grown, never per request, so no pinned
// allocation or release sits on the request path).
struct Slot {
    mlp_nbr *nbr = nullptr;
    DevBuf pos, species;
    float *h_pos = nullptr;      // pinned, SoA 3 x cap
    int *h_species = nullptr;    // pinned, cap
    int h_cap = 0;
    bool busy = false;
};

// One request's part of a wave: its slot's pruned graph and its offsets in
// the packed batch.
struct PackDesc {
    const int *rowc, *perm, *sp, *colc, *revc;
    const float4 *geom;
    int n, ne, aoff, eoff;
};

// Host side of one wave: pinned buffers its results are copied into (one
// copy each for the energies and the forces of the whole batch) and the atom
// offsets of its systems.  Two alternate, so the next wave can be launched
// before the finished one is unpacked.
struct WaveHost {
    double *energies = nullptr;
    float *forces = nullptr;   // SoA 3 x nt, the batch's rows
    PackDesc *desc = nullptr;  // the requests' pack descriptors (copied to the device)
    size_t e_cap = 0, f_cap = 0, d_cap = 0;
    std::vector<int> seg;      // B + 1 atom offsets
    int64_t nt = 0;
};

int ensure_pinned(void **p, size_t *cap, size_t bytes) {
    if (bytes <= *cap) return 0;
    if (*p) hipHostFree(*p);
    *p = nullptr;
    *cap = 0;
    const size_t want = bytes + bytes / 4;
    if (hipHostMalloc(p, want, 0) != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return fail(MLP_ERR_OOM, "pinned allocation failed");
    }
    *cap = want;
    return 0;
}

int ensure_staging(Slot &sl, int n) {
    if (n <= sl.h_cap) return 0;
    if (sl.h_pos) hipHostFree(sl.h_pos);
    if (sl.h_species) hipHostFree(sl.h_species);
    sl.h_pos = nullptr;
    sl.h_species = nullptr;
    sl.h_cap = 0;
    const int cap = n + n / 4;
    if (hipHostMalloc((void **)&sl.h_pos, sizeof(float) * 3 * (size_t)cap, 0) != hipSuccess ||
        hipHostMalloc((void **)&sl.h_species, sizeof(int) * (size_t)cap, 0) != hipSuccess) {
        (void)hipGetLastError();
        return fail(MLP_ERR_OOM, "pinned staging allocation failed");
    }
    sl.h_cap = cap;
    return 0;
}

// Packs every request of a wave (blockIdx.y = request) in one launch:
// atom rows (row offsets shifted by the request's edge offset, internal
// order and species shifted by its atom offset), and edge rows (columns and
// reverse indices shifted likewise, geometry copied).
__global__ void k_pack_wave(const PackDesc *__restrict__ D, int *__restrict__ browc, int *__restrict__ bperm,
                            int *__restrict__ bsp, int8_t *__restrict__ bhop, int *__restrict__ bcol,
                            int *__restrict__ brev, float4 *__restrict__ bgeom) {
    const PackDesc d = D[blockIdx.y];
    const bool last = blockIdx.y == gridDim.y - 1;
    const int span = max(d.n + 1, d.ne);
    for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < span; k += gridDim.x * blockDim.x) {
        if (k < d.n) {
            browc[d.aoff + k] = d.eoff + d.rowc[k];
            bperm[d.aoff + k] = d.aoff + d.perm[k];
            bsp[d.aoff + k] = d.sp[k];
            bhop[d.aoff + k] = 0;
        } else if (k == d.n && last) {
            browc[d.aoff + d.n] = d.eoff + d.rowc[d.n];
        }
        if (k < d.ne) {
            bcol[d.eoff + k] = d.aoff + d.colc[k];
            brev[d.eoff + k] = d.eoff + d.revc[k];
            bgeom[d.eoff + k] = d.geom[k];
        }
    }
}

// Device bytes of one system of n atoms: activations of every layer, the
// adjoint's work arrays and graph buffers for up to 120 neighbours within
// rc + skin per atom.
static size_t footprint(const mlp_model *m, int n) {
    const size_t F = m->F, T = m->T;
    const size_t act = (layer_work_per_feature((int)F) * T + 4 + adjoint_work_per_feature((int)F) + 1) * F * 4 + 64;
    const size_t nslot = (size_t)msg_slots((int)F, (int)T, false);   // the adjoint's edge sums (at most)
    const size_t graph = 120 * (60 + 16 * nslot) + 96;
    return (size_t)n * (act + graph) + (1u << 20);
}

}  // namespace mlp

using namespace mlp;

struct mlp_server {
    mlp_model *m = nullptr;
    size_t budget = 0, reserved = 0;
    int max_slots = 0;
    int device = 0;
    std::vector<Slot> slots;
    std::mutex mu;
    std::condition_variable cv;
    bool stop = false;
    std::thread th;
    std::deque<Req *> pending;
    std::unordered_map<uint64_t, Req *> all;
    std::vector<Req *> ready, running;
    uint64_t next_ticket = 1;
    // admitted requests are prepared (copied, graph built and pruned) by a
    // few worker threads, each with its own stream, so the host round trips
    // of one preparation overlap the others and the running wave
    std::deque<Req *> to_prep;
    int n_prep_busy = 0;
    bool stop_workers = false;
    std::vector<std::thread> workers;
    std::vector<hipStream_t> s_preps;
    hipStream_t s_comp = nullptr;
    hipEvent_t ev_wave = nullptr;
    bool wave_in_flight = false;
    mlp_nbr batch;              // packed graph + activations of the running wave
    DevBuf seg, energies, forces, pdesc;
    WaveHost wh[2];             // host side of the wave in flight (wh[cur]) and of the one before
    int cur = 0;
    float skin = 0.0f;
};

namespace {

void fail_req(Req *r, int code, const char *msg) {
    r->state = code < 0 ? code : -5;
    r->err = r->state;
    r->errmsg = msg ? msg : "";
}

// Copy, build and prune one admitted request on the prep stream.  Runs
// without the lock and changes no state a poller reads: the caller publishes
// the outcome (ready, or failed with the slot released) under the lock, so a
// poller never sees a failed request while the scheduler still holds it.
int prepare(mlp_server *S, Req *r, hipStream_t sp, std::string *msg) {
    Slot &sl = S->slots[r->slot];
    int *G = &sl.nbr->n_grows;
    int rc = sl.pos.ensure(sizeof(float) * 3 * (size_t)r->n, 1.2, G);
    if (!rc) rc = sl.species.ensure(sizeof(int) * (size_t)r->n, 1.2, G);
    if (!rc) rc = ensure_staging(sl, r->n);
    if (!rc) {
        std::memcpy(sl.h_pos, r->pos.data(), sizeof(float) * 3 * r->n);
        std::memcpy(sl.h_species, r->species.data(), sizeof(int) * r->n);
    }
    if (!rc && (hipMemcpyAsync(sl.pos.p, sl.h_pos, sizeof(float) * 3 * r->n, hipMemcpyHostToDevice, sp) !=
                    hipSuccess ||
                hipMemcpyAsync(sl.species.p, sl.h_species, sizeof(int) * r->n, hipMemcpyHostToDevice, sp) !=
                    hipSuccess))
        rc = fail(MLP_ERR_DEVICE, "request upload failed");
    mlp_nbr *g = sl.nbr;
    if (!rc) rc = build_graph(S->m, g, sl.pos.as<float>(), sl.species.as<int>(), r->n, r->n, r->box, S->skin, sp);
    if (!rc) rc = prune_graph(S->m, g, sl.pos.as<float>(), sp);
    int Ec = 0;
    if (!rc && (hipMemcpyAsync(&Ec, g->rowc.as<int>() + r->n, sizeof(int), hipMemcpyDeviceToHost, sp) !=
                    hipSuccess ||
                hipStreamSynchronize(sp) != hipSuccess))
        rc = fail(MLP_ERR_DEVICE, "prep stream failed");
    if (rc) {
        (void)hipStreamSynchronize(sp);   // nothing of this request is still in flight on the slot
        *msg = mlp_last_error();
        return rc;
    }
    r->n_edges = Ec;
    return 0;
}

// Pack all ready requests and launch one evaluation on the compute stream.
int launch_wave(mlp_server *S) {
    std::vector<Req *> &W = S->running;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        W.swap(S->ready);
        S->ready.clear();
    }
    const int B = (int)W.size();
    int64_t Nt = 0, Et = 0;
    for (Req *r : W) {
        Nt += r->n;
        Et += r->n_edges;
    }
    mlp_nbr &g = S->batch;
    int *G = &g.n_grows;
    int rc;
    if ((rc = g.rowc.ensure(sizeof(int) * (Nt + 1), 1.25, G)) || (rc = g.perm.ensure(sizeof(int) * Nt, 1.25, G)) ||
        (rc = g.species.ensure(sizeof(int) * Nt, 1.25, G)) || (rc = g.hop.ensure(Nt + 16, 1.25, G)) ||
        (rc = g.colc.ensure(sizeof(int) * Et + 16, 1.25, G)) || (rc = g.revc.ensure(sizeof(int) * Et + 16, 1.25, G)) ||
        (rc = g.geom.ensure(sizeof(float4) * Et + 16, 1.25, G)) ||
        (rc = S->seg.ensure(sizeof(int) * (B + 1), 1.25, G)) ||
        (rc = S->pdesc.ensure(sizeof(PackDesc) * B, 1.25, G)) ||
        (rc = S->energies.ensure(sizeof(double) * B, 1.25, G)) ||
        (rc = S->forces.ensure(sizeof(float) * 3 * Nt, 1.25, G)))
        return rc;
    // this wave's host buffers: the other pair than the previous wave's,
    // which may not be unpacked yet
    S->cur ^= 1;
    WaveHost &H = S->wh[S->cur];
    if ((rc = ensure_pinned((void **)&H.energies, &H.e_cap, sizeof(double) * B)) ||
        (rc = ensure_pinned((void **)&H.forces, &H.f_cap, sizeof(float) * 3 * (size_t)Nt)) ||
        (rc = ensure_pinned((void **)&H.desc, &H.d_cap, sizeof(PackDesc) * B)))
        return rc;
    H.seg.assign(B + 1, 0);
    H.nt = Nt;
    // one launch packs every request: its descriptor holds the slot's graph
    // and its offsets in the batch
    int64_t aoff = 0, eoff = 0, span = 1;
    for (int b = 0; b < B; b++) {
        Req *r = W[b];
        mlp_nbr *sg = S->slots[r->slot].nbr;
        H.desc[b] = PackDesc{sg->rowc.as<int>(), sg->perm.as<int>(), sg->species.as<int>(), sg->colc.as<int>(),
                             sg->revc.as<int>(), sg->geom.as<float4>(), r->n, (int)r->n_edges, (int)aoff, (int)eoff};
        span = std::max<int64_t>(span, std::max<int64_t>(r->n + 1, r->n_edges));
        H.seg[b] = (int)aoff;
        aoff += r->n;
        eoff += r->n_edges;
    }
    HIP_TRY(hipMemcpyAsync(S->pdesc.p, H.desc, sizeof(PackDesc) * B, hipMemcpyHostToDevice, S->s_comp));
    k_pack_wave<<<dim3((unsigned)std::min<int64_t>((span + 255) / 256, 1024), (unsigned)B), 256, 0, S->s_comp>>>(
        S->pdesc.as<PackDesc>(), g.rowc.as<int>(), g.perm.as<int>(), g.species.as<int>(), g.hop.as<int8_t>(),
        g.colc.as<int>(), g.revc.as<int>(), g.geom.as<float4>());
    {
        std::lock_guard<std::mutex> lk(S->mu);
        for (Req *r : W) {
            r->state = 3;
            r->batch_size = B;
        }
    }
    H.seg[B] = (int)aoff;
    HIP_TRY(hipMemcpyAsync(S->seg.p, H.seg.data(), sizeof(int) * (B + 1), hipMemcpyHostToDevice, S->s_comp));
    g.n_atoms = (int)Nt;
    g.n_local = (int)Nt;
    g.n_edges_skin = Et;
    g.n_builds = 1;
    if ((rc = evaluate(S->m, &g, S->s_comp, S->energies.as<double>(), S->forces.as<float>(), nullptr, B,
                       S->seg.as<int>())))
        return rc;
    // the results come back in two copies (the whole batch's energies and
    // forces); each request's rows are taken out on the host
    HIP_TRY(hipMemcpyAsync(H.energies, S->energies.p, sizeof(double) * B, hipMemcpyDeviceToHost, S->s_comp));
    HIP_TRY(hipMemcpyAsync(H.forces, S->forces.p, sizeof(float) * 3 * (size_t)Nt, hipMemcpyDeviceToHost, S->s_comp));
    HIP_TRY(hipEventRecord(S->ev_wave, S->s_comp));
    S->wave_in_flight = true;
    return 0;
}

// Unpack a completed wave (its requests `done`, its host buffers `H`).
void finish_wave(mlp_server *S, std::vector<Req *> &done, const WaveHost &H) {
    const auto now = clk::now();
    // the rows of each request, out of the batch's SoA forces, before the lock
    for (size_t b = 0; b < done.size(); b++) {
        Req *r = done[b];
        r->energy = H.energies[b];
        r->forces.resize(3 * (size_t)r->n);
        for (int d = 0; d < 3; d++) {
            const float *hf = H.forces + (size_t)d * H.nt + H.seg[b];
            std::copy(hf, hf + r->n, r->forces.begin() + (size_t)d * r->n);
        }
    }
    std::lock_guard<std::mutex> lk(S->mu);
    for (size_t b = 0; b < done.size(); b++) {
        Req *r = done[b];
        r->t_done = now;
        r->state = 4;
        S->slots[r->slot].busy = false;
        S->reserved -= r->bytes;
        r->slot = -1;
    }
    done.clear();
    S->cv.notify_all();
}

// One preparation worker: takes admitted requests, prepares them on its own
// stream and publishes each as ready (or failed, its slot released).
void prep_worker(mlp_server *S, int k) {
    hipSetDevice(S->device);
    for (;;) {
        Req *r = nullptr;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            S->cv.wait(lk, [&] { return S->stop_workers || !S->to_prep.empty(); });
            if (S->to_prep.empty()) break;
            r = S->to_prep.front();
            S->to_prep.pop_front();
            S->n_prep_busy++;
        }
        std::string msg;
        const int rc = prepare(S, r, S->s_preps[k], &msg);
        {
            std::lock_guard<std::mutex> lk(S->mu);
            if (rc == 0) {
                r->state = 2;
                S->ready.push_back(r);
            } else {
                fail_req(r, rc, msg.c_str());
                S->slots[r->slot].busy = false;
                S->reserved -= r->bytes;
                r->slot = -1;
                r->t_done = clk::now();
            }
            S->n_prep_busy--;
        }
        S->cv.notify_all();
    }
}

// Launch a wave of every ready request; if the launch fails, its requests
// fail (and their slots are released).
void start_wave(mlp_server *S) {
    const int rc = launch_wave(S);
    if (!rc) return;
    // kernels of the partly launched wave may still read the slots
    (void)hipStreamSynchronize(S->s_comp);
    std::lock_guard<std::mutex> lk(S->mu);
    for (Req *r : S->running) {
        fail_req(r, rc, mlp_last_error());
        S->slots[r->slot].busy = false;
        S->reserved -= r->bytes;
        r->slot = -1;
        r->t_done = clk::now();
    }
    S->running.clear();
}

// The scheduler: admission in arrival order, and waves.  When a wave
// completes, the next one, of every request ready by then, is launched and
// then the completed one is unpacked.
void scheduler(mlp_server *S) {
    hipSetDevice(S->device);
    for (;;) {
        bool admitted = false, have_ready = false;
        {
            std::unique_lock<std::mutex> lk(S->mu);
            if (!S->wave_in_flight && S->pending.empty() && S->ready.empty())
                S->cv.wait_for(lk, std::chrono::microseconds(200));
            if (S->stop && S->pending.empty() && S->to_prep.empty() && S->n_prep_busy == 0 && S->ready.empty() &&
                !S->wave_in_flight)
                break;
            // admission in arrival order: a free slot and room in the budget
            while (!S->pending.empty()) {
                Req *r = S->pending.front();
                int free_slot = -1;
                for (int k = 0; k < (int)S->slots.size(); k++)
                    if (!S->slots[k].busy) {
                        free_slot = k;
                        break;
                    }
                if (free_slot < 0 || S->reserved + r->bytes > S->budget) break;
                S->pending.pop_front();
                S->slots[free_slot].busy = true;
                S->reserved += r->bytes;
                r->slot = free_slot;
                r->state = 1;
                r->t_admit = clk::now();
                S->to_prep.push_back(r);
                admitted = true;
            }
            have_ready = !S->ready.empty();
        }
        if (admitted) S->cv.notify_all();
        if (S->wave_in_flight) {
            const hipError_t q = hipEventQuery(S->ev_wave);
            if (q == hipSuccess) {
                // the next wave goes to the device before the finished one is
                // unpacked on the host (it uses the other host buffers)
                std::vector<Req *> done;
                done.swap(S->running);
                const int dcur = S->cur;
                S->wave_in_flight = false;
                {
                    std::lock_guard<std::mutex> lk(S->mu);
                    have_ready = !S->ready.empty();
                }
                if (have_ready) start_wave(S);
                have_ready = false;
                finish_wave(S, done, S->wh[dcur]);
            } else if (q != hipErrorNotReady) {
                // the wave failed on the device: its requests fail instead of waiting forever
                (void)hipStreamSynchronize(S->s_comp);
                std::lock_guard<std::mutex> lk(S->mu);
                for (Req *r : S->running) {
                    fail_req(r, MLP_ERR_DEVICE, "evaluation failed on the device");
                    S->slots[r->slot].busy = false;
                    S->reserved -= r->bytes;
                    r->slot = -1;
                    r->t_done = clk::now();
                }
                S->running.clear();
                S->wave_in_flight = false;
            }
        }
        if (!S->wave_in_flight && have_ready) start_wave(S);
        // a wave in flight: poll its event for a few tens of microseconds
        // (yielding) before the next admission round; a sleep here overshot
        // to 50-500 us and left the device idle between waves
        if (S->wave_in_flight)
            for (int k = 0; k < 64 && hipEventQuery(S->ev_wave) == hipErrorNotReady; k++) std::this_thread::yield();
    }
}

void free_req(Req *r) { delete r; }

}  // namespace

extern "C" {

int mlp_server_create(mlp_model *m, size_t hbm_budget_bytes, int32_t max_slots, mlp_server **out) {
    if (!m || !out || max_slots < 1 || hbm_budget_bytes == 0) return fail(MLP_ERR_INVALID_ARG, "bad argument");
    if (m->al || m->mc) return fail(MLP_ERR_INVALID_ARG, "the server's admission model is PaiNN's; serve a PaiNN model");
    mlp_server *S = new mlp_server();
    S->m = m;
    S->budget = hbm_budget_bytes;
    S->max_slots = max_slots;
    S->skin = 0.0f;
    hipGetDevice(&S->device);
    S->slots.resize(max_slots);
    for (auto &sl : S->slots) sl.nbr = new mlp_nbr();
    S->s_preps.assign(PREP_WORKERS, nullptr);
    bool streams_ok = true;
    for (hipStream_t &sp : S->s_preps) streams_ok &= hipStreamCreateWithFlags(&sp, hipStreamNonBlocking) == hipSuccess;
    if (!streams_ok ||
        hipStreamCreateWithFlags(&S->s_comp, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&S->ev_wave, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        for (hipStream_t sp : S->s_preps)
            if (sp) hipStreamDestroy(sp);
        if (S->s_comp) hipStreamDestroy(S->s_comp);
        for (auto &sl : S->slots) mlp_nbr_destroy(sl.nbr);
        delete S;
        return fail(MLP_ERR_DEVICE, "stream creation failed");
    }
    for (int k = 0; k < PREP_WORKERS; k++) S->workers.emplace_back(prep_worker, S, k);
    S->th = std::thread(scheduler, S);
    *out = S;
    return MLP_OK;
}

int mlp_server_destroy(mlp_server *S) {
    if (!S) return MLP_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (Req *r : S->pending) {
            fail_req(r, MLP_ERR_UNKNOWN_TICKET, "server destroyed");
        }
        S->pending.clear();
    }
    S->cv.notify_all();
    if (S->th.joinable()) S->th.join();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop_workers = true;
    }
    S->cv.notify_all();
    for (std::thread &w : S->workers)
        if (w.joinable()) w.join();
    hipStreamSynchronize(S->s_comp);
    for (hipStream_t sp : S->s_preps)
        if (sp) hipStreamSynchronize(sp);
    for (auto &kv : S->all) free_req(kv.second);
    for (auto &sl : S->slots) {
        sl.pos.release();
        sl.species.release();
        if (sl.h_pos) hipHostFree(sl.h_pos);
        if (sl.h_species) hipHostFree(sl.h_species);
        mlp_nbr_destroy(sl.nbr);
    }
    DevBuf *bufs[] = {&S->batch.rowc, &S->batch.perm, &S->batch.species, &S->batch.hop, &S->batch.colc,
                      &S->batch.revc, &S->batch.geom, &S->batch.act, &S->batch.G, &S->batch.Gs, &S->seg, &S->energies,
                      &S->forces, &S->pdesc};
    for (DevBuf *b : bufs) b->release();
    for (WaveHost &H : S->wh) {
        if (H.energies) hipHostFree(H.energies);
        if (H.forces) hipHostFree(H.forces);
        if (H.desc) hipHostFree(H.desc);
    }
    hipEventDestroy(S->ev_wave);
    for (hipStream_t sp : S->s_preps)
        if (sp) hipStreamDestroy(sp);
    hipStreamDestroy(S->s_comp);
    delete S;
    return MLP_OK;
}

int mlp_submit(mlp_server *S, const mlp_request *q, uint64_t *ticket) {
    if (!S || !q || !ticket || !q->pos || !q->species || q->n_atoms <= 0)
        return fail(MLP_ERR_INVALID_ARG, "bad request");
    const size_t bytes = footprint(S->m, q->n_atoms);
    if (bytes > S->budget) return fail(MLP_ERR_INVALID_ARG, "request exceeds the server's device-memory budget");
    for (int d = 0; d < 3; d++)
        if (!(q->box[d] > 0.0)) return fail(MLP_ERR_INVALID_ARG, "served systems must be periodic (box > 0)");
    Req *r = new Req();
    r->n = q->n_atoms;
    std::memcpy(r->box, q->box, sizeof(r->box));
    r->bytes = bytes;
    r->pos.assign(q->pos, q->pos + 3 * (size_t)r->n);
    r->species.assign(q->species, q->species + (size_t)r->n);
    r->t_submit = clk::now();
    {
        std::lock_guard<std::mutex> lk(S->mu);
        r->ticket = S->next_ticket++;
        S->pending.push_back(r);
        S->all[r->ticket] = r;
    }
    S->cv.notify_all();
    *ticket = r->ticket;
    return MLP_OK;
}

int mlp_poll(mlp_server *S, uint64_t ticket, double *energy, float *forces, mlp_timing *timing) {
    if (!S) return fail(MLP_ERR_INVALID_ARG, "null server");
    Req *r = nullptr;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        auto it = S->all.find(ticket);
        if (it == S->all.end()) return fail(MLP_ERR_UNKNOWN_TICKET, "unknown or retired ticket");
        r = it->second;
        if (r->state >= 0 && r->state < 4) return MLP_PENDING;
        S->all.erase(it);
    }
    int rc = MLP_OK;
    if (r->state < 0) {
        rc = fail(r->err, r->errmsg);
    } else {
        if (energy) *energy = r->energy;
        if (forces) std::memcpy(forces, r->forces.data(), sizeof(float) * 3 * r->n);
        if (timing) {
            timing->latency_us = std::chrono::duration<double, std::micro>(r->t_done - r->t_submit).count();
            timing->queue_us = std::chrono::duration<double, std::micro>(r->t_admit - r->t_submit).count();
            timing->batch_size = r->batch_size;
        }
    }
    free_req(r);
    return rc;
}

}  // extern "C"
