// C ABI of libmlp: model and neighbour handles, evaluation, MD step.
#include "../../include/mlp.h"
#include "internal.h"
#include "header_json.h"

#include <vector>

#include <cctype>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>

namespace mlp {
const char *last_error_cstr();
int hop_histogram(mlp_model *m, mlp_nbr *g, hipStream_t s, int *hist_host, int64_t *ehist_host);
int export_edges(mlp_nbr *g, const int *row, const int *col, int32_t *dst, int32_t *src, hipStream_t s);
}

using namespace mlp;

// Minimal reader for the flat top-level JSON object of the model header.
namespace {
using mlp_json::JsonTop;
using mlp_json::get_int;
using mlp_json::get_int_list;
using mlp_json::get_num;
using mlp_json::parse_top;
int status(int rc) { return rc; }
}  // namespace

mlp::LayerW mlp_model::layer(int t) const {
    LayerW L;
    const size_t *o = off_layer[t];
    L.W1 = at(o[0]); L.b1 = at(o[1]); L.W2 = at(o[2]); L.b2 = at(o[3]);
    L.A = at(o[4]); L.c = at(o[5]); L.U = at(o[6]); L.V = at(o[7]);
    L.W3 = at(o[8]); L.b3 = at(o[9]); L.W4 = at(o[10]); L.b4 = at(o[11]);
    return L;
}

// An Allegro model (single tensor-product layer): header fields n_species,
// r_c, n_basis, envelope_p, mlp_2b, channels (per degree l = 0..l_max),
// latent_hidden, out_hidden, env_scale; basis "bessel", envelope
// "polynomial".  The neighbour graph treats it as one layer (strictly local).
static int create_allegro(const JsonTop &j, const float *weights, size_t n_weights, int precision, mlp_model **out) {
    long S, NB, p, LH, OH;
    double rc, nu;
    std::vector<long> d2b, ch;
    if (!get_int(j, "n_species", &S) || !get_int(j, "n_basis", &NB) || !get_int(j, "envelope_p", &p) ||
        !get_int(j, "latent_hidden", &LH) || !get_int(j, "out_hidden", &OH) || !get_num(j, "r_c", &rc) ||
        !get_num(j, "env_scale", &nu) || !get_int_list(j, "mlp_2b", &d2b) || !get_int_list(j, "channels", &ch))
        return fail(MLP_ERR_INVALID_ARG, "allegro header lacks n_species, n_basis, envelope_p, mlp_2b, channels, "
                                         "latent_hidden, out_hidden, r_c or env_scale");
    auto str = [&](const char *k) { auto it = j.kv.find(k); return it == j.kv.end() ? std::string() : it->second; };
    if (str("basis") != "bessel" || str("envelope") != "polynomial")
        return fail(MLP_ERR_INVALID_ARG, "allegro: basis must be bessel and envelope polynomial");
    if (d2b.size() > 6 || ch.size() > 4 || ch.empty())
        return fail(MLP_ERR_INVALID_ARG, "allegro: at most 6 two-body widths and degrees 0..3");
    if (precision != MLP_FP32 && precision != MLP_BF16 && precision != MLP_BF16_FAST &&
        precision != MLP_BF16_NODE && precision != MLP_BF16_NODE_X3)
        return fail(MLP_ERR_INVALID_ARG, "unknown precision");
    AlDims d;
    d.S = (int)S;
    d.NB = (int)NB;
    d.p = (int)p;
    d.n2b = (int)d2b.size();
    for (size_t q = 0; q < d2b.size(); q++) d.d2b[q] = (int)d2b[q];
    d.lmax = (int)ch.size() - 1;
    d.NC = 0;
    for (size_t q = 0; q < ch.size(); q++) {
        if (ch[q] < 0 || ch[q] > 64) return fail(MLP_ERR_INVALID_ARG, "allegro: channel count out of range");
        d.ch[q] = (int)ch[q];
        d.NC += (int)ch[q];
    }
    d.D = d.d2b[d.n2b - 1];
    d.LH = (int)LH;
    d.OH = (int)OH;
    d.rc = (float)rc;
    d.nu = (float)nu;
    mlp_model *m = new mlp_model();
    m->F = 0;
    m->K = 0;
    m->T = 1;
    m->S = (int)S;
    m->rc = (float)rc;
    m->eps = 0.f;
    m->precision = precision;
    m->n_weights = n_weights;
    if (int rc2 = allegro_create(m, d, weights, n_weights)) {
        delete m;
        return rc2;
    }
    *out = m;
    return MLP_OK;
}

// A MACE model (two layers): header fields n_species, r_c, n_basis,
// envelope_p, l_max, channels, correlation, radial_hidden, readout_hidden,
// avg_neighbors; basis "bessel", envelope "polynomial".  The neighbour graph
// treats it as two layers (receptive field 2 r_c).
static int create_mace(const JsonTop &j, const float *weights, size_t n_weights, int precision, mlp_model **out) {
    long S, NB, p, lmax, K, corr, RH;
    double rc, navg;
    std::vector<long> rh;
    if (!get_int(j, "n_species", &S) || !get_int(j, "n_basis", &NB) || !get_int(j, "envelope_p", &p) ||
        !get_int(j, "l_max", &lmax) || !get_int(j, "channels", &K) || !get_int(j, "correlation", &corr) ||
        !get_int(j, "readout_hidden", &RH) || !get_num(j, "r_c", &rc) || !get_num(j, "avg_neighbors", &navg) ||
        !get_int_list(j, "radial_hidden", &rh))
        return fail(MLP_ERR_INVALID_ARG, "mace header lacks n_species, n_basis, envelope_p, l_max, channels, "
                                         "correlation, radial_hidden, readout_hidden, r_c or avg_neighbors");
    auto str = [&](const char *k) { auto it = j.kv.find(k); return it == j.kv.end() ? std::string() : it->second; };
    if (str("basis") != "bessel" || str("envelope") != "polynomial")
        return fail(MLP_ERR_INVALID_ARG, "mace: basis must be bessel and envelope polynomial");
    if (rh.empty() || rh.size() > 4) return fail(MLP_ERR_INVALID_ARG, "mace: radial_hidden needs 1..4 widths");
    if (precision != MLP_FP32 && precision != MLP_BF16 && precision != MLP_BF16_FAST &&
        precision != MLP_BF16_NODE && precision != MLP_BF16_NODE_X3)
        return fail(MLP_ERR_INVALID_ARG, "unknown precision");
    auto in = [](long v, long lo, long hi) { return v >= lo && v <= hi; };
    if (!in(S, 1, 64) || !in(NB, 1, 16) || !in(p, 1, 8) || !in(lmax, 0, 8) || !in(K, 1, 1024) || !in(corr, 1, 8) ||
        !in(RH, 1, 1024))
        return fail(MLP_ERR_INVALID_ARG, "mace: header value out of range");
    McDims d;
    d.S = (int)S;
    d.NB = (int)NB;
    d.p = (int)p;
    d.lmax = (int)lmax;
    d.K = (int)K;
    d.corr = (int)corr;
    d.nrad = (int)rh.size();
    for (size_t q = 0; q < rh.size(); q++) {
        if (!in(rh[q], 1, 4096)) return fail(MLP_ERR_INVALID_ARG, "mace: radial width out of range");
        d.rh[q] = (int)rh[q];
    }
    d.RH = (int)RH;
    d.rc = (float)rc;
    d.navg = (float)navg;
    mlp_model *m = new mlp_model();
    m->F = 0;
    m->K = 0;
    m->T = 2;
    m->S = (int)S;
    m->rc = (float)rc;
    m->eps = 0.f;
    m->precision = precision;
    m->n_weights = n_weights;
    if (int rc2 = mace_create(m, d, weights, n_weights)) {
        delete m;
        return rc2;
    }
    *out = m;
    return MLP_OK;
}

extern "C" {

const char *mlp_last_error(void) { return last_error_cstr(); }

int mlp_model_create(const char *header_json, const float *weights, size_t n_weights, int precision,
                     mlp_model **out) {
    if (!header_json || !weights || !out) return fail(MLP_ERR_INVALID_ARG, "null argument");
    *out = nullptr;
    JsonTop j = parse_top(header_json);
    if (!j.ok) return fail(MLP_ERR_INVALID_ARG, "model header is not a JSON object");
    {
        auto it = j.kv.find("model");
        if (it != j.kv.end() && it->second == "allegro") return create_allegro(j, weights, n_weights, precision, out);
        if (it != j.kv.end() && it->second == "mace") return create_mace(j, weights, n_weights, precision, out);
    }
    long F, K, T, S;
    double rc, eps;
    if (!get_int(j, "F", &F) || !get_int(j, "K", &K) || !get_int(j, "T", &T) || !get_int(j, "n_species", &S) ||
        !get_num(j, "r_c", &rc) || !get_num(j, "eps", &eps))
        return fail(MLP_ERR_INVALID_ARG, "model header lacks F, K, T, n_species, r_c or eps");
    auto str = [&](const char *k) { auto it = j.kv.find(k); return it == j.kv.end() ? std::string() : it->second; };
    if (str("model") != "painn") return fail(MLP_ERR_INVALID_ARG, "model must be \"painn\"");
    if (str("basis") != "bessel_sin_over_r") return fail(MLP_ERR_INVALID_ARG, "basis must be bessel_sin_over_r");
    if (str("envelope") != "cosine") return fail(MLP_ERR_INVALID_ARG, "envelope must be cosine");
    if (!(F == 16 || F == 32 || F == 64 || F == 128)) return fail(MLP_ERR_INVALID_ARG, "F must be 16, 32, 64 or 128");
    if (K < 1 || K > MLP_MAX_K || T < 1 || T > MLP_MAX_LAYERS || S < 1)
        return fail(MLP_ERR_INVALID_ARG, "K, T or n_species out of range");
    {
        static const int ok[][2] = {{128, 20}, {32, 8}, {64, 20}, {128, 8}, {32, 20}, {64, 8}, {16, 6}};
        bool found = false;
        for (auto &p : ok) found |= (p[0] == F && p[1] == K);
        if (!found) return fail(MLP_ERR_INVALID_ARG, "(F, K) combination is not compiled in this build");
    }
    if (!(rc > 0.0) || !(eps > 0.0)) return fail(MLP_ERR_INVALID_ARG, "r_c and eps must be positive");
    if (precision != MLP_FP32 && precision != MLP_BF16 && precision != MLP_BF16_FAST &&
        precision != MLP_BF16_NODE && precision != MLP_BF16_NODE_X3)
        return fail(MLP_ERR_INVALID_ARG, "unknown precision");
    mlp_model *m = new mlp_model();
    m->F = (int)F; m->K = (int)K; m->T = (int)T; m->S = (int)S;
    m->rc = (float)rc; m->eps = (float)eps; m->precision = precision;
    size_t off = 0;
    m->off_emb = off; off += (size_t)S * F;
    const size_t sizes[12] = {(size_t)F * F, (size_t)F, 3 * (size_t)F * F, 3 * (size_t)F, 3 * (size_t)F * K,
                              3 * (size_t)F, (size_t)F * F, (size_t)F * F, 2 * (size_t)F * F, (size_t)F,
                              3 * (size_t)F * F, 3 * (size_t)F};
    for (int t = 0; t < T; t++)
        for (int b = 0; b < 12; b++) {
            m->off_layer[t][b] = off;
            off += sizes[b];
        }
    m->off_W5 = off; off += (size_t)(F / 2) * F;
    m->off_b5 = off; off += F / 2;
    m->off_w6 = off; off += F / 2;
    m->off_b6 = off; off += 1;
    if (off != n_weights) {
        delete m;
        return fail(MLP_ERR_INVALID_ARG, "weight count " + std::to_string(n_weights) + " does not match the header (" +
                                             std::to_string(off) + ")");
    }
    m->n_weights = off;
    if (hipMalloc(&m->w_dev, sizeof(float) * off) != hipSuccess) {
        (void)hipGetLastError();
        delete m;
        return fail(MLP_ERR_OOM, "weight allocation failed");
    }
    if (hipMemcpy(m->w_dev, weights, sizeof(float) * off, hipMemcpyHostToDevice) != hipSuccess) {
        hipFree(m->w_dev);
        delete m;
        return fail(MLP_ERR_DEVICE, "weight copy failed");
    }
    // the weight matrices of the node GEMMs, packed once as B operands
    struct Item {
        const float *W;
        int R, C;
        bool tr;
        mlp::PackedW *dst;
        bool parts3 = false;
    };
    std::vector<Item> items;
    const int Fi = (int)F;
    for (int t = 0; t < (int)T; t++) {
        const mlp::LayerW L = m->layer(t);
        // U and V are adjacent ([U; V] is one 2F x F row-major matrix)
        const float *Wm[5] = {L.W1, L.W2, L.U, L.W3, L.W4};
        const int R[5] = {Fi, 3 * Fi, 2 * Fi, Fi, 3 * Fi}, C[5] = {Fi, Fi, Fi, 2 * Fi, Fi};
        for (int q = 0; q < 5; q++) {
            items.push_back({Wm[q], R[q], C[q], false, &m->pk[t][q]});
            items.push_back({Wm[q], R[q], C[q], true, &m->pk[t][5 + q]});
        }
        if (Fi == 64 || Fi == 128) items.push_back({L.W4, 3 * Fi, Fi, true, &m->pk[t][mlp::WP_W4TP], true});
    }
    items.push_back({m->at(m->off_W5), Fi / 2, Fi, false, &m->pk_W5});
    items.push_back({m->at(m->off_W5), Fi / 2, Fi, true, &m->pk_W5t});
    size_t pk_bytes = 0;
    for (const Item &it : items) pk_bytes += mlp::packed_bytes(it.R, it.C, it.tr);
    int prc = hipMalloc(&m->pk_dev, pk_bytes) == hipSuccess ? 0 : MLP_ERR_OOM;
    for (size_t q = 0, o = 0; prc == 0 && q < items.size(); q++) {
        const Item &it = items[q];
        if (mlp::pack_weight(nullptr, it.W, it.R, it.C, it.tr, (char *)m->pk_dev + o, it.dst, it.parts3))
            prc = MLP_ERR_DEVICE;
        o += mlp::packed_bytes(it.R, it.C, it.tr);
    }
    // first-layer phi per species, followed by the scratch of its two GEMMs
    float *tab = nullptr;
    if (prc == 0 && hipMalloc(&tab, sizeof(float) * 5 * (size_t)S * F) != hipSuccess) prc = MLP_ERR_OOM;
    if (prc == 0) {
        m->phi0_dev = tab;
        prc = mlp::first_layer_table(m, nullptr, tab + 3 * (size_t)S * F);
    }
    if (prc == 0 && hipDeviceSynchronize() != hipSuccess) prc = MLP_ERR_DEVICE;
    // the factorised first layer's species-scaled filter weights (up to four species)
    if (prc == 0) prc = mlp::first_layer_factor(m);
    if (prc) {
        (void)hipGetLastError();
        if (tab) hipFree(tab);
        if (m->pk_l0_dev) hipFree(m->pk_l0_dev);
        if (m->pk_dev) hipFree(m->pk_dev);
        hipFree(m->w_dev);
        delete m;
        return fail(prc, "weight packing failed");
    }
    *out = m;
    return MLP_OK;
}

int mlp_model_destroy(mlp_model *m) {
    if (!m) return MLP_OK;
    allegro_destroy(m);
    mace_destroy(m);
    if (m->w_dev) hipFree(m->w_dev);
    if (m->wb_dev) hipFree(m->wb_dev);
    if (m->pk_dev) hipFree(m->pk_dev);
    if (m->phi0_dev) hipFree(m->phi0_dev);
    if (m->pk_l0_dev) hipFree(m->pk_l0_dev);
    delete m;
    return MLP_OK;
}

int mlp_build_neighbors(mlp_model *m, const float *pos, const int32_t *species, int32_t n_atoms, int32_t n_local,
                        const double box[3], float skin, void *stream, mlp_nbr **inout) {
    if (!m || !pos || !species || !box || !inout) return fail(MLP_ERR_INVALID_ARG, "null argument");
    mlp_nbr *g = *inout;
    bool created = false;
    if (!g) {
        g = new mlp_nbr();
        created = true;
    }
    int rc = build_graph(m, g, pos, species, n_atoms, n_local, box, skin, (hipStream_t)stream);
    if (rc) {
        if (created) {
            mlp_nbr_destroy(g);
        }
        return rc;
    }
    *inout = g;
    return MLP_OK;
}

static void release_all(mlp_nbr *g) {
    if (g->h_flag) {
        hipHostFree(g->h_flag);
        g->h_flag = nullptr;
    }
    DevBuf *bufs[] = {&g->perm, &g->iperm, &g->cell_of, &g->cell_start, &g->cell_cnt, &g->cell_fill, &g->tmp_idx,
                      &g->pos_build, &g->species, &g->row, &g->col, &g->rev, &g->rowc, &g->colc, &g->revc,
                      &g->geom, &g->map, &g->oldidx, &g->cnt, &g->hop, &g->pos4, &g->scan_tmp, &g->flags,
                      &g->red, &g->ghost_ptr, &g->ghost_list, &g->ghost_cnt, &g->act, &g->G, &g->Gs, &g->Fint, &g->Uatom};
    for (DevBuf *b : bufs) b->release();
}

static int64_t held_bytes(mlp_nbr *g) {
    DevBuf *bufs[] = {&g->perm, &g->iperm, &g->cell_of, &g->cell_start, &g->cell_cnt, &g->cell_fill, &g->tmp_idx,
                      &g->pos_build, &g->species, &g->row, &g->col, &g->rev, &g->rowc, &g->colc, &g->revc,
                      &g->geom, &g->map, &g->oldidx, &g->cnt, &g->hop, &g->pos4, &g->scan_tmp, &g->flags,
                      &g->red, &g->ghost_ptr, &g->ghost_list, &g->ghost_cnt, &g->act, &g->G, &g->Gs, &g->Fint, &g->Uatom};
    int64_t t = 0;
    for (DevBuf *b : bufs) t += (int64_t)b->bytes;
    return t;
}

int mlp_nbr_destroy(mlp_nbr *g) {
    if (!g) return MLP_OK;
    release_all(g);
    delete g;
    return MLP_OK;
}

int mlp_energy_forces(mlp_model *m, mlp_nbr *g, const float *pos, int32_t n_atoms, int32_t n_local,
                      const int32_t *ghost_owner, void *stream, double *energy, float *forces, float *atom_energy,
                      mlp_stats *stats) {
    if (!m || !g || !pos || !energy) return fail(MLP_ERR_INVALID_ARG, "null argument");
    if (g->n_builds == 0) return fail(MLP_ERR_INVALID_ARG, "neighbour handle was never built");
    if (n_atoms != g->n_atoms || n_local != g->n_local)
        return fail(MLP_ERR_INVALID_ARG, "atom counts differ from the last neighbour build");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    const bool fold = forces && ghost_owner && n_atoms > n_local;
    // the owner map is validated before anything is computed
    if (fold && (rc = prepare_owner_map(g, ghost_owner, s))) return rc;
    if ((rc = prune_graph(m, g, pos, s))) return rc;
    if ((rc = compute_hops(m, g, s))) return rc;
    if ((rc = evaluate(m, g, s, energy, forces, atom_energy))) return rc;
    if (fold && (rc = fold_ghosts(g, forces, s))) return rc;
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        int hist[MLP_MAX_LAYERS + 2] = {0};
        int64_t ehist[MLP_MAX_LAYERS + 2] = {0};
        if ((rc = hop_histogram(m, g, s, hist, ehist))) return rc;
        int Ec = 0;
        if (hipMemcpyAsync(&Ec, g->rowc.as<int>() + g->n_atoms, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess)
            return fail(MLP_ERR_DEVICE, "statistics readback failed");
        stats->n_edges_skin = g->n_edges_skin;
        stats->n_edges = Ec;
        stats->n_atoms = g->n_atoms;
        stats->n_local = g->n_local;
        int run = 0;
        int64_t erun = 0;
        for (int t = 0; t <= m->T && t < 8; t++) {
            run += hist[t];
            erun += ehist[t];
            stats->n_within_hops[t] = run;
            stats->n_edges_within_hops[t] = erun;
        }
        for (int d = 0; d < 3; d++) stats->n_cells[d] = g->nc[d];
        stats->max_cell_occupancy = g->max_occ;
        stats->n_builds = g->n_builds;
        stats->n_grows = g->n_grows;
        stats->device_bytes = held_bytes(g);
    }
    return MLP_OK;
}

int mlp_nbr_check_displacement(mlp_nbr *g, const float *pos, int32_t n_atoms, void *stream, int32_t *exceeds) {
    if (!g || !pos || !exceeds) return fail(MLP_ERR_INVALID_ARG, "null argument");
    if (g->n_builds == 0) return fail(MLP_ERR_INVALID_ARG, "neighbour handle was never built");
    if (n_atoms != g->n_atoms) return fail(MLP_ERR_INVALID_ARG, "atom count differs from the last neighbour build");
    bool ex = false;
    int rc = max_displacement_exceeds(g, pos, 0.5f * g->skin, (hipStream_t)stream, &ex);
    if (rc) return rc;
    *exceeds = ex ? 1 : 0;
    return MLP_OK;
}

int mlp_md_step(mlp_model *m, mlp_nbr *g, float *pos, float *vel, float *forces, const float *inv_mass,
                const int32_t *species, int32_t n, const double box[3], float skin, float dt, void *stream,
                double *energy, int32_t *rebuilt) {
    if (!m || !g || !pos || !vel || !forces || !inv_mass || !species || !box || !energy)
        return fail(MLP_ERR_INVALID_ARG, "null argument");
    if (g->n_builds == 0 || g->n_atoms != n || g->n_local != n)
        return fail(MLP_ERR_INVALID_ARG, "MD step needs a periodic system built on this handle");
    hipStream_t s = (hipStream_t)stream;
    int rc;
    if ((rc = verlet_kick_drift(pos, vel, forces, inv_mass, n, box, dt, s))) return rc;
    bool exceeds = false;
    if ((rc = max_displacement_exceeds(g, pos, 0.5f * g->skin, s, &exceeds))) return rc;
    if (rebuilt) *rebuilt = exceeds ? 1 : 0;
    if (exceeds) {
        mlp_nbr *gg = g;
        if ((rc = mlp_build_neighbors(m, pos, species, n, n, box, skin, stream, &gg))) return rc;
    }
    if ((rc = mlp_energy_forces(m, g, pos, n, n, nullptr, stream, energy, forces, nullptr, nullptr))) return rc;
    return verlet_kick(vel, forces, inv_mass, n, dt, s);
}

int mlp_nbr_edges(mlp_nbr *g, int32_t which, int32_t *dst, int32_t *src, int64_t cap, int64_t *n_edges,
                  void *stream) {
    if (!g || !n_edges || (which != 0 && which != 1)) return fail(MLP_ERR_INVALID_ARG, "bad argument");
    if (g->n_builds == 0) return fail(MLP_ERR_INVALID_ARG, "neighbour handle was never built");
    hipStream_t s = (hipStream_t)stream;
    const int *row = which ? g->rowc.as<int>() : g->row.as<int>();
    const int *col = which ? g->colc.as<int>() : g->col.as<int>();
    if (which && !row) return fail(MLP_ERR_INVALID_ARG, "no evaluation has pruned this graph yet");
    int E = 0;
    if (hipMemcpyAsync(&E, row + g->n_atoms, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(MLP_ERR_DEVICE, "edge count readback failed");
    *n_edges = E;
    if (E > cap) return fail(MLP_ERR_CAPACITY, "edge arrays too small");
    if (!dst || !src) return fail(MLP_ERR_INVALID_ARG, "null edge arrays");
    int rc = export_edges(g, row, col, dst, src, s);
    if (rc) return rc;
    if (hipStreamSynchronize(s) != hipSuccess) return fail(MLP_ERR_DEVICE, "edge export failed");
    return MLP_OK;
}

}  // extern "C"
