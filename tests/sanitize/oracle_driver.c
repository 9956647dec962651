/* Driver of the FP64 oracle (oracle/oracle.c) for the AddressSanitizer /
 * UndefinedBehaviorSanitizer build made by tests/test_sanitizers.py.  It runs
 * every exported routine on small seeded systems: a periodic box smaller than
 * twice the cutoff (several images per pair), an open domain, an isolated
 * atom, a single atom, and an empty-capacity neighbour query.  Inputs are
 * random numbers only; any out-of-bounds access or undefined behaviour
 * aborts, and non-finite results or a non-zero net force fail. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t orc_model_size(const int32_t *dims);
int64_t orc_neighbors(const double *pos, int n, const double *box, double cut, int64_t cap, int32_t *dst,
                      int32_t *src, double *dvec);
int64_t orc_neighbors_f32(const float *pos, int n, const float *box, float rc, float skin, int64_t cap,
                          int32_t *dst, int32_t *src);
void orc_hops(int n, int n_local, int64_t E, const int32_t *dst, const int32_t *src, int T, int8_t *hop);
double orc_energy_forces(const int32_t *dims, const double *rc_eps, const double *W, int64_t nW, const double *pos,
                         const int32_t *Z, int n, int n_local, const double *box, double *forces,
                         double *atom_energy, int64_t *n_edges_out);

static uint64_t st = 12345;
static double urand(void) { /* xorshift64*, uniform in [0, 1) */
    st ^= st >> 12; st ^= st << 25; st ^= st >> 27;
    return (double)((st * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}
static double nrand(void) { return sqrt(-2.0 * log(1.0 - urand())) * cos(6.283185307179586 * urand()); }

static int run_case(const char *name, int n, int n_local, const double box[3], double extent, int F, int K, int T,
                    int S) {
    int32_t dims[4] = {F, K, T, S};
    double rc_eps[2] = {5.0, 1e-8};
    int64_t nW = orc_model_size(dims);
    double *W = malloc(sizeof(double) * (size_t)nW);
    for (int64_t q = 0; q < nW; q++) W[q] = 0.15 * nrand();
    double *pos = malloc(sizeof(double) * 3 * (size_t)n);
    float *posf = malloc(sizeof(float) * 3 * (size_t)n);
    int32_t *Z = malloc(sizeof(int32_t) * (size_t)n);
    for (int i = 0; i < n; i++) {
        for (int d = 0; d < 3; d++) {
            double L = box[d] > 0 ? box[d] : extent;
            pos[3 * i + d] = (double)(float)(urand() * L);
            posf[3 * i + d] = (float)pos[3 * i + d];
        }
        Z[i] = (int32_t)(urand() * S);
    }
    double *Fo = calloc(3 * (size_t)n, sizeof(double)), *U = calloc((size_t)n, sizeof(double));
    int64_t E = -1;
    double e = orc_energy_forces(dims, rc_eps, W, nW, pos, Z, n, n_local, box, Fo, U, &E);
    int bad = !isfinite(e);
    double net[3] = {0, 0, 0}, fmax = 0;
    for (int i = 0; i < n; i++)
        for (int d = 0; d < 3; d++) {
            bad |= !isfinite(Fo[3 * i + d]);
            net[d] += Fo[3 * i + d];
            fmax = fmax > fabs(Fo[3 * i + d]) ? fmax : fabs(Fo[3 * i + d]);
        }
    for (int d = 0; d < 3; d++) bad |= fabs(net[d]) > 1e-9 * (1.0 + fmax) * n;
    /* neighbour routines: count, then fill; a zero-capacity call only counts */
    int64_t En = orc_neighbors(pos, n, box, 5.5, 0, NULL, NULL, NULL);
    int32_t *dst = malloc(sizeof(int32_t) * (size_t)(En + 1)), *src = malloc(sizeof(int32_t) * (size_t)(En + 1));
    double *dv = malloc(sizeof(double) * 3 * (size_t)(En + 1));
    bad |= orc_neighbors(pos, n, box, 5.5, En, dst, src, dv) != En;
    int8_t *hop = malloc((size_t)n);
    orc_hops(n, n_local, En, dst, src, T, hop);
    for (int i = 0; i < n; i++) bad |= hop[i] < 0 || hop[i] > T + 1;
    float boxf[3] = {(float)box[0], (float)box[1], (float)box[2]};
    int single_image = 1;
    for (int d = 0; d < 3; d++) single_image &= box[d] == 0 || 5.5 < 0.5 * box[d];
    if (single_image) {
        int64_t Ef = orc_neighbors_f32(posf, n, boxf, 5.0f, 0.5f, 0, NULL, NULL);
        int32_t *d2 = malloc(sizeof(int32_t) * (size_t)(Ef + 1)), *s2 = malloc(sizeof(int32_t) * (size_t)(Ef + 1));
        bad |= orc_neighbors_f32(posf, n, boxf, 5.0f, 0.5f, Ef, d2, s2) != Ef;
        free(d2);
        free(s2);
    }
    printf("%-28s n=%4d local=%4d edges(rc)=%6lld E=%.6e net=(%.1e %.1e %.1e) %s\n", name, n, n_local,
           (long long)E, e, net[0], net[1], net[2], bad ? "BAD" : "ok");
    free(W); free(pos); free(posf); free(Z); free(Fo); free(U); free(dst); free(src); free(dv); free(hop);
    return bad;
}

int main(void) {
    int bad = 0;
    const double small[3] = {7.3, 8.1, 9.4};     /* below 2 rc: several images per pair */
    const double cube[3] = {12.42, 12.42, 12.42};
    const double open_[3] = {0, 0, 0};
    const double slab[3] = {12.0, 12.0, 0};
    bad |= run_case("periodic multi-image", 24, 24, small, 0, 16, 6, 2, 2);
    bad |= run_case("periodic water-size box", 96, 96, cube, 0, 32, 8, 2, 2);
    bad |= run_case("open domain with ghosts", 80, 30, open_, 14.0, 16, 6, 3, 1);
    bad |= run_case("slab (one open dimension)", 60, 60, slab, 30.0, 16, 6, 2, 3);
    bad |= run_case("isolated atoms", 3, 3, open_, 400.0, 16, 6, 2, 1);
    bad |= run_case("single atom", 1, 1, open_, 1.0, 16, 6, 1, 1);
    return bad;
}
