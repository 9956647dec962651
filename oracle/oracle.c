/*
 * FP64 CPU oracle for the PaiNN-form semi-local message-passing potential and
 * its forces.  TEST INFRASTRUCTURE ONLY: tests, the smoke check and the CPU
 * baseline leg of the benchmark may call it; the product path never does.
 * It shares no code with the GPU library.
 *
 * What it computes (plain definitions, step by step, in double precision):
 *   - the directed neighbour graph: every ordered pair (i <- j, image n) with
 *     0 < |r_j + n.L - r_i| < cutoff (Results, "Distributed potential
 *     computation": atoms share an edge if closer than the cutoff);
 *   - per-atom energies U_i of a T-layer PaiNN network evaluated on that graph
 *     (Methods, "Graph Neural Networks", message and update equations;
 *     "Chosen Architectures": PaiNN correlates pairs of neighbour features per
 *     layer).  The layer equations are the PaiNN paper's, which the paper
 *     cites but does not print; the reading used here is:
 *       phi_j = W2 silu(W1 s_j + b1) + b2                       (F -> 3F)
 *       w_ij  = (A e(r_ij) + c) * fc(r_ij),  e_k = sin(k pi r/rc)/r,
 *               fc = (cos(pi r/rc) + 1)/2 for r < rc             (K -> 3F)
 *       x_ij  = phi_j o w_ij = [x_vv | x_s | x_vs]
 *       s_i  += sum_j x_s ;  v_i += sum_j (v_j o x_vv + rhat_ij (x) x_vs)
 *       Uv = U v, Vv = V v (per Cartesian row), n = sqrt(sum_d Vv_d^2 + eps)
 *       a = W4 silu(W3 [s; n] + b3) + b4 = [a_vv | a_sv | a_ss]
 *       v += a_vv o Uv ;  s += a_sv o <Uv, Vv> + a_ss
 *     readout U_i = w6 . silu(W5 s_i + b5) + b6 after layer T;
 *   - the energy E = sum of U_i over local atoms (Eq. 1) and the forces
 *     F_k = -dE/dr_k on every atom, local and ghost (Eq. 2: the partial
 *     forces of the local energy with respect to all atoms of the domain).
 *     The derivative is taken by a hand-written reverse pass; the edge
 *     gradient G_e = dE/d(r_j - r_i) enters F as
 *     F_k = sum_{e into k} G_e - sum_{e out of k} G_e.
 *
 * Pins (tests/): brute-force neighbour sets; central finite differences;
 * zero net force; rotation / reflection / translation / permutation
 * invariance; periodic replication; isolated atoms (node-only recursion); an
 * embedded-atom special case evaluated by a textbook EAM loop; the collinear
 * dimer closed form; ghost-shell domain == periodic system.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXL 16

typedef struct {
    const double *W1, *b1, *W2, *b2, *A, *c, *U, *V, *W3, *b3, *W4, *b4;
} layer_t;

typedef struct {
    int F, K, T, S;
    double rc, eps;
    const double *emb;
    layer_t L[MAXL];
    const double *W5, *b5, *w6, *b6;
} model_t;

/* Parameter order: emb, then per layer W1 b1 W2 b2 A c U V W3 b3 W4 b4, then
 * W5 b5 w6 b6.  Matrices are [out][in] row-major.  Returns the count used. */
static int64_t parse_model(model_t *m, const int32_t *dims, const double *rc_eps, const double *w)
{
    int64_t off = 0;
    int F = dims[0], K = dims[1], T = dims[2], S = dims[3];
    m->F = F; m->K = K; m->T = T; m->S = S;
    m->rc = rc_eps[0]; m->eps = rc_eps[1];
#define TAKE(ptr, cnt) do { (ptr) = w + off; off += (int64_t)(cnt); } while (0)
    TAKE(m->emb, (int64_t)S * F);
    for (int t = 0; t < T; t++) {
        layer_t *l = &m->L[t];
        TAKE(l->W1, F * F); TAKE(l->b1, F);
        TAKE(l->W2, 3 * F * F); TAKE(l->b2, 3 * F);
        TAKE(l->A, 3 * F * K); TAKE(l->c, 3 * F);
        TAKE(l->U, F * F); TAKE(l->V, F * F);
        TAKE(l->W3, F * 2 * F); TAKE(l->b3, F);
        TAKE(l->W4, 3 * F * F); TAKE(l->b4, 3 * F);
    }
    TAKE(m->W5, (F / 2) * F); TAKE(m->b5, F / 2); TAKE(m->w6, F / 2); TAKE(m->b6, 1);
#undef TAKE
    return off;
}

int64_t orc_model_size(const int32_t *dims)
{
    int64_t F = dims[0], K = dims[1], T = dims[2], S = dims[3];
    int64_t per = F * F + F + 3 * F * F + 3 * F + 3 * F * K + 3 * F + 2 * F * F + 2 * F * F + F + 3 * F * F + 3 * F;
    return S * F + T * per + (F / 2) * F + F / 2 + F / 2 + 1;
}

static double silu(double x) { return x / (1.0 + exp(-x)); }
static double dsilu(double x)
{
    double sg = 1.0 / (1.0 + exp(-x));
    return sg * (1.0 + x * (1.0 - sg));
}

/* y = W x + b, W [nout][nin] */
static void matvec(const double *W, const double *b, const double *x, int nout, int nin, double *y)
{
    for (int o = 0; o < nout; o++) {
        double acc = b ? b[o] : 0.0;
        for (int k = 0; k < nin; k++) acc += W[(int64_t)o * nin + k] * x[k];
        y[o] = acc;
    }
}

/* xbar += W^T ybar */
static void matTvec_acc(const double *W, const double *ybar, int nout, int nin, double *xbar)
{
    for (int o = 0; o < nout; o++) {
        double g = ybar[o];
        if (g == 0.0) continue;
        for (int k = 0; k < nin; k++) xbar[k] += W[(int64_t)o * nin + k] * g;
    }
}

/* ------------------------------------------------------------------------ */
/* Neighbour graph, FP64, brute force over periodic images.                 */
/* ------------------------------------------------------------------------ */

/* Image shift range for dimension d. */
static int image_range(const double *box, double cut, int d)
{
    if (box[d] <= 0.0) return 0;
    return (int)ceil(cut / box[d]) + 1;
}

static int min_image_ok(const double *box, double cut)
{
    for (int d = 0; d < 3; d++)
        if (box[d] > 0.0 && !(cut < 0.5 * box[d])) return 0;
    return 1;
}

/* Visit all edges of row i in (j, image) lexicographic order.  When every
 * periodic length exceeds twice the cutoff at most one image of j can lie
 * within the cutoff, namely the nearest one, and only it is examined. */
static int64_t row_edges(const double *pos, int n, const double *box, double cut, int i,
                         int32_t *src, double *dvec)
{
    double cut2 = cut * cut;
    int64_t cnt = 0;
    int mi = min_image_ok(box, cut);
    int m[3];
    for (int d = 0; d < 3; d++) m[d] = mi ? 0 : image_range(box, cut, d);
    for (int j = 0; j < n; j++) {
        double base[3];
        for (int d = 0; d < 3; d++) {
            base[d] = pos[3 * j + d] - pos[3 * i + d];
            if (mi && box[d] > 0.0) base[d] -= box[d] * nearbyint(base[d] / box[d]);
        }
        for (int a = -m[0]; a <= m[0]; a++)
            for (int b = -m[1]; b <= m[1]; b++)
                for (int c = -m[2]; c <= m[2]; c++) {
                    double dv[3] = {base[0] + a * box[0], base[1] + b * box[1], base[2] + c * box[2]};
                    double r2 = dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2];
                    if (r2 >= cut2 || r2 == 0.0) continue;
                    if (j == i && a == 0 && b == 0 && c == 0) continue;
                    if (src) {
                        src[cnt] = j;
                        dvec[3 * cnt + 0] = dv[0];
                        dvec[3 * cnt + 1] = dv[1];
                        dvec[3 * cnt + 2] = dv[2];
                    }
                    cnt++;
                }
    }
    return cnt;
}

/* Directed edges (dst i <- src j) with 0 < |d| < cut, d = r_j + n.L - r_i.
 * Sorted by dst, then src, then image.  Returns E; arrays filled when cap >= E. */
int64_t orc_neighbors(const double *pos, int n, const double *box, double cut, int64_t cap,
                      int32_t *dst, int32_t *src, double *dvec)
{
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 16)
    for (int i = 0; i < n; i++) cnt[i + 1] = row_edges(pos, n, box, cut, i, NULL, NULL);
    for (int i = 0; i < n; i++) cnt[i + 1] += cnt[i];
    int64_t E = cnt[n];
    if (cap >= E && dst) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < n; i++) {
            int64_t o = cnt[i];
            int64_t k = row_edges(pos, n, box, cut, i, src + o, dvec + 3 * o);
            for (int64_t e = 0; e < k; e++) dst[o + e] = i;
        }
    }
    free(cnt);
    return E;
}

/* Single-precision pair decision, used only where a float comparison decides
 * an integer result (which pairs are neighbours), so that the oracle takes
 * that decision in the same precision and by the same formula as the device:
 *   dx = x_j - x_i; dx -= L if dx > L/2; dx += L if dx < -L/2 (periodic dims)
 *   r2 = fma(dz, dz, fma(dy, dy, dx * dx));   keep iff r2 < cut*cut (float)
 * with cut = rc + skin in float.  Positions must lie in [0, L). */
int64_t orc_neighbors_f32(const float *pos, int n, const float *box, float rc, float skin,
                          int64_t cap, int32_t *dst, int32_t *src)
{
    volatile float cutv = rc + skin;
    float cut = cutv;
    volatile float c2v = cut * cut;
    float cut2 = c2v;
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int pass = 0; pass < 2; pass++) {
#pragma omp parallel for schedule(dynamic, 16)
        for (int i = 0; i < n; i++) {
            int64_t c = 0, o = pass ? cnt[i] : 0;
            for (int j = 0; j < n; j++) {
                if (j == i) continue;
                float d[3];
                for (int k = 0; k < 3; k++) {
                    volatile float dk = pos[3 * j + k] - pos[3 * i + k];
                    float L = box[k];
                    if (L > 0.0f) {
                        float h = 0.5f * L;
                        if (dk > h) dk = dk - L;
                        else if (dk < -h) dk = dk + L;
                    }
                    d[k] = dk;
                }
                float r2 = fmaf(d[2], d[2], fmaf(d[1], d[1], d[0] * d[0]));
                if (r2 < cut2) {
                    if (pass) { dst[o + c] = i; src[o + c] = j; }
                    c++;
                }
            }
            if (!pass) cnt[i + 1] = c;
        }
        if (!pass) {
            for (int i = 0; i < n; i++) cnt[i + 1] += cnt[i];
            if (cap < cnt[n] || !dst) break;
        }
    }
    int64_t E = cnt[n];
    free(cnt);
    return E;
}

/* Hop distance from the local atoms over a directed edge list, capped at
 * T + 1: the set an atom belongs to after T rounds of pseudo-messages sent
 * from the local atoms, each receiver sending in the next round (Results,
 * "Distributed potential computation", pruning). */
void orc_hops(int n, int n_local, int64_t E, const int32_t *dst, const int32_t *src, int T, int8_t *hop)
{
    for (int i = 0; i < n; i++) hop[i] = (int8_t)(i < n_local ? 0 : T + 1);
    for (int t = 1; t <= T; t++) {
        for (int64_t e = 0; e < E; e++) {
            int i = dst[e], j = src[e];
            /* a message travels from an atom that has one (hop <= t-1) to its neighbour */
            if (hop[i] == t - 1 && hop[j] > t) hop[j] = (int8_t)t;
            if (hop[j] == t - 1 && hop[i] > t) hop[i] = (int8_t)t;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Energy and forces                                                        */
/* ------------------------------------------------------------------------ */

typedef struct {
    double r, rhat[3];
    double fc, dfc;
} geom_t;

static void edge_geom(const double *d, double rc, geom_t *g)
{
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    g->r = r;
    for (int k = 0; k < 3; k++) g->rhat[k] = d[k] / r;
    if (r < rc) {
        g->fc = 0.5 * (cos(M_PI * r / rc) + 1.0);
        g->dfc = -0.5 * (M_PI / rc) * sin(M_PI * r / rc);
    } else {
        g->fc = 0.0;
        g->dfc = 0.0;
    }
}

/* Filter w(r) (3F) and, when dw != NULL, its derivative dw/dr. */
static void filter(const model_t *m, const layer_t *l, const geom_t *g, double *w, double *dw)
{
    int F3 = 3 * m->F, K = m->K;
    double e[64], de[64];
    for (int k = 1; k <= K; k++) {
        double a = k * M_PI / m->rc;
        e[k - 1] = sin(a * g->r) / g->r;
        de[k - 1] = a * cos(a * g->r) / g->r - sin(a * g->r) / (g->r * g->r);
    }
    for (int f = 0; f < F3; f++) {
        double lin = l->c[f], dlin = 0.0;
        for (int k = 0; k < K; k++) {
            lin += l->A[(int64_t)f * K + k] * e[k];
            dlin += l->A[(int64_t)f * K + k] * de[k];
        }
        w[f] = lin * g->fc;
        if (dw) dw[f] = dlin * g->fc + lin * g->dfc;
    }
}

typedef struct {
    /* layer inputs */
    double *s, *v;
    /* intermediates */
    double *h1, *phi, *s1, *v1, *Uv, *Vv, *nrm, *h3, *a;
} lstate_t;

double orc_energy_forces(const int32_t *dims, const double *rc_eps, const double *W, int64_t nW,
                         const double *pos, const int32_t *Z, int n, int n_local, const double *box,
                         double *forces, double *atom_energy, int64_t *n_edges_out)
{
    model_t m;
    if (dims[2] > MAXL || dims[1] > 64) return NAN;
    if (parse_model(&m, dims, rc_eps, W) != nW) return NAN;
    const int F = m.F, F3 = 3 * F, T = m.T, Fh = F / 2;

    /* graph */
    int64_t E = orc_neighbors(pos, n, box, m.rc, 0, NULL, NULL, NULL);
    int32_t *dst = (int32_t *)malloc(sizeof(int32_t) * (E + 1));
    int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (E + 1));
    double *dvec = (double *)malloc(sizeof(double) * 3 * (E + 1));
    orc_neighbors(pos, n, box, m.rc, E, dst, src, dvec);
    if (n_edges_out) *n_edges_out = E;
    int64_t *rowp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t e = 0; e < E; e++) rowp[dst[e] + 1]++;
    for (int i = 0; i < n; i++) rowp[i + 1] += rowp[i];
    /* edges grouped by source */
    int64_t *srcp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int64_t *bysrc = (int64_t *)malloc(sizeof(int64_t) * (E + 1));
    for (int64_t e = 0; e < E; e++) srcp[src[e] + 1]++;
    for (int i = 0; i < n; i++) srcp[i + 1] += srcp[i];
    {
        int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
        memcpy(fill, srcp, sizeof(int64_t) * (n + 1));
        for (int64_t e = 0; e < E; e++) bysrc[fill[src[e]]++] = e;
        free(fill);
    }
    geom_t *geo = (geom_t *)malloc(sizeof(geom_t) * (E + 1));
#pragma omp parallel for
    for (int64_t e = 0; e < E; e++) edge_geom(dvec + 3 * e, m.rc, &geo[e]);

    /* per-layer storage */
    lstate_t *st = (lstate_t *)calloc(T + 1, sizeof(lstate_t));
    for (int t = 0; t <= T; t++) {
        st[t].s = (double *)calloc((size_t)n * F, sizeof(double));
        st[t].v = (double *)calloc((size_t)n * F3, sizeof(double));
        if (t == T) break;
        st[t].h1 = (double *)malloc(sizeof(double) * n * F);
        st[t].phi = (double *)malloc(sizeof(double) * n * F3);
        st[t].s1 = (double *)malloc(sizeof(double) * n * F);
        st[t].v1 = (double *)malloc(sizeof(double) * n * F3);
        st[t].Uv = (double *)malloc(sizeof(double) * n * F3);
        st[t].Vv = (double *)malloc(sizeof(double) * n * F3);
        st[t].nrm = (double *)malloc(sizeof(double) * n * F);
        st[t].h3 = (double *)malloc(sizeof(double) * n * F);
        st[t].a = (double *)malloc(sizeof(double) * n * F3);
    }

    /* embedding: s0 = emb[Z], v0 = 0 */
    for (int i = 0; i < n; i++)
        for (int f = 0; f < F; f++) st[0].s[(int64_t)i * F + f] = m.emb[(int64_t)Z[i] * F + f];

    /* ---------------- forward ---------------- */
    for (int t = 0; t < T; t++) {
        const layer_t *l = &m.L[t];
        lstate_t *S = &st[t];
#pragma omp parallel
        {
            double *tmp = (double *)malloc(sizeof(double) * 2 * F);
#pragma omp for
            for (int i = 0; i < n; i++) {
                double *h1 = S->h1 + (int64_t)i * F;
                matvec(l->W1, l->b1, S->s + (int64_t)i * F, F, F, h1);
                for (int f = 0; f < F; f++) tmp[f] = silu(h1[f]);
                matvec(l->W2, l->b2, tmp, F3, F, S->phi + (int64_t)i * F3);
            }
            free(tmp);
        }
        /* messages, gathered per destination atom */
#pragma omp parallel
        {
            double *w = (double *)malloc(sizeof(double) * F3);
#pragma omp for schedule(dynamic, 16)
            for (int i = 0; i < n; i++) {
                double *s1 = S->s1 + (int64_t)i * F, *v1 = S->v1 + (int64_t)i * F3;
                for (int f = 0; f < F; f++) s1[f] = S->s[(int64_t)i * F + f];
                for (int f = 0; f < F3; f++) v1[f] = S->v[(int64_t)i * F3 + f];
                for (int64_t e = rowp[i]; e < rowp[i + 1]; e++) {
                    int j = src[e];
                    const geom_t *g = &geo[e];
                    filter(&m, l, g, w, NULL);
                    const double *phj = S->phi + (int64_t)j * F3, *vj = S->v + (int64_t)j * F3;
                    for (int f = 0; f < F; f++) {
                        double xvv = phj[f] * w[f];
                        double xs = phj[F + f] * w[F + f];
                        double xvs = phj[2 * F + f] * w[2 * F + f];
                        s1[f] += xs;
                        for (int d = 0; d < 3; d++)
                            v1[d * F + f] += vj[d * F + f] * xvv + g->rhat[d] * xvs;
                    }
                }
            }
            free(w);
        }
        /* update block */
#pragma omp parallel
        {
            double *sn = (double *)malloc(sizeof(double) * 2 * F);
            double *a3 = (double *)malloc(sizeof(double) * F);
#pragma omp for
            for (int i = 0; i < n; i++) {
                const double *s1 = S->s1 + (int64_t)i * F, *v1 = S->v1 + (int64_t)i * F3;
                double *Uv = S->Uv + (int64_t)i * F3, *Vv = S->Vv + (int64_t)i * F3;
                double *nrm = S->nrm + (int64_t)i * F, *h3 = S->h3 + (int64_t)i * F, *a = S->a + (int64_t)i * F3;
                for (int d = 0; d < 3; d++) {
                    matvec(l->U, NULL, v1 + d * F, F, F, Uv + d * F);
                    matvec(l->V, NULL, v1 + d * F, F, F, Vv + d * F);
                }
                for (int f = 0; f < F; f++) {
                    double q = m.eps;
                    for (int d = 0; d < 3; d++) q += Vv[d * F + f] * Vv[d * F + f];
                    nrm[f] = sqrt(q);
                    sn[f] = s1[f];
                    sn[F + f] = nrm[f];
                }
                matvec(l->W3, l->b3, sn, F, 2 * F, h3);
                for (int f = 0; f < F; f++) a3[f] = silu(h3[f]);
                matvec(l->W4, l->b4, a3, F3, F, a);
                double *so = st[t + 1].s + (int64_t)i * F, *vo = st[t + 1].v + (int64_t)i * F3;
                for (int f = 0; f < F; f++) {
                    double sp = 0.0;
                    for (int d = 0; d < 3; d++) {
                        sp += Uv[d * F + f] * Vv[d * F + f];
                        vo[d * F + f] = v1[d * F + f] + a[f] * Uv[d * F + f];
                    }
                    so[f] = s1[f] + a[F + f] * sp + a[2 * F + f];
                }
            }
            free(sn);
            free(a3);
        }
    }

    /* readout and energy (Eq. 1: sum over local atoms) */
    double *gs = (double *)calloc((size_t)n * F, sizeof(double));
    double *gv = (double *)calloc((size_t)n * F3, sizeof(double));
    double *Ui = (double *)malloc(sizeof(double) * n);
#pragma omp parallel
    {
        double *h5 = (double *)malloc(sizeof(double) * Fh);
        double *g5 = (double *)malloc(sizeof(double) * Fh);
#pragma omp for
        for (int i = 0; i < n; i++) {
            matvec(m.W5, m.b5, st[T].s + (int64_t)i * F, Fh, F, h5);
            double u = m.b6[0];
            for (int k = 0; k < Fh; k++) u += m.w6[k] * silu(h5[k]);
            Ui[i] = u;
            if (i < n_local) {
                for (int k = 0; k < Fh; k++) g5[k] = m.w6[k] * dsilu(h5[k]);
                matTvec_acc(m.W5, g5, Fh, F, gs + (int64_t)i * F);
            }
        }
        free(h5);
        free(g5);
    }
    double E_tot = 0.0;
    for (int i = 0; i < n_local; i++) E_tot += Ui[i];
    if (atom_energy) memcpy(atom_energy, Ui, sizeof(double) * n);

    /* ---------------- reverse pass ---------------- */
    double *G = (double *)calloc((size_t)3 * (E + 1), sizeof(double));
    double *gs1 = (double *)malloc(sizeof(double) * n * F);
    double *gv1 = (double *)malloc(sizeof(double) * n * F3);
    double *gphi = (double *)malloc(sizeof(double) * n * F3);
    for (int t = T - 1; t >= 0; t--) {
        const layer_t *l = &m.L[t];
        lstate_t *S = &st[t];
        /* update block: (gs, gv) are gradients w.r.t. the layer output */
#pragma omp parallel
        {
            double *ga = (double *)malloc(sizeof(double) * F3);
            double *ga3 = (double *)malloc(sizeof(double) * F);
            double *gsn = (double *)malloc(sizeof(double) * 2 * F);
            double *gUv = (double *)malloc(sizeof(double) * F3);
            double *gVv = (double *)malloc(sizeof(double) * F3);
#pragma omp for
            for (int i = 0; i < n; i++) {
                const double *Uv = S->Uv + (int64_t)i * F3, *Vv = S->Vv + (int64_t)i * F3;
                const double *a = S->a + (int64_t)i * F3, *h3 = S->h3 + (int64_t)i * F;
                const double *nrm = S->nrm + (int64_t)i * F;
                const double *g_s = gs + (int64_t)i * F, *g_v = gv + (int64_t)i * F3;
                for (int f = 0; f < F; f++) {
                    double sp = 0.0, gavv = 0.0;
                    for (int d = 0; d < 3; d++) {
                        sp += Uv[d * F + f] * Vv[d * F + f];
                        gavv += g_v[d * F + f] * Uv[d * F + f];
                    }
                    ga[f] = gavv;
                    ga[F + f] = g_s[f] * sp;
                    ga[2 * F + f] = g_s[f];
                    for (int d = 0; d < 3; d++) {
                        gUv[d * F + f] = g_v[d * F + f] * a[f] + g_s[f] * a[F + f] * Vv[d * F + f];
                        gVv[d * F + f] = g_s[f] * a[F + f] * Uv[d * F + f];
                    }
                }
                for (int f = 0; f < F; f++) ga3[f] = 0.0;
                matTvec_acc(l->W4, ga, F3, F, ga3);
                for (int f = 0; f < F; f++) ga3[f] *= dsilu(h3[f]);
                for (int f = 0; f < 2 * F; f++) gsn[f] = 0.0;
                matTvec_acc(l->W3, ga3, F, 2 * F, gsn);
                for (int f = 0; f < F; f++)
                    for (int d = 0; d < 3; d++) gVv[d * F + f] += gsn[F + f] * Vv[d * F + f] / nrm[f];
                double *o_s = gs1 + (int64_t)i * F, *o_v = gv1 + (int64_t)i * F3;
                for (int f = 0; f < F; f++) o_s[f] = g_s[f] + gsn[f];
                for (int q = 0; q < F3; q++) o_v[q] = g_v[q];
                for (int d = 0; d < 3; d++) {
                    matTvec_acc(l->U, gUv + d * F, F, F, o_v + d * F);
                    matTvec_acc(l->V, gVv + d * F, F, F, o_v + d * F);
                }
            }
            free(ga); free(ga3); free(gsn); free(gUv); free(gVv);
        }
        /* message block, organised by source atom j (its out-edges i <- j) */
#pragma omp parallel
        {
            double *w = (double *)malloc(sizeof(double) * F3);
            double *dw = (double *)malloc(sizeof(double) * F3);
#pragma omp for schedule(dynamic, 16)
            for (int j = 0; j < n; j++) {
                const double *phj = S->phi + (int64_t)j * F3, *vj = S->v + (int64_t)j * F3;
                double *gpj = gphi + (int64_t)j * F3;
                double *gvj = gv + (int64_t)j * F3;      /* residual part already equals gv1 below */
                for (int q = 0; q < F3; q++) gpj[q] = 0.0;
                for (int q = 0; q < F3; q++) gvj[q] = gv1[(int64_t)j * F3 + q];
                for (int64_t p = srcp[j]; p < srcp[j + 1]; p++) {
                    int64_t e = bysrc[p];
                    int i = dst[e];
                    const geom_t *g = &geo[e];
                    filter(&m, l, g, w, dw);
                    const double *gsi = gs1 + (int64_t)i * F, *gvi = gv1 + (int64_t)i * F3;
                    double gr = 0.0, grh[3] = {0.0, 0.0, 0.0};
                    for (int f = 0; f < F; f++) {
                        double gxs = gsi[f];
                        double gxvv = 0.0, gxvs = 0.0;
                        for (int d = 0; d < 3; d++) {
                            gxvv += gvi[d * F + f] * vj[d * F + f];
                            gxvs += gvi[d * F + f] * g->rhat[d];
                        }
                        double xvv = phj[f] * w[f];
                        double xvs = phj[2 * F + f] * w[2 * F + f];
                        for (int d = 0; d < 3; d++) {
                            gvj[d * F + f] += gvi[d * F + f] * xvv;
                            grh[d] += gvi[d * F + f] * xvs;
                        }
                        gpj[f] += gxvv * w[f];
                        gpj[F + f] += gxs * w[F + f];
                        gpj[2 * F + f] += gxvs * w[2 * F + f];
                        gr += gxvv * phj[f] * dw[f] + gxs * phj[F + f] * dw[F + f] + gxvs * phj[2 * F + f] * dw[2 * F + f];
                    }
                    double rd = grh[0] * g->rhat[0] + grh[1] * g->rhat[1] + grh[2] * g->rhat[2];
                    for (int d = 0; d < 3; d++)
                        G[3 * e + d] += gr * g->rhat[d] + (grh[d] - rd * g->rhat[d]) / g->r;
                }
            }
            free(w); free(dw);
        }
        /* message-function MLP, and the residual into the layer input */
#pragma omp parallel
        {
            double *ga1 = (double *)malloc(sizeof(double) * F);
#pragma omp for
            for (int j = 0; j < n; j++) {
                const double *h1 = S->h1 + (int64_t)j * F;
                for (int f = 0; f < F; f++) ga1[f] = 0.0;
                matTvec_acc(l->W2, gphi + (int64_t)j * F3, F3, F, ga1);
                for (int f = 0; f < F; f++) ga1[f] *= dsilu(h1[f]);
                double *o = gs + (int64_t)j * F;
                for (int f = 0; f < F; f++) o[f] = gs1[(int64_t)j * F + f];
                matTvec_acc(l->W1, ga1, F, F, o);
            }
            free(ga1);
        }
    }

    /* forces: F_k = sum_{e into k} G_e - sum_{e out of k} G_e */
    if (forces) {
#pragma omp parallel for
        for (int k = 0; k < n; k++) {
            double f[3] = {0.0, 0.0, 0.0};
            for (int64_t e = rowp[k]; e < rowp[k + 1]; e++)
                for (int d = 0; d < 3; d++) f[d] += G[3 * e + d];
            for (int64_t p = srcp[k]; p < srcp[k + 1]; p++)
                for (int d = 0; d < 3; d++) f[d] -= G[3 * bysrc[p] + d];
            for (int d = 0; d < 3; d++) forces[3 * k + d] = f[d];
        }
    }

    for (int t = 0; t <= T; t++) {
        free(st[t].s); free(st[t].v);
        if (t == T) break;
        free(st[t].h1); free(st[t].phi); free(st[t].s1); free(st[t].v1); free(st[t].Uv);
        free(st[t].Vv); free(st[t].nrm); free(st[t].h3); free(st[t].a);
    }
    free(st); free(gs); free(gv); free(Ui); free(G); free(gs1); free(gv1); free(gphi);
    free(dst); free(src); free(dvec); free(rowp); free(srcp); free(bysrc); free(geo);
    return E_tot;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
