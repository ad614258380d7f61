/*
 * FP64 CPU oracle for the cylindrical-grid cone-beam projectors and SART.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the package smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code with the HIP path.
 *
 * What it computes (paper, Sec. 2 and 2.2):
 *   - pose:           X' = R X + T                                  (Eq. 1)
 *   - cell membership: r = sqrt(x'^2+y'^2), theta = atan2(y',x'), h = z'
 *                                                                    (Eq. 2)
 *   - system matrix:  t_jl = length of ray j (source -> pixel centre)
 *                     inside ring-sector cell l                      (Eq. 6)
 *   - SART:           per ordered subset (one projection, or several;
 *                     all of them is SIRT), mu_m += lam * w_m *
 *                     sum_j t_jm * wp_j (p_j - sum_l t_jl mu_l) / sum_l t_jl
 *                     / sum_j t_jm, j over the rays of the subset    (Eq. 7)
 *                     with the voxel weight map w_m of the weighted back-
 *                     projection (Sec. 2.2, last paragraph).
 *
 * Method for t_jl (plain definition, no traversal): for each ray collect every
 * parameter t in (0,1) at which it meets a cell boundary -- both roots of each
 * shell quadric, the crossing with each full plane through the axis holding a
 * sector edge, each axial plane -- sort them, and give each sub-interval to the
 * cell containing its midpoint (classified with Eq. 2).  Each open
 * sub-interval then lies in exactly one cell, including the second piece of a
 * ray that re-enters a non-convex ring sector.
 *
 * Conventions: grid r_i = r_min + i dr, h_m = h_min + m dh,
 * theta_b = theta0 + b dtheta, dtheta = 2 pi / N_theta; cells are half-open
 * [lower, upper); volumes are (N_h, N_theta, N_r) C order; pixel (v, u) of a
 * view has centre D + (u - (W-1)/2) U + (v - (H-1)/2) V; projections are
 * (views, rows, cols).  Zero denominators in Eq. 7 (sum_l t_jl = 0 or
 * sum_j t_jm = 0) contribute nothing.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t n_h, n_theta, n_r;
    double r_min, r_max, h_min, h_max, theta0;
} orc_grid;

typedef struct {
    orc_grid g;
    int32_t n_views, det_rows, det_cols;
    const double *views; /* n_views x 12, stage frame */
    double R[9], T[3];
} orc_scan;

/* ---------------------------------------------------------------- geometry */

/* Eq. 1: stage -> object frame. */
static void to_object(const orc_scan *s, const double X[3], double out[3]) {
    for (int i = 0; i < 3; ++i)
        out[i] = s->R[3 * i] * X[0] + s->R[3 * i + 1] * X[1] + s->R[3 * i + 2] * X[2] + s->T[i];
}

/* Source and pixel centre of ray (k, v, u), in the object frame. */
static void ray_ends(const orc_scan *s, int k, int v, int u, double a[3], double e[3]) {
    const double *w = s->views + 12 * (size_t)k;
    double du = u - 0.5 * (s->det_cols - 1), dv = v - 0.5 * (s->det_rows - 1);
    double E[3];
    for (int i = 0; i < 3; ++i) E[i] = w[3 + i] + du * w[6 + i] + dv * w[9 + i];
    to_object(s, w, a);
    to_object(s, E, e);
}

/* Eq. 2 classification of a point; returns the flat cell index or -1. */
static int64_t classify(const orc_grid *g, const double X[3]) {
    double r = hypot(X[0], X[1]);
    double dr = (g->r_max - g->r_min) / g->n_r;
    double dh = (g->h_max - g->h_min) / g->n_h;
    double fr = floor((r - g->r_min) / dr);
    double fh = floor((X[2] - g->h_min) / dh);
    if (fr < 0 || fr >= g->n_r || fh < 0 || fh >= g->n_h) return -1;
    int64_t it = 0;
    if (g->n_theta > 1) {
        double two_pi = 2.0 * M_PI;
        double th = fmod(atan2(X[1], X[0]) - g->theta0, two_pi);
        if (th < 0) th += two_pi;
        it = (int64_t)floor(th / (two_pi / g->n_theta));
        if (it >= g->n_theta) it = 0;
        if (it < 0) it = 0;
    }
    return ((int64_t)fh * g->n_theta + it) * g->n_r + (int64_t)fr;
}

static int cmp_double(const void *x, const void *y) {
    double a = *(const double *)x, b = *(const double *)y;
    return (a > b) - (a < b);
}

/* Upper bound on the number of candidate parameters of one ray. */
static int max_candidates(const orc_grid *g) {
    return 2 + 2 * (g->n_r + 1) + g->n_theta + (g->n_h + 1);
}

/*
 * All (cell, length) pieces of one ray, in order along the ray.  `cand` is
 * scratch of max_candidates() doubles.  Returns the number of pieces written
 * (a cell can appear twice for a re-entering ray).
 */
static int ray_pieces(const orc_grid *g, const double a[3], const double e[3],
                      double *cand, int64_t *cells, double *lens) {
    double d[3] = {e[0] - a[0], e[1] - a[1], e[2] - a[2]};
    double len = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    int nc = 0;
    cand[nc++] = 0.0;
    cand[nc++] = 1.0;
    /* shells: A t^2 + 2 B t + (C - r^2) = 0, stable root pair */
    double A = d[0] * d[0] + d[1] * d[1];
    double B = a[0] * d[0] + a[1] * d[1];
    double C = a[0] * a[0] + a[1] * a[1];
    double dr = (g->r_max - g->r_min) / g->n_r;
    if (A > 0.0) {
        for (int i = 0; i <= g->n_r; ++i) {
            double ri = g->r_min + i * dr;
            if (ri <= 0.0) continue;
            double c0 = C - ri * ri;
            double disc = B * B - A * c0;
            if (disc <= 0.0) continue;
            double q = -(B + copysign(sqrt(disc), B));
            double t1 = q / A;
            if (t1 > 0.0 && t1 < 1.0) cand[nc++] = t1;
            if (q != 0.0) {
                double t2 = c0 / q;
                if (t2 > 0.0 && t2 < 1.0) cand[nc++] = t2;
            }
        }
    }
    /* sector edges: full planes through the axis, normal m_b = (-sin, cos, 0) */
    if (g->n_theta > 1) {
        double dth = 2.0 * M_PI / g->n_theta;
        for (int b = 0; b < g->n_theta; ++b) {
            double th = g->theta0 + b * dth;
            double mx = -sin(th), my = cos(th);
            double den = mx * d[0] + my * d[1];
            if (den == 0.0) continue;
            double t = -(mx * a[0] + my * a[1]) / den;
            if (t > 0.0 && t < 1.0) cand[nc++] = t;
        }
    }
    /* axial planes */
    if (d[2] != 0.0) {
        double dh = (g->h_max - g->h_min) / g->n_h;
        for (int m = 0; m <= g->n_h; ++m) {
            double t = (g->h_min + m * dh - a[2]) / d[2];
            if (t > 0.0 && t < 1.0) cand[nc++] = t;
        }
    }
    qsort(cand, nc, sizeof(double), cmp_double);
    int np = 0;
    for (int i = 0; i + 1 < nc; ++i) {
        double t0 = cand[i], t1 = cand[i + 1];
        if (!(t1 > t0)) continue;
        double tm = 0.5 * (t0 + t1);
        double X[3] = {a[0] + tm * d[0], a[1] + tm * d[1], a[2] + tm * d[2]};
        int64_t l = classify(g, X);
        if (l < 0) continue;
        cells[np] = l;
        lens[np] = (t1 - t0) * len;
        ++np;
    }
    return np;
}

/* ------------------------------------------------------------ public: rays */

int orc_max_pieces(const orc_grid *g) { return max_candidates(g); }

/* Pieces of one ray given by its object-frame end points. */
int orc_ray_pieces(const orc_grid *g, const double a[3], const double e[3],
                   int64_t *cells, double *lens) {
    double *cand = (double *)malloc(sizeof(double) * max_candidates(g));
    int n = ray_pieces(g, a, e, cand, cells, lens);
    free(cand);
    return n;
}

/* Object-frame end points of ray (k, v, u). */
void orc_ray_ends(const orc_scan *s, int k, int v, int u, double a[3], double e[3]) {
    ray_ends(s, k, v, u, a, e);
}

/* ------------------------------------------------------- threaded workers */

typedef struct {
    const orc_scan *s;
    int view_begin, view_end;
    int64_t ray_lo, ray_hi; /* global ray index range, ray = (k - view_begin) * H*W + v*W + u */
    const double *x;        /* FP input volume, or NULL */
    double *q;              /* FP output rays (indexed from view_begin) */
    double *rowsum;         /* sum_l t_jl per ray, or NULL */
    const double *y;        /* BP input per ray, or NULL */
    double *bp;             /* private BP accumulator (V), or NULL */
    double *colsum;         /* private column sums (V), or NULL */
    const int64_t *sample;  /* optional explicit ray list */
} work_t;

static void *worker(void *arg) {
    work_t *w = (work_t *)arg;
    const orc_scan *s = w->s;
    int maxc = max_candidates(&s->g);
    double *cand = (double *)malloc(sizeof(double) * maxc);
    int64_t *cells = (int64_t *)malloc(sizeof(int64_t) * maxc);
    double *lens = (double *)malloc(sizeof(double) * maxc);
    int64_t per_view = (int64_t)s->det_rows * s->det_cols;
    for (int64_t jj = w->ray_lo; jj < w->ray_hi; ++jj) {
        int64_t j = w->sample ? w->sample[jj] : jj;
        int k = w->view_begin + (int)(j / per_view);
        int64_t pix = j % per_view;
        int v = (int)(pix / s->det_cols), u = (int)(pix % s->det_cols);
        double a[3], e[3];
        ray_ends(s, k, v, u, a, e);
        int np = ray_pieces(&s->g, a, e, cand, cells, lens);
        if (w->x) {
            double acc = 0.0;
            for (int i = 0; i < np; ++i) acc += lens[i] * w->x[cells[i]];
            w->q[jj] = acc;
        }
        if (w->rowsum) {
            double acc = 0.0;
            for (int i = 0; i < np; ++i) acc += lens[i];
            w->rowsum[jj] = acc;
        }
        if (w->bp) {
            double yj = w->y[j];
            if (yj != 0.0)
                for (int i = 0; i < np; ++i) w->bp[cells[i]] += lens[i] * yj;
        }
        if (w->colsum)
            for (int i = 0; i < np; ++i) w->colsum[cells[i]] += lens[i];
    }
    free(cand);
    free(cells);
    free(lens);
    return NULL;
}

static void run_threads(work_t *ws, int nthreads) {
    if (nthreads <= 1) {
        worker(&ws[0]);
        return;
    }
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * nthreads);
    for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], NULL, worker, &ws[t]);
    for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
    free(th);
}

static void split(work_t *ws, int nthreads, int64_t n) {
    for (int t = 0; t < nthreads; ++t) {
        ws[t].ray_lo = n * t / nthreads;
        ws[t].ray_hi = n * (t + 1) / nthreads;
    }
}

/* ---------------------------------------------------- public: projectors */

/* q[ray] = sum_l t_jl x_l for every ray of views [vb, ve); rowsum optional. */
void orc_fp(const orc_scan *s, const double *x, int vb, int ve, double *q, double *rowsum,
            int nthreads) {
    if (nthreads < 1) nthreads = 1;
    int64_t n = (int64_t)(ve - vb) * s->det_rows * s->det_cols;
    work_t *ws = (work_t *)calloc(nthreads, sizeof(work_t));
    for (int t = 0; t < nthreads; ++t) {
        ws[t].s = s; ws[t].view_begin = vb; ws[t].view_end = ve;
        ws[t].x = x; ws[t].q = q; ws[t].rowsum = rowsum;
    }
    split(ws, nthreads, n);
    run_threads(ws, nthreads);
    free(ws);
}

/* FP of an explicit list of rays (indices relative to view vb). */
void orc_fp_rays(const orc_scan *s, const double *x, int vb, const int64_t *rays, int64_t n,
                 double *q, double *rowsum, int nthreads) {
    if (nthreads < 1) nthreads = 1;
    work_t *ws = (work_t *)calloc(nthreads, sizeof(work_t));
    for (int t = 0; t < nthreads; ++t) {
        ws[t].s = s; ws[t].view_begin = vb; ws[t].view_end = s->n_views;
        ws[t].x = x; ws[t].q = q; ws[t].rowsum = rowsum; ws[t].sample = rays;
    }
    split(ws, nthreads, n);
    run_threads(ws, nthreads);
    free(ws);
}

/*
 * out_l = sum_j t_jl y_j over the rays of views [vb, ve) (y indexed from vb);
 * colsum_l = sum_j t_jl optional.  Each thread accumulates into a private
 * volume; the private volumes are added in thread order, so the result is
 * deterministic for a given thread count.
 */
void orc_bp(const orc_scan *s, const double *y, int vb, int ve, double *out, double *colsum,
            int nthreads) {
    if (nthreads < 1) nthreads = 1;
    int64_t V = (int64_t)s->g.n_h * s->g.n_theta * s->g.n_r;
    int64_t n = (int64_t)(ve - vb) * s->det_rows * s->det_cols;
    work_t *ws = (work_t *)calloc(nthreads, sizeof(work_t));
    for (int t = 0; t < nthreads; ++t) {
        ws[t].s = s; ws[t].view_begin = vb; ws[t].view_end = ve;
        ws[t].y = y;
        ws[t].bp = (double *)calloc(V, sizeof(double));
        ws[t].colsum = colsum ? (double *)calloc(V, sizeof(double)) : NULL;
    }
    split(ws, nthreads, n);
    run_threads(ws, nthreads);
    memset(out, 0, sizeof(double) * V);
    if (colsum) memset(colsum, 0, sizeof(double) * V);
    for (int t = 0; t < nthreads; ++t) {
        for (int64_t l = 0; l < V; ++l) out[l] += ws[t].bp[l];
        if (colsum)
            for (int64_t l = 0; l < V; ++l) colsum[l] += ws[t].colsum[l];
        free(ws[t].bp);
        free(ws[t].colsum);
    }
    free(ws);
}

/* ------------------------------------------------------------ public: SART */

typedef struct {
    int32_t n_iter;
    double lambda;
    int32_t nonneg;
    const int32_t *view_order; /* NULL = 0..n_views-1 */
    int32_t start_iter, start_view;
    int32_t subset; /* projections per ordered subset; <= 1: one (plain SART) */
} orc_sart_params;

/*
 * Weighted SART, Eq. 7, with ordered subsets of `subset` projections: the
 * view order is cut into consecutive groups of `subset` positions (the last
 * one may be shorter), and each group is one update step.  All views of a
 * group are projected from the same mu, their residuals rho_j are formed, and
 * c_m = sum_j t_jm rho_j and n_m = sum_j t_jm run over every ray of the group
 * before mu_m += lam w_m c_m / n_m.  subset = 1 is the paper's setting (one
 * projection per update); subset = n_views is SIRT.
 * vol: in = prior mu(0), out = result.  proj: (views, rows, cols) measured
 * line integrals.  pw: per-pixel weights or NULL (= 1).  vw: per-voxel
 * weights or NULL (= 1).  If resid_out is non-NULL it receives, per
 * iteration, sum_j (p_j - q_j)^2 over all views as seen during the sweep.
 * The resume point (start_iter, start_view) counts positions in view_order
 * and must fall on a group boundary.
 */
int orc_sart(const orc_scan *s, const orc_sart_params *P, const double *proj, const double *pw,
             const double *vw, double *vol, double *resid_out, int nthreads) {
    int64_t V = (int64_t)s->g.n_h * s->g.n_theta * s->g.n_r;
    int64_t per_view = (int64_t)s->det_rows * s->det_cols;
    int m = P->subset > 1 ? P->subset : 1;
    if (m > s->n_views) m = s->n_views;
    if (m < 1) m = 1;
    double *q = (double *)malloc(sizeof(double) * per_view);
    double *L = (double *)malloc(sizeof(double) * per_view);
    double *rho = (double *)malloc(sizeof(double) * per_view * m);
    double *c = (double *)malloc(sizeof(double) * V);
    double *nsum = (double *)malloc(sizeof(double) * V);
    double *ck = (double *)malloc(sizeof(double) * V);
    double *nk = (double *)malloc(sizeof(double) * V);
    if (!q || !L || !rho || !c || !nsum || !ck || !nk) return -2;
    for (int it = P->start_iter; it < P->n_iter; ++it) {
        double r2 = 0.0;
        int kv0 = (it == P->start_iter) ? P->start_view : 0;
        for (int g0 = kv0; g0 < s->n_views; g0 += m) {
            int cnt = s->n_views - g0 < m ? s->n_views - g0 : m;
            /* residuals of every view of the group, from the same mu */
            for (int i = 0; i < cnt; ++i) {
                int k = P->view_order ? P->view_order[g0 + i] : g0 + i;
                orc_fp(s, vol, k, k + 1, q, L, nthreads);
                const double *p = proj + per_view * (size_t)k;
                double *rk = rho + per_view * (size_t)i;
                for (int64_t j = 0; j < per_view; ++j) {
                    double res = p[j] - q[j];
                    r2 += res * res;
                    double w = pw ? pw[per_view * (size_t)k + j] : 1.0;
                    rk[j] = (L[j] > 0.0) ? w * res / L[j] : 0.0;
                }
            }
            /* column sums over all rays of the group */
            for (int i = 0; i < cnt; ++i) {
                int k = P->view_order ? P->view_order[g0 + i] : g0 + i;
                double *cc = i == 0 ? c : ck, *nn = i == 0 ? nsum : nk;
                orc_bp(s, rho + per_view * (size_t)i, k, k + 1, cc, nn, nthreads);
                if (i > 0)
                    for (int64_t l = 0; l < V; ++l) {
                        c[l] += ck[l];
                        nsum[l] += nk[l];
                    }
            }
            for (int64_t l = 0; l < V; ++l) {
                if (!(nsum[l] > 0.0)) continue;
                double w = vw ? vw[l] : 1.0;
                double nv = vol[l] + P->lambda * w * c[l] / nsum[l];
                if (P->nonneg && nv < 0.0) nv = 0.0;
                vol[l] = nv;
            }
        }
        if (resid_out) resid_out[it] = r2;
    }
    free(q); free(L); free(rho); free(c); free(nsum); free(ck); free(nk);
    return 0;
}

/* ------------------------------------------------- explicit sparse matrix */

/*
 * Rows of A for views [vb, ve) in CSR form, used by the small-size tests.
 * First call with cells == NULL to get the row pointer (indptr, n_rays + 1
 * entries); then call again with cells/lens of indptr[n_rays] entries.
 */
int64_t orc_build_csr(const orc_scan *s, int vb, int ve, int64_t *indptr, int64_t *cells,
                      double *lens) {
    int maxc = max_candidates(&s->g);
    double *cand = (double *)malloc(sizeof(double) * maxc);
    int64_t *cc = (int64_t *)malloc(sizeof(int64_t) * maxc);
    double *ll = (double *)malloc(sizeof(double) * maxc);
    int64_t per_view = (int64_t)s->det_rows * s->det_cols;
    int64_t n = (int64_t)(ve - vb) * per_view;
    int64_t pos = 0;
    if (indptr) indptr[0] = 0;
    for (int64_t j = 0; j < n; ++j) {
        int k = vb + (int)(j / per_view);
        int64_t pix = j % per_view;
        double a[3], e[3];
        ray_ends(s, k, (int)(pix / s->det_cols), (int)(pix % s->det_cols), a, e);
        int np = ray_pieces(&s->g, a, e, cand, cc, ll);
        if (cells) {
            memcpy(cells + pos, cc, sizeof(int64_t) * np);
            memcpy(lens + pos, ll, sizeof(double) * np);
        }
        pos += np;
        if (indptr) indptr[j + 1] = pos;
    }
    free(cand); free(cc); free(ll);
    return pos;
}
