/* Sanitizer driver for the FP64 oracle (test infrastructure only): builds
 * with the oracle source in the same translation unit and runs FP, BP, SART
 * (one and several projections per update) and the CSR build on small scans,
 * including a hollow grid, a one-sector grid and a posed object.  Exit status
 * 0 when every output is finite. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../oracle/cyl_oracle.c"

static void circular(double *v, int n, double sod, double sdd, double p) {
    for (int k = 0; k < n; ++k) {
        double phi = 6.283185307179586 * k / n, c = cos(phi), s = sin(phi);
        double *w = v + 12 * k;
        w[0] = -sod * c; w[1] = -sod * s; w[2] = 0.0;
        w[3] = (sdd - sod) * c; w[4] = (sdd - sod) * s; w[5] = 0.0;
        w[6] = -p * s; w[7] = p * c; w[8] = 0.0;
        w[9] = 0.0; w[10] = 0.0; w[11] = p;
    }
}

static int finite_all(const double *x, int64_t n) {
    for (int64_t i = 0; i < n; ++i)
        if (!isfinite(x[i])) return 0;
    return 1;
}

static int run(orc_grid g, int posed) {
    double views[12 * 5];
    circular(views, 5, 40.0, 80.0, 1.1);
    orc_scan s;
    s.g = g;
    s.n_views = 5;
    s.det_rows = 7;
    s.det_cols = 9;
    s.views = views;
    for (int i = 0; i < 9; ++i) s.R[i] = (i % 4 == 0) ? 1.0 : 0.0;
    s.T[0] = s.T[1] = s.T[2] = 0.0;
    if (posed) {
        double a = 0.3, c = cos(a), sn = sin(a);
        double R[9] = {c, 0.0, sn, 0.0, 1.0, 0.0, -sn, 0.0, c};
        for (int i = 0; i < 9; ++i) s.R[i] = R[i];
        s.T[0] = 0.4; s.T[1] = -0.3; s.T[2] = 0.2;
    }
    const int64_t V = (int64_t)g.n_h * g.n_theta * g.n_r, P = (int64_t)s.n_views * s.det_rows * s.det_cols;
    double *x = malloc(sizeof(double) * V), *q = malloc(sizeof(double) * P), *L = malloc(sizeof(double) * P);
    double *b = malloc(sizeof(double) * V), *n = malloc(sizeof(double) * V), *w = malloc(sizeof(double) * V);
    double *r = malloc(sizeof(double) * P);
    for (int64_t i = 0; i < V; ++i) {
        x[i] = 0.01 * (double)((i * 7919) % 101);
        w[i] = 0.5 + 0.5 * (double)(i % 2);
    }
    orc_fp(&s, x, 0, s.n_views, q, L, 2);
    orc_bp(&s, q, 0, s.n_views, b, n, 2);
    int ok = finite_all(q, P) && finite_all(L, P) && finite_all(b, V) && finite_all(n, V);
    for (int subset = 1; subset <= 3; subset += 2) {
        orc_sart_params prm = {2, 0.5, 1, NULL, 0, 0, subset};
        for (int64_t i = 0; i < V; ++i) b[i] = 0.9 * x[i];
        ok = ok && orc_sart(&s, &prm, q, NULL, w, b, r, 2) == 0 && finite_all(b, V);
    }
    int64_t nnz = orc_build_csr(&s, 0, 1, NULL, NULL, NULL);
    int64_t *ip = malloc(sizeof(int64_t) * (s.det_rows * s.det_cols + 1));
    int64_t *cells = malloc(sizeof(int64_t) * (nnz > 0 ? nnz : 1));
    double *lens = malloc(sizeof(double) * (nnz > 0 ? nnz : 1));
    ok = ok && orc_build_csr(&s, 0, 1, ip, cells, lens) == nnz && finite_all(lens, nnz);
    free(x); free(q); free(L); free(b); free(n); free(w); free(r); free(ip); free(cells); free(lens);
    return ok;
}

int main(void) {
    orc_grid grids[3] = {{4, 8, 4, 1.5, 6.0, -2.0, 4.0, 0.3}, {3, 1, 3, 0.0, 6.0, -3.0, 3.0, 0.0},
                         {7, 37, 19, 0.0, 6.0, -3.0, 3.0, 0.0}};
    for (int i = 0; i < 3; ++i)
        for (int posed = 0; posed < 2; ++posed)
            if (!run(grids[i], posed)) {
                printf("non-finite output, grid %d posed %d\n", i, posed);
                return 1;
            }
    printf("oracle sanitizer run: ok\n");
    return 0;
}
