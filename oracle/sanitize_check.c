/*
 * sanitize_check.c -- TEST INFRASTRUCTURE ONLY: a driver of the oracle for
 * sanitizer builds (AddressSanitizer + UndefinedBehaviorSanitizer). It
 * compiles psc_oracle.c into the same program and runs every entry point
 * the tests use on a 3D Poisson 7-point grid: hierarchies with each
 * aggregation, prolongator and smoother setting, the V-cycles, PCG, FCG in
 * all its forms (FP64 / FP32 V-cycle, learned, l1-Jacobi alternate), the
 * network's forward, loss gradient, Adam step and apply.
 *
 *   sanitize_check <n>
 */
#include "psc_oracle.c"

#include <stdio.h>

static void poisson(int n, int **rp, int **ci, double **v) {
    int N = n * n * n, k = 0;
    *rp = malloc(sizeof(int) * (size_t)(N + 1));
    *ci = malloc(sizeof(int) * (size_t)N * 7);
    *v = malloc(sizeof(double) * (size_t)N * 7);
    (*rp)[0] = 0;
    for (int i = 0; i < N; i++) {
        int x = i % n, y = (i / n) % n, z = i / (n * n);
        int nb[7] = {z > 0 ? i - n * n : -1, y > 0 ? i - n : -1, x > 0 ? i - 1 : -1, i,
                     x + 1 < n ? i + 1 : -1, y + 1 < n ? i + n : -1, z + 1 < n ? i + n * n : -1};
        for (int q = 0; q < 7; q++) {
            if (nb[q] < 0) continue;
            (*ci)[k] = nb[q];
            (*v)[k] = nb[q] == i ? 6.0 : -1.0;
            k++;
        }
        (*rp)[i + 1] = k;
    }
}

int main(int argc, char **argv) {
    int n = argc > 1 ? atoi(argv[1]) : 12;
    int N = n * n * n;
    int *rp, *ci;
    double *v;
    poisson(n, &rp, &ci, &v);
    double *b = malloc(sizeof(double) * N), *x = malloc(sizeof(double) * N), *z = malloc(sizeof(double) * N);
    for (int i = 0; i < N; i++) b[i] = sin(0.37 * i) + 0.5;
    /* settings: sweeps, prol, nu, nu_double, aggr, smoother, coarse_pcg */
    int cfg[][7] = {{2, 0, 1, 0, 0, 0, 0}, {3, 1, 4, 0, 0, 0, 0}, {3, 0, 2, 1, 0, 0, 40}, {2, 1, 4, 0, 1, 0, 0},
                    {2, 0, 1, 0, 0, 1, 0}, {2, 0, 1, 0, 0, 2, 0}, {2, 0, 2, 0, 0, 3, 0}};
    int ncfg = (int)(sizeof(cfg) / sizeof(cfg[0]));
    int np = orc_net_param_count();
    double *params = malloc(sizeof(double) * np);
    for (int i = 0; i < np; i++) params[i] = 0.1 * sin(1.3 * i);
    for (int c = 0; c < ncfg; c++) {
        orc_hier *h = NULL;
        int st = orc_build(N, rp, ci, v, cfg[c][0], 20, 30, 30, cfg[c][1], cfg[c][2], cfg[c][3], cfg[c][4], 0.01,
                           cfg[c][5], 0.1, 0, 1, cfg[c][6], 1e-4, &h);
        if (st != ORC_OK) { fprintf(stderr, "build %d failed: %d\n", c, st); return 1; }
        orc_vcycle(h, b, z);
        orc_vcycle32(h, b, z);
        int it, fb, ne;
        double rr;
        for (int i = 0; i < N; i++) x[i] = 0.0;
        st = orc_pcg(h, ORC_PREC_VCYCLE, b, x, 1e-6, 200, &it, &rr, NULL);
        printf("config %d: %d levels, PCG %d its (status %d)\n", c, orc_nlevels(h), it, st);
        for (int form = 0; form < 2; form++) {
            for (int i = 0; i < N; i++) x[i] = 0.0;
            orc_fcg(h, form, NULL, 0, 0, 0, b, x, 1e-6, 200, &it, &rr, &fb, &ne);
            for (int i = 0; i < N; i++) x[i] = 0.0;
            orc_fcg(h, form, params, n, n, n, b, x, 1e-6, 200, &it, &rr, &fb, &ne);
            for (int i = 0; i < N; i++) x[i] = 0.0;
            orc_fcg(h, form | ORC_ALT_JACOBI, NULL, 0, 0, 0, b, x, 1e-6, 200, &it, &rr, &fb, &ne);
        }
        orc_free(h);
    }
    /* network: a batch of two 6^3 crops */
    int D = 6, B = 2, cells = B * D * D * D;
    double *in = malloc(sizeof(double) * cells), *tg = malloc(sizeof(double) * cells);
    double *out = malloc(sizeof(double) * cells), *g = malloc(sizeof(double) * np);
    double *m = calloc(np, sizeof(double)), *vv = calloc(np, sizeof(double));
    for (int i = 0; i < cells; i++) { in[i] = cos(0.11 * i); tg[i] = 0.3 * in[i]; }
    orc_net_forward(params, 1, B, D, D, D, in, out, NULL);
    double loss = orc_net_loss_grad(params, 1, B, D, D, D, in, tg, 1, g);
    orc_adam_step(np, params, m, vv, g, 1, 1e-3, 0.9, 0.999, 1e-8);
    orc_net_apply(params, n, n, n, b, z);
    printf("net loss %.6e\nsanitize check ok\n", loss);
    free(in); free(tg); free(out); free(g); free(m); free(vv); free(params);
    free(b); free(x); free(z); free(rp); free(ci); free(v);
    return 0;
}
