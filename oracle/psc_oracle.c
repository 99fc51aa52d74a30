/*
 * psc_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, obviously-correct FP64 CPU implementation of the solve phase
 * of the paper's method: conjugate gradient preconditioned by an
 * aggregation-based algebraic multigrid V-cycle. Only tests, the smoke check
 * and the benchmark's CPU-baseline leg may load this file's library; the
 * product path never does. It shares no code with the HIP library.
 *
 * What each part follows:
 *   - AMG as a stationary iteration, Galerkin coarse operators
 *     A_{l+1} = P_l^T A_l P_l and the V-cycle error propagation with one
 *     pre- and one post-sweep: Section "AMG4PSBLAS", eq. (amg).
 *   - Coupled aggregation by compatible weighted matching, the tentative
 *     prolongator P^ = blockdiag(w_e) (+) diag(w_s/|w_s|) and k matching
 *     sweeps giving aggregates of size <= 2^k: Section "Aggregation
 *     strategies", eq. (prolongator); optionally the smoothed prolongator
 *     P = (I - omega D^-1 A) P^, omega = 1/||D^-1 A||_inf (same section).
 *   - l1-Jacobi smoother M_l = diag(A_l) + diag(sum_{j!=i} |a_ij|):
 *     Section "GPU enabled smoothers".
 *   - AINV and INVK smoothers, G_l = Z D^-1 Z^T ~ A_l^-1 with Z unit upper
 *     triangular (incomplete A-biconjugation with a drop tolerance; inverse
 *     of an incomplete LDL^T factor with levels of fill): same section.
 *   - A polynomial smoother (named as future work in the Conclusions): the
 *     fourth-kind Chebyshev smoother on the l1-Jacobi preconditioned operator.
 *   - Conjugate gradient / flexible CG to a relative residual tolerance:
 *     Section "Numerical Example".
 * Readings where the paper is silent (edge weights, tie order, weight
 * quantisation, the graph of the second sweep, coarsest solve, FCG variant,
 * the learned preconditioner) are stated at the function that takes each.
 *
 * Parity pins live in tests/test_oracle_*.py. Functions marked
 * "parity unpinned" have no independent pin.
 *
 * Build: gcc -O2 -std=gnu11 -fopenmp -ffp-contract=off -fPIC -shared (no
 * fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_NOCONV 1
#define ORC_ERR_ARG -1
#define ORC_ERR_NOT_SPD -2
#define ORC_ERR_NAN -3
#define ORC_ERR_OOM -5
#define ORC_ERR_COARSEN -6

#define ORC_MAXLEV 64

/*
 * Row-independent loops (y_i = sum_k a_ik x_k, elementwise vector updates)
 * may run on several host threads: every row is still computed by one thread
 * in the same order, so the results are identical for any thread count.
 * Dot products, restrictions (scatter sums) and the whole setup stay serial.
 */
#ifdef _OPENMP
#include <omp.h>
#define ORC_ROWS _Pragma("omp parallel for schedule(static) if (n >= 65536)")
#else
#define ORC_ROWS
#endif

/* Threads used by the row loops (<= 0: leave the OpenMP default). */
void orc_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* CSR helpers                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    int n;
    int *rp;      /* n+1 */
    int *ci;      /* nnz, ascending per row */
    double *v;    /* nnz */
} csr;

static void csr_free(csr *a) {
    free(a->rp); free(a->ci); free(a->v);
    a->rp = NULL; a->ci = NULL; a->v = NULL;
}

/* y = A x, each row summed in ascending column order */
void orc_spmv(int n, const int *rp, const int *ci, const double *v,
              const double *x, double *y) {
    ORC_ROWS
    for (int i = 0; i < n; i++) {
        double s = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; k++) s += v[k] * x[ci[k]];
        y[i] = s;
    }
}

static double dot(int n, const double *a, const double *b) {
    double s = 0.0;
    for (int i = 0; i < n; i++) s += a[i] * b[i];
    return s;
}

/*
 * Canonical Galerkin sum (Section "AMG4PSBLAS": A_{l+1} = P^T A P for a
 * prolongator with one nonzero per row):
 *   C[I,J] = sum over i in I (ascending), then stored entries j of row i
 *            (ascending) with agg[j] = J, of (s_i * a_ij) * s_j.
 * Every structurally reached (I,J) is stored, even if its value is zero.
 * Rows of C have ascending columns.
 */
static int galerkin(const csr *a, const int *agg, int nc, const double *s, csr *c) {
    int n = a->n;
    int *cnt = calloc((size_t)nc + 1, sizeof(int));
    int *mem = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!cnt || !mem) { free(cnt); free(mem); return ORC_ERR_OOM; }
    for (int i = 0; i < n; i++) cnt[agg[i] + 1]++;
    for (int I = 0; I < nc; I++) cnt[I + 1] += cnt[I];
    int *fill = malloc(sizeof(int) * (size_t)(nc + 1));
    memcpy(fill, cnt, sizeof(int) * (size_t)(nc + 1));
    for (int i = 0; i < n; i++) mem[fill[agg[i]]++] = i;   /* members ascending */
    free(fill);

    double *acc = calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
    int *mark = malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    int *list = malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    for (int J = 0; J < nc; J++) mark[J] = -1;

    /* first pass: count */
    size_t cap = 0;
    int *rp = malloc(sizeof(int) * (size_t)(nc + 1));
    rp[0] = 0;
    for (int I = 0; I < nc; I++) {
        int len = 0;
        for (int m = cnt[I]; m < cnt[I + 1]; m++) {
            int i = mem[m];
            for (int k = a->rp[i]; k < a->rp[i + 1]; k++) {
                int J = agg[a->ci[k]];
                if (mark[J] != I) { mark[J] = I; len++; }
            }
        }
        rp[I + 1] = rp[I] + len;
    }
    cap = (size_t)rp[nc];
    int *ci = malloc(sizeof(int) * (cap > 0 ? cap : 1));
    double *v = malloc(sizeof(double) * (cap > 0 ? cap : 1));
    for (int J = 0; J < nc; J++) mark[J] = -1;
    for (int I = 0; I < nc; I++) {
        int len = 0;
        for (int m = cnt[I]; m < cnt[I + 1]; m++) {
            int i = mem[m];
            for (int k = a->rp[i]; k < a->rp[i + 1]; k++) {
                int J = agg[a->ci[k]];
                double t = (s[i] * a->v[k]) * s[a->ci[k]];
                if (mark[J] != I) { mark[J] = I; acc[J] = t; list[len++] = J; }
                else acc[J] += t;
            }
        }
        /* sort the touched columns ascending (insertion sort; rows are short) */
        for (int x = 1; x < len; x++) {
            int key = list[x], y = x - 1;
            while (y >= 0 && list[y] > key) { list[y + 1] = list[y]; y--; }
            list[y + 1] = key;
        }
        for (int x = 0; x < len; x++) {
            ci[rp[I] + x] = list[x];
            v[rp[I] + x] = acc[list[x]];
        }
    }
    free(acc); free(mark); free(list); free(cnt); free(mem);
    c->n = nc; c->rp = rp; c->ci = ci; c->v = v;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Matching (Section "Aggregation strategies", coupled aggregation)         */
/* ------------------------------------------------------------------------ */

typedef struct { long long q; int i, j; } edge;

static int edge_cmp(const void *pa, const void *pb) {
    const edge *a = pa, *b = pb;
    if (a->q != b->q) return a->q > b->q ? -1 : 1;     /* weight descending */
    if (a->i != b->i) return a->i < b->i ? -1 : 1;     /* then smaller end ascending */
    if (a->j != b->j) return a->j < b->j ? -1 : 1;     /* then larger end ascending */
    return 0;
}

/* Edge weight of the compatible weighted matching, in terms of the scaled
 * operator S = diag(w) A diag(w) (block-summed at a second sweep):
 *   c_ij = 1 - 2 S_ij / (S_ii + S_jj),
 * quantised as q = llround(c * 2^30); only edges with q > 0 take part. */
long long orc_edge_key(double sij, double sii, double sjj) {
    double c = 1.0 - 2.0 * sij / (sii + sjj);
    return llround(c * 1073741824.0);
}

/*
 * One matching sweep on the symmetric graph of S (CSR, ascending columns,
 * diagonal present). Greedy over eligible edges (i<j) in the strict order
 * (q desc, i asc, j asc): an edge joins the matching when both ends are
 * still free. Under a strict total order this is the unique
 * locally-dominant matching, a 1/2-approximation of the maximum-weight
 * matching. mate[i] = partner or -1. Returns the number of matched pairs.
 */
int orc_match(int n, const int *rp, const int *ci, const double *S, int *mate) {
    double *dg = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; i++) {
        dg[i] = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; k++) if (ci[k] == i) dg[i] = S[k];
    }
    size_t ne = 0;
    for (int i = 0; i < n; i++)
        for (int k = rp[i]; k < rp[i + 1]; k++) if (ci[k] > i) ne++;
    edge *E = malloc(sizeof(edge) * (ne > 0 ? ne : 1));
    size_t m = 0;
    for (int i = 0; i < n; i++)
        for (int k = rp[i]; k < rp[i + 1]; k++) {
            int j = ci[k];
            if (j <= i) continue;
            long long q = orc_edge_key(S[k], dg[i], dg[j]);
            if (q > 0) { E[m].q = q; E[m].i = i; E[m].j = j; m++; }
        }
    qsort(E, m, sizeof(edge), edge_cmp);
    for (int i = 0; i < n; i++) mate[i] = -1;
    int pairs = 0;
    for (size_t e = 0; e < m; e++) {
        if (mate[E[e].i] < 0 && mate[E[e].j] < 0) {
            mate[E[e].i] = E[e].j; mate[E[e].j] = E[e].i; pairs++;
        }
    }
    free(E); free(dg);
    return pairs;
}

/* Pairs and singletons of a matching as aggregates, numbered by ascending
 * smallest member. Returns the number of aggregates. */
static int pairs_to_aggregates(int n, const int *mate, int *agg) {
    int nc = 0;
    for (int i = 0; i < n; i++) agg[i] = -1;
    for (int i = 0; i < n; i++) {
        if (agg[i] >= 0) continue;
        agg[i] = nc;
        if (mate[i] >= 0) agg[mate[i]] = nc;
        nc++;
    }
    return nc;
}

/* ------------------------------------------------------------------------ */
/* Factored approximate inverse smoothers (Section "GPU enabled smoothers", */
/* AINV and INVK): G = Z D^-1 Z^T ~ A^-1 with Z unit upper triangular, so   */
/* that a sweep x <- x + G (b - A x) needs only products with A, Z^T and Z. */
/* ------------------------------------------------------------------------ */

/* Z stored by columns: column k holds rows zi[zr[k] .. zr[k+1]) (ascending)
 * with values zv; d[k] > 0. n = 0 means "no such smoother". */
typedef struct { int n; int *zr, *zi; double *zv, *d; } fai;

static void fai_free(fai *s) { free(s->zr); free(s->zi); free(s->zv); free(s->d); s->n = 0; }

/* growable column store */
typedef struct { long long len, cap; int *idx; double *val; } colbuf;
static int colbuf_push(colbuf *b, int i, double v) {
    if (b->len == b->cap) {
        long long nc = b->cap ? 2 * b->cap : 1024;
        int *ni = realloc(b->idx, sizeof(int) * (size_t)nc);
        if (!ni) return ORC_ERR_OOM;
        b->idx = ni;
        double *nv = realloc(b->val, sizeof(double) * (size_t)nc);
        if (!nv) return ORC_ERR_OOM;
        b->val = nv;
        b->cap = nc;
    }
    b->idx[b->len] = i;
    b->val[b->len] = v;
    b->len++;
    return ORC_OK;
}

/* binary heap of ints; sign = +1: smallest first, -1: largest first */
typedef struct { int *a; int len; int sign; } iheap;
static void heap_push(iheap *h, int x) {
    int i = h->len++;
    h->a[i] = x;
    while (i > 0) {
        int p = (i - 1) / 2;
        if (h->sign * h->a[p] <= h->sign * h->a[i]) break;
        int t = h->a[p]; h->a[p] = h->a[i]; h->a[i] = t;
        i = p;
    }
}
static int heap_pop(iheap *h) {
    int top = h->a[0];
    h->a[0] = h->a[--h->len];
    int i = 0;
    for (;;) {
        int l = 2 * i + 1, r = l + 1, m = i;
        if (l < h->len && h->sign * h->a[l] < h->sign * h->a[m]) m = l;
        if (r < h->len && h->sign * h->a[r] < h->sign * h->a[m]) m = r;
        if (m == i) break;
        int t = h->a[m]; h->a[m] = h->a[i]; h->a[i] = t;
        i = m;
    }
    return top;
}

/* AINV candidates reached from the support index s: every finished column
 * i in (cur, k) with an entry in a row adjacent to s */
static void ainv_reach(const csr *A, int s, int cur, int k, const int *rhead, const int *rnext,
                       const int *rcol, int *mark, iheap *hp) {
    for (int q = A->rp[s]; q < A->rp[s + 1]; q++)
        for (int e = rhead[A->ci[q]]; e >= 0; e = rnext[e]) {
            const int i = rcol[e];
            if (i > cur && i < k && mark[i] != k) { mark[i] = k; heap_push(hp, i); }
        }
}

static int int_cmp(const void *a, const void *b) {
    int x = *(const int *)a, y = *(const int *)b;
    return (x > y) - (x < y);
}

/* (A z)_r for the dense vector z: sum over row r of A in column order */
static double row_dot(const csr *A, int r, const double *z) {
    double s = 0.0;
    for (int q = A->rp[r]; q < A->rp[r + 1]; q++) s += A->v[q] * z[A->ci[q]];
    return s;
}

/*
 * AINV: incomplete A-biconjugation of the SPD matrix A (W = Z by symmetry),
 * in the stabilised form whose pivots are d_i = z_i^T A z_i > 0. The process
 * starts from z_j = e_j; for i = 0, 1, ... the columns j > i are made
 * A-conjugate to z_i: z_j <- z_j - (z_i^T A z_j / d_i) z_i whenever that
 * coefficient is non-zero, and after each such update the entries r != j of
 * z_j with |z_rj| sqrt(a_rr / a_jj) < tau are dropped (the drop tolerance
 * applies to the matrix scaled to unit diagonal). Column k is final once
 * the steps i < k have been applied to it, so it is formed here column by
 * column, applying those steps in ascending i; a step whose coefficient is
 * zero changes nothing and is skipped. The candidates i for column k are
 * the columns with an entry in a row adjacent (in A) to an entry of z_k.
 */
static int ainv_build(const csr *A, double tau, fai *S) {
    const int n = A->n;
    int st = ORC_OK;
    double *dg = malloc(sizeof(double) * (size_t)n);
    double *z = calloc((size_t)n, sizeof(double));
    char *in = calloc((size_t)n, 1);
    int *sup = malloc(sizeof(int) * (size_t)n);
    int *mark = malloc(sizeof(int) * (size_t)n);
    iheap hp = {malloc(sizeof(int) * (size_t)n), 0, 1};
    /* rows of the finished columns: for row r, the columns i with z_ri != 0 */
    int *rhead = malloc(sizeof(int) * (size_t)n);
    colbuf rl = {0, 0, NULL, NULL};   /* idx: column i, val unused; linked by rnext */
    int *rnext = NULL;
    long long rnext_cap = 0;
    colbuf col = {0, 0, NULL, NULL};
    S->n = n;
    S->zr = malloc(sizeof(int) * (size_t)(n + 1));
    S->d = malloc(sizeof(double) * (size_t)n);
    if (!dg || !z || !in || !sup || !mark || !hp.a || !rhead || !S->zr || !S->d) { st = ORC_ERR_OOM; goto out; }
    for (int i = 0; i < n; i++) {
        dg[i] = 0.0;
        for (int q = A->rp[i]; q < A->rp[i + 1]; q++) if (A->ci[q] == i) dg[i] = A->v[q];
        if (!(dg[i] > 0.0)) { st = ORC_ERR_NOT_SPD; goto out; }
        mark[i] = -1;
        rhead[i] = -1;
    }
    S->zr[0] = 0;
    for (int k = 0; k < n; k++) {
        int ns = 0;
        sup[ns++] = k;
        in[k] = 1;
        z[k] = 1.0;
        hp.len = 0;
        int cur = -1;   /* the step being applied; candidates must exceed it */
        ainv_reach(A, k, cur, k, rhead, rnext, rl.idx, mark, &hp);
        while (hp.len > 0) {
            const int i = heap_pop(&hp);
            cur = i;
            /* coefficient z_i^T A z over the entries of column i */
            double p = 0.0;
            for (int e = S->zr[i]; e < S->zr[i + 1]; e++) p += col.val[e] * row_dot(A, col.idx[e], z);
            if (p == 0.0) continue;
            const double alpha = p / S->d[i];
            for (int e = S->zr[i]; e < S->zr[i + 1]; e++) {
                const int r = col.idx[e];
                if (!in[r]) {
                    in[r] = 1;
                    z[r] = 0.0;
                    sup[ns++] = r;
                    ainv_reach(A, r, cur, k, rhead, rnext, rl.idx, mark, &hp);
                }
                z[r] -= alpha * col.val[e];
            }
            /* drop small entries (never the unit diagonal) */
            int w = 0;
            for (int t = 0; t < ns; t++) {
                const int r = sup[t];
                if (r != k && fabs(z[r]) * sqrt(dg[r] / dg[k]) < tau) { in[r] = 0; z[r] = 0.0; }
                else sup[w++] = r;
            }
            ns = w;
        }
        qsort(sup, (size_t)ns, sizeof(int), int_cmp);
        /* pivot d_k = z^T A z, rows ascending */
        double dk = 0.0;
        for (int t = 0; t < ns; t++) dk += z[sup[t]] * row_dot(A, sup[t], z);
        if (!(dk > 0.0)) { st = ORC_ERR_NOT_SPD; goto out; }
        S->d[k] = dk;
        for (int t = 0; t < ns; t++) {
            const int r = sup[t];
            if ((st = colbuf_push(&col, r, z[r]))) goto out;
            if ((st = colbuf_push(&rl, k, 0.0))) goto out;
            if (rl.len > rnext_cap) {
                rnext_cap = rl.cap;
                int *nn = realloc(rnext, sizeof(int) * (size_t)rnext_cap);
                if (!nn) { st = ORC_ERR_OOM; goto out; }
                rnext = nn;
            }
            rnext[rl.len - 1] = rhead[r];
            rhead[r] = (int)(rl.len - 1);
        }
        if (col.len > 2147483647LL) { st = ORC_ERR_OOM; goto out; }
        S->zr[k + 1] = (int)col.len;
        for (int t = 0; t < ns; t++) { in[sup[t]] = 0; z[sup[t]] = 0.0; }
    }
    S->zi = col.idx;
    S->zv = col.val;
    col.idx = NULL;
    col.val = NULL;
out:
    free(dg); free(z); free(in); free(sup); free(mark); free(hp.a); free(rhead);
    free(rl.idx); free(rl.val); free(rnext); free(col.idx); free(col.val);
    if (st) fai_free(S);
    return st;
}

/*
 * INVK: an incomplete factorisation A ~ L D L^T with level-of-fill fill1
 * (L unit lower triangular; original entries have level 0, a fill entry
 * created through pivot m has level lev(i,m) + lev(j,m) + 1 and is kept when
 * that is at most fill1), followed by the sparse inverse Z ~ L^-T whose
 * column k solves L^T z = e_k on a limited pattern: z_k = 1 (level -1), and
 * z_r = -sum_{j > r} l_jr z_j for r < k taken in descending order, an entry
 * r being kept when its level, one more than the smallest level of the
 * entries j it is computed from, is at most fill2. G = Z D^-1 Z^T.
 * A non-positive pivot is a breakdown (ORC_ERR_NOT_SPD).
 */
static int invk_build(const csr *A, int fill1, int fill2, fai *S) {
    const int n = A->n;
    int st = ORC_OK;
    /* L by rows (strictly lower part, ascending columns) */
    int *lr = malloc(sizeof(int) * (size_t)(n + 1));
    colbuf lrow = {0, 0, NULL, NULL};
    double *w = calloc((size_t)n, sizeof(double));
    int *lev = malloc(sizeof(int) * (size_t)n);
    char *in = calloc((size_t)n, 1);
    int *sup = malloc(sizeof(int) * (size_t)n);
    int *mark = malloc(sizeof(int) * (size_t)n);
    iheap hp = {malloc(sizeof(int) * (size_t)n), 0, 1};
    colbuf col = {0, 0, NULL, NULL};
    S->n = n;
    S->zr = malloc(sizeof(int) * (size_t)(n + 1));
    S->d = malloc(sizeof(double) * (size_t)n);
    /* the factorisation needs column access to finished rows: a growable
     * per-column list kept as a linked list of (row, value, level) */
    int *chead = malloc(sizeof(int) * (size_t)n), *ctail = malloc(sizeof(int) * (size_t)n);
    int *cnext = NULL, *crow = NULL, *clev = NULL;
    double *cval = NULL;
    long long clen = 0, ccap = 0;
    if (!lr || !w || !lev || !in || !sup || !mark || !hp.a || !S->zr || !S->d || !chead || !ctail) {
        st = ORC_ERR_OOM; goto out;
    }
    for (int i = 0; i < n; i++) { chead[i] = ctail[i] = -1; mark[i] = -1; }
    lr[0] = 0;
    for (int i = 0; i < n; i++) {
        int ns = 0;
        hp.len = 0;
        for (int q = A->rp[i]; q < A->rp[i + 1]; q++) {
            const int c = A->ci[q];
            if (c > i) continue;
            w[c] = A->v[q];
            lev[c] = 0;
            in[c] = 1;
            sup[ns++] = c;
            if (c < i) heap_push(&hp, c);
        }
        if (!in[i]) { st = ORC_ERR_NOT_SPD; goto out; }
        /* symbolic pass: the row's final pattern, every level the minimum
         * over all pivots (a pivot's own level is final when it is reached) */
        while (hp.len > 0) {
            const int m = heap_pop(&hp);
            for (int e = chead[m]; e >= 0; e = cnext[e]) {
                const int j = crow[e];
                const int nl = lev[m] + clev[e] + 1;
                if (in[j]) {
                    if (nl < lev[j]) lev[j] = nl;
                } else if (nl <= fill1) {
                    in[j] = 1;
                    w[j] = 0.0;
                    lev[j] = nl;
                    sup[ns++] = j;
                    heap_push(&hp, j);
                }
            }
        }
        qsort(sup, (size_t)ns, sizeof(int), int_cmp);
        /* numeric pass over that pattern, pivots ascending:
         * l_im = w_m / d_m, w_j -= l_im d_m l_jm, w_i -= l_im d_m l_im */
        for (int t = 0; t < ns && sup[t] < i; t++) {
            const int m = sup[t];
            const double lim = w[m] / S->d[m];
            w[m] = lim;
            for (int e = chead[m]; e >= 0; e = cnext[e])
                if (in[crow[e]]) w[crow[e]] -= lim * S->d[m] * cval[e];
            w[i] -= lim * S->d[m] * lim;
        }
        if (!(w[i] > 0.0)) { st = ORC_ERR_NOT_SPD; goto out; }
        S->d[i] = w[i];
        for (int t = 0; t < ns; t++) {
            const int m = sup[t];
            if (m == i) continue;
            if ((st = colbuf_push(&lrow, m, w[m]))) goto out;
            /* append (i, l_im) to column m (rows arrive in ascending order) */
            if (clen == ccap) {
                ccap = ccap ? 2 * ccap : 1024;
                int *a1 = realloc(cnext, sizeof(int) * (size_t)ccap);
                if (!a1) { st = ORC_ERR_OOM; goto out; }
                cnext = a1;
                int *a2 = realloc(crow, sizeof(int) * (size_t)ccap);
                if (!a2) { st = ORC_ERR_OOM; goto out; }
                crow = a2;
                int *a3 = realloc(clev, sizeof(int) * (size_t)ccap);
                if (!a3) { st = ORC_ERR_OOM; goto out; }
                clev = a3;
                double *a4 = realloc(cval, sizeof(double) * (size_t)ccap);
                if (!a4) { st = ORC_ERR_OOM; goto out; }
                cval = a4;
            }
            crow[clen] = i; cval[clen] = w[m]; clev[clen] = lev[m]; cnext[clen] = -1;
            if (ctail[m] < 0) chead[m] = (int)clen; else cnext[ctail[m]] = (int)clen;
            ctail[m] = (int)clen;
            clen++;
        }
        lr[i + 1] = (int)lrow.len;
        for (int t = 0; t < ns; t++) { in[sup[t]] = 0; w[sup[t]] = 0.0; }
    }
    /* Z = L^-T column by column (descending row order) */
    {
        iheap mh = {hp.a, 0, -1};
        S->zr[0] = 0;
        for (int k = 0; k < n; k++) {
            int ns = 0;
            w[k] = 1.0;
            lev[k] = -1;
            in[k] = 1;
            sup[ns++] = k;
            mh.len = 0;
            for (int e = lr[k]; e < lr[k + 1]; e++) {
                const int r = lrow.idx[e];
                if (mark[r] != k) { mark[r] = k; heap_push(&mh, r); }
            }
            while (mh.len > 0) {
                const int r = heap_pop(&mh);
                double s = 0.0;
                int lv = 2147483647;
                for (int e = chead[r]; e >= 0; e = cnext[e]) {
                    const int j = crow[e];
                    if (j > k || !in[j]) continue;
                    s += cval[e] * w[j];
                    if (lev[j] + 1 < lv) lv = lev[j] + 1;
                }
                if (lv > fill2) continue;
                w[r] = -s;
                lev[r] = lv;
                in[r] = 1;
                sup[ns++] = r;
                for (int e = lr[r]; e < lr[r + 1]; e++) {
                    const int r2 = lrow.idx[e];
                    if (mark[r2] != k) { mark[r2] = k; heap_push(&mh, r2); }
                }
            }
            qsort(sup, (size_t)ns, sizeof(int), int_cmp);
            for (int t = 0; t < ns; t++)
                if ((st = colbuf_push(&col, sup[t], w[sup[t]]))) goto out;
            if (col.len > 2147483647LL) { st = ORC_ERR_OOM; goto out; }
            S->zr[k + 1] = (int)col.len;
            for (int t = 0; t < ns; t++) { in[sup[t]] = 0; w[sup[t]] = 0.0; }
        }
        hp.a = mh.a;
    }
    S->zi = col.idx;
    S->zv = col.val;
    col.idx = NULL;
    col.val = NULL;
out:
    free(lr); free(lrow.idx); free(lrow.val);
    free(w); free(lev); free(in); free(sup); free(mark); free(hp.a); free(col.idx); free(col.val);
    free(chead); free(ctail); free(cnext); free(crow); free(clev); free(cval);
    if (st) fai_free(S);
    return st;
}

/* u = Z D^-1 Z^T t: y_k = (sum over column k, rows ascending, of z_rk t_r)
 * / d_k, then u_r = sum over k ascending of z_rk y_k. */
static void fai_apply(const fai *S, const double *t, double *u, double *y) {
    const int n = S->n;
    for (int k = 0; k < n; k++) {
        double s = 0.0;
        for (int e = S->zr[k]; e < S->zr[k + 1]; e++) s += S->zv[e] * t[S->zi[e]];
        y[k] = s / S->d[k];
    }
    for (int r = 0; r < n; r++) u[r] = 0.0;
    for (int k = 0; k < n; k++)
        for (int e = S->zr[k]; e < S->zr[k + 1]; e++) u[S->zi[e]] += S->zv[e] * y[k];
}

/* The same in float with float copies of the factors: y_k = sum of
 * (float)(z_rk / d_k) t_r, u_r = sum of (float)z_rk y_k. */
static void fai_apply32(const fai *S, const float *t, float *u, float *y) {
    const int n = S->n;
    for (int k = 0; k < n; k++) {
        float s = 0.0f;
        for (int e = S->zr[k]; e < S->zr[k + 1]; e++) s += (float)(S->zv[e] / S->d[k]) * t[S->zi[e]];
        y[k] = s;
    }
    for (int r = 0; r < n; r++) u[r] = 0.0f;
    for (int k = 0; k < n; k++)
        for (int e = S->zr[k]; e < S->zr[k + 1]; e++) u[S->zi[e]] += (float)S->zv[e] * y[k];
}

/* ------------------------------------------------------------------------ */
/* Hierarchy                                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
    csr A;
    double *w;      /* near-kernel sample at this level (w = 1 at level 0) */
    double *minv;   /* l1-Jacobi: 1 / (a_ii + sum_{j!=i} |a_ij|) */
    int nc;         /* next level size (0 at the coarsest) */
    int *agg;       /* aggregate of each row */
    double *p;      /* value of row i of the tentative prolongator P^ */
    csr P;          /* prolongator used by the V-cycle: P^ itself, or smoothed */
    double omega;   /* smoothed prolongator: damping 1 / ||D^-1 A||_inf */
    double *L;      /* coarsest only: dense lower Cholesky factor, row-major */
    fai S;          /* AINV / INVK smoother (S.n = 0 with l1-Jacobi) */
} orc_level;

typedef struct {
    int nlev;
    int sweeps;
    int coarse_sweeps;   /* > 0: the coarsest level is solved by this many l1-Jacobi sweeps */
    int coarse_pcg;      /* > 0: the coarsest level is solved by at most this many PCG iterations */
    double coarse_rtol;  /* their relative residual tolerance */
    int prol;            /* 0: tentative prolongator, 1: smoothed */
    int nu;              /* l1-Jacobi sweeps before and after the coarse correction (level 0) */
    int nu_double;       /* 1: variable V-cycle, nu_l = nu * 2^l (the paper's VMATCH) */
    int aggr;            /* 0: coupled matching aggregation, 1: decoupled VBM */
    double theta;        /* VBM strength threshold */
    int smoother;        /* 0: l1-Jacobi, 1: AINV, 2: INVK, 3: Chebyshev polynomial (levels above the coarsest) */
    double tau;          /* AINV drop tolerance */
    int fill1, fill2;    /* INVK fill levels of the factor and of its inverse */
    orc_level lev[ORC_MAXLEV];
} orc_hier;

void orc_free(orc_hier *h) {
    if (!h) return;
    for (int l = 0; l < h->nlev; l++) {
        orc_level *L = &h->lev[l];
        csr_free(&L->A);
        free(L->w); free(L->minv); free(L->agg); free(L->p); free(L->L);
        csr_free(&L->P);
        fai_free(&L->S);
    }
    free(h);
}

/* l1-Jacobi inverse diagonal (Section "GPU enabled smoothers"):
 * d_i = a_ii + (sum over j != i, ascending, of |a_ij|). */
static int l1_diag_inv(const csr *a, double *minv) {
    for (int i = 0; i < a->n; i++) {
        double dii = 0.0, off = 0.0;
        int has = 0;
        for (int k = a->rp[i]; k < a->rp[i + 1]; k++) {
            if (a->ci[k] == i) { dii = a->v[k]; has = 1; }
            else off += fabs(a->v[k]);
        }
        if (!has || !(dii > 0.0)) return ORC_ERR_NOT_SPD;
        minv[i] = 1.0 / (dii + off);
    }
    return ORC_OK;
}

/* Dense Cholesky A = L L^T of the coarsest matrix (lower triangle read). */
static int dense_cholesky(const csr *a, double *L) {
    int n = a->n;
    for (size_t t = 0; t < (size_t)n * n; t++) L[t] = 0.0;
    for (int i = 0; i < n; i++)
        for (int k = a->rp[i]; k < a->rp[i + 1]; k++)
            if (a->ci[k] <= i) L[(size_t)i * n + a->ci[k]] = a->v[k];
    for (int j = 0; j < n; j++) {
        double d = L[(size_t)j * n + j];
        for (int k = 0; k < j; k++) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(d > 0.0)) return ORC_ERR_NOT_SPD;
        double ljj = sqrt(d);
        L[(size_t)j * n + j] = ljj;
        for (int i = j + 1; i < n; i++) {
            double s = L[(size_t)i * n + j];
            for (int k = 0; k < j; k++) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = s / ljj;
        }
    }
    return ORC_OK;
}

static void chol_solve(int n, const double *L, const double *b, double *x) {
    for (int i = 0; i < n; i++) {
        double s = b[i];
        for (int k = 0; k < i; k++) s -= L[(size_t)i * n + k] * x[k];
        x[i] = s / L[(size_t)i * n + i];
    }
    for (int i = n - 1; i >= 0; i--) {
        double s = x[i];
        for (int k = i + 1; k < n; k++) s -= L[(size_t)k * n + i] * x[k];
        x[i] = s / L[(size_t)i * n + i];
    }
}

/*
 * One level of coarsening by `sweeps` matching sweeps (Section "Aggregation
 * strategies"). Sweep 1 matches the graph of S = diag(w) A diag(w); sweep
 * s+1 matches the graph of the block sums of S over the aggregates of sweep
 * s (the tentative Galerkin operator of the previous sweeps, up to the
 * normalisation, which the edge weight does not see). The final aggregates
 * are numbered by ascending smallest level-l member.
 */
/*
 * Decoupled Vanek-Mandel-Brezina aggregation (Section "Aggregation
 * strategies"): j is strongly coupled to i when j != i and
 * |a_ij| >= theta sqrt(a_ii a_jj). In ascending node order:
 *   1. a node whose strong neighbours are all unaggregated forms an
 *      aggregate with them;
 *   2. each node still unaggregated joins the aggregate (from step 1) of its
 *      strong neighbour with the largest |a_ij| (ties: smaller j);
 *   3. each node still unaggregated forms an aggregate with its
 *      unaggregated strong neighbours.
 * Aggregates are numbered in order of creation.
 */
static int vbm_aggregate(const csr *A, double theta, int *agg, int *nc_out) {
    int n = A->n, nc = 0;
    double *d = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    int *a1 = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    if (!d || !a1) { free(d); free(a1); return ORC_ERR_OOM; }
    for (int i = 0; i < n; i++) {
        d[i] = 0.0;
        for (int k = A->rp[i]; k < A->rp[i + 1]; k++) if (A->ci[k] == i) d[i] = A->v[k];
        agg[i] = -1;
    }
#define STRONG(i, k) (A->ci[k] != (i) && fabs(A->v[k]) >= theta * sqrt(d[i] * d[A->ci[k]]))
    for (int i = 0; i < n; i++) {
        if (agg[i] != -1) continue;
        int free_all = 1;
        for (int k = A->rp[i]; k < A->rp[i + 1]; k++)
            if (STRONG(i, k) && agg[A->ci[k]] != -1) { free_all = 0; break; }
        if (!free_all) continue;
        agg[i] = nc;
        for (int k = A->rp[i]; k < A->rp[i + 1]; k++) if (STRONG(i, k)) agg[A->ci[k]] = nc;
        nc++;
    }
    memcpy(a1, agg, sizeof(int) * (size_t)n);
    for (int i = 0; i < n; i++) {
        if (a1[i] != -1) continue;
        int best = -1;
        double bv = -1.0;
        for (int k = A->rp[i]; k < A->rp[i + 1]; k++) {
            if (!STRONG(i, k) || a1[A->ci[k]] == -1) continue;
            double v = fabs(A->v[k]);
            if (v > bv) { bv = v; best = a1[A->ci[k]]; }     /* columns ascending: ties keep the smaller j */
        }
        if (best != -1) agg[i] = best;
    }
    for (int i = 0; i < n; i++) {
        if (agg[i] != -1) continue;
        agg[i] = nc;
        for (int k = A->rp[i]; k < A->rp[i + 1]; k++)
            if (STRONG(i, k) && agg[A->ci[k]] == -1) agg[A->ci[k]] = nc;
        nc++;
    }
#undef STRONG
    free(d); free(a1);
    *nc_out = nc;
    return ORC_OK;
}

/*
 * Smoothed prolongator (Section "Aggregation strategies"): P = (I - omega
 * D^-1 A) P^ with D = diag(A), omega = 1 / ||D^-1 A||_inf, and P^ the
 * tentative prolongator (row i: value p_i in column agg_i). Row i:
 *   t_J  = sum over stored j of row i (ascending) with agg_j = J of a_ij p_j,
 *   P_iJ = [J = agg_i] p_i - (omega / a_ii) t_J,
 * every reached J stored, columns ascending.
 */
static int smoothed_prolongator(const csr *A, const int *agg, const double *p, int nc,
                                double omega, csr *P) {
    int n = A->n;
    double *acc = calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
    int *mark = malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    int *list = malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    int *rp = malloc(sizeof(int) * (size_t)(n + 1));
    if (!acc || !mark || !list || !rp) { free(acc); free(mark); free(list); free(rp); return ORC_ERR_OOM; }
    for (int J = 0; J < nc; J++) mark[J] = -1;
    rp[0] = 0;
    for (int i = 0; i < n; i++) {
        int len = 0;
        for (int k = A->rp[i]; k < A->rp[i + 1]; k++) {
            int J = agg[A->ci[k]];
            if (mark[J] != i) { mark[J] = i; len++; }
        }
        rp[i + 1] = rp[i] + len;
    }
    int nnz = rp[n];
    int *ci = malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    double *v = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    for (int J = 0; J < nc; J++) mark[J] = -1;
    for (int i = 0; i < n; i++) {
        int len = 0;
        double aii = 0.0;
        for (int k = A->rp[i]; k < A->rp[i + 1]; k++) {
            int j = A->ci[k], J = agg[j];
            if (j == i) aii = A->v[k];
            double t = A->v[k] * p[j];
            if (mark[J] != i) { mark[J] = i; acc[J] = t; list[len++] = J; }
            else acc[J] += t;
        }
        for (int x = 1; x < len; x++) {
            int key = list[x], y = x - 1;
            while (y >= 0 && list[y] > key) { list[y + 1] = list[y]; y--; }
            list[y + 1] = key;
        }
        for (int x = 0; x < len; x++) {
            int J = list[x];
            double pk = (J == agg[i]) ? p[i] : 0.0;
            ci[rp[i] + x] = J;
            v[rp[i] + x] = pk - (omega / aii) * acc[J];
        }
    }
    free(acc); free(mark); free(list);
    P->n = n; P->rp = rp; P->ci = ci; P->v = v;
    return ORC_OK;
}

/*
 * General Galerkin product A_c = P^T (A P) (Section "AMG4PSBLAS") for a
 * prolongator with several nonzeros per row, in a fixed order:
 *   T[i,J] = sum over stored j of row i (ascending), then entries (J, p_jJ)
 *            of row j of P (ascending), of a_ij p_jJ;
 *   C[I,J] = sum over rows i ascending with P_iI stored, of P_iI T[i,J].
 * Every structurally reached entry is stored; rows of C ascending.
 */
static int galerkin_general(const csr *A, const csr *P, int nc, csr *C) {
    int n = A->n;
    double *acc = calloc((size_t)(nc > 0 ? nc : 1), sizeof(double));
    int *mark = malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    int *list = malloc(sizeof(int) * (size_t)(nc > 0 ? nc : 1));
    /* T = A P, row by row */
    csr T;
    T.n = n;
    T.rp = malloc(sizeof(int) * (size_t)(n + 1));
    T.rp[0] = 0;
    size_t cap = (size_t)(A->rp[n] > 0 ? A->rp[n] : 1) * 4, used = 0;
    T.ci = malloc(sizeof(int) * cap);
    T.v = malloc(sizeof(double) * cap);
    for (int J = 0; J < nc; J++) mark[J] = -1;
    for (int i = 0; i < n; i++) {
        int len = 0;
        for (int k = A->rp[i]; k < A->rp[i + 1]; k++) {
            int j = A->ci[k];
            for (int m = P->rp[j]; m < P->rp[j + 1]; m++) {
                int J = P->ci[m];
                double t = A->v[k] * P->v[m];
                if (mark[J] != i) { mark[J] = i; acc[J] = t; list[len++] = J; }
                else acc[J] += t;
            }
        }
        for (int x = 1; x < len; x++) {
            int key = list[x], y = x - 1;
            while (y >= 0 && list[y] > key) { list[y + 1] = list[y]; y--; }
            list[y + 1] = key;
        }
        if (used + (size_t)len > cap) {
            while (used + (size_t)len > cap) cap *= 2;
            T.ci = realloc(T.ci, sizeof(int) * cap);
            T.v = realloc(T.v, sizeof(double) * cap);
        }
        for (int x = 0; x < len; x++) { T.ci[used] = list[x]; T.v[used] = acc[list[x]]; used++; }
        T.rp[i + 1] = (int)used;
    }
    /* rows of P^T: for each coarse I the fine rows i ascending with P_iI */
    int *tc = calloc((size_t)nc + 1, sizeof(int));
    for (int m = 0; m < P->rp[n]; m++) tc[P->ci[m] + 1]++;
    for (int I = 0; I < nc; I++) tc[I + 1] += tc[I];
    int *fill = malloc(sizeof(int) * (size_t)(nc + 1));
    memcpy(fill, tc, sizeof(int) * (size_t)(nc + 1));
    int *ti = malloc(sizeof(int) * (size_t)(P->rp[n] > 0 ? P->rp[n] : 1));
    double *tv = malloc(sizeof(double) * (size_t)(P->rp[n] > 0 ? P->rp[n] : 1));
    for (int i = 0; i < n; i++)
        for (int m = P->rp[i]; m < P->rp[i + 1]; m++) {
            int o = fill[P->ci[m]]++;
            ti[o] = i;
            tv[o] = P->v[m];
        }
    free(fill);
    /* C = P^T T */
    int *crp = malloc(sizeof(int) * (size_t)(nc + 1));
    crp[0] = 0;
    size_t ccap = (size_t)(nc > 0 ? nc : 1) * 8, cused = 0;
    int *cci = malloc(sizeof(int) * ccap);
    double *cv = malloc(sizeof(double) * ccap);
    for (int J = 0; J < nc; J++) mark[J] = -1;
    for (int I = 0; I < nc; I++) {
        int len = 0;
        for (int o = tc[I]; o < tc[I + 1]; o++) {
            int i = ti[o];
            double pi = tv[o];
            for (int m = T.rp[i]; m < T.rp[i + 1]; m++) {
                int J = T.ci[m];
                double t = pi * T.v[m];
                if (mark[J] != I) { mark[J] = I; acc[J] = t; list[len++] = J; }
                else acc[J] += t;
            }
        }
        for (int x = 1; x < len; x++) {
            int key = list[x], y = x - 1;
            while (y >= 0 && list[y] > key) { list[y + 1] = list[y]; y--; }
            list[y + 1] = key;
        }
        if (cused + (size_t)len > ccap) {
            while (cused + (size_t)len > ccap) ccap *= 2;
            cci = realloc(cci, sizeof(int) * ccap);
            cv = realloc(cv, sizeof(double) * ccap);
        }
        for (int x = 0; x < len; x++) { cci[cused] = list[x]; cv[cused] = acc[list[x]]; cused++; }
        crp[I + 1] = (int)cused;
    }
    free(tc); free(ti); free(tv); csr_free(&T);
    free(acc); free(mark); free(list);
    C->n = nc; C->rp = crp; C->ci = cci; C->v = cv;
    return ORC_OK;
}

static int coarsen(const csr *A, const double *w, int sweeps, int *agg, int *nc_out) {
    int n = A->n;
    /* S = diag(w) A diag(w) */
    int *ident = malloc(sizeof(int) * (size_t)(n > 0 ? n : 1));
    for (int i = 0; i < n; i++) { ident[i] = i; agg[i] = i; }
    csr S;
    int st = galerkin(A, ident, n, w, &S);
    free(ident);
    if (st) return st;
    double *one = NULL;
    int ncur = n;
    for (int s = 0; s < sweeps; s++) {
        int *mate = malloc(sizeof(int) * (size_t)(ncur > 0 ? ncur : 1));
        int *a2 = malloc(sizeof(int) * (size_t)(ncur > 0 ? ncur : 1));
        orc_match(ncur, S.rp, S.ci, S.v, mate);
        int nnew = pairs_to_aggregates(ncur, mate, a2);
        for (int i = 0; i < n; i++) agg[i] = a2[agg[i]];
        if (s + 1 < sweeps) {
            free(one);
            one = malloc(sizeof(double) * (size_t)(ncur > 0 ? ncur : 1));
            for (int i = 0; i < ncur; i++) one[i] = 1.0;
            csr S2;
            st = galerkin(&S, a2, nnew, one, &S2);
            csr_free(&S);
            if (st) { free(mate); free(a2); free(one); return st; }
            S = S2;
        }
        free(mate); free(a2);
        ncur = nnew;
    }
    csr_free(&S);
    free(one);
    /* renumber by ascending smallest member (kept explicit for clarity) */
    int *ren = malloc(sizeof(int) * (size_t)(ncur > 0 ? ncur : 1));
    for (int I = 0; I < ncur; I++) ren[I] = -1;
    int nc = 0;
    for (int i = 0; i < n; i++) {
        if (ren[agg[i]] < 0) ren[agg[i]] = nc++;
        agg[i] = ren[agg[i]];
    }
    free(ren);
    *nc_out = nc;
    return ORC_OK;
}

static int csr_copy(int n, const int *rp, const int *ci, const double *v, csr *a) {
    long nnz = rp[n];
    a->n = n;
    a->rp = malloc(sizeof(int) * (size_t)(n + 1));
    a->ci = malloc(sizeof(int) * (size_t)(nnz > 0 ? nnz : 1));
    a->v = malloc(sizeof(double) * (size_t)(nnz > 0 ? nnz : 1));
    if (!a->rp || !a->ci || !a->v) return ORC_ERR_OOM;
    memcpy(a->rp, rp, sizeof(int) * (size_t)(n + 1));
    memcpy(a->ci, ci, sizeof(int) * (size_t)nnz);
    memcpy(a->v, v, sizeof(double) * (size_t)nnz);
    return ORC_OK;
}

/*
 * Hierarchy build. For each level: if n_l <= coarse_max it is the coarsest
 * level and is factored by dense Cholesky. Otherwise aggregate, form
 * w_{l+1}[I] = sqrt(sum_{i in I} w_i^2) (ascending members), the tentative
 * prolongator value p_i = w_i / w_{l+1}[agg_i] (eq. prolongator: the column
 * of an aggregate is w restricted to it, normalised), the Galerkin operator
 * A_{l+1} = P^T A_l P (eq. amg context), and the l1-Jacobi diagonal.
 * Stall guard: if n_{l+1} > 0.9 n_l, level l+1 becomes the coarsest; it is
 * factored when it has at most 2000 rows, otherwise it is solved by
 * coarse_sweeps l1-Jacobi sweeps (ORC_ERR_COARSEN when coarse_sweeps < 1).
 */
int orc_build(int n, const int *rp, const int *ci, const double *v,
              int sweeps, int coarse_max, int max_levels, int coarse_sweeps, int prol, int nu,
              int nu_double, int aggr, double theta, int smoother, double tau, int fill1, int fill2,
              int coarse_pcg, double coarse_rtol, orc_hier **out) {
    *out = NULL;
    if (n <= 0 || sweeps < 1 || max_levels < 1 || max_levels > ORC_MAXLEV || prol < 0 || prol > 1 ||
        nu < 1 || nu_double < 0 || nu_double > 1 || aggr < 0 || aggr > 1 || !(theta >= 0.0 && theta < 1.0) ||
        smoother < 0 || smoother > 3 || !(tau >= 0.0) || fill1 < 0 || fill2 < 0 || coarse_pcg < 0 ||
        !(coarse_rtol >= 0.0))
        return ORC_ERR_ARG;
    orc_hier *h = calloc(1, sizeof(orc_hier));
    h->sweeps = sweeps;
    h->prol = prol;
    h->nu = nu;
    h->nu_double = nu_double;
    h->aggr = aggr;
    h->theta = theta;
    h->smoother = smoother;
    h->tau = tau;
    h->fill1 = fill1;
    h->fill2 = fill2;
    h->coarse_rtol = coarse_rtol;
    int st = csr_copy(n, rp, ci, v, &h->lev[0].A);
    if (st) { orc_free(h); return st; }
    h->lev[0].w = malloc(sizeof(double) * (size_t)n);
    for (int i = 0; i < n; i++) h->lev[0].w[i] = 1.0;
    h->nlev = 1;
    for (int l = 0;; l++) {
        orc_level *L = &h->lev[l];
        int nl = L->A.n;
        L->minv = malloc(sizeof(double) * (size_t)nl);
        st = l1_diag_inv(&L->A, L->minv);
        if (st) { orc_free(h); return st; }
        int force_coarsest = (l + 1 >= max_levels);
        int stalled = 0;
        if (l > 0) {
            int nprev = h->lev[l - 1].A.n;
            if ((double)nl > 0.9 * (double)nprev) { force_coarsest = 1; stalled = 1; }
        }
        if (nl <= coarse_max || force_coarsest) {
            L->nc = 0;
            if (stalled && nl > 2000) {
                /* coarsening stalled on a level too large for a dense factor:
                 * it is solved by a fixed number of l1-Jacobi sweeps from zero
                 * (the paper's l1-Jacobi coarsest solver, Section "GPU enabled
                 * smoothers", Fig. prec_build), a fixed SPD operator */
                if (coarse_sweeps < 1) { orc_free(h); return ORC_ERR_COARSEN; }
                h->coarse_sweeps = coarse_sweeps;
                break;
            }
            if (coarse_pcg > 0) {
                /* inexact coarsest solve by PCG instead of the dense factor */
                h->coarse_pcg = coarse_pcg;
                break;
            }
            L->L = malloc(sizeof(double) * (size_t)nl * nl);
            st = dense_cholesky(&L->A, L->L);
            if (st) { orc_free(h); return st; }
            break;
        }
        /* smoother of a level that is not the coarsest */
        if (smoother == 1) st = ainv_build(&L->A, tau, &L->S);
        else if (smoother == 2) st = invk_build(&L->A, fill1, fill2, &L->S);
        if (st) { orc_free(h); return st; }
        L->agg = malloc(sizeof(int) * (size_t)nl);
        int nc = 0;
        if (aggr == 0) st = coarsen(&L->A, L->w, sweeps, L->agg, &nc);
        else st = vbm_aggregate(&L->A, theta, L->agg, &nc);
        if (st) { orc_free(h); return st; }
        L->nc = nc;
        orc_level *C = &h->lev[l + 1];
        C->w = malloc(sizeof(double) * (size_t)nc);
        L->p = malloc(sizeof(double) * (size_t)nl);
        if (aggr == 0) {
            /* matching: P^ columns are the normalised restrictions of w */
            for (int I = 0; I < nc; I++) C->w[I] = 0.0;
            for (int i = 0; i < nl; i++) C->w[L->agg[i]] += L->w[i] * L->w[i];
            for (int I = 0; I < nc; I++) C->w[I] = sqrt(C->w[I]);
            for (int i = 0; i < nl; i++) L->p[i] = L->w[i] / C->w[L->agg[i]];
        } else {
            /* VBM, eq. (prolongator_vbm): P^_{i,agg_i} = w_i; the coarse sample is 1 */
            for (int I = 0; I < nc; I++) C->w[I] = 1.0;
            for (int i = 0; i < nl; i++) L->p[i] = L->w[i];
        }
        if (prol == 0) {
            /* tentative: P = P^, one entry per row; canonical Galerkin sum */
            L->P.n = nl;
            L->P.rp = malloc(sizeof(int) * (size_t)(nl + 1));
            L->P.ci = malloc(sizeof(int) * (size_t)(nl > 0 ? nl : 1));
            L->P.v = malloc(sizeof(double) * (size_t)(nl > 0 ? nl : 1));
            for (int i = 0; i < nl; i++) { L->P.rp[i] = i; L->P.ci[i] = L->agg[i]; L->P.v[i] = L->p[i]; }
            L->P.rp[nl] = nl;
            st = galerkin(&L->A, L->agg, nc, L->p, &C->A);
        } else {
            /* omega = 1 / max_i sum_j |a_ij| / a_ii */
            double norm = 0.0;
            for (int i = 0; i < nl; i++) {
                double s = 0.0, aii = 0.0;
                for (int k = L->A.rp[i]; k < L->A.rp[i + 1]; k++) {
                    s += fabs(L->A.v[k]);
                    if (L->A.ci[k] == i) aii = L->A.v[k];
                }
                if (s / aii > norm) norm = s / aii;
            }
            L->omega = 1.0 / norm;
            st = smoothed_prolongator(&L->A, L->agg, L->p, nc, L->omega, &L->P);
            if (!st) st = galerkin_general(&L->A, &L->P, nc, &C->A);
        }
        if (st) { orc_free(h); return st; }
        h->nlev = l + 2;
    }
    *out = h;
    return ORC_OK;
}

int orc_nlevels(const orc_hier *h) { return h->nlev; }

int orc_level_info(const orc_hier *h, int l, int *n, long long *nnz, int *nc) {
    if (l < 0 || l >= h->nlev) return ORC_ERR_ARG;
    const orc_level *L = &h->lev[l];
    if (n) *n = L->A.n;
    if (nnz) *nnz = L->A.rp[L->A.n];
    if (nc) *nc = L->nc;
    return ORC_OK;
}

/* Copy out level data; any pointer may be NULL. agg/p only below the coarsest. */
int orc_level_get(const orc_hier *h, int l, int *rp, int *ci, double *v,
                  int *agg, double *p, double *w, double *minv) {
    if (l < 0 || l >= h->nlev) return ORC_ERR_ARG;
    const orc_level *L = &h->lev[l];
    int n = L->A.n;
    long nnz = L->A.rp[n];
    if (rp) memcpy(rp, L->A.rp, sizeof(int) * (size_t)(n + 1));
    if (ci) memcpy(ci, L->A.ci, sizeof(int) * (size_t)nnz);
    if (v) memcpy(v, L->A.v, sizeof(double) * (size_t)nnz);
    if (agg && L->agg) memcpy(agg, L->agg, sizeof(int) * (size_t)n);
    if (p && L->p) memcpy(p, L->p, sizeof(double) * (size_t)n);
    if (w) memcpy(w, L->w, sizeof(double) * (size_t)n);
    if (minv) memcpy(minv, L->minv, sizeof(double) * (size_t)n);
    return ORC_OK;
}

int orc_coarse_factor(const orc_hier *h, double *Lout) {
    const orc_level *L = &h->lev[h->nlev - 1];
    int n = L->A.n;
    if (!L->L) return ORC_ERR_ARG;
    memcpy(Lout, L->L, sizeof(double) * (size_t)n * n);
    return ORC_OK;
}

int orc_coarse_sweeps(const orc_hier *h) { return h->coarse_sweeps; }

/* The prolongator of level l (below the coarsest) as CSR; nnz via orc_prol_nnz. */
long long orc_prol_nnz(const orc_hier *h, int l) {
    if (l < 0 || l >= h->nlev - 1) return -1;
    return h->lev[l].P.rp[h->lev[l].P.n];
}

int orc_prol_get(const orc_hier *h, int l, int *rp, int *ci, double *v, double *omega) {
    if (l < 0 || l >= h->nlev - 1) return ORC_ERR_ARG;
    const csr *P = &h->lev[l].P;
    memcpy(rp, P->rp, sizeof(int) * (size_t)(P->n + 1));
    memcpy(ci, P->ci, sizeof(int) * (size_t)P->rp[P->n]);
    memcpy(v, P->v, sizeof(double) * (size_t)P->rp[P->n]);
    if (omega) *omega = h->lev[l].omega;
    return ORC_OK;
}

/* The AINV / INVK factor of level l: nnz of Z (-1 when the level has none),
 * then Z by columns (zr n+1, zi / zv nnz) and the pivots d (n). */
long long orc_fai_nnz(const orc_hier *h, int l) {
    if (l < 0 || l >= h->nlev || !h->lev[l].S.n) return -1;
    return h->lev[l].S.zr[h->lev[l].S.n];
}

int orc_fai_get(const orc_hier *h, int l, int *zr, int *zi, double *zv, double *d) {
    if (orc_fai_nnz(h, l) < 0) return ORC_ERR_ARG;
    const fai *S = &h->lev[l].S;
    memcpy(zr, S->zr, sizeof(int) * (size_t)(S->n + 1));
    memcpy(zi, S->zi, sizeof(int) * (size_t)S->zr[S->n]);
    memcpy(zv, S->zv, sizeof(double) * (size_t)S->zr[S->n]);
    memcpy(d, S->d, sizeof(double) * (size_t)S->n);
    return ORC_OK;
}

/* Stand-alone factorisations of an SPD CSR matrix (for the pins): kind 1
 * AINV(tau), kind 2 INVK(fill1, fill2). The result is kept in a small
 * handle read with orc_fai_single_get and released with orc_fai_single_free. */
fai *orc_fai_single(int n, const int *rp, const int *ci, const double *v, int kind, double tau,
                    int fill1, int fill2, int *status) {
    csr a;
    *status = csr_copy(n, rp, ci, v, &a);
    if (*status) return NULL;
    fai *S = calloc(1, sizeof(fai));
    if (kind == 1) *status = ainv_build(&a, tau, S);
    else if (kind == 2) *status = invk_build(&a, fill1, fill2, S);
    else *status = ORC_ERR_ARG;
    csr_free(&a);
    if (*status) { free(S); return NULL; }
    return S;
}

long long orc_fai_single_nnz(const fai *S) { return S->zr[S->n]; }

void orc_fai_single_get(const fai *S, int *zr, int *zi, double *zv, double *d) {
    memcpy(zr, S->zr, sizeof(int) * (size_t)(S->n + 1));
    memcpy(zi, S->zi, sizeof(int) * (size_t)S->zr[S->n]);
    memcpy(zv, S->zv, sizeof(double) * (size_t)S->zr[S->n]);
    memcpy(d, S->d, sizeof(double) * (size_t)S->n);
}

void orc_fai_single_free(fai *S) {
    if (!S) return;
    fai_free(S);
    free(S);
}

/* Coarsest-level solve in FP64: dense Cholesky, or l1-Jacobi sweeps from
 * x = 0 (x <- x + M^{-1}(b - A x)) when the hierarchy says so. */
/* The paper's coarsest solver in its tests (Section "Algorithmic tests"): at
 * most coarse_pcg iterations of CG preconditioned by l1-Jacobi, from x = 0,
 * stopped when ||r|| <= coarse_rtol ||b|| (the tolerance is a reading; the
 * paper gives only the iteration cap). Textbook PCG: z = M^-1 r, p = z,
 * alpha = (r.z)/(p.Ap), x += alpha p, r -= alpha Ap, beta = (r'.z')/(r.z),
 * p = z' + beta p; a non-positive p.Ap or r.z ends the iteration. */
static void coarse_pcg_solve(const orc_level *L, int maxit, double rtol, const double *b, double *x) {
    const int n = L->A.n;
    double *r = malloc(sizeof(double) * (size_t)n), *z = malloc(sizeof(double) * (size_t)n),
           *p = malloc(sizeof(double) * (size_t)n), *q = malloc(sizeof(double) * (size_t)n);
    for (int i = 0; i < n; i++) { x[i] = 0.0; r[i] = b[i]; }
    const double bn = sqrt(dot(n, b, b));
    if (bn > 0.0) {
        for (int i = 0; i < n; i++) { z[i] = L->minv[i] * r[i]; p[i] = z[i]; }
        double rz = dot(n, r, z);
        for (int it = 0; it < maxit && rz > 0.0; it++) {
            orc_spmv(n, L->A.rp, L->A.ci, L->A.v, p, q);
            const double pq = dot(n, p, q);
            if (!(pq > 0.0)) break;
            const double alpha = rz / pq;
            for (int i = 0; i < n; i++) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            if (sqrt(dot(n, r, r)) <= rtol * bn) break;
            for (int i = 0; i < n; i++) z[i] = L->minv[i] * r[i];
            const double rz2 = dot(n, r, z);
            const double beta = rz2 / rz;
            for (int i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
            rz = rz2;
        }
    }
    free(r); free(z); free(p); free(q);
}

static void coarse_solve(const orc_hier *h, const double *b, double *x) {
    const orc_level *L = &h->lev[h->nlev - 1];
    int n = L->A.n;
    if (h->coarse_pcg) { coarse_pcg_solve(L, h->coarse_pcg, h->coarse_rtol, b, x); return; }
    if (!h->coarse_sweeps) { chol_solve(n, L->L, b, x); return; }
    double *t = malloc(sizeof(double) * (size_t)n);
    for (int i = 0; i < n; i++) x[i] = 0.0;
    for (int k = 0; k < h->coarse_sweeps; k++) {
        orc_spmv(n, L->A.rp, L->A.ci, L->A.v, x, t);
        for (int i = 0; i < n; i++) x[i] += L->minv[i] * (b[i] - t[i]);
    }
    free(t);
}

/* ------------------------------------------------------------------------ */
/* Polynomial smoother (the paper names polynomial smoothers as GPU-friendly */
/* future work without fixing one). Reading: the fourth-kind Chebyshev      */
/* smoother of Lottes (2023, "Optimal polynomial smoothers for multigrid    */
/* V-cycles") on the l1-Jacobi preconditioned operator M^-1 A, with the     */
/* spectral bound rho = 1: A <= M holds for the l1 diagonal because M - A   */
/* is diagonally dominant with a non-negative diagonal. Degree nu (= the    */
/* sweep count) error propagation W_nu(I - 2 M^-1 A) / (2 nu + 1), W the    */
/* Chebyshev polynomial of the fourth kind.                                 */
/* ------------------------------------------------------------------------ */

/* x <- x + q(M^-1 A) M^-1 (b - A x) by the three-term recurrence
 *   r_0 = b - A x_0 (b when from_zero, x_0 = 0), d_0 = (4/3) M^-1 r_0,
 *   x_k = x_{k-1} + d_{k-1}, r_k = r_{k-1} - A d_{k-1},
 *   d_k = (2k-1)/(2k+3) d_{k-1} + (8k+4)/(2k+3) M^-1 r_k   (k = 1 .. nu-1),
 *   x_nu = x_{nu-1} + d_{nu-1}.
 * r, d, t: n-vectors of scratch. */
static void cheb4_smooth(const orc_level *L, int nu, const double *b, double *x, int from_zero,
                         double *r, double *d, double *t) {
    const int n = L->A.n;
    if (from_zero) {
        for (int i = 0; i < n; i++) { x[i] = 0.0; r[i] = b[i]; }
    } else {
        orc_spmv(n, L->A.rp, L->A.ci, L->A.v, x, t);
        for (int i = 0; i < n; i++) r[i] = b[i] - t[i];
    }
    for (int i = 0; i < n; i++) d[i] = (4.0 / 3.0) * L->minv[i] * r[i];
    for (int k = 1; k < nu; k++) {
        const double ak = (double)(2 * k - 1) / (double)(2 * k + 3);
        const double bk = (double)(8 * k + 4) / (double)(2 * k + 3);
        orc_spmv(n, L->A.rp, L->A.ci, L->A.v, d, t);
        for (int i = 0; i < n; i++) {
            x[i] += d[i];
            r[i] -= t[i];
            d[i] = ak * d[i] + bk * L->minv[i] * r[i];
        }
    }
    for (int i = 0; i < n; i++) x[i] += d[i];
}

/* The same in float: level values rounded to float, coefficients computed
 * in double and rounded to float. */
static void cheb4_smooth32(const orc_level *L, int nu, const float *b, float *x, int from_zero,
                           float *r, float *d, float *t) {
    const int n = L->A.n;
    if (from_zero) {
        for (int i = 0; i < n; i++) { x[i] = 0.0f; r[i] = b[i]; }
    } else {
        for (int i = 0; i < n; i++) {
            float s = 0.0f;
            for (int q = L->A.rp[i]; q < L->A.rp[i + 1]; q++) s += (float)L->A.v[q] * x[L->A.ci[q]];
            t[i] = s;
        }
        for (int i = 0; i < n; i++) r[i] = b[i] - t[i];
    }
    const float c0 = (float)(4.0 / 3.0);
    for (int i = 0; i < n; i++) d[i] = c0 * (float)L->minv[i] * r[i];
    for (int k = 1; k < nu; k++) {
        const float ak = (float)((double)(2 * k - 1) / (double)(2 * k + 3));
        const float bk = (float)((double)(8 * k + 4) / (double)(2 * k + 3));
        for (int i = 0; i < n; i++) {
            float s = 0.0f;
            for (int q = L->A.rp[i]; q < L->A.rp[i + 1]; q++) s += (float)L->A.v[q] * d[L->A.ci[q]];
            t[i] = s;
        }
        for (int i = 0; i < n; i++) {
            x[i] += d[i];
            r[i] -= t[i];
            d[i] = ak * d[i] + bk * (float)L->minv[i] * r[i];
        }
    }
    for (int i = 0; i < n; i++) x[i] += d[i];
}

/* The degree-nu smoother from x = 0 on one matrix, in FP64 (for the pins). */
void orc_cheb4_apply(int n, const int *rp, const int *ci, const double *v, int nu, const double *b, double *x) {
    orc_level L;
    memset(&L, 0, sizeof(L));
    csr_copy(n, rp, ci, v, &L.A);
    L.minv = malloc(sizeof(double) * (size_t)n);
    l1_diag_inv(&L.A, L.minv);
    double *r = malloc(sizeof(double) * (size_t)n), *d = malloc(sizeof(double) * (size_t)n),
           *t = malloc(sizeof(double) * (size_t)n);
    cheb4_smooth(&L, nu, b, x, 1, r, d, t);
    free(r); free(d); free(t); free(L.minv);
    csr_free(&L.A);
}

/* ------------------------------------------------------------------------ */
/* V-cycle (eq. amg, with nu sweeps): nu pre-sweeps from a zero guess,     */
/* coarse correction, nu post-sweeps; coarsest level by coarse_solve.       */
/* ------------------------------------------------------------------------ */

/* Smoothing sweeps on level l: nu, or nu * 2^l for the variable V-cycle
 * (capped at 4096 sweeps). */
static int level_sweeps(const orc_hier *h, int l) {
    if (!h->nu_double) return h->nu;
    int s = h->nu << (l < 12 ? l : 12);
    return s < 4096 ? s : 4096;
}

static void vcycle_level(const orc_hier *h, int l, const double *b, double *x) {
    const orc_level *L = &h->lev[l];
    int n = L->A.n;
    if (l == h->nlev - 1) { coarse_solve(h, b, x); return; }
    int nc = L->nc;
    const csr *P = &L->P;
    double *r = malloc(sizeof(double) * (size_t)n);
    double *bc = malloc(sizeof(double) * (size_t)nc);
    double *xc = malloc(sizeof(double) * (size_t)nc);
    /* pre-smoothing from x = 0: x = M^{-1} b, then nu_l - 1 sweeps
     * x += M^{-1} (b - A x); with AINV / INVK, M^{-1} is G = Z D^-1 Z^T */
    const int nu = level_sweeps(h, l);
    double *t = NULL, *y = NULL;
    if (h->smoother == 3) {
        /* polynomial smoother of degree nu from x = 0 (r, t, y as its scratch) */
        t = malloc(sizeof(double) * (size_t)n);
        y = malloc(sizeof(double) * (size_t)n);
        cheb4_smooth(L, nu, b, x, 1, r, t, y);
    } else if (L->S.n) {
        t = malloc(sizeof(double) * (size_t)n);
        y = malloc(sizeof(double) * (size_t)n);
        fai_apply(&L->S, b, x, y);
    } else {
        ORC_ROWS
        for (int i = 0; i < n; i++) x[i] = L->minv[i] * b[i];
    }
    for (int k = 1; k < nu && h->smoother != 3; k++) {
        orc_spmv(n, L->A.rp, L->A.ci, L->A.v, x, r);
        if (L->S.n) {
            ORC_ROWS
            for (int i = 0; i < n; i++) r[i] = b[i] - r[i];
            fai_apply(&L->S, r, t, y);
            ORC_ROWS
            for (int i = 0; i < n; i++) x[i] += t[i];
        } else {
            ORC_ROWS
            for (int i = 0; i < n; i++) x[i] += L->minv[i] * (b[i] - r[i]);
        }
    }
    /* residual r = b - A x */
    orc_spmv(n, L->A.rp, L->A.ci, L->A.v, x, r);
    ORC_ROWS
    for (int i = 0; i < n; i++) r[i] = b[i] - r[i];
    /* restriction b_c = P^T r (fine rows ascending, then row entries) */
    for (int I = 0; I < nc; I++) bc[I] = 0.0;
    for (int i = 0; i < n; i++)
        for (int m = P->rp[i]; m < P->rp[i + 1]; m++) bc[P->ci[m]] += P->v[m] * r[i];
    vcycle_level(h, l + 1, bc, xc);
    /* prolongation and correction x += P x_c */
    ORC_ROWS
    for (int i = 0; i < n; i++) {
        double s = 0.0;
        for (int m = P->rp[i]; m < P->rp[i + 1]; m++) s += P->v[m] * xc[P->ci[m]];
        x[i] += s;
    }
    /* nu_l post-smoothing sweeps x += M^{-1} (b - A x); the polynomial
     * smoother of degree nu from the corrected x */
    if (h->smoother == 3) cheb4_smooth(L, nu, b, x, 0, r, t, y);
    for (int k = 0; k < nu && h->smoother != 3; k++) {
        orc_spmv(n, L->A.rp, L->A.ci, L->A.v, x, r);
        if (L->S.n) {
            ORC_ROWS
            for (int i = 0; i < n; i++) r[i] = b[i] - r[i];
            fai_apply(&L->S, r, t, y);
            ORC_ROWS
            for (int i = 0; i < n; i++) x[i] += t[i];
        } else {
            ORC_ROWS
            for (int i = 0; i < n; i++) x[i] += L->minv[i] * (b[i] - r[i]);
        }
    }
    free(r); free(bc); free(xc); free(t); free(y);
}

void orc_vcycle(const orc_hier *h, const double *b, double *x) {
    vcycle_level(h, 0, b, x);
}

/*
 * The same V-cycle evaluated in FP32 (the mixed-precision form): the level
 * operators, prolongator values and l1 diagonals are the FP64 ones rounded
 * to nearest float, the input is rounded to float, every level operation is
 * done in float, the coarsest solve is done in FP64 on the float input
 * widened to double and rounded back to float, and the result is widened to
 * double.
 */
static void vcycle32_level(const orc_hier *h, int l, const float *b, float *x) {
    const orc_level *L = &h->lev[l];
    int n = L->A.n;
    if (l == h->nlev - 1) {
        double *bd = malloc(sizeof(double) * (size_t)n);
        double *xd = malloc(sizeof(double) * (size_t)n);
        for (int i = 0; i < n; i++) bd[i] = (double)b[i];
        coarse_solve(h, bd, xd);
        for (int i = 0; i < n; i++) x[i] = (float)xd[i];
        free(bd); free(xd);
        return;
    }
    int nc = L->nc;
    const csr *P = &L->P;
    float *r = malloc(sizeof(float) * (size_t)n);
    float *bc = malloc(sizeof(float) * (size_t)nc);
    float *xc = malloc(sizeof(float) * (size_t)nc);
    const int nu = level_sweeps(h, l);
    float *t = NULL, *y = NULL;
    if (h->smoother == 3) {
        t = malloc(sizeof(float) * (size_t)n);
        y = malloc(sizeof(float) * (size_t)n);
        cheb4_smooth32(L, nu, b, x, 1, r, t, y);
    } else if (L->S.n) {
        t = malloc(sizeof(float) * (size_t)n);
        y = malloc(sizeof(float) * (size_t)n);
        fai_apply32(&L->S, b, x, y);
    } else {
        ORC_ROWS
        for (int i = 0; i < n; i++) x[i] = (float)L->minv[i] * b[i];
    }
    for (int k = 1; k < nu && h->smoother != 3; k++) {
        ORC_ROWS
        for (int i = 0; i < n; i++) {
            float s = 0.0f;
            for (int q = L->A.rp[i]; q < L->A.rp[i + 1]; q++) s += (float)L->A.v[q] * x[L->A.ci[q]];
            r[i] = s;
        }
        if (L->S.n) {
            ORC_ROWS
            for (int i = 0; i < n; i++) r[i] = b[i] - r[i];
            fai_apply32(&L->S, r, t, y);
            ORC_ROWS
            for (int i = 0; i < n; i++) x[i] += t[i];
        } else {
            ORC_ROWS
            for (int i = 0; i < n; i++) x[i] += (float)L->minv[i] * (b[i] - r[i]);
        }
    }
    ORC_ROWS
    for (int i = 0; i < n; i++) {
        float s = 0.0f;
        for (int q = L->A.rp[i]; q < L->A.rp[i + 1]; q++) s += (float)L->A.v[q] * x[L->A.ci[q]];
        r[i] = b[i] - s;
    }
    for (int I = 0; I < nc; I++) bc[I] = 0.0f;
    for (int i = 0; i < n; i++)
        for (int m = P->rp[i]; m < P->rp[i + 1]; m++) bc[P->ci[m]] += (float)P->v[m] * r[i];
    vcycle32_level(h, l + 1, bc, xc);
    ORC_ROWS
    for (int i = 0; i < n; i++) {
        float s = 0.0f;
        for (int m = P->rp[i]; m < P->rp[i + 1]; m++) s += (float)P->v[m] * xc[P->ci[m]];
        x[i] += s;
    }
    if (h->smoother == 3) cheb4_smooth32(L, nu, b, x, 0, r, t, y);
    for (int k = 0; k < nu && h->smoother != 3; k++) {
        ORC_ROWS
        for (int i = 0; i < n; i++) {
            float s = 0.0f;
            for (int q = L->A.rp[i]; q < L->A.rp[i + 1]; q++) s += (float)L->A.v[q] * x[L->A.ci[q]];
            r[i] = s;
        }
        if (L->S.n) {
            ORC_ROWS
            for (int i = 0; i < n; i++) r[i] = b[i] - r[i];
            fai_apply32(&L->S, r, t, y);
            ORC_ROWS
            for (int i = 0; i < n; i++) x[i] += t[i];
        } else {
            ORC_ROWS
            for (int i = 0; i < n; i++) x[i] += (float)L->minv[i] * (b[i] - r[i]);
        }
    }
    free(r); free(bc); free(xc); free(t); free(y);
}

void orc_vcycle32(const orc_hier *h, const double *b, double *x) {
    int n = h->lev[0].A.n;
    float *bf = malloc(sizeof(float) * (size_t)n);
    float *xf = malloc(sizeof(float) * (size_t)n);
    ORC_ROWS
    for (int i = 0; i < n; i++) bf[i] = (float)b[i];
    vcycle32_level(h, 0, bf, xf);
    ORC_ROWS
    for (int i = 0; i < n; i++) x[i] = (double)xf[i];
    free(bf); free(xf);
}

/* ------------------------------------------------------------------------ */
/* Preconditioned CG (plain form)                                           */
/* ------------------------------------------------------------------------ */

#define ORC_PREC_VCYCLE 0
#define ORC_PREC_NONE 1
#define ORC_PREC_L1JACOBI 2
#define ORC_PREC_JACOBI 3
#define ORC_PREC_VCYCLE32 4

static void apply_prec(const orc_hier *h, int prec, const double *r, double *z) {
    const orc_level *L = &h->lev[0];
    int n = L->A.n;
    switch (prec) {
    case ORC_PREC_VCYCLE: orc_vcycle(h, r, z); break;
    case ORC_PREC_VCYCLE32: orc_vcycle32(h, r, z); break;
    case ORC_PREC_NONE: memcpy(z, r, sizeof(double) * (size_t)n); break;
    case ORC_PREC_L1JACOBI: for (int i = 0; i < n; i++) z[i] = L->minv[i] * r[i]; break;
    default: /* Jacobi with diag(A) */
        for (int i = 0; i < n; i++) {
            double d = 1.0;
            for (int k = L->A.rp[i]; k < L->A.rp[i + 1]; k++) if (L->A.ci[k] == i) d = L->A.v[k];
            z[i] = r[i] / d;
        }
    }
}

/*
 * PCG with x in/out as the initial guess. Stops when the recursive residual
 * satisfies ||r||_2 <= rtol ||b||_2 (Section "Numerical Example": relative
 * tolerance on the residual). relres is the true ||b - A x|| / ||b||.
 * hist (optional, 2*maxit doubles): alpha_k, beta_k of each iteration.
 */
int orc_pcg(const orc_hier *h, int prec, const double *b, double *x, double rtol,
            int maxit, int *iters, double *relres, double *hist) {
    const orc_level *L = &h->lev[0];
    int n = L->A.n;
    double nb = sqrt(dot(n, b, b));
    *iters = 0;
    if (isnan(nb) || isinf(nb)) return ORC_ERR_NAN;
    if (nb == 0.0) { for (int i = 0; i < n; i++) x[i] = 0.0; *relres = 0.0; return ORC_OK; }
    double *r = malloc(sizeof(double) * (size_t)n), *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n), *q = malloc(sizeof(double) * (size_t)n);
    orc_spmv(n, L->A.rp, L->A.ci, L->A.v, x, q);
    ORC_ROWS
    for (int i = 0; i < n; i++) r[i] = b[i] - q[i];
    int st = ORC_NOCONV, k = 0;
    if (sqrt(dot(n, r, r)) <= rtol * nb) st = ORC_OK;
    else {
        apply_prec(h, prec, r, z);
        memcpy(p, z, sizeof(double) * (size_t)n);
        double rho = dot(n, r, z);
        if (!(rho > 0.0)) st = isnan(rho) ? ORC_ERR_NAN : ORC_ERR_NOT_SPD;
        while (st == ORC_NOCONV && k < maxit) {
            orc_spmv(n, L->A.rp, L->A.ci, L->A.v, p, q);
            double pq = dot(n, p, q);
            if (!(pq > 0.0)) { st = isnan(pq) ? ORC_ERR_NAN : ORC_ERR_NOT_SPD; break; }
            double alpha = rho / pq;
            ORC_ROWS
            for (int i = 0; i < n; i++) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
            k++;
            double rr = dot(n, r, r);
            if (isnan(rr)) { st = ORC_ERR_NAN; break; }
            if (hist) hist[2 * (k - 1)] = alpha;
            if (sqrt(rr) <= rtol * nb) { st = ORC_OK; if (hist) hist[2 * (k - 1) + 1] = 0.0; break; }
            apply_prec(h, prec, r, z);
            double rho2 = dot(n, r, z);
            if (!(rho2 > 0.0)) { st = isnan(rho2) ? ORC_ERR_NAN : ORC_ERR_NOT_SPD; break; }
            double beta = rho2 / rho;
            if (hist) hist[2 * (k - 1) + 1] = beta;
            ORC_ROWS
            for (int i = 0; i < n; i++) p[i] = z[i] + beta * p[i];
            rho = rho2;
        }
    }
    *iters = k;
    orc_spmv(n, L->A.rp, L->A.ci, L->A.v, x, q);
    ORC_ROWS
    for (int i = 0; i < n; i++) r[i] = b[i] - q[i];
    *relres = sqrt(dot(n, r, r)) / nb;
    free(r); free(z); free(p); free(q);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Learned preconditioner: 3-layer 3x3x3 convolutional network              */
/* ------------------------------------------------------------------------ */
/*
 * Parity unpinned by the paper (the network is not part of it); pinned by
 * the tests against a library convolution, central finite differences and
 * closed-form Adam special cases.
 *
 * Parameters (C = 16 channels): W1[C][1][27] b1[C] W2[C][C][27] b2[C]
 * W3[1][C][27] b3[1]; tap t = (dz*3+dy)*3+dx acts at offset (dz-1,dy-1,dx-1).
 * A field of B samples, each D x H x W (x fastest), zero outside.
 *   h1 = GELU(conv1(u) + b1), h2 = GELU(conv2(h1) + b2), out = conv3(h2) + b3
 * GELU(t) = t * Phi(t) = 0.5 t (1 + erf(t / sqrt 2)).
 * With round_bf16 set, u, h1 and h2 (and the weights) are rounded to
 * bfloat16 (round to nearest even, via float) before the convolution that
 * reads them; sums are formed in double.
 */

#define NET_C 16
#define NET_P (NET_C * 27 + NET_C + NET_C * NET_C * 27 + NET_C + NET_C * 27 + 1)

int orc_net_param_count(void) { return NET_P; }

double orc_bf16(double x) {
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) {          /* inf / nan: truncate, keep nan quiet */
        if (u & 0x007fffffu) u |= 0x00400000u;
        u &= 0xffff0000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u += 0x7fffu + lsb;
        u &= 0xffff0000u;
    }
    memcpy(&f, &u, 4);
    return (double)f;
}

static double gelu(double t) { return 0.5 * t * (1.0 + erf(t / sqrt(2.0))); }
static double gelu_d(double t) {
    return 0.5 * (1.0 + erf(t / sqrt(2.0))) + t * exp(-0.5 * t * t) / sqrt(2.0 * M_PI);
}

/* out[co] = bias[co] + sum_ci sum_t W[co][ci][t] * in[ci](cell + off_t) */
static void conv3(int cin, int cout, const double *W, const double *bias,
                  int D, int H, int Wd, const double *in, double *out) {
    size_t cells = (size_t)D * H * Wd;
    for (int co = 0; co < cout; co++)
        for (int z = 0; z < D; z++)
            for (int y = 0; y < H; y++)
                for (int x = 0; x < Wd; x++) {
                    double s = bias ? bias[co] : 0.0;
                    for (int ci = 0; ci < cin; ci++)
                        for (int t = 0; t < 27; t++) {
                            int zz = z + t / 9 - 1, yy = y + (t / 3) % 3 - 1, xx = x + t % 3 - 1;
                            if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= Wd) continue;
                            s += W[((size_t)co * cin + ci) * 27 + t] *
                                 in[(size_t)ci * cells + ((size_t)zz * H + yy) * Wd + xx];
                        }
                    out[(size_t)co * cells + ((size_t)z * H + y) * Wd + x] = s;
                }
}

typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3;
    double *buf;    /* rounded weight copy */
} netw;

static void net_split(const double *params, int round_bf16, netw *nw) {
    nw->buf = malloc(sizeof(double) * NET_P);
    for (int i = 0; i < NET_P; i++) nw->buf[i] = round_bf16 ? orc_bf16(params[i]) : params[i];
    /* biases stay FP32-exact: only weight taps are rounded */
    const double *q = nw->buf;
    nw->W1 = q; q += NET_C * 27;
    nw->b1 = params + (q - nw->buf); q += NET_C;
    nw->W2 = q; q += NET_C * NET_C * 27;
    nw->b2 = params + (q - nw->buf); q += NET_C;
    nw->W3 = q; q += NET_C * 27;
    nw->b3 = params + (q - nw->buf);
}

/*
 * Forward pass for B samples of D x H x W. in: B*cells, out: B*cells.
 * act (optional, 2*B*C*cells + 2*B*C*cells doubles): pre-activations a1, a2
 * and rounded activations h1, h2 per sample, kept for the backward pass.
 */
void orc_net_forward(const double *params, int round_bf16, int B, int D, int H, int Wd,
                     const double *in, double *out, double *act) {
    size_t cells = (size_t)D * H * Wd;
    netw nw;
    net_split(params, round_bf16, &nw);
    double *u = malloc(sizeof(double) * cells);
    double *a1 = malloc(sizeof(double) * NET_C * cells), *h1 = malloc(sizeof(double) * NET_C * cells);
    double *a2 = malloc(sizeof(double) * NET_C * cells), *h2 = malloc(sizeof(double) * NET_C * cells);
    for (int b = 0; b < B; b++) {
        const double *ib = in + (size_t)b * cells;
        for (size_t c = 0; c < cells; c++) u[c] = round_bf16 ? orc_bf16(ib[c]) : ib[c];
        conv3(1, NET_C, nw.W1, nw.b1, D, H, Wd, u, a1);
        for (size_t c = 0; c < NET_C * cells; c++) {
            double g = gelu(a1[c]);
            h1[c] = round_bf16 ? orc_bf16(g) : g;
        }
        conv3(NET_C, NET_C, nw.W2, nw.b2, D, H, Wd, h1, a2);
        for (size_t c = 0; c < NET_C * cells; c++) {
            double g = gelu(a2[c]);
            h2[c] = round_bf16 ? orc_bf16(g) : g;
        }
        conv3(NET_C, 1, nw.W3, nw.b3, D, H, Wd, h2, out + (size_t)b * cells);
        if (act) {
            double *ab = act + (size_t)b * 4 * NET_C * cells;
            memcpy(ab, a1, sizeof(double) * NET_C * cells);
            memcpy(ab + NET_C * cells, h1, sizeof(double) * NET_C * cells);
            memcpy(ab + 2 * NET_C * cells, a2, sizeof(double) * NET_C * cells);
            memcpy(ab + 3 * NET_C * cells, h2, sizeof(double) * NET_C * cells);
        }
    }
    free(u); free(a1); free(h1); free(a2); free(h2); free(nw.buf);
}

/* gin[ci] += sum_co sum_t W[co][ci][t] * gout[co](cell - off_t) (transpose conv) */
static void conv3_dgrad(int cin, int cout, const double *W, int D, int H, int Wd,
                        const double *gout, double *gin) {
    size_t cells = (size_t)D * H * Wd;
    for (size_t c = 0; c < (size_t)cin * cells; c++) gin[c] = 0.0;
    for (int co = 0; co < cout; co++)
        for (int z = 0; z < D; z++)
            for (int y = 0; y < H; y++)
                for (int x = 0; x < Wd; x++) {
                    double g = gout[(size_t)co * cells + ((size_t)z * H + y) * Wd + x];
                    if (g == 0.0) continue;
                    for (int ci = 0; ci < cin; ci++)
                        for (int t = 0; t < 27; t++) {
                            int zz = z + t / 9 - 1, yy = y + (t / 3) % 3 - 1, xx = x + t % 3 - 1;
                            if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= Wd) continue;
                            gin[(size_t)ci * cells + ((size_t)zz * H + yy) * Wd + xx] +=
                                W[((size_t)co * cin + ci) * 27 + t] * g;
                        }
                }
}

/* gW[co][ci][t] += sum_cell gout[co](cell) * in[ci](cell + off_t); gb[co] += sum gout */
static void conv3_wgrad(int cin, int cout, int D, int H, int Wd, const double *in,
                        const double *gout, double *gW, double *gb) {
    size_t cells = (size_t)D * H * Wd;
    for (int co = 0; co < cout; co++)
        for (int z = 0; z < D; z++)
            for (int y = 0; y < H; y++)
                for (int x = 0; x < Wd; x++) {
                    double g = gout[(size_t)co * cells + ((size_t)z * H + y) * Wd + x];
                    gb[co] += g;
                    for (int ci = 0; ci < cin; ci++)
                        for (int t = 0; t < 27; t++) {
                            int zz = z + t / 9 - 1, yy = y + (t / 3) % 3 - 1, xx = x + t % 3 - 1;
                            if (zz < 0 || zz >= D || yy < 0 || yy >= H || xx < 0 || xx >= Wd) continue;
                            gW[((size_t)co * cin + ci) * 27 + t] +=
                                g * in[(size_t)ci * cells + ((size_t)zz * H + yy) * Wd + xx];
                        }
                }
}

/*
 * Loss and gradient: loss = mean over samples and interior cells (those at
 * least `margin` cells from every face) of (out - target)^2. The rounding
 * to bfloat16 is treated as the identity in the backward pass. grad (NET_P
 * doubles) receives d loss / d params. Returns the loss.
 */
double orc_net_loss_grad(const double *params, int round_bf16, int B, int D, int H, int Wd,
                         const double *in, const double *target, int margin, double *grad) {
    size_t cells = (size_t)D * H * Wd;
    double *out = malloc(sizeof(double) * (size_t)B * cells);
    double *act = malloc(sizeof(double) * (size_t)B * 4 * NET_C * cells);
    orc_net_forward(params, round_bf16, B, D, H, Wd, in, out, act);
    netw nw;
    net_split(params, round_bf16, &nw);
    size_t cnt = (size_t)B * (D - 2 * margin) * (H - 2 * margin) * (Wd - 2 * margin);
    double loss = 0.0;
    double *g3 = malloc(sizeof(double) * cells);
    double *g2 = malloc(sizeof(double) * NET_C * cells), *g1 = malloc(sizeof(double) * NET_C * cells);
    double *u = malloc(sizeof(double) * cells);
    if (grad) for (int i = 0; i < NET_P; i++) grad[i] = 0.0;
    double *gW1 = grad, *gb1 = grad ? grad + NET_C * 27 : NULL;
    double *gW2 = grad ? gb1 + NET_C : NULL, *gb2 = grad ? gW2 + NET_C * NET_C * 27 : NULL;
    double *gW3 = grad ? gb2 + NET_C : NULL, *gb3 = grad ? gW3 + NET_C * 27 : NULL;
    for (int b = 0; b < B; b++) {
        const double *ob = out + (size_t)b * cells, *tb = target + (size_t)b * cells;
        for (int z = 0; z < D; z++)
            for (int y = 0; y < H; y++)
                for (int x = 0; x < Wd; x++) {
                    size_t c = ((size_t)z * H + y) * Wd + x;
                    int in_ = z >= margin && z < D - margin && y >= margin && y < H - margin &&
                              x >= margin && x < Wd - margin;
                    double d = in_ ? ob[c] - tb[c] : 0.0;
                    loss += d * d;
                    g3[c] = 2.0 * d / (double)cnt;
                }
        if (!grad) continue;
        const double *ab = act + (size_t)b * 4 * NET_C * cells;
        const double *a1 = ab, *h1 = ab + NET_C * cells, *a2 = ab + 2 * NET_C * cells, *h2 = ab + 3 * NET_C * cells;
        conv3_wgrad(NET_C, 1, D, H, Wd, h2, g3, gW3, gb3);
        conv3_dgrad(NET_C, 1, nw.W3, D, H, Wd, g3, g2);
        for (size_t c = 0; c < NET_C * cells; c++) g2[c] *= gelu_d(a2[c]);
        conv3_wgrad(NET_C, NET_C, D, H, Wd, h1, g2, gW2, gb2);
        conv3_dgrad(NET_C, NET_C, nw.W2, D, H, Wd, g2, g1);
        for (size_t c = 0; c < NET_C * cells; c++) g1[c] *= gelu_d(a1[c]);
        const double *ib = in + (size_t)b * cells;
        for (size_t c = 0; c < cells; c++) u[c] = round_bf16 ? orc_bf16(ib[c]) : ib[c];
        conv3_wgrad(1, NET_C, D, H, Wd, u, g1, gW1, gb1);
    }
    free(out); free(act); free(g3); free(g2); free(g1); free(u); free(nw.buf);
    return loss / (double)cnt;
}

/*
 * One Adam step (t = 1-based step count): m = b1 m + (1-b1) g;
 * v = b2 v + (1-b2) g^2; p -= lr * (m/(1-b1^t)) / (sqrt(v/(1-b2^t)) + eps).
 */
void orc_adam_step(int np, double *p, double *m, double *v, const double *g, int t,
                   double lr, double b1, double b2, double eps) {
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int i = 0; i < np; i++) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
}

/* z = s * net(r / s), s = ||r||_2 / sqrt(N), on one nx x ny x nz grid. */
void orc_net_apply(const double *params, int nx, int ny, int nz, const double *r, double *z) {
    size_t N = (size_t)nx * ny * nz;
    double s = sqrt(dot((int)N, r, r) / (double)N);
    if (s == 0.0) { for (size_t i = 0; i < N; i++) z[i] = 0.0; return; }
    double *u = malloc(sizeof(double) * N);
    for (size_t i = 0; i < N; i++) u[i] = r[i] / s;
    orc_net_forward(params, 1, 1, nz, ny, nx, u, z, NULL);
    for (size_t i = 0; i < N; i++) z[i] *= s;
    free(u);
}

/* ------------------------------------------------------------------------ */
/* Flexible CG, FCG(1)                                                      */
/* ------------------------------------------------------------------------ */
/*
 * Flexible CG (Section "Numerical Example" uses FCG) with one stored
 * direction: z = B_k r; p = z - ((z.q_prev)/(p_prev.q_prev)) p_prev;
 * q = A p; alpha = (p.r)/(p.q); x += alpha p; r -= alpha q.
 * When the recursive residual passes ||r|| <= rtol ||b||, the true residual
 * b - A x is formed; if it also passes the solve ends, otherwise r is
 * replaced by it and the direction history restarts.
 *
 * B_k: form 0 = FP64 V-cycle, form 1 = FP32 V-cycle (orc_vcycle32).
 * With params != NULL (learned form), iterations k = 1, 3, 5, ... use the
 * network z = s net(r/s) instead; if z.r <= 0 that step takes the V-cycle
 * instead. The network is switched off for the rest of the solve when a
 * network step leaves ||r_new|| > 0.9 ||r_old|| (stagnation), or when two
 * network steps in a row fail z.r > 0. *fallbacks counts scheduled network
 * steps that ran the V-cycle instead, *net_evals the network applications.
 * form | ORC_ALT_JACOBI (comparison arm of the learned form, params unused):
 * the same schedule and rules with one l1-Jacobi sweep from zero on level 0,
 * z = M_0^-1 r, in place of the network.
 */
#define ORC_ALT_JACOBI 4
int orc_fcg(const orc_hier *h, int form, const double *params, int nx, int ny, int nz,
            const double *b, double *x, double rtol, int maxit, int *iters, double *relres,
            int *fallbacks, int *net_evals) {
    const orc_level *L = &h->lev[0];
    int n = L->A.n;
    double nb = sqrt(dot(n, b, b));
    *iters = 0;
    if (fallbacks) *fallbacks = 0;
    if (net_evals) *net_evals = 0;
    if (isnan(nb) || isinf(nb)) return ORC_ERR_NAN;
    if (nb == 0.0) { for (int i = 0; i < n; i++) x[i] = 0.0; *relres = 0.0; return ORC_OK; }
    const int alt_jacobi = (form & ORC_ALT_JACOBI) != 0;
    form &= 3;
    if (alt_jacobi) params = NULL;
    if (params && (size_t)nx * ny * nz != (size_t)n) return ORC_ERR_ARG;
    double *r = malloc(sizeof(double) * (size_t)n), *z = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n), *q = malloc(sizeof(double) * (size_t)n);
    double *pp = malloc(sizeof(double) * (size_t)n), *qp = malloc(sizeof(double) * (size_t)n);
    orc_spmv(n, L->A.rp, L->A.ci, L->A.v, x, q);
    ORC_ROWS
    for (int i = 0; i < n; i++) r[i] = b[i] - q[i];
    const int learned = params != NULL || alt_jacobi;
    int st = ORC_NOCONV, k = 0, have_prev = 0, net_on = learned, net_fails = 0;
    double pqp = 0.0;
    if (sqrt(dot(n, r, r)) <= rtol * nb) st = ORC_OK;
    while (st == ORC_NOCONV && k < maxit) {
        int use_net = net_on && (k % 2 == 1);
        int vform = form == 1 ? ORC_PREC_VCYCLE32 : ORC_PREC_VCYCLE;
        if (use_net) {
            if (alt_jacobi) {
                for (int i = 0; i < n; i++) z[i] = L->minv[i] * r[i];
            } else {
                orc_net_apply(params, nx, ny, nz, r, z);
            }
            if (net_evals) (*net_evals)++;
            if (!(dot(n, z, r) > 0.0)) {
                apply_prec(h, vform, r, z);
                use_net = 0;
                if (fallbacks) (*fallbacks)++;
                if (++net_fails >= 2) net_on = 0;
            } else {
                net_fails = 0;
            }
        } else {
            if (learned && !net_on && k % 2 == 1 && fallbacks) (*fallbacks)++;
            apply_prec(h, vform, r, z);
        }
        if (have_prev) {
            double beta = dot(n, z, qp) / pqp;
            ORC_ROWS
            for (int i = 0; i < n; i++) p[i] = z[i] - beta * pp[i];
        } else {
            memcpy(p, z, sizeof(double) * (size_t)n);
        }
        orc_spmv(n, L->A.rp, L->A.ci, L->A.v, p, q);
        double pq = dot(n, p, q);
        if (isnan(pq)) { st = ORC_ERR_NAN; break; }
        if (!(pq > 0.0)) { st = ORC_ERR_NOT_SPD; break; }
        double rr_old = dot(n, r, r);
        double alpha = dot(n, p, r) / pq;
        ORC_ROWS
        for (int i = 0; i < n; i++) { x[i] += alpha * p[i]; r[i] -= alpha * q[i]; }
        k++;
        double rr = dot(n, r, r);
        if (isnan(rr)) { st = ORC_ERR_NAN; break; }
        if (use_net && sqrt(rr) > 0.9 * sqrt(rr_old)) net_on = 0;
        memcpy(pp, p, sizeof(double) * (size_t)n);
        memcpy(qp, q, sizeof(double) * (size_t)n);
        pqp = pq;
        have_prev = 1;
        if (sqrt(rr) <= rtol * nb) {
            orc_spmv(n, L->A.rp, L->A.ci, L->A.v, x, q);
            ORC_ROWS
            for (int i = 0; i < n; i++) q[i] = b[i] - q[i];
            if (sqrt(dot(n, q, q)) <= rtol * nb) { st = ORC_OK; break; }
            memcpy(r, q, sizeof(double) * (size_t)n);
            have_prev = 0;
        }
    }
    *iters = k;
    orc_spmv(n, L->A.rp, L->A.ci, L->A.v, x, q);
    ORC_ROWS
    for (int i = 0; i < n; i++) r[i] = b[i] - q[i];
    *relres = sqrt(dot(n, r, r)) / nb;
    free(r); free(z); free(p); free(q); free(pp); free(qp);
    return st;
}
