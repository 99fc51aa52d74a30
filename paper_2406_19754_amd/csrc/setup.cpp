// setup.cpp -- host-side construction of the matching-based AMG hierarchy.
//
// Follows the paper's Section "AMG4PSBLAS" (Galerkin coarse operators),
// Section "Aggregation strategies" (coupled aggregation by compatible
// weighted matching, tentative prolongator of eq. (prolongator), k matching
// sweeps) and Section "GPU enabled smoothers" (l1-Jacobi diagonal). The
// paper leaves the edge weights, the matching algorithm's tie order and the
// graph of later sweeps to its references; this file takes the readings:
//   * edge weight of {i,j} on the scaled operator S = diag(w) A diag(w):
//       c = 1 - 2 S_ij / (S_ii + S_jj), taken from the entry of the row
//       min(i,j), quantised q = llround(c 2^30); only q > 0 is eligible;
//   * the matching is the unique locally-dominant matching under the strict
//     order (q desc, min(i,j) asc, max(i,j) asc), a 1/2-approximate
//     maximum-weight matching; it is computed here by parallel rounds of
//     mutual "heaviest free neighbour" proposals;
//   * sweep s+1 matches the graph of the block sums of S over the aggregates
//     of sweep s; aggregates are numbered by ascending smallest member;
//   * w_{l+1}[I] = sqrt(sum_{i in I} w_i^2), p_i = w_i / w_{l+1}[agg_i];
//   * Galerkin sums C[I,J] = sum_{i in I asc} sum_{j in row i asc,
//     agg j = J} (s_i a_ij) s_j, with every reached (I,J) stored.
// Setup is not part of the solve time; it is parallel with OpenMP.
#include "setup.h"

#include <algorithm>
#include <iterator>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <omp.h>

#include "../../include/psc.h"

namespace psc {

namespace {

struct Csr {
    int64_t n = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
};

// exclusive prefix sum of cnt[0..n) into off[0..n], returns total
int64_t prefix(const std::vector<int64_t>& cnt, std::vector<int64_t>& off) {
    off.resize(cnt.size() + 1);
    off[0] = 0;
    for (size_t i = 0; i < cnt.size(); i++) off[i + 1] = off[i] + cnt[i];
    return off.back();
}

// Members of each aggregate in ascending order (counting sort, stable).
void members_of(const std::vector<int32_t>& agg, int64_t nc, std::vector<int64_t>& start,
                std::vector<int32_t>& mem) {
    std::vector<int64_t> cnt(nc, 0);
    for (size_t i = 0; i < agg.size(); i++) cnt[agg[i]]++;
    prefix(cnt, start);
    mem.resize(agg.size());
    std::vector<int64_t> pos(start.begin(), start.end() - 1);
    for (size_t i = 0; i < agg.size(); i++) mem[pos[agg[i]]++] = (int32_t)i;
}

// C = A B (B has ncols columns). Row i of C sums, for each stored a_ij in
// ascending j and then each entry (J, b_jJ) of row j of B in ascending J, the
// product a_ij b_jJ into C[i,J] in that arrival order; columns ascending,
// every reached entry stored.
void spgemm_raw(int64_t n, const int32_t* arp, const int32_t* aci, const double* av, const int32_t* brp,
                const int32_t* bci, const double* bv, int64_t ncols, Csr& C) {
    // Row i of C: the products a_ik b_kj in the order k ascending (row i of
    // A), then row k of B, summed per column j in that order (the first
    // product of a column assigns, later ones add); columns stored ascending.
    // A dense accumulator per thread keeps that order without sorting the
    // products; only the distinct columns are sorted.
    C.n = n;
    C.rp.assign(n + 1, 0);
#pragma omp parallel
    {
        std::vector<int64_t> tag(ncols, -1);
#pragma omp for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n; i++) {
            int32_t cnt = 0;
            for (int32_t k = arp[i]; k < arp[i + 1]; k++) {
                const int32_t j = aci[k];
                for (int32_t m = brp[j]; m < brp[j + 1]; m++)
                    if (tag[bci[m]] != i) {
                        tag[bci[m]] = i;
                        cnt++;
                    }
            }
            C.rp[i + 1] = cnt;
        }
    }
    for (int64_t i = 0; i < n; i++) C.rp[i + 1] += C.rp[i];
    C.ci.resize(C.rp[n]);
    C.v.resize(C.rp[n]);
#pragma omp parallel
    {
        std::vector<int64_t> tag(ncols, -1);
        std::vector<double> acc(ncols);
        std::vector<int32_t> cols;
#pragma omp for schedule(dynamic, 1024)
        for (int64_t i = 0; i < n; i++) {
            cols.clear();
            for (int32_t k = arp[i]; k < arp[i + 1]; k++) {
                const int32_t j = aci[k];
                for (int32_t m = brp[j]; m < brp[j + 1]; m++) {
                    const int32_t c = bci[m];
                    const double x = av[k] * bv[m];
                    if (tag[c] != i) {
                        tag[c] = i;
                        acc[c] = x;
                        cols.push_back(c);
                    } else {
                        acc[c] += x;
                    }
                }
            }
            std::sort(cols.begin(), cols.end());
            int64_t o = C.rp[i];
            for (int32_t c : cols) {
                C.ci[o] = c;
                C.v[o] = acc[c];
                o++;
            }
        }
    }
}

void spgemm(const Csr& A, const Csr& B, int64_t ncols, Csr& C) {
    (void)ncols;
    spgemm_raw(A.n, A.rp.data(), A.ci.data(), A.v.data(), B.rp.data(), B.ci.data(), B.v.data(), ncols, C);
}

// Transpose of an n x ncols CSR: row J lists (i, v_iJ) for i ascending.
void transpose(const Csr& P, int64_t ncols, Csr& R) {
    const int64_t n = P.n;
    R.n = ncols;
    R.rp.assign(ncols + 1, 0);
    for (int64_t m = 0; m < P.rp[n]; m++) R.rp[P.ci[m] + 1]++;
    for (int64_t J = 0; J < ncols; J++) R.rp[J + 1] += R.rp[J];
    R.ci.resize(P.rp[n]);
    R.v.resize(P.rp[n]);
    std::vector<int32_t> pos(R.rp.begin(), R.rp.end() - 1);
    for (int64_t i = 0; i < n; i++)
        for (int32_t m = P.rp[i]; m < P.rp[i + 1]; m++) {
            const int32_t o = pos[P.ci[m]]++;
            R.ci[o] = (int32_t)i;
            R.v[o] = P.v[m];
        }
}

// Galerkin sum in canonical order (see file header). s == nullptr means s = 1.
void galerkin(const Csr& a, const std::vector<int32_t>& agg, int64_t nc, const double* s,
              Csr& c) {
    std::vector<int64_t> start;
    std::vector<int32_t> mem;
    members_of(agg, nc, start, mem);
    std::vector<int64_t> len(nc, 0);
    // pass 1: row lengths; pass 2: values. A row's contributions are few, so
    // a short list with linear search keeps them in arrival order.
    for (int pass = 0; pass < 2; pass++) {
        std::vector<int64_t> off;
        if (pass == 1) {
            prefix(len, off);
            c.n = nc;
            c.rp.resize(nc + 1);
            for (int64_t I = 0; I <= nc; I++) c.rp[I] = (int32_t)off[I];
            c.ci.resize(off[nc]);
            c.v.resize(off[nc]);
        }
#pragma omp parallel
        {
            std::vector<int32_t> cols;
            std::vector<double> vals;
            std::vector<std::pair<int32_t, double>> tmp;
#pragma omp for schedule(dynamic, 4096)
            for (int64_t I = 0; I < nc; I++) {
                cols.clear();
                vals.clear();
                for (int64_t m = start[I]; m < start[I + 1]; m++) {
                    int32_t i = mem[m];
                    double si = s ? s[i] : 1.0;
                    for (int32_t k = a.rp[i]; k < a.rp[i + 1]; k++) {
                        int32_t j = a.ci[k];
                        int32_t J = agg[j];
                        double t = s ? (si * a.v[k]) * s[j] : a.v[k];
                        size_t q = 0;
                        while (q < cols.size() && cols[q] != J) q++;
                        if (q == cols.size()) { cols.push_back(J); vals.push_back(t); }
                        else vals[q] += t;
                    }
                }
                if (pass == 0) { len[I] = (int64_t)cols.size(); continue; }
                tmp.resize(cols.size());
                for (size_t q = 0; q < cols.size(); q++) tmp[q] = {cols[q], vals[q]};
                std::sort(tmp.begin(), tmp.end(),
                          [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                              return x.first < y.first;
                          });
                int64_t o = off[I];
                for (size_t q = 0; q < tmp.size(); q++) { c.ci[o + q] = tmp[q].first; c.v[o + q] = tmp[q].second; }
            }
        }
    }
}

// position of column j in row i (binary search), -1 if absent
inline int64_t find_col(const Csr& a, int32_t i, int32_t j) {
    const int32_t* b = a.ci.data() + a.rp[i];
    const int32_t* e = a.ci.data() + a.rp[i + 1];
    const int32_t* f = std::lower_bound(b, e, j);
    return (f != e && *f == j) ? (int64_t)(f - a.ci.data()) : -1;
}

// Strict edge order: does edge {i,a} with key qa come before {i,b} with key qb?
inline bool edge_first(int64_t qa, int32_t i, int32_t a, int64_t qb, int32_t b) {
    if (qa != qb) return qa > qb;
    int32_t amin = std::min(i, a), amax = std::max(i, a);
    int32_t bmin = std::min(i, b), bmax = std::max(i, b);
    if (amin != bmin) return amin < bmin;
    return amax < bmax;
}

// Locally-dominant matching of the graph of S. mate[i] = partner or -1.
void ld_matching(const Csr& S, std::vector<int32_t>& mate) {
    const int64_t n = S.n;
    const int64_t nnz = S.rp[n];
    std::vector<double> dg(n, 0.0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        int64_t k = find_col(S, (int32_t)i, (int32_t)i);
        dg[i] = k >= 0 ? S.v[k] : 0.0;
    }
    // key of each stored entry; the key of {i,j} is computed from the entry
    // of row min(i,j) so both rows see the same value
    std::vector<int64_t> key(nnz);
#pragma omp parallel for schedule(dynamic, 2048)
    for (int64_t i = 0; i < n; i++) {
        for (int32_t k = S.rp[i]; k < S.rp[i + 1]; k++) {
            int32_t j = S.ci[k];
            if (j == i) { key[k] = -1; continue; }
            int32_t lo = std::min<int32_t>((int32_t)i, j), hi = std::max<int32_t>((int32_t)i, j);
            int64_t kk = (j > i) ? k : find_col(S, lo, hi);
            if (kk < 0) { key[k] = -1; continue; }
            double sij = S.v[kk];
            double c = 1.0 - 2.0 * sij / (dg[lo] + dg[hi]);
            long long q = llround(c * 1073741824.0);
            key[k] = q > 0 ? (int64_t)q : -1;
        }
    }
    mate.assign(n, -1);
    std::vector<int32_t> cand(n, -1);
    auto best_free = [&](int64_t i) -> int32_t {
        int32_t best = -1;
        int64_t bq = 0;
        for (int32_t k = S.rp[i]; k < S.rp[i + 1]; k++) {
            if (key[k] < 0) continue;
            int32_t j = S.ci[k];
            if (mate[j] >= 0) continue;
            if (best < 0 || edge_first(key[k], (int32_t)i, j, bq, best)) { best = j; bq = key[k]; }
        }
        return best;
    };
    std::vector<int32_t> active(n);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; i++) { cand[i] = best_free(i); active[i] = (int32_t)i; }
    std::vector<uint8_t> is_active(n, 1), dirty(n, 0);
    int nt = omp_get_max_threads();
    std::vector<std::vector<int32_t>> tl_matched(nt), tl_dirty(nt);
    while (!active.empty()) {
        // 1) match mutual proposals among the active vertices
        int64_t na = (int64_t)active.size();
#pragma omp parallel
        {
            auto& out = tl_matched[omp_get_thread_num()];
            out.clear();
#pragma omp for schedule(static)
            for (int64_t t = 0; t < na; t++) {
                int32_t i = active[t];
                int32_t j = cand[i];
                if (j < 0 || cand[j] != i) continue;
                // record the pair once: by the smaller end, or by i if j is not active
                if (i < j || !is_active[j]) {
                    mate[i] = j;
                    mate[j] = i;
                    out.push_back(i);
                    out.push_back(j);
                }
            }
        }
        size_t newly = 0;
        for (auto& v : tl_matched) newly += v.size();
        for (int32_t i : active) is_active[i] = 0;
        if (newly == 0) break;
        // 2) free neighbours that proposed to a newly matched vertex re-propose
#pragma omp parallel
        {
            auto& out = tl_dirty[omp_get_thread_num()];
            out.clear();
            for (int t = 0; t < nt; t++) {
                const auto& ml = tl_matched[t];
#pragma omp for schedule(static) nowait
                for (int64_t q = 0; q < (int64_t)ml.size(); q++) {
                    int32_t m = ml[q];
                    for (int32_t k = S.rp[m]; k < S.rp[m + 1]; k++) {
                        int32_t u = S.ci[k];
                        if (mate[u] >= 0 || cand[u] != m) continue;
                        if (__atomic_exchange_n(&dirty[u], (uint8_t)1, __ATOMIC_RELAXED) == 0) out.push_back(u);
                    }
                }
            }
        }
        active.clear();
        for (auto& v : tl_dirty) active.insert(active.end(), v.begin(), v.end());
        int64_t nd = (int64_t)active.size();
#pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t t = 0; t < nd; t++) {
            int32_t u = active[t];
            cand[u] = best_free(u);
            dirty[u] = 0;
            is_active[u] = 1;
        }
    }
}

// Aggregates of a matching, numbered by ascending smallest member.
int64_t pairs_to_aggs(const std::vector<int32_t>& mate, std::vector<int32_t>& agg) {
    const int64_t n = (int64_t)mate.size();
    agg.assign(n, -1);
    int64_t nc = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t m = mate[i];
        if (m < 0 || m > i) agg[i] = (int32_t)nc++;
        else agg[i] = agg[m];
    }
    return nc;
}

// Decoupled Vanek-Mandel-Brezina aggregation (Section "Aggregation
// strategies"): j is strongly coupled to i when j != i and
// |a_ij| >= theta sqrt(a_ii a_jj). Sequential, ascending node order:
//   1. a node whose strong neighbours are all unaggregated forms an
//      aggregate with them;
//   2. each node still unaggregated joins the aggregate (from step 1) of its
//      strong neighbour with the largest |a_ij| (ties: smaller j);
//   3. each node still unaggregated forms an aggregate with its unaggregated
//      strong neighbours.
// Aggregates are numbered in order of creation.
void vbm_aggregate(const Csr& A, double theta, std::vector<int32_t>& agg, int64_t& nc_out) {
    const int64_t n = A.n;
    std::vector<double> d(n, 0.0);
    for (int64_t i = 0; i < n; i++)
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; k++)
            if (A.ci[k] == i) d[i] = A.v[k];
    auto strong = [&](int64_t i, int32_t k) {
        return A.ci[k] != i && std::fabs(A.v[k]) >= theta * std::sqrt(d[i] * d[A.ci[k]]);
    };
    agg.assign(n, -1);
    int32_t nc = 0;
    for (int64_t i = 0; i < n; i++) {
        if (agg[i] != -1) continue;
        bool free_all = true;
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; k++)
            if (strong(i, k) && agg[A.ci[k]] != -1) { free_all = false; break; }
        if (!free_all) continue;
        agg[i] = nc;
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; k++)
            if (strong(i, k)) agg[A.ci[k]] = nc;
        nc++;
    }
    const std::vector<int32_t> a1 = agg;
    for (int64_t i = 0; i < n; i++) {
        if (a1[i] != -1) continue;
        int32_t best = -1;
        double bv = -1.0;
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; k++) {
            if (!strong(i, k) || a1[A.ci[k]] == -1) continue;
            const double v = std::fabs(A.v[k]);
            if (v > bv) { bv = v; best = a1[A.ci[k]]; }
        }
        if (best != -1) agg[i] = best;
    }
    for (int64_t i = 0; i < n; i++) {
        if (agg[i] != -1) continue;
        agg[i] = nc;
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; k++)
            if (strong(i, k) && agg[A.ci[k]] == -1) agg[A.ci[k]] = nc;
        nc++;
    }
    nc_out = nc;
}

int coarsen(const Csr& A, const std::vector<double>& w, int sweeps, std::vector<int32_t>& agg,
            int64_t& nc_out) {
    const int64_t n = A.n;
    // S = diag(w) A diag(w), same pattern as A
    Csr S;
    S.n = n;
    S.rp = A.rp;
    S.ci = A.ci;
    S.v.resize(A.v.size());
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; i++)
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; k++) S.v[k] = (w[i] * A.v[k]) * w[A.ci[k]];
    agg.resize(n);
    for (int64_t i = 0; i < n; i++) agg[i] = (int32_t)i;
    int64_t ncur = n;
    for (int s = 0; s < sweeps; s++) {
        std::vector<int32_t> mate, a2;
        ld_matching(S, mate);
        int64_t nnew = pairs_to_aggs(mate, a2);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < n; i++) agg[i] = a2[agg[i]];
        if (s + 1 < sweeps) {
            Csr S2;
            galerkin(S, a2, nnew, nullptr, S2);
            S = std::move(S2);
        }
        ncur = nnew;
    }
    // explicit renumbering by ascending smallest level-l member
    std::vector<int32_t> ren(ncur, -1);
    int64_t nc = 0;
    for (int64_t i = 0; i < n; i++) {
        int32_t& r = ren[agg[i]];
        if (r < 0) r = (int32_t)nc++;
        agg[i] = r;
    }
    nc_out = nc;
    return PSC_OK;
}

int l1_inverse_diag(const Csr& A, std::vector<double>& minv) {
    minv.resize(A.n);
    std::atomic<int> bad(0);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < A.n; i++) {
        double d = 0.0, off = 0.0;
        bool has = false;
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; k++) {
            if (A.ci[k] == i) { d = A.v[k]; has = true; }
            else off += std::fabs(A.v[k]);
        }
        if (!has || !(d > 0.0)) { bad = 1; minv[i] = 0.0; }
        else minv[i] = 1.0 / (d + off);
    }
    return bad ? PSC_ERR_NOT_SPD : PSC_OK;
}

// Dense Cholesky of the coarsest matrix and its explicit inverse
// inv = L^-T L^-1 (applied as one matrix-vector product on the device).
int coarse_inverse(const Csr& A, std::vector<double>& inv) {
    const int64_t n = A.n;
    std::vector<double> L((size_t)n * n, 0.0);
    for (int64_t i = 0; i < n; i++)
        for (int32_t k = A.rp[i]; k < A.rp[i + 1]; k++)
            if (A.ci[k] <= i) L[(size_t)i * n + A.ci[k]] = A.v[k];
    for (int64_t j = 0; j < n; j++) {
        double d = L[(size_t)j * n + j];
        for (int64_t k = 0; k < j; k++) d -= L[(size_t)j * n + k] * L[(size_t)j * n + k];
        if (!(d > 0.0)) return PSC_ERR_NOT_SPD;
        double ljj = std::sqrt(d);
        L[(size_t)j * n + j] = ljj;
        for (int64_t i = j + 1; i < n; i++) {
            double s = L[(size_t)i * n + j];
            for (int64_t k = 0; k < j; k++) s -= L[(size_t)i * n + k] * L[(size_t)j * n + k];
            L[(size_t)i * n + j] = s / ljj;
        }
    }
    inv.assign((size_t)n * n, 0.0);
    std::vector<double> y(n);
    for (int64_t c = 0; c < n; c++) {
        for (int64_t i = 0; i < n; i++) {                 // L y = e_c
            double s = (i == c) ? 1.0 : 0.0;
            for (int64_t k = 0; k < i; k++) s -= L[(size_t)i * n + k] * y[k];
            y[i] = s / L[(size_t)i * n + i];
        }
        for (int64_t i = n - 1; i >= 0; i--) {            // L^T x = y
            double s = y[i];
            for (int64_t k = i + 1; k < n; k++) s -= L[(size_t)k * n + i] * y[k];
            y[i] = s / L[(size_t)i * n + i];
        }
        for (int64_t i = 0; i < n; i++) inv[(size_t)i * n + c] = y[i];
    }
    return PSC_OK;
}

// The numeric part of coarsening level l, given its aggregates F.agg and
// F.nc: the next sample vector, the tentative prolongator values, the
// prolongator the V-cycle uses (tentative or smoothed) and the Galerkin
// operator of level l + 1 (Cl). Shared by the build and the numeric rebuild.
void level_numeric(const Csr& A, const SetupOpts& o, HostLevel& F, HostLevel& Cl) {
    const int64_t nc = F.nc;
    Cl.n = nc;
    std::vector<int64_t> start;
    std::vector<int32_t> mem;
    members_of(F.agg, nc, start, mem);
    Cl.w.resize(nc);
    F.p.resize(F.n);
    if (o.aggr == 0) {
        // matching: P^ columns are the normalised restrictions of w
#pragma omp parallel for schedule(static)
        for (int64_t I = 0; I < nc; I++) {
            double s = 0.0;
            for (int64_t m = start[I]; m < start[I + 1]; m++) s += F.w[mem[m]] * F.w[mem[m]];
            Cl.w[I] = std::sqrt(s);
        }
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < F.n; i++) F.p[i] = F.w[i] / Cl.w[F.agg[i]];
    } else {
        // VBM, eq. (prolongator_vbm): P^_{i,agg_i} = w_i; the coarse sample is 1
        std::fill(Cl.w.begin(), Cl.w.end(), 1.0);
        for (int64_t i = 0; i < F.n; i++) F.p[i] = F.w[i];
    }
    Csr Ac;
    if (o.prol == 0) {
        // tentative: one entry per row, canonical Galerkin sum
        F.prp.resize(F.n + 1);
        for (int64_t i = 0; i <= F.n; i++) F.prp[i] = (int32_t)i;
        F.pci = F.agg;
        F.pv = F.p;
        galerkin(A, F.agg, nc, F.p.data(), Ac);
    } else if (o.device_products && [&] {
                   // the same products on the GPU (bit-identical); a row too wide
                   // for its kernels, or any device error, leaves them to the host
                   std::string derr;
                   return gpu_smoothed_products(A.n, A.rp.data(), A.ci.data(), A.v.data(), F.agg.data(),
                                                F.p.data(), nc, F.omega, F.prp, F.pci, F.pv, F.aprp, F.apci,
                                                F.apv, Ac.rp, Ac.ci, Ac.v, derr) == PSC_OK;
               }()) {
        Ac.n = nc;
    } else {
        // smoothed: omega = 1 / max_i sum_j |a_ij| / a_ii, then
        // P_iJ = [J = agg_i] p_i - (omega / a_ii) (A P^)_iJ and C = P^T (A P)
        double norm = 0.0;
        for (int64_t i = 0; i < A.n; i++) {
            double sabs = 0.0, aii = 0.0;
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; k++) {
                sabs += std::fabs(A.v[k]);
                if (A.ci[k] == i) aii = A.v[k];
            }
            if (sabs / aii > norm) norm = sabs / aii;
        }
        F.omega = 1.0 / norm;
        Csr Ph, T;
        Ph.n = F.n;
        Ph.rp.resize(F.n + 1);
        for (int64_t i = 0; i <= F.n; i++) Ph.rp[i] = (int32_t)i;
        Ph.ci = F.agg;
        Ph.v = F.p;
        spgemm(A, Ph, nc, T);
        Csr Pm;
        Pm.n = F.n;
        Pm.rp = T.rp;
        Pm.ci = T.ci;
        Pm.v.resize(T.v.size());
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < F.n; i++) {
            double aii = 0.0;
            for (int32_t k = A.rp[i]; k < A.rp[i + 1]; k++)
                if (A.ci[k] == i) aii = A.v[k];
            for (int32_t m = T.rp[i]; m < T.rp[i + 1]; m++) {
                const double pk = T.ci[m] == F.agg[i] ? F.p[i] : 0.0;
                Pm.v[m] = pk - (F.omega / aii) * T.v[m];
            }
        }
        Csr AP, R;
        spgemm(A, Pm, nc, AP);
        transpose(Pm, nc, R);
        spgemm(R, AP, nc, Ac);
        F.prp.swap(Pm.rp);
        F.pci.swap(Pm.ci);
        F.pv.swap(Pm.v);
        // kept for the split smoothing operator (I - M^-1 A) P
        F.aprp.swap(AP.rp);
        F.apci.swap(AP.ci);
        F.apv.swap(AP.v);
    }
    Cl.rp.swap(Ac.rp);
    Cl.ci.swap(Ac.ci);
    Cl.v.swap(Ac.v);
}

bool trace_on() {
    static const bool on = std::getenv("PSC_SETUP_TRACE") != nullptr;
    return on;
}

}  // namespace

PhaseTimer::PhaseTimer(const char* n) : name(n), t0(omp_get_wtime()) {}
PhaseTimer::~PhaseTimer() {
    if (trace_on()) std::fprintf(stderr, "[psc setup] %s %.3f\n", name, omp_get_wtime() - t0);
}

void pack_ell(int64_t nrows, const int32_t* rp, const int32_t* ci, const double* v,
              std::vector<long long>& off, std::vector<double>& val, std::vector<int>& col) {
    const int S = 64;
    int64_t ns = (nrows + S - 1) / S;
    off.assign(ns + 1, 0);
    std::vector<long long> width(ns, 0);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < ns; s++) {
        int wmax = 0;
        for (int64_t r = s * S; r < std::min<int64_t>(nrows, (s + 1) * S); r++)
            wmax = std::max(wmax, rp[r + 1] - rp[r]);
        width[s] = wmax;
    }
    for (int64_t s = 0; s < ns; s++) off[s + 1] = off[s] + width[s] * S;
    if (v) val.resize(off[ns]);
    else val.clear();
    col.resize(off[ns]);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < ns; s++) {
        int w = (int)width[s];
        for (int lane = 0; lane < S; lane++) {
            int64_t r = s * S + lane;
            int len = r < nrows ? rp[r + 1] - rp[r] : 0;
            int last = (r < nrows && len > 0) ? ci[rp[r + 1] - 1] : 0;
            for (int k = 0; k < w; k++) {
                long long slot = off[s] + (long long)k * S + lane;
                if (k < len) {
                    if (v) val[slot] = v[rp[r] + k];
                    col[slot] = ci[rp[r] + k];
                } else {
                    if (v) val[slot] = 0.0;
                    col[slot] = last;
                }
            }
        }
    }
}

void pack_ell_capped(int64_t nrows, const int32_t* rp, const int32_t* ci, const double* v, int cap,
                     std::vector<long long>& off, std::vector<double>& val, std::vector<int>& col,
                     std::vector<long long>& xs, std::vector<int>& xc, std::vector<unsigned char>& xl,
                     std::vector<long long>& xsrc) {
    const int S = 64;
    const int64_t ns = (nrows + S - 1) / S;
    off.assign(ns + 1, 0);
    xs.assign(ns + 1, 0);
    xc.clear();
    xl.clear();
    xsrc.clear();
    for (int64_t s = 0; s < ns; s++) {
        int w = 0;
        for (int64_t r = s * S; r < std::min<int64_t>(nrows, (s + 1) * S); r++) {
            const int len = rp[r + 1] - rp[r];
            w = std::max(w, std::min(len, cap));
            for (int32_t q = rp[r] + cap; q < rp[r + 1]; q++) {
                xc.push_back(ci[q]);
                xl.push_back((unsigned char)(r - s * S));
                xsrc.push_back(q);
            }
        }
        off[s + 1] = off[s] + (long long)w * S;
        xs[s + 1] = (long long)xc.size();
    }
    if (v) val.assign(off[ns], 0.0);
    else val.clear();
    col.resize(off[ns]);
#pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < ns; s++) {
        const int w = (int)((off[s + 1] - off[s]) / S);
        for (int lane = 0; lane < S; lane++) {
            const int64_t r = s * S + lane;
            const int len = r < nrows ? std::min(rp[r + 1] - rp[r], cap) : 0;
            const int last = (r < nrows && len > 0) ? ci[rp[r] + len - 1] : 0;
            for (int k = 0; k < w; k++) {
                const long long slot = off[s] + (long long)k * S + lane;
                if (k < len) {
                    if (v) val[slot] = v[rp[r] + k];
                    col[slot] = ci[rp[r] + k];
                } else {
                    col[slot] = last;
                }
            }
        }
    }
}

int choose_ell_cap(int64_t nrows, const int32_t* rp) {
    const int S = 64;
    const int64_t ns = (nrows + S - 1) / S;
    int wmax = 0;
    for (int64_t r = 0; r < nrows; r++) wmax = std::max(wmax, rp[r + 1] - rp[r]);
    if (wmax <= 8 || ns == 0) return 0;
    std::vector<int> len((size_t)ns * S, 0), sw(ns, 0);
    for (int64_t r = 0; r < nrows; r++) len[r] = rp[r + 1] - rp[r];
    long long plain = 0;
    for (int64_t s = 0; s < ns; s++) {
        for (int l = 0; l < S; l++) sw[s] = std::max(sw[s], len[s * S + l]);
        plain += sw[s];
    }
    long long best = plain;
    int best_cap = 0;
    for (int cap = 1; cap < wmax && cap <= 48; cap++) {
        long long c = 0;
        for (int64_t s = 0; s < ns && c < best; s++) {
            c += std::min(sw[s], cap);
            if (sw[s] <= cap) continue;
            long long e = 0;
            for (int l = 0; l < S; l++) e += std::max(0, len[s * S + l] - cap);
            c += 3 * ((e + S - 1) / S);
        }
        if (c < best) {
            best = c;
            best_cap = cap;
        }
    }
    return (best_cap > 0 && best * 10 <= plain * 9) ? best_cap : 0;
}

void pack_ell_paired(int64_t nrows, const int32_t* rp, const int32_t* ci, const double* v,
                     std::vector<long long>& off, std::vector<double>& val, std::vector<int>& col) {
    const int64_t ns = (nrows + 63) / 64, nb = (ns + 1) / 2;
    std::vector<long long> width(nb, 0), base(nb + 1, 0);
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; b++) {
        int wmax = 0;
        for (int64_t r = b * 128; r < std::min<int64_t>(nrows, (b + 1) * 128); r++)
            wmax = std::max(wmax, rp[r + 1] - rp[r]);
        width[b] = wmax;
    }
    for (int64_t b = 0; b < nb; b++) base[b + 1] = base[b] + width[b] * 128;
    off.assign(ns + 2, base[nb]);
    for (int64_t s = 0; s < ns; s++) off[s] = base[s >> 1] + (s & 1) * 64;
    if (v) val.resize(base[nb]);
    else val.clear();
    col.resize(base[nb]);
#pragma omp parallel for schedule(static)
    for (int64_t b = 0; b < nb; b++) {
        const int w = (int)width[b];
        for (int r = 0; r < 128; r++) {
            const int64_t row = b * 128 + r;
            const int len = row < nrows ? rp[row + 1] - rp[row] : 0;
            const int last = (row < nrows && len > 0) ? ci[rp[row + 1] - 1] : 0;
            for (int k = 0; k < w; k++) {
                const long long slot = base[b] + (long long)k * 128 + r;
                if (k < len) {
                    if (v) val[slot] = v[rp[row] + k];
                    col[slot] = ci[rp[row] + k];
                } else {
                    if (v) val[slot] = 0.0;
                    col[slot] = last;
                }
            }
        }
    }
}

int validate_csr(int64_t n, const int32_t* rp, const int32_t* ci, const double* v,
                 std::string& err) {
    if (n <= 0 || !rp || !ci || !v) { err = "n must be positive and arrays non-NULL"; return PSC_ERR_ARG; }
    if (rp[0] != 0) { err = "rowptr[0] must be 0"; return PSC_ERR_ARG; }
    for (int64_t i = 0; i < n; i++)
        if (rp[i + 1] < rp[i]) { err = "rowptr must be non-decreasing"; return PSC_ERR_ARG; }
    std::atomic<int> st(PSC_OK);
    std::atomic<int64_t> bad_row(-1);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; i++) {
        bool diag = false;
        int local = PSC_OK;
        for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
            int32_t j = ci[k];
            if (j < 0 || j >= n) { local = PSC_ERR_ARG; break; }
            if (k > rp[i] && ci[k - 1] >= j) { local = PSC_ERR_ARG; break; }
            if (!std::isfinite(v[k])) { local = PSC_ERR_ARG; break; }
            if (j == i) { diag = true; if (!(v[k] > 0.0)) local = PSC_ERR_NOT_SPD; }
        }
        if (local == PSC_OK && !diag) local = PSC_ERR_NOT_SPD;
        if (local != PSC_OK) { st = local; bad_row = i; }
    }
    if (st != PSC_OK) {
        err = (st == PSC_ERR_ARG ? "malformed CSR row " : "missing or non-positive diagonal in row ") +
              std::to_string(bad_row.load());
        return st;
    }
    // structural symmetry (the matching reads each edge from its upper entry)
    std::atomic<int64_t> asym(-1);
    Csr view;
    view.n = n;
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t i = 0; i < n; i++) {
        for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
            int32_t j = ci[k];
            const int32_t* b = ci + rp[j];
            const int32_t* e = ci + rp[j + 1];
            const int32_t* f = std::lower_bound(b, e, (int32_t)i);
            if (f == e || *f != i) { asym = i; break; }
        }
    }
    if (asym >= 0) {
        err = "matrix is not structurally symmetric (row " + std::to_string(asym.load()) + ")";
        return PSC_ERR_ARG;
    }
    return PSC_OK;
}

int build_hierarchy(int64_t n, const int32_t* rp, const int32_t* ci, const double* v,
                    const SetupOpts& o, HostHier& H, std::string& err) {
    if (o.sweeps < 1 || o.sweeps > 8 || o.coarse_max < 1 || o.max_levels < 1 ||
        o.max_levels > PSC_MAX_LEVELS || o.coarse_sweeps < 0 || o.coarse_sweeps > 1000 || o.aggr < 0 ||
        o.aggr > 1 || !(o.theta >= 0.0 && o.theta < 1.0) || o.smoother < 0 || o.smoother > 3 ||
        !(o.tau >= 0.0) || o.fill1 < 0 || o.fill1 > 64 || o.fill2 < 0 || o.fill2 > 64 || o.coarse_pcg < 0 ||
        o.coarse_pcg > 10000 || !(o.coarse_rtol >= 0.0)) {
        err = "invalid hierarchy options";
        return PSC_ERR_ARG;
    }
    H.lev.clear();
    H.lev.emplace_back();
    {
        HostLevel& L0 = H.lev[0];
        L0.n = n;
        L0.rp.assign(rp, rp + n + 1);
        L0.ci.assign(ci, ci + rp[n]);
        L0.v.assign(v, v + rp[n]);
        L0.w.assign(n, 1.0);
    }
    for (int l = 0;; l++) {
        Csr A;
        A.n = H.lev[l].n;
        A.rp.swap(H.lev[l].rp);
        A.ci.swap(H.lev[l].ci);
        A.v.swap(H.lev[l].v);
        int st = l1_inverse_diag(A, H.lev[l].minv);
        if (st != PSC_OK) { err = "non-positive l1 diagonal on level " + std::to_string(l); return st; }
        bool coarsest = (A.n <= o.coarse_max) || (l + 1 >= o.max_levels);
        bool stalled = l > 0 && (double)A.n > 0.9 * (double)H.lev[l - 1].n;
        if (stalled && A.n > 2000) {
            // Coarsening stalled above the dense-factor limit: this level is
            // the coarsest and is solved by a fixed number of l1-Jacobi sweeps.
            if (o.coarse_sweeps < 1) {
                err = "coarsening stalled at level " + std::to_string(l) + " with " + std::to_string(A.n) + " rows";
                return PSC_ERR_COARSEN;
            }
            H.lev[l].nc = 0;
            H.coarse_sweeps = o.coarse_sweeps;
            H.coarse_inv.clear();
            H.lev[l].rp.swap(A.rp);
            H.lev[l].ci.swap(A.ci);
            H.lev[l].v.swap(A.v);
            break;
        }
        if (coarsest || stalled) {
            if (A.n > 4096) { err = "coarsest level too large for a dense solve"; return PSC_ERR_COARSEN; }
            H.lev[l].nc = 0;
            H.coarse_sweeps = 0;
            H.coarse_pcg = o.coarse_pcg;
            H.coarse_rtol = o.coarse_rtol;
            if (o.coarse_pcg > 0) H.coarse_inv.clear();   // inexact PCG solve instead of the factor
            else st = coarse_inverse(A, H.coarse_inv);
            H.lev[l].rp.swap(A.rp);
            H.lev[l].ci.swap(A.ci);
            H.lev[l].v.swap(A.v);
            if (st != PSC_OK) { err = "Cholesky breakdown on the coarsest level"; return st; }
            break;
        }
        int64_t nc = 0;
        std::vector<int32_t> agg;
        bool have_agg = false;
        PhaseTimer pt_level("coarsen level (aggregation + numerics)");
        if (o.device && o.aggr == 0) {
            // matching on the GPU; with the tentative prolongator the whole
            // coarsening (the smoothed one takes the aggregates, its products
            // are formed below on the host)
            std::vector<double> gp, gwc, gcv;
            std::vector<int32_t> gcrp, gcci;
            st = gpu_coarsen_level(A.n, A.rp.data(), A.ci.data(), A.v.data(), H.lev[l].w.data(), o.sweeps,
                                   o.prol == 0, agg, nc, gp, gwc, gcrp, gcci, gcv, err);
            if (st == PSC_OK && o.prol != 0) {
                have_agg = true;
            } else if (st == PSC_OK) {
                H.lev.emplace_back();
                HostLevel& F = H.lev[l];
                HostLevel& Cl = H.lev[l + 1];
                F.nc = nc;
                F.agg.swap(agg);
                F.p.swap(gp);
                F.prp.resize(F.n + 1);
                for (int64_t i = 0; i <= F.n; i++) F.prp[i] = (int32_t)i;
                F.pci = F.agg;
                F.pv = F.p;
                Cl.n = nc;
                Cl.w.swap(gwc);
                Cl.rp.swap(gcrp);
                Cl.ci.swap(gcci);
                Cl.v.swap(gcv);
                F.rp.swap(A.rp);
                F.ci.swap(A.ci);
                F.v.swap(A.v);
                continue;
            }
            if (st != PSC_OK && st != PSC_ERR_STATE) return st;
            if (st != PSC_OK) err.clear();
        }
        if (!have_agg) {
            PhaseTimer pt("host aggregation");
            if (o.aggr == 0) coarsen(A, H.lev[l].w, o.sweeps, agg, nc);
            else vbm_aggregate(A, o.theta, agg, nc);
        }
        H.lev.emplace_back();
        HostLevel& F = H.lev[l];
        HostLevel& Cl = H.lev[l + 1];
        F.nc = nc;
        F.agg.swap(agg);
        {
            PhaseTimer pt("level numerics (prolongator, Galerkin)");
            level_numeric(A, o, F, Cl);
        }
        F.rp.swap(A.rp);
        F.ci.swap(A.ci);
        F.v.swap(A.v);
    }
    return build_smoothers(H, o, err);
}

int build_smoothers(HostHier& H, const SetupOpts& o, std::string& err) {
    PhaseTimer pt("smoother factors");
    // AINV / INVK smoothers of the levels above the coarsest
    if (o.smoother == 1 || o.smoother == 2) {
        for (size_t l = 0; l + 1 < H.lev.size(); l++) {
            HostLevel& F = H.lev[l];
            const int st = o.smoother == 1
                               ? build_ainv(F.n, F.rp.data(), F.ci.data(), F.v.data(), o.tau, F.fai, err)
                               : build_invk(F.n, F.rp.data(), F.ci.data(), F.v.data(), o.fill1, o.fill2, F.fai, err);
            if (st != PSC_OK) {
                err += " (level " + std::to_string(l) + ")";
                return st;
            }
        }
    }
    return PSC_OK;
}

int rebuild_numeric(HostHier& H, const double* v0, const SetupOpts& o, std::string& err) {
    const size_t L = H.lev.size();
    if (L == 0) {
        err = "empty hierarchy";
        return PSC_ERR_STATE;
    }
    {
        HostLevel& L0 = H.lev[0];
        const int64_t nnz = L0.rp[L0.n];
        for (int64_t i = 0; i < L0.n; i++) {
            bool diag = false;
            for (int32_t k = L0.rp[i]; k < L0.rp[i + 1]; k++) diag = diag || (L0.ci[k] == i && v0[k] > 0.0);
            if (!diag) {
                err = "row " + std::to_string(i) + " has no positive diagonal";
                return PSC_ERR_NOT_SPD;
            }
        }
        L0.v.assign(v0, v0 + nnz);
    }
    for (size_t l = 0; l < L; l++) {
        HostLevel& F = H.lev[l];
        Csr A;
        A.n = F.n;
        A.rp.swap(F.rp);
        A.ci.swap(F.ci);
        A.v.swap(F.v);
        int st = l1_inverse_diag(A, F.minv);
        if (st == PSC_OK && l + 1 == L && H.coarse_sweeps == 0 && H.coarse_pcg == 0)
            st = coarse_inverse(A, H.coarse_inv);
        if (st == PSC_OK && l + 1 < L) level_numeric(A, o, F, H.lev[l + 1]);
        F.rp.swap(A.rp);
        F.ci.swap(A.ci);
        F.v.swap(A.v);
        if (st != PSC_OK) {
            err = l + 1 == L ? "Cholesky breakdown on the coarsest level" : "non-positive l1 diagonal";
            return st;
        }
    }
    for (auto& F : H.lev) F.fai = HostFai();
    return build_smoothers(H, o, err);
}

// S P = (I - M^-1 A_l) P_l as CSR over the rows of A_l with aggregate
// columns: with (A P)_iJ from spgemm (ascending j, then row j of P),
//   sp_iJ = P_iJ - minv_i (A P)_iJ
// (the columns of row i of P are among those of row i of A P: a_ii is stored).
void jacobi_smoothed_prolongator(const HostLevel& H, const double* minv, std::vector<int32_t>& rp,
                                 std::vector<int32_t>& ci, std::vector<double>& v) {
    Csr T;
    if (!H.aprp.empty()) {
        // A P as formed by the level's Galerkin product (the same product)
        T.n = H.n;
        T.rp = H.aprp;
        T.ci = H.apci;
        T.v = H.apv;
    } else {
        spgemm_raw(H.n, H.rp.data(), H.ci.data(), H.v.data(), H.prp.data(), H.pci.data(), H.pv.data(), H.nc, T);
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < H.n; i++) {
        int32_t m = H.prp[i];
        for (int32_t k = T.rp[i]; k < T.rp[i + 1]; k++) {
            double pk = 0.0;
            if (m < H.prp[i + 1] && H.pci[m] == T.ci[k]) pk = H.pv[m++];
            T.v[k] = pk - minv[i] * T.v[k];
        }
    }
    rp.swap(T.rp);
    ci.swap(T.ci);
    v.swap(T.v);
}

void tentative_sp_pattern(const HostLevel& H, std::vector<int32_t>& rp, std::vector<int32_t>& ci) {
    const int64_t n = H.n;
    rp.assign(n + 1, 0);
    auto row = [&](int64_t i, int32_t* out) {
        // distinct aggregates of row i's columns, ascending (rows are short)
        int32_t cnt = 0;
        for (int32_t k = H.rp[i]; k < H.rp[i + 1]; k++) {
            const int32_t J = H.agg[H.ci[k]];
            int32_t q = 0;
            while (q < cnt && out[q] < J) q++;
            if (q < cnt && out[q] == J) continue;
            for (int32_t u = cnt; u > q; u--) out[u] = out[u - 1];
            out[q] = J;
            cnt++;
        }
        return cnt;
    };
    int32_t wmax = 0;
    for (int64_t i = 0; i < n; i++) wmax = std::max(wmax, H.rp[i + 1] - H.rp[i]);
#pragma omp parallel
    {
        std::vector<int32_t> buf(wmax + 1);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; i++) rp[i + 1] = row(i, buf.data());
    }
    for (int64_t i = 0; i < n; i++) rp[i + 1] += rp[i];
    ci.resize(rp[n]);
#pragma omp parallel
    {
        std::vector<int32_t> buf(wmax + 1);
#pragma omp for schedule(static)
        for (int64_t i = 0; i < n; i++) {
            const int32_t c = row(i, buf.data());
            std::copy(buf.begin(), buf.begin() + c, ci.begin() + rp[i]);
        }
    }
}

bool pack_dia(int64_t nrows, int64_t ncols, const int32_t* rp, const int32_t* ci, const double* v,
              long long max_slots, std::vector<int32_t>& start, std::vector<int32_t>& offs,
              std::vector<double>& val, std::vector<int32_t>* uniform) {
    start.clear();
    offs.clear();
    val.clear();
    if (uniform) uniform->clear();
    if (nrows + 64 + ncols >= (int64_t)1 << 30) return false;
    const int64_t ns = (nrows + 63) / 64;
    std::vector<int64_t> cnt(ns + 1, 0);
    auto slice_offsets = [&](int64_t s, std::vector<int32_t>& o) {
        o.clear();
        const int64_t r1 = std::min<int64_t>(nrows, (s + 1) * 64);
        for (int64_t i = s * 64; i < r1; i++)
            for (int32_t k = rp[i]; k < rp[i + 1]; k++) o.push_back((int32_t)(ci[k] - i));
        std::sort(o.begin(), o.end());
        o.erase(std::unique(o.begin(), o.end()), o.end());
    };
    // union of the slices' offsets (kept while it has at most 8 members)
    std::vector<int32_t> uni;
    bool uni_ok = uniform != nullptr;
#pragma omp parallel
    {
        std::vector<int32_t> o, mine;
        bool mine_ok = true;
#pragma omp for schedule(static)
        for (int64_t s = 0; s < ns; s++) {
            slice_offsets(s, o);
            cnt[s + 1] = (int64_t)o.size();
            if (mine_ok) {
                std::vector<int32_t> u;
                std::set_union(mine.begin(), mine.end(), o.begin(), o.end(), std::back_inserter(u));
                mine.swap(u);
                mine_ok = mine.size() <= 8;
            }
        }
#pragma omp critical
        {
            if (!mine_ok) uni_ok = false;
            if (uni_ok) {
                std::vector<int32_t> u;
                std::set_union(uni.begin(), uni.end(), mine.begin(), mine.end(), std::back_inserter(u));
                uni.swap(u);
                if (uni.size() > 8) uni_ok = false;
            }
        }
    }
    if (uni_ok && !uni.empty() && (int64_t)uni.size() * ns * 64 <= max_slots &&
        (int64_t)uni.size() * ns < ((int64_t)1 << 31)) {
        // uniform layout: every slice holds the union's diagonals
        const int64_t nd = (int64_t)uni.size();
        start.resize(ns + 1);
        for (int64_t s = 0; s <= ns; s++) start[s] = (int32_t)(s * nd);
        offs.resize(ns * nd);
        for (int64_t s = 0; s < ns; s++) std::copy(uni.begin(), uni.end(), offs.begin() + s * nd);
        *uniform = uni;
        if (!v) return true;
        val.assign((size_t)(ns * nd) * 64, 0.0);
#pragma omp parallel for schedule(static)
        for (int64_t s = 0; s < ns; s++) {
            const int64_t r1 = std::min<int64_t>(nrows, (s + 1) * 64);
            for (int64_t i = s * 64; i < r1; i++)
                for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
                    const int32_t d = (int32_t)(ci[k] - i);
                    const int64_t kk = std::lower_bound(uni.begin(), uni.end(), d) - uni.begin();
                    val[(size_t)(s * nd + kk) * 64 + (size_t)(i - s * 64)] = v[k];
                }
        }
        return true;
    }
    for (int64_t s = 0; s < ns; s++) cnt[s + 1] += cnt[s];
    if (cnt[ns] * 64 > max_slots || cnt[ns] >= ((int64_t)1 << 31)) return false;
    start.resize(ns + 1);
    for (int64_t s = 0; s <= ns; s++) start[s] = (int32_t)cnt[s];
    offs.resize(cnt[ns]);
    if (v) val.assign((size_t)cnt[ns] * 64, 0.0);
#pragma omp parallel
    {
        std::vector<int32_t> o;
#pragma omp for schedule(static)
        for (int64_t s = 0; s < ns; s++) {
            slice_offsets(s, o);
            std::copy(o.begin(), o.end(), offs.begin() + cnt[s]);
            if (!v) continue;
            const int64_t r1 = std::min<int64_t>(nrows, (s + 1) * 64);
            for (int64_t i = s * 64; i < r1; i++) {
                for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
                    const int32_t d = (int32_t)(ci[k] - i);
                    const int64_t kk = std::lower_bound(o.begin(), o.end(), d) - o.begin();
                    val[(size_t)(cnt[s] + kk) * 64 + (size_t)(i - s * 64)] = v[k];
                }
            }
        }
    }
    return true;
}

}  // namespace psc
