// fai.cpp -- host construction of the factored approximate inverse smoothers.
//
// Section "GPU enabled smoothers" names two smoothers besides l1-Jacobi that
// approximate A_l^-1 by sparse triangular factors, so that applying them
// needs only sparse matrix-vector products:
//   AINV: an incomplete A-biconjugation (the symmetric case, W = Z);
//   INVK: the inverse of the factors of an incomplete LDL^T decomposition.
// Both give G = Z D^-1 Z^T with Z unit upper triangular and D > 0 diagonal.
// The readings taken here (the paper defers the algorithms to its
// references):
//   * AINV is the stabilised biconjugation, pivots d_i = z_i^T A z_i (> 0
//     for SPD A); column k receives the updates z_k -= (z_i^T A z_k / d_i) z_i
//     of the steps i < k in ascending order, each followed by dropping the
//     entries r != k with |z_rk| sqrt(a_rr / a_kk) < tau (the tolerance acts
//     on the matrix scaled to unit diagonal); a zero coefficient skips the
//     step;
//   * INVK factors with level-of-fill fill1 (entry levels: 0 on the pattern
//     of A, lev(i,m) + lev(j,m) + 1 for fill through pivot m; each row's
//     pattern is fixed first, then eliminated), then inverts L^T on a
//     pattern limited by fill2: z_k = 1 at level -1, and entry r < k of
//     column k is kept when 1 + min over the entries j it is computed from
//     of their level is at most fill2.
// Every sum runs in a fixed order (ascending indices), so the factors are
// the same bit for bit on every run.
#include <algorithm>
#include <cmath>
#include <functional>
#include <queue>
#include <vector>

#include "setup.h"
#include "../../include/psc.h"

namespace psc {

namespace {

// Diagonal of a CSR matrix; false when an entry is missing or not positive.
bool positive_diagonal(int64_t n, const int32_t* rp, const int32_t* ci, const double* v, std::vector<double>& dg) {
    dg.assign(n, 0.0);
    for (int64_t i = 0; i < n; i++) {
        for (int32_t q = rp[i]; q < rp[i + 1]; q++)
            if (ci[q] == i) dg[i] = v[q];
        if (!(dg[i] > 0.0)) return false;
    }
    return true;
}

// Sparse accumulator: dense values with a membership flag and the list of
// members (in insertion order).
struct Spa {
    std::vector<double> val;
    std::vector<char> on;
    std::vector<int32_t> idx;
    explicit Spa(int64_t n) : val(n, 0.0), on(n, 0) { idx.reserve(64); }
    bool add(int32_t r) {
        if (on[r]) return false;
        on[r] = 1;
        val[r] = 0.0;
        idx.push_back(r);
        return true;
    }
    void clear() {
        for (int32_t r : idx) { on[r] = 0; val[r] = 0.0; }
        idx.clear();
    }
};

using MinHeap = std::priority_queue<int32_t, std::vector<int32_t>, std::greater<int32_t>>;

}  // namespace

int build_ainv(int64_t n, const int32_t* rp, const int32_t* ci, const double* v, double tau, HostFai& F,
               std::string& err) {
    std::vector<double> dg;
    if (!positive_diagonal(n, rp, ci, v, dg)) { err = "AINV: non-positive diagonal"; return PSC_ERR_NOT_SPD; }
    F.zr.assign(1, 0);
    F.zi.clear();
    F.zv.clear();
    F.d.assign(n, 0.0);
    // transpose structure of the finished columns: for row r the chain of
    // columns i with z_ri != 0 (first[r], then link[e])
    std::vector<int32_t> first(n, -1), link, owner;
    std::vector<int32_t> seen(n, -1);
    Spa z(n);
    MinHeap cand;
    // (A z)_r over row r in column order
    auto arow = [&](int32_t r) {
        double s = 0.0;
        for (int32_t q = rp[r]; q < rp[r + 1]; q++) s += v[q] * z.val[ci[q]];
        return s;
    };
    for (int64_t k = 0; k < n; k++) {
        const int32_t kk = (int32_t)k;
        int32_t step = -1;
        // queue every finished column i in (step, k) that has an entry in a
        // row adjacent to the new support index s
        auto reach = [&](int32_t s) {
            for (int32_t q = rp[s]; q < rp[s + 1]; q++)
                for (int32_t e = first[ci[q]]; e >= 0; e = link[e]) {
                    const int32_t i = owner[e];
                    if (i > step && i < kk && seen[i] != kk) { seen[i] = kk; cand.push(i); }
                }
        };
        z.add(kk);
        z.val[kk] = 1.0;
        reach(kk);
        while (!cand.empty()) {
            const int32_t i = cand.top();
            cand.pop();
            step = i;
            const int64_t b0 = F.zr[i], b1 = F.zr[i + 1];
            double p = 0.0;
            for (int64_t e = b0; e < b1; e++) p += F.zv[e] * arow(F.zi[e]);
            if (p == 0.0) continue;
            const double alpha = p / F.d[i];
            for (int64_t e = b0; e < b1; e++) {
                const int32_t r = F.zi[e];
                if (z.add(r)) reach(r);
                z.val[r] -= alpha * F.zv[e];
            }
            // drop on the unit-diagonal scale, never the diagonal itself
            size_t keep = 0;
            for (size_t t = 0; t < z.idx.size(); t++) {
                const int32_t r = z.idx[t];
                if (r != kk && std::fabs(z.val[r]) * std::sqrt(dg[r] / dg[kk]) < tau) {
                    z.on[r] = 0;
                    z.val[r] = 0.0;
                } else {
                    z.idx[keep++] = r;
                }
            }
            z.idx.resize(keep);
        }
        std::sort(z.idx.begin(), z.idx.end());
        double dk = 0.0;
        for (int32_t r : z.idx) dk += z.val[r] * arow(r);
        if (!(dk > 0.0)) { err = "AINV: non-positive pivot"; return PSC_ERR_NOT_SPD; }
        F.d[k] = dk;
        for (int32_t r : z.idx) {
            F.zi.push_back(r);
            F.zv.push_back(z.val[r]);
            link.push_back(first[r]);
            owner.push_back(kk);
            first[r] = (int32_t)(owner.size() - 1);
        }
        if (owner.size() > (size_t)INT32_MAX) { err = "AINV: factor too large"; return PSC_ERR_OOM; }
        F.zr.push_back((int64_t)F.zi.size());
        z.clear();
    }
    return PSC_OK;
}

int build_invk(int64_t n, const int32_t* rp, const int32_t* ci, const double* v, int fill1, int fill2,
               HostFai& F, std::string& err) {
    // L (unit lower, strictly lower part) by rows and by columns
    std::vector<int64_t> lrp(1, 0);
    std::vector<int32_t> lci;
    std::vector<double> lv;
    struct ColEntry {
        int32_t row;
        int32_t lev;
        double val;
    };
    std::vector<std::vector<ColEntry>> lcol(n);
    F.d.assign(n, 0.0);
    std::vector<double> w(n, 0.0);
    std::vector<int32_t> lev(n, 0);
    std::vector<char> on(n, 0);
    std::vector<int32_t> pat;
    MinHeap piv;
    for (int64_t i = 0; i < n; i++) {
        const int32_t ii = (int32_t)i;
        pat.clear();
        for (int32_t q = rp[i]; q < rp[i + 1]; q++) {
            const int32_t c = ci[q];
            if (c > ii) continue;
            w[c] = v[q];
            lev[c] = 0;
            on[c] = 1;
            pat.push_back(c);
            if (c < ii) piv.push(c);
        }
        if (!on[ii]) { err = "INVK: missing diagonal"; return PSC_ERR_NOT_SPD; }
        // symbolic: the final pattern and levels of row i
        while (!piv.empty()) {
            const int32_t m = piv.top();
            piv.pop();
            for (const ColEntry& e : lcol[m]) {
                const int32_t nl = lev[m] + e.lev + 1;
                if (on[e.row]) {
                    lev[e.row] = std::min(lev[e.row], nl);
                } else if (nl <= fill1) {
                    on[e.row] = 1;
                    w[e.row] = 0.0;
                    lev[e.row] = nl;
                    pat.push_back(e.row);
                    piv.push(e.row);
                }
            }
        }
        std::sort(pat.begin(), pat.end());
        // numeric elimination over that pattern, pivots ascending
        for (int32_t m : pat) {
            if (m == ii) break;
            const double lim = w[m] / F.d[m];
            w[m] = lim;
            for (const ColEntry& e : lcol[m])
                if (on[e.row]) w[e.row] -= lim * F.d[m] * e.val;
            w[ii] -= lim * F.d[m] * lim;
        }
        if (!(w[ii] > 0.0)) { err = "INVK: non-positive pivot in the incomplete factorisation"; return PSC_ERR_NOT_SPD; }
        F.d[i] = w[ii];
        for (int32_t m : pat) {
            if (m == ii) continue;
            lci.push_back(m);
            lv.push_back(w[m]);
            lcol[m].push_back(ColEntry{ii, lev[m], w[m]});
        }
        lrp.push_back((int64_t)lci.size());
        for (int32_t m : pat) { on[m] = 0; w[m] = 0.0; }
    }
    // Z = L^-T, column k by descending rows
    F.zr.assign(1, 0);
    F.zi.clear();
    F.zv.clear();
    std::priority_queue<int32_t> rows;   // largest first
    std::vector<int32_t> mark(n, -1);
    for (int64_t k = 0; k < n; k++) {
        const int32_t kk = (int32_t)k;
        pat.clear();
        w[kk] = 1.0;
        lev[kk] = -1;
        on[kk] = 1;
        pat.push_back(kk);
        for (int64_t e = lrp[k]; e < lrp[k + 1]; e++)
            if (mark[lci[e]] != kk) { mark[lci[e]] = kk; rows.push(lci[e]); }
        while (!rows.empty()) {
            const int32_t r = rows.top();
            rows.pop();
            double s = 0.0;
            int32_t lvl = INT32_MAX;
            for (const ColEntry& e : lcol[r]) {
                if (e.row > kk || !on[e.row]) continue;
                s += e.val * w[e.row];
                lvl = std::min(lvl, lev[e.row] + 1);
            }
            if (lvl > fill2) continue;
            w[r] = -s;
            lev[r] = lvl;
            on[r] = 1;
            pat.push_back(r);
            for (int64_t e = lrp[r]; e < lrp[r + 1]; e++)
                if (mark[lci[e]] != kk) { mark[lci[e]] = kk; rows.push(lci[e]); }
        }
        std::sort(pat.begin(), pat.end());
        for (int32_t r : pat) {
            F.zi.push_back(r);
            F.zv.push_back(w[r]);
        }
        F.zr.push_back((int64_t)F.zi.size());
        for (int32_t r : pat) { on[r] = 0; w[r] = 0.0; }
    }
    if (F.zi.size() > (size_t)INT32_MAX) { err = "INVK: factor too large"; return PSC_ERR_OOM; }
    return PSC_OK;
}

}  // namespace psc
