// host_check.cpp -- CPU-only driver of the library's host-side setup code,
// for sanitizer builds (AddressSanitizer + UndefinedBehaviorSanitizer, and
// ThreadSanitizer for the OpenMP loops). Not part of libpsc.
//
// It replays, on the host, the build sequence of one process that builds
// several hierarchies in a row (the default matching hierarchy, then
// INVK(0,0), INVK(0,1), AINV, the smoothed prolongator and VBM), each
// followed by the host-side packing that the device upload performs (hacked
// ELL and DIA layouts, the tentative S P pattern, the smoothed S P, R = P^T)
// and a numeric rebuild. The GPU coarsening entry points are replaced by
// stubs that report "does not fit the device kernels", so the build takes
// the host path for every level (the device path computes the same results).
//
//   host_check <n> [repeats] [names]   3D Poisson 7-point on an n^3 grid;
//   names: comma-separated configurations to run (default: all)
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "setup.h"
#include "../../include/psc.h"

namespace psc {
int gpu_coarsen_level(int64_t, const int32_t*, const int32_t*, const double*, const double*, int, bool,
                      std::vector<int32_t>&, int64_t&, std::vector<double>&, std::vector<double>&,
                      std::vector<int32_t>&, std::vector<int32_t>&, std::vector<double>&, std::string& err) {
    err = "host check: no device";
    return PSC_ERR_STATE;
}
int gpu_smoothed_products(int64_t, const int32_t*, const int32_t*, const double*, const int32_t*, const double*,
                          int64_t, double&, std::vector<int32_t>&, std::vector<int32_t>&, std::vector<double>&,
                          std::vector<int32_t>&, std::vector<int32_t>&, std::vector<double>&,
                          std::vector<int32_t>&, std::vector<int32_t>&, std::vector<double>&, std::string& err) {
    err = "host check: no device";
    return PSC_ERR_STATE;
}
}  // namespace psc

using namespace psc;

static void poisson(int n, std::vector<int32_t>& rp, std::vector<int32_t>& ci, std::vector<double>& v) {
    const int64_t N = (int64_t)n * n * n;
    rp.assign(1, 0);
    ci.clear();
    v.clear();
    for (int64_t i = 0; i < N; i++) {
        const int x = (int)(i % n), y = (int)((i / n) % n), z = (int)(i / ((int64_t)n * n));
        const int64_t nb[7] = {z > 0 ? i - (int64_t)n * n : -1, y > 0 ? i - n : -1, x > 0 ? i - 1 : -1, i,
                               x + 1 < n ? i + 1 : -1, y + 1 < n ? i + n : -1,
                               z + 1 < n ? i + (int64_t)n * n : -1};
        for (int k = 0; k < 7; k++) {
            if (nb[k] < 0) continue;
            ci.push_back((int32_t)nb[k]);
            v.push_back(nb[k] == i ? 6.0 : -1.0);
        }
        rp.push_back((int32_t)ci.size());
    }
}

// the host-side packing of the device upload, level by level
static long long pack_levels(const HostHier& H) {
    long long sum = 0;
    for (size_t l = 0; l < H.lev.size(); l++) {
        const HostLevel& L = H.lev[l];
        std::vector<long long> off;
        std::vector<double> val;
        std::vector<int> col;
        pack_ell(L.n, L.rp.data(), L.ci.data(), L.v.data(), off, val, col);
        std::vector<int32_t> start, offs, uni;
        std::vector<double> dv;
        pack_dia(L.n, L.n, L.rp.data(), L.ci.data(), L.v.data(), off.back() * 4 / 3, start, offs, dv, &uni);
        sum += off.back() + (long long)dv.size();
        const int cap = choose_ell_cap(L.n, L.rp.data());
        if (cap > 0) {
            std::vector<long long> coff, xs, xsrc;
            std::vector<double> cval;
            std::vector<int> ccol, xc;
            std::vector<unsigned char> xl;
            pack_ell_capped(L.n, L.rp.data(), L.ci.data(), L.v.data(), cap, coff, cval, ccol, xs, xc, xl, xsrc);
            sum += coff.back() + (long long)xsrc.size();
        }
        if (l + 1 == H.lev.size()) break;
        std::vector<int32_t> sprp, spci;
        std::vector<double> spv;
        if ((int64_t)L.pci.size() == L.n) {
            tentative_sp_pattern(L, sprp, spci);
            sum += (long long)spci.size();
        }
        jacobi_smoothed_prolongator(L, L.minv.data(), sprp, spci, spv);
        sum += (long long)spv.size();
        std::vector<long long> poff;
        std::vector<double> pval;
        std::vector<int> pcol;
        pack_ell_paired(L.n, sprp.data(), spci.data(), spv.data(), poff, pval, pcol);
        sum += poff.back();
    }
    return sum;
}

// The capped hacked-ELL packing of rows whose lengths vary widely (a long row
// every 37 rows): every row's entries must come back, in CSR order, from its
// slots followed by its overflow record.
static int check_capped() {
    const int64_t n = 1000;
    std::vector<int32_t> rp(1, 0), ci;
    std::vector<double> v;
    for (int64_t i = 0; i < n; i++) {
        const int len = i % 37 == 5 ? 150 + (int)(i % 7) : 1 + (int)(i % 5);
        for (int k = 0; k < len; k++) {
            ci.push_back((int32_t)((i + 3 * k) % n));
            v.push_back(1.0 + (double)(i * 1000 + k));
        }
        rp.push_back((int32_t)ci.size());
    }
    const int cap = choose_ell_cap(n, rp.data());
    if (cap <= 0) {
        std::fprintf(stderr, "capped: no cap chosen for irregular rows\n");
        return 1;
    }
    std::vector<long long> off, xs, xsrc;
    std::vector<double> val;
    std::vector<int> col, xc;
    std::vector<unsigned char> xl;
    pack_ell_capped(n, rp.data(), ci.data(), v.data(), cap, off, val, col, xs, xc, xl, xsrc);
    for (int64_t i = 0; i < n; i++) {
        const int64_t s = i / 64;
        const int lane = (int)(i % 64);
        const int w = (int)((off[s + 1] - off[s]) / 64);
        std::vector<int> gc;
        std::vector<double> gv;
        for (int k = 0; k < w; k++) {
            const long long slot = off[s] + (long long)k * 64 + lane;
            if (k < rp[i + 1] - rp[i]) {
                gc.push_back(col[slot]);
                gv.push_back(val[slot]);
            } else if (val[slot] != 0.0) {
                std::fprintf(stderr, "capped: row %lld padding slot holds %g\n", (long long)i, val[slot]);
                return 1;
            }
        }
        int prev = -1;
        for (long long e = xs[s]; e < xs[s + 1]; e++) {
            if ((int)xl[e] < prev) {
                std::fprintf(stderr, "capped: slice %lld overflow not in lane order\n", (long long)s);
                return 1;
            }
            prev = xl[e];
            if (xl[e] != lane) continue;
            gc.push_back(xc[e]);
            gv.push_back(v[xsrc[e]]);
        }
        if ((int32_t)gc.size() != rp[i + 1] - rp[i]) {
            std::fprintf(stderr, "capped: row %lld has %zu entries, CSR %d\n", (long long)i, gc.size(), rp[i + 1] - rp[i]);
            return 1;
        }
        for (size_t k = 0; k < gc.size(); k++)
            if (gc[k] != ci[rp[i] + k] || gv[k] != v[rp[i] + k]) {
                std::fprintf(stderr, "capped: row %lld entry %zu differs\n", (long long)i, k);
                return 1;
            }
    }
    std::printf("capped layout: cap %d, %zu overflow entries, rows reproduced\n", cap, xc.size());
    return 0;
}

int main(int argc, char** argv) {
    if (check_capped()) return 1;
    const int n = argc > 1 ? std::atoi(argv[1]) : 32;
    const int reps = argc > 2 ? std::atoi(argv[2]) : 1;
    const std::string only = argc > 3 ? std::string(",") + argv[3] + "," : std::string();
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
    poisson(n, rp, ci, v);
    struct Cfg {
        const char* name;
        SetupOpts o;
    };
    std::vector<Cfg> cfgs;
    SetupOpts base;
    base.device = true;   // device path requested; the stubs send it to the host
    cfgs.push_back({"default", base});
    SetupOpts o = base;
    o.smoother = 2; o.fill1 = 0; o.fill2 = 0;
    cfgs.push_back({"invk00", o});
    o.fill2 = 1;
    cfgs.push_back({"invk01", o});
    o = base;
    o.smoother = 1; o.tau = 0.1;
    cfgs.push_back({"ainv", o});
    o = base;
    o.sweeps = 3; o.prol = 1; o.device_products = true;
    cfgs.push_back({"smatch", o});
    o = base;
    o.aggr = 1; o.prol = 1;
    cfgs.push_back({"vbm", o});
    for (int r = 0; r < reps; r++) {
        for (const Cfg& c : cfgs) {
            if (!only.empty() && only.find(std::string(",") + c.name + ",") == std::string::npos) continue;
            HostHier H;
            std::string err;
            int st = build_hierarchy((int64_t)n * n * n, rp.data(), ci.data(), v.data(), c.o, H, err);
            if (st != PSC_OK) {
                std::fprintf(stderr, "%s: build failed (%d): %s\n", c.name, st, err.c_str());
                return 1;
            }
            const long long packed = pack_levels(H);
            std::vector<double> v2(v);
            for (size_t k = 0; k < v2.size(); k++) v2[k] *= 1.0 + 0.25 * (double)(k % 3 == 0);
            // keep the matrix symmetric: scale rows and columns alike (s_i a_ij s_j)
            for (int64_t i = 0; i + 1 < (int64_t)rp.size(); i++)
                for (int32_t k = rp[i]; k < rp[i + 1]; k++) {
                    const double si = 1.0 + 0.25 * (double)(i % 3 == 0), sj = 1.0 + 0.25 * (double)(ci[k] % 3 == 0);
                    v2[k] = si * v[k] * sj;
                }
            st = rebuild_numeric(H, v2.data(), c.o, err);
            if (st != PSC_OK) {
                std::fprintf(stderr, "%s: rebuild failed (%d): %s\n", c.name, st, err.c_str());
                return 1;
            }
            std::printf("%s: %zu levels, packed %lld slots, rebuilt\n", c.name, H.lev.size(), packed);
            std::fflush(stdout);
        }
    }
    std::printf("host check ok\n");
    return 0;
}
