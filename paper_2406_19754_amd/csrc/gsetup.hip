// gsetup.hip -- coarsening of one hierarchy level on the GPU.
//
// Computes, for the default setting (coupled aggregation by compatible
// weighted matching with the tentative prolongator; Section "Aggregation
// strategies", eq. (prolongator); Section "AMG4PSBLAS" for the Galerkin
// product), exactly what the host functions coarsen(), the w/p loop and
// galerkin() in setup.cpp compute:
//   * matching keys q = llround((1 - 2 s_ij / (s_ii + s_jj)) 2^30) of the
//     scaled operator S = diag(w) A diag(w), and the unique locally-dominant
//     matching under the order (q desc, min asc, max asc), found by rounds of
//     mutual proposals in which only vertices whose partner was taken
//     propose again;
//   * aggregates numbered by ascending smallest member, k sweeps on the
//     block sums of S;
//   * w_{l+1}[I] = sqrt(sum over members ascending of w_i^2),
//     p_i = w_i / w_{l+1}[agg_i], and A_{l+1}[I,J] = sum over members i of I
//     ascending, then row entries ascending, of (p_i a_ij) p_j, with the
//     columns of a coarse row sorted.
// Every floating-point step is a separately rounded operation in the host's
// order (no contraction in this file), so the hierarchy is bit-identical to
// the host one.
// Member lists come from merging the sorted pairs of each sweep (an
// aggregate has at most 2^sweeps members); the only other primitive is an
// integer exclusive scan. Rows with more than GS_MAXC distinct coarse
// columns are reported so the caller can build that level on the host.
//
// For the smoothed prolongator (Section "Aggregation strategies", the
// prolongator smoothed by one damped Jacobi step) the level's products run
// here as well: omega = 1 / max_i sum_j |a_ij| / a_ii, T = A P^ and
// P = P^ - (omega / a_ii) T row by row, A P, R = P^T and the Galerkin
// operator R (A P), each sparse product summed as the host's: for row i the
// products a_ik b_kj for k ascending, then row k of B ascending, added into
// column j in that order (the first assigns), columns stored ascending.
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/psc.h"
#include "setup.h"

// This file is compiled with -ffp-contract=off (the rest of the library
// with contraction on): a multiply feeding an add must not become one fused
// operation here, or sums differ from the host's.

namespace psc {

namespace {

constexpr int GS_WG = 256;
constexpr int GS_MAXC = 64;      // distinct coarse columns one coarse row may collect

#define GS_CHK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess) {                                                       \
            err = std::string(#call) + ": " + hipGetErrorString(e_);                  \
            return PSC_ERR_HIP;                                                       \
        }                                                                             \
    } while (0)

__device__ __forceinline__ long long gs_llround(double x) {
    // round half away from zero: t = trunc(x) and |x - t| are exact
    const double t = trunc(x);
    long long r = (long long)t;
    if (fabs(__dsub_rn(x, t)) >= 0.5) r += x > 0.0 ? 1 : -1;
    return r;
}

// strict edge order of the matching: does {i,a} (key qa) come before {i,b} (key qb)?
__device__ __forceinline__ bool gs_edge_first(long long qa, int i, int a, long long qb, int b) {
    if (qa != qb) return qa > qb;
    const int amin = min(i, a), amax = max(i, a), bmin = min(i, b), bmax = max(i, b);
    if (amin != bmin) return amin < bmin;
    return amax < bmax;
}

__device__ __forceinline__ int gs_find(const int* rp, const int* ci, int i, int j) {
    int lo = rp[i], hi = rp[i + 1];
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (ci[mid] < j) lo = mid + 1;
        else hi = mid;
    }
    return (lo < rp[i + 1] && ci[lo] == j) ? lo : -1;
}

__global__ void k_gs_scale(int n, const int* rp, const int* ci, const double* v, const double* w, double* s) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int k = rp[i]; k < rp[i + 1]; k++) s[k] = __dmul_rn(__dmul_rn(w[i], v[k]), w[ci[k]]);
}

__global__ void k_gs_diag(int n, const int* rp, const int* ci, const double* v, double* dg) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int k = gs_find(rp, ci, i, i);
        dg[i] = k >= 0 ? v[k] : 0.0;
    }
}

// key of every stored entry, computed from the entry of row min(i,j)
__global__ void k_gs_keys(int n, const int* rp, const int* ci, const double* v, const double* dg, long long* key) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        for (int k = rp[i]; k < rp[i + 1]; k++) {
            const int j = ci[k];
            if (j == i) { key[k] = -1; continue; }
            const int lo = min(i, j), hi = max(i, j);
            const int kk = j > i ? k : gs_find(rp, ci, lo, hi);
            if (kk < 0) { key[k] = -1; continue; }
            const double c = __dsub_rn(1.0, __ddiv_rn(__dmul_rn(2.0, v[kk]), __dadd_rn(dg[lo], dg[hi])));
            const long long q = gs_llround(__dmul_rn(c, 1073741824.0));
            key[k] = q > 0 ? q : -1;
        }
    }
}

__device__ __forceinline__ int gs_best_free(int i, const int* rp, const int* ci, const long long* key,
                                            const int* mate) {
    int best = -1;
    long long bq = 0;
    for (int k = rp[i]; k < rp[i + 1]; k++) {
        if (key[k] < 0) continue;
        const int j = ci[k];
        if (mate[j] >= 0) continue;
        if (best < 0 || gs_edge_first(key[k], i, j, bq, best)) {
            best = j;
            bq = key[k];
        }
    }
    return best;
}

__global__ void k_gs_unmatch(int n, int* mate) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) mate[i] = -1;
}

__global__ void k_gs_cand_all(int n, const int* rp, const int* ci, const long long* key, const int* mate, int* cand) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        cand[i] = gs_best_free(i, rp, ci, key, mate);
}

// a free vertex whose proposed partner was taken proposes again (mate is
// not written in this kernel, so every vertex sees the same state)
__global__ void k_gs_propose(int n, const int* rp, const int* ci, const long long* key, const int* mate, int* cand) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (mate[i] >= 0) continue;
        const int c = cand[i];
        if (c >= 0 && mate[c] >= 0) cand[i] = gs_best_free(i, rp, ci, key, mate);
    }
}

// mutual proposals become matched pairs; the smaller end writes both mates
// (no other thread can write either entry: each vertex proposes to one)
__global__ void k_gs_match(int n, const int* cand, int* mate, int* count) {
    int local = 0;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        if (mate[i] >= 0) continue;
        const int u = cand[i];
        if (u > i && cand[u] == i) {
            mate[i] = u;
            mate[u] = i;
            local++;
        }
    }
    if (local) atomicAdd(count, local);
}

// ---- integer exclusive scan (three passes, fixed order: exact) ------------
__global__ void k_gs_scan_block(int n, const int* in, int* out, int* bsum) {
    __shared__ int sh[GS_WG];
    const int i = blockIdx.x * GS_WG + threadIdx.x;
    const int x = i < n ? in[i] : 0;
    sh[threadIdx.x] = x;
    __syncthreads();
    for (int o = 1; o < GS_WG; o <<= 1) {
        const int t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    if (i < n) out[i] = sh[threadIdx.x] - x;
    if (threadIdx.x == GS_WG - 1) bsum[blockIdx.x] = sh[GS_WG - 1];
}

__global__ void k_gs_scan_sums(int nb, int* bsum, int* total) {
    // one workgroup: sequential chunks, each scanned in shared memory
    __shared__ int sh[GS_WG];
    __shared__ int carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += GS_WG) {
        const int i = base + threadIdx.x;
        const int x = i < nb ? bsum[i] : 0;
        sh[threadIdx.x] = x;
        __syncthreads();
        for (int o = 1; o < GS_WG; o <<= 1) {
            const int t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) bsum[i] = carry + sh[threadIdx.x] - x;
        __syncthreads();
        if (threadIdx.x == 0) carry += sh[GS_WG - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *total = carry;
}

__global__ void k_gs_scan_add(int n, int* out, const int* bsum) {
    const int i = blockIdx.x * GS_WG + threadIdx.x;
    if (i < n) out[i] += bsum[blockIdx.x];
}

// ---- aggregates of one matching sweep --------------------------------------
__global__ void k_gs_rep(int n, const int* mate, int* rep) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        rep[i] = (mate[i] < 0 || mate[i] > i) ? 1 : 0;
}

// a2[v]: aggregate of vertex v (numbered by smallest member); first[I]: that member
__global__ void k_gs_pairs(int n, const int* mate, const int* scan, int* a2, int* first) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int m = mate[i];
        if (m < 0 || m > i) {
            a2[i] = scan[i];
            first[scan[i]] = i;
        } else {
            a2[i] = scan[m];
        }
    }
}

// fine members of the new aggregates: merge the sorted lists of the (one or
// two) vertices joined by the sweep; lists are padded with -1
__global__ void k_gs_merge(int nc, int stride, const int* first, const int* mate, const int* mem_in, int* mem_out) {
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < nc; I += gridDim.x * blockDim.x) {
        const int a = first[I], b = mate[a];
        const int* la = mem_in + (long long)a * stride;
        int* o = mem_out + (long long)I * 2 * stride;
        int x = 0, y = 0, k = 0;
        if (b < 0) {
            for (; x < stride; x++) o[k++] = la[x];
        } else {
            const int* lb = mem_in + (long long)b * stride;
            while (x < stride || y < stride) {
                const int va = x < stride ? la[x] : -1, vb = y < stride ? lb[y] : -1;
                if (va < 0 && vb < 0) break;
                if (vb < 0 || (va >= 0 && va < vb)) { o[k++] = va; x++; }
                else { o[k++] = vb; y++; }
            }
        }
        for (; k < 2 * stride; k++) o[k] = -1;
    }
}

__global__ void k_gs_compose(int n, int* agg, const int* a2) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) agg[i] = a2[agg[i]];
}

// w_{l+1} and p from the member lists
__global__ void k_gs_wp(int nc, int stride, const int* mem, const double* w, double* wc) {
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < nc; I += gridDim.x * blockDim.x) {
        double s = 0.0;
        for (int m = 0; m < stride; m++) {
            const int i = mem[(long long)I * stride + m];
            if (i < 0) break;
            s = __dadd_rn(s, __dmul_rn(w[i], w[i]));
        }
        wc[I] = __dsqrt_rn(s);
    }
}

__global__ void k_gs_p(int n, const double* w, const double* wc, const int* agg, double* p) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = __ddiv_rn(w[i], wc[agg[i]]);
}

// Galerkin product in the canonical order. Members of coarse row I come from
// mem (stride entries, -1 padded). s == nullptr: t = a_ij, else
// t = (s_i a_ij) s_j. pass 0 writes the row lengths, pass 1 the sorted row.
__global__ void k_gs_galerkin(int nc, int stride, const int* mem, const int* rp, const int* ci, const double* v,
                              const int* agg, const double* s, int pass, int* len, const int* crp, int* cci,
                              double* cv, int* overflow) {
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < nc; I += gridDim.x * blockDim.x) {
        int cols[GS_MAXC];
        double vals[GS_MAXC];
        int nq = 0;
        bool over = false;
        for (int m = 0; m < stride && !over; m++) {
            const int i = mem[(long long)I * stride + m];
            if (i < 0) break;
            const double si = s ? s[i] : 1.0;
            for (int k = rp[i]; k < rp[i + 1]; k++) {
                const int j = ci[k];
                const int J = agg[j];
                const double t = s ? __dmul_rn(__dmul_rn(si, v[k]), s[j]) : v[k];
                int q = 0;
                while (q < nq && cols[q] != J) q++;
                if (q == nq) {
                    if (nq == GS_MAXC) { over = true; break; }
                    cols[nq] = J;
                    vals[nq] = t;
                    nq++;
                } else {
                    vals[q] = __dadd_rn(vals[q], t);
                }
            }
        }
        if (over) {
            atomicOr(overflow, 1);
            if (pass == 0) len[I] = 0;
            continue;
        }
        if (pass == 0) {
            len[I] = nq;
            continue;
        }
        // insertion sort by column (columns are distinct)
        for (int x = 1; x < nq; x++) {
            const int c = cols[x];
            const double cvv = vals[x];
            int y = x - 1;
            while (y >= 0 && cols[y] > c) {
                cols[y + 1] = cols[y];
                vals[y + 1] = vals[y];
                y--;
            }
            cols[y + 1] = c;
            vals[y + 1] = cvv;
        }
        const int o = crp[I];
        for (int x = 0; x < nq; x++) {
            cci[o + x] = cols[x];
            cv[o + x] = vals[x];
        }
    }
}

__global__ void k_gs_pairs_members(int nc, const int* first, const int* mate, int* mem2) {
    for (int I = blockIdx.x * blockDim.x + threadIdx.x; I < nc; I += gridDim.x * blockDim.x) {
        const int a = first[I], b = mate[a];
        mem2[2 * I] = a;
        mem2[2 * I + 1] = b > a ? b : -1;
    }
}

__global__ void k_gs_iota(int n, int* mem) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) mem[i] = i;
}

// device buffer that frees itself
template <typename T>
struct DBuf {
    T* p = nullptr;
    ~DBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t count) {
        if (p) (void)hipFree(p);
        p = nullptr;
        return hipMalloc((void**)&p, (count > 0 ? count : 1) * sizeof(T));
    }
};

inline int gs_grid(long long n) {
    long long g = (n + GS_WG - 1) / GS_WG;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

// exclusive scan of in[0..n) into out, total into *total_host
int gs_scan(hipStream_t st, int n, const int* in, int* out, int& total_host, std::string& err) {
    const int nb = (n + GS_WG - 1) / GS_WG;
    DBuf<int> bsum, tot;
    GS_CHK(bsum.alloc(nb > 0 ? nb : 1));
    GS_CHK(tot.alloc(1));
    if (n > 0) k_gs_scan_block<<<nb, GS_WG, 0, st>>>(n, in, out, bsum.p);
    k_gs_scan_sums<<<1, GS_WG, 0, st>>>(nb, bsum.p, tot.p);
    if (n > 0) k_gs_scan_add<<<nb, GS_WG, 0, st>>>(n, out, bsum.p);
    GS_CHK(hipGetLastError());
    GS_CHK(hipMemcpyAsync(&total_host, tot.p, sizeof(int), hipMemcpyDeviceToHost, st));
    GS_CHK(hipStreamSynchronize(st));
    return PSC_OK;
}

// Galerkin product on the device; returns PSC_ERR_STATE when a coarse row
// collects more than GS_MAXC columns
int gs_galerkin(hipStream_t st, int nc, int stride, const int* mem, int n, const int* rp, const int* ci,
                const double* v, const int* agg, const double* s, DBuf<int>& crp, DBuf<int>& cci,
                DBuf<double>& cv, int& cnnz, std::string& err) {
    DBuf<int> len, over;
    GS_CHK(len.alloc(nc));
    GS_CHK(over.alloc(1));
    GS_CHK(hipMemsetAsync(over.p, 0, sizeof(int), st));
    k_gs_galerkin<<<gs_grid(nc), GS_WG, 0, st>>>(nc, stride, mem, rp, ci, v, agg, s, 0, len.p, nullptr, nullptr,
                                                 nullptr, over.p);
    GS_CHK(hipGetLastError());
    int ov = 0;
    GS_CHK(hipMemcpyAsync(&ov, over.p, sizeof(int), hipMemcpyDeviceToHost, st));
    GS_CHK(hipStreamSynchronize(st));
    if (ov) return PSC_ERR_STATE;
    GS_CHK(crp.alloc(nc + 1));
    int total = 0;
    int r = gs_scan(st, nc, len.p, crp.p, total, err);
    if (r) return r;
    GS_CHK(hipMemcpyAsync(crp.p + nc, &total, sizeof(int), hipMemcpyHostToDevice, st));
    GS_CHK(cci.alloc(total));
    GS_CHK(cv.alloc(total));
    k_gs_galerkin<<<gs_grid(nc), GS_WG, 0, st>>>(nc, stride, mem, rp, ci, v, agg, s, 1, nullptr, crp.p, cci.p,
                                                 cv.p, over.p);
    GS_CHK(hipGetLastError());
    GS_CHK(hipStreamSynchronize(st));
    cnnz = total;
    return PSC_OK;
}

constexpr int SG_CAP = 1024;            // distinct columns one product row may collect
constexpr int SG_WAVES = GS_WG / 64;
constexpr int SG_MAX_AROW = 64;        // longest operator row the device products take

// C = A B, one row per wavefront: the row's distinct columns and their sums
// in LDS, each product looked up by the whole wavefront (ballot) and added by
// one lane, in the order the products arrive. pass 0 writes the row lengths,
// pass 1 the row with its columns sorted (rank of each column). A row with
// more than SG_CAP columns sets *overflow.
__global__ __launch_bounds__(GS_WG) void k_sg_spgemm(int n, const int* __restrict__ arp, const int* __restrict__ aci,
                                                     const double* __restrict__ av, const int* __restrict__ brp,
                                                     const int* __restrict__ bci, const double* __restrict__ bv,
                                                     int pass, int* __restrict__ len, const int* __restrict__ crp,
                                                     int* __restrict__ cci, double* __restrict__ cv, int* overflow) {
    __shared__ int scol[SG_WAVES][SG_CAP];
    __shared__ double sval[SG_WAVES][SG_CAP];
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    int* cols = scol[wv];
    double* vals = sval[wv];
    for (int i = blockIdx.x * SG_WAVES + wv; i < n; i += gridDim.x * SG_WAVES) {
        int nq = 0;
        bool over = false;
        for (int ka = arp[i]; ka < arp[i + 1] && !over; ka++) {
            const int k = aci[ka];
            const double a = av[ka];
            for (int kb = brp[k]; kb < brp[k + 1]; kb++) {
                const int J = bci[kb];
                const double x = __dmul_rn(a, bv[kb]);
                int pos = -1;
                for (int base = 0; base < nq && pos < 0; base += 64) {
                    const int q = base + lane;
                    const unsigned long long m = __ballot(q < nq && cols[q] == J);
                    if (m) pos = base + __ffsll((long long)m) - 1;
                }
                if (pos >= 0) {
                    if (lane == 0) vals[pos] = __dadd_rn(vals[pos], x);
                } else if (nq == SG_CAP) {
                    over = true;
                    break;
                } else {
                    if (lane == 0) {
                        cols[nq] = J;
                        vals[nq] = x;
                    }
                    nq++;
                }
                // the next lookup reads what lane 0 wrote (one wavefront: in order)
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                __builtin_amdgcn_wave_barrier();
            }
        }
        if (over) {
            if (lane == 0) {
                atomicOr(overflow, 1);
                if (pass == 0) len[i] = 0;
            }
            continue;
        }
        if (pass == 0) {
            if (lane == 0) len[i] = nq;
            continue;
        }
        const int o = crp[i];
        for (int q = lane; q < nq; q += 64) {
            const int c = cols[q];
            int rank = 0;
            for (int u = 0; u < nq; u++) rank += cols[u] < c ? 1 : 0;
            cci[o + rank] = c;
            cv[o + rank] = vals[q];
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
}

// max over rows of sum_j |a_ij| / a_ii (positive values order like their bit
// patterns as signed integers; the host's maximum starts at 0 as well)
__global__ void k_sg_ratio(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                           const double* __restrict__ v, long long* maxbits) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double sabs = 0.0, aii = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; k++) {
            sabs = __dadd_rn(sabs, fabs(v[k]));
            if (ci[k] == i) aii = v[k];
        }
        const double r = sabs / aii;
        if (r > 0.0) atomicMax(maxbits, __double_as_longlong(r));
    }
}

// P = P^ - (omega / a_ii) T in place of T (T = A P^, same pattern)
__global__ void k_sg_pm(int n, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                        const int* __restrict__ agg, const double* __restrict__ p, double omega,
                        const int* __restrict__ trp, const int* __restrict__ tci, double* __restrict__ tv) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        double aii = 0.0;
        for (int k = rp[i]; k < rp[i + 1]; k++)
            if (ci[k] == i) aii = v[k];
        const double f = omega / aii;
        for (int m = trp[i]; m < trp[i + 1]; m++) {
            const double pk = tci[m] == agg[i] ? p[i] : 0.0;
            tv[m] = __dsub_rn(pk, __dmul_rn(f, tv[m]));
        }
    }
}

__global__ void k_sg_rows(int n, const int* __restrict__ rp, int* __restrict__ row) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        for (int m = rp[i]; m < rp[i + 1]; m++) row[m] = i;
}

__global__ void k_sg_count(int nnz, const int* __restrict__ col, int* __restrict__ cnt) {
    for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < nnz; m += gridDim.x * blockDim.x)
        atomicAdd(&cnt[col[m]], 1);
}

// R = P^T from the entries sorted stably by column: R row J lists the rows i
// of column J ascending
__global__ void k_sg_tfill(int nnz, const int* __restrict__ order, const int* __restrict__ row,
                           const double* __restrict__ pv, int* __restrict__ rci, double* __restrict__ rv) {
    for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < nnz; t += gridDim.x * blockDim.x) {
        const int m = order[t];
        rci[t] = row[m];
        rv[t] = pv[m];
    }
}

// S P = (I - M^-1 A) P for the tentative prolongator (one entry p_j at
// column agg_j in row j of P), in place in the build's hacked-ELL slots of S P:
// row i's columns are the distinct aggregates of its columns, ascending, so
// its length is their count; (A P)_iJ sums a_ij p_j over the row's entries
// ascending with agg_j = J (the first product assigns), as the host's sparse
// product does, and s_iJ = [J = agg_i] p_i - minv_i (A P)_iJ.
__global__ void k_gs_tentative_sp(long long n, const long long* __restrict__ a_off, const int* __restrict__ a_col,
                                  const double* __restrict__ a_val, const int32_t* __restrict__ a_rp,
                                  const int32_t* __restrict__ agg, const double* __restrict__ p,
                                  const double* __restrict__ minv, const long long* __restrict__ sp_off,
                                  const int* __restrict__ sp_col, double* __restrict__ sp_val,
                                  float* __restrict__ sp_val32, int sp_pair) {
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const long long s = i >> 6;
        const int lane = (int)(i & 63);
        const long long ao = a_off[s] + lane, so = sp_off[s] + lane;
        const int la = a_rp[i + 1] - a_rp[i];
        int ls = 0;
        for (int q = 0; q < la; q++) {
            const int J = agg[a_col[ao + (long long)q * 64]];
            bool first = true;
            for (int u = 0; u < q && first; u++) first = agg[a_col[ao + (long long)u * 64]] != J;
            ls += first ? 1 : 0;
        }
        // never past the slice (same pattern as at build); the paired layout
        // keeps one width per 128-row block and a slot stride of 128
        const int wsp = sp_pair ? (int)((sp_off[(s & ~1ll) + 2] - sp_off[s & ~1ll]) >> 7)
                                : (int)((sp_off[s + 1] - sp_off[s]) >> 6);
        const long long sstride = sp_pair ? 128 : 64;
        if (ls > wsp) ls = wsp;
        const int ai = agg[i];
        const double mi = minv[i];
        for (int q = 0; q < ls; q++) {
            const long long slot = so + (long long)q * sstride;
            const int J = sp_col[slot];
            double t = 0.0;
            bool any = false;
            for (int u = 0; u < la; u++) {
                const int c = a_col[ao + (long long)u * 64];
                if (agg[c] != J) continue;
                const double x = a_val[ao + (long long)u * 64] * p[c];
                t = any ? t + x : x;
                any = true;
            }
            const double pk = J == ai ? p[i] : 0.0;
            const double val = pk - mi * t;
            sp_val[slot] = val;
            if (sp_val32) sp_val32[slot] = (float)val;
        }
    }
}

inline int sg_grid(long long rows) {
    long long g = (rows + SG_WAVES - 1) / SG_WAVES;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

// C = A B on the device (row lengths, scan, rows); PSC_ERR_STATE when a row
// of C would collect more than SG_CAP columns
int sg_spgemm(hipStream_t st, int n, const int* arp, const int* aci, const double* av, const int* brp, const int* bci,
              const double* bv, DBuf<int>& crp, DBuf<int>& cci, DBuf<double>& cv, int& cnnz, std::string& err) {
    DBuf<int> len, over;
    GS_CHK(len.alloc(n));
    GS_CHK(over.alloc(1));
    GS_CHK(hipMemsetAsync(over.p, 0, sizeof(int), st));
    k_sg_spgemm<<<sg_grid(n), GS_WG, 0, st>>>(n, arp, aci, av, brp, bci, bv, 0, len.p, nullptr, nullptr, nullptr,
                                              over.p);
    GS_CHK(hipGetLastError());
    int ov = 0;
    GS_CHK(hipMemcpyAsync(&ov, over.p, sizeof(int), hipMemcpyDeviceToHost, st));
    GS_CHK(hipStreamSynchronize(st));
    if (ov) return PSC_ERR_STATE;
    GS_CHK(crp.alloc((size_t)n + 1));
    int total = 0;
    int r = gs_scan(st, n, len.p, crp.p, total, err);
    if (r) return r;
    if (total < 0) return PSC_ERR_STATE;
    GS_CHK(hipMemcpyAsync(crp.p + n, &total, sizeof(int), hipMemcpyHostToDevice, st));
    GS_CHK(cci.alloc(total));
    GS_CHK(cv.alloc(total));
    k_sg_spgemm<<<sg_grid(n), GS_WG, 0, st>>>(n, arp, aci, av, brp, bci, bv, 1, nullptr, crp.p, cci.p, cv.p, over.p);
    GS_CHK(hipGetLastError());
    GS_CHK(hipStreamSynchronize(st));
    cnnz = total;
    return PSC_OK;
}

template <typename T>
int sg_download(hipStream_t st, const DBuf<T>& d, size_t count, std::vector<T>& out, std::string& err) {
    out.resize(count);
    if (count) GS_CHK(hipMemcpyAsync(out.data(), d.p, count * sizeof(T), hipMemcpyDeviceToHost, st));
    return PSC_OK;
}

}  // namespace

int gpu_coarsen_level(int64_t n64, const int32_t* hrp, const int32_t* hci, const double* hv, const double* hw,
                      int sweeps, bool want_coarse, std::vector<int32_t>& agg_out, int64_t& nc_out,
                      std::vector<double>& p_out,
                      std::vector<double>& wc_out, std::vector<int32_t>& crp_out, std::vector<int32_t>& cci_out,
                      std::vector<double>& cv_out, std::string& err) {
    const int64_t nnz64 = hrp[n64];
    if (n64 >= ((int64_t)1 << 30) || nnz64 >= ((int64_t)1 << 31) || (sweeps < 1) || sweeps > 6) {
        err = "level too large for device coarsening";
        return PSC_ERR_STATE;
    }
    const int n = (int)n64, nnz = (int)nnz64;
    hipStream_t st;
    GS_CHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } guard{st};

    DBuf<int> rp, ci, agg;
    DBuf<double> v, w, S;
    GS_CHK(rp.alloc(n + 1));
    GS_CHK(ci.alloc(nnz));
    GS_CHK(v.alloc(nnz));
    GS_CHK(w.alloc(n));
    GS_CHK(S.alloc(nnz));
    GS_CHK(agg.alloc(n));
    GS_CHK(hipMemcpyAsync(rp.p, hrp, (n + 1) * sizeof(int), hipMemcpyHostToDevice, st));
    GS_CHK(hipMemcpyAsync(ci.p, hci, (size_t)nnz * sizeof(int), hipMemcpyHostToDevice, st));
    GS_CHK(hipMemcpyAsync(v.p, hv, (size_t)nnz * sizeof(double), hipMemcpyHostToDevice, st));
    GS_CHK(hipMemcpyAsync(w.p, hw, (size_t)n * sizeof(double), hipMemcpyHostToDevice, st));
    k_gs_scale<<<gs_grid(n), GS_WG, 0, st>>>(n, rp.p, ci.p, v.p, w.p, S.p);
    k_gs_iota<<<gs_grid(n), GS_WG, 0, st>>>(n, agg.p);

    // current matching graph (level rows at sweep 0, then block sums)
    const int* grp = rp.p;
    const int* gci = ci.p;
    const double* gv = S.p;
    int gn = n;
    DBuf<int> g2rp, g2ci, g3rp, g3ci;
    DBuf<double> g2v, g3v;
    // member lists of the current graph's vertices (stride 1: the rows themselves)
    DBuf<int> mem, mem2;
    GS_CHK(mem.alloc(n));
    k_gs_iota<<<gs_grid(n), GS_WG, 0, st>>>(n, mem.p);
    int stride = 1;
    int nc = n;
    DBuf<int> count;
    GS_CHK(count.alloc(1));
    int* hcount = nullptr;
    GS_CHK(hipHostMalloc((void**)&hcount, sizeof(int)));
    struct HostGuard {
        int* p;
        ~HostGuard() { (void)hipHostFree(p); }
    } hguard{hcount};

    for (int sw = 0; sw < sweeps; sw++) {
        DBuf<double> dg;
        DBuf<long long> key;
        DBuf<int> mate, cand, rep, scan, a2, first;
        int enz = 0;
        GS_CHK(hipMemcpyAsync(&enz, grp + gn, sizeof(int), hipMemcpyDeviceToHost, st));
        GS_CHK(hipStreamSynchronize(st));
        GS_CHK(dg.alloc(gn));
        GS_CHK(key.alloc(enz));
        GS_CHK(mate.alloc(gn));
        GS_CHK(cand.alloc(gn));
        k_gs_diag<<<gs_grid(gn), GS_WG, 0, st>>>(gn, grp, gci, gv, dg.p);
        k_gs_keys<<<gs_grid(gn), GS_WG, 0, st>>>(gn, grp, gci, gv, dg.p, key.p);
        k_gs_unmatch<<<gs_grid(gn), GS_WG, 0, st>>>(gn, mate.p);
        k_gs_cand_all<<<gs_grid(gn), GS_WG, 0, st>>>(gn, grp, gci, key.p, mate.p, cand.p);
        GS_CHK(hipGetLastError());
        // rounds: match mutual proposals, re-propose where the partner was taken
        for (int round = 0;; round++) {
            GS_CHK(hipMemsetAsync(count.p, 0, sizeof(int), st));
            k_gs_match<<<gs_grid(gn), GS_WG, 0, st>>>(gn, cand.p, mate.p, count.p);
            k_gs_propose<<<gs_grid(gn), GS_WG, 0, st>>>(gn, grp, gci, key.p, mate.p, cand.p);
            GS_CHK(hipMemcpyAsync(hcount, count.p, sizeof(int), hipMemcpyDeviceToHost, st));
            GS_CHK(hipStreamSynchronize(st));
            if (*hcount == 0) break;
            if (round > gn) {
                err = "device matching did not terminate";
                return PSC_ERR_HIP;
            }
        }
        // aggregates of this sweep, numbered by smallest member
        GS_CHK(rep.alloc(gn));
        GS_CHK(scan.alloc(gn));
        k_gs_rep<<<gs_grid(gn), GS_WG, 0, st>>>(gn, mate.p, rep.p);
        int nnew = 0;
        int r = gs_scan(st, gn, rep.p, scan.p, nnew, err);
        if (r) return r;
        GS_CHK(a2.alloc(gn));
        GS_CHK(first.alloc(nnew));
        k_gs_pairs<<<gs_grid(gn), GS_WG, 0, st>>>(gn, mate.p, scan.p, a2.p, first.p);
        k_gs_compose<<<gs_grid(n), GS_WG, 0, st>>>(n, agg.p, a2.p);
        GS_CHK(mem2.alloc((size_t)nnew * 2 * stride));
        k_gs_merge<<<gs_grid(nnew), GS_WG, 0, st>>>(nnew, stride, first.p, mate.p, mem.p, mem2.p);
        GS_CHK(hipGetLastError());
        std::swap(mem.p, mem2.p);
        stride *= 2;
        if (sw + 1 < sweeps) {
            // block sums of the matching graph for the next sweep (s = 1)
            DBuf<int> pm;
            GS_CHK(pm.alloc((size_t)nnew * 2));
            k_gs_pairs_members<<<gs_grid(nnew), GS_WG, 0, st>>>(nnew, first.p, mate.p, pm.p);
            DBuf<int>& orp = (sw % 2 == 0) ? g2rp : g3rp;
            DBuf<int>& oci = (sw % 2 == 0) ? g2ci : g3ci;
            DBuf<double>& ov = (sw % 2 == 0) ? g2v : g3v;
            int cnnz = 0;
            r = gs_galerkin(st, nnew, 2, pm.p, gn, grp, gci, gv, a2.p, nullptr, orp, oci, ov, cnnz, err);
            if (r) return r;
            grp = orp.p;
            gci = oci.p;
            gv = ov.p;
            gn = nnew;
        }
        nc = nnew;
    }
    // w_{l+1}, p and A_{l+1}
    DBuf<double> wc, p;
    GS_CHK(wc.alloc(nc));
    GS_CHK(p.alloc(n));
    k_gs_wp<<<gs_grid(nc), GS_WG, 0, st>>>(nc, stride, mem.p, w.p, wc.p);
    k_gs_p<<<gs_grid(n), GS_WG, 0, st>>>(n, w.p, wc.p, agg.p, p.p);
    GS_CHK(hipGetLastError());
    DBuf<int> crp, cci;
    DBuf<double> cv;
    int cnnz = 0;
    if (want_coarse) {
        int r = gs_galerkin(st, nc, stride, mem.p, n, rp.p, ci.p, v.p, agg.p, p.p, crp, cci, cv, cnnz, err);
        if (r) return r;
    }
    agg_out.resize(n);
    p_out.resize(n);
    wc_out.resize(nc);
    GS_CHK(hipMemcpyAsync(agg_out.data(), agg.p, (size_t)n * sizeof(int), hipMemcpyDeviceToHost, st));
    GS_CHK(hipMemcpyAsync(p_out.data(), p.p, (size_t)n * sizeof(double), hipMemcpyDeviceToHost, st));
    GS_CHK(hipMemcpyAsync(wc_out.data(), wc.p, (size_t)nc * sizeof(double), hipMemcpyDeviceToHost, st));
    if (want_coarse) {
        crp_out.resize(nc + 1);
        cci_out.resize(cnnz);
        cv_out.resize(cnnz);
        GS_CHK(hipMemcpyAsync(crp_out.data(), crp.p, (size_t)(nc + 1) * sizeof(int), hipMemcpyDeviceToHost, st));
        GS_CHK(hipMemcpyAsync(cci_out.data(), cci.p, (size_t)cnnz * sizeof(int), hipMemcpyDeviceToHost, st));
        GS_CHK(hipMemcpyAsync(cv_out.data(), cv.p, (size_t)cnnz * sizeof(double), hipMemcpyDeviceToHost, st));
    }
    GS_CHK(hipStreamSynchronize(st));
    nc_out = nc;
    return PSC_OK;
}


int gpu_tentative_sp(void* stream, int64_t n, const long long* a_off, const int* a_col, const double* a_val,
                     const int32_t* a_rp, const int32_t* agg, const double* p, const double* minv,
                     const long long* sp_off, const int* sp_col, double* sp_val, float* sp_val32, int sp_pair,
                     std::string& err) {
    hipStream_t st = (hipStream_t)stream;
    k_gs_tentative_sp<<<gs_grid(n), GS_WG, 0, st>>>(n, a_off, a_col, a_val, a_rp, agg, p, minv, sp_off, sp_col,
                                                     sp_val, sp_val32, sp_pair);
    GS_CHK(hipGetLastError());
    GS_CHK(hipStreamSynchronize(st));
    return PSC_OK;
}

int gpu_smoothed_products(int64_t n64, const int32_t* hrp, const int32_t* hci, const double* hv, const int32_t* hagg,
                          const double* hp, int64_t nc64, double& omega, std::vector<int32_t>& prp_out,
                          std::vector<int32_t>& pci_out, std::vector<double>& pv_out, std::vector<int32_t>& aprp_out,
                          std::vector<int32_t>& apci_out, std::vector<double>& apv_out,
                          std::vector<int32_t>& crp_out, std::vector<int32_t>& cci_out, std::vector<double>& cv_out,
                          std::string& err) {
    const int64_t nnz64 = hrp[n64];
    if (n64 >= ((int64_t)1 << 30) || nnz64 >= ((int64_t)1 << 31) || nc64 < 1 || nc64 > n64) {
        err = "level too large for device products";
        return PSC_ERR_STATE;
    }
    const int n = (int)n64, nnz = (int)nnz64, nc = (int)nc64;
    // wide operator rows make product rows too wide and slow for one
    // wavefront's sequential sums: those levels stay on the host
    for (int i = 0; i < n; i++)
        if (hrp[i + 1] - hrp[i] > SG_MAX_AROW) {
            err = "operator rows too wide for device products";
            return PSC_ERR_STATE;
        }
    hipStream_t st;
    GS_CHK(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));
    struct StreamGuard {
        hipStream_t s;
        ~StreamGuard() { (void)hipStreamDestroy(s); }
    } guard{st};
    DBuf<int> rp, ci, agg, iota;
    DBuf<double> v, p;
    GS_CHK(rp.alloc((size_t)n + 1));
    GS_CHK(ci.alloc(nnz));
    GS_CHK(v.alloc(nnz));
    GS_CHK(agg.alloc(n));
    GS_CHK(p.alloc(n));
    GS_CHK(iota.alloc((size_t)n + 1));
    GS_CHK(hipMemcpyAsync(rp.p, hrp, ((size_t)n + 1) * sizeof(int), hipMemcpyHostToDevice, st));
    GS_CHK(hipMemcpyAsync(ci.p, hci, (size_t)nnz * sizeof(int), hipMemcpyHostToDevice, st));
    GS_CHK(hipMemcpyAsync(v.p, hv, (size_t)nnz * sizeof(double), hipMemcpyHostToDevice, st));
    GS_CHK(hipMemcpyAsync(agg.p, hagg, (size_t)n * sizeof(int), hipMemcpyHostToDevice, st));
    GS_CHK(hipMemcpyAsync(p.p, hp, (size_t)n * sizeof(double), hipMemcpyHostToDevice, st));
    k_gs_iota<<<gs_grid((long long)n + 1), GS_WG, 0, st>>>(n + 1, iota.p);
    // omega = 1 / max_i sum_j |a_ij| / a_ii
    DBuf<long long> mb;
    GS_CHK(mb.alloc(1));
    GS_CHK(hipMemsetAsync(mb.p, 0, sizeof(long long), st));
    k_sg_ratio<<<gs_grid(n), GS_WG, 0, st>>>(n, rp.p, ci.p, v.p, mb.p);
    GS_CHK(hipGetLastError());
    long long bits = 0;
    GS_CHK(hipMemcpyAsync(&bits, mb.p, sizeof(long long), hipMemcpyDeviceToHost, st));
    GS_CHK(hipStreamSynchronize(st));
    double norm = 0.0;
    static_assert(sizeof(norm) == sizeof(bits), "64-bit double");
    std::memcpy(&norm, &bits, sizeof(norm));
    omega = 1.0 / norm;
    // T = A P^ (P^: row i holds p_i at column agg_i), then P in place
    DBuf<int> trp, tci;
    DBuf<double> tv;
    int tnnz = 0;
    int r = sg_spgemm(st, n, rp.p, ci.p, v.p, iota.p, agg.p, p.p, trp, tci, tv, tnnz, err);
    if (r) return r;
    k_sg_pm<<<gs_grid(n), GS_WG, 0, st>>>(n, rp.p, ci.p, v.p, agg.p, p.p, omega, trp.p, tci.p, tv.p);
    GS_CHK(hipGetLastError());
    // A P
    DBuf<int> aprp, apci;
    DBuf<double> apv;
    int apnnz = 0;
    r = sg_spgemm(st, n, rp.p, ci.p, v.p, trp.p, tci.p, tv.p, aprp, apci, apv, apnnz, err);
    if (r) return r;
    // R = P^T: entries sorted stably by column keep their rows ascending
    DBuf<int> row, keys_out, order, idx, cnt, rrp, rci;
    DBuf<double> rv;
    GS_CHK(row.alloc(tnnz));
    GS_CHK(keys_out.alloc(tnnz));
    GS_CHK(order.alloc(tnnz));
    GS_CHK(idx.alloc(tnnz));
    GS_CHK(cnt.alloc(nc));
    GS_CHK(rrp.alloc((size_t)nc + 1));
    GS_CHK(rci.alloc(tnnz));
    GS_CHK(rv.alloc(tnnz));
    k_sg_rows<<<gs_grid(n), GS_WG, 0, st>>>(n, trp.p, row.p);
    k_gs_iota<<<gs_grid(tnnz), GS_WG, 0, st>>>(tnnz, idx.p);
    GS_CHK(hipMemsetAsync(cnt.p, 0, (size_t)nc * sizeof(int), st));
    k_sg_count<<<gs_grid(tnnz), GS_WG, 0, st>>>(tnnz, tci.p, cnt.p);
    GS_CHK(hipGetLastError());
    int end_bit = 1;
    while (end_bit < 31 && ((int64_t)1 << end_bit) < nc64) end_bit++;
    size_t tmp_bytes = 0;
    GS_CHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, tci.p, keys_out.p, idx.p, order.p, tnnz, 0, end_bit,
                                             st));
    DBuf<char> tmp;
    GS_CHK(tmp.alloc(tmp_bytes));
    GS_CHK(hipcub::DeviceRadixSort::SortPairs(tmp.p, tmp_bytes, tci.p, keys_out.p, idx.p, order.p, tnnz, 0, end_bit,
                                             st));
    int rtotal = 0;
    r = gs_scan(st, nc, cnt.p, rrp.p, rtotal, err);
    if (r) return r;
    if (rtotal != tnnz) {
        err = "device transpose lost entries";
        return PSC_ERR_HIP;
    }
    GS_CHK(hipMemcpyAsync(rrp.p + nc, &rtotal, sizeof(int), hipMemcpyHostToDevice, st));
    k_sg_tfill<<<gs_grid(tnnz), GS_WG, 0, st>>>(tnnz, order.p, row.p, tv.p, rci.p, rv.p);
    GS_CHK(hipGetLastError());
    // A_{l+1} = R (A P)
    DBuf<int> crp, cci;
    DBuf<double> cv;
    int cnnz = 0;
    r = sg_spgemm(st, nc, rrp.p, rci.p, rv.p, aprp.p, apci.p, apv.p, crp, cci, cv, cnnz, err);
    if (r) return r;
    if ((r = sg_download(st, trp, (size_t)n + 1, prp_out, err))) return r;
    if ((r = sg_download(st, tci, (size_t)tnnz, pci_out, err))) return r;
    if ((r = sg_download(st, tv, (size_t)tnnz, pv_out, err))) return r;
    if ((r = sg_download(st, aprp, (size_t)n + 1, aprp_out, err))) return r;
    if ((r = sg_download(st, apci, (size_t)apnnz, apci_out, err))) return r;
    if ((r = sg_download(st, apv, (size_t)apnnz, apv_out, err))) return r;
    if ((r = sg_download(st, crp, (size_t)nc + 1, crp_out, err))) return r;
    if ((r = sg_download(st, cci, (size_t)cnnz, cci_out, err))) return r;
    if ((r = sg_download(st, cv, (size_t)cnnz, cv_out, err))) return r;
    GS_CHK(hipStreamSynchronize(st));
    return PSC_OK;
}

}  // namespace psc
