// amg.hip -- gfx950 kernels and C ABI of the AMG-preconditioned CG solve phase.
//
// Method (arXiv 2406.19754): CG / flexible CG preconditioned by the V-cycle
// of eq. (amg), Section "AMG4PSBLAS": one l1-Jacobi pre-sweep from a zero
// guess, restriction with P^T, recursive coarse correction, prolongation and
// one l1-Jacobi post-sweep; the coarsest level is solved exactly. The matrix
// storage is hacked ELLPACK (Section "GPU support"): rows in groups of one
// wavefront (64 rows here) stored as independent ELLPACK blocks.
//
// MI355X mapping:
//   * one lane per row, one wavefront per 64-row slice, column-major slice
//     layout so each load instruction of a wavefront reads 512 contiguous
//     bytes of values and 256 of indices, streamed with non-temporal loads
//     so the gathered vectors keep the L2 and Infinity Cache;
//   * streaming kernels run a grid of up to 131072 workgroups in which
//     workgroup b walks a contiguous range of slices in launch order, so the
//     8 XCDs (which receive workgroups round-robin) sweep the same region at
//     once and share the neighbour gathers through the Infinity Cache; on a
//     stencil level the range is sized so that a z-plane is a multiple of 8
//     ranges (the rows a plane away are then swept on the same die,
//     grid_lvl); an optional remap (PSC_TUNE_XCD) gives each XCD one
//     contiguous eighth of the rows instead, which measured slower;
//   * every dot product is fused into the kernel that produces one of its
//     operands: wavefront shuffles, then LDS, then one partial per
//     workgroup; a one-workgroup finishing kernel adds the partials in a
//     fixed order and updates the Krylov scalars on the device --
//     deterministic, no atomics, no fences, no host sync (a device-scope
//     fence per workgroup would write back the XCD's L2 each time);
//   * the V-cycle never stores the pre-smoothed iterate: x = M^-1 b is
//     recomputed where it is needed, the pre-smoothing kernel writes only
//     the residual, and prolongation is fused into the post-smoothing kernel;
//   * the whole iteration is captured once as a HIP graph and replayed;
//     kernels of iterations launched past convergence exit at entry.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <type_traits>
#include <unordered_map>
#include <vector>

#include "../../include/psc.h"
#include "kernels.h"
#include "net.h"
#include "setup.h"

namespace psc {

thread_local std::string g_err;

static int fail(int st, const std::string& msg) {
    g_err = msg;
    return st;
}

#define HIPCHK(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            return fail(PSC_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Block order. Workgroups are dealt round-robin to the 8 accelerator dies
// (block b runs on die b % 8). By default a block takes the work in launch
// order, so all dies sweep the same region at once and share the neighbour
// gathers through the Infinity Cache; measured faster (5 % on the 256^3 PCG
// iteration) than giving each die its own contiguous chunk, which keeps the
// gathers in the die's L2. PSC_TUNE_XCD = 1 selects the chunked order:
// XCD x receives ids x, x+8, ... and maps them to the contiguous range
// [x*G/8, (x+1)*G/8) (G = gridDim.x, always a multiple of 8).
__constant__ int g_xcd_chunked = 0;

__device__ __forceinline__ int logical_block() {
    if (!g_xcd_chunked) return blockIdx.x;
    int g8 = gridDim.x / NXCD;
    return (blockIdx.x % NXCD) * g8 + blockIdx.x / NXCD;
}

__device__ __forceinline__ void chunk_range(long long total, long long& lo, long long& hi) {
    int lb = logical_block();
    long long per = (total + gridDim.x - 1) / gridDim.x;
    lo = (long long)lb * per;
    hi = lo + per;
    if (hi > total) hi = total;
    if (lo > total) lo = total;
}

template <typename T>
__device__ __forceinline__ T ntload(const T* p) {
    return __builtin_nontemporal_load(p);
}

// Mirror the stop flag to host-mapped memory. Only the final state is
// needed by the host loop, so the system-scope fence is paid once per solve.
__device__ __forceinline__ void publish(Ctl* c, HostCtl* hc) {
    if (hc && c->done) {
        hc->done = c->done;
        hc->iter = c->iter;
        hc->status = c->status;
        hc->fallbacks = c->fallbacks;
        __threadfence_system();
    }
}

enum Fin {
    FIN_NONE = 0,
    FIN_INIT,         // s0 = ||b||^2, s1 = ||r0||^2
    FIN_ALPHA_PCG,    // s0 = p.q
    FIN_ALPHA_FCG,    // s0 = p.q, s1 = p.r
    FIN_UPDATE_PCG,   // s0 = ||r||^2
    FIN_UPDATE_FCG,   // s0 = ||r||^2
    FIN_RHO_INIT,     // s0 = r.z
    FIN_RHO,          // s0 = r.z
    FIN_BETA_FCG,     // s0 = z.q_prev
    FIN_TRUE,         // s0 = ||b - A x||^2 (r replaced by it)
    FIN_STORE,        // out0 = s0, out1 = s1
    FIN_NETCHECK,     // s0 = z.r, s1 = z.q_prev of a network step
};

__device__ void finalize(int fin, double s0, double s1, Ctl* c, HostCtl* hc) {
    switch (fin) {
    case FIN_INIT:
        c->nb2 = s0;
        c->rr = s1;
        c->rr_old = s1;
        if (!isfinite(s0) || !isfinite(s1)) { c->status = PSC_ERR_NAN; c->done = 1; }
        else if (s0 == 0.0) { c->status = PSC_OK; c->done = 1; }
        else if (sqrt(s1) <= c->rtol * sqrt(s0)) { c->status = PSC_OK; c->done = 1; }
        break;
    case FIN_ALPHA_PCG:
        c->pq = s0;
        if (isnan(s0)) { c->status = PSC_ERR_NAN; c->done = 1; c->alpha = 0.0; }
        else if (!(s0 > 0.0)) { c->status = PSC_ERR_NOT_SPD; c->done = 1; c->alpha = 0.0; }
        else c->alpha = c->rho / s0;
        break;
    case FIN_ALPHA_FCG:
        c->pq = s0;
        c->pr = s1;
        // on a breakdown alpha = 0: the deferred x update of the fused forms
        // (already applied for the previous direction) is not repeated
        if (isnan(s0) || isnan(s1)) { c->status = PSC_ERR_NAN; c->done = 1; c->alpha = 0.0; }
        else if (!(s0 > 0.0)) { c->status = PSC_ERR_NOT_SPD; c->done = 1; c->alpha = 0.0; }
        else { c->alpha = s1 / s0; c->pq_prev = s0; c->have_prev = 1; }
        break;
    case FIN_UPDATE_PCG:
    case FIN_UPDATE_FCG:
        c->rr_old = c->rr;
        c->rr = s0;
        c->iter += 1;
        c->redo = 0;
        if (c->use_net && c->net_on && sqrt(s0) > 0.9 * sqrt(c->rr_old)) {   // network stagnates
            c->net_on = 0;
            if (hc) {   // once per solve: lets the host drop the network kernels
                hc->net_off = 1;
                __threadfence_system();
            }
        }
        if (isnan(s0)) { c->status = PSC_ERR_NAN; c->done = 1; }
        else if (sqrt(s0) <= c->rtol * sqrt(c->nb2)) {
            if (fin == FIN_UPDATE_PCG) { c->status = PSC_OK; c->done = 1; }
            else c->check = 1;
        } else if (c->iter >= c->maxit) { c->status = PSC_NOCONV; c->done = 1; }
        break;
    case FIN_RHO_INIT:
        if (isnan(s0)) { c->status = PSC_ERR_NAN; c->done = 1; }
        else if (!(s0 > 0.0)) { c->status = PSC_ERR_NOT_SPD; c->done = 1; }
        c->rho = s0;
        break;
    case FIN_RHO:
        if (isnan(s0)) { c->status = PSC_ERR_NAN; c->done = 1; }
        else if (!(s0 > 0.0)) { c->status = PSC_ERR_NOT_SPD; c->done = 1; }
        else { c->beta = s0 / c->rho; c->rho = s0; }
        break;
    case FIN_BETA_FCG:
        c->zq = s0;
        c->beta = c->have_prev ? s0 / c->pq_prev : 0.0;
        break;
    case FIN_TRUE:
        if (!c->check) break;          // no true-residual check was due this iteration
        c->check = 0;
        if (isnan(s0)) { c->status = PSC_ERR_NAN; c->done = 1; }
        else if (sqrt(s0) <= c->rtol * sqrt(c->nb2)) { c->status = PSC_OK; c->done = 1; }
        else {
            c->have_prev = 0;
            c->rr = s0;
            c->redo = 1;
            if (c->iter >= c->maxit) { c->status = PSC_NOCONV; c->done = 1; }
        }
        break;
    case FIN_STORE:
        c->out0 = s0;
        c->out1 = s1;
        break;
    case FIN_NETCHECK:
        c->zr = s0;
        if (!(s0 > 0.0)) {
            // not a descent direction: the V-cycle runs instead; a second
            // such step in a row switches the network off for the solve
            c->use_net = 0;
            c->fallbacks += 1;
            if (++c->net_fails >= 2) {
                c->net_on = 0;
                if (hc) {
                    hc->net_off = 1;
                    __threadfence_system();
                }
            }
        } else {
            c->net_fails = 0;
            c->zq = s1;
            c->beta = c->have_prev ? s1 / c->pq_prev : 0.0;
        }
        break;
    default:
        break;
    }
    publish(c, hc);
}

struct Red {
    double* part;      // 2 doubles per workgroup
    Ctl* ctl;          // control block (finaliser target, and the gate)
    HostCtl* hctl;     // host-mapped mirror (may be NULL)
    int fin;           // finaliser run by k_finish
    int gmode;         // GateMode applied with ctl
};

__device__ __forceinline__ bool skip_red(const Red& R) { return gate_skip(Gate{R.ctl, R.gmode}); }

// Block-reduce (s0, s1) and store this workgroup's partial pair. The
// partials are added in a fixed order by k_finish, launched right after
// (the kernel boundary makes them visible); no atomics, no fences.
__device__ void block_partial(double s0, double s1, double* part) {
    __shared__ double red[2][WG / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    if (lane == 0) { red[0][w] = s0; red[1][w] = s1; }
    __syncthreads();
    if (threadIdx.x == 0) {
        const int lb = logical_block();
        part[2 * lb] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        part[2 * lb + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

// Optional middle stage for large grids: workgroup f adds the partial pairs
// [f*per, (f+1)*per) in order into out[2f], out[2f+1].
__global__ __launch_bounds__(WG) void k_finish_mid(Red R, int nblk, double* __restrict__ out) {
    if (skip_red(R)) return;
    __shared__ double red[2][WG / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int per = (nblk + gridDim.x - 1) / gridDim.x;
    const int lo = blockIdx.x * per, hi = min(nblk, lo + per);
    double a = 0.0, b = 0.0;
    for (int i = lo + threadIdx.x; i < hi; i += WG) {
        a += R.part[2 * i];
        b += R.part[2 * i + 1];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) { red[0][w] = a; red[1][w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        out[2 * blockIdx.x] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        out[2 * blockIdx.x + 1] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
    }
}

// Last stage: one workgroup adds the nblk partial pairs in a fixed order
// and runs the finaliser on the control block.
__global__ __launch_bounds__(WG) void k_finish(Red R, int nblk) {
    if (skip_red(R)) return;
    __shared__ double red[2][WG / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double a = 0.0, b = 0.0;
    for (int i = threadIdx.x; i < nblk; i += WG) {
        a += R.part[2 * i];
        b += R.part[2 * i + 1];
    }
    a = wave_sum(a);
    b = wave_sum(b);
    if (lane == 0) { red[0][w] = a; red[1][w] = b; }
    __syncthreads();
    if (threadIdx.x == 0) {
        a = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        b = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        finalize(R.fin, a, b, R.ctl, R.hctl);
    }
}

// Row sum over one hacked-ELL row: sum_k val[k] * g(col[k]) in slot order
// (ascending column order of the CSR input; padded slots carry 0). Slices of
// width <= 8 (every stencil slice) issue all value and index loads before
// the first gather, so a wavefront keeps up to 16 streaming loads and 8
// gathers in flight; wider slices take the general loop.
template <typename T, typename G, int U = 8, int GB = 4>
__device__ __forceinline__ T ell_row(const Ell<T>& A, long long s, int lane, G g) {
    if (A.pair) {
        // paired layout: one width per 128-row block, slot stride 128
        const long long o = A.off[s], b0 = A.off[s & ~1ll];
        const int w = (int)((A.off[(s & ~1ll) + 2] - b0) >> 7);
        const T* vp = A.val + o + lane;
        const int* cp = A.col + o + lane;
        T acc = T(0);
        int k = 0;
        for (; k + GB <= w; k += GB) {
            T v[GB];
            int c[GB];
#pragma unroll
            for (int j = 0; j < GB; j++) {
                v[j] = ntload(vp + (k + j) * 2 * SLICE);
                c[j] = ntload(cp + (k + j) * 2 * SLICE);
            }
            T gv[GB];
#pragma unroll
            for (int j = 0; j < GB; j++) gv[j] = g(c[j]);
#pragma unroll
            for (int j = 0; j < GB; j++) acc += v[j] * gv[j];
        }
        for (; k < w; k++) acc += ntload(vp + k * 2 * SLICE) * g(ntload(cp + k * 2 * SLICE));
        return acc;
    }
    const long long o = A.off[s];
    const int w = (int)((A.off[s + 1] - o) >> 6);
    const T* vp = A.val + o + lane;
    const int* cp = A.col + o + lane;
    T acc = T(0);
    if (U == 4 && w <= 8) {
        // two batches of four slots: fewer live registers, higher occupancy
#pragma unroll
        for (int b0 = 0; b0 < 8; b0 += 4) {
            T v[4];
            int c[4];
#pragma unroll
            for (int k = 0; k < 4; k++) {
                if (b0 + k < w) {
                    v[k] = ntload(vp + (b0 + k) * SLICE);
                    c[k] = ntload(cp + (b0 + k) * SLICE);
                }
            }
            T gv[4];
#pragma unroll
            for (int k = 0; k < 4; k++)
                if (b0 + k < w) gv[k] = g(c[k]);
#pragma unroll
            for (int k = 0; k < 4; k++)
                if (b0 + k < w) acc += v[k] * gv[k];
        }
        return acc;
    }
    if (w <= 8) {
        T v[8];
        int c[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if (k < w) {
                v[k] = ntload(vp + k * SLICE);
                c[k] = ntload(cp + k * SLICE);
            }
        }
        T gv[8];
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < w) gv[k] = g(c[k]);
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < w) acc += v[k] * gv[k];
        return acc;
    }
    // wider rows: batches of GB slots, every load of a batch issued before
    // its gathers (GB = 8 for operators with wide rows -- restriction and the
    // coarse operators of smoothed hierarchies -- at the price of registers)
    int k = 0;
    for (; k + GB <= w; k += GB) {
        T v[GB];
        int c[GB];
#pragma unroll
        for (int j = 0; j < GB; j++) {
            v[j] = ntload(vp + j * SLICE);
            c[j] = ntload(cp + j * SLICE);
        }
        T gv[GB];
#pragma unroll
        for (int j = 0; j < GB; j++) gv[j] = g(c[j]);
#pragma unroll
        for (int j = 0; j < GB; j++) acc += v[j] * gv[j];
        vp += GB * SLICE;
        cp += GB * SLICE;
    }
    for (; k < w; k++) {
        T v0 = ntload(vp);
        int c0 = ntload(cp);
        acc += v0 * g(c0);
        vp += SLICE;
        cp += SLICE;
    }
    return acc;
}

// Lanes of one wavefront exchanging values through LDS: order the writes of
// every lane before the reads that follow.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Overflow of slice s in a capped layout (see EllC), as the row sum of each
// lane's row (0 for rows without overflow). The wavefront takes the entries
// 64 at a time (a round), lane j one entry, four rounds with all their loads
// and gathers in flight together; within a round a row's entries are adjacent
// lanes, summed by a segmented inclusive scan (distances 1, 2, 4, ..., 32,
// each adding the partial sum d lanes down when it belongs to the same row),
// and the last lane of each run adds its sum to the row's slot in LDS (one
// writer per row and round, rounds in order). The wavefront's LDS accesses
// run in program order, and the compiler keeps the order of these (their
// addresses may alias). With nq > 1 (the split form) wavefront q of nq takes
// the rounds q, q + nq, q + 2 nq, ... and returns its part of each row's sum.
// Every lane of the wavefront must call this with the same s; workgroups of
// up to 1024 threads.
template <typename T, typename G>
__device__ __forceinline__ T ell_ovf(const EllC<T>& A, long long s, int lane, G g, int q = 0, int nq = 1) {
    constexpr int RB = 4;
    __shared__ T ov_acc[16][SLICE];
    T* acc = ov_acc[threadIdx.x >> 6];
    acc[lane] = T(0);
    const long long e0 = A.xs[s], e1 = A.xs[s + 1];
    const long long step = (long long)nq * SLICE;
    wave_lds_sync();
    for (long long base = e0 + (long long)q * SLICE; base < e1; base += RB * step) {
        T v[RB], p[RB];
        int c[RB], key[RB];
#pragma unroll
        for (int t = 0; t < RB; t++) {
            const long long e = base + t * step + lane;
            key[t] = SLICE + lane;   // lanes past the end: a key of their own
            v[t] = T(0);
            c[t] = 0;
            if (e < e1) {
                key[t] = A.xl[e];
                v[t] = A.xv[e];
                c[t] = A.xc[e];
            }
        }
#pragma unroll
        for (int t = 0; t < RB; t++) p[t] = base + t * step + lane < e1 ? v[t] * g(c[t]) : T(0);
#pragma unroll
        for (int t = 0; t < RB; t++) {
#pragma unroll
            for (int d = 1; d < SLICE; d <<= 1) {
                const T q = __shfl_up(p[t], d);
                const int kq = __shfl_up(key[t], d);
                if (lane >= d && kq == key[t]) p[t] += q;
            }
        }
#pragma unroll
        for (int t = 0; t < RB; t++) {
            const int kn = __shfl_down(key[t], 1);
            if (key[t] < SLICE && (lane == SLICE - 1 || kn != key[t])) acc[key[t]] += p[t];
        }
    }
    wave_lds_sync();
    return acc[lane];
}

// Row sum over one row of a capped layout: its slots, then its overflow.
// Wave-uniform s.
template <typename T, typename G, int U = 8, int GB = 4>
__device__ __forceinline__ T ell_row(const EllC<T>& A, long long s, int lane, G g) {
    T acc = ell_row<T, G, U, GB>(static_cast<const Ell<T>&>(A), s, lane, g);
    return acc + ell_ovf(A, s, lane, g);
}

// Operators with wide rows (the coarse operators, transfers and smoothed
// prolongators of smoothed hierarchies: hundreds to thousands of slots per
// row) are latency-bound with one lane per row walking its slots, and their
// few slices leave most of the GPU idle. GB = GB_SPLIT selects the split
// form: the WG / 64 wavefronts of a workgroup share each slice, wavefront q
// taking the slots q, q + 4, q + 8, ... of all its 64 rows (batches of 8,
// every load of a batch issued before its gathers); the partial sums meet in
// LDS and wavefront 0 adds them in a fixed order and finishes the rows.
constexpr int GB_SPLIT = 0;
constexpr int OVF_SPLIT_ROUNDS = 8;   // capped layouts: overflow rounds per slice above which it takes the split form
constexpr int SPLIT_W = 48;
static_assert(WG == 256, "the split form adds four wavefronts' partial sums");   // hacked-ELL slots per row above which a level takes the split form

template <typename T, typename G>
__device__ __forceinline__ T ell_row_part(const Ell<T>& A, long long s, int lane, int q, G g) {
    constexpr int NQ = WG / 64, B = 8;
    long long o, stride;
    int w;
    if (A.pair) {
        const long long b0 = A.off[s & ~1ll];
        o = A.off[s];
        w = (int)((A.off[(s & ~1ll) + 2] - b0) >> 7);
        stride = 2 * SLICE;
    } else {
        o = A.off[s];
        w = (int)((A.off[s + 1] - o) >> 6);
        stride = SLICE;
    }
    const T* vp = A.val + o + lane;
    const int* cp = A.col + o + lane;
    T acc = T(0);
    int k = q;
    for (; k + (B - 1) * NQ < w; k += B * NQ) {
        T v[B];
        int c[B];
#pragma unroll
        for (int j = 0; j < B; j++) {
            v[j] = ntload(vp + (long long)(k + j * NQ) * stride);
            c[j] = ntload(cp + (long long)(k + j * NQ) * stride);
        }
        T gv[B];
#pragma unroll
        for (int j = 0; j < B; j++) gv[j] = g(c[j]);
#pragma unroll
        for (int j = 0; j < B; j++) acc += v[j] * gv[j];
    }
    for (; k < w; k += NQ) acc += ntload(vp + (long long)k * stride) * g(ntload(cp + (long long)k * stride));
    return acc;
}

// The split form's loop over the slices of this workgroup's chunk: row sums
// a = sum_k v_k g(col_k), then epi(row, a) on wavefront 0. Every thread of the
// workgroup runs the loop (two barriers per slice).
template <typename MT, typename G, typename E>
__device__ __forceinline__ void ell_split_slices(const MT& A, G g, E epi) {
    using T = typename MT::value_type;
    __shared__ T part[WG / 64][SLICE];
    long long lo, hi;
    chunk_range(A.nslices, lo, hi);
    const int lane = threadIdx.x & 63, q = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    for (long long s = lo; s < hi; s++) {
        T a = ell_row_part(static_cast<const Ell<T>&>(A), s, lane, q, g);
        if constexpr (std::is_same<MT, EllC<T>>::value) a += ell_ovf(A, s, lane, g, q, WG / 64);
        part[q][lane] = a;
        __syncthreads();
        if (q == 0) {
            const T a = (part[0][lane] + part[1][lane]) + (part[2][lane] + part[3][lane]);
            const long long row = s * SLICE + lane;
            if (row < A.nrows) epi(row, a);
        }
        __syncthreads();
    }
}

// Two rows of two different slices (s1, s2, both of width <= 8) computed
// together: all value and index loads of both slices are issued before the
// first gather, doubling the loads a wavefront keeps in flight.
template <typename T, typename G>
__device__ __forceinline__ void ell_row2(const Ell<T>& A, long long s1, long long s2, int lane, G g, T& a1, T& a2) {
    if (A.pair) {
        a1 = ell_row(A, s1, lane, g);
        a2 = ell_row(A, s2, lane, g);
        return;
    }
    const long long o1 = A.off[s1], o2 = A.off[s2];
    const int w1 = (int)((A.off[s1 + 1] - o1) >> 6), w2 = (int)((A.off[s2 + 1] - o2) >> 6);
    if (w1 > 8 || w2 > 8) {
        a1 = ell_row(A, s1, lane, g);
        a2 = ell_row(A, s2, lane, g);
        return;
    }
    const T* vp1 = A.val + o1 + lane;
    const int* cp1 = A.col + o1 + lane;
    const T* vp2 = A.val + o2 + lane;
    const int* cp2 = A.col + o2 + lane;
    T v1[8], v2[8];
    int c1[8], c2[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        if (k < w1) { v1[k] = ntload(vp1 + k * SLICE); c1[k] = ntload(cp1 + k * SLICE); }
        if (k < w2) { v2[k] = ntload(vp2 + k * SLICE); c2[k] = ntload(cp2 + k * SLICE); }
    }
    T g1[8], g2[8];
#pragma unroll
    for (int k = 0; k < 8; k++) {
        if (k < w1) g1[k] = g(c1[k]);
        if (k < w2) g2[k] = g(c2[k]);
    }
    T acc1 = T(0), acc2 = T(0);
#pragma unroll
    for (int k = 0; k < 8; k++) {
        if (k < w1) acc1 += v1[k] * g1[k];
        if (k < w2) acc2 += v2[k] * g2[k];
    }
    a1 = acc1;
    a2 = acc2;
}

// ---- buffer-load path ------------------------------------------------------
// Raw buffer loads address memory as a scalar descriptor (base, byte size)
// plus a 32-bit per-lane byte offset: one VGPR per gathered address instead
// of a 64-bit pointer pair, an immediate offset for the slot stride, and a
// zero (not a fault) for an offset past the end. Descriptor word 3 for the
// gfx9 family is 0x00020000; aux bit 1 is the non-temporal hint.
typedef __amdgpu_buffer_rsrc_t rsrc_t;
__device__ __forceinline__ rsrc_t brsrc(const void* p, long long bytes) {
    const long long cap = 0xffffffffll;
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)(bytes < cap ? bytes : cap),
                                             0x00020000);
}
template <typename T, int AUX>
struct BLoad;
template <int AUX>
struct BLoad<double, AUX> {
    static __device__ __forceinline__ double f(rsrc_t r, unsigned off) {
        return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, AUX));
    }
};
template <int AUX>
struct BLoad<float, AUX> {
    static __device__ __forceinline__ float f(rsrc_t r, unsigned off) {
        return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, AUX));
    }
};
template <int AUX>
struct BLoad<int, AUX> {
    static __device__ __forceinline__ int f(rsrc_t r, unsigned off) {
        return __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, 0, AUX);
    }
};
// aux 0: default caching (gathers); aux 2: non-temporal (matrix streams)
template <typename T, int AUX = 0>
__device__ __forceinline__ T bload(rsrc_t r, unsigned off) {
    return BLoad<T, AUX>::f(r, off);
}
// gathered vector element: g[c]
template <typename T>
struct BVec {
    rsrc_t r;
    __device__ __forceinline__ T operator[](int c) const { return bload<T>(r, (unsigned)c * sizeof(T)); }
};
template <typename T>
__device__ __forceinline__ BVec<T> bvec(const T* p, long long n) { return BVec<T>{brsrc(p, n * (long long)sizeof(T))}; }

// ell_row with the slice's values and columns read through per-slice
// descriptors (s must be wave-uniform).
template <typename T, typename G>
__device__ __forceinline__ T ell_row_buf(const Ell<T>& A, long long s, int lane, G g) {
    if (A.pair) return ell_row(A, s, lane, g);
    const long long o = A.off[s];
    const int w = (int)((A.off[s + 1] - o) >> 6);
    const rsrc_t rv = brsrc(A.val + o, (long long)w * SLICE * sizeof(T));
    const rsrc_t rc = brsrc(A.col + o, (long long)w * SLICE * 4);
    const unsigned lv = (unsigned)lane * sizeof(T), lc = (unsigned)lane * 4u;
    T acc = T(0);
    if (w <= 8) {
        T v[8];
        int c[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if (k < w) {
                v[k] = bload<T, 2>(rv, lv + k * SLICE * sizeof(T));
                c[k] = bload<int, 2>(rc, lc + k * SLICE * 4);
            }
        }
        T gv[8];
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < w) gv[k] = g(c[k]);
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < w) acc += v[k] * gv[k];
        return acc;
    }
    for (int k = 0; k < w; k++)
        acc += bload<T, 2>(rv, lv + (unsigned)k * SLICE * sizeof(T)) * g(bload<int, 2>(rc, lc + (unsigned)k * SLICE * 4));
    return acc;
}

// The capped layout reads its slots with plain loads, then its overflow.
template <typename T, typename G>
__device__ __forceinline__ T ell_row_buf(const EllC<T>& A, long long s, int lane, G g) {
    return ell_row(A, s, lane, g);
}
template <typename T, typename G>
__device__ __forceinline__ void ell_row2(const EllC<T>& A, long long s1, long long s2, int lane, G g, T& a1, T& a2) {
    a1 = ell_row(A, s1, lane, g);
    a2 = ell_row(A, s2, lane, g);
}

// wave-uniform wave index of this thread within its workgroup
__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Vector range of this workgroup, in whole 512-element units so that the
// bulk is walked with 16-byte (2 x FP64) loads.
__device__ __forceinline__ void vchunk_range(long long total, long long& lo, long long& hi) {
    const int lb = logical_block();
    long long per = (total + gridDim.x - 1) / gridDim.x;
    per = (per + 2 * WG - 1) / (2 * WG) * (2 * WG);
    lo = (long long)lb * per;
    hi = lo + per;
    if (hi > total) hi = total;
    if (lo > total) lo = total;
}

// Row sum over one hacked-DIA row: sum_k val[k] * g(row + offs[k]) in
// ascending offset (= column) order. Offsets are wave-uniform (scalar
// loads); a column that falls outside [0, ncols) belongs to a zero value and
// is clamped to a valid index. Slices of at most 8 diagonals issue every
// value load before the first gather.
template <typename T, typename G, int GB = 4>
__device__ __forceinline__ T dia_row(const Dia<T>& A, long long s, int lane, G g) {
    if (A.nd > 0) {
        // uniform offsets (kernel argument): no per-slice metadata load
        const int nd = A.nd;
        const int row = (int)(s * SLICE) + lane;
        const int cmax = (int)A.ncols - 1;
        const int ks = A.pair ? 2 * SLICE : SLICE;   // diagonal stride
        const T* vp = A.val + (A.pair ? (s >> 1) * (long long)nd * 2 * SLICE + (s & 1) * SLICE
                                      : s * (long long)nd * SLICE) + lane;
        if (nd == 7) {
            // 7-point stencils: the diagonal count known at compile time, so
            // no branch per diagonal (a gather that combines several loads
            // would otherwise wait for each diagonal's before the next)
            T v[7];
            int c[7];
#pragma unroll
            for (int k = 0; k < 7; k++) {
                v[k] = ntload(vp + k * ks);
                c[k] = min(max(row + A.uo[k], 0), cmax);
            }
            T gv[7];
#pragma unroll
            for (int k = 0; k < 7; k++) gv[k] = g(c[k]);
            T acc = T(0);
#pragma unroll
            for (int k = 0; k < 7; k++) acc += v[k] * gv[k];
            return acc;
        }
        T v[8];
        int c[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if (k < nd) {
                v[k] = ntload(vp + k * ks);
                c[k] = min(max(row + A.uo[k], 0), cmax);
            }
        }
        T gv[8];
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < nd) gv[k] = g(c[k]);
        T acc = T(0);
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < nd) acc += v[k] * gv[k];
        return acc;
    }
    const int k0 = A.start[s];
    const int nd = A.start[s + 1] - k0;
    const int row = (int)(s * SLICE) + lane;
    const int cmax = (int)A.ncols - 1;
    // a paired layout is uniform: k0 = s * nd
    const int ks = A.pair ? 2 * SLICE : SLICE;
    const T* vp = A.val + (A.pair ? (s >> 1) * (long long)nd * 2 * SLICE + (s & 1) * SLICE
                                  : (long long)k0 * SLICE) + lane;
    const int* op = A.offs + k0;
    T acc = T(0);
    if (nd <= 8) {
        T v[8];
        int c[8];
#pragma unroll
        for (int k = 0; k < 8; k++) {
            if (k < nd) {
                v[k] = ntload(vp + k * ks);
                c[k] = min(max(row + op[k], 0), cmax);
            }
        }
        T gv[8];
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < nd) gv[k] = g(c[k]);
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < nd) acc += v[k] * gv[k];
        return acc;
    }
    int k = 0;
    for (; k + GB <= nd; k += GB) {
        T v[GB];
        int c[GB];
#pragma unroll
        for (int j = 0; j < GB; j++) {
            v[j] = ntload(vp + (k + j) * ks);
            c[j] = min(max(row + op[k + j], 0), cmax);
        }
        T gv[GB];
#pragma unroll
        for (int j = 0; j < GB; j++) gv[j] = g(c[j]);
#pragma unroll
        for (int j = 0; j < GB; j++) acc += v[j] * gv[j];
    }
    for (; k < nd; k++) {
        const T v0 = ntload(vp + k * ks);
        acc += v0 * g(min(max(row + op[k], 0), cmax));
    }
    return acc;
}

// ---- two rows per lane on the paired uniform hacked-DIA layout -----------
// A wavefront takes one 128-row block S and lane l its rows 2l and 2l+1:
// every value load and, inside the matrix, every gather reads two
// consecutive elements with one 8- or 16-byte access. gp(c) returns
// {g(c), g(c+1)}; g1(c) one element (blocks whose gathers leave [0, ncols),
// where the index is clamped and the value is zero).
template <typename T>
struct V2;
template <>
struct V2<double> {
    typedef double u __attribute__((ext_vector_type(2), aligned(8)));    // any 8-byte address
    typedef double a __attribute__((ext_vector_type(2), aligned(16)));   // values of the layout
};
template <>
struct V2<float> {
    typedef float u __attribute__((ext_vector_type(2), aligned(4)));
    typedef float a __attribute__((ext_vector_type(2), aligned(8)));
};
template <typename T>
using v2u = typename V2<T>::u;
template <typename T>
using v2a = typename V2<T>::a;

template <typename T>
__device__ __forceinline__ v2u<T> ld2(const T* p) { return *(const v2u<T>*)p; }
template <typename T>
__device__ __forceinline__ void st2(T* p, T a, T b) { *(v2u<T>*)p = v2u<T>{a, b}; }

template <typename T>
__device__ __forceinline__ bool dia_pair_on(const Dia<T>& A) { return A.pair && A.nd > 0; }

// number of 128-row blocks of a paired layout
template <typename T>
__device__ __forceinline__ long long dia_blocks(const Dia<T>& A) { return (A.nslices + 1) >> 1; }

// Row sums a0, a1 of the two rows 2 lane, 2 lane + 1 of block S of a paired
// uniform hacked-DIA operator: a = sum_k v_k cb(gl(column_k)). gl loads what
// one entry needs (any type), cb turns it into the two rows' operands; every
// gl of the block is issued before any cb, so that the loads of all diagonals
// are in flight together (a cb that used its loads at once would make each
// diagonal wait for the previous one's). g1 gives one row's operand at a
// clamped column (blocks at the ends of the matrix).
template <typename T, typename GL, typename CB, typename G1>
__device__ __forceinline__ void dia_pair_rows_lc(const Dia<T>& A, long long S, int lane, GL gl, CB cb, G1 g1, T& a0,
                                                 T& a1) {
    const int nd = A.nd;
    const long long r0 = S * (2 * SLICE) + 2 * lane;
    const v2a<T>* vp = (const v2a<T>*)(A.val + S * (long long)nd * 2 * SLICE) + lane;
    v2a<T> v[8];
#pragma unroll
    for (int k = 0; k < 8; k++)
        if (k < nd) v[k] = ntload(vp + k * SLICE);
    const long long b0 = S * (2 * SLICE);
    // wave-uniform: every row of the block exists and every gather is in range
    const bool inner = b0 + A.uo[0] >= 0 && b0 + 2 * SLICE - 1 + A.uo[nd - 1] < A.ncols &&
                       b0 + 2 * SLICE <= A.nrows;
    T s0 = T(0), s1 = T(0);
    if (inner && nd == 7) {
        // 7-point stencils: no branch per diagonal
        decltype(gl(0ll)) g[7];
#pragma unroll
        for (int k = 0; k < 7; k++) g[k] = gl(r0 + A.uo[k]);
#pragma unroll
        for (int k = 0; k < 7; k++) {
            const v2u<T> c = cb(g[k]);
            s0 += v[k].x * c.x;
            s1 += v[k].y * c.y;
        }
    } else if (inner) {
        decltype(gl(0ll)) g[8];
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < nd) g[k] = gl(r0 + A.uo[k]);
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < nd) {
                const v2u<T> c = cb(g[k]);
                s0 += v[k].x * c.x;
                s1 += v[k].y * c.y;
            }
    } else {
        const long long cmax = A.ncols - 1;
#pragma unroll
        for (int k = 0; k < 8; k++)
            if (k < nd) {
                const long long c0 = min(max(r0 + A.uo[k], 0ll), cmax), c1 = min(max(r0 + 1 + A.uo[k], 0ll), cmax);
                s0 += v[k].x * g1((int)c0);
                s1 += v[k].y * g1((int)c1);
            }
    }
    a0 = s0;
    a1 = s1;
}

// The same with gp giving the two rows' operands directly.
template <typename T, typename GP, typename G1>
__device__ __forceinline__ void dia_pair_rows(const Dia<T>& A, long long S, int lane, GP gp, G1 g1, T& a0, T& a1) {
    dia_pair_rows_lc(A, S, lane, gp, [](const v2u<T>& g) { return g; }, g1, a0, a1);
}

// Two gathered FP64 vectors of one entry.
struct Gather2 {
    v2u<double> a, b;
};
// Two gathered vectors of any element types.
template <typename A, typename B>
struct GatherAB {
    v2u<A> a;
    v2u<B> b;
};

// Row sum of either storage format; GB is the batch of the wide-row path.
template <int GB = 4, typename T, typename G>
__device__ __forceinline__ T mat_row(const Ell<T>& A, long long s, int lane, G g) {
    return ell_row<T, G, 8, GB>(A, s, lane, g);
}
template <int GB = 4, typename T, typename G>
__device__ __forceinline__ T mat_row(const EllC<T>& A, long long s, int lane, G g) {
    return ell_row<T, G, 8, GB>(A, s, lane, g);
}
template <int GB = 4, typename T, typename G>
__device__ __forceinline__ T mat_row(const Dia<T>& A, long long s, int lane, G g) {
    return dia_row<T, G, GB>(A, s, lane, g);
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// y = A x
template <typename M, bool BUF = false, int GB = 4>
__global__ __launch_bounds__(WG) void k_spmv(M A, const typename M::value_type* __restrict__ x,
                                             typename M::value_type* __restrict__ y, Gate g) {
    using T = typename M::value_type;
    if (gate_skip(g)) return;
    if constexpr (GB == GB_SPLIT) {
        if constexpr (is_ell<M>::value)
            ell_split_slices(A, [&](int c) { return x[c]; }, [&](long long row, T a) { y[row] = a; });
        return;
    }
    constexpr int GBN = GB == GB_SPLIT ? 4 : GB;   // (the split form returned above)
    long long lo, hi;
    const int lane = threadIdx.x & 63, w = wave_id();
    if constexpr (std::is_same<M, Dia<T>>::value) {
        if (dia_pair_on(A)) {
            chunk_range(dia_blocks(A), lo, hi);
            for (long long S = lo + w; S < hi; S += WG / 64) {
                T a0, a1;
                dia_pair_rows(A, S, lane, [&](long long c) { return ld2(x + c); }, [&](int c) { return x[c]; }, a0, a1);
                const long long row = S * (2 * SLICE) + 2 * lane;
                if (row + 1 < A.nrows) st2(y + row, a0, a1);
                else if (row < A.nrows) y[row] = a0;
            }
            return;
        }
    }
    chunk_range(A.nslices, lo, hi);
    const BVec<T> bx = bvec(x, A.ncols);
    for (long long s = lo + w; s < hi; s += WG / 64) {
        T acc;
        if constexpr (BUF) acc = ell_row_buf(A, s, lane, [&](int c) { return bx[c]; });
        else acc = mat_row<GBN>(A, s, lane, [&](int c) { return x[c]; });
        long long row = s * SLICE + lane;
        if (row < A.nrows) y[row] = acc;
    }
}

// y = A x, two slices per wavefront in flight (slices s and s + 4 of the
// workgroup's chunk).
template <typename T>
__global__ __launch_bounds__(WG) void k_spmv2(Ell<T> A, const T* __restrict__ x, T* __restrict__ y, Gate g) {
    if (gate_skip(g)) return;
    long long lo, hi;
    chunk_range(A.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = wave_id();
    auto gx = [&](int c) { return x[c]; };
    long long s = lo + w;
    for (; s + WG / 64 < hi; s += 2 * (WG / 64)) {
        T a1, a2;
        ell_row2(A, s, s + WG / 64, lane, gx, a1, a2);
        const long long r1 = s * SLICE + lane, r2 = (s + WG / 64) * SLICE + lane;
        if (r1 < A.nrows) y[r1] = a1;
        if (r2 < A.nrows) y[r2] = a2;
    }
    if (s < hi) {
        T a = ell_row(A, s, lane, gx);
        const long long r1 = s * SLICE + lane;
        if (r1 < A.nrows) y[r1] = a;
    }
}

// q = A p with partials (p.q, p.r); r may be NULL.
template <typename M>
__global__ __launch_bounds__(WG) void k_spmv_dot(M A, const double* __restrict__ p,
                                                 double* __restrict__ q, const double* __restrict__ r,
                                                 Red R) {
    if (skip_red(R)) return;
    long long lo, hi;
    chunk_range(A.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double s0 = 0.0, s1 = 0.0;
    for (long long s = lo + w; s < hi; s += WG / 64) {
        double acc = mat_row(A, s, lane, [&](int c) { return p[c]; });
        long long row = s * SLICE + lane;
        if (row < A.nrows) {
            q[row] = acc;
            double pi = p[row];
            s0 += pi * acc;
            if (r) s1 += pi * r[row];
        }
    }
    block_partial(s0, s1, R.part);
}

// r = b - A x with partials (b.b, r.r). With only_if_check, runs only when
// the control block asks for a true-residual check.
template <typename M>
__global__ __launch_bounds__(WG) void k_resid(M A, const double* __restrict__ b,
                                              const double* __restrict__ x, double* __restrict__ r,
                                              int only_if_check, Red R) {
    if (skip_red(R)) return;
    if (only_if_check && !R.ctl->check) return;
    long long lo, hi;
    chunk_range(A.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    double s0 = 0.0, s1 = 0.0;
    for (long long s = lo + w; s < hi; s += WG / 64) {
        double acc = mat_row(A, s, lane, [&](int c) { return x[c]; });
        long long row = s * SLICE + lane;
        if (row < A.nrows) {
            double bi = b[row];
            double ri = bi - acc;
            r[row] = ri;
            s0 += bi * bi;
            s1 += ri * ri;
        }
    }
    if (only_if_check) block_partial(s1, 0.0, R.part);
    else block_partial(s0, s1, R.part);
}

// x += alpha p; r -= alpha q; partial r.r
__global__ __launch_bounds__(WG) void k_update(long long n, double* __restrict__ x,
                                               double* __restrict__ r, const double* __restrict__ p,
                                               const double* __restrict__ q, Red R) {
    if (skip_red(R)) return;
    const double alpha = R.ctl->alpha;
    long long lo, hi;
    vchunk_range(n, lo, hi);
    double s0 = 0.0;
    long long i = lo + 2 * threadIdx.x;
    for (; i + 1 < hi; i += 2 * WG) {
        const double2 pp = *(const double2*)(p + i), qq = *(const double2*)(q + i);
        double2 xx = *(const double2*)(x + i), rr = *(const double2*)(r + i);
        xx.x += alpha * pp.x;
        xx.y += alpha * pp.y;
        rr.x -= alpha * qq.x;
        rr.y -= alpha * qq.y;
        *(double2*)(x + i) = xx;
        *(double2*)(r + i) = rr;
        s0 += rr.x * rr.x;
        s0 += rr.y * rr.y;
    }
    if (i < hi) {   // odd tail (last element of the vector)
        x[i] += alpha * p[i];
        const double ri = r[i] - alpha * q[i];
        r[i] = ri;
        s0 += ri * ri;
    }
    block_partial(s0, 0.0, R.part);
}

// PCG: p = z + beta p.  FCG: p = z - beta p (p = z without a previous direction).
__global__ __launch_bounds__(WG) void k_pupdate(long long n, double* __restrict__ p,
                                                const double* __restrict__ z, int fcg, Gate g) {
    if (gate_skip(g)) return;
    const int keep = fcg ? g.ctl->have_prev : 1;
    const double beta = keep ? (fcg ? -g.ctl->beta : g.ctl->beta) : 0.0;
    long long lo, hi;
    vchunk_range(n, lo, hi);
    long long i = lo + 2 * threadIdx.x;
    if (!keep) {
        for (; i + 1 < hi; i += 2 * WG) *(double2*)(p + i) = *(const double2*)(z + i);
        if (i < hi) p[i] = z[i];
        return;
    }
    for (; i + 1 < hi; i += 2 * WG) {
        const double2 zz = *(const double2*)(z + i);
        double2 pp = *(const double2*)(p + i);
        pp.x = zz.x + beta * pp.x;
        pp.y = zz.y + beta * pp.y;
        *(double2*)(p + i) = pp;
    }
    if (i < hi) p[i] = z[i] + beta * p[i];
}

// Fused PCG, first pass: p_new = z + beta p_old (own row, and recomputed
// for every gathered neighbour), q = A p_new, the x update deferred from the
// previous iteration x += alpha_prev p_old, and the partial p_new.q.
// alpha in the control block still holds alpha_prev here (0 at the start).
template <typename M, bool BUF = false>
__global__ __launch_bounds__(WG) void k_spmv_pfuse(M A, const double* __restrict__ z,
                                                   const double* __restrict__ pold, double* __restrict__ pnew,
                                                   double* __restrict__ q, double* __restrict__ x, Red R) {
    if (skip_red(R)) return;
    const double beta = R.ctl->beta, alpha_prev = R.ctl->alpha;
    long long lo, hi;
    const int lane = threadIdx.x & 63, w = wave_id();
    double s0 = 0.0;
    if constexpr (std::is_same<M, Dia<double>>::value) {
        if (dia_pair_on(A)) {
            chunk_range(dia_blocks(A), lo, hi);
            for (long long S = lo + w; S < hi; S += WG / 64) {
                double a0, a1;
                dia_pair_rows_lc(
                    A, S, lane, [&](long long c) { return Gather2{ld2(pold + c), ld2(z + c)}; },
                    [&](const Gather2& t) {
                        return v2u<double>{fma(beta, t.a.x, t.b.x), fma(beta, t.a.y, t.b.y)};
                    },
                    [&](int c) { return fma(beta, pold[c], z[c]); }, a0, a1);
                const long long row = S * (2 * SLICE) + 2 * lane;
                if (row + 1 < A.nrows) {
                    const v2u<double> po = ld2(pold + row), zz = ld2(z + row), xx = ld2((const double*)x + row);
                    const double p0 = fma(beta, po.x, zz.x), p1 = fma(beta, po.y, zz.y);
                    // p_new and x are read again only in the next iteration, after the whole
                    // V-cycle, and q mostly from HBM anyway (the residual update streams
                    // it after the reduction; at 384^3 it is larger than the Infinity
                    // Cache): non-temporal stores (pass 1 1031 -> 1013 us at 384^3)
                    __builtin_nontemporal_store(v2a<double>{p0, p1}, (v2a<double>*)(pnew + row));
                    __builtin_nontemporal_store(v2a<double>{a0, a1}, (v2a<double>*)(q + row));
                    __builtin_nontemporal_store(v2a<double>{fma(alpha_prev, po.x, xx.x), fma(alpha_prev, po.y, xx.y)},
                                                 (v2a<double>*)(x + row));
                    s0 += p0 * a0;
                    s0 += p1 * a1;
                } else if (row < A.nrows) {
                    const double po = pold[row];
                    const double pn = fma(beta, po, z[row]);
                    pnew[row] = pn;
                    q[row] = a0;
                    x[row] = fma(alpha_prev, po, x[row]);
                    s0 += pn * a0;
                }
            }
            block_partial(s0, 0.0, R.part);
            return;
        }
    }
    chunk_range(A.nslices, lo, hi);
    const BVec<double> bz = bvec(z, A.ncols), bp = bvec(pold, A.ncols);
    for (long long s = lo + w; s < hi; s += WG / 64) {
        double acc;
        if constexpr (BUF) acc = ell_row_buf(A, s, lane, [&](int c) { return fma(beta, bp[c], bz[c]); });
        else acc = mat_row(A, s, lane, [&](int c) { return fma(beta, pold[c], z[c]); });
        long long row = s * SLICE + lane;
        if (row < A.nrows) {
            const double po = pold[row];
            const double pn = fma(beta, po, z[row]);
            pnew[row] = pn;
            q[row] = acc;
            x[row] = fma(alpha_prev, po, x[row]);
            s0 += pn * acc;
        }
    }
    block_partial(s0, 0.0, R.part);
}

// Fused PCG, second pass: r_new = r_old - alpha q (own row, and recomputed for
// every gathered neighbour), the level-0 pre-smoothing residual
// r0 = r_new - A (minv .* r_new), and the partial ||r_new||^2.
template <int U = 8, bool BUF = false>
__global__ __launch_bounds__(WG) void k_update_pre(Ell<double> A, const double* __restrict__ minv,
                                                   const double* __restrict__ rold, const double* __restrict__ q,
                                                   double* __restrict__ rnew, double* __restrict__ r0, Red R) {
    if (skip_red(R)) return;
    const double nalpha = -R.ctl->alpha;
    long long lo, hi;
    chunk_range(A.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = wave_id();
    const BVec<double> bm = bvec(minv, A.ncols), bq = bvec(q, A.ncols), br = bvec(rold, A.ncols);
    double s0 = 0.0;
    for (long long s = lo + w; s < hi; s += WG / 64) {
        double acc;
        if constexpr (BUF) {
            acc = ell_row_buf(A, s, lane, [&](int c) { return bm[c] * fma(nalpha, bq[c], br[c]); });
        } else {
            auto g = [&](int c) { return minv[c] * fma(nalpha, q[c], rold[c]); };
            acc = ell_row<double, decltype(g), U>(A, s, lane, g);
        }
        long long row = s * SLICE + lane;
        if (row < A.nrows) {
            const double rn = fma(nalpha, q[row], rold[row]);
            rnew[row] = rn;
            r0[row] = rn - acc;
            s0 += rn * rn;
        }
    }
    block_partial(s0, 0.0, R.part);
}

// Fused FCG(1), first pass: p_new = z - beta p_old (p_new = z without a
// previous direction), q = A p_new, the deferred x += alpha_prev p_old, and
// the partials (p_new.q, p_new.r_old). Held to 168 registers, three waves
// per SIMD: the compiler's 170 would allow only two, measured 2 % slower at
// 384^3 (two registers spill). TZ = float: z read from its FP32 copy (the
// mixed form's V-cycle output) and widened.
template <typename M, bool BUF = false, typename TZ = double>
__global__ __launch_bounds__(WG) __attribute__((amdgpu_waves_per_eu(3))) void k_spmv_pfuse_fcg(M A, const TZ* __restrict__ z,
                                                       const double* __restrict__ pold, double* __restrict__ pnew,
                                                       double* __restrict__ q, double* __restrict__ x,
                                                       const double* __restrict__ rold, Red R) {
    if (skip_red(R)) return;
    const double nb = R.ctl->have_prev ? -R.ctl->beta : 0.0, alpha_prev = R.ctl->alpha;
    long long lo, hi;
    const int lane = threadIdx.x & 63, w = wave_id();
    double s0 = 0.0, s1 = 0.0;
    if constexpr (std::is_same<M, Dia<double>>::value) {
        if (dia_pair_on(A)) {
            chunk_range(dia_blocks(A), lo, hi);
            for (long long S = lo + w; S < hi; S += WG / 64) {
                double a0, a1;
                dia_pair_rows_lc(
                    A, S, lane, [&](long long c) { return GatherAB<double, TZ>{ld2(pold + c), ld2(z + c)}; },
                    [&](const GatherAB<double, TZ>& t) {
                        return v2u<double>{fma(nb, t.a.x, (double)t.b.x), fma(nb, t.a.y, (double)t.b.y)};
                    },
                    [&](int c) { return fma(nb, pold[c], (double)z[c]); }, a0, a1);
                const long long row = S * (2 * SLICE) + 2 * lane;
                if (row + 1 < A.nrows) {
                    const v2u<double> po = ld2(pold + row), xx = ld2((const double*)x + row), rr = ld2(rold + row);
                    const v2u<TZ> zz = ld2(z + row);
                    const double p0 = fma(nb, po.x, (double)zz.x), p1 = fma(nb, po.y, (double)zz.y);
                    __builtin_nontemporal_store(v2a<double>{p0, p1}, (v2a<double>*)(pnew + row));
                    __builtin_nontemporal_store(v2a<double>{a0, a1}, (v2a<double>*)(q + row));
                    __builtin_nontemporal_store(v2a<double>{fma(alpha_prev, po.x, xx.x), fma(alpha_prev, po.y, xx.y)},
                                                 (v2a<double>*)(x + row));
                    s0 += p0 * a0;
                    s0 += p1 * a1;
                    s1 += p0 * rr.x;
                    s1 += p1 * rr.y;
                } else if (row < A.nrows) {
                    const double po = pold[row];
                    const double pn = fma(nb, po, (double)z[row]);
                    pnew[row] = pn;
                    q[row] = a0;
                    x[row] = fma(alpha_prev, po, x[row]);
                    s0 += pn * a0;
                    s1 += pn * rold[row];
                }
            }
            block_partial(s0, s1, R.part);
            return;
        }
    }
    chunk_range(A.nslices, lo, hi);
    const BVec<TZ> bz = bvec(z, A.ncols);
    const BVec<double> bp = bvec(pold, A.ncols);
    for (long long s = lo + w; s < hi; s += WG / 64) {
        double acc;
        if constexpr (BUF) acc = ell_row_buf(A, s, lane, [&](int c) { return fma(nb, bp[c], (double)bz[c]); });
        else acc = mat_row(A, s, lane, [&](int c) { return fma(nb, pold[c], (double)z[c]); });
        long long row = s * SLICE + lane;
        if (row < A.nrows) {
            const double po = pold[row];
            const double pn = fma(nb, po, (double)z[row]);
            pnew[row] = pn;
            q[row] = acc;
            x[row] = fma(alpha_prev, po, x[row]);
            s0 += pn * acc;
            s1 += pn * rold[row];
        }
    }
    block_partial(s0, s1, R.part);
}

// Fused update + level-0 pre-smoothing in the V-cycle's precision T:
// r_new = r_old - alpha q (FP64), r0 = (T)r_new - A_T ((T)minv .* (T)r_new).
template <typename T, bool BUF = false>
__global__ __launch_bounds__(WG) void k_update_pre_t(Ell<T> A, const T* __restrict__ minv,
                                                     const double* __restrict__ rold, const double* __restrict__ q,
                                                     double* __restrict__ rnew, T* __restrict__ r0, Red R) {
    if (skip_red(R)) return;
    const double nalpha = -R.ctl->alpha;
    long long lo, hi;
    chunk_range(A.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = wave_id();
    const BVec<T> bm = bvec(minv, A.ncols);
    const BVec<double> bq = bvec(q, A.ncols), br = bvec(rold, A.ncols);
    double s0 = 0.0;
    for (long long s = lo + w; s < hi; s += WG / 64) {
        T acc;
        if constexpr (BUF) acc = ell_row_buf(A, s, lane, [&](int c) { return bm[c] * (T)fma(nalpha, bq[c], br[c]); });
        else acc = ell_row(A, s, lane, [&](int c) { return minv[c] * (T)fma(nalpha, q[c], rold[c]); });
        long long row = s * SLICE + lane;
        if (row < A.nrows) {
            const double rn = fma(nalpha, q[row], rold[row]);
            rnew[row] = rn;
            r0[row] = (T)rn - acc;
            s0 += rn * rn;
        }
    }
    block_partial(s0, 0.0, R.part);
}

// Fused FCG true residual (only when the recursive test passed): x lags by
// its last update, so r = b - A (x + alpha p) with the sum formed for every
// gathered neighbour; the partial ||r||^2 feeds FIN_TRUE.
template <typename M>
__global__ __launch_bounds__(WG) void k_resid_lag(M A, const double* __restrict__ b,
                                                  const double* __restrict__ x, const double* __restrict__ p,
                                                  double* __restrict__ r, Red R) {
    if (skip_red(R) || !R.ctl->check) return;
    const double alpha = R.ctl->alpha;
    long long lo, hi;
    chunk_range(A.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = wave_id();
    double s0 = 0.0;
    for (long long s = lo + w; s < hi; s += WG / 64) {
        double acc = mat_row(A, s, lane, [&](int c) { return fma(alpha, p[c], x[c]); });
        long long row = s * SLICE + lane;
        if (row < A.nrows) {
            const double ri = b[row] - acc;
            r[row] = ri;
            s0 += ri * ri;
        }
    }
    block_partial(s0, 0.0, R.part);
}

// x += alpha p once the fused iteration has stopped (its last x update is deferred).
__global__ __launch_bounds__(WG) void k_final_axpy(long long n, double* __restrict__ x, const double* __restrict__ p,
                                                   const Ctl* ctl) {
    const double alpha = ctl->alpha;
    long long lo, hi;
    chunk_range(n, lo, hi);
    for (long long i = lo + threadIdx.x; i < hi; i += WG) x[i] = fma(alpha, p[i], x[i]);
}

// partials (a.b, 0) for a dot product not fused elsewhere
__global__ __launch_bounds__(WG) void k_dot(long long n, const double* __restrict__ a,
                                            const double* __restrict__ b, Red R) {
    if (skip_red(R)) return;
    long long lo, hi;
    chunk_range(n, lo, hi);
    double s0 = 0.0;
    for (long long i = lo + threadIdx.x; i < hi; i += WG) s0 += a[i] * b[i];
    block_partial(s0, 0.0, R.part);
}

template <typename TD, typename TS>
__global__ __launch_bounds__(WG) void k_copy(long long n, TD* __restrict__ d, const TS* __restrict__ s,
                                             Gate g) {
    if (gate_skip(g)) return;
    long long lo, hi;
    chunk_range(n, lo, hi);
    for (long long i = lo + threadIdx.x; i < hi; i += WG) d[i] = (TD)s[i];
}

template <typename T>
__global__ __launch_bounds__(WG) void k_fill(long long n, T* __restrict__ d, T v) {
    long long lo, hi;
    chunk_range(n, lo, hi);
    for (long long i = lo + threadIdx.x; i < hi; i += WG) d[i] = v;
}

__global__ void k_ctl_init(Ctl* c, HostCtl* hc, double rtol, int maxit, int form) {
    if (threadIdx.x == 0) {
        c->rtol = rtol;
        c->nb2 = c->rr = c->rr_old = c->rho = c->alpha = c->beta = 0.0;
        c->pq = c->pr = c->zq = c->zr = c->pq_prev = c->out0 = c->out1 = 0.0;
        c->done = 0;
        c->iter = 0;
        c->status = PSC_NOCONV;
        c->maxit = maxit;
        c->check = 0;
        c->have_prev = 0;
        c->net_on = 0;
        c->use_net = 0;
        c->fallbacks = 0;
        c->form = form;
        c->redo = 0;
        c->net_fails = 0;
        if (hc) {
            hc->done = 0;
            hc->iter = 0;
            hc->status = PSC_NOCONV;
            hc->fallbacks = 0;
            hc->net_off = 0;
            __threadfence_system();
        }
    }
}

__global__ void k_set_net_on(Ctl* c) {
    if (threadIdx.x == 0) c->net_on = 1;
}

// Pre-smoothing from a zero guess and its residual, one pass:
//   r_i = b_i - sum_j a_ij (minv_j b_j)       (the iterate M^-1 b is not stored)
template <typename T, typename TB, bool BUF = false>
__global__ __launch_bounds__(WG) void k_pre(Ell<T> A, const T* __restrict__ minv,
                                            const TB* __restrict__ b, T* __restrict__ r, Gate g) {
    if (gate_skip(g)) return;
    long long lo, hi;
    chunk_range(A.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = wave_id();
    const BVec<T> bm = bvec(minv, A.ncols);
    const BVec<TB> bb = bvec(b, A.ncols);
    for (long long s = lo + w; s < hi; s += WG / 64) {
        T acc;
        if constexpr (BUF) acc = ell_row_buf(A, s, lane, [&](int c) { return bm[c] * (T)bb[c]; });
        else acc = ell_row(A, s, lane, [&](int c) { return minv[c] * (T)b[c]; });
        long long row = s * SLICE + lane;
        if (row < A.nrows) r[row] = (T)b[row] - acc;
    }
}

// Prolongation fused with the post-smoothing sweep:
//   xs_j = minv_j b_j + p_j xc[agg_j]   (pre-smoothed iterate + coarse correction)
//   x_i  = xs_i + minv_i (b_i - sum_j a_ij xs_j)
// With R.fin != FIN_NONE, also the partial sum of x_i * d_i.
template <typename T, typename TB, typename TX, int U = 8, bool BUF = false>
__global__ __launch_bounds__(WG) void k_post(Ell<T> A, const T* __restrict__ minv,
                                             const TB* __restrict__ b, const int* __restrict__ agg,
                                             const T* __restrict__ pv, const T* __restrict__ xc, long long nc,
                                             TX* __restrict__ x, const double* __restrict__ d, Red R) {
    if (skip_red(R)) return;
    long long lo, hi;
    chunk_range(A.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = wave_id();
    const BVec<T> bm = bvec(minv, A.ncols), bp = bvec(pv, A.ncols), bx = bvec(xc, nc);
    const BVec<TB> bb = bvec(b, A.ncols);
    const BVec<int> ba = bvec(agg, A.ncols);
    double s0 = 0.0;
    auto xs = [&](int c) { return minv[c] * (T)b[c] + pv[c] * xc[agg[c]]; };
    for (long long s = lo + w; s < hi; s += WG / 64) {
        T acc;
        if constexpr (BUF) acc = ell_row_buf(A, s, lane, [&](int c) { return bm[c] * (T)bb[c] + bp[c] * bx[ba[c]]; });
        else acc = ell_row<T, decltype(xs), U>(A, s, lane, xs);
        long long row = s * SLICE + lane;
        if (row < A.nrows) {
            int i = (int)row;
            T xi = xs(i) + minv[i] * ((T)b[i] - acc);
            x[row] = (TX)xi;
            if (d) s0 += (double)(TX)xi * d[row];
        }
    }
    if (R.fin != FIN_NONE) block_partial(s0, 0.0, R.part);
}

// ---- split-operator forms of the smoothing sweeps --------------------------
// With the scaled operator AM = A M^-1 (values a_ij minv_j in A's layout) the
// pre-smoothing residual r = b - AM b gathers one vector. Post-smoothing of
// xs = M^-1 b + P xc is x = xs + M^-1 (b - A xs) = M^-1 (b + r) + S P xc with
// S = I - M^-1 A, so with the smoothed prolongator SP = P - M^-1 A P (rows of
// A, aggregate columns) it gathers only the coarse correction:
//   x_i = minv_i (b_i + r_i) + sum_J sp_iJ xc_J.
// These give the sweeps of k_pre / k_post up to rounding.

// r_i = b_i - sum_j am_ij b_j
//
// hp != nullptr (paired uniform DIA levels whose row pairs 2k, 2k+1 share an
// aggregate and a prolongator value, see DevLevel::R2): also the pair sums
// hp[k] = r_2k + r_2k+1, which the restriction then reads instead of r.
template <typename M, typename TB, int GB = 4>
__global__ __launch_bounds__(WG) void k_pre_s(M AM, const TB* __restrict__ b, typename M::value_type* __restrict__ r,
                                              Gate g, typename M::value_type* __restrict__ hp) {
    using T = typename M::value_type;
    if (gate_skip(g)) return;
    if constexpr (GB == GB_SPLIT) {
        if constexpr (is_ell<M>::value)
            ell_split_slices(AM, [&](int c) { return (T)b[c]; }, [&](long long row, T a) { r[row] = (T)b[row] - a; });
        return;
    }
    constexpr int GBN = GB == GB_SPLIT ? 4 : GB;   // (the split form returned above)
    long long lo, hi;
    const int lane = threadIdx.x & 63, w = wave_id();
    if constexpr (std::is_same<M, Dia<T>>::value) {
        if (dia_pair_on(AM)) {
            chunk_range(dia_blocks(AM), lo, hi);
            for (long long S = lo + w; S < hi; S += WG / 64) {
                T a0, a1;
                dia_pair_rows_lc(
                    AM, S, lane, [&](long long c) { return ld2(b + c); },
                    [&](const v2u<TB>& bb) { return v2u<T>{(T)bb.x, (T)bb.y}; }, [&](int c) { return (T)b[c]; },
                    a0, a1);
                const long long row = S * (2 * SLICE) + 2 * lane;
                if (row + 1 < AM.nrows) {
                    const v2u<TB> bb = ld2(b + row);
                    const T r0 = (T)bb.x - a0, r1 = (T)bb.y - a1;
                    __builtin_nontemporal_store(v2a<T>{r0, r1}, (v2a<T>*)(r + row));
                    if (hp) hp[row >> 1] = r0 + r1;
                } else if (row < AM.nrows) {
                    r[row] = (T)b[row] - a0;
                }
            }
            return;
        }
    }
    chunk_range(AM.nslices, lo, hi);
    for (long long s = lo + w; s < hi; s += WG / 64) {
        const T acc = mat_row<GBN>(AM, s, lane, [&](int c) { return (T)b[c]; });
        const long long row = s * SLICE + lane;
        if (row < AM.nrows) r[row] = (T)b[row] - acc;
    }
}

// Fused update + level-0 pre-smoothing with AM in precision T:
// r_new = r_old - alpha q (FP64), r0 = (T)r_new - AM_T (T)r_new, partial ||r_new||^2.
// hp: the pair sums of r0 as in k_pre_s.
template <typename M>
__global__ __launch_bounds__(WG) void k_update_pre_s(M AM, const double* __restrict__ rold,
                                                     const double* __restrict__ q, double* __restrict__ rnew,
                                                     typename M::value_type* __restrict__ r0, Red R,
                                                     typename M::value_type* __restrict__ hp) {
    using T = typename M::value_type;
    if (skip_red(R)) return;
    const double nalpha = -R.ctl->alpha;
    long long lo, hi;
    const int lane = threadIdx.x & 63, w = wave_id();
    double s0 = 0.0;
    if constexpr (std::is_same<M, Dia<T>>::value) {
        if (dia_pair_on(AM)) {
            chunk_range(dia_blocks(AM), lo, hi);
            for (long long S = lo + w; S < hi; S += WG / 64) {
                T a0, a1;
                dia_pair_rows_lc(
                    AM, S, lane, [&](long long c) { return Gather2{ld2(q + c), ld2(rold + c)}; },
                    [&](const Gather2& t) {
                        return v2u<T>{(T)fma(nalpha, t.a.x, t.b.x), (T)fma(nalpha, t.a.y, t.b.y)};
                    },
                    [&](int c) { return (T)fma(nalpha, q[c], rold[c]); }, a0, a1);
                const long long row = S * (2 * SLICE) + 2 * lane;
                if (row + 1 < AM.nrows) {
                    const v2u<double> qq = ld2(q + row), rr = ld2(rold + row);
                    const double n0 = fma(nalpha, qq.x, rr.x), n1 = fma(nalpha, qq.y, rr.y);
                    st2(rnew + row, n0, n1);
                    const T z0 = (T)n0 - a0, z1 = (T)n1 - a1;
                    st2(r0 + row, z0, z1);
                    if (hp) hp[row >> 1] = z0 + z1;
                    s0 += n0 * n0;
                    s0 += n1 * n1;
                } else if (row < AM.nrows) {
                    const double rn = fma(nalpha, q[row], rold[row]);
                    rnew[row] = rn;
                    r0[row] = (T)rn - a0;
                    s0 += rn * rn;
                }
            }
            block_partial(s0, 0.0, R.part);
            return;
        }
    }
    chunk_range(AM.nslices, lo, hi);
    for (long long s = lo + w; s < hi; s += WG / 64) {
        const T acc = mat_row(AM, s, lane, [&](int c) { return (T)fma(nalpha, q[c], rold[c]); });
        const long long row = s * SLICE + lane;
        if (row < AM.nrows) {
            const double rn = fma(nalpha, q[row], rold[row]);
            rnew[row] = rn;
            r0[row] = (T)rn - acc;
            s0 += rn * rn;
        }
    }
    block_partial(s0, 0.0, R.part);
}

// Post-smoothing with prolongation through SP (see above); with
// R.fin != FIN_NONE also the partial sum of x_i * d_i.
template <typename T, typename TB, typename TX, int GB = 4>
__global__ __launch_bounds__(WG) void k_post_s(Ell<T> SP, const T* __restrict__ minv, const TB* __restrict__ b,
                                               const T* __restrict__ r, const T* __restrict__ xc,
                                               TX* __restrict__ x, const double* __restrict__ d, Red R) {
    if (skip_red(R)) return;
    long long lo, hi;
    const int lane = threadIdx.x & 63, w = wave_id();
    double s0 = 0.0;
    if constexpr (GB == GB_SPLIT) {
        ell_split_slices(SP, [&](int c) { return xc[c]; }, [&](long long row, T a) {
            const T xi = minv[row] * ((T)b[row] + r[row]) + a;
            x[row] = (TX)xi;
            if (d) s0 += (double)(TX)xi * d[row];
        });
        if (R.fin != FIN_NONE) block_partial(s0, 0.0, R.part);
        return;
    }
    constexpr int GBN = GB == GB_SPLIT ? 4 : GB;   // (the split form returned above)
    if (SP.pair) {
        // two rows per lane: their values (8/16 bytes) and columns (8 bytes)
        // with one load per slot
        typedef int i2 __attribute__((ext_vector_type(2), aligned(8)));
        chunk_range((SP.nslices + 1) >> 1, lo, hi);
        for (long long S = lo + w; S < hi; S += WG / 64) {
            const long long b0 = SP.off[2 * S];
            const int ws = (int)((SP.off[2 * S + 2] - b0) >> 7);
            const v2a<T>* vp = (const v2a<T>*)(SP.val + b0) + lane;
            const i2* cp = (const i2*)(SP.col + b0) + lane;
            T a0 = T(0), a1 = T(0);
            int k = 0;
            // FP64: the usual widths (5 and 6 slots: a tentative prolongator's
            // own aggregate and its stencil neighbours' ones) in one batch,
            // every slot's loads and gathers in flight together (same sums,
            // same order); FP32 levels keep the batches of GBN, which measure
            // faster there
            auto whole = [&](auto wc) {
                constexpr int W = decltype(wc)::value;
                v2a<T> v[W];
                i2 c[W];
#pragma unroll
                for (int j = 0; j < W; j++) {
                    v[j] = ntload(vp + j * SLICE);
                    c[j] = ntload(cp + j * SLICE);
                }
                T g0[W], g1[W];
#pragma unroll
                for (int j = 0; j < W; j++) {
                    g0[j] = xc[c[j].x];
                    g1[j] = xc[c[j].y];
                }
#pragma unroll
                for (int j = 0; j < W; j++) {
                    a0 += v[j].x * g0[j];
                    a1 += v[j].y * g1[j];
                }
                k = W;
            };
            if constexpr (sizeof(T) == 8) {
                if (ws == 5) whole(std::integral_constant<int, 5>{});
                else if (ws == 6) whole(std::integral_constant<int, 6>{});
            }
            for (; k + GBN <= ws; k += GBN) {
                v2a<T> v[GBN];
                i2 c[GBN];
#pragma unroll
                for (int j = 0; j < GBN; j++) {
                    v[j] = ntload(vp + (k + j) * SLICE);
                    c[j] = ntload(cp + (k + j) * SLICE);
                }
                T g0[GBN], g1[GBN];
#pragma unroll
                for (int j = 0; j < GBN; j++) {
                    g0[j] = xc[c[j].x];
                    g1[j] = xc[c[j].y];
                }
#pragma unroll
                for (int j = 0; j < GBN; j++) {
                    a0 += v[j].x * g0[j];
                    a1 += v[j].y * g1[j];
                }
            }
            for (; k < ws; k++) {
                const v2a<T> v = ntload(vp + k * SLICE);
                const i2 c = ntload(cp + k * SLICE);
                a0 += v.x * xc[c.x];
                a1 += v.y * xc[c.y];
            }
            const long long row = S * (2 * SLICE) + 2 * lane;
            if (row + 1 < SP.nrows) {
                const v2u<T> m = ld2(minv + row), rr = ld2(r + row);
                const v2u<TB> bb = ld2(b + row);
                const T x0 = m.x * ((T)bb.x + rr.x) + a0, x1 = m.y * ((T)bb.y + rr.y) + a1;
                st2(x + row, (TX)x0, (TX)x1);
                if (d) {
                    const v2u<double> dd = ld2(d + row);
                    s0 += (double)(TX)x0 * dd.x;
                    s0 += (double)(TX)x1 * dd.y;
                }
            } else if (row < SP.nrows) {
                const T xi = minv[row] * ((T)b[row] + r[row]) + a0;
                x[row] = (TX)xi;
                if (d) s0 += (double)(TX)xi * d[row];
            }
        }
        if (R.fin != FIN_NONE) block_partial(s0, 0.0, R.part);
        return;
    }
    chunk_range(SP.nslices, lo, hi);
    for (long long s = lo + w; s < hi; s += WG / 64) {
        const T acc = mat_row<GBN>(SP, s, lane, [&](int c) { return xc[c]; });
        const long long row = s * SLICE + lane;
        if (row < SP.nrows) {
            const T xi = minv[row] * ((T)b[row] + r[row]) + acc;
            x[row] = (TX)xi;
            if (d) s0 += (double)(TX)xi * d[row];
        }
    }
    if (R.fin != FIN_NONE) block_partial(s0, 0.0, R.part);
}

// Pre-smoothing sweep k >= 2 from a zero guess, carried as the running sum
// s_k = b + r_1 + ... + r_{k-1} (so x_k = M^-1 s_k): with s_k = s_{k-1} + r_{k-1}
// formed for the own row and every gathered neighbour,
//   r_k = b - AM s_k,   and s_k, r_k are stored.
template <typename M, typename TB, typename TS, int GB = 4>
__global__ __launch_bounds__(WG) void k_presweep(M AM, const TB* __restrict__ b, const TS* __restrict__ sprev,
                                                 const typename M::value_type* __restrict__ rprev,
                                                 typename M::value_type* __restrict__ sout,
                                                 typename M::value_type* __restrict__ rout, Gate g) {
    using T = typename M::value_type;
    if (gate_skip(g)) return;
    if constexpr (GB == GB_SPLIT) {
        if constexpr (is_ell<M>::value)
            ell_split_slices(AM, [&](int c) { return (T)sprev[c] + rprev[c]; }, [&](long long row, T a) {
                sout[row] = (T)sprev[row] + rprev[row];
                rout[row] = (T)b[row] - a;
            });
        return;
    }
    constexpr int GBN = GB == GB_SPLIT ? 4 : GB;   // (the split form returned above)
    long long lo, hi;
    const int lane = threadIdx.x & 63, w = wave_id();
    if constexpr (std::is_same<M, Dia<T>>::value) {
        if (dia_pair_on(AM)) {
            // two rows per lane, every diagonal's loads in flight together
            chunk_range(dia_blocks(AM), lo, hi);
            for (long long S = lo + w; S < hi; S += WG / 64) {
                T a0, a1;
                dia_pair_rows_lc(
                    AM, S, lane, [&](long long c) { return GatherAB<TS, T>{ld2(sprev + c), ld2(rprev + c)}; },
                    [&](const GatherAB<TS, T>& t) { return v2u<T>{(T)t.a.x + t.b.x, (T)t.a.y + t.b.y}; },
                    [&](int c) { return (T)sprev[c] + rprev[c]; }, a0, a1);
                const long long row = S * (2 * SLICE) + 2 * lane;
                if (row + 1 < AM.nrows) {
                    const v2u<TS> sp = ld2(sprev + row);
                    const v2u<T> rp = ld2(rprev + row);
                    const v2u<TB> bb = ld2(b + row);
                    st2(sout + row, (T)sp.x + rp.x, (T)sp.y + rp.y);
                    st2(rout + row, (T)bb.x - a0, (T)bb.y - a1);
                } else if (row < AM.nrows) {
                    sout[row] = (T)sprev[row] + rprev[row];
                    rout[row] = (T)b[row] - a0;
                }
            }
            return;
        }
    }
    chunk_range(AM.nslices, lo, hi);
    for (long long s = lo + w; s < hi; s += WG / 64) {
        const T acc = mat_row<GBN>(AM, s, lane, [&](int c) { return (T)sprev[c] + rprev[c]; });
        const long long row = s * SLICE + lane;
        if (row < AM.nrows) {
            sout[row] = (T)sprev[row] + rprev[row];
            rout[row] = (T)b[row] - acc;
        }
    }
}

// One l1-Jacobi sweep x_out = x_in + M^-1 (b - A x_in) (post-smoothing sweeps
// after the first); with R.fin != FIN_NONE also the partial sum of x_out * d.
template <typename M, typename TB, typename TX, int GB = 4>
__global__ __launch_bounds__(WG) void k_sweep(M A, const typename M::value_type* __restrict__ minv,
                                              const TB* __restrict__ b,
                                              const typename M::value_type* __restrict__ xin, TX* __restrict__ xout,
                                              const double* __restrict__ d, Red R) {
    using T = typename M::value_type;
    if (skip_red(R)) return;
    double s0 = 0.0;
    if constexpr (GB == GB_SPLIT) {
        if constexpr (is_ell<M>::value)
            ell_split_slices(A, [&](int c) { return xin[c]; }, [&](long long row, T a) {
                const T xi = xin[row] + minv[row] * ((T)b[row] - a);
                xout[row] = (TX)xi;
                if (d) s0 += (double)(TX)xi * d[row];
            });
        if (R.fin != FIN_NONE) block_partial(s0, 0.0, R.part);
        return;
    }
    constexpr int GBN = GB == GB_SPLIT ? 4 : GB;   // (the split form returned above)
    long long lo, hi;
    const int lane = threadIdx.x & 63, w = wave_id();
    if constexpr (std::is_same<M, Dia<T>>::value) {
        if (dia_pair_on(A)) {
            // two rows per lane
            chunk_range(dia_blocks(A), lo, hi);
            for (long long S = lo + w; S < hi; S += WG / 64) {
                T a0, a1;
                dia_pair_rows(A, S, lane, [&](long long c) { return ld2(xin + c); }, [&](int c) { return xin[c]; },
                              a0, a1);
                const long long row = S * (2 * SLICE) + 2 * lane;
                if (row + 1 < A.nrows) {
                    const v2u<T> xx = ld2(xin + row), mm = ld2(minv + row);
                    const v2u<TB> bb = ld2(b + row);
                    const T x0 = xx.x + mm.x * ((T)bb.x - a0), x1 = xx.y + mm.y * ((T)bb.y - a1);
                    st2(xout + row, (TX)x0, (TX)x1);
                    if (d) {
                        const v2u<double> dd = ld2(d + row);
                        s0 += (double)(TX)x0 * dd.x;
                        s0 += (double)(TX)x1 * dd.y;
                    }
                } else if (row < A.nrows) {
                    const T xi = xin[row] + minv[row] * ((T)b[row] - a0);
                    xout[row] = (TX)xi;
                    if (d) s0 += (double)(TX)xi * d[row];
                }
            }
            if (R.fin != FIN_NONE) block_partial(s0, 0.0, R.part);
            return;
        }
    }
    chunk_range(A.nslices, lo, hi);
    for (long long s = lo + w; s < hi; s += WG / 64) {
        const T acc = mat_row<GBN>(A, s, lane, [&](int c) { return xin[c]; });
        const long long row = s * SLICE + lane;
        if (row < A.nrows) {
            const T xi = xin[row] + minv[row] * ((T)b[row] - acc);
            xout[row] = (TX)xi;
            if (d) s0 += (double)(TX)xi * d[row];
        }
    }
    if (R.fin != FIN_NONE) block_partial(s0, 0.0, R.part);
}

// Coarsest level: x = A_L^{-1} b with the explicit inverse (column-major), FP64.
template <typename TB, typename TX>
__global__ __launch_bounds__(WG) void k_coarse(int n, const double* __restrict__ invT,
                                               const TB* __restrict__ b, TX* __restrict__ x,
                                               Gate g) {
    if (gate_skip(g)) return;
    __shared__ double bs[4096];
    for (int i = threadIdx.x; i < n; i += WG) bs[i] = (double)b[i];
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += WG) {
        double s = 0.0;
        for (int k = 0; k < n; k++) s += invT[(size_t)k * n + i] * bs[k];
        x[i] = (TX)s;
    }
}

// Coarsest level by at most maxit iterations of l1-Jacobi preconditioned CG
// from x = 0, stopped at ||r|| <= rtol ||b||, in FP64, in one workgroup of
// CPCG_WG threads: thread t owns rows t, t + CPCG_WG, ... (at most
// CPCG_ROWS), keeping x, r, z and q in registers; the direction p lives in
// LDS, where the product A p gathers it (hacked-ELL rows, padding is 0).
// Block sums are formed in a fixed order and broadcast, so every thread
// takes the same branches and the loop ends after at most maxit iterations.
constexpr int CPCG_WG = 1024;
constexpr int CPCG_ROWS = 4;
constexpr int CPCG_MAX = CPCG_WG * CPCG_ROWS;

__device__ double cpcg_sum(double v, double* red) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    v = wave_sum(v);
    __syncthreads();   // earlier readers of red are done
    if (lane == 0) red[w] = v;
    __syncthreads();
    double t = 0.0;
    for (int k = 0; k < CPCG_WG / 64; k++) t += red[k];
    return t;
}

// The solve itself, for a workgroup of CPCG_WG threads; p (at least n
// doubles) and red (CPCG_WG / 64 doubles) are LDS scratch.
template <typename TB, typename TX>
__device__ void coarse_pcg_block(const Ell<double>& A, const double* __restrict__ minv, const TB* b, TX* x,
                                 int maxit, double rtol, double* p, double* red) {
    const int n = (int)A.nrows;
    double xr[CPCG_ROWS], rr[CPCG_ROWS], zr[CPCG_ROWS], qr[CPCG_ROWS];
    double bb = 0.0, rz0 = 0.0;
#pragma unroll
    for (int k = 0; k < CPCG_ROWS; k++) {
        const int i = threadIdx.x + k * CPCG_WG;
        xr[k] = 0.0;
        rr[k] = i < n ? (double)b[i] : 0.0;
        zr[k] = i < n ? minv[i] * rr[k] : 0.0;
        if (i < n) p[i] = zr[k];
        bb += rr[k] * rr[k];
        rz0 += rr[k] * zr[k];
    }
    const double bn = sqrt(cpcg_sum(bb, red));
    double rz = cpcg_sum(rz0, red);
    if (bn > 0.0) {
        for (int it = 0; it < maxit && rz > 0.0; it++) {
            __syncthreads();   // p complete
            double pq = 0.0;
#pragma unroll
            for (int k = 0; k < CPCG_ROWS; k++) {
                const int i = threadIdx.x + k * CPCG_WG;
                qr[k] = 0.0;
                if (i < n) {
                    const long long s = i / SLICE, o = A.off[s];
                    const int w = (int)((A.off[s + 1] - o) / SLICE), lane = i % SLICE;
                    double acc = 0.0;
                    for (int e = 0; e < w; e++) acc += A.val[o + (long long)e * SLICE + lane] * p[A.col[o + (long long)e * SLICE + lane]];
                    qr[k] = acc;
                    pq += p[i] * acc;
                }
            }
            pq = cpcg_sum(pq, red);
            if (!(pq > 0.0)) break;
            const double alpha = rz / pq;
            double rn = 0.0;
#pragma unroll
            for (int k = 0; k < CPCG_ROWS; k++) {
                const int i = threadIdx.x + k * CPCG_WG;
                if (i < n) {
                    xr[k] += alpha * p[i];
                    rr[k] -= alpha * qr[k];
                    rn += rr[k] * rr[k];
                }
            }
            rn = cpcg_sum(rn, red);
            if (sqrt(rn) <= rtol * bn) break;
            double rz2 = 0.0;
#pragma unroll
            for (int k = 0; k < CPCG_ROWS; k++) {
                const int i = threadIdx.x + k * CPCG_WG;
                zr[k] = i < n ? minv[i] * rr[k] : 0.0;
                rz2 += rr[k] * zr[k];
            }
            rz2 = cpcg_sum(rz2, red);
            const double beta = rz2 / rz;
            // every read of p in this iteration happened before the sums above
#pragma unroll
            for (int k = 0; k < CPCG_ROWS; k++) {
                const int i = threadIdx.x + k * CPCG_WG;
                if (i < n) p[i] = zr[k] + beta * p[i];
            }
            rz = rz2;
        }
    }
#pragma unroll
    for (int k = 0; k < CPCG_ROWS; k++) {
        const int i = threadIdx.x + k * CPCG_WG;
        if (i < n) x[i] = (TX)xr[k];
    }
}

template <typename TB, typename TX>
__global__ __launch_bounds__(CPCG_WG) void k_coarse_pcg(Ell<double> A, const double* __restrict__ minv,
                                                        const TB* __restrict__ b, TX* __restrict__ x, int maxit,
                                                        double rtol, Gate g) {
    if (gate_skip(g)) return;
    __shared__ double p[CPCG_MAX];
    __shared__ double red[CPCG_WG / 64];
    coarse_pcg_block<TB, TX>(A, minv, b, x, maxit, rtol, p, red);
}

// ---- the small levels in one workgroup --------------------------------------
// Below a few thousand rows a level's pre-smoothing, restriction and
// post-smoothing are dominated by launch and drain time; levels t..L-1
// (ending in the coarsest solve) can run in one workgroup of 16 waves: each
// wave takes whole 64-row slices, and a workgroup barrier separates the
// steps.
constexpr int TAIL_WG = 1024;
constexpr int TAIL_MAX_ROWS = 4096;
constexpr int TAIL_LDS_BYTES = 160 * 1024;   // gfx950: 160 KB of LDS per workgroup
constexpr long long TAIL_MAX_LEVEL_BYTES = 512 * 1024;   // operator bytes of one tail level's sweep

template <typename T>
struct TailLevel {
    Ell<T> am_ell;     // A M^-1 in hacked ELL (used when dia == 0)
    Dia<T> am_dia;     // A M^-1 in hacked DIA
    Ell<T> a_ell;      // A (post-smoothing sweeps after the first)
    Dia<T> a_dia;
    int dia;
    int nu;            // smoothing sweeps on this level
    Ell<T> R;          // restriction to the next level
    Ell<T> SP;         // (I - M^-1 A) P
    const T* minv;
    T *b, *x;          // the first tail level's input and output (device memory)
};

template <typename T>
struct TailDesc {
    int t, L, nL;
    int lds_elems;                 // LDS elements of levels t .. L-1 (b, r and, with nu > 1, s)
    int base[PSC_MAX_LEVELS];      // element offset of level l's b (r follows, then s)
    const double* invT;            // dense coarsest solve (cmaxit == 0)
    int cmaxit;                    // > 0: coarsest by at most cmaxit PCG iterations (FP64)
    int cpcg_off;                  // byte offset of the PCG direction and sums in LDS
    double crtol;
    Ell<double> cA;                // coarsest operator and l1 inverse diagonal for the PCG
    const double* cminv;
    TailLevel<T> lev[PSC_MAX_LEVELS];
};

// LDS array of a tail level that holds its final post-smoothed x: the first
// post sweep writes over r (one sweep) or over s, later sweeps alternate.
__host__ __device__ inline int tail_xslot(int nu) { return nu == 1 ? 1 : (nu % 2 == 0 ? 1 : 2); }

// Levels t .. L-1 of the V-cycle in one workgroup: b, r (and s with several
// sweeps) of every such level live in LDS, and x is written over r or s once
// the post-smoothing has read them (level t's b is read from and its x
// written to device memory, where the neighbouring launches exchange them),
// so a step waits on an LDS barrier instead of a device-memory round trip;
// only the operators come from the L2. nu sweeps of the split smoother per
// level (sweep k of the pre-smoothing: s_k = s_{k-1} + r_{k-1} with s_1 = b,
// r_k = b - A M^-1 s_k; post: x = M^-1 (s + r) + S P x_c, then
// x += M^-1 (b - A x)), dense or PCG coarsest. Same arithmetic as k_pre_s,
// k_presweep, k_spmv on R, k_coarse or k_coarse_pcg, k_post_s and k_sweep.
// The operators are the levels' plain hacked ELL (or DIA), never the capped
// copies.
template <typename T>
__global__ __launch_bounds__(TAIL_WG) void k_tail(const TailDesc<T>* __restrict__ D, Gate g) {
    if (gate_skip(g)) return;
    extern __shared__ __align__(16) unsigned char tail_lds[];
    T* lds = reinterpret_cast<T*>(tail_lds);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = TAIL_WG / 64;
    const int t = D->t, L = D->L;
    {
        const T* bg = D->lev[t].b;
        T* bt = lds + D->base[t];
        const int n = (int)D->lev[t].am_ell.nrows;
        for (int i = threadIdx.x; i < n; i += TAIL_WG) bt[i] = bg[i];
        __syncthreads();
    }
    for (int l = t; l < L - 1; l++) {
        const TailLevel<T>& V = D->lev[l];
        const long long ns = V.am_ell.nslices, n = V.am_ell.nrows;
        const T* b = lds + D->base[l];
        T* r = lds + D->base[l] + n;
        T* sv = lds + D->base[l] + 2 * n;
        for (long long s = wv; s < ns; s += nw) {
            const T acc = V.dia ? dia_row(V.am_dia, s, lane, [&](int c) { return b[c]; })
                                : ell_row(V.am_ell, s, lane, [&](int c) { return b[c]; });
            const long long row = s * SLICE + lane;
            if (row < n) r[row] = b[row] - acc;
        }
        __syncthreads();
        for (int k = 2; k <= V.nu; k++) {
            for (int i = threadIdx.x; i < n; i += TAIL_WG) sv[i] = (k == 2 ? b[i] : sv[i]) + r[i];
            __syncthreads();
            for (long long s = wv; s < ns; s += nw) {
                const T acc = V.dia ? dia_row(V.am_dia, s, lane, [&](int c) { return (T)sv[c]; })
                                    : ell_row(V.am_ell, s, lane, [&](int c) { return (T)sv[c]; });
                const long long row = s * SLICE + lane;
                if (row < n) r[row] = b[row] - acc;
            }
            __syncthreads();
        }
        T* bc = lds + D->base[l + 1];
        for (long long s = wv; s < V.R.nslices; s += nw) {
            const T acc = ell_row(V.R, s, lane, [&](int c) { return (T)r[c]; });
            const long long row = s * SLICE + lane;
            if (row < V.R.nrows) bc[row] = acc;
        }
        __syncthreads();
    }
    {
        const int nL = D->nL;
        const T* bL = lds + D->base[L - 1];
        T* xL = lds + D->base[L - 1] + nL;
        if (D->cmaxit > 0) {
            double* pd = reinterpret_cast<double*>(tail_lds + D->cpcg_off);
            coarse_pcg_block<T, T>(D->cA, D->cminv, bL, xL, D->cmaxit, D->crtol, pd, pd + CPCG_MAX);
        } else {
            for (int i = threadIdx.x; i < nL; i += TAIL_WG) {
                double s = 0.0;
                for (int k = 0; k < nL; k++) s += D->invT[(size_t)k * nL + i] * (double)bL[k];
                xL[i] = (T)s;
            }
        }
        __syncthreads();
    }
    for (int l = L - 2; l >= t; l--) {
        const TailLevel<T>& V = D->lev[l];
        const long long ns = V.SP.nslices, n = V.SP.nrows;
        const long long nc = D->lev[l + 1].am_ell.nrows;
        const int cslot = l + 1 == L - 1 ? 1 : tail_xslot(D->lev[l + 1].nu);
        const T* b = lds + D->base[l];
        T* r = lds + D->base[l] + n;
        T* sv = lds + D->base[l] + 2 * n;
        const T* xc = lds + D->base[l + 1] + cslot * nc;
        T* xg = V.x;
        // first sweep, fused with the prolongation; x over r (one sweep) or s
        T* x = V.nu == 1 ? r : sv;
        const T* s_nu = V.nu == 1 ? b : sv;
        for (long long s = wv; s < ns; s += nw) {
            const T acc = ell_row(V.SP, s, lane, [&](int c) { return xc[c]; });
            const long long row = s * SLICE + lane;
            if (row < n) {
                const T xi = V.minv[row] * (s_nu[row] + r[row]) + acc;
                x[row] = xi;
                if (l == t && V.nu == 1) xg[row] = xi;
            }
        }
        __syncthreads();
        for (int k = 2; k <= V.nu; k++) {
            const T* xin = x;
            T* xo = x == sv ? r : sv;
            for (long long s = wv; s < ns; s += nw) {
                const T acc = V.dia ? dia_row(V.a_dia, s, lane, [&](int c) { return xin[c]; })
                                    : ell_row(V.a_ell, s, lane, [&](int c) { return xin[c]; });
                const long long row = s * SLICE + lane;
                if (row < n) {
                    const T xi = xin[row] + V.minv[row] * (b[row] - acc);
                    xo[row] = xi;
                    if (l == t && k == V.nu) xg[row] = xi;
                }
            }
            __syncthreads();
            x = xo;
        }
    }
}

// Coarsest level solved by l1-Jacobi sweeps in FP64 (used when coarsening
// stalls above the dense-factor limit). One sweep from x_in:
//   x_out_i = x_in_i + minv_i (b_i - sum_j a_ij x_in_j);
// x_in == nullptr stands for the zero guess (x_out = minv b).
template <typename M, typename TB, typename TX, int GB = 4>
__global__ __launch_bounds__(WG) void k_jacobi(M A, const double* __restrict__ minv,
                                               const TB* __restrict__ b, const double* __restrict__ xin,
                                               TX* __restrict__ xout, Gate g) {
    if (gate_skip(g)) return;
    long long lo, hi;
    if constexpr (GB == GB_SPLIT) {
        // rows wider than SPLIT_W slots: the four wavefronts share each slice
        if constexpr (is_ell<M>::value) {
            if (xin) {
                ell_split_slices(A, [&](int c) { return xin[c]; }, [&](long long row, double a) {
                    xout[row] = (TX)(xin[row] + minv[row] * ((double)b[row] - a));
                });
            } else {
                chunk_range(A.nslices, lo, hi);
                for (long long s = lo; s < hi; s++) {
                    const long long row = s * SLICE + threadIdx.x;
                    if (threadIdx.x < SLICE && row < A.nrows) xout[row] = (TX)(minv[row] * (double)b[row]);
                }
            }
        }
        return;
    }
    constexpr int GBN = GB == GB_SPLIT ? 4 : GB;   // (the split form returned above)
    chunk_range(A.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = wave_id();
    for (long long s = lo + w; s < hi; s += WG / 64) {
        const long long row = s * SLICE + lane;
        if (!xin) {
            if (row < A.nrows) xout[row] = (TX)(minv[row] * (double)b[row]);
            continue;
        }
        double acc = mat_row<GBN>(A, s, lane, [&](int c) { return xin[c]; });
        if (row < A.nrows) xout[row] = (TX)(xin[row] + minv[row] * ((double)b[row] - acc));
    }
}

// ---------------------------------------------------------------------------
// handle
// ---------------------------------------------------------------------------


// ---------------------------------------------------------------------------
// Factored approximate inverse smoothers (AINV / INVK): a sweep is
// x <- x + Z (W (b - A x)) with W = D^-1 Z^T, both stored as hacked ELL
// over their rows. Four streaming kernels: the residual, the two factor
// products and the prolongation; the V-cycle order is that of the l1-Jacobi
// form.
// ---------------------------------------------------------------------------

// t = b - A x (x = NULL: t = b)
template <typename M, typename TB, int GB = 4>
__global__ __launch_bounds__(WG) void k_fres(M A, const TB* __restrict__ b, const typename M::value_type* __restrict__ x,
                                             typename M::value_type* __restrict__ t, Gate g) {
    using T = typename M::value_type;
    if (gate_skip(g)) return;
    long long lo, hi;
    if constexpr (GB == GB_SPLIT) {
        // rows wider than SPLIT_W slots: the four wavefronts share each slice
        if constexpr (is_ell<M>::value) {
            if (x) {
                ell_split_slices(A, [&](int c) { return x[c]; }, [&](long long row, T a) { t[row] = (T)b[row] - a; });
            } else {
                chunk_range(A.nslices, lo, hi);
                for (long long s = lo; s < hi; s++) {
                    const long long row = s * SLICE + threadIdx.x;
                    if (threadIdx.x < SLICE && row < A.nrows) t[row] = (T)b[row];
                }
            }
        }
        return;
    }
    constexpr int GBN = GB == GB_SPLIT ? 4 : GB;   // (the split form returned above)
    chunk_range(A.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = wave_id();
    for (long long s = lo + w; s < hi; s += WG / 64) {
        const T acc = x ? mat_row<GBN>(A, s, lane, [&](int c) { return x[c]; }) : T(0);
        const long long row = s * SLICE + lane;
        if (row < A.nrows) t[row] = (T)b[row] - acc;
    }
}

// u = W t with the input read in its own precision TB and rounded to T
template <typename T, typename TB, int GB = 4>
__global__ __launch_bounds__(WG) void k_fw(Ell<T> W, const TB* __restrict__ t, T* __restrict__ u, Gate g) {
    if (gate_skip(g)) return;
    long long lo, hi;
    chunk_range(W.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = wave_id();
    for (long long s = lo + w; s < hi; s += WG / 64) {
        const T acc = mat_row<GB>(W, s, lane, [&](int c) { return (T)t[c]; });
        const long long row = s * SLICE + lane;
        if (row < W.nrows) u[row] = acc;
    }
}

// xout = xin + Z u (xin = NULL: xout = Z u); with R.fin != FIN_NONE also the
// partial sum of xout * d
template <typename T, typename TX, int GB = 4>
__global__ __launch_bounds__(WG) void k_fz(Ell<T> Z, const T* __restrict__ u, const T* xin, TX* xout,
                                           const double* __restrict__ d, Red R) {
    if (skip_red(R)) return;
    long long lo, hi;
    chunk_range(Z.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = wave_id();
    double s0 = 0.0;
    for (long long s = lo + w; s < hi; s += WG / 64) {
        const T acc = mat_row<GB>(Z, s, lane, [&](int c) { return u[c]; });
        const long long row = s * SLICE + lane;
        if (row < Z.nrows) {
            const T xi = (xin ? xin[row] : T(0)) + acc;
            xout[row] = (TX)xi;
            if (d) s0 += (double)(TX)xi * d[row];
        }
    }
    if (R.fin != FIN_NONE) block_partial(s0, 0.0, R.part);
}

// x += P xc (general prolongator, aggregate columns)
template <typename T, int GB = 4>
__global__ __launch_bounds__(WG) void k_fprol(Ell<T> P, const T* __restrict__ xc, T* __restrict__ x, Gate g) {
    if (gate_skip(g)) return;
    long long lo, hi;
    chunk_range(P.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = wave_id();
    for (long long s = lo + w; s < hi; s += WG / 64) {
        const T acc = mat_row<GB>(P, s, lane, [&](int c) { return xc[c]; });
        const long long row = s * SLICE + lane;
        if (row < P.nrows) x[row] += acc;
    }
}

// ---------------------------------------------------------------------------
// Polynomial smoother: the fourth-kind Chebyshev recurrence on M^-1 A with
// the bound 1 (A <= M for the l1 diagonal). Step k (1-based) takes
// (x, r, d) = (x_{k-1}, r_{k-1}, d_{k-1}) to
//   r_k = r_{k-1} - A d_{k-1},  x_k = x_{k-1} + d_{k-1},
//   d_k = a_k d_{k-1} + b_k M^-1 r_k,
// with d_0 = c0 M^-1 r_0 formed on the fly for every gathered column in the
// first step (FIRST: r_0 = sv, x_0 = xin or 0). fold: the last step of a
// post-smoothing writes x_{k+1} = x_k + d_k to xout (with the partial sum of
// xout * d when R.fin != FIN_NONE) and stores nothing else; otherwise r and x
// are updated in place and d_k goes to dout (when not NULL).
// ---------------------------------------------------------------------------
template <typename M, typename TB, typename TX, bool FIRST, int GB = 4>
__global__ __launch_bounds__(WG) void k_cheb(M A, const typename M::value_type* __restrict__ minv,
                                             const TB* __restrict__ sv, const typename M::value_type* __restrict__ din,
                                             const typename M::value_type* xin, typename M::value_type* r,
                                             typename M::value_type* x, TX* xout,
                                             typename M::value_type* __restrict__ dout, typename M::value_type c0,
                                             typename M::value_type ak, typename M::value_type bk, int fold,
                                             const double* __restrict__ d, Red R) {
    using T = typename M::value_type;
    if (skip_red(R)) return;
    long long lo, hi;
    chunk_range(A.nslices, lo, hi);
    const int lane = threadIdx.x & 63, w = wave_id();
    double s0 = 0.0;
    for (long long sl = lo + w; sl < hi; sl += WG / 64) {
        T ad;
        if constexpr (FIRST) ad = mat_row<GB>(A, sl, lane, [&](int c) { return c0 * minv[c] * (T)sv[c]; });
        else ad = mat_row<GB>(A, sl, lane, [&](int c) { return din[c]; });
        const long long row = sl * SLICE + lane;
        if (row < A.nrows) {
            T dself, rprev, xprev;
            if constexpr (FIRST) {
                dself = c0 * minv[row] * (T)sv[row];
                rprev = (T)sv[row];
                xprev = xin ? xin[row] : T(0);
            } else {
                dself = din[row];
                rprev = r[row];
                xprev = x[row];
            }
            const T rk = rprev - ad;
            const T xk = xprev + dself;
            if (fold) {
                const T xo = xk + (ak * dself + bk * minv[row] * rk);
                xout[row] = (TX)xo;
                if (d) s0 += (double)(TX)xo * d[row];
            } else {
                r[row] = rk;
                x[row] = xk;
                if (dout) dout[row] = ak * dself + bk * minv[row] * rk;
            }
        }
    }
    if (R.fin != FIN_NONE) block_partial(s0, 0.0, R.part);
}

// Degree-1 post-smoothing: xout = x + c0 M^-1 t (t = b - A x), with the
// partial sum of xout * d when R.fin != FIN_NONE.
template <typename T, typename TX>
__global__ __launch_bounds__(WG) void k_cheb_fin(long long nslices, long long n, const T* __restrict__ x,
                                                 const T* __restrict__ minv, const T* __restrict__ t, T c0,
                                                 TX* xout, const double* __restrict__ d, Red R) {
    if (skip_red(R)) return;
    long long lo, hi;
    chunk_range(nslices, lo, hi);
    double s0 = 0.0;
    for (long long i = lo * SLICE + threadIdx.x; i < hi * SLICE && i < n; i += WG) {
        const T xo = x[i] + c0 * minv[i] * t[i];
        xout[i] = (TX)xo;
        if (d) s0 += (double)(TX)xo * d[i];
    }
    if (R.fin != FIN_NONE) block_partial(s0, 0.0, R.part);
}

// Fused-iteration residual update without pre-smoothing (the factored
// smoothers start the V-cycle from r): r_new = r_old - alpha q, partial
// ||r_new||^2 (same reduction layout as k_update_pre_s).
__global__ __launch_bounds__(WG) void k_rupdate(long long nslices, long long n, const double* __restrict__ rold,
                                                const double* __restrict__ q, double* __restrict__ rnew, Red R,
                                                float* __restrict__ rnew32 = nullptr) {
    if (skip_red(R)) return;
    const double nalpha = -R.ctl->alpha;
    long long lo, hi;
    chunk_range(nslices, lo, hi);
    const long long end = hi * SLICE < n ? hi * SLICE : n;
    double s0 = 0.0;
    // two elements per thread (16-byte loads, aligned: the range starts on an
    // even index); q and r_old are loaded non-temporally, so that they do not
    // displace r_new, which the pre-smoothing pass gathers next (measured:
    // the two passes 961 -> 949 us at 384^3)
    long long i = lo * SLICE + 2 * threadIdx.x;
    for (; i + 1 < end; i += 2 * WG) {
        const v2a<double> qq = ntload((const v2a<double>*)(q + i)), rr = ntload((const v2a<double>*)(rold + i));
        const double r0 = fma(nalpha, qq.x, rr.x), r1 = fma(nalpha, qq.y, rr.y);
        st2(rnew + i, r0, r1);
        if (rnew32) st2(rnew32 + i, (float)r0, (float)r1);
        s0 += r0 * r0;
        s0 += r1 * r1;
    }
    if (i < end) {   // odd tail (last element)
        const double rn = fma(nalpha, q[i], rold[i]);
        rnew[i] = rn;
        if (rnew32) rnew32[i] = (float)rn;
        s0 += rn * rn;
    }
    block_partial(s0, 0.0, R.part);
}

struct GraphEntry {
    int form;
    const psc_net* net;
    uint64_t gen;
    hipGraphExec_t exec;
};

template <typename T>
struct DevEll {
    long long* off = nullptr;
    T* val = nullptr;
    int* col = nullptr;
    float* val32 = nullptr;
    long long nrows = 0, nslices = 0, slots = 0, ncols = 0, nnz = 0;
    int wmax = 0;                          // widest slice (entries per row)
    int pair = 0;                          // paired 128-row layout (see Ell)
    // capped layout (see Ell): per-slice overflow ranges and their entries
    long long* xs = nullptr;
    int* xc = nullptr;
    unsigned char* xl = nullptr;
    T* xv = nullptr;
    float* xv32 = nullptr;
    int cap = 0;                           // slots per row kept in the slices (0: plain layout)
    long long xents = 0;                   // overflow entries
    bool ovf_split = false;                // a slice's overflow is long: the split form shares it
    Ell<T> view() const {
        Ell<T> e{off, val, col, nrows, nslices, ncols};
        e.pair = pair;
        return e;
    }
    Ell<float> view32() const {
        Ell<float> e{off, val32, col, nrows, nslices, ncols};
        e.pair = pair;
        return e;
    }
    // the capped layout (xs != nullptr)
    EllC<T> cview() const {
        EllC<T> e;
        static_cast<Ell<T>&>(e) = view();
        e.xs = xs, e.xv = xv, e.xc = xc, e.xl = xl;
        return e;
    }
    EllC<float> cview32() const {
        EllC<float> e;
        static_cast<Ell<float>&>(e) = view32();
        e.xs = xs, e.xv = xv32, e.xc = xc, e.xl = xl;
        return e;
    }
};

// Hacked-DIA copy of a level operator; the scaled operator A M^-1 shares
// its start and offset arrays.
struct DevDia {
    int* start = nullptr;
    int* offs = nullptr;
    double* val = nullptr;
    float* val32 = nullptr;
    long long nrows = 0, nslices = 0, ncols = 0, slots = 0;
    int ndmax = 0;                         // most diagonals in one slice
    bool on() const { return start != nullptr; }
    int nd = 0;                            // uniform offsets in use (0: per-slice offsets)
    int nd_u = 0;                          // uniform offset count of the layout (0: not uniform)
    int uo[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int pair = 0;                          // paired 128-row layout (every uniform layout)
    template <typename T>
    Dia<T> make(const T* v) const {
        Dia<T> d{start, offs, v, nrows, nslices, ncols};
        d.nd = nd;
        for (int k = 0; k < 8; k++) d.uo[k] = uo[k];
        d.pair = pair;
        return d;
    }
    Dia<double> view(const double* v) const { return make<double>(v); }
    Dia<float> view32(const float* v) const { return make<float>(v); }
};

struct DevLevel {
    long long n = 0, nc = 0, nnz = 0;
    int nu = 1;                           // l1-Jacobi sweeps before and after the coarse correction
    DevDia Ad;                            // A in hacked DIA when that stores fewer bytes
    double* amd = nullptr;                // A M^-1 values in Ad's layout
    float* amd32 = nullptr;
    DevEll<double> A, R;                  // R = P^T (coarse rows, members as columns)
    DevEll<double> SP;                    // smoothed prolongator P - M^-1 A P
    // Pair restriction: when rows 2k and 2k+1 always share an aggregate and a
    // prolongator value (Poisson's 2x2x1 aggregates on the paired DIA
    // layout), R r = R2 h with h_k = r_2k + r_2k+1 (written by the
    // pre-smoothing pass) and R2 the coarse rows over pairs (value p_2k):
    // half the vector and half the entries. R2.off == nullptr: not eligible.
    DevEll<double> R2;
    double* h2 = nullptr;
    float* h2_32 = nullptr;
    double* am = nullptr;                 // A M^-1 values in A's hacked-ELL layout
    float* am32 = nullptr;
    Ell<double> am_view() const { Ell<double> e = A.view(); e.val = am; return e; }
    Ell<float> am_view32() const { Ell<float> e = A.view32(); e.val = am32; return e; }
    // capped hacked-ELL copy of A (and A M^-1 in its slots and records) for
    // levels whose row lengths vary widely; Ac.off == nullptr: none
    DevEll<double> Ac;
    double *acm = nullptr, *acm_x = nullptr;
    float *acm32 = nullptr, *acm32_x = nullptr;
    EllC<double> acm_view() const { EllC<double> e = Ac.cview(); e.val = acm; e.xv = acm_x; return e; }
    EllC<float> acm_view32() const { EllC<float> e = Ac.cview32(); e.val = acm32; e.xv = acm32_x; return e; }
    double* minv = nullptr;
    float* minv32 = nullptr;
    int* agg = nullptr;
    double* pval = nullptr;
    float* pval32 = nullptr;
    double *b = nullptr, *x = nullptr, *r = nullptr;      // level vectors (FP64 form)
    float *b32 = nullptr, *x32 = nullptr, *r32 = nullptr; // level vectors (FP32 form)
    // more than one smoothing sweep: second residual buffer, running sums
    // s (two buffers) and two post-smoothing iterates, per precision
    double *rb = nullptr, *s = nullptr, *sb = nullptr, *xt = nullptr, *xt2 = nullptr;
    float *rb32 = nullptr, *s32 = nullptr, *sb32 = nullptr, *xt32 = nullptr, *xt232 = nullptr;
    // AINV / INVK smoother: Z and W = D^-1 Z^T by rows, the prolongator P,
    // and the sweep's residual t and factor product u
    DevEll<double> Z, W, P;
    double *ft = nullptr, *fu = nullptr;
    float *ft32 = nullptr, *fu32 = nullptr;
    double* fd = nullptr;                  // polynomial smoother: second direction buffer
    float* fd32 = nullptr;
};

// Per-precision views of a level's vectors and operators.
template <typename T>
struct LV;
template <>
struct LV<double> {
    static double* b(DevLevel& V) { return V.b; }
    static double* x(DevLevel& V) { return V.x; }
    static double* r(DevLevel& V) { return V.r; }
    static double* rb(DevLevel& V) { return V.rb; }
    static double* s(DevLevel& V) { return V.s; }
    static double* sb(DevLevel& V) { return V.sb; }
    static double* xt(DevLevel& V) { return V.xt; }
    static double* xt2(DevLevel& V) { return V.xt2; }
    static const double* minv(const DevLevel& V) { return V.minv; }
    static Ell<double> R(const DevLevel& V) { return V.R.view(); }
    static Ell<double> R2(const DevLevel& V) { return V.R2.view(); }
    static double* h2(DevLevel& V) { return V.h2; }
    static Ell<double> SP(const DevLevel& V) { return V.SP.view(); }
    static Ell<double> A(const DevLevel& V) { return V.A.view(); }
    static const double* pv(const DevLevel& V) { return V.pval; }
    static double* ft(DevLevel& V) { return V.ft; }
    static double* fu(DevLevel& V) { return V.fu; }
    static double* fd(DevLevel& V) { return V.fd; }
    static Ell<double> Z(const DevLevel& V) { return V.Z.view(); }
    static Ell<double> W(const DevLevel& V) { return V.W.view(); }
    static Ell<double> P(const DevLevel& V) { return V.P.view(); }
};
template <>
struct LV<float> {
    static float* b(DevLevel& V) { return V.b32; }
    static float* x(DevLevel& V) { return V.x32; }
    static float* r(DevLevel& V) { return V.r32; }
    static float* rb(DevLevel& V) { return V.rb32; }
    static float* s(DevLevel& V) { return V.s32; }
    static float* sb(DevLevel& V) { return V.sb32; }
    static float* xt(DevLevel& V) { return V.xt32; }
    static float* xt2(DevLevel& V) { return V.xt232; }
    static const float* minv(const DevLevel& V) { return V.minv32; }
    static Ell<float> R(const DevLevel& V) { return V.R.view32(); }
    static Ell<float> R2(const DevLevel& V) { return V.R2.view32(); }
    static float* h2(DevLevel& V) { return V.h2_32; }
    static Ell<float> SP(const DevLevel& V) { return V.SP.view32(); }
    static Ell<float> A(const DevLevel& V) { return V.A.view32(); }
    static const float* pv(const DevLevel& V) { return V.pval32; }
    static float* ft(DevLevel& V) { return V.ft32; }
    static float* fu(DevLevel& V) { return V.fu32; }
    static float* fd(DevLevel& V) { return V.fd32; }
    static Ell<float> Z(const DevLevel& V) { return V.Z.view32(); }
    static Ell<float> W(const DevLevel& V) { return V.W.view32(); }
    static Ell<float> P(const DevLevel& V) { return V.P.view32(); }
};

}  // namespace psc

struct psc_hier {
    psc::HostHier host;
    std::vector<psc::DevLevel> lev;
    double* coarse_invT = nullptr;
    int coarse_n = 0;
    hipStream_t stream = nullptr;         // library work stream (owned, capturable)
    hipStream_t user_stream = nullptr;    // caller's stream; joined at entry and exit
    hipEvent_t ev_join[2] = {nullptr, nullptr};
    int device = 0;
    psc_amg_opts opts;
    bool has32 = false;
    // solver state
    psc::Ctl* ctl = nullptr;
    psc::HostCtl* hctl = nullptr;
    psc::HostCtl* hctl_dev = nullptr;
    double* part = nullptr;
    double* part2 = nullptr;              // middle-stage partials (2 x 256 doubles)
    double *xs = nullptr, *bs = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
    double *r2 = nullptr, *p2 = nullptr;  // second buffers of the fused PCG iteration
    bool fused_pcg = true;                // PCG form: fused two-pass iteration
    bool unroll4 = false;                 // gather in batches of 4 in the FP64 post / update+pre kernels
    int bufload = 2;                      // buffer descriptors: 0 none, 1 all ELL kernels, 2 post-smoothing only
    bool spmv2 = false;                   // plain SpMV / restriction: two slices per wavefront
    bool split = true;                    // smoothing sweeps through A M^-1 and A P
    bool dia = true;                      // use the hacked-DIA copies where a level has them
    bool capped = true;                   // use the capped hacked-ELL copies where a level has them
    bool pair_r = true;                   // pair restriction where a level is eligible
    bool dia_uniform = true;              // a level with <= 8 distinct offsets keeps them in the kernel argument
    bool dia_align = true;                // grids aligned to the largest DIA offset (grid_lvl)
    bool mixed_split = true;              // FP32 V-cycle: residual update and pre-smoothing as two passes
    bool fp64_split = true;               // FP64 V-cycle: the same two passes
    float* r32 = nullptr;                 // FP32 copy of the outer residual (mixed_split)
    float* z32 = nullptr;                 // the FP32 V-cycle's output of the mixed form, kept in FP32
    bool mixed_z32 = true;
    // Small levels in one workgroup (k_tail): off by default. Under graph
    // replay each small kernel costs about as much as one latency-bound round
    // inside the tail, so the per-level launches are as fast or faster
    // (measured at 128^3 and 256^3); without graphs the tail saves launches.
    bool tail = true;
    int tail_rows = -1;                   // largest level (rows) the tail takes; -1: automatic
    int tail_t = 0;                       // first level of the tail (0: no tail)
    int tail_lds = 0;                     // elements of the tail's LDS arrays
    int tail_pcg_bytes = 0;               // LDS after them for a PCG coarsest solve
    psc::TailDesc<double>* tail64 = nullptr;   // device descriptors (built at setup)
    psc::TailDesc<float>* tail32 = nullptr;
    bool tail_dia = true;                 // the DIA setting the descriptors were built with
    int nu = 1;                           // l1-Jacobi sweeps before and after the coarse correction
    bool fai = false;                     // AINV / INVK smoother on the levels above the coarsest
    bool cheb = false;                    // polynomial (fourth-kind Chebyshev) smoother
    std::vector<void*> allocs;
    std::vector<void*> lev_allocs;        // per-level device data (released by a numeric rebuild)
    int64_t lev_bytes = 0;
    bool lev_phase = false;               // dalloc records into lev_allocs
    // refresh: a numeric rebuild writes new values into the existing level
    // buffers (same sizes), skipping allocations and index arrays
    bool refresh = false;
    std::unordered_map<void*, size_t> asize;   // bytes of every level allocation
    void* stage = nullptr;                // rebuild staging of CSR rows and values (freed after it)
    size_t stage_bytes = 0;
    int64_t device_bytes = 0;
    double setup_seconds = 0.0;
    double rebuild_seconds = 0.0;         // last numeric rebuild
    bool stale = false;                   // a numeric rebuild failed: solves refused until one succeeds
    int gmax = psc::GDEF;                 // workgroup cap of the streaming kernels
    // captured iterations, one per (form, network, network generation)
    std::vector<psc::GraphEntry> graphs;
    // timing: 0 off, 1 every level-0 kernel and the whole V-cycle, 2 only
    // the outer SpMV pass (kernel id 0)
    int timing = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
    std::vector<int> ev_kind;
    std::vector<int> ev_iter;             // iteration a timed launch belongs to (-1: outside the loop)
    int t_iter = -1;                      // iteration being issued
    size_t ev_used = 0;
    int64_t t_count[PSC_TIMING_KERNELS] = {0};
    double t_ms[PSC_TIMING_KERNELS] = {0};
    std::vector<hipEvent_t> ring;
};

namespace psc {

static int dalloc(psc_hier* h, void** p, size_t bytes) {
    if (bytes == 0) bytes = 64;
    if (h->refresh) {
        // reuse the buffer of the same size; anything else needs a full re-upload
        auto it = *p ? h->asize.find(*p) : h->asize.end();
        if (it == h->asize.end() || it->second != bytes) return PSC_ERR_STATE;
        return PSC_OK;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return fail(PSC_ERR_OOM, "hipMalloc of " + std::to_string(bytes) + " bytes failed");
    (h->lev_phase ? h->lev_allocs : h->allocs).push_back(*p);
    if (h->lev_phase) {
        h->lev_bytes += (int64_t)bytes;
        h->asize[*p] = bytes;
    }
    h->device_bytes += (int64_t)bytes;
    return PSC_OK;
}

// Order the library's work stream after the caller's stream (entry) and the
// caller's stream after the library's work (exit).
static int join_in(psc_hier* h) {
    HIPCHK(hipEventRecord(h->ev_join[0], h->user_stream));
    HIPCHK(hipStreamWaitEvent(h->stream, h->ev_join[0], 0));
    return PSC_OK;
}
static int join_out(psc_hier* h) {
    HIPCHK(hipEventRecord(h->ev_join[1], h->stream));
    HIPCHK(hipStreamWaitEvent(h->user_stream, h->ev_join[1], 0));
    return PSC_OK;
}

template <typename T>
static int upload(psc_hier* h, T** d, const T* src, size_t count) {
    int st = dalloc(h, (void**)d, count * sizeof(T));
    if (st) return st;
    HIPCHK(hipMemcpy(*d, src, count * sizeof(T), hipMemcpyHostToDevice));
    return PSC_OK;
}

// Hacked-ELL copy of a CSR operator packed on the host (the factored
// smoothers' W and Z and their prolongator). value_pattern: the sparsity
// depends on the values (AINV factors), so a refresh rewrites the index
// arrays too (same sizes) instead of keeping them.
static int upload_ell(psc_hier* h, DevEll<double>& E, int64_t nrows, int64_t ncols, const int32_t* rp,
                      const int32_t* ci, const double* v, bool fp32, bool value_pattern = false) {
    std::vector<long long> off;
    std::vector<double> val;
    std::vector<int> col;
    pack_ell(nrows, rp, ci, v, off, val, col);
    E.nrows = nrows;
    E.ncols = ncols;
    E.nslices = (long long)off.size() - 1;
    E.slots = off.back();
    E.nnz = rp[nrows];
    for (size_t q = 0; q + 1 < off.size(); q++) E.wmax = std::max(E.wmax, (int)((off[q + 1] - off[q]) / SLICE));
    int st;
    if (h->refresh && !value_pattern) {
        // the pattern is the one uploaded at build: new values only
        if (E.off == nullptr || E.col == nullptr) return PSC_ERR_STATE;
    } else {
        if ((st = upload(h, &E.off, off.data(), off.size()))) return st;
        if ((st = upload(h, &E.col, col.data(), col.size()))) return st;
    }
    if ((st = upload(h, &E.val, val.data(), val.size()))) return st;
    if (fp32) {
        std::vector<float> v32(val.size());
        for (size_t i = 0; i < val.size(); i++) v32[i] = (float)val[i];
        if ((st = upload(h, &E.val32, v32.data(), v32.size()))) return st;
    }
    return PSC_OK;
}

// Numeric rebuild on an unchanged pattern: row i's new CSR values go into
// the slots the build gave them, hacked ELL (entry q of the row at
// off[s] + 64 q + lane, or off[s] + 128 q + lane in the paired layout) and,
// when the level has one, hacked DIA (slot
// (start[s] + k) 64 + lane, k the slice's diagonal of the entry's column),
// with A M^-1 (a_ij minv_j) and the FP32 copies formed on the way (a paired
// layout places slice s at (s >> 1) nd 128 + (s & 1) 64 with diagonal
// stride 128). Padding and empty diagonal slots keep the zeros the build wrote.
__global__ void k_refresh_values(long long n, const int32_t* __restrict__ rp, const double* __restrict__ v,
                                 const double* __restrict__ mv, const long long* __restrict__ off,
                                 const int* __restrict__ col, double* __restrict__ val, float* __restrict__ val32,
                                 double* __restrict__ am, float* __restrict__ am32, const int* __restrict__ dstart,
                                 const int* __restrict__ doffs, double* __restrict__ dval,
                                 float* __restrict__ dval32, double* __restrict__ damd,
                                 float* __restrict__ damd32, int dpair, int epair) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const long long s = i >> 6;
    const int lane = (int)(i & 63);
    const long long o = off[s] + lane;
    const long long estride = epair ? 2 * SLICE : SLICE;   // paired hacked ELL: slot stride 128
    const int32_t b = rp[i], e = rp[i + 1];
    const int k0 = dstart ? dstart[s] : 0, k1 = dstart ? dstart[s + 1] : 0;
    for (int32_t q = b; q < e; q++) {
        const long long slot = o + (long long)(q - b) * estride;
        const double x = v[q];
        const int c = col[slot];
        val[slot] = x;
        if (val32) val32[slot] = (float)x;
        double y = 0.0;
        if (am) {
            y = x * mv[c];
            am[slot] = y;
            if (am32) am32[slot] = (float)y;
        }
        if (dstart) {
            // the slice's offsets ascend: binary search for this column's diagonal
            const int d = c - (int)i;
            int lo = k0, hi = k1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (doffs[mid] < d) lo = mid + 1;
                else hi = mid;
            }
            const int k = lo;
            if (k < k1 && doffs[k] == d) {
                // paired layout: slice s is half (s & 1) of block s >> 1
                const long long ds = dpair ? (s >> 1) * (long long)(k1 - k0) * 2 * SLICE + (k - k0) * 2 * SLICE +
                                                 (s & 1) * SLICE + lane
                                           : (long long)k * SLICE + lane;
                dval[ds] = x;
                if (dval32) dval32[ds] = (float)x;
                if (damd) {
                    damd[ds] = y;
                    if (damd32) damd32[ds] = (float)y;
                }
            }
        }
    }
}

// The staging buffer lives only while the level data are filled (build or
// rebuild).
static void release_stage(psc_hier* h) {
    if (h->stage) (void)hipFree(h->stage);
    h->stage = nullptr;
    h->stage_bytes = 0;
}

// Device side of a refresh: stage the rows and values of a CSR operator with
// the pattern uploaded at build and scatter them (see k_refresh_values).
// mv != nullptr also refreshes A M^-1 (am / amd and their FP32 copies).
static int refresh_values(psc_hier* h, DevEll<double>& E, const DevDia* G, int64_t n, const int32_t* rp,
                          const double* v, const double* mv, double* am, float* am32, double* amd, float* amd32,
                          const int32_t** staged_rp = nullptr) {
    if (!E.off || !E.col || !E.val || E.nrows != n || E.nnz != (long long)rp[n]) return PSC_ERR_STATE;
    const size_t brp = ((size_t)(n + 1) * sizeof(int32_t) + 255) & ~(size_t)255;
    const size_t bv = ((size_t)rp[n] * sizeof(double) + 255) & ~(size_t)255;
    const size_t bm = mv ? (size_t)n * sizeof(double) : 0;
    const size_t need = brp + bv + bm;
    if (h->stage_bytes < need) {
        if (h->stage) HIPCHK(hipFree(h->stage));
        h->stage = nullptr;
        h->stage_bytes = 0;
        if (hipMalloc(&h->stage, need) != hipSuccess) return fail(PSC_ERR_OOM, "staging allocation failed");
        h->stage_bytes = need;
    }
    char* sb = (char*)h->stage;
    int32_t* drp = (int32_t*)sb;
    double* dv = (double*)(sb + brp);
    double* dm = mv ? (double*)(sb + brp + bv) : nullptr;
    HIPCHK(hipMemcpyAsync(drp, rp, (size_t)(n + 1) * sizeof(int32_t), hipMemcpyHostToDevice, h->stream));
    if (rp[n] > 0) HIPCHK(hipMemcpyAsync(dv, v, (size_t)rp[n] * sizeof(double), hipMemcpyHostToDevice, h->stream));
    if (mv) HIPCHK(hipMemcpyAsync(dm, mv, bm, hipMemcpyHostToDevice, h->stream));
    const bool dia = G && G->on();
    const long long blocks = (n + WG - 1) / WG;
    k_refresh_values<<<(unsigned)blocks, WG, 0, h->stream>>>(
        n, drp, dv, dm, E.off, E.col, E.val, E.val32, mv ? am : nullptr, mv ? am32 : nullptr,
        dia ? G->start : nullptr, dia ? G->offs : nullptr, dia ? G->val : nullptr, dia ? G->val32 : nullptr,
        (dia && mv) ? amd : nullptr, (dia && mv) ? amd32 : nullptr, dia ? G->pair : 0, E.pair);
    HIPCHK(hipGetLastError());
    // the staging buffer and the host arrays are reused or released next
    HIPCHK(hipStreamSynchronize(h->stream));
    if (staged_rp) *staged_rp = drp;   // valid until the next refresh_values call
    return PSC_OK;
}

// Allocation cleared to zero (padding and empty diagonal slots of a layout).
static int zalloc(psc_hier* h, void** p, size_t bytes) {
    int st = dalloc(h, p, bytes);
    if (st) return st;
    HIPCHK(hipMemsetAsync(*p, 0, bytes, h->stream));
    return PSC_OK;
}

// Hacked-ELL layout of a CSR operator on the device: slice offsets and
// columns packed on the host, value arrays (FP64, FP32 when fp32, and A M^-1
// when am != nullptr) allocated and cleared, for refresh_values to fill.
static int upload_ell_layout(psc_hier* h, DevEll<double>& E, int64_t nrows, int64_t ncols, const int32_t* rp,
                             const int32_t* ci, bool fp32, double** am = nullptr, float** am32 = nullptr,
                             bool paired = false) {
    std::vector<long long> off;
    std::vector<double> none;
    std::vector<int> col;
    E.nrows = nrows;
    E.ncols = ncols;
    E.nnz = rp[nrows];
    E.nslices = (nrows + SLICE - 1) / SLICE;
    E.pair = paired ? 1 : 0;
    if (paired) {
        pack_ell_paired(nrows, rp, ci, nullptr, off, none, col);
        E.slots = off.back();
        for (long long q = 0; q < E.nslices; q += 2)
            E.wmax = std::max(E.wmax, (int)((off[q + 2] - off[q]) / (2 * SLICE)));
    } else {
        pack_ell(nrows, rp, ci, nullptr, off, none, col);
        E.slots = off.back();
        for (size_t q = 0; q + 1 < off.size(); q++) E.wmax = std::max(E.wmax, (int)((off[q + 1] - off[q]) / SLICE));
    }
    int st;
    if ((st = upload(h, &E.off, off.data(), off.size()))) return st;
    if ((st = upload(h, &E.col, col.data(), col.size()))) return st;
    const size_t slots = (size_t)E.slots;
    if ((st = zalloc(h, (void**)&E.val, slots * sizeof(double)))) return st;
    if (fp32 && (st = zalloc(h, (void**)&E.val32, slots * sizeof(float)))) return st;
    if (am) {
        if ((st = zalloc(h, (void**)am, slots * sizeof(double)))) return st;
        if (fp32 && (st = zalloc(h, (void**)am32, slots * sizeof(float)))) return st;
    }
    return PSC_OK;
}

// Capped hacked-ELL copy of level operator A (see Ell) with, when mv is
// given, A M^-1 (a_ij mv_j) in the same slots and overflow, and FP32 copies
// when f32; built for levels of at least capped_min_rows rows when
// choose_ell_cap finds a cap that pays, refilled with the same cap by a
// numeric rebuild.
static std::vector<float> to32(const std::vector<double>& a);
static int upload_capped(psc_hier* h, DevLevel& D, const HostLevel& H, const double* mv, bool f32) {
    const int min_rows = h->opts.capped_min_rows;
    if (!h->refresh && (min_rows <= 0 || H.n < min_rows)) return PSC_OK;
    const int cap = h->refresh ? D.Ac.cap : choose_ell_cap(H.n, H.rp.data());
    if (cap <= 0) return PSC_OK;
    std::vector<long long> off, xs, xsrc;
    std::vector<double> val;
    std::vector<int> col, xc;
    std::vector<unsigned char> xl;
    pack_ell_capped(H.n, H.rp.data(), H.ci.data(), H.v.data(), cap, off, val, col, xs, xc, xl, xsrc);
    DevEll<double>& E = D.Ac;
    E.cap = cap;
    E.nrows = H.n;
    E.ncols = H.n;
    E.nnz = H.rp[H.n];
    E.nslices = (long long)off.size() - 1;
    E.slots = off.back();
    E.xents = (long long)xsrc.size();
    // slices with more than OVF_SPLIT_ROUNDS rounds of 64 overflow entries
    // bound the launch by their wavefront: the split form gives them four
    long long most = 0;
    for (size_t q = 0; q + 1 < xs.size(); q++) most = std::max(most, xs[q + 1] - xs[q]);
    E.ovf_split = most > (long long)OVF_SPLIT_ROUNDS * SLICE;
    E.wmax = 0;
    for (size_t q = 0; q + 1 < off.size(); q++) E.wmax = std::max(E.wmax, (int)((off[q + 1] - off[q]) / SLICE));
    std::vector<double> xv(xsrc.size());
    for (size_t e = 0; e < xsrc.size(); e++) xv[e] = H.v[xsrc[e]];
    int st;
    if ((st = upload(h, &E.off, off.data(), off.size()))) return st;
    if ((st = upload(h, &E.col, col.data(), col.size()))) return st;
    if ((st = upload(h, &E.xs, xs.data(), xs.size()))) return st;
    if ((st = upload(h, &E.xc, xc.data(), xc.size()))) return st;
    if ((st = upload(h, &E.xl, xl.data(), xl.size()))) return st;
    if ((st = upload(h, &E.val, val.data(), val.size()))) return st;
    if ((st = upload(h, &E.xv, xv.data(), xv.size()))) return st;
    if (f32) {
        auto v32 = to32(val), x32 = to32(xv);
        if ((st = upload(h, &E.val32, v32.data(), v32.size()))) return st;
        if ((st = upload(h, &E.xv32, x32.data(), x32.size()))) return st;
    }
    if (mv) {
        // A M^-1: the same product as the plain layout's refresh (a_ij mv_j);
        // padding slots hold 0
        std::vector<double> am(val.size()), amx(xv.size());
        for (size_t k = 0; k < val.size(); k++) am[k] = val[k] * mv[col[k]];
        for (size_t e = 0; e < xv.size(); e++) amx[e] = xv[e] * mv[xc[e]];
        if ((st = upload(h, &D.acm, am.data(), am.size()))) return st;
        if ((st = upload(h, &D.acm_x, amx.data(), amx.size()))) return st;
        if (f32) {
            auto a32 = to32(am), ax32 = to32(amx);
            if ((st = upload(h, &D.acm32, a32.data(), a32.size()))) return st;
            if ((st = upload(h, &D.acm32_x, ax32.data(), ax32.size()))) return st;
        }
    }
    return PSC_OK;
}

// Pair restriction of level D (see DevLevel::R2): eligible when P is
// tentative, the row count even, and rows 2k and 2k+1 share their aggregate
// and their prolongator value for every k; R2 holds the coarse rows over the
// pairs (ascending), value p_2k, and h2 (h2_32) the pair sums. A numeric
// rebuild refills R2's values, or turns it off when the pairs no longer agree.
static int upload_pair_r(psc_hier* h, DevLevel& D, const HostLevel& H, bool f32) {
    const int64_t n = H.n;
    bool ok = n > 0 && n % 2 == 0 && (int64_t)H.pci.size() == n && (int64_t)H.prp.size() == n + 1 &&
              H.prp[n] == n && (int64_t)H.pv.size() == n;
    for (int64_t k = 0; ok && k < n / 2; k++)
        ok = H.pci[2 * k] == H.pci[2 * k + 1] && H.pv[2 * k] == H.pv[2 * k + 1];
    if (!ok || (h->refresh && D.R2.off == nullptr)) {
        D.R2.off = nullptr;   // (a rebuild keeps the buffers until the handle is freed)
        return PSC_OK;
    }
    const int64_t np = n / 2;
    std::vector<int32_t> rrp(H.nc + 1, 0), rci(np);
    std::vector<double> rv(np);
    for (int64_t k = 0; k < np; k++) rrp[H.pci[2 * k] + 1]++;
    for (int64_t I = 0; I < H.nc; I++) rrp[I + 1] += rrp[I];
    std::vector<int32_t> pos(rrp.begin(), rrp.end() - 1);
    for (int64_t k = 0; k < np; k++) {
        const int32_t o = pos[H.pci[2 * k]]++;
        rci[o] = (int32_t)k;
        rv[o] = H.pv[2 * k];
    }
    int st;
    if (!h->refresh && (st = upload_ell_layout(h, D.R2, H.nc, np, rrp.data(), rci.data(), f32))) return st;
    if ((st = refresh_values(h, D.R2, nullptr, H.nc, rrp.data(), rv.data(), nullptr, nullptr, nullptr, nullptr,
                             nullptr)))
        return st;
    if ((st = dalloc(h, (void**)&D.h2, np * sizeof(double)))) return st;
    if (f32 && (st = dalloc(h, (void**)&D.h2_32, np * sizeof(float)))) return st;
    return PSC_OK;
}

static std::vector<float> to32(const std::vector<double>& a) {
    std::vector<float> r(a.size());
    for (size_t i = 0; i < a.size(); i++) r[i] = (float)a[i];
    return r;
}

// AINV / INVK factors of a level: W = D^-1 Z^T (row k = column k of Z over
// d_k) and Z by rows, the prolongator P, and the sweep vectors.
static int upload_fai(psc_hier* h, DevLevel& D, const HostLevel& H, bool f32) {
    const HostFai& F = H.fai;
    const int64_t n = H.n;
    int st;
    if (h->cheb) {
        // polynomial smoother: P and three work vectors per precision
        if ((st = upload_ell(h, D.P, n, H.nc, H.prp.data(), H.pci.data(), H.pv.data(), f32))) return st;
        for (double** q : {&D.ft, &D.fu, &D.fd})
            if ((st = dalloc(h, (void**)q, n * sizeof(double)))) return st;
        if (f32)
            for (float** q : {&D.ft32, &D.fu32, &D.fd32})
                if ((st = dalloc(h, (void**)q, n * sizeof(float)))) return st;
        return PSC_OK;
    }
    if ((int64_t)F.zr.size() != n + 1) return fail(PSC_ERR_STATE, "smoother factor missing on a level");
    const size_t nz = F.zi.size();
    std::vector<int32_t> wrp(n + 1), zrp(n + 1, 0), zci(nz);
    std::vector<double> wv(nz), zv(nz);
    for (int64_t k = 0; k <= n; k++) wrp[k] = (int32_t)F.zr[k];
    for (int64_t k = 0; k < n; k++)
        for (int64_t e = F.zr[k]; e < F.zr[k + 1]; e++) wv[e] = F.zv[e] / F.d[k];
    // rows of Z: columns ascending within a row
    for (size_t e = 0; e < nz; e++) zrp[F.zi[e] + 1]++;
    for (int64_t r = 0; r < n; r++) zrp[r + 1] += zrp[r];
    std::vector<int32_t> pos(zrp.begin(), zrp.end() - 1);
    for (int64_t k = 0; k < n; k++)
        for (int64_t e = F.zr[k]; e < F.zr[k + 1]; e++) {
            const int32_t o = pos[F.zi[e]]++;
            zci[o] = (int32_t)k;
            zv[o] = F.zv[e];
        }
    if ((st = upload_ell(h, D.W, n, n, wrp.data(), F.zi.data(), wv.data(), f32, true)))
        return st;
    if ((st = upload_ell(h, D.Z, n, n, zrp.data(), zci.data(), zv.data(), f32, true)))
        return st;
    if ((st = upload_ell(h, D.P, n, H.nc, H.prp.data(), H.pci.data(), H.pv.data(), f32))) return st;
    for (double** q : {&D.ft, &D.fu})
        if ((st = dalloc(h, (void**)q, n * sizeof(double)))) return st;
    if (f32)
        for (float** q : {&D.ft32, &D.fu32})
            if ((st = dalloc(h, (void**)q, n * sizeof(float)))) return st;
    return PSC_OK;
}

static int grid_of(const psc_hier* h, long long units_per_block_4, long long total) {
    // one workgroup per 4 slices (or 1024 vector elements) up to the cap,
    // rounded up to a multiple of the XCD count
    long long g = (total + units_per_block_4 - 1) / units_per_block_4;
    if (g > h->gmax) g = h->gmax;
    if (g < 1) g = 1;
    g = (g + NXCD - 1) / NXCD * NXCD;
    return (int)g;
}

static inline int grid_ell(const psc_hier* h, long long nslices) { return grid_of(h, 4, nslices); }

// Grid of the kernels that sweep level V's rows. Workgroup b runs on die
// b % 8 and its four wavefronts take `per` consecutive 128-row blocks of a
// paired layout one at a time, so per >= 4 keeps every wavefront busy (the
// default grid of four 64-row slices per workgroup leaves two of them idle).
// When V is read from a paired uniform hacked-DIA copy whose largest offset
// D is a whole number of blocks per die (D = 8 k 128 rows: the plane of a 3D
// stencil), `per` is also chosen to divide k, so that the rows D away from a
// workgroup's rows belong to a workgroup D / (128 per) = a multiple of 8
// launches away, on the same die: those gathers then find the lines the die
// fetched a plane earlier in its L2 instead of fetching them again through
// the fabric (PSC_TUNE_DIA_ALIGN = 0 skips this choice).
static bool split_A(const psc_hier* h, const DevLevel& V);

static int grid_lvl(const psc_hier* h, const DevLevel& V) {
    if (split_A(h, V)) return grid_of(h, 1, V.A.nslices);   // one slice per workgroup
    const int g = grid_ell(h, V.A.nslices);
    const DevDia& G = V.Ad;
    if (!h->dia || !G.on() || !G.pair || G.nd <= 0) return g;
    const long long nb = (G.nslices + 1) / 2;
    const long long per0 = std::max<long long>((nb + g - 1) / g, WG / 64);
    auto grid_for = [&](long long per) {
        const long long gg = (nb + per - 1) / per;
        return (gg + NXCD - 1) / NXCD * NXCD;
    };
    if (h->dia_align) {
        long long D = 0;
        for (int k = 0; k < G.nd; k++) D = std::max(D, (long long)std::abs(G.uo[k]));
        if (D > 0 && D % (2 * SLICE * NXCD) == 0) {
            const long long k8 = D / (2 * SLICE * NXCD);
            for (long long per = per0; per <= 2 * per0 && per <= k8; per++) {
                if (k8 % per) continue;
                const long long gg = grid_for(per);
                if (gg <= h->gmax && (nb + gg - 1) / gg == per) return (int)gg;
            }
        }
    }
    return (int)std::min<long long>(grid_for(per0), h->gmax);
}

// Call f with the level operator (FP64 / FP32) or its scaled form A M^-1 in
// the storage the level uses: hacked DIA when present and enabled, else the
// capped hacked ELL when present and enabled, else hacked ELL. All have the
// same slices, so grids do not change.
static inline bool capped_on(const psc_hier* h, const DevLevel& V) { return h->capped && V.Ac.off != nullptr; }
template <typename F>
static void with_A(const psc_hier* h, const DevLevel& V, F f) {
    if (h->dia && V.Ad.on()) f(V.Ad.view(V.Ad.val));
    else if (capped_on(h, V)) f(V.Ac.cview());
    else f(V.A.view());
}
template <typename F>
static void with_A32(const psc_hier* h, const DevLevel& V, F f) {
    if (h->dia && V.Ad.on()) f(V.Ad.view32(V.Ad.val32));
    else if (capped_on(h, V)) f(V.Ac.cview32());
    else f(V.A.view32());
}
template <typename F>
static void with_AM(const psc_hier* h, const DevLevel& V, F f) {
    if (h->dia && V.Ad.on()) f(V.Ad.view(V.amd));
    else if (capped_on(h, V) && V.acm) f(V.acm_view());
    else f(V.am_view());
}
template <typename F>
static void with_AM32(const psc_hier* h, const DevLevel& V, F f) {
    if (h->dia && V.Ad.on()) f(V.Ad.view32(V.amd32));
    else if (capped_on(h, V) && V.acm32) f(V.acm_view32());
    else f(V.am_view32());
}
template <typename T, typename F>
static void with_A_t(const psc_hier* h, const DevLevel& V, F f) {
    if constexpr (std::is_same<T, float>::value) with_A32(h, V, f);
    else with_A(h, V, f);
}
template <typename T, typename F>
static void with_AM_t(const psc_hier* h, const DevLevel& V, F f) {
    if constexpr (std::is_same<T, float>::value) with_AM32(h, V, f);
    else with_AM(h, V, f);
}
// Rows wider than 8 entries take the 8-slot batch kernels (more registers,
// more loads in flight); stencil operators keep the 4-slot ones.
static bool wide_A(const psc_hier* h, const DevLevel& V) {
    return (h->dia && V.Ad.on()) ? V.Ad.ndmax > 8 : (capped_on(h, V) ? V.Ac.wmax : V.A.wmax) > 8;
}
// Level V's operator read from hacked ELL with rows wider than SPLIT_W slots:
// its kernels take the split form (GB_SPLIT) on one slice per workgroup.
static bool split_A(const psc_hier* h, const DevLevel& V) {
    if (h->dia && V.Ad.on()) return false;
    if (capped_on(h, V)) return V.Ac.wmax > SPLIT_W || V.Ac.ovf_split;
    return V.A.wmax > SPLIT_W;
}
// Level V restricts pair sums (see DevLevel::R2): eligible, enabled, and
// its one pre-smoothing sweep runs the paired uniform DIA path that writes
// them.
static bool use_pr(const psc_hier* h, const DevLevel& V) {
    return h->pair_r && V.R2.off != nullptr && h->split && h->dia && V.Ad.on() && V.Ad.pair && V.Ad.nd > 0 &&
           V.nu == 1;
}
template <typename T>
static T* pr_out(const psc_hier* h, DevLevel& V) {
    return use_pr(h, V) ? LV<T>::h2(V) : nullptr;
}
// The mixed form's z in FP32: the FP32 V-cycle computes it in FP32, so the
// FP32 copy holds exactly the values the FP64 one would (the level-0
// post-smoothing writes it, the next outer pass widens it on reading), in
// half the bytes. l1-Jacobi split V-cycle only.
static float* mixed_z(const psc_hier* h) {
    return (h->mixed_z32 && h->z32 && h->split && !h->fai && !h->cheb && h->lev.size() > 1 && h->bufload != 1)
               ? h->z32
               : nullptr;
}
static inline int grid_vec(const psc_hier* h, long long n) { return grid_of(h, 1024, n); }

// ---------------------------------------------------------------------------
// timing
// ---------------------------------------------------------------------------

struct TimeScope {
    psc_hier* h;
    int kind;
    size_t idx = (size_t)-1;
    TimeScope(psc_hier* hh, int k) : h(hh), kind(k) {
        if (!h->timing || (h->timing == 2 && kind != 0)) return;
        if (h->ev_used >= h->ev_pool.size()) {
            hipEvent_t a, b;
            if (hipEventCreate(&a) != hipSuccess) return;
            if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
            h->ev_pool.push_back({a, b});
            h->ev_kind.push_back(0);
            h->ev_iter.push_back(-1);
        }
        idx = h->ev_used++;
        h->ev_kind[idx] = kind;
        h->ev_iter[idx] = h->t_iter;
        (void)hipEventRecord(h->ev_pool[idx].first, h->stream);
    }
    ~TimeScope() {
        if (idx != (size_t)-1) (void)hipEventRecord(h->ev_pool[idx].second, h->stream);
    }
};

// Accumulate the recorded launch durations. After a solve of `iters`
// iterations, launches issued past convergence (they exit at entry) are left
// out: the outer-pass kernels (ids 0-2) of iteration i ran when i < iters, the
// V-cycle kernels (ids 3-7) when i < iters - vc_lag (vc_lag = 1 where the
// V-cycle closes an iteration, after its convergence test; 0 where it opens
// one). iters < 0: keep every launch.
static void timing_collect(psc_hier* h, int iters = -1, int vc_lag = 0) {
    if (!h->timing || h->ev_used == 0) return;
    (void)hipStreamSynchronize(h->stream);
    for (size_t i = 0; i < h->ev_used; i++) {
        const int it = h->ev_iter[i];
        if (iters >= 0 && it >= 0 && it >= (h->ev_kind[i] <= 2 ? iters : iters - vc_lag)) continue;
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, h->ev_pool[i].first, h->ev_pool[i].second) == hipSuccess) {
            h->t_count[h->ev_kind[i]] += 1;
            h->t_ms[h->ev_kind[i]] += ms;
        }
    }
    h->ev_used = 0;
}

// ---------------------------------------------------------------------------
// launch helpers (variant selection)
// ---------------------------------------------------------------------------

// Pre-smoothing from zero and its residual on level V, in the V-cycle's
// precision T (r = b - A M^-1 b).
template <typename T, typename TB>
static void launch_pre(psc_hier* h, DevLevel& V, const TB* b, T* r, Gate g, int grid = 0) {
    const int gr = grid ? grid : grid_lvl(h, V);
    constexpr bool f32 = std::is_same<T, float>::value;
    if (h->split) {
        const bool wide = wide_A(h, V), spl = split_A(h, V);
        T* hp = pr_out<T>(h, V);
        auto go = [&](auto AM) {
            if (spl) k_pre_s<decltype(AM), TB, GB_SPLIT><<<gr, WG, 0, h->stream>>>(AM, b, r, g, hp);
            else if (wide) k_pre_s<decltype(AM), TB, 8><<<gr, WG, 0, h->stream>>>(AM, b, r, g, hp);
            else k_pre_s<decltype(AM), TB, 4><<<gr, WG, 0, h->stream>>>(AM, b, r, g, hp);
        };
        if constexpr (f32) with_AM32(h, V, go);
        else with_AM(h, V, go);
        return;
    }
    const T* minv;
    Ell<T> A;
    if constexpr (f32) { minv = V.minv32; A = V.A.view32(); }
    else { minv = V.minv; A = V.A.view(); }
    if (h->bufload == 1) k_pre<T, TB, true><<<gr, WG, 0, h->stream>>>(A, minv, b, r, g);
    else k_pre<T, TB, false><<<gr, WG, 0, h->stream>>>(A, minv, b, r, g);
}

// y = A x for an operator in either storage; the variant knobs apply to ELL.
template <typename M>
static void launch_spmv(psc_hier* h, const M& A, const typename M::value_type* x, typename M::value_type* y,
                        Gate g, bool wide = false, bool split = false) {
    using T = typename M::value_type;
    const int gr = grid_ell(h, A.nslices);
    if constexpr (is_ell<M>::value) {
        if (split) {
            k_spmv<M, false, GB_SPLIT><<<grid_of(h, 1, A.nslices), WG, 0, h->stream>>>(A, x, y, g);
            return;
        }
        if constexpr (std::is_same<M, Ell<T>>::value) {
            if (h->spmv2) {
                // two slices per wavefront: half the workgroups of the one-slice grid
                k_spmv2<T><<<grid_of(h, 8, A.nslices), WG, 0, h->stream>>>(A, x, y, g);
                return;
            }
        }
        if (h->bufload == 1) {
            k_spmv<M, true><<<gr, WG, 0, h->stream>>>(A, x, y, g);
            return;
        }
    }
    if (wide) k_spmv<M, false, 8><<<gr, WG, 0, h->stream>>>(A, x, y, g);
    else k_spmv<M, false, 4><<<gr, WG, 0, h->stream>>>(A, x, y, g);
}

template <typename T, typename TB, typename TX>
static void launch_post(psc_hier* h, int gr, const Ell<T>& A, const Ell<T>& SP, const T* minv, const TB* b,
                        const T* r, const int* agg, const T* pv, const T* xc, long long nc, TX* x, const double* d,
                        const Red& R) {
    if (h->split) k_post_s<T, TB, TX><<<gr, WG, 0, h->stream>>>(SP, minv, b, r, xc, x, d, R);
    else if (h->bufload >= 1) k_post<T, TB, TX, 8, true><<<gr, WG, 0, h->stream>>>(A, minv, b, agg, pv, xc, nc, x, d, R);
    else if (h->unroll4) k_post<T, TB, TX, 4, false><<<gr, WG, 0, h->stream>>>(A, minv, b, agg, pv, xc, nc, x, d, R);
    else k_post<T, TB, TX, 8, false><<<gr, WG, 0, h->stream>>>(A, minv, b, agg, pv, xc, nc, x, d, R);
}

// ---------------------------------------------------------------------------
// V-cycle
// ---------------------------------------------------------------------------

static Red red_of(psc_hier* h, int fin, int gmode = GATE_DONE) {
    return Red{h->part, h->ctl, h->hctl_dev, fin, gmode};
}

// Remaining reduction stages for a kernel launched with `grid` workgroups:
// up to 1024 partial pairs are added by one workgroup; more go through a
// middle stage of up to 256 workgroups first (fixed order either way).
static void finish(psc_hier* h, const Red& R, int grid) {
    if (R.fin == FIN_NONE) return;
    if (grid <= 1024) {
        k_finish<<<1, WG, 0, h->stream>>>(R, grid);
        return;
    }
    const int mid = std::min(256, (grid + WG - 1) / WG);
    k_finish_mid<<<mid, WG, 0, h->stream>>>(R, grid, h->part2);
    Red R2 = R;
    R2.part = h->part2;
    k_finish<<<1, WG, 0, h->stream>>>(R2, mid);
}

// Coarsest solve x = B_L b: the explicit dense inverse, or coarse_sweeps
// l1-Jacobi sweeps in FP64 from zero. The sweeps alternate between the
// level's FP64 x and r buffers so that the last one lands in x (TX = double)
// or is rounded into the FP32 x32 (TX = float).
template <typename TB, typename TX>
static void coarse_solve(psc_hier* h, const TB* b, TX* x, Gate g) {
    DevLevel& C = h->lev.back();
    if (h->host.coarse_pcg > 0) {
        k_coarse_pcg<TB, TX><<<1, CPCG_WG, 0, h->stream>>>(C.A.view(), C.minv, b, x, h->host.coarse_pcg,
                                                          h->host.coarse_rtol, g);
        return;
    }
    const int K = h->host.coarse_sweeps;
    if (K == 0) {
        k_coarse<TB, TX><<<1, WG, 0, h->stream>>>(h->coarse_n, h->coarse_invT, b, x, g);
        return;
    }
    const int gr = grid_lvl(h, C);
    const bool wide = wide_A(h, C), spl = split_A(h, C);
    with_A(h, C, [&](auto A) {
        using M = decltype(A);
        const double* xin = nullptr;
        for (int k = 1; k < K; k++) {
            double* xo = ((K - k) % 2 == 0) ? C.x : C.r;
            if (spl) k_jacobi<M, TB, double, GB_SPLIT><<<gr, WG, 0, h->stream>>>(A, C.minv, b, xin, xo, g);
            else if (wide) k_jacobi<M, TB, double, 8><<<gr, WG, 0, h->stream>>>(A, C.minv, b, xin, xo, g);
            else k_jacobi<M, TB, double, 4><<<gr, WG, 0, h->stream>>>(A, C.minv, b, xin, xo, g);
            xin = xo;
        }
        if (spl) k_jacobi<M, TB, TX, GB_SPLIT><<<gr, WG, 0, h->stream>>>(A, C.minv, b, xin, x, g);
        else if (wide) k_jacobi<M, TB, TX, 8><<<gr, WG, 0, h->stream>>>(A, C.minv, b, xin, x, g);
        else k_jacobi<M, TB, TX, 4><<<gr, WG, 0, h->stream>>>(A, C.minv, b, xin, x, g);
    });
}

// Descriptors of the small levels run by k_tail: levels t..L-1 with at most
// TAIL_MAX_ROWS rows (t >= 1, at least one level above the coarsest), for a
// V-cycle with l1-Jacobi sweeps on the split operators and a dense coarsest
// solve.
template <typename T>
static TailLevel<T> tail_level(const psc_hier* h, const DevLevel& V) {
    TailLevel<T> e{};
    constexpr bool f32 = std::is_same<T, float>::value;
    if constexpr (f32) {
        e.am_ell = V.am_view32();
        if (V.Ad.on()) e.am_dia = V.Ad.view32(V.amd32);
        e.a_ell = V.A.view32();
        if (V.Ad.on()) e.a_dia = V.Ad.view32(V.Ad.val32);
        e.R = V.R.view32();
        e.SP = V.SP.view32();
        e.minv = V.minv32;
        e.b = V.b32;
        e.x = V.x32;
    } else {
        e.am_ell = V.am_view();
        if (V.Ad.on()) e.am_dia = V.Ad.view(V.amd);
        e.a_ell = V.A.view();
        if (V.Ad.on()) e.a_dia = V.Ad.view(V.Ad.val);
        e.R = V.R.view();
        e.SP = V.SP.view();
        e.minv = V.minv;
        e.b = V.b;
        e.x = V.x;
    }
    e.dia = (h->dia && V.Ad.on()) ? 1 : 0;
    e.nu = V.nu;
    return e;
}

static int build_tail(psc_hier* h) {
    const int L = (int)h->lev.size();
    h->tail_t = 0;
    if (L < 3 || h->host.coarse_sweeps > 0 || !h->split || h->fai || h->cheb) return PSC_OK;
    const bool cpcg = h->host.coarse_pcg > 0;
    if (cpcg && h->lev[L - 1].n > CPCG_MAX) return PSC_OK;
    // the PCG coarsest solve's direction and block sums (FP64, after the level arrays)
    const long long pcg_bytes = cpcg ? (long long)(CPCG_MAX + CPCG_WG / 64) * sizeof(double) : 0;
    for (int l = 0; l < L - 1; l++)
        if (h->lev[l].nu < 1) return PSC_OK;
    // automatic: the levels up to 1024 rows with one sweep per level (taking
    // the 4096-row level as well measured the same), up to 4096 rows with
    // several, where each sweep would otherwise be a launch of its own
    const int rows = h->tail_rows >= 0 ? h->tail_rows : ((h->nu > 1 || h->opts.vcycle_double) ? 4096 : 1024);
    // one workgroup streams a level's operators through one compute unit: by
    // default a level joins only while a sweep's operator bytes stay small
    // enough to be latency-bound there (wide coarse operators, as the smoothed
    // prolongator and VBM build, run faster spread over the chip); an explicit
    // row limit is taken as given
    auto op_bytes = [&](int l) {
        const DevLevel& V = h->lev[l];
        const long long a = (h->dia && V.Ad.on()) ? V.Ad.slots * 8LL : V.A.slots * 12LL;
        return a + V.SP.slots * 12LL;
    };
    int t = L - 1;
    while (t - 1 >= 1 && h->lev[t - 1].n <= rows && (h->tail_rows >= 0 || op_bytes(t - 1) <= TAIL_MAX_LEVEL_BYTES))
        t--;
    if (t > L - 2 || h->lev[L - 1].n > TAIL_MAX_ROWS) return PSC_OK;
    // LDS: b and r (and s) of levels t .. L-1, x over r or s (FP64 sized, so
    // the FP32 tail fits too); drop the largest tail levels until that fits in
    // what a workgroup may take
    int dev = 0, lds_max = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    lds_max = std::min(lds_max, TAIL_LDS_BYTES);
    auto width = [&](int l) { return (l < L - 1 && h->lev[l].nu > 1) ? 3 : 2; };   // b, r (, s)
    auto lds_of = [&](int t0) {
        long long e = 0;
        for (int l = t0; l < L; l++) e += width(l) * h->lev[l].n;
        return e;
    };
    while (t <= L - 2 && lds_of(t) * (long long)sizeof(double) + pcg_bytes > lds_max) t++;
    if (t > L - 2) return PSC_OK;
    const int lds_bytes = (int)(lds_of(t) * (long long)sizeof(double) + pcg_bytes);
    // the limit is per kernel and process-wide: raise it to what the device
    // allows, never to this handle's size (another handle may need more)
    if (lds_bytes > 64 * 1024 &&
        (hipFuncSetAttribute((const void*)k_tail<double>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max) !=
             hipSuccess ||
         hipFuncSetAttribute((const void*)k_tail<float>, hipFuncAttributeMaxDynamicSharedMemorySize, lds_max) !=
             hipSuccess)) {
        // the runtime refuses more than 64 KB: keep to that
        (void)hipGetLastError();
        while (t <= L - 2 && lds_of(t) * (long long)sizeof(double) + pcg_bytes > 64 * 1024) t++;
        if (t > L - 2) return PSC_OK;
    }
    TailDesc<double> d64{};
    TailDesc<float> d32{};
    {
        int e = 0;
        for (int l = t; l < L; l++) {
            d64.base[l] = d32.base[l] = e;
            e += width(l) * (int)h->lev[l].n;
        }
        d64.lds_elems = d32.lds_elems = e;
    }
    d64.t = d32.t = t;
    d64.L = d32.L = L;
    d64.nL = d32.nL = h->coarse_n;
    d64.invT = d32.invT = h->coarse_invT;
    d64.cmaxit = d32.cmaxit = cpcg ? h->host.coarse_pcg : 0;
    d64.crtol = d32.crtol = h->host.coarse_rtol;
    d64.cA = d32.cA = h->lev[L - 1].A.view();
    d64.cminv = d32.cminv = h->lev[L - 1].minv;
    d64.cpcg_off = (int)(((long long)d64.lds_elems * (long long)sizeof(double) + 7) & ~7LL);
    d32.cpcg_off = (int)(((long long)d32.lds_elems * (long long)sizeof(float) + 7) & ~7LL);
    for (int l = t; l < L; l++) {
        d64.lev[l] = tail_level<double>(h, h->lev[l]);
        if (h->has32) d32.lev[l] = tail_level<float>(h, h->lev[l]);
    }
    int st;
    if (!h->tail64 && (st = dalloc(h, (void**)&h->tail64, sizeof(TailDesc<double>)))) return st;
    if (h->has32 && !h->tail32 && (st = dalloc(h, (void**)&h->tail32, sizeof(TailDesc<float>)))) return st;
    HIPCHK(hipMemcpy(h->tail64, &d64, sizeof(d64), hipMemcpyHostToDevice));
    if (h->has32) HIPCHK(hipMemcpy(h->tail32, &d32, sizeof(d32), hipMemcpyHostToDevice));
    h->tail_dia = h->dia;
    h->tail_lds = d64.lds_elems;
    h->tail_pcg_bytes = (int)pcg_bytes;
    h->tail_t = t;
    return PSC_OK;
}

template <typename T>
static const TailDesc<T>* tail_desc(const psc_hier* h) {
    if constexpr (std::is_same<T, float>::value) return h->tail32;
    else return h->tail64;
}

// Residual buffer of pre-smoothing sweep k (1..nu) on a level: the buffers
// alternate so that the last sweep's residual lands in r (read by the
// restriction and the first post-smoothing sweep).
template <typename T>
static T* pre_rbuf(const psc_hier*, DevLevel& V, int k) {
    return ((V.nu - k) % 2 == 0) ? LV<T>::r(V) : LV<T>::rb(V);
}

// nu pre-smoothing sweeps from zero on level V (b: the level's right-hand
// side, FP64 at level 0). Sweep 1 is skipped when a fused kernel has done it.
template <typename T, typename TB>
static void pre_sweeps(psc_hier* h, DevLevel& V, const TB* b, bool skip1, Gate g) {
    const int gr = grid_lvl(h, V);
    if (!skip1) launch_pre(h, V, b, pre_rbuf<T>(h, V, 1), g);
    const T* rp = pre_rbuf<T>(h, V, 1);
    const T* sp = nullptr;
    for (int k = 2; k <= V.nu; k++) {
        T* so = ((V.nu - k) % 2 == 0) ? LV<T>::s(V) : LV<T>::sb(V);
        T* ro = pre_rbuf<T>(h, V, k);
        const bool wide = wide_A(h, V), spl = split_A(h, V);
        with_AM_t<T>(h, V, [&](auto AM) {
            using M = decltype(AM);
            if (k == 2) {
                if (spl) k_presweep<M, TB, TB, GB_SPLIT><<<gr, WG, 0, h->stream>>>(AM, b, b, rp, so, ro, g);
                else if (wide) k_presweep<M, TB, TB, 8><<<gr, WG, 0, h->stream>>>(AM, b, b, rp, so, ro, g);
                else k_presweep<M, TB, TB, 4><<<gr, WG, 0, h->stream>>>(AM, b, b, rp, so, ro, g);
            } else {
                if (spl) k_presweep<M, TB, T, GB_SPLIT><<<gr, WG, 0, h->stream>>>(AM, b, sp, rp, so, ro, g);
                else if (wide) k_presweep<M, TB, T, 8><<<gr, WG, 0, h->stream>>>(AM, b, sp, rp, so, ro, g);
                else k_presweep<M, TB, T, 4><<<gr, WG, 0, h->stream>>>(AM, b, sp, rp, so, ro, g);
            }
        });
        sp = so;
        rp = ro;
    }
}

// nu post-smoothing sweeps on level V after the coarse correction xc; the
// first is fused with the prolongation (x = M^-1 (s_nu + r_nu) + S P xc,
// with s_1 = b), the others are plain sweeps through two scratch iterates.
// The last writes out (FP64 z at level 0) with the reduction Rf.
template <typename T, typename TB, typename TX>
static void post_sweeps(psc_hier* h, DevLevel& V, const TB* b, TX* out, const T* xc, const double* d,
                        const Red& Rf) {
    const int gr = grid_lvl(h, V);
    Red Rn = Rf;
    Rn.fin = FIN_NONE;
    const Ell<T> SP = LV<T>::SP(V);
    const T* r = LV<T>::r(V);
    const T* minv = LV<T>::minv(V);
    const bool wsp = V.SP.wmax > 8, ssp = V.SP.wmax > SPLIT_W, wa = wide_A(h, V), sa = split_A(h, V);
    if (V.nu == 1) {
        if (ssp) k_post_s<T, TB, TX, GB_SPLIT><<<gr, WG, 0, h->stream>>>(SP, minv, b, r, xc, out, d, Rf);
        else if (wsp) k_post_s<T, TB, TX, 8><<<gr, WG, 0, h->stream>>>(SP, minv, b, r, xc, out, d, Rf);
        else k_post_s<T, TB, TX, 4><<<gr, WG, 0, h->stream>>>(SP, minv, b, r, xc, out, d, Rf);
        return;
    }
    T* ta = LV<T>::xt(V);
    T* tb = LV<T>::xt2(V);
    const T* sn = LV<T>::s(V);
    if (ssp) k_post_s<T, T, T, GB_SPLIT><<<gr, WG, 0, h->stream>>>(SP, minv, sn, r, xc, ta, nullptr, Rn);
    else if (wsp) k_post_s<T, T, T, 8><<<gr, WG, 0, h->stream>>>(SP, minv, sn, r, xc, ta, nullptr, Rn);
    else k_post_s<T, T, T, 4><<<gr, WG, 0, h->stream>>>(SP, minv, sn, r, xc, ta, nullptr, Rn);
    const T* xin = ta;
    for (int k = 2; k <= V.nu; k++) {
        with_A_t<T>(h, V, [&](auto A) {
            using M = decltype(A);
            if (k == V.nu) {
                if (sa) k_sweep<M, TB, TX, GB_SPLIT><<<gr, WG, 0, h->stream>>>(A, minv, b, xin, out, d, Rf);
                else if (wa) k_sweep<M, TB, TX, 8><<<gr, WG, 0, h->stream>>>(A, minv, b, xin, out, d, Rf);
                else k_sweep<M, TB, TX, 4><<<gr, WG, 0, h->stream>>>(A, minv, b, xin, out, d, Rf);
            } else {
                T* xo = xin == ta ? tb : ta;
                if (sa) k_sweep<M, TB, T, GB_SPLIT><<<gr, WG, 0, h->stream>>>(A, minv, b, xin, xo, nullptr, Rn);
                else if (wa) k_sweep<M, TB, T, 8><<<gr, WG, 0, h->stream>>>(A, minv, b, xin, xo, nullptr, Rn);
                else k_sweep<M, TB, T, 4><<<gr, WG, 0, h->stream>>>(A, minv, b, xin, xo, nullptr, Rn);
                xin = xo;
            }
        });
    }
}

// The V-cycle below level 0's right-hand side r0 in precision T (split sweeps).
// r0_32: when not NULL, an FP32 copy of r0 ((float) r0 element by element),
// read by the FP32 level-0 post-smoothing instead of r0 (same values, half
// the bytes).
template <typename T>
static void vcycle_t(psc_hier* h, const double* r0, double* z0, const double* d, const Red& R, Gate g,
                     bool skip_pre0, const float* r0_32 = nullptr, float* z32 = nullptr) {
    const int L = (int)h->lev.size();
    Red R0 = R;
    R0.fin = FIN_NONE;
    // levels from tl on run in one workgroup (k_tail) when that is set up
    const bool tail = h->tail && h->tail_t > 0 && h->split && h->tail_dia == h->dia;
    const int tl = tail ? h->tail_t : L - 1;
    for (int l = 0; l < tl; l++) {
        DevLevel& V = h->lev[l];
        if (!(l == 0 && skip_pre0 && V.nu == 1)) {
            TimeScope t(h, l == 0 ? 2 : 7);
            if (l == 0) pre_sweeps<T, double>(h, V, r0, skip_pre0, g);
            else pre_sweeps<T, T>(h, V, (const T*)LV<T>::b(V), false, g);
        }
        {
            TimeScope t(h, l == 0 ? 3 : 7);
            if (use_pr(h, V))
                launch_spmv(h, LV<T>::R2(V), (const T*)LV<T>::h2(V), LV<T>::b(h->lev[l + 1]), g, V.R2.wmax > 8);
            else
                launch_spmv(h, LV<T>::R(V), (const T*)LV<T>::r(V), LV<T>::b(h->lev[l + 1]), g, V.R.wmax > 8,
                            V.R.wmax > SPLIT_W);
        }
    }
    if (tail) {
        TimeScope t(h, 7);
        const size_t lds = (((size_t)h->tail_lds * sizeof(T) + 7) & ~(size_t)7) + (size_t)h->tail_pcg_bytes;
        k_tail<T><<<1, TAIL_WG, lds, h->stream>>>(tail_desc<T>(h), g);
    } else {
        DevLevel& C = h->lev[L - 1];
        TimeScope t(h, 7);
        coarse_solve<T, T>(h, (const T*)LV<T>::b(C), LV<T>::x(C), g);
    }
    for (int l = tl - 1; l >= 0; l--) {
        DevLevel& V = h->lev[l];
        const T* xc = LV<T>::x(h->lev[l + 1]);
        if (l == 0) {
            {
                TimeScope t(h, 4);
                if constexpr (std::is_same<T, float>::value) {
                    // z32: the output kept in FP32 (its values are FP32 anyway)
                    if (h->split && r0_32 && z32) post_sweeps<T, float, float>(h, V, r0_32, z32, xc, d, R);
                    else if (h->split && r0_32) post_sweeps<T, float, double>(h, V, r0_32, z0, xc, d, R);
                    else if (h->split && z32) post_sweeps<T, double, float>(h, V, r0, z32, xc, d, R);
                    else if (h->split) post_sweeps<T, double, double>(h, V, r0, z0, xc, d, R);
                }
                if constexpr (std::is_same<T, double>::value) {
                    if (h->split) post_sweeps<T, double, double>(h, V, r0, z0, xc, d, R);
                }
                if (!h->split)
                    launch_post(h, grid_lvl(h, V), LV<T>::A(V), LV<T>::SP(V), LV<T>::minv(V), r0, (const T*)LV<T>::r(V),
                                V.agg, LV<T>::pv(V), xc, V.nc, z0, d, R);
            }
            finish(h, R, grid_lvl(h, V));
        } else {
            TimeScope t(h, 7);
            if (h->split) post_sweeps<T, T, T>(h, V, (const T*)LV<T>::b(V), LV<T>::x(V), xc, nullptr, R0);
            else launch_post(h, grid_lvl(h, V), LV<T>::A(V), LV<T>::SP(V), LV<T>::minv(V), (const T*)LV<T>::b(V),
                             (const T*)LV<T>::r(V), V.agg, LV<T>::pv(V), xc, V.nc, LV<T>::x(V), (const double*)nullptr,
                             R0);
        }
    }
}

// The V-cycle with the AINV / INVK smoother in precision T: on each level
// above the coarsest, nu sweeps x <- x + Z W (b - A x) from x = 0 (the first
// is x = Z W b), the residual r = b - A x restricted; after the coarse
// correction x += P x_c, nu more sweeps, the last one at level 0 writing z0
// (FP64) with the fused dot z0 . d.
template <typename T>
static void vcycle_fai(psc_hier* h, const double* r0, double* z0, const double* d, const Red& R, Gate g) {
    const int L = (int)h->lev.size();
    Red R0 = R;
    R0.fin = FIN_NONE;
    hipStream_t st = h->stream;
    auto wide = [](const DevEll<double>& E) { return E.wmax > 8; };
    // t = b - A x
    auto resid = [&](DevLevel& V, auto b, const T* x, T* t) {
        using TB = std::remove_const_t<std::remove_pointer_t<decltype(b)>>;
        const int gr = grid_lvl(h, V);
        const bool wa = wide_A(h, V), sa = split_A(h, V);
        with_A_t<T>(h, V, [&](auto A) {
            using M = decltype(A);
            if (sa) k_fres<M, TB, GB_SPLIT><<<gr, WG, 0, st>>>(A, b, x, t, g);
            else if (wa) k_fres<M, TB, 8><<<gr, WG, 0, st>>>(A, b, x, t, g);
            else k_fres<M, TB, 4><<<gr, WG, 0, st>>>(A, b, x, t, g);
        });
    };
    auto wprod = [&](DevLevel& V, auto t, T* u) {
        using TB = std::remove_const_t<std::remove_pointer_t<decltype(t)>>;
        const int gr = grid_ell(h, V.W.nslices);
        if (wide(V.W)) k_fw<T, TB, 8><<<gr, WG, 0, st>>>(LV<T>::W(V), t, u, g);
        else k_fw<T, TB, 4><<<gr, WG, 0, st>>>(LV<T>::W(V), t, u, g);
    };
    auto zprod = [&](DevLevel& V, const T* u, const T* xin, auto xout, const double* dd, const Red& Rz) {
        using TX = std::remove_pointer_t<decltype(xout)>;
        const int gr = grid_ell(h, V.Z.nslices);
        if (wide(V.Z)) k_fz<T, TX, 8><<<gr, WG, 0, st>>>(LV<T>::Z(V), u, xin, xout, dd, Rz);
        else k_fz<T, TX, 4><<<gr, WG, 0, st>>>(LV<T>::Z(V), u, xin, xout, dd, Rz);
    };
    for (int l = 0; l < L - 1; l++) {
        DevLevel& V = h->lev[l];
        TimeScope ts(h, l == 0 ? 2 : 7);
        T* x = LV<T>::x(V);
        T* t = LV<T>::ft(V);
        T* u = LV<T>::fu(V);
        auto pre = [&](auto b) {
            wprod(V, b, u);
            zprod(V, u, (const T*)nullptr, x, nullptr, R0);
            for (int k = 2; k <= V.nu; k++) {
                resid(V, b, x, t);
                wprod(V, (const T*)t, u);
                zprod(V, u, x, x, nullptr, R0);
            }
            resid(V, b, x, LV<T>::r(V));
        };
        if (l == 0) pre(r0);
        else pre((const T*)LV<T>::b(V));
        launch_spmv(h, LV<T>::R(V), (const T*)LV<T>::r(V), LV<T>::b(h->lev[l + 1]), g, V.R.wmax > 8, V.R.wmax > SPLIT_W);
    }
    {
        DevLevel& C = h->lev[L - 1];
        TimeScope ts(h, 7);
        coarse_solve<T, T>(h, (const T*)LV<T>::b(C), LV<T>::x(C), g);
    }
    for (int l = L - 2; l >= 0; l--) {
        DevLevel& V = h->lev[l];
        TimeScope ts(h, l == 0 ? 4 : 7);
        T* x = LV<T>::x(V);
        T* t = LV<T>::ft(V);
        T* u = LV<T>::fu(V);
        const int gp = grid_ell(h, V.P.nslices);
        if (wide(V.P)) k_fprol<T, 8><<<gp, WG, 0, st>>>(LV<T>::P(V), LV<T>::x(h->lev[l + 1]), x, g);
        else k_fprol<T, 4><<<gp, WG, 0, st>>>(LV<T>::P(V), LV<T>::x(h->lev[l + 1]), x, g);
        for (int k = 1; k <= V.nu; k++) {
            if (l == 0) resid(V, r0, x, t);
            else resid(V, (const T*)LV<T>::b(V), x, t);
            wprod(V, (const T*)t, u);
            if (l == 0 && k == V.nu) zprod(V, u, x, z0, d, R);
            else zprod(V, u, x, x, nullptr, R0);
        }
        if (l == 0) finish(h, R, grid_ell(h, V.Z.nslices));
    }
}

// The V-cycle with the polynomial smoother in precision T: on each level
// above the coarsest, nu recurrence steps from x = 0 (the last leaves r_nu for
// the restriction); after x += P x_c and t = b - A x, nu more steps from x,
// the last folded into the output (FP64 z0 with the fused dot at level 0).
template <typename T>
static void vcycle_cheb(psc_hier* h, const double* r0, double* z0, const double* d, const Red& R, Gate g) {
    const int L = (int)h->lev.size();
    Red R0 = R;
    R0.fin = FIN_NONE;
    hipStream_t st = h->stream;
    const T c0 = (T)(4.0 / 3.0);
    auto coef = [](int k, T& ak, T& bk) {
        ak = (T)((double)(2 * k - 1) / (double)(2 * k + 3));
        bk = (T)((double)(8 * k + 4) / (double)(2 * k + 3));
    };
    // one recurrence step on level V (FIRST: from r_0 = sv, x_0 = xin)
    auto step = [&](DevLevel& V, bool first, auto sv, const T* din, const T* xin, auto xout, T* dout, int k,
                    bool fold, const double* dd, const Red& Rs) {
        using TB = std::remove_const_t<std::remove_pointer_t<decltype(sv)>>;
        using TX = std::remove_pointer_t<decltype(xout)>;
        T ak = T(0), bk = T(0);
        if (fold || dout) coef(k, ak, bk);
        const int gr = grid_lvl(h, V);
        const bool wa = wide_A(h, V);
        T* r = LV<T>::r(V);
        T* x = LV<T>::x(V);
        const T* minv = LV<T>::minv(V);
        with_A_t<T>(h, V, [&](auto A) {
            using M = decltype(A);
            if (first) {
                if (wa) k_cheb<M, TB, TX, true, 8><<<gr, WG, 0, st>>>(A, minv, sv, din, xin, r, x, xout, dout, c0, ak, bk, fold, dd, Rs);
                else k_cheb<M, TB, TX, true, 4><<<gr, WG, 0, st>>>(A, minv, sv, din, xin, r, x, xout, dout, c0, ak, bk, fold, dd, Rs);
            } else {
                if (wa) k_cheb<M, TB, TX, false, 8><<<gr, WG, 0, st>>>(A, minv, sv, din, xin, r, x, xout, dout, c0, ak, bk, fold, dd, Rs);
                else k_cheb<M, TB, TX, false, 4><<<gr, WG, 0, st>>>(A, minv, sv, din, xin, r, x, xout, dout, c0, ak, bk, fold, dd, Rs);
            }
        });
    };
    for (int l = 0; l < L - 1; l++) {
        DevLevel& V = h->lev[l];
        TimeScope ts(h, l == 0 ? 2 : 7);
        const int nu = V.nu;
        T* da = LV<T>::fu(V);
        T* db = LV<T>::fd(V);
        auto pre = [&](auto b) {
            step(V, true, b, (const T*)nullptr, (const T*)nullptr, (T*)nullptr, nu > 1 ? da : (T*)nullptr, 1, false,
                 nullptr, R0);
            const T* cur = da;
            for (int k = 2; k <= nu; k++) {
                T* nxt = cur == da ? db : da;
                step(V, false, (const T*)nullptr, cur, (const T*)nullptr, (T*)nullptr, k < nu ? nxt : (T*)nullptr, k,
                     false, nullptr, R0);
                cur = nxt;
            }
        };
        if (l == 0) pre(r0);
        else pre((const T*)LV<T>::b(V));
        launch_spmv(h, LV<T>::R(V), (const T*)LV<T>::r(V), LV<T>::b(h->lev[l + 1]), g, V.R.wmax > 8, V.R.wmax > SPLIT_W);
    }
    {
        DevLevel& C = h->lev[L - 1];
        TimeScope ts(h, 7);
        coarse_solve<T, T>(h, (const T*)LV<T>::b(C), LV<T>::x(C), g);
    }
    for (int l = L - 2; l >= 0; l--) {
        DevLevel& V = h->lev[l];
        TimeScope ts(h, l == 0 ? 4 : 7);
        const int nu = V.nu;
        T* x = LV<T>::x(V);
        T* t = LV<T>::ft(V);
        T* da = LV<T>::fu(V);
        T* db = LV<T>::fd(V);
        const int gr = grid_lvl(h, V);
        const int gp = grid_ell(h, V.P.nslices);
        if (V.P.wmax > 8) k_fprol<T, 8><<<gp, WG, 0, st>>>(LV<T>::P(V), LV<T>::x(h->lev[l + 1]), x, g);
        else k_fprol<T, 4><<<gp, WG, 0, st>>>(LV<T>::P(V), LV<T>::x(h->lev[l + 1]), x, g);
        const bool wa = wide_A(h, V), sa = split_A(h, V);
        auto res = [&](auto b) {
            using TB = std::remove_const_t<std::remove_pointer_t<decltype(b)>>;
            with_A_t<T>(h, V, [&](auto A) {
                using M = decltype(A);
                if (sa) k_fres<M, TB, GB_SPLIT><<<gr, WG, 0, st>>>(A, b, x, t, g);
                else if (wa) k_fres<M, TB, 8><<<gr, WG, 0, st>>>(A, b, x, t, g);
                else k_fres<M, TB, 4><<<gr, WG, 0, st>>>(A, b, x, t, g);
            });
        };
        if (l == 0) res(r0);
        else res((const T*)LV<T>::b(V));
        auto post = [&](auto out, const double* dd, const Red& Rz) {
            using TX = std::remove_pointer_t<decltype(out)>;
            if (nu == 1) {
                k_cheb_fin<T, TX><<<gr, WG, 0, st>>>(V.A.nslices, V.n, x, LV<T>::minv(V), t, c0, out, dd, Rz);
                return;
            }
            const T* cur = nullptr;
            for (int k = 1; k <= nu - 1; k++) {
                const bool fold = k == nu - 1;
                T* nxt = cur == da ? db : da;
                if (k == 1)
                    step(V, true, (const T*)t, (const T*)nullptr, (const T*)x, out, fold ? (T*)nullptr : nxt, k, fold,
                         fold ? dd : nullptr, fold ? Rz : R0);
                else
                    step(V, false, (const T*)nullptr, cur, (const T*)nullptr, out, fold ? (T*)nullptr : nxt, k, fold,
                         fold ? dd : nullptr, fold ? Rz : R0);
                cur = nxt;
            }
        };
        if (l == 0) {
            post(z0, d, R);
            finish(h, R, gr);
        } else {
            post(x, nullptr, R0);
        }
    }
}

// z = B r on level 0. prec: PSC_FP64 / PSC_FP32. fin/d: optional fused dot
// z.d at level 0 with finaliser fin. g gates every kernel (g.ctl == NULL:
// standalone V-cycle, always runs, no fused dot).
// z32 (FP32 V-cycle only, see mixed_z): the output goes there instead of z0.
static void vcycle(psc_hier* h, int prec, const double* r0, double* z0, int fin, const double* d,
                   Gate g, bool skip_pre0 = false, const float* r0_32 = nullptr, float* z32 = nullptr) {
    hipStream_t st = h->stream;
    const int L = (int)h->lev.size();
    Red R = red_of(h, fin, g.ctl ? g.mode : GATE_NONE);
    Red R0 = R;
    R0.fin = FIN_NONE;
    TimeScope whole(h, 6);
    if (L == 1) {
        coarse_solve<double, double>(h, r0, z0, g);
        if (fin != FIN_NONE) {
            int gr = grid_vec(h, h->lev[0].n);
            k_dot<<<gr, WG, 0, st>>>(h->lev[0].n, z0, d, R);
            finish(h, R, gr);
        }
        return;
    }
    if (h->fai) {
        // the factored smoothers start from r; no fused level-0 pre-smoothing
        if (prec == PSC_FP64) vcycle_fai<double>(h, r0, z0, d, R, g);
        else vcycle_fai<float>(h, r0, z0, d, R, g);
        return;
    }
    if (h->cheb) {
        if (prec == PSC_FP64) vcycle_cheb<double>(h, r0, z0, d, R, g);
        else vcycle_cheb<float>(h, r0, z0, d, R, g);
        return;
    }
    if (prec == PSC_FP64) vcycle_t<double>(h, r0, z0, d, R, g, skip_pre0);
    else vcycle_t<float>(h, r0, z0, d, R, g, skip_pre0, r0_32, z32);
}

// ---------------------------------------------------------------------------
// solve loops
// ---------------------------------------------------------------------------

static const int LAG = 2;     // iterations the GPU may run ahead of the host check
static const int RING = 8;

// forms: 0 PCG + FP64 V-cycle; 1 FCG(1) + FP64 V-cycle; 2 FCG(1) + FP32
// V-cycle; 3 / 4: forms 1 / 2 with the learned network on odd iterations.
static const int FORM_FUSED = 5;     // PCG, fused two-pass iteration, issued two iterations at a time
static const int FORM_FFUSED64 = 6;  // FCG(1) + FP64 V-cycle, fused, two iterations at a time
static const int FORM_FFUSED32 = 7;  // FCG(1) + FP32 V-cycle, fused, two iterations at a time
static const int FORM_FNET64 = 8;    // FORM_FFUSED64 with the learned network on odd iterations
static const int FORM_FNET32 = 9;    // FORM_FFUSED32 with the learned network on odd iterations
static inline bool form_net(int form) { return form == 3 || form == 4 || form == FORM_FNET64 || form == FORM_FNET32; }
static inline bool form_fused(int form) { return form >= FORM_FUSED; }
static inline int form_prec(int form) {
    return (form == 2 || form == 4 || form == FORM_FFUSED32 || form == FORM_FNET32) ? PSC_FP32 : PSC_FP64;
}

__global__ void k_iter_begin(Ctl* c, HostCtl* hc, int has_net) {
    if (threadIdx.x != 0 || c->done) return;
    const int odd = c->iter & 1;
    c->use_net = has_net && c->net_on && odd;
    if (has_net && !c->net_on && odd) c->fallbacks += 1;
}

// partials (z.r, z.q) of a network step
__global__ __launch_bounds__(WG) void k_dot2(long long n, const double* __restrict__ z,
                                             const double* __restrict__ r, const double* __restrict__ q,
                                             Red R) {
    if (skip_red(R)) return;
    long long lo, hi;
    chunk_range(n, lo, hi);
    double s0 = 0.0, s1 = 0.0;
    for (long long i = lo + threadIdx.x; i < hi; i += WG) {
        double zi = z[i];
        s0 += zi * r[i];
        s1 += zi * q[i];
    }
    block_partial(s0, s1, R.part);
}

// Issue one iteration of the given form. Every kernel exits at entry once
// the control block says the solve is over.
static int issue_iteration(psc_hier* h, int form, psc_net* net) {
    hipStream_t st = h->stream;
    DevLevel& L0 = h->lev[0];
    const long long n = L0.n;
    const int ge = grid_lvl(h, L0), gv = grid_vec(h, n);
    const Gate gd{h->ctl, GATE_DONE};
    if (form == FORM_FUSED) {
        // two iterations (even, odd) with the p and r buffers swapped between them
        const int it0 = h->t_iter;
        for (int parity = 0; parity < 2; parity++) {
            if (it0 >= 0) h->t_iter = it0 + parity;
            double* pold = parity ? h->p2 : h->p;
            double* pnew = parity ? h->p : h->p2;
            double* rold = parity ? h->r2 : h->r;
            double* rnew = parity ? h->r : h->r2;
            {
                TimeScope t(h, 0);
                if (h->bufload == 1)
                    k_spmv_pfuse<Ell<double>, true><<<ge, WG, 0, st>>>(L0.A.view(), h->z, pold, pnew, h->q, h->xs, red_of(h, FIN_ALPHA_PCG));
                else
                    with_A(h, L0, [&](auto A) {
                        k_spmv_pfuse<decltype(A)><<<ge, WG, 0, st>>>(A, h->z, pold, pnew, h->q, h->xs, red_of(h, FIN_ALPHA_PCG));
                    });
            }
            finish(h, red_of(h, FIN_ALPHA_PCG), ge);
            {
                TimeScope t(h, 2);
                if (h->fai || h->cheb)
                    k_rupdate<<<ge, WG, 0, st>>>(L0.A.nslices, n, rold, h->q, rnew, red_of(h, FIN_UPDATE_PCG));
                else if (h->split && h->fp64_split) {
                    // r = r - alpha q, then the level-0 pre-smoothing residual
                    // gathering r: the same values as the fused pass, half its gathers
                    k_rupdate<<<ge, WG, 0, st>>>(L0.A.nslices, n, rold, h->q, rnew, red_of(h, FIN_UPDATE_PCG));
                    with_AM(h, L0, [&](auto AM) {
                        k_pre_s<decltype(AM), double, 4><<<ge, WG, 0, st>>>(AM, rnew, pre_rbuf<double>(h, L0, 1), gd,
                                                                            pr_out<double>(h, L0));
                    });
                } else if (h->split)
                    with_AM(h, L0, [&](auto AM) {
                        k_update_pre_s<decltype(AM)><<<ge, WG, 0, st>>>(AM, rold, h->q, rnew, pre_rbuf<double>(h, L0, 1),
                                                                        red_of(h, FIN_UPDATE_PCG), pr_out<double>(h, L0));
                    });
                else if (h->bufload == 1)
                    k_update_pre<8, true><<<ge, WG, 0, st>>>(L0.A.view(), L0.minv, rold, h->q, rnew, L0.r, red_of(h, FIN_UPDATE_PCG));
                else if (h->unroll4)
                    k_update_pre<4><<<ge, WG, 0, st>>>(L0.A.view(), L0.minv, rold, h->q, rnew, L0.r, red_of(h, FIN_UPDATE_PCG));
                else
                    k_update_pre<8><<<ge, WG, 0, st>>>(L0.A.view(), L0.minv, rold, h->q, rnew, L0.r, red_of(h, FIN_UPDATE_PCG));
            }
            finish(h, red_of(h, FIN_UPDATE_PCG), ge);
            vcycle(h, PSC_FP64, rnew, h->z, FIN_RHO, rnew, gd, true);
        }
        return PSC_OK;
    }
    if (form == FORM_FFUSED64 || form == FORM_FFUSED32 || form == FORM_FNET64 || form == FORM_FNET32) {
        const bool f32 = form == FORM_FFUSED32 || form == FORM_FNET32;
        const bool netf = form == FORM_FNET64 || form == FORM_FNET32;
        // the mixed forms keep z in FP32 (see mixed_z); a network step's FP64 z
        // is rounded into it for the outer pass
        float* z32 = (form == FORM_FFUSED32 || form == FORM_FNET32) ? mixed_z(h) : nullptr;
        // The true residual and the redo of the pre-smoothing run only in the
        // iterations whose recursive residual passed the test, but are launched
        // in every one: on a grid of at most 1024 workgroups their early exit
        // costs a few microseconds instead of tens.
        const int gq = std::min(ge, 1024);
        const int it0 = h->t_iter;
        for (int parity = 0; parity < 2; parity++) {
            if (it0 >= 0) h->t_iter = it0 + parity;
            double* pold = parity ? h->p2 : h->p;
            double* pnew = parity ? h->p : h->p2;
            double* rold = parity ? h->r2 : h->r;
            double* rnew = parity ? h->r : h->r2;
            {
                TimeScope t(h, 0);
                if (h->bufload == 1)
                    k_spmv_pfuse_fcg<Ell<double>, true><<<ge, WG, 0, st>>>(L0.A.view(), h->z, pold, pnew, h->q, h->xs, rold, red_of(h, FIN_ALPHA_FCG));
                else if (z32)
                    with_A(h, L0, [&](auto A) {
                        k_spmv_pfuse_fcg<decltype(A), false, float><<<ge, WG, 0, st>>>(
                            A, z32, pold, pnew, h->q, h->xs, rold, red_of(h, FIN_ALPHA_FCG));
                    });
                else
                    with_A(h, L0, [&](auto A) {
                        k_spmv_pfuse_fcg<decltype(A)><<<ge, WG, 0, st>>>(A, h->z, pold, pnew, h->q, h->xs, rold, red_of(h, FIN_ALPHA_FCG));
                    });
            }
            finish(h, red_of(h, FIN_ALPHA_FCG), ge);
            {
                TimeScope t(h, 2);
                if (h->fai || h->cheb) {
                    k_rupdate<<<ge, WG, 0, st>>>(L0.A.nslices, n, rold, h->q, rnew, red_of(h, FIN_UPDATE_FCG));
                } else if (h->split) {
                    if (f32 && h->mixed_split) {
                        // r = r - alpha q (also rounded to FP32), then the FP32
                        // pre-smoothing residual gathering the FP32 copy: the same
                        // values as the fused pass, fewer FP64 gathers
                        k_rupdate<<<ge, WG, 0, st>>>(L0.A.nslices, n, rold, h->q, rnew, red_of(h, FIN_UPDATE_FCG),
                                                     h->r32);
                        const bool wide = wide_A(h, L0);
                        with_AM32(h, L0, [&](auto AM) {
                            using M = decltype(AM);
                            if (wide) k_pre_s<M, float, 8><<<ge, WG, 0, st>>>(AM, h->r32, pre_rbuf<float>(h, L0, 1), gd,
                                                                              pr_out<float>(h, L0));
                            else k_pre_s<M, float, 4><<<ge, WG, 0, st>>>(AM, h->r32, pre_rbuf<float>(h, L0, 1), gd,
                                                                         pr_out<float>(h, L0));
                        });
                    } else if (f32)
                        with_AM32(h, L0, [&](auto AM) {
                            k_update_pre_s<decltype(AM)><<<ge, WG, 0, st>>>(AM, rold, h->q, rnew, pre_rbuf<float>(h, L0, 1),
                                                                            red_of(h, FIN_UPDATE_FCG), pr_out<float>(h, L0));
                        });
                    else if (h->fp64_split) {
                        k_rupdate<<<ge, WG, 0, st>>>(L0.A.nslices, n, rold, h->q, rnew, red_of(h, FIN_UPDATE_FCG));
                        with_AM(h, L0, [&](auto AM) {
                            k_pre_s<decltype(AM), double, 4><<<ge, WG, 0, st>>>(AM, rnew, pre_rbuf<double>(h, L0, 1),
                                                                                gd, pr_out<double>(h, L0));
                        });
                    } else
                        with_AM(h, L0, [&](auto AM) {
                            k_update_pre_s<decltype(AM)><<<ge, WG, 0, st>>>(AM, rold, h->q, rnew, pre_rbuf<double>(h, L0, 1),
                                                                            red_of(h, FIN_UPDATE_FCG), pr_out<double>(h, L0));
                        });
                } else if (f32) {
                    if (h->bufload == 1)
                        k_update_pre_t<float, true><<<ge, WG, 0, st>>>(L0.A.view32(), L0.minv32, rold, h->q, rnew, L0.r32, red_of(h, FIN_UPDATE_FCG));
                    else
                        k_update_pre_t<float, false><<<ge, WG, 0, st>>>(L0.A.view32(), L0.minv32, rold, h->q, rnew, L0.r32, red_of(h, FIN_UPDATE_FCG));
                } else {
                    if (h->bufload == 1)
                        k_update_pre_t<double, true><<<ge, WG, 0, st>>>(L0.A.view(), L0.minv, rold, h->q, rnew, L0.r, red_of(h, FIN_UPDATE_FCG));
                    else
                        k_update_pre_t<double, false><<<ge, WG, 0, st>>>(L0.A.view(), L0.minv, rold, h->q, rnew, L0.r, red_of(h, FIN_UPDATE_FCG));
                }
            }
            finish(h, red_of(h, FIN_UPDATE_FCG), ge);
            with_A(h, L0, [&](auto A) {
                k_resid_lag<decltype(A)><<<gq, WG, 0, st>>>(A, h->bs, h->xs, pnew, rnew, red_of(h, FIN_TRUE));
            });
            finish(h, red_of(h, FIN_TRUE), gq);
            // after a residual replacement, redo the level-0 pre-smoothing from the true residual
            const Gate gr{h->ctl, GATE_REDO};
            // the FP32 copy of r (mixed form, split passes) read by the level-0 post-smoothing
            const float* r32v = (f32 && h->split && h->mixed_split && !(h->fai || h->cheb)) ? h->r32 : nullptr;
            if (h->fai || h->cheb) {
                // these smoothers have no fused pre-smoothing to redo
            } else if (f32) {
                if (r32v) k_copy<float, double><<<gq, WG, 0, st>>>(n, h->r32, rnew, gr);
                launch_pre(h, L0, (const double*)rnew, pre_rbuf<float>(h, L0, 1), gr, gq);
            } else {
                launch_pre(h, L0, (const double*)rnew, pre_rbuf<double>(h, L0, 1), gr, gq);
            }
            if (!netf) {
                vcycle(h, f32 ? PSC_FP32 : PSC_FP64, rnew, h->z, FIN_BETA_FCG, h->q, gd, true, r32v, z32);
                continue;
            }
            // learned form: odd iterations try z = net(r); the V-cycle (its
            // level-0 pre-smoothing already done above) runs when the network
            // step is not taken. net == NULL: the network was switched off for
            // this solve, only the step accounting remains.
            k_iter_begin<<<1, 64, 0, st>>>(h->ctl, h->hctl_dev, 1);
            if (net) {
                int rs = net_launch_apply(net, st, rnew, h->z, &h->ctl->rr, n, Gate{h->ctl, GATE_NET});
                if (rs) return rs;
                Red Rn = red_of(h, FIN_NETCHECK, GATE_NET);
                k_dot2<<<gv, WG, 0, st>>>(n, h->z, rnew, h->q, Rn);
                finish(h, Rn, gv);
                if (z32) k_copy<float, double><<<gv, WG, 0, st>>>(n, z32, h->z, Gate{h->ctl, GATE_NET});
            }
            vcycle(h, f32 ? PSC_FP32 : PSC_FP64, rnew, h->z, FIN_BETA_FCG, h->q, Gate{h->ctl, GATE_VC}, true, r32v,
                   z32);
        }
        return PSC_OK;
    }
    if (form == 0) {
        {
            TimeScope t(h, 0);
            with_A(h, L0, [&](auto A) {
                k_spmv_dot<decltype(A)><<<ge, WG, 0, st>>>(A, h->p, h->q, nullptr, red_of(h, FIN_ALPHA_PCG));
            });
        }
        finish(h, red_of(h, FIN_ALPHA_PCG), ge);
        {
            TimeScope t(h, 1);
            k_update<<<gv, WG, 0, st>>>(n, h->xs, h->r, h->p, h->q, red_of(h, FIN_UPDATE_PCG));
        }
        finish(h, red_of(h, FIN_UPDATE_PCG), gv);
        vcycle(h, PSC_FP64, h->r, h->z, FIN_RHO, h->r, gd);
        {
            TimeScope t(h, 5);
            k_pupdate<<<gv, WG, 0, st>>>(n, h->p, h->z, 0, gd);
        }
        return PSC_OK;
    }
    const int prec = form_prec(form);
    if (form_net(form)) {
        k_iter_begin<<<1, 64, 0, st>>>(h->ctl, h->hctl_dev, 1);
        if (net) {   // NULL: the network was switched off for this solve
            int rs = net_launch_apply(net, st, h->r, h->z, &h->ctl->rr, n, Gate{h->ctl, GATE_NET});
            if (rs) return rs;
            Red Rn = red_of(h, FIN_NETCHECK, GATE_NET);
            k_dot2<<<gv, WG, 0, st>>>(n, h->z, h->r, h->q, Rn);
            finish(h, Rn, gv);
        }
        vcycle(h, prec, h->r, h->z, FIN_BETA_FCG, h->q, Gate{h->ctl, GATE_VC});
    } else {
        vcycle(h, prec, h->r, h->z, FIN_BETA_FCG, h->q, gd);
    }
    {
        TimeScope t(h, 5);
        k_pupdate<<<gv, WG, 0, st>>>(n, h->p, h->z, 1, gd);
    }
    {
        TimeScope t(h, 0);
        with_A(h, L0, [&](auto A) {
            k_spmv_dot<decltype(A)><<<ge, WG, 0, st>>>(A, h->p, h->q, h->r, red_of(h, FIN_ALPHA_FCG));
        });
    }
    finish(h, red_of(h, FIN_ALPHA_FCG), ge);
    {
        TimeScope t(h, 1);
        k_update<<<gv, WG, 0, st>>>(n, h->xs, h->r, h->p, h->q, red_of(h, FIN_UPDATE_FCG));
    }
    finish(h, red_of(h, FIN_UPDATE_FCG), gv);
    with_A(h, L0, [&](auto A) {
        k_resid<decltype(A)><<<ge, WG, 0, st>>>(A, h->bs, h->xs, h->r, 1, red_of(h, FIN_TRUE));
    });
    finish(h, red_of(h, FIN_TRUE), ge);
    return PSC_OK;
}

static int get_graph(psc_hier* h, int form, psc_net* net, hipGraphExec_t* out) {
    const uint64_t gen = net ? net_generation(net) : 0;
    for (auto& e : h->graphs)
        if (e.form == form && e.net == net && e.gen == gen) { *out = e.exec; return PSC_OK; }
    hipGraph_t g;
    HIPCHK(hipStreamBeginCapture(h->stream, hipStreamCaptureModeRelaxed));
    int rs = issue_iteration(h, form, net);
    hipError_t ec = hipStreamEndCapture(h->stream, &g);
    if (rs) return rs;
    if (ec != hipSuccess) return fail(PSC_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    hipGraphExec_t ge;
    hipError_t e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(PSC_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    h->graphs.push_back(GraphEntry{form, net, gen, ge});
    *out = ge;
    return PSC_OK;
}

static void drop_graphs(psc_hier* h) {
    for (auto& e : h->graphs) (void)hipGraphExecDestroy(e.exec);
    h->graphs.clear();
}

static int read_ctl(psc_hier* h, Ctl* c) {
    HIPCHK(hipMemcpyAsync(c, h->ctl, sizeof(Ctl), hipMemcpyDeviceToHost, h->stream));
    HIPCHK(hipStreamSynchronize(h->stream));
    return PSC_OK;
}

// Common start of a solve: internal copies of b and x0, control block,
// r = b - A x0 with ||b||^2 and ||r||^2. Returns the control block.
static int solve_begin(psc_hier* h, int form, const double* b_dev, const double* x_dev, double rtol,
                       int32_t maxit, Ctl* c) {
    hipStream_t st = h->stream;
    DevLevel& L0 = h->lev[0];
    const long long n = L0.n;
    const int ge = grid_lvl(h, L0);
    HIPCHK(hipMemcpyAsync(h->bs, b_dev, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(h->xs, x_dev, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    k_ctl_init<<<1, 64, 0, st>>>(h->ctl, h->hctl_dev, rtol, maxit, form);
    with_A(h, L0, [&](auto A) {
        k_resid<decltype(A)><<<ge, WG, 0, st>>>(A, h->bs, h->xs, h->r, 0, red_of(h, FIN_INIT));
    });
    finish(h, red_of(h, FIN_INIT), ge);
    HIPCHK(hipGetLastError());
    return read_ctl(h, c);
}

// Shared driver of psc_pcg_solve (form 0) and psc_fcg_solve (forms 1-4).
static int solve_impl(psc_hier* h, int form, psc_net* net, const double* b_dev, double* x_dev,
                      double rtol, int32_t maxit, int32_t* iters, double* relres, int32_t* fallbacks) {
    if (!b_dev || !x_dev || !iters || !relres) return fail(PSC_ERR_ARG, "NULL argument");
    if (!(rtol > 0.0) || maxit < 0) return fail(PSC_ERR_ARG, "rtol must be > 0 and maxit >= 0");
    if (form_prec(form) == PSC_FP32 && !h->has32) return fail(PSC_ERR_STATE, "FP32 V-cycle needs build_fp32");
    hipStream_t st = h->stream;
    DevLevel& L0 = h->lev[0];
    const long long n = L0.n;
    const int gv = grid_vec(h, n), ge = grid_lvl(h, L0);
    if (form_net(form)) {
        int rs = net_check_grid(net, n);
        if (rs) return rs;
    }
    Ctl c;
    int rs = solve_begin(h, form, b_dev, x_dev, rtol, maxit, &c);
    if (rs) return rs;
    if (c.status == PSC_ERR_NAN) return fail(PSC_ERR_NAN, "NaN or Inf in the right-hand side or initial guess");
    if (c.nb2 == 0.0) {
        k_fill<double><<<gv, WG, 0, st>>>(n, x_dev, 0.0);
        HIPCHK(hipStreamSynchronize(st));
        *iters = 0;
        *relres = 0.0;
        if (fallbacks) *fallbacks = 0;
        return PSC_OK;
    }
    const bool use_graph = h->opts.use_graph && !h->timing;
    const bool fused = form <= 4 && h->fused_pcg && h->lev.size() > 1;
    static const int fused_of[5] = {FORM_FUSED, FORM_FFUSED64, FORM_FFUSED32, FORM_FNET64, FORM_FNET32};
    if (fused) form = fused_of[form];
    if (!c.done) {
        const Gate gd{h->ctl, GATE_DONE};
        if (form == FORM_FUSED) {
            vcycle(h, PSC_FP64, h->r, h->z, FIN_RHO_INIT, h->r, gd);
            k_fill<double><<<gv, WG, 0, st>>>(n, h->p, 0.0);   // p_old of the first iteration (beta = 0)
        } else if (fused) {
            k_fill<double><<<gv, WG, 0, st>>>(n, h->q, 0.0);
            k_fill<double><<<gv, WG, 0, st>>>(n, h->p, 0.0);
            vcycle(h, form_prec(form), h->r, h->z, FIN_BETA_FCG, h->q, gd, false, nullptr,
                   (form == FORM_FFUSED32 || form == FORM_FNET32) ? mixed_z(h) : nullptr);   // z = B r0, beta = 0
            if (form_net(form)) k_set_net_on<<<1, 64, 0, st>>>(h->ctl);
        } else if (form == 0) {
            vcycle(h, PSC_FP64, h->r, h->z, FIN_RHO_INIT, h->r, gd);
            k_copy<double, double><<<gv, WG, 0, st>>>(n, h->p, h->z, gd);
        } else {
            k_fill<double><<<gv, WG, 0, st>>>(n, h->q, 0.0);
            if (form_net(form)) k_set_net_on<<<1, 64, 0, st>>>(h->ctl);
        }
        hipGraphExec_t gexec = nullptr;
        if (use_graph) {
            rs = get_graph(h, form, net, &gexec);
            if (rs) return rs;
        }
        const int per_launch = fused ? 2 : 1;
        psc_net* inet = net;
        for (int k = 0; k * per_launch < maxit; k++) {
            if (use_graph) HIPCHK(hipGraphLaunch(gexec, st));
            else {
                h->t_iter = k * per_launch;
                rs = issue_iteration(h, form, inet);
                h->t_iter = -1;
                if (rs) return rs;
            }
            HIPCHK(hipEventRecord(h->ring[k % RING], st));
            if (k >= LAG) {
                HIPCHK(hipEventSynchronize(h->ring[(k - LAG) % RING]));
                if (h->hctl->done) break;
                if (inet && h->hctl->net_off) {
                    // the network is off for the rest of this solve: replay
                    // iterations without its kernels
                    inet = nullptr;
                    if (use_graph && (rs = get_graph(h, form, nullptr, &gexec))) return rs;
                }
            }
        }
        HIPCHK(hipGetLastError());
        HIPCHK(hipStreamSynchronize(st));
        rs = read_ctl(h, &c);
        if (rs) return rs;
        // the V-cycle closes the iteration in the fused forms and in PCG
        timing_collect(h, c.iter, (fused || form == 0) ? 1 : 0);
        if (fused) {
            // the last iteration's x update is deferred: x += alpha p_last
            k_final_axpy<<<gv, WG, 0, st>>>(n, h->xs, (c.iter & 1) ? h->p2 : h->p, h->ctl);
        }
    }
    // true residual in FP64 (ungated: runs after convergence)
    {
        Red Rs{h->part, h->ctl, nullptr, FIN_STORE, GATE_NONE};
        with_A(h, L0, [&](auto A) {
            k_resid<decltype(A)><<<ge, WG, 0, st>>>(A, h->bs, h->xs, h->q, 0, Rs);
        });
        finish(h, Rs, ge);
    }
    HIPCHK(hipMemcpyAsync(x_dev, h->xs, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    Ctl c2;
    rs = read_ctl(h, &c2);
    if (rs) return rs;
    int status = c.status;
    if (status == PSC_ERR_NAN) return fail(PSC_ERR_NAN, "NaN met during the iteration");
    if (status == PSC_ERR_NOT_SPD) return fail(PSC_ERR_NOT_SPD, "CG breakdown (p.q <= 0 or r.z <= 0)");
    *iters = c.iter;
    *relres = std::sqrt(c2.out1) / std::sqrt(c2.out0);
    if (fallbacks) *fallbacks = c.fallbacks;
    if (c.done == 0) status = PSC_NOCONV;
    if (status == PSC_NOCONV) g_err = "maximum number of iterations reached";
    return status;
}

static int solve(psc_hier* h, int form, psc_net* net, const double* b_dev, double* x_dev, double rtol,
                 int32_t maxit, int32_t* iters, double* relres, int32_t* fallbacks) {
    if (!h) return fail(PSC_ERR_ARG, "NULL handle");
    if (!h->ctl) return fail(PSC_ERR_STATE, "hierarchy was built host-only");
    if (h->stale) return fail(PSC_ERR_STATE, "the last numeric rebuild failed");
    HIPCHK(hipSetDevice(h->device));
    int st = join_in(h);
    if (st) return st;
    st = solve_impl(h, form, net, b_dev, x_dev, rtol, maxit, iters, relres, fallbacks);
    int j = join_out(h);
    return st ? st : j;
}

// Scaled crops (r/s, z/s), s = sqrt(rr/N), of the current PCG pair. One
// thread per crop cell; origins holds cpi (z, y, x) corners.
__global__ __launch_bounds__(WG) void k_crop(const double* __restrict__ r, const double* __restrict__ z,
                                             const double* rr, long long N, int nx, int ny,
                                             const int* __restrict__ origins, int cpi, int crop,
                                             float* __restrict__ out_r, float* __restrict__ out_z,
                                             Gate g) {
    if (gate_skip(g)) return;
    const long long per = (long long)crop * crop * crop;
    const long long t = (long long)blockIdx.x * WG + threadIdx.x;
    if (t >= per * cpi) return;
    const int c = (int)(t / per);
    const long long w = t % per;
    const int cx = (int)(w % crop), cy = (int)((w / crop) % crop), cz = (int)(w / ((long long)crop * crop));
    const long long gi = ((long long)(origins[3 * c] + cz) * ny + (origins[3 * c + 1] + cy)) * nx +
                         (origins[3 * c + 2] + cx);
    const double s = sqrt(*rr / (double)N);
    const double inv = s > 0.0 ? 1.0 / s : 0.0;
    out_r[t] = (float)(r[gi] * inv);
    out_z[t] = (float)(z[gi] * inv);
}

static int pairs_impl(psc_hier* h, const double* b_dev, int nx, int ny, int nz, double rtol, int maxit,
                      int crop, int cpi, const int32_t* origins, int n_origins, float* r_out,
                      float* z_out, int capacity, int32_t* count) {
    hipStream_t st = h->stream;
    DevLevel& L0 = h->lev[0];
    const long long n = L0.n;
    const int gv = grid_vec(h, n);
    int* d_orig = nullptr;
    HIPCHK(hipMallocAsync((void**)&d_orig, sizeof(int) * 3 * (size_t)n_origins, st));
    std::unique_ptr<int, std::function<void(int*)>> guard(d_orig, [st](int* p) { (void)hipFreeAsync(p, st); });
    HIPCHK(hipMemcpyAsync(d_orig, origins, sizeof(int) * 3 * (size_t)n_origins, hipMemcpyHostToDevice, st));
    double* x0 = nullptr;
    HIPCHK(hipMallocAsync((void**)&x0, sizeof(double) * n, st));
    std::unique_ptr<double, std::function<void(double*)>> guard2(x0, [st](double* p) { (void)hipFreeAsync(p, st); });
    k_fill<double><<<gv, WG, 0, st>>>(n, x0, 0.0);
    Ctl c;
    int rs = solve_begin(h, 0, b_dev, x0, rtol, maxit, &c);
    if (rs) return rs;
    if (c.status == PSC_ERR_NAN) return fail(PSC_ERR_NAN, "NaN or Inf in the right-hand side");
    if (c.done) return PSC_OK;
    const Gate gd{h->ctl, GATE_DONE};
    vcycle(h, PSC_FP64, h->r, h->z, FIN_RHO_INIT, h->r, gd);
    k_copy<double, double><<<gv, WG, 0, st>>>(n, h->p, h->z, gd);
    const long long per = (long long)crop * crop * crop;
    for (int k = 0;; k++) {
        // the pair (r_k, B r_k) is in (h->r, h->z)
        if ((k + 1) * cpi <= n_origins && *count + cpi <= capacity) {
            long long tot = per * cpi;
            k_crop<<<(unsigned)((tot + WG - 1) / WG), WG, 0, st>>>(
                h->r, h->z, &h->ctl->rr, n, nx, ny, d_orig + 3 * (size_t)k * cpi, cpi, crop,
                r_out + per * (*count), z_out + per * (*count), gd);
            HIPCHK(hipGetLastError());
            HIPCHK(hipStreamSynchronize(st));
            if (h->hctl->done) break;
            *count += cpi;
        }
        if (k >= maxit) break;
        if ((rs = issue_iteration(h, 0, nullptr))) return rs;
        HIPCHK(hipStreamSynchronize(st));
        if (h->hctl->done) break;
    }
    HIPCHK(hipStreamSynchronize(st));
    return PSC_OK;
}

// Host setup options of a handle.
static SetupOpts setup_opts_of(const psc_hier* h) {
    SetupOpts so;
    so.sweeps = h->opts.sweeps;
    so.coarse_max = h->opts.coarse_max;
    so.max_levels = h->opts.max_levels;
    so.coarse_sweeps = h->opts.coarse_sweeps;
    so.prol = h->opts.smoothed_prol;
    so.aggr = h->opts.aggregation;
    so.theta = h->opts.vbm_theta;
    so.device = h->opts.setup_device != 0 && !h->opts.host_only;
    so.device_products = so.device && h->opts.setup_device_products != 0;
    so.smoother = h->opts.smoother;
    so.tau = h->opts.ainv_tau;
    so.fill1 = h->opts.invk_fill;
    so.fill2 = h->opts.invk_inv_fill;
    so.coarse_pcg = h->opts.coarse_pcg_iters;
    so.coarse_rtol = h->opts.coarse_rtol;
    return so;
}

// Device copies of every level (operators, split operators, DIA copies,
// smoother data, level vectors) and of the coarsest solve, from the host
// hierarchy. Allocations go to h->lev_allocs so that a numeric rebuild can
// release and redo them.
static int upload_levels(psc_hier* h) {
    const bool f32 = h->has32;
    const int L = (int)h->host.lev.size();
    const bool cheb1 = h->opts.smoother == PSC_SMOOTH_CHEB4 && !h->cheb;
    if (!h->refresh) {
        h->lev.assign(L, DevLevel{});
        h->coarse_invT = nullptr;
    } else if ((int)h->lev.size() != L) {
        return PSC_ERR_STATE;
    }
    h->lev_phase = true;
    struct PhaseEnd {
        psc_hier* h;
        ~PhaseEnd() { h->lev_phase = false; }
    } phase_end{h};
    int st = PSC_OK;
    for (int l = 0; l < L; l++) {
        HostLevel& H = h->host.lev[l];
        DevLevel& D = h->lev[l];
        D.n = H.n;
        D.nc = H.nc;
        D.nnz = H.rp[H.n];
        D.nu = h->opts.vcycle_double ? std::min(h->nu << std::min(l, 12), 4096) : h->nu;
        // the smoother's inverse diagonal: M^-1, or (4/3) M^-1 for the degree-1
        // polynomial smoother (never on the coarsest level, whose sweeps stay l1-Jacobi)
        std::vector<double> wminv;
        if (cheb1 && l < L - 1) {
            wminv.resize(H.n);
            const double c0 = 4.0 / 3.0;
            for (int64_t i = 0; i < H.n; i++) wminv[i] = c0 * H.minv[i];
        }
        const std::vector<double>& mv = wminv.empty() ? H.minv : wminv;
        // A, its hacked-DIA copy and A M^-1 in both: the layouts are packed
        // on the host at build (kept by a refresh: same pattern), the values
        // scattered into them on the device
        if (!h->refresh) {
            if ((st = upload_ell_layout(h, D.A, H.n, H.n, H.rp.data(), H.ci.data(), f32,
                                        l < L - 1 ? &D.am : nullptr, &D.am32)))
                return st;
            // hacked-DIA copy when it stores at most 4/3 of the ELL slots (8
            // instead of 12 bytes per slot: at least 11 % fewer bytes)
            std::vector<int32_t> dstart, doffs, duo;
            std::vector<double> none;
            if (pack_dia(H.n, H.n, H.rp.data(), H.ci.data(), nullptr, D.A.slots * 4 / 3, dstart, doffs, none,
                         &duo)) {
                DevDia& G = D.Ad;
                G.nrows = H.n;
                G.ncols = H.n;
                G.nslices = (long long)dstart.size() - 1;
                G.slots = (long long)dstart.back() * SLICE;
                for (size_t q = 0; q + 1 < dstart.size(); q++)
                    G.ndmax = std::max(G.ndmax, dstart[q + 1] - dstart[q]);
                G.nd_u = (int)duo.size();
                G.nd = h->dia_uniform ? G.nd_u : 0;
                for (size_t k = 0; k < duo.size() && k < 8; k++) G.uo[k] = duo[k];
                // uniform layouts are stored in 128-row blocks (an odd last
                // slice gets an empty partner)
                G.pair = G.nd_u > 0 ? 1 : 0;
                if (G.pair && (G.nslices & 1)) G.slots += (long long)G.nd_u * SLICE;
                if ((st = upload(h, &G.start, dstart.data(), dstart.size()))) return st;
                if ((st = upload(h, &G.offs, doffs.data(), doffs.size()))) return st;
                const size_t slots = (size_t)G.slots;
                if ((st = zalloc(h, (void**)&G.val, slots * sizeof(double)))) return st;
                if (f32 && (st = zalloc(h, (void**)&G.val32, slots * sizeof(float)))) return st;
                if (l < L - 1) {
                    if ((st = zalloc(h, (void**)&D.amd, slots * sizeof(double)))) return st;
                    if (f32 && (st = zalloc(h, (void**)&D.amd32, slots * sizeof(float)))) return st;
                }
            }
        }
        const int32_t* a_rp_dev = nullptr;   // A's rows staged on the device (kept until R is filled)
        if ((st = refresh_values(h, D.A, &D.Ad, H.n, H.rp.data(), H.v.data(), l < L - 1 ? mv.data() : nullptr,
                                 D.am, D.am32, D.amd, D.amd32, &a_rp_dev)))
            return st;
        if (!D.Ad.on() && (st = upload_capped(h, D, H, l < L - 1 ? mv.data() : nullptr, f32))) return st;
        if ((st = upload(h, &D.minv, mv.data(), H.n))) return st;
        if (f32) {
            auto m32 = to32(mv);
            if ((st = upload(h, &D.minv32, m32.data(), m32.size()))) return st;
        }
        if (l == 0 && (h->fai || h->cheb) && L > 1) {
            // the smoothed iterate of level 0 (the other levels keep it in x)
            if ((st = dalloc(h, (void**)&D.x, H.n * sizeof(double)))) return st;
            if (f32 && (st = dalloc(h, (void**)&D.x32, H.n * sizeof(float)))) return st;
        }
        if (l > 0) {
            if ((st = dalloc(h, (void**)&D.b, H.n * sizeof(double)))) return st;
            if ((st = dalloc(h, (void**)&D.x, H.n * sizeof(double)))) return st;
            if (f32) {
                if ((st = dalloc(h, (void**)&D.b32, H.n * sizeof(float)))) return st;
                if ((st = dalloc(h, (void**)&D.x32, H.n * sizeof(float)))) return st;
            }
        }
        if (l == L - 1 && l > 0 && h->host.coarse_sweeps > 0) {
            if ((st = dalloc(h, (void**)&D.r, H.n * sizeof(double)))) return st;
        }
        if (l < L - 1 && D.nu > 1) {
            for (double** q : {&D.rb, &D.s, &D.sb, &D.xt, &D.xt2})
                if ((st = dalloc(h, (void**)q, H.n * sizeof(double)))) return st;
            if (f32)
                for (float** q : {&D.rb32, &D.s32, &D.sb32, &D.xt32, &D.xt232})
                    if ((st = dalloc(h, (void**)q, H.n * sizeof(float)))) return st;
        }
        if (l < L - 1) {
            if ((st = dalloc(h, (void**)&D.r, H.n * sizeof(double)))) return st;
            if (f32 && (st = dalloc(h, (void**)&D.r32, H.n * sizeof(float)))) return st;
            if ((st = upload(h, &D.agg, H.agg.data(), H.n))) return st;
            if ((st = upload(h, &D.pval, H.p.data(), H.n))) return st;
            if (f32) {
                auto p32 = to32(H.p);
                if ((st = upload(h, &D.pval32, p32.data(), p32.size()))) return st;
            }
            // smoothed prolongator S P = (I - M^-1 A) P of the split post-smoothing
            // sweep. Tentative prolongator (row i: p_i at agg_i): its layout is
            // the distinct aggregates of each row's columns, its values are formed
            // on the device from A's slots (before R reuses the staging)
            const bool tentative = (int64_t)H.pci.size() == H.n && (int64_t)H.prp.size() == H.n + 1 &&
                                   H.prp[H.n] == H.n && !h->opts.smoothed_prol;
            const bool sp_on_device = tentative && a_rp_dev != nullptr;
            if (sp_on_device) {
                if (!h->refresh) {
                    std::vector<int32_t> sprp, spci;
                    tentative_sp_pattern(H, sprp, spci);
                    if ((st = upload_ell_layout(h, D.SP, H.n, H.nc, sprp.data(), spci.data(), f32, nullptr, nullptr,
                                                true)))
                        return st;
                }
                if (!D.SP.off || !D.SP.col || !D.SP.val || D.SP.nrows != H.n) return PSC_ERR_STATE;
                std::string err;
                if ((st = gpu_tentative_sp((void*)h->stream, H.n, D.A.off, D.A.col, D.A.val, a_rp_dev, D.agg, D.pval,
                                           D.minv, D.SP.off, D.SP.col, D.SP.val, D.SP.val32, D.SP.pair, err)))
                    return fail(st, err);
            }
            // R = P^T as CSR over coarse rows: fine rows ascending
            const size_t pn = H.pci.size();
            std::vector<int32_t> rrp(H.nc + 1, 0), rci(pn);
            std::vector<double> rv(pn);
            for (size_t m = 0; m < pn; m++) rrp[H.pci[m] + 1]++;
            for (int64_t I = 0; I < H.nc; I++) rrp[I + 1] += rrp[I];
            std::vector<int32_t> pos(rrp.begin(), rrp.end() - 1);
            for (int64_t i = 0; i < H.n; i++) {
                for (int32_t m = H.prp[i]; m < H.prp[i + 1]; m++) {
                    int32_t o = pos[H.pci[m]]++;
                    rci[o] = (int32_t)i;
                    rv[o] = H.pv[m];
                }
            }
            if (!h->refresh && (st = upload_ell_layout(h, D.R, H.nc, H.n, rrp.data(), rci.data(), f32))) return st;
            if ((st = refresh_values(h, D.R, nullptr, H.nc, rrp.data(), rv.data(), nullptr, nullptr, nullptr, nullptr,
                                     nullptr)))
                return st;
            if ((st = upload_pair_r(h, D, H, f32))) return st;
            // general prolongator: S P from the host's sparse product
            if (!sp_on_device) {
                std::vector<int32_t> sprp, spci;
                std::vector<double> spv;
                jacobi_smoothed_prolongator(H, mv.data(), sprp, spci, spv);
                if (!h->refresh &&
                    (st = upload_ell_layout(h, D.SP, H.n, H.nc, sprp.data(), spci.data(), f32, nullptr, nullptr,
                                            true)))
                    return st;
                if ((st = refresh_values(h, D.SP, nullptr, H.n, sprp.data(), spv.data(), nullptr, nullptr, nullptr,
                                         nullptr, nullptr)))
                    return st;
            }
            // the kept A P is not needed after this (a rebuild forms it again)
            std::vector<int32_t>().swap(H.aprp);
            std::vector<int32_t>().swap(H.apci);
            std::vector<double>().swap(H.apv);
            if (h->fai || h->cheb) {
                if ((st = upload_fai(h, D, H, f32))) return st;
            }
        }
    }
    // coarsest inverse, stored transposed for coalesced reads
    h->coarse_n = (int)h->host.lev[L - 1].n;
    if (h->host.coarse_sweeps == 0 && h->host.coarse_pcg == 0) {
        int nc = h->coarse_n;
        std::vector<double> invT((size_t)nc * nc);
        for (int i = 0; i < nc; i++)
            for (int k = 0; k < nc; k++) invT[(size_t)k * nc + i] = h->host.coarse_inv[(size_t)i * nc + k];
        if ((st = upload(h, &h->coarse_invT, invT.data(), invT.size()))) return st;
    }
    return PSC_OK;
}

}  // namespace psc

using namespace psc;

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

const char* psc_last_error(void) { return g_err.c_str(); }

void psc_amg_opts_default(psc_amg_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->sweeps = 2;
    o->coarse_max = 200;
    o->max_levels = 30;
    o->build_fp32 = 0;
    o->use_graph = 1;
    o->coarse_sweeps = 30;
    o->smoothed_prol = 0;
    o->smoother_sweeps = 1;
    o->aggregation = PSC_AGGR_MATCHING;
    o->vbm_theta = 0.01;
    o->setup_device = 1;
    o->setup_device_products = 0;
    o->smoother = PSC_SMOOTH_L1JACOBI;
    o->invk_fill = 0;
    o->invk_inv_fill = 1;
    o->ainv_tau = 0.1;
    o->coarse_pcg_iters = 0;
    o->coarse_rtol = 1e-4;
    o->capped_min_rows = 65536;
}

void psc_hier_free(psc_hier* h) {
    if (!h) return;
    if (h->opts.host_only) { delete h; return; }
    (void)hipSetDevice(h->device);
    if (h->stream) (void)hipStreamSynchronize(h->stream);
    for (auto& g : h->graphs) (void)hipGraphExecDestroy(g.exec);
    for (auto& e : h->ev_pool) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto& e : h->ring) (void)hipEventDestroy(e);
    for (auto& e : h->ev_join)
        if (e) (void)hipEventDestroy(e);
    if (h->stream) (void)hipStreamDestroy(h->stream);
    for (void* p : h->allocs) (void)hipFree(p);
    for (void* p : h->lev_allocs) (void)hipFree(p);
    if (h->stage) (void)hipFree(h->stage);
    if (h->hctl) (void)hipHostFree(h->hctl);
    delete h;
}

int psc_amg_build(int32_t n, const int32_t* rp, const int32_t* ci, const double* v,
                  const psc_amg_opts* opts, void* hip_stream, psc_hier** out) {
    if (!out) return fail(PSC_ERR_ARG, "out is NULL");
    *out = nullptr;
    auto t0 = std::chrono::steady_clock::now();
    std::string err;
    int st = validate_csr(n, rp, ci, v, err);
    if (st) return fail(st, err);
    std::unique_ptr<psc_hier, void (*)(psc_hier*)> h(new psc_hier(), psc_hier_free);
    if (opts) h->opts = *opts;
    else psc_amg_opts_default(&h->opts);
    h->user_stream = (hipStream_t)hip_stream;
    if (!h->opts.host_only) {
        HIPCHK(hipGetDevice(&h->device));
        HIPCHK(hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking));
        for (auto& e : h->ev_join) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        HIPCHK(hipStreamSynchronize(h->user_stream));
    }
    SetupOpts so = setup_opts_of(h.get());
    if (so.smoother < 0 || so.smoother > 3 || !(so.tau >= 0.0) || so.fill1 < 0 || so.fill1 > 64 || so.fill2 < 0 ||
        so.fill2 > 64)
        return fail(PSC_ERR_ARG, "smoother must be 0..3, ainv_tau >= 0, INVK fill levels 0..64");
    h->fai = so.smoother == PSC_SMOOTH_AINV || so.smoother == PSC_SMOOTH_INVK;
    // The degree-1 polynomial smoother is l1-Jacobi weighted 4/3: it runs on
    // the l1 path with the weight folded into M^-1 (and so into A M^-1 and
    // (I - M^-1 A) P); higher degrees take the recurrence kernels.
    const bool cheb1 = so.smoother == PSC_SMOOTH_CHEB4 && h->opts.smoother_sweeps == 1 && !h->opts.vcycle_double;
    h->cheb = so.smoother == PSC_SMOOTH_CHEB4 && !cheb1;
    if (h->opts.smoother_sweeps < 1 || h->opts.smoother_sweeps > 16 || h->opts.smoothed_prol < 0 ||
        h->opts.smoothed_prol > 1)
        return fail(PSC_ERR_ARG, "smoother_sweeps must be 1..16 and smoothed_prol 0 or 1");
    h->nu = h->opts.smoother_sweeps;
    if (h->opts.vcycle_double < 0 || h->opts.vcycle_double > 1)
        return fail(PSC_ERR_ARG, "vcycle_double must be 0 or 1");
    if (h->opts.capped_min_rows < 0) return fail(PSC_ERR_ARG, "capped_min_rows must be >= 0");
    {
        PhaseTimer pt("hierarchy (host and device coarsening)");
        st = build_hierarchy(n, rp, ci, v, so, h->host, err);
    }
    if (st) return fail(st, err);
    const bool f32 = h->opts.build_fp32 != 0;
    h->has32 = f32;
    const int L = (int)h->host.lev.size();
    h->lev.resize(L);
    if (h->opts.host_only) {
        for (int l = 0; l < L; l++) {
            h->lev[l].n = h->host.lev[l].n;
            h->lev[l].nc = h->host.lev[l].nc;
            h->lev[l].nnz = h->host.lev[l].rp[h->host.lev[l].n];
        }
        h->coarse_n = (int)h->host.lev[L - 1].n;
        h->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        *out = h.release();
        return PSC_OK;
    }
    {
        PhaseTimer pt("pack and upload levels");
            if (h->host.coarse_pcg > 0 && h->host.lev.back().n > CPCG_MAX)
            return fail(PSC_ERR_ARG, "the PCG coarsest solver takes at most 4096 rows");
        st = upload_levels(h.get());
        release_stage(h.get());
        if (st) return st;
    }
    // solver workspace
    const int64_t N = n;
    if ((st = dalloc(h.get(), (void**)&h->ctl, sizeof(Ctl)))) return st;
    if ((st = dalloc(h.get(), (void**)&h->part, 2 * GMAX * sizeof(double)))) return st;
    if ((st = dalloc(h.get(), (void**)&h->part2, 2 * 256 * sizeof(double)))) return st;
    for (double** p : {&h->xs, &h->bs, &h->r, &h->z, &h->p, &h->q, &h->r2, &h->p2})
        if ((st = dalloc(h.get(), (void**)p, N * sizeof(double)))) return st;
    if (f32 && (st = dalloc(h.get(), (void**)&h->r32, N * sizeof(float)))) return st;
    if (f32 && (st = dalloc(h.get(), (void**)&h->z32, N * sizeof(float)))) return st;
    HIPCHK(hipHostMalloc((void**)&h->hctl, sizeof(HostCtl), hipHostMallocMapped | hipHostMallocCoherent));
    std::memset(h->hctl, 0, sizeof(HostCtl));
    HIPCHK(hipHostGetDevicePointer((void**)&h->hctl_dev, h->hctl, 0));
    h->ring.resize(RING);
    for (auto& e : h->ring) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    k_ctl_init<<<1, 64, 0, h->stream>>>(h->ctl, h->hctl_dev, 1e-6, 1, 0);
    HIPCHK(hipGetLastError());
    if ((st = build_tail(h.get()))) return st;
    HIPCHK(hipStreamSynchronize(h->stream));
    h->setup_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = h.release();
    return PSC_OK;
}

int psc_amg_rebuild(psc_hier* h, const double* val) {
    if (!h || !val) return fail(PSC_ERR_ARG, "NULL argument");
    auto t0 = std::chrono::steady_clock::now();
    std::string err;
    if (!h->opts.host_only) {
        HIPCHK(hipSetDevice(h->device));
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    h->stale = true;
    int st;
    {
        PhaseTimer pt("rebuild numerics");
        st = rebuild_numeric(h->host, val, setup_opts_of(h), err);
    }
    if (st) return fail(st, err);
    if (!h->opts.host_only) {
        // new values into the existing buffers when every size matches (the
        // captured iterations stay valid); otherwise release and re-upload
        h->refresh = true;
        {
            PhaseTimer pt("rebuild: refresh level values");
            st = upload_levels(h);
        }
        h->refresh = false;
        if (st == PSC_ERR_STATE) {
            g_err.clear();
            drop_graphs(h);   // they point at the buffers released below
            for (void* p : h->lev_allocs) (void)hipFree(p);
            h->lev_allocs.clear();
            h->asize.clear();
            h->device_bytes -= h->lev_bytes;
            h->lev_bytes = 0;
            st = upload_levels(h);
        }
        release_stage(h);
        if (st) return st;
        if ((st = build_tail(h))) return st;
        HIPCHK(hipStreamSynchronize(h->stream));
    }
    h->stale = false;
    h->rebuild_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return PSC_OK;
}

int psc_pcg_solve(psc_hier* h, const double* b, double* x, double rtol, int32_t maxit,
                  int32_t* iters, double* relres) {
    return solve(h, 0, nullptr, b, x, rtol, maxit, iters, relres, nullptr);
}

int psc_fcg_solve(psc_hier* h, psc_net* net, int32_t vprec, const double* b, double* x,
                  double rtol, int32_t maxit, int32_t* iters, double* relres, int32_t* fallbacks) {
    if (vprec != PSC_FP64 && vprec != PSC_FP32) return fail(PSC_ERR_ARG, "vcycle_prec must be PSC_FP64 or PSC_FP32");
    int form = (vprec == PSC_FP32 ? 2 : 1) + (net ? 2 : 0);
    return solve(h, form, net, b, x, rtol, maxit, iters, relres, fallbacks);
}

int psc_pairs_collect(psc_hier* h, const double* b, int32_t nx, int32_t ny, int32_t nz, double rtol,
                      int32_t maxit, int32_t crop, int32_t cpi, const int32_t* origins, int32_t n_origins,
                      float* r_out, float* z_out, int32_t capacity, int32_t* count) {
    if (!h || !b || !origins || !r_out || !z_out || !count) return fail(PSC_ERR_ARG, "NULL argument");
    if (!h->ctl) return fail(PSC_ERR_STATE, "hierarchy was built host-only");
    if (h->stale) return fail(PSC_ERR_STATE, "the last numeric rebuild failed");
    if ((long long)nx * ny * nz != h->lev[0].n) return fail(PSC_ERR_ARG, "grid does not match the matrix size");
    if (crop < 1 || crop > nx || crop > ny || crop > nz || cpi < 1 || n_origins < 0 || capacity < 0 ||
        *count < 0 || *count > capacity || maxit < 0 || !(rtol > 0.0))
        return fail(PSC_ERR_ARG, "bad crop, count or capacity");
    for (int i = 0; i < n_origins; i++) {
        const int dims[3] = {nz, ny, nx};
        for (int a = 0; a < 3; a++)
            if (origins[3 * i + a] < 0 || origins[3 * i + a] + crop > dims[a])
                return fail(PSC_ERR_ARG, "crop origin out of range");
    }
    HIPCHK(hipSetDevice(h->device));
    int st = join_in(h);
    if (st) return st;
    st = pairs_impl(h, b, nx, ny, nz, rtol, maxit, crop, cpi, origins, n_origins, r_out, z_out, capacity, count);
    int j = join_out(h);
    return st ? st : j;
}

int psc_hier_info(const psc_hier* h, psc_hier_stats* s) {
    if (!h || !s) return fail(PSC_ERR_ARG, "NULL argument");
    std::memset(s, 0, sizeof(*s));
    const int L = (int)h->lev.size();
    s->levels = L;
    double z0 = (double)h->lev[0].nnz, zs = 0.0, vb64 = 0.0, vb32 = 0.0;
    for (int l = 0; l < L; l++) {
        const DevLevel& D = h->lev[l];
        s->rows[l] = D.n;
        s->nnz[l] = D.nnz;
        s->ell_slots[l] = D.A.slots;
        s->dia_slots[l] = D.Ad.slots;
        s->capped_cap[l] = D.Ac.off ? D.Ac.cap : 0;
        s->capped_slots[l] = D.Ac.off ? D.Ac.slots + D.Ac.xents : 0;
        s->pair_restrict[l] = use_pr(h, D) ? 1 : 0;
        if (l + 1 < L) {
            s->p_nnz[l] = (int64_t)h->host.lev[l].pci.size();
            s->omega[l] = h->host.lev[l].omega;
        }
        zs += (double)D.nnz;
        // bytes per stored entry of A (and A M^-1) in the storage the kernels read
        const bool dia = h->dia && D.Ad.on();
        const double m64 = dia ? 8 : 12, m32 = dia ? 4 : 8;
        if (l < L - 1) {
            double Z = (double)D.nnz, N = (double)D.n, Nc = (double)D.nc, Zp = (double)D.SP.nnz;
            s->sp_nnz[l] = D.SP.nnz;
            // level 0 reads b and writes x in FP64 in both forms
            const double e0 = l == 0 ? 1.0 : 0.0;
            if (h->fai) {
                // AINV / INVK: W and Z (Zf entries each, hacked ELL), A for the
                // residuals, P and R for the transfers.
                // pre: W b (b gathered, u written), Z u (u gathered, x written);
                // sweeps 2..nu: residual (A, x gathered, b read, t written), W t,
                // x += Z u (x read and written); residual r; restriction;
                // post: x += P x_c, then nu sweeps of residual, W t, x += Z u
                const double Zf = (double)D.Z.nnz, Zr = (double)h->host.lev[l].pci.size(), nu = D.nu;
                const double res64 = Z * m64 + 24 * N, w64 = Zf * 12 + 16 * N, z64 = Zf * 12 + 24 * N;
                const double res32 = Z * m32 + 12 * N, w32 = Zf * 8 + 8 * N, z32 = Zf * 8 + 12 * N;
                s->smoother_nnz[l] = D.Z.nnz;
                vb64 += w64 + (z64 - 8 * N) + (nu - 1) * (res64 + w64 + z64) + res64 + Zr * 12 + 8 * N + 8 * Nc +
                        Zr * 12 + 8 * Nc + 16 * N + nu * (res64 + w64 + z64);
                vb32 += w32 + (z32 - 4 * N) + (nu - 1) * (res32 + w32 + z32) + res32 + Zr * 8 + 4 * N + 4 * Nc +
                        Zr * 8 + 4 * Nc + 8 * N + nu * (res32 + w32 + z32) + e0 * 4 * N * (2 * nu + 2);
            } else if (h->cheb) {
                // polynomial smoother: each recurrence step reads A and gathers the
                // direction, reads and writes r and x, reads M^-1, writes d (48 N
                // bytes of vectors in FP64); pre: nu steps; restriction; post:
                // x += P x_c, t = b - A x, then nu - 1 steps (the last writes x
                // once) or, for nu = 1, one vector pass
                const double Zr = (double)h->host.lev[l].pci.size(), nu = D.nu;
                const double st64 = Z * m64 + 48 * N, st32 = Z * m32 + 24 * N;
                vb64 += nu * st64 + Zr * 12 + 8 * N + 8 * Nc + Zr * 12 + 8 * Nc + 16 * N + Z * m64 + 24 * N +
                        (nu > 1 ? (nu - 1) * st64 : 32 * N);
                vb32 += nu * st32 + Zr * 8 + 4 * N + 4 * Nc + Zr * 8 + 4 * Nc + 8 * N + Z * m32 + 12 * N +
                        (nu > 1 ? (nu - 1) * st32 : 16 * N) + e0 * 12 * N;
            } else if (h->split) {
                // pre sweep 1: A M^-1, b gathered, r written; sweeps 2..nu: A M^-1,
                // s and r gathered, b read, s and r written; restriction: R
                // (nnz(P) entries), r, b_c; post sweep 1: S P, s (or b), minv, r
                // read, x_c gathered, x written; sweeps 2..nu: A, x gathered, b and
                // minv read, x written
                // (pair restriction: the pre sweep also writes N/2 pair sums, the
                // restriction reads them with N/2 entries instead of r with nnz(P))
                const double nu = D.nu;
                const bool pr = use_pr(h, D);
                const double Zr = pr ? 0.5 * N : (double)h->host.lev[l].pci.size(), Nr = pr ? 0.5 * N : N;
                vb64 += Z * m64 + 16 * N + (pr ? 4 * N : 0) + (nu - 1) * (Z * m64 + 40 * N) + Zr * 12 + 8 * Nr +
                        8 * Nc + Zp * 12 + 32 * N + 8 * Nc + (nu - 1) * (Z * m64 + 32 * N);
                vb32 += Z * m32 + 8 * N + (pr ? 2 * N : 0) + (nu - 1) * (Z * m32 + 20 * N) + Zr * 8 + 4 * Nr +
                        4 * Nc + Zp * 8 + 16 * N + 4 * Nc + (nu - 1) * (Z * m32 + 16 * N) + e0 * 12 * N;
            } else {
                // pre: A, b and minv gathered, r written; restriction: R, r, b_c;
                // post: A, b, minv, p, agg, x_c gathered, x written
                vb64 += 2 * Z * 12 + N * 12 * 2 /* P and R */ + N * (8 * 8) + Nc * 8 * 2;
                vb32 += 2 * Z * 8 + N * 8 * 2 + N * (8 * 4) + Nc * 4 * 2 + e0 * 12 * N;
            }
        } else if (h->host.coarse_sweeps > 0) {
            // sweeps: A and x gathered, b and minv read, x written
            double K = h->host.coarse_sweeps, Z = (double)D.nnz, N = (double)D.n;
            vb64 += (K - 1) * (Z * m64 + N * 8 * 4) + N * 8 * 3;
            vb32 += (K - 1) * (Z * m64 + N * 8 * 3 + N * 4) + N * (8 + 4 + 4);
        } else {
            double n2 = (double)D.n * D.n;
            vb64 += 8 * n2;
            vb32 += 8 * n2;
        }
    }
    s->operator_complexity = zs / z0;
    s->vcycle_bytes_fp64 = vb64;
    s->vcycle_bytes_fp32 = vb32;
    s->spmv_bytes_fp64 = z0 * ((h->dia && h->lev[0].Ad.on()) ? 8 : 12) + 2 * 8 * (double)h->lev[0].n;
    s->setup_seconds = h->setup_seconds;
    s->device_bytes = h->device_bytes;
    s->coarse_sweeps = h->host.coarse_sweeps;
    s->smoother_sweeps = h->nu;
    s->vcycle_double = h->opts.vcycle_double;
    s->aggregation = h->opts.aggregation;
    s->smoothed_prol = h->opts.smoothed_prol;
    s->smoother = h->opts.smoother;
    s->rebuild_seconds = h->rebuild_seconds;
    s->coarse_pcg_iters = h->host.coarse_pcg;
    const bool tail = h->tail && h->tail_t > 0 && h->split && h->tail_dia == h->dia;
    s->tail_level = tail ? h->tail_t : 0;
    s->tail_lds_bytes = tail ? h->tail_lds * (int)sizeof(double) + h->tail_pcg_bytes : 0;
    if (h->opts.host_only)
        for (int l = 0; l + 1 < L; l++) s->smoother_nnz[l] = (int64_t)h->host.lev[l].fai.zi.size();
    return PSC_OK;
}

int psc_hier_export_smoother(const psc_hier* h, int32_t l, int64_t* colptr, int32_t* row, double* val,
                             double* d) {
    if (!h || l < 0 || l + 1 >= (int)h->host.lev.size() || h->host.lev[l].fai.empty())
        return fail(PSC_ERR_ARG, "level has no AINV / INVK factor");
    const HostFai& F = h->host.lev[l].fai;
    if (colptr) std::memcpy(colptr, F.zr.data(), F.zr.size() * sizeof(int64_t));
    if (row) std::memcpy(row, F.zi.data(), F.zi.size() * sizeof(int32_t));
    if (val) std::memcpy(val, F.zv.data(), F.zv.size() * sizeof(double));
    if (d) std::memcpy(d, F.d.data(), F.d.size() * sizeof(double));
    return PSC_OK;
}

int psc_hier_export_level(const psc_hier* h, int32_t l, int32_t* agg, double* p, double* minv,
                          int32_t* rp, int32_t* ci, double* v) {
    if (!h || l < 0 || l >= (int)h->host.lev.size()) return fail(PSC_ERR_ARG, "bad level");
    const HostLevel& H = h->host.lev[l];
    if (agg && !H.agg.empty()) std::memcpy(agg, H.agg.data(), H.n * sizeof(int32_t));
    if (p && !H.p.empty()) std::memcpy(p, H.p.data(), H.n * sizeof(double));
    if (minv) std::memcpy(minv, H.minv.data(), H.n * sizeof(double));
    if (rp) std::memcpy(rp, H.rp.data(), (H.n + 1) * sizeof(int32_t));
    if (ci) std::memcpy(ci, H.ci.data(), H.ci.size() * sizeof(int32_t));
    if (v) std::memcpy(v, H.v.data(), H.v.size() * sizeof(double));
    return PSC_OK;
}

int psc_hier_export_prolongator(const psc_hier* h, int32_t l, int32_t* rp, int32_t* ci, double* v) {
    if (!h || l < 0 || l + 1 >= (int)h->host.lev.size()) return fail(PSC_ERR_ARG, "bad level");
    const HostLevel& H = h->host.lev[l];
    if (rp) std::memcpy(rp, H.prp.data(), H.prp.size() * sizeof(int32_t));
    if (ci) std::memcpy(ci, H.pci.data(), H.pci.size() * sizeof(int32_t));
    if (v) std::memcpy(v, H.pv.data(), H.pv.size() * sizeof(double));
    return PSC_OK;
}

int psc_net_create_l1jacobi(const psc_hier* h, void* hip_stream, psc_net** out) {
    if (!h || !out) return fail(PSC_ERR_ARG, "NULL argument");
    *out = nullptr;
    if (h->host.lev.empty() || (int64_t)h->host.lev[0].minv.size() != h->host.lev[0].n)
        return fail(PSC_ERR_STATE, "hierarchy holds no level-0 l1 diagonal");
    HIPCHK(hipSetDevice(h->device));
    return net_create_jacobi(h->host.lev[0].minv.data(), h->host.lev[0].n, hip_stream, out);
}

int psc_vcycle_apply(psc_hier* h, int32_t prec, const double* r, double* z) {
    if (!h || !r || !z) return fail(PSC_ERR_ARG, "NULL argument");
    if (!h->ctl) return fail(PSC_ERR_STATE, "hierarchy was built host-only");
    if (h->stale) return fail(PSC_ERR_STATE, "the last numeric rebuild failed");
    if (prec != PSC_FP64 && prec != PSC_FP32) return fail(PSC_ERR_ARG, "prec must be PSC_FP64 or PSC_FP32");
    if (prec == PSC_FP32 && !h->has32) return fail(PSC_ERR_STATE, "FP32 V-cycle needs build_fp32");
    HIPCHK(hipSetDevice(h->device));
    int st = join_in(h);
    if (st) return st;
    vcycle(h, prec, r, z, FIN_NONE, nullptr, Gate{nullptr, GATE_NONE});
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    timing_collect(h);
    return join_out(h);
}

int psc_spmv(psc_hier* h, int32_t l, int32_t prec, const void* x, void* y) {
    if (!h || !x || !y || l < 0 || l >= (int)h->lev.size()) return fail(PSC_ERR_ARG, "bad argument");
    if (prec == PSC_FP32 && !h->has32) return fail(PSC_ERR_STATE, "FP32 copies not built");
    if (!h->ctl) return fail(PSC_ERR_STATE, "hierarchy was built host-only");
    if (h->stale) return fail(PSC_ERR_STATE, "the last numeric rebuild failed");
    HIPCHK(hipSetDevice(h->device));
    int st = join_in(h);
    if (st) return st;
    DevLevel& D = h->lev[l];
    {
        TimeScope t(h, l == 0 ? 0 : 7);
        if (prec == PSC_FP64)
            with_A(h, D, [&](auto A) {
                launch_spmv(h, A, (const double*)x, (double*)y, Gate{nullptr, GATE_NONE}, wide_A(h, D));
            });
        else
            with_A32(h, D, [&](auto A) {
                launch_spmv(h, A, (const float*)x, (float*)y, Gate{nullptr, GATE_NONE}, wide_A(h, D));
            });
    }
    HIPCHK(hipGetLastError());
    HIPCHK(hipStreamSynchronize(h->stream));
    timing_collect(h);
    return join_out(h);
}

int psc_timing_enable(psc_hier* h, int32_t on) {
    if (!h) return fail(PSC_ERR_ARG, "NULL handle");
    if (on < 0 || on > 2) return fail(PSC_ERR_ARG, "timing mode must be 0, 1 or 2");
    timing_collect(h);
    h->timing = on;
    return PSC_OK;
}

int psc_timing_get(psc_hier* h, int64_t* counts, double* total_ms) {
    if (!h) return fail(PSC_ERR_ARG, "NULL handle");
    timing_collect(h);
    for (int k = 0; k < PSC_TIMING_KERNELS; k++) {
        if (counts) counts[k] = h->t_count[k];
        if (total_ms) total_ms[k] = h->t_ms[k];
        h->t_count[k] = 0;
        h->t_ms[k] = 0.0;
    }
    return PSC_OK;
}

int psc_tune(psc_hier* h, int32_t key, int32_t value) {
    if (!h) return fail(PSC_ERR_ARG, "NULL handle");
    if (key == PSC_TUNE_BUFLOAD) {
        if (value < 0 || value > 2) return fail(PSC_ERR_ARG, "buffer-load mode must be 0, 1 or 2");
        h->bufload = value;
        drop_graphs(h);
        return PSC_OK;
    }
    if (key == PSC_TUNE_DIA) {
        h->dia = value != 0;
        drop_graphs(h);
        return build_tail(h);
    }
    if (key == PSC_TUNE_FP64_SPLIT) {
        h->fp64_split = value != 0;
        drop_graphs(h);
        return PSC_OK;
    }
    if (key == PSC_TUNE_MIXED_SPLIT) {
        h->mixed_split = value != 0;
        drop_graphs(h);
        return PSC_OK;
    }
    if (key == PSC_TUNE_DIA_UNIFORM) {
        h->dia_uniform = value != 0;
        for (auto& D : h->lev) D.Ad.nd = h->dia_uniform ? D.Ad.nd_u : 0;
        drop_graphs(h);
        return build_tail(h);
    }
    if (key == PSC_TUNE_DIA_ALIGN) {
        h->dia_align = value != 0;
        drop_graphs(h);
        return PSC_OK;
    }
    if (key == PSC_TUNE_CAPPED) {
        h->capped = value != 0;
        drop_graphs(h);
        return PSC_OK;
    }
    if (key == PSC_TUNE_PAIR_R) {
        h->pair_r = value != 0;
        drop_graphs(h);
        return PSC_OK;
    }
    if (key == PSC_TUNE_MIXED_Z32) {
        h->mixed_z32 = value != 0;
        drop_graphs(h);
        return PSC_OK;
    }
    if (key == PSC_TUNE_XCD) {
        const int v = value != 0;
        HIPCHK(hipSetDevice(h->device));
        HIPCHK(hipStreamSynchronize(h->stream));
        HIPCHK(hipMemcpyToSymbol(HIP_SYMBOL(g_xcd_chunked), &v, sizeof(int)));
        drop_graphs(h);
        return PSC_OK;
    }
    if (key == PSC_TUNE_TAIL) {
        if (value < 0 || value > TAIL_MAX_ROWS) return fail(PSC_ERR_ARG, "tail row limit must be 0..4096");
        h->tail = value != 0;
        h->tail_rows = value;
        drop_graphs(h);
        return build_tail(h);
    }
    if (key == PSC_TUNE_SPLIT) {
        if (value == 0 && (h->nu > 1 || h->opts.vcycle_double || h->opts.smoothed_prol))
            return fail(PSC_ERR_ARG, "the gathering sweeps support only one sweep with the tentative prolongator");
        h->split = value != 0;
        build_tail(h);
        drop_graphs(h);
        return PSC_OK;
    }
    if (key == PSC_TUNE_SPMV2) {
        h->spmv2 = value != 0;
        drop_graphs(h);
        return PSC_OK;
    }
    if (key == PSC_TUNE_UNROLL4) {
        h->unroll4 = value != 0;
        drop_graphs(h);
        return PSC_OK;
    }
    if (key == PSC_TUNE_FUSED_PCG) {
        h->fused_pcg = value != 0;
        drop_graphs(h);
        return PSC_OK;
    }
    if (key == PSC_TUNE_GRID_MAX) {
        if (value < NXCD || value > GMAX || value % NXCD) return fail(PSC_ERR_ARG, "grid cap must be a multiple of 8 in [8, 131072]");
        h->gmax = value;
        drop_graphs(h);
        return PSC_OK;
    }
    return fail(PSC_ERR_ARG, "unknown tuning key");
}

}  // extern "C"

