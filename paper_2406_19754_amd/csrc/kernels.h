// kernels.h -- device-side building blocks shared by the HIP sources of libpsc.
#pragma once
#include <type_traits>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace psc {

constexpr int WG = 256;        // threads per workgroup: 4 wavefronts of 64
constexpr int SLICE = 64;      // rows per hacked-ELL slice: one wavefront
constexpr int NXCD = 8;        // accelerator complex dies; workgroups are dealt round-robin
constexpr int GMAX = 131072;   // largest grid of the streaming kernels (PSC_TUNE_GRID_MAX)
constexpr int GDEF = 131072;   // their default cap

// Solver control block, device resident. Scalars of the Krylov recurrence
// live here so no host round trip is needed between kernels.
struct Ctl {
    double rtol, nb2, rr, rr_old, rho, alpha, beta, pq, pr, zq, zr, pq_prev, out0, out1;
    int done, iter, status, maxit;
    int check, have_prev, net_on, use_net, fallbacks, form;
    int redo;      // fused FCG: the residual was replaced, redo the level-0 pre-smoothing
    int net_fails; // consecutive network steps whose output failed z.r > 0
};

// Which kernels of an iteration run: GATE_NONE always; GATE_DONE until the
// solve is over; GATE_NET only on a network step; GATE_VC only on a V-cycle
// step (the choice is made on the device, see ctl->use_net).
enum GateMode { GATE_NONE = 0, GATE_DONE = 1, GATE_NET = 2, GATE_VC = 3, GATE_REDO = 4 };
struct Gate {
    const Ctl* ctl;
    int mode;
};
__device__ __forceinline__ bool gate_skip(const Gate& g) {
    if (!g.ctl || g.mode == GATE_NONE) return false;
    if (g.ctl->done) return true;
    if (g.mode == GATE_NET) return !g.ctl->use_net;
    if (g.mode == GATE_VC) return g.ctl->use_net != 0;
    if (g.mode == GATE_REDO) return !g.ctl->redo;
    return false;
}

// Host-mapped mirror polled by the host loop.
struct HostCtl {
    int done, iter, status, fallbacks;
    int net_off;   // the learned network was switched off for the rest of the solve
};

// Hacked-ELL operator: slices of 64 rows; slice s holds its w_s columns
// column-major at [off[s], off[s+1]) (w_s = (off[s+1]-off[s])/64).
//
// Paired layout (pair = 1): slices 2S and 2S+1 form a block of 128 rows with
// one width w_S (the larger of the two), block-major: entry k of row r of the
// block at off[2S] + k*128 + r, so one lane reads two consecutive rows'
// entries with one 16-byte (FP64 values) or 8-byte (indices, FP32 values)
// load. off[s] = off[2S] + (s & 1)*64 is slice s's first entry, the slot
// stride is 128, w_S = (off[2S+2] - off[2S]) / 128, and off holds nslices + 2
// entries (the last two equal: the total).
//
template <typename T>
struct Ell {
    using value_type = T;
    const long long* off;
    const T* val;
    const int* col;
    long long nrows;
    long long nslices;
    long long ncols;
    int pair = 0;
};

// Capped hacked ELL (never paired): the slices hold at most a cap of slots
// per row; a longer row's remaining entries go to the overflow of its slice,
// entries xs[s] .. xs[s+1]-1 (values xv, columns xc, and xl = the lane of
// their row), grouped by row in lane order, each row's in CSR order. A
// wavefront takes them 64 at a time, one per lane, and sums each row's run
// with a segmented scan across the lanes (fixed order). A type of its own, so
// that only the kernels instantiated for it carry the overflow code.
template <typename T>
struct EllC : Ell<T> {
    const long long* xs = nullptr;
    const T* xv = nullptr;
    const int* xc = nullptr;
    const unsigned char* xl = nullptr;
};

template <typename M>
struct is_ell : std::false_type {};
template <typename T>
struct is_ell<Ell<T>> : std::true_type {};
template <typename T>
struct is_ell<EllC<T>> : std::true_type {};

// Hacked-DIA operator (the hacked diagonal format of the PSBLAS extensions):
// slice s of 64 rows holds the diagonals start[s] .. start[s+1]-1, with
// offsets offs[k] = column - row (ascending) and values at val[k*64 + lane],
// zero where the row stores nothing on that diagonal. A 7-point stencil slice
// keeps 7 diagonals: 8 bytes per entry instead of 12 for hacked ELL.
//
// Uniform variant (nd > 0): every slice holds the same nd <= 8 diagonals, at
// the offsets uo[0..nd) carried in the kernel argument itself (start[s] =
// s*nd still holds), so a slice needs no metadata load before its gathers.
//
// Paired layout (pair = 1, every uniform layout): the slices are stored two
// by two as blocks of 128 rows, block S holding diagonal k of its rows r at
// val[S*nd*128 + k*128 + r], so that one lane can read two consecutive rows
// with one 16-byte load; slice s of 64 rows starts at (s>>1)*nd*128 +
// (s&1)*64 with a diagonal stride of 128.
template <typename T>
struct Dia {
    using value_type = T;
    const int* start;
    const int* offs;
    const T* val;
    long long nrows;
    long long nslices;
    long long ncols;
    int nd = 0;
    int uo[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int pair = 0;
};

}  // namespace psc
