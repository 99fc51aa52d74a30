// setup.h -- host-side AMG hierarchy construction (internal to libpsc).
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace psc {

// Factored approximate inverse G = Z D^-1 Z^T of a level (AINV / INVK
// smoothers): Z unit upper triangular by columns (column k: rows
// zi[zr[k] .. zr[k+1]) ascending, values zv), pivots d.
struct HostFai {
    std::vector<int64_t> zr;
    std::vector<int32_t> zi;
    std::vector<double> zv, d;
    bool empty() const { return zr.size() < 2; }
};

// One level of the host hierarchy. A_l is CSR with ascending columns.
struct HostLevel {
    int64_t n = 0;
    std::vector<int32_t> rp, ci;
    std::vector<double> v;
    std::vector<double> w;      // near-kernel sample vector at this level
    std::vector<double> minv;   // l1-Jacobi inverse diagonal
    int64_t nc = 0;             // rows of the next level (0 at the coarsest)
    std::vector<int32_t> agg;   // aggregate of each row
    std::vector<double> p;      // the entry of row i of the tentative prolongator
    // prolongator the V-cycle uses (CSR, aggregate columns): the tentative one,
    // or the smoothed (I - omega D^-1 A) P^ with omega = 1/||D^-1 A||_inf
    std::vector<int32_t> prp, pci;
    std::vector<double> pv;
    double omega = 0.0;
    // A_l P_l when the smoothed prolongator's Galerkin product formed it
    // (reused for (I - M^-1 A) P; empty otherwise)
    std::vector<int32_t> aprp, apci;
    std::vector<double> apv;
    HostFai fai;                // AINV / INVK smoother (empty with l1-Jacobi)
};

struct HostHier {
    std::vector<HostLevel> lev;
    std::vector<double> coarse_inv;   // dense inverse of the coarsest A, row-major
    int coarse_sweeps = 0;            // > 0: coarsest solved by l1-Jacobi sweeps instead
    int coarse_pcg = 0;               // > 0: coarsest solved by at most this many l1-Jacobi PCG iterations
    double coarse_rtol = 1e-4;        // their relative residual tolerance
};

struct SetupOpts {
    int sweeps = 2;
    int coarse_max = 200;
    int max_levels = 30;
    int coarse_sweeps = 30;
    int prol = 0;               // 0 tentative prolongator, 1 smoothed
    int aggr = 0;               // 0 coupled matching, 1 decoupled VBM
    double theta = 0.01;        // VBM strength threshold
    bool device = false;        // coarsen matching / tentative levels on the GPU
    bool device_products = false;   // smoothed prolongator: its products on the GPU
    int smoother = 0;           // 0 l1-Jacobi, 1 AINV, 2 INVK, 3 polynomial (levels above the coarsest)
    double tau = 0.1;           // AINV drop tolerance
    int fill1 = 0, fill2 = 1;   // INVK fill levels of the factor and of its inverse
    int coarse_pcg = 0;         // > 0: factored coarsest replaced by at most this many PCG iterations
    double coarse_rtol = 1e-4;
};

// Setup phase trace: with the environment variable PSC_SETUP_TRACE set, the
// build prints "[psc setup] <phase> <seconds>" lines to stderr.
struct PhaseTimer {
    const char* name;
    double t0;
    explicit PhaseTimer(const char* n);
    ~PhaseTimer();
};

// Status codes follow psc.h.
int validate_csr(int64_t n, const int32_t* rp, const int32_t* ci, const double* v,
                 std::string& err);
int build_hierarchy(int64_t n, const int32_t* rp, const int32_t* ci, const double* v,
                    const SetupOpts& o, HostHier& H, std::string& err);

// AINV / INVK factors of every level above the coarsest (nothing for the
// other smoothers).
int build_smoothers(HostHier& H, const SetupOpts& o, std::string& err);

// Numeric-only rebuild: new values v0 of A_0 on the sparsity pattern the
// hierarchy was built with. Aggregates, prolongator patterns and the
// coarsest-level choice are kept; everything that depends on the values
// (l1 diagonals, smoothed prolongators, Galerkin values, the coarsest
// factor, AINV / INVK factors) is recomputed in the build's order, so the
// result equals a build that reached the same aggregates.
int rebuild_numeric(HostHier& H, const double* v0, const SetupOpts& o, std::string& err);

// AINV / INVK factors of one SPD CSR matrix (Section "GPU enabled smoothers").
int build_ainv(int64_t n, const int32_t* rp, const int32_t* ci, const double* v, double tau, HostFai& F,
               std::string& err);
int build_invk(int64_t n, const int32_t* rp, const int32_t* ci, const double* v, int fill1, int fill2,
               HostFai& F, std::string& err);

// S P = (I - M_l^-1 A_l) P_l, the level's prolongator after one (weighted)
// l1-Jacobi sweep with the inverse diagonal minv (rows of A_l, aggregate
// columns), CSR with ascending columns.
void jacobi_smoothed_prolongator(const HostLevel& H, const double* minv, std::vector<int32_t>& rp,
                                 std::vector<int32_t>& ci, std::vector<double>& v);

// One level's coarsening on the GPU (matching aggregation, tentative
// prolongator): aggregates, p, the next sample vector and (want_coarse) the
// Galerkin product, bit-identical to the host path. Returns PSC_ERR_STATE when the
// level does not fit the device kernels (the caller then uses the host).
int gpu_coarsen_level(int64_t n, const int32_t* rp, const int32_t* ci, const double* v, const double* w,
                      int sweeps, bool want_coarse, std::vector<int32_t>& agg, int64_t& nc, std::vector<double>& p,
                      std::vector<double>& wc, std::vector<int32_t>& crp, std::vector<int32_t>& cci,
                      std::vector<double>& cv, std::string& err);

// The smoothed prolongator's products of one level on the GPU, bit-identical
// to the host's: omega, P = (I - omega D^-1 A) P^ (CSR), A P (CSR) and the
// Galerkin operator P^T (A P) (CSR), from the level's CSR, its aggregates and
// p (P^_{i,agg_i} = p_i). Returns PSC_ERR_STATE when a product row exceeds
// the device kernels' column capacity (the caller then uses the host).
int gpu_smoothed_products(int64_t n, const int32_t* rp, const int32_t* ci, const double* v, const int32_t* agg,
                          const double* p, int64_t nc, double& omega, std::vector<int32_t>& prp,
                          std::vector<int32_t>& pci, std::vector<double>& pv, std::vector<int32_t>& aprp,
                          std::vector<int32_t>& apci, std::vector<double>& apv, std::vector<int32_t>& crp,
                          std::vector<int32_t>& cci, std::vector<double>& cv, std::string& err);

// Pattern of S P for the tentative prolongator (one entry per row of P, at
// column agg_i): row i holds the distinct aggregates of its columns,
// ascending, which is the pattern jacobi_smoothed_prolongator stores.
void tentative_sp_pattern(const HostLevel& H, std::vector<int32_t>& rp, std::vector<int32_t>& ci);

// Numeric rebuild, tentative prolongator: S P = (I - M^-1 A) P recomputed on
// the device into the build's hacked-ELL slots of S P (sp_pair: the paired
// layout) from A's refreshed
// hacked-ELL values (a_rp: A's row pointers, device), agg, p and minv, with
// the host's summation order (bit-identical to jacobi_smoothed_prolongator).
// Every pointer is a device pointer; stream is a hipStream_t.
int gpu_tentative_sp(void* stream, int64_t n, const long long* a_off, const int* a_col, const double* a_val,
                     const int32_t* a_rp, const int32_t* agg, const double* p, const double* minv,
                     const long long* sp_off, const int* sp_col, double* sp_val, float* sp_val32, int sp_pair,
                     std::string& err);

// Pack CSR rows into hacked DIA with 64-row slices (offsets ascending per
// slice, values diagonal-major in a slice, zeros where a row has no entry).
// Returns false and packs nothing when the diagonal slots would exceed
// max_ratio times max_slots, or when row + offset could leave int32.
// v == NULL packs the layout only (start, offs, uniform; val left empty).
// With uniform != NULL and at most 8 distinct offsets over the whole matrix,
// every slice gets all of them (zeros where a row has no entry) and *uniform
// receives the offsets (ascending); otherwise it is left empty.
bool pack_dia(int64_t nrows, int64_t ncols, const int32_t* rp, const int32_t* ci, const double* v,
              long long max_slots, std::vector<int32_t>& start, std::vector<int32_t>& offs,
              std::vector<double>& val, std::vector<int32_t>* uniform = nullptr);

// Pack CSR rows into hacked ELL with 64-row slices (column-major in a
// slice). Padding slots carry value 0 and repeat the row's last column (0 for
// rows past the end), so every slot reads a valid, usually cached, entry.
// v == NULL packs the layout only (off and col; val left empty).
void pack_ell(int64_t nrows, const int32_t* rp, const int32_t* ci, const double* v,
              std::vector<long long>& off, std::vector<double>& val, std::vector<int>& col);

// The same in the paired layout of two 64-row slices per 128-row block (one
// width per block; entry k of block row r at off[2S] + 128 k + r; off[s] =
// off[2S] + 64 (s & 1); off has nslices + 2 entries, the last two the total).
void pack_ell_paired(int64_t nrows, const int32_t* rp, const int32_t* ci, const double* v,
                     std::vector<long long>& off, std::vector<double>& val, std::vector<int>& col);

// Capped hacked ELL for operators whose row lengths vary widely (a few long
// rows in most slices, as on the stalled coarse levels of strongly varying
// coefficients): every slice stores at most `cap` slots per row, and the
// entries of a longer row past its first `cap` go to the overflow of its
// slice: entries xs[s] .. xs[s+1]-1, grouped by row in lane order (CSR order
// within a row), with columns xc, the row's lane xl and the CSR position xsrc
// (for filling values). v == NULL packs the layout only.
void pack_ell_capped(int64_t nrows, const int32_t* rp, const int32_t* ci, const double* v, int cap,
                     std::vector<long long>& off, std::vector<double>& val, std::vector<int>& col,
                     std::vector<long long>& xs, std::vector<int>& xc, std::vector<unsigned char>& xl,
                     std::vector<long long>& xsrc);

// Cap for pack_ell_capped, or 0 when the plain layout is as good. A slice's
// cost is counted in wavefront loads: min(w_s, cap) for its capped slots plus
// three per 64 overflow entries (a load, a gather and the cross-lane scan);
// the cheapest cap up to 48 (the widest one-row-per-lane slices) is taken
// when it costs at most 0.9 of the plain layout's sum of slice widths.
int choose_ell_cap(int64_t nrows, const int32_t* rp);

}  // namespace psc
