/*
 * psc.h -- C ABI of the MI355X (gfx950) AMG-preconditioned CG library.
 *
 * The library implements the solve phase of the method of D'Ambra,
 * Durastante and Filippone, "PSCToolkit: solving sparse linear systems with
 * a large number of GPUs" (arXiv 2406.19754): conjugate gradient
 * preconditioned by an algebraic multigrid V-cycle built by coupled
 * aggregation based on compatible weighted matching, with l1-Jacobi
 * smoothing. Two further forms run inside flexible CG: a V-cycle evaluated
 * in FP32, and a small learned convolutional preconditioner alternated with
 * the V-cycle.
 *
 * Conventions for every entry point:
 *   - Return value is a status code (PSC_OK = 0, PSC_NOCONV = 1, errors < 0),
 *     in the spirit of the paper's `info` argument (Section "PSBLAS
 *     applications"). No C++ exception crosses this boundary.
 *   - psc_last_error() returns a thread-local message for the last error.
 *   - Pointers named *_host are host memory; pointers named *_dev are device
 *     memory on the GPU that was current when the handle was created. All
 *     arrays are dense, contiguous, and owned by the caller; the library
 *     never keeps a caller pointer after a call returns.
 *   - All device work of a handle is issued on the HIP stream given at
 *     creation (NULL = the null stream). Calls on one handle are not
 *     thread-safe; distinct handles are independent.
 *   - Out-parameters are written only on PSC_OK, except that iteration
 *     counts and residuals are also written on PSC_NOCONV.
 */
#ifndef PSC_H
#define PSC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes -------------------------------------------------------- */
#define PSC_OK            0
#define PSC_NOCONV        1   /* maxit reached; iters / relres are valid */
#define PSC_ERR_ARG      -1   /* malformed argument (CSR structure, sizes, NULL) */
#define PSC_ERR_NOT_SPD  -2   /* non-positive diagonal, Cholesky or CG breakdown */
#define PSC_ERR_NAN      -3   /* NaN / Inf met in the right-hand side or iteration */
#define PSC_ERR_HIP      -4   /* a HIP runtime call failed */
#define PSC_ERR_OOM      -5   /* host or device allocation failed */
#define PSC_ERR_COARSEN  -6   /* coarsening stalled above the coarsest-size limit */
#define PSC_ERR_STATE    -7   /* handle not in a state that allows the call */
#define PSC_ERR_IO       -8   /* checkpoint file cannot be opened, read or written, or is not one */

/* ---- precisions ---------------------------------------------------------- */
#define PSC_FP64 0
#define PSC_FP32 1

typedef struct psc_hier psc_hier;   /* opaque: owns all device memory of a hierarchy */
typedef struct psc_net  psc_net;    /* opaque: owns the learned preconditioner       */

/*
 * Hierarchy options. psc_amg_opts_default() fills the defaults:
 *   sweeps = 2       pairwise matching sweeps per level; aggregates hold at
 *                    most 2^sweeps rows (Section "Aggregation strategies",
 *                    multiple matching sweeps).
 *   coarse_max = 200 a level with at most this many rows is the coarsest one
 *                    and is solved exactly by dense Cholesky.
 *   max_levels = 30  hard cap on the number of levels.
 *   coarse_sweeps = 30  when coarsening stalls (a level keeps more than 0.9
 *                    of the rows of the level above) that level becomes the
 *                    coarsest; with at most 2000 rows it is factored, else
 *                    it is solved by this many FP64 l1-Jacobi sweeps from a
 *                    zero guess (the l1-Jacobi coarsest solver of Section
 *                    "GPU enabled smoothers"). 0 makes such a stall an error.
 *   smoothed_prol = 0  1: the smoothed prolongator P = (I - omega D^-1 A) P^
 *                    of the tentative P^, D = diag(A), omega = 1/||D^-1 A||_inf
 *                    (Section "Aggregation strategies"), with the general
 *                    Galerkin product A_{l+1} = P^T A_l P; with sweeps = 3 and
 *                    smoother_sweeps = 4 this is the paper's SMATCH setting.
 *   smoother_sweeps = 1  l1-Jacobi sweeps before and after the coarse
 *                    correction on every level (1..16; the paper's examples
 *                    use 4).
 *   vcycle_double = 0  1: variable V-cycle, level l smooths with
 *                    smoother_sweeps * 2^l sweeps (capped at 4096); with
 *                    sweeps = 3, the tentative prolongator and
 *                    smoother_sweeps = 2 this is the paper's VMATCH setting.
 *   aggregation = 0  PSC_AGGR_MATCHING: coupled aggregation by compatible
 *                    weighted matching (sweeps matching sweeps per level);
 *                    PSC_AGGR_VBM: decoupled Vanek-Mandel-Brezina
 *                    aggregation of strongly coupled neighbourhoods,
 *                    |a_ij| >= vbm_theta sqrt(a_ii a_jj), with
 *                    P^_{i,agg(i)} = w_i (Section "Aggregation strategies");
 *                    with smoothed_prol = 1 and smoother_sweeps = 4 this is
 *                    the paper's VBM setting. sweeps is ignored for VBM.
 *   vbm_theta = 0.01 strength threshold of PSC_AGGR_VBM, in [0, 1).
 *   setup_device = 1  coarsen on the GPU where the setting allows it
 *                    (matching aggregation with the tentative prolongator):
 *                    matching, aggregates, prolongator and Galerkin product
 *                    are computed by device kernels in the host setup's
 *                    arithmetic order, so the hierarchy is the same bit for
 *                    bit; levels the kernels cannot take (a coarse row with
 *                    more than 64 distinct columns) fall back to the host.
 *                    Ignored (host setup) with host_only.
 *   setup_device_products = 0  with setup_device and the smoothed
 *                    prolongator, also form omega, P, A P and the Galerkin
 *                    product P^T (A P) on the GPU (sparse products summed in
 *                    the host's order: the same hierarchy bit for bit); levels
 *                    whose operator rows exceed 64 entries, or whose product
 *                    rows exceed 1024 columns, stay on the host. Off by
 *                    default: the products travel back to the host, and those
 *                    transfers cost about what the host's products do.
 *   build_fp32 = 0   also build the FP32 copies of the level operators that
 *                    the mixed-precision V-cycle needs.
 *   use_graph = 1    capture the per-iteration kernel sequence as a HIP
 *                    graph and replay it.
 *   smoother = 0     PSC_SMOOTH_L1JACOBI; PSC_SMOOTH_AINV or PSC_SMOOTH_INVK
 *                    replace M_l^-1 in every smoothing sweep of the levels
 *                    above the coarsest by G_l = Z D^-1 Z^T ~ A_l^-1, Z unit
 *                    upper triangular, D > 0 diagonal (Section "GPU enabled
 *                    smoothers"): AINV by the stabilised incomplete
 *                    A-biconjugation with drop tolerance ainv_tau (applied to
 *                    the matrix scaled to unit diagonal); INVK by the inverse
 *                    of an incomplete LDL^T factor with level of fill
 *                    invk_fill, inverted on a pattern of level invk_inv_fill.
 *                    A sweep is x <- x + Z (D^-1 Z^T (b - A x)): products with
 *                    A, D^-1 Z^T and Z. The coarsest solve is unchanged. The
 *                    factors are built on the host (setup_device does not
 *                    apply to them); PSC_ERR_NOT_SPD on a non-positive pivot.
 *                    PSC_SMOOTH_CHEB4: a polynomial smoother (polynomial
 *                    smoothers are named as GPU-friendly future work in the
 *                    Conclusions): the fourth-kind Chebyshev smoother of degree
 *                    smoother_sweeps on the l1-Jacobi preconditioned operator
 *                    M^-1 A with the bound 1 (A <= M for the l1 diagonal), so
 *                    no eigenvalue estimate is needed; its error propagation is
 *                    W_nu(I - 2 M^-1 A) / (2 nu + 1), W the Chebyshev polynomial
 *                    of the fourth kind. Degree 1 is l1-Jacobi weighted 4/3.
 *   coarse_pcg_iters = 0  > 0: the coarsest level, where it would be
 *                    factored, is solved instead by at most this many
 *                    iterations of CG preconditioned by l1-Jacobi from a zero
 *                    guess, stopped at ||r|| <= coarse_rtol ||b|| (the paper's
 *                    coarsest solver in its tests, Section "Algorithmic tests",
 *                    with 40 iterations). The V-cycle then depends nonlinearly
 *                    on its input: use psc_fcg_solve. Runs in one workgroup;
 *                    the coarsest level must have at most 4096 rows
 *                    (PSC_ERR_ARG otherwise). Coarsest levels left by a stall
 *                    above 2000 rows keep their l1-Jacobi sweeps.
 *   coarse_rtol = 1e-4  tolerance of that solve (>= 0; 0: always the cap).
 *   ainv_tau = 0.1   AINV drop tolerance (>= 0).
 *   invk_fill = 0, invk_inv_fill = 1   INVK levels of fill (0..64).
 *   capped_min_rows = 65536  levels with at least this many rows whose row
 *                    lengths vary widely get a capped hacked-ELL copy
 *                    (PSC_TUNE_CAPPED); smaller levels are bound by their
 *                    longest slice, not by the bytes read, and keep the plain
 *                    layout. 1: every level where a cap pays; 0: none.
 *   host_only = 0    build the hierarchy on the host only and make no HIP
 *                    call (for inspection with psc_hier_info and
 *                    psc_hier_export_level on machines without a GPU);
 *                    solve and apply calls then return PSC_ERR_STATE.
 */
#define PSC_AGGR_MATCHING 0
#define PSC_AGGR_VBM 1
#define PSC_SMOOTH_L1JACOBI 0
#define PSC_SMOOTH_AINV 1
#define PSC_SMOOTH_INVK 2
#define PSC_SMOOTH_CHEB4 3

typedef struct {
    int32_t sweeps;
    int32_t coarse_max;
    int32_t max_levels;
    int32_t build_fp32;
    int32_t use_graph;
    int32_t host_only;
    int32_t coarse_sweeps;
    int32_t smoothed_prol;
    int32_t smoother_sweeps;
    int32_t vcycle_double;
    int32_t aggregation;
    int32_t setup_device;
    int32_t smoother;
    int32_t invk_fill;
    int32_t invk_inv_fill;
    int32_t setup_device_products;
    double  vbm_theta;
    double  ainv_tau;
    int32_t coarse_pcg_iters;
    int32_t capped_min_rows;
    double  coarse_rtol;
} psc_amg_opts;

void psc_amg_opts_default(psc_amg_opts* opts);

/*
 * Build the AMG hierarchy of the n x n symmetric positive-definite matrix A
 * given in CSR form (Section "AMG4PSBLAS": Galerkin coarse operators
 * A_{l+1} = P_l^T A_l P_l; Section "Aggregation strategies": coupled
 * aggregation by compatible weighted matching with tentative prolongator,
 * eq. (prolongator); Section "GPU enabled smoothers": l1-Jacobi diagonal).
 *   n           rows (> 0)
 *   rowptr_host n+1 int32, rowptr[0] = 0, non-decreasing
 *   col_host    rowptr[n] int32 column indices, strictly ascending per row,
 *               in [0, n); every row holds its diagonal
 *   val_host    rowptr[n] FP64 values; diagonal entries must be > 0
 *   opts        NULL for defaults
 *   hip_stream  hipStream_t used for all device work of the handle
 *   out         receives the handle; release with psc_hier_free
 * With setup_device = 1 (the default) the coarsening of the matching
 * setting runs on the GPU (matching, aggregates, prolongator, Galerkin
 * product) and the values of every storage format are filled on the GPU;
 * the layouts, the smoother setup of other settings and the coarsest factor
 * are computed on the host (the paper's build is mostly host-side). The CSR
 * arrays are copied; the caller keeps them.
 * Errors: PSC_ERR_ARG (malformed CSR or options), PSC_ERR_NOT_SPD
 * (diagonal <= 0 or coarsest Cholesky breakdown), PSC_ERR_COARSEN (a stall
 * above 2000 rows with coarse_sweeps = 0, or a coarsest level forced by
 * max_levels above 4096 rows), PSC_ERR_OOM, PSC_ERR_HIP.
 * Symmetry is assumed, not checked.
 */
int psc_amg_build(int32_t n, const int32_t* rowptr_host, const int32_t* col_host,
                  const double* val_host, const psc_amg_opts* opts, void* hip_stream,
                  psc_hier** out);

/*
 * Numeric-only rebuild: replace the values of A (same n, rowptr and col as
 * at psc_amg_build; val_host holds rowptr[n] FP64 values) and recompute
 * everything that depends on them -- l1 diagonals, smoothed prolongators,
 * Galerkin operators A_{l+1} = P_l^T A_l P_l, the coarsest factor, AINV /
 * INVK factors -- while keeping the aggregates, the prolongator patterns and
 * the level structure, so no matching runs (Section "GPU support": the
 * toolkit updates the coefficients of an existing matrix whose structure is
 * preserved, and splits the AMG build so that parts of it can be redone on
 * an assembled hierarchy, because building is mostly host-side). The result is
 * the hierarchy a build would give if it reached the same aggregates. Device
 * copies are refreshed and captured iterations dropped; the handle's
 * options, stream and workspace stay. Not thread-safe with work in flight on
 * the handle (the call synchronizes its stream first).
 * Errors: PSC_ERR_ARG (NULL), PSC_ERR_NOT_SPD (a diagonal <= 0 or a
 * Cholesky / incomplete-factorisation breakdown), PSC_ERR_HIP, PSC_ERR_OOM.
 * After an error the handle refuses solves and applies (PSC_ERR_STATE) until
 * a rebuild succeeds.
 */
int psc_amg_rebuild(psc_hier* h, const double* val_host);

/*
 * Preconditioned conjugate gradient with the FP64 V-cycle (one l1-Jacobi
 * pre- and post-sweep, coarsest solve as chosen at build; Section "AMG4PSBLAS",
 * eq. (amg)) as the preconditioner. Stops when the recursive residual
 * satisfies ||r||_2 <= rtol ||b||_2 (Section "Numerical Example").
 *   b_dev    n FP64, right-hand side
 *   x_dev    n FP64, in: initial guess, out: solution
 *   iters    out: iterations taken
 *   relres   out: true relative residual ||b - A x||_2 / ||b||_2 in FP64
 * b = 0 gives x = 0, iters = 0. Returns PSC_NOCONV when maxit is reached,
 * PSC_ERR_NAN when b or an iterate holds NaN/Inf, PSC_ERR_NOT_SPD on a
 * breakdown (p.q <= 0 or r.z <= 0); x_dev then holds the last iterate
 * before the breakdown.
 */
int psc_pcg_solve(psc_hier* h, const double* b_dev, double* x_dev, double rtol,
                  int32_t maxit, int32_t* iters, double* relres);

/*
 * Flexible CG with one stored direction, FCG(1) (the paper runs its tests
 * with flexible CG, Section "Numerical Example"): z = B_k r,
 * p = z - ((z.q_prev)/(p_prev.q_prev)) p_prev, q = A p,
 * alpha = (p.r)/(p.q). When the recursive residual passes the test the
 * true residual b - A x is formed in FP64; if it fails, r is replaced by it
 * and the directions restart.
 *   vcycle_prec  PSC_FP64, or PSC_FP32 (the V-cycle in FP32: level
 *                operators, smoothing and transfers in FP32, the coarsest
 *                solve in FP64; needs build_fp32)
 *   net          NULL for the V-cycle only; else the iterations k = 1, 3,
 *                5, ... (counting from 0) apply the learned network
 *                z = s net(r/s), s = ||r||/sqrt(n), with the V-cycle taken
 *                instead when z.r <= 0. The network is switched off for the
 *                rest of the solve when a network step leaves
 *                ||r_new|| > 0.9 ||r_old|| (stagnation), or when two
 *                scheduled network steps in a row fail z.r > 0. The grid
 *                declared with psc_net_set_grid must have nx*ny*nz = n.
 *   fallbacks    out (may be NULL): scheduled network steps that ran the
 *                V-cycle instead (also those after the switch-off)
 * Other arguments and errors as for psc_pcg_solve.
 */
int psc_fcg_solve(psc_hier* h, psc_net* net, int32_t vcycle_prec, const double* b_dev,
                  double* x_dev, double rtol, int32_t maxit, int32_t* iters,
                  double* relres, int32_t* fallbacks);

/* Hierarchy statistics. Arrays hold one entry per level. */
#define PSC_MAX_LEVELS 32
typedef struct {
    int32_t levels;
    int64_t rows[PSC_MAX_LEVELS];
    int64_t nnz[PSC_MAX_LEVELS];
    int64_t ell_slots[PSC_MAX_LEVELS];       /* padded hacked-ELL slots of A_l */
    double  operator_complexity;             /* sum nnz(A_l) / nnz(A_0) */
    double  vcycle_bytes_fp64;               /* algorithmic bytes of one V-cycle (current kernels) */
    double  vcycle_bytes_fp32;
    double  spmv_bytes_fp64;                 /* algorithmic bytes of y = A_0 x: nnz x (8 + 4 in
                                                hacked ELL, 8 in hacked DIA) + 16 n */
    double  setup_seconds;                   /* host setup wall time */
    int64_t device_bytes;                    /* device memory held by the handle */
    int32_t coarse_sweeps;                   /* 0: coarsest factored, else l1-Jacobi sweeps */
    int64_t sp_nnz[PSC_MAX_LEVELS];          /* nonzeros of the smoothed prolongator
                                                (I - M_l^-1 A_l) P_l (0 at the coarsest) */
    int64_t dia_slots[PSC_MAX_LEVELS];       /* hacked-DIA slots of A_l, 0 when A_l has no DIA copy */
    int64_t p_nnz[PSC_MAX_LEVELS];           /* nonzeros of the prolongator P_l (0 at the coarsest) */
    double  omega[PSC_MAX_LEVELS];           /* smoothed prolongator damping per level (0: tentative) */
    int32_t smoother_sweeps;
    int32_t smoothed_prol;
    int32_t vcycle_double;
    int32_t aggregation;
    int32_t smoother;
    int64_t smoother_nnz[PSC_MAX_LEVELS];    /* AINV / INVK: nonzeros of Z_l (0 otherwise) */
    double  rebuild_seconds;                 /* wall time of the last psc_amg_rebuild (0: none) */
    int32_t coarse_pcg_iters;                /* > 0: coarsest solved by at most this many PCG iterations */
    int32_t tail_level;                      /* first level run by the one-workgroup tail (0: none) */
    int32_t tail_lds_bytes;                  /* LDS of the FP64 tail kernel (0: none) */
    int32_t capped_cap[PSC_MAX_LEVELS];      /* slots per row of A_l's capped hacked-ELL copy
                                                (PSC_TUNE_CAPPED; 0: no such copy) */
    int64_t capped_slots[PSC_MAX_LEVELS];    /* its slice slots, plus its overflow entries */
    int32_t pair_restrict[PSC_MAX_LEVELS];   /* 1: level l restricts pair sums (PSC_TUNE_PAIR_R) */
} psc_hier_stats;

int psc_hier_info(const psc_hier* h, psc_hier_stats* s);

/*
 * Copy one level's setup data to host arrays (for tests). Any pointer may
 * be NULL. agg_host (rows[l] int32): aggregate of each row; p_host
 * (rows[l] FP64): value of the single prolongator entry of each row;
 * minv_host (rows[l] FP64): l1-Jacobi inverse diagonal; rowptr/col/val:
 * A_l in CSR (rows[l]+1, nnz[l], nnz[l]). agg and p are only defined below
 * the coarsest level.
 */
int psc_hier_export_level(const psc_hier* h, int32_t level, int32_t* agg_host,
                          double* p_host, double* minv_host, int32_t* rowptr_host,
                          int32_t* col_host, double* val_host);

/*
 * Copy the prolongator P_l the V-cycle uses (the tentative one, or the
 * smoothed one) as CSR with aggregate columns: rowptr_host rows[l]+1 int32,
 * col_host / val_host p_nnz[l] entries. Levels below the coarsest only
 * (else PSC_ERR_ARG).
 */
int psc_hier_export_prolongator(const psc_hier* h, int32_t level, int32_t* rowptr_host,
                                int32_t* col_host, double* val_host);

/*
 * Copy the AINV / INVK factor of level l (levels above the coarsest of a
 * hierarchy built with that smoother, else PSC_ERR_ARG): Z by columns,
 * colptr_host rows[l]+1 int64, row_host / val_host smoother_nnz[l] entries
 * (rows ascending in a column, the unit diagonal included), d_host rows[l]
 * FP64 pivots; G_l = Z diag(d)^-1 Z^T. Any pointer may be NULL.
 */
int psc_hier_export_smoother(const psc_hier* h, int32_t level, int64_t* colptr_host, int32_t* row_host,
                             double* val_host, double* d_host);

/* z = B r: one V-cycle (FP64 or FP32 form) on device vectors of size n. */
int psc_vcycle_apply(psc_hier* h, int32_t prec, const double* r_dev, double* z_dev);

/* y = A_l x on level l's hacked-ELL operator, FP64 (prec = PSC_FP64) or
 * its FP32 copy (x and y are then float*). For tests and bandwidth runs. */
int psc_spmv(psc_hier* h, int32_t level, int32_t prec, const void* x_dev, void* y_dev);

/*
 * Kernel timing. When enabled (on = 1), the library records HIP events on its
 * stream around every launch of the level-0 kernels during solves (which
 * disables graph replay) and accumulates their durations; on = 2 records
 * only the outer SpMV pass (kernel id 0), so the rest of each iteration runs
 * back to back as in a replay. Launches issued past convergence (they exit at
 * entry) are not counted. psc_timing_get returns, per kernel id, the launch
 * count and the total milliseconds, and resets. The V-cycle ids count the
 * V-cycle-only forms exactly (on a learned step the V-cycle is skipped).
 * Kernel ids: 0 outer SpMV (+p.q), 1 CG update (+||r||^2), 2 level-0
 * pre-smoothing + residual, 3 level-0 restriction, 4 level-0 prolongation +
 * post-smoothing (+r.z), 5 direction update, 6 whole V-cycle.
 */
#define PSC_TIMING_KERNELS 8
int psc_timing_enable(psc_hier* h, int32_t on);
int psc_timing_get(psc_hier* h, int64_t* counts, double* total_ms);

/*
 * Tuning. PSC_TUNE_GRID_MAX caps the number of workgroups of the streaming
 * kernels (multiple of 8, at most 131072; default 131072; invalidates captured
 * graphs). PSC_TUNE_FUSED_PCG (default 1) selects the fused CG / FCG(1)
 * iteration (V-cycle-only forms): the direction update and the (deferred)
 * x update ride in the SpMV pass, the residual update rides in the level-0
 * pre-smoothing pass; 0 selects the one-kernel-per-operation sequence. Both
 * give the same iterates up to rounding. PSC_TUNE_UNROLL4 (default 0): the FP64 post-smoothing and fused
 * update kernels gather a 7-point row in two batches of four slots (fewer
 * registers, more waves) instead of one batch of eight.
 */
#define PSC_TUNE_GRID_MAX 1
#define PSC_TUNE_FUSED_PCG 2
#define PSC_TUNE_UNROLL4 3
/* PSC_TUNE_BUFLOAD: which hacked-ELL kernels read the matrix and gather
 * vectors through buffer descriptors (32-bit offsets, fewer registers):
 * 0 none, 1 all, 2 (default) the prolongation + post-smoothing kernel. */
#define PSC_TUNE_BUFLOAD 4
/* PSC_TUNE_SPMV2 (default 0): the plain SpMV and the restriction process two
 * slices per wavefront concurrently. */
#define PSC_TUNE_SPMV2 5
/* PSC_TUNE_SPLIT (default 1; must stay 1 for smoothed prolongators or more
 * than one smoothing sweep, else PSC_ERR_ARG): the smoothing sweeps use two operators stored
 * at build, A M^-1 (pre-smoothing r = b - A M^-1 b, one gathered vector) and
 * the smoothed prolongator S P = (I - M^-1 A) P (post-smoothing with
 * prolongation, x = M^-1 (b + r) + S P x_c), the same sweeps up to rounding;
 * 0 gathers through A, M^-1, P and the aggregate map instead. The BUFLOAD
 * and UNROLL4 keys select among the gathering kernels only. */
#define PSC_TUNE_SPLIT 6
/* PSC_TUNE_DIA (default 1): kernels that support it read a level operator
 * (and A M^-1) from its hacked-DIA copy, which the build keeps for a level
 * when its diagonal slots are at most 4/3 of its ELL slots (7-point
 * stencils: 8 bytes per entry instead of 12); 0 reads hacked ELL. */
#define PSC_TUNE_DIA 7
/* PSC_TUNE_TAIL (default: automatic, up to 1024 rows with one smoothing sweep
 * per level and 4096 with more, and only levels whose sweep reads at most
 * 512 KB of operators): the levels with at most `value` rows (value <= 4096),
 * down to the dense coarsest solve, run in one kernel of one workgroup per V-cycle
 * (l1-Jacobi sweeps on the split operators; dense or PCG coarsest), whose
 * vectors are held in LDS (16 bytes per row, 24 with several sweeps, within
 * the device's LDS per workgroup: the largest such levels are left out until
 * they fit); 0 launches their kernels one by one. */
#define PSC_TUNE_TAIL 8
/* PSC_TUNE_DIA_UNIFORM (default 1): a level whose hacked-DIA copy has at most 8
 * distinct diagonals over the whole matrix stores every slice with all of them
 * and passes the offsets in the kernel argument (no per-slice metadata load);
 * 0 reads the per-slice offset arrays instead (same values and results). */
#define PSC_TUNE_DIA_UNIFORM 9
/* PSC_TUNE_XCD (default 0): 1 makes the streaming kernels give each
 * accelerator die a contiguous chunk of the work (workgroups are dealt to the
 * 8 dies round robin); 0 lets workgroups take the work in launch order, which
 * measured faster (all dies share the neighbour gathers through the Infinity
 * Cache). This setting is per device and applies to every handle on it. */
#define PSC_TUNE_XCD 10
/* PSC_TUNE_MIXED_SPLIT (default 1): in the FP32-V-cycle FCG iteration, the
 * residual update r -= alpha q (with an FP32 copy of r) and the level-0 FP32
 * pre-smoothing residual run as two passes, the second gathering the FP32 copy;
 * 0 fuses them, recomputing r at every gathered neighbour from FP64 r and q.
 * Same values either way. */
#define PSC_TUNE_MIXED_SPLIT 11
/* PSC_TUNE_FP64_SPLIT (default 1): the same two passes with the FP64 V-cycle
 * (r -= alpha q, then the level-0 pre-smoothing residual gathering r); 0 fuses
 * them into one pass that recomputes r at every gathered neighbour. Same
 * values either way. */
#define PSC_TUNE_FP64_SPLIT 12
/* PSC_TUNE_DIA_ALIGN (default 1): a level read from a paired uniform hacked-DIA
 * copy (which gets at least one 128-row block per wavefront in any case) whose
 * largest diagonal offset is a multiple of 8 x 128 rows (the plane of a 3D
 * stencil) gets a grid whose blocks per workgroup divide that offset over 8,
 * so the rows a plane away are swept by a workgroup on the same accelerator
 * die (workgroups are dealt to the 8 dies round robin) and its gathers hit
 * that die's L2; 0 skips that choice. The reductions' partial sums are added
 * in a fixed order either way; their grouping follows the grid, so results
 * agree up to rounding. */
#define PSC_TUNE_DIA_ALIGN 13
/* PSC_TUNE_CAPPED (default 1): a level without a hacked-DIA copy, with at
 * least capped_min_rows rows, whose row lengths vary so widely that its
 * hacked-ELL slices are mostly padding (a few long rows in most 64-row
 * slices, as on the stalled coarse levels of strongly varying coefficients)
 * is read, by the kernels that take it (smoothing sweeps, residuals, the
 * l1-Jacobi coarsest solve, psc_spmv), from a copy whose slices keep at most
 * a cap of slots per row, the rest of each longer row in an overflow that one
 * wavefront sums with a segmented scan; the build keeps that copy when it
 * costs at most 0.9 of the plain layout's wavefront loads. 0 reads the plain
 * hacked ELL. Same values up to rounding (overflow entries are summed in scan
 * order). */
#define PSC_TUNE_CAPPED 14
/* PSC_TUNE_PAIR_R (default 1): on a level whose rows 2k and 2k+1 always share
 * an aggregate and a prolongator value (Poisson's 2x2x1 aggregates of the
 * first levels) and whose one pre-smoothing sweep reads the paired uniform
 * hacked-DIA layout, that sweep also writes the pair sums r_2k + r_2k+1 and
 * the restriction reads them with one entry per pair (Section "Multigrid
 * preconditioners": b_c = P^T r, summed over pairs first): half the vector
 * and half the index and value bytes of R. 0 restricts r itself. Same values
 * up to rounding. */
#define PSC_TUNE_PAIR_R 15
/* PSC_TUNE_MIXED_Z32 (default 1): the mixed forms (FCG(1) with the FP32
 * V-cycle, l1-Jacobi split smoother) keep the V-cycle's output z in FP32, the
 * precision it is computed in: the level-0 post-smoothing writes 4 bytes per
 * row instead of 8 and the next outer pass gathers them and widens them
 * exactly (the same values bit for bit). In the learned form with the FP32
 * V-cycle, a network step's z (from BF16 activations) is rounded to FP32 for
 * the outer pass; its acceptance test reads the FP64 z. 0 keeps z in FP64. */
#define PSC_TUNE_MIXED_Z32 16
int psc_tune(psc_hier* h, int32_t key, int32_t value);

void psc_hier_free(psc_hier* h);

/* ---- learned preconditioner ---------------------------------------------- */
/*
 * A 3-layer 3x3x3 convolutional network with C = 16 channels:
 *   h1 = GELU(W1 * u + b1), h2 = GELU(W2 * h1 + b2), out = W3 * h2 + b3,
 * zero padding, GELU(t) = t Phi(t). Inputs and activations are bfloat16,
 * convolution sums are FP32 (MFMA for the 16 -> 16 layer); weights are kept
 * as an FP32 master copy and a bfloat16 working copy.
 * Parameter layout (psc_net_param_count() = 7809 floats):
 *   W1[16][1][27] b1[16] W2[16][16][27] b2[16] W3[1][16][27] b3[1],
 * tap t = (dz*3+dy)*3+dx acting at offset (dz-1, dy-1, dx-1).
 */
int32_t psc_net_param_count(void);
int psc_net_create(const float* params_host, void* hip_stream, psc_net** out);
int psc_net_get_params(const psc_net* net, float* params_host);
int psc_net_set_params(psc_net* net, const float* params_host);

/* z = s net(r/s), s = ||r||_2/sqrt(n), on an nx x ny x nz grid (x fastest). */
int psc_net_apply(psc_net* net, const double* r_dev, double* z_dev, int32_t nx,
                  int32_t ny, int32_t nz);

/*
 * psc_net_apply without any device allocation, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). Same result as psc_net_apply (the same
 * kernels); its scratch (the norm reduction, 8.5 KB, and with the unfused
 * kernels of psc_net_tune the activations, 66 bytes per cell) lives in a
 * fixed array of about 17.3 MB that every device the library runs on holds
 * until the process ends. Grids above
 * PSC_NET_NOALLOC_MAX_CELLS cells (64^3) return PSC_ERR_ARG. The handle's own
 * grid buffers are neither used nor changed. All calls on one device share
 * that array: calls that overlap on one device (several host threads, or
 * several streams) race and give wrong results; serialise them.
 */
#define PSC_NET_NOALLOC_MAX_CELLS 262144
int psc_net_apply_noalloc(psc_net* net, const double* r_dev, double* z_dev, int32_t nx,
                          int32_t ny, int32_t nz);

/*
 * The comparison arm of the learned form: a network handle whose "network"
 * is one l1-Jacobi sweep from zero on the finest level, z = M_0^-1 r with
 * M_0 = diag(a_ii + sum_{j != i} |a_ij|) (Section "GPU enabled smoothers"),
 * taken in psc_fcg_solve's schedule exactly where the network would be (same
 * z.r > 0 test, fallback and switch-off rules). The handle copies M_0^-1 from
 * h (h may be freed afterwards) and acts on vectors of h's size only;
 * psc_net_apply and psc_net_apply_noalloc give z = M_0^-1 r; calls that need
 * weights (get/set params, training, save) return PSC_ERR_STATE. Release with
 * psc_net_free. Errors: PSC_ERR_ARG (NULL), PSC_ERR_STATE (h holds no
 * finest-level diagonal), PSC_ERR_OOM, PSC_ERR_HIP.
 */
int psc_net_create_l1jacobi(const psc_hier* h, void* hip_stream, psc_net** out);

/* Declare the grid used by psc_fcg_solve (n = nx*ny*nz). */
int psc_net_set_grid(psc_net* net, int32_t nx, int32_t ny, int32_t nz);

/*
 * Inference kernels of psc_net_apply, psc_net_apply_noalloc and the network
 * steps of psc_fcg_solve. PSC_NET_TUNE_FUSED (default 1): one kernel computes
 * the three layers, walking 16 x 16 columns of the grid plane by plane with
 * the activations in LDS (16 bytes of HBM traffic per cell: r in, z out;
 * every layer on MFMA, the third as 27 tap projections of each cell summed
 * over its neighbours); 0: one kernel per layer with bfloat16 activation
 * fields in device memory (66 bytes per cell, allocated by psc_net_set_grid).
 * The two agree up to FP32 summation order, which can move a bfloat16
 * rounding of an activation. Without layers (the l1-Jacobi alternate) the
 * call does nothing. Errors: PSC_ERR_ARG (NULL handle, unknown key),
 * PSC_ERR_OOM, PSC_ERR_HIP.
 */
#define PSC_NET_TUNE_FUSED 1
int psc_net_tune(psc_net* net, int32_t key, int32_t value);

/*
 * Batched forward / loss-gradient on B cubic crops of side D (float, device):
 *   in_dev, target_dev, out_dev: B*D^3 floats.
 * psc_net_loss_grad: loss = mean over samples and cells at least `margin`
 * from every face of (out - target)^2; grad_host receives d loss / d params
 * (7809 floats), computed by the backward kernels (bfloat16 rounding
 * treated as identity). Returns the loss in *loss.
 */
int psc_net_forward_batch(psc_net* net, const float* in_dev, float* out_dev, int32_t B,
                          int32_t D);
int psc_net_loss_grad(psc_net* net, const float* in_dev, const float* target_dev,
                      int32_t B, int32_t D, int32_t margin, float* loss, float* grad_host);

/*
 * Collect training pairs from preconditioned CG runs: runs PCG on b_dev and,
 * after every iteration k, crops `crops_per_iter` cubes of side `crop` at
 * the corners origins_host[(k*crops_per_iter + c)*3 + {0,1,2}] = (z,y,x)
 * from (r_k / s_k, z_k / s_k) with z_k = B r_k and s_k = ||r_k||/sqrt(n),
 * appending them as floats to r_out_dev / z_out_dev (capacity crops).
 * n_origins: number of origin triples provided. *count is in/out: the
 * number of crops already stored, advanced by the crops added.
 */
int psc_pairs_collect(psc_hier* h, const double* b_dev, int32_t nx, int32_t ny, int32_t nz,
                      double rtol, int32_t maxit, int32_t crop, int32_t crops_per_iter,
                      const int32_t* origins_host, int32_t n_origins, float* r_out_dev,
                      float* z_out_dev, int32_t capacity, int32_t* count);

/*
 * Train with Adam (FP32 master weights, bfloat16 working copy refreshed
 * after each step) on stored crops: step s uses the `batch` crops
 * order_host[s*batch .. s*batch+batch-1]. Loss as psc_net_loss_grad.
 * losses_host (steps floats, may be NULL) receives each step's loss.
 */
int psc_net_train(psc_net* net, const float* r_dev, const float* z_dev, int32_t ncrops,
                  int32_t crop, int32_t margin, const int32_t* order_host, int32_t steps,
                  int32_t batch, float lr, float beta1, float beta2, float eps,
                  float* losses_host);

/*
 * Checkpoint / resume of a network (the caller owns `path`; the files are the
 * caller's). The file is little-endian: a 40-byte header
 *   char magic[8] = "PSCNET01"; uint32 header_bytes = 40, nparams = 7809,
 *   channels = 16, ksize = 3, flags (bit 0: Adam moments follow), reserved;
 *   int64 adam_t (optimiser steps taken)
 * then nparams FP32 master weights in the layout above, then (flag bit 0)
 * the first and second Adam moment vectors, nparams floats each.
 * psc_net_save writes the current master weights and Adam state (waits for
 * the network's pending work first). psc_net_load creates a new handle
 * bound to `hip_stream` with those weights (the bfloat16 working copy is
 * derived from them) and restores the Adam state, so psc_net_train resumes
 * where the saved run stopped. Errors: PSC_ERR_ARG (NULL), PSC_ERR_IO
 * (open/read/write failure, bad magic, a header that does not match this
 * network, a truncated file or trailing bytes), PSC_ERR_HIP / PSC_ERR_OOM
 * from the device; on error *out is NULL and no handle is leaked.
 */
int psc_net_save(const psc_net* net, const char* path);
int psc_net_load(const char* path, void* hip_stream, psc_net** out);

void psc_net_free(psc_net* net);

const char* psc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* PSC_H */
