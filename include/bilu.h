/*
 * bilu.h -- block incomplete LU (BILU) on one AMD Instinct MI355X (gfx950).
 *
 * Method: Bollhoefer, Schenk and Verbosio, "High Performance Block
 * Incomplete LU Factorization" (arXiv 1908.10169).  The library computes the
 * Crout-type block ILU of Sec. 2.2 on a permuted matrix
 *
 *      P^T A P  ~  L S U,   L, U^T unit block lower triangular,
 *                           S block diagonal, D_K = S_K^{-1} stored,
 *
 * with the initial blocking of Sec. 3.2 (cosine) and Sec. 3.4 (ILU(1,tau)),
 * the symmetric reordering of Sec. 3.3, the perturbation of Sec. 3.6 and the
 * progressive aggregation of Sec. 3.5, and uses it as the preconditioner
 * M = P L S U P^T of Sec. 3.7 (no scaling/matching: D_l = D_r = Pi = I)
 * inside flexible GMRES.
 *
 * Conventions
 *  - 0-based CSR: rowptr int64[n+1], colind int32[nnz] strictly increasing
 *    within each row, val double[nnz] finite.
 *  - Host arrays are borrowed for the duration of a call and copied.
 *  - Device arrays are plain HIP device pointers owned by the caller;
 *    work is enqueued on the handle's stream (the stream given at create;
 *    NULL = the default stream) and calls that return results to the host
 *    synchronize that stream.
 *  - Every entry point returns a bilu_status; no C++ exception, abort or
 *    exit crosses this boundary.  bilu_last_error() gives a message.
 *  - A handle is not thread-safe.
 */
#ifndef BILU_H
#define BILU_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BILU_OK = 0,
  BILU_WARN_PERTURBED = 1,      /* factor succeeded, some pivot blocks perturbed */
  BILU_WARN_NOT_CONVERGED = 2,  /* solver stopped at maxit above rtol           */
  BILU_ERR_INVALID = -1,        /* bad argument or malformed CSR                 */
  BILU_ERR_NO_MEMORY = -2,      /* device or host allocation, or a capacity cap  */
  BILU_ERR_STATE = -3,          /* call order: analyze before factor before apply */
  BILU_ERR_SINGULAR = -4,       /* a pivot block stayed singular after perturbing */
  BILU_ERR_DEVICE = -5,         /* HIP runtime error or kernel-reported fault     */
  BILU_ERR_INTERNAL = -6
} bilu_status;

/* Sec. 3.3 ordering of the compressed graph: nested dissection by recursive
 * level-structure bisection, none (the caller's order), or multilevel nested
 * dissection (heavy-edge coarsening, greedy growing, Fiduccia-Mattheyses
 * refinement, minimum vertex cover separators; slower, smaller separators) */
typedef enum {
  BILU_ORDER_ND = 0,
  BILU_ORDER_NATURAL = 1,
  BILU_ORDER_ND_MULTILEVEL = 2
} bilu_ordering;
typedef enum { BILU_PREC_F64 = 0, BILU_PREC_F32 = 1, BILU_PREC_BF16 = 2 } bilu_precision;
typedef enum { BILU_NORM_INF = 0, BILU_NORM_TWO = 1 } bilu_drop_norm;

typedef struct {
  int use_cosine;        /* Sec. 3.2 initial blocking (default 1)                     */
  int use_ilu1t;         /* Sec. 3.4 ILU(1,tau) block growth (default 1)              */
  int use_aggregation;   /* Sec. 3.5 progressive aggregation (default 1)              */
  int max_block;         /* cap on block widths, 1..128 (default 128)                 */
  double cos_eps;        /* cosine threshold (default 0.8)                            */
  int ordering;          /* bilu_ordering of the compressed graph (default ND)        */
  const int64_t* pre_perm; /* optional host permutation new->old applied to A before  */
                         /* the cosine step (NULL = identity); read during analyze    */
  int drop_norm;         /* bilu_drop_norm of the scaled block rows/columns (INF)     */
  double perturb_tau;    /* Sec. 3.6 absolute tolerance (default 1e-2)                */
  double perturb_rho;    /* Sec. 3.6 relative tolerance (default 1e-1)                */
  double pivot_eps;      /* pivot |u_jj| <= pivot_eps*max|S| triggers perturbation    */
  int beta_one;          /* 0: beta_j = max|column j| (default); 1: beta_j = 1        */
  int update_precision;  /* bilu_precision of the Schur-complement products (F64),   */
                         /* also the precision L and W are stored in; pivot blocks,  */
                         /* drop norms and the solver stay FP64                      */
  size_t heap_bytes;     /* factor heap size; 0 = sized from nnz(A).  A heap that    */
                         /* proves too small grows and the sweep runs again          */
                         /* (counted in bilu_stats.heap_regrows)                     */
  int collect_timing;    /* 1: time kernels with HIP events on the handle's stream;  */
                         /* 2: also trace every block of the factor kernel           */
  int factor_path;       /* 0 (default): blocks up to 16 wide stage their data in    */
                         /* LDS, or in global scratch when it does not fit; others  */
                         /* take the general path.  1: every block takes the general */
                         /* path.  2: global staging wherever it fits.  All three   */
                         /* compute identical bits                                   */
  int apply_path;        /* 0 (default): the apply runs as one dataflow launch, one  */
                         /* wave per block, blocks taken in workgroup-index order   */
                         /* (no workgroup has to be resident); a wait that times    */
                         /* out is counted in apply_faults and reported as          */
                         /* BILU_ERR_DEVICE by the next bilu_sync or                */
                         /* bilu_fgmres_solve.  1: one launch per dependency level. */
                         /* 2: as 0, blocks taken in the order workgroups draw a    */
                         /* ticket when they start (no assumption on start order;  */
                         /* slower).  All compute identical bits                     */
  int use_mwm;           /* 1: Sec. 3.1 first: the handle factors D_l A D_r Pi     */
                         /* (bilu_mwm) instead of A; apply, spmv and fgmres still   */
                         /* act on A in its own numbering (default 0).              */
                         /* 2: Sec. 5, eq. (smwm), for symmetric A: the symmetric  */
                         /* matching; the handle factors D A D (d_i = sqrt(dl_i    */
                         /* dr_i) from bilu_mwm) with the matching's 1x1 and 2x2   */
                         /* pivots kept whole by the cosine groups, which form on  */
                         /* the compressed companion matrix (a pivot's row is the  */
                         /* union of its rows, columns replaced by their pivots),  */
                         /* listed along pre_perm; M stays symmetric.  Both route  */
                         /* the analysis through the host                           */
  int analyze_path;      /* 0 (default): bilu_analyze checks the entries, searches  */
                         /* the cosine candidates and builds P A P^T on the device  */
                         /* (the host keeps the limits, the greedy replay and the   */
                         /* ordering); 1: all on the host.  Both give the same      */
                         /* permutation, groups and matrix bit for bit.  nnz >= 2^31 */
                         /* takes the host path                                      */
  int apply_precision;   /* bilu_precision the apply reads L and W in: F64 (default) */
                         /* or F32 (an FP32 copy made after the factorization).     */
                         /* With FP32 or BF16 updates, L and W are stored in that   */
                         /* precision and the apply reads them as stored; D and the */
                         /* vectors are FP64 in every form                           */
  int update_mfma;       /* 1: the Schur-update terms of blocks up to 16 wide are  */
                         /* computed as 16x16 matrix-core tiles (FP64 16x16x4, FP32 */
                         /* 16x16x4 or BF16 16x16x16 with FP32 accumulation); 0     */
                         /* (default): scalar fused multiply-adds, which measure    */
                         /* faster on narrow blocks.  Both give the same patterns   */
                         /* up to rounding of the products                           */
  int deterministic;     /* 1 (default): every run gives the same bits: the update   */
                         /* terms of a block are materialized and subtracted in     */
                         /* predecessor order.  0: blocks up to 16 wide subtract     */
                         /* each term as it is computed, with atomic adds (faster;  */
                         /* results vary at rounding level between runs, patterns   */
                         /* only where a drop norm is within rounding of tau).      */
                         /* update_mfma = 1 implies 1                                */
  double drop_log_margin; /* > 0: log every drop decision whose norm is within      */
                         /* drop_log_margin * tau of tau (block, row i or column ~j, */
                         /* norm), for replaying ambiguous decisions; exported by  */
                         /* bilu_export_factors.  0 (default): no log               */
  int workers_per_cu;    /* workgroups of the factor sweep per compute unit: 0       */
                         /* (default) as many as fit (two), or 1                     */
  int use_tuning;        /* 1 (default): a table loaded with bilu_load_tuning that  */
                         /* has an entry for the update precision, block-width     */
                         /* class and deterministic setting of a factorization     */
                         /* supplies those of workers_per_cu, update_mfma,         */
                         /* factor_path and apply_path left at 0 (and, for         */
                         /* deterministic = 0, the order of accumulation); 0: the  */
                         /* options as given                                         */
} bilu_options;

typedef struct bilu_handle bilu_handle;

typedef struct {
  int64_t iterations;    /* Arnoldi steps (FGMRES) or steps (SQMR) taken              */
  int64_t restarts;      /* restart cycles started                                    */
  double rel_residual;   /* true ||b - A x||_2 / ||b||_2 at exit                      */
  double seconds;        /* wall time of the call                                     */
  int converged;
} bilu_solve_info;

typedef struct {
  int64_t n, nnz_a;
  int64_t ngroups;            /* cosine groups                                        */
  int64_t nblocks_initial;    /* blocks after ILU(1,tau), before aggregation         */
  int64_t nblocks;            /* final blocks                                         */
  int64_t max_width;
  double avg_width, std_width;
  int64_t nnz_l, nnz_w, nnz_d;/* stored factor entries                               */
  int64_t merges, perturbed_blocks;
  int64_t factor_levels;      /* longest chain of possible updaters in the sweep     */
  int64_t apply_levels_fwd, apply_levels_bwd;
  double flops_update;        /* counted Schur-update flops (2 m p q per product)    */
  double bytes_apply;         /* algorithmic bytes of one preconditioner apply        */
  double t_analyze, t_ilu1t, t_factor_device, t_aggregate, t_factor;  /* seconds   */
  /* with collect_timing: device time (HIP events) of the factor kernels of
   * the last bilu_factor, and of all applies / products since it */
  double dev_ms_factor, dev_ms_apply, dev_ms_spmv;
  int64_t n_factor_launches, n_apply, n_spmv;
  double bytes_factor;        /* algorithmic bytes of the factor kernels             */
  /* host wall time of the phases of the last bilu_factor (seconds):
   * [0] ILU(1,tau) sets, [1] ILU(1,tau) block growth, [2] factor launch
   * preparation, [3] factor kernel to completion, [4] aggregation, [5] apply
   * plan, [6] final statistics, [7] unused */
  double t_phase[8];
  int64_t apply_faults;       /* dataflow applies whose dependency wait timed out     */
                              /* since analyze (0 unless the device misbehaves)       */
  int64_t heap_regrows;       /* sweeps of the last factor rerun with a larger heap   */
  double r_kept;              /* ||(L S U - A)_Omega||_F / ||A||_F of the last factor,  */
                              /* from bilu_kept_residual (-1 until it is called)      */
  /* drop decisions of the last sweep (Alg. 1 in block form: a candidate block
   * row (column) is dropped when its scaled norm is <= tau) */
  int64_t drops_rows, drops_cols;
  double drop_margin_min;     /* smallest |norm - tau| / tau over all decisions      */
                              /* (-1 when tau = 0 or no candidate was tested)         */
  int64_t drop_log_count;     /* decisions within drop_log_margin of tau (logged      */
                              /* up to 2^20, exported with the factors)               */
  int64_t tuning_applied;     /* 1 when a tuned entry set the last factorization's    */
                              /* kernel settings                                       */
  int64_t max_width_initial;  /* widest block of the initial partition                */
  int64_t ilu1t_host;         /* 1 when the ILU(1,tau) partition of the last          */
                              /* factorization came from the host computation (a      */
                              /* device kernel capacity was exceeded), else 0         */
} bilu_stats;

/* Library-allocated host copy of the factors (for checking), final blocks. */
typedef struct {
  int64_t n, nblocks, nblocks_initial;
  int64_t* perm;           /* [n] new -> old                                         */
  int64_t* starts;         /* [nblocks+1]                                            */
  int64_t* starts_initial; /* [nblocks_initial+1]                                    */
  int64_t* group_starts;   /* [ngroups+1] cosine groups in the permuted numbering    */
  int64_t ngroups;
  int64_t* r_ptr;          /* [nblocks+1] offsets into r_idx                         */
  int32_t* r_idx;          /* rows of L per block, ascending                         */
  int64_t* c_ptr;          /* [nblocks+1]                                            */
  int32_t* c_idx;          /* columns of U per block, ascending                      */
  double* l_val;           /* per block |R_K| x q row-major, blocks concatenated     */
  double* w_val;           /* per block q x |C_K| column-major                       */
  double* d_val;           /* per block q x q row-major                              */
  /* the drop-decision log of the sweep (drop_log_margin > 0), in the order
   * the decisions were taken: initial block, candidate (row i, or ~j for
   * column j, permuted numbering) and the scaled norm compared with tau */
  int64_t ndrop_log;
  int64_t* drop_block;
  int64_t* drop_index;
  double* drop_norm;
} bilu_factors_host;

/* Defaults: the paper's constants (Sec. 3.2, 3.4-3.6). */
void bilu_default_options(bilu_options* opt);

/* Create a handle.  opt may be NULL (defaults).  hip_stream is a hipStream_t
 * (NULL = default stream).  Returns BILU_ERR_INVALID on bad options. */
bilu_status bilu_create(bilu_handle** h, const bilu_options* opt, void* hip_stream);

/* Sec. 3.2-3.3 (preprocessing steps 2-3 of Sec. 3.7): validate the CSR,
 * cosine-group the rows, compress, order the compressed graph, expand the
 * permutation, and keep the permuted matrix (CSR and CSC) in device memory.
 * Host arrays (rowptr n+1 entries, colind and val rowptr[n] each), read
 * during the call only.  With analyze_path = 0 the matrix is copied to the
 * device first and the entry checks, the cosine search and the permutation
 * run there.  Synchronous.  Errors: BILU_ERR_INVALID (n <= 0,
 * unsorted/duplicate/out-of-range column, non-finite value, bad pre_perm),
 * BILU_ERR_NO_MEMORY, BILU_ERR_DEVICE. */
bilu_status bilu_analyze(bilu_handle* h, int64_t n, const int64_t* rowptr,
                         const int32_t* colind, const double* val);

/* bilu_analyze for a matrix already in device memory (Sec. 3.2-3.3, as
 * bilu_analyze): rowptr (n+1), colind and val (rowptr[n] entries each) are
 * device arrays owned by the caller, read during the call only.  rowptr is
 * copied to the host and checked there before any entry is read; the entries
 * are checked on the device.  With use_mwm = 1 or 2, analyze_path = 1 or
 * nnz >= 2^31 the matrix is copied to the host and analyzed as by
 * bilu_analyze.  The handle ends as bilu_analyze would leave it, bit for bit.
 * Same errors as bilu_analyze, plus BILU_ERR_DEVICE.  Synchronous. */
bilu_status bilu_analyze_device(bilu_handle* h, int64_t n, const int64_t* rowptr,
                                const int32_t* colind, const double* val);

/* Sec. 3.4-3.6 and Sec. 2.2: guess the initial blocks with ILU(1,tau), run
 * the block Crout sweep on the GPU with drop tolerance tau >= 0 (tau = 0
 * drops only exactly-zero rows/columns), perturb singular pivot blocks, and
 * aggregate blocks progressively.  May be called again with another tau.
 * Returns BILU_OK, BILU_WARN_PERTURBED, BILU_ERR_SINGULAR, BILU_ERR_STATE
 * (no analyze), BILU_ERR_NO_MEMORY, BILU_ERR_DEVICE.  Synchronous. */
bilu_status bilu_factor(bilu_handle* h, double tau);

/* Numeric refactorization for a sequence of matrices with one pattern
 * (the paper's time-step matrices, Sec. 4): val (device array, rowptr[n]
 * doubles in the entry order of the matrix given to bilu_analyze) replaces
 * A's values; the block Crout sweep of Sec. 2.2 (dropping with tau,
 * perturbation, aggregation) runs again on the initial blocks of the last
 * bilu_factor, without the cosine step, the ordering or ILU(1,tau).  The
 * result is what the sweep gives on that partition, so it equals the last
 * factor bit for bit when val holds the same values and tau is the same.
 * Errors: BILU_ERR_STATE before bilu_factor, BILU_ERR_INVALID (non-finite
 * value: nothing changes; use_mwm; nnz >= 2^31), and those of bilu_factor.
 * Synchronous. */
bilu_status bilu_refactor(bilu_handle* h, double tau, const double* val);

/* Numeric refactorization with frozen patterns, for the same sequences:
 * val (as for bilu_refactor) replaces A's values and the last factor's
 * values are recomputed on its own blocks (after aggregation), row lists
 * R_K, column lists C_K and storage: the Crout panels of Sec. 2.2 restricted
 * to the stored positions (updates L_J W_J only where both ends are
 * stored), the pivot blocks inverted with the perturbation of Sec. 3.6,
 * L_K = C(R_K, K) D_K and W_K = C(K, C_K).  Nothing is dropped or merged,
 * so the apply plan is kept; (L S U)_Omega = A_Omega holds on the stored
 * positions Omega for the new values.  All blocks run in one launch,
 * ordered by dependency level, each after its predecessors (a bounded wait;
 * BILU_ERR_DEVICE when it times out).  bilu_kept_residual afterwards:
 * BILU_ERR_STATE when the
 * last factor had merged blocks (its sweep's positions are no longer the
 * factor's).  Errors: BILU_ERR_STATE before bilu_factor, BILU_ERR_INVALID
 * (non-finite value: nothing changes; use_mwm; nnz >= 2^31),
 * BILU_ERR_SINGULAR, BILU_ERR_DEVICE; BILU_WARN_PERTURBED when pivot blocks
 * were perturbed.  Synchronous. */
bilu_status bilu_refactor_frozen(bilu_handle* h, const double* val);

/* Factor count independent analyzed handles in one launch of the factor
 * sweep (many matrices at once).  hs[i] is factored with drop tolerance
 * taus[i]; every handle ends as bilu_factor(hs[i], taus[i]) would leave it,
 * with the same factor bit for bit.  The handles must be distinct, on the
 * same device, and agree in drop_norm, beta_one, perturb_tau, perturb_rho,
 * pivot_eps, update_precision, update_mfma, deterministic and factor_path
 * (BILU_ERR_INVALID
 * otherwise); blocking and aggregation options may differ.  The launch runs
 * on hs[0]'s stream.  The device counters of the launch (flops_update, the
 * update part of bytes_factor, dev_ms_factor, factor_levels) describe the
 * whole batch in every handle's statistics.  Returns the first error, else
 * BILU_WARN_PERTURBED if any handle perturbed a pivot block, else BILU_OK;
 * errors of the common launch are reported on hs[0].  Synchronous. */
bilu_status bilu_factor_batched(bilu_handle** hs, int count, const double* taus);

/* Sec. 3.7: y = M^{-1} x = P (L S U)^{-1} P^T x, multiplying by D_K
 * (Sec. 2.2).  x, y: device arrays of n doubles in the original numbering,
 * x != y.  Asynchronous on the handle's stream.  BILU_ERR_STATE before a
 * successful factor. */
bilu_status bilu_apply(bilu_handle* h, const double* x, double* y);

/* bilu_apply for callers that cannot allocate device memory (code under
 * stream capture, serving loops, harnesses that forbid allocation): the
 * same arguments, result and bits as bilu_apply, but its three work vectors
 * (n doubles each) live in a fixed 48 MiB array per device that the library
 * holds until the process ends, instead of the handle's workspace; it calls
 * no allocator.  n is limited to 2^21 = 2,097,152 unknowns
 * (BILU_ERR_INVALID beyond, with a message).  Every call on one device
 * shares that device's array: calls that overlap on one device (other
 * streams, other handles, other threads) race and must be serialized by the
 * caller.  Asynchronous on the handle's stream; HIP event timing is not
 * recorded for it. */
bilu_status bilu_apply_noalloc(bilu_handle* h, const double* x, double* y);

/* Wait for the handle's stream; BILU_ERR_DEVICE if the runtime reports an
 * error left by asynchronous calls (bilu_apply, bilu_spmv), or if a
 * dataflow apply since the last check timed out in a dependency wait (its
 * output is then invalid; counted in bilu_stats.apply_faults). */
bilu_status bilu_sync(bilu_handle* h);

/* y = A x with the analyzed matrix (original numbering), device arrays. */
bilu_status bilu_spmv(bilu_handle* h, const double* x, double* y);

/* Right-preconditioned restarted flexible GMRES(restart) for A x = b with M
 * from bilu_factor.  b, x: device arrays (original numbering); x holds the
 * initial guess on entry and the solution on exit.  Stops when the
 * residual estimate reaches rtol*||b|| and the true residual confirms it,
 * or after maxit Arnoldi steps.  info (host, may be NULL) receives counts
 * and the true relative residual.  Returns BILU_OK or
 * BILU_WARN_NOT_CONVERGED.  Synchronous. */
bilu_status bilu_fgmres_solve(bilu_handle* h, const double* b, double* x, int restart,
                              double rtol, int maxit, bilu_solve_info* info);

/* Simplified QMR (Sec. 5, the solver used there with the symmetric block
 * factorization; Freund and Nachtigal 1995) for a symmetric A, with M from
 * bilu_factor as preconditioner.  On symmetric data the factorization is
 * symmetric (the kept columns of U are the transposed kept rows of L), so M
 * is symmetric up to rounding; it may be indefinite.  b, x: device arrays
 * (original numbering); x holds the initial guess on entry and the
 * solution on exit.  Stops when the normwise backward error in the
 * infinity norm, ||b - A x|| / (||A|| ||x|| + ||b||), of the updated QMR
 * residual is <= tol and the true residual confirms it, after maxit steps,
 * or at a breakdown (q^T A q = 0 or r^T M^{-1} r = 0).  info (host, may be
 * NULL): steps in iterations, restarts 0, the true 2-norm relative
 * residual; *backward_error (host, may be NULL): the true backward error at
 * exit.  With use_mwm = 2 the iteration runs on D A D x^ = D b, x = D x^,
 * and the stopping test stays on A x = b.  BILU_ERR_INVALID when the
 * handle uses the nonsymmetric matching (use_mwm = 1: its one-sided
 * permutation and scalings make M nonsymmetric) or for tol < 0,
 * maxit < 0.  Returns BILU_OK or BILU_WARN_NOT_CONVERGED.  Synchronous. */
bilu_status bilu_sqmr_solve(bilu_handle* h, const double* b, double* x, double tol, int maxit,
                            bilu_solve_info* info, double* backward_error);

/* Host-only structural preprocessing (no GPU is touched): the cosine
 * groups (Sec. 3.2), the ordering of the compressed graph (Sec. 3.3) and the
 * ILU(1,tau) initial partition (Sec. 3.4) that bilu_analyze + bilu_factor
 * would use (with use_mwm = 2 also the symmetric matching, on D A D; the
 * nonsymmetric matching, use_mwm = 1, is not applied here).  perm (n
 * entries, new -> old), group_starts (n+1 entries) and block_starts (n+1
 * entries) are caller-allocated host arrays; *ngroups and *nblocks receive
 * the counts.  Same errors as bilu_analyze. */
bilu_status bilu_preprocess(const bilu_options* opt, int64_t n, const int64_t* rowptr,
                            const int32_t* colind, const double* val, double tau,
                            int64_t* perm, int64_t* group_starts, int64_t* ngroups,
                            int64_t* block_starts, int64_t* nblocks);

/* Sec. 3.1, eq. (mwm): maximum weight matching (a maximum product
 * transversal) of the n x n CSR matrix A and the diagonal scalings with
 * which D_l A D_r Pi has |entries| <= 1 and unit diagonal magnitudes.
 * Host-only (no handle, no GPU).  rowptr [n+1], colind [nnz] (0-based,
 * any order within a row), val [nnz]; caller-allocated outputs: sigma [n]
 * (the column matched to row i, i.e. Pi[sigma(i), i] = 1, so column i of
 * A Pi is column sigma(i) of A), dl [n] and dr [n] (the diagonals of D_l,
 * D_r).  Entries equal to zero do not count.  BILU_ERR_SINGULAR when A has
 * no perfect matching on its nonzero entries (or an empty row or column),
 * BILU_ERR_INVALID on bad arguments. */
bilu_status bilu_mwm(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* val,
                     int64_t* sigma, double* dl, double* dr);

/* Kept-pattern residual of the last factorization (Sec. 2.2: the Crout step
 * reproduces A exactly on the stored positions):
 *   *r_kept = ||(L S U - A)_Omega||_F / ||A||_F,
 * Omega = the diagonal blocks, R_K x K and K x C_K of the sweep's factor
 * (before aggregation), computed on the device in FP64 from the stored L, W
 * (in their storage precision) and S_K.  Rounding level in the FP64 form;
 * it measures the precision of the stored factor and of the updates in the
 * mixed forms, and perturbed pivot blocks.  Also kept in
 * bilu_stats.r_kept.  BILU_ERR_STATE before a factorization.  Synchronous. */
bilu_status bilu_kept_residual(bilu_handle* h, double* r_kept);

/* Load the tuning table written by the project's tuner
 * (paper_1908_10169_amd/tune.py): a JSON object whose "entries" array holds
 * flat objects with the integer fields precision (bilu_precision),
 * width_class (0: the widest initial block is at most 16 columns, 1: wider),
 * reproducible (1: for handles with deterministic = 1, 0: for the others),
 * workers_per_cu, update_mfma, factor_path, apply_path and deterministic
 * (which must be 1 where reproducible is 1).
 * Process-wide; replaces any table loaded before; path NULL or "" clears it.
 * Without an explicit call, the table shipped beside the library for the
 * device's architecture (tuning/<gfx...>.json next to libbilu.so) is loaded
 * at the first factorization, if present.  Handles with use_tuning = 1 use
 * the entry that matches each factorization.  BILU_ERR_INVALID if the file cannot be read or a field is
 * out of range (the table is then unchanged). */
bilu_status bilu_load_tuning(const char* path);
/* Entries in the loaded tuning table. */
int64_t bilu_tuning_entries(void);

/* Statistics of the last analyze/factor (block sizes as in the paper's
 * tables of Sec. 3.2-3.5: number, max, average, standard deviation). */
bilu_status bilu_get_stats(const bilu_handle* h, bilu_stats* st);

/* Host copies of permutation, partition and factors; free with
 * bilu_free_factors. */
bilu_status bilu_export_factors(const bilu_handle* h, bilu_factors_host* out);
void bilu_free_factors(bilu_factors_host* f);

/* Per-block trace of the last factor kernel (collect_timing = 2): 24 values
 * per initial block in block order, device wall-clock ticks: pushed to the
 * ready queue, taken by a worker, its possible-update set built, candidates
 * built, done; then the block whose retraction made it ready (0 for blocks
 * ready at the start), the count that retraction removed, and the worker;
 * fields 8..15 time the end of the column panel, row panel, pivot, drop
 * norms, heap allocation, factor writes, list pushes and successor counts;
 * fields 16..19 are the numbers of column and row predecessors and of
 * candidate rows and columns; fields 20..23 (narrow blocks only) time the
 * end of the list offsets, of the list staging, of the position searches
 * and candidate compaction, and of the candidate sort.  out may be NULL to
 * query *nrecords; capacity counts uint64 values.  BILU_ERR_STATE without a
 * trace. */
bilu_status bilu_export_trace(const bilu_handle* h, uint64_t* out, int64_t capacity,
                              int64_t* nrecords, double* ticks_per_second);

void bilu_destroy(bilu_handle* h);
const char* bilu_status_string(bilu_status s);
const char* bilu_last_error(const bilu_handle* h);

#ifdef __cplusplus
}
#endif
#endif /* BILU_H */
