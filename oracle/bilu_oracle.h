/*
 * Block incomplete LU (BILU) -- plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, sequential reference
 * that the GPU library is checked against.  Only the test suite, the smoke
 * check and the benchmark's CPU-baseline leg may load it.  It shares no code
 * with the GPU library.
 *
 * It follows Bollhoefer, Schenk and Verbosio, "High Performance Block
 * Incomplete LU Factorization" (arXiv 1908.10169):
 *   - Sec. 2.1, Alg. 1   Crout ILU (the scalar special case),
 *   - Sec. 2.2           Crout-type block ILU, A ~ L D^{-1} U,
 *   - Sec. 3.2           cosine-based blocking with the mu+2sigma filter,
 *   - Sec. 3.3           compression + symmetric reordering (the ordering is
 *                        an input here: natural, or a caller permutation),
 *   - Sec. 3.4           simplified ILU(1,tau) guess of the initial blocks,
 *   - Sec. 3.5           progressive aggregation,
 *   - Sec. 3.6           perturbation of singular diagonal blocks,
 *   - Sec. 3.7           the preconditioner composition,
 * plus restarted flexible GMRES (Saad 1993) as the Krylov driver.
 *
 * Conventions: CSR input with sorted, unique column indices, 0-based.
 * Stored factors, per block K with rows first..last (width q):
 *   R_K  sorted scalar rows  > last kept in block column K of L,
 *   L_K  |R_K| x q  row-major, unit-scaled:  L(i,K) = C(i,K) * D_K,
 *   C_K  sorted scalar cols  > last kept in block row K of U,
 *   W_K  q x |C_K|  column-major, unscaled block row (U(K,:) = D_K W_K),
 *   D_K  q x q row-major, the inverse of the pivot block S_K.
 * so that the permuted matrix satisfies  A ~ L S U  with L, U unit block
 * triangular and S = blockdiag(D_K^{-1}).
 */
#ifndef BILU_ORACLE_H
#define BILU_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int use_cosine;       /* Sec. 3.2 initial blocking                        */
  int use_ilu1t;        /* Sec. 3.4 ILU(1,tau) block growth                 */
  int use_aggregation;  /* Sec. 3.5 progressive aggregation                 */
  int max_block;        /* cap on any block width                           */
  double tau;           /* drop tolerance                                   */
  double cos_eps;       /* cosine threshold (0.8 -> integer test 5ov^2>=4nn)*/
  double pert_tau;      /* Sec. 3.6 absolute perturbation tolerance        */
  double pert_rho;      /* Sec. 3.6 relative perturbation tolerance        */
  double pivot_eps;     /* relative pivot size that triggers perturbation   */
  int beta_one;         /* reading of the undefined beta_j: 0 -> delta_j, 1 -> 1 */
  int drop_norm;        /* 0 = max-abs (inf) norm, 1 = Euclidean norm       */
  int sym_perturb;      /* Sec. 5: a failed inversion perturbs each column's */
                        /* selected entry and its mirror together (symmetric */
                        /* pivot blocks stay symmetric)                      */
} orc_options;

void orc_default_options(orc_options* o);

typedef struct orc_handle orc_handle;

orc_handle* orc_create(void);
void orc_destroy(orc_handle* h);

/* Full pipeline: optional caller pre-permutation (new->old, may be NULL),
 * cosine blocking, natural order of the groups, ILU(1,tau) guess, Crout
 * sweep with dropping, perturbation and aggregation.  Returns 0 on success,
 * 1 when a block stayed singular, -1 on invalid input. */
int orc_run(orc_handle* h, int64_t n, const int64_t* rowptr,
            const int32_t* colind, const double* val, const int64_t* pre_perm,
            const orc_options* opt);
/* orc_run with units (Sec. 5, the symmetric variant): the pre-permuted
 * index range splits into nunits contiguous units [unit_starts[u],
 * unit_starts[u+1]) (1x1 and 2x2 pivots of the symmetric matching) that no
 * group splits; the cosine test runs on the compressed companion matrix
 * (a unit's row is the union of its rows, columns replaced by their units)
 * and a group holds at most max_block scalars.  Both scalars of a 2x2
 * pivot take the pivot block's largest magnitude in place of |a_kk| in
 * the ILU(1,tau) thresholds.  partner (n entries in the final numbering,
 * the other scalar of each 2x2 pivot or -1; may be NULL) names the 2x2
 * pivots when the units are coarser (groups given by the caller); NULL:
 * the units of two scalars.  unit_starts NULL: orc_run. */
int orc_run_units(orc_handle* h, int64_t n, const int64_t* rowptr,
                  const int32_t* colind, const double* val, const int64_t* pre_perm,
                  int64_t nunits, const int64_t* unit_starts, const int64_t* partner,
                  const orc_options* opt);

/* Same, but with a caller-given block partition of the permuted matrix
 * (starts[0]=0 < ... < starts[nblocks]=n); cosine and ILU(1,tau) skipped. */
int orc_run_partition(orc_handle* h, int64_t n, const int64_t* rowptr,
                      const int32_t* colind, const double* val,
                      const int64_t* perm, int64_t nblocks,
                      const int64_t* starts, const orc_options* opt);

/* --- individual preprocessing steps (for pins) ----------------------- */
/* Sec. 3.2: cosine groups of the matrix; perm (new->old) lists groups in
 * seed order, members ascending; group_starts has ngroups+1 entries.     */
int64_t orc_cosine(int64_t n, const int64_t* rowptr, const int32_t* colind,
                   double cos_eps, int max_block, int64_t* perm,
                   int64_t* group_starts, int64_t* n_ignored);
/* Sec. 3.4: ILU(1,tau) growth over units; returns the number of blocks.  */
int64_t orc_ilu1t(int64_t n, const int64_t* rowptr, const int32_t* colind,
                  const double* val, int64_t nunits, const int64_t* unit_starts,
                  double tau, int max_block, int64_t* block_starts);
/* Sec. 3.4: the estimated sets I~_k (rows > k) and J~_k (cols > k).   */
int64_t orc_ilu1t_sets(int64_t n, const int64_t* rowptr, const int32_t* colind,
                       const double* val, int64_t k, double tau, int64_t* I,
                       int64_t* nI, int64_t* J, int64_t* nJ);
/* Sec. 3.6: perturb + invert one dense q x q block (row-major, in place
 * into dinv).  Returns the number of perturbation rounds, -1 if singular. */
int orc_perturb_invert(int q, const double* s, double alpha,
                       const orc_options* opt, double* s_used, double* dinv);

/* --- results ---------------------------------------------------------- */
int64_t orc_n(const orc_handle* h);
int64_t orc_nblocks(const orc_handle* h);          /* final (after merges) */
int64_t orc_nblocks_initial(const orc_handle* h);  /* before merges        */
void orc_get_perm(const orc_handle* h, int64_t* perm);          /* new->old */
void orc_get_starts(const orc_handle* h, int64_t* starts);      /* final    */
void orc_get_starts_initial(const orc_handle* h, int64_t* starts);
void orc_get_group_starts(const orc_handle* h, int64_t* starts, int64_t* ngroups);
/* sizes: nR[K], nC[K] per final block; totals returned through pointers */
void orc_get_counts(const orc_handle* h, int64_t* nR, int64_t* nC);
/* concatenated per final block in block order */
void orc_get_factors(const orc_handle* h, int64_t* R, double* L, int64_t* C,
                     double* W, double* D);
void orc_get_stats(const orc_handle* h, int64_t* out /* 16 */);
/* drop-decision log of the sweep: one entry per candidate row / column
 * with its block, scalar index, kind (0 row of L, 1 column of U), norm
 * and kept flag.  Returns the number of entries (arrays may be NULL). */
int64_t orc_get_droplog(const orc_handle* h, int64_t* block, int64_t* index,
                        int32_t* kind, double* norm, int32_t* kept);
/* merge log: one entry per aggregation test: K, p, q, mu, nu, merged */
int64_t orc_get_mergelog(const orc_handle* h, int64_t* rec /* 6 per entry */);

/* y = M^{-1} x in the original numbering (Sec. 3.7 with D_l=D_r=Pi=I). */
void orc_apply(const orc_handle* h, const double* x, double* y);

typedef struct {
  int64_t iterations;  /* Arnoldi steps (FGMRES), steps (SQMR)            */
  int64_t restarts;    /* cycles started                                   */
  double rel_residual; /* true ||b-Ax||/||b|| at exit                      */
  int converged;
} orc_solve_info;

/* Right-preconditioned FGMRES(restart) on the original matrix. x holds the
 * initial guess on entry. */
void orc_fgmres(const orc_handle* h, const double* b, double* x, int restart,
                double rtol, int maxit, orc_solve_info* info);
/* orc_fgmres that also writes the residual estimate after every Arnoldi
 * step (maxit entries at most) to resid_history (may be NULL). */
void orc_fgmres_hist(const orc_handle* h, const double* b, double* x, int restart,
                     double rtol, int maxit, orc_solve_info* info, double* resid_history);
/* FGMRES with M = I (unpreconditioned), on any CSR matrix. */
void orc_fgmres_plain(int64_t n, const int64_t* rowptr, const int32_t* colind,
                      const double* val, const double* b, double* x,
                      int restart, double rtol, int maxit,
                      orc_solve_info* info, double* resid_history);

/* Simplified QMR (Sec. 5; Freund and Nachtigal 1995) for symmetric A with
 * M from the run as preconditioner.  Stops when the infinity-norm backward
 * error ||b - A x|| / (||A|| ||x|| + ||b||) of the updated QMR residual is
 * <= tol and the true residual confirms it, after maxit steps, or at a
 * breakdown.  info->rel_residual is the true 2-norm relative residual;
 * *eta (may be NULL) the true backward error at exit; tau_history (may be
 * NULL, maxit entries) the quasi-residual norm after every step. */
void orc_sqmr(const orc_handle* h, const double* b, double* x, double tol, int maxit,
              orc_solve_info* info, double* eta, double* tau_history);
/* orc_sqmr with M = I, on any CSR matrix. */
void orc_sqmr_plain(int64_t n, const int64_t* rowptr, const int32_t* colind,
                    const double* val, const double* b, double* x, double tol,
                    int maxit, orc_solve_info* info, double* eta, double* tau_history);

/* ||(L S U - A)_Omega||_F / ||A||_F over the stored positions Omega of the
 * blocks the sweep computed (before merges). */
double orc_kept_residual(const orc_handle* h);
/* The same over the stored positions of the final blocks. */
double orc_final_residual(const orc_handle* h);
/* Refactorization with frozen patterns: val (A's values in its entry
 * order, same pattern) replaces A's values; the final blocks, R_K and C_K
 * stay and L, W, D (and S) are recomputed on them, nothing dropped or
 * merged.  0 on success, 1 singular, -1 invalid. */
int orc_refactor_frozen(orc_handle* h, const double* val);
/* y = (L S U) x in the permuted numbering. */
void orc_lsu_matvec(const orc_handle* h, const double* x, double* y);

/* Test hook of the pins (not part of the method): adds delta to stored value
 * pos of L_K (which 0) or W_K (which 1) of final block k; 0 or -1. */
int orc_plant(orc_handle* h, int which, int64_t k, int64_t pos, double delta);

/* timings of the last run, seconds: analyze, ilu1t, factor */
void orc_get_times(const orc_handle* h, double* t3);

#ifdef __cplusplus
}
#endif
#endif
