// Simplified QMR (Freund and Nachtigal 1995; Freund and Jarre 1997), the
// Krylov solver Sec. 5 pairs with the block incomplete factorization of a
// symmetric matrix.  A is symmetric, M the block ILU from bilu_factor (on
// symmetric data the sweep is symmetric: the columns of U repeat the rows
// of L, so M is symmetric up to rounding, and it may be indefinite).  The
// preconditioner splits as M1 = I, M2 = M: per step one product with A, one
// application of M^{-1}, three dot products.  FP64 throughout, in the
// permuted numbering (permutations preserve inner products and maximum
// norms).
//
// With the symmetric matching (use_mwm = 2) the iteration runs on
// D A D x^ = D b (x = D x^); M stays symmetric.
//
// Stopping test: the normwise backward error of A x = b in the infinity
// norm, eta = ||b - A x|| / (||A|| ||x|| + ||b||), evaluated on the QMR
// residual that the iteration updates (rq -= A d, with A d kept by its own
// recurrence) and confirmed with the true residual; a step whose update
// met the tolerance but whose true residual does not is resumed.  Under
// the scaling, x = D x^ and b - A x = D^{-1} (D b - D A D x^).
//
// As in the FGMRES driver the host queues step k + 1 before it reads
// whether step k - 1 stopped (flags copied to pinned memory); the kernels of
// a step queued behind the stopping one do no work.
#include <chrono>
#include <cmath>

#include "internal.h"

namespace bilu {

namespace {
struct SqGuard {
  bilu_handle* h;
  hipEvent_t ev[2];
  ~SqGuard() {
    h->run_skip = nullptr;
    for (hipEvent_t e : ev)
      if (e) h->ev_pool.push_back(e);
  }
};

double backward_error(double rmax, double anorm, double xmax, double bmax) {
  return rmax == 0.0 ? 0.0 : rmax / (anorm * xmax + bmax);
}
}  // namespace

bilu_status sqmr(bilu_handle* h, const double* b_orig, double* x_orig, double tol, int maxit,
                 bilu_solve_info* info, double* eta_out) {
  using clk = std::chrono::steady_clock;
  const auto t_start = clk::now();
  if (maxit < 0 || !(tol >= 0)) return fail(h, BILU_ERR_INVALID, "bad solver parameters");
  if (h->mwm && !h->mwm_sym)
    return fail(h, BILU_ERR_INVALID,
                "SQMR needs a symmetric preconditioner; the matching's one-sided permutation "
                "and scalings make M nonsymmetric (use_mwm = 2 keeps it symmetric)");
  const int64_t n = h->n;
  hipStream_t st = h->stream;
  // workspace: b, x, r, rq, q, t, u, d, sv, apply temporary
  const int64_t cols = 10;
  if (h->w_cols < cols) {
    if (h->w_vec.alloc((size_t)cols * n) != hipSuccess)
      return fail(h, BILU_ERR_NO_MEMORY, "solver workspace");
    h->w_cols = cols;
  }
  double* b = h->w_vec.p;
  double* x = b + n;
  double* r = x + n;
  double* rq = r + n;
  double* q = rq + n;
  double* t = q + n;
  double* u = t + n;
  double* d = u + n;
  double* sv = d + n;
  double* tmp = sv + n;
  double* red = h->w_red.p;
  hipError_t ae = h->w_gm.alloc(kSqSlots + 2 * kSqParts);
  if (ae == hipSuccess) ae = h->w_flags.alloc(4);
  int* hflags = ae == hipSuccess ? h->w_hflags.get<int>(8, &ae) : nullptr;
  if (ae != hipSuccess || !hflags) return fail(h, BILU_ERR_NO_MEMORY, "solver workspace");
  SqState g{h->w_gm.p, h->w_gm.p + kSqSlots, h->w_flags.p};
  SqGuard guard{h, {h->ev_get(), h->ev_get()}};
  hipEvent_t* ev = guard.ev;
  if (!ev[0] || !ev[1]) return fail(h, BILU_ERR_DEVICE, "solver: events");
  const int* flags = g.flags;
  auto device_error = [&]() { return fail(h, BILU_ERR_DEVICE, "solver: device error"); };
  double hs[kSqSlots];
  auto read_scalars = [&]() {
    return hipMemcpyAsync(hs, g.s, sizeof(hs), hipMemcpyDeviceToHost, st) == hipSuccess &&
           hipStreamSynchronize(st) == hipSuccess;
  };
  // the scales between the iterated and A's own vectors (NULL: none)
  const double* rscale = h->sl_inv();  // b - A x = rscale .* (b^ - A^ x^)
  const double* xscale = h->sr();      // x = xscale .* x^
  // true residual b^ - A^ x^ into t; the maxima of A's residual and of x,
  // and the 2-norm of A's residual (formed in tmp, free outside applies)
  auto true_residual = [&]() {
    h->run_skip = nullptr;
    spmv_permuted(h, x, t);
    launch_sub(st, n, b, t, t);
    const double* ro = t;
    if (rscale) {
      launch_mul(st, n, rscale, t, tmp);
      ro = tmp;
    }
    launch_amax(st, n, ro, nullptr, red, g.s + kSqRmax);
    launch_amax(st, n, x, xscale, red, g.s + kSqXmax);
    launch_dot(st, n, ro, ro, red, g.s + kSqRR);
  };

  launch_gather(st, n, h->d_perm.p, h->sl(), b_orig, b);
  launch_gather(st, n, h->perm_col(), h->sr_inv(), x_orig, x);
  launch_row_amax(st, n, h->d_rp.p, h->d_ci.p, h->d_rv.p, h->sl_inv(), h->sr_inv(), red,
                  g.s + kSqAnorm);
  launch_amax(st, n, b_orig, nullptr, red, g.s + kSqBmax);
  launch_dot(st, n, b_orig, b_orig, red, g.s + kSqEta);  // ||b||^2, read once below
  true_residual();
  if (!read_scalars()) return device_error();
  const double anorm = hs[kSqAnorm], bmax = hs[kSqBmax], bnorm = std::sqrt(hs[kSqEta]);
  double resid2 = hs[kSqRR];
  double eta = backward_error(hs[kSqRmax], anorm, hs[kSqXmax], bmax);
  int64_t steps = 0;
  int converged = eta <= tol ? 1 : 0;
  if (!converged && maxit > 0) {
    // r = rq = b^ - A^ x^ (in t), q = M^{-1} r, rho = r^T q, tau = ||r||
    if (hipMemcpyAsync(r, t, n * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(rq, t, n * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemsetAsync(d, 0, n * sizeof(double), st) != hipSuccess ||
        hipMemsetAsync(sv, 0, n * sizeof(double), st) != hipSuccess)
      return device_error();
    bilu_status s0 = apply_permuted(h, r, q, tmp);
    if (s0 != BILU_OK) return s0;
    launch_dot(st, n, r, q, red, g.s + kSqRhoNew);
    launch_dot(st, n, r, r, red, g.s + kSqRR);  // the iterated residual's norm
    launch_sq_init(st, g);
    // the second half of a step: u = M^{-1} r, rho_new = r^T u, q = u + beta q
    auto tail = [&]() -> bilu_status {
      bilu_status s = apply_permuted(h, r, u, tmp);
      if (s != BILU_OK) return s;
      launch_dot(st, n, r, u, red, g.s + kSqRhoNew, flags);
      launch_sq_direction(st, n, g, u, q);
      return BILU_OK;
    };
    bool resume = false;
    while (true) {
      h->run_skip = flags;
      if (resume) {
        launch_sq_resume(st, g);
        bilu_status s = tail();
        if (s != BILU_OK) return s;
      }
      for (int64_t j = 0;; ++j) {
        spmv_permuted(h, q, t);
        launch_dot(st, n, q, t, red, g.s + kSqSigma, flags);
        launch_sq_alpha(st, g);
        launch_axpy(st, n, g.s + kSqAlpha, -1.0, t, r, flags);
        launch_dot(st, n, r, r, red, g.s + kSqRR, flags);
        launch_sq_theta(st, g);
        launch_sq_update(st, n, g, q, t, d, sv, x, rq, xscale, rscale, tol, maxit);
        bilu_status s = tail();
        if (s != BILU_OK) return s;
        int* hf = hflags + 4 * (j & 1);
        if (hipMemcpyAsync(hf, g.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
            hipEventRecord(ev[j & 1], st) != hipSuccess)
          return device_error();
        if (j > 0) {
          if (hipEventSynchronize(ev[(j - 1) & 1]) != hipSuccess) return device_error();
          if (hflags[4 * ((j - 1) & 1)]) break;
        }
      }
      h->run_skip = nullptr;
      int fl[4];
      if (hipMemcpyAsync(fl, g.flags, sizeof(fl), hipMemcpyDeviceToHost, st) != hipSuccess ||
          !read_scalars())
        return device_error();
      steps = fl[2];
      const double rho = hs[kSqRho];
      if (fl[1] != 1) break;  // breakdown or maxit
      true_residual();
      if (!read_scalars()) return device_error();
      if (backward_error(hs[kSqRmax], anorm, hs[kSqXmax], bmax) <= tol) {
        converged = 1;
        break;
      }
      if (steps >= maxit || rho == 0.0) break;
      resume = true;
    }
    true_residual();
    if (!read_scalars()) return device_error();
    resid2 = hs[kSqRR];
    eta = backward_error(hs[kSqRmax], anorm, hs[kSqXmax], bmax);
  }
  // x is written back only when a step changed it (the round trip through
  // the scaling could move its last bits)
  if (steps > 0) launch_scatter(st, n, h->perm_col(), h->sr(), x, x_orig);
  if (hipStreamSynchronize(st) != hipSuccess) return device_error();
  int64_t faults = 0;
  if (apply_faults(h, &faults) != BILU_OK) return BILU_ERR_DEVICE;
  if (info) {
    info->iterations = steps;
    info->restarts = 0;
    info->rel_residual = bnorm > 0 ? std::sqrt(resid2) / bnorm : 0.0;
    info->converged = converged;
    info->seconds = std::chrono::duration<double>(clk::now() - t_start).count();
  }
  if (eta_out) *eta_out = eta;
  return converged ? BILU_OK : BILU_WARN_NOT_CONVERGED;
}

}  // namespace bilu
