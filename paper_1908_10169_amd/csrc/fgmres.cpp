// Restarted flexible GMRES (Saad, SIAM J. Sci. Comput. 14, 1993) with the
// block ILU as right preconditioner, FP64 throughout.  Vectors live on the
// GPU; the (m+1) x m Hessenberg matrix, its Givens rotations and the small
// triangular solve stay on the host, which reads one column of H per
// Arnoldi step.  Orthogonalization is modified Gram-Schmidt.  The iteration
// runs in the permuted numbering (permutations preserve norms and inner
// products), so neither the apply nor the product permutes vectors.
#include <chrono>
#include <cmath>

#include "internal.h"

namespace bilu {

bilu_status fgmres(bilu_handle* h, const double* b_orig, double* x_orig, int m, double rtol,
                   int maxit, bilu_solve_info* info) {
  using clk = std::chrono::steady_clock;
  const auto t_start = clk::now();
  if (m < 1 || maxit < 0 || !(rtol >= 0)) return fail(h, BILU_ERR_INVALID, "bad solver parameters");
  const int64_t n = h->n;
  hipStream_t st = h->stream;
  // workspace: V (m+1), Z (m), w, r, b, x, apply temporary (permuted numbering)
  const int64_t cols = 2 * (int64_t)m + 6;
  if (h->w_cols < cols) {
    if (h->w_vec.alloc((size_t)cols * n) != hipSuccess)
      return fail(h, BILU_ERR_NO_MEMORY, "solver workspace");
    h->w_cols = cols;
  }
  double* base = h->w_vec.p;
  auto V = [&](int j) { return base + (int64_t)j * n; };
  auto Z = [&](int j) { return base + (int64_t)(m + 1 + j) * n; };
  double* w = base + (int64_t)(2 * m + 1) * n;
  double* r = w + n;
  double* b = r + n;
  double* x = b + n;
  double* tmp = x + n;  // apply intermediate
  double* red = h->w_red.p;          // dot partials
  DevArray<double> hcol;             // device column of H: m+3 scalars
  if (hcol.alloc(m + 3) != hipSuccess) return fail(h, BILU_ERR_NO_MEMORY, "solver workspace");

  // b in A's row space, x in its column space (with use_mwm the iteration
  // runs on the scaled system; the stopping test uses A's own residual)
  launch_gather(st, n, h->d_perm.p, h->sl(), b_orig, b);
  launch_gather(st, n, h->perm_col(), h->sr_inv(), x_orig, x);
  auto norm = [&](const double* v, double* slot) {
    launch_dot(st, n, v, v, red, slot);
  };
  // 2-norm of the residual of A x = b behind the permuted one (tmp is free
  // outside the applies)
  auto true_norm = [&](const double* v, double* slot) {
    if (h->sl_inv()) {
      launch_mul(st, n, h->sl_inv(), v, tmp);
      norm(tmp, slot);
    } else {
      norm(v, slot);
    }
  };
  double hbuf[2];
  norm(b, hcol.p);
  true_norm(b, hcol.p + 1);
  if (hipMemcpyAsync(hbuf, hcol.p, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(h, BILU_ERR_DEVICE, "solver: device error");
  const double bnorm = std::sqrt(hbuf[1]);
  const double target = rtol * bnorm;
  const double target_inner = rtol * std::sqrt(hbuf[0]);  // same as target without use_mwm

  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), col(m + 3);
  int64_t it = 0, cycles = 0;
  int converged = 0;
  double resid = 0.0;
  while (true) {
    spmv_permuted(h, x, r);
    launch_sub(st, n, b, r, r);
    norm(r, hcol.p);
    true_norm(r, hcol.p + 1);
    if (hipMemcpyAsync(hbuf, hcol.p, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(h, BILU_ERR_DEVICE, "solver: device error");
    const double beta = std::sqrt(hbuf[0]);
    resid = std::sqrt(hbuf[1]);
    if (resid <= target) {
      converged = 1;
      break;
    }
    if (it >= maxit) break;
    ++cycles;
    launch_scale(st, n, 1.0 / beta, r, V(0));
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      bilu_status s = apply_permuted(h, V(j), Z(j), tmp);
      if (s != BILU_OK) return s;
      spmv_permuted(h, Z(j), w);
      norm(w, hcol.p + m + 1);  // ||A z_j|| before orthogonalization
      for (int i = 0; i <= j; ++i) {
        launch_dot(st, n, w, V(i), red, hcol.p + i);
        launch_axpy(st, n, hcol.p + i, -1.0, V(i), w);
      }
      norm(w, hcol.p + j + 1);
      if (hipMemcpyAsync(col.data(), hcol.p, (m + 3) * sizeof(double), hipMemcpyDeviceToHost, st) !=
              hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess)
        return fail(h, BILU_ERR_DEVICE, "solver: device error");
      const double hn = std::sqrt(col[j + 1]);
      const double wn0 = std::sqrt(col[m + 1]);
      for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = col[i];
      H[(size_t)(j + 1) * m + j] = hn;
      ++it;
      for (int i = 0; i < j; ++i) {
        const double a0 = H[(size_t)i * m + j], a1 = H[(size_t)(i + 1) * m + j];
        H[(size_t)i * m + j] = cs[i] * a0 + sn[i] * a1;
        H[(size_t)(i + 1) * m + j] = -sn[i] * a0 + cs[i] * a1;
      }
      const double hjj = H[(size_t)j * m + j], hj1 = H[(size_t)(j + 1) * m + j];
      if (hj1 == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else if (std::fabs(hj1) > std::fabs(hjj)) {
        const double t = hjj / hj1;
        sn[j] = 1.0 / std::sqrt(1.0 + t * t);
        cs[j] = sn[j] * t;
      } else {
        const double t = hj1 / hjj;
        cs[j] = 1.0 / std::sqrt(1.0 + t * t);
        sn[j] = cs[j] * t;
      }
      H[(size_t)j * m + j] = cs[j] * hjj + sn[j] * hj1;
      H[(size_t)(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      const double est = std::fabs(g[j + 1]);
      const bool breakdown = hn <= 1e-14 * wn0;
      if (!breakdown) launch_scale(st, n, 1.0 / hn, w, V(j + 1));
      jend = j + 1;
      if (est <= target_inner || breakdown || it >= maxit) break;
    }
    for (int i = jend - 1; i >= 0; --i) {
      double acc = g[i];
      for (int k = i + 1; k < jend; ++k) acc -= H[(size_t)i * m + k] * y[k];
      y[i] = acc / H[(size_t)i * m + i];
    }
    for (int i = 0; i < jend; ++i) launch_axpy_host(st, n, y[i], Z(i), x);
  }
  launch_scatter(st, n, h->perm_col(), h->sr(), x, x_orig);
  if (hipStreamSynchronize(st) != hipSuccess) return fail(h, BILU_ERR_DEVICE, "solver: device error");
  int64_t faults = 0;
  if (apply_faults(h, &faults) != BILU_OK) return BILU_ERR_DEVICE;
  if (info) {
    info->iterations = it;
    info->restarts = cycles;
    info->rel_residual = bnorm > 0 ? resid / bnorm : 0.0;
    info->converged = converged;
    info->seconds = std::chrono::duration<double>(clk::now() - t_start).count();
  }
  return converged ? BILU_OK : BILU_WARN_NOT_CONVERGED;
}

}  // namespace bilu
