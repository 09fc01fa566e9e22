// Restarted flexible GMRES (Saad, SIAM J. Sci. Comput. 14, 1993) with the
// block ILU as right preconditioner, FP64 throughout.  Vectors, the
// (m+1) x m Hessenberg matrix, its Givens rotations, the residual estimate
// and the small triangular solve all live on the GPU.  Orthogonalization
// is modified Gram-Schmidt.  The iteration runs in the permuted numbering
// (permutations preserve norms and inner products), so neither the apply
// nor the product permutes vectors.
//
// The host enqueues Arnoldi step j + 1 before it reads whether step j
// ended the cycle (a flag copied to pinned memory), so the GPU never waits
// for the host inside a cycle; once a step has set the flag, the kernels of
// the step queued behind it do no work.  The host synchronizes with the
// stream once per cycle, for the residual of the restart.
#include <chrono>
#include <cmath>

#include "internal.h"

namespace bilu {

namespace {
// On every exit from the solve: clears the solver's skip flag and returns
// the step events to the handle's pool.
struct SolveGuard {
  bilu_handle* h;
  hipEvent_t ev[2];
  ~SolveGuard() {
    h->run_skip = nullptr;
    for (hipEvent_t e : ev)
      if (e) h->ev_pool.push_back(e);
  }
};
}  // namespace

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
  double* red = h->w_red.p;  // dot partials
  // device state: H, cs, sn, g, y, the step's dot products (m + 3), 1/h(j+1,j)
  const size_t gm_len = (size_t)(m + 1) * m + 2 * (size_t)m + (m + 1) + m + (m + 3) + 1;
  hipError_t ae = h->w_gm.alloc(gm_len);
  if (ae == hipSuccess) ae = h->w_flags.alloc(4);
  int* hflags = ae == hipSuccess ? h->w_hflags.get<int>(8, &ae) : nullptr;
  if (ae != hipSuccess || !hflags) return fail(h, BILU_ERR_NO_MEMORY, "solver workspace");
  GmState gs{};
  gs.H = h->w_gm.p;
  gs.cs = gs.H + (size_t)(m + 1) * m;
  gs.sn = gs.cs + m;
  gs.g = gs.sn + m;
  gs.y = gs.g + (m + 1);
  double* hcol = gs.y + m;
  gs.hcol = hcol;
  gs.inv_hn = hcol + (m + 3);
  gs.flags = h->w_flags.p;
  SolveGuard guard{h, {h->ev_get(), h->ev_get()}};
  hipEvent_t* ev = guard.ev;
  if (!ev[0] || !ev[1]) return fail(h, BILU_ERR_DEVICE, "solver: events");

  // b in A's row space, x in its column space (with use_mwm the iteration
  // runs on the scaled system; the stopping test uses A's own residual)
  launch_gather(st, n, h->d_perm.p, h->sl(), b_orig, b);
  launch_gather(st, n, h->perm_col(), h->sr_inv(), x_orig, x);
  auto norm = [&](const double* v, double* slot, const int* skip) {
    launch_dot(st, n, v, v, red, slot, skip);
  };
  // 2-norm of the residual of A x = b behind the permuted one (tmp is free
  // outside the applies)
  auto true_norm = [&](const double* v, double* slot) {
    if (h->sl_inv()) {
      launch_mul(st, n, h->sl_inv(), v, tmp);
      norm(tmp, slot, nullptr);
    } else {
      norm(v, slot, nullptr);
    }
  };
  double hbuf[2];
  norm(b, hcol, nullptr);
  true_norm(b, hcol + 1);
  if (hipMemcpyAsync(hbuf, hcol, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return fail(h, BILU_ERR_DEVICE, "solver: device error");
  const double bnorm = std::sqrt(hbuf[1]);
  const double target = rtol * bnorm;
  const double target_inner = rtol * std::sqrt(hbuf[0]);  // same as target without use_mwm

  int64_t it = 0, cycles = 0;
  int converged = 0;
  double resid = 0.0;
  while (true) {
    h->run_skip = nullptr;
    spmv_permuted(h, x, r);
    launch_sub(st, n, b, r, r);
    norm(r, hcol, nullptr);
    true_norm(r, hcol + 1);
    if (hipMemcpyAsync(hbuf, hcol, 2 * sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
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
    launch_gm_init(st, gs, m, beta);
    // the cycle's steps; each runs only while the flag is clear
    h->run_skip = gs.flags;
    for (int j = 0; j < m; ++j) {
      bilu_status s = apply_permuted(h, V(j), Z(j), tmp);
      if (s != BILU_OK) return s;
      spmv_permuted(h, Z(j), w);
      norm(w, hcol + m + 1, gs.flags);  // ||A z_j|| before orthogonalization
      for (int i = 0; i <= j; ++i) {
        launch_dot(st, n, w, V(i), red, hcol + i, gs.flags);
        launch_axpy(st, n, hcol + i, -1.0, V(i), w, gs.flags);
      }
      norm(w, hcol + j + 1, gs.flags);
      launch_gm_update(st, gs, j, m, target_inner, it, maxit);
      launch_scale_dev(st, n, gs.inv_hn, w, V(j + 1), gs.flags);  // unused after the last step
      int* hf = hflags + 4 * (j & 1);
      if (hipMemcpyAsync(hf, gs.flags, 4 * sizeof(int), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipEventRecord(ev[j & 1], st) != hipSuccess)
        return fail(h, BILU_ERR_DEVICE, "solver: device error");
      // step j + 1 is queued behind step j before the host looks at step j - 1
      if (j > 0) {
        if (hipEventSynchronize(ev[(j - 1) & 1]) != hipSuccess)
          return fail(h, BILU_ERR_DEVICE, "solver: device error");
        if (hflags[4 * ((j - 1) & 1)]) break;
      }
    }
    launch_gm_solve(st, gs, m);
    h->run_skip = nullptr;
    int fl[4];
    if (hipMemcpyAsync(fl, gs.flags, sizeof(fl), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return fail(h, BILU_ERR_DEVICE, "solver: device error");
    const int jend = fl[1];
    it += jend;
    for (int i = 0; i < jend; ++i) launch_axpy(st, n, gs.y + i, 1.0, Z(i), x);
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
