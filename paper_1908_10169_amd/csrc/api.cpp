// C ABI of the BILU library (declared in include/bilu.h).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <exception>
#include <new>

#include "internal.h"

namespace bilu {

bilu_status fail(bilu_handle* h, bilu_status s, const std::string& msg) {
  if (h) h->err = msg;
  return s;
}

bilu_status hip_check(bilu_handle* h, hipError_t e, const char* what) {
  std::string msg = std::string(what) + ": " + hipGetErrorString(e);
  if (e == hipErrorOutOfMemory) return fail(h, BILU_ERR_NO_MEMORY, msg);
  return fail(h, BILU_ERR_DEVICE, msg);
}

}  // namespace bilu

hipEvent_t bilu_handle::ev_get() {
  if (!ev_pool.empty()) {
    hipEvent_t e = ev_pool.back();
    ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

void bilu_handle::ev_resolve() {
  if (ev_pending.empty()) return;
  (void)hipStreamSynchronize(stream);
  for (const EventPair& p : ev_pending) {
    float ms = 0.f;
    if (p.a && p.b && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
      if (p.kind == 0) stats.dev_ms_factor += ms;
      if (p.kind == 1) { stats.dev_ms_apply += ms; stats.n_apply++; }
      if (p.kind == 2) { stats.dev_ms_spmv += ms; stats.n_spmv++; }
    }
    if (p.a) ev_pool.push_back(p.a);
    if (p.b) ev_pool.push_back(p.b);
  }
  ev_pending.clear();
}

bilu_handle::~bilu_handle() {
  for (const EventPair& p : ev_pending) {
    if (p.a) (void)hipEventDestroy(p.a);
    if (p.b) (void)hipEventDestroy(p.b);
  }
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
}

using namespace bilu;

#define GUARD_BEGIN try {
#define GUARD_END                                                         \
  }                                                                       \
  catch (const std::bad_alloc&) {                                         \
    return fail(h, BILU_ERR_NO_MEMORY, "host allocation failed");        \
  }                                                                       \
  catch (const std::exception& ex) {                                      \
    return fail(h, BILU_ERR_INTERNAL, ex.what());                        \
  }                                                                       \
  catch (...) {                                                           \
    return fail(h, BILU_ERR_INTERNAL, "unknown exception");              \
  }

namespace bilu {

// After the sweep: the sweep's factor becomes the handle's, then
// aggregation (Sec. 3.5), the apply plan and the statistics.
bilu_status finish_factor(bilu_handle* h, std::chrono::steady_clock::time_point t0) {
  bilu_status s = BILU_OK;
  h->kept_stale = false;
  h->frozen.ready = false;  // a new factor: the frozen schedule is rebuilt on demand
  h->stats.r_kept = -1.0;  // computed on request (bilu_kept_residual)
  h->nb = h->stats.nblocks_initial;
  h->bstart = h->bstart0;
  h->fv = FactorView{};
  h->fv.nb = (int)h->nb;
  h->fv.bstart = h->d_bstart.p;
  h->fv.blockOf = h->d_blockof.p;
  h->fv.nr = h->d_nr.p;
  h->fv.nc = h->d_nc.p;
  h->fv.roff = h->d_roff.p;
  h->fv.coff = h->d_coff.p;
  h->fv.loff = h->d_loff.p;
  h->fv.woff = h->d_woff.p;
  h->fv.doff = h->d_doff.p;
  h->fv.idx = h->d_idx_heap.p;
  h->fv.val = h->d_val_heap.p;
  h->fv.vprec = h->opt.update_precision;
  h->fv.dval = h->d_dval.p;
  h->f_val_len = h->val_used;
  auto t1 = std::chrono::steady_clock::now();
  if (h->opt.use_aggregation) {
    s = aggregate_device(h);
    if (s != BILU_OK) return s;
  }
  auto t2 = std::chrono::steady_clock::now();
  h->stats.t_aggregate = std::chrono::duration<double>(t2 - t1).count();
  h->stats.t_phase[4] = h->stats.t_aggregate;
  s = build_apply_plan(h);
  if (s != BILU_OK) return s;
  auto t3 = std::chrono::steady_clock::now();
  h->stats.t_phase[5] = std::chrono::duration<double>(t3 - t2).count();
  // block statistics and stored entries of the final factor
  {
    const int64_t nb = h->nb;
    std::vector<int32_t> nr(nb), nc(nb);
    if (hipMemcpy(nr.data(), h->fv.nr, nb * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(nc.data(), h->fv.nc, nb * 4, hipMemcpyDeviceToHost) != hipSuccess)
      return fail(h, BILU_ERR_DEVICE, "stats copy");
    double sum = 0, sum2 = 0;
    int64_t mx = 0, nl = 0, nw = 0, nd = 0, ir = 0, ic = 0;
    for (int64_t b = 0; b < nb; ++b) {
      int64_t q = h->bstart[b + 1] - h->bstart[b];
      sum += q;
      sum2 += double(q) * q;
      mx = std::max(mx, q);
      nl += nr[b] * q;
      nw += nc[b] * q;
      nd += q * q;
      ir += nr[b];
      ic += nc[b];
    }
    h->stats.nblocks = nb;
    h->stats.max_width = mx;
    h->stats.avg_width = sum / nb;
    h->stats.std_width = std::sqrt(std::max(0.0, sum2 / nb - (sum / nb) * (sum / nb)));
    h->stats.nnz_l = nl;
    h->stats.nnz_w = nw;
    h->stats.nnz_d = nd;
    // one apply reads every stored value and row/column index once and
    // moves six vectors of n doubles: x and y across the boundary, their
    // permuted copies, and t (written, then read)
    h->stats.bytes_apply = 8.0 * double(nl + nw + nd) + 4.0 * double(ir + ic) + 48.0 * h->n;
    // factor: A once (value + index), the L_J/W_J reads of the updates, the
    // written factors and their indices
    h->stats.bytes_factor += 12.0 * double(h->nnz) + 8.0 * double(nl + nw + nd) +
                             4.0 * double(ir + ic);
  }
  {
    auto t4 = std::chrono::steady_clock::now();
    h->stats.t_phase[6] = std::chrono::duration<double>(t4 - t3).count();
    h->stats.t_factor = std::chrono::duration<double>(t4 - t0).count();
  }
  h->state = 2;
  return h->stats.perturbed_blocks > 0 ? BILU_WARN_PERTURBED : BILU_OK;
}

}  // namespace bilu

namespace {

bool rowptr_monotone(int64_t n, const int64_t* rp) {
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) return false;
  return true;
}

void analyze_done(bilu_handle* h, std::chrono::steady_clock::time_point t0) {
  h->stats = bilu_stats{};
  h->stats.n = h->n;
  h->stats.nnz_a = h->nnz;
  h->stats.ngroups = (int64_t)h->group_starts.size() - 1;
  h->stats.t_analyze = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  h->state = 1;
}

}  // namespace

extern "C" {

void bilu_default_options(bilu_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->use_cosine = 1;
  o->use_ilu1t = 1;
  o->use_aggregation = 1;
  o->max_block = 128;
  o->cos_eps = 0.8;
  o->ordering = BILU_ORDER_ND;
  o->pre_perm = nullptr;
  o->drop_norm = BILU_NORM_INF;
  o->perturb_tau = 1e-2;
  o->perturb_rho = 1e-1;
  o->pivot_eps = 1e-12;
  o->beta_one = 0;
  o->update_precision = BILU_PREC_F64;
  o->heap_bytes = 0;
  o->deterministic = 1;
  o->workers_per_cu = 0;
  o->use_tuning = 1;
}

bilu_status bilu_create(bilu_handle** out, const bilu_options* opt, void* stream) {
  if (!out) return BILU_ERR_INVALID;
  *out = nullptr;
  bilu_handle* h = nullptr;
  try {
    h = new bilu_handle();
  } catch (...) {
    return BILU_ERR_NO_MEMORY;
  }
  if (opt)
    h->opt = *opt;
  else
    bilu_default_options(&h->opt);
  if (h->opt.max_block < 1 || h->opt.max_block > kMaxWidth || !(h->opt.cos_eps >= 0.0) ||
      h->opt.cos_eps > 1.0 || h->opt.ordering < 0 || h->opt.ordering > 2 ||
      h->opt.update_precision < 0 || h->opt.update_precision > 2 || h->opt.drop_norm < 0 ||
      h->opt.drop_norm > 1 || h->opt.factor_path < 0 || h->opt.factor_path > 2 ||
      h->opt.apply_path < 0 || h->opt.apply_path > 2 || h->opt.use_mwm < 0 || h->opt.use_mwm > 2 ||
      h->opt.analyze_path < 0 || h->opt.analyze_path > 1 || h->opt.apply_precision < 0 ||
      h->opt.apply_precision > 1 || h->opt.update_mfma < 0 || h->opt.update_mfma > 1 ||
      h->opt.deterministic < 0 || h->opt.deterministic > 1 || h->opt.workers_per_cu < 0 ||
      h->opt.workers_per_cu > 8 || h->opt.use_tuning < 0 || h->opt.use_tuning > 1 ||
      !(h->opt.drop_log_margin >= 0.0)) {
    delete h;
    return BILU_ERR_INVALID;
  }
  h->stream = reinterpret_cast<hipStream_t>(stream);
  *out = h;
  return BILU_OK;
}

void bilu_destroy(bilu_handle* h) {
  if (!h) return;
  (void)hipStreamSynchronize(h->stream);
  delete h;
}

namespace {
// use_mwm = 2 (Sec. 5): the symmetric matching.  The analyzed matrix is
// D A D (A's pattern, values in sv); its 1x1 and 2x2 pivot units, listed
// along the caller's pre_perm, go to h->sym_order / h->sym_ustart.
bilu_status sym_prepare(bilu_handle* h, int64_t n, const int64_t* rowptr, const int32_t* colind,
                        const double* val, std::vector<double>& d, std::vector<double>& sv) {
  if (n <= 0 || !rowptr || !colind || !val || rowptr[0] != 0)
    return fail(h, BILU_ERR_INVALID, "null CSR or n<=0");
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return fail(h, BILU_ERR_INVALID, "rowptr not monotone");
  if (h->opt.pre_perm) {
    std::vector<char> seen(n, 0);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t p = h->opt.pre_perm[i];
      if (p < 0 || p >= n || seen[p]) return fail(h, BILU_ERR_INVALID, "pre_perm is not a permutation");
      seen[p] = 1;
    }
  }
  std::string why;
  const bilu_status ms = sym_matching_host(n, rowptr, colind, val, h->opt.pre_perm, d,
                                           h->sym_order, h->sym_ustart, &why);
  if (ms != BILU_OK) return fail(h, ms, "symmetric matching: " + why);
  sv.resize(rowptr[n]);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) sv[k] = (d[i] * val[k]) * d[colind[k]];
  return BILU_OK;
}
}  // namespace

bilu_status bilu_analyze(bilu_handle* h, int64_t n, const int64_t* rowptr, const int32_t* colind,
                         const double* val) {
  if (!h) return BILU_ERR_INVALID;
  GUARD_BEGIN
  auto t0 = std::chrono::steady_clock::now();
  h->state = 0;
  h->ilu_static = false;
  h->mwm = false;
  h->mwm_sym = false;
  h->sym_order.clear();
  h->sym_ustart.clear();
  h->sym_partner.clear();
  // Sec. 3.1 (use_mwm = 1): analyze D_l A D_r Pi instead of A; Sec. 5
  // (use_mwm = 2): D A D with the symmetric matching's pivot units
  std::vector<int64_t> sigma;
  std::vector<double> dl, dr;
  std::vector<int64_t> m_rp;
  std::vector<int32_t> m_ci;
  std::vector<double> m_v;
  std::vector<double> sym_d;
  if (h->opt.use_mwm == 2) {
    const bilu_status ss = sym_prepare(h, n, rowptr, colind, val, sym_d, m_v);
    if (ss != BILU_OK) return ss;
    val = m_v.data();
  } else if (h->opt.use_mwm) {
    if (n <= 0 || !rowptr || !colind || !val || rowptr[0] != 0)
      return fail(h, BILU_ERR_INVALID, "null CSR or n<=0");
    for (int64_t i = 0; i < n; ++i)
      if (rowptr[i + 1] < rowptr[i]) return fail(h, BILU_ERR_INVALID, "rowptr not monotone");
    sigma.resize(n);
    dl.resize(n);
    dr.resize(n);
    std::string why;
    const bilu_status ms = mwm_host(n, rowptr, colind, val, sigma.data(), dl.data(), dr.data(), &why);
    if (ms != BILU_OK) return fail(h, ms, "maximum weight matching: " + why);
    // column j of A becomes column sigma^{-1}(j); rows keep their order and
    // are re-sorted by the new column index
    std::vector<int32_t> pos(n);
    for (int64_t k = 0; k < n; ++k) pos[sigma[k]] = (int32_t)k;
    m_rp.assign(rowptr, rowptr + n + 1);
    m_ci.resize(rowptr[n]);
    m_v.resize(rowptr[n]);
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t i = 0; i < n; ++i) {
      row.clear();
      for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
        row.push_back({pos[colind[k]], (dl[i] * val[k]) * dr[colind[k]]});
      std::sort(row.begin(), row.end(),
                [](const std::pair<int32_t, double>& x, const std::pair<int32_t, double>& y) {
                  return x.first < y.first;
                });
      for (size_t t = 0; t < row.size(); ++t) {
        m_ci[rowptr[i] + t] = row[t].first;
        m_v[rowptr[i] + t] = row[t].second;
      }
    }
    rowptr = m_rp.data();
    colind = m_ci.data();
    val = m_v.data();
  }
  hipStream_t st = h->stream;
#define CK(x)                                          \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return hip_check(h, e_, #x); \
  } while (0)
  if (h->opt.analyze_path == 0 && h->opt.use_mwm != 2 && n > 0 && n <= INT32_MAX - 1 && rowptr &&
      colind && val &&
      rowptr[0] == 0 && rowptr_monotone(n, rowptr) && rowptr[n] <= INT32_MAX) {
    // the matrix goes to HBM as it is; checks, cosine search and P A P^T there
    const int64_t nnz = rowptr[n];
    DevArray<int64_t> a_rp;
    DevArray<int32_t> a_ci;
    DevArray<double> a_v;
    CK(a_rp.alloc(n + 1));
    CK(a_ci.alloc(std::max<int64_t>(1, nnz)));
    CK(a_v.alloc(std::max<int64_t>(1, nnz)));
    CK(hipMemcpyAsync(a_rp.p, rowptr, (n + 1) * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(a_ci.p, colind, nnz * 4, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(a_v.p, val, nnz * 8, hipMemcpyHostToDevice, st));
    bilu_status s = analyze_device(h, n, a_rp.p, a_ci.p, a_v.p, rowptr);
    if (s != BILU_OK) return s;
  } else {
    bilu_status s = analyze_host(h, n, rowptr, colind, val);
    if (s != BILU_OK) return s;
    const int64_t nnz = h->nnz;
    CK(h->d_rp.alloc(n + 1));
    CK(h->d_ci.alloc(nnz));
    CK(h->d_rv.alloc(nnz));
    CK(h->d_cp.alloc(n + 1));
    CK(h->d_ri.alloc(nnz));
    CK(h->d_cv.alloc(nnz));
    CK(h->d_perm.alloc(n));
    std::vector<int32_t> p32(h->perm.begin(), h->perm.end());
    CK(hipMemcpyAsync(h->d_rp.p, h->prp.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_ci.p, h->pci.data(), nnz * 4, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_rv.p, h->pv.data(), nnz * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_cp.p, h->pcp.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_ri.p, h->pri.data(), nnz * 4, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_cv.p, h->pcv.data(), nnz * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_perm.p, p32.data(), n * 4, hipMemcpyHostToDevice, st));
    // value maps for bilu_refactor, from A's pattern on the device
    if (nnz <= INT32_MAX) {
      DevArray<int64_t> a_rp;
      DevArray<int32_t> a_ci;
      CK(a_rp.alloc(n + 1));
      CK(a_ci.alloc(std::max<int64_t>(1, nnz)));
      CK(hipMemcpyAsync(a_rp.p, rowptr, (n + 1) * 8, hipMemcpyHostToDevice, st));
      CK(hipMemcpyAsync(a_ci.p, colind, nnz * 4, hipMemcpyHostToDevice, st));
      s = value_maps(h, a_rp.p, a_ci.p, false);
      if (s != BILU_OK) return s;
    }
    CK(hipStreamSynchronize(st));
  }
  if (h->opt.use_mwm) {
    // boundary of the scaled system: rows by perm with D_l, columns by
    // sigma o perm with D_r (symmetric matching: both by perm with D)
    const bool sym = h->opt.use_mwm == 2;
    std::vector<int32_t> pc(n);
    std::vector<double> sl(n), sli(n), sr(n), sri(n);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t p = h->perm[i], c = sym ? p : sigma[p];
      pc[i] = (int32_t)c;
      sl[i] = sym ? sym_d[p] : dl[p];
      sli[i] = 1.0 / sl[i];
      sr[i] = sym ? sym_d[c] : dr[c];
      sri[i] = 1.0 / sr[i];
    }
    CK(h->d_perm_col.alloc(n));
    CK(h->d_sl.alloc(n));
    CK(h->d_sl_inv.alloc(n));
    CK(h->d_sr.alloc(n));
    CK(h->d_sr_inv.alloc(n));
    CK(hipMemcpyAsync(h->d_perm_col.p, pc.data(), n * 4, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_sl.p, sl.data(), n * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_sl_inv.p, sli.data(), n * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_sr.p, sr.data(), n * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_sr_inv.p, sri.data(), n * 8, hipMemcpyHostToDevice, st));
    h->mwm = true;
    h->mwm_sym = sym;
  }
  CK(hipStreamSynchronize(st));
#undef CK
  analyze_done(h, t0);
  return BILU_OK;
  GUARD_END
}

bilu_status bilu_analyze_device(bilu_handle* h, int64_t n, const int64_t* rowptr,
                                const int32_t* colind, const double* val) {
  if (!h) return BILU_ERR_INVALID;
  GUARD_BEGIN
  auto t0 = std::chrono::steady_clock::now();
  if (n <= 0 || !rowptr || !colind || !val) return fail(h, BILU_ERR_INVALID, "null CSR or n<=0");
  if (n > INT32_MAX - 1) return fail(h, BILU_ERR_INVALID, "n exceeds int32 range");
  hipStream_t st = h->stream;
  std::vector<int64_t> rp(n + 1);
  hipError_t e = hipMemcpyAsync(rp.data(), rowptr, (n + 1) * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_check(h, e, "bilu_analyze_device: rowptr");
  if (rp[0] != 0) return fail(h, BILU_ERR_INVALID, "rowptr[0] != 0");
  if (!rowptr_monotone(n, rp.data())) return fail(h, BILU_ERR_INVALID, "rowptr not monotone");
  const int64_t nnz = rp[n];
  if (h->opt.use_mwm || h->opt.analyze_path == 1 || nnz > INT32_MAX) {
    // the host route, on a host copy of the matrix
    std::vector<int32_t> ci(nnz);
    std::vector<double> v(nnz);
    if (nnz > 0) {
      e = hipMemcpyAsync(ci.data(), colind, nnz * 4, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipMemcpyAsync(v.data(), val, nnz * 8, hipMemcpyDeviceToHost, st);
      if (e == hipSuccess) e = hipStreamSynchronize(st);
      if (e != hipSuccess) return hip_check(h, e, "bilu_analyze_device: entries");
    }
    const bilu_status s = bilu_analyze(h, n, rp.data(), ci.data(), v.data());
    if (s == BILU_OK) h->stats.t_analyze = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return s;
  }
  h->state = 0;
  h->ilu_static = false;
  h->mwm = false;
  const bilu_status s = analyze_device(h, n, rowptr, colind, val, rp.data());
  if (s != BILU_OK) return s;
  analyze_done(h, t0);
  return BILU_OK;
  GUARD_END
}


bilu_status bilu_factor(bilu_handle* h, double tau) {
  if (!h) return BILU_ERR_INVALID;
  if (h->state < 1) return fail(h, BILU_ERR_STATE, "bilu_factor before bilu_analyze");
  if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(h, BILU_ERR_INVALID, "tau must be >= 0");
  GUARD_BEGIN
  auto t0 = std::chrono::steady_clock::now();
  h->state = 1;
  h->ev_resolve();
  h->stats.dev_ms_factor = h->stats.dev_ms_apply = h->stats.dev_ms_spmv = 0.0;
  h->stats.n_apply = h->stats.n_spmv = 0;
  bilu_status s = factor_device(h, tau);
  if (s != BILU_OK) return s;
  return finish_factor(h, t0);
  GUARD_END
}

bilu_status bilu_refactor(bilu_handle* h, double tau, const double* val) {
  if (!h) return BILU_ERR_INVALID;
  if (h->state < 2) return fail(h, BILU_ERR_STATE, "bilu_refactor before bilu_factor");
  if (!val) return fail(h, BILU_ERR_INVALID, "bilu_refactor: null values");
  if (!(tau >= 0.0) || !std::isfinite(tau)) return fail(h, BILU_ERR_INVALID, "tau must be >= 0");
  if (h->mwm) return fail(h, BILU_ERR_INVALID, "bilu_refactor: not with use_mwm");
  if (h->nnz > 0 && !h->d_vmap_r.p) return fail(h, BILU_ERR_INVALID, "bilu_refactor: nnz >= 2^31");
  GUARD_BEGIN
  auto t0 = std::chrono::steady_clock::now();
  bilu_status s = refactor_values(h, val);
  if (s != BILU_OK) return s;  // nothing changed: the previous factor stands
  h->state = 1;
  h->ev_resolve();
  h->stats.dev_ms_factor = h->stats.dev_ms_apply = h->stats.dev_ms_spmv = 0.0;
  h->stats.n_apply = h->stats.n_spmv = 0;
  h->stats.t_ilu1t = 0.0;
  h->stats.t_phase[0] = h->stats.t_phase[1] = 0.0;
  s = factor_sweep(h, tau, nullptr, nullptr);
  if (s != BILU_OK) return s;
  return finish_factor(h, t0);
  GUARD_END
}

bilu_status bilu_refactor_frozen(bilu_handle* h, const double* val) {
  if (!h) return BILU_ERR_INVALID;
  if (h->state < 2) return fail(h, BILU_ERR_STATE, "bilu_refactor_frozen before bilu_factor");
  if (!val) return fail(h, BILU_ERR_INVALID, "bilu_refactor_frozen: null values");
  if (h->mwm) return fail(h, BILU_ERR_INVALID, "bilu_refactor_frozen: not with use_mwm");
  if (h->nnz > 0 && !h->d_vmap_r.p)
    return fail(h, BILU_ERR_INVALID, "bilu_refactor_frozen: nnz >= 2^31");
  GUARD_BEGIN
  auto t0 = std::chrono::steady_clock::now();
  bilu_status s = refactor_values(h, val);
  if (s != BILU_OK) return s;  // nothing changed: the previous factor stands
  h->state = 1;                // until the new values are complete
  h->ev_resolve();
  h->stats.perturbed_blocks = 0;
  s = frozen_refactor(h);
  if (s != BILU_OK) return s;
  s = refresh_apply_values(h);
  if (s != BILU_OK) return s;
  h->kept_stale = h->fv.dval != h->d_dval.p;
  h->stats.r_kept = -1.0;
  h->stats.t_factor = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  h->state = 2;
  return h->stats.perturbed_blocks > 0 ? BILU_WARN_PERTURBED : BILU_OK;
  GUARD_END
}

bilu_status bilu_factor_batched(bilu_handle** hs, int count, const double* taus) {
  if (!hs || !taus || count < 1) return BILU_ERR_INVALID;
  for (int i = 0; i < count; ++i) {
    if (!hs[i]) return BILU_ERR_INVALID;
    for (int j = 0; j < i; ++j)
      if (hs[j] == hs[i]) return fail(hs[i], BILU_ERR_INVALID, "a handle appears twice in the batch");
    if (hs[i]->state < 1) return fail(hs[i], BILU_ERR_STATE, "bilu_factor_batched before bilu_analyze");
    if (!(taus[i] >= 0.0) || !std::isfinite(taus[i]))
      return fail(hs[i], BILU_ERR_INVALID, "tau must be >= 0");
  }
  try {
    return factor_batched(hs, count, taus);
  } catch (const std::bad_alloc&) {
    return fail(hs[0], BILU_ERR_NO_MEMORY, "host allocation failed");
  } catch (...) {
    return fail(hs[0], BILU_ERR_INTERNAL, "unexpected exception");
  }
}

bilu_status bilu_apply(bilu_handle* h, const double* x, double* y) {
  if (!h || !x || !y || x == y) return fail(h, BILU_ERR_INVALID, "bilu_apply: bad pointers");
  if (h->state < 2) return fail(h, BILU_ERR_STATE, "bilu_apply before bilu_factor");
  GUARD_BEGIN
  const int64_t n = h->n;
  if (h->w_cols < 3) {
    if (h->w_vec.alloc((size_t)3 * n) != hipSuccess) return fail(h, BILU_ERR_NO_MEMORY, "workspace");
    h->w_cols = 3;
  }
  double* xp = h->w_vec.p;
  double* yp = xp + n;
  double* tp = yp + n;
  // x lives in A's row space, y in its column space
  launch_gather(h->stream, n, h->d_perm.p, h->sl(), x, xp);
  bilu_status s = apply_permuted(h, xp, yp, tp);
  if (s != BILU_OK) return s;
  launch_scatter(h->stream, n, h->perm_col(), h->sr(), yp, y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_check(h, e, "bilu_apply");
  return BILU_OK;
  GUARD_END
}

bilu_status bilu_spmv(bilu_handle* h, const double* x, double* y) {
  if (!h || !x || !y || x == y) return fail(h, BILU_ERR_INVALID, "bilu_spmv: bad pointers");
  if (h->state < 1) return fail(h, BILU_ERR_STATE, "bilu_spmv before bilu_analyze");
  GUARD_BEGIN
  const int64_t n = h->n;
  if (h->w_cols < 3) {
    if (h->w_vec.alloc((size_t)3 * n) != hipSuccess) return fail(h, BILU_ERR_NO_MEMORY, "workspace");
    h->w_cols = 3;
  }
  double* xp = h->w_vec.p;
  double* yp = xp + n;
  // x lives in A's column space, y in its row space
  launch_gather(h->stream, n, h->perm_col(), h->sr_inv(), x, xp);
  spmv_permuted(h, xp, yp);
  launch_scatter(h->stream, n, h->d_perm.p, h->sl_inv(), yp, y);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_check(h, e, "bilu_spmv");
  return BILU_OK;
  GUARD_END
}

bilu_status bilu_fgmres_solve(bilu_handle* h, const double* b, double* x, int restart, double rtol,
                              int maxit, bilu_solve_info* info) {
  if (!h || !b || !x || b == x) return fail(h, BILU_ERR_INVALID, "bilu_fgmres_solve: bad pointers");
  if (h->state < 2) return fail(h, BILU_ERR_STATE, "bilu_fgmres_solve before bilu_factor");
  GUARD_BEGIN
  return fgmres(h, b, x, restart, rtol, maxit, info);
  GUARD_END
}

bilu_status bilu_sqmr_solve(bilu_handle* h, const double* b, double* x, double tol, int maxit,
                            bilu_solve_info* info, double* backward_error) {
  if (!h || !b || !x || b == x) return fail(h, BILU_ERR_INVALID, "bilu_sqmr_solve: bad pointers");
  if (h->state < 2) return fail(h, BILU_ERR_STATE, "bilu_sqmr_solve before bilu_factor");
  GUARD_BEGIN
  return sqmr(h, b, x, tol, maxit, info, backward_error);
  GUARD_END
}

bilu_status bilu_mwm(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* val,
                     int64_t* sigma, double* dl, double* dr) {
  if (n < 0) return BILU_ERR_INVALID;
  if (n == 0) return BILU_OK;
  if (!rowptr || !colind || !val || !sigma || !dl || !dr || rowptr[0] != 0) return BILU_ERR_INVALID;
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return BILU_ERR_INVALID;
  try {
    std::string why;
    return bilu::mwm_host(n, rowptr, colind, val, sigma, dl, dr, &why);
  } catch (const std::bad_alloc&) {
    return BILU_ERR_NO_MEMORY;
  } catch (...) {
    return BILU_ERR_INTERNAL;
  }
}

bilu_status bilu_preprocess(const bilu_options* opt, int64_t n, const int64_t* rowptr,
                            const int32_t* colind, const double* val, double tau, int64_t* perm,
                            int64_t* group_starts, int64_t* ngroups, int64_t* block_starts,
                            int64_t* nblocks) {
  if (!perm || !group_starts || !ngroups || !block_starts || !nblocks) return BILU_ERR_INVALID;
  if (!(tau >= 0.0) || !std::isfinite(tau)) return BILU_ERR_INVALID;
  bilu_handle tmp;
  bilu_handle* h = &tmp;
  if (opt)
    h->opt = *opt;
  else
    bilu_default_options(&h->opt);
  if (h->opt.max_block < 1 || h->opt.max_block > kMaxWidth) return BILU_ERR_INVALID;
  if (h->opt.use_mwm < 0 || h->opt.use_mwm > 2) return BILU_ERR_INVALID;
  GUARD_BEGIN
  std::vector<double> sym_d, sym_v;
  if (h->opt.use_mwm == 2) {
    // the symmetric matching's units and scaled values, as bilu_analyze
    const bilu_status ss = sym_prepare(h, n, rowptr, colind, val, sym_d, sym_v);
    if (ss != BILU_OK) return ss;
    val = sym_v.data();
  }
  bilu_status s = analyze_host(h, n, rowptr, colind, val);
  if (s != BILU_OK) return s;
  std::copy(h->perm.begin(), h->perm.end(), perm);
  std::copy(h->group_starts.begin(), h->group_starts.end(), group_starts);
  *ngroups = (int64_t)h->group_starts.size() - 1;
  std::vector<int32_t> bs;
  *nblocks = ilu1t_partition(h, tau, bs);
  std::copy(bs.begin(), bs.end(), block_starts);
  return BILU_OK;
  GUARD_END
}

bilu_status bilu_kept_residual(bilu_handle* h, double* r_kept) {
  if (!h || !r_kept) return fail(h, BILU_ERR_INVALID, "bilu_kept_residual: null argument");
  if (h->state < 2) return fail(h, BILU_ERR_STATE, "bilu_kept_residual before bilu_factor");
  if (h->kept_stale)
    return fail(h, BILU_ERR_STATE,
                "bilu_kept_residual: the frozen refactorization of a factor with merged blocks");
  GUARD_BEGIN
  return kept_residual(h, r_kept);
  GUARD_END
}

bilu_status bilu_sync(bilu_handle* h) {
  if (!h) return BILU_ERR_INVALID;
  hipError_t e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_check(h, e, "bilu_sync");
  int64_t faults = 0;
  return apply_faults(h, &faults);
}

bilu_status bilu_get_stats(const bilu_handle* hc, bilu_stats* st) {
  bilu_handle* h = const_cast<bilu_handle*>(hc);
  if (!h || !st) return BILU_ERR_INVALID;
  h->ev_resolve();
  *st = h->stats;
  return BILU_OK;
}

bilu_status bilu_export_factors(const bilu_handle* hc, bilu_factors_host* out) {
  bilu_handle* h = const_cast<bilu_handle*>(hc);
  if (!h || !out) return BILU_ERR_INVALID;
  if (h->state < 2) return fail(h, BILU_ERR_STATE, "export before factor");
  GUARD_BEGIN
  std::memset(out, 0, sizeof(*out));
  const int64_t n = h->n, nb = h->nb;
  std::vector<int32_t> nr(nb), nc(nb);
  std::vector<int64_t> roff(nb), coff(nb), loff(nb), woff(nb);
  const FactorView& fv = h->fv;
  if (hipMemcpy(nr.data(), fv.nr, nb * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(nc.data(), fv.nc, nb * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(roff.data(), fv.roff, nb * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(coff.data(), fv.coff, nb * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(loff.data(), fv.loff, nb * 8, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(woff.data(), fv.woff, nb * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(h, BILU_ERR_DEVICE, "export copy");
  int64_t tr = 0, tc = 0, tl = 0, tw = 0, td = 0;
  for (int64_t b = 0; b < nb; ++b) {
    int64_t q = h->bstart[b + 1] - h->bstart[b];
    tr += nr[b];
    tc += nc[b];
    tl += nr[b] * q;
    tw += nc[b] * q;
    td += q * q;
  }
  int64_t idx_len = 0, val_len = 0;
  for (int64_t b = 0; b < nb; ++b) {
    int64_t q = h->bstart[b + 1] - h->bstart[b];
    idx_len = std::max(idx_len, std::max(roff[b] + nr[b], coff[b] + nc[b]));
    val_len = std::max(val_len, std::max(loff[b] + nr[b] * q, woff[b] + nc[b] * q));
  }
  std::vector<int32_t> idx(idx_len);
  std::vector<double> val;
  // copy only what is referenced: gather per block from device heaps
  out->n = n;
  out->nblocks = nb;
  out->nblocks_initial = (int64_t)h->bstart0.size() - 1;
  out->ngroups = (int64_t)h->group_starts.size() - 1;
  out->perm = new int64_t[n];
  out->starts = new int64_t[nb + 1];
  out->starts_initial = new int64_t[h->bstart0.size()];
  out->group_starts = new int64_t[h->group_starts.size()];
  out->r_ptr = new int64_t[nb + 1];
  out->c_ptr = new int64_t[nb + 1];
  out->r_idx = new int32_t[std::max<int64_t>(1, tr)];
  out->c_idx = new int32_t[std::max<int64_t>(1, tc)];
  out->l_val = new double[std::max<int64_t>(1, tl)];
  out->w_val = new double[std::max<int64_t>(1, tw)];
  out->d_val = new double[std::max<int64_t>(1, td)];
  std::copy(h->perm.begin(), h->perm.end(), out->perm);
  for (int64_t b = 0; b <= nb; ++b) out->starts[b] = h->bstart[b];
  for (size_t b = 0; b < h->bstart0.size(); ++b) out->starts_initial[b] = h->bstart0[b];
  std::copy(h->group_starts.begin(), h->group_starts.end(), out->group_starts);
  // whole heaps are copied once (simple; export is a checking path); stored
  // FP32 / BF16 values are widened to double exactly
  std::vector<double> vheap(val_len);
  const int vb = value_bytes(fv.vprec);
  std::vector<unsigned char> raw((size_t)val_len * vb);
  if (hipMemcpy(idx.data(), fv.idx, idx.size() * 4, hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(raw.data(), fv.val, raw.size(), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(out->d_val, fv.dval, td * 8, hipMemcpyDeviceToHost) != hipSuccess) {
    bilu_free_factors(out);
    return fail(h, BILU_ERR_DEVICE, "export copy");
  }
  // the drop-decision log
  if (h->drop_log_n > 0) {
    const int64_t m = h->drop_log_n;
    std::vector<int32_t> lb(m), li(m);
    out->drop_norm = new double[m];
    out->drop_block = new int64_t[m];
    out->drop_index = new int64_t[m];
    if (hipMemcpy(lb.data(), h->d_log_blk.p, m * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(li.data(), h->d_log_idx.p, m * 4, hipMemcpyDeviceToHost) != hipSuccess ||
        hipMemcpy(out->drop_norm, h->d_log_nrm.p, m * 8, hipMemcpyDeviceToHost) != hipSuccess) {
      bilu_free_factors(out);
      return fail(h, BILU_ERR_DEVICE, "export copy");
    }
    for (int64_t i = 0; i < m; ++i) {
      out->drop_block[i] = lb[i];
      out->drop_index[i] = li[i];
    }
    out->ndrop_log = m;
  }
  for (int64_t i = 0; i < val_len; ++i) {
    if (vb == 8) {
      std::memcpy(&vheap[i], raw.data() + 8 * i, 8);
    } else if (vb == 4) {
      float x;
      std::memcpy(&x, raw.data() + 4 * i, 4);
      vheap[i] = x;
    } else {
      uint16_t b;
      std::memcpy(&b, raw.data() + 2 * i, 2);
      const uint32_t u = (uint32_t)b << 16;
      float x;
      std::memcpy(&x, &u, 4);
      vheap[i] = x;
    }
  }
  int64_t ar = 0, ac = 0, al = 0, aw = 0;
  out->r_ptr[0] = out->c_ptr[0] = 0;
  for (int64_t b = 0; b < nb; ++b) {
    int64_t q = h->bstart[b + 1] - h->bstart[b];
    std::copy(idx.begin() + roff[b], idx.begin() + roff[b] + nr[b], out->r_idx + ar);
    std::copy(idx.begin() + coff[b], idx.begin() + coff[b] + nc[b], out->c_idx + ac);
    std::copy(vheap.begin() + loff[b], vheap.begin() + loff[b] + nr[b] * q, out->l_val + al);
    std::copy(vheap.begin() + woff[b], vheap.begin() + woff[b] + nc[b] * q, out->w_val + aw);
    ar += nr[b];
    ac += nc[b];
    al += nr[b] * q;
    aw += nc[b] * q;
    out->r_ptr[b + 1] = ar;
    out->c_ptr[b + 1] = ac;
  }
  return BILU_OK;
  GUARD_END
}

bilu_status bilu_export_trace(const bilu_handle* hc, uint64_t* out, int64_t capacity,
                              int64_t* nrecords, double* ticks_per_second) {
  bilu_handle* h = const_cast<bilu_handle*>(hc);
  if (!h || !nrecords) return BILU_ERR_INVALID;
  if (!h->d_trace.p) return fail(h, BILU_ERR_STATE, "no trace: factor with collect_timing = 2");
  const int64_t m = (int64_t)h->d_trace.n;
  *nrecords = m / kTraceFields;
  if (ticks_per_second) {
    int dev = 0, khz = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    *ticks_per_second = khz > 0 ? 1e3 * khz : 1e8;
  }
  if (!out) return BILU_OK;
  if (capacity < m) return fail(h, BILU_ERR_INVALID, "trace buffer too small");
  if (hipMemcpy(out, h->d_trace.p, m * 8, hipMemcpyDeviceToHost) != hipSuccess)
    return fail(h, BILU_ERR_DEVICE, "trace copy");
  return BILU_OK;
}

void bilu_free_factors(bilu_factors_host* f) {
  if (!f) return;
  delete[] f->perm;
  delete[] f->starts;
  delete[] f->starts_initial;
  delete[] f->group_starts;
  delete[] f->r_ptr;
  delete[] f->c_ptr;
  delete[] f->r_idx;
  delete[] f->c_idx;
  delete[] f->l_val;
  delete[] f->w_val;
  delete[] f->d_val;
  delete[] f->drop_block;
  delete[] f->drop_index;
  delete[] f->drop_norm;
  std::memset(f, 0, sizeof(*f));
}

const char* bilu_status_string(bilu_status s) {
  switch (s) {
    case BILU_OK: return "BILU_OK";
    case BILU_WARN_PERTURBED: return "BILU_WARN_PERTURBED";
    case BILU_WARN_NOT_CONVERGED: return "BILU_WARN_NOT_CONVERGED";
    case BILU_ERR_INVALID: return "BILU_ERR_INVALID";
    case BILU_ERR_NO_MEMORY: return "BILU_ERR_NO_MEMORY";
    case BILU_ERR_STATE: return "BILU_ERR_STATE";
    case BILU_ERR_SINGULAR: return "BILU_ERR_SINGULAR";
    case BILU_ERR_DEVICE: return "BILU_ERR_DEVICE";
    case BILU_ERR_INTERNAL: return "BILU_ERR_INTERNAL";
  }
  return "unknown status";
}

const char* bilu_last_error(const bilu_handle* h) { return h ? h->err.c_str() : "null handle"; }

}  // extern "C"
