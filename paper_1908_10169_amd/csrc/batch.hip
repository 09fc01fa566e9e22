// Batched factorization: many independent matrices in one sweep launch.
//
// Every handle keeps its own analysis (cosine groups, ordering) and gets its
// own ILU(1,tau) partition with its own tau.  Their permuted matrices are
// then placed on the diagonal of one block-diagonal system, with per-block
// tau and perturbation scale alpha, and a single launch of the factor
// kernel sweeps all of them: the dataflow needs no change, since no block
// of one matrix can update a block of another.  Afterwards each handle's
// blocks are compacted into its own factor storage (indices rebased to its
// numbering), and aggregation, the apply plan and the statistics run per
// handle.  Each handle's factor equals the one bilu_factor computes for it
// alone, bit for bit: every block performs the same arithmetic in the same
// order.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "internal.h"

namespace bilu {
namespace {

__global__ void offset_ptr(int64_t count, const int64_t* p, int64_t add, int64_t* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = p[i] + add;
}

__global__ void offset_idx(int64_t count, const int32_t* p, int32_t add, int32_t* out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = p[i] + add;
}

__global__ void batch_block_of(const int32_t* bstart, int nb, int32_t* blockOf) {
  const int b = blockIdx.x * blockDim.y + threadIdx.y;
  if (b >= nb) return;
  for (int i = bstart[b] + threadIdx.x; i < bstart[b + 1]; i += blockDim.x) blockOf[i] = b;
}

struct SplitArgs {
  int nb, b0, n0;                       // blocks of the handle; first block / row in the system
  const int32_t* bstart;                // system partition
  const int32_t* nr; const int32_t* nc; // system per-block counts
  const int64_t* roff; const int64_t* coff; const int64_t* loff; const int64_t* woff;
  const int32_t* idx; const void* val;
  const int64_t* new_roff; const int64_t* new_loff;  // handle layout: rows, columns; L, W
  int32_t* out_idx; void* out_val;
  int vprec;                                          // precision of the stored L, W
};

// One workgroup per block: copy R_K, C_K (rebased), L_K, W_K.
__global__ void split_blocks(SplitArgs a) {
  for (int k = blockIdx.x; k < a.nb; k += gridDim.x) {
    const int K = a.b0 + k;
    const int q = a.bstart[K + 1] - a.bstart[K];
    const int nr = a.nr[K], nc = a.nc[K];
    const int64_t ro = a.new_roff[k], lo = a.new_loff[k];
    for (int t = threadIdx.x; t < nr; t += blockDim.x) a.out_idx[ro + t] = a.idx[a.roff[K] + t] - a.n0;
    for (int t = threadIdx.x; t < nc; t += blockDim.x)
      a.out_idx[ro + nr + t] = a.idx[a.coff[K] + t] - a.n0;
    for (int t = threadIdx.x; t < nr * q; t += blockDim.x)
      value_store(a.out_val, a.vprec, lo + t, value_load(a.val, a.vprec, a.loff[K] + t));
    for (int t = threadIdx.x; t < nc * q; t += blockDim.x)
      value_store(a.out_val, a.vprec, lo + (int64_t)nr * q + t,
                  value_load(a.val, a.vprec, a.woff[K] + t));
  }
}

unsigned grid_for(int64_t count) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(65536, (count + 255) / 256));
}

}  // namespace

bilu_status factor_batched(bilu_handle** hs, int count, const double* taus) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  bilu_handle* h0 = hs[0];
  // what the sweep computes must agree across the batch
  for (int i = 1; i < count; ++i) {
    const bilu_options& a = h0->opt;
    const bilu_options& b = hs[i]->opt;
    if (a.drop_norm != b.drop_norm || a.beta_one != b.beta_one || a.perturb_tau != b.perturb_tau ||
        a.perturb_rho != b.perturb_rho || a.pivot_eps != b.pivot_eps ||
        a.update_precision != b.update_precision || a.factor_path != b.factor_path ||
        a.update_mfma != b.update_mfma || a.deterministic != b.deterministic ||
        h0->mwm_sym != hs[i]->mwm_sym)
      return fail(hs[i], BILU_ERR_INVALID,
                  "batched factorization: drop norm, perturbation (and its symmetric form), "
                  "pivot threshold, update precision, matrix-core use, determinism and kernel "
                  "path must agree across the batch");
  }
  // ---- per-handle partitions (a3)
  for (int i = 0; i < count; ++i) {
    bilu_handle* h = hs[i];
    h->state = 1;
    h->ev_resolve();
    h->stats.dev_ms_factor = h->stats.dev_ms_apply = h->stats.dev_ms_spmv = 0.0;
    h->stats.n_apply = h->stats.n_spmv = 0;
    if (factor_partition(h, taus[i]) < 0) return fail(h, BILU_ERR_INTERNAL, "partition failed");
  }
  // ---- the block-diagonal system
  bilu_handle sys;
  sys.opt = h0->opt;
  sys.stream = h0->stream;
  std::vector<int64_t> n0(count + 1, 0), z0(count + 1, 0), b0(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    n0[i + 1] = n0[i] + hs[i]->n;
    z0[i + 1] = z0[i] + hs[i]->nnz;
    b0[i + 1] = b0[i] + (int64_t)hs[i]->bstart0.size() - 1;
  }
  if (n0[count] > INT32_MAX - 1) return fail(h0, BILU_ERR_INVALID, "batch exceeds int32 indices");
  sys.n = n0[count];
  sys.nnz = z0[count];
  const int64_t nb = b0[count];
  hipStream_t st = sys.stream;
#define CK(x)                                              \
  do {                                                     \
    hipError_t e_ = (x);                                   \
    if (e_ != hipSuccess) return hip_check(h0, e_, #x);    \
  } while (0)
  CK(sys.d_rp.alloc(sys.n + 1));
  CK(sys.d_cp.alloc(sys.n + 1));
  CK(sys.d_ci.alloc(std::max<int64_t>(1, sys.nnz)));
  CK(sys.d_ri.alloc(std::max<int64_t>(1, sys.nnz)));
  CK(sys.d_rv.alloc(std::max<int64_t>(1, sys.nnz)));
  CK(sys.d_cv.alloc(std::max<int64_t>(1, sys.nnz)));
  sys.bstart0.assign(1, 0);
  std::vector<double> tau_blk, alpha_blk;
  tau_blk.reserve(nb);
  alpha_blk.reserve(nb);
  for (int i = 0; i < count; ++i) {
    const bilu_handle* h = hs[i];
    const int64_t n = h->n, z = h->nnz;
    // pointers: n+1 entries; the next matrix overwrites the shared last one
    // with the same value
    offset_ptr<<<grid_for(n + 1), 256, 0, st>>>(n + 1, h->d_rp.p, z0[i], sys.d_rp.p + n0[i]);
    offset_ptr<<<grid_for(n + 1), 256, 0, st>>>(n + 1, h->d_cp.p, z0[i], sys.d_cp.p + n0[i]);
    offset_idx<<<grid_for(z), 256, 0, st>>>(z, h->d_ci.p, (int32_t)n0[i], sys.d_ci.p + z0[i]);
    offset_idx<<<grid_for(z), 256, 0, st>>>(z, h->d_ri.p, (int32_t)n0[i], sys.d_ri.p + z0[i]);
    CK(hipMemcpyAsync(sys.d_rv.p + z0[i], h->d_rv.p, z * sizeof(double), hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(sys.d_cv.p + z0[i], h->d_cv.p, z * sizeof(double), hipMemcpyDeviceToDevice, st));
    for (size_t b = 1; b < h->bstart0.size(); ++b) {
      sys.bstart0.push_back((int32_t)(h->bstart0[b] + n0[i]));
      tau_blk.push_back(taus[i]);
      alpha_blk.push_back(h->alpha);
    }
  }
  CK(hipGetLastError());
  // ---- one sweep (a4-a8) over every block of the batch
  bilu_status s = factor_sweep(&sys, 0.0, &tau_blk, &alpha_blk);
  if (s != BILU_OK) {
    h0->err = "batched factorization: " + sys.err;
    return s;
  }
  CK(hipStreamSynchronize(st));
  sys.ev_resolve();
  // ---- each handle's blocks into its own storage
  std::vector<int32_t> nr(nb), nc(nb), pflag(nb);
  CK(hipMemcpy(nr.data(), sys.d_nr.p, nb * 4, hipMemcpyDeviceToHost));
  CK(hipMemcpy(nc.data(), sys.d_nc.p, nb * 4, hipMemcpyDeviceToHost));
  CK(hipMemcpy(pflag.data(), sys.d_pflag.p, nb * 4, hipMemcpyDeviceToHost));
  for (int i = 0; i < count; ++i) {
    bilu_handle* h = hs[i];
    const int64_t nbi = b0[i + 1] - b0[i], n = h->n;
    const std::vector<int32_t>& bs = h->bstart0;
    std::vector<int64_t> roff(nbi), coff(nbi), loff(nbi), woff(nbi);
    h->doff_h.assign(nbi + 1, 0);
    int64_t io = 0, vo = 0;
    int perturbed = 0;
    for (int64_t k = 0; k < nbi; ++k) {
      const int64_t K = b0[i] + k, q = bs[k + 1] - bs[k];
      roff[k] = io;
      coff[k] = io + nr[K];
      io += nr[K] + nc[K];
      loff[k] = vo;
      woff[k] = vo + nr[K] * q;
      vo += (int64_t)(nr[K] + nc[K]) * q;
      h->doff_h[k + 1] = h->doff_h[k] + q * q;
      perturbed += pflag[K];
    }
    CK(h->d_bstart.alloc(nbi + 1));
    CK(h->d_blockof.alloc(n));
    CK(h->d_roff.alloc(nbi));
    CK(h->d_coff.alloc(nbi));
    CK(h->d_loff.alloc(nbi));
    CK(h->d_woff.alloc(nbi));
    CK(h->d_doff.alloc(nbi + 1));
    CK(h->d_nr.alloc(nbi));
    CK(h->d_nc.alloc(nbi));
    CK(h->d_dval.alloc(h->doff_h[nbi]));
    CK(h->d_sval.alloc(h->doff_h[nbi]));
    CK(h->d_idx_heap.alloc(std::max<int64_t>(1, io)));
    CK(h->d_val_heap.alloc(std::max<int64_t>(1, vo) * value_bytes(h->opt.update_precision)));
    CK(hipMemcpyAsync(h->d_bstart.p, bs.data(), (nbi + 1) * 4, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_roff.p, roff.data(), nbi * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_coff.p, coff.data(), nbi * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_loff.p, loff.data(), nbi * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_woff.p, woff.data(), nbi * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_doff.p, h->doff_h.data(), (nbi + 1) * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->d_nr.p, sys.d_nr.p + b0[i], nbi * 4, hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(h->d_nc.p, sys.d_nc.p + b0[i], nbi * 4, hipMemcpyDeviceToDevice, st));
    const int64_t d0 = sys.doff_h[b0[i]];
    CK(hipMemcpyAsync(h->d_dval.p, sys.d_dval.p + d0, h->doff_h[nbi] * 8, hipMemcpyDeviceToDevice, st));
    CK(hipMemcpyAsync(h->d_sval.p, sys.d_sval.p + d0, h->doff_h[nbi] * 8, hipMemcpyDeviceToDevice, st));
    {
      dim3 blk(64, 4);
      batch_block_of<<<dim3((unsigned)((nbi + 3) / 4)), blk, 0, st>>>(h->d_bstart.p, (int)nbi,
                                                                    h->d_blockof.p);
    }
    SplitArgs sa{};
    sa.nb = (int)nbi;
    sa.b0 = (int)b0[i];
    sa.n0 = (int)n0[i];
    sa.bstart = sys.d_bstart.p;
    sa.nr = sys.d_nr.p;
    sa.nc = sys.d_nc.p;
    sa.roff = sys.d_roff.p;
    sa.coff = sys.d_coff.p;
    sa.loff = sys.d_loff.p;
    sa.woff = sys.d_woff.p;
    sa.idx = sys.d_idx_heap.p;
    sa.val = sys.d_val_heap.p;
    sa.new_roff = h->d_roff.p;
    sa.new_loff = h->d_loff.p;
    sa.out_idx = h->d_idx_heap.p;
    sa.out_val = h->d_val_heap.p;
    sa.vprec = h->opt.update_precision;
    split_blocks<<<(unsigned)std::min<int64_t>(nbi, 4096), 64, 0, st>>>(sa);
    CK(hipGetLastError());
    // device counters of the one launch describe the whole batch
    h->stats.nblocks_initial = nbi;
    h->idx_used = io;
    h->val_used = vo;
    h->stats.perturbed_blocks = perturbed;
    h->stats.flops_update = sys.stats.flops_update;
    h->stats.bytes_factor = sys.stats.bytes_factor;
    h->stats.factor_levels = sys.stats.factor_levels;
    h->stats.t_factor_device = sys.stats.t_factor_device;
    h->stats.t_phase[2] = sys.stats.t_phase[2];
    h->stats.t_phase[3] = sys.stats.t_phase[3];
    h->stats.dev_ms_factor = sys.stats.dev_ms_factor;
    h->stats.n_factor_launches = 1;
    // the settings of the common sweep; the apply path stays the handle's own
    // unless a tuned entry chose it
    h->eff = sys.eff;
    if (!sys.stats.tuning_applied) h->eff.apply_path = h->opt.apply_path;
    h->stats.tuning_applied = sys.stats.tuning_applied;
    h->stats.max_width_initial = sys.stats.max_width_initial;
  }
  CK(hipStreamSynchronize(st));
  // ---- aggregation, apply plan, statistics per handle
  bilu_status worst = BILU_OK;
  for (int i = 0; i < count; ++i) {
    const bilu_status r = finish_factor(hs[i], t0);
    if (r < 0) return r;
    if (r == BILU_WARN_PERTURBED) worst = r;
  }
  return worst;
#undef CK
}

}  // namespace bilu
