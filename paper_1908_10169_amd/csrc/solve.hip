// Preconditioner apply (Sec. 3.7, multiplying by D as in Sec. 2.2), sparse
// matrix-vector product and the vector kernels of flexible GMRES.
//
// Apply, in the permuted numbering, for the final blocks K:
//   forward   t_K = x_K - sum_J L_J(rows in K, :) t_J      (L unit, J < K)
//   backward  z_K = D_K (t_K - sum_{j in C_K} W_K(:, j) z_j)
// One wave per block; blocks of one dependency level run in one launch.
// Sums run over J in increasing order and over stored entries in storage
// order, so results are run-to-run identical.
#include <algorithm>
#include <numeric>

#include "internal.h"
#include "wg.h"

namespace bilu {
namespace {

constexpr int kDotBlocks = 512;

struct ApplyArgs {
  const int32_t* bstart;
  const int32_t* nr;
  const int32_t* nc;
  const int64_t* roff;
  const int64_t* coff;
  const int64_t* loff;
  const int64_t* woff;
  const int64_t* doff;
  const int32_t* idx;
  const double* val;
  const double* dval;
  const int32_t* fw_ptr;
  const int32_t* fw_j;
  const int32_t* fw_r0;
  const int32_t* fw_cnt;
  const int32_t* sched;
  int begin, end;
};

__global__ void __launch_bounds__(256) forward_level(ApplyArgs a, const double* x, double* t) {
  const int w = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int idx = a.begin + w;
  if (idx >= a.end) return;
  const int lane = threadIdx.x & 63;
  const int K = a.sched[idx];
  const int f = a.bstart[K], q = a.bstart[K + 1] - f;
  for (int r = lane; r < q; r += 64) {
    double acc = 0.0;
    for (int e = a.fw_ptr[K]; e < a.fw_ptr[K + 1]; ++e) {
      const int J = a.fw_j[e], r0 = a.fw_r0[e], cnt = a.fw_cnt[e];
      const int fJ = a.bstart[J], pJ = a.bstart[J + 1] - fJ;
      const int32_t* RJ = a.idx + a.roff[J];
      const double* LJ = a.val + a.loff[J];
      for (int ir = r0; ir < r0 + cnt; ++ir) {
        if (RJ[ir] != f + r) continue;
        const double* lr = LJ + (int64_t)ir * pJ;
        for (int c = 0; c < pJ; ++c) acc = fma(lr[c], t[fJ + c], acc);
      }
    }
    t[f + r] = x[f + r] - acc;
  }
}

__global__ void __launch_bounds__(256) backward_level(ApplyArgs a, const double* t, double* z) {
  __shared__ double sv[4][kMaxWidth];
  const int wv = threadIdx.x >> 6;
  const int idx = a.begin + blockIdx.x * 4 + wv;
  const bool active = idx < a.end;
  const int lane = threadIdx.x & 63;
  int K = 0, f = 0, q = 0;
  if (active) {
    K = a.sched[idx];
    f = a.bstart[K];
    q = a.bstart[K + 1] - f;
    const int nC = a.nc[K];
    const int32_t* CK = a.idx + a.coff[K];
    const double* WK = a.val + a.woff[K];
    for (int r = lane; r < q; r += 64) {
      double acc = 0.0;
      for (int cj = 0; cj < nC; ++cj) acc = fma(WK[(int64_t)cj * q + r], z[CK[cj]], acc);
      sv[wv][r] = t[f + r] - acc;
    }
  }
  __syncthreads();
  if (active) {
    const double* DK = a.dval + a.doff[K];
    for (int r = lane; r < q; r += 64) {
      double acc = 0.0;
      for (int c = 0; c < q; ++c) acc = fma(DK[r * q + c], sv[wv][c], acc);
      z[f + r] = acc;
    }
  }
}

// Forward lists of each block: predecessors J with rows inside K, sorted, and
// the range of those rows inside R_J.
__global__ void __launch_bounds__(256) build_forward_lists(
    int nb, const int32_t* bstart, const int32_t* cnt_arr, const int32_t* list,
    const int32_t* ovf_head, const int32_t* ovf_j, const int32_t* ovf_next, const int32_t* nr,
    const int64_t* roff, const int32_t* idx, const int32_t* fw_ptr, int32_t* fw_j,
    int32_t* fw_r0, int32_t* fw_cnt, int* err) {
  __shared__ int keys[kPredCap];
  const int K = blockIdx.x;
  if (K >= nb) return;
  const int cnt = cnt_arr[K];
  if (cnt > kPredCap) {
    if (threadIdx.x == 0) atomicExch(err, kDevPredOverflow);
    return;
  }
  const int inl = min(cnt, kListCap);
  for (int t = threadIdx.x; t < inl; t += blockDim.x) keys[t] = list[(int64_t)K * kListCap + t];
  if (threadIdx.x == 0) {
    int node = ovf_head[K], at = kListCap;
    while (node >= 0 && at < cnt) {
      keys[at++] = ovf_j[node];
      node = ovf_next[node];
    }
  }
  __syncthreads();
  wg_bitonic_sort(keys, cnt);
  const int f = bstart[K], l = bstart[K + 1] - 1;
  const int base = fw_ptr[K];
  for (int e = threadIdx.x; e < cnt; e += blockDim.x) {
    const int J = keys[e];
    const int32_t* RJ = idx + roff[J];
    const int m = nr[J];
    int lo = 0, hi = m;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (RJ[mid] < f) lo = mid + 1; else hi = mid;
    }
    int r0 = lo;
    hi = m;
    while (lo < hi) {
      int mid = (lo + hi) >> 1;
      if (RJ[mid] <= l) lo = mid + 1; else hi = mid;
    }
    fw_j[base + e] = J;
    fw_r0[base + e] = r0;
    fw_cnt[base + e] = lo - r0;
  }
}

// y = A x, CSR, 8 lanes per row.
__global__ void __launch_bounds__(256) spmv_csr(int64_t n, const int64_t* rp, const int32_t* ci,
                                                const double* v, const double* x, double* y) {
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 3;
  const int sub = threadIdx.x & 7;
  double acc = 0.0;
  if (row < n)
    for (int64_t k = rp[row] + sub; k < rp[row + 1]; k += 8) acc = fma(v[k], x[ci[k]], acc);
  acc += __shfl_xor(acc, 1, 64);
  acc += __shfl_xor(acc, 2, 64);
  acc += __shfl_xor(acc, 4, 64);
  if (row < n && sub == 0) y[row] = acc;
}

__global__ void gather_k(int64_t n, const int32_t* perm, const double* x, double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = x[perm[i]];
}
__global__ void scatter_k(int64_t n, const int32_t* perm, const double* x, double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[perm[i]] = x[i];
}
__global__ void axpy_dev_k(int64_t n, const double* alpha, double sign, const double* x, double* y) {
  const double a = sign * *alpha;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = fma(a, x[i], y[i]);
}
__global__ void axpy_k(int64_t n, double a, const double* x, double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = fma(a, x[i], y[i]);
}
__global__ void scale_k(int64_t n, double a, const double* x, double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}
__global__ void sub_k(int64_t n, const double* b, const double* ax, double* r) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    r[i] = b[i] - ax[i];
}

// Deterministic dot product: fixed grid of partial sums, then one block
// adds the partials in index order.
__global__ void __launch_bounds__(256) dot_partial(int64_t n, const double* x, const double* y,
                                                   double* partial) {
  __shared__ double sw[4];
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc = fma(x[i], y[i], acc);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (sw[0] + sw[1]) + (sw[2] + sw[3]);
}
__global__ void __launch_bounds__(256) dot_final(int nparts, const double* partial, double* out) {
  __shared__ double sw[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += partial[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = (sw[0] + sw[1]) + (sw[2] + sw[3]);
}

inline unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

}  // namespace

void launch_gather(hipStream_t s, int64_t n, const int32_t* perm, const double* x, double* y) {
  gather_k<<<grid_for(n), 256, 0, s>>>(n, perm, x, y);
}
void launch_scatter(hipStream_t s, int64_t n, const int32_t* perm, const double* x, double* y) {
  scatter_k<<<grid_for(n), 256, 0, s>>>(n, perm, x, y);
}
void launch_axpy(hipStream_t s, int64_t n, const double* alpha_dev, double sign, const double* x,
                 double* y) {
  axpy_dev_k<<<grid_for(n), 256, 0, s>>>(n, alpha_dev, sign, x, y);
}
void launch_axpy_host(hipStream_t s, int64_t n, double alpha, const double* x, double* y) {
  axpy_k<<<grid_for(n), 256, 0, s>>>(n, alpha, x, y);
}
void launch_scale(hipStream_t s, int64_t n, double alpha, const double* x, double* y) {
  scale_k<<<grid_for(n), 256, 0, s>>>(n, alpha, x, y);
}
void launch_sub(hipStream_t s, int64_t n, const double* b, const double* ax, double* r) {
  sub_k<<<grid_for(n), 256, 0, s>>>(n, b, ax, r);
}
void launch_dot(hipStream_t s, int64_t n, const double* x, const double* y, double* partial,
                double* out) {
  dot_partial<<<kDotBlocks, 256, 0, s>>>(n, x, y, partial);
  dot_final<<<1, 256, 0, s>>>(kDotBlocks, partial, out);
}

bilu_status spmv_permuted(bilu_handle* h, const double* x, double* y) {
  const int64_t n = h->n;
  spmv_csr<<<(unsigned)((n * 8 + 255) / 256), 256, 0, h->stream>>>(n, h->d_rp.p, h->d_ci.p,
                                                                   h->d_rv.p, x, y);
  return BILU_OK;
}

// Forward lists and apply levels for the final factor.
bilu_status build_apply_plan(bilu_handle* h) {
  hipStream_t st = h->stream;
  const int64_t nb = h->nb;
#define CK(x)                                          \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return hip_check(h, e_, #x); \
  } while (0)
  std::vector<int32_t> cnt(nb), ptr(nb + 1, 0);
  CK(hipMemcpyAsync(cnt.data(), h->d_row_cnt.p, nb * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  for (int64_t k = 0; k < nb; ++k) ptr[k + 1] = ptr[k] + cnt[k];
  CK(h->fw_ptr.alloc(nb + 1));
  CK(h->fw_j.alloc(std::max<int32_t>(1, ptr[nb])));
  CK(h->fw_r0.alloc(std::max<int32_t>(1, ptr[nb])));
  CK(h->fw_cnt.alloc(std::max<int32_t>(1, ptr[nb])));
  CK(hipMemcpyAsync(h->fw_ptr.p, ptr.data(), (nb + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
  int* err = h->d_status.p + 4;
  CK(hipMemsetAsync(err, 0, sizeof(int), st));
  build_forward_lists<<<(unsigned)nb, 256, 0, st>>>(
      (int)nb, h->d_bstart.p, h->d_row_cnt.p, h->d_row_list.p, h->d_row_ovf.p, h->d_ovf_j.p,
      h->d_ovf_next.p, h->d_nr.p, h->d_roff.p, h->d_idx_heap.p, h->fw_ptr.p, h->fw_j.p, h->fw_r0.p,
      h->fw_cnt.p, err);
  CK(hipGetLastError());
  int e = 0;
  CK(hipMemcpyAsync(&e, err, sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (e) return fail(h, BILU_ERR_NO_MEMORY, "forward list exceeds capacity");
  // schedule: the factorization's tree levels are valid for both sweeps
  h->apply_sched = h->sched;
  h->apply_ptr = h->sched_ptr;
  h->stats.apply_levels_fwd = (int64_t)h->apply_ptr.size() - 1;
  h->stats.apply_levels_bwd = h->stats.apply_levels_fwd;
  CK(h->w_red.alloc(kDotBlocks + 64));
  return BILU_OK;
#undef CK
}

bilu_status apply_permuted(bilu_handle* h, const double* x, double* y, double* t) {
  hipStream_t st = h->stream;
  ApplyArgs a{};
  a.bstart = h->d_bstart.p;
  a.nr = h->d_nr.p;
  a.nc = h->d_nc.p;
  a.roff = h->d_roff.p;
  a.coff = h->d_coff.p;
  a.loff = h->d_loff.p;
  a.woff = h->d_woff.p;
  a.doff = h->d_doff.p;
  a.idx = h->d_idx_heap.p;
  a.val = h->d_val_heap.p;
  a.dval = h->d_dval.p;
  a.fw_ptr = h->fw_ptr.p;
  a.fw_j = h->fw_j.p;
  a.fw_r0 = h->fw_r0.p;
  a.fw_cnt = h->fw_cnt.p;
  if (!h->d_apply_sched.p) {
    if (h->d_apply_sched.alloc(h->apply_sched.size()) != hipSuccess)
      return fail(h, BILU_ERR_NO_MEMORY, "apply schedule");
    (void)hipMemcpyAsync(h->d_apply_sched.p, h->apply_sched.data(),
                         h->apply_sched.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
  }
  a.sched = h->d_apply_sched.p;
  const int nlev = (int)h->apply_ptr.size() - 1;
  for (int L = 0; L < nlev; ++L) {
    a.begin = h->apply_ptr[L];
    a.end = h->apply_ptr[L + 1];
    const int cnt = a.end - a.begin;
    forward_level<<<(unsigned)((cnt + 3) / 4), 256, 0, st>>>(a, x, t);
  }
  for (int L = nlev - 1; L >= 0; --L) {
    a.begin = h->apply_ptr[L];
    a.end = h->apply_ptr[L + 1];
    const int cnt = a.end - a.begin;
    backward_level<<<(unsigned)((cnt + 3) / 4), 256, 0, st>>>(a, t, y);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_check(h, e, "apply launch");
  return BILU_OK;
}

}  // namespace bilu
