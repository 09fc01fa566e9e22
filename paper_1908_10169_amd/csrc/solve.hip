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

#include <hipcub/hipcub.hpp>

#include "internal.h"
#include "wg.h"

namespace bilu {
namespace {

constexpr int kDotBlocks = 512;

// ---------------------------------------------------------------------------
// Apply plan builders (run once per factorization)
// ---------------------------------------------------------------------------
// Runs of consecutive rows of R_J that fall into one block K.
__global__ void __launch_bounds__(256) fw_count(FactorView f, int32_t* cnt) {
  const int J = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (J >= f.nb) return;
  const int lane = threadIdx.x & 63;
  const int32_t* R = f.idx + f.roff[J];
  const int m = f.nr[J];
  for (int i = lane; i < m; i += 64) {
    const int K = f.blockOf[R[i]];
    if (i == 0 || f.blockOf[R[i - 1]] != K) atomicAdd(&cnt[K], 1);
  }
}

// Packed (J, first row index in R_J, row count) keys, sorted later per block.
__global__ void __launch_bounds__(256) fw_fill(FactorView f, const int32_t* ptr, int32_t* fillc,
                                               unsigned long long* keys) {
  const int J = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (J >= f.nb) return;
  const int lane = threadIdx.x & 63;
  const int32_t* R = f.idx + f.roff[J];
  const int m = f.nr[J];
  for (int i = lane; i < m; i += 64) {
    const int K = f.blockOf[R[i]];
    if (i == 0 || f.blockOf[R[i - 1]] != K) {
      int e = i + 1;
      while (e < m && f.blockOf[R[e]] == K) ++e;
      const int pos = atomicAdd(&fillc[K], 1);
      keys[ptr[K] + pos] = ((unsigned long long)J << 32) | ((unsigned long long)i << 8) |
                           (unsigned long long)(e - i);
    }
  }
}

// Sort each block's keys (ascending J) and unpack them.
__global__ void __launch_bounds__(64) fw_sort(int nb, const int32_t* ptr, unsigned long long* keys,
                                              int32_t* fw_j, int32_t* fw_r0, int32_t* fw_cnt) {
  const int K = blockIdx.x;
  if (K >= nb) return;
  const int b = ptr[K], m = ptr[K + 1] - b;
  if (threadIdx.x == 0) {
    unsigned long long* k = keys + b;
    for (int i = 1; i < m; ++i) {  // insertion sort: lists are short
      unsigned long long v = k[i];
      int j = i - 1;
      while (j >= 0 && k[j] > v) {
        k[j + 1] = k[j];
        --j;
      }
      k[j + 1] = v;
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < m; i += blockDim.x) {
    const unsigned long long v = keys[b + i];
    fw_j[b + i] = (int32_t)(v >> 32);
    fw_r0[b + i] = (int32_t)((v >> 8) & 0xffffff);
    fw_cnt[b + i] = (int32_t)(v & 0xff);
  }
}

// Distinct blocks of C_K (successors of K in the backward sweep).
__global__ void __launch_bounds__(256) bw_count(FactorView f, int32_t* cnt) {
  const int K = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (K >= f.nb) return;
  const int lane = threadIdx.x & 63;
  const int32_t* Cc = f.idx + f.coff[K];
  const int m = f.nc[K];
  int c = 0;
  for (int i = lane; i < m; i += 64) c += (i == 0 || f.blockOf[Cc[i - 1]] != f.blockOf[Cc[i]]);
  c = wave_sum(c);
  if (lane == 0) cnt[K] = c;
}
__global__ void __launch_bounds__(64) bw_fill(FactorView f, const int32_t* ptr, int32_t* bw_b) {
  const int K = blockIdx.x;
  if (K >= f.nb || threadIdx.x != 0) return;
  const int32_t* Cc = f.idx + f.coff[K];
  const int m = f.nc[K];
  int at = ptr[K];
  for (int i = 0; i < m; ++i) {
    const int B = f.blockOf[Cc[i]];
    if (i == 0 || f.blockOf[Cc[i - 1]] != B) bw_b[at++] = B;
  }
}

// Row-major copy of L: row i lists, for every block J (ascending) whose L_J
// holds row i, the q_J entries L_J(i, :) at columns first(J)..last(J).
__global__ void __launch_bounds__(256) lr_count(FactorView f, const int32_t* fw_ptr,
                                                const int32_t* fw_j, const int32_t* fw_r0,
                                                const int32_t* fw_cnt, int64_t* lr_cnt) {
  const int K = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (K >= f.nb) return;
  const int lane = threadIdx.x & 63;
  const int fK = f.bstart[K], q = f.bstart[K + 1] - fK;
  for (int r = lane; r < q; r += 64) {
    int64_t c = 0;
    for (int e = fw_ptr[K]; e < fw_ptr[K + 1]; ++e) {
      const int J = fw_j[e];
      const int32_t* R = f.idx + f.roff[J];
      for (int i = fw_r0[e]; i < fw_r0[e] + fw_cnt[e]; ++i)
        if (R[i] == fK + r) c += f.bstart[J + 1] - f.bstart[J];
    }
    lr_cnt[fK + r] = c;
  }
}
__global__ void __launch_bounds__(256) lr_fill(FactorView f, const int32_t* fw_ptr,
                                               const int32_t* fw_j, const int32_t* fw_r0,
                                               const int32_t* fw_cnt, const int64_t* lr_ptr,
                                               int32_t* lr_col, double* lr_val) {
  const int K = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (K >= f.nb) return;
  const int lane = threadIdx.x & 63;
  const int fK = f.bstart[K], q = f.bstart[K + 1] - fK;
  for (int r = lane; r < q; r += 64) {
    int64_t at = lr_ptr[fK + r];
    for (int e = fw_ptr[K]; e < fw_ptr[K + 1]; ++e) {
      const int J = fw_j[e];
      const int fJ = f.bstart[J], pJ = f.bstart[J + 1] - fJ;
      const int32_t* R = f.idx + f.roff[J];
      const double* L = f.val + f.loff[J];
      for (int i = fw_r0[e]; i < fw_r0[e] + fw_cnt[e]; ++i)
        if (R[i] == fK + r)
          for (int c = 0; c < pJ; ++c) {
            lr_col[at] = fJ + c;
            lr_val[at] = L[(int64_t)i * pJ + c];
            ++at;
          }
    }
  }
}

// ---------------------------------------------------------------------------
// Level-scheduled sweeps.  Blocks are grouped by their depth in the actual
// dependency graph of the factor (forward: predecessors J whose L_J has rows
// in K; backward: blocks holding the columns of U_K); one launch per level,
// one wave per block, no waiting inside a kernel.
// ---------------------------------------------------------------------------
struct SweepArgs {
  FactorView f;
  const int64_t* lr_ptr;
  const int32_t* lr_col;
  const double* lr_val;
  const int32_t* sched;
  int begin, end;
};

// forward: t_K = x_K - sum over stored L(i, j) t_j, rows of K from the
// row-major copy (groups of lanes per row, fixed reduction tree)
__global__ void __launch_bounds__(256) forward_level(SweepArgs a, const double* x, double* t) {
  const int w = a.begin + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= a.end) return;
  const int lane = threadIdx.x & 63;
  const int K = a.sched[w];
  const int f = a.f.bstart[K], q = a.f.bstart[K + 1] - f;
  int qp = 1;
  while (qp < q && qp < 64) qp <<= 1;
  const int g = 64 / qp;  // lanes per row
  for (int r0 = 0; r0 < q; r0 += qp) {
    const int r = r0 + lane / g, sub = lane % g;
    double acc = 0.0;
    if (r < q) {
      const int64_t b = a.lr_ptr[f + r], e = a.lr_ptr[f + r + 1];
      for (int64_t k = b + sub; k < e; k += g) acc = fma(a.lr_val[k], t[a.lr_col[k]], acc);
    }
    for (int o = g >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (r < q && sub == 0) t[f + r] = x[f + r] - acc;
  }
}

// backward: z_K = D_K (t_K - W_K z(C_K)); lanes over the columns of W_K,
// 16 rows at a time, wave-wide reduction; v staged in LDS per wave
__global__ void __launch_bounds__(256) backward_level(SweepArgs a, const double* t, double* z) {
  __shared__ double sv[4][kMaxWidth];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int w = a.begin + blockIdx.x * 4 + wv;
  const bool active = w < a.end;
  int K = 0, f = 0, q = 0;
  if (active) {
    K = a.sched[w];
    f = a.f.bstart[K];
    q = a.f.bstart[K + 1] - f;
    const int m = a.f.nc[K];
    const int32_t* Cc = a.f.idx + a.f.coff[K];
    const double* W = a.f.val + a.f.woff[K];
    for (int c0 = 0; c0 < q; c0 += 16) {
      const int cn = min(16, q - c0);
      double p[16];
#pragma unroll
      for (int r = 0; r < 16; ++r) p[r] = 0.0;
      for (int j = lane; j < m; j += 64) {
        const double zj = z[Cc[j]];
        const double* wc = W + (int64_t)j * q + c0;
#pragma unroll
        for (int r = 0; r < 16; ++r)
          if (r < cn) p[r] = fma(wc[r], zj, p[r]);
      }
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        if (r >= cn) break;  // wave-uniform
        double v = p[r];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == r) sv[wv][c0 + r] = t[f + c0 + r] - v;
      }
    }
  }
  __syncthreads();
  if (active) {
    const double* D = a.f.dval + a.f.doff[K];
    for (int r = lane; r < q; r += 64) {
      double acc = 0.0;
      for (int c = 0; c < q; ++c) acc = fma(D[r * q + c], sv[wv][c], acc);
      z[f + r] = acc;
    }
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
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->opt.collect_timing) {
    e0 = h->ev_get();
    e1 = h->ev_get();
    if (e0) (void)hipEventRecord(e0, h->stream);
  }
  spmv_csr<<<(unsigned)((n * 8 + 255) / 256), 256, 0, h->stream>>>(n, h->d_rp.p, h->d_ci.p,
                                                                   h->d_rv.p, x, y);
  if (h->opt.collect_timing) {
    if (e1) (void)hipEventRecord(e1, h->stream);
    h->ev_record(2, e0, e1);
  }
  return BILU_OK;
}

// Apply plan of the factor in h->fv: forward/backward dependency lists and
// the row-major copy of L.
// Exclusive prefix of in[0..count) into out[0..count] on the device (out[count]
// is the total); returns the total.
template <class T>
static hipError_t device_scan(bilu_handle* h, const T* in, T* out, int64_t count, T* total) {
  hipStream_t st = h->stream;
  size_t bytes = 0;
  hipError_t e = hipcub::DeviceScan::InclusiveSum(nullptr, bytes, in, out + 1, (int)count, st);
  if (e != hipSuccess) return e;
  if ((e = h->d_scan_tmp.alloc(bytes + 1)) != hipSuccess) return e;
  if ((e = hipMemsetAsync(out, 0, sizeof(T), st)) != hipSuccess) return e;
  if (count > 0 &&
      (e = hipcub::DeviceScan::InclusiveSum(h->d_scan_tmp.p, bytes, in, out + 1, (int)count, st)) !=
          hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(total, out + count, sizeof(T), hipMemcpyDeviceToHost, st)) != hipSuccess)
    return e;
  return hipStreamSynchronize(st);
}

bilu_status build_apply_plan(bilu_handle* h) {
  hipStream_t st = h->stream;
  const FactorView& f = h->fv;
  const int64_t nb = f.nb, n = h->n;
#define CK(x)                                          \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return hip_check(h, e_, #x); \
  } while (0)
  const unsigned gw = (unsigned)((nb + 3) / 4);  // one wave per block
  DevArray<int32_t> cnt;
  CK(cnt.alloc(nb + 1));
  CK(hipMemsetAsync(cnt.p, 0, (nb + 1) * sizeof(int32_t), st));
  fw_count<<<gw, 256, 0, st>>>(f, cnt.p);
  CK(h->fw_ptr.alloc(nb + 1));
  int32_t nfw = 0;
  CK(device_scan<int32_t>(h, cnt.p, h->fw_ptr.p, nb, &nfw));
  const int64_t ne = std::max<int64_t>(1, nfw);
  CK(h->fw_j.alloc(ne));
  CK(h->fw_r0.alloc(ne));
  CK(h->fw_cnt.alloc(ne));
  DevArray<unsigned long long> keys;
  CK(keys.alloc(ne));
  CK(hipMemsetAsync(cnt.p, 0, (nb + 1) * sizeof(int32_t), st));
  fw_fill<<<gw, 256, 0, st>>>(f, h->fw_ptr.p, cnt.p, keys.p);
  fw_sort<<<(unsigned)nb, 64, 0, st>>>((int)nb, h->fw_ptr.p, keys.p, h->fw_j.p, h->fw_r0.p,
                                       h->fw_cnt.p);
  // backward successor blocks
  bw_count<<<gw, 256, 0, st>>>(f, cnt.p);
  CK(h->bw_ptr.alloc(nb + 1));
  int32_t nbw = 0;
  CK(device_scan<int32_t>(h, cnt.p, h->bw_ptr.p, nb, &nbw));
  CK(h->bw_b.alloc(std::max<int32_t>(1, nbw)));
  bw_fill<<<(unsigned)nb, 64, 0, st>>>(f, h->bw_ptr.p, h->bw_b.p);
  // row-major L
  CK(h->lr_ptr.alloc(n + 1));
  DevArray<int64_t> lc;
  CK(lc.alloc(n));
  lr_count<<<gw, 256, 0, st>>>(f, h->fw_ptr.p, h->fw_j.p, h->fw_r0.p, h->fw_cnt.p, lc.p);
  int64_t nlr = 0;
  CK(device_scan<int64_t>(h, lc.p, h->lr_ptr.p, n, &nlr));
  CK(h->lr_col.alloc(std::max<int64_t>(1, nlr)));
  CK(h->lr_val.alloc(std::max<int64_t>(1, nlr)));
  lr_fill<<<gw, 256, 0, st>>>(f, h->fw_ptr.p, h->fw_j.p, h->fw_r0.p, h->fw_cnt.p, h->lr_ptr.p,
                              h->lr_col.p, h->lr_val.p);
  CK(hipGetLastError());
  // dependency levels (actual graph of the factor), computed on the host
  {
    std::vector<int32_t> fp(nb + 1), fj(std::max<int32_t>(1, nfw)), bp(nb + 1),
        bb(std::max<int32_t>(1, nbw));
    CK(hipMemcpyAsync(fp.data(), h->fw_ptr.p, (nb + 1) * 4, hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(bp.data(), h->bw_ptr.p, (nb + 1) * 4, hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(fj.data(), h->fw_j.p, fj.size() * 4, hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(bb.data(), h->bw_b.p, bb.size() * 4, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    auto levels = [&](bool fwd, std::vector<int32_t>& sched, std::vector<int32_t>& lptr) {
      std::vector<int32_t> lev(nb, 0);
      int32_t top = 0;
      for (int64_t s0 = 0; s0 < nb; ++s0) {
        const int64_t K = fwd ? s0 : nb - 1 - s0;
        int32_t l = 0;
        if (fwd)
          for (int32_t e = fp[K]; e < fp[K + 1]; ++e) l = std::max(l, lev[fj[e]] + 1);
        else
          for (int32_t e = bp[K]; e < bp[K + 1]; ++e) l = std::max(l, lev[bb[e]] + 1);
        lev[K] = l;
        top = std::max(top, l);
      }
      lptr.assign(top + 2, 0);
      for (int64_t K = 0; K < nb; ++K) lptr[lev[K] + 1]++;
      for (int32_t l = 0; l <= top; ++l) lptr[l + 1] += lptr[l];
      sched.resize(nb);
      std::vector<int32_t> at(lptr.begin(), lptr.end() - 1);
      for (int64_t K = 0; K < nb; ++K) sched[at[lev[K]]++] = (int32_t)K;
    };
    std::vector<int32_t> sf, sb;
    levels(true, sf, h->lev_f_ptr);
    levels(false, sb, h->lev_b_ptr);
    CK(h->lev_f.alloc(nb));
    CK(h->lev_b.alloc(nb));
    CK(hipMemcpyAsync(h->lev_f.p, sf.data(), nb * 4, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->lev_b.p, sb.data(), nb * 4, hipMemcpyHostToDevice, st));
    h->stats.apply_levels_fwd = (int64_t)h->lev_f_ptr.size() - 1;
    h->stats.apply_levels_bwd = (int64_t)h->lev_b_ptr.size() - 1;
  }
  CK(h->w_red.alloc(kDotBlocks + 64));
  CK(hipStreamSynchronize(st));
  return BILU_OK;
#undef CK
}

bilu_status apply_permuted(bilu_handle* h, const double* x, double* y, double* t) {
  hipStream_t st = h->stream;
  SweepArgs a{};
  a.f = h->fv;
  a.lr_ptr = h->lr_ptr.p;
  a.lr_col = h->lr_col.p;
  a.lr_val = h->lr_val.p;
  a.sched = h->lev_f.p;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (h->opt.collect_timing) {
    e0 = h->ev_get();
    e1 = h->ev_get();
    if (e0) (void)hipEventRecord(e0, st);
  }
  const int nf = (int)h->lev_f_ptr.size() - 1;
  for (int L = 0; L < nf; ++L) {
    a.begin = h->lev_f_ptr[L];
    a.end = h->lev_f_ptr[L + 1];
    forward_level<<<(unsigned)((a.end - a.begin + 3) / 4), 256, 0, st>>>(a, x, t);
  }
  a.sched = h->lev_b.p;
  const int nbk = (int)h->lev_b_ptr.size() - 1;
  for (int L = 0; L < nbk; ++L) {
    a.begin = h->lev_b_ptr[L];
    a.end = h->lev_b_ptr[L + 1];
    backward_level<<<(unsigned)((a.end - a.begin + 3) / 4), 256, 0, st>>>(a, t, y);
  }
  if (h->opt.collect_timing) {
    if (e1) (void)hipEventRecord(e1, st);
    h->ev_record(1, e0, e1);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_check(h, e, "apply launch");
  return BILU_OK;
}

}  // namespace bilu
