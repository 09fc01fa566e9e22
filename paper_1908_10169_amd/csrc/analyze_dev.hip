// Preprocessing steps 2-3 of Sec. 3.7 with the matrix resident in HBM: the
// CSR checks, the cosine candidate search of Sec. 3.2, and the permuted
// matrix P A P^T with its transpose (Sec. 3.3).
//
// The host keeps what is sequential or O(n) on index arrays: the mu + 2 sigma
// limits (summed in index order, as the host path does), the greedy replay
// of the seeds, the nested dissection of the compressed graph and the
// expansion of the permutation.  The result is the one of the host path bit
// for bit.
//
//   1. entries_check: column indices in range and strictly increasing per
//      row, values finite, max |a_ij|, and the column counts.
//   2. A1 = A(pre, pre): rows gathered with their columns renumbered (their
//      order within a row left as it comes), and the columns of A1 filled by
//      atomic positions (row order left as it comes).  The cosine test needs
//      only pair counts, so neither order matters.
//   3. cos_rows<false>: one wave per seed row i counts |pat(i) & pat(j)| for
//      every later row j reached through the columns of row i in an LDS hash
//      table and keeps the number of rows that pass the test;
//      cos_rows<true> repeats the count and writes the passing rows
//      ascending.  A row with more than kHash distinct later rows is counted
//      on the host from a copy of A1's pattern.
//   4. P A P^T in CSR (each row ascending by column) and in CSC (each column
//      ascending by row) by radix sorts of (row, column) keys.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <hipcub/hipcub.hpp>
#include <numeric>

#include "internal.h"

namespace bilu {
namespace {

constexpr int kT = 256;         // threads of the streaming kernels (4 waves)
constexpr int kHashBits = 9;
constexpr int kHash = 1 << kHashBits;  // distinct later rows per seed held in LDS

int stream_grid(int64_t rows) {
  const int64_t b = (rows + kT / 64 - 1) / (kT / 64);
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 8192));
}

// Column indices in range and strictly increasing per row (rowptr was checked
// on the host), values finite; max |a_ij| and the column counts.  Error bits:
// 1 range, 2 order, 4 non-finite.  One wave per row.
__global__ __launch_bounds__(kT) void entries_check(int64_t n, const int64_t* __restrict__ rp,
                                                    const int32_t* __restrict__ ci,
                                                    const double* __restrict__ v,
                                                    int* __restrict__ bad,
                                                    unsigned long long* __restrict__ amax,
                                                    int32_t* __restrict__ ccount) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  int f = 0;
  double mx = 0.0;
  for (int64_t i = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; i < n; i += nw) {
    const int64_t b = rp[i], e = rp[i + 1];
    for (int64_t k = b + lane; k < e; k += 64) {
      const int32_t c = ci[k];
      if (c < 0 || c >= n) {
        f |= 1;
      } else {
        atomicAdd(&ccount[c], 1);
        if (k > b && c <= ci[k - 1]) f |= 2;
      }
      const double x = v[k];
      if (!isfinite(x)) f |= 4;
      else mx = fmax(mx, fabs(x));
    }
  }
  for (int o = 32; o; o >>= 1) {
    f |= __shfl_xor(f, o);
    mx = fmax(mx, __shfl_xor(mx, o));
  }
  __shared__ int sf[kT / 64];
  __shared__ double sm[kT / 64];
  if (lane == 0) {
    sf[threadIdx.x >> 6] = f;
    sm[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kT / 64; ++w) {
      f |= sf[w];
      mx = fmax(mx, sm[w]);
    }
    if (f) atomicOr(bad, f);
    if (mx > 0.0) atomicMax(amax, (unsigned long long)__double_as_longlong(mx));
  }
}

// inv[p[i]] = i
__global__ void invert_perm(int64_t n, const int32_t* __restrict__ p, int32_t* __restrict__ inv) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += stride)
    inv[p[i]] = (int32_t)i;
}

// Row r of A(pre, pre) = row pre[r] of A with columns renumbered by inv.
__global__ __launch_bounds__(kT) void gather_rows(int64_t n, const int64_t* __restrict__ rp,
                                                  const int32_t* __restrict__ ci,
                                                  const int32_t* __restrict__ pre,
                                                  const int32_t* __restrict__ inv,
                                                  const int64_t* __restrict__ rp1,
                                                  int32_t* __restrict__ ci1) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; r < n; r += nw) {
    const int64_t b = rp[pre[r]], d = rp1[r], len = rp1[r + 1] - d;
    for (int64_t t = lane; t < len; t += 64) ci1[d + t] = inv[ci[b + t]];
  }
}

// Columns of A1: entry (r, c) lands at an atomic position of column c.
__global__ __launch_bounds__(kT) void scatter_cols(int64_t n, const int64_t* __restrict__ rp1,
                                                   const int32_t* __restrict__ ci1,
                                                   unsigned long long* __restrict__ fill,
                                                   int32_t* __restrict__ ri1) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t r = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; r < n; r += nw)
    for (int64_t k = rp1[r] + lane; k < rp1[r + 1]; k += 64) {
      const unsigned long long pos = atomicAdd(&fill[ci1[k]], 1ull);
      ri1[pos] = (int32_t)r;
    }
}

struct CosArgs {
  int64_t n;
  const int64_t* rp1;  // rows of A1 (column order irrelevant)
  const int32_t* ci1;
  const int64_t* cp1;  // columns of A1 (row order irrelevant)
  const int32_t* ri1;
  const uint8_t* skip;
  int int_test;        // eps = 0.8: the test 5 ov^2 >= 4 |pat(i)| |pat(j)| in integers
  double eps;
  int32_t* cnt;        // per seed: rows passing, -1 past the table, 0 skipped
  const int64_t* off;  // fill pass: where each seed's rows go
  int32_t* out;
};

// Sec. 3.2: row j > i is a candidate of seed i when
// |pat(i) & pat(j)|^2 >= eps |pat(i)| |pat(j)|, neither row being skipped.
// One wave (the whole workgroup) per seed row.
template <bool kFill>
__global__ __launch_bounds__(64) void cos_rows(CosArgs a) {
  __shared__ int32_t key[kHash];
  __shared__ int32_t hit[kHash];
  __shared__ int32_t lst[kHash];
  const int lane = threadIdx.x;
  for (int64_t i = blockIdx.x; i < a.n; i += gridDim.x) {
    if (a.skip[i]) {
      if (!kFill && lane == 0) a.cnt[i] = 0;
      continue;
    }
    if (kFill && a.cnt[i] <= 0) continue;
    for (int s = lane; s < kHash; s += 64) {
      key[s] = -1;
      hit[s] = 0;
    }
    __syncthreads();
    int ovf = 0;
    const int64_t b = a.rp1[i], e = a.rp1[i + 1];
    for (int64_t k = b + lane; k < e && !ovf; k += 64) {
      const int32_t c = a.ci1[k];
      const int64_t ce = a.cp1[c + 1];
      for (int64_t m = a.cp1[c]; m < ce; ++m) {
        const int32_t j = a.ri1[m];
        if (j <= i || a.skip[j]) continue;
        uint32_t h = ((uint32_t)j * 2654435761u) >> (32 - kHashBits);
        int probes = 0;
        for (;;) {
          const int32_t old = atomicCAS(&key[h], -1, j);
          if (old == -1 || old == j) {
            atomicAdd(&hit[h], 1);
            break;
          }
          if (++probes == kHash) {  // every slot holds another row
            ovf = 1;
            break;
          }
          h = (h + 1) & (kHash - 1);
        }
        if (ovf) break;
      }
    }
    if (__syncthreads_or(ovf)) {
      if (!kFill && lane == 0) a.cnt[i] = -1;
      continue;
    }
    const int64_t rci = e - b;
    int m = 0;
    for (int s0 = 0; s0 < kHash; s0 += 64) {
      const int32_t j = key[s0 + lane];
      bool ok = false;
      if (j >= 0) {
        const int64_t ov = hit[s0 + lane];
        const int64_t rcj = a.rp1[j + 1] - a.rp1[j];
        ok = a.int_test ? (5 * ov * ov >= 4 * rci * rcj)
                        : (double(ov) * ov >= a.eps * double(rci) * double(rcj));
      }
      const unsigned long long bal = __ballot(ok);
      if (ok) lst[m + __popcll(bal & ((1ull << lane) - 1ull))] = j;
      m += __popcll(bal);
    }
    if (!kFill) {
      if (lane == 0) a.cnt[i] = m;
      __syncthreads();
      continue;
    }
    __syncthreads();
    int32_t* o = a.out + a.off[i];
    for (int t = lane; t < m; t += 64) {
      const int32_t x = lst[t];
      int r = 0;
      for (int u = 0; u < m; ++u) r += lst[u] < x;
      o[r] = x;
    }
    __syncthreads();
  }
}

// Keys of the entries of P A P^T: (new row, new column) for the CSR, or
// (new column, new row) for the CSC; the payload is the entry's index in A.
template <bool kByCol>
__global__ __launch_bounds__(kT) void entry_keys(int64_t n, const int64_t* __restrict__ rp,
                                                 const int32_t* __restrict__ ci,
                                                 const int32_t* __restrict__ inv, int bits,
                                                 unsigned long long* __restrict__ key,
                                                 int32_t* __restrict__ idx) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t o = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) >> 6; o < n; o += nw) {
    const unsigned long long r = (unsigned long long)inv[o];
    for (int64_t k = rp[o] + lane; k < rp[o + 1]; k += 64) {
      const unsigned long long c = (unsigned long long)inv[ci[k]];
      key[k] = kByCol ? ((c << bits) | r) : ((r << bits) | c);
      idx[k] = (int32_t)k;
    }
  }
}

// Sorted keys -> index array (the low field).
__global__ void key_low(int64_t nnz, const unsigned long long* __restrict__ key,
                        unsigned long long mask, int32_t* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nnz; t += stride)
    out[t] = (int32_t)(key[t] & mask);
}

// Values of P A P^T through the maps: out_r[t] = v[mr[t]], out_c[t] = v[mc[t]].
__global__ void gather_values(int64_t nnz, const double* __restrict__ v,
                              const int32_t* __restrict__ mr, const int32_t* __restrict__ mc,
                              double* __restrict__ out_r, double* __restrict__ out_c) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nnz; t += stride) {
    out_r[t] = v[mr[t]];
    out_c[t] = v[mc[t]];
  }
}

// Values finite (bit 4 of bad otherwise) and max |v|.
__global__ __launch_bounds__(kT) void values_check(int64_t nnz, const double* __restrict__ v,
                                                   int* __restrict__ bad,
                                                   unsigned long long* __restrict__ amax) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int f = 0;
  double mx = 0.0;
  for (int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; t < nnz; t += stride) {
    const double x = v[t];
    if (!isfinite(x)) f = 4;
    else mx = fmax(mx, fabs(x));
  }
  for (int o = 32; o; o >>= 1) {
    f |= __shfl_xor(f, o);
    mx = fmax(mx, __shfl_xor(mx, o));
  }
  __shared__ int sf[kT / 64];
  __shared__ double sm[kT / 64];
  const int lane = threadIdx.x & 63;
  if (lane == 0) {
    sf[threadIdx.x >> 6] = f;
    sm[threadIdx.x >> 6] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kT / 64; ++w) {
      f |= sf[w];
      mx = fmax(mx, sm[w]);
    }
    if (f) atomicOr(bad, f);
    if (mx > 0.0) atomicMax(amax, (unsigned long long)__double_as_longlong(mx));
  }
}

int flat_grid(int64_t items) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((items + kT - 1) / kT, 16384));
}

// Host candidate search of one seed (a row past the LDS table): the same test
// over A1's pattern, rows ascending.
void host_candidates(int64_t i, const std::vector<int64_t>& rp1, const std::vector<int32_t>& ci1,
                     const std::vector<int64_t>& cp1, const std::vector<int32_t>& ri1,
                     const std::vector<uint8_t>& skip, double eps, std::vector<int32_t>& hits,
                     std::vector<int32_t>& out) {
  const bool int_test = (eps == 0.8);
  std::vector<int32_t> seen;
  for (int64_t k = rp1[i]; k < rp1[i + 1]; ++k) {
    const int32_t c = ci1[k];
    for (int64_t m = cp1[c]; m < cp1[c + 1]; ++m) {
      const int32_t j = ri1[m];
      if (j <= i || skip[j]) continue;
      if (hits[j]++ == 0) seen.push_back(j);
    }
  }
  std::sort(seen.begin(), seen.end());
  const int64_t rci = rp1[i + 1] - rp1[i];
  out.clear();
  for (int32_t j : seen) {
    const int64_t ov = hits[j];
    hits[j] = 0;
    const int64_t rcj = rp1[j + 1] - rp1[j];
    const bool ok = int_test ? (5 * ov * ov >= 4 * rci * rcj)
                             : (double(ov) * ov >= eps * double(rci) * double(rcj));
    if (ok) out.push_back(j);
  }
}

}  // namespace

bilu_status analyze_device(bilu_handle* h, int64_t n, const int64_t* d_a_rp,
                           const int32_t* d_a_ci, const double* d_a_v, const int64_t* rowptr) {
  if (n <= 0 || !rowptr || !d_a_rp || !d_a_ci || !d_a_v)
    return fail(h, BILU_ERR_INVALID, "null CSR or n<=0");
  if (n > INT32_MAX - 1) return fail(h, BILU_ERR_INVALID, "n exceeds int32 range");
  if (rowptr[0] != 0) return fail(h, BILU_ERR_INVALID, "rowptr[0] != 0");
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return fail(h, BILU_ERR_INVALID, "rowptr not monotone");
  const int64_t nnz = rowptr[n];
  if (nnz > INT32_MAX) return fail(h, BILU_ERR_INVALID, "the device analyze takes nnz < 2^31");
  hipStream_t st = h->stream;
#define CK(x)                                          \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return hip_check(h, e_, #x); \
  } while (0)

  // 1. entries
  DevArray<int> d_bad;
  DevArray<unsigned long long> d_amax;
  DevArray<int32_t> d_cc;
  CK(d_bad.alloc(1));
  CK(d_amax.alloc(1));
  CK(d_cc.alloc(n));
  CK(hipMemsetAsync(d_bad.p, 0, sizeof(int), st));
  CK(hipMemsetAsync(d_amax.p, 0, sizeof(unsigned long long), st));
  CK(hipMemsetAsync(d_cc.p, 0, n * sizeof(int32_t), st));
  if (nnz > 0) {
    entries_check<<<stream_grid(n), kT, 0, st>>>(n, d_a_rp, d_a_ci, d_a_v, d_bad.p, d_amax.p,
                                                  d_cc.p);
    CK(hipGetLastError());
  }
  int bad = 0;
  unsigned long long amax = 0;
  std::vector<int32_t> ccount(n);
  CK(hipMemcpyAsync(&bad, d_bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(&amax, d_amax.p, sizeof(amax), hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(ccount.data(), d_cc.p, n * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (bad & 1) return fail(h, BILU_ERR_INVALID, "column index out of range");
  if (bad & 2) return fail(h, BILU_ERR_INVALID, "column indices not strictly increasing");
  if (bad & 4) return fail(h, BILU_ERR_INVALID, "non-finite value");
  h->n = n;
  h->nnz = nnz;
  double alpha;
  std::memcpy(&alpha, &amax, sizeof(alpha));
  h->alpha = alpha;
  h->prp.clear();
  h->pci.clear();
  h->pv.clear();
  h->pcp.clear();
  h->pri.clear();
  h->pcv.clear();

  std::vector<int64_t> pre;
  if (!pre_permutation(h, n, pre)) return fail(h, BILU_ERR_INVALID, "pre_perm is not a permutation");
  const bool ident = h->opt.pre_perm == nullptr;

  // 2. A1 = A(pre, pre), when the cosine step or the ordering reads it
  const bool need_nd =
      h->opt.ordering == BILU_ORDER_ND || h->opt.ordering == BILU_ORDER_ND_MULTILEVEL;
  std::vector<int64_t> rp1(n + 1, 0), cp1(n + 1, 0);
  DevArray<int32_t> d_pre, d_inv, d_ci1, d_ri1;
  DevArray<int64_t> d_rp1, d_cp1;
  DevArray<unsigned long long> d_fill;
  const int32_t* ci1 = d_a_ci;
  const int64_t* drp1 = d_a_rp;
  if (h->opt.use_cosine || need_nd) {
    for (int64_t r = 0; r < n; ++r) rp1[r + 1] = rp1[r] + (rowptr[pre[r] + 1] - rowptr[pre[r]]);
    if (!ident) {
      std::vector<int32_t> p32(n);
      for (int64_t i = 0; i < n; ++i) p32[i] = (int32_t)pre[i];
      CK(d_pre.alloc(n));
      CK(d_inv.alloc(n));
      CK(d_rp1.alloc(n + 1));
      CK(d_ci1.alloc(std::max<int64_t>(1, nnz)));
      CK(hipMemcpyAsync(d_pre.p, p32.data(), n * 4, hipMemcpyHostToDevice, st));
      CK(hipMemcpyAsync(d_rp1.p, rp1.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
      invert_perm<<<flat_grid(n), kT, 0, st>>>(n, d_pre.p, d_inv.p);
      gather_rows<<<stream_grid(n), kT, 0, st>>>(n, d_a_rp, d_a_ci, d_pre.p, d_inv.p, d_rp1.p,
                                                  d_ci1.p);
      CK(hipGetLastError());
      CK(hipStreamSynchronize(st));  // the host staging arrays end here
      ci1 = d_ci1.p;
      drp1 = d_rp1.p;
    }
  }

  // 3. cosine groups
  std::vector<int64_t> q, gs;
  std::vector<int32_t> ci1_h;  // A1's rows on the host, when needed
  if (h->opt.use_cosine) {
    std::vector<int64_t> rc(n), cc(n);
    for (int64_t i = 0; i < n; ++i) {
      rc[i] = rp1[i + 1] - rp1[i];
      cc[i] = ccount[pre[i]];
    }
    for (int64_t i = 0; i < n; ++i) cp1[i + 1] = cp1[i] + cc[i];
    double lim_r, lim_c;
    cosine_limits(n, nnz, rc.data(), cc.data(), &lim_r, &lim_c);
    std::vector<uint8_t> skip(n);
    for (int64_t i = 0; i < n; ++i) skip[i] = rc[i] > lim_r || cc[i] > lim_c;
    DevArray<uint8_t> d_skip;
    DevArray<int32_t> d_cnt;
    CK(d_skip.alloc(n));
    CK(d_cnt.alloc(n));
    CK(d_cp1.alloc(n + 1));
    CK(d_fill.alloc(n + 1));
    CK(d_ri1.alloc(std::max<int64_t>(1, nnz)));
    CK(hipMemcpyAsync(d_skip.p, skip.data(), n, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(d_cp1.p, cp1.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(d_fill.p, cp1.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
    const int64_t* rp1d = drp1;  // A's own rowptr when pre is the identity
    scatter_cols<<<stream_grid(n), kT, 0, st>>>(n, rp1d, ci1, d_fill.p, d_ri1.p);
    CK(hipGetLastError());
    CosArgs ca{};
    ca.n = n;
    ca.rp1 = rp1d;
    ca.ci1 = ci1;
    ca.cp1 = d_cp1.p;
    ca.ri1 = d_ri1.p;
    ca.skip = d_skip.p;
    ca.int_test = h->opt.cos_eps == 0.8;
    ca.eps = h->opt.cos_eps;
    ca.cnt = d_cnt.p;
    const int cgrid = (int)std::min<int64_t>(n, 16384);
    cos_rows<false><<<cgrid, 64, 0, st>>>(ca);
    CK(hipGetLastError());
    std::vector<int32_t> cnt(n);
    CK(hipMemcpyAsync(cnt.data(), d_cnt.p, n * 4, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    std::vector<int64_t> off(n + 1, 0);
    std::vector<int64_t> over;
    for (int64_t i = 0; i < n; ++i) {
      if (cnt[i] < 0) over.push_back(i);
      off[i + 1] = off[i] + std::max(0, cnt[i]);
    }
    const int64_t total = off[n];
    std::vector<int32_t> list(total);
    if (total > 0) {
      DevArray<int64_t> d_off;
      DevArray<int32_t> d_out;
      CK(d_off.alloc(n + 1));
      CK(d_out.alloc(total));
      CK(hipMemcpyAsync(d_off.p, off.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
      ca.off = d_off.p;
      ca.out = d_out.p;
      cos_rows<true><<<cgrid, 64, 0, st>>>(ca);
      CK(hipGetLastError());
      CK(hipMemcpyAsync(list.data(), d_out.p, total * 4, hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
    }
    // seeds past the LDS table: the host, from A1's pattern
    std::vector<std::vector<int32_t>> over_list(over.size());
    if (!over.empty()) {
      ci1_h.resize(nnz);
      std::vector<int32_t> ri1_h(nnz);
      CK(hipMemcpyAsync(ci1_h.data(), ci1, nnz * 4, hipMemcpyDeviceToHost, st));
      CK(hipMemcpyAsync(ri1_h.data(), d_ri1.p, nnz * 4, hipMemcpyDeviceToHost, st));
      CK(hipStreamSynchronize(st));
      std::vector<int32_t> hits(n, 0);
      for (size_t t = 0; t < over.size(); ++t)
        host_candidates(over[t], rp1, ci1_h, cp1, ri1_h, skip, h->opt.cos_eps, hits, over_list[t]);
    }
    // greedy replay: seeds ascending, members ascending, at most max_block
    std::vector<char> taken(n, 0);
    q.reserve(n);
    gs.assign(1, 0);
    size_t ov_at = 0;
    for (int64_t i = 0; i < n; ++i) {
      const int32_t* L = list.data() + off[i];
      int64_t len = off[i + 1] - off[i];
      if (ov_at < over.size() && over[ov_at] == i) {
        L = over_list[ov_at].data();
        len = (int64_t)over_list[ov_at].size();
        ++ov_at;
      }
      if (taken[i]) continue;
      taken[i] = 1;
      q.push_back(i);
      int members = 1;
      for (int64_t k = 0; k < len && members < h->opt.max_block; ++k) {
        const int32_t j = L[k];
        if (taken[j]) continue;
        taken[j] = 1;
        q.push_back(j);
        ++members;
      }
      gs.push_back((int64_t)q.size());
    }
  } else {
    q.resize(n);
    std::iota(q.begin(), q.end(), 0);
    gs.resize(n + 1);
    std::iota(gs.begin(), gs.end(), 0);
  }

  // ordering of the groups and the expansion (host)
  const int64_t ng = (int64_t)gs.size() - 1;
  if (need_nd && ng > 8 && ci1_h.empty()) {
    ci1_h.resize(nnz);
    CK(hipMemcpyAsync(ci1_h.data(), ci1, nnz * 4, hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
  }
  const bilu_status os =
      order_and_expand(h, rp1.data(), ci1_h.empty() ? nullptr : ci1_h.data(), pre, q, gs);
  if (os != BILU_OK) return os;

  // 4. P A P^T, CSR and CSC
  std::vector<int64_t> prp(n + 1, 0), pcp(n + 1, 0);
  std::vector<int32_t> perm32(n);
  for (int64_t r = 0; r < n; ++r) {
    const int64_t o = h->perm[r];
    perm32[r] = (int32_t)o;
    prp[r + 1] = prp[r] + (rowptr[o + 1] - rowptr[o]);
    pcp[r + 1] = pcp[r] + ccount[o];
  }
  CK(h->d_rp.alloc(n + 1));
  CK(h->d_ci.alloc(nnz));
  CK(h->d_rv.alloc(nnz));
  CK(h->d_cp.alloc(n + 1));
  CK(h->d_ri.alloc(nnz));
  CK(h->d_cv.alloc(nnz));
  CK(h->d_perm.alloc(n));
  CK(hipMemcpyAsync(h->d_perm.p, perm32.data(), n * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(h->d_rp.p, prp.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(h->d_cp.p, pcp.data(), (n + 1) * 8, hipMemcpyHostToDevice, st));
  {
    const bilu_status ms = value_maps(h, d_a_rp, d_a_ci, true);
    if (ms != BILU_OK) return ms;
  }
  if (nnz > 0) {
    gather_values<<<flat_grid(nnz), kT, 0, st>>>(nnz, d_a_v, h->d_vmap_r.p, h->d_vmap_c.p,
                                                 h->d_rv.p, h->d_cv.p);
    CK(hipGetLastError());
  }
  CK(hipStreamSynchronize(st));
#undef CK
  return BILU_OK;
}

// For every position of the CSR (and of the CSC) of P A P^T the index of
// the entry of A it holds, from d_perm (new -> old) and A's pattern in device
// memory; with write_idx also the column (row) index arrays.  Two radix
// sorts of (row, column) and (column, row) keys, payload the entry index;
// the keys are unique, so CSR rows ascend by column and CSC columns by row.
bilu_status value_maps(bilu_handle* h, const int64_t* d_a_rp, const int32_t* d_a_ci,
                       bool write_idx) {
  const int64_t n = h->n, nnz = h->nnz;
  h->d_vmap_r.release();
  h->d_vmap_c.release();
  if (nnz > INT32_MAX) return BILU_OK;  // no maps: bilu_refactor reports it
  hipStream_t st = h->stream;
#define CK(x)                                          \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return hip_check(h, e_, #x); \
  } while (0)
  CK(h->d_vmap_r.alloc(std::max<int64_t>(1, nnz)));
  CK(h->d_vmap_c.alloc(std::max<int64_t>(1, nnz)));
  if (nnz == 0) return BILU_OK;
  const int nbits = std::max(1, 64 - __builtin_clzll((unsigned long long)std::max<int64_t>(1, n - 1)));
  DevArray<int32_t> d_inv, i_in;
  DevArray<unsigned long long> k_in, k_out;
  CK(d_inv.alloc(n));
  CK(k_in.alloc(nnz));
  CK(k_out.alloc(nnz));
  CK(i_in.alloc(nnz));
  invert_perm<<<flat_grid(n), kT, 0, st>>>(n, h->d_perm.p, d_inv.p);
  CK(hipGetLastError());
  const int end_bit = 2 * nbits;
  size_t tb = 0;
  CK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, k_in.p, k_out.p, i_in.p, h->d_vmap_r.p,
                                        (int)nnz, 0, end_bit, st));
  DevArray<char> tmp;
  CK(tmp.alloc(std::max<size_t>(tb, 1)));
  const unsigned long long mask = (1ull << nbits) - 1ull;
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 0)
      entry_keys<false><<<stream_grid(n), kT, 0, st>>>(n, d_a_rp, d_a_ci, d_inv.p, nbits, k_in.p,
                                                        i_in.p);
    else
      entry_keys<true><<<stream_grid(n), kT, 0, st>>>(n, d_a_rp, d_a_ci, d_inv.p, nbits, k_in.p,
                                                       i_in.p);
    CK(hipGetLastError());
    CK(hipcub::DeviceRadixSort::SortPairs(tmp.p, tb, k_in.p, k_out.p, i_in.p,
                                          pass == 0 ? h->d_vmap_r.p : h->d_vmap_c.p, (int)nnz, 0,
                                          end_bit, st));
    if (write_idx) {
      key_low<<<flat_grid(nnz), kT, 0, st>>>(nnz, k_out.p, mask, pass == 0 ? h->d_ci.p : h->d_ri.p);
      CK(hipGetLastError());
    }
  }
  CK(hipStreamSynchronize(st));  // the temporaries end here
#undef CK
  return BILU_OK;
}

// New values of the analyzed pattern (device array, A's own entry order)
// into P A P^T's CSR and CSC; max |a_ij| for the perturbation scale.
bilu_status refactor_values(bilu_handle* h, const double* d_val) {
  const int64_t nnz = h->nnz;
  hipStream_t st = h->stream;
#define CK(x)                                          \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return hip_check(h, e_, #x); \
  } while (0)
  DevArray<int> d_bad;
  DevArray<unsigned long long> d_amax;
  CK(d_bad.alloc(1));
  CK(d_amax.alloc(1));
  CK(hipMemsetAsync(d_bad.p, 0, sizeof(int), st));
  CK(hipMemsetAsync(d_amax.p, 0, sizeof(unsigned long long), st));
  if (nnz > 0) {
    values_check<<<flat_grid(nnz), kT, 0, st>>>(nnz, d_val, d_bad.p, d_amax.p);
    CK(hipGetLastError());
  }
  int bad = 0;
  unsigned long long amax = 0;
  CK(hipMemcpyAsync(&bad, d_bad.p, sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipMemcpyAsync(&amax, d_amax.p, sizeof(amax), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (bad) return fail(h, BILU_ERR_INVALID, "non-finite value");
  if (nnz > 0) {
    gather_values<<<flat_grid(nnz), kT, 0, st>>>(nnz, d_val, h->d_vmap_r.p, h->d_vmap_c.p,
                                                 h->d_rv.p, h->d_cv.p);
    CK(hipGetLastError());
  }
  CK(hipStreamSynchronize(st));
#undef CK
  double alpha;
  std::memcpy(&alpha, &amax, sizeof(alpha));
  h->alpha = alpha;
  h->prp.clear();          // host copies, if any, hold the old values
  h->ilu_static = false;   // so does the diagonal kept for ILU(1,tau)
  return BILU_OK;
}

// Host copies of the permuted matrix, for the host ILU(1,tau) step after a
// device analyze.
bilu_status ensure_host_matrix(bilu_handle* h) {
  if (!h->prp.empty()) return BILU_OK;
  const int64_t n = h->n, nnz = h->nnz;
  h->prp.resize(n + 1);
  h->pci.resize(nnz);
  h->pv.resize(nnz);
  h->pcp.resize(n + 1);
  h->pri.resize(nnz);
  h->pcv.resize(nnz);
  hipStream_t st = h->stream;
  hipError_t e = hipMemcpyAsync(h->prp.data(), h->d_rp.p, (n + 1) * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h->pcp.data(), h->d_cp.p, (n + 1) * 8, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess && nnz > 0) {
    e = hipMemcpyAsync(h->pci.data(), h->d_ci.p, nnz * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h->pv.data(), h->d_rv.p, nnz * 8, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h->pri.data(), h->d_ri.p, nnz * 4, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h->pcv.data(), h->d_cv.p, nnz * 8, hipMemcpyDeviceToHost, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) {
    h->prp.clear();
    return hip_check(h, e, "copy of the permuted matrix to the host");
  }
  return BILU_OK;
}

}  // namespace bilu
