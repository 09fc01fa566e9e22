// Kept-pattern residual of the sweep's factor (before aggregation):
//
//   r_kept = ||(L S U - A)_Omega||_F / ||A||_F,
//
// Omega the stored positions: every diagonal block K x K, R_K x K and
// K x C_K.  In exact arithmetic the Crout step of Sec. 2.2 reproduces A on
// exactly these positions (the updates it subtracts are the products L S U
// leaves there), so r_kept measures rounding, the precision of the stored
// L and W and of the Schur updates, and perturbed pivot blocks; dropped
// positions are not counted.  With U = D W, L S U on Omega is
//   column panel (i >= first(K), j in K):
//     sum over J < K of L_J(i,:) W_J(:,j)  +  [i in K] S_K(i,j)
//                                          +  [i in R_K] L_K(i,:) S_K(:,j)
//   row panel (i in K, j in C_K):
//     sum over J < K of L_J(i,:) W_J(:,j)  +  W_K(i,j).
// One workgroup per block K builds both panels in FP64 from the stored
// factor (predecessors in ascending order, each term to its own position:
// the sum is deterministic), then one partial sum of squares per block;
// the partials and ||A||_F^2 are reduced in a fixed order.
#include <algorithm>
#include <cmath>

#include <hipcub/hipcub.hpp>

#include "internal.h"

namespace bilu {
namespace {

constexpr int kKeptThreads = 256;
constexpr int kKeptGroups = 2048;

struct KeptArgs {
  FactorView f;                       // the sweep's factor
  const double* sval;                 // S_K = D_K^{-1}, q x q row-major at f.doff
  const int64_t* rp; const int32_t* ci; const double* rv;  // permuted A, CSR
  const int64_t* cp; const int32_t* ri; const double* cv;  // and CSC
  // column predecessors of K: J (ascending) with C_J[s0, s0 + cnt) inside K
  const int32_t* cptr; const int32_t* cj; const int32_t* cs0; const int32_t* ccnt;
  // row predecessors of K: J (ascending) with R_J[s0, s0 + cnt) inside K
  const int32_t* rptr; const int32_t* rj; const int32_t* rs0; const int32_t* rcnt;
  double* scratch; int64_t slot;      // per workgroup: (q + |R_K|) q + q |C_K| doubles
  double* partial;                    // [nb] sums of squares
};

__device__ __forceinline__ int find_index(const int32_t* lst, int cnt, int x) {
  int lo = 0, hi = cnt;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (lst[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return (lo < cnt && lst[lo] == x) ? lo : -1;
}
__device__ __forceinline__ int first_at_least(const int32_t* lst, int cnt, int x) {
  int lo = 0, hi = cnt;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (lst[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// sum over t < p of L(lo + t) W(wo + t), stored values widened to FP64
__device__ __forceinline__ double dot_stored(const FactorView& f, int64_t lo, int64_t wo, int p) {
  double acc = 0.0;
  for (int t = 0; t < p; ++t) acc = fma(value_load(f.val, f.vprec, lo + t), value_load(f.val, f.vprec, wo + t), acc);
  return acc;
}

__global__ void __launch_bounds__(kKeptThreads) kept_kernel(KeptArgs a) {
  __shared__ double red[kKeptThreads / 64];
  const int tid = threadIdx.x, nt = blockDim.x;
  const FactorView& f = a.f;
  double* P = a.scratch + (int64_t)blockIdx.x * a.slot;
  for (int K = blockIdx.x; K < f.nb; K += gridDim.x) {
    const int fK = f.bstart[K], q = f.bstart[K + 1] - fK, lK = fK + q - 1;
    const int nrK = f.nr[K], ncK = f.nc[K];
    const int32_t* RK = f.idx + f.roff[K];
    const int32_t* CK = f.idx + f.coff[K];
    double* Cp = P;                          // (q + nrK) x q, row-major
    double* Rp = P + (int64_t)(q + nrK) * q; // column z of the row panel: Rp[z q + r]
    const int64_t np_ = (int64_t)(q + nrK) * q + (int64_t)q * ncK;
    for (int64_t e = tid; e < np_; e += nt) P[e] = 0.0;
    __syncthreads();
    // A on Omega
    for (int c = 0; c < q; ++c)
      for (int64_t m = a.cp[fK + c] + tid; m < a.cp[fK + c + 1]; m += nt) {
        const int i = a.ri[m];
        if (i < fK) continue;
        const int z = i <= lK ? i - fK : (nrK ? find_index(RK, nrK, i) : -1);
        if (z < 0) continue;
        Cp[(int64_t)(i <= lK ? z : q + z) * q + c] = a.cv[m];
      }
    for (int r = 0; r < q; ++r)
      for (int64_t m = a.rp[fK + r] + tid; m < a.rp[fK + r + 1]; m += nt) {
        const int j = a.ci[m];
        if (j <= lK) continue;
        const int z = find_index(CK, ncK, j);
        if (z >= 0) Rp[(int64_t)z * q + r] = a.rv[m];
      }
    __syncthreads();
    // column predecessors, ascending: L_J(i,:) W_J(:,j), i >= first(K), j in K
    for (int e = a.cptr[K]; e < a.cptr[K + 1]; ++e) {
      const int J = a.cj[e], c0 = a.cs0[e], cc = a.ccnt[e];
      const int pJ = f.bstart[J + 1] - f.bstart[J];
      const int nrJ = f.nr[J];
      const int32_t* RJ = f.idx + f.roff[J];
      const int32_t* CJ = f.idx + f.coff[J];
      const int r_lo = first_at_least(RJ, nrJ, fK);
      const int work = (nrJ - r_lo) * cc;
      for (int w = tid; w < work; w += nt) {
        const int rix = r_lo + w / cc, cix = c0 + w % cc;
        const int i = RJ[rix];
        const int z = i <= lK ? i - fK : (nrK ? find_index(RK, nrK, i) : -1);
        if (z < 0) continue;
        const double t = dot_stored(f, f.loff[J] + (int64_t)rix * pJ, f.woff[J] + (int64_t)cix * pJ, pJ);
        Cp[(int64_t)(i <= lK ? z : q + z) * q + (CJ[cix] - fK)] -= t;
      }
      __syncthreads();
    }
    // K's own term: S_K on the diagonal block, L_K S_K below it
    const double* SK = a.sval + f.doff[K];
    for (int e = tid; e < (q + nrK) * q; e += nt) {
      const int z = e / q, c = e % q;
      double t;
      if (z < q) {
        t = SK[z * q + c];
      } else {
        t = 0.0;
        const int64_t lo = f.loff[K] + (int64_t)(z - q) * q;
        for (int k = 0; k < q; ++k) t = fma(value_load(f.val, f.vprec, lo + k), SK[k * q + c], t);
      }
      Cp[e] -= t;
    }
    // row predecessors, ascending: L_J(i,:) W_J(:,j), i in K, j in C_K
    for (int e = a.rptr[K]; e < a.rptr[K + 1]; ++e) {
      const int J = a.rj[e], r0 = a.rs0[e], rc = a.rcnt[e];
      const int pJ = f.bstart[J + 1] - f.bstart[J];
      const int ncJ = f.nc[J];
      const int32_t* RJ = f.idx + f.roff[J];
      const int32_t* CJ = f.idx + f.coff[J];
      const int c_lo = first_at_least(CJ, ncJ, lK + 1);
      const int work = rc * (ncJ - c_lo);
      for (int w = tid; w < work; w += nt) {
        const int rix = r0 + w % rc, cix = c_lo + w / rc;
        const int z = find_index(CK, ncK, CJ[cix]);
        if (z < 0) continue;
        const double t = dot_stored(f, f.loff[J] + (int64_t)rix * pJ, f.woff[J] + (int64_t)cix * pJ, pJ);
        Rp[(int64_t)z * q + (RJ[rix] - fK)] -= t;
      }
      __syncthreads();
    }
    // K's own term: W_K (q x |C_K| column-major, the layout of Rp)
    for (int64_t e = tid; e < (int64_t)q * ncK; e += nt) Rp[e] -= value_load(f.val, f.vprec, f.woff[K] + e);
    __syncthreads();
    double acc = 0.0;
    for (int64_t e = tid; e < np_; e += nt) acc = fma(P[e], P[e], acc);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((tid & 63) == 0) red[tid >> 6] = acc;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < nt / 64; ++w) s += red[w];
      a.partial[K] = s;
    }
    __syncthreads();
  }
}

struct Square {
  __host__ __device__ double operator()(double x) const { return x * x; }
};

}  // namespace

bilu_status kept_residual(bilu_handle* h, double* out) {
  hipStream_t st = h->stream;
  const int64_t nb = (int64_t)h->bstart0.size() - 1;
#define CK(x)                                          \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return hip_check(h, e_, #x); \
  } while (0)
  // the sweep's factor: the handle's per-block arrays and heaps (aggregation
  // writes the merged factor elsewhere)
  FactorView f{};
  f.nb = (int)nb;
  f.bstart = h->d_bstart.p;
  f.blockOf = h->d_blockof.p;
  f.nr = h->d_nr.p;
  f.nc = h->d_nc.p;
  f.roff = h->d_roff.p;
  f.coff = h->d_coff.p;
  f.loff = h->d_loff.p;
  f.woff = h->d_woff.p;
  f.doff = h->d_doff.p;
  f.idx = h->d_idx_heap.p;
  f.val = h->d_val_heap.p;
  f.vprec = h->opt.update_precision;
  f.dval = h->d_dval.p;
  DevArray<int32_t> cptr, cj, cs0, ccnt, rptr, rj, rs0, rcnt;
  bilu_status s = block_runs(h, f, true, cptr, cj, cs0, ccnt);
  if (s != BILU_OK) return s;
  s = block_runs(h, f, false, rptr, rj, rs0, rcnt);
  if (s != BILU_OK) return s;
  // panel sizes
  std::vector<int32_t> nr(nb), nc(nb);
  CK(hipMemcpy(nr.data(), h->d_nr.p, nb * 4, hipMemcpyDeviceToHost));
  CK(hipMemcpy(nc.data(), h->d_nc.p, nb * 4, hipMemcpyDeviceToHost));
  int64_t slot = 1;
  for (int64_t k = 0; k < nb; ++k) {
    const int64_t q = h->bstart0[k + 1] - h->bstart0[k];
    slot = std::max<int64_t>(slot, (q + nr[k]) * q + q * nc[k]);
  }
  const int64_t groups = std::max<int64_t>(1, std::min<int64_t>(nb, kKeptGroups));
  DevArray<double> scratch, partial, sums;
  CK(scratch.alloc(groups * slot));
  CK(partial.alloc(nb));
  CK(sums.alloc(2));
  KeptArgs a{};
  a.f = f;
  a.sval = h->d_sval.p;
  a.rp = h->d_rp.p; a.ci = h->d_ci.p; a.rv = h->d_rv.p;
  a.cp = h->d_cp.p; a.ri = h->d_ri.p; a.cv = h->d_cv.p;
  a.cptr = cptr.p; a.cj = cj.p; a.cs0 = cs0.p; a.ccnt = ccnt.p;
  a.rptr = rptr.p; a.rj = rj.p; a.rs0 = rs0.p; a.rcnt = rcnt.p;
  a.scratch = scratch.p;
  a.slot = slot;
  a.partial = partial.p;
  kept_kernel<<<(unsigned)groups, kKeptThreads, 0, st>>>(a);
  CK(hipGetLastError());
  size_t bytes = 0;
  hipcub::TransformInputIterator<double, Square, const double*> sq(h->d_rv.p, Square{});
  CK(hipcub::DeviceReduce::Sum(nullptr, bytes, partial.p, sums.p, (int)nb, st));
  size_t bytes2 = 0;
  CK(hipcub::DeviceReduce::Sum(nullptr, bytes2, sq, sums.p + 1, (int)h->nnz, st));
  CK(h->d_scan_tmp.alloc(std::max(bytes, bytes2) + 1));
  CK(hipcub::DeviceReduce::Sum(h->d_scan_tmp.p, bytes, partial.p, sums.p, (int)nb, st));
  CK(hipcub::DeviceReduce::Sum(h->d_scan_tmp.p, bytes2, sq, sums.p + 1, (int)h->nnz, st));
  double hs[2];
  CK(hipMemcpyAsync(hs, sums.p, sizeof(hs), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  *out = hs[1] > 0.0 ? std::sqrt(hs[0] / hs[1]) : 0.0;
  h->stats.r_kept = *out;
  return BILU_OK;
#undef CK
}

}  // namespace bilu
