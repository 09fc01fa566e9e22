// ILU(1,tau) guess of the initial block partition (Sec. 3.4) on the GPU.
//
// Sets.  For every scalar k of the permuted matrix, the estimated column set
// of L is
//   I~_k = { i > k : |a_ik| >= tau |a_kk| }
//        u { i > k : exists j < k with a_jk != 0, a_ij != 0 and
//                    |a_ij a_jk| >= tau |a_jj a_kk| },
// and the row set J~_k of U is the same with the roles of rows and columns
// exchanged.  One wave computes both sets of one k: it dedups the direct
// entries and the fill candidates in an LDS hash and writes them to a
// padded per-k slot.  A source j whose largest off-diagonal entry cannot
// pass the fill test with a_jk is skipped without reading its column (the
// bound is exact, so the sets do not change).
//
// Growth.  A block started at unit s (a cosine group) takes the next unit
// while the dense count f' = (r'+s'+l') l' stays within 4/3 of the scalar
// count c' or within c' + 4 l', where r' (s') counts the union of the
// blocks' sets beyond the new last index and c' sums |I~|+|J~|+1 over its
// columns.  Whether a unit joins depends only on where the block started,
// so one wave per unit s computes the end g(s) of a block started there;
// the host follows s -> g(s) from s = 0, which is the sequential rule.
//
// Real comparisons are the plain products and compares above (no fused
// operations), so the partition equals the sequential host computation bit
// for bit.  Capacity overflows are reported and the caller then computes
// the partition on the host.
#include <algorithm>
#include <chrono>
#include <cmath>

#include "internal.h"
#include "wg.h"

namespace bilu {
namespace {

constexpr int kSetCap = 96;        // entries of one set (per k and side)
constexpr int kSetHash = 256;      // LDS hash slots of one wave (sets)
constexpr int kSrcCap = 128;       // fill sources (entries before the diagonal)
constexpr int kCandBatch = 4;      // fill candidates per lane in flight
constexpr int kGrowHash = 512;     // LDS hash slots of one wave per side (growth)
constexpr int kWaves = 4;          // waves per workgroup

struct IluArgs {
  int n, nu, maxb;
  double tau;
  const int64_t* cp; const int32_t* ri; const double* cv;   // CSC
  const int64_t* rp; const int32_t* ci; const double* rv;   // CSR
  const double* dg;                // diagonal entries (0 when absent)
  const double* cmax;              // largest |a_ij|, i != j, of column j (CSC)
  const double* rmax;              // largest |a_ji|, i != j, of row j (CSR)
  const int64_t* gs;               // unit starts [nu+1]
  int32_t* iset; int32_t* jset;    // [n * kSetCap]
  int32_t* icnt; int32_t* jcnt;    // [n]
  int32_t* gend;                   // [nu]
  int* overflow;
};

__global__ void diag_kernel(int n, const int64_t* rp, const int32_t* ci, const double* rv,
                            double* dg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double d = 0.0;
  for (int64_t m = rp[i]; m < rp[i + 1]; ++m)
    if (ci[m] == i) d = rv[m];
  dg[i] = d;
}

// Sec. 5: both scalars of a 2x2 pivot (partner >= 0) take the pivot
// block's largest magnitude in place of their diagonal.
__global__ void pair_dg_kernel(int n, const int32_t* partner, const int64_t* rp, const int32_t* ci,
                               const double* rv, double* dg) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = partner[i];
  if (p < 0) return;
  auto at = [&](int r, int c) {
    int64_t lo = rp[r], hi = rp[r + 1];
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ci[mid] < c) lo = mid + 1; else hi = mid;
    }
    return lo < rp[r + 1] && ci[lo] == c ? fabs(rv[lo]) : 0.0;
  };
  dg[i] = fmax(fmax(at(i, i), at(p, p)), fmax(at(i, p), at(p, i)));
}

// Largest off-diagonal magnitude of every row (CSR) or column (CSC).
__global__ void offdiag_max_kernel(int n, const int64_t* ptr, const int32_t* idx, const double* val,
                                   double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double m = 0.0;
  for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e)
    if (idx[e] != i) m = fmax(m, fabs(val[e]));
  out[i] = m;
}

// Wave-local insert; false when the table is full.
__device__ __forceinline__ bool wave_insert(int* table, int slots, int key, int* count) {
  unsigned h = (unsigned(key) * 2654435761u) & (unsigned)(slots - 1);
  for (int probe = 0; probe < slots; ++probe) {
    const int old = atomicCAS(&table[h], -1, key);
    if (old == -1) {
      atomicAdd(count, 1);
      return true;
    }
    if (old == key) return true;
    h = (h + 1) & (unsigned)(slots - 1);
  }
  return false;
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

struct SetLds {
  int hash[kWaves][kSetHash];
  int src[kWaves][kSrcCap];        // fill source index j (L) / i (U)
  double srcv[kWaves][kSrcCap];    // a_jk (L) / a_ki (U)
  double srcd[kWaves][kSrcCap];    // a_jj of the source
  long long srcp[kWaves][kSrcCap]; // start of the source's column (row)
  int off[kWaves][kSrcCap + 1];    // prefix of the source lengths
  int misc[kWaves][4];
};

// One side of the sets of k: (ptr, idx, val) is the CSC for I~_k and the
// CSR for J~_k.  Writes the set to out[0..cnt) and returns cnt, or -1.
__device__ int one_set(const IluArgs& a, const int64_t* ptr, const int32_t* idx, const double* val,
                       const double* smax, int k, SetLds& s, int w, int32_t* out) {
  const int lane = threadIdx.x & 63;
  int* hash = s.hash[w];
  int* misc = s.misc[w];
  for (int t = lane; t < kSetHash; t += 64) hash[t] = -1;
  if (lane == 0) {
    misc[0] = 0;  // unique keys
    misc[1] = 0;  // overflow
    misc[2] = 0;  // sources
  }
  wave_sync();
  const double akk = fabs(a.dg[k]);
  const double dk = a.dg[k];
  const int64_t b = ptr[k], e = ptr[k + 1];
  for (int64_t m = b + lane; m < e; m += 64) {
    const int i = idx[m];
    const double v = val[m];
    if (i > k && fabs(v) >= a.tau * akk)
      if (!wave_insert(hash, kSetHash, i, &misc[0])) misc[1] = 1;
    // a source none of whose entries can pass the fill test is left out:
    // every candidate product is at most |smax_i v| in magnitude (rounding
    // is monotone), compared with the candidate test's own threshold
    if (i < k && fabs(smax[i] * v) >= a.tau * fabs(a.dg[i] * dk)) {
      const int o = atomicAdd(&misc[2], 1);
      if (o < kSrcCap) {
        s.src[w][o] = i;
        s.srcv[w][o] = v;
      } else {
        misc[1] = 1;
      }
    }
  }
  wave_sync();
  const int nsrc = min(misc[2], kSrcCap);
  // lengths of the sources' columns (rows), then a wave prefix
  int base = 0;
  for (int t0 = 0; t0 < nsrc; t0 += 64) {
    const int t = t0 + lane;
    int len = 0;
    if (t < nsrc) {
      const int j = s.src[w][t];
      const int64_t p0 = ptr[j];
      len = (int)(ptr[j + 1] - p0);
      s.srcp[w][t] = p0;
      s.srcd[w][t] = a.dg[j];
    }
    int incl = len;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o, 64);
      if (lane >= o) incl += y;
    }
    if (t < nsrc) s.off[w][t] = base + incl - len;
    base += __shfl(incl, 63, 64);
  }
  if (lane == 0) s.off[w][nsrc] = base;
  wave_sync();
  const int total = base;
  for (int x0 = 0; x0 < total; x0 += 64 * kCandBatch) {
    // sources first (LDS), then every candidate's loads, then the tests
    int iv[kCandBatch], sl[kCandBatch];
    double vv[kCandBatch];
#pragma unroll
    for (int u = 0; u < kCandBatch; ++u) {
      const int x = x0 + u * 64 + lane;
      sl[u] = -1;
      if (x < total) {
        // source t with off[t] <= x < off[t+1]
        int lo = 0, hi = nsrc;
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (s.off[w][mid] <= x)
            lo = mid;
          else
            hi = mid;
        }
        const int64_t m2 = s.srcp[w][lo] + (x - s.off[w][lo]);
        iv[u] = idx[m2];
        vv[u] = val[m2];
        sl[u] = lo;
      }
    }
#pragma unroll
    for (int u = 0; u < kCandBatch; ++u) {
      if (sl[u] < 0 || iv[u] <= k) continue;
      const double thr = a.tau * fabs(s.srcd[w][sl[u]] * dk);
      if (fabs(vv[u] * s.srcv[w][sl[u]]) >= thr)
        if (!wave_insert(hash, kSetHash, iv[u], &misc[0])) misc[1] = 1;
    }
  }
  wave_sync();
  const int cnt = misc[0];
  if (misc[1] || cnt > kSetCap) return -1;
  if (lane == 0) misc[3] = 0;
  wave_sync();
  for (int t = lane; t < kSetHash; t += 64) {
    const int key = hash[t];
    if (key >= 0) out[atomicAdd(&misc[3], 1)] = key;
  }
  wave_sync();
  return cnt;
}

__global__ void __launch_bounds__(64 * kWaves) ilu_sets_kernel(IluArgs a) {
  __shared__ SetLds s;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int k = blockIdx.x * kWaves + w; k < a.n; k += gridDim.x * kWaves) {
    const int ci_ = one_set(a, a.cp, a.ri, a.cv, a.cmax, k, s, w, a.iset + (int64_t)k * kSetCap);
    const int cj_ = one_set(a, a.rp, a.ci, a.rv, a.rmax, k, s, w, a.jset + (int64_t)k * kSetCap);
    if (lane == 0) {
      a.icnt[k] = ci_;
      a.jcnt[k] = cj_;
      if (ci_ < 0 || cj_ < 0) atomicExch(a.overflow, 1);
    }
  }
}

// Growth hash: committed key x >= 0, tentative key stored as -x-2, empty -1.
__device__ __forceinline__ int grow_insert(int* table, int key) {
  unsigned h = (unsigned(key) * 2654435761u) & (unsigned)(kGrowHash - 1);
  const int tent = -key - 2;
  for (int probe = 0; probe < kGrowHash; ++probe) {
    const int old = atomicCAS(&table[h], -1, tent);
    if (old == -1 || old == key || old == tent) return 1;
    h = (h + 1) & (unsigned)(kGrowHash - 1);
  }
  return 0;
}

struct GrowLds {
  int rows[kWaves][kGrowHash];
  int cols[kWaves][kGrowHash];
  int misc[kWaves][4];
};

__global__ void __launch_bounds__(64 * kWaves) ilu_grow_kernel(IluArgs a) {
  __shared__ GrowLds s;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int* R = s.rows[w];
  int* Cc = s.cols[w];
  int* misc = s.misc[w];
  for (int u0 = blockIdx.x * kWaves + w; u0 < a.nu; u0 += gridDim.x * kWaves) {
    for (int t = lane; t < kGrowHash; t += 64) {
      R[t] = -1;
      Cc[t] = -1;
    }
    if (lane == 0) misc[0] = 0;  // overflow
    wave_sync();
    const int64_t s0 = a.gs[u0];
    long long scal = 0;
    int u = u0;
    bool first = true;
    while (u < a.nu) {
      const int64_t e2 = a.gs[u + 1];
      const int64_t w2 = e2 - s0;
      if (!first && w2 > a.maxb) break;
      // the unit's entries, tentative
      long long sc2 = scal;
      for (int64_t k = a.gs[u]; k < e2; ++k) {
        const int ni = a.icnt[k], nj = a.jcnt[k];
        for (int t = lane; t < ni + nj; t += 64) {
          const bool row = t < ni;
          const int key = row ? a.iset[k * kSetCap + t] : a.jset[k * kSetCap + t - ni];
          if (!grow_insert(row ? R : Cc, key)) misc[0] = 1;
        }
        sc2 += ni + nj + 1;
      }
      wave_sync();
      if (misc[0]) break;
      bool grow = true;
      if (!first) {
        // union beyond the new last index
        const int last = (int)(e2 - 1);
        int r2 = 0, c2 = 0;
        for (int t = lane; t < kGrowHash; t += 64) {
          const int x = R[t], y = Cc[t];
          r2 += (x >= 0 ? x : -x - 2) > last && x != -1;
          c2 += (y >= 0 ? y : -y - 2) > last && y != -1;
        }
        r2 = wave_sum(r2);
        c2 = wave_sum(c2);
        const long long f2 = ((long long)r2 + c2 + w2) * w2;
        grow = 3 * f2 <= 4 * sc2 || f2 <= sc2 + 4 * w2;
      }
      if (!grow) break;
      // commit the unit
      for (int t = lane; t < kGrowHash; t += 64) {
        if (R[t] < -1) R[t] = -R[t] - 2;
        if (Cc[t] < -1) Cc[t] = -Cc[t] - 2;
      }
      wave_sync();
      scal = sc2;
      first = false;
      ++u;
    }
    if (lane == 0) {
      a.gend[u0] = u;
      if (misc[0]) atomicExch(a.overflow, 1);
    }
    wave_sync();
  }
}

}  // namespace

// Device ILU(1,tau) partition.  Returns the block count, or -1 when a set or
// a growing block exceeded the kernel capacities (the caller then uses the
// host computation).  t_sets receives the wall time of the set kernel.
int64_t ilu1t_partition_device(bilu_handle* h, double tau, std::vector<int32_t>& bstart,
                               double* t_sets) {
  using clk = std::chrono::steady_clock;
  const auto t0 = clk::now();
  const int64_t n = h->n;
  const auto& gs = h->group_starts;
  const int64_t nu = (int64_t)gs.size() - 1;
  hipStream_t st = h->stream;
  // the unit starts and the diagonal depend on the analyzed matrix only
  if (!h->ilu_static) {
    if (h->d_ilu_gs.alloc(gs.size()) != hipSuccess || h->d_ilu_dg.alloc(3 * n) != hipSuccess ||
        hipMemcpyAsync(h->d_ilu_gs.p, gs.data(), gs.size() * sizeof(int64_t), hipMemcpyHostToDevice,
                       st) != hipSuccess)
      return -1;
    diag_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>((int)n, h->d_rp.p, h->d_ci.p, h->d_rv.p,
                                                             h->d_ilu_dg.p);
    if (!h->sym_partner.empty()) {
      if (h->d_partner.alloc(n) != hipSuccess ||
          hipMemcpyAsync(h->d_partner.p, h->sym_partner.data(), n * sizeof(int32_t),
                         hipMemcpyHostToDevice, st) != hipSuccess)
        return -1;
      pair_dg_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
          (int)n, h->d_partner.p, h->d_rp.p, h->d_ci.p, h->d_rv.p, h->d_ilu_dg.p);
    }
    offdiag_max_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
        (int)n, h->d_cp.p, h->d_ri.p, h->d_cv.p, h->d_ilu_dg.p + n);
    offdiag_max_kernel<<<(unsigned)((n + 255) / 256), 256, 0, st>>>(
        (int)n, h->d_rp.p, h->d_ci.p, h->d_rv.p, h->d_ilu_dg.p + 2 * n);
    if (hipGetLastError() != hipSuccess) return -1;
    h->ilu_static = true;
  }
  if (h->d_ilu_set.alloc(2 * n * kSetCap) != hipSuccess ||
      h->d_ilu_cnt.alloc(2 * n + nu + 1) != hipSuccess)
    return -1;
  IluArgs a{};
  a.n = (int)n;
  a.nu = (int)nu;
  a.maxb = h->opt.max_block;
  a.tau = tau;
  a.cp = h->d_cp.p; a.ri = h->d_ri.p; a.cv = h->d_cv.p;
  a.rp = h->d_rp.p; a.ci = h->d_ci.p; a.rv = h->d_rv.p;
  a.dg = h->d_ilu_dg.p;
  a.cmax = h->d_ilu_dg.p + n;
  a.rmax = h->d_ilu_dg.p + 2 * n;
  a.gs = h->d_ilu_gs.p;
  a.iset = h->d_ilu_set.p;
  a.jset = h->d_ilu_set.p + n * kSetCap;
  a.icnt = h->d_ilu_cnt.p;
  a.jcnt = h->d_ilu_cnt.p + n;
  a.gend = h->d_ilu_cnt.p + 2 * n;
  a.overflow = h->d_ilu_cnt.p + 2 * n + nu;
  if (hipMemsetAsync(a.overflow, 0, sizeof(int), st) != hipSuccess) return -1;
  const unsigned g1 = (unsigned)std::min<int64_t>((n + kWaves - 1) / kWaves, 65536);
  ilu_sets_kernel<<<g1, 64 * kWaves, 0, st>>>(a);
  if (hipStreamSynchronize(st) != hipSuccess) return -1;
  const auto t1 = clk::now();
  if (t_sets) *t_sets = std::chrono::duration<double>(t1 - t0).count();
  const unsigned g2 = (unsigned)std::min<int64_t>((nu + kWaves - 1) / kWaves, 65536);
  ilu_grow_kernel<<<g2, 64 * kWaves, 0, st>>>(a);
  std::vector<int32_t> gend(nu + 1);
  if (hipMemcpyAsync(gend.data(), a.gend, (nu + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, st) !=
          hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess)
    return -1;
  if (gend[nu] != 0) return -1;  // overflow flag
  bstart.assign(1, 0);
  for (int64_t u = 0; u < nu;) {
    const int64_t g = gend[u];
    if (g <= u || g > nu) return -1;
    bstart.push_back((int32_t)gs[g]);
    u = g;
  }
  return (int64_t)bstart.size() - 1;
}

}  // namespace bilu
