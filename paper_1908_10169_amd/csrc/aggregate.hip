// Progressive aggregation (Sec. 3.5) of consecutive blocks, after the sweep.
//
// Decision.  After step K the live block P (blocks a..K-1 merged so far) and
// K merge when nu <= 1.2 mu or nu <= mu + 2(p+q) (integer form 5 nu <= 6 mu),
// and p+q <= max_block, with
//   mu = p (p + r + s + r' + s') + q (q + t + t'),   nu = (p+q)(p+q+u+v),
// r, s the rows of L_P inside / below K, t = |R_K|, u the size of the union
// of P's rows below K with R_K, and r', s', t', v the same for the columns
// of U.  The counts depend only on patterns, and whether K joins depends only
// on where the live block started, so one wave per block a computes the end
// of a group started at a; the host follows those ends from a = 0, which is
// the sequential rule.
//
// Merge.  A merge rewrites L S U without changing it (no dropping at merge
// time).  For a group G of consecutive blocks with unit lower (upper) block
// triangular coupling L_GG (U_GG, blocks D_J W_J inside G) and pivot blocks
// S_J = D_J^{-1}, the merged block has
//   D^ = U_GG^{-1} diag(D_J) L_GG^{-1},  L^ = L_{R,G} L_GG^{-1},
//   W^ = L_GG W_{G,C},
// with R (C) the union of the members' rows (columns) beyond the group: the
// closed form of merging the members pairwise in order.  One workgroup
// builds each group in a slot of its LDS (of global scratch when the widest
// block's four w x w matrices do not fit kMergeLdsSlot).
#include <algorithm>
#include <chrono>
#include <numeric>

#include "internal.h"
#include "wg.h"

namespace bilu {
namespace {

constexpr int kAggHash = 1024;   // LDS hash slots per wave and side (decisions)
constexpr int kAggWaves = 4;
constexpr int kMergeThreads = 256;
constexpr int kMergeSort = 4096; // rows (columns) of a merged block sorted in LDS
constexpr int64_t kMergeLdsSlot = 24576;  // bytes: the work matrices stay in LDS up to this

struct DecideArgs {
  int nb, maxb;
  const int32_t* bstart;
  const int32_t* nr; const int32_t* nc;
  const int64_t* roff; const int64_t* coff;
  const int32_t* idx;
  int32_t* gend;   // [nb]
  int32_t* gnr;    // [nb] rows of the group's merged block
  int32_t* gnc;    // [nb]
  int* overflow;
};

__device__ __forceinline__ void wsync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// committed key x >= 0, tentative -x-2, empty -1; counts new keys
__device__ __forceinline__ bool agg_insert(int* table, int key, int* added) {
  unsigned h = (unsigned(key) * 2654435761u) & (unsigned)(kAggHash - 1);
  const int tent = -key - 2;
  for (int probe = 0; probe < kAggHash; ++probe) {
    const int old = atomicCAS(&table[h], -1, tent);
    if (old == -1) {
      atomicAdd(added, 1);
      return true;
    }
    if (old == key || old == tent) return true;
    h = (h + 1) & (unsigned)(kAggHash - 1);
  }
  return false;
}

struct DecideLds {
  int rows[kAggWaves][kAggHash];
  int cols[kAggWaves][kAggHash];
  int misc[kAggWaves][4];
};

__global__ void __launch_bounds__(64 * kAggWaves) agg_decide_kernel(DecideArgs a) {
  __shared__ DecideLds s;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  int* R = s.rows[w];
  int* Cc = s.cols[w];
  int* misc = s.misc[w];
  for (int g0 = blockIdx.x * kAggWaves + w; g0 < a.nb; g0 += gridDim.x * kAggWaves) {
    for (int t = lane; t < kAggHash; t += 64) {
      R[t] = -1;
      Cc[t] = -1;
    }
    if (lane == 0) {
      misc[0] = 0;  // overflow
      misc[1] = 0;  // new rows
      misc[2] = 0;  // new columns
    }
    wsync();
    // the starting block
    {
      const int n1 = a.nr[g0], n2 = a.nc[g0];
      for (int t = lane; t < n1 + n2; t += 64) {
        const bool row = t < n1;
        const int key = row ? a.idx[a.roff[g0] + t] : a.idx[a.coff[g0] + t - n1];
        if (!agg_insert(row ? R : Cc, key, &misc[row ? 1 : 2])) misc[0] = 1;
      }
      wsync();
      for (int t = lane; t < kAggHash; t += 64) {
        if (R[t] < -1) R[t] = -R[t] - 2;
        if (Cc[t] < -1) Cc[t] = -Cc[t] - 2;
      }
      wsync();
    }
    int p = a.bstart[g0 + 1] - a.bstart[g0];
    int cur_r = a.nr[g0], cur_c = a.nc[g0];
    int K = g0 + 1;
    while (K < a.nb && !misc[0]) {
      const int fK = a.bstart[K], lK = a.bstart[K + 1] - 1, q = lK - fK + 1, wd = p + q;
      if (wd > a.maxb) break;
      // r, s (r', s'): the live block's rows (columns) inside / below K
      int r = 0, sb = 0, r2 = 0, s2 = 0;
      for (int t = lane; t < kAggHash; t += 64) {
        const int x = R[t], y = Cc[t];
        r += x >= fK && x <= lK;
        sb += x > lK;
        r2 += y >= fK && y <= lK;
        s2 += y > lK;
      }
      r = wave_sum(r);
      sb = wave_sum(sb);
      r2 = wave_sum(r2);
      s2 = wave_sum(s2);
      if (lane == 0) {
        misc[1] = 0;
        misc[2] = 0;
      }
      wsync();
      const int t1 = a.nr[K], t2 = a.nc[K];
      for (int t = lane; t < t1 + t2; t += 64) {
        const bool row = t < t1;
        const int key = row ? a.idx[a.roff[K] + t] : a.idx[a.coff[K] + t - t1];
        if (!agg_insert(row ? R : Cc, key, &misc[row ? 1 : 2])) misc[0] = 1;
      }
      wsync();
      if (misc[0]) break;
      const long long u = sb + misc[1], v = s2 + misc[2];
      const long long mu = (long long)p * (p + r + sb + r2 + s2) + (long long)q * (q + t1 + t2);
      const long long nu = (long long)wd * (wd + u + v);
      const bool merge = (5 * nu <= 6 * mu || nu <= mu + 2 * wd) && wd <= a.maxb;
      if (!merge) break;
      for (int t = lane; t < kAggHash; t += 64) {
        if (R[t] < -1) R[t] = -R[t] - 2;
        if (Cc[t] < -1) Cc[t] = -Cc[t] - 2;
      }
      wsync();
      p = wd;
      cur_r = (int)u;
      cur_c = (int)v;
      ++K;
    }
    if (lane == 0) {
      a.gend[g0] = K;
      a.gnr[g0] = cur_r;
      a.gnc[g0] = cur_c;
      if (misc[0]) atomicExch(a.overflow, 1);
    }
    wsync();
  }
}

struct MergeArgs {
  int ngroups;
  const int32_t* gfirst;   // [ngroups+1] first initial block of each final block
  FactorView in;           // the sweep's factor (initial blocks)
  // final factor
  const int64_t* froff; const int64_t* fcoff; const int64_t* floff; const int64_t* fwoff;
  const int64_t* fdoff;
  const int32_t* fnr; const int32_t* fnc;
  int32_t* fidx; void* fval; double* fdval;   // fval in the precision in.vprec
  double* scratch; int64_t slot_doubles;   // per workgroup: 4 w^2 doubles
  int lds_slot;   // 1: the slot is the launch's dynamic LDS, not scratch
  int* err;
  int copy_all;   // 0: blocks that merged with nothing stay in place (only D_K is copied)
};

struct MergeLds {
  int keys[kMergeSort];
  int misc[8];
};

// Position of x in the sorted list lst[0..cnt), or -1.
__device__ __forceinline__ int find_sorted(const int32_t* lst, int cnt, int x) {
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

// Sorted union of the members' indices beyond last into out (LDS sort);
// returns the count or -1 when it does not fit.
__device__ int merged_index_set(const MergeArgs& a, int b0, int b1, int last, bool rows,
                                MergeLds& s, int* out) {
  const int tid = threadIdx.x;
  if (tid == 0) s.misc[0] = 0;
  __syncthreads();
  for (int J = b0; J < b1; ++J) {
    const int cnt = rows ? a.in.nr[J] : a.in.nc[J];
    const int32_t* lst = a.in.idx + (rows ? a.in.roff[J] : a.in.coff[J]);
    for (int t = tid; t < cnt; t += blockDim.x) {
      const int x = lst[t];
      if (x <= last) continue;
      // an index that an earlier block of the group holds is taken there,
      // so the LDS holds the union itself, not the sum of the list lengths
      bool seen = false;
      for (int J2 = b0; J2 < J && !seen; ++J2)
        seen = find_sorted(a.in.idx + (rows ? a.in.roff[J2] : a.in.coff[J2]),
                           rows ? a.in.nr[J2] : a.in.nc[J2], x) >= 0;
      if (seen) continue;
      const int o = atomicAdd(&s.misc[0], 1);
      if (o < kMergeSort) s.keys[o] = x;
    }
  }
  __syncthreads();
  const int m = s.misc[0];
  if (m > kMergeSort) return -1;
  wg_bitonic_sort(s.keys, m);
  // unique, in order: keep first of each run
  if (tid == 0) s.misc[1] = 0;
  __syncthreads();
  // exclusive positions by a block scan over runs
  int cnt = 0;
  const int per = (m + blockDim.x - 1) / blockDim.x;
  const int i0 = tid * per, i1 = min(m, i0 + per);
  for (int i = i0; i < i1; ++i) cnt += (i == 0 || s.keys[i] != s.keys[i - 1]);
  int total = 0;
  int pos = wg_exclusive_scan(cnt, s.misc + 2, &total);
  for (int i = i0; i < i1; ++i)
    if (i == 0 || s.keys[i] != s.keys[i - 1]) out[pos++] = s.keys[i];
  __syncthreads();
  return total;
}


__global__ void __launch_bounds__(kMergeThreads) agg_merge_kernel(MergeArgs a) {
  __shared__ MergeLds s;
  extern __shared__ double s_slot[];
  const int tid = threadIdx.x, nt = blockDim.x;
  // L_GG (w x w), then L_GG^{-1}, U_GG and the product below; every step
  // of the two triangular solves reads the rows before it, so the slot sits
  // in LDS whenever it fits
  double* Lg = a.lds_slot ? s_slot : a.scratch + (int64_t)blockIdx.x * a.slot_doubles;
  for (int g = blockIdx.x; g < a.ngroups; g += gridDim.x) {
    const int b0 = a.gfirst[g], b1 = a.gfirst[g + 1];
    const int f0 = a.in.bstart[b0], last = a.in.bstart[b1] - 1, w = last - f0 + 1;
    int32_t* Rout = a.fidx + a.froff[g];
    int32_t* Cout = a.fidx + a.fcoff[g];
    const int64_t lout = a.floff[g], wout = a.fwoff[g];  // L^, W^ offsets in fval
    const int vp = a.in.vprec;
    double* Dout = a.fdval + a.fdoff[g];
    const int nrg = a.fnr[g], ncg = a.fnc[g];
    if (b1 - b0 == 1) {
      // a block that merged with nothing: copy (D_K only when it stays in place)
      const int J = b0;
      if (!a.copy_all) {
        for (int t = tid; t < w * w; t += nt) Dout[t] = a.in.dval[a.in.doff[J] + t];
        continue;
      }
      for (int t = tid; t < nrg; t += nt) Rout[t] = a.in.idx[a.in.roff[J] + t];
      for (int t = tid; t < ncg; t += nt) Cout[t] = a.in.idx[a.in.coff[J] + t];
      for (int t = tid; t < nrg * w; t += nt)
        value_store(a.fval, vp, lout + t, value_load(a.in.val, vp, a.in.loff[J] + t));
      for (int t = tid; t < ncg * w; t += nt)
        value_store(a.fval, vp, wout + t, value_load(a.in.val, vp, a.in.woff[J] + t));
      for (int t = tid; t < w * w; t += nt) Dout[t] = a.in.dval[a.in.doff[J] + t];
      continue;
    }
    double* Li = Lg + w * w;      // L_GG^{-1}
    double* Ug = Li + w * w;      // U_GG
    double* Tm = Ug + w * w;      // diag(D_J) L_GG^{-1}
    // L_GG and U_GG: unit diagonal, member couplings
    for (int e = tid; e < w * w; e += nt) {
      const int x = e / w, y = e % w;
      Lg[e] = x == y ? 1.0 : 0.0;
      Ug[e] = x == y ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int J = b0; J < b1; ++J) {
      const int oJ = a.in.bstart[J] - f0, qJ = a.in.bstart[J + 1] - a.in.bstart[J];
      const int nr = a.in.nr[J], nc = a.in.nc[J];
      const int32_t* RJ = a.in.idx + a.in.roff[J];
      const int32_t* CJ = a.in.idx + a.in.coff[J];
      const int64_t LJ = a.in.loff[J], WJ = a.in.woff[J];
      const double* DJ = a.in.dval + a.in.doff[J];
      for (int e = tid; e < nr * qJ; e += nt) {
        const int z = e / qJ, c = e % qJ;
        const int x = RJ[z];
        if (x <= last) Lg[(x - f0) * w + oJ + c] = value_load(a.in.val, vp, LJ + (int64_t)z * qJ + c);
      }
      for (int e = tid; e < nc * qJ; e += nt) {
        const int z = e / qJ, r = e % qJ;
        const int y = CJ[z];
        if (y <= last) {
          double acc = 0.0;
          for (int t = 0; t < qJ; ++t)
            acc = fma(DJ[r * qJ + t], value_load(a.in.val, vp, WJ + (int64_t)z * qJ + t), acc);
          Ug[(oJ + r) * w + (y - f0)] = acc;
        }
      }
    }
    __syncthreads();
    // L_GG^{-1}, column by column (forward substitution)
    for (int y = tid; y < w; y += nt) {
      for (int x = 0; x < w; ++x) {
        double v = x == y ? 1.0 : 0.0;
        if (x > y) {
          double acc = 0.0;
          for (int z = y; z < x; ++z) acc = fma(Lg[x * w + z], Li[z * w + y], acc);
          v = -acc;
        }
        Li[x * w + y] = v;
      }
    }
    __syncthreads();
    // Tm = diag(D_J) L_GG^{-1}
    for (int e = tid; e < w * w; e += nt) {
      const int x = e / w, y = e % w;
      int J = b0;
      while (a.in.bstart[J + 1] - f0 <= x) ++J;
      const int oJ = a.in.bstart[J] - f0, qJ = a.in.bstart[J + 1] - a.in.bstart[J];
      const double* DJ = a.in.dval + a.in.doff[J];
      double acc = 0.0;
      for (int t = 0; t < qJ; ++t) acc = fma(DJ[(x - oJ) * qJ + t], Li[(oJ + t) * w + y], acc);
      Tm[e] = acc;
    }
    __syncthreads();
    // D^ = U_GG^{-1} Tm (back substitution per column, in place: row x
    // reads the finished rows below it), then out
    for (int y = tid; y < w; y += nt) {
      for (int x = w - 1; x >= 0; --x) {
        double acc = Tm[x * w + y];
        for (int z = x + 1; z < w; ++z) acc = fma(-Ug[x * w + z], Tm[z * w + y], acc);
        Tm[x * w + y] = acc;
      }
    }
    __syncthreads();
    for (int e = tid; e < w * w; e += nt) Dout[e] = Tm[e];
    // rows of the merged block: L^ = L_{R,G} L_GG^{-1}
    {
      const int m = merged_index_set(a, b0, b1, last, true, s, Rout);
      if (m != nrg) {
        if (tid == 0) atomicCAS(a.err, 0, 1);
        return;
      }
    }
    // the position of every merged row in every member's row list, found
    // once per (member, row) into the LDS key array when it fits, else per
    // entry below
    const int nmem = b1 - b0;
    const bool rtab = nmem * nrg <= kMergeSort;
    if (rtab) {
      for (int e = tid; e < nmem * nrg; e += nt) {
        const int J = b0 + e / nrg;
        s.keys[e] = find_sorted(a.in.idx + a.in.roff[J], a.in.nr[J], Rout[e % nrg]);
      }
      __syncthreads();
    }
    for (int e = tid; e < nrg * w; e += nt) {
      const int z = e / w, y = e % w;
      double acc = 0.0;
      for (int J = b0; J < b1; ++J) {
        const int oJ = a.in.bstart[J] - f0, qJ = a.in.bstart[J + 1] - a.in.bstart[J];
        if (oJ + qJ <= y) continue;  // L_GG^{-1} is lower triangular
        const int pz = rtab ? s.keys[(J - b0) * nrg + z]
                            : find_sorted(a.in.idx + a.in.roff[J], a.in.nr[J], Rout[z]);
        if (pz < 0) continue;
        const int64_t row = a.in.loff[J] + (int64_t)pz * qJ;
        for (int c = 0; c < qJ; ++c)
          acc = fma(value_load(a.in.val, vp, row + c), Li[(oJ + c) * w + y], acc);
      }
      value_store(a.fval, vp, lout + (int64_t)z * w + y, acc);
    }
    __syncthreads();
    // columns: W^ = L_GG W_{G,C}
    {
      const int m = merged_index_set(a, b0, b1, last, false, s, Cout);
      if (m != ncg) {
        if (tid == 0) atomicCAS(a.err, 0, 1);
        return;
      }
    }
    const bool ctab = nmem * ncg <= kMergeSort;  // as for the rows
    if (ctab) {
      for (int e = tid; e < nmem * ncg; e += nt) {
        const int J = b0 + e / ncg;
        s.keys[e] = find_sorted(a.in.idx + a.in.coff[J], a.in.nc[J], Cout[e % ncg]);
      }
      __syncthreads();
    }
    for (int e = tid; e < ncg * w; e += nt) {
      const int z = e / w, x = e % w;
      double acc = 0.0;
      for (int J = b0; J < b1; ++J) {
        const int oJ = a.in.bstart[J] - f0, qJ = a.in.bstart[J + 1] - a.in.bstart[J];
        if (oJ > x) break;  // L_GG is lower triangular
        const int pz = ctab ? s.keys[(J - b0) * ncg + z]
                            : find_sorted(a.in.idx + a.in.coff[J], a.in.nc[J], Cout[z]);
        if (pz < 0) continue;
        const int64_t col = a.in.woff[J] + (int64_t)pz * qJ;
        for (int c = 0; c < qJ; ++c)
          acc = fma(Lg[x * w + oJ + c], value_load(a.in.val, vp, col + c), acc);
      }
      value_store(a.fval, vp, wout + (int64_t)z * w + x, acc);
    }
    __syncthreads();
  }
}

// Offsets of the final blocks when the unmerged ones stay in place: every
// group first takes its first member's offsets, then the merged groups get
// theirs from the compact list (group, rows, columns, L, W offsets).
__global__ void agg_offsets(int ng, const int32_t* gfirst, FactorView in, int64_t* roff,
                            int64_t* coff, int64_t* loff, int64_t* woff) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= ng) return;
  const int J = gfirst[g];
  roff[g] = in.roff[J];
  coff[g] = in.coff[J];
  loff[g] = in.loff[J];
  woff[g] = in.woff[J];
}
__global__ void agg_offsets_merged(int m, const int64_t* list, int64_t* roff, int64_t* coff,
                                   int64_t* loff, int64_t* woff) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  const int64_t* e = list + 5 * (int64_t)i;
  roff[e[0]] = e[1];
  coff[e[0]] = e[2];
  loff[e[0]] = e[3];
  woff[e[0]] = e[4];
}

// Rows, columns and first index of every final block, from its first
// initial block (index ng gives the end of the last one).
__global__ void agg_gather(int ng, const int32_t* gfirst, const int32_t* gnr, const int32_t* gnc,
                           const int32_t* bstart0, int32_t* fnr, int32_t* fnc, int32_t* fbs) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g > ng) return;
  const int J = gfirst[g];
  fbs[g] = bstart0[J];
  if (g < ng) {
    fnr[g] = gnr[J];
    fnc[g] = gnc[J];
  }
}

__global__ void agg_block_of(const int32_t* bstart, int nb, int32_t* blockOf) {
  const int b = blockIdx.x * blockDim.y + threadIdx.y;
  if (b >= nb) return;
  for (int i = bstart[b] + threadIdx.x; i < bstart[b + 1]; i += blockDim.x) blockOf[i] = b;
}

}  // namespace

bilu_status aggregate_device(bilu_handle* h) {
  hipStream_t st = h->stream;
  const int64_t nb = (int64_t)h->bstart0.size() - 1;
  const int64_t n = h->n;
#define CK(x)                                              \
  do {                                                     \
    hipError_t e_ = (x);                                   \
    if (e_ != hipSuccess) return hip_check(h, e_, #x);     \
  } while (0)
  // ---- decisions
  DevArray<int32_t> dec;
  CK(dec.alloc(3 * nb + 1));
  DecideArgs da{};
  da.nb = (int)nb;
  da.maxb = h->opt.max_block;
  da.bstart = h->d_bstart.p;
  da.nr = h->d_nr.p;
  da.nc = h->d_nc.p;
  da.roff = h->d_roff.p;
  da.coff = h->d_coff.p;
  da.idx = h->d_idx_heap.p;
  da.gend = dec.p;
  da.gnr = dec.p + nb;
  da.gnc = dec.p + 2 * nb;
  da.overflow = dec.p + 3 * nb;
  CK(hipMemsetAsync(da.overflow, 0, sizeof(int), st));
  const unsigned g1 = (unsigned)std::min<int64_t>((nb + kAggWaves - 1) / kAggWaves, 65536);
  agg_decide_kernel<<<g1, 64 * kAggWaves, 0, st>>>(da);
  CK(hipGetLastError());
  hipError_t pe = hipSuccess;
  int32_t* hdec = h->pin_dec.get<int32_t>(3 * nb + 1, &pe);
  CK(pe);
  CK(hipMemcpyAsync(hdec, dec.p, (3 * nb + 1) * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (hdec[3 * nb] != 0)
    return fail(h, BILU_ERR_NO_MEMORY, "aggregation: a merged block exceeds the decision capacity");
  const int32_t* gnr = hdec + nb;  // rows / columns of a group, by its first block
  const int32_t* gnc = hdec + 2 * nb;
  // ---- groups: follow the ends from block 0
  std::vector<int32_t>& gfirst = h->agg_gfirst;
  gfirst.clear();
  for (int64_t a0 = 0; a0 < nb;) {
    const int64_t e = hdec[a0];
    if (e <= a0 || e > nb) return fail(h, BILU_ERR_INTERNAL, "aggregation: bad group end");
    gfirst.push_back((int32_t)a0);
    a0 = e;
  }
  const int64_t ng = (int64_t)gfirst.size();
  gfirst.push_back((int32_t)nb);
  h->stats.merges = nb - ng;
  if (ng == nb) return BILU_OK;  // nothing merged: the sweep's factor is final
  std::vector<int32_t>& fbs = h->agg_fbs;
  fbs.resize(ng + 1);
  // staged uploads: group firsts, then D offsets, then the merged-group list
  int64_t nmerged = 0;
  for (int64_t g = 0; g < ng; ++g) nmerged += gfirst[g + 1] - gfirst[g] > 1;
  const size_t up_words = (size_t)(ng + 2) / 2 + 1 + (size_t)(ng + 1) + 5 * (size_t)nmerged;
  int64_t* up = h->pin_up.get<int64_t>(up_words, &pe);
  CK(pe);
  int32_t* up_gfirst = reinterpret_cast<int32_t*>(up);
  int64_t* fdoff = up + (ng + 2) / 2 + 1;
  int64_t* mlist = fdoff + ng + 1;
  std::copy(gfirst.begin(), gfirst.end(), up_gfirst);
  fdoff[0] = 0;
  int64_t wmax = 1;
  for (int64_t g = 0; g < ng; ++g) {
    fbs[g] = h->bstart0[gfirst[g]];
    const int64_t w = h->bstart0[gfirst[g + 1]] - h->bstart0[gfirst[g]];
    wmax = std::max(wmax, w);
    fdoff[g + 1] = fdoff[g] + w * w;
  }
  fbs[ng] = (int32_t)n;
  // merged blocks go after the sweep's data in its own heaps when they fit;
  // blocks that merged with nothing then stay where they are
  int64_t mi = h->idx_used, mv = h->val_used, m = 0;
  for (int64_t g = 0; g < ng; ++g) {
    if (gfirst[g + 1] - gfirst[g] == 1) continue;
    const int64_t w = fbs[g + 1] - fbs[g];
    const int64_t r = gnr[gfirst[g]], c = gnc[gfirst[g]];
    int64_t* e = mlist + 5 * m++;
    e[0] = g;
    e[1] = mi;
    e[2] = mi + r;
    e[3] = mv;
    e[4] = mv + r * w;
    mi += r + c;
    mv += (r + c) * w;
  }
  const int vbytes = value_bytes(h->fv.vprec);
  const bool in_place =
      mi <= (int64_t)h->d_idx_heap.n && mv * vbytes <= (int64_t)h->d_val_heap.n;
  CK(h->f_bstart.alloc(ng + 1));
  CK(h->f_blockof.alloc(n));
  CK(h->f_nr.alloc(ng));
  CK(h->f_nc.alloc(ng));
  CK(h->f_roff.alloc(ng));
  CK(h->f_coff.alloc(ng));
  CK(h->f_loff.alloc(ng));
  CK(h->f_woff.alloc(ng));
  CK(h->f_doff.alloc(ng + 1));
  CK(h->f_dval.alloc(fdoff[ng]));
  DevArray<int32_t> d_gfirst;
  CK(d_gfirst.alloc(ng + 1));
  CK(hipMemcpyAsync(d_gfirst.p, up_gfirst, (ng + 1) * 4, hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(h->f_doff.p, fdoff, (ng + 1) * 8, hipMemcpyHostToDevice, st));
  agg_gather<<<(unsigned)((ng + 256) / 256), 256, 0, st>>>((int)ng, d_gfirst.p, dec.p + nb,
                                                           dec.p + 2 * nb, h->d_bstart.p, h->f_nr.p,
                                                           h->f_nc.p, h->f_bstart.p);
  CK(hipGetLastError());
  DevArray<int64_t> d_mlist;
  int64_t vo_total = 0;  // values of the separate storage (not in place)
  if (in_place) {
    agg_offsets<<<(unsigned)((ng + 255) / 256), 256, 0, st>>>((int)ng, d_gfirst.p, h->fv, h->f_roff.p,
                                                             h->f_coff.p, h->f_loff.p, h->f_woff.p);
    if (m > 0) {
      CK(d_mlist.alloc(5 * m));
      CK(hipMemcpyAsync(d_mlist.p, mlist, 5 * m * 8, hipMemcpyHostToDevice, st));
      agg_offsets_merged<<<(unsigned)((m + 255) / 256), 256, 0, st>>>(
          (int)m, d_mlist.p, h->f_roff.p, h->f_coff.p, h->f_loff.p, h->f_woff.p);
    }
    CK(hipGetLastError());
  } else {
    // every block is copied: consecutive offsets
    std::vector<int64_t>& off = h->agg_off;
    off.resize(4 * ng);
    int64_t io = 0, vo = 0;
    for (int64_t g = 0; g < ng; ++g) {
      const int64_t w = fbs[g + 1] - fbs[g];
      const int64_t r = gnr[gfirst[g]], c = gnc[gfirst[g]];
      off[g] = io;
      off[ng + g] = io + r;
      off[2 * ng + g] = vo;
      off[3 * ng + g] = vo + r * w;
      io += r + c;
      vo += (r + c) * w;
    }
    CK(h->f_idx.alloc(std::max<int64_t>(1, io)));
    CK(h->f_val.alloc(std::max<int64_t>(1, vo) * vbytes));
    vo_total = vo;
    CK(hipMemcpyAsync(h->f_roff.p, off.data(), ng * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->f_coff.p, off.data() + ng, ng * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->f_loff.p, off.data() + 2 * ng, ng * 8, hipMemcpyHostToDevice, st));
    CK(hipMemcpyAsync(h->f_woff.p, off.data() + 3 * ng, ng * 8, hipMemcpyHostToDevice, st));
  }
  {
    dim3 blk(64, 4);
    agg_block_of<<<dim3((unsigned)((ng + 3) / 4)), blk, 0, st>>>(h->f_bstart.p, (int)ng,
                                                                h->f_blockof.p);
  }
  // ---- merged blocks
  // A merged group's steps are short and separated by workgroup barriers,
  // so the merge is bound by latency: launch as many workgroups as can be
  // resident.  Each owns a slot of 4 w_max^2 doubles: dynamic LDS when that
  // fits kMergeLdsSlot, else global scratch, kept within 256 MiB when the
  // blocks are wide.
  const int64_t slot_doubles = 4 * wmax * wmax;
  const bool lds_slot = 8 * slot_doubles <= kMergeLdsSlot;
  const size_t dyn = lds_slot ? (size_t)(8 * slot_doubles) : 0;
  int64_t slots = 1024;
  {
    int dev = 0, cus = 0, per_cu = 0;
    CK(hipGetDevice(&dev));
    CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(
        &per_cu, reinterpret_cast<const void*>(agg_merge_kernel), kMergeThreads, dyn));
    const int64_t resident = (int64_t)std::max(cus, 1) * std::max(per_cu, 1);
    const int64_t cap =
        lds_slot ? resident : std::max<int64_t>(1024, (int64_t(256) << 20) / (8 * slot_doubles));
    slots = std::max<int64_t>(1, std::min({ng, resident, cap}));
  }
  DevArray<int> err;
  if (!lds_slot) CK(h->d_agg_scratch.alloc(slots * slot_doubles));
  CK(err.alloc(1));
  CK(hipMemsetAsync(err.p, 0, sizeof(int), st));
  MergeArgs ma{};
  ma.ngroups = (int)ng;
  ma.gfirst = d_gfirst.p;
  ma.in = h->fv;
  ma.froff = h->f_roff.p;
  ma.fcoff = h->f_coff.p;
  ma.floff = h->f_loff.p;
  ma.fwoff = h->f_woff.p;
  ma.fdoff = h->f_doff.p;
  ma.fnr = h->f_nr.p;
  ma.fnc = h->f_nc.p;
  ma.fidx = in_place ? h->d_idx_heap.p : h->f_idx.p;
  ma.fval = in_place ? h->d_val_heap.p : h->f_val.p;
  ma.copy_all = in_place ? 0 : 1;
  ma.fdval = h->f_dval.p;
  ma.scratch = lds_slot ? nullptr : h->d_agg_scratch.p;
  ma.slot_doubles = slot_doubles;
  ma.lds_slot = lds_slot ? 1 : 0;
  ma.err = err.p;
  agg_merge_kernel<<<(unsigned)slots, kMergeThreads, dyn, st>>>(ma);
  CK(hipGetLastError());
  int herr = 0;
  CK(hipMemcpyAsync(&herr, err.p, sizeof(int), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  if (herr) return fail(h, BILU_ERR_NO_MEMORY, "aggregation: a merged block exceeds the merge capacity");
  // ---- the merged factor becomes the final one
  h->nb = ng;
  h->bstart.assign(fbs.begin(), fbs.end());
  h->final_is_initial = false;
  FactorView& f = h->fv;
  f.nb = (int)ng;
  f.bstart = h->f_bstart.p;
  f.blockOf = h->f_blockof.p;
  f.nr = h->f_nr.p;
  f.nc = h->f_nc.p;
  f.roff = h->f_roff.p;
  f.coff = h->f_coff.p;
  f.loff = h->f_loff.p;
  f.woff = h->f_woff.p;
  f.doff = h->f_doff.p;
  f.idx = in_place ? h->d_idx_heap.p : h->f_idx.p;
  f.val = in_place ? h->d_val_heap.p : h->f_val.p;
  h->f_val_len = in_place ? mv : vo_total;
  f.dval = h->f_dval.p;
  return BILU_OK;
#undef CK
}

}  // namespace bilu
