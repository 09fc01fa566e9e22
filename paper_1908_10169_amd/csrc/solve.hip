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
#include <climits>
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
// Runs of consecutive rows of R_J (columns of C_J with cols) that fall into
// one block K.
__global__ void __launch_bounds__(256) fw_count(FactorView f, int32_t* cnt, int cols) {
  const int J = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (J >= f.nb) return;
  const int lane = threadIdx.x & 63;
  const int32_t* R = f.idx + (cols ? f.coff[J] : f.roff[J]);
  const int m = cols ? f.nc[J] : f.nr[J];
  for (int i = lane; i < m; i += 64) {
    const int K = f.blockOf[R[i]];
    if (i == 0 || f.blockOf[R[i - 1]] != K) atomicAdd(&cnt[K], 1);
  }
}

// Packed (J, first index in R_J (C_J), count) keys, sorted later per block.
__global__ void __launch_bounds__(256) fw_fill(FactorView f, const int32_t* ptr, int32_t* fillc,
                                               unsigned long long* keys, int cols) {
  const int J = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (J >= f.nb) return;
  const int lane = threadIdx.x & 63;
  const int32_t* R = f.idx + (cols ? f.coff[J] : f.roff[J]);
  const int m = cols ? f.nc[J] : f.nr[J];
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

// Sort each block's keys (ascending J; the keys of a block are distinct)
// and unpack them.  One wave per block: up to 64 keys are ranked in
// registers, longer lists by an insertion sort of lane 0.
__global__ void __launch_bounds__(256) fw_sort(int nb, const int32_t* ptr, unsigned long long* keys,
                                               int32_t* fw_j, int32_t* fw_r0, int32_t* fw_cnt) {
  const int K = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (K >= nb) return;  // no workgroup barrier below
  const int lane = threadIdx.x & 63;
  const int b = ptr[K], m = ptr[K + 1] - b;
  auto put = [&](int i, unsigned long long v) {
    fw_j[b + i] = (int32_t)(v >> 32);
    fw_r0[b + i] = (int32_t)((v >> 8) & 0xffffff);
    fw_cnt[b + i] = (int32_t)(v & 0xff);
  };
  if (m <= 64) {
    const unsigned long long v = lane < m ? keys[b + lane] : ~0ull;
    int r = 0;
    for (int j = 0; j < m; ++j) r += __shfl(v, j, 64) < v;
    if (lane < m) put(r, v);
    return;
  }
  if (lane == 0) {
    unsigned long long* k = keys + b;
    for (int i = 1; i < m; ++i) {
      unsigned long long v = k[i];
      int j = i - 1;
      while (j >= 0 && k[j] > v) {
        k[j + 1] = k[j];
        --j;
      }
      k[j + 1] = v;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  for (int i = lane; i < m; i += 64) put(i, keys[b + i]);
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
// One wave per block: the first column of every run of one block, in
// order (ballot compaction 64 columns at a time).
__global__ void __launch_bounds__(256) bw_fill(FactorView f, const int32_t* ptr, int32_t* bw_b) {
  const int K = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (K >= f.nb) return;
  const int lane = threadIdx.x & 63;
  const int32_t* Cc = f.idx + f.coff[K];
  const int m = f.nc[K];
  int at = ptr[K];
  for (int i0 = 0; i0 < m; i0 += 64) {
    const int i = i0 + lane;
    const int B = i < m ? f.blockOf[Cc[i]] : -1;
    const bool head = i < m && (i == 0 || f.blockOf[Cc[i - 1]] != B);
    const unsigned long long hm = __ballot(head);
    if (head) bw_b[at + __popcll(hm & ((1ull << lane) - 1ull))] = B;
    at += __popcll(hm);
  }
}

// Order of the level computation below.  A block's key starts as the
// largest sweep depth among the initial blocks it holds (depth0 over the
// initial partition, blockOf0 its row map; both read within bounds whatever
// they hold).  Keys only grow, and only to values already present.
__global__ void plan_keys(int nb, const int32_t* bstart, const int32_t* blockOf0, int nb0,
                          const int* depth0, int* key) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nb) return;
  const int i0 = bstart[g], i1 = bstart[g + 1] - 1;
  const int b0 = min(max(blockOf0[i0], 0), nb0 - 1);
  const int b1 = min(max(blockOf0[i1], 0), nb0 - 1);
  int k = 0;
  for (int b = b0; b <= b1 && b - b0 <= i1 - i0; ++b) k = max(k, depth0[b]);
  key[g] = k;
}
// One relaxation pass, one wave per block K: key(K) rises to the keys of
// the blocks it depends on forward (fw lists), and the blocks it depends on
// backward (bw lists) rise to key(K).  *changed is set when a key rose.  A
// pass that changes nothing read constant keys throughout, so afterwards
// key(J) <= key(K) for every forward dependency J of K and key(B) >= key(K)
// for every backward one B.
__global__ void __launch_bounds__(256) plan_relax(int nb, const int32_t* fptr, const int32_t* fj,
                                                  const int32_t* bptr, const int32_t* bb, int* key,
                                                  int* changed) {
  const int K = blockIdx.x * 4 + (int)(threadIdx.x >> 6);
  if (K >= nb) return;
  const int lane = threadIdx.x & 63;
  int m = 0;
  for (int e = fptr[K] + lane; e < fptr[K + 1]; e += 64)
    m = max(m, __hip_atomic_load(&key[fj[e]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = max(m, __shfl_xor(m, o, 64));
  int kk = __hip_atomic_load(&key[K], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (m > kk) {
    if (lane == 0 && atomicMax(&key[K], m) < m) atomicExch(changed, 1);
    kk = m;
  }
  for (int e = bptr[K] + lane; e < bptr[K + 1]; e += 64) {
    const int B = bb[e];
    if (__hip_atomic_load(&key[B], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < kk &&
        atomicMax(&key[B], kk) < kk)
      atomicExch(changed, 1);
  }
}

// Dependency levels of the apply: level(K) = 1 + the largest level of the
// blocks K depends on (0 without any); forward over fw lists (J < K),
// backward over bw lists (B > K).  One wave per block: even slots 2i hold
// the forward blocks in the order ord (ascending index when ord is null),
// odd slots 2i+1 the backward blocks in the reverse order.  ord lists every
// forward dependency of a block before it, and so every backward one after
// it: every dependency of a slot sits at a lower slot.
// Workgroup g runs slots 4g..4g+3, g its index (the hardware starts a
// launch's workgroups in index order) or, with ticket, the order in which
// workgroups took a ticket when they started.  Either way every workgroup
// holding a lower slot has started before the one holding the lowest
// unfinished slot, so that slot's wave is running with its dependencies
// done: the launch needs no workgroup to be resident for another to make
// progress.  Waits are bounded; a timeout sets *err.  Levels start at -1.
__global__ void __launch_bounds__(256) apply_levels(int nb, const int32_t* fptr, const int32_t* fj,
                                                    const int32_t* bptr, const int32_t* bb,
                                                    const int32_t* ord, int* lf, int* lb, int* err,
                                                    int* ticket, unsigned long long wait_ticks) {
  __shared__ int s_id;
  int id = blockIdx.x;
  if (ticket) {
    if (threadIdx.x == 0) s_id = atomicAdd(ticket, 1);
    __syncthreads();
    id = s_id;
  }
  const int lane = threadIdx.x & 63;
  const int s = id * 4 + (int)(threadIdx.x >> 6);
  if (s >= 2 * nb) return;  // no workgroup barrier below
  // the two directions interleave (they do not depend on each other): even
  // slots forward along ord, odd slots backward along its reverse
  const bool fwd = (s & 1) == 0;
  const int p = fwd ? s >> 1 : nb - 1 - (s >> 1);
  const int K = ord ? ord[p] : p;
  const int32_t* ptr = fwd ? fptr : bptr;
  const int32_t* adj = fwd ? fj : bb;
  int* lev = fwd ? lf : lb;
  const int e0 = ptr[K], e1 = ptr[K + 1];
  int l = 0;
  const unsigned long long t0 = wall_clock64();
  for (int e = e0; e < e1; e += 64) {
    const int J = e + lane < e1 ? adj[e + lane] : -1;
    int v = J >= 0 ? __hip_atomic_load(&lev[J], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    while (!__all(v >= 0)) {
      __builtin_amdgcn_s_sleep(1);
      // the level's reload, the error word and the clock go out together
      const int nv = v < 0 ? __hip_atomic_load(&lev[J], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : v;
      const int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const unsigned long long now = wall_clock64();
      v = nv;
      if (e != 0) return;
      if (now - t0 > wait_ticks && !__all(v >= 0)) {
        if (lane == 0) atomicExch(err, 1);
        return;
      }
    }
    if (J >= 0) l = max(l, v + 1);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) l = max(l, __shfl_xor(l, o, 64));
  if (lane == 0) __hip_atomic_store(&lev[K], l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// First position of every level in the sorted levels (every level from 0 to
// the largest one holds a block: a block of level l depends on one of l - 1).
__global__ void level_starts(int nb, const int* sorted, int* start) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  if (i == 0 || sorted[i - 1] != sorted[i]) start[sorted[i]] = i;
  if (i == nb - 1) start[sorted[i] + 1] = nb;
}
__global__ void slot_rows(int nb, const int32_t* sched, const int32_t* bstart, int2* fq) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int K = sched[i];
  fq[i] = make_int2(bstart[K], bstart[K + 1] - bstart[K]);
}
__global__ void iota_k(int n, int32_t* v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

// Row-major copy of L: row i lists, for every block J (ascending) whose L_J
// holds row i, the q_J entries L_J(i, :) at columns first(J)..last(J).
// One wave per block K: the dependencies of K (ascending J) are read 64 at
// a time, then their rows in K 64 at a time; lane r (and r + 64) then takes
// row r of K through them in that order.  kFill = false counts the entries
// of each row into lr_cnt; kFill = true writes them from lr_ptr on.
template <bool kFill, class T>
__global__ void __launch_bounds__(256) lr_build(FactorView f, const int32_t* fw_ptr,
                                                const int32_t* fw_j, const int32_t* fw_r0,
                                                const int32_t* fw_cnt, const int64_t* lr_ptr,
                                                int64_t* lr_cnt, int32_t* lr_col, T* lr_val) {
  __shared__ int sOff[4][65];             // prefix of the dependencies' row counts
  __shared__ int sR0[4][64], sF[4][64], sP[4][64];
  __shared__ long long sRoff[4][64], sLoff[4][64];
  __shared__ int sRow[4][64], sLe[4][64], sI[4][64];
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int K = blockIdx.x * 4 + wv;
  if (K >= f.nb) return;  // no workgroup barrier below
  const int fK = f.bstart[K], q = f.bstart[K + 1] - fK;
  const int e0 = fw_ptr[K], e1 = fw_ptr[K + 1];
  int64_t at0 = 0, at1 = 0;  // rows lane and lane + 64: next position, or count
  if (kFill) {
    if (lane < q) at0 = lr_ptr[fK + lane];
    if (lane + 64 < q) at1 = lr_ptr[fK + lane + 64];
  }
  auto wave_sync = []() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
  };
  for (int c0 = e0; c0 < e1; c0 += 64) {
    const int e = c0 + lane;
    int cnt = 0;
    if (e < e1) {
      const int J = fw_j[e];
      cnt = fw_cnt[e];
      const int fJ = f.bstart[J];
      sR0[wv][lane] = fw_r0[e];
      sF[wv][lane] = fJ;
      sP[wv][lane] = f.bstart[J + 1] - fJ;
      sRoff[wv][lane] = f.roff[J];
      sLoff[wv][lane] = f.loff[J];
    }
    int incl = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int t = __shfl_up(incl, o, 64);
      if (lane >= o) incl += t;
    }
    sOff[wv][lane + 1] = incl;
    if (lane == 0) sOff[wv][0] = 0;
    const int mc = __shfl(incl, 63, 64);
    wave_sync();
    for (int t0 = 0; t0 < mc; t0 += 64) {
      const int t = t0 + lane;
      if (t < mc) {
        int lo = 0, hi = 64;  // last dependency with sOff <= t
        while (hi - lo > 1) {
          const int mid = (lo + hi) >> 1;
          if (sOff[wv][mid] <= t)
            lo = mid;
          else
            hi = mid;
        }
        const int i = sR0[wv][lo] + (t - sOff[wv][lo]);
        sRow[wv][lane] = f.idx[sRoff[wv][lo] + i] - fK;
        sLe[wv][lane] = lo;
        sI[wv][lane] = i;
      }
      wave_sync();
      const int tn = min(64, mc - t0);
      if (kFill) {
        // lane u copies item u: its row's next position plus the items of
        // the same row before it in this chunk
        const int myr = lane < tn ? sRow[wv][lane] : 0;
        const long long b0 = __shfl((long long)at0, myr & 63, 64);
        const long long b1 = __shfl((long long)at1, myr & 63, 64);
        if (lane < tn) {
          int64_t pos = myr < 64 ? b0 : b1;
          for (int u = 0; u < lane; ++u)
            if (sRow[wv][u] == myr) pos += sP[wv][sLe[wv][u]];
          const int le = sLe[wv][lane];
          const int pJ = sP[wv][le], fJ = sF[wv][le];
          const int64_t L = sLoff[wv][le] + (int64_t)sI[wv][lane] * pJ;
          for (int c = 0; c < pJ; ++c) {
            lr_col[pos + c] = fJ + c;
            lr_val[pos + c] = from_double<T>(value_load(f.val, f.vprec, L + c));
          }
        }
      }
      // the rows' owner lanes advance past this chunk's items
      for (int u = 0; u < tn; ++u) {
        const int r = sRow[wv][u];
        const int pJ = sP[wv][sLe[wv][u]];
        if (r == lane) at0 += pJ;
        else if (r == lane + 64) at1 += pJ;
      }
      wave_sync();
    }
  }
  if (!kFill) {
    if (lane < q) lr_cnt[fK + lane] = at0;
    if (lane + 64 < q) lr_cnt[fK + lane + 64] = at1;
  }
}

// ---------------------------------------------------------------------------
// Level-scheduled sweeps.  Blocks are grouped by their depth in the actual
// dependency graph of the factor (forward: predecessors J whose L_J has rows
// in K; backward: blocks holding the columns of U_K); one launch per level,
// one wave per block, no waiting inside a kernel.
// ---------------------------------------------------------------------------
template <class T>
struct SweepArgs {
  FactorView f;
  const int64_t* lr_ptr;
  const int32_t* lr_col;
  const T* lr_val;     // row-major L in the apply precision
  const T* wval;       // W values in the apply precision, at f.woff
  const int32_t* sched;
  const int2* fq;  // forward: first row and width of each scheduled block
  int begin, end;
  const int* skip;  // when set and nonzero (a converged solver step): no work
};

// forward: t_K = x_K - sum over stored L(i, j) t_j, rows of K from the
// row-major copy (groups of lanes per row, fixed reduction tree)
template <class T>
__global__ void __launch_bounds__(256) forward_level(SweepArgs<T> a, const double* x, double* t) {
  if (a.skip && *a.skip) return;
  const int w = a.begin + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (w >= a.end) return;
  const int lane = threadIdx.x & 63;
  const int2 fq = a.fq[w];
  const int f = fq.x, q = fq.y;
  int qp = 1;
  while (qp < q && qp < 64) qp <<= 1;
  const int g = 64 / qp;  // lanes per row
  for (int r0 = 0; r0 < q; r0 += qp) {
    const int r = r0 + lane / g, sub = lane % g;
    double acc = 0.0;
    if (r < q) {
      const int64_t b = a.lr_ptr[f + r], e = a.lr_ptr[f + r + 1];
      for (int64_t k = b + sub; k < e; k += g) acc = fma(as_double(a.lr_val[k]), t[a.lr_col[k]], acc);
    }
    for (int o = g >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (r < q && sub == 0) t[f + r] = x[f + r] - acc;
  }
}

// backward: z_K = D_K (t_K - W_K z(C_K)); as in the forward sweep, groups
// of lanes per row: lane (jj, r) takes row r of W_K over the columns
// jj, jj + g, ... (W_K is column-major, so a wave reads it contiguously),
// then a fixed reduction tree over jj; v staged in LDS per wave
template <class T>
__global__ void __launch_bounds__(256) backward_level(SweepArgs<T> a, const double* t, double* z) {
  __shared__ double sv[4][kMaxWidth];
  if (a.skip && *a.skip) return;  // uniform: before the barrier
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
    const T* W = a.wval + a.f.woff[K];
    int qp = 1;
    while (qp < q && qp < 64) qp <<= 1;
    const int g = 64 / qp;  // column groups
    for (int r0 = 0; r0 < q; r0 += qp) {
      const int r = r0 + (lane & (qp - 1)), jj = lane / qp;
      double acc = 0.0;
      if (r < q)
        for (int j = jj; j < m; j += g) acc = fma(as_double(W[(int64_t)j * q + r]), z[Cc[j]], acc);
      for (int o = 32; o >= qp; o >>= 1) acc += __shfl_xor(acc, o, 64);
      if (jj == 0 && r < q) sv[wv][r] = t[f + r] - acc;
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

// ---------------------------------------------------------------------------
// Dataflow apply: one launch runs every forward block, then every backward
// block, in the plan's level order (slots 0..nb-1 forward, nb..2nb-1
// backward), one wave per slot: workgroup g runs slots 4g + wave, g its
// index (the hardware starts a launch's workgroups in index order) or, with
// ticketed, its rank in an atomic ticket counter taken when it starts (no
// assumption on the start order; one atomic on one address per workgroup,
// several times slower).  A value of t (z) is its own ready mark: both start
// as kPending, a bit pattern (a signalling NaN) that no arithmetic
// produces, and a consumer polls the value with device-scope atomic loads
// until the producer's atomic store replaces it.  Every dependency of a
// slot sits at a lower slot, and every workgroup holding a lower slot has
// started before the one holding the lowest unfinished slot, so that slot's
// inputs are all published and every wait ends, with no workgroup having to
// be resident for another.  Waits are bounded anyway (err).
// The arithmetic is that of forward_level and backward_level, in the same
// order.
// ---------------------------------------------------------------------------
// both halves 0x7ff4b11e: a signalling NaN, set with a 32-bit fill
constexpr unsigned kPendingHalf = 0x7ff4b11eu;
constexpr unsigned long long kPending = ((unsigned long long)kPendingHalf << 32) | kPendingHalf;

template <class T>
struct FlowApplyArgs {
  FactorView f;
  const int64_t* lr_ptr;
  const int32_t* lr_col;
  const T* lr_val;       // row-major L in the apply precision
  const T* wval;         // W values in the apply precision, at f.woff
  const int2* fq;        // forward slots: first row and width
  const int32_t* lev_b;  // backward slots: block
  int nb;
  const double* x;
  unsigned long long* t;
  unsigned long long* z;
  int* err;             // [0] set on a timeout; [1] slot, [2] side, [3] awaited index;
                        // [4] the ticket counter
  int ticketed;         // 1: slots by ticket; 0: by workgroup index (dispatch order)
  unsigned long long wait_ticks;
  const int* skip;      // when set and nonzero (a converged solver step): no work
};

// Values of t (side 0) or z (side 1) at idx for the lanes with has set, once
// every one of them is published; the whole wave waits together (no lane
// spins on its own).  On a timeout the first one records where it waited.
template <class A>
__device__ __forceinline__ unsigned long long peek_value(const A& a, int side, bool has,
                                                         int64_t idx) {
  return has ? __hip_atomic_load((side ? a.z : a.t) + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
             : 0ull;
}
// As await_values, from a value v read before (peek_value).
template <class A>
__device__ __forceinline__ double await_from(const A& a, int side, bool has, int64_t idx,
                                             unsigned long long v, unsigned long long t0, bool& bad,
                                             int slot) {
  unsigned long long* p = (side ? a.z : a.t) + (has ? idx : 0);
  while (!__all(!has || v != kPending)) {
    if (__any(bad)) {
      bad = true;
      return 0.0;
    }
    __builtin_amdgcn_s_sleep(1);
    // the value's reload, the error word and the clock go out together
    // (one round trip per poll)
    const unsigned long long nv =
        has && v == kPending ? __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : v;
    const int err = __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned long long now = wall_clock64();
    v = nv;
    if (err != 0) {
      bad = true;
      return 0.0;
    }
    if (now - t0 > a.wait_ticks && !__all(!has || v != kPending)) {
      if (has && v == kPending && atomicCAS(&a.err[0], 0, 1) == 0) {
        a.err[1] = slot;
        a.err[2] = side;
        a.err[3] = (int)idx;
      }
      bad = true;
      return 0.0;
    }
  }
  return __longlong_as_double((long long)v);
}
template <class A>
__device__ __forceinline__ double await_values(const A& a, int side, bool has, int64_t idx,
                                               unsigned long long t0, bool& bad, int slot) {
  return await_from(a, side, has, idx, peek_value(a, side, has, idx), t0, bad, slot);
}
__device__ __forceinline__ void publish_value(unsigned long long* p, double v) {
  __hip_atomic_store(p, (unsigned long long)__double_as_longlong(v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = max(v, __shfl_xor(v, o, 64));
  return v;
}

constexpr int kPre = 4;  // dependency steps of the dataflow apply loaded together

template <class T>
__global__ void __launch_bounds__(256) apply_flow(FlowApplyArgs<T> a) {
  __shared__ double sv[4][kMaxWidth];
  __shared__ int s_id;
  if (a.skip && *a.skip) return;  // uniform across the launch
  int id = blockIdx.x;
  if (a.ticketed) {
    if (threadIdx.x == 0) s_id = atomicAdd(&a.err[4], 1);
    __syncthreads();
    id = s_id;
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int s = id * 4 + wv;
  // no workgroup barrier below: each wave runs its own slot
  if (s < 2 * a.nb) {
    const unsigned long long t0 = wall_clock64();
    const int2 cur = s < a.nb ? a.fq[s] : make_int2(a.lev_b[s - a.nb], 0);
    bool bad = false;
    if (s < a.nb) {
      const int f = cur.x, q = cur.y;
      int qp = 1;
      while (qp < q && qp < 64) qp <<= 1;
      const int g = 64 / qp;  // lanes per row
      for (int r0 = 0; r0 < q; r0 += qp) {
        const int r = r0 + lane / g, sub = lane % g;
        int64_t b = 0, e = 0;
        if (r < q) {
          b = a.lr_ptr[f + r] + sub;
          e = a.lr_ptr[f + r + 1];
        }
        const int steps = wave_max_int(b < e ? (int)((e - b + g - 1) / g) : 0);
        const double xv = r < q && sub == 0 ? a.x[f + r] : 0.0;
        double acc = 0.0;
        // kPre steps at a time: their index, value and t loads go out
        // together, then the sum runs in step order
        for (int i0 = 0; i0 < steps; i0 += kPre) {
          int col[kPre];
          double lv[kPre];
          unsigned long long tv0[kPre];
          bool has[kPre];
#pragma unroll
          for (int u = 0; u < kPre; ++u) {
            const int64_t k = b + (int64_t)(i0 + u) * g;
            has[u] = i0 + u < steps && k < e;
            col[u] = has[u] ? a.lr_col[k] : 0;
            lv[u] = has[u] ? as_double(a.lr_val[k]) : 0.0;
          }
#pragma unroll
          for (int u = 0; u < kPre; ++u) tv0[u] = peek_value(a, 0, has[u], col[u]);
#pragma unroll
          for (int u = 0; u < kPre; ++u) {
            const double tv = await_from(a, 0, has[u], col[u], tv0[u], t0, bad, s);
            if (has[u]) acc = fma(lv[u], tv, acc);
          }
        }
        for (int o = g >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (r < q && sub == 0) publish_value(&a.t[f + r], xv - acc);
      }
    } else {
      const int K = cur.x;
      const int f = a.f.bstart[K], q = a.f.bstart[K + 1] - f;
      const int m = a.f.nc[K];
      const int32_t* Cc = a.f.idx + a.f.coff[K];
      const T* W = a.wval + a.f.woff[K];
      int qp = 1;
      while (qp < q && qp < 64) qp <<= 1;
      const int g = 64 / qp;  // column groups
      const int steps = (m + g - 1) / g;
      for (int r0 = 0; r0 < q; r0 += qp) {
        const int r = r0 + (lane & (qp - 1)), jj = lane / qp;
        const bool own = jj == 0 && r < q;
        const unsigned long long tv0 = peek_value(a, 0, own, f + r);  // usually there
        double acc = 0.0;
        for (int i0 = 0; i0 < steps; i0 += kPre) {
          int col[kPre];
          double wv[kPre];
          unsigned long long zv0[kPre];
          bool has[kPre];
#pragma unroll
          for (int u = 0; u < kPre; ++u) {
            const int j = jj + (i0 + u) * g;
            has[u] = i0 + u < steps && r < q && j < m;
            col[u] = has[u] ? Cc[j] : 0;
            wv[u] = has[u] ? as_double(W[(int64_t)j * q + r]) : 0.0;
          }
#pragma unroll
          for (int u = 0; u < kPre; ++u) zv0[u] = peek_value(a, 1, has[u], col[u]);
#pragma unroll
          for (int u = 0; u < kPre; ++u) {
            const double zv = await_from(a, 1, has[u], col[u], zv0[u], t0, bad, s);
            if (has[u]) acc = fma(wv[u], zv, acc);
          }
        }
        for (int o = 32; o >= qp; o >>= 1) acc += __shfl_xor(acc, o, 64);
        const double tv = await_from(a, 0, own, f + r, tv0, t0, bad, s);
        if (own) sv[wv][r] = tv - acc;
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
      const double* D = a.f.dval + a.f.doff[K];
      for (int r = lane; r < q; r += 64) {
        double acc = 0.0;
        for (int c = 0; c < q; ++c) acc = fma(D[r * q + c], sv[wv][c], acc);
        publish_value(&a.z[f + r], acc);
      }
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
    }
    if (__any(bad)) return;
  }
}

// Before a dataflow apply: t and z become kPending and the ticket and wait
// words are cleared.  A timeout of the previous apply (err[0]) is added to
// err[5], which only apply_faults() reads and clears, so no fault is lost.
// A fill kernel rather than a memset, so a captured graph can hold it.
__global__ void apply_reset(int64_t n, unsigned long long* t, unsigned long long* z, int* err,
                            const int* skip) {
  if (skip && *skip) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    t[i] = kPending;
    z[i] = kPending;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (err[0]) err[5] += 1;
    for (int k = 0; k < 5; ++k) err[k] = 0;
  }
}

// y = A x, CSR, 8 lanes per row.
__global__ void __launch_bounds__(256) spmv_csr(int64_t n, const int64_t* rp, const int32_t* ci,
                                                const double* v, const double* x, double* y,
                                                const int* skip) {
  if (skip && *skip) return;
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

__global__ void gather_k(int64_t n, const int32_t* perm, const double* scale, const double* x,
                         double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (perm ? x[perm[i]] : x[i]) * (scale ? scale[i] : 1.0);
}
__global__ void scatter_k(int64_t n, const int32_t* perm, const double* scale, const double* x,
                          double* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    y[perm[i]] = scale ? x[i] * scale[i] : x[i];
}
__global__ void axpy_dev_k(int64_t n, const double* alpha, double sign, const double* x, double* y,
                           const int* skip) {
  if (skip && *skip) return;
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
__global__ void scale_dev_k(int64_t n, const double* alpha, const double* x, double* y,
                            const int* skip) {
  if (skip && *skip) return;
  const double a = *alpha;
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
                                                   double* partial, const int* skip) {
  __shared__ double sw[4];
  if (skip && *skip) return;
  double acc = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    acc = fma(x[i], y[i], acc);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = (sw[0] + sw[1]) + (sw[2] + sw[3]);
}
__global__ void __launch_bounds__(256) dot_final(int nparts, const double* partial, double* out,
                                                 const int* skip) {
  __shared__ double sw[4];
  if (skip && *skip) return;
  double acc = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) acc += partial[i];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *out = (sw[0] + sw[1]) + (sw[2] + sw[3]);
}

// FP32 copies of FP64 factor values (apply_precision F32).
__global__ void convert_values(int64_t n, const double* x, float* y) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    y[i] = (float)x[i];
}

// Calls f with a value of the type that holds values of precision prec.
template <class F>
void with_value_type(int prec, F&& f) {
  if (prec == kValF32)
    f(float{});
  else if (prec == kValBF16)
    f(uint16_t{});
  else
    f(double{});
}

// FGMRES on the device: the Hessenberg column of step j, its Givens
// rotation and the residual estimate, and the triangular solve of a cycle,
// by one thread, with the operations (no contraction into fused
// multiply-adds, IEEE square root and division) of the host version.
// flags: [0] the cycle is done (the solver's kernels skip their work),
// [1] steps taken (jend), [2] breakdown.
__global__ void gm_init(GmState g, int m, double beta) {
  if (threadIdx.x != 0) return;
  g.g[0] = beta;
  for (int i = 1; i <= m; ++i) g.g[i] = 0.0;
  g.flags[0] = g.flags[1] = g.flags[2] = g.flags[3] = 0;
}
__global__ void gm_update(GmState g, int j, int m, double target_inner, long long it_before,
                          long long maxit) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0 || g.flags[0]) return;
  const double* col = g.hcol;
  double* H = g.H;
  const double hn = sqrt(col[j + 1]);
  const double wn0 = sqrt(col[m + 1]);
  for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = col[i];
  H[(size_t)(j + 1) * m + j] = hn;
  for (int i = 0; i < j; ++i) {
    const double a0 = H[(size_t)i * m + j], a1 = H[(size_t)(i + 1) * m + j];
    H[(size_t)i * m + j] = g.cs[i] * a0 + g.sn[i] * a1;
    H[(size_t)(i + 1) * m + j] = -g.sn[i] * a0 + g.cs[i] * a1;
  }
  const double hjj = H[(size_t)j * m + j], hj1 = H[(size_t)(j + 1) * m + j];
  if (hj1 == 0.0) {
    g.cs[j] = 1.0;
    g.sn[j] = 0.0;
  } else if (fabs(hj1) > fabs(hjj)) {
    const double t = hjj / hj1;
    g.sn[j] = 1.0 / sqrt(1.0 + t * t);
    g.cs[j] = g.sn[j] * t;
  } else {
    const double t = hj1 / hjj;
    g.cs[j] = 1.0 / sqrt(1.0 + t * t);
    g.sn[j] = g.cs[j] * t;
  }
  H[(size_t)j * m + j] = g.cs[j] * hjj + g.sn[j] * hj1;
  H[(size_t)(j + 1) * m + j] = 0.0;
  g.g[j + 1] = -g.sn[j] * g.g[j];
  g.g[j] = g.cs[j] * g.g[j];
  const double est = fabs(g.g[j + 1]);
  const bool breakdown = hn <= 1e-14 * wn0;
  *g.inv_hn = breakdown ? 0.0 : 1.0 / hn;
  g.flags[1] = j + 1;
  g.flags[2] = breakdown ? 1 : 0;
  if (est <= target_inner || breakdown || it_before + j + 1 >= maxit || j + 1 >= m) g.flags[0] = 1;
}
__global__ void gm_solve(GmState g, int m) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0) return;
  const int jend = g.flags[1];
  for (int i = jend - 1; i >= 0; --i) {
    double acc = g.g[i];
    for (int k = i + 1; k < jend; ++k) acc -= g.H[(size_t)i * m + k] * g.y[k];
    g.y[i] = acc / g.H[(size_t)i * m + i];
  }
}

// SQMR on the device.  The scalar recurrences of a step run on one thread
// with the operations of the host version (no contraction into fused
// multiply-adds, IEEE square root and division); a kernel that finds the
// stop flag set does nothing.
__device__ inline double block_max(double v, double* sw) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sw[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = fmax(fmax(sw[0], sw[1]), fmax(sw[2], sw[3]));
  __syncthreads();
  return r;
}
__global__ void sq_init(SqState g) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0) return;
  g.s[kSqTau] = sqrt(g.s[kSqRR]);
  g.s[kSqTheta] = 0.0;
  g.s[kSqRho] = g.s[kSqRhoNew];
  g.flags[0] = g.flags[1] = g.flags[2] = g.flags[3] = 0;
}
__global__ void sq_resume(SqState g) {
  if (threadIdx.x == 0) g.flags[0] = g.flags[1] = 0;
}
// alpha = rho_{k-1} / sigma; rho_{k-1} becomes the previous step's value
__global__ void sq_alpha(SqState g) {
  if (threadIdx.x != 0 || g.flags[0]) return;
  const double rho = g.s[kSqRhoNew];
  g.s[kSqRho] = rho;
  const double sigma = g.s[kSqSigma];
  if (sigma == 0.0) {
    g.flags[1] = 2;
    g.flags[0] = 1;
    return;
  }
  g.s[kSqAlpha] = rho / sigma;
}
__global__ void sq_theta(SqState g) {
#pragma clang fp contract(off)
  if (threadIdx.x != 0 || g.flags[0]) return;
  const double theta_old = g.s[kSqTheta];
  const double theta = sqrt(g.s[kSqRR]) / g.s[kSqTau];
  const double c = 1.0 / sqrt(1.0 + theta * theta);
  const double c2 = c * c;
  g.s[kSqTau] = g.s[kSqTau] * theta * c;
  g.s[kSqTheta] = theta;
  g.s[kSqCd] = c2 * theta_old * theta_old;
  g.s[kSqCq] = c2 * g.s[kSqAlpha];
}
__global__ void __launch_bounds__(256) sq_update(int64_t n, SqState g, const double* q,
                                                 const double* t, double* d, double* sv,
                                                 double* x, double* rq, const double* xs,
                                                 const double* rs) {
#pragma clang fp contract(off)
  __shared__ double sw[4];
  if (g.flags[0]) return;
  const double cd = g.s[kSqCd], cq = g.s[kSqCq];
  double mx = 0.0, mr = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double di = cd * d[i] + cq * q[i];
    const double si = cd * sv[i] + cq * t[i];
    const double xi = x[i] + di;
    const double ri = rq[i] - si;
    d[i] = di;
    sv[i] = si;
    x[i] = xi;
    rq[i] = ri;
    mx = fmax(mx, fabs(xs ? xi * xs[i] : xi));
    mr = fmax(mr, fabs(rs ? ri * rs[i] : ri));
  }
  mx = block_max(mx, sw);
  mr = block_max(mr, sw);
  if (threadIdx.x == 0) {
    g.part[blockIdx.x] = mx;
    g.part[kSqParts + blockIdx.x] = mr;
  }
}
// the maxima, eta = ||rq|| / (||A|| ||x|| + ||b||) and the stop test
__global__ void __launch_bounds__(256) sq_check(SqState g, double tol, long long maxit) {
#pragma clang fp contract(off)
  __shared__ double sw[4];
  if (g.flags[0]) return;
  double mx = 0.0, mr = 0.0;
  for (int i = threadIdx.x; i < kSqParts; i += blockDim.x) {
    mx = fmax(mx, g.part[i]);
    mr = fmax(mr, g.part[kSqParts + i]);
  }
  mx = block_max(mx, sw);
  mr = block_max(mr, sw);
  if (threadIdx.x != 0) return;
  g.s[kSqXmax] = mx;
  g.s[kSqRmax] = mr;
  const double eta = mr == 0.0 ? 0.0 : mr / (g.s[kSqAnorm] * mx + g.s[kSqBmax]);
  g.s[kSqEta] = eta;
  const int steps = g.flags[2] + 1;
  g.flags[2] = steps;
  int why = 0;
  if (eta <= tol)
    why = 1;
  else if (steps >= maxit)
    why = 3;
  else if (g.s[kSqRho] == 0.0)
    why = 2;
  if (why) {
    g.flags[1] = why;
    g.flags[0] = 1;
  }
}
__global__ void sq_direction(int64_t n, SqState g, const double* u, double* q) {
#pragma clang fp contract(off)
  if (g.flags[0]) return;
  const double beta = g.s[kSqRhoNew] / g.s[kSqRho];
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    q[i] = u[i] + beta * q[i];
}
// max_i |v_i w_i| (rp NULL), or the largest row sum max_i rs_i sum_k
// |v_k| cs_{ci_k} of a CSR matrix (scales NULL: 1)
__global__ void __launch_bounds__(256) amax_partial(int64_t n, const int64_t* rp,
                                                    const int32_t* ci, const double* v,
                                                    const double* rs, const double* cs,
                                                    double* partial) {
  __shared__ double sw[4];
  double m = 0.0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if (rp) {
      double a = 0.0;
      for (int64_t k = rp[i]; k < rp[i + 1]; ++k) a += fabs(cs ? v[k] * cs[ci[k]] : v[k]);
      m = fmax(m, rs ? a * rs[i] : a);
    } else {
      m = fmax(m, fabs(rs ? v[i] * rs[i] : v[i]));
    }
  }
  m = block_max(m, sw);
  if (threadIdx.x == 0) partial[blockIdx.x] = m;
}
__global__ void __launch_bounds__(256) amax_final(int nparts, const double* partial, double* out) {
  __shared__ double sw[4];
  double m = 0.0;
  for (int i = threadIdx.x; i < nparts; i += blockDim.x) m = fmax(m, partial[i]);
  m = block_max(m, sw);
  if (threadIdx.x == 0) *out = m;
}

inline unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 4096));
}

}  // namespace

void launch_gather(hipStream_t s, int64_t n, const int32_t* perm, const double* scale, const double* x,
                   double* y) {
  gather_k<<<grid_for(n), 256, 0, s>>>(n, perm, scale, x, y);
}
void launch_scatter(hipStream_t s, int64_t n, const int32_t* perm, const double* scale,
                    const double* x, double* y) {
  scatter_k<<<grid_for(n), 256, 0, s>>>(n, perm, scale, x, y);
}
void launch_mul(hipStream_t s, int64_t n, const double* w, const double* x, double* y) {
  gather_k<<<grid_for(n), 256, 0, s>>>(n, nullptr, w, x, y);
}
void launch_axpy(hipStream_t s, int64_t n, const double* alpha_dev, double sign, const double* x,
                 double* y, const int* skip) {
  axpy_dev_k<<<grid_for(n), 256, 0, s>>>(n, alpha_dev, sign, x, y, skip);
}
void launch_axpy_host(hipStream_t s, int64_t n, double alpha, const double* x, double* y) {
  axpy_k<<<grid_for(n), 256, 0, s>>>(n, alpha, x, y);
}
void launch_scale(hipStream_t s, int64_t n, double alpha, const double* x, double* y) {
  scale_k<<<grid_for(n), 256, 0, s>>>(n, alpha, x, y);
}
void launch_scale_dev(hipStream_t s, int64_t n, const double* alpha_dev, const double* x, double* y,
                      const int* skip) {
  scale_dev_k<<<grid_for(n), 256, 0, s>>>(n, alpha_dev, x, y, skip);
}
void launch_sub(hipStream_t s, int64_t n, const double* b, const double* ax, double* r) {
  sub_k<<<grid_for(n), 256, 0, s>>>(n, b, ax, r);
}
void launch_gm_init(hipStream_t s, const GmState& g, int m, double beta) {
  gm_init<<<1, 64, 0, s>>>(g, m, beta);
}
void launch_gm_update(hipStream_t s, const GmState& g, int j, int m, double target_inner,
                      int64_t it_before, int64_t maxit) {
  gm_update<<<1, 64, 0, s>>>(g, j, m, target_inner, (long long)it_before, (long long)maxit);
}
void launch_gm_solve(hipStream_t s, const GmState& g, int m) { gm_solve<<<1, 64, 0, s>>>(g, m); }
void launch_dot(hipStream_t s, int64_t n, const double* x, const double* y, double* partial,
                double* out, const int* skip) {
  dot_partial<<<kDotBlocks, 256, 0, s>>>(n, x, y, partial, skip);
  dot_final<<<1, 256, 0, s>>>(kDotBlocks, partial, out, skip);
}

void launch_sq_init(hipStream_t s, const SqState& g) { sq_init<<<1, 64, 0, s>>>(g); }
void launch_sq_resume(hipStream_t s, const SqState& g) { sq_resume<<<1, 64, 0, s>>>(g); }
void launch_sq_alpha(hipStream_t s, const SqState& g) { sq_alpha<<<1, 64, 0, s>>>(g); }
void launch_sq_theta(hipStream_t s, const SqState& g) { sq_theta<<<1, 64, 0, s>>>(g); }
void launch_sq_update(hipStream_t s, int64_t n, const SqState& g, const double* q, const double* t,
                      double* d, double* sv, double* x, double* rq, const double* xs,
                      const double* rs, double tol, int64_t maxit) {
  sq_update<<<kSqParts, 256, 0, s>>>(n, g, q, t, d, sv, x, rq, xs, rs);
  sq_check<<<1, 256, 0, s>>>(g, tol, (long long)maxit);
}
void launch_sq_direction(hipStream_t s, int64_t n, const SqState& g, const double* u, double* q) {
  sq_direction<<<grid_for(n), 256, 0, s>>>(n, g, u, q);
}
void launch_amax(hipStream_t s, int64_t n, const double* x, const double* w, double* partial,
                 double* out) {
  amax_partial<<<kDotBlocks, 256, 0, s>>>(n, nullptr, nullptr, x, w, nullptr, partial);
  amax_final<<<1, 256, 0, s>>>(kDotBlocks, partial, out);
}
void launch_row_amax(hipStream_t s, int64_t n, const int64_t* rp, const int32_t* ci,
                     const double* v, const double* rs, const double* cs, double* partial,
                     double* out) {
  amax_partial<<<kDotBlocks, 256, 0, s>>>(n, rp, ci, v, rs, cs, partial);
  amax_final<<<1, 256, 0, s>>>(kDotBlocks, partial, out);
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
                                                                   h->d_rv.p, x, y, h->run_skip);
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

// For every block K, the blocks J whose stored rows (cols: columns) fall into
// K, ascending, each with the first position of that run in R_J (C_J) and
// its length: ptr [nb+1], then j, s0 and cnt per entry.
bilu_status block_runs(bilu_handle* h, const FactorView& f, bool cols, DevArray<int32_t>& ptr,
                       DevArray<int32_t>& j, DevArray<int32_t>& s0, DevArray<int32_t>& cnt) {
  hipStream_t st = h->stream;
  const int64_t nb = f.nb;
#define CK(x)                                          \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return hip_check(h, e_, #x); \
  } while (0)
  const unsigned gw = (unsigned)((nb + 3) / 4);  // one wave per block
  DevArray<int32_t> c;
  CK(c.alloc(nb + 1));
  CK(hipMemsetAsync(c.p, 0, (nb + 1) * sizeof(int32_t), st));
  fw_count<<<gw, 256, 0, st>>>(f, c.p, cols ? 1 : 0);
  CK(ptr.alloc(nb + 1));
  int32_t total = 0;
  CK(device_scan<int32_t>(h, c.p, ptr.p, nb, &total));
  const int64_t ne = std::max<int64_t>(1, total);
  CK(j.alloc(ne));
  CK(s0.alloc(ne));
  CK(cnt.alloc(ne));
  DevArray<unsigned long long> keys;
  CK(keys.alloc(ne));
  CK(hipMemsetAsync(c.p, 0, (nb + 1) * sizeof(int32_t), st));
  fw_fill<<<gw, 256, 0, st>>>(f, ptr.p, c.p, keys.p, cols ? 1 : 0);
  fw_sort<<<gw, 256, 0, st>>>((int)nb, ptr.p, keys.p, j.p, s0.p, cnt.p);
  CK(hipGetLastError());
  CK(hipStreamSynchronize(st));  // keys and counts are freed here
  return BILU_OK;
#undef CK
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
  {
    const bilu_status rs = block_runs(h, f, false, h->fw_ptr, h->fw_j, h->fw_r0, h->fw_cnt);
    if (rs != BILU_OK) return rs;
  }
  // backward successor blocks
  bw_count<<<gw, 256, 0, st>>>(f, cnt.p);
  CK(h->bw_ptr.alloc(nb + 1));
  int32_t nbw = 0;
  CK(device_scan<int32_t>(h, cnt.p, h->bw_ptr.p, nb, &nbw));
  CK(h->bw_b.alloc(std::max<int32_t>(1, nbw)));
  bw_fill<<<gw, 256, 0, st>>>(f, h->bw_ptr.p, h->bw_b.p);
  // the precision the apply reads L and W in: the stored one, or FP32
  // copies of FP64 values (apply_precision)
  h->apply_prec = f.vprec != kValF64 ? f.vprec
                  : h->opt.apply_precision == BILU_PREC_F32 ? kValF32
                                                             : kValF64;
  if (h->apply_prec != f.vprec) {
    CK(h->d_apply_val.alloc(std::max<int64_t>(1, h->f_val_len) * value_bytes(h->apply_prec)));
    convert_values<<<grid_for(h->f_val_len), 256, 0, st>>>(
        h->f_val_len, static_cast<const double*>(f.val),
        reinterpret_cast<float*>(h->d_apply_val.p));
  }
  // row-major L
  CK(h->lr_ptr.alloc(n + 1));
  DevArray<int64_t> lc;
  CK(lc.alloc(n));
  lr_build<false, double><<<gw, 256, 0, st>>>(f, h->fw_ptr.p, h->fw_j.p, h->fw_r0.p, h->fw_cnt.p,
                                               nullptr, lc.p, nullptr, nullptr);
  int64_t nlr = 0;
  CK(device_scan<int64_t>(h, lc.p, h->lr_ptr.p, n, &nlr));
  CK(h->lr_col.alloc(std::max<int64_t>(1, nlr)));
  CK(h->lr_val.alloc(std::max<int64_t>(1, nlr) * value_bytes(h->apply_prec)));
  with_value_type(h->apply_prec, [&](auto tag) {
    using T = decltype(tag);
    lr_build<true, T><<<gw, 256, 0, st>>>(f, h->fw_ptr.p, h->fw_j.p, h->fw_r0.p, h->fw_cnt.p,
                                          h->lr_ptr.p, nullptr, h->lr_col.p,
                                          reinterpret_cast<T*>(h->lr_val.p));
  });
  CK(hipGetLastError());
  // dependency levels (actual graph of the factor) on the device, then the
  // blocks of each direction ordered by (level, index)
  {
    DevArray<int> lev, misc;
    CK(lev.alloc(2 * nb));
    CK(misc.alloc(4));
    CK(hipMemsetAsync(lev.p, 0xff, 2 * nb * sizeof(int), st));
    CK(hipMemsetAsync(misc.p, 0, 4 * sizeof(int), st));
    // one wave per block and direction, ordinary launch (workgroups take
    // their slots from a ticket counter)
    const int64_t groups = std::max<int64_t>(1, (2 * nb + 3) / 4);
    unsigned long long wait = h->wait_ticks ? h->wait_ticks : (unsigned long long)1e9;
    int* lf = lev.p;
    int* lb = lev.p + nb;
    int* top = misc.p;
    int* err = misc.p + 2;
    int* ticket = h->eff.apply_path == 2 ? misc.p + 3 : nullptr;
    int nbi = (int)nb;
    // the slots in the order of the sweep's dependency depths, made
    // consistent with the apply's own dependencies by relaxation passes (a
    // merged block can hold a deeper member than a block that depends on
    // it); block order when the depths are not there or the passes do not
    // settle
    DevArray<int32_t> key, ord, sorted_keys, seq;
    const int32_t* slot_order = nullptr;
    const int64_t nb0 = h->stats.nblocks_initial;
    if (nb0 > 0 && h->d_flow.p && h->d_flow.n >= (size_t)(5 * nb0 + 8) && h->d_blockof.p &&
        h->d_blockof.n >= (size_t)n) {
      constexpr int kRounds = 8, kPasses = 2;
      DevArray<int> changed;
      CK(key.alloc(nb));
      CK(changed.alloc(kRounds * kPasses));
      CK(hipMemsetAsync(changed.p, 0, kRounds * kPasses * sizeof(int), st));
      plan_keys<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(nbi, f.bstart, h->d_blockof.p,
                                                             (int)nb0, h->d_flow.p + 3 * nb0, key.p);
      CK(hipGetLastError());
      bool settled = false;
      for (int r = 0; r < kRounds && !settled; ++r) {
        for (int q = 0; q < kPasses; ++q)
          plan_relax<<<gw, 256, 0, st>>>(nbi, h->fw_ptr.p, h->fw_j.p, h->bw_ptr.p, h->bw_b.p, key.p,
                                         changed.p + r * kPasses + q);
        CK(hipGetLastError());
        int last = 1;
        CK(hipMemcpyAsync(&last, changed.p + r * kPasses + kPasses - 1, sizeof(int),
                          hipMemcpyDeviceToHost, st));
        CK(hipStreamSynchronize(st));
        settled = last == 0;
      }
      if (settled) {
        // (key, index) ascending: a stable sort of the indices by key
        CK(ord.alloc(nb));
        CK(sorted_keys.alloc(nb));
        CK(seq.alloc(nb));
        iota_k<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(nbi, seq.p);
        CK(hipGetLastError());
        size_t bytes = 0;
        CK(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, key.p, sorted_keys.p, seq.p, ord.p,
                                              nbi, 0, 32, st));
        CK(h->d_scan_tmp.alloc(bytes + 1));
        CK(hipcub::DeviceRadixSort::SortPairs(h->d_scan_tmp.p, bytes, key.p, sorted_keys.p, seq.p,
                                              ord.p, nbi, 0, 32, st));
        slot_order = ord.p;
      }
    }
    apply_levels<<<(unsigned)groups, 256, 0, st>>>((int)nb, h->fw_ptr.p, h->fw_j.p, h->bw_ptr.p,
                                                  h->bw_b.p, slot_order, lf, lb, err, ticket, wait);
    CK(hipGetLastError());
    {
      // the largest level of each direction
      size_t rb = 0;
      CK(hipcub::DeviceReduce::Max(nullptr, rb, lf, top, nbi, st));
      CK(h->d_scan_tmp.alloc(rb + 1));
      CK(hipcub::DeviceReduce::Max(h->d_scan_tmp.p, rb, lf, top, nbi, st));
      CK(hipcub::DeviceReduce::Max(h->d_scan_tmp.p, rb, lb, top + 1, nbi, st));
    }
    int hm[4];
    CK(hipMemcpyAsync(hm, misc.p, sizeof(hm), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (hm[2]) return fail(h, BILU_ERR_DEVICE, "apply plan: a dependency wait timed out");
    // (level, index) order: stable radix sort of the levels with the indices
    DevArray<int32_t> idx, keys_out, starts;
    CK(idx.alloc(nb));
    CK(keys_out.alloc(2 * nb));
    CK(starts.alloc((int64_t)hm[0] + hm[1] + 4));
    CK(h->lev_f.alloc(nb));
    CK(h->lev_b.alloc(nb));
    iota_k<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(nbi, idx.p);
    CK(hipGetLastError());
    int bits = 1;
    while ((1 << bits) <= std::max(hm[0], hm[1])) ++bits;
    size_t bytes = 0;
    CK(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, lf, keys_out.p, idx.p, h->lev_f.p, nbi, 0,
                                          bits, st));
    CK(h->d_scan_tmp.alloc(bytes + 1));
    CK(hipcub::DeviceRadixSort::SortPairs(h->d_scan_tmp.p, bytes, lf, keys_out.p, idx.p, h->lev_f.p,
                                          nbi, 0, bits, st));
    CK(hipcub::DeviceRadixSort::SortPairs(h->d_scan_tmp.p, bytes, lb, keys_out.p + nb, idx.p,
                                          h->lev_b.p, nbi, 0, bits, st));
    int* sf = starts.p;
    int* sb = starts.p + hm[0] + 2;
    level_starts<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(nbi, keys_out.p, sf);
    CK(h->lev_f_fq.alloc(nb));
    slot_rows<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(nbi, h->lev_f.p, f.bstart, h->lev_f_fq.p);
    level_starts<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(nbi, keys_out.p + nb, sb);
    CK(hipGetLastError());
    h->lev_f_ptr.assign(hm[0] + 2, 0);
    h->lev_b_ptr.assign(hm[1] + 2, 0);
    CK(hipMemcpyAsync(h->lev_f_ptr.data(), sf, (hm[0] + 2) * sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(h->lev_b_ptr.data(), sb, (hm[1] + 2) * sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    for (const auto* v : {&h->lev_f_ptr, &h->lev_b_ptr})
      for (size_t l = 0; l + 1 < v->size(); ++l)
        if ((*v)[l] >= (*v)[l + 1] || v->back() != nb)
          return fail(h, BILU_ERR_INTERNAL, "apply plan: inconsistent dependency levels");
    h->stats.apply_levels_fwd = (int64_t)h->lev_f_ptr.size() - 1;
    h->stats.apply_levels_bwd = (int64_t)h->lev_b_ptr.size() - 1;
  }
  CK(h->w_red.alloc(kDotBlocks + 64));
  CK(h->d_apply_err.alloc(8));
  CK(hipMemsetAsync(h->d_apply_err.p, 0, 8 * sizeof(int), st));
  CK(hipStreamSynchronize(st));
  return BILU_OK;
#undef CK
}

bilu_status refresh_apply_values(bilu_handle* h) {
  hipStream_t st = h->stream;
  const FactorView& f = h->fv;
  const int64_t nb = f.nb;
  const unsigned gw = (unsigned)((nb + 3) / 4);
  if (h->apply_prec != f.vprec)
    convert_values<<<grid_for(h->f_val_len), 256, 0, st>>>(
        h->f_val_len, static_cast<const double*>(f.val), reinterpret_cast<float*>(h->d_apply_val.p));
  with_value_type(h->apply_prec, [&](auto tag) {
    using T = decltype(tag);
    lr_build<true, T><<<gw, 256, 0, st>>>(f, h->fw_ptr.p, h->fw_j.p, h->fw_r0.p, h->fw_cnt.p,
                                          h->lr_ptr.p, nullptr, h->lr_col.p,
                                          reinterpret_cast<T*>(h->lr_val.p));
  });
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return hip_check(h, e, "refresh apply values");
  return BILU_OK;
}

// W values the apply reads: the stored ones, or their FP32 copy.
template <class T>
static const T* apply_w(const bilu_handle* h) {
  return reinterpret_cast<const T*>(h->apply_prec == h->fv.vprec ? h->fv.val
                                                                  : (const void*)h->d_apply_val.p);
}

// One launch per dependency level (forward_level, backward_level).
template <class T>
static void apply_levels_launch(bilu_handle* h, const double* x, double* y, double* t) {
  hipStream_t st = h->stream;
  SweepArgs<T> a{};
  a.f = h->fv;
  a.lr_ptr = h->lr_ptr.p;
  a.lr_col = h->lr_col.p;
  a.lr_val = reinterpret_cast<const T*>(h->lr_val.p);
  a.wval = apply_w<T>(h);
  a.sched = h->lev_f.p;
  a.fq = h->lev_f_fq.p;
  a.skip = h->run_skip;
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
}

bilu_status apply_permuted(bilu_handle* h, const double* x, double* y, double* t, bool timed) {
  hipStream_t st = h->stream;
  const int64_t n = h->n;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  timed = timed && h->opt.collect_timing;
  if (timed) {
    e0 = h->ev_get();
    e1 = h->ev_get();
    if (e0) (void)hipEventRecord(e0, st);
  }
  with_value_type(h->apply_prec, [&](auto tag) {
  using T = decltype(tag);
  if (h->eff.apply_path == 1) {
    apply_levels_launch<T>(h, x, y, t);
  } else {
    FlowApplyArgs<T> a{};
    a.f = h->fv;
    a.lr_ptr = h->lr_ptr.p;
    a.lr_col = h->lr_col.p;
    a.lr_val = reinterpret_cast<const T*>(h->lr_val.p);
    a.wval = apply_w<T>(h);
    a.fq = h->lev_f_fq.p;
    a.lev_b = h->lev_b.p;
    a.nb = (int)h->fv.nb;
    a.x = x;
    a.t = reinterpret_cast<unsigned long long*>(t);
    a.z = reinterpret_cast<unsigned long long*>(y);
    a.err = h->d_apply_err.p;
    // every wait ends (see apply_flow); the bound only catches a fault
    a.wait_ticks = (h->wait_ticks ? h->wait_ticks : (unsigned long long)1e9) / 5;
    a.ticketed = h->eff.apply_path == 2 ? 1 : 0;
    a.skip = h->run_skip;
    apply_reset<<<grid_for(n), 256, 0, st>>>(n, a.t, a.z, a.err, a.skip);
    apply_flow<T><<<(unsigned)((2 * h->fv.nb + 3) / 4), 256, 0, st>>>(a);
  }
  });
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_check(h, e, "apply launch");
  if (timed) {
    if (e1) (void)hipEventRecord(e1, st);
    h->ev_record(1, e0, e1);
  }
  return BILU_OK;
}

// Dataflow applies whose waits timed out since the last call (synchronizes
// the stream); the count is cleared.
bilu_status apply_faults(bilu_handle* h, int64_t* count) {
  *count = 0;
  if (!h->d_apply_err.p) return BILU_OK;
  int e[6];
  hipStream_t st = h->stream;
  hipError_t r = hipMemcpyAsync(e, h->d_apply_err.p, sizeof(e), hipMemcpyDeviceToHost, st);
  if (r == hipSuccess) r = hipStreamSynchronize(st);
  if (r != hipSuccess) return hip_check(h, r, "apply status");
  *count = (int64_t)e[5] + (e[0] ? 1 : 0);
  if (*count == 0) return BILU_OK;
  // clear both words (the next apply_reset would count e[0] again)
  r = hipMemsetAsync(h->d_apply_err.p, 0, 8 * sizeof(int), st);
  if (r == hipSuccess) r = hipStreamSynchronize(st);
  if (r != hipSuccess) return hip_check(h, r, "apply status");
  h->stats.apply_faults += *count;
  return fail(h, BILU_ERR_DEVICE,
              "apply: a dependency wait timed out (slot " + std::to_string(e[1]) + ", side " +
                  std::to_string(e[2]) + ", index " + std::to_string(e[3]) + ")");
}

}  // namespace bilu
