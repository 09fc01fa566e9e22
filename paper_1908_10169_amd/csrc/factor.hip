// Numeric block Crout sweep (Sec. 2.2) on the GPU.
//
// One workgroup computes one block column K of L and block row K of U:
//   1. the predecessors J whose stored block row has columns inside K (for
//      the column panel) or whose block column has rows inside K (for the
//      row panel) are read from K's predecessor lists, which every finished
//      J appends itself to;
//   2. candidate rows/columns (structural entries of A plus the stored
//      rows/columns of those J) are deduplicated in an LDS hash and sorted;
//   3. the panels are gathered from A and updated C -= L_J W_J for every J
//      in increasing order (fixed order: results are run-to-run identical);
//   4. the pivot block S_K is perturbed if needed (Sec. 3.6) and inverted by
//      Gauss-Jordan elimination with partial pivoting (lowest row on ties);
//   5. rows L(i,K) = C(i,K) D_K and columns D_K R(K,j) are dropped when
//      their norm is <= tau, the kept ones compacted into the factor heap
//      (L scaled, W = R unscaled), and K is appended to the predecessor lists
//      of the blocks it will update.
// Scheduling.  J can update K > J only if K holds one of J's candidate rows
// or columns, i.e. (a) A couples J and K, or (b) a predecessor I of J has
// stored rows (columns) in K and J among its stored column (row) blocks.
// pending[K] counts these possible updaters with multiplicity: (a) once per
// entry of A coupling K to an earlier block, set before the sweep; (b) is
// added by I when it finishes, for every pair (J, K)
// its stored patterns create, before I retracts its own counts; J retracts
// all of its counts once its factor is written and it has appended itself
// to the lists of the blocks it really updates.  Every possible updater of
// K is therefore counted before its own cause is retracted, so pending[K]
// reaches zero once, when K's predecessor lists are complete.  The
// retraction that reaches zero pushes K to a queue; running workgroups
// claim queue positions in ascending order and take the blocks there, so
// blocks run in readiness order and the critical path is the longest chain
// of possible updates after dropping, not the elimination-tree height.
// Queue waits are bounded in wall-clock time and end on any reported error.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include <hipcub/hipcub.hpp>

#include "internal.h"
#include "wg.h"

namespace bilu {
namespace {

// Device-scope ordering.  A block's results become visible to blocks on
// other XCDs by a release (L2 write-back) before it retracts its counts; a
// worker acquires (L2 invalidate) once after taking a block from the queue.
// Both act on whole caches that every wave of the workgroup shares (its
// CU's L1 and its XCD's L2), so wave 0 issues them for the workgroup, one
// of each per block.
__device__ __forceinline__ void release_agent() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void acquire_agent() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
// The cache operation of wave 0 has completed (it counts as a vector memory
// operation) before the barrier lets the other waves go on.
__device__ __forceinline__ void wait_vector_memory() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }
// Every wave waits until its own stores are acknowledged (they are in the
// L2), then wave 0 writes the L2 back; no wave goes on before that is done.
__device__ __forceinline__ void wg_release_agent() {
  wait_vector_memory();
  __syncthreads();
  if (threadIdx.x < 64) {
    release_agent();
    wait_vector_memory();
  }
  __syncthreads();
}
// Wave 0 invalidates; the barrier keeps every wave's later loads after it.
__device__ __forceinline__ void wg_acquire_agent() {
  if (threadIdx.x < 64) {
    acquire_agent();
    wait_vector_memory();
  }
  __syncthreads();
}

__device__ __forceinline__ void raise_error(const FactorArgs& a, int code, int blk) {
  if (atomicCAS(a.err, 0, code) == 0) atomicExch(a.err_block, blk);
}

__device__ __forceinline__ unsigned hash_slot(int key) {
  return (unsigned(key) * 2654435761u) & (kHashSlots - 1);
}

// Insert key into the LDS hash; counts new keys in *count.  Returns false
// when the table is full.
__device__ __forceinline__ bool hash_insert(int* table, int key, int* count) {
  unsigned h = hash_slot(key);
  for (int probe = 0; probe < kHashSlots; ++probe) {
    int old = atomicCAS(&table[h], -1, key);
    if (old == -1) {
      atomicAdd(count, 1);
      return true;
    }
    if (old == key) return true;
    h = (h + 1) & (kHashSlots - 1);
  }
  return false;
}

// Insert into a table of n slots (a power of two); false when full.
__device__ __forceinline__ bool hash_insert_n(int* table, int n, int key, int* count) {
  unsigned h = (unsigned(key) * 2654435761u) & (unsigned)(n - 1);
  for (int probe = 0; probe < n; ++probe) {
    int old = atomicCAS(&table[h], -1, key);
    if (old == -1) {
      atomicAdd(count, 1);
      return true;
    }
    if (old == key) return true;
    h = (h + 1) & (unsigned)(n - 1);
  }
  return false;
}

// As hash_insert_n; a new key also goes to list[count] (when below cap).
__device__ __forceinline__ bool hash_insert_list(int* table, int n, int key, int* count, int* list,
                                                 int cap) {
  unsigned h = (unsigned(key) * 2654435761u) & (unsigned)(n - 1);
  for (int probe = 0; probe < n; ++probe) {
    // most keys are repeats: a plain read settles them without an atomic
    int old = __hip_atomic_load(&table[h], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (old == -1) old = atomicCAS(&table[h], -1, key);
    if (old == -1) {
      const int o = atomicAdd(count, 1);
      if (o < cap) list[o] = key;
      return true;
    }
    if (old == key) return true;
    h = (h + 1) & (unsigned)(n - 1);
  }
  return false;
}

// As hash_insert_n, returning the slot of the key, or -1 when the table is full.
__device__ __forceinline__ int hash_insert_at_n(int* table, int n, int key, int* count) {
  unsigned h = (unsigned(key) * 2654435761u) & (unsigned)(n - 1);
  for (int probe = 0; probe < n; ++probe) {
    int old = atomicCAS(&table[h], -1, key);
    if (old == -1) {
      atomicAdd(count, 1);
      return (int)h;
    }
    if (old == key) return (int)h;
    h = (h + 1) & (unsigned)(n - 1);
  }
  return -1;
}

// As hash_insert, returning the slot of the key, or -1 when the table is full.
__device__ __forceinline__ int hash_insert_at(int* table, int key, int* count) {
  unsigned h = hash_slot(key);
  for (int probe = 0; probe < kHashSlots; ++probe) {
    int old = atomicCAS(&table[h], -1, key);
    if (old == -1) {
      atomicAdd(count, 1);
      return (int)h;
    }
    if (old == key) return (int)h;
    h = (h + 1) & (kHashSlots - 1);
  }
  return -1;
}

// Read the predecessor list of a block (inline part + overflow chain) into
// LDS and sort it.  Returns the count, or -1 on overflow.
__device__ __forceinline__ int load_preds(const FactorArgs& a, const int32_t* cnt_arr, const int32_t* list,
                          const int32_t* ovf_head, int K, int* s_pred, int* s_misc) {
  const int cnt = cnt_arr[K];
  if (cnt > kPredCap) return -1;
  const int inl = min(cnt, kListCap);
  for (int t = threadIdx.x; t < inl; t += blockDim.x) s_pred[t] = list[(int64_t)K * kListCap + t];
  if (threadIdx.x == 0) {
    int node = ovf_head[K];
    int at = kListCap;
    while (node >= 0 && at < cnt) {
      s_pred[at++] = a.ovf_j[node];
      node = a.ovf_next[node];
    }
    s_misc[0] = (cnt > kListCap && at != cnt) ? 1 : 0;
  }
  __syncthreads();
  if (s_misc[0]) return -1;
  __syncthreads();
  wg_bitonic_sort(s_pred, cnt);
  return cnt;
}

// Append block K to the predecessor list of block B.
__device__ __forceinline__ void push_pred_at(const FactorArgs& a, int32_t* list, int32_t* ovf_head, int B,
                                             int K, int pos) {
  if (pos < kListCap) {
    list[(int64_t)B * kListCap + pos] = K;
    return;
  }
  int node = atomicAdd(a.ovf_top, 1);
  if (node >= a.ovf_cap) {
    raise_error(a, kDevListOverflow, K);
    return;
  }
  a.ovf_j[node] = K;
  a.ovf_next[node] = atomicExch(&ovf_head[B], node);
}
__device__ __forceinline__ void push_pred(const FactorArgs& a, int32_t* cnt_arr, int32_t* list,
                                          int32_t* ovf_head, int B, int K) {
  push_pred_at(a, list, ovf_head, B, K, atomicAdd(&cnt_arr[B], 1));
}

__device__ __forceinline__ double dot_strided(const double* x, const double* y, int p) {
  double acc = 0.0;
  for (int t = 0; t < p; ++t) acc = fma(x[t], y[t], acc);
  return acc;
}

// One stored factor value (L or W) as a double: the heap holds them in the
// update precision.
__device__ __forceinline__ double load_factor(const FactorArgs& a, int64_t o) {
  return value_load(a.val_heap, a.update_prec, o);
}

// One Schur-update term L_J(i,:) W_J(:,j) of length p, from value-heap
// offsets lo (row of L_J) and wo (column of W_J): FP64, or FP32 / BF16
// inputs (the stored values) with FP32 accumulation.
__device__ __forceinline__ double update_term(const FactorArgs& a, int64_t lo, int64_t wo, int p) {
  if (a.update_prec == 1) {
    const float* v = static_cast<const float*>(a.val_heap);
    float acc = 0.0f;
    for (int t = 0; t < p; ++t) acc = fmaf(v[lo + t], v[wo + t], acc);
    return (double)acc;
  }
  if (a.update_prec == 2) {
    const uint16_t* v = static_cast<const uint16_t*>(a.val_heap);
    float acc = 0.0f;
    for (int t = 0; t < p; ++t) acc = fmaf(bf16_float(v[lo + t]), bf16_float(v[wo + t]), acc);
    return (double)acc;
  }
  const double* v = static_cast<const double*>(a.val_heap);
  return dot_strided(v + lo, v + wo, p);
}

// Store a factor value at value-heap offset o, rounded to the update
// precision (the drop test has already seen the FP64 value).
__device__ __forceinline__ void store_factor(const FactorArgs& a, int64_t o, double v) {
  value_store(a.val_heap, a.update_prec, o, v);
}

// Sec. 3.6 perturbation of column j of the q x q row-major matrix m: the
// largest-magnitude entry (lowest row on ties), or the diagonal when
// 2|m_jj| >= |m_kj|, becomes m_kj (1 + rho beta) + sign(m_kj) tau alpha.
__device__ __forceinline__ void perturb_column(double* m, int q, int j, const FactorArgs& a,
                                               double alpha) {
  int k = 0;
  double dmax = -1.0;
  for (int i = 0; i < q; ++i) {
    double v = fabs(m[i * q + j]);
    if (v > dmax) {
      dmax = v;
      k = i;
    }
  }
  if (2.0 * fabs(m[j * q + j]) >= fabs(m[k * q + j])) k = j;
  const double beta = a.beta_one ? 1.0 : dmax;
  const double d = m[k * q + j];
  m[k * q + j] = d * (1.0 + a.pert_rho * beta) + (d < 0.0 ? -1.0 : 1.0) * a.pert_tau * alpha;
}

__device__ __forceinline__ void perturb_row(double* m, int q, int i, const FactorArgs& a,
                                            double alpha) {
  int k = 0;
  double dmax = -1.0;
  for (int j = 0; j < q; ++j) {
    double v = fabs(m[i * q + j]);
    if (v > dmax) {
      dmax = v;
      k = j;
    }
  }
  if (2.0 * fabs(m[i * q + i]) >= fabs(m[i * q + k])) k = i;
  const double beta = a.beta_one ? 1.0 : dmax;
  const double d = m[i * q + k];
  m[i * q + k] = d * (1.0 + a.pert_rho * beta) + (d < 0.0 ? -1.0 : 1.0) * a.pert_tau * alpha;
}

// Sec. 5, the symmetrized perturbation: column j's entry is chosen as in
// perturb_column and the same new value is written at (k, j) and at its
// mirror (j, k).  Columns are taken one after the other (a mirror lands in
// another column).
__device__ __forceinline__ void perturb_symmetric(double* m, int q, int j, const FactorArgs& a,
                                                  double alpha) {
  int k = 0;
  double dmax = -1.0;
  for (int i = 0; i < q; ++i) {
    double v = fabs(m[i * q + j]);
    if (v > dmax) {
      dmax = v;
      k = i;
    }
  }
  if (2.0 * fabs(m[j * q + j]) >= fabs(m[k * q + j])) k = j;
  const double beta = a.beta_one ? 1.0 : dmax;
  const double d = m[k * q + j];
  const double nv = d * (1.0 + a.pert_rho * beta) + (d < 0.0 ? -1.0 : 1.0) * a.pert_tau * alpha;
  m[k * q + j] = nv;
  m[j * q + k] = nv;
}

// Thread group of a cooperative step: the whole workgroup, or wave 0 alone
// (wave-synchronous: LDS accesses of one wave complete in order, so a fence
// that stops compiler reordering is the only synchronisation needed).
template <bool kWave>
struct Group {
  __device__ static int id() { return kWave ? (int)(threadIdx.x & 63) : (int)threadIdx.x; }
  __device__ static int size() { return kWave ? 64 : (int)blockDim.x; }
  __device__ static void sync() {
    if (kWave) {
      __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
      __builtin_amdgcn_wave_barrier();
    } else {
      __syncthreads();
    }
  }
};

// In-place Gauss-Jordan inverse of the q x q row-major LDS matrix w with
// partial pivoting.  Returns false (uniformly) when a pivot is not above
// eps * smax.  kWave: run by wave 0 alone (no workgroup barriers).  s_f: q doubles, s_ip: q ints, s_misc: >= 4 ints.
template <bool kWave>
__device__ __forceinline__ bool gauss_jordan_inverse(double* w, int q, double smax, double eps, double* s_f,
                                     int* s_ip, int* s_misc) {
  using G = Group<kWave>;
  const int tid = G::id(), nth = G::size();
  for (int k = 0; k < q; ++k) {
    // pivot search by wave 0: max |w_ik|, i >= k, lowest i on ties
    if (tid < 64) {
      double bv = -1.0;
      int bi = q;
      for (int i = k + tid; i < q; i += 64) {
        double v = fabs(w[i * q + k]);
        if (v > bv || (v == bv && i < bi)) {
          bv = v;
          bi = i;
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        double ov = __shfl_xor(bv, o, 64);
        int oi = __shfl_xor(bi, o, 64);
        if (ov > bv || (ov == bv && oi < bi)) {
          bv = ov;
          bi = oi;
        }
      }
      if (tid == 0) {
        s_misc[0] = bi;
        double u = (bi < q) ? w[bi * q + k] : 0.0;
        s_misc[1] = (bi < q && u != 0.0 && fabs(u) > eps * smax && isfinite(u)) ? 1 : 0;
      }
    }
    G::sync();
    const int p = s_misc[0];
    if (!s_misc[1]) return false;
    if (p != k)
      for (int j = tid; j < q; j += nth) {
        double t = w[k * q + j];
        w[k * q + j] = w[p * q + j];
        w[p * q + j] = t;
      }
    if (tid == 0) s_ip[k] = p;
    G::sync();
    const double d = w[k * q + k];
    G::sync();
    for (int j = tid; j < q; j += nth) w[k * q + j] = (j == k ? 1.0 : w[k * q + j]) / d;
    for (int i = tid; i < q; i += nth) s_f[i] = w[i * q + k];
    G::sync();
    for (int e = tid; e < q * q; e += nth) {
      const int i = e / q, j = e - i * q;
      if (i == k) continue;
      const double base = (j == k) ? 0.0 : w[e];
      w[e] = fma(-s_f[i], w[k * q + j], base);
    }
    G::sync();
  }
  for (int k = q - 1; k >= 0; --k) {
    const int p = s_ip[k];
    if (p != k)
      for (int i = tid; i < q; i += nth) {
        double t = w[i * q + k];
        w[i * q + k] = w[i * q + p];
        w[i * q + p] = t;
      }
    G::sync();
  }
  return true;
}

// Fast path limits: blocks up to kFastWidth wide with at most kFastPreds
// predecessors, whose predecessor lists, candidates and panels fit in LDS.
constexpr int kFastWidth = 16;
constexpr int kFastPreds = 120;     // column + row predecessors
constexpr int kFastStage = 3072;    // staged list entries
constexpr int kFastBuf = 2048;      // doubles: panels + update terms
constexpr int kFastExtra = 256;     // candidate rows (columns) beyond the block
constexpr int kFastSegs = 2 + 2 * kFastPreds;
// LDS variant: candidates hash in s.hash[0, kFastCandSlots); K's own counts
// (blocks it may update) in a second table of kFastOwnSlots keys followed by
// their counts.
constexpr int kFastCandSlots = 2048;
constexpr int kFastOwnSlots = 512;
constexpr int kFastOwn = kFastCandSlots;                  // keys
constexpr int kFastOwnCnt = kFastCandSlots + kFastOwnSlots;  // counts
// The same path with its staged lists and panels in the worker's global
// slot, for blocks beyond the LDS capacities; the per-predecessor data stays
// in LDS (in the space the LDS variant uses for lists and panels).
constexpr int kBigPreds = 300;
// The global variant's own-count table (keys, then counts) at the end of
// the LDS variant's panel and metadata space, when the predecessor data
// leaves room for it; else that variant counts in a pass of its own after
// the factor writes.
constexpr int kGOwnSlots = 1024;
constexpr int kBigStage = 65536;
constexpr int kBigBuf = 65536;

// Per-predecessor data of the fast path.  lo/hi/lo2 are positions in J's
// lists: for a column predecessor, C_J[lo, hi) lie inside K and R_J[lo2, nr)
// are rows >= first(K); for a row predecessor, R_J[lo, hi) lie inside K and
// C_J[lo2, nc) are columns > last(K).  ioff: first update term of J.
struct PredMeta {
  long long roff, coff, loff, woff, troff, tcoff;
  int nr, nc, p, ntr, ntc, lo, hi, lo2, ioff, pad;
};
// bytes of the LDS variant's panel and metadata space (contiguous in Lds)
constexpr int kRegionBytes = sizeof(double) * kFastBuf + sizeof(PredMeta) * kFastPreds;

struct alignas(16) Lds {
  int hash[kHashSlots];     // candidate dedup; reused as keep flags; panels of
                            // the global variant while the terms accumulate
  int cand[kCandCap];       // sorted candidate rows
  int candc[kCandCap];      // sorted candidate columns
  union {
    struct {                // general path
      int pred[kPredCap];   // predecessors of the column panel
      int rpred[kPredCap];  // predecessors of the row panel
      int ann[kAnnCap];     // blocks this block may update
      int annc[kAnnCap];    // ... and the count it retracts from each
    } g;
    struct {                // fast path
      double buf[kFastBuf];           // panels, then update terms
      PredMeta meta[kFastPreds];      // column predecessors, then row ones
      int stage[kFastStage];          // staged lists (see factor_block_fast)
      int segoff[kFastSegs + 1];
      int useg[2 + kFastPreds + 1];   // offsets of the lists of K's own counts
      int pred[kFastPreds];
      int rpred[kFastPreds];
      long long cpk[kFastWidth + 1];  // A's column (row) pointers of K
      long long rpk[kFastWidth + 1];
    } x;
  };
  int misc[32];
  int scan[20];
  int ip[kMaxWidth];
  double f[kMaxWidth];
  double smax;
  double tau_k, alpha_k;    // drop tolerance and perturbation scale of the block
  long long off[2];
  long long hcur[2], hend[2];  // the worker's heap chunks (values, indices); kept across blocks
  // the worker's share of the launch counters, added once when it ends
  unsigned long long acc_flops, acc_bytes;
  unsigned long long acc_drop[3];  // rows dropped, columns dropped, smallest margin (bits)
  int acc_depth;
};
// updater_set counts per hash slot in cand[] followed by candc[]
static_assert(2 * kCandCap >= kHashSlots, "count slots");
static_assert(offsetof(Lds, candc) == offsetof(Lds, cand) + sizeof(int) * kCandCap, "layout");
static_assert(offsetof(Lds, x.buf) % 16 == 0 && 2 * 4 * (kThreads / 2) <= kHashSlots,
              "rank sort: 16-byte reads of the candidate lists");
static_assert(kFastWidth + kFastExtra <= 512 && 2560 + kFastExtra <= kFastStage, "stage layout");
static_assert(2 + 2 * kFastPreds <= kThreads && kFastPreds <= kThreads, "one thread per segment");
static_assert(2 * kFastExtra <= kFastBuf * 2, "candidate staging in buf");
static_assert(6 * kCandCap <= kBigStage && 2 * kCandCap <= 2 * kBigBuf, "global stage layout");
static_assert(sizeof(PredMeta) % 8 == 0, "PredMeta alignment");
// doubles of a worker slot used by the global variant of the fast path
constexpr int64_t kBigSlotDoubles = kBigBuf + kBigStage / 2 + 8;
static_assert(kBigPreds * sizeof(PredMeta) <= sizeof(double) * kFastBuf + sizeof(PredMeta) * kFastPreds,
              "global variant: predecessor data in LDS");
static_assert(2 * kBigPreds + 4 + 2 * kBigPreds + kBigPreds + 3 <= kFastStage,
              "global variant: list offsets and own-count offsets in LDS");
static_assert(kRegionBytes % 16 == 0 && 8 * kGOwnSlots < kRegionBytes, "global variant: own-count table");
static_assert(offsetof(Lds, x.meta) == offsetof(Lds, x.buf) + sizeof(double) * kFastBuf,
              "global variant: the predecessor data spans buf and meta");
static_assert(kThreads >= 192 && kListCap <= 64 && kFastWidth + 1 <= 32, "phase-1 thread map");
static_assert(kFastOwnCnt + kFastOwnSlots <= kHashSlots && 2 * kFastExtra <= kFastCandSlots / 2 &&
                  1024 + kFastExtra <= kFastCandSlots,
              "LDS variant hash layout");

// Build the sorted set of candidate indices into out[] from the structural
// entries of A (lists ptr/idx over [lo, hi], keeping idx >= min_keep) plus
// the stored rows (or columns) of the predecessors preds[0..npred).
// Returns the count or -1 on overflow.
__device__ __forceinline__ int build_candidates(Lds& s, int* out, const int64_t* ptr, const int32_t* idx, int lo,
                                int hi, int min_keep, const int* preds, int npred,
                                const FactorArgs& a, bool rows, int diag_first, int diag_last) {
  for (int t = threadIdx.x; t < kHashSlots; t += blockDim.x) s.hash[t] = -1;
  if (threadIdx.x == 0) {
    s.misc[4] = 0;  // unique count
    s.misc[5] = 0;  // overflow flag
  }
  __syncthreads();
  for (int i = diag_first + (int)threadIdx.x; i <= diag_last; i += blockDim.x)
    if (!hash_insert(s.hash, i, &s.misc[4])) s.misc[5] = 1;
  for (int c = lo; c <= hi; ++c) {
    const int64_t b = ptr[c], e = ptr[c + 1];
    for (int64_t m = b + threadIdx.x; m < e; m += blockDim.x) {
      int r = idx[m];
      if (r >= min_keep)
        if (!hash_insert(s.hash, r, &s.misc[4])) s.misc[5] = 1;
    }
  }
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int pi = wid; pi < npred; pi += nw) {
    const int J = preds[pi];
    const int cnt = rows ? a.nr[J] : a.nc[J];
    const int32_t* lst = a.idx_heap + (rows ? a.roff[J] : a.coff[J]);
    for (int t = lane; t < cnt; t += 64) {
      int r = lst[t];
      if (r >= min_keep)
        if (!hash_insert(s.hash, r, &s.misc[4])) s.misc[5] = 1;
    }
  }
  __syncthreads();
  const int m = s.misc[4];
  if (s.misc[5] || m > kCandCap) return -1;
  if (threadIdx.x == 0) s.misc[6] = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < kHashSlots; t += blockDim.x) {
    int k = s.hash[t];
    if (k >= 0) out[atomicAdd(&s.misc[6], 1)] = k;
  }
  __syncthreads();
  wg_bitonic_sort(out, m);
  return m;
}

__device__ __forceinline__ void trace_at(const FlowArgs& d, int K, int field,
                                         unsigned long long v) {
  if (d.trace) d.trace[(int64_t)K * kTraceFields + field] = v;
}

// Claim the next queue position for the calling worker: positions past the
// seeded ones ([0, L), L in misc[28]) are handed out in ascending order to
// workers that are running, so the lowest position still waiting for its
// block always belongs to a worker that will take it; no worker has to be
// resident for another to make progress.
__device__ __forceinline__ int claim_position(const FlowArgs& d, const Lds& s) {
  return s.misc[28] + atomicAdd(d.claim, 1);
}

// Push block B to the ready queue; who and why are traced.  Only the
// retraction that brings B's count to zero calls this, so a second push of B
// is a protocol error; the mark and the queue slot are taken together.
__device__ __forceinline__ void push_ready(const FactorArgs& a, const FlowArgs& d, int B, int by,
                                           int why) {
  const int again = atomicExch(&d.enq[B], 1);
  const int pos = atomicAdd(d.tail, 1);
  trace_at(d, B, 0, wall_clock64());
  trace_at(d, B, 5, (unsigned long long)by);
  trace_at(d, B, 6, (unsigned long long)why);
  if (again != 0 || pos >= a.nb) {
    raise_error(a, kDevProtocol, by);
    return;
  }
  __hip_atomic_store(&d.queue[pos], B, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The blocks K may update, each with the count K holds in its pending
// counter: 1 for every entry of A's block column and block row K that lies
// in a block B > K, plus 1 for every (column predecessor J, row block B > K
// of J) and (row predecessor J, column block B > K of J).  Keys go to s.g.ann, counts to s.g.annc; returns the
// number of keys or -1 on overflow.
__device__ __forceinline__ int updater_set(const FactorArgs& a, int K, Lds& s, int np, int npr) {
  int* cnt = s.cand;  // per hash slot, over cand[] and candc[] (built later)
  for (int t = threadIdx.x; t < kHashSlots; t += blockDim.x) {
    s.hash[t] = -1;
    cnt[t] = 0;
  }
  if (threadIdx.x == 0) {
    s.misc[4] = 0;
    s.misc[5] = 0;
  }
  __syncthreads();
  const int f = a.bstart[K], l = a.bstart[K + 1] - 1;
  for (int c = f; c <= l; ++c) {
    for (int64_t m = a.cp[c] + threadIdx.x; m < a.cp[c + 1]; m += blockDim.x) {
      const int B = a.bri[m];
      if (B > K) {
        const int h = hash_insert_at(s.hash, B, &s.misc[4]);
        if (h < 0) s.misc[5] = 1;
        else atomicAdd(&cnt[h], 1);
      }
    }
    for (int64_t m = a.rp[c] + threadIdx.x; m < a.rp[c + 1]; m += blockDim.x) {
      const int B = a.bci[m];
      if (B > K) {
        const int h = hash_insert_at(s.hash, B, &s.misc[4]);
        if (h < 0) s.misc[5] = 1;
        else atomicAdd(&cnt[h], 1);
      }
    }
  }
  const int wid = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  for (int pi = wid; pi < np + npr; pi += nw) {
    const bool col = pi < np;
    const int J = col ? s.g.pred[pi] : s.g.rpred[pi - np];
    const int n = col ? a.ntr[J] : a.ntc[J];
    const int32_t* lst = a.idx_heap + (col ? a.troff[J] : a.tcoff[J]);
    for (int t = lane; t < n; t += 64) {
      const int B = lst[t];
      if (B > K) {
        const int h = hash_insert_at(s.hash, B, &s.misc[4]);
        if (h < 0) s.misc[5] = 1;
        else atomicAdd(&cnt[h], 1);
      }
    }
  }
  __syncthreads();
  const int m = s.misc[4];
  if (s.misc[5] || m > kAnnCap) return -1;
  if (threadIdx.x == 0) s.misc[6] = 0;
  __syncthreads();
  for (int t = threadIdx.x; t < kHashSlots; t += blockDim.x) {
    const int k = s.hash[t];
    if (k >= 0) {
      const int o = atomicAdd(&s.misc[6], 1);
      s.g.ann[o] = k;
      s.g.annc[o] = cnt[t];
    }
  }
  __syncthreads();
  return m;
}

// Retract K's counts; the retraction that brings a count to zero makes that
// block ready.  Every write of K is visible before this is called.
__device__ __forceinline__ void retract(const FactorArgs& a, const FlowArgs& d, const Lds& s, int m, int K) {
  const int dK = __hip_atomic_load(&d.depth[K], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
  for (int t = threadIdx.x; t < m; t += blockDim.x) {
    const int B = s.g.ann[t], c = s.g.annc[t];
    atomicMax(&d.depth[B], dK);
    const int old = atomicSub(&d.pending[B], c);
    if (old < c) raise_error(a, kDevProtocol, K);
    if (old == c) push_ready(a, d, B, K, c);
  }
}

// Count, for every block B of K's stored rows (columns), the blocks J < B
// of K's stored columns (rows): each such J becomes a possible updater of
// B once K is done.  B's own count from K is still held, so B cannot have
// started.
__device__ __forceinline__ void add_successor_counts(const FactorArgs& a, const FlowArgs& d, const int32_t* tr,
                                     int ntr, const int32_t* tc, int ntc, int K) {
  for (int t = threadIdx.x; t < ntr + ntc; t += blockDim.x) {
    const bool row = t < ntr;
    const int B = row ? tr[t] : tc[t - ntr];
    const int c = row ? lower_bound(tc, ntc, B) : lower_bound(tr, ntr, B);
    if (c > 0 && atomicAdd(&d.pending[B], c) <= 0) raise_error(a, kDevProtocol, K);
  }
}

// Append block K to the predecessor list of block B (which must not have
// started its numeric phase yet).
__device__ __forceinline__ void push_checked(const FactorArgs& a, const FlowArgs& d,
                                             int32_t* cnt_arr, int32_t* list, int32_t* ovf_head,
                                             int B, int K) {
  if (__hip_atomic_load(&d.started[B], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
    raise_error(a, kDevProtocol, K);
  push_pred(a, cnt_arr, list, ovf_head, B, K);
}

// Pivot block (Sec. 3.6, Sec. 2.2): copy the q x q leading rows of the
// column panel into sS, perturb all-zero columns and rows, then invert into
// sW by Gauss-Jordan; a failed inversion perturbs every column and row of
// sS and retries (at most 3 rounds).  Returns false
// (uniformly) after reporting a block that stays singular.  kWave: run by
// wave 0 alone.
template <bool kWave>
__device__ __forceinline__ bool pivot_block(const FactorArgs& a, int K, int q, const double* Cp, double* sS,
                            double* sW, Lds& s, double alpha) {
  using G = Group<kWave>;
  const int tid = G::id(), nth = G::size();
  for (int e = tid; e < q * q; e += nth) sS[e] = Cp[e];
  if (tid == 0) s.misc[12] = 0;
  G::sync();
  // all-zero columns, then all-zero rows, are perturbed before factoring
  for (int j = tid; j < q; j += nth) {
    bool zero = true;
    for (int i = 0; i < q; ++i) zero = zero && sS[i * q + j] == 0.0;
    if (zero) {
      perturb_column(sS, q, j, a, alpha);
      s.misc[12] = 1;
    }
  }
  G::sync();
  for (int i = tid; i < q; i += nth) {
    bool zero = true;
    for (int j = 0; j < q; ++j) zero = zero && sS[i * q + j] == 0.0;
    if (zero) {
      perturb_row(sS, q, i, a, alpha);
      s.misc[12] = 1;
    }
  }
  G::sync();
  int rounds = s.misc[12];
  for (int attempt = 0;; ++attempt) {
    double mx = 0.0;
    int finite = 1;
    for (int e = tid; e < q * q; e += nth) {
      double v = sS[e];
      sW[e] = v;
      if (!isfinite(v)) finite = 0;
      mx = fmax(mx, fabs(v));
    }
    mx = wave_max(mx);
    finite = __all(finite);
    if (tid == 0) {
      s.misc[13] = 1;
      s.smax = 0.0;
    }
    G::sync();
    if ((tid & 63) == 0) {
      if (!finite) s.misc[13] = 0;
      // non-negative doubles order like their bit patterns
      atomicMax(reinterpret_cast<unsigned long long*>(&s.smax),
                (unsigned long long)__double_as_longlong(mx));
    }
    G::sync();
    const double smax = s.smax;
    bool ok = s.misc[13] && gauss_jordan_inverse<kWave>(sW, q, smax, a.pivot_eps, s.f, s.ip, s.misc);
    G::sync();
    if (ok) break;
    if (attempt == 3) {
      if (tid == 0) raise_error(a, kDevSingular, K);
      return false;
    }
    if (a.sym_pert) {
      if (tid == 0)
        for (int j = 0; j < q; ++j) perturb_symmetric(sS, q, j, a, alpha);
      G::sync();
    } else {
      for (int j = tid; j < q; j += nth) perturb_column(sS, q, j, a, alpha);
      G::sync();
      for (int i = tid; i < q; i += nth) perturb_row(sS, q, i, a, alpha);
      G::sync();
    }
    ++rounds;
  }
  if (tid == 0 && rounds > 0) {
    atomicAdd(a.n_perturbed, 1);
    if (a.pflag) a.pflag[K] = 1;
  }
  G::sync();
  return true;
}

// Pivot block of width q <= 8 in wave 0's registers (lane i q + j holds
// entry (i, j)), for the common case only: no all-zero row or column, every
// entry finite and every pivot above eps * smax.  Returns false (uniformly,
// nothing written) otherwise; the caller then runs pivot_block, which also
// perturbs.  The inverse takes the operations of gauss_jordan_inverse in the
// same order, so both give the same bits.
__device__ __forceinline__ bool pivot_regs(const FactorArgs& a, int q, const double* Cp, double* sS,
                                           double* sW) {
  const int lane = threadIdx.x & 63;
  const bool in = lane < q * q;
  const int i = in ? lane / q : 0, j = in ? lane - i * q : 0;
  const double c0 = in ? Cp[lane] : 0.0;
  double v = c0;
  const unsigned long long nz = __ballot(in && v != 0.0);
  for (int c = 0; c < q; ++c) {
    unsigned long long colm = 0, rowm = 0;
    for (int r = 0; r < q; ++r) {
      colm |= 1ull << (r * q + c);
      rowm |= 1ull << (c * q + r);
    }
    if ((nz & colm) == 0 || (nz & rowm) == 0) return false;
  }
  if (!__all(!in || isfinite(v))) return false;
  const double smax = wave_max(in ? fabs(v) : 0.0);
  unsigned piv = 0;  // 3 bits per step
  for (int k = 0; k < q; ++k) {
    // max |w_rk| over r >= k, lowest r on ties
    double bv = -1.0;
    int bi = q;
    for (int r = k; r < q; ++r) {
      const double x = fabs(__shfl(v, r * q + k, 64));
      if (x > bv) {
        bv = x;
        bi = r;
      }
    }
    if (bi >= q) return false;
    const double u = __shfl(v, bi * q + k, 64);
    if (!(u != 0.0 && fabs(u) > a.pivot_eps * smax && isfinite(u))) return false;
    piv |= (unsigned)bi << (3 * k);
    if (bi != k) v = __shfl(v, i == k ? bi * q + j : (i == bi ? k * q + j : lane), 64);
    const double dk = __shfl(v, k * q + k, 64);
    if (i == k) v = (j == k ? 1.0 : v) / dk;
    const double fi = __shfl(v, i * q + k, 64);
    const double wk = __shfl(v, k * q + j, 64);
    if (i != k) v = fma(-fi, wk, j == k ? 0.0 : v);
  }
  for (int k = q - 1; k >= 0; --k) {
    const int p = (int)((piv >> (3 * k)) & 7u);
    if (p != k) v = __shfl(v, j == k ? i * q + p : (j == p ? i * q + k : lane), 64);
  }
  if (in) {
    sW[lane] = v;
    sS[lane] = c0;
  }
  return true;
}

// D_K (sW) and the pivot block used (sS) into the factor storage; called in
// the write phase with the other factor stores.
__device__ __forceinline__ void store_pivot(const FactorArgs& a, int K, int q, const double* sS,
                                            const double* sW) {
  for (int e = threadIdx.x; e < q * q; e += blockDim.x) {
    a.dval[a.doff[K] + e] = sW[e];
    a.sval[a.doff[K] + e] = sS[e];
  }
}

// Drop test (Alg. 1 in block form): row z of L is kept iff the norm of
// C(z, K) D_K exceeds tau, column z of U iff the norm of D_K R(K, z) does.
// Drop decisions of block K (Alg. 1 in block form): keep_r[z] / keep_c[z]
// for the candidate rows cand[z] (z >= q) and columns candc[z].  The block's
// drops and the smallest relative margin |norm - tau| / tau go to the
// worker's LDS counters acc (rows dropped, columns dropped, margin bits);
// with a.log_margin > 0 the decisions within that margin of tau are logged.
__device__ __forceinline__ void drop_flags(const FactorArgs& a, const double* Cp, const double* Rp, int mc, int mcc,
                           int q, const double* sW, int* keep_r, int* keep_c, double tau, int K,
                           const int* cand, const int* candc, unsigned long long* acc) {
  const int tid = threadIdx.x;
  const bool two = a.drop_norm == 1;
  unsigned long long dr = 0, dc = 0;
  double mg = INFINITY;
  auto decide = [&](double nrm, int side, int idx) {
    if (tau > 0.0) {
      const double m = fabs(nrm - tau) / tau;
      mg = fmin(mg, m);
      if (m <= a.log_margin) {
        const int at = (int)atomicAdd(a.drop_ctr + 3, 1ull);
        if (at < a.log_cap) {
          a.log_blk[at] = K;
          a.log_idx[at] = side ? ~idx : idx;
          a.log_nrm[at] = nrm;
        }
      }
    }
    return nrm > tau;
  };
  for (int z = q + tid; z < mc; z += blockDim.x) {
    const double* row = Cp + (int64_t)z * q;
    double nrm = 0.0;
    for (int c = 0; c < q; ++c) {
      double v = 0.0;
      for (int t = 0; t < q; ++t) v = fma(row[t], sW[t * q + c], v);
      nrm = two ? fma(v, v, nrm) : fmax(nrm, fabs(v));
    }
    if (two) nrm = sqrt(nrm);
    const bool keep = decide(nrm, 0, cand[z]);
    keep_r[z] = keep ? 1 : 0;
    dr += keep ? 0 : 1;
  }
  for (int z = tid; z < mcc; z += blockDim.x) {
    const double* col = Rp + (int64_t)z * q;
    double nrm = 0.0;
    for (int r = 0; r < q; ++r) {
      double acc = 0.0;
      for (int t = 0; t < q; ++t) acc = fma(sW[r * q + t], col[t], acc);
      nrm = two ? fma(acc, acc, nrm) : fmax(nrm, fabs(acc));
    }
    if (two) nrm = sqrt(nrm);
    const bool keep = decide(nrm, 1, candc[z]);
    keep_c[z] = keep ? 1 : 0;
    dc += keep ? 0 : 1;
  }
  // per wave, then one LDS atomic each (non-negative doubles order like
  // their bit patterns)
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    dr += __shfl_xor(dr, o, 64);
    dc += __shfl_xor(dc, o, 64);
    mg = fmin(mg, __shfl_xor(mg, o, 64));
  }
  if ((tid & 63) == 0) {
    if (dr) atomicAdd(&acc[0], dr);
    if (dc) atomicAdd(&acc[1], dc);
    if (mg < INFINITY) atomicMin(&acc[2], (unsigned long long)__double_as_longlong(mg));
  }
  __syncthreads();
}

// Heap space for one block (run by one thread): nv values and ni indices from
// the worker's current chunks; a chunk that runs short is replaced by a new
// one of at least a.val_chunk (a.idx_chunk) entries from the shared top.
// Offsets go to s.off; false when the heap is exhausted.
__device__ __forceinline__ bool heap_take(const FactorArgs& a, Lds& s, long long nv, long long ni) {
  const bool nv_new = s.hcur[0] + nv > s.hend[0];
  const bool ni_new = s.hcur[1] + ni > s.hend[1];
  const long long tv = max(nv, (long long)a.val_chunk), ti = max(ni, (long long)a.idx_chunk);
  // both atomics in flight together
  const long long bv = nv_new ? (long long)atomicAdd(a.val_top, (unsigned long long)tv) : 0;
  const long long bi = ni_new ? (long long)atomicAdd(a.idx_top, (unsigned long long)ti) : 0;
  bool ok = true;
  if (nv_new) {
    s.hcur[0] = bv;
    s.hend[0] = min(bv + tv, (long long)a.val_cap);
    ok = ok && bv + nv <= a.val_cap;
  }
  if (ni_new) {
    s.hcur[1] = bi;
    s.hend[1] = min(bi + ti, (long long)a.idx_cap);
    ok = ok && bi + ni <= a.idx_cap;
  }
  s.off[0] = s.hcur[0];
  s.off[1] = s.hcur[1];
  s.hcur[0] += nv;
  s.hcur[1] += ni;
  return ok;
}

// Returns false (uniformly) when the block reported an error.
__device__ __forceinline__ bool factor_block(const FactorArgs& a, const FlowArgs& d, int K, int slot, Lds& s,
                             double* s_dyn) {
  const int tid = threadIdx.x;
  const int f = a.bstart[K], l = a.bstart[K + 1] - 1, q = l - f + 1;
  if (q > kMaxWidth) {
    if (tid == 0) raise_error(a, kDevWidth, K);
    return false;
  }
  double* Cp = a.scratch + (int64_t)slot * a.slot_doubles;   // kCandCap x q, row-major
  double* Rp = Cp + (int64_t)kCandCap * q;                     // q x kCandCap, column-major
  double flops = 0.0, ubytes = 0.0;

  // ---------------- predecessors, announcement, then candidates
  const int np = load_preds(a, a.col_cnt, a.col_list, a.col_ovf, K, s.g.pred, s.misc);
  if (np < 0) {
    if (tid == 0) raise_error(a, kDevPredOverflow, K);
    return false;
  }
  const int npr = load_preds(a, a.row_cnt, a.row_list, a.row_ovf, K, s.g.rpred, s.misc);
  if (npr < 0) {
    if (tid == 0) raise_error(a, kDevPredOverflow, K);
    return false;
  }
  if (tid == 0) {
    __hip_atomic_store(&d.started[K], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s.acc_depth = max(s.acc_depth,
                      __hip_atomic_load(&d.depth[K], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1);
  }
  const int na = updater_set(a, K, s, np, npr);
  if (na < 0) {
    if (tid == 0) raise_error(a, kDevAnnOverflow, K);
    return false;
  }
  if (tid == 0) trace_at(d, K, 2, wall_clock64());
  const int mc = build_candidates(s, s.cand, a.cp, a.ri, f, l, l + 1, s.g.pred, np, a, true, f, l);
  if (mc < 0) {
    if (tid == 0) raise_error(a, kDevCandOverflow, K);
    return false;
  }
  const int mcc = build_candidates(s, s.candc, a.rp, a.ci, f, l, l + 1, s.g.rpred, npr, a, false,
                                   1, 0);
  if (mcc < 0) {
    if (tid == 0) raise_error(a, kDevCandOverflow, K);
    return false;
  }
  if (tid == 0) {
    trace_at(d, K, 3, wall_clock64());
    trace_at(d, K, 16, (unsigned long long)np);
    trace_at(d, K, 17, (unsigned long long)npr);
    trace_at(d, K, 18, (unsigned long long)mc);
    trace_at(d, K, 19, (unsigned long long)mcc);
  }

  // ---------------- column panel: rows >= f of block column K
  for (int e = tid; e < mc * q; e += blockDim.x) Cp[e] = 0.0;
  __syncthreads();
  for (int c = f; c <= l; ++c) {
    for (int64_t m = a.cp[c] + tid; m < a.cp[c + 1]; m += blockDim.x) {
      int r = a.ri[m];
      if (r >= f) Cp[(int64_t)lower_bound(s.cand, mc, r) * q + (c - f)] = a.cv[m];
    }
  }
  __syncthreads();
  for (int pi = 0; pi < np; ++pi) {
    const int J = s.g.pred[pi];
    const int pJ = a.bstart[J + 1] - a.bstart[J];
    const int nRJ = a.nr[J], nCJ = a.nc[J];
    const int32_t* RJ = a.idx_heap + a.roff[J];
    const int32_t* CJ = a.idx_heap + a.coff[J];
    if (tid == 0) {
      s.misc[8] = 0;
      s.misc[9] = 0;
      s.misc[10] = 0;
    }
    __syncthreads();
    int c0 = 0, c1 = 0, r0 = 0;
    for (int t = tid; t < nCJ; t += blockDim.x) {
      int c = CJ[t];
      c0 += c < f;
      c1 += c <= l;
    }
    for (int t = tid; t < nRJ; t += blockDim.x) r0 += RJ[t] < f;
    c0 = wave_sum(c0);
    c1 = wave_sum(c1);
    r0 = wave_sum(r0);
    if ((tid & 63) == 0) {
      atomicAdd(&s.misc[8], c0);
      atomicAdd(&s.misc[9], c1);
      atomicAdd(&s.misc[10], r0);
    }
    __syncthreads();
    c0 = s.misc[8];
    c1 = s.misc[9];
    r0 = s.misc[10];
    const int ncol = c1 - c0, nrow = nRJ - r0;
    const int work = ncol * nrow;
    for (int w = tid; w < work; w += blockDim.x) {
      const int ri = r0 + w / ncol, cj = c0 + w % ncol;
      const int z = lower_bound(s.cand, mc, RJ[ri]);
      const double acc =
          update_term(a, a.loff[J] + (int64_t)ri * pJ, a.woff[J] + (int64_t)cj * pJ, pJ);
      Cp[(int64_t)z * q + (CJ[cj] - f)] -= acc;
    }
    flops += 2.0 * work * pJ;
    ubytes += (double)a.elem_bytes * pJ * (nrow + ncol);
    __syncthreads();
  }

  if (tid == 0) trace_at(d, K, 8, wall_clock64());
  // ---------------- row panel: columns > l of block row K
  for (int e = tid; e < mcc * q; e += blockDim.x) Rp[e] = 0.0;
  __syncthreads();
  for (int r = f; r <= l; ++r) {
    for (int64_t m = a.rp[r] + tid; m < a.rp[r + 1]; m += blockDim.x) {
      int c = a.ci[m];
      if (c > l) Rp[(int64_t)lower_bound(s.candc, mcc, c) * q + (r - f)] = a.rv[m];
    }
  }
  __syncthreads();
  for (int pi = 0; pi < npr; ++pi) {
    const int J = s.g.rpred[pi];
    const int pJ = a.bstart[J + 1] - a.bstart[J];
    const int nRJ = a.nr[J], nCJ = a.nc[J];
    const int32_t* RJ = a.idx_heap + a.roff[J];
    const int32_t* CJ = a.idx_heap + a.coff[J];
    if (tid == 0) {
      s.misc[8] = 0;
      s.misc[9] = 0;
      s.misc[10] = 0;
    }
    __syncthreads();
    int r0 = 0, r1 = 0, c0 = 0;
    for (int t = tid; t < nRJ; t += blockDim.x) {
      int r = RJ[t];
      r0 += r < f;
      r1 += r <= l;
    }
    for (int t = tid; t < nCJ; t += blockDim.x) c0 += CJ[t] <= l;
    r0 = wave_sum(r0);
    r1 = wave_sum(r1);
    c0 = wave_sum(c0);
    if ((tid & 63) == 0) {
      atomicAdd(&s.misc[8], r0);
      atomicAdd(&s.misc[9], r1);
      atomicAdd(&s.misc[10], c0);
    }
    __syncthreads();
    r0 = s.misc[8];
    r1 = s.misc[9];
    c0 = s.misc[10];
    const int nrow = r1 - r0, ncol = nCJ - c0;
    const int work = nrow * ncol;
    for (int w = tid; w < work; w += blockDim.x) {
      const int ri = r0 + w % nrow, cj = c0 + w / nrow;
      const int z = lower_bound(s.candc, mcc, CJ[cj]);
      const double acc =
          update_term(a, a.loff[J] + (int64_t)ri * pJ, a.woff[J] + (int64_t)cj * pJ, pJ);
      Rp[(int64_t)z * q + (RJ[ri] - f)] -= acc;
    }
    flops += 2.0 * work * pJ;
    ubytes += (double)a.elem_bytes * pJ * (nrow + ncol);
    __syncthreads();
  }

  if (tid == 0) trace_at(d, K, 9, wall_clock64());
  // ---------------- pivot block: perturb (Sec. 3.6) + invert
  // q x q perturbed pivot block and work/inverse: LDS up to width 64,
  // the slot's scratch beyond the panels for wider blocks
  double* big = Rp + (int64_t)kCandCap * q;
  const bool lds = a.lds_pivot && q <= kLdsPivotWidth;
  double* sS = lds ? s_dyn : big;
  double* sW = lds ? s_dyn + q * q : big + q * q;
  if (!pivot_block<false>(a, K, q, Cp, sS, sW, s, a.alpha_blk ? a.alpha_blk[K] : a.alpha)) return false;

  if (tid == 0) trace_at(d, K, 10, wall_clock64());
  // ---------------- drop: rows of L (scaled) and columns of U (D R)
  int* keep_r = s.hash;                 // flags for rows q..mc-1
  int* keep_c = s.hash + kCandCap;      // flags for cols 0..mcc-1
  drop_flags(a, Cp, Rp, mc, mcc, q, sW, keep_r, keep_c, a.tau_blk ? a.tau_blk[K] : a.tau, K, s.cand,
             s.candc, s.acc_drop);
  if (tid == 0) trace_at(d, K, 11, wall_clock64());
  constexpr int kPer = kCandCap / kThreads;  // flags per thread
  int fr[kPer], fc[kPer];
  int sr = 0, sc = 0;
  for (int k = 0; k < kPer; ++k) {
    const int z = tid * kPer + k;
    fr[k] = (z >= q && z < mc) ? keep_r[z] : 0;
    fc[k] = (z < mcc) ? keep_c[z] : 0;
    sr += fr[k];
    sc += fc[k];
  }
  int mk = 0, nk = 0;
  const int pr = wg_exclusive_scan(sr, s.scan, &mk);
  const int pc = wg_exclusive_scan(sc, s.scan, &nk);
  // distinct blocks of the kept rows (columns): a kept entry starts a new
  // block when the previous kept entry lies in another block
  int br = 0, bc = 0;
  for (int k = 0; k < kPer; ++k) {
    const int z = tid * kPer + k;
    if (fr[k]) {
      int y = z - 1;
      while (y >= q && !keep_r[y]) --y;
      br += y < q || a.blockOf[s.cand[y]] != a.blockOf[s.cand[z]];
    }
    if (fc[k]) {
      int y = z - 1;
      while (y >= 0 && !keep_c[y]) --y;
      bc += y < 0 || a.blockOf[s.candc[y]] != a.blockOf[s.candc[z]];
    }
  }
  int ntr = 0, ntc = 0;
  const int pbr = wg_exclusive_scan(br, s.scan, &ntr);
  const int pbc = wg_exclusive_scan(bc, s.scan, &ntc);
  if (tid == 0) {
    const bool over = !heap_take(a, s, (long long)(mk + nk) * q, (long long)(mk + nk + ntr + ntc));
    s.misc[16] = over ? 1 : 0;
    if (over) raise_error(a, kDevHeapOverflow, K);
  }
  __syncthreads();
  if (s.misc[16]) return false;
  if (tid == 0) trace_at(d, K, 12, wall_clock64());
  const int64_t vo = s.off[0];
  store_pivot(a, K, q, sS, sW);
  const int64_t io = s.off[1];
  int32_t* Rout = a.idx_heap + io;
  int32_t* Cout = Rout + mk;
  int32_t* TRout = Cout + nk;
  int32_t* TCout = TRout + ntr;
  {
    int posr = pbr, posc = pbc;
    for (int k = 0; k < kPer; ++k) {
      const int z = tid * kPer + k;
      if (fr[k]) {
        int y = z - 1;
        while (y >= q && !keep_r[y]) --y;
        const int B = a.blockOf[s.cand[z]];
        if (y < q || a.blockOf[s.cand[y]] != B) TRout[posr++] = B;
      }
      if (fc[k]) {
        int y = z - 1;
        while (y >= 0 && !keep_c[y]) --y;
        const int B = a.blockOf[s.candc[z]];
        if (y < 0 || a.blockOf[s.candc[y]] != B) TCout[posc++] = B;
      }
    }
  }
  {
    int pos = pr;
    for (int k = 0; k < kPer; ++k) {
      if (!fr[k]) continue;
      const int z = tid * kPer + k;
      const double* row = Cp + (int64_t)z * q;
      for (int c = 0; c < q; ++c) {
        double acc = 0.0;
        for (int t = 0; t < q; ++t) acc = fma(row[t], sW[t * q + c], acc);
        store_factor(a, vo + (int64_t)pos * q + c, acc);
      }
      Rout[pos] = s.cand[z];
      ++pos;
    }
    pos = pc;
    for (int k = 0; k < kPer; ++k) {
      if (!fc[k]) continue;
      const int z = tid * kPer + k;
      for (int r = 0; r < q; ++r)
        store_factor(a, vo + (int64_t)mk * q + (int64_t)pos * q + r, Rp[(int64_t)z * q + r]);
      Cout[pos] = s.candc[z];
      ++pos;
    }
  }
  if (tid == 0) {
    a.roff[K] = io;
    a.nr[K] = mk;
    a.coff[K] = io + mk;
    a.nc[K] = nk;
    a.loff[K] = vo;
    a.woff[K] = vo + (int64_t)mk * q;
    a.troff[K] = io + mk + nk;
    a.ntr[K] = ntr;
    a.tcoff[K] = io + mk + nk + ntr;
    a.ntc[K] = ntc;
    s.acc_flops += (unsigned long long)flops;
    s.acc_bytes += (unsigned long long)ubytes;
  }
  __syncthreads();
  if (tid == 0) trace_at(d, K, 13, wall_clock64());
  // K updates the row panels of the blocks holding its rows of L and the
  // column panels of the blocks holding its columns of U.
  for (int t = tid; t < mk; t += blockDim.x) {
    const int b = a.blockOf[Rout[t]];
    if (t == 0 || a.blockOf[Rout[t - 1]] != b)
      push_checked(a, d, a.row_cnt, a.row_list, a.row_ovf, b, K);
  }
  for (int t = tid; t < nk; t += blockDim.x) {
    const int b = a.blockOf[Cout[t]];
    if (t == 0 || a.blockOf[Cout[t - 1]] != b)
      push_checked(a, d, a.col_cnt, a.col_list, a.col_ovf, b, K);
  }
  __syncthreads();
  if (tid == 0) trace_at(d, K, 14, wall_clock64());
  add_successor_counts(a, d, TRout, ntr, TCout, ntc, K);
  // publish: every write and count of this block is visible before the
  // retraction
  wg_release_agent();
  if (tid == 0) trace_at(d, K, 15, wall_clock64());
  retract(a, d, s, na, K);
  if (tid == 0) trace_at(d, K, 4, wall_clock64());
  return true;
}

// ---------------------------------------------------------------------------
// Fast path for narrow blocks (q <= kFastWidth, at most kFastPreds
// predecessors, lists, candidates and panels within LDS).  Same arithmetic
// in the same order as factor_block, so both paths give identical bits; it
// differs in how data moves: a few batched rounds of global loads instead of
// one round per predecessor, panels in LDS, rank sorts, and the update terms
// L_J(i,:) W_J(:,j) computed for all predecessors at once, then subtracted
// in predecessor order.  Returns kFastFallback (before any global side
// effect other than the started flag) when the block does not fit.
// ---------------------------------------------------------------------------
enum FastResult : int { kFastDone = 0, kFastFallback = 1, kFastError = 2, kFastBig = 3 };

// Segments of the staged lists: 0 rows of A's block column K (CSC), 1 columns
// of A's block row K (CSR), then R_J and C_J of every column predecessor,
// then R_J and C_J of every row predecessor.
__device__ __forceinline__ const int32_t* fast_list(const FactorArgs& a, const Lds& s,
                                                    const PredMeta* meta, int sg, int np, int npr) {
  if (sg == 0) return a.ri + s.x.cpk[0];
  if (sg == 1) return a.ci + s.x.rpk[0];
  int t = sg - 2;
  if (t < np) return a.idx_heap + meta[t].roff;
  t -= np;
  if (t < np) return a.idx_heap + meta[t].coff;
  t -= np;
  if (t < npr) return a.idx_heap + meta[np + t].roff;
  t -= npr;
  return a.idx_heap + meta[np + t].coff;
}

// In-place exclusive prefix of v[0..m) for any m (all threads); returns the
// total.
__device__ __forceinline__ int wg_scan_array(int* v, int m, int* tmp) {
  int carry = 0;
  for (int base = 0; base < m; base += blockDim.x) {
    const int i = base + threadIdx.x;
    const int x = i < m ? v[i] : 0;
    int tot = 0;
    const int ex = wg_exclusive_scan(x, tmp, &tot);
    if (i < m) v[i] = carry + ex;
    carry += tot;
  }
  __syncthreads();
  return carry;
}

// Exclusive prefix of v[0..m), m <= 64, by one wave; the total goes to *tot.
__device__ __forceinline__ void wave_scan_array(int* v, int m, int* tot) {
  const int lane = threadIdx.x & 63;
  const int x = lane < m ? v[lane] : 0;
  int incl = x;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int t = __shfl_up(incl, o, 64);
    if (lane >= o) incl += t;
  }
  if (lane < m) v[lane] = incl - x;
  if (lane == 63) *tot = incl;
}

// Last s in [0, n) with off[s] <= e (off ascending, off[n] > e).
__device__ __forceinline__ int last_le(const int* off, int n, int e) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (off[mid] <= e)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Entry e of A's columns (e < nA0) or rows of block K in the staged lists:
// where its value is and its position in the panels (-1: outside them).
struct AEntry {
  const double* src;
  int tgt;
};
__device__ __forceinline__ AEntry a_entry(const FactorArgs& a, const Lds& s, const int* stage, int e,
                                          int nA0, int f, int l, int q, int mc, int mcc) {
  if (e < nA0) {
    const int r = stage[e];
    const long long m = s.x.cpk[0] + e;
    int tgt = -1;
    if (r >= f) {
      int c = 0;
      while (s.x.cpk[c + 1] <= m) ++c;
      tgt = lower_bound(s.cand, mc, r) * q + c;
    }
    return {a.cv + m, tgt};
  }
  const int c = stage[e];
  const long long m = s.x.rpk[0] + (e - nA0);
  int tgt = -1;
  if (c > l) {
    int r = 0;
    while (s.x.rpk[r + 1] <= m) ++r;
    tgt = mc * q + lower_bound(s.candc, mcc, c) * q + r;
  }
  return {a.rv + m, tgt};
}

// ---------------------------------------------------------------------------
// Schur-update terms on the matrix cores.  The terms of one predecessor J
// form a dense product T = L_J(rows, :) W_J(:, cols) of size M x N with
// contraction p_J (Sec. 2.2, Fig. 2): for a column predecessor the rows of
// R_J at or below first(K) times the columns of C_J inside K; for a row
// predecessor the rows of R_J inside K times the columns of C_J beyond K.
// A wave computes one 16 x 16 tile of T with v_mfma 16x16 instructions,
// each lane loading its operand fragments straight from the factor heap
// (one value of L and one of W per lane and k-step, instead of a whole row
// and column per term), and writes each term with its panel position to
// Tm / Ti exactly as the scalar loop does, so the ordered accumulation that
// follows is unchanged.  FP64 inputs use the FP64 instruction (16x16x4),
// FP32 inputs 16x16x4 with FP32 accumulation, BF16 inputs 16x16x16 with
// FP32 accumulation.  Lane layout (checked on the device): operand lane l
// holds row (column) l % 16 of k-group l / 16; the result element i of lane
// l is row 4 (l / 16) + i (FP64: l / 16 + 4 i) of column l % 16.
// kG: the staged lists and panels live in the worker's global slot.
// ---------------------------------------------------------------------------
// 16-byte loads of stored factor values at their natural alignment (the
// hardware accepts loads aligned to their element size)
typedef double wide_f64 __attribute__((ext_vector_type(2), aligned(8)));
typedef float wide_f32 __attribute__((ext_vector_type(4), aligned(4)));
typedef uint16_t wide_bf16 __attribute__((ext_vector_type(8), aligned(2)));
// Slack in values after the end of the value heap: the last 16-byte load of
// a row may reach past the last stored value.
constexpr int64_t kHeapSlack = 16;
// Records of near-tie drop decisions kept at most (drop_log_margin > 0).
constexpr int kDropLogCap = 1 << 20;

typedef double mfma_d4 __attribute__((ext_vector_type(4)));
typedef float mfma_f4 __attribute__((ext_vector_type(4)));
typedef short mfma_s4 __attribute__((ext_vector_type(4)));

template <int kPrec>
struct TileAcc;
template <>
struct TileAcc<0> {
  using T = mfma_d4;
};
template <>
struct TileAcc<1> {
  using T = mfma_f4;
};
template <>
struct TileAcc<2> {
  using T = mfma_f4;
};

// Operand fragment of one lane for k-step k0: FP64 / FP32 one value, BF16
// four (k = k0 + 4 kg + j); off = -1 or k >= p pads with zero.
template <int kPrec>
struct Frag;
template <>
struct Frag<0> {
  using T = double;
  static constexpr int kStep = 4;
  __device__ static T load(const void* v, int64_t off, int k0, int kg, int p) {
    const int k = k0 + kg;
    return (off >= 0 && k < p) ? static_cast<const double*>(v)[off + k] : 0.0;
  }
};
template <>
struct Frag<1> {
  using T = float;
  static constexpr int kStep = 4;
  __device__ static T load(const void* v, int64_t off, int k0, int kg, int p) {
    const int k = k0 + kg;
    return (off >= 0 && k < p) ? static_cast<const float*>(v)[off + k] : 0.0f;
  }
};
template <>
struct Frag<2> {
  using T = mfma_s4;
  static constexpr int kStep = 16;
  __device__ static T load(const void* v, int64_t off, int k0, int kg, int p) {
    T x;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = k0 + 4 * kg + j;
      x[j] = (short)((off >= 0 && k < p) ? static_cast<const uint16_t*>(v)[off + k] : 0);
    }
    return x;
  }
};
template <int kPrec>
__device__ __forceinline__ typename TileAcc<kPrec>::T mfma_step(typename Frag<kPrec>::T x,
                                                                typename Frag<kPrec>::T y,
                                                                typename TileAcc<kPrec>::T c) {
  if constexpr (kPrec == 0)
    return __builtin_amdgcn_mfma_f64_16x16x4f64(x, y, c, 0, 0, 0);
  else if constexpr (kPrec == 1)
    return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(x, y, c, 0, 0, 0);
}

// Geometry of one tile: its predecessor, the tile's rows a0.. and columns
// b0.. of the product, and this lane's operand offsets.
struct TileGeo {
  int t, M, N, a0, b0;
  int64_t la, wb;
  int p;
  bool live;
};

// Values of the terms e in [i0, i1) of all predecessors into Tm (their
// panel positions are already in Ti).  Each wave takes kTiles tiles at a
// time: their operand fragments for one k-step are loaded together, then
// their matrix-core steps issued, so the loads of several tiles are in
// flight at once.  fmeta[t].pad holds the first tile of predecessor t,
// ntiles their total.
template <int kPrec>
__device__ __forceinline__ void mfma_terms(const FactorArgs& a, const PredMeta* fmeta, int npt,
                                           int np, int i0, int i1, double* Tm, int ntiles) {
  constexpr int kTiles = 4;
  const int lane = threadIdx.x & 63, kg = lane >> 4;
  const int nw = blockDim.x >> 6;
  for (int base = (int)(threadIdx.x >> 6); base < ntiles; base += nw * kTiles) {
    TileGeo g[kTiles];
    int pmax = 0;
#pragma unroll
    for (int u = 0; u < kTiles; ++u) {
      const int task = base + u * nw;
      g[u].live = false;
      g[u].la = g[u].wb = -1;
      g[u].p = 0;
      g[u].t = g[u].M = g[u].N = g[u].a0 = g[u].b0 = 0;
      if (task >= ntiles) continue;
      int lo_t = 0, hi_t = npt;  // the predecessor: last t with first tile <= task
      while (hi_t - lo_t > 1) {
        const int mid = (lo_t + hi_t) >> 1;
        if (fmeta[mid].pad <= task)
          lo_t = mid;
        else
          hi_t = mid;
      }
      const int t = lo_t;
      const PredMeta& m = fmeta[t];
      const bool colp = t < np;
      const int M = colp ? m.nr - m.lo2 : m.hi - m.lo;
      const int N = colp ? m.hi - m.lo : m.nc - m.lo2;
      const int tn = (N + 15) >> 4;
      const int a0 = (task - m.pad) / tn * 16, b0 = (task - m.pad) % tn * 16;
      const int a1 = min(M, a0 + 16), b1 = min(N, b0 + 16);
      // the tile's first and last term (column predecessors number their
      // terms row by row, row predecessors column by column)
      const int emin = colp ? m.ioff + a0 * N + b0 : m.ioff + b0 * M + a0;
      const int emax = colp ? m.ioff + (a1 - 1) * N + (b1 - 1) : m.ioff + (b1 - 1) * M + (a1 - 1);
      if (emax < i0 || emin >= i1) continue;
      const int ra = a0 + (lane & 15), cb = b0 + (lane & 15);
      g[u] = TileGeo{t, M, N, a0, b0,
                     ra < M ? m.loff + (int64_t)((colp ? m.lo2 : m.lo) + ra) * m.p : -1,
                     cb < N ? m.woff + (int64_t)((colp ? m.lo : m.lo2) + cb) * m.p : -1, m.p,
                     true};
      pmax = max(pmax, m.p);
    }
    typename TileAcc<kPrec>::T acc[kTiles];
#pragma unroll
    for (int u = 0; u < kTiles; ++u) acc[u] = typename TileAcc<kPrec>::T{0, 0, 0, 0};
    for (int k0 = 0; k0 < pmax; k0 += Frag<kPrec>::kStep) {
      typename Frag<kPrec>::T x[kTiles], y[kTiles];
#pragma unroll
      for (int u = 0; u < kTiles; ++u) {
        x[u] = Frag<kPrec>::load(a.val_heap, g[u].la, k0, kg, g[u].p);
        y[u] = Frag<kPrec>::load(a.val_heap, g[u].wb, k0, kg, g[u].p);
      }
#pragma unroll
      for (int u = 0; u < kTiles; ++u)
        if (g[u].live && k0 < g[u].p) acc[u] = mfma_step<kPrec>(x[u], y[u], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < kTiles; ++u) {
      if (!g[u].live) continue;
      const bool colp = g[u].t < np;
      const PredMeta& m = fmeta[g[u].t];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int ar = kPrec == 0 ? g[u].a0 + kg + 4 * i : g[u].a0 + 4 * kg + i;
        const int bc = g[u].b0 + (lane & 15);
        if (ar >= g[u].M || bc >= g[u].N) continue;
        const int e = colp ? m.ioff + ar * g[u].N + bc : m.ioff + bc * g[u].M + ar;
        if (e >= i0 && e < i1) Tm[e - i0] = (double)acc[u][i];
      }
    }
  }
}

// Rank sort of distinct keys: dst[#{u : src[u] < src[i]}] = src[i] for
// every i < m.  The calling thread takes keys lt, lt + ln, ... (at most
// kRankKeys of them, so m <= kRankKeys * ln) and counts against all of src
// in one pass, reading four keys per 16-byte LDS load (src 16-byte aligned).
constexpr int kRankKeys = 4;
__device__ __forceinline__ void rank_place(const int* src, int m, int* dst, int lt, int ln) {
  int v[kRankKeys], r[kRankKeys];
#pragma unroll
  for (int e = 0; e < kRankKeys; ++e) {
    const int i = lt + e * ln;
    v[e] = i < m ? src[i] : INT32_MIN;  // INT32_MIN: counts nothing
    r[e] = 0;
  }
  const int m4 = m & ~3;
  for (int u = 0; u < m4; u += 4) {
    const int4 w = *reinterpret_cast<const int4*>(src + u);
#pragma unroll
    for (int e = 0; e < kRankKeys; ++e)
      r[e] += (w.x < v[e]) + (w.y < v[e]) + (w.z < v[e]) + (w.w < v[e]);
  }
  for (int u = m4; u < m; ++u) {
    const int w = src[u];
#pragma unroll
    for (int e = 0; e < kRankKeys; ++e) r[e] += w < v[e];
  }
#pragma unroll
  for (int e = 0; e < kRankKeys; ++e) {
    const int i = lt + e * ln;
    if (i < m) dst[r[e]] = v[e];
  }
}

template <bool kG>
__device__ __forceinline__ int factor_block_fast(const FactorArgs& a, const FlowArgs& d, int K,
                                                 Lds& s, double* s_dyn, double* gslot, int next_pos) {
  const int tid = threadIdx.x, nt = blockDim.x;
  // entries per thread and pass of the staging loop: a pass covers a
  // typical LDS-variant block and the unrolled body stays small for the
  // instruction cache; the global variant stages far longer lists
  constexpr int kBatch = kG ? 12 : 4;
  // storage: LDS, or (kG) the worker's global slot for blocks beyond the LDS
  // capacities; per-candidate arrays sit at multiples of cSpace in stage
  constexpr int cStage = kG ? kBigStage : kFastStage;
  constexpr int cPreds = kG ? kBigPreds : kFastPreds;
  constexpr int cBuf = kG ? kBigBuf : kFastBuf;
  constexpr int cExtra = kG ? kCandCap - kFastWidth : kFastExtra;
  constexpr int cSpace = kG ? kCandCap : 512;
  const int fallback = kG ? kFastFallback : kFastBig;
  double* fbuf;
  PredMeta* fmeta;
  int *stage, *fseg, *fpred, *frpred;
  if (kG) {
    // global: panels and staged lists; LDS: predecessor data over the LDS
    // variant's panel, metadata and stage space
    fbuf = gslot;
    stage = reinterpret_cast<int*>(gslot + kBigBuf);
    fmeta = reinterpret_cast<PredMeta*>(s.x.buf);
    fseg = s.x.stage;
    fpred = fseg + 2 * kBigPreds + 4;
    frpred = fpred + kBigPreds;
  } else {
    fbuf = s.x.buf;
    fmeta = s.x.meta;
    stage = s.x.stage;
    fseg = s.x.segoff;
    fpred = s.x.pred;
    frpred = s.x.rpred;
  }
  // ---- phase 1: predecessor counts and inline lists, block range.  The
  // global variant resumes from the LDS variant's rounds 1 and 2 when that
  // variant gave the block up after them (misc[31]): the counts, range,
  // sorted predecessors, their data and A's pointers of K are in LDS.
  const bool resume = kG && s.misc[31] != 0;
  int* rawc = stage;
  int* rawr = stage + cPreds;
  if (resume) {
  } else if (tid < kListCap) {
    rawc[tid] = a.col_list[(int64_t)K * kListCap + tid];
  } else if (tid >= 64 && tid < 64 + kListCap) {
    rawr[tid - 64] = a.row_list[(int64_t)K * kListCap + tid - 64];
  } else if (tid == 128) {
    s.misc[0] = a.col_cnt[K];
  } else if (tid == 129) {
    s.misc[1] = a.row_cnt[K];
  } else if (tid == 130) {
    s.misc[2] = a.bstart[K];
  } else if (tid == 131) {
    s.misc[3] = a.bstart[K + 1];
  } else if (tid == 132) {
    __hip_atomic_store(&d.started[K], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // every updater's depth is in: K became ready after their retractions
    const int dep = __hip_atomic_load(&d.depth[K], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s.misc[24] = dep;
    s.acc_depth = max(s.acc_depth, dep + 1);
  } else if (tid == 133) {
    s.tau_k = a.tau_blk ? a.tau_blk[K] : a.tau;
  } else if (tid == 134) {
    s.alpha_k = a.alpha_blk ? a.alpha_blk[K] : a.alpha;
  }
  if (tid == 0) s.misc[8] = 0;
  __syncthreads();
  const int np = s.misc[0], npr = s.misc[1];
  const int f = s.misc[2], l = s.misc[3] - 1, q = l - f + 1;
  if (q > kFastWidth || !a.lds_pivot) return kFastFallback;
  if (np + npr > cPreds) return fallback;
  // K's own counts come with the staging pass (phase 3) in the LDS variant
  // and, when its predecessor data leaves room for the table, in the global
  // variant (gown, over the end of the LDS variant's panel and metadata)
  const bool ownearly =
      !kG || (np + npr) * (int)sizeof(PredMeta) <= kRegionBytes - 8 * kGOwnSlots;
  int* const gown = reinterpret_cast<int*>(reinterpret_cast<char*>(s.x.buf) + kRegionBytes) -
                    2 * kGOwnSlots;
  int* const fuseg = kG ? fpred + 2 * kBigPreds : s.x.useg;  // offsets of the own-count lists
  if (resume) {
    for (int t = tid; t < np; t += nt) fpred[t] = s.x.pred[t];
    for (int t = tid; t < npr; t += nt) frpred[t] = s.x.rpred[t];
  } else if (np > kListCap || npr > kListCap) {
    // overflow chains: one serial walk per list
    if ((tid == 0 && np > kListCap) || (tid == 64 && npr > kListCap)) {
      const bool col = tid == 0;
      const int cnt = col ? np : npr;
      int* raw = col ? rawc : rawr;
      int node = col ? a.col_ovf[K] : a.row_ovf[K];
      int at = kListCap;
      while (node >= 0 && at < cnt) {
        raw[at++] = a.ovf_j[node];
        node = a.ovf_next[node];
      }
      if (at != cnt) s.misc[8] = 1;
    }
    __syncthreads();
    if (s.misc[8]) return kFastFallback;  // the general path reports it
  }
  // ascending predecessor order (entries are distinct): rank sort
  for (int t = resume ? np + npr : tid; t < np + npr; t += nt) {
    const bool col = t < np;
    const int* raw = col ? rawc : rawr;
    const int m = col ? np : npr, i = col ? t : t - np;
    const int v = raw[i];
    int r = 0;
    for (int u = 0; u < m; ++u) r += raw[u] < v;
    (col ? fpred : frpred)[r] = v;
  }
  __syncthreads();

  // ---- phase 2: predecessor data, A's pointers of K; clear the hash
  if (resume)  // the LDS variant's data (s.x.meta lies above the first
               // cPreds entries of the global variant's fmeta, s.x.buf)
    for (int t = tid; t < np + npr; t += nt) fmeta[t] = s.x.meta[t];
  for (int t = resume ? np + npr : tid; t < np + npr; t += nt) {
    const int J = t < np ? fpred[t] : frpred[t - np];
    PredMeta& m = fmeta[t];
    m.roff = a.roff[J];
    m.coff = a.coff[J];
    m.loff = a.loff[J];
    m.woff = a.woff[J];
    m.troff = a.troff[J];
    m.tcoff = a.tcoff[J];
    m.nr = a.nr[J];
    m.nc = a.nc[J];
    m.ntr = a.ntr[J];
    m.ntc = a.ntc[J];
    m.p = a.bstart[J + 1] - a.bstart[J];
  }
  if (!resume && tid >= 128 && tid <= 128 + q) s.x.cpk[tid - 128] = a.cp[f + tid - 128];
  if (!resume && tid >= 160 && tid <= 160 + q) s.x.rpk[tid - 160] = a.rp[f + tid - 160];
  for (int t = tid; t < kHashSlots; t += nt) s.hash[t] = (!kG && t >= kFastOwnCnt) ? 0 : -1;
  if (tid == 0) {
    s.misc[4] = 0;
    s.misc[5] = 0;
    s.misc[6] = 0;
    s.misc[7] = 0;
    s.misc[9] = 0;
    s.misc[10] = 0;
    s.misc[31] = kG ? 0 : 1;  // rounds 1 and 2 done (read after the barrier)
  }
  __syncthreads();
  if (tid == 0) trace_at(d, K, 2, wall_clock64());
  const int nseg = 2 + 2 * (np + npr);
  {
    for (int g = tid; g < nseg; g += nt) {
      int len;
      if (g == 0) {
        len = (int)(s.x.cpk[q] - s.x.cpk[0]);
      } else if (g == 1) {
        len = (int)(s.x.rpk[q] - s.x.rpk[0]);
      } else {
        int t = g - 2;
        if (t < np) {
          len = fmeta[t].nr;
        } else if ((t -= np) < np) {
          len = fmeta[t].nc;
        } else if ((t -= np) < npr) {
          len = fmeta[np + t].nr;
        } else {
          t -= npr;
          len = fmeta[np + t].nc;
        }
      }
      fseg[g] = len;
    }
    if (ownearly)
      for (int g = tid; g < 2 + np + npr; g += nt)
        fuseg[g] = g == 0   ? (int)(s.x.cpk[q] - s.x.cpk[0])
                   : g == 1 ? (int)(s.x.rpk[q] - s.x.rpk[0])
                   : g - 2 < np ? fmeta[g - 2].ntr
                                : fmeta[g - 2].ntc;
    if (kG && ownearly)  // after the barrier that ends the resumed copy of s.x.meta
      for (int t = tid; t < 2 * kGOwnSlots; t += nt) gown[t] = t < kGOwnSlots ? -1 : 0;
    __syncthreads();
    const int nu = 2 + np + npr;
    if (nseg <= 64 && nu <= 64) {
      // both offset arrays at once, by waves 0 and 1
      if (tid < 64)
        wave_scan_array(fseg, nseg, &fseg[nseg]);
      else if (ownearly && tid < 128)
        wave_scan_array(fuseg, nu, &fuseg[nu]);
      __syncthreads();
      if (fseg[nseg] > cStage) return fallback;
    } else {
      const int total = wg_scan_array(fseg, nseg, s.scan);
      if (tid == 0) fseg[nseg] = total;
      if (ownearly) {
        const int tot = wg_scan_array(fuseg, nu, s.scan);
        if (tid == 0) fuseg[nu] = tot;
      }
      if (total > cStage) return fallback;
      __syncthreads();
    }
  }
  const int* segoff = fseg;
  const int total = segoff[nseg];
  if (tid == 0) trace_at(d, K, 20, wall_clock64());

  // ---- phase 3: stage every list; candidate rows (keys r) and columns
  // (keys ~c) beyond the block go to one hash, and each new key to keys[]
  int* keys = reinterpret_cast<int*>(fbuf) + 2 * cExtra;
  // K's own counts come with the same pass (LDS variant): A's entries of K
  // in later blocks, TR_J > K of column predecessors, TC_J > K of row
  // predecessors; entries [total, total + totu) of the combined index range
  const int nu = 2 + np + npr, totu = ownearly ? fuseg[nu] : 0;
  const int tall = total + totu;
  // the column lists of column predecessors and the row lists of row
  // predecessors (one contiguous range of segments) are only searched for
  // the block's own range: the global variant reads them from the heap and
  // does not stage them; the LDS variant stages them (searches in LDS are
  // cheaper than in the heap)
  const int gA = segoff[2 + np], gap = kG ? segoff[2 + 2 * np + npr] - gA : 0;
  const int tv = tall - gap;
  for (int base = 0; base < tv; base += kBatch * nt) {
    int v[kBatch], sgk[kBatch];
    // each entry's segment (in segoff, or in useg for K's own counts), kept
    // for the insertion pass
#pragma unroll
    for (int k = 0; k < kBatch; ++k) {
      const int ev = base + tid + k * nt;
      const int e = ev < gA ? ev : ev + gap;
      sgk[k] = e < total ? last_le(segoff, nseg, e) : last_le(fuseg, nu, e - total);
    }
    for (int k = 0; k < kBatch; ++k) {
      const int ev = base + tid + k * nt;
      const int e = ev < gA ? ev : ev + gap;
      if (ev >= tv) {
      } else if (e < total) {
        const int sg = sgk[k];
        v[k] = fast_list(a, s, fmeta, sg, np, npr)[e - segoff[sg]];
      } else if (e < tall) {
        const int sg = sgk[k];
        const int i = e - total - fuseg[sg];
        if (sg == 0)
          v[k] = a.bri[s.x.cpk[0] + i];
        else if (sg == 1)
          v[k] = a.bci[s.x.rpk[0] + i];
        else if (sg - 2 < np)
          v[k] = a.idx_heap[fmeta[sg - 2].troff + i];
        else
          v[k] = a.idx_heap[fmeta[sg - 2].tcoff + i];
      }
    }
    for (int k = 0; k < kBatch; ++k) {
      const int ev = base + tid + k * nt;
      if (ev >= tv) break;
      const int e = ev < gA ? ev : ev + gap;
      if (e < total) {
        stage[e] = v[k];
        const int sg = sgk[k];
        const bool rowc = sg == 0 || (sg >= 2 && sg < 2 + np);
        const bool colc = sg == 1 || sg >= 2 + 2 * np + npr;
        if ((rowc || colc) && v[k] > l)
          if (!hash_insert_list(s.hash, kG ? kHashSlots : kFastCandSlots, rowc ? v[k] : ~v[k],
                                &s.misc[4], keys, 2 * cExtra))
            s.misc[5] = 1;
      } else if (v[k] > K) {  // e < tall: only when ownearly
        int* const tab = kG ? gown : s.hash + kFastOwn;
        const int h = hash_insert_at_n(tab, kG ? kGOwnSlots : kFastOwnSlots, v[k], &s.misc[9]);
        if (h < 0)
          s.misc[10] = 1;
        else
          atomicAdd(&tab[(kG ? kGOwnSlots : kFastOwnSlots) + h], 1);
      }
    }
  }
  __syncthreads();
  if (tid == 0) trace_at(d, K, 21, wall_clock64());
  if (!kG && s.misc[10]) return kFastBig;
  // the global variant's early table overflowed: it counts after the writes
  const bool ownlate = kG && (!ownearly || s.misc[10] != 0);
  if (s.misc[5] || s.misc[4] > 2 * cExtra) return fallback;
  // positions inside the predecessors' sorted lists (the three searches of
  // a predecessor step together, so their loads overlap)
  for (int t = tid; t < np + npr; t += nt) {
    PredMeta& m = fmeta[t];
    const int* A;
    const int* B;
    int na, nb_, ka, kb;
    if (t < np) {
      A = kG ? a.idx_heap + m.coff : stage + segoff[2 + np + t];  // C: lo, hi
      B = stage + segoff[2 + t];       // R: lo2
      na = m.nc;
      nb_ = m.nr;
      ka = f;
      kb = f;
    } else {
      const int u = t - np;
      A = kG ? a.idx_heap + m.roff : stage + segoff[2 + 2 * np + u];  // R: lo, hi
      B = stage + segoff[2 + 2 * np + npr + u];  // C: lo2
      na = m.nr;
      nb_ = m.nc;
      ka = f;
      kb = l + 1;
    }
    int lo0 = 0, hi0 = na, lo1 = 0, hi1 = na, lo2 = 0, hi2 = nb_;
    while (lo0 < hi0 || lo1 < hi1 || lo2 < hi2) {
      const int m0 = (lo0 + hi0) >> 1, m1 = (lo1 + hi1) >> 1, m2 = (lo2 + hi2) >> 1;
      const int v0 = lo0 < hi0 ? A[m0] : 0, v1 = lo1 < hi1 ? A[m1] : 0, v2 = lo2 < hi2 ? B[m2] : 0;
      if (lo0 < hi0) {
        if (v0 < ka) lo0 = m0 + 1; else hi0 = m0;
      }
      if (lo1 < hi1) {
        if (v1 < l + 1) lo1 = m1 + 1; else hi1 = m1;
      }
      if (lo2 < hi2) {
        if (v2 < kb) lo2 = m2 + 1; else hi2 = m2;
      }
    }
    m.lo = lo0;
    m.hi = lo1;
    m.lo2 = lo2;
  }
  // candidate rows to tmpR, columns to tmpC (wave-compacted)
  int* tmpR = reinterpret_cast<int*>(fbuf);
  int* tmpC = tmpR + cExtra;
  {
    const int nkeys = s.misc[4];
    const int lane = tid & 63;
    const unsigned long long below = (1ull << lane) - 1ull;
    for (int t0 = 0; t0 < nkeys; t0 += nt) {
      const int t = t0 + tid;
      const int key = t < nkeys ? keys[t] : -1;
      const bool isr = t < nkeys && key >= 0, isc = t < nkeys && key <= -2;
      const unsigned long long mr = __ballot(isr), mcl = __ballot(isc);
      int br = 0, bc = 0;
      if (lane == 0) {
        if (mr) br = atomicAdd(&s.misc[6], __popcll(mr));
        if (mcl) bc = atomicAdd(&s.misc[7], __popcll(mcl));
      }
      br = __shfl(br, 0, 64);
      bc = __shfl(bc, 0, 64);
      if (isr) {
        const int o = br + __popcll(mr & below);
        if (o < cExtra) tmpR[o] = key;
      }
      if (isc) {
        const int o = bc + __popcll(mcl & below);
        if (o < cExtra) tmpC[o] = ~key;
      }
    }
  }
  __syncthreads();
  if (tid == 0) trace_at(d, K, 22, wall_clock64());
  const int nrow = s.misc[6], ncol = s.misc[7];
  const int mc = q + nrow, mcc = ncol;
  if (nrow > cExtra || ncol > cExtra || (mc + mcc) * q > cBuf - kThreads) return fallback;
  int p2r = 1, p2c = 1;
  while (p2r < nrow) p2r <<= 1;
  while (p2c < ncol) p2c <<= 1;
  // rank sort: rows by the first half of the threads, columns by the second
  constexpr int kRankMax = kRankKeys * (kThreads / 2);
  const bool rank_sort = nrow <= kRankMax && ncol <= kRankMax;
  if (!rank_sort && (q + p2r > kCandCap || p2c > kCandCap)) return kFastFallback;
  if (rank_sort) {
    const int* srcR = tmpR;
    const int* srcC = tmpC;
    if (kG) {
      // the lists sit in global scratch: rank them from LDS (the candidate
      // hash is no longer needed)
      for (int t = tid; t < nrow; t += nt) s.hash[t] = tmpR[t];
      for (int t = tid; t < ncol; t += nt) s.hash[kRankMax + t] = tmpC[t];
      __syncthreads();
      srcR = s.hash;
      srcC = s.hash + kRankMax;
    }
    const int half = nt >> 1;
    if (tid < half)
      rank_place(srcR, nrow, s.cand + q, tid, half);
    else
      rank_place(srcC, ncol, s.candc, tid - half, half);
  } else {
    for (int t = tid; t < nrow; t += nt) s.cand[q + t] = tmpR[t];
    for (int t = tid; t < ncol; t += nt) s.candc[t] = tmpC[t];
    __syncthreads();
    wg_bitonic_sort(s.cand + q, nrow);
    wg_bitonic_sort(s.candc, ncol);
  }
  for (int t = tid; t < q; t += nt) s.cand[t] = f + t;
  if (tid == 0) trace_at(d, K, 23, wall_clock64());
  // update terms per predecessor: column panel (rows >= f) x (columns in K),
  // row panel (rows in K) x (columns > l); their offsets by one wave when
  // there are at most 64 predecessors
  int nterms;
  if (np + npr <= 64) {
    if (tid < 64) {
      int x = 0;
      if (tid < np + npr) {
        const PredMeta& m = fmeta[tid];
        x = tid < np ? (m.nr - m.lo2) * (m.hi - m.lo) : (m.hi - m.lo) * (m.nc - m.lo2);
      }
      int incl = x;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if (tid >= o) incl += t;
      }
      if (tid < np + npr) fmeta[tid].ioff = incl - x;
      if (tid == 63) s.misc[26] = incl;
    }
    __syncthreads();
    nterms = s.misc[26];
  } else {
    __syncthreads();
    for (int t = tid; t < np + npr; t += nt) {
      const PredMeta& m = fmeta[t];
      fpred[t] = t < np ? (m.nr - m.lo2) * (m.hi - m.lo) : (m.hi - m.lo) * (m.nc - m.lo2);
    }
    __syncthreads();
    nterms = wg_scan_array(fpred, np + npr, s.scan);
    for (int t = tid; t < np + npr; t += nt) fmeta[t].ioff = fpred[t];
    __syncthreads();
  }
  // matrix-core tiles: the first 16 x 16 tile of every predecessor's term
  // product (in PredMeta::pad) and their total
  int ntiles = 0;
  if (a.mfma) {
    __syncthreads();
    if (tid < 64) {  // wave 0 scans 64 predecessors at a time
      int base = 0;
      for (int t0 = 0; t0 < np + npr; t0 += 64) {
        const int t = t0 + tid;
        int x = 0;
        if (t < np + npr) {
          const PredMeta& m = fmeta[t];
          const int M = t < np ? m.nr - m.lo2 : m.hi - m.lo;
          const int N = t < np ? m.hi - m.lo : m.nc - m.lo2;
          x = ((M + 15) >> 4) * ((N + 15) >> 4);
        }
        int incl = x;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
          const int y = __shfl_up(incl, o, 64);
          if (tid >= o) incl += y;
        }
        if (t < np + npr) fmeta[t].pad = base + incl - x;
        base += __shfl(incl, 63, 64);
      }
      if (tid == 0) s.misc[30] = base;
    }
    __syncthreads();
    ntiles = s.misc[30];
  }
  if (tid == 0) {
    trace_at(d, K, 3, wall_clock64());
    trace_at(d, K, 16, (unsigned long long)np);
    trace_at(d, K, 17, (unsigned long long)npr);
    trace_at(d, K, 18, (unsigned long long)mc);
    trace_at(d, K, 19, (unsigned long long)mcc);
  }

  // ---- phase 4: A's values into the panels, update terms (chunked)
  double* Cp = fbuf;                    // mc x q, row-major
  double* Rp = Cp + mc * q;             // mcc x q (column z of the row panel)
  double* const Tm = Rp + mcc * q;      // update terms
  // a chunk holds cap terms and, after them, each term's panel position
  // (without a.det the terms go straight into the panels: one chunk)
  const int cap = a.det ? (cBuf - (mc + mcc) * q) * 2 / 3 : max(nterms, 1);
  int* Ti = reinterpret_cast<int*>(Tm + cap);
  // the panels accumulate in P: the global variant's go to LDS when both
  // fit the hash area (free from the candidate sort to the drop test) and
  // are copied to the global slot afterwards
  const int npanel = (mc + mcc) * q;
  const bool lpanel = kG && npanel <= kHashSlots / 2;
  double* P = lpanel ? reinterpret_cast<double*>(s.hash) : fbuf;
  for (int e = tid; e < npanel; e += nt) P[e] = 0.0;
  __syncthreads();
  // A's entries of K: panel position (-1: outside the panels) and value
  const int nA0 = segoff[1], nA = segoff[2];
  for (int e = nt + tid; e < nA; e += nt) {  // beyond the first nt entries (rare)
    const AEntry x = a_entry(a, s, stage, e, nA0, f, l, q, mc, mcc);
    if (x.tgt >= 0) {
      if (a.det)
        P[x.tgt] = *x.src;
      else
        atomicAdd(&P[x.tgt], *x.src);  // the terms may already be arriving
    }
  }
  // the first nt: loaded now, stored with the first chunk of terms, so both
  // loads share one round trip
  int a_tgt = -1;
  double a_val = 0.0;
  if (tid < nA) {
    const AEntry x = a_entry(a, s, stage, tid, nA0, f, l, q, mc, mcc);
    a_tgt = x.tgt;
    if (a_tgt >= 0) a_val = *x.src;
  }
  const int npt = np + npr;
  constexpr int kU = 4;  // terms per thread in flight
  for (int i0 = 0; i0 < nterms; i0 += cap) {
    const int i1 = min(nterms, i0 + cap);
    if (a.mfma) {
      if (a.update_prec == 0)
        mfma_terms<0>(a, fmeta, npt, np, i0, i1, Tm, ntiles);
      else if (a.update_prec == 1)
        mfma_terms<1>(a, fmeta, npt, np, i0, i1, Tm, ntiles);
      else
        mfma_terms<2>(a, fmeta, npt, np, i0, i1, Tm, ntiles);
    }
    for (int e0 = i0 + tid; e0 < i1; e0 += kU * nt) {
      // (1) the predecessor and the (row, column) pair of each term
      // each term's row and column index: one from the staged lists (so),
      // the one inside K (ho) from the heap in the global variant, from the
      // staged lists in the LDS variant
      int64_t lo[kU], wo[kU], ho[kU];
      int pp[kU], so[kU];
      bool colp[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * nt;
        lo[u] = wo[u] = ho[u] = 0;
        pp[u] = 0;
        so[u] = 0;
        colp[u] = true;
        if (e < i1) {
          int lo_t = 0, hi_t = npt;  // last t with ioff <= e
          while (hi_t - lo_t > 1) {
            const int mid = (lo_t + hi_t) >> 1;
            if (fmeta[mid].ioff <= e)
              lo_t = mid;
            else
              hi_t = mid;
          }
          const int t = lo_t;
          const PredMeta& m = fmeta[t];
          const int w = e - m.ioff;
          int ri, cj;
          if (t < np) {
            const int nc = m.hi - m.lo;
            ri = m.lo2 + w / nc;
            cj = m.lo + w % nc;
            so[u] = segoff[2 + t] + ri;
            ho[u] = kG ? m.coff + cj : (int64_t)segoff[2 + np + t] + cj;
          } else {
            const int nr = m.hi - m.lo;
            ri = m.lo + w % nr;
            cj = m.lo2 + w / nr;
            so[u] = segoff[2 + 2 * np + npr + (t - np)] + cj;
            ho[u] = kG ? m.roff + ri : (int64_t)segoff[2 + 2 * np + (t - np)] + ri;
            colp[u] = false;
          }
          lo[u] = m.loff + (int64_t)ri * m.p;
          wo[u] = m.woff + (int64_t)cj * m.p;
          pp[u] = m.p;
        }
      }
      // (2) all loads first: row and column indices, then L_J and W_J values
      int rr[kU], cc[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int sv = stage[so[u]];
        const int hv = kG ? a.idx_heap[ho[u]] : stage[ho[u]];
        rr[u] = colp[u] ? sv : hv;
        cc[u] = colp[u] ? hv : sv;
      }
      double acc[kU];
      if (a.mfma) {
        // values come from the matrix-core tiles; only positions here
      } else {
        // the terms' values: each thread's kU dot products in step, the
        // rows of L_J and columns of W_J read 16 bytes at a time (2 FP64,
        // 4 FP32 or 8 BF16 values per load; the value heap has slack past
        // its end for the last partial load), the products taken in index
        // order with one fused multiply-add each, as update_term does
        int pmax = 0;
#pragma unroll
        for (int u = 0; u < kU; ++u) pmax = max(pmax, pp[u]);
        if (a.update_prec == 0) {
          const double* v = static_cast<const double*>(a.val_heap);
#pragma unroll
          for (int u = 0; u < kU; ++u) acc[u] = 0.0;
          for (int t0 = 0; t0 < pmax; t0 += 2) {
            wide_f64 x[kU], y[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
              // only while the row lasts: at most 1 values past its end
              x[u] = t0 < pp[u] ? *reinterpret_cast<const wide_f64*>(v + lo[u] + t0) : wide_f64{};
              y[u] = t0 < pp[u] ? *reinterpret_cast<const wide_f64*>(v + wo[u] + t0) : wide_f64{};
            }
#pragma unroll
            for (int u = 0; u < kU; ++u)
#pragma unroll
              for (int k = 0; k < 2; ++k)
                if (t0 + k < pp[u]) acc[u] = fma(x[u][k], y[u][k], acc[u]);
          }
        } else if (a.update_prec == 1) {
          const float* v = static_cast<const float*>(a.val_heap);
          float fa[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) fa[u] = 0.0f;
          for (int t0 = 0; t0 < pmax; t0 += 4) {
            wide_f32 x[kU], y[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
              // only while the row lasts: at most 3 values past its end
              x[u] = t0 < pp[u] ? *reinterpret_cast<const wide_f32*>(v + lo[u] + t0) : wide_f32{};
              y[u] = t0 < pp[u] ? *reinterpret_cast<const wide_f32*>(v + wo[u] + t0) : wide_f32{};
            }
#pragma unroll
            for (int u = 0; u < kU; ++u)
#pragma unroll
              for (int k = 0; k < 4; ++k)
                if (t0 + k < pp[u]) fa[u] = fmaf(x[u][k], y[u][k], fa[u]);
          }
#pragma unroll
          for (int u = 0; u < kU; ++u) acc[u] = (double)fa[u];
        } else {
          const uint16_t* v = static_cast<const uint16_t*>(a.val_heap);
          float fa[kU];
#pragma unroll
          for (int u = 0; u < kU; ++u) fa[u] = 0.0f;
          for (int t0 = 0; t0 < pmax; t0 += 8) {
            wide_bf16 x[kU], y[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u) {
              // only while the row lasts: at most 7 values past its end
              x[u] = t0 < pp[u] ? *reinterpret_cast<const wide_bf16*>(v + lo[u] + t0) : wide_bf16{};
              y[u] = t0 < pp[u] ? *reinterpret_cast<const wide_bf16*>(v + wo[u] + t0) : wide_bf16{};
            }
#pragma unroll
            for (int u = 0; u < kU; ++u)
#pragma unroll
              for (int k = 0; k < 8; ++k)
                if (t0 + k < pp[u]) fa[u] = fmaf(bf16_float(x[u][k]), bf16_float(y[u][k]), fa[u]);
          }
#pragma unroll
          for (int u = 0; u < kU; ++u) acc[u] = (double)fa[u];
        }
      }
      // (3) positions in the panels: the candidate row (column) of each
      // term by branch-free lower bounds stepping together
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * nt;
        if (e < i1) {
          const int pos = colp[u] ? lower_bound(s.cand, mc, rr[u]) * q + (cc[u] - f)
                                  : mc * q + lower_bound(s.candc, mcc, cc[u]) * q + (rr[u] - f);
          if (a.det) {
            if (!a.mfma) Tm[e - i0] = acc[u];
            Ti[e - i0] = pos;
          } else {
            atomicAdd(&P[pos], -acc[u]);  // any order: not run-to-run reproducible
          }
        }
      }
    }
    if (i0 == 0 && a_tgt >= 0) {
      if (a.det)
        P[a_tgt] = a_val;
      else
        atomicAdd(&P[a_tgt], a_val);
    }
    __syncthreads();
    if (i0 == 0 && tid == 0) trace_at(d, K, 9, wall_clock64());  // first chunk's terms done
    if (!a.det) continue;  // the terms are in the panels already
    // (4) in predecessor order (a predecessor's terms hit distinct
    // entries).  Column predecessors update only the column panel and row
    // predecessors only the row panel, so the k-th of each go together.
    // Each thread's first kAhead entries of the next pair are loaded before
    // the barrier of the current one.
    constexpr int kAhead = 2;
    const int kmax = max(np, npr);
    int ra0 = 0, rna = 0, rb0 = 0, rnab = 0;  // the current pair's term ranges
    int pi[kAhead];
    double pv[kAhead];
    auto fetch = [&](int k) {
      int a0 = 0, a1 = 0, b0 = 0, b1 = 0;
      if (k < np) {
        a0 = max(i0, fmeta[k].ioff);
        a1 = min(i1, k + 1 < npt ? fmeta[k + 1].ioff : nterms);
      }
      if (k < npr) {
        const int t = np + k;
        b0 = max(i0, fmeta[t].ioff);
        b1 = min(i1, t + 1 < npt ? fmeta[t + 1].ioff : nterms);
      }
      ra0 = a0;
      rb0 = b0;
      rna = max(0, a1 - a0);
      rnab = rna + max(0, b1 - b0);
#pragma unroll
      for (int r = 0; r < kAhead; ++r) {
        const int x = tid + r * nt;
        pi[r] = -1;
        if (x < rnab) {
          const int e = (x < rna ? ra0 + x : rb0 + (x - rna)) - i0;
          pi[r] = Ti[e];
          pv[r] = Tm[e];
        }
      }
    };
    if (kmax > 0) fetch(0);
    for (int k = 0; k < kmax; ++k) {
      // a pair's positions are distinct: all reads, then all writes
#pragma unroll
      for (int r = 0; r < kAhead; ++r)
        if (pi[r] >= 0) P[pi[r]] -= pv[r];
      for (int x = tid + kAhead * nt; x < rnab; x += nt) {  // beyond the loaded ones
        const int e = (x < rna ? ra0 + x : rb0 + (x - rna)) - i0;
        P[Ti[e]] -= Tm[e];
      }
      const bool any = rnab > 0;  // uniform
      if (k + 1 < kmax) fetch(k + 1);
      if (any) __syncthreads();
    }
  }
  if (nterms == 0 && a_tgt >= 0) P[a_tgt] = a_val;  // no chunk ran (no term can race)
  __syncthreads();
  // the LDS panels stay there through the pivot, drop test and factor
  // writes when the keep flags fit the LDS after the predecessor data (the
  // global variant keeps that data over the LDS variant's panel, metadata
  // and nothing else there); else they go to the global slot
  int* const keep_lds = reinterpret_cast<int*>(fmeta + npt);
  const bool lkeep =
      lpanel && (int64_t)(mc + mcc) * (int64_t)sizeof(int) + (int64_t)npt * (int64_t)sizeof(PredMeta) <=
                    (int64_t)kRegionBytes - (ownlate ? 0 : 8 * kGOwnSlots);
  if (lpanel && !lkeep) {
    for (int e = tid; e < npanel; e += nt) fbuf[e] = P[e];
    __syncthreads();
  }
  if (lkeep) {
    Cp = P;
    Rp = P + mc * q;
  }
  if (tid == 0) {
    const unsigned long long now = wall_clock64();
    trace_at(d, K, 8, now);
    if (nterms == 0) trace_at(d, K, 9, now);
  }

  // ---- pivot block and drop test (shared with the general path)
  double* sS = s_dyn;
  double* sW = s_dyn + q * q;
  // wave 0 takes the pivot block; the other waves meanwhile look up the
  // blocks of the candidate rows and columns (the staged lists are done)
  int* keep_r = lkeep ? keep_lds : s.hash;
  int* keep_c = lkeep ? keep_lds + mc : s.hash + (kG ? kCandCap : 1024);  // below the own-count table
  int* rblk = stage;                // block of candidate row z
  int* cblk = stage + cSpace;       // block of candidate column z
  int* rbp = stage + 2 * cSpace;    // position in TR_K of the first kept row of a block
  int* cbp = stage + 3 * cSpace;
  int* trL = stage + 4 * cSpace;    // TR_K and TC_K
  int* tcL = stage + 5 * cSpace;
  if (tid < 64) {
    const bool ok = (q <= 8 && pivot_regs(a, q, Cp, sS, sW)) ||
                    pivot_block<true>(a, K, q, Cp, sS, sW, s, s.alpha_k);
    if (tid == 0) s.misc[14] = ok ? 1 : 0;
  } else {
    for (int z = q + tid - 64; z < mc; z += nt - 64) rblk[z] = a.blockOf[s.cand[z]];
    for (int z = tid - 64; z < mcc; z += nt - 64) cblk[z] = a.blockOf[s.candc[z]];
  }
  __syncthreads();
  if (!s.misc[14]) return kFastError;
  if (tid == 0) trace_at(d, K, 10, wall_clock64());
  drop_flags(a, Cp, Rp, mc, mcc, q, sW, keep_r, keep_c, s.tau_k, K, s.cand, s.candc, s.acc_drop);
  if (tid == 0) trace_at(d, K, 11, wall_clock64());

  // ---- positions of kept rows / columns and of their distinct blocks
  // (one wave, 64 candidates per step)
  if (tid < 64) {
    const unsigned long long lt = (1ull << tid) - 1ull;
    for (int side = 0; side < 2; ++side) {
      int* keep = side ? keep_c : keep_r;
      const int* blk = side ? cblk : rblk;
      int* bp = side ? cbp : rbp;
      const int z0 = side ? 0 : q, z1 = side ? mcc : mc;
      int cpos = 0, cb = 0, lastb = -1;
      for (int zb = z0; zb < z1; zb += 64) {
        const int z = zb + tid;
        const bool in = z < z1;
        const int kp = in ? keep[z] : 0;
        const int b = in ? blk[z] : -1;
        const unsigned long long m = __ballot(kp);
        const unsigned long long below = m & lt;
        const int pl = below ? 63 - __clzll(below) : 0;
        const int pb = __shfl(b, pl, 64);
        const bool nb = kp && (below ? pb : lastb) != b;
        const unsigned long long bm = __ballot(nb);
        if (in) {
          keep[z] = kp ? cpos + __popcll(below) : -1;
          bp[z] = nb ? cb + __popcll(bm & lt) : -1;
        }
        if (m) lastb = __shfl(b, 63 - __clzll(m), 64);
        cpos += __popcll(m);
        cb += __popcll(bm);
      }
      if (tid == 0) {
        s.misc[20 + 2 * side] = cpos;
        s.misc[21 + 2 * side] = cb;
      }
    }
  }
  __syncthreads();
  const int mk = s.misc[20], ntr = s.misc[21], nk = s.misc[22], ntc = s.misc[23];
  if (tid == 0) {
    const bool over = !heap_take(a, s, (long long)(mk + nk) * q, (long long)(mk + nk + ntr + ntc));
    s.misc[16] = over ? 1 : 0;
    if (over) raise_error(a, kDevHeapOverflow, K);
  }
  __syncthreads();
  if (s.misc[16]) return kFastError;
  if (tid == 0) trace_at(d, K, 12, wall_clock64());
  const int64_t vo = s.off[0];
  store_pivot(a, K, q, sS, sW);
  const int64_t io = s.off[1];
  int32_t* Rout = a.idx_heap + io;
  int32_t* Cout = Rout + mk;
  int32_t* TRout = Cout + nk;
  int32_t* TCout = TRout + ntr;
  for (int w = tid; w < (mc - q) * q; w += nt) {
    const int z = q + w / q, c = w % q;
    const int p = keep_r[z];
    if (p >= 0) {
      double acc = 0.0;
      for (int t = 0; t < q; ++t) acc = fma(Cp[z * q + t], sW[t * q + c], acc);
      store_factor(a, vo + (int64_t)p * q + c, acc);
    }
  }
  for (int w = tid; w < mcc * q; w += nt) {
    const int z = w / q, r = w % q;
    const int p = keep_c[z];
    if (p >= 0) store_factor(a, vo + (int64_t)mk * q + (int64_t)p * q + r, Rp[z * q + r]);
  }
  for (int z = q + tid; z < mc; z += nt) {
    const int p = keep_r[z];
    if (p >= 0) {
      Rout[p] = s.cand[z];
      const int b = rbp[z];
      if (b >= 0) {
        TRout[b] = rblk[z];
        trL[b] = rblk[z];
      }
    }
  }
  for (int z = tid; z < mcc; z += nt) {
    const int p = keep_c[z];
    if (p >= 0) {
      Cout[p] = s.candc[z];
      const int b = cbp[z];
      if (b >= 0) {
        TCout[b] = cblk[z];
        tcL[b] = cblk[z];
      }
    }
  }
  if (tid == 0) {
    a.roff[K] = io;
    a.nr[K] = mk;
    a.coff[K] = io + mk;
    a.nc[K] = nk;
    a.loff[K] = vo;
    a.woff[K] = vo + (int64_t)mk * q;
    a.troff[K] = io + mk + nk;
    a.ntr[K] = ntr;
    a.tcoff[K] = io + mk + nk + ntr;
    a.ntc[K] = ntc;
  } else if (tid >= 64 && tid < 128) {
    // the update flops and bytes of the block, one wave over the predecessors
    double flops = 0.0, ubytes = 0.0;
    for (int t = tid - 64; t < npt; t += 64) {
      const PredMeta& m = fmeta[t];
      const int nr = t < np ? m.nr - m.lo2 : m.hi - m.lo;
      const int nc = t < np ? m.hi - m.lo : m.nc - m.lo2;
      flops += 2.0 * nr * nc * m.p;
      ubytes += (double)a.elem_bytes * m.p * (nr + nc);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      flops += __shfl_xor(flops, o, 64);
      ubytes += __shfl_xor(ubytes, o, 64);
    }
    if (tid == 64) {
      s.acc_flops += (unsigned long long)flops;
      s.acc_bytes += (unsigned long long)ubytes;
    }
  }
  __syncthreads();
  if (tid == 0) trace_at(d, K, 13, wall_clock64());
  // TR_K and TC_K in LDS for the lookups below (the candidate lists are no
  // longer needed)
  const int* trS = trL;
  const int* tcS = tcL;
  if (kG) {
    for (int t = tid; t < ntr; t += nt) s.cand[t] = trL[t];
    for (int t = tid; t < ntc; t += nt) s.candc[t] = tcL[t];
    trS = s.cand;
    tcS = s.candc;
    __syncthreads();
  }
  // K updates the row panels of the blocks of its rows of L and the column
  // panels of the blocks of its columns of U; with the same pass, the
  // successor counts (as add_successor_counts)
  for (int t = tid; t < ntr + ntc; t += nt) {
    const bool row = t < ntr;
    const int B = row ? trS[t] : tcS[t - ntr];
    const int c = row ? lower_bound(tcS, ntc, B) : lower_bound(trS, ntr, B);
    int32_t* cnt_arr = row ? a.row_cnt : a.col_cnt;
    // the three accesses are independent: all in flight before any result
    // is used
    const int started = __hip_atomic_load(&d.started[B], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int pos = atomicAdd(&cnt_arr[B], 1);
    const int before = atomicAdd(&d.pending[B], c);
    if (started || (c > 0 && before <= 0)) raise_error(a, kDevProtocol, K);
    push_pred_at(a, row ? a.row_list : a.col_list, row ? a.row_ovf : a.col_ovf, B, K, pos);
  }
  if (tid == 0) trace_at(d, K, 14, wall_clock64());
  if (ownlate) __syncthreads();  // trS / tcS overlay the counts cleared below

  // ---- K's own counts (as updater_set): A's entries of K in later blocks,
  // TR_J > K of column predecessors, TC_J > K of row predecessors; the LDS
  // variant built them while staging
  int* own = ownlate ? s.hash : kG ? gown : s.hash + kFastOwn;
  int* cnt = ownlate ? s.cand : kG ? gown + kGOwnSlots : s.hash + kFastOwnCnt;  // per hash slot
  const int own_slots = ownlate ? kHashSlots : kG ? kGOwnSlots : kFastOwnSlots;
  if (ownlate) {
  for (int t = tid; t < kHashSlots; t += nt) {
    s.hash[t] = -1;
    cnt[t] = 0;
  }
  if (tid == 0) {
    s.misc[4] = 0;
    s.misc[5] = 0;
  }
  const int nseg2 = 2 + npt;
  {
    for (int g = tid; g < nseg2; g += nt)
      fseg[g] = g == 0   ? (int)(s.x.cpk[q] - s.x.cpk[0])
                : g == 1 ? (int)(s.x.rpk[q] - s.x.rpk[0])
                : g - 2 < np ? fmeta[g - 2].ntr
                             : fmeta[g - 2].ntc;
    __syncthreads();
    const int tot = wg_scan_array(fseg, nseg2, s.scan);
    if (tid == 0) fseg[nseg2] = tot;
    __syncthreads();
  }
  const int tot2 = fseg[nseg2];
  for (int base = 0; base < tot2; base += kBatch * nt) {
    int v[kBatch];
    for (int k = 0; k < kBatch; ++k) {
      const int e = base + tid + k * nt;
      if (e < tot2) {
        const int sg = last_le(fseg, nseg2, e);
        const int i = e - fseg[sg];
        if (sg == 0)
          v[k] = a.bri[s.x.cpk[0] + i];
        else if (sg == 1)
          v[k] = a.bci[s.x.rpk[0] + i];
        else if (sg - 2 < np)
          v[k] = a.idx_heap[fmeta[sg - 2].troff + i];
        else
          v[k] = a.idx_heap[fmeta[sg - 2].tcoff + i];
      }
    }
    for (int k = 0; k < kBatch; ++k) {
      const int e = base + tid + k * nt;
      if (e < tot2 && v[k] > K) {
        const int h = hash_insert_at(s.hash, v[k], &s.misc[4]);
        if (h < 0)
          s.misc[5] = 1;
        else
          atomicAdd(&cnt[h], 1);
      }
    }
  }
  __syncthreads();
  if (s.misc[5]) {
    if (tid == 0) raise_error(a, kDevAnnOverflow, K);
    return kFastError;
  }
  }
  if (tid == 0) trace_at(d, K, 15, wall_clock64());
  // publish: every write and count of this block is visible before the
  // retraction
  wg_release_agent();
  const int dK = s.misc[24] + 1;
  // the worker's next queue position (claimed here when next_pos < 0) and
  // the block already there, read while the retractions are in flight
  // (misc[25] = -1: not filled yet)
  if (tid == nt - 1) {
    const int p = next_pos >= 0 ? next_pos : claim_position(d, s);
    s.misc[29] = p;
    s.misc[25] =
        p < a.nb ? __hip_atomic_load(&d.queue[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
  }
  for (int t = tid; t < own_slots; t += nt) {
    const int B = own[t];
    if (B < 0) continue;
    const int c = cnt[t];
    atomicMax(&d.depth[B], dK);
    const int old = atomicSub(&d.pending[B], c);
    if (old < c) raise_error(a, kDevProtocol, K);
    if (old == c) push_ready(a, d, B, K, c);
  }
  if (tid == 0) trace_at(d, K, 4, wall_clock64());
  return kFastDone;
}

// The next seeded block for the calling workgroup, or -1 when they are all
// taken.  The counter moves only while seeded blocks are left, so it stays
// within the seeded count (misc[28]) plus the number of workers.
__device__ __forceinline__ int take_seeded(const FlowArgs& d, Lds& s) {
  if (threadIdx.x == 0) {
    const int L = s.misc[28];
    const int li = __hip_atomic_load(d.leaf_head, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < L
                       ? atomicAdd(d.leaf_head, 1)
                       : L;
    s.misc[27] =
        li < L ? __hip_atomic_load(&d.queue[li], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
  }
  __syncthreads();
  const int KS = s.misc[27];
  __syncthreads();
  return KS;
}

// Worker.  The blocks that nothing can update are seeded at queue positions
// [0, L) before the launch; any worker that would otherwise wait takes the
// next of them from a shared counter.  Positions L, L + 1, ... are filled in
// the order blocks become ready during the sweep; a running worker claims
// one of them at a time (claim_position), in ascending order, and waits for
// its block, taking seeded blocks while it is still empty.  A worker claims
// its next position while its current block retracts its counts, so a
// block made ready during the sweep waits at most for one worker's current
// block, not behind the seeded ones.  Every claimed position belongs to a
// running worker and positions fill in ascending order, so progress needs
// no worker to be resident: the launch is an ordinary one.
// One instance per update precision (0 FP64, 1 FP32, 2 BF16): the constant
// removes the other precisions' code from the instance that runs.
template <int kPrec>
__global__ void __launch_bounds__(kThreads, 2) factor_worker_kernel(FactorArgs a_in, FlowArgs d) {
  FactorArgs a = a_in;
  a.update_prec = kPrec;
  __shared__ Lds s;
  extern __shared__ double s_dyn[];
  const int slot = blockIdx.x;
  if (threadIdx.x == 0) {
    s.hcur[0] = s.hcur[1] = s.hend[0] = s.hend[1] = 0;
    s.acc_flops = s.acc_bytes = 0;
    s.acc_drop[0] = s.acc_drop[1] = 0;
    s.acc_drop[2] = (unsigned long long)__double_as_longlong(INFINITY);
    s.acc_depth = 0;
    // the seeded count, kept in LDS (misc[28]) to spare registers
    s.misc[28] = __hip_atomic_load(d.nleaves, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s.misc[29] = claim_position(d, s);
  }
  __syncthreads();
  int next = -1;  // the block at position pos when already known
  int pos = s.misc[29];
  while (true) {
    // pick the next block: the one at this worker's position, or a seeded
    // one while that position is still empty or once the positions are done
    int K = -1, next_pos = -1;  // next_pos < 0: claim a new position
    if (pos < a.nb) {
      const unsigned long long t0 = wall_clock64();
      K = next;  // uniform: read from LDS after a barrier
      bool seeded = false;
      while (K < 0) {
        K = __hip_atomic_load(&d.queue[pos], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int stop = __hip_atomic_load(a.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                         wall_clock64() - t0 > d.wait_ticks;
        if (__syncthreads_or(stop)) {
          if (threadIdx.x == 0) raise_error(a, kDevSpin, pos);
          return;
        }
        if (__syncthreads_and(K >= 0)) break;
        K = take_seeded(d, s);
        if (K >= 0) {
          seeded = true;
          break;
        }
        __builtin_amdgcn_s_sleep(2);
      }
      if (seeded) next_pos = pos;  // still this worker's position
    } else {
      K = take_seeded(d, s);
      if (K < 0) break;
      next_pos = pos;  // no position left to claim
    }
    // the block; next is the block at the worker's next position if it is
    // already there, else -1
    wg_acquire_agent();
    if (threadIdx.x == 0) {
      trace_at(d, K, 1, wall_clock64());
      trace_at(d, K, 7, (unsigned long long)blockIdx.x);
    }
    if (threadIdx.x == 0) {
      s.misc[25] = -1;
      s.misc[29] = -1;  // set by the fast path when it claims or reads ahead
      s.misc[31] = 0;   // set by the LDS variant once its rounds 1 and 2 are done
    }
    int r = kFastFallback;
    if (a.fast_path == 1) r = factor_block_fast<false>(a, d, K, s, s_dyn, nullptr, next_pos);
    if (r == kFastBig || a.fast_path == 2) {
      __syncthreads();
      r = factor_block_fast<true>(a, d, K, s, s_dyn, a.scratch + (int64_t)slot * a.slot_doubles,
                                  next_pos);
    }
    if (r == kFastFallback) {
      __syncthreads();
      factor_block(a, d, K, slot, s, s_dyn);
    }
    __syncthreads();
    // the next position: read ahead by the fast path, else kept (seeded
    // block, or none left) or claimed now
    if (threadIdx.x == 0 && s.misc[29] < 0) {
      s.misc[29] = next_pos >= 0 ? next_pos : claim_position(d, s);
      s.misc[25] = -1;
    }
    __syncthreads();
    next = s.misc[25];
    pos = s.misc[29];
    __syncthreads();  // s.misc[25] and s.misc[29] are reset by the next block
  }
  if (threadIdx.x == 0) {
    atomicAdd(a.flops, s.acc_flops);
    atomicAdd(a.drop_ctr + 0, s.acc_drop[0]);
    atomicAdd(a.drop_ctr + 1, s.acc_drop[1]);
    atomicMin(a.drop_ctr + 2, s.acc_drop[2]);
    atomicAdd(a.upd_bytes, s.acc_bytes);
    atomicMax(d.max_depth, s.acc_depth);
  }
}

__global__ void fill_block_of(const int32_t* bstart, int nb, int32_t* blockOf) {
  int b = blockIdx.x * blockDim.y + threadIdx.y;
  if (b >= nb) return;
  for (int i = bstart[b] + threadIdx.x; i < bstart[b + 1]; i += blockDim.x) blockOf[i] = b;
}

// out[m] = blockOf[idx[m]] for every stored entry.
__global__ void map_blocks(const int32_t* idx, int64_t nnz, const int32_t* blockOf, int32_t* out) {
  for (int64_t m = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; m < nnz;
       m += (int64_t)gridDim.x * blockDim.x)
    out[m] = blockOf[idx[m]];
}

// pending[K] += entries of A's rows and columns of K that lie in earlier
// blocks.  16 lanes per index i (row i and column i), reading its entries
// contiguously.
__global__ void __launch_bounds__(256) static_pending(int n, const int64_t* rp, const int32_t* bci,
                                                      const int64_t* cp, const int32_t* bri,
                                                      const int32_t* blockOf, int* pending) {
  const int i = blockIdx.x * 16 + (threadIdx.x >> 4);
  const int sub = threadIdx.x & 15;
  int c = 0, K = 0;
  if (i < n) {
    K = blockOf[i];
    for (int64_t m = rp[i] + sub; m < rp[i + 1]; m += 16) c += bci[m] < K;
    for (int64_t m = cp[i] + sub; m < cp[i + 1]; m += 16) c += bri[m] < K;
  }
#pragma unroll
  for (int o = 8; o > 0; o >>= 1) c += __shfl_xor(c, o, 16);
  if (i < n && sub == 0 && c) atomicAdd(&pending[K], c);
}

// Blocks that nothing can update start in the ready queue: flagged here,
// listed in ascending order by a device select.
__global__ void seed_flags(int nb, const int* pending, int* enq, unsigned char* flag) {
  const int K = blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= nb) return;
  const bool seed = pending[K] == 0;
  flag[K] = seed ? 1 : 0;
  if (seed) enq[K] = 1;
}

}  // namespace

// ---------------------------------------------------------------------------
// Refactorization with frozen patterns: new values of A on the last
// factor's final blocks, row and column lists and storage.  Block K's panels
// are the Crout ones of Sec. 2.2 restricted to the stored positions:
//   C(i, j) = A(i, j) - sum over J < K of L_J(i,:) W_J(:,j),
// for i in K or R_K and j in K (column panel), i in K and j in C_K (row
// panel), the terms taken per predecessor J in ascending order and only
// where both ends are stored; then D_K = S_K^-1 (the sweep's pivot routine,
// perturbation included), L_K = C(R_K, K) D_K and W_K = C(K, C_K).  Nothing
// is dropped and nothing merges.  One workgroup per block, all blocks in one
// launch ordered by dependency level: a block waits (bounded) until every
// predecessor has published its values.  The FP64 panels sit in the scratch
// arrays PL (at the L offsets), PW (at the W offsets) and PD (at the pivot
// offsets).
// ---------------------------------------------------------------------------
// One predecessor of the frozen refactorization as the pair loop reads it.
struct FrozenPred {
  long long roff, coff, loff, woff;  // the block's list and value offsets
  int J, s0, cnt;                    // the block and its run inside K
  int p;                             // its width
  int len;                           // length of its row (column) list
  int first;                         // first row from K on (first column beyond K)
  int pad[2];
};
static_assert(sizeof(FrozenPred) == 64, "layout");
// predecessors staged in LDS, over the general path's annotation lists
constexpr int kFrozenStaged = (int)(2 * kAnnCap * sizeof(int) / sizeof(FrozenPred));
static_assert(offsetof(Lds, g.annc) == offsetof(Lds, g.ann) + sizeof(int) * kAnnCap &&
                  offsetof(Lds, g.ann) % alignof(FrozenPred) == 0,
              "layout");
struct FrozenArgs {
  FactorView f;            // the factor rewritten in place (val, dval)
  double* val64;           // = f.val when it is FP64 (else null)
  void* val;               // the stored values (f.val), written
  double* dval;            // D_K, written
  double* sval;            // S_K at the same offsets, or null
  double *PL, *PW, *PD;    // FP64 panels
  double* piv;             // 2 q^2 pivot scratch per block at 2 doff, when not in LDS
  const int64_t *cp, *rp;  // P A P^T: CSC and CSR
  const int32_t *ri, *ci;
  const double *cv, *rv;
  // per block: the blocks J whose C_J (cptr) or R_J (rptr) has a run inside
  // K, ascending, with the run's first position and length
  const int32_t *cptr, *cj, *cs0, *ccnt;
  const int32_t *rptr, *rj, *rs0, *rcnt;
  const int32_t* sched;    // the blocks by (level, index): every predecessor earlier
  int nb;
  int* done;               // per block: set once its values are published
  unsigned long long wait; // bound of a dependency wait (wall-clock ticks)
  FactorArgs fa;           // perturbation settings and status words of the sweep
};

// Position of key in the sorted list x[0..m) or -1.
__device__ __forceinline__ int find_sorted(const int* x, int m, int key) {
  int lo = 0, hi = m;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (x[mid] < key) lo = mid + 1; else hi = mid;
  }
  return lo < m && x[lo] == key ? lo : -1;
}

// One update term of the stored values in precision prec (FP64: fused
// multiply-adds in index order; FP32 / BF16: the same in FP32).
__device__ __forceinline__ double frozen_term(const void* heap, int prec, int64_t lo, int64_t wo,
                                              int p) {
  if (prec == kValF64) {
    const double* v = static_cast<const double*>(heap);
    double acc = 0.0;
    for (int k = 0; k < p; ++k) acc = fma(v[lo + k], v[wo + k], acc);
    return acc;
  }
  float acc = 0.0f;
  for (int k = 0; k < p; ++k)
    acc = fmaf((float)value_load(heap, prec, lo + k), (float)value_load(heap, prec, wo + k), acc);
  return (double)acc;
}

__global__ void __launch_bounds__(kThreads) frozen_block_kernel(FrozenArgs a) {
  __shared__ Lds s;
  extern __shared__ double s_dyn[];
  const int w = blockIdx.x;
  if (w >= a.nb) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const FactorView& f = a.f;
  const int K = a.sched[w];
  // K's values are published (or K gave up) for the blocks that wait on it
  auto publish = [&]() {
    wg_release_agent();
    if (tid == 0) __hip_atomic_store(&a.done[K], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  };
  const int f0 = f.bstart[K], q = f.bstart[K + 1] - f0, l0 = f0 + q - 1;
  const int nr = f.nr[K], nc = f.nc[K];
  const int32_t* RK = f.idx + f.roff[K];
  const int32_t* CK = f.idx + f.coff[K];
  // FP64 panels: in LDS (the candidate hash, unused here) when they fit,
  // else in the scratch arrays
  const bool lp = (int64_t)(nr + nc + q) * q <= kHashSlots / 2;
  double* PL = lp ? reinterpret_cast<double*>(s.hash) : a.PL + f.loff[K];  // nr x q, row-major
  double* PW = lp ? PL + (int64_t)nr * q : a.PW + f.woff[K];              // q x nc, column-major
  double* PD = lp ? PW + (int64_t)nc * q : a.PD + f.doff[K];              // q x q, row-major
  // K's lists in LDS when they fit (searched for every term)
  const bool lr = nr <= kCandCap, lc = nc <= kCandCap;
  for (int t = tid; t < nr && lr; t += nt) s.cand[t] = RK[t];
  for (int t = tid; t < nc && lc; t += nt) s.candc[t] = CK[t];
  const int* Rl = lr ? s.cand : RK;
  const int* Cl = lc ? s.candc : CK;
  for (int e = tid; e < nr * q; e += nt) PL[e] = 0.0;
  for (int e = tid; e < nc * q; e += nt) PW[e] = 0.0;
  for (int e = tid; e < q * q; e += nt) PD[e] = 0.0;
  __syncthreads();
  // A's entries on the stored positions (each position once)
  for (int c = 0; c < q; ++c) {
    const int64_t b = a.cp[f0 + c], e = a.cp[f0 + c + 1];
    for (int64_t m = b + tid; m < e; m += nt) {
      const int r = a.ri[m];
      if (r < f0) continue;
      if (r <= l0) {
        PD[(r - f0) * q + c] = a.cv[m];
      } else {
        const int i = find_sorted(Rl, nr, r);
        if (i >= 0) PL[(int64_t)i * q + c] = a.cv[m];
      }
    }
  }
  for (int r = 0; r < q; ++r) {
    const int64_t b = a.rp[f0 + r], e = a.rp[f0 + r + 1];
    for (int64_t m = b + tid; m < e; m += nt) {
      const int j = a.ci[m];
      if (j <= l0) continue;
      const int k = find_sorted(Cl, nc, j);
      if (k >= 0) PW[(int64_t)k * q + r] = a.rv[m];
    }
  }
  // per predecessor (column-panel ones first, then row-panel ones): the
  // block, its run inside K, its width and list and value offsets, and its
  // first row from the block on (column panel) or first column beyond the
  // block (row panel); staged in LDS all at once when they fit, else read
  // per pair
  const int x0c = a.cptr[K], ncp = a.cptr[K + 1] - x0c;
  const int x0r = a.rptr[K], nrp = a.rptr[K + 1] - x0r;
  auto first_from = [&](const int32_t* v, int m, int key, bool beyond) {
    int lo = 0, hi = m;  // first position with v >= key (beyond: v > key)
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (beyond ? v[mid] <= key : v[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
  };
  auto load_pred = [&](int t) {
    FrozenPred m;
    const bool col = t < ncp;
    const int x = col ? x0c + t : x0r + t - ncp;
    m.J = col ? a.cj[x] : a.rj[x];
    m.s0 = col ? a.cs0[x] : a.rs0[x];
    m.cnt = col ? a.ccnt[x] : a.rcnt[x];
    m.p = f.bstart[m.J + 1] - f.bstart[m.J];
    m.roff = f.roff[m.J];
    m.coff = f.coff[m.J];
    m.loff = f.loff[m.J];
    m.woff = f.woff[m.J];
    m.len = col ? f.nr[m.J] : f.nc[m.J];
    m.first = col ? first_from(f.idx + m.roff, m.len, f0, false)
                  : first_from(f.idx + m.coff, m.len, l0, true);
    return m;
  };
  FrozenPred* md = reinterpret_cast<FrozenPred*>(s.g.ann);
  const bool staged = ncp + nrp <= kFrozenStaged;
  for (int t = tid; staged && t < ncp + nrp; t += nt) md[t] = load_pred(t);
  // every predecessor has published its values (bounded wait; the
  // structure read above is the old factor's and does not change)
  {
    const unsigned long long t0 = wall_clock64();
    bool stop = false;
    for (int t = tid; t < ncp + nrp && !stop; t += nt) {
      const int J = t < ncp ? a.cj[x0c + t] : a.rj[x0r + t - ncp];
      int ready = __hip_atomic_load(&a.done[J], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      while (!ready) {
        __builtin_amdgcn_s_sleep(1);
        // the flag's reload, the error word and the clock go out together
        ready = __hip_atomic_load(&a.done[J], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const int err = __hip_atomic_load(a.fa.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long now = wall_clock64();
        if (!ready && (err != 0 || now - t0 > a.wait)) {
          stop = true;
          break;
        }
      }
    }
    if (__syncthreads_or(stop)) {
      if (tid == 0) raise_error(a.fa, kDevSpin, K);
      publish();
      return;
    }
    wg_acquire_agent();
  }
  // the k-th column-panel predecessor (columns running inside K) and the
  // k-th row-panel predecessor (rows running inside K) together, in
  // ascending order: they update different panels, and one predecessor's
  // terms hit distinct entries, so one barrier per pair keeps every entry's
  // terms in block order
  for (int k = 0; k < max(ncp, nrp); ++k) {
    FrozenPred mc{}, mr{};
    if (k < ncp) mc = staged ? md[k] : load_pred(k);
    if (k < nrp) mr = staged ? md[ncp + k] : load_pred(ncp + k);
    const int c0 = mc.s0, cn = mc.cnt, pc = mc.p, loc = mc.first;
    const int rows = k < ncp ? mc.len - loc : 0;
    const int32_t* RJc = f.idx + mc.roff;
    const int32_t* CJc = f.idx + mc.coff;
    const int r0 = mr.s0, rn = mr.cnt, pr = mr.p, lor = mr.first;
    const int cols = k < nrp ? mr.len - lor : 0;
    const int32_t* RJr = f.idx + mr.roff;
    const int32_t* CJr = f.idx + mr.coff;
    const int na = rows * cn, nab = na + (k < nrp ? rn * cols : 0);
    // term e of the pair and its entry (null: the position is not stored)
    auto term_at = [&](int e, double*& dst) -> double {
      dst = nullptr;
      if (e < na) {
        const int i = loc + e / cn, t = c0 + e % cn;
        const int r = RJc[i];
        double* row;
        if (r <= l0) {
          row = PD + (r - f0) * q;
        } else {
          const int ii = find_sorted(Rl, nr, r);
          if (ii < 0) return 0.0;
          row = PL + (int64_t)ii * q;
        }
        dst = row + (CJc[t] - f0);
        return frozen_term(f.val, f.vprec, mc.loff + (int64_t)i * pc, mc.woff + (int64_t)t * pc,
                           pc);
      }
      const int e2 = e - na;
      const int i = r0 + e2 % rn, t = lor + e2 / rn;
      const int kk = find_sorted(Cl, nc, CJr[t]);
      if (kk < 0) return 0.0;
      dst = PW + (int64_t)kk * q + (RJr[i] - f0);
      return frozen_term(f.val, f.vprec, mr.loff + (int64_t)i * pr, mr.woff + (int64_t)t * pr,
                         pr);
    };
    // a pair's terms hit distinct entries, so four of them are formed
    // (their loads in flight together) before they are subtracted
    constexpr int kU = 4;
    for (int e0 = tid; e0 < nab; e0 += kU * nt) {
      double v[kU];
      double* d[kU];
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int e = e0 + u * nt;
        d[u] = nullptr;
        v[u] = e < nab ? term_at(e, d[u]) : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kU; ++u)
        if (d[u]) *d[u] -= v[u];
    }
    __syncthreads();
  }
  // pivot block (the sweep's routine and perturbation), then L_K and W_K
  double* sS = a.piv ? a.piv + 2 * f.doff[K] : s_dyn;
  double* sW = sS + q * q;
  if (tid == 0) s.alpha_k = a.fa.alpha;
  __syncthreads();
  if (tid < 64) {
    const bool ok = (q <= 8 && pivot_regs(a.fa, q, PD, sS, sW)) ||
                    pivot_block<true>(a.fa, K, q, PD, sS, sW, s, s.alpha_k);
    if (tid == 0) s.misc[14] = ok ? 1 : 0;
  }
  __syncthreads();
  if (!s.misc[14]) {  // reported through the status words
    publish();
    return;
  }
  const int64_t dof = f.doff[K];
  for (int e = tid; e < q * q; e += nt) {
    a.dval[dof + e] = sW[e];
    if (a.sval) a.sval[dof + e] = sS[e];
  }
  for (int e = tid; e < nr * q; e += nt) {
    const int i = e / q, c = e % q;
    double acc = 0.0;
    for (int t = 0; t < q; ++t) acc = fma(PL[(int64_t)i * q + t], sW[t * q + c], acc);
    value_store(a.val, f.vprec, f.loff[K] + e, acc);
  }
  for (int e = tid; e < nc * q; e += nt) value_store(a.val, f.vprec, f.woff[K] + e, PW[e]);
  publish();
}

// Dependency levels of the frozen refactorization: level(K) = 1 + the
// largest level of the blocks whose columns (cptr) or rows (rptr) run
// inside K, all of them earlier.  One wave per block in ascending order of
// workgroups (every dependency at a lower slot, the hardware starts
// workgroups in index order); bounded waits.
__global__ void __launch_bounds__(256) frozen_levels(int nb, const int32_t* cptr, const int32_t* cj,
                                                     const int32_t* rptr, const int32_t* rj,
                                                     int* lev, int* err, unsigned long long wait) {
  const int K = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (K >= nb) return;  // no workgroup barrier below
  const int lane = threadIdx.x & 63;
  int l = 0;
  const unsigned long long t0 = wall_clock64();
  for (int side = 0; side < 2; ++side) {
    const int32_t* ptr = side ? rptr : cptr;
    const int32_t* adj = side ? rj : cj;
    for (int e = ptr[K]; e < ptr[K + 1]; e += 64) {
      const int J = e + lane < ptr[K + 1] ? adj[e + lane] : -1;
      int v = J >= 0 ? __hip_atomic_load(&lev[J], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
      while (!__all(v >= 0)) {
        __builtin_amdgcn_s_sleep(1);
        // the level's reload, the error word and the clock go out together
        const int nv = v < 0 ? __hip_atomic_load(&lev[J], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : v;
        const int e = __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const unsigned long long now = wall_clock64();
        v = nv;
        if (e != 0) return;
        if (now - t0 > wait && !__all(v >= 0)) {
          if (lane == 0) atomicExch(err, 1);
          return;
        }
      }
      if (J >= 0) l = max(l, v + 1);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) l = max(l, __shfl_xor(l, o, 64));
  if (lane == 0) __hip_atomic_store(&lev[K], l, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Ends of every block's value ranges (L and W) and pivot range, maximum.
__global__ void frozen_extent(FactorView f, unsigned long long* mx) {
  const int K = blockIdx.x * blockDim.x + threadIdx.x;
  if (K >= f.nb) return;
  const int64_t q = f.bstart[K + 1] - f.bstart[K];
  const int64_t e = max(f.loff[K] + f.nr[K] * q, f.woff[K] + f.nc[K] * q);
  atomicMax(mx, (unsigned long long)e);
  atomicMax(mx + 1, (unsigned long long)(f.doff[K] + q * q));
  atomicMax(mx + 2, (unsigned long long)q);
}
__global__ void frozen_iota(int n, int32_t* v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

// ---------------------------------------------------------------------------
// Host driver
// ---------------------------------------------------------------------------
int64_t factor_partition(bilu_handle* h, double tau) {
  using clk = std::chrono::steady_clock;
  auto t0 = clk::now();
  std::vector<int32_t>& bs = h->bstart0;
  double t_sets = 0.0;
  // ILU(1,tau) on the device; the host computation when a kernel capacity
  // was exceeded (or the step is off)
  int64_t nb = h->opt.use_ilu1t ? ilu1t_partition_device(h, tau, bs, &t_sets) : -1;
  h->stats.ilu1t_host = nb < 0 && h->opt.use_ilu1t ? 1 : 0;
  if (nb < 0) {
    (void)hipGetLastError();
    if (ensure_host_matrix(h) != BILU_OK) return -1;
    nb = ilu1t_partition(h, tau, bs, &t_sets);
  }
  h->stats.t_ilu1t = std::chrono::duration<double>(clk::now() - t0).count();
  h->stats.t_phase[0] = t_sets;
  h->stats.t_phase[1] = h->stats.t_ilu1t - t_sets;
  return nb;
}

bilu_status factor_device(bilu_handle* h, double tau) {
  if (factor_partition(h, tau) < 0) return fail(h, BILU_ERR_INTERNAL, "partition failed");
  return factor_sweep(h, tau, nullptr, nullptr);
}

bilu_status factor_sweep(bilu_handle* h, double tau, const std::vector<double>* tau_blk,
                         const std::vector<double>* alpha_blk) {
  using clk = std::chrono::steady_clock;
  auto t1 = clk::now();
  h->stats.heap_regrows = 0;
  const int64_t n = h->n;
  const std::vector<int32_t>& bs = h->bstart0;
  const int64_t nb = (int64_t)bs.size() - 1;
  int32_t maxq = 0;
  for (int64_t b = 0; b < nb; ++b) maxq = std::max(maxq, bs[b + 1] - bs[b]);
  if (maxq > kMaxWidth) return fail(h, BILU_ERR_INVALID, "block wider than the kernel limit");
  // the settings of this sweep: the options, or the tuned entry for its
  // precision, width class and reproducibility requirement
  {
    TunedEntry& e = h->eff;
    e.precision = h->opt.update_precision;
    e.width_class = maxq > kFastWidth ? 1 : 0;
    e.reproducible = h->opt.deterministic;
    h->stats.max_width_initial = maxq;
    e.workers_per_cu = h->opt.workers_per_cu;
    e.update_mfma = h->opt.update_mfma;
    e.factor_path = h->opt.factor_path;
    e.apply_path = h->opt.apply_path;
    e.deterministic = h->opt.deterministic;
    TunedEntry t;
    h->stats.tuning_applied = 0;
    // a tuned entry supplies the settings left at their defaults (0); a
    // setting the caller chose stays
    if (h->opt.use_tuning && tuned_entry(e.precision, e.width_class, h->opt.deterministic, &t)) {
      if (e.workers_per_cu == 0) e.workers_per_cu = t.workers_per_cu;
      if (e.update_mfma == 0) e.update_mfma = t.update_mfma;
      if (e.factor_path == 0) e.factor_path = t.factor_path;
      if (e.apply_path == 0) e.apply_path = t.apply_path;
      if (e.deterministic == 0) e.deterministic = t.deterministic;
      h->stats.tuning_applied = 1;
    }
  }
  h->doff_h.assign(nb + 1, 0);
  for (int64_t b = 0; b < nb; ++b) {
    int64_t q = bs[b + 1] - bs[b];
    h->doff_h[b + 1] = h->doff_h[b] + q * q;
  }
  hipStream_t st = h->stream;
#define CK(x)                                              \
  do {                                                     \
    hipError_t e_ = (x);                                   \
    if (e_ != hipSuccess) return hip_check(h, e_, #x);     \
  } while (0)
  CK(h->d_bstart.alloc(nb + 1));
  CK(h->d_blockof.alloc(n));
  CK(h->d_roff.alloc(nb));
  CK(h->d_coff.alloc(nb));
  CK(h->d_loff.alloc(nb));
  CK(h->d_woff.alloc(nb));
  CK(h->d_doff.alloc(nb + 1));
  CK(h->d_nr.alloc(nb));
  CK(h->d_nc.alloc(nb));
  CK(h->d_dval.alloc(h->doff_h[nb]));
  CK(h->d_sval.alloc(h->doff_h[nb]));
  CK(h->d_col_cnt.alloc(nb));
  CK(h->d_row_cnt.alloc(nb));
  CK(h->d_col_list.alloc((size_t)nb * kListCap));
  CK(h->d_row_list.alloc((size_t)nb * kListCap));
  CK(h->d_col_ovf.alloc(nb));
  CK(h->d_row_ovf.alloc(nb));
  int64_t ovf_cap = std::max<int64_t>(1 << 16, 2 * nb);
  CK(h->d_status.alloc(8));
  CK(h->d_counters.alloc(4));
  CK(h->d_troff.alloc(nb));
  CK(h->d_tcoff.alloc(nb));
  CK(h->d_ntr.alloc(nb));
  CK(h->d_ntc.alloc(nb));
  CK(h->d_flow.alloc(5 * nb + 8));
  CK(hipMemcpyAsync(h->d_bstart.p, bs.data(), (nb + 1) * sizeof(int32_t), hipMemcpyHostToDevice, st));
  CK(hipMemcpyAsync(h->d_doff.p, h->doff_h.data(), (nb + 1) * sizeof(int64_t), hipMemcpyHostToDevice, st));
  {
    dim3 blk(64, 4);
    fill_block_of<<<dim3((unsigned)((nb + 3) / 4)), blk, 0, st>>>(h->d_bstart.p, (int)nb, h->d_blockof.p);
    const int64_t nnz = h->nnz;
    CK(h->d_bri.alloc(std::max<int64_t>(1, nnz)));
    CK(h->d_bci.alloc(std::max<int64_t>(1, nnz)));
    const unsigned g = (unsigned)std::min<int64_t>(65536, (nnz + 255) / 256 + 1);
    map_blocks<<<g, 256, 0, st>>>(h->d_ri.p, nnz, h->d_blockof.p, h->d_bri.p);
    map_blocks<<<g, 256, 0, st>>>(h->d_ci.p, nnz, h->d_blockof.p, h->d_bci.p);
    CK(hipGetLastError());
  }
  int64_t val_cap = h->opt.heap_bytes ? (int64_t)(h->opt.heap_bytes / sizeof(double))
                                      : std::max<int64_t>(1 << 20, 4 * h->nnz);
  int64_t idx_cap = std::max<int64_t>(1 << 20, 2 * h->nnz);
  // workers: as many workgroups as can be resident at once (more would only
  // start when others end); each owns one scratch slot
  const size_t dyn = maxq <= kLdsPivotWidth ? 2 * sizeof(double) * maxq * maxq : 0;
  int dev = 0, cus = 0, per_cu = 0;
  CK(hipGetDevice(&dev));
  CK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const void* worker = h->opt.update_precision == 1   ? reinterpret_cast<const void*>(factor_worker_kernel<1>)
                      : h->opt.update_precision == 2 ? reinterpret_cast<const void*>(factor_worker_kernel<2>)
                                                     : reinterpret_cast<const void*>(factor_worker_kernel<0>);
  CK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, worker, kThreads, dyn));
  if (h->eff.workers_per_cu > 0) per_cu = std::min(per_cu, h->eff.workers_per_cu);
  const int64_t workers = std::min<int64_t>(nb, std::max<int64_t>(1, (int64_t)cus * std::max(per_cu, 1)));
  const int64_t mq = std::max<int32_t>(maxq, 1);
  const int64_t slot_doubles = std::max<int64_t>(2 * (int64_t)kCandCap * mq + 2 * mq * mq,
                                                  h->eff.factor_path != 1 ? kBigSlotDoubles : 0);
  if ((int64_t)h->d_scratch.n < workers * slot_doubles) CK(h->d_scratch.alloc(workers * slot_doubles));
  h->scratch_slots = workers;
  h->slot_doubles = slot_doubles;
  if (h->wait_ticks == 0) {
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
      h->wait_ticks = (unsigned long long)(kWaitSeconds * 1e3 * khz);
    else
      h->wait_ticks = (unsigned long long)(kWaitSeconds * 1e8);
  }
  auto t2 = clk::now();
  h->stats.t_phase[2] = std::chrono::duration<double>(t2 - t1).count();
  // a heap or overflow pool that proves too small grows, and the sweep runs
  // again from the start
  for (int attempt = 0; attempt < 16; ++attempt) {
    if ((int64_t)h->d_val_heap.n < (val_cap + kHeapSlack) * value_bytes(h->opt.update_precision))
      CK(h->d_val_heap.alloc((val_cap + kHeapSlack) * value_bytes(h->opt.update_precision)));
    CK(h->d_ovf_j.alloc(ovf_cap));
    CK(h->d_ovf_next.alloc(ovf_cap));
    if ((int64_t)h->d_idx_heap.n < idx_cap) CK(h->d_idx_heap.alloc(idx_cap));
    CK(hipMemsetAsync(h->d_col_cnt.p, 0, nb * sizeof(int32_t), st));
    CK(hipMemsetAsync(h->d_row_cnt.p, 0, nb * sizeof(int32_t), st));
    CK(hipMemsetAsync(h->d_col_ovf.p, 0xff, nb * sizeof(int32_t), st));
    CK(hipMemsetAsync(h->d_row_ovf.p, 0xff, nb * sizeof(int32_t), st));
    CK(hipMemsetAsync(h->d_status.p, 0, 8 * sizeof(int), st));
    CK(hipMemsetAsync(h->d_counters.p, 0, 4 * sizeof(unsigned long long), st));
    {
      const double inf = INFINITY;
      unsigned long long init[4] = {0, 0, 0, 0};
      std::memcpy(&init[2], &inf, 8);
      CK(h->d_drop_ctr.alloc(4));
      CK(hipMemcpyAsync(h->d_drop_ctr.p, init, sizeof(init), hipMemcpyHostToDevice, st));
      CK(hipStreamSynchronize(st));  // init is on the host stack
    }
    // pending, started, enqueued, depth = 0; queue = -1; tail, max depth,
    // seeded-block counter, seeded count, claimed positions = 0
    CK(hipMemsetAsync(h->d_flow.p, 0, 4 * nb * sizeof(int), st));
    CK(hipMemsetAsync(h->d_flow.p + 4 * nb, 0xff, nb * sizeof(int), st));
    CK(hipMemsetAsync(h->d_flow.p + 5 * nb, 0, 8 * sizeof(int), st));
    static_pending<<<(unsigned)((n + 15) / 16), 256, 0, st>>>(
        (int)n, h->d_rp.p, h->d_bci.p, h->d_cp.p, h->d_bri.p, h->d_blockof.p, h->d_flow.p);
    {
      DevArray<unsigned char> flag;
      CK(flag.alloc(nb));
      seed_flags<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>((int)nb, h->d_flow.p,
                                                               h->d_flow.p + 2 * nb, flag.p);
      CK(hipGetLastError());
      hipcub::CountingInputIterator<int> ids(0);
      size_t bytes = 0;
      CK(hipcub::DeviceSelect::Flagged(nullptr, bytes, ids, flag.p, h->d_flow.p + 4 * nb,
                                       h->d_flow.p + 5 * nb, (int)nb, st));
      CK(h->d_scan_tmp.alloc(bytes + 1));
      CK(hipcub::DeviceSelect::Flagged(h->d_scan_tmp.p, bytes, ids, flag.p, h->d_flow.p + 4 * nb,
                                       h->d_flow.p + 5 * nb, (int)nb, st));
      CK(hipStreamSynchronize(st));  // the flags end here
    }
    // the seeded count: the tail before any block has run
    CK(hipMemcpyAsync(h->d_flow.p + 5 * nb + 3, h->d_flow.p + 5 * nb, sizeof(int),
                      hipMemcpyDeviceToDevice, st));
    FactorArgs a{};
    a.n = (int)n;
    a.nb = (int)nb;
    a.cp = h->d_cp.p; a.ri = h->d_ri.p; a.cv = h->d_cv.p;
    a.rp = h->d_rp.p; a.ci = h->d_ci.p; a.rv = h->d_rv.p;
    a.bstart = h->d_bstart.p;
    a.blockOf = h->d_blockof.p;
    a.tau = tau;
    a.alpha = h->alpha;
    a.tau_blk = nullptr;
    a.alpha_blk = nullptr;
    a.pflag = nullptr;
    if (tau_blk && alpha_blk) {
      CK(h->d_tau_blk.alloc(nb));
      CK(h->d_alpha_blk.alloc(nb));
      CK(h->d_pflag.alloc(nb));
      CK(hipMemcpyAsync(h->d_tau_blk.p, tau_blk->data(), nb * 8, hipMemcpyHostToDevice, st));
      CK(hipMemcpyAsync(h->d_alpha_blk.p, alpha_blk->data(), nb * 8, hipMemcpyHostToDevice, st));
      CK(hipMemsetAsync(h->d_pflag.p, 0, nb * sizeof(int), st));
      a.tau_blk = h->d_tau_blk.p;
      a.alpha_blk = h->d_alpha_blk.p;
      a.pflag = h->d_pflag.p;
    }
    a.pert_tau = h->opt.perturb_tau;
    a.pert_rho = h->opt.perturb_rho;
    a.sym_pert = h->mwm_sym ? 1 : 0;
    a.pivot_eps = h->opt.pivot_eps;
    a.beta_one = h->opt.beta_one;
    a.drop_norm = h->opt.drop_norm;
    a.update_prec = h->opt.update_precision;
    a.fast_path = h->eff.factor_path == 0 ? 1 : h->eff.factor_path == 2 ? 2 : 0;
    a.mfma = h->eff.update_mfma == 1 ? 1 : 0;
    // the ordered accumulation of the terms is what makes runs bit-identical;
    // matrix-core tiles always use it
    a.det = h->eff.deterministic || a.mfma ? 1 : 0;
    a.lds_pivot = dyn > 0 ? 1 : 0;
    a.roff = h->d_roff.p; a.nr = h->d_nr.p; a.coff = h->d_coff.p; a.nc = h->d_nc.p;
    a.loff = h->d_loff.p; a.woff = h->d_woff.p; a.doff = h->d_doff.p;
    a.dval = h->d_dval.p; a.sval = h->d_sval.p;
    a.idx_heap = h->d_idx_heap.p; a.idx_cap = (int64_t)h->d_idx_heap.n; a.idx_top = h->d_counters.p + 0;
    a.elem_bytes = value_bytes(h->opt.update_precision);
    a.val_heap = h->d_val_heap.p;
    a.val_cap = (int64_t)(h->d_val_heap.n / a.elem_bytes) - kHeapSlack;
    a.val_top = h->d_counters.p + 1;
    // per-worker chunks: at most an eighth of either heap sits unused in them
    a.val_chunk = std::min<int64_t>(8192, a.val_cap / (8 * workers));
    a.idx_chunk = std::min<int64_t>(4096, a.idx_cap / (8 * workers));
    a.col_cnt = h->d_col_cnt.p; a.col_list = h->d_col_list.p; a.col_ovf = h->d_col_ovf.p;
    a.row_cnt = h->d_row_cnt.p; a.row_list = h->d_row_list.p; a.row_ovf = h->d_row_ovf.p;
    a.ovf_j = h->d_ovf_j.p; a.ovf_next = h->d_ovf_next.p; a.ovf_top = h->d_status.p + 3;
    a.ovf_cap = (int32_t)ovf_cap;
    a.scratch = h->d_scratch.p;
    a.slot_doubles = slot_doubles;
    a.sched = nullptr;
    a.begin = 0;
    a.end = (int)nb;
    a.err = h->d_status.p + 0;
    a.err_block = h->d_status.p + 1;
    a.n_perturbed = h->d_status.p + 2;
    a.flops = h->d_counters.p + 2;
    a.drop_ctr = h->d_drop_ctr.p;
    a.log_margin = h->opt.drop_log_margin > 0.0 ? h->opt.drop_log_margin : -1.0;
    a.log_cap = 0;
    a.log_blk = a.log_idx = nullptr;
    a.log_nrm = nullptr;
    if (h->opt.drop_log_margin > 0.0) {
      CK(h->d_log_blk.alloc(kDropLogCap));
      CK(h->d_log_idx.alloc(kDropLogCap));
      CK(h->d_log_nrm.alloc(kDropLogCap));
      a.log_cap = kDropLogCap;
      a.log_blk = h->d_log_blk.p;
      a.log_idx = h->d_log_idx.p;
      a.log_nrm = h->d_log_nrm.p;
    }
    a.upd_bytes = h->d_counters.p + 3;
    a.troff = h->d_troff.p;
    a.ntr = h->d_ntr.p;
    a.tcoff = h->d_tcoff.p;
    a.ntc = h->d_ntc.p;
    a.bri = h->d_bri.p;
    a.bci = h->d_bci.p;
    FlowArgs d{};
    d.pending = h->d_flow.p;
    d.started = h->d_flow.p + nb;
    d.enq = h->d_flow.p + 2 * nb;
    d.depth = h->d_flow.p + 3 * nb;
    d.queue = h->d_flow.p + 4 * nb;
    d.tail = h->d_flow.p + 5 * nb;
    d.max_depth = h->d_flow.p + 5 * nb + 1;
    d.leaf_head = h->d_flow.p + 5 * nb + 2;
    d.nleaves = h->d_flow.p + 5 * nb + 3;
    d.claim = h->d_flow.p + 5 * nb + 4;
    d.wait_ticks = h->wait_ticks;
    d.trace = nullptr;
    if (h->opt.collect_timing >= 2) {
      CK(h->d_trace.alloc((size_t)nb * kTraceFields));
      CK(hipMemsetAsync(h->d_trace.p, 0, (size_t)nb * kTraceFields * 8, st));
      d.trace = h->d_trace.p;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (h->opt.collect_timing) {
      e0 = h->ev_get();
      e1 = h->ev_get();
      if (e0) (void)hipEventRecord(e0, st);
    }
    // an ordinary launch: workers claim queue positions as they run, so
    // none relies on another being resident
    void* kargs[] = {&a, &d};
    CK(hipLaunchKernel(worker, dim3((unsigned)workers), dim3(kThreads), kargs, dyn, st));
    if (h->opt.collect_timing) {
      if (e1) (void)hipEventRecord(e1, st);
      h->ev_record(0, e0, e1);
    }
    h->stats.n_factor_launches = 1;
    CK(hipGetLastError());
    int status[8];
    unsigned long long ctr[4];
    CK(hipMemcpyAsync(status, h->d_status.p, sizeof(status), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(ctr, h->d_counters.p, sizeof(ctr), hipMemcpyDeviceToHost, st));
    int max_depth = 0;
    CK(hipMemcpyAsync(&max_depth, h->d_flow.p + 5 * nb + 1, sizeof(int), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (status[0] == kDevHeapOverflow) {
      val_cap = std::max<int64_t>(val_cap * 4, (int64_t)ctr[1] * 2);
      idx_cap = std::max<int64_t>(idx_cap * 4, (int64_t)ctr[0] * 2);
      ++h->stats.heap_regrows;
      continue;
    }
    if (status[0] == kDevListOverflow && ovf_cap < INT32_MAX / 4) {
      ovf_cap *= 4;
      continue;
    }
    if (status[0] != kDevOk) {
      static const char* what[] = {"ok", "candidate set exceeds the per-block capacity",
                                   "predecessor list exceeds the per-block capacity",
                                   "factor heap exhausted", "predecessor overflow pool exhausted",
                                   "pivot block singular after perturbation",
                                   "block wider than the kernel limit", "dependency wait timed out",
                                   "dependency protocol violated", "no free scratch slot",
                                   "announcement set exceeds the per-block capacity"};
      // kDevSpin reports the queue position that was never filled
      std::string msg = std::string("factor kernel: ") + what[std::min(status[0], 10)] +
                        " (block " + std::to_string(status[1]) + ")";
      return fail(h, status[0] == kDevSingular ? BILU_ERR_SINGULAR
                     : (status[0] == kDevSpin || status[0] == kDevProtocol || status[0] == kDevSlot)
                         ? BILU_ERR_DEVICE
                         : BILU_ERR_NO_MEMORY,
                  msg);
    }
    h->stats.perturbed_blocks = status[2];
    {
      unsigned long long dc[4];
      CK(hipMemcpy(dc, h->d_drop_ctr.p, sizeof(dc), hipMemcpyDeviceToHost));
      double mg;
      std::memcpy(&mg, &dc[2], 8);
      h->stats.drops_rows = (int64_t)dc[0];
      h->stats.drops_cols = (int64_t)dc[1];
      h->stats.drop_margin_min = std::isfinite(mg) ? mg : -1.0;
      h->drop_log_n = a.log_cap > 0 ? std::min<int64_t>((int64_t)dc[3], a.log_cap) : 0;
      h->stats.drop_log_count = (int64_t)dc[3];
    }
    h->stats.flops_update = (double)ctr[2];
    h->stats.bytes_factor = (double)ctr[3];  // completed with A and output bytes by the caller
    h->stats.factor_levels = max_depth;
    auto t3 = clk::now();
    h->stats.t_factor_device = std::chrono::duration<double>(t3 - t2).count();
    h->stats.t_phase[3] = h->stats.t_factor_device;
    h->stats.nblocks_initial = nb;
    h->idx_used = (int64_t)ctr[0];
    h->val_used = (int64_t)ctr[1];
    return BILU_OK;
  }
  return fail(h, BILU_ERR_NO_MEMORY, "factor heap could not be sized");
#undef CK
}


// Refactorization with frozen patterns (see frozen_block_kernel): the values
// of A were replaced (refactor_values); the last factor's blocks, lists and
// storage stay, its values are recomputed.
bilu_status frozen_refactor(bilu_handle* h) {
#define CK(x)                                          \
  do {                                                 \
    hipError_t e_ = (x);                               \
    if (e_ != hipSuccess) return hip_check(h, e_, #x); \
  } while (0)
  hipStream_t st = h->stream;
  const FactorView& f = h->fv;
  const int nb = f.nb;
  const unsigned long long wait = h->wait_ticks ? h->wait_ticks : (unsigned long long)1e9;
  FrozenPlan& fp = h->frozen;
  if (!fp.ready) {
    // the schedule depends on the factor's structure only: built once per
    // factorization.  The blocks whose columns run inside each block (its
    // rows: the apply plan's forward lists of the same factor)
    const bilu_status rs = block_runs(h, f, true, fp.cptr, fp.cj, fp.cs0, fp.ccnt);
    if (rs != BILU_OK) return rs;
    // levels, the blocks ordered by (level, index)
    DevArray<int> lev, misc;
    DevArray<unsigned long long> ext;
    CK(lev.alloc(std::max(1, nb)));
    CK(misc.alloc(4));
    CK(ext.alloc(3));
    CK(hipMemsetAsync(lev.p, 0xff, nb * sizeof(int), st));
    CK(hipMemsetAsync(misc.p, 0, 4 * sizeof(int), st));
    CK(hipMemsetAsync(ext.p, 0, 3 * sizeof(unsigned long long), st));
    frozen_levels<<<(unsigned)((nb + 3) / 4), 256, 0, st>>>(nb, fp.cptr.p, fp.cj.p, h->fw_ptr.p,
                                                            h->fw_j.p, lev.p, misc.p + 2, wait);
    frozen_extent<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(f, ext.p);
    CK(hipGetLastError());
    size_t rb = 0;
    CK(hipcub::DeviceReduce::Max(nullptr, rb, lev.p, misc.p, nb, st));
    CK(h->d_scan_tmp.alloc(rb + 1));
    CK(hipcub::DeviceReduce::Max(h->d_scan_tmp.p, rb, lev.p, misc.p, nb, st));
    int hm[4];
    CK(hipMemcpyAsync(hm, misc.p, sizeof(hm), hipMemcpyDeviceToHost, st));
    CK(hipMemcpyAsync(fp.ext, ext.p, sizeof(fp.ext), hipMemcpyDeviceToHost, st));
    CK(hipStreamSynchronize(st));
    if (hm[2]) return fail(h, BILU_ERR_DEVICE, "refactor: a dependency wait timed out");
    const int maxlev = hm[0];
    DevArray<int32_t> idx, keys_out;
    CK(idx.alloc(nb));
    CK(fp.sched.alloc(nb));
    CK(keys_out.alloc(nb));
    frozen_iota<<<(unsigned)((nb + 255) / 256), 256, 0, st>>>(nb, idx.p);
    int bits = 1;
    while ((1 << bits) <= maxlev) ++bits;
    size_t bytes = 0;
    CK(hipcub::DeviceRadixSort::SortPairs(nullptr, bytes, lev.p, keys_out.p, idx.p, fp.sched.p, nb,
                                          0, bits, st));
    CK(h->d_scan_tmp.alloc(bytes + 1));
    CK(hipcub::DeviceRadixSort::SortPairs(h->d_scan_tmp.p, bytes, lev.p, keys_out.p, idx.p,
                                          fp.sched.p, nb, 0, bits, st));
    // FP64 panels (for blocks whose panels do not fit the LDS) and pivot
    // scratch, kept with the schedule
    CK(fp.pv.alloc(std::max<unsigned long long>(1, fp.ext[0])));
    CK(fp.pd.alloc(std::max<unsigned long long>(1, fp.ext[1])));
    if ((int)fp.ext[2] > kLdsPivotWidth) CK(fp.piv.alloc(2 * std::max<unsigned long long>(1, fp.ext[1])));
    CK(fp.done.alloc(std::max(1, nb)));
    CK(hipStreamSynchronize(st));
    fp.ready = true;
  }
  CK(hipMemsetAsync(fp.done.p, 0, nb * sizeof(int), st));
  const int maxq = (int)fp.ext[2];
  const bool lds_pivot = maxq <= kLdsPivotWidth;
  const size_t dyn = lds_pivot ? 2 * sizeof(double) * maxq * maxq : 0;
  CK(hipMemsetAsync(h->d_status.p, 0, 3 * sizeof(int), st));
  FrozenArgs a{};
  a.f = f;
  a.val = const_cast<void*>(f.val);
  a.dval = const_cast<double*>(f.dval);
  // S_K too when the factor is the sweep's own (no merges), so the
  // kept-pattern residual stays defined
  a.sval = f.dval == h->d_dval.p ? h->d_sval.p : nullptr;
  a.PL = fp.pv.p;
  a.PW = fp.pv.p;
  a.PD = fp.pd.p;
  a.piv = lds_pivot ? nullptr : fp.piv.p;
  a.cp = h->d_cp.p; a.ri = h->d_ri.p; a.cv = h->d_cv.p;
  a.rp = h->d_rp.p; a.ci = h->d_ci.p; a.rv = h->d_rv.p;
  a.cptr = fp.cptr.p; a.cj = fp.cj.p; a.cs0 = fp.cs0.p; a.ccnt = fp.ccnt.p;
  a.rptr = h->fw_ptr.p; a.rj = h->fw_j.p; a.rs0 = h->fw_r0.p; a.rcnt = h->fw_cnt.p;
  a.sched = fp.sched.p;
  a.nb = nb;
  a.done = fp.done.p;
  a.wait = wait;
  a.fa.alpha = h->alpha;
  a.fa.pert_tau = h->opt.perturb_tau;
  a.fa.pert_rho = h->opt.perturb_rho;
  a.fa.sym_pert = h->mwm_sym ? 1 : 0;
  a.fa.pivot_eps = h->opt.pivot_eps;
  a.fa.beta_one = h->opt.beta_one;
  a.fa.pflag = nullptr;
  a.fa.err = h->d_status.p + 0;
  a.fa.err_block = h->d_status.p + 1;
  a.fa.n_perturbed = h->d_status.p + 2;
  // one launch: workgroup w takes the w-th block by (level, index), so
  // every block it waits on sits at a lower workgroup, which the hardware
  // has started before it; no workgroup needs another to be resident
  if (nb > 0) frozen_block_kernel<<<(unsigned)nb, kThreads, dyn, st>>>(a);
  CK(hipGetLastError());
  int status[3];
  CK(hipMemcpyAsync(status, h->d_status.p, sizeof(status), hipMemcpyDeviceToHost, st));
  CK(hipStreamSynchronize(st));
  h->stats.perturbed_blocks = status[2];
  if (status[0] == kDevSingular)
    return fail(h, BILU_ERR_SINGULAR, "refactor: a pivot block stayed singular (block " +
                                          std::to_string(status[1]) + ")");
  if (status[0] != 0) return fail(h, BILU_ERR_DEVICE, "refactor: device error " + std::to_string(status[0]));
  return BILU_OK;
#undef CK
}

}  // namespace bilu
