// Internal declarations of the BILU library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <chrono>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/bilu.h"
#include "values.h"

namespace bilu {

// Capacities of the per-block work of the factor kernel.
constexpr int kThreads = 256;      // threads per workgroup (4 wave64)
constexpr int kHashSlots = 4096;   // LDS hash of candidate rows/columns
constexpr int kCandCap = 2048;     // unique candidate rows (or columns) per block
constexpr int kPredCap = 1024;     // predecessors per block panel
constexpr int kListCap = 64;       // inline capacity of a block's predecessor list
constexpr int kMaxWidth = 128;     // widest pivot block
constexpr int kLdsPivotWidth = 64; // pivot blocks up to this width live in LDS

// Error codes written by kernels into the device status word.
enum DevErr : int {
  kDevOk = 0,
  kDevCandOverflow = 1,
  kDevPredOverflow = 2,
  kDevHeapOverflow = 3,
  kDevListOverflow = 4,
  kDevSingular = 5,
  kDevWidth = 6,
  kDevSpin = 7,
  kDevProtocol = 8,
  kDevSlot = 9,
  kDevAnnOverflow = 10,
};

// Device array owned by a handle.  alloc() keeps the existing allocation
// when it is large enough (refactoring does not free and reallocate).
// Pinned host memory that only grows (hipHostMalloc); used for staging
// copies between host and device without a pageable bounce.
struct PinnedBuf {
  void* p = nullptr;
  size_t bytes = 0;
  PinnedBuf() = default;
  PinnedBuf(const PinnedBuf&) = delete;
  PinnedBuf& operator=(const PinnedBuf&) = delete;
  ~PinnedBuf() {
    if (p) (void)hipHostFree(p);
  }
  template <class T>
  T* get(size_t count, hipError_t* err) {
    const size_t b = count * sizeof(T);
    if (b > bytes) {
      if (p) (void)hipHostFree(p);
      p = nullptr;
      bytes = 0;
      *err = hipHostMalloc(&p, b, hipHostMallocDefault);
      if (*err != hipSuccess) {
        p = nullptr;
        return nullptr;
      }
      bytes = b;
    }
    *err = hipSuccess;
    return static_cast<T*>(p);
  }
};

template <class T>
struct DevArray {
  T* p = nullptr;
  size_t n = 0;    // elements in use
  size_t cap = 0;  // elements allocated
  ~DevArray() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = cap = 0;
  }
  hipError_t alloc(size_t count) {
    if (count <= cap && p) {
      n = count;
      return hipSuccess;
    }
    release();
    if (count == 0) return hipSuccess;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), count * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    n = cap = count;
    return hipSuccess;
  }
};

// Everything the factor kernels read and write, passed by value.
struct FactorArgs {
  int n, nb;
  const int64_t* cp;      // CSC of the permuted matrix
  const int32_t* ri;
  const double* cv;
  const int64_t* rp;      // CSR of the permuted matrix
  const int32_t* ci;
  const double* rv;
  const int32_t* bstart;  // [nb+1]
  const int32_t* blockOf; // [n]
  double tau, alpha, pert_tau, pert_rho, pivot_eps;
  const double* tau_blk;           // per-block tau and alpha (batched factorization) or null
  const double* alpha_blk;
  int* pflag;                      // per-block perturbed flag or null
  int beta_one, drop_norm, update_prec;
  int sym_pert;                    // Sec. 5: symmetrized perturbation (symmetric matching)
  int fast_path;                   // 1: LDS staging where it fits, 2: global staging, 0: general only
  int mfma;                        // fast path: update terms as matrix-core tiles
  int det;                         // fast path: terms subtracted in predecessor order
  int lds_pivot;                   // dynamic LDS holds 2 q^2 doubles for every block
  // factor storage, per block
  int64_t* roff;  int32_t* nr;     // rows of L  : idx heap
  int64_t* coff;  int32_t* nc;     // cols of U  : idx heap
  int64_t* loff;  int64_t* woff;   // values     : val heap
  const int64_t* doff;             // D / S      : prefix of q^2
  double* dval;
  double* sval;
  int32_t* idx_heap; int64_t idx_cap; unsigned long long* idx_top;
  void* val_heap;  int64_t val_cap; unsigned long long* val_top;  // L, W in update_prec
  int64_t idx_chunk, val_chunk;    // entries a worker takes from a heap top at once
  int elem_bytes;                  // bytes of one stored L / W value (8, 4 or 2)
  // predecessor lists: inline + overflow linked list
  int32_t* col_cnt; int32_t* col_list; int32_t* col_ovf;
  int32_t* row_cnt; int32_t* row_list; int32_t* row_ovf;
  int32_t* ovf_j; int32_t* ovf_next; int32_t* ovf_top; int32_t ovf_cap;
  // per-workgroup scratch (panels)
  double* scratch; int64_t slot_doubles;
  // schedule
  const int32_t* sched; int begin, end;
  // status / counters
  int* err; int* err_block; int* n_perturbed;
  unsigned long long* flops;
  unsigned long long* upd_bytes;  // bytes of L_J rows + W_J columns read by updates
  // drop decisions: [0] rows dropped, [1] columns dropped, [2] smallest
  // |norm - tau| / tau (double bits), [3] decisions logged (may exceed log_cap)
  unsigned long long* drop_ctr;
  double log_margin;               // log decisions with |norm - tau| <= log_margin * tau
  int log_cap;
  int32_t* log_blk; int32_t* log_idx; double* log_nrm;  // idx: row i, or ~j for column j
  // block-level patterns: distinct blocks of R_K (tr) and of C_K (tc) in the
  // idx heap, and the static distinct blocks > K of A's pattern of K
  int64_t* troff; int32_t* ntr;
  int64_t* tcoff; int32_t* ntc;
  // block of the row (column) of every CSC (CSR) entry of A
  const int32_t* bri; const int32_t* bci;
};

constexpr int kAnnCap = 2048;      // distinct blocks one block may still update

// Dependency bookkeeping of the factor kernel.
struct FlowArgs {
  int* pending;            // unfinished possible updaters (with multiplicity)
  int* depth;              // longest chain of possible updaters ending at the block
  int* max_depth;
  int* started;            // numeric phase begun (checks the protocol)
  int* enq;                // block pushed to the ready queue
  int* queue;              // ready queue, filled in readiness order (-1 = empty)
  int* tail;               // next free queue position
  int* leaf_head;          // next of the seeded positions [0, *nleaves) to take
  const int* nleaves;      // blocks seeded before the launch
  int* claim;              // positions past the seeded ones claimed so far
  unsigned long long wait_ticks;
  // optional per-block trace (kTraceFields per block, wall-clock ticks):
  // pushed, popped, updater set built, candidates built, done, the block
  // whose retraction made it ready, the count it retracted, worker; then
  // the end of the column panel, row panel, pivot, drop norms, heap
  // allocation, factor writes, list pushes, successor counts; then the
  // numbers of column and row predecessors, candidate rows and columns
  unsigned long long* trace;
};

constexpr int kTraceFields = 24;

// Bound of one dependency wait in seconds: a wait that exceeds it reports
// an error instead of hanging.
constexpr double kWaitSeconds = 10.0;

// Device view of a block factor (initial or aggregated), used by the apply
// and by export.  Per block K: rows R_K (nr, at idx+roff), columns C_K
// (nc, at idx+coff), L_K (nr x q row-major at val+loff), W_K (q x nc
// column-major at val+woff), both in precision vprec (values.h), D_K (q x q
// row-major at dval+doff, FP64).
struct FactorView {
  int nb = 0;
  const int32_t* bstart = nullptr;
  const int32_t* blockOf = nullptr;
  const int32_t* nr = nullptr;
  const int32_t* nc = nullptr;
  const int64_t* roff = nullptr;
  const int64_t* coff = nullptr;
  const int64_t* loff = nullptr;
  const int64_t* woff = nullptr;
  const int64_t* doff = nullptr;
  const int32_t* idx = nullptr;
  const void* val = nullptr;
  int vprec = 0;
  const double* dval = nullptr;
};


// The frozen refactorization's schedule: per block the runs of the blocks
// whose columns fall inside it, the blocks by dependency level, the largest
// value and pivot offsets and width (ext), FP64 scratch and done flags.  It
// depends on the factor's structure only.
struct FrozenPlan {
  bool ready = false;
  DevArray<int32_t> cptr, cj, cs0, ccnt, sched;
  DevArray<int> done;
  DevArray<double> pv, pd, piv;
  unsigned long long ext[3] = {0, 0, 0};
};

// tuning.cpp: tuned settings for one update precision and block-width
// class (0: the widest initial block is at most 16, 1: wider), for handles
// that require reproducible results (reproducible = 1) or not
struct TunedEntry {
  int precision = 0, width_class = 0, reproducible = 1;
  int workers_per_cu = 0;  // 0: as many as fit
  int update_mfma = 0, factor_path = 0, apply_path = 0, deterministic = 1;
};
bool tuned_entry(int precision, int width_class, int reproducible, TunedEntry* out);

}  // namespace bilu

struct bilu_handle {
  bilu_options opt{};
  hipStream_t stream = nullptr;
  std::string err;
  int state = 0;  // 0 created, 1 analyzed, 2 factored
  int64_t n = 0, nnz = 0;
  double alpha = 0.0;

  // ---- analyze (host)
  std::vector<int64_t> perm;          // new -> old
  std::vector<int64_t> group_starts;  // cosine groups, permuted numbering
  std::vector<int64_t> prp;           // permuted CSR
  std::vector<int32_t> pci;
  std::vector<double> pv;
  std::vector<int64_t> pcp;           // permuted CSC
  std::vector<int32_t> pri;
  std::vector<double> pcv;
  // ---- analyze (device)
  bilu::DevArray<int64_t> d_rp, d_cp;
  bilu::DevArray<int32_t> d_ci, d_ri, d_perm;
  bilu::DevArray<double> d_rv, d_cv;
  // entry of A held by each position of the CSR / CSC (bilu_refactor)
  bilu::DevArray<int32_t> d_vmap_r, d_vmap_c;

  // ---- factor: partition + schedule (host)
  std::vector<int32_t> bstart0;       // initial partition
  bilu::DevArray<int64_t> d_troff, d_tcoff;
  bilu::DevArray<unsigned long long> d_trace;  // collect_timing == 2
  // ILU(1,tau) on the device: unit starts, diagonal, padded sets, counts
  bilu::DevArray<int64_t> d_ilu_gs;
  bilu::DevArray<double> d_ilu_dg;
  bilu::DevArray<int32_t> d_ilu_set, d_ilu_cnt;
  bilu::DevArray<int32_t> d_ntr, d_ntc, d_bri, d_bci;
  bilu::DevArray<int> d_flow;        // pending, started, enqueued, depth, queue, tail, max depth
  unsigned long long wait_ticks = 0; // bound of one dependency wait (wall-clock ticks)
  std::vector<int64_t> doff_h;
  // ---- factor storage (device)
  bilu::DevArray<int32_t> d_bstart, d_blockof;
  bilu::DevArray<int64_t> d_roff, d_coff, d_loff, d_woff, d_doff;
  bilu::DevArray<int32_t> d_nr, d_nc;
  bilu::DevArray<double> d_dval, d_sval;
  bilu::DevArray<int32_t> d_idx_heap;
  bilu::DevArray<unsigned char> d_val_heap;  // L, W values in the update precision (bytes)
  bilu::DevArray<int32_t> d_col_cnt, d_col_list, d_col_ovf, d_row_cnt, d_row_list, d_row_ovf;
  bilu::DevArray<int32_t> d_ovf_j, d_ovf_next;
  bilu::DevArray<double> d_scratch;
  bilu::DevArray<int> d_status;                  // err, err_block, n_perturbed, ovf_top
  bilu::DevArray<unsigned long long> d_counters; // idx_top, val_top, flops
  bilu::DevArray<unsigned long long> d_drop_ctr; // drops, margin, log count
  bilu::DevArray<int32_t> d_log_blk, d_log_idx;  // near-tie drop decisions
  bilu::DevArray<double> d_log_nrm;
  int64_t drop_log_n = 0;                        // records in the log
  int64_t scratch_slots = 0, slot_doubles = 0;
  int64_t idx_used = 0, val_used = 0;  // heap entries the last sweep allocated

  // ---- final factor (after aggregation), used by apply
  int64_t nb = 0;                    // final block count
  std::vector<int32_t> bstart;       // final partition (host)
  bilu::DevArray<int32_t> f_bstart, f_blockof, f_nr, f_nc;
  bilu::DevArray<int64_t> f_roff, f_coff, f_loff, f_woff, f_doff;
  bilu::DevArray<int32_t> f_idx;     // idx heap of the final factor
  bilu::DevArray<unsigned char> f_val;  // merged L, W values (bytes, update precision)
  bilu::DevArray<double> f_dval;
  bool final_is_initial = true;      // no merge happened: f_* alias the factor storage
  int64_t f_val_len = 0;             // values of the final factor's value array in use
  bool ilu_static = false;
  // Sec. 3.1 (use_mwm): the factored matrix is D_l A D_r Pi.  Vectors cross
  // the boundary by row (perm, sl / sl_inv) or by column (perm_col = sigma o
  // perm, sr / sr_inv); without it perm_col = perm and no scaling.
  bool mwm = false;
  // use_mwm = 2 (Sec. 5): symmetric scaling D on both sides, no column
  // permutation; sym_order (new -> old) lists the 1x1 and 2x2 pivot units
  // that the cosine groups keep whole, sym_ustart their boundaries
  bool mwm_sym = false;
  std::vector<int64_t> sym_order, sym_ustart;
  // the other scalar of each 2x2 pivot in the final numbering (-1: a 1x1
  // pivot; empty without the symmetric matching), for ILU(1,tau)
  std::vector<int32_t> sym_partner;
  bilu::DevArray<int32_t> d_partner;
  bilu::DevArray<int32_t> d_perm_col;
  bilu::DevArray<double> d_sl, d_sl_inv, d_sr, d_sr_inv;
  const int32_t* perm_col() const { return mwm ? d_perm_col.p : d_perm.p; }
  const double* sl() const { return mwm ? d_sl.p : nullptr; }
  const double* sl_inv() const { return mwm ? d_sl_inv.p : nullptr; }
  const double* sr() const { return mwm ? d_sr.p : nullptr; }
  const double* sr_inv() const { return mwm ? d_sr_inv.p : nullptr; }
  bilu::PinnedBuf pin_dec, pin_up;     // aggregation: decisions down, group data up
  std::vector<int32_t> agg_gfirst, agg_fbs;
  std::vector<int64_t> agg_off;        // final offsets (copying path) and D offsets           // unit starts and diagonal of the analyzed matrix on the device
  bilu::DevArray<double> d_agg_scratch;  // merge workspace (4 w^2 doubles per slot)
  bilu::DevArray<double> d_tau_blk, d_alpha_blk;  // batched factorization only
  bilu::DevArray<int> d_pflag;
  bilu::FactorView fv;               // the factor the apply uses
  // apply plan: predecessor blocks of the forward sweep (sorted, with the
  // range of their rows inside the block), successor blocks of the backward
  // sweep, and a row-major copy of L
  bilu::DevArray<int32_t> fw_ptr, fw_j, fw_r0, fw_cnt, bw_ptr, bw_b;
  bilu::DevArray<int64_t> lr_ptr;
  bilu::DevArray<int32_t> lr_col;
  bilu::DevArray<unsigned char> lr_val;          // row-major L in the apply precision (bytes)
  int apply_prec = 0;                            // precision of the values the apply reads
  bilu::DevArray<unsigned char> d_apply_val;     // FP32 copy of L, W when apply_prec differs
  bilu::DevArray<int32_t> lev_f, lev_b;          // blocks by forward / backward level
  bilu::DevArray<int2> lev_f_fq;                 // first row and width of lev_f's blocks
  bilu::DevArray<int> d_apply_err;              // dataflow apply: wait words, ticket, fault count
  bilu::DevArray<unsigned char> d_scan_tmp;      // device-scan workspace
  std::vector<int32_t> lev_f_ptr, lev_b_ptr;

  // ---- solver workspace
  bilu::DevArray<double> w_vec;      // scratch vectors
  bilu::DevArray<double> w_red;      // reduction partials
  int64_t w_cols = 0;
  bilu::DevArray<double> w_gm;       // FGMRES state on the device (GmState)
  bilu::DevArray<int> w_flags;       // its flags
  bilu::PinnedBuf w_hflags;          // host copies of the flags, one per step parity
  // set by the solver while it runs steps ahead: the apply, the product and
  // the vector kernels do no work once the int it points to is nonzero
  const int* run_skip = nullptr;
  // the kept-pattern residual no longer describes the factor (a frozen
  // refactorization of a factor with merged blocks)
  bool kept_stale = false;
  // the frozen refactorization's schedule and scratch (factor.hip), kept
  // from one call to the next until the factor changes
  bilu::FrozenPlan frozen;

  // settings in effect for the last factorization: the options, or a tuned
  // entry for its precision and block-width class (use_tuning)
  bilu::TunedEntry eff{};
  bilu_stats stats{};

  // event timing (collect_timing): pending event pairs, resolved by stats
  struct EventPair {
    hipEvent_t a, b;
    int kind;  // 0 factor, 1 apply, 2 spmv
  };
  std::vector<EventPair> ev_pending;
  std::vector<hipEvent_t> ev_pool;
  hipEvent_t ev_get();
  void ev_record(int kind, hipEvent_t a, hipEvent_t b) { ev_pending.push_back({a, b, kind}); }
  void ev_resolve();
  ~bilu_handle();
};

namespace bilu {


// error helpers
bilu_status fail(bilu_handle* h, bilu_status s, const std::string& msg);
bilu_status hip_check(bilu_handle* h, hipError_t e, const char* what);

// analyze.cpp
bilu_status analyze_host(bilu_handle* h, int64_t n, const int64_t* rowptr,
                         const int32_t* colind, const double* val);
int64_t ilu1t_partition(const bilu_handle* h, double tau, std::vector<int32_t>& bstart,
                        double* t_sets = nullptr);
void cosine_limits(int64_t n, int64_t nnz, const int64_t* rc, const int64_t* cc, double* lim_r,
                   double* lim_c);
bool pre_permutation(const bilu_handle* h, int64_t n, std::vector<int64_t>& pre);
// mlnd.cpp: multilevel nested dissection of a graph (CSR without self loops,
// symmetric) with vertex weights vw; order[i] is the vertex at position i
void mlnd_order(const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
                const std::vector<int32_t>& vw, std::vector<int32_t>& order);
bilu_status order_and_expand(bilu_handle* h, const int64_t* rp1, const int32_t* ci1,
                             const std::vector<int64_t>& pre, const std::vector<int64_t>& q,
                             const std::vector<int64_t>& gs);

// analyze_dev.hip
bilu_status analyze_device(bilu_handle* h, int64_t n, const int64_t* d_rowptr,
                           const int32_t* d_colind, const double* d_val, const int64_t* rowptr);
bilu_status ensure_host_matrix(bilu_handle* h);
bilu_status value_maps(bilu_handle* h, const int64_t* d_a_rp, const int32_t* d_a_ci,
                       bool write_idx);
bilu_status refactor_values(bilu_handle* h, const double* d_val);

// ilu1t.hip
int64_t ilu1t_partition_device(bilu_handle* h, double tau, std::vector<int32_t>& bstart,
                               double* t_sets);

// factor.hip
bilu_status factor_device(bilu_handle* h, double tau);
int64_t factor_partition(bilu_handle* h, double tau);   // a3 into h->bstart0
bilu_status factor_sweep(bilu_handle* h, double tau, const std::vector<double>* tau_blk,
                         const std::vector<double>* alpha_blk);

// batch.hip
bilu_status factor_batched(bilu_handle** hs, int count, const double* taus);

// api.cpp
bilu_status finish_factor(bilu_handle* h, std::chrono::steady_clock::time_point t0);

// aggregate.hip
bilu_status aggregate_device(bilu_handle* h);

// solve.hip
bilu_status build_apply_plan(bilu_handle* h);
// For every block K of f, the blocks J whose stored rows (cols: columns)
// fall into K, ascending, with the first position of the run in R_J (C_J)
// and its length (ptr [nb+1]; j, s0, cnt per entry).  Synchronous.
// factor.hip: the last factor's values recomputed on its frozen patterns
bilu_status frozen_refactor(bilu_handle* h);
// solve.hip: the apply's copies of the factor values (row-major L, FP32
// copy) made again from the factor, its patterns unchanged
bilu_status refresh_apply_values(bilu_handle* h);
bilu_status block_runs(bilu_handle* h, const FactorView& f, bool cols, DevArray<int32_t>& ptr,
                       DevArray<int32_t>& j, DevArray<int32_t>& s0, DevArray<int32_t>& cnt);
// kept.hip: ||(L S U - A)_Omega||_F / ||A||_F of the sweep's factor (before
// aggregation), Omega its stored positions; FP64.  Synchronous.
bilu_status kept_residual(bilu_handle* h, double* out);
// Sec. 3.1 maximum weight matching on the host (mwm.cpp); *why explains a
// failure.
bilu_status mwm_host(int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                     int64_t* sigma, double* dl, double* dr, std::string* why);
// Sec. 5 symmetric matching (mwm.cpp): the symmetrized scaling d, the 1x1
// and 2x2 pivot units in the order their first index is met along pre
// (NULL: identity), order new -> old, unit boundaries ustart.
bilu_status sym_matching_host(int64_t n, const int64_t* rp, const int32_t* ci,
                              const double* val, const int64_t* pre, std::vector<double>& d,
                              std::vector<int64_t>& order, std::vector<int64_t>& ustart,
                              std::string* why);
// timed: record HIP events around it when collect_timing is on (events may
// be created, so allocation-free callers pass false)
bilu_status apply_permuted(bilu_handle* h, const double* x, double* y, double* t,
                           bool timed = true);
// Dataflow applies whose waits timed out since the last call (synchronizes
// the handle's stream; BILU_ERR_DEVICE when *count > 0).
bilu_status apply_faults(bilu_handle* h, int64_t* count);
bilu_status spmv_permuted(bilu_handle* h, const double* x, double* y);
// y[i] = x[perm[i]] (times scale[i] when given); scatter: y[perm[i]] = x[i]
// (times scale[i])
void launch_gather(hipStream_t s, int64_t n, const int32_t* perm, const double* scale, const double* x,
                   double* y);
void launch_scatter(hipStream_t s, int64_t n, const int32_t* perm, const double* scale,
                    const double* x, double* y);
void launch_mul(hipStream_t s, int64_t n, const double* w, const double* x, double* y);  // y = w .* x
// skip: when set and nonzero at run time (a converged solver step), the
// kernels do no work
void launch_axpy(hipStream_t s, int64_t n, const double* alpha_dev, double sign, const double* x,
                 double* y, const int* skip = nullptr);
void launch_axpy_host(hipStream_t s, int64_t n, double alpha, const double* x, double* y);
void launch_scale(hipStream_t s, int64_t n, double alpha, const double* x, double* y);
void launch_scale_dev(hipStream_t s, int64_t n, const double* alpha_dev, const double* x, double* y,
                      const int* skip = nullptr);
void launch_dot(hipStream_t s, int64_t n, const double* x, const double* y, double* partial,
                double* out, const int* skip = nullptr);
// FGMRES state on the device (solve.hip): H is (m+1) x m row-major, hcol the
// dot products of the current step (m + 3 values)
struct GmState {
  double* H;
  double* cs;
  double* sn;
  double* g;
  double* y;
  const double* hcol;
  double* inv_hn;
  int* flags;
};
void launch_gm_init(hipStream_t s, const GmState& g, int m, double beta);
void launch_gm_update(hipStream_t s, const GmState& g, int j, int m, double target_inner,
                      int64_t it_before, int64_t maxit);
void launch_gm_solve(hipStream_t s, const GmState& g, int m);
void launch_sub(hipStream_t s, int64_t n, const double* b, const double* ax, double* r);

// SQMR state on the device (solve.hip): scalar slots of s, the partial
// maxima (2 * kSqParts) and the flags: [0] the solve stopped (the solver's
// kernels skip their work), [1] why (1 the updated backward error met the
// tolerance, 2 breakdown, 3 maxit), [2] steps taken.
enum SqSlot {
  kSqRho = 0,   // r^T M^{-1} r of the previous step
  kSqRhoNew,    // of this step
  kSqTau,       // quasi-residual norm
  kSqTheta,
  kSqSigma,     // q^T A q
  kSqRR,        // r^T r
  kSqAlpha,
  kSqCd,        // c^2 theta_old^2
  kSqCq,        // c^2 alpha
  kSqRmax,      // ||rq||_inf
  kSqXmax,      // ||x||_inf
  kSqAnorm,     // ||A||_inf
  kSqBmax,      // ||b||_inf
  kSqEta,       // backward error of the updated residual
  kSqSlots = 16
};
constexpr int kSqParts = 512;
struct SqState {
  double* s;
  double* part;
  int* flags;
};
void launch_sq_init(hipStream_t s, const SqState& g);
void launch_sq_resume(hipStream_t s, const SqState& g);
void launch_sq_alpha(hipStream_t s, const SqState& g);
void launch_sq_theta(hipStream_t s, const SqState& g);
// d = cd d + cq q, sv = cd sv + cq t, x += d, rq -= sv, then the maxima of
// |x .* xs| and |rq .* rs| (scales NULL: 1), the backward error and the
// stop test
void launch_sq_update(hipStream_t s, int64_t n, const SqState& g, const double* q, const double* t,
                      double* d, double* sv, double* x, double* rq, const double* xs,
                      const double* rs, double tol, int64_t maxit);
// q = u + (rho_new / rho) q
void launch_sq_direction(hipStream_t s, int64_t n, const SqState& g, const double* u, double* q);
// *out = max_i |x_i w_i| (w NULL: 1); *out = max_i rs_i sum_k |v_k| cs_{ci_k}
// over the rows of a CSR matrix (scales NULL: 1)
void launch_amax(hipStream_t s, int64_t n, const double* x, const double* w, double* partial,
                 double* out);
void launch_row_amax(hipStream_t s, int64_t n, const int64_t* rp, const int32_t* ci,
                     const double* v, const double* rs, const double* cs, double* partial,
                     double* out);

// fgmres.cpp
bilu_status fgmres(bilu_handle* h, const double* b, double* x, int restart, double rtol,
                   int maxit, bilu_solve_info* info);
// sqmr.cpp
bilu_status sqmr(bilu_handle* h, const double* b, double* x, double tol, int maxit,
                 bilu_solve_info* info, double* eta);

}  // namespace bilu
