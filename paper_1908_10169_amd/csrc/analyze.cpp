// Host-side structural preprocessing of the BILU library:
//   - CSR validation,
//   - cosine-based grouping of rows with similar patterns (Sec. 3.2),
//   - compression to the group graph, ordering, expansion (Sec. 3.3),
//   - the simplified ILU(1,tau) guess of the initial blocks (Sec. 3.4),
//   - the block elimination tree that schedules the numeric sweep.
// Integer and comparison work only; all numeric factorization runs on the GPU.
#include <algorithm>
#include <chrono>
#include <atomic>
#include <cmath>
#include <numeric>
#include <thread>

#include "internal.h"

namespace bilu {

// Sec. 3.2: rows (columns) with more than mu + 2 sigma entries stay out of
// the cosine groups; mu is the mean entry count, sigma the standard
// deviation of the row (column) counts, summed in index order.
void cosine_limits(int64_t n, int64_t nnz, const int64_t* rc, const int64_t* cc, double* lim_r,
                   double* lim_c) {
  const double mean = double(nnz) / double(n);
  double vr = 0.0, vc = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    vr += (rc[i] - mean) * (rc[i] - mean);
    vc += (cc[i] - mean) * (cc[i] - mean);
  }
  *lim_r = mean + 2.0 * std::sqrt(vr / n);
  *lim_c = mean + 2.0 * std::sqrt(vc / n);
}

namespace {

// Run body(lo, hi) over [0, n) on the host's cores.
template <class F>
void parallel_for(int64_t n, F body) {
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  if (n < 4096 || nt == 1) {
    body(int64_t(0), n);
    return;
  }
  std::vector<std::thread> th;
  int64_t chunk = (n + nt - 1) / nt;
  for (unsigned t = 0; t < nt; ++t) {
    int64_t lo = t * chunk, hi = std::min<int64_t>(n, lo + chunk);
    if (lo >= hi) break;
    th.emplace_back([=] { body(lo, hi); });
  }
  for (auto& x : th) x.join();
}

struct Csr {
  int64_t n = 0;
  std::vector<int64_t> rp;
  std::vector<int32_t> ci;
  std::vector<double> v;
};

// Transpose (CSR -> CSC), rows of each column ascending.
Csr transpose(const Csr& a) {
  Csr t;
  t.n = a.n;
  t.rp.assign(a.n + 1, 0);
  for (int32_t c : a.ci) t.rp[c + 1]++;
  std::partial_sum(t.rp.begin(), t.rp.end(), t.rp.begin());
  t.ci.resize(a.ci.size());
  t.v.resize(a.v.size());
  std::vector<int64_t> fill(t.rp.begin(), t.rp.end() - 1);
  for (int64_t i = 0; i < a.n; ++i)
    for (int64_t k = a.rp[i]; k < a.rp[i + 1]; ++k) {
      int64_t d = fill[a.ci[k]]++;
      t.ci[d] = (int32_t)i;
      t.v[d] = a.v[k];
    }
  return t;
}

// B = A(perm, perm) with perm new -> old; columns re-sorted per row.
Csr permute(const Csr& a, const std::vector<int64_t>& perm) {
  const int64_t n = a.n;
  std::vector<int32_t> inv(n);
  for (int64_t i = 0; i < n; ++i) inv[perm[i]] = (int32_t)i;
  Csr b;
  b.n = n;
  b.rp.assign(n + 1, 0);
  for (int64_t i = 0; i < n; ++i) b.rp[i + 1] = a.rp[perm[i] + 1] - a.rp[perm[i]];
  std::partial_sum(b.rp.begin(), b.rp.end(), b.rp.begin());
  b.ci.resize(a.ci.size());
  b.v.resize(a.v.size());
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t i = lo; i < hi; ++i) {
      int64_t o = perm[i];
      row.clear();
      for (int64_t k = a.rp[o]; k < a.rp[o + 1]; ++k) row.emplace_back(inv[a.ci[k]], a.v[k]);
      std::sort(row.begin(), row.end(),
                [](const auto& x, const auto& y) { return x.first < y.first; });
      int64_t d = b.rp[i];
      for (auto& e : row) {
        b.ci[d] = e.first;
        b.v[d++] = e.second;
      }
    }
  });
  return b;
}

// ---------------------------------------------------------------------------
// Sec. 3.2 cosine grouping.  Row j > i joins the group seeded by row i when
// |pat(i) & pat(j)|^2 >= eps |pat(i)| |pat(j)| and neither row nor column
// of j (or i) has more than mu + 2 sigma entries.  The test involves only
// the pair, so candidates are found for every seed in parallel and the
// greedy seed order (ascending i, members ascending j, at most max_block
// members) is replayed afterwards.  With width (rows of a compressed matrix
// standing for width[i] scalars) a group holds at most max_block scalars
// and a close row that would overflow it is passed over.
// ---------------------------------------------------------------------------
void cosine(const Csr& a, const Csr& at, double eps, int max_block, std::vector<int64_t>& q,
            std::vector<int64_t>& gstart, const std::vector<int64_t>* width = nullptr) {
  const int64_t n = a.n;
  std::vector<int64_t> rc(n), cc(n);
  for (int64_t i = 0; i < n; ++i) {
    rc[i] = a.rp[i + 1] - a.rp[i];
    cc[i] = at.rp[i + 1] - at.rp[i];
  }
  double lim_r, lim_c;
  cosine_limits(n, a.rp[n], rc.data(), cc.data(), &lim_r, &lim_c);
  std::vector<char> skip(n);
  for (int64_t i = 0; i < n; ++i) skip[i] = rc[i] > lim_r || cc[i] > lim_c;

  // candidates per seed, found in parallel
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  int64_t chunk = (n + nt - 1) / nt;
  std::vector<std::vector<int64_t>> cptr(nt), clist(nt);
  std::vector<std::thread> th;
  const bool int_test = (eps == 0.8);
  for (unsigned t = 0; t < nt; ++t) {
    th.emplace_back([&, t] {
      int64_t lo = std::min<int64_t>(n, t * chunk), hi = std::min<int64_t>(n, lo + chunk);
      std::vector<int32_t> hits(n, 0);
      std::vector<int64_t> seen;
      auto& P = cptr[t];
      auto& Lst = clist[t];
      P.push_back(0);
      for (int64_t i = lo; i < hi; ++i) {
        if (!skip[i]) {
          seen.clear();
          for (int64_t k = a.rp[i]; k < a.rp[i + 1]; ++k) {
            const int32_t c = a.ci[k];
            for (int64_t m = at.rp[c + 1] - 1; m >= at.rp[c]; --m) {
              const int64_t j = at.ci[m];
              if (j <= i) break;
              if (skip[j]) continue;
              if (hits[j]++ == 0) seen.push_back(j);
            }
          }
          std::sort(seen.begin(), seen.end());
          for (int64_t j : seen) {
            const int64_t ov = hits[j];
            hits[j] = 0;
            bool ok = int_test ? (5 * ov * ov >= 4 * rc[i] * rc[j])
                               : (double(ov) * ov >= eps * double(rc[i]) * double(rc[j]));
            if (ok) Lst.push_back(j);
          }
        }
        P.push_back((int64_t)Lst.size());
      }
    });
  }
  for (auto& x : th) x.join();
  std::vector<char> taken(n, 0);
  q.clear();
  q.reserve(n);
  gstart.assign(1, 0);
  for (unsigned t = 0; t < nt; ++t) {
    int64_t lo = std::min<int64_t>(n, t * chunk);
    for (int64_t i = lo; i < lo + (int64_t)cptr[t].size() - 1; ++i) {
      if (taken[i]) continue;
      taken[i] = 1;
      q.push_back(i);
      int64_t members = width ? (*width)[i] : 1;
      for (int64_t k = cptr[t][i - lo]; k < cptr[t][i - lo + 1] && members < max_block; ++k) {
        int64_t j = clist[t][k];
        const int64_t wj = width ? (*width)[j] : 1;
        if (taken[j] || members + wj > max_block) continue;
        taken[j] = 1;
        q.push_back(j);
        members += wj;
      }
      gstart.push_back((int64_t)q.size());
    }
  }
}

// ---------------------------------------------------------------------------
// Sec. 3.3 ordering of the compressed (group) graph: nested dissection by
// recursive level-structure bisection.  A pseudo-peripheral vertex of each
// connected part is found by repeated breadth-first search; the middle
// level (the first level holding half of the part) is the separator,
// reduced to the vertices that touch the far side; both sides are ordered
// first and the separator last.  Parts of at most 8 vertices are listed in
// ascending order.
// ---------------------------------------------------------------------------
struct Graph {
  int64_t n = 0;
  std::vector<int64_t> xadj;
  std::vector<int32_t> adj;
};

// Shared state of one ordering.  Concurrent tasks own disjoint vertex sets:
// level and mark are only touched for a task's own vertices, and part is
// read for foreign vertices only to see that they are foreign (any label of
// another task differs from the reader's own).
struct NdState {
  const Graph& g;
  std::vector<std::atomic<int32_t>> part;
  std::vector<int32_t> level, mark;
  std::atomic<int32_t> next_label{1};
  std::atomic<int> threads{1};
  int max_threads = 1;
  int32_t* out;
  NdState(const Graph& gr, int32_t* o) : g(gr), part(gr.n), level(gr.n, 0), mark(gr.n, 0), out(o) {
    for (auto& x : part) x.store(0, std::memory_order_relaxed);
  }
  int32_t label() { return next_label.fetch_add(1, std::memory_order_relaxed); }
  int32_t part_of(int32_t v) const { return part[v].load(std::memory_order_relaxed); }
};

struct NdTask {
  std::vector<int32_t> verts;
  bool emit;    // a separator, already sorted
  int64_t off;  // where its order starts
};

// Breadth-first search inside the part of src; records levels.
void nd_bfs(NdState& S, int32_t src, int32_t label, std::vector<int32_t>& seq) {
  seq.clear();
  seq.push_back(src);
  S.level[src] = 0;
  S.mark[src] = label;
  const int32_t pt = S.part_of(src);
  for (size_t hd = 0; hd < seq.size(); ++hd) {
    const int32_t v = seq[hd];
    for (int64_t k = S.g.xadj[v]; k < S.g.xadj[v + 1]; ++k) {
      const int32_t w = S.g.adj[k];
      if (S.part_of(w) != pt || S.mark[w] == label) continue;
      S.mark[w] = label;
      S.level[w] = S.level[v] + 1;
      seq.push_back(w);
    }
  }
}

// One step on a task: either its order is written (a separator, a part of at
// most 8 vertices, or a part without a level structure of depth 2), or its
// children are returned in output order with their offsets.
void nd_step(NdState& S, NdTask& t, std::vector<NdTask>& kids, std::vector<int32_t>& seq) {
  kids.clear();
  auto write = [&](std::vector<int32_t>& v) {
    std::copy(v.begin(), v.end(), S.out + t.off);
  };
  if (t.emit || t.verts.size() <= 8) {
    if (!t.emit) std::sort(t.verts.begin(), t.verts.end());
    write(t.verts);
    return;
  }
  const int32_t lab = S.label();
  for (int32_t v : t.verts) S.part[v].store(lab, std::memory_order_relaxed);
  // connected components of the part, ordered one after another
  std::vector<std::vector<int32_t>> comps;
  const int32_t cm = S.label();
  for (int32_t v : t.verts) {
    if (S.mark[v] == cm) continue;
    nd_bfs(S, v, cm, seq);
    comps.push_back(seq);
  }
  if (comps.size() > 1) {
    int64_t at = t.off;
    for (auto& c : comps) {
      const int64_t sz = (int64_t)c.size();
      kids.push_back(NdTask{std::move(c), false, at});
      at += sz;
    }
    return;
  }
  // one connected part: pseudo-peripheral start vertex
  std::vector<int32_t> comp = std::move(comps[0]);
  int32_t start = *std::min_element(comp.begin(), comp.end());
  int32_t depth = -1;
  for (int it = 0; it < 4; ++it) {
    nd_bfs(S, start, S.label(), seq);
    const int32_t far = seq.back();
    if (S.level[far] <= depth) break;
    depth = S.level[far];
    start = far;
  }
  const int32_t lbl = S.label();
  nd_bfs(S, start, lbl, seq);
  const int32_t maxlev = S.level[seq.back()];
  if (maxlev < 2) {
    std::sort(comp.begin(), comp.end());
    write(comp);
    return;
  }
  // separator level: the first whose cumulative size reaches half
  std::vector<int64_t> cnt(maxlev + 1, 0);
  for (int32_t v : seq) cnt[S.level[v]]++;
  int64_t acc = 0;
  int32_t mid = 1;
  for (int32_t l = 0; l <= maxlev; ++l) {
    acc += cnt[l];
    if (2 * acc >= (int64_t)seq.size()) {
      mid = std::min(std::max(l, 1), maxlev - 1);
      break;
    }
  }
  NdTask left{{}, false, 0}, right{{}, false, 0}, sep{{}, true, 0};
  for (int32_t v : seq) {
    const int32_t l = S.level[v];
    if (l < mid) {
      left.verts.push_back(v);
    } else if (l > mid) {
      right.verts.push_back(v);
    } else {
      bool far_side = false;
      for (int64_t k = S.g.xadj[v]; k < S.g.xadj[v + 1] && !far_side; ++k) {
        const int32_t w = S.g.adj[k];
        far_side = S.part_of(w) == lab && S.mark[w] == lbl && S.level[w] == mid + 1;
      }
      (far_side ? sep.verts : left.verts).push_back(v);
    }
  }
  std::sort(sep.verts.begin(), sep.verts.end());
  // both sides first, the separator last
  left.off = t.off;
  right.off = left.off + (int64_t)left.verts.size();
  sep.off = right.off + (int64_t)right.verts.size();
  kids.push_back(std::move(left));
  kids.push_back(std::move(right));
  kids.push_back(std::move(sep));
}

// A subtree on the calling thread, with an explicit stack.
void nd_serial(NdState& S, NdTask root) {
  std::vector<NdTask> stack, kids;
  std::vector<int32_t> seq;
  stack.push_back(std::move(root));
  while (!stack.empty()) {
    NdTask t = std::move(stack.back());
    stack.pop_back();
    nd_step(S, t, kids, seq);
    for (auto& k : kids) stack.push_back(std::move(k));
  }
}

// Large parts hand their children to other threads while threads are free;
// each child writes its own range of the order, so the result does not
// depend on the schedule.
void nd_parallel(NdState& S, NdTask t) {
  constexpr size_t kSpawn = 16384;  // smallest part worth a thread
  std::vector<NdTask> kids;
  std::vector<int32_t> seq;
  nd_step(S, t, kids, seq);
  std::vector<std::thread> th;
  for (size_t i = 0; i < kids.size(); ++i) {
    NdTask& k = kids[i];
    const bool big = k.verts.size() >= kSpawn && !k.emit;
    if (big && i + 1 < kids.size() &&
        S.threads.fetch_add(1, std::memory_order_relaxed) < S.max_threads) {
      th.emplace_back([&S, task = std::move(k)]() mutable {
        nd_parallel(S, std::move(task));
        S.threads.fetch_sub(1, std::memory_order_relaxed);
      });
      continue;
    }
    if (big && i + 1 < kids.size()) S.threads.fetch_sub(1, std::memory_order_relaxed);
    if (big) nd_parallel(S, std::move(k));
    else nd_serial(S, std::move(k));
  }
  for (auto& x : th) x.join();
}

void nd_order(const Graph& g, std::vector<int32_t>& order) {
  const int64_t n = g.n;
  order.assign(n, 0);
  NdState S(g, order.data());
  S.max_threads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  NdTask root{std::vector<int32_t>(n), false, 0};
  std::iota(root.verts.begin(), root.verts.end(), 0);
  nd_parallel(S, std::move(root));
}

}  // namespace

// Sec. 3.3: order the groups (natural, or nested dissection of the
// compressed graph, built from the rows rp1/ci1 of A(pre, pre); the column
// order inside a row does not matter) and expand them: perm (new -> old)
// lists the groups contiguously, members in their order.
bilu_status order_and_expand(bilu_handle* h, const int64_t* rp1, const int32_t* ci1,
                             const std::vector<int64_t>& pre, const std::vector<int64_t>& q,
                             const std::vector<int64_t>& gs) {
  const int64_t n = h->n;
  const int64_t ng = (int64_t)gs.size() - 1;

  // group order: natural, or nested dissection of the compressed graph
  std::vector<int32_t> gorder(ng);
  std::iota(gorder.begin(), gorder.end(), 0);
  if ((h->opt.ordering == BILU_ORDER_ND || h->opt.ordering == BILU_ORDER_ND_MULTILEVEL) && ng > 8) {
    if (!ci1) return fail(h, BILU_ERR_INTERNAL, "ordering: the column indices are missing");
    std::vector<int32_t> gof(n);
    for (int64_t g = 0; g < ng; ++g)
      for (int64_t k = gs[g]; k < gs[g + 1]; ++k) gof[q[k]] = (int32_t)g;
    // edges of B + B^T: the out-neighbours of each group, sorted and unique
    std::vector<std::vector<int32_t>> nb(ng);
    parallel_for(ng, [&](int64_t lo, int64_t hi) {
      for (int64_t g = lo; g < hi; ++g) {
        auto& v = nb[g];
        for (int64_t k = gs[g]; k < gs[g + 1]; ++k) {
          int64_t r = q[k];
          for (int64_t m = rp1[r]; m < rp1[r + 1]; ++m) {
            int32_t h2 = gof[ci1[m]];
            if (h2 != g) v.push_back(h2);
          }
        }
        std::sort(v.begin(), v.end());
        v.erase(std::unique(v.begin(), v.end()), v.end());
      }
    });
    // in-neighbours, ascending by construction
    std::vector<int64_t> iptr(ng + 1, 0);
    for (int64_t g = 0; g < ng; ++g)
      for (int32_t h2 : nb[g]) iptr[h2 + 1]++;
    std::partial_sum(iptr.begin(), iptr.end(), iptr.begin());
    std::vector<int32_t> iadj(iptr[ng]);
    {
      std::vector<int64_t> fill(iptr.begin(), iptr.end() - 1);
      for (int64_t g = 0; g < ng; ++g)
        for (int32_t h2 : nb[g]) iadj[fill[h2]++] = (int32_t)g;
    }
    // the union of both lists per group
    Graph gr;
    gr.n = ng;
    gr.xadj.assign(ng + 1, 0);
    auto merge = [&](int64_t g, int32_t* out) {
      const auto& a = nb[g];
      const int32_t* b = iadj.data() + iptr[g];
      const int32_t* be = iadj.data() + iptr[g + 1];
      size_t i = 0;
      int64_t c = 0;
      while (i < a.size() || b < be) {
        int32_t x;
        if (b == be || (i < a.size() && a[i] < *b)) x = a[i++];
        else if (i == a.size() || *b < a[i]) x = *b++;
        else {
          x = a[i++];
          ++b;
        }
        if (out) out[c] = x;
        ++c;
      }
      return c;
    };
    parallel_for(ng, [&](int64_t lo, int64_t hi) {
      for (int64_t g = lo; g < hi; ++g) gr.xadj[g + 1] = merge(g, nullptr);
    });
    std::partial_sum(gr.xadj.begin(), gr.xadj.end(), gr.xadj.begin());
    gr.adj.resize(gr.xadj[ng]);
    parallel_for(ng, [&](int64_t lo, int64_t hi) {
      for (int64_t g = lo; g < hi; ++g) merge(g, gr.adj.data() + gr.xadj[g]);
    });
    if (h->opt.ordering == BILU_ORDER_ND_MULTILEVEL) {
      std::vector<int32_t> vw(ng);
      for (int64_t g = 0; g < ng; ++g) vw[g] = (int32_t)(gs[g + 1] - gs[g]);
      mlnd_order(gr.xadj, gr.adj, vw, gorder);
    } else {
      nd_order(gr, gorder);
    }
    if ((int64_t)gorder.size() != ng) return fail(h, BILU_ERR_INTERNAL, "ordering lost vertices");
  }
  // expand: groups contiguous, members in their order
  h->perm.resize(n);
  h->group_starts.assign(1, 0);
  int64_t at = 0;
  for (int64_t gi = 0; gi < ng; ++gi) {
    int64_t g = gorder[gi];
    for (int64_t k = gs[g]; k < gs[g + 1]; ++k) h->perm[at++] = pre[q[k]];
    h->group_starts.push_back(at);
  }
  return BILU_OK;
}

// The caller's pre-permutation (identity when absent); false when it is not
// a permutation.
bool pre_permutation(const bilu_handle* h, int64_t n, std::vector<int64_t>& pre) {
  pre.resize(n);
  if (!h->opt.pre_perm) {
    std::iota(pre.begin(), pre.end(), 0);
    return true;
  }
  std::vector<char> seen(n, 0);
  for (int64_t i = 0; i < n; ++i) {
    const int64_t p = h->opt.pre_perm[i];
    if (p < 0 || p >= n || seen[p]) return false;
    seen[p] = 1;
    pre[i] = p;
  }
  return true;
}

// ---------------------------------------------------------------------------
bilu_status analyze_host(bilu_handle* h, int64_t n, const int64_t* rowptr,
                         const int32_t* colind, const double* val) {
  if (n <= 0 || !rowptr || !colind || !val) return fail(h, BILU_ERR_INVALID, "null CSR or n<=0");
  if (n > INT32_MAX - 1) return fail(h, BILU_ERR_INVALID, "n exceeds int32 range");
  if (rowptr[0] != 0) return fail(h, BILU_ERR_INVALID, "rowptr[0] != 0");
  for (int64_t i = 0; i < n; ++i)
    if (rowptr[i + 1] < rowptr[i]) return fail(h, BILU_ERR_INVALID, "rowptr not monotone");
  const int64_t nnz = rowptr[n];
  std::atomic<int> bad{0};
  parallel_for(n, [&](int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi && !bad.load(std::memory_order_relaxed); ++i)
      for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
        if (colind[k] < 0 || colind[k] >= n) bad = 1;
        else if (k > rowptr[i] && colind[k] <= colind[k - 1]) bad = 2;
        else if (!std::isfinite(val[k])) bad = 3;
      }
  });
  if (bad == 1) return fail(h, BILU_ERR_INVALID, "column index out of range");
  if (bad == 2) return fail(h, BILU_ERR_INVALID, "column indices not strictly increasing");
  if (bad == 3) return fail(h, BILU_ERR_INVALID, "non-finite value");

  Csr a;
  a.n = n;
  a.rp.assign(rowptr, rowptr + n + 1);
  a.ci.assign(colind, colind + nnz);
  a.v.assign(val, val + nnz);
  h->n = n;
  h->nnz = nnz;
  h->alpha = 0.0;
  for (double x : a.v) h->alpha = std::max(h->alpha, std::fabs(x));

  // optional caller pre-permutation (with the symmetric matching: the
  // units listed along it)
  std::vector<int64_t> pre;
  const bool units = !h->sym_ustart.empty();
  if (units)
    pre = h->sym_order;
  else if (!pre_permutation(h, n, pre))
    return fail(h, BILU_ERR_INVALID, "pre_perm is not a permutation");
  Csr a1 = h->opt.pre_perm || units ? permute(a, pre) : a;

  // cosine groups
  std::vector<int64_t> q, gs;
  if (units) {
    // Sec. 5: groups of the compressed companion matrix (a unit's row is
    // the union of its rows, every column replaced by its unit), expanded;
    // without the cosine step every unit is a group
    const std::vector<int64_t>& us = h->sym_ustart;
    const int64_t nu = (int64_t)us.size() - 1;
    std::vector<int64_t> unit_of(n), width(nu), qu, gu;
    for (int64_t u = 0; u < nu; ++u) {
      width[u] = us[u + 1] - us[u];
      for (int64_t i = us[u]; i < us[u + 1]; ++i) unit_of[i] = u;
    }
    if (h->opt.use_cosine) {
      Csr c;
      c.n = nu;
      c.rp.assign(1, 0);
      std::vector<int32_t> row;
      for (int64_t u = 0; u < nu; ++u) {
        row.clear();
        for (int64_t i = us[u]; i < us[u + 1]; ++i)
          for (int64_t k = a1.rp[i]; k < a1.rp[i + 1]; ++k) row.push_back((int32_t)unit_of[a1.ci[k]]);
        std::sort(row.begin(), row.end());
        row.erase(std::unique(row.begin(), row.end()), row.end());
        c.ci.insert(c.ci.end(), row.begin(), row.end());
        c.rp.push_back((int64_t)c.ci.size());
      }
      c.v.assign(c.ci.size(), 0.0);
      cosine(c, transpose(c), h->opt.cos_eps, h->opt.max_block, qu, gu, &width);
    } else {
      qu.resize(nu);
      std::iota(qu.begin(), qu.end(), 0);
      gu.resize(nu + 1);
      std::iota(gu.begin(), gu.end(), 0);
    }
    gs.assign(1, 0);
    for (size_t g = 0; g + 1 < gu.size(); ++g) {
      for (int64_t k = gu[g]; k < gu[g + 1]; ++k)
        for (int64_t i = us[qu[k]]; i < us[qu[k] + 1]; ++i) q.push_back(i);
      gs.push_back((int64_t)q.size());
    }
  } else if (h->opt.use_cosine) {
    Csr a1t = transpose(a1);
    cosine(a1, a1t, h->opt.cos_eps, h->opt.max_block, q, gs);
  } else {
    q.resize(n);
    std::iota(q.begin(), q.end(), 0);
    gs.resize(n + 1);
    std::iota(gs.begin(), gs.end(), 0);
  }
  const bilu_status os = order_and_expand(h, a1.rp.data(), a1.ci.data(), pre, q, gs);
  if (os != BILU_OK) return os;
  h->sym_partner.clear();
  if (units) {
    // the 2x2 pivots in the final numbering
    std::vector<int64_t> pos(n);
    for (int64_t i = 0; i < n; ++i) pos[h->perm[i]] = i;
    h->sym_partner.assign(n, -1);
    const std::vector<int64_t>& us = h->sym_ustart;
    for (size_t u = 0; u + 1 < us.size(); ++u)
      if (us[u + 1] - us[u] == 2) {
        const int64_t p0 = pos[h->sym_order[us[u]]], p1 = pos[h->sym_order[us[u] + 1]];
        h->sym_partner[p0] = (int32_t)p1;
        h->sym_partner[p1] = (int32_t)p0;
      }
  }
  Csr p = permute(a, h->perm);
  Csr pt = transpose(p);
  h->prp = std::move(p.rp);
  h->pci = std::move(p.ci);
  h->pv = std::move(p.v);
  h->pcp = std::move(pt.rp);
  h->pri = std::move(pt.ci);
  h->pcv = std::move(pt.v);
  return BILU_OK;
}

// ---------------------------------------------------------------------------
// Sec. 3.4: for every scalar k the estimated column pattern I~_k of L (rows
// i > k with |a_ik| >= tau |a_kk|, plus rows i reached through an original
// a_ij a_jk, j < k, with |a_ij a_jk| >= tau |a_jj a_kk|) and, symmetrically,
// J~_k of U.  Blocks grow unit by unit (cosine groups) while the dense
// block count f' = (r'+s'+l')*l' stays within 4/3 of the scalar count c' or
// within c' + 4 l'; r', s' count the union rows/columns beyond the block.
// ---------------------------------------------------------------------------
int64_t ilu1t_partition(const bilu_handle* h, double tau, std::vector<int32_t>& bstart,
                        double* t_sets) {
  const auto t_start = std::chrono::steady_clock::now();
  const int64_t n = h->n;
  const auto& gs = h->group_starts;
  const int64_t nu = (int64_t)gs.size() - 1;
  bstart.assign(1, 0);
  if (!h->opt.use_ilu1t) {
    for (int64_t u = 0; u < nu; ++u) bstart.push_back((int32_t)gs[u + 1]);
    return nu;
  }
  const auto& rp = h->prp;
  const auto& ci = h->pci;
  const auto& rv = h->pv;
  const auto& cp = h->pcp;
  const auto& ri = h->pri;
  const auto& cv = h->pcv;
  std::vector<double> dg(n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k)
      if (ci[k] == i) dg[i] = rv[k];
  // Sec. 5: both scalars of a 2x2 pivot take the pivot block's largest
  // magnitude in place of |a_kk| (a zero diagonal inside a 2x2 pivot would
  // pass every candidate)
  if (!h->sym_partner.empty()) {
    auto at = [&](int64_t r, int64_t c) {
      const auto b = ci.begin() + rp[r], e = ci.begin() + rp[r + 1];
      const auto it = std::lower_bound(b, e, (int32_t)c);
      return it != e && *it == c ? std::fabs(rv[it - ci.begin()]) : 0.0;
    };
    std::vector<double> d2(dg);
    for (int64_t i = 0; i < n; ++i) {
      const int64_t p = h->sym_partner[i];
      if (p >= 0) d2[i] = std::max(std::max(at(i, i), at(p, p)), std::max(at(i, p), at(p, i)));
    }
    dg.swap(d2);
  }
  // per-k sets, computed in parallel into per-range buffers
  unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  int64_t chunk = (n + nt - 1) / nt;
  std::vector<std::vector<int32_t>> Ibuf(nt), Jbuf(nt);
  std::vector<int64_t> Iptr(n + 1, 0), Jptr(n + 1, 0);
  std::vector<int32_t> Icnt(n), Jcnt(n);
  std::vector<std::thread> th;
  for (unsigned t = 0; t < nt; ++t) {
    th.emplace_back([&, t] {
      int64_t lo = std::min<int64_t>(n, t * chunk), hi = std::min<int64_t>(n, lo + chunk);
      std::vector<int32_t> stamp(n, -1);
      auto& IB = Ibuf[t];
      auto& JB = Jbuf[t];
      for (int64_t k = lo; k < hi; ++k) {
        const double akk = std::fabs(dg[k]);
        size_t s0 = IB.size();
        for (int64_t m = cp[k]; m < cp[k + 1]; ++m) {
          int32_t i = ri[m];
          if (i > k && std::fabs(cv[m]) >= tau * akk && stamp[i] != (int32_t)k) {
            stamp[i] = (int32_t)k;
            IB.push_back(i);
          }
        }
        for (int64_t m = cp[k]; m < cp[k + 1]; ++m) {
          int32_t j = ri[m];
          if (j >= k) break;
          const double ajk = cv[m];
          const double thr = tau * std::fabs(dg[j] * dg[k]);
          for (int64_t m2 = cp[j + 1] - 1; m2 >= cp[j]; --m2) {
            int32_t i = ri[m2];
            if (i <= k) break;
            if (stamp[i] != (int32_t)k && std::fabs(cv[m2] * ajk) >= thr) {
              stamp[i] = (int32_t)k;
              IB.push_back(i);
            }
          }
        }
        Icnt[k] = (int32_t)(IB.size() - s0);
        // row k of U, stamps shifted to keep them apart from the column pass
        const int32_t sk = (int32_t)(k + n);
        size_t t0 = JB.size();
        for (int64_t m = rp[k]; m < rp[k + 1]; ++m) {
          int32_t j = ci[m];
          if (j > k && std::fabs(rv[m]) >= tau * akk && stamp[j] != sk) {
            stamp[j] = sk;
            JB.push_back(j);
          }
        }
        for (int64_t m = rp[k]; m < rp[k + 1]; ++m) {
          int32_t i = ci[m];
          if (i >= k) break;
          const double aki = rv[m];
          const double thr = tau * std::fabs(dg[i] * dg[k]);
          for (int64_t m2 = rp[i + 1] - 1; m2 >= rp[i]; --m2) {
            int32_t j = ci[m2];
            if (j <= k) break;
            if (stamp[j] != sk && std::fabs(aki * rv[m2]) >= thr) {
              stamp[j] = sk;
              JB.push_back(j);
            }
          }
        }
        Jcnt[k] = (int32_t)(JB.size() - t0);
      }
    });
  }
  for (auto& x : th) x.join();
  // flatten offsets (per-thread buffers are in k order)
  for (int64_t k = 0; k < n; ++k) {
    Iptr[k + 1] = Iptr[k] + Icnt[k];
    Jptr[k + 1] = Jptr[k] + Jcnt[k];
  }
  std::vector<int32_t> Iall(Iptr[n]), Jall(Jptr[n]);
  {
    int64_t oi = 0, oj = 0;
    for (unsigned t = 0; t < nt; ++t) {
      std::copy(Ibuf[t].begin(), Ibuf[t].end(), Iall.begin() + oi);
      std::copy(Jbuf[t].begin(), Jbuf[t].end(), Jall.begin() + oj);
      oi += (int64_t)Ibuf[t].size();
      oj += (int64_t)Jbuf[t].size();
    }
  }
  if (t_sets)
    *t_sets = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
  // Growth.  Whether unit u joins the block that starts at unit s depends
  // only on s and u, so the end g(s) of a block started at s is computed for
  // every s in parallel; the partition then follows s -> g(s) from s = 0,
  // which is exactly the sequential greedy growth.  Marks: 2s = row (column)
  // of the block started at s, 2s+1 = tentatively added by the next unit.
  const int maxb = h->opt.max_block;
  std::vector<int64_t> gend(nu);
  auto count_beyond = [](const std::vector<int32_t>& v, int64_t last) {
    int64_t c = 0;
    for (int32_t x : v) c += x > last;
    return c;
  };
  auto grow_range = [&](int64_t ulo, int64_t uhi) {
    std::vector<uint32_t> rmark(n, UINT32_MAX), cmark(n, UINT32_MAX);
    std::vector<int32_t> rows, cols, addr, addc;
    for (int64_t s = ulo; s < uhi; ++s) {
      const uint32_t mk = (uint32_t)(2 * s), tent = mk + 1;
      rows.clear();
      cols.clear();
      const int64_t s0 = gs[s];
      int64_t scal = 0;
      for (int64_t k = s0; k < gs[s + 1]; ++k) {
        for (int64_t m = Iptr[k]; m < Iptr[k + 1]; ++m)
          if (rmark[Iall[m]] != mk) {
            rmark[Iall[m]] = mk;
            rows.push_back(Iall[m]);
          }
        for (int64_t m = Jptr[k]; m < Jptr[k + 1]; ++m)
          if (cmark[Jall[m]] != mk) {
            cmark[Jall[m]] = mk;
            cols.push_back(Jall[m]);
          }
        scal += Icnt[k] + Jcnt[k] + 1;
      }
      int64_t u = s + 1;
      while (u < nu) {
        const int64_t e2 = gs[u + 1];
        const int64_t w2 = e2 - s0;
        if (w2 > maxb) break;
        // union beyond the new last index, the new unit's entries tentative
        int64_t r2 = count_beyond(rows, e2 - 1), c2 = count_beyond(cols, e2 - 1);
        int64_t sc2 = scal;
        addr.clear();
        addc.clear();
        for (int64_t k = gs[u]; k < e2; ++k) {
          for (int64_t m = Iptr[k]; m < Iptr[k + 1]; ++m) {
            const int32_t i = Iall[m];
            if (rmark[i] != mk && rmark[i] != tent) {
              rmark[i] = tent;
              addr.push_back(i);
            }
          }
          for (int64_t m = Jptr[k]; m < Jptr[k + 1]; ++m) {
            const int32_t j = Jall[m];
            if (cmark[j] != mk && cmark[j] != tent) {
              cmark[j] = tent;
              addc.push_back(j);
            }
          }
          sc2 += Icnt[k] + Jcnt[k] + 1;
        }
        r2 += count_beyond(addr, e2 - 1);
        c2 += count_beyond(addc, e2 - 1);
        const int64_t f2 = (r2 + c2 + w2) * w2;
        if (!(3 * f2 <= 4 * sc2 || f2 <= sc2 + 4 * w2)) break;
        for (int32_t i : addr) rmark[i] = mk;
        for (int32_t j : addc) cmark[j] = mk;
        rows.insert(rows.end(), addr.begin(), addr.end());
        cols.insert(cols.end(), addc.begin(), addc.end());
        scal = sc2;
        ++u;
      }
      gend[s] = u;
    }
  };
  {
    const int64_t uchunk = (nu + nt - 1) / nt;
    std::vector<std::thread> tg;
    for (unsigned t = 0; t < nt; ++t) {
      const int64_t lo = std::min<int64_t>(nu, t * uchunk), hi = std::min<int64_t>(nu, lo + uchunk);
      if (lo < hi) tg.emplace_back(grow_range, lo, hi);
    }
    for (auto& x : tg) x.join();
  }
  for (int64_t u = 0; u < nu; u = gend[u]) bstart.push_back((int32_t)gs[gend[u]]);
  return (int64_t)bstart.size() - 1;
}

}  // namespace bilu
