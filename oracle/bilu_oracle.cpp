// Block incomplete LU (BILU) -- plain FP64 CPU oracle.
//
// TEST INFRASTRUCTURE ONLY: the sequential reference the GPU library is
// checked against.  Written from the paper (arXiv 1908.10169); every
// function names the section it follows.  Nothing here is tuned: plain
// loops, no BLAS, one thread, one block column at a time in the order the
// Crout sweep of Sec. 2.1/2.2 prescribes.
//
// Readings of passages that the paper leaves open are marked "Reading:".

#include "bilu_oracle.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

namespace {

using i64 = int64_t;
using Clock = std::chrono::steady_clock;

// ---------------------------------------------------------------------------
// Sparse matrix with sorted column indices (CSR); also used for CSC.
// ---------------------------------------------------------------------------
struct Mat {
  i64 n = 0;
  std::vector<i64> rp;
  std::vector<i64> ci;
  std::vector<double> v;
};

Mat from_csr(i64 n, const int64_t* rp, const int32_t* ci, const double* v) {
  Mat a;
  a.n = n;
  a.rp.assign(rp, rp + n + 1);
  i64 nnz = rp[n];
  a.ci.resize(nnz);
  a.v.resize(nnz);
  for (i64 k = 0; k < nnz; ++k) {
    a.ci[k] = ci[k];
    a.v[k] = v ? v[k] : 1.0;
  }
  return a;
}

Mat transpose(const Mat& a) {
  Mat t;
  t.n = a.n;
  t.rp.assign(a.n + 1, 0);
  for (i64 k = 0; k < a.rp[a.n]; ++k) t.rp[a.ci[k] + 1]++;
  for (i64 i = 0; i < a.n; ++i) t.rp[i + 1] += t.rp[i];
  t.ci.resize(a.ci.size());
  t.v.resize(a.v.size());
  std::vector<i64> next(t.rp.begin(), t.rp.end() - 1);
  for (i64 i = 0; i < a.n; ++i)
    for (i64 k = a.rp[i]; k < a.rp[i + 1]; ++k) {
      i64 p = next[a.ci[k]]++;
      t.ci[p] = i;
      t.v[p] = a.v[k];
    }
  return t;
}

// B(i, j) = A(perm[i], perm[j]),  perm: new -> old.
Mat permute_sym(const Mat& a, const std::vector<i64>& perm) {
  std::vector<i64> inv(a.n);
  for (i64 i = 0; i < a.n; ++i) inv[perm[i]] = i;
  Mat b;
  b.n = a.n;
  b.rp.assign(a.n + 1, 0);
  for (i64 i = 0; i < a.n; ++i) {
    i64 o = perm[i];
    b.rp[i + 1] = b.rp[i] + (a.rp[o + 1] - a.rp[o]);
  }
  b.ci.resize(a.ci.size());
  b.v.resize(a.v.size());
  std::vector<std::pair<i64, double>> row;
  for (i64 i = 0; i < a.n; ++i) {
    i64 o = perm[i];
    row.clear();
    for (i64 k = a.rp[o]; k < a.rp[o + 1]; ++k) row.push_back({inv[a.ci[k]], a.v[k]});
    std::sort(row.begin(), row.end(),
              [](const std::pair<i64, double>& x, const std::pair<i64, double>& y) {
                return x.first < y.first;
              });
    for (size_t k = 0; k < row.size(); ++k) {
      b.ci[b.rp[i] + k] = row[k].first;
      b.v[b.rp[i] + k] = row[k].second;
    }
  }
  return b;
}

double entry(const Mat& a, i64 i, i64 j) {
  auto b = a.ci.begin() + a.rp[i], e = a.ci.begin() + a.rp[i + 1];
  auto it = std::lower_bound(b, e, j);
  if (it != e && *it == j) return a.v[it - a.ci.begin()];
  return 0.0;
}

double sgn(double x) { return x < 0.0 ? -1.0 : 1.0; }  // Reading: sign(0) = +1

// ---------------------------------------------------------------------------
// Sec. 3.2: cosine-based blocking with the mu + 2 sigma filter.
// ---------------------------------------------------------------------------
// Two rows are grouped when the square of the size of their pattern overlap
// is at least eps times the product of their pattern sizes; only rows j > i
// that share a column with row i (upper part of A A^T) and are not yet in a
// group are considered.  Rows or columns with more than mu + 2 sigma entries
// are left out of the grouping.
// Readings: a left-out index becomes a group of its own; the test compares
// against the seed row i; groups are listed in seed order, members
// ascending; a group never exceeds max_block members.  With width (the
// rows of a compressed matrix stand for width[i] scalars) a group never
// exceeds max_block scalars: a close row that would overflow it is passed
// over.
i64 cosine_groups(const Mat& a, double eps, int max_block, std::vector<i64>& perm,
                  std::vector<i64>& gstart, i64* n_ignored,
                  const std::vector<i64>* width = nullptr) {
  const i64 n = a.n;
  Mat at = transpose(a);
  std::vector<i64> nzr(n), nzc(n);
  for (i64 i = 0; i < n; ++i) nzr[i] = a.rp[i + 1] - a.rp[i];
  for (i64 j = 0; j < n; ++j) nzc[j] = at.rp[j + 1] - at.rp[j];
  double mu = double(a.rp[n]) / double(n);
  double sr = 0, sc = 0;
  for (i64 i = 0; i < n; ++i) {
    sr += (nzr[i] - mu) * (nzr[i] - mu);
    sc += (nzc[i] - mu) * (nzc[i] - mu);
  }
  sr = std::sqrt(sr / n);
  sc = std::sqrt(sc / n);
  std::vector<char> ignored(n, 0);
  i64 nig = 0;
  for (i64 i = 0; i < n; ++i) {
    if (nzr[i] > mu + 2 * sr || nzc[i] > mu + 2 * sc) {
      ignored[i] = 1;
      ++nig;
    }
  }
  if (n_ignored) *n_ignored = nig;
  std::vector<char> assigned(n, 0);
  std::vector<i64> cnt(n, 0), touched;
  perm.clear();
  gstart.assign(1, 0);
  const bool int_test = (eps == 0.8);
  for (i64 i = 0; i < n; ++i) {
    if (assigned[i]) continue;
    assigned[i] = 1;
    perm.push_back(i);
    if (!ignored[i]) {
      touched.clear();
      for (i64 k = a.rp[i]; k < a.rp[i + 1]; ++k) {
        i64 c = a.ci[k];
        for (i64 m = at.rp[c]; m < at.rp[c + 1]; ++m) {
          i64 j = at.ci[m];
          if (j <= i || assigned[j] || ignored[j]) continue;
          if (cnt[j] == 0) touched.push_back(j);
          cnt[j]++;
        }
      }
      std::sort(touched.begin(), touched.end());
      i64 members = width ? (*width)[i] : 1;
      for (i64 j : touched) {
        i64 ov = cnt[j];
        bool close;
        if (int_test)
          close = 5 * ov * ov >= 4 * nzr[i] * nzr[j];
        else
          close = double(ov) * double(ov) >= eps * double(nzr[i]) * double(nzr[j]);
        const i64 wj = width ? (*width)[j] : 1;
        if (close && members + wj <= max_block) {
          assigned[j] = 1;
          perm.push_back(j);
          members += wj;
        }
      }
      for (i64 j : touched) cnt[j] = 0;
    }
    gstart.push_back((i64)perm.size());
  }
  return (i64)gstart.size() - 1;
}

// Sec. 5 (symmetric variant): the compressed companion matrix.  Units are
// contiguous index ranges [us[u], us[u+1]) (a 1x1 or a 2x2 pivot of the
// symmetric matching); row u of the result is the union of the unit's rows
// with every column index replaced by its unit (pattern only).
Mat compress_units(const Mat& a, const std::vector<i64>& us) {
  const i64 nu = (i64)us.size() - 1;
  std::vector<i64> unit_of(a.n);
  for (i64 u = 0; u < nu; ++u)
    for (i64 i = us[u]; i < us[u + 1]; ++i) unit_of[i] = u;
  Mat c;
  c.n = nu;
  c.rp.assign(1, 0);
  std::vector<i64> row;
  for (i64 u = 0; u < nu; ++u) {
    row.clear();
    for (i64 i = us[u]; i < us[u + 1]; ++i)
      for (i64 k = a.rp[i]; k < a.rp[i + 1]; ++k) row.push_back(unit_of[a.ci[k]]);
    std::sort(row.begin(), row.end());
    row.erase(std::unique(row.begin(), row.end()), row.end());
    c.ci.insert(c.ci.end(), row.begin(), row.end());
    c.rp.push_back((i64)c.ci.size());
  }
  c.v.assign(c.ci.size(), 0.0);
  return c;
}

// ---------------------------------------------------------------------------
// Sec. 3.4: simplified ILU(1,tau) estimate of the pattern of column k of L
// and row k of U, and the block growth rule built on it.
// ---------------------------------------------------------------------------
struct Ilu1tSets {
  std::vector<i64> I;  // estimated rows i > k of column k of L
  std::vector<i64> J;  // estimated cols j > k of row k of U
};

// Column k: entries a_ik (i > k) with |a_ik| >= tau |a_kk|, plus fill rows
// i > k created by a_ij a_jk (j < k) with |a_ij a_jk| >= tau |a_jj a_kk|.
// Row k symmetric.  Only entries of the original matrix enter (ILU(1)).
Ilu1tSets ilu1t_sets(const Mat& a, const Mat& at, const std::vector<double>& dg,
                     i64 k, double tau) {
  Ilu1tSets s;
  const double akk = dg[k];
  // column k of L
  for (i64 m = at.rp[k]; m < at.rp[k + 1]; ++m) {
    i64 i = at.ci[m];
    double aik = at.v[m];
    if (i > k && std::fabs(aik) >= tau * std::fabs(akk)) s.I.push_back(i);
  }
  for (i64 m = at.rp[k]; m < at.rp[k + 1]; ++m) {
    i64 j = at.ci[m];
    if (j >= k) continue;
    double ajk = at.v[m];
    for (i64 m2 = at.rp[j]; m2 < at.rp[j + 1]; ++m2) {
      i64 i = at.ci[m2];
      if (i <= k) continue;
      double aij = at.v[m2];
      if (std::fabs(aij * ajk) >= tau * std::fabs(dg[j] * akk)) s.I.push_back(i);
    }
  }
  // row k of U
  for (i64 m = a.rp[k]; m < a.rp[k + 1]; ++m) {
    i64 j = a.ci[m];
    double akj = a.v[m];
    if (j > k && std::fabs(akj) >= tau * std::fabs(akk)) s.J.push_back(j);
  }
  for (i64 m = a.rp[k]; m < a.rp[k + 1]; ++m) {
    i64 i = a.ci[m];
    if (i >= k) continue;
    double aki = a.v[m];
    for (i64 m2 = a.rp[i]; m2 < a.rp[i + 1]; ++m2) {
      i64 j = a.ci[m2];
      if (j <= k) continue;
      double aij = a.v[m2];
      if (std::fabs(aki * aij) >= tau * std::fabs(dg[i] * akk)) s.J.push_back(j);
    }
  }
  std::sort(s.I.begin(), s.I.end());
  s.I.erase(std::unique(s.I.begin(), s.I.end()), s.I.end());
  std::sort(s.J.begin(), s.J.end());
  s.J.erase(std::unique(s.J.begin(), s.J.end()), s.J.end());
  return s;
}

// Union of sorted x with sorted y, keeping only entries > last.
std::vector<i64> union_above(const std::vector<i64>& x, const std::vector<i64>& y, i64 last) {
  std::vector<i64> out;
  out.reserve(x.size() + y.size());
  size_t p = 0, q = 0;
  while (p < x.size() || q < y.size()) {
    i64 v;
    if (q >= y.size() || (p < x.size() && x[p] < y[q]))
      v = x[p++];
    else if (p >= x.size() || y[q] < x[p])
      v = y[q++];
    else {
      v = x[p++];
      ++q;
    }
    if (v > last) out.push_back(v);
  }
  return out;
}

// Growth rule: a block of width l with r rows below it in L, s columns right
// of it in U and c scalar entries is enlarged by the next unit as long as
// the new dense count f' = (r'+s'+l')*l' satisfies f' <= 4/3 c' or
// f' <= c' + 4 l', where c' adds |I_k| + |J_k| + 1 for each new column k.
// Readings: the unit of growth is a cosine group (a scalar without the
// cosine step); |I|, |J| in c' are the estimated sets; the diagonal is the
// "+1"; widths never exceed max_block.
// Sec. 5 (symmetric variant, 1x1 and 2x2 pivots): with partner (the other
// index of a scalar's 2x2 pivot, -1 for a 1x1 pivot) both scalars of a 2x2
// pivot take the pivot block's largest magnitude in place of |a_kk| in the
// thresholds.  Reading: the paper says only that ILU(1,tau) is modified to
// deal with 1x1 and 2x2 pivots; a zero diagonal inside a 2x2 pivot would
// otherwise pass every candidate.
i64 ilu1t_blocks(const Mat& a, const std::vector<i64>& ustart, double tau, int max_block,
                 bool grow, std::vector<i64>& bstart, const std::vector<i64>* partner = nullptr) {
  Mat at = transpose(a);
  std::vector<double> dg(a.n, 0.0);
  for (i64 i = 0; i < a.n; ++i) dg[i] = entry(a, i, i);
  if (partner && !partner->empty()) {
    std::vector<double> d2(dg);
    for (i64 i = 0; i < a.n; ++i) {
      const i64 p = (*partner)[i];
      if (p < 0) continue;
      d2[i] = std::max(std::max(std::fabs(entry(a, i, i)), std::fabs(entry(a, p, p))),
                       std::max(std::fabs(entry(a, i, p)), std::fabs(entry(a, p, i))));
    }
    dg.swap(d2);
  }
  const i64 nu = (i64)ustart.size() - 1;
  bstart.assign(1, 0);
  i64 u = 0;
  while (u < nu) {
    i64 s0 = ustart[u], e0 = ustart[u + 1];
    std::vector<i64> rows, cols;
    i64 c = 0;
    for (i64 k = s0; grow && k < e0; ++k) {
      Ilu1tSets st = ilu1t_sets(a, at, dg, k, tau);
      rows = union_above(rows, st.I, e0 - 1);
      cols = union_above(cols, st.J, e0 - 1);
      c += (i64)st.I.size() + (i64)st.J.size() + 1;
    }
    i64 l = e0 - s0;
    ++u;
    while (grow && u < nu) {
      i64 s1 = ustart[u], e1 = ustart[u + 1];
      i64 l2 = l + (e1 - s1);
      if (l2 > max_block) break;
      std::vector<i64> rows2 = union_above(rows, {}, e1 - 1);
      std::vector<i64> cols2 = union_above(cols, {}, e1 - 1);
      i64 c2 = c;
      for (i64 k = s1; k < e1; ++k) {
        Ilu1tSets st = ilu1t_sets(a, at, dg, k, tau);
        rows2 = union_above(rows2, st.I, e1 - 1);
        cols2 = union_above(cols2, st.J, e1 - 1);
        c2 += (i64)st.I.size() + (i64)st.J.size() + 1;
      }
      i64 f2 = ((i64)rows2.size() + (i64)cols2.size() + l2) * l2;
      if (3 * f2 <= 4 * c2 || f2 <= c2 + 4 * l2) {
        rows.swap(rows2);
        cols.swap(cols2);
        c = c2;
        l = l2;
        ++u;
      } else {
        break;
      }
    }
    bstart.push_back(bstart.back() + l);
  }
  return (i64)bstart.size() - 1;
}

// ---------------------------------------------------------------------------
// Sec. 3.6: perturbation of a singular or ill-conditioned diagonal block,
// then LU with partial pivoting inside the block and explicit inversion
// (Sec. 2.2: the diagonal blocks are factored and inverted).
// ---------------------------------------------------------------------------
// Column j: the entry of largest magnitude d_kj (lowest k on ties), or the
// diagonal when 2|d_jj| >= |d_kj|, becomes d_kj (1 + rho beta_j) +
// sign(d_kj) tau alpha.  Rows analogously afterwards.
// Readings: beta_j := delta_j (max |column j|) unless beta_one; all-zero
// columns/rows are perturbed before factoring; a pivot with |u_jj| <=
// pivot_eps * max|S| marks the block ill-conditioned, then every column and
// then every row is perturbed and the block refactored, at most 3 times.
void perturb_col(std::vector<double>& m, int q, int j, double alpha, const orc_options& o) {
  int k = 0;
  double dmax = -1.0;
  for (int i = 0; i < q; ++i)
    if (std::fabs(m[i * q + j]) > dmax) {
      dmax = std::fabs(m[i * q + j]);
      k = i;
    }
  if (2.0 * std::fabs(m[j * q + j]) >= std::fabs(m[k * q + j])) k = j;
  double beta = o.beta_one ? 1.0 : dmax;
  double d = m[k * q + j];
  m[k * q + j] = d * (1.0 + o.pert_rho * beta) + sgn(d) * o.pert_tau * alpha;
}

void perturb_row(std::vector<double>& m, int q, int i, double alpha, const orc_options& o) {
  int k = 0;
  double dmax = -1.0;
  for (int j = 0; j < q; ++j)
    if (std::fabs(m[i * q + j]) > dmax) {
      dmax = std::fabs(m[i * q + j]);
      k = j;
    }
  if (2.0 * std::fabs(m[i * q + i]) >= std::fabs(m[i * q + k])) k = i;
  double beta = o.beta_one ? 1.0 : dmax;
  double d = m[i * q + k];
  m[i * q + k] = d * (1.0 + o.pert_rho * beta) + sgn(d) * o.pert_tau * alpha;
}

// Sec. 5, the symmetrized perturbation (reading: the paper names it only):
// column j's entry is chosen as in perturb_col and the same new value is
// written at (k, j) and at its mirror (j, k), one column after the other.
void perturb_sym(std::vector<double>& m, int q, int j, double alpha, const orc_options& o) {
  int k = 0;
  double dmax = -1.0;
  for (int i = 0; i < q; ++i)
    if (std::fabs(m[i * q + j]) > dmax) {
      dmax = std::fabs(m[i * q + j]);
      k = i;
    }
  if (2.0 * std::fabs(m[j * q + j]) >= std::fabs(m[k * q + j])) k = j;
  double beta = o.beta_one ? 1.0 : dmax;
  double d = m[k * q + j];
  const double nv = d * (1.0 + o.pert_rho * beta) + sgn(d) * o.pert_tau * alpha;
  m[k * q + j] = nv;
  m[j * q + k] = nv;
}

// LU with partial pivoting (lowest index wins ties).  Returns false when a
// pivot is not above pivot_eps * max|m|.
bool getrf(std::vector<double> lu, int q, double pivot_eps, std::vector<double>& out,
           std::vector<int>& piv) {
  double smax = 0.0;
  for (double x : lu) {
    if (!std::isfinite(x)) return false;
    smax = std::max(smax, std::fabs(x));
  }
  piv.assign(q, 0);
  for (int j = 0; j < q; ++j) {
    int p = j;
    double best = std::fabs(lu[j * q + j]);
    for (int i = j + 1; i < q; ++i)
      if (std::fabs(lu[i * q + j]) > best) {
        best = std::fabs(lu[i * q + j]);
        p = i;
      }
    piv[j] = p;
    if (p != j)
      for (int c = 0; c < q; ++c) std::swap(lu[j * q + c], lu[p * q + c]);
    double u = lu[j * q + j];
    if (!(std::fabs(u) > pivot_eps * smax) || u == 0.0) return false;
    for (int i = j + 1; i < q; ++i) {
      double f = lu[i * q + j] / u;
      lu[i * q + j] = f;
      for (int c = j + 1; c < q; ++c) lu[i * q + c] -= f * lu[j * q + c];
    }
  }
  out.swap(lu);
  return true;
}

// Inverse from the LU factors: solve LU x = P e_j for every j.
void lu_inverse(const std::vector<double>& lu, const std::vector<int>& piv, int q,
                std::vector<double>& inv) {
  inv.assign((size_t)q * q, 0.0);
  std::vector<double> x(q);
  for (int j = 0; j < q; ++j) {
    for (int i = 0; i < q; ++i) x[i] = (i == j) ? 1.0 : 0.0;
    for (int i = 0; i < q; ++i) std::swap(x[i], x[piv[i]]);
    for (int i = 0; i < q; ++i)
      for (int c = 0; c < i; ++c) x[i] -= lu[i * q + c] * x[c];
    for (int i = q - 1; i >= 0; --i) {
      for (int c = i + 1; c < q; ++c) x[i] -= lu[i * q + c] * x[c];
      x[i] /= lu[i * q + i];
    }
    for (int i = 0; i < q; ++i) inv[i * q + j] = x[i];
  }
}

// Returns number of perturbation rounds (0 = none), -1 if still singular.
int perturb_invert(int q, std::vector<double> m, double alpha, const orc_options& o,
                   std::vector<double>& s_used, std::vector<double>& dinv) {
  int rounds = 0;
  bool pre = false;
  for (int j = 0; j < q; ++j) {
    bool zero = true;
    for (int i = 0; i < q; ++i) zero = zero && m[i * q + j] == 0.0;
    if (zero) {
      perturb_col(m, q, j, alpha, o);
      pre = true;
    }
  }
  for (int i = 0; i < q; ++i) {
    bool zero = true;
    for (int j = 0; j < q; ++j) zero = zero && m[i * q + j] == 0.0;
    if (zero) {
      perturb_row(m, q, i, alpha, o);
      pre = true;
    }
  }
  if (pre) rounds = 1;
  std::vector<double> lu;
  std::vector<int> piv;
  for (int attempt = 0;; ++attempt) {
    if (getrf(m, q, o.pivot_eps, lu, piv)) break;
    if (attempt == 3) return -1;
    if (o.sym_perturb) {
      for (int j = 0; j < q; ++j) perturb_sym(m, q, j, alpha, o);
    } else {
      for (int j = 0; j < q; ++j) perturb_col(m, q, j, alpha, o);
      for (int i = 0; i < q; ++i) perturb_row(m, q, i, alpha, o);
    }
    ++rounds;
  }
  lu_inverse(lu, piv, q, dinv);
  s_used = m;
  return rounds;
}

// ---------------------------------------------------------------------------
// Factor storage
// ---------------------------------------------------------------------------
struct Block {
  i64 first = 0;
  int q = 0;
  bool alive = true;
  bool computed = false;  // created by the sweep (not by a merge)
  std::vector<i64> R;     // rows > last, sorted
  std::vector<double> L;  // |R| x q row-major
  std::vector<i64> C;     // cols > last, sorted
  std::vector<double> W;  // q x |C| column-major
  std::vector<double> D;  // q x q row-major, inverse pivot block
  std::vector<double> S;  // q x q row-major, pivot block actually used
  i64 last() const { return first + q - 1; }
};

struct DropRec {
  i64 block, index;
  int kind;
  double norm;
  int kept;
};

double drop_norm(const double* x, int len, i64 stride, int kind) {
  double r = 0.0;
  if (kind == 1) {
    for (int t = 0; t < len; ++t) r += x[t * stride] * x[t * stride];
    return std::sqrt(r);
  }
  for (int t = 0; t < len; ++t) r = std::max(r, std::fabs(x[t * stride]));
  return r;
}

}  // namespace

// ---------------------------------------------------------------------------
// Handle
// ---------------------------------------------------------------------------
struct orc_handle {
  i64 n = 0;
  Mat A;                       // original
  Mat P;                       // permuted  (P(i,j) = A(perm[i], perm[j]))
  std::vector<i64> perm;       // new -> old
  std::vector<i64> gstart;     // cosine groups in permuted numbering
  std::vector<i64> partner;    // the other scalar of a 2x2 pivot (-1: 1x1), permuted numbering
  std::vector<i64> start0;     // initial partition
  std::vector<Block> blocks;   // all blocks ever created (dead ones merged)
  std::vector<int> live;       // ids of final blocks in order
  std::vector<DropRec> droplog;
  std::vector<i64> mergelog;   // K, p, q, mu, nu, merged
  i64 n_ignored = 0, n_perturbed = 0, n_merges = 0;
  int singular = 0;
  double alpha = 0.0;
  double t_analyze = 0, t_ilu1t = 0, t_factor = 0;
  orc_options opt{};
};

namespace {

// ---------------------------------------------------------------------------
// Sec. 3.5: progressive aggregation test and merge of the live block P
// (immediately preceding) with the block K just computed.
// ---------------------------------------------------------------------------
// Counts: p, q widths; r, s rows of L_P inside K / below K; t rows of L_K;
// r', s', t' the same for the columns of U; u, v the sizes of the row and
// column unions of the merged block.  mu = p(p+r+s+r'+s') + q(q+t+t'),
// nu = (p+q)(p+q+u+v); merge when nu <= 1.2 mu or nu <= mu + 2(p+q).
// The merged factors follow from rewriting the 2x2 block product so that
// the merged pivot block absorbs L_{K,P} and U_{P,K}:
//   D^ = [[I, -U_PK], [0, I]] diag(D_P, D_K) [[I, 0], [-X, I]],
//   L^ = [L_P - L_K X, L_K],   W^ = [W_P; W_K + X W_P],
// X = rows of L_P inside K, U_PK = D_P Y, Y = columns of W_P inside K.
// Readings: the lower-left block of the printed merged inverse is
// D^_{k,k-1}; nothing is re-dropped after a merge; widths <= max_block.
bool try_merge(orc_handle* h, int pid, int kid) {
  Block& P = h->blocks[pid];
  Block& K = h->blocks[kid];
  const int p = P.q, q = K.q, w = p + q;
  const i64 fK = K.first, lK = K.last();
  i64 r = 0, s = 0, r2 = 0, s2 = 0;
  for (i64 i : P.R) (i <= lK ? r : s)++;
  for (i64 j : P.C) (j <= lK ? r2 : s2)++;
  i64 t = (i64)K.R.size(), t2 = (i64)K.C.size();
  std::vector<i64> PRb, PCb;
  for (i64 i : P.R)
    if (i > lK) PRb.push_back(i);
  for (i64 j : P.C)
    if (j > lK) PCb.push_back(j);
  std::vector<i64> Ru = union_above(PRb, K.R, lK);
  std::vector<i64> Cu = union_above(PCb, K.C, lK);
  i64 u = (i64)Ru.size(), v = (i64)Cu.size();
  i64 mu = (i64)p * (p + r + s + r2 + s2) + (i64)q * (q + t + t2);
  i64 nu = (i64)w * (w + u + v);
  bool merge = (5 * nu <= 6 * mu || nu <= mu + 2 * w) && w <= h->opt.max_block;
  h->mergelog.insert(h->mergelog.end(), {fK, p, q, mu, nu, merge ? 1 : 0});
  if (!merge) return false;

  // X (q x p): rows of L_P inside K;  Y (p x q): columns of W_P inside K.
  std::vector<double> X((size_t)q * p, 0.0), Y((size_t)p * q, 0.0);
  for (size_t a = 0; a < P.R.size(); ++a)
    if (P.R[a] <= lK)
      for (int c = 0; c < p; ++c) X[(P.R[a] - fK) * p + c] = P.L[a * p + c];
  for (size_t a = 0; a < P.C.size(); ++a)
    if (P.C[a] <= lK)
      for (int c = 0; c < p; ++c) Y[c * q + (P.C[a] - fK)] = P.W[a * p + c];
  // U_PK = D_P Y (p x q);  DX = D_K X (q x p)
  std::vector<double> U((size_t)p * q, 0.0), DX((size_t)q * p, 0.0);
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < q; ++j) {
      double acc = 0.0;
      for (int k = 0; k < p; ++k) acc += P.D[i * p + k] * Y[k * q + j];
      U[i * q + j] = acc;
    }
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < p; ++j) {
      double acc = 0.0;
      for (int k = 0; k < q; ++k) acc += K.D[i * q + k] * X[k * p + j];
      DX[i * p + j] = acc;
    }
  Block M;
  M.first = P.first;
  M.q = w;
  M.D.assign((size_t)w * w, 0.0);
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) {
      double acc = 0.0;
      for (int k = 0; k < q; ++k) acc += U[i * q + k] * DX[k * p + j];
      M.D[i * w + j] = P.D[i * p + j] + acc;
    }
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < q; ++j) {
      double acc = 0.0;
      for (int k = 0; k < q; ++k) acc += U[i * q + k] * K.D[k * q + j];
      M.D[i * w + p + j] = -acc;
    }
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < p; ++j) M.D[(p + i) * w + j] = -DX[i * p + j];
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) M.D[(p + i) * w + p + j] = K.D[i * q + j];
  // merged pivot block S^ = [[S_P, Y], [X S_P, X Y + S_K]] (kept for metrics)
  M.S.assign((size_t)w * w, 0.0);
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < p; ++j) M.S[i * w + j] = P.S[i * p + j];
  for (int i = 0; i < p; ++i)
    for (int j = 0; j < q; ++j) M.S[i * w + p + j] = Y[i * q + j];
  for (int i = 0; i < q; ++i) {
    for (int j = 0; j < p; ++j) {
      double acc = 0.0;
      for (int k = 0; k < p; ++k) acc += X[i * p + k] * P.S[k * p + j];
      M.S[(p + i) * w + j] = acc;
    }
    for (int j = 0; j < q; ++j) {
      double acc = 0.0;
      for (int k = 0; k < p; ++k) acc += X[i * p + k] * Y[k * q + j];
      M.S[(p + i) * w + p + j] = acc + K.S[i * q + j];
    }
  }
  // L^ rows
  M.R = Ru;
  M.L.assign(Ru.size() * w, 0.0);
  {
    size_t a = 0, b = 0;  // cursors into PRb-in-P.R and K.R
    std::vector<i64> pidx;  // position of each P row > lK inside P.R
    for (size_t z = 0; z < P.R.size(); ++z)
      if (P.R[z] > lK) pidx.push_back((i64)z);
    for (size_t z = 0; z < Ru.size(); ++z) {
      i64 i = Ru[z];
      double* out = &M.L[z * w];
      bool inP = a < pidx.size() && P.R[pidx[a]] == i;
      bool inK = b < K.R.size() && K.R[b] == i;
      if (inP)
        for (int c = 0; c < p; ++c) out[c] = P.L[pidx[a] * p + c];
      if (inK) {
        for (int c = 0; c < p; ++c) {
          double acc = 0.0;
          for (int k = 0; k < q; ++k) acc += K.L[b * q + k] * X[k * p + c];
          out[c] -= acc;
        }
        for (int c = 0; c < q; ++c) out[p + c] = K.L[b * q + c];
      }
      if (inP) ++a;
      if (inK) ++b;
    }
  }
  // W^ columns
  M.C = Cu;
  M.W.assign(Cu.size() * w, 0.0);
  {
    size_t a = 0, b = 0;
    std::vector<i64> pidx;
    for (size_t z = 0; z < P.C.size(); ++z)
      if (P.C[z] > lK) pidx.push_back((i64)z);
    for (size_t z = 0; z < Cu.size(); ++z) {
      i64 j = Cu[z];
      double* out = &M.W[z * w];
      bool inP = a < pidx.size() && P.C[pidx[a]] == j;
      bool inK = b < K.C.size() && K.C[b] == j;
      if (inP)
        for (int c = 0; c < p; ++c) out[c] = P.W[pidx[a] * p + c];
      if (inK)
        for (int c = 0; c < q; ++c) out[p + c] = K.W[b * q + c];
      if (inP)
        for (int i = 0; i < q; ++i) {
          double acc = 0.0;
          for (int k = 0; k < p; ++k) acc += X[i * p + k] * P.W[pidx[a] * p + k];
          out[p + i] += acc;
        }
      if (inP) ++a;
      if (inK) ++b;
    }
  }
  h->blocks[pid].alive = false;
  h->blocks[kid].alive = false;
  h->blocks.push_back(std::move(M));
  return true;
}

// ---------------------------------------------------------------------------
// Sec. 2.2: Crout-type block ILU over the given partition, with dropping
// (Alg. 1 in block form), perturbation (Sec. 3.6) and, optionally,
// progressive aggregation after every step (Sec. 3.5).
// ---------------------------------------------------------------------------
// Step K (rows/cols first..last, width q):
//  column panel  C(i,K) = A(i,K) - sum_J L_J(i,:) W_J(:,K)  for i >= first,
//                over live J whose block row has columns inside K,
//  row panel     R(K,j) = A(K,j) - sum_J L_J(K,:) W_J(:,j)  for j > last,
//                over live J whose block column has rows inside K,
//  pivot block   S_K = C(K,K), D_K = S_K^{-1} (perturbed if needed),
//  L(i,K) = C(i,K) D_K  kept iff ||L(i,K)|| > tau,
//  U(K,j) = D_K R(K,j)  kept iff ||U(K,j)|| > tau, stored unscaled W = R.
// Sums run over J in increasing position; candidates are the structural
// entries of A and the stored rows/columns of the contributing J.
int crout_sweep(orc_handle* h) {
  const Mat& a = h->P;
  const i64 n = a.n;
  const orc_options& o = h->opt;
  Mat at = transpose(a);
  h->alpha = 0.0;
  for (double x : a.v) h->alpha = std::max(h->alpha, std::fabs(x));
  std::vector<std::vector<int>> rowOwners(n), colOwners(n);
  std::vector<i64> pos(n, -1);
  h->blocks.clear();
  h->live.clear();
  h->droplog.clear();
  h->mergelog.clear();
  h->n_perturbed = h->n_merges = 0;
  h->singular = 0;
  const i64 nb = (i64)h->start0.size() - 1;
  std::vector<int> preds;
  std::vector<i64> cand;
  for (i64 kb = 0; kb < nb; ++kb) {
    const i64 f = h->start0[kb], l = h->start0[kb + 1] - 1;
    const int q = (int)(l - f + 1);
    // ---------------- column panel
    preds.clear();
    for (i64 c = f; c <= l; ++c)
      for (int id : colOwners[c])
        if (h->blocks[id].alive) preds.push_back(id);
    std::sort(preds.begin(), preds.end(),
              [&](int x, int y) { return h->blocks[x].first < h->blocks[y].first; });
    preds.erase(std::unique(preds.begin(), preds.end()), preds.end());
    cand.clear();
    for (i64 i = f; i <= l; ++i) {
      pos[i] = i - f;
      cand.push_back(i);
    }
    for (i64 c = f; c <= l; ++c)
      for (i64 m = at.rp[c]; m < at.rp[c + 1]; ++m) {
        i64 i = at.ci[m];
        if (i > l && pos[i] < 0) {
          pos[i] = 0;
          cand.push_back(i);
        }
      }
    for (int id : preds)
      for (i64 i : h->blocks[id].R)
        if (i > l && pos[i] < 0) {
          pos[i] = 0;
          cand.push_back(i);
        }
    std::sort(cand.begin() + q, cand.end());
    for (size_t z = 0; z < cand.size(); ++z) pos[cand[z]] = (i64)z;
    std::vector<double> Cp(cand.size() * q, 0.0);
    for (i64 c = f; c <= l; ++c)
      for (i64 m = at.rp[c]; m < at.rp[c + 1]; ++m) {
        i64 i = at.ci[m];
        if (i >= f) Cp[pos[i] * q + (c - f)] = at.v[m];
      }
    for (int id : preds) {
      const Block& J = h->blocks[id];
      const int pJ = J.q;
      for (size_t cj = 0; cj < J.C.size(); ++cj) {
        i64 c = J.C[cj];
        if (c < f || c > l) continue;
        for (size_t ri = 0; ri < J.R.size(); ++ri) {
          i64 i = J.R[ri];
          if (i < f) continue;
          double acc = 0.0;
          for (int t = 0; t < pJ; ++t) acc += J.L[ri * pJ + t] * J.W[cj * pJ + t];
          Cp[pos[i] * q + (c - f)] -= acc;
        }
      }
    }
    // ---------------- row panel
    std::vector<int> rpreds;
    for (i64 r = f; r <= l; ++r)
      for (int id : rowOwners[r])
        if (h->blocks[id].alive) rpreds.push_back(id);
    std::sort(rpreds.begin(), rpreds.end(),
              [&](int x, int y) { return h->blocks[x].first < h->blocks[y].first; });
    rpreds.erase(std::unique(rpreds.begin(), rpreds.end()), rpreds.end());
    std::vector<i64> candc;
    std::vector<i64>& posc = pos;  // reuse after clearing the rows
    for (i64 i : cand) pos[i] = -1;
    for (i64 r = f; r <= l; ++r)
      for (i64 m = a.rp[r]; m < a.rp[r + 1]; ++m) {
        i64 j = a.ci[m];
        if (j > l && posc[j] < 0) {
          posc[j] = 0;
          candc.push_back(j);
        }
      }
    for (int id : rpreds)
      for (i64 j : h->blocks[id].C)
        if (j > l && posc[j] < 0) {
          posc[j] = 0;
          candc.push_back(j);
        }
    std::sort(candc.begin(), candc.end());
    for (size_t z = 0; z < candc.size(); ++z) posc[candc[z]] = (i64)z;
    std::vector<double> Rp(candc.size() * q, 0.0);  // column-major q x |candc|
    for (i64 r = f; r <= l; ++r)
      for (i64 m = a.rp[r]; m < a.rp[r + 1]; ++m) {
        i64 j = a.ci[m];
        if (j > l) Rp[posc[j] * q + (r - f)] = a.v[m];
      }
    for (int id : rpreds) {
      const Block& J = h->blocks[id];
      const int pJ = J.q;
      for (size_t cj = 0; cj < J.C.size(); ++cj) {
        i64 j = J.C[cj];
        if (j <= l) continue;
        for (size_t ri = 0; ri < J.R.size(); ++ri) {
          i64 r = J.R[ri];
          if (r < f || r > l) continue;
          double acc = 0.0;
          for (int t = 0; t < pJ; ++t) acc += J.L[ri * pJ + t] * J.W[cj * pJ + t];
          Rp[posc[j] * q + (r - f)] -= acc;
        }
      }
    }
    for (i64 j : candc) posc[j] = -1;
    // ---------------- pivot block
    Block K;
    K.first = f;
    K.q = q;
    K.computed = true;
    std::vector<double> S((size_t)q * q);
    for (int i = 0; i < q; ++i)
      for (int j = 0; j < q; ++j) S[i * q + j] = Cp[i * q + j];
    int rounds = perturb_invert(q, S, h->alpha, o, K.S, K.D);
    if (rounds < 0) {
      h->singular = 1;
      return 1;
    }
    if (rounds > 0) ++h->n_perturbed;
    // ---------------- scale + drop (column of L)
    std::vector<double> row(q);
    for (size_t z = q; z < cand.size(); ++z) {
      for (int c = 0; c < q; ++c) {
        double acc = 0.0;
        for (int t = 0; t < q; ++t) acc += Cp[z * q + t] * K.D[t * q + c];
        row[c] = acc;
      }
      double nr = drop_norm(row.data(), q, 1, o.drop_norm);
      bool keep = nr > o.tau;
      h->droplog.push_back({kb, cand[z], 0, nr, keep ? 1 : 0});
      if (keep) {
        K.R.push_back(cand[z]);
        K.L.insert(K.L.end(), row.begin(), row.end());
      }
    }
    // ---------------- scale + drop (row of U)
    std::vector<double> col(q);
    for (size_t z = 0; z < candc.size(); ++z) {
      for (int r = 0; r < q; ++r) {
        double acc = 0.0;
        for (int t = 0; t < q; ++t) acc += K.D[r * q + t] * Rp[z * q + t];
        col[r] = acc;
      }
      double nr = drop_norm(col.data(), q, 1, o.drop_norm);
      bool keep = nr > o.tau;
      h->droplog.push_back({kb, candc[z], 1, nr, keep ? 1 : 0});
      if (keep) {
        K.C.push_back(candc[z]);
        K.W.insert(K.W.end(), Rp.begin() + z * q, Rp.begin() + (z + 1) * q);
      }
    }
    // ---------------- register, then aggregate
    int kid = (int)h->blocks.size();
    h->blocks.push_back(std::move(K));
    int cur = kid;
    if (o.use_aggregation && !h->live.empty()) {
      int pid = h->live.back();
      if (try_merge(h, pid, kid)) {
        h->live.pop_back();
        cur = (int)h->blocks.size() - 1;
        ++h->n_merges;
      }
    }
    h->live.push_back(cur);
    const Block& B = h->blocks[cur];
    for (i64 i : B.R) rowOwners[i].push_back(cur);
    for (i64 j : B.C) colOwners[j].push_back(cur);
  }
  return 0;
}

int run_common(orc_handle* h, const orc_options* opt) {
  auto t1 = Clock::now();
  h->start0.clear();
  i64 nu = (i64)h->gstart.size() - 1;
  (void)nu;
  ilu1t_blocks(h->P, h->gstart, h->opt.tau, h->opt.max_block, h->opt.use_ilu1t != 0, h->start0,
               &h->partner);
  auto t2 = Clock::now();
  h->t_ilu1t = std::chrono::duration<double>(t2 - t1).count();
  (void)opt;
  int rc = crout_sweep(h);
  h->t_factor = std::chrono::duration<double>(Clock::now() - t2).count();
  return rc;
}

bool valid_csr(i64 n, const int64_t* rp, const int32_t* ci, const double* v) {
  if (n <= 0 || rp[0] != 0) return false;
  for (i64 i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return false;
    for (i64 k = rp[i]; k < rp[i + 1]; ++k) {
      if (ci[k] < 0 || ci[k] >= n) return false;
      if (k > rp[i] && ci[k] <= ci[k - 1]) return false;
      if (v && !std::isfinite(v[k])) return false;
    }
  }
  return true;
}

}  // namespace

// ---------------------------------------------------------------------------
// C API
// ---------------------------------------------------------------------------
extern "C" {

void orc_default_options(orc_options* o) {
  o->use_cosine = 1;
  o->use_ilu1t = 1;
  o->use_aggregation = 1;
  o->max_block = 128;
  o->tau = 1e-2;
  o->cos_eps = 0.8;
  o->pert_tau = 1e-2;
  o->pert_rho = 1e-1;
  o->pivot_eps = 1e-12;
  o->beta_one = 0;
  o->drop_norm = 0;
  o->sym_perturb = 0;
}

orc_handle* orc_create(void) { return new orc_handle(); }
void orc_destroy(orc_handle* h) { delete h; }

int orc_run(orc_handle* h, int64_t n, const int64_t* rowptr, const int32_t* colind,
            const double* val, const int64_t* pre_perm, const orc_options* opt) {
  return orc_run_units(h, n, rowptr, colind, val, pre_perm, 0, nullptr, nullptr, opt);
}

int orc_run_units(orc_handle* h, int64_t n, const int64_t* rowptr, const int32_t* colind,
                  const double* val, const int64_t* pre_perm, int64_t nunits,
                  const int64_t* unit_starts, const int64_t* partner, const orc_options* opt) {
  if (!valid_csr(n, rowptr, colind, val)) return -1;
  if (unit_starts) {
    if (nunits < 1 || unit_starts[0] != 0 || unit_starts[nunits] != n) return -1;
    for (i64 u = 0; u < nunits; ++u)
      if (unit_starts[u + 1] <= unit_starts[u]) return -1;
  }
  h->partner.clear();
  auto t0 = Clock::now();
  h->opt = *opt;
  h->n = n;
  h->A = from_csr(n, rowptr, colind, val);
  std::vector<i64> pre(n);
  for (i64 i = 0; i < n; ++i) pre[i] = pre_perm ? pre_perm[i] : i;
  Mat A1 = permute_sym(h->A, pre);
  std::vector<i64> q, gs;
  if (unit_starts) {
    // Sec. 5: the groups are formed on the compressed companion matrix and
    // expanded; without the cosine step every unit is a group
    std::vector<i64> us(unit_starts, unit_starts + nunits + 1), width(nunits), qu, gu;
    for (i64 u = 0; u < nunits; ++u) width[u] = us[u + 1] - us[u];
    if (opt->use_cosine) {
      cosine_groups(compress_units(A1, us), opt->cos_eps, opt->max_block, qu, gu,
                    &h->n_ignored, &width);
    } else {
      qu.resize(nunits);
      gu.resize(nunits + 1);
      for (i64 u = 0; u < nunits; ++u) qu[u] = u;
      for (i64 u = 0; u <= nunits; ++u) gu[u] = u;
      h->n_ignored = 0;
    }
    gs.assign(1, 0);
    for (size_t g = 0; g + 1 < gu.size(); ++g) {
      for (i64 k = gu[g]; k < gu[g + 1]; ++k)
        for (i64 i = us[qu[k]]; i < us[qu[k] + 1]; ++i) q.push_back(i);
      gs.push_back((i64)q.size());
    }
    // the 2x2 pivots in the final numbering (the groups keep the group
    // order, so q is that numbering): the units of two scalars, unless the
    // caller gives them
    if (partner) {
      h->partner.assign(partner, partner + n);
    } else {
      std::vector<i64> qinv(n);
      for (i64 i = 0; i < n; ++i) qinv[q[i]] = i;
      h->partner.assign(n, -1);
      for (i64 u = 0; u < nunits; ++u)
        if (us[u + 1] - us[u] == 2) {
          const i64 p0 = qinv[us[u]], p1 = qinv[us[u] + 1];
          h->partner[p0] = p1;
          h->partner[p1] = p0;
        }
    }
  } else if (opt->use_cosine) {
    cosine_groups(A1, opt->cos_eps, opt->max_block, q, gs, &h->n_ignored);
  } else {
    q.resize(n);
    gs.resize(n + 1);
    for (i64 i = 0; i < n; ++i) q[i] = i;
    for (i64 i = 0; i <= n; ++i) gs[i] = i;
    h->n_ignored = 0;
  }
  // Sec. 3.3: groups kept contiguous; the group order is the natural one
  // (the caller's pre-permutation carries any fill-reducing ordering).
  h->perm.resize(n);
  for (i64 i = 0; i < n; ++i) h->perm[i] = pre[q[i]];
  h->gstart = gs;
  h->P = permute_sym(h->A, h->perm);
  h->t_analyze = std::chrono::duration<double>(Clock::now() - t0).count();
  return run_common(h, opt);
}

int orc_run_partition(orc_handle* h, int64_t n, const int64_t* rowptr, const int32_t* colind,
                      const double* val, const int64_t* perm, int64_t nblocks,
                      const int64_t* starts, const orc_options* opt) {
  if (!valid_csr(n, rowptr, colind, val)) return -1;
  if (starts[0] != 0 || starts[nblocks] != n) return -1;
  for (i64 b = 0; b < nblocks; ++b)
    if (starts[b + 1] <= starts[b]) return -1;
  h->opt = *opt;
  h->n = n;
  h->partner.clear();
  h->A = from_csr(n, rowptr, colind, val);
  h->perm.resize(n);
  for (i64 i = 0; i < n; ++i) h->perm[i] = perm ? perm[i] : i;
  h->P = permute_sym(h->A, h->perm);
  h->gstart.assign(starts, starts + nblocks + 1);
  h->start0.assign(starts, starts + nblocks + 1);
  auto t2 = Clock::now();
  int rc = crout_sweep(h);
  h->t_factor = std::chrono::duration<double>(Clock::now() - t2).count();
  return rc;
}

int64_t orc_cosine(int64_t n, const int64_t* rowptr, const int32_t* colind, double cos_eps,
                   int max_block, int64_t* perm, int64_t* group_starts, int64_t* n_ignored) {
  Mat a = from_csr(n, rowptr, colind, nullptr);
  std::vector<i64> p, g;
  i64 ng = cosine_groups(a, cos_eps, max_block, p, g, n_ignored);
  std::copy(p.begin(), p.end(), perm);
  std::copy(g.begin(), g.end(), group_starts);
  return ng;
}

int64_t orc_ilu1t(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* val,
                  int64_t nunits, const int64_t* unit_starts, double tau, int max_block,
                  int64_t* block_starts) {
  Mat a = from_csr(n, rowptr, colind, val);
  std::vector<i64> us(unit_starts, unit_starts + nunits + 1), bs;
  i64 nb = ilu1t_blocks(a, us, tau, max_block, true, bs);
  std::copy(bs.begin(), bs.end(), block_starts);
  return nb;
}

int64_t orc_ilu1t_sets(int64_t n, const int64_t* rowptr, const int32_t* colind,
                        const double* val, int64_t k, double tau, int64_t* I, int64_t* nI,
                        int64_t* J, int64_t* nJ) {
  Mat a = from_csr(n, rowptr, colind, val);
  Mat at = transpose(a);
  std::vector<double> dg(n, 0.0);
  for (i64 i = 0; i < n; ++i) dg[i] = entry(a, i, i);
  Ilu1tSets st = ilu1t_sets(a, at, dg, k, tau);
  *nI = (int64_t)st.I.size();
  *nJ = (int64_t)st.J.size();
  if (I) std::copy(st.I.begin(), st.I.end(), I);
  if (J) std::copy(st.J.begin(), st.J.end(), J);
  return *nI + *nJ;
}

int orc_perturb_invert(int q, const double* s, double alpha, const orc_options* opt,
                       double* s_used, double* dinv) {
  std::vector<double> m(s, s + (size_t)q * q), su, di;
  int r = perturb_invert(q, m, alpha, *opt, su, di);
  if (r >= 0) {
    std::copy(su.begin(), su.end(), s_used);
    std::copy(di.begin(), di.end(), dinv);
  }
  return r;
}

int64_t orc_n(const orc_handle* h) { return h->n; }
int64_t orc_nblocks(const orc_handle* h) { return (int64_t)h->live.size(); }
int64_t orc_nblocks_initial(const orc_handle* h) { return (int64_t)h->start0.size() - 1; }

void orc_get_perm(const orc_handle* h, int64_t* perm) {
  std::copy(h->perm.begin(), h->perm.end(), perm);
}
void orc_get_starts(const orc_handle* h, int64_t* starts) {
  size_t k = 0;
  for (int id : h->live) starts[k++] = h->blocks[id].first;
  starts[k] = h->n;
}
void orc_get_starts_initial(const orc_handle* h, int64_t* starts) {
  std::copy(h->start0.begin(), h->start0.end(), starts);
}
void orc_get_group_starts(const orc_handle* h, int64_t* starts, int64_t* ngroups) {
  *ngroups = (int64_t)h->gstart.size() - 1;
  if (starts) std::copy(h->gstart.begin(), h->gstart.end(), starts);
}
void orc_get_counts(const orc_handle* h, int64_t* nR, int64_t* nC) {
  size_t k = 0;
  for (int id : h->live) {
    nR[k] = (int64_t)h->blocks[id].R.size();
    nC[k] = (int64_t)h->blocks[id].C.size();
    ++k;
  }
}
void orc_get_factors(const orc_handle* h, int64_t* R, double* L, int64_t* C, double* W,
                     double* D) {
  for (int id : h->live) {
    const Block& B = h->blocks[id];
    R = std::copy(B.R.begin(), B.R.end(), R);
    L = std::copy(B.L.begin(), B.L.end(), L);
    C = std::copy(B.C.begin(), B.C.end(), C);
    W = std::copy(B.W.begin(), B.W.end(), W);
    D = std::copy(B.D.begin(), B.D.end(), D);
  }
}
void orc_get_stats(const orc_handle* h, int64_t* out) {
  for (int k = 0; k < 16; ++k) out[k] = 0;
  int64_t nnzL = 0, nnzW = 0, nnzD = 0, maxw = 0;
  for (int id : h->live) {
    const Block& B = h->blocks[id];
    nnzL += (int64_t)B.R.size() * B.q;
    nnzW += (int64_t)B.C.size() * B.q;
    nnzD += (int64_t)B.q * B.q;
    maxw = std::max<int64_t>(maxw, B.q);
  }
  out[0] = (int64_t)h->start0.size() - 1;
  out[1] = (int64_t)h->live.size();
  out[2] = h->n_merges;
  out[3] = h->n_perturbed;
  out[4] = nnzL;
  out[5] = nnzW;
  out[6] = nnzD;
  out[7] = maxw;
  out[8] = (int64_t)h->gstart.size() - 1;
  out[9] = h->n_ignored;
  out[10] = h->singular;
  out[11] = (int64_t)h->A.rp[h->n];
}
int64_t orc_get_droplog(const orc_handle* h, int64_t* block, int64_t* index, int32_t* kind,
                        double* norm, int32_t* kept) {
  size_t k = 0;
  if (block)
    for (const DropRec& d : h->droplog) {
      block[k] = d.block;
      index[k] = d.index;
      kind[k] = d.kind;
      norm[k] = d.norm;
      kept[k] = d.kept;
      ++k;
    }
  return (int64_t)h->droplog.size();
}
int64_t orc_get_mergelog(const orc_handle* h, int64_t* rec) {
  if (rec) std::copy(h->mergelog.begin(), h->mergelog.end(), rec);
  return (int64_t)h->mergelog.size() / 6;
}

// Sec. 3.7 with D_l = D_r = Pi = I:  M = P (L S U) P^T,  y = M^{-1} x.
// Forward:  t_K = x_K - sum_{J<K} L_{K,J} t_J   (L unit),
// backward: z_K = D_K (t_K - sum_{j in C_K} W_K(:,j) z_j)  (U = D W).
void orc_apply(const orc_handle* h, const double* x, double* y) {
  const i64 n = h->n;
  std::vector<double> t(n);
  for (i64 i = 0; i < n; ++i) t[i] = x[h->perm[i]];
  for (int id : h->live) {
    const Block& B = h->blocks[id];
    for (size_t ri = 0; ri < B.R.size(); ++ri) {
      double acc = 0.0;
      for (int c = 0; c < B.q; ++c) acc += B.L[ri * B.q + c] * t[B.first + c];
      t[B.R[ri]] -= acc;
    }
  }
  std::vector<double> z(n, 0.0), v;
  for (auto it = h->live.rbegin(); it != h->live.rend(); ++it) {
    const Block& B = h->blocks[*it];
    v.assign(t.begin() + B.first, t.begin() + B.first + B.q);
    for (size_t cj = 0; cj < B.C.size(); ++cj)
      for (int r = 0; r < B.q; ++r) v[r] -= B.W[cj * B.q + r] * z[B.C[cj]];
    for (int r = 0; r < B.q; ++r) {
      double acc = 0.0;
      for (int c = 0; c < B.q; ++c) acc += B.D[r * B.q + c] * v[c];
      z[B.first + r] = acc;
    }
  }
  for (i64 i = 0; i < n; ++i) y[h->perm[i]] = z[i];
}

}  // extern "C"

namespace {

void spmv(const Mat& a, const double* x, double* y) {
  for (i64 i = 0; i < a.n; ++i) {
    double acc = 0.0;
    for (i64 k = a.rp[i]; k < a.rp[i + 1]; ++k) acc += a.v[k] * x[a.ci[k]];
    y[i] = acc;
  }
}

double dot(const std::vector<double>& x, const std::vector<double>& y) {
  double acc = 0.0;
  for (size_t i = 0; i < x.size(); ++i) acc += x[i] * y[i];
  return acc;
}

// Restarted flexible GMRES (Saad, SIAM J. Sci. Comput. 14, 1993) with right
// preconditioning, modified Gram-Schmidt and Givens rotations.  The Givens
// estimate is checked after every Arnoldi step; a cycle that meets it is
// confirmed with the true residual and restarted if that is not met.
// Happy breakdown: h_{j+1,j} <= 1e-14 ||A z_j||.
template <class Prec>
void fgmres(const Mat& a, Prec prec, const double* b, double* x, int m, double rtol, int maxit,
            orc_solve_info* info, double* hist) {
  const i64 n = a.n;
  std::vector<double> bb(b, b + n);
  const double bnorm = std::sqrt(dot(bb, bb));
  std::vector<std::vector<double>> V(m + 1, std::vector<double>(n)), Z(m, std::vector<double>(n));
  std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), yv(m), r(n), w(n);
  i64 it = 0, cycles = 0;
  int converged = 0;
  const double target = rtol * bnorm;
  while (true) {
    spmv(a, x, r.data());
    for (i64 i = 0; i < n; ++i) r[i] = b[i] - r[i];
    double beta = std::sqrt(dot(r, r));
    if (beta <= target) {
      converged = 1;
      break;
    }
    if (it >= maxit) break;
    ++cycles;
    for (i64 i = 0; i < n; ++i) V[0][i] = r[i] / beta;
    std::fill(g.begin(), g.end(), 0.0);
    g[0] = beta;
    int jend = 0;
    for (int j = 0; j < m; ++j) {
      prec(V[j].data(), Z[j].data());
      spmv(a, Z[j].data(), w.data());
      double wn0 = std::sqrt(dot(w, w));
      for (int i = 0; i <= j; ++i) {
        double hij = dot(w, V[i]);
        H[i * m + j] = hij;
        for (i64 k = 0; k < n; ++k) w[k] -= hij * V[i][k];
      }
      double hn = std::sqrt(dot(w, w));
      H[(j + 1) * m + j] = hn;
      ++it;
      for (int i = 0; i < j; ++i) {
        double t1 = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
        H[(i + 1) * m + j] = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
        H[i * m + j] = t1;
      }
      double aa = H[j * m + j], bv = H[(j + 1) * m + j];
      if (bv == 0.0) {
        cs[j] = 1.0;
        sn[j] = 0.0;
      } else if (std::fabs(bv) > std::fabs(aa)) {
        double t1 = aa / bv;
        sn[j] = 1.0 / std::sqrt(1.0 + t1 * t1);
        cs[j] = sn[j] * t1;
      } else {
        double t1 = bv / aa;
        cs[j] = 1.0 / std::sqrt(1.0 + t1 * t1);
        sn[j] = cs[j] * t1;
      }
      H[j * m + j] = cs[j] * aa + sn[j] * bv;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      double est = std::fabs(g[j + 1]);
      if (hist) hist[it - 1] = est;
      bool breakdown = hn <= 1e-14 * wn0;
      if (!breakdown)
        for (i64 k = 0; k < n; ++k) V[j + 1][k] = w[k] / hn;
      jend = j + 1;
      if (est <= target || breakdown || it >= maxit) break;
    }
    for (int i = jend - 1; i >= 0; --i) {
      double acc = g[i];
      for (int k = i + 1; k < jend; ++k) acc -= H[i * m + k] * yv[k];
      yv[i] = acc / H[i * m + i];
    }
    for (int i = 0; i < jend; ++i)
      for (i64 k = 0; k < n; ++k) x[k] += yv[i] * Z[i][k];
  }
  spmv(a, x, r.data());
  for (i64 i = 0; i < n; ++i) r[i] = b[i] - r[i];
  info->iterations = it;
  info->restarts = cycles;
  info->rel_residual = std::sqrt(dot(r, r)) / bnorm;
  info->converged = converged;
}


double norm_inf(const double* v, i64 n) {
  double m = 0.0;
  for (i64 i = 0; i < n; ++i) m = std::max(m, std::fabs(v[i]));
  return m;
}

// ||A||_inf: the largest row sum of magnitudes.
double mat_norm_inf(const Mat& a) {
  double m = 0.0;
  for (i64 i = 0; i < a.n; ++i) {
    double s = 0.0;
    for (i64 k = a.rp[i]; k < a.rp[i + 1]; ++k) s += std::fabs(a.v[k]);
    m = std::max(m, s);
  }
  return m;
}

// Normwise backward error of x in the infinity norm (Rigal and Gaches,
// J. ACM 14, 1967): the smallest eta with (A + E) x = b + f,
// ||E|| <= eta ||A||, ||f|| <= eta ||b||.  0 when the residual is 0.
double backward_error(double rmax, double anorm, double xmax, double bmax) {
  if (rmax == 0.0) return 0.0;
  return rmax / (anorm * xmax + bmax);
}

// Simplified QMR (Freund and Nachtigal 1995; Freund and Jarre 1997), the
// Krylov solver of Sec. 5 for symmetric A with a symmetric, possibly
// indefinite preconditioner M (the preconditioner splits as M1 = I,
// M2 = M).  One product with A and one application of M^{-1} per step;
// r is the Lanczos (BiCG) residual, tau the quasi-residual norm, and
// ||b - A x_k||_2 <= sqrt(k + 1) tau_k.  The QMR residual b - A x is kept
// by the recurrence rq -= A d, with A d = cd (A d_old) + cq (A q).
// Stopping test: the backward error eta of x on the updated QMR residual,
// confirmed with the true residual (Reading: Sec. 5 names the backward
// error and the tolerance 1e-6, not its norm; it is taken in the infinity
// norm).  Breakdown (q^T A q = 0 or r^T M^{-1} r = 0) stops the solve.
// hist (may be NULL): tau_k after step k.
template <class Prec>
void sqmr(const Mat& a, Prec prec, const double* b, double* x, double tol, int maxit,
          orc_solve_info* info, double* eta_out, double* hist) {
  const i64 n = a.n;
  std::vector<double> r(n), rq(n), q(n), t(n), u(n), d(n, 0.0), s(n, 0.0), tr(n);
  const double anorm = mat_norm_inf(a);
  const double bmax = norm_inf(b, n);
  spmv(a, x, r.data());
  for (i64 i = 0; i < n; ++i) r[i] = b[i] - r[i];
  rq = r;
  double eta = backward_error(norm_inf(rq.data(), n), anorm, norm_inf(x, n), bmax);
  i64 it = 0;
  int converged = eta <= tol ? 1 : 0;
  if (!converged && maxit > 0) {
    double tau = std::sqrt(dot(r, r));
    prec(r.data(), q.data());
    double theta = 0.0;
    double rho = dot(r, q);
    while (true) {
      spmv(a, q.data(), t.data());
      const double sigma = dot(q, t);
      if (sigma == 0.0) break;
      const double alpha = rho / sigma;
      for (i64 i = 0; i < n; ++i) r[i] -= alpha * t[i];
      const double theta_old = theta;
      theta = std::sqrt(dot(r, r)) / tau;
      const double c = 1.0 / std::sqrt(1.0 + theta * theta);
      const double c2 = c * c;
      tau = tau * theta * c;
      const double cd = c2 * theta_old * theta_old, cq = c2 * alpha;
      for (i64 i = 0; i < n; ++i) {
        d[i] = cd * d[i] + cq * q[i];
        s[i] = cd * s[i] + cq * t[i];
        x[i] += d[i];
        rq[i] -= s[i];
      }
      ++it;
      if (hist) hist[it - 1] = tau;
      eta = backward_error(norm_inf(rq.data(), n), anorm, norm_inf(x, n), bmax);
      if (eta <= tol) {
        spmv(a, x, tr.data());
        for (i64 i = 0; i < n; ++i) tr[i] = b[i] - tr[i];
        if (backward_error(norm_inf(tr.data(), n), anorm, norm_inf(x, n), bmax) <= tol) {
          converged = 1;
          break;
        }
      }
      if (it >= maxit || rho == 0.0) break;
      prec(r.data(), u.data());
      const double rho_new = dot(r, u);
      const double beta = rho_new / rho;
      rho = rho_new;
      for (i64 i = 0; i < n; ++i) q[i] = u[i] + beta * q[i];
    }
  }
  spmv(a, x, tr.data());
  for (i64 i = 0; i < n; ++i) tr[i] = b[i] - tr[i];
  std::vector<double> bb(b, b + n);
  const double bnorm = std::sqrt(dot(bb, bb));
  info->iterations = it;
  info->restarts = 0;
  info->rel_residual = bnorm > 0.0 ? std::sqrt(dot(tr, tr)) / bnorm : 0.0;
  info->converged = converged;
  if (eta_out) *eta_out = backward_error(norm_inf(tr.data(), n), anorm, norm_inf(x, n), bmax);
}

}  // namespace

extern "C" {

void orc_fgmres(const orc_handle* h, const double* b, double* x, int restart, double rtol,
                int maxit, orc_solve_info* info) {
  orc_fgmres_hist(h, b, x, restart, rtol, maxit, info, nullptr);
}

void orc_fgmres_hist(const orc_handle* h, const double* b, double* x, int restart, double rtol,
                     int maxit, orc_solve_info* info, double* resid_history) {
  fgmres(
      h->A, [h](const double* in, double* out) { orc_apply(h, in, out); }, b, x, restart, rtol,
      maxit, info, resid_history);
}

void orc_fgmres_plain(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* val,
                      const double* b, double* x, int restart, double rtol, int maxit,
                      orc_solve_info* info, double* resid_history) {
  Mat a = from_csr(n, rowptr, colind, val);
  fgmres(
      a, [n](const double* in, double* out) { std::copy(in, in + n, out); }, b, x, restart, rtol,
      maxit, info, resid_history);
}

void orc_sqmr(const orc_handle* h, const double* b, double* x, double tol, int maxit,
              orc_solve_info* info, double* eta, double* tau_history) {
  sqmr(
      h->A, [h](const double* in, double* out) { orc_apply(h, in, out); }, b, x, tol, maxit,
      info, eta, tau_history);
}

void orc_sqmr_plain(int64_t n, const int64_t* rowptr, const int32_t* colind, const double* val,
                    const double* b, double* x, double tol, int maxit, orc_solve_info* info,
                    double* eta, double* tau_history) {
  Mat a = from_csr(n, rowptr, colind, val);
  sqmr(
      a, [n](const double* in, double* out) { std::copy(in, in + n, out); }, b, x, tol, maxit,
      info, eta, tau_history);
}

// (L S U) x in the permuted numbering: W = S U is the non-unit upper factor
// with W(K,K) = S_K, so L S U x = L (W x).
void orc_lsu_matvec(const orc_handle* h, const double* x, double* y) {
  const i64 n = h->n;
  std::vector<double> v(n, 0.0);
  for (int id : h->live) {
    const Block& B = h->blocks[id];
    for (int r = 0; r < B.q; ++r) {
      double acc = 0.0;
      for (int c = 0; c < B.q; ++c) acc += B.S[r * B.q + c] * x[B.first + c];
      for (size_t cj = 0; cj < B.C.size(); ++cj) acc += B.W[cj * B.q + r] * x[B.C[cj]];
      v[B.first + r] = acc;
    }
  }
  std::copy(v.begin(), v.end(), y);
  for (int id : h->live) {
    const Block& B = h->blocks[id];
    for (size_t ri = 0; ri < B.R.size(); ++ri) {
      double acc = 0.0;
      for (int c = 0; c < B.q; ++c) acc += B.L[ri * B.q + c] * v[B.first + c];
      y[B.R[ri]] += acc;
    }
  }
}

// ||(L S U - A)_Omega||_F / ||A||_F, Omega = diagonal blocks, R_K x K, K x C_K
// of the blocks as the sweep computed them (before any merge: merged blocks
// also store zero-filled positions whose values were dropped).  L S U is
// taken from the final (merged) factors; entry (i,j) of L W is the sparse
// dot product of row i of L with column j of W.
namespace {
// ||(L S U - A)_Omega||_F / ||A||_F; Omega: the positions of the blocks the
// sweep computed (before merges), or of the final blocks (live).
double omega_residual(const orc_handle* h, bool live) {
  const i64 n = h->n;
  std::vector<std::vector<std::pair<i64, double>>> Lrow(n), Wcol(n);
  for (i64 i = 0; i < n; ++i) Lrow[i].push_back({i, 1.0});
  for (int id : h->live) {
    const Block& B = h->blocks[id];
    for (size_t ri = 0; ri < B.R.size(); ++ri)
      for (int c = 0; c < B.q; ++c) Lrow[B.R[ri]].push_back({B.first + c, B.L[ri * B.q + c]});
    for (int c = 0; c < B.q; ++c)
      for (int r = 0; r < B.q; ++r) Wcol[B.first + c].push_back({B.first + r, B.S[r * B.q + c]});
    for (size_t cj = 0; cj < B.C.size(); ++cj)
      for (int r = 0; r < B.q; ++r) Wcol[B.C[cj]].push_back({B.first + r, B.W[cj * B.q + r]});
  }
  auto cmp = [](const std::pair<i64, double>& x, const std::pair<i64, double>& y) {
    return x.first < y.first;
  };
  for (i64 i = 0; i < n; ++i) {
    std::sort(Lrow[i].begin(), Lrow[i].end(), cmp);
    std::sort(Wcol[i].begin(), Wcol[i].end(), cmp);
  }
  auto lw = [&](i64 i, i64 j) {
    const auto& x = Lrow[i];
    const auto& y = Wcol[j];
    size_t p = 0, q = 0;
    double acc = 0.0;
    while (p < x.size() && q < y.size()) {
      if (x[p].first < y[q].first)
        ++p;
      else if (y[q].first < x[p].first)
        ++q;
      else
        acc += x[p++].second * y[q++].second;
    }
    return acc;
  };
  double num = 0.0, den = 0.0;
  for (double x : h->A.v) den += x * x;
  const Mat& a = h->P;
  std::vector<char> is_live(h->blocks.size(), 0);
  for (int id : h->live) is_live[id] = 1;
  for (size_t id = 0; id < h->blocks.size(); ++id) {
    const Block& B = h->blocks[id];
    if (live ? !is_live[id] : !B.computed) continue;
    for (int r = 0; r < B.q; ++r)
      for (int c = 0; c < B.q; ++c) {
        double d = lw(B.first + r, B.first + c) - entry(a, B.first + r, B.first + c);
        num += d * d;
      }
    for (i64 i : B.R)
      for (int c = 0; c < B.q; ++c) {
        double d = lw(i, B.first + c) - entry(a, i, B.first + c);
        num += d * d;
      }
    for (i64 j : B.C)
      for (int r = 0; r < B.q; ++r) {
        double d = lw(B.first + r, j) - entry(a, B.first + r, j);
        num += d * d;
      }
  }
  return std::sqrt(num / den);
}
}  // namespace

double orc_kept_residual(const orc_handle* h) { return omega_residual(h, false); }
double orc_final_residual(const orc_handle* h) { return omega_residual(h, true); }

// Refactorization with frozen patterns (a variant for sequences of matrices
// with one pattern, not a step of the paper): the final blocks and their
// lists R_K, C_K stay, the values follow the new A.  For K in order, the
// Crout panels of Sec. 2.2 on the stored positions only,
//   C(i, j) = A(i, j) - sum over earlier final blocks J of L_J(i,:) W_J(:,j),
// the sum over the J whose lists hold both i (R_J) and j (C_J), in order;
// then S_K = C(K, K) perturbed and inverted as in the sweep (Sec. 3.6),
// L_K = C(R_K, K) D_K and W_K = C(K, C_K).  Nothing is dropped or merged.
int orc_refactor_frozen(orc_handle* h, const double* val) {
  if (h->live.empty()) return -1;
  for (size_t e = 0; e < h->A.v.size(); ++e) {
    if (!std::isfinite(val[e])) return -1;
  }
  std::copy(val, val + h->A.v.size(), h->A.v.begin());
  h->P = permute_sym(h->A, h->perm);
  const Mat& a = h->P;
  const orc_options& o = h->opt;
  h->alpha = 0.0;
  for (double x : a.v) h->alpha = std::max(h->alpha, std::fabs(x));
  h->n_perturbed = 0;
  h->singular = 0;
  std::vector<int> order(h->live.begin(), h->live.end());
  for (size_t k = 0; k < order.size(); ++k) {
    Block& K = h->blocks[order[k]];
    const int q = K.q;
    const i64 f = K.first, l = K.last();
    const size_t nR = K.R.size(), nC = K.C.size();
    // panel rows: K's own, then R_K; row panel columns: C_K
    auto rowpos = [&](i64 i) -> i64 {
      if (i >= f && i <= l) return i - f;
      auto it = std::lower_bound(K.R.begin(), K.R.end(), i);
      return it != K.R.end() && *it == i ? q + (i64)(it - K.R.begin()) : -1;
    };
    auto colpos = [&](i64 j) -> i64 {
      auto it = std::lower_bound(K.C.begin(), K.C.end(), j);
      return it != K.C.end() && *it == j ? (i64)(it - K.C.begin()) : -1;
    };
    std::vector<double> Cp((q + nR) * (size_t)q), Rp((size_t)q * nC);
    for (int r = 0; r < q; ++r)
      for (int c = 0; c < q; ++c) Cp[(size_t)r * q + c] = entry(a, f + r, f + c);
    for (size_t t = 0; t < nR; ++t)
      for (int c = 0; c < q; ++c) Cp[(q + t) * q + c] = entry(a, K.R[t], f + c);
    for (int r = 0; r < q; ++r)
      for (size_t t = 0; t < nC; ++t) Rp[(size_t)r * nC + t] = entry(a, f + r, K.C[t]);
    for (size_t jb = 0; jb < k; ++jb) {
      const Block& J = h->blocks[order[jb]];
      const int p = J.q;
      auto term = [&](size_t tr, size_t tc) {
        double acc = 0.0;
        for (int u = 0; u < p; ++u) acc += J.L[tr * p + u] * J.W[tc * p + u];
        return acc;
      };
      for (size_t tc = 0; tc < J.C.size(); ++tc) {
        const i64 j = J.C[tc];
        if (j < f) continue;
        const bool in_k = j <= l;
        const i64 cj = in_k ? -1 : colpos(j);
        if (!in_k && cj < 0) continue;
        for (size_t tr = 0; tr < J.R.size(); ++tr) {
          const i64 i = J.R[tr];
          if (in_k) {  // column panel: rows of K and R_K
            const i64 ri = rowpos(i);
            if (ri >= 0) Cp[(size_t)ri * q + (j - f)] -= term(tr, tc);
          } else if (i >= f && i <= l) {  // row panel: rows of K
            Rp[(size_t)(i - f) * nC + cj] -= term(tr, tc);
          }
        }
      }
    }
    std::vector<double> S(Cp.begin(), Cp.begin() + (size_t)q * q);
    const int rounds = perturb_invert(q, S, h->alpha, o, K.S, K.D);
    if (rounds < 0) {
      h->singular = 1;
      return 1;
    }
    if (rounds > 0) ++h->n_perturbed;
    for (size_t t = 0; t < nR; ++t)
      for (int c = 0; c < q; ++c) {
        double acc = 0.0;
        for (int u = 0; u < q; ++u) acc += Cp[(q + t) * q + u] * K.D[(size_t)u * q + c];
        K.L[t * q + c] = acc;
      }
    for (size_t t = 0; t < nC; ++t)
      for (int r = 0; r < q; ++r) K.W[t * q + r] = Rp[(size_t)r * nC + t];
  }
  return 0;
}

// Test hook of the pins, not part of the method: adds delta to the stored
// value pos of L_K (which = 0, row-major) or W_K (which = 1, column-major) of
// final block k, so that a pin can show the kept-pattern residual responds
// to a defect.  Returns 0, or -1 when the position does not exist.
int orc_plant(orc_handle* h, int which, int64_t k, int64_t pos, double delta) {
  if (k < 0 || k >= (int64_t)h->live.size()) return -1;
  Block& B = h->blocks[h->live[k]];
  std::vector<double>& v = which == 0 ? B.L : B.W;
  if (which < 0 || which > 1 || pos < 0 || pos >= (int64_t)v.size()) return -1;
  v[pos] += delta;
  return 0;
}

void orc_get_times(const orc_handle* h, double* t3) {
  t3[0] = h->t_analyze;
  t3[1] = h->t_ilu1t;
  t3[2] = h->t_factor;
}

}  // extern "C"
