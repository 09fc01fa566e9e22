// Maximum weight matching of Sec. 3.1 (eq. (mwm)) on the host.
//
// A maximum product transversal maximizes prod_i |a_{i,sigma(i)}|.  With
// colmax_j = max_i |a_ij| and c_ij = log(colmax_j) - log|a_ij| >= 0 on the
// nonzero entries it is the linear assignment problem min sum c_{i,sigma(i)},
// solved here by successive shortest augmenting paths: duals u (rows) and
// v (columns) keep every reduced cost c_ij - u_i - v_j non-negative; a greedy
// pass first matches rows along zero reduced costs, then for every row left
// Dijkstra over alternating paths finds the nearest free column, the duals of
// the rows and columns reached before it move by their distance deficit
// (keeping reduced costs non-negative and making the path tight), and the
// path is flipped.  D_l = exp(u), D_r = exp(v) / colmax then give
// |(D_l A D_r)_ij| = exp(u_i + v_j - c_ij) <= 1, with equality on the
// matching.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <queue>
#include <vector>

#include "internal.h"

namespace bilu {

bilu_status mwm_host(int64_t n, const int64_t* rp, const int32_t* ci, const double* val,
                     int64_t* sigma, double* dl, double* dr, std::string* why) {
  std::vector<double> colmax(n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t m = rp[i]; m < rp[i + 1]; ++m) {
      if (ci[m] < 0 || ci[m] >= n) {
        *why = "column index out of range";
        return BILU_ERR_INVALID;
      }
      colmax[ci[m]] = std::max(colmax[ci[m]], std::fabs(val[m]));
    }
  for (int64_t j = 0; j < n; ++j)
    if (!(colmax[j] > 0.0) || !std::isfinite(colmax[j])) {
      *why = "a column without finite nonzero entries";
      return BILU_ERR_SINGULAR;
    }
  // costs of the nonzero entries, row by row
  std::vector<int64_t> ptr(n + 1, 0);
  std::vector<int32_t> col;
  std::vector<double> cost;
  col.reserve(rp[n]);
  cost.reserve(rp[n]);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t m = rp[i]; m < rp[i + 1]; ++m) {
      const double x = std::fabs(val[m]);
      if (x != 0.0) {
        col.push_back(ci[m]);
        cost.push_back(std::log(colmax[ci[m]]) - std::log(x));
      }
    }
    ptr[i + 1] = (int64_t)col.size();
  }
  std::vector<double> u(n), v(n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    if (ptr[i] == ptr[i + 1]) {
      *why = "a row without nonzero entries";
      return BILU_ERR_SINGULAR;
    }
    double mn = cost[ptr[i]];
    for (int64_t m = ptr[i] + 1; m < ptr[i + 1]; ++m) mn = std::min(mn, cost[m]);
    u[i] = mn;
  }
  std::vector<int64_t> row_of(n, -1), col_of(n, -1);
  // greedy: a zero reduced cost to a free column
  for (int64_t i = 0; i < n; ++i)
    for (int64_t m = ptr[i]; m < ptr[i + 1]; ++m) {
      const int32_t j = col[m];
      if (row_of[j] < 0 && cost[m] - u[i] - v[j] <= 0.0) {
        row_of[j] = i;
        col_of[i] = j;
        break;
      }
    }
  // shortest augmenting paths for the rows left
  std::vector<double> dist(n), fin(n);
  std::vector<int64_t> pred(n);
  std::vector<int64_t> stamp(n, -1), done_stamp(n, -1), row_stamp(n, -1);
  std::vector<double> d_row(n);
  std::vector<int64_t> touched_cols, touched_rows;
  using Item = std::pair<double, int64_t>;
  std::priority_queue<Item, std::vector<Item>, std::greater<Item>> heap;
  for (int64_t r = 0; r < n; ++r) {
    if (col_of[r] >= 0) continue;
    touched_cols.clear();
    touched_rows.clear();
    while (!heap.empty()) heap.pop();
    row_stamp[r] = r;
    d_row[r] = 0.0;
    touched_rows.push_back(r);
    auto relax = [&](int64_t i, double di) {
      for (int64_t m = ptr[i]; m < ptr[i + 1]; ++m) {
        const int32_t k = col[m];
        if (done_stamp[k] == r) continue;
        const double nd = di + cost[m] - u[i] - v[k];
        if (stamp[k] != r || nd < dist[k]) {
          stamp[k] = r;
          dist[k] = nd;
          pred[k] = i;
          heap.push({nd, k});
        }
      }
    };
    relax(r, 0.0);
    int64_t free_col = -1;
    double delta = 0.0;
    while (!heap.empty()) {
      const auto [d, j] = heap.top();
      heap.pop();
      if (done_stamp[j] == r || d > dist[j]) continue;
      done_stamp[j] = r;
      fin[j] = d;
      touched_cols.push_back(j);
      if (row_of[j] < 0) {
        free_col = j;
        delta = d;
        break;
      }
      const int64_t i = row_of[j];
      row_stamp[i] = r;
      d_row[i] = d;
      touched_rows.push_back(i);
      relax(i, d);
    }
    if (free_col < 0) {
      *why = "no perfect matching on the nonzero entries (structurally singular)";
      return BILU_ERR_SINGULAR;
    }
    for (int64_t i : touched_rows)
      if (d_row[i] < delta) u[i] += delta - d_row[i];
    for (int64_t j : touched_cols)
      if (fin[j] < delta) v[j] -= delta - fin[j];
    for (int64_t j = free_col;;) {
      const int64_t i = pred[j];
      const int64_t prev = col_of[i];
      row_of[j] = i;
      col_of[i] = j;
      if (i == r) break;
      j = prev;
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    sigma[i] = col_of[i];
    dl[i] = std::exp(u[i]);
  }
  for (int64_t j = 0; j < n; ++j) dr[j] = std::exp(v[j]) / colmax[j];
  return BILU_OK;
}

// Sec. 5, eq. (smwm): the symmetric matching of the symmetric variant
// (Duff and Pralet, SIAM J. Matrix Anal. Appl. 27, 2005).  For symmetric A
// the symmetrized scaling d_i = sqrt(dl_i dr_i) of a maximum product
// matching keeps |d_i a_ij d_j| <= 1 with the matched entries at magnitude
// one.  The matching's cycles give the pivots: a fixed point a 1x1 pivot, a
// 2-cycle a 2x2 pivot; a longer cycle c_0 -> c_1 -> ... (c_0 its smallest
// index) is cut into consecutive pairs (c_0, c_1), (c_2, c_3), ...; an odd
// cycle first leaves out as a 1x1 pivot its member with the largest scaled
// diagonal |a_ii| d_i d_i (the first in cycle order on ties) and pairs the
// rest from the member after it on.  A pair lists its smaller index first.
// The units are listed in the order their first index is met along pre
// (identity when NULL): order (new -> old) and their boundaries ustart.
bilu_status sym_matching_host(int64_t n, const int64_t* rp, const int32_t* ci,
                              const double* val, const int64_t* pre, std::vector<double>& d,
                              std::vector<int64_t>& order, std::vector<int64_t>& ustart,
                              std::string* why) {
  std::vector<int64_t> sigma(n);
  std::vector<double> dl(n), dr(n);
  const bilu_status ms = mwm_host(n, rp, ci, val, sigma.data(), dl.data(), dr.data(), why);
  if (ms != BILU_OK) return ms;
  d.resize(n);
  std::vector<double> diag(n, 0.0);
  for (int64_t i = 0; i < n; ++i) {
    d[i] = std::sqrt(dl[i] * dr[i]);
    for (int64_t m = rp[i]; m < rp[i + 1]; ++m)
      if (ci[m] == i) diag[i] = std::fabs(val[m]);
  }
  for (int64_t i = 0; i < n; ++i) diag[i] = diag[i] * d[i] * d[i];
  // units: unit_first[u], unit_second[u] (-1 for a 1x1 pivot)
  std::vector<int64_t> unit(n, -1), ufirst, usecond, cyc, rest;
  for (int64_t s0 = 0; s0 < n; ++s0) {
    if (unit[s0] >= 0) continue;
    cyc.assign(1, s0);
    for (int64_t j = sigma[s0]; j != s0; j = sigma[j]) cyc.push_back(j);
    const int64_t L = (int64_t)cyc.size();
    rest.clear();
    if (L % 2 == 1) {
      int64_t best = 0;
      for (int64_t k = 1; k < L; ++k)
        if (diag[cyc[k]] > diag[cyc[best]]) best = k;
      unit[cyc[best]] = (int64_t)ufirst.size();
      ufirst.push_back(cyc[best]);
      usecond.push_back(-1);
      for (int64_t t = 1; t < L; ++t) rest.push_back(cyc[(best + t) % L]);
    } else {
      rest = cyc;
    }
    for (size_t t = 0; t + 1 < rest.size(); t += 2) {
      const int64_t a = std::min(rest[t], rest[t + 1]), b = std::max(rest[t], rest[t + 1]);
      unit[a] = unit[b] = (int64_t)ufirst.size();
      ufirst.push_back(a);
      usecond.push_back(b);
    }
  }
  std::vector<char> done(ufirst.size(), 0);
  order.clear();
  order.reserve(n);
  ustart.assign(1, 0);
  for (int64_t k = 0; k < n; ++k) {
    const int64_t i = pre ? pre[k] : k;
    const int64_t u = unit[i];
    if (done[u]) continue;
    done[u] = 1;
    order.push_back(ufirst[u]);
    if (usecond[u] >= 0) order.push_back(usecond[u]);
    ustart.push_back((int64_t)order.size());
  }
  return BILU_OK;
}

}  // namespace bilu
