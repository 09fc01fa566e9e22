// Multilevel nested dissection of the compressed (group) graph, the
// ordering step of Sec. 3.3 by the multilevel scheme: the graph is coarsened
// by heavy-edge matchings, the coarsest graph is bisected by greedy graph
// growing from several seeds, each bisection is improved by boundary
// Fiduccia-Mattheyses passes while it is projected back to the finer graphs,
// and the vertex separator is a minimum vertex cover of the cut edges
// (Hopcroft-Karp matching and Koenig's construction).  Both sides are
// ordered first, recursively, and the separator last.  Vertex weights are
// the group sizes, so the halves balance scalars, not groups.  Every random
// choice comes from a generator seeded by the part itself, and parts write
// disjoint ranges of the order, so the result does not depend on threads.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <numeric>
#include <queue>
#include <thread>
#include <vector>

#include "internal.h"

namespace bilu {
namespace {

struct WGraph {
  int32_t n = 0;
  std::vector<int32_t> xadj, adj, ew, vw;  // CSR, edge and vertex weights
  int64_t total_vw() const { return std::accumulate(vw.begin(), vw.end(), (int64_t)0); }
};

// splitmix64
struct Rng {
  uint64_t s;
  explicit Rng(uint64_t seed) : s(seed) {}
  uint64_t next() {
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  }
  int32_t below(int32_t m) { return (int32_t)(next() % (uint64_t)m); }
};

// One level of coarsening by a heavy-edge matching; cmap maps fine to coarse
// vertices.  Returns false when the graph shrinks by less than a tenth.
bool coarsen(const WGraph& g, Rng& rng, WGraph& c, std::vector<int32_t>& cmap) {
  const int32_t n = g.n;
  std::vector<int32_t> perm(n), match(n, -1);
  std::iota(perm.begin(), perm.end(), 0);
  for (int32_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[rng.below(i + 1)]);
  for (int32_t v : perm) {
    if (match[v] >= 0) continue;
    int32_t best = v, bw = -1;
    for (int32_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k) {
      const int32_t u = g.adj[k];
      if (match[u] < 0 && u != v && g.ew[k] > bw) {
        bw = g.ew[k];
        best = u;
      }
    }
    match[v] = best;
    match[best] = v;
  }
  cmap.assign(n, -1);
  int32_t nc = 0;
  for (int32_t v = 0; v < n; ++v)
    if (cmap[v] < 0) {
      cmap[v] = nc;
      cmap[match[v]] = nc;
      ++nc;
    }
  if (nc > n - n / 10) return false;
  c.n = nc;
  c.vw.assign(nc, 0);
  c.xadj.assign(nc + 1, 0);
  c.adj.clear();
  c.ew.clear();
  std::vector<int32_t> pos(nc, -1);
  std::vector<int32_t> rep(nc, -1);  // the first fine vertex of each coarse one
  for (int32_t v = 0; v < n; ++v)
    if (rep[cmap[v]] < 0) rep[cmap[v]] = v;
  for (int32_t cv = 0; cv < nc; ++cv) {
    const int32_t a = rep[cv], b = match[a];
    const int32_t start = (int32_t)c.adj.size();
    for (int pass = 0; pass < (b == a ? 1 : 2); ++pass) {
      const int32_t f = pass == 0 ? a : b;
      c.vw[cv] += g.vw[f];
      for (int32_t k = g.xadj[f]; k < g.xadj[f + 1]; ++k) {
        const int32_t cu = cmap[g.adj[k]];
        if (cu == cv) continue;
        if (pos[cu] < start) {
          pos[cu] = (int32_t)c.adj.size();
          c.adj.push_back(cu);
          c.ew.push_back(g.ew[k]);
        } else {
          c.ew[pos[cu]] += g.ew[k];
        }
      }
    }
    c.xadj[cv + 1] = (int32_t)c.adj.size();
  }
  return true;
}

int64_t cut_of(const WGraph& g, const std::vector<uint8_t>& part) {
  int64_t cut = 0;
  for (int32_t v = 0; v < g.n; ++v)
    for (int32_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k)
      if (part[g.adj[k]] != part[v]) cut += g.ew[k];
  return cut / 2;
}

// Boundary Fiduccia-Mattheyses passes: moves of single vertices by largest
// cut reduction from the side that keeps the balance, each vertex at most
// once per pass, rolled back to the best balanced state of the pass.
void fm_refine(const WGraph& g, std::vector<uint8_t>& part, int64_t maxdev, int passes) {
  const int32_t n = g.n;
  std::vector<int64_t> gain(n);
  std::vector<uint8_t> locked(n);
  int64_t w[2] = {0, 0};
  for (int32_t v = 0; v < n; ++v) w[part[v]] += g.vw[v];
  const int64_t tot = w[0] + w[1];
  auto dev = [&](int64_t w0) { return std::llabs(2 * w0 - tot); };
  for (int pass = 0; pass < passes; ++pass) {
    for (int32_t v = 0; v < n; ++v) {
      int64_t ext = 0, in = 0;
      for (int32_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k)
        (part[g.adj[k]] != part[v] ? ext : in) += g.ew[k];
      gain[v] = ext - in;
    }
    std::fill(locked.begin(), locked.end(), 0);
    // lazy priority queues per side: (gain, vertex)
    std::priority_queue<std::pair<int64_t, int32_t>> pq[2];
    for (int32_t v = 0; v < n; ++v) {
      bool bnd = false;
      for (int32_t k = g.xadj[v]; k < g.xadj[v + 1] && !bnd; ++k) bnd = part[g.adj[k]] != part[v];
      if (bnd) pq[part[v]].push({gain[v], v});
    }
    std::vector<int32_t> moved;
    int64_t cur = 0, best = 0;
    int64_t bestdev = dev(w[0]);
    size_t bestlen = 0;
    int since = 0;
    const int kLimit = std::max(50, n / 50);
    while (since < kLimit) {
      // the side to move from: the heavier one, or either while balanced
      int from = -1;
      int64_t bg = INT64_MIN;
      for (int s = 0; s < 2; ++s) {
        while (!pq[s].empty()) {
          const auto [gv, v] = pq[s].top();
          if (locked[v] || part[v] != s || gv != gain[v]) {
            pq[s].pop();
            continue;
          }
          break;
        }
        if (pq[s].empty()) continue;
        const int32_t v = pq[s].top().second;
        const int64_t w0 = w[0] + (s == 0 ? -g.vw[v] : g.vw[v]);
        if (dev(w0) > std::max<int64_t>(maxdev, dev(w[0]))) continue;  // would break the balance
        if (pq[s].top().first > bg) {
          bg = pq[s].top().first;
          from = s;
        }
      }
      if (from < 0) break;
      const int32_t v = pq[from].top().second;
      pq[from].pop();
      locked[v] = 1;
      part[v] = (uint8_t)(1 - from);
      w[from] -= g.vw[v];
      w[1 - from] += g.vw[v];
      cur += gain[v];
      moved.push_back(v);
      for (int32_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k) {
        const int32_t u = g.adj[k];
        if (locked[u]) continue;
        gain[u] += part[u] == part[v] ? -2 * g.ew[k] : 2 * g.ew[k];
        pq[part[u]].push({gain[u], u});
      }
      const int64_t d = dev(w[0]);
      if (cur > best || (cur == best && d < bestdev)) {
        if (d <= std::max<int64_t>(maxdev, bestdev)) {
          best = cur;
          bestdev = d;
          bestlen = moved.size();
          since = 0;
          continue;
        }
      }
      ++since;
    }
    for (size_t i = moved.size(); i > bestlen; --i) {  // roll back
      const int32_t v = moved[i - 1];
      w[part[v]] -= g.vw[v];
      part[v] ^= 1;
      w[part[v]] += g.vw[v];
    }
    if (best <= 0) break;
  }
}

// Bisection of a small graph by growing a region from a seed (always the
// frontier vertex with the most edge weight into the region) to half the
// weight; the best of several seeds after refinement.
void initial_bisection(const WGraph& g, Rng& rng, int64_t maxdev, std::vector<uint8_t>& best) {
  const int32_t n = g.n;
  const int64_t tot = g.total_vw();
  int64_t bestcut = INT64_MAX;
  std::vector<uint8_t> part(n);
  std::vector<int64_t> conn(n);
  const int tries = std::min<int32_t>(n, 8);
  for (int t = 0; t < tries; ++t) {
    std::fill(part.begin(), part.end(), 1);
    std::fill(conn.begin(), conn.end(), 0);
    std::priority_queue<std::pair<int64_t, int32_t>> pq;
    int64_t w0 = 0;
    int32_t seed = rng.below(n);
    while (2 * w0 < tot) {
      int32_t v = -1;
      while (!pq.empty()) {
        const auto [c, u] = pq.top();
        pq.pop();
        if (part[u] == 1 && c == conn[u]) {
          v = u;
          break;
        }
      }
      if (v < 0) {  // a new component, or the first seed
        if (part[seed] == 0)
          for (seed = 0; seed < n && part[seed] == 0; ++seed) {
          }
        if (seed >= n) break;
        v = seed;
      }
      part[v] = 0;
      w0 += g.vw[v];
      for (int32_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k) {
        const int32_t u = g.adj[k];
        if (part[u] == 1) {
          conn[u] += g.ew[k];
          pq.push({conn[u], u});
        }
      }
    }
    fm_refine(g, part, maxdev, 4);
    const int64_t c = cut_of(g, part);
    if (c < bestcut) {
      bestcut = c;
      best = part;
    }
  }
}

// Edge bisection of g: part[v] in {0, 1}.
void bisect(const WGraph& g0, Rng& rng, std::vector<uint8_t>& part) {
  std::vector<WGraph> levels;
  std::vector<std::vector<int32_t>> maps;
  const WGraph* cur = &g0;
  while (cur->n > 120) {
    WGraph c;
    std::vector<int32_t> cmap;
    if (!coarsen(*cur, rng, c, cmap)) break;
    levels.push_back(std::move(c));
    maps.push_back(std::move(cmap));
    cur = &levels.back();
  }
  int32_t maxvw = 0;
  for (int32_t x : g0.vw) maxvw = std::max(maxvw, x);
  const int64_t tot = g0.total_vw();
  const int64_t maxdev = std::max<int64_t>(tot / 20, 2 * (int64_t)maxvw);
  initial_bisection(*cur, rng, maxdev, part);
  for (int i = (int)levels.size() - 1; i >= 0; --i) {
    const WGraph& fine = i > 0 ? levels[i - 1] : g0;
    std::vector<uint8_t> fp(fine.n);
    for (int32_t v = 0; v < fine.n; ++v) fp[v] = part[maps[i][v]];
    part.swap(fp);
    fm_refine(fine, part, maxdev, 3);
  }
}

// Minimum vertex cover of the cut edges (Koenig): a maximum matching of the
// bipartite graph between the boundary vertices of side 0 and side 1 by
// Hopcroft-Karp, then the side-0 vertices not reachable from an unmatched
// side-0 vertex by alternating paths, and the side-1 vertices that are.
std::vector<uint8_t> cut_cover(const WGraph& g, const std::vector<uint8_t>& part) {
  const int32_t n = g.n;
  std::vector<int32_t> mate(n, -1), dist(n);
  std::vector<int32_t> left;  // boundary vertices of side 0
  for (int32_t v = 0; v < n; ++v) {
    if (part[v] != 0) continue;
    for (int32_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k)
      if (part[g.adj[k]] == 1) {
        left.push_back(v);
        break;
      }
  }
  const int32_t kInf = INT32_MAX;
  auto bfs = [&]() {
    std::queue<int32_t> q;
    bool found = false;
    for (int32_t v : left) {
      if (mate[v] < 0) {
        dist[v] = 0;
        q.push(v);
      } else {
        dist[v] = kInf;
      }
    }
    while (!q.empty()) {
      const int32_t v = q.front();
      q.pop();
      for (int32_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k) {
        const int32_t u = g.adj[k];
        if (part[u] != 1) continue;
        const int32_t w = mate[u];
        if (w < 0) {
          found = true;
        } else if (dist[w] == kInf) {
          dist[w] = dist[v] + 1;
          q.push(w);
        }
      }
    }
    return found;
  };
  // iterative augmenting-path search along the BFS layers
  std::vector<int32_t> it(n), stk;
  auto dfs = [&](int32_t root) {
    stk.assign(1, root);
    it[root] = g.xadj[root];
    while (!stk.empty()) {
      const int32_t v = stk.back();
      bool advanced = false;
      while (it[v] < g.xadj[v + 1]) {
        const int32_t u = g.adj[it[v]++];
        if (part[u] != 1) continue;
        const int32_t w = mate[u];
        if (w < 0) {
          // augment along the stack: each left vertex takes the right vertex
          // it advanced through
          int32_t right = u;
          for (size_t i = stk.size(); i-- > 0;) {
            const int32_t l = stk[i];
            const int32_t prev = mate[l];
            mate[l] = right;
            mate[right] = l;
            right = prev;
          }
          return true;
        }
        if (dist[w] == dist[v] + 1) {
          it[w] = g.xadj[w];
          stk.push_back(w);
          advanced = true;
          break;
        }
      }
      if (!advanced && stk.back() == v) {
        dist[v] = kInf;
        stk.pop_back();
      }
    }
    return false;
  };
  while (bfs())
    for (int32_t v : left)
      if (mate[v] < 0) dfs(v);
  // alternating reachability from the unmatched side-0 boundary vertices
  std::vector<uint8_t> reach(n, 0);
  std::queue<int32_t> q;
  for (int32_t v : left)
    if (mate[v] < 0) {
      reach[v] = 1;
      q.push(v);
    }
  while (!q.empty()) {
    const int32_t v = q.front();
    q.pop();
    for (int32_t k = g.xadj[v]; k < g.xadj[v + 1]; ++k) {
      const int32_t u = g.adj[k];
      if (part[u] != 1 || reach[u] || mate[u] == v) continue;
      reach[u] = 1;
      const int32_t w = mate[u];
      if (w >= 0 && !reach[w]) {
        reach[w] = 1;
        q.push(w);
      }
    }
  }
  std::vector<uint8_t> cover(n, 0);
  for (int32_t v : left)
    if (!reach[v]) cover[v] = 1;
  for (int32_t v = 0; v < n; ++v)
    if (part[v] == 1 && reach[v]) cover[v] = 1;
  return cover;
}

struct MlState {
  const std::vector<int64_t>& xadj;
  const std::vector<int32_t>& adj;
  const std::vector<int32_t>& vw;
  int32_t* out;
  std::atomic<int> threads{1};
  int max_threads = 1;
};

// The subgraph induced by verts (local numbering), unit edge weights.
void induced(const MlState& S, const std::vector<int32_t>& verts, std::vector<int32_t>& local,
             WGraph& g) {
  g.n = (int32_t)verts.size();
  g.xadj.assign(g.n + 1, 0);
  g.adj.clear();
  g.vw.resize(g.n);
  for (int32_t i = 0; i < g.n; ++i) local[verts[i]] = i;
  for (int32_t i = 0; i < g.n; ++i) {
    const int32_t v = verts[i];
    g.vw[i] = S.vw[v];
    for (int64_t k = S.xadj[v]; k < S.xadj[v + 1]; ++k) {
      const int32_t u = local[S.adj[k]];
      if (u >= 0) g.adj.push_back(u);
    }
    g.xadj[i + 1] = (int32_t)g.adj.size();
  }
  g.ew.assign(g.adj.size(), 1);
  for (int32_t v : verts) local[v] = -1;
}

constexpr size_t kLeaf = 8;

// Orders verts into S.out[off, off + |verts|).
void ml_nd(MlState& S, std::vector<int32_t> verts, int64_t off, int depth) {
  if (verts.size() <= kLeaf) {
    std::sort(verts.begin(), verts.end());
    std::copy(verts.begin(), verts.end(), S.out + off);
    return;
  }
  WGraph g;
  {
    // global -> local numbering, all -1 between uses (induced() resets it)
    thread_local std::vector<int32_t> local;
    if (local.size() != S.xadj.size() - 1) local.assign(S.xadj.size() - 1, -1);
    induced(S, verts, local, g);
  }
  Rng rng(0x5eed ^ ((uint64_t)verts.size() << 20) ^ (uint64_t)verts.front() ^ ((uint64_t)depth << 52));
  std::vector<uint8_t> part;
  bisect(g, rng, part);
  const std::vector<uint8_t> cover = cut_cover(g, part);
  std::vector<int32_t> a, b, s;
  for (int32_t i = 0; i < g.n; ++i)
    (cover[i] ? s : part[i] == 0 ? a : b).push_back(verts[i]);
  if (a.empty() || b.empty()) {  // no useful separator: keep the part as it is
    std::sort(verts.begin(), verts.end());
    std::copy(verts.begin(), verts.end(), S.out + off);
    return;
  }
  verts.clear();
  verts.shrink_to_fit();
  std::sort(s.begin(), s.end());
  std::copy(s.begin(), s.end(), S.out + off + (int64_t)a.size() + (int64_t)b.size());
  const int64_t offb = off + (int64_t)a.size();
  constexpr size_t kSpawn = 8192;
  if (a.size() >= kSpawn && S.threads.fetch_add(1) < S.max_threads) {
    std::thread t([&S, va = std::move(a), off, depth]() mutable {
      ml_nd(S, std::move(va), off, depth + 1);
      S.threads.fetch_sub(1);
    });
    ml_nd(S, std::move(b), offb, depth + 1);
    t.join();
    return;
  }
  if (a.size() >= kSpawn) S.threads.fetch_sub(1);
  ml_nd(S, std::move(a), off, depth + 1);
  ml_nd(S, std::move(b), offb, depth + 1);
}

}  // namespace

void mlnd_order(const std::vector<int64_t>& xadj, const std::vector<int32_t>& adj,
                const std::vector<int32_t>& vw, std::vector<int32_t>& order) {
  const int64_t n = (int64_t)xadj.size() - 1;
  order.assign(n, 0);
  MlState S{xadj, adj, vw, order.data()};
  S.max_threads = (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<int32_t> all(n);
  std::iota(all.begin(), all.end(), 0);
  ml_nd(S, std::move(all), 0, 0);
}

}  // namespace bilu
