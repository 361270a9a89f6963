// Host-side symbolic work for sparse pencils (see host_sparse.h).
#include "host_sparse.h"

#include <algorithm>
#include <cstdio>
#include <numeric>

namespace feast_host {

std::string check_pattern(int64_t n, const int32_t *rp, const int32_t *ci, int64_t nnz) {
  char buf[160];
  if (rp[0] != 0 || rp[n] != nnz) {
    std::snprintf(buf, sizeof buf, "rowptr[0] = %d and rowptr[n] = %d (nnz = %lld)", rp[0], rp[n],
                  static_cast<long long>(nnz));
    return buf;
  }
  std::vector<int64_t> seen(static_cast<size_t>(n), -1);
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) {
      std::snprintf(buf, sizeof buf, "rowptr decreases at row %lld", static_cast<long long>(i));
      return buf;
    }
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int32_t c = ci[e];
      if (c < 0 || c >= n) {
        std::snprintf(buf, sizeof buf, "column index %d out of range in row %lld", c,
                      static_cast<long long>(i));
        return buf;
      }
      if (seen[c] == i) {
        std::snprintf(buf, sizeof buf, "column %d appears twice in row %lld", c,
                      static_cast<long long>(i));
        return buf;
      }
      seen[c] = i;
    }
  }
  return std::string();
}

namespace {

// adjacency of the symmetrised pattern without the diagonal (sorted, unique),
// in one CSR array: adj[v] is the range of v's neighbours
struct Adjacency {
  std::vector<int64_t> off;
  std::vector<int32_t> nb;
  struct Range {
    const int32_t *b, *e;
    const int32_t *begin() const { return b; }
    const int32_t *end() const { return e; }
    size_t size() const { return static_cast<size_t>(e - b); }
  };
  Range operator[](int64_t v) const { return {nb.data() + off[v], nb.data() + off[v + 1]}; }
};

// transpose of an n x n pattern by counting sort: the rows of the result come
// out sorted (rows of the input are scanned in increasing order)
void transpose(int64_t n, const int32_t *rp, const int32_t *ci, std::vector<int64_t> &trp,
               std::vector<int32_t> &tci) {
  trp.assign(static_cast<size_t>(n) + 1, 0);
  for (int64_t e = 0; e < rp[n]; ++e) ++trp[ci[e] + 1];
  for (int64_t i = 0; i < n; ++i) trp[i + 1] += trp[i];
  tci.resize(static_cast<size_t>(rp[n]));
  std::vector<int64_t> fill(trp.begin(), trp.end() - 1);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t e = rp[i]; e < rp[i + 1]; ++e) tci[fill[ci[e]]++] = static_cast<int32_t>(i);
}

Adjacency adjacency(const Pattern &P) {
  const int64_t n = P.n;
  // T = P^T and S = T^T = P, both with sorted rows; row v of the symmetrised
  // pattern is the merge of S's row v and T's row v
  std::vector<int64_t> trp, srp;
  std::vector<int32_t> tci, sci;
  transpose(n, P.rp.data(), P.ci.data(), trp, tci);
  std::vector<int32_t> trp32(trp.begin(), trp.end());
  transpose(n, trp32.data(), tci.data(), srp, sci);
  Adjacency A;
  A.off.assign(static_cast<size_t>(n) + 1, 0);
  A.nb.reserve(2 * sci.size());
  for (int64_t v = 0; v < n; ++v) {
    int64_t x = srp[v], y = trp[v];
    const int64_t xe = srp[v + 1], ye = trp[v + 1];
    int32_t last = -1;
    while (x < xe || y < ye) {
      const int32_t c = (y >= ye || (x < xe && sci[x] <= tci[y])) ? sci[x++] : tci[y++];
      if (c != v && c != last) A.nb.push_back(c);
      last = c;
    }
    A.off[v + 1] = static_cast<int64_t>(A.nb.size());
  }
  return A;
}

// breadth-first levels from `root` inside its component; returns the vertices
// of the last level and the number of levels
int bfs_levels(const Adjacency &adj, int32_t root,
               std::vector<int32_t> &level, std::vector<int32_t> &last) {
  std::vector<int32_t> cur{root}, next;
  level[root] = 0;
  std::vector<int32_t> touched{root};
  int depth = 0;
  while (true) {
    next.clear();
    for (int32_t v : cur)
      for (int32_t w : adj[v])
        if (level[w] < 0) {
          level[w] = depth + 1;
          next.push_back(w);
          touched.push_back(w);
        }
    if (next.empty()) break;
    cur.swap(next);
    ++depth;
  }
  last = cur;
  for (int32_t v : touched) level[v] = -1;
  return depth + 1;
}

}  // namespace

std::vector<int32_t> rcm_order(const Pattern &P) {
  const int64_t n = P.n;
  const auto adj = adjacency(P);
  std::vector<int32_t> order;
  order.reserve(static_cast<size_t>(n));
  std::vector<char> placed(static_cast<size_t>(n), 0);
  std::vector<int32_t> level(static_cast<size_t>(n), -1), last;
  // vertices by (degree, index): the start of each new component is the
  // first unplaced one
  std::vector<int32_t> by_degree(static_cast<size_t>(n));
  std::iota(by_degree.begin(), by_degree.end(), 0);
  std::stable_sort(by_degree.begin(), by_degree.end(),
                   [&](int32_t a, int32_t b) { return adj[a].size() < adj[b].size(); });
  auto lower_degree = [&](int32_t a, int32_t b) {
    return adj[a].size() < adj[b].size() || (adj[a].size() == adj[b].size() && a < b);
  };
  size_t next_start = 0;
  while (order.size() < static_cast<size_t>(n)) {
    while (placed[by_degree[next_start]]) ++next_start;
    int32_t root = by_degree[next_start];
    // pseudo-peripheral vertex: move to the lowest-degree vertex of the last
    // level while that lengthens the level structure
    int depth = bfs_levels(adj, root, level, last);
    for (int it = 0; it < 16; ++it) {
      const int32_t cand = *std::min_element(last.begin(), last.end(), lower_degree);
      std::vector<int32_t> last2;
      const int d2 = bfs_levels(adj, cand, level, last2);
      if (d2 <= depth) break;
      root = cand;
      depth = d2;
      last.swap(last2);
    }
    // Cuthill-McKee from root
    size_t head = order.size();
    order.push_back(root);
    placed[root] = 1;
    std::vector<int32_t> nb;
    while (head < order.size()) {
      const int32_t v = order[head++];
      nb.clear();
      for (int32_t w : adj[v])
        if (!placed[w]) nb.push_back(w);
      std::sort(nb.begin(), nb.end(), lower_degree);
      for (int32_t w : nb) {
        placed[w] = 1;
        order.push_back(w);
      }
    }
  }
  std::reverse(order.begin(), order.end());
  return order;
}

void band_widths(const Pattern &P, const std::vector<int32_t> &perm, int64_t *kl, int64_t *ku) {
  std::vector<int32_t> inv(static_cast<size_t>(P.n));
  if (perm.empty())
    std::iota(inv.begin(), inv.end(), 0);
  else
    for (int64_t i = 0; i < P.n; ++i) inv[perm[i]] = static_cast<int32_t>(i);
  int64_t l = 0, u = 0;
  for (int64_t i = 0; i < P.n; ++i)
    for (int32_t e = P.rp[i]; e < P.rp[i + 1]; ++e) {
      const int64_t d = static_cast<int64_t>(inv[P.ci[e]]) - inv[i];
      l = std::max(l, -d);
      u = std::max(u, d);
    }
  *kl = l;
  *ku = u;
}

std::vector<int32_t> band_order(const Pattern &P, int64_t *kl, int64_t *ku) {
  std::vector<int32_t> perm = rcm_order(P);
  int64_t l1 = 0, u1 = 0, l0 = 0, u0 = 0;
  band_widths(P, perm, &l1, &u1);
  band_widths(P, std::vector<int32_t>(), &l0, &u0);
  if (l0 + u0 <= l1 + u1) {
    std::iota(perm.begin(), perm.end(), 0);
    l1 = l0;
    u1 = u0;
  }
  *kl = l1;
  *ku = u1;
  return perm;
}

UnionPattern union_reordered(const Pattern &A, const Pattern &B, const std::vector<int32_t> &perm) {
  const int64_t n = A.n;
  std::vector<int32_t> inv(static_cast<size_t>(n));
  for (int64_t i = 0; i < n; ++i) inv[perm[i]] = static_cast<int32_t>(i);
  UnionPattern U;
  U.P.n = n;
  U.P.rp.assign(static_cast<size_t>(n) + 1, 0);
  U.P.ci.reserve(A.ci.size() + B.ci.size());
  U.mapA.reserve(A.ci.size() + B.ci.size());
  U.mapB.reserve(A.ci.size() + B.ci.size());
  std::vector<int64_t> slot(static_cast<size_t>(n), -1);  // position of an old column in this row
  struct Ent {
    int32_t col, a, b;
  };
  std::vector<Ent> row;
  for (int64_t r = 0; r < n; ++r) {
    const int32_t o = perm[r];
    row.clear();
    for (int32_t e = A.rp[o]; e < A.rp[o + 1]; ++e) {
      slot[A.ci[e]] = static_cast<int64_t>(row.size());
      row.push_back({inv[A.ci[e]], e, -1});
    }
    for (int32_t e = B.rp[o]; e < B.rp[o + 1]; ++e) {
      const int64_t s = slot[B.ci[e]];
      if (s >= 0)
        row[s].b = e;
      else
        row.push_back({inv[B.ci[e]], -1, e});
    }
    for (int32_t e = A.rp[o]; e < A.rp[o + 1]; ++e) slot[A.ci[e]] = -1;
    std::sort(row.begin(), row.end(), [](const Ent &x, const Ent &y) { return x.col < y.col; });
    for (const Ent &x : row) {
      U.P.ci.push_back(x.col);
      U.mapA.push_back(x.a);
      U.mapB.push_back(x.b);
    }
    U.P.rp[r + 1] = static_cast<int32_t>(U.P.ci.size());
  }
  return U;
}

}  // namespace feast_host
