// Geometric nested dissection of the element grid (host, integer only).
//
// Recursive bisection of the (i, j) element coordinates (paper Sec.
// "Scalability study of spaND"), defining interiors, separators and
// interfaces at every level 0 <= l < lmax (Sec. "Sparsified Nested
// Dissection algorithm").  Exact rule (the paper leaves it open):
//  * heap-numbered tree, root 1, children 2k, 2k+1; depth d <-> level L-1-d;
//  * split axis x if the box is at least as wide as tall, else y;
//    mid = lo + (hi-lo)/2; left box: coord < mid; right box: coord >= mid;
//  * separator = vertices of the node with coord >= mid that have a grid
//    neighbour (wrap edges in periodic directions) in the node with
//    coord < mid; the right child keeps the right box minus the separator;
//  * level-l cluster key of a live element = (its node, the depth-(L-1-l)
//    box containing it); clusters ordered by key, elements ascending;
//  * merge: (S, B) at level l+1 gathers (S, 2B) then (S, 2B+1) of level l;
//  * elimination permutation: elements by (level of node, node, element).
#include <algorithm>
#include <array>
#include <cmath>

#include "internal.h"

namespace spand {

int default_levels(int64_t K) {
  double v = std::log2(double(K) / 32.0);
  int L = int(std::lround(v)) + 1;
  return L < 1 ? 1 : L;
}

static void grid_neighbours(int nx, int ny, bool px, bool py, int i, int j, int out[4], int &cnt) {
  static const int di[4] = {1, -1, 0, 0}, dj[4] = {0, 0, 1, -1};
  cnt = 0;
  for (int t = 0; t < 4; ++t) {
    int ii = i + di[t], jj = j + dj[t];
    if (px) ii = ii < 0 ? ii + nx : (ii >= nx ? ii - nx : ii);
    if (py) jj = jj < 0 ? jj + ny : (jj >= ny ? jj - ny : jj);
    if (ii < 0 || ii >= nx || jj < 0 || jj >= ny) continue;
    int f = jj * nx + ii;
    if (ii == i && jj == j) continue;   // a one-wide periodic direction wraps onto itself
    bool dup = false;
    for (int q = 0; q < cnt; ++q) dup |= (out[q] == f);
    if (!dup) out[cnt++] = f;
  }
}

NDResult nested_dissection(int nx, int ny, bool px, bool py, int L) {
  NDResult R;
  R.nx = nx;
  R.ny = ny;
  R.L = L;
  const int K = nx * ny;
  std::vector<int> ex(K), ey(K);
  for (int e = 0; e < K; ++e) {
    ex[e] = e % nx;
    ey[e] = e / nx;
  }
  // grid neighbours of every element, once (-1 = none)
  std::vector<std::array<int, 4>> nbr(K);
  for (int e = 0; e < K; ++e) {
    int tmp[4], cnt;
    grid_neighbours(nx, ny, px, py, ex[e], ey[e], tmp, cnt);
    nbr[e] = {-1, -1, -1, -1};
    for (int q = 0; q < cnt; ++q) nbr[e][q] = tmp[q];
  }
  // node ids are below 2^L <= 2K: dense tables indexed by node id
  const size_t nnode = size_t(1) << L;
  std::vector<int32_t> node_of(K, -1);
  std::vector<int> node_lv(nnode, -1);
  std::vector<std::array<int, 4>> boxes(nnode);
  std::vector<std::vector<int32_t>> box_at(L, std::vector<int32_t>(K, 0));
  for (int e = 0; e < K; ++e) box_at[0][e] = 1;
  boxes[1] = {0, nx, 0, ny};
  // Breadth-first over the tree.  The live set of node k is its box minus
  // the separators of its ancestors, i.e. the elements of the box that no
  // node has claimed yet; scanning the box row by row visits them in
  // ascending order.
  std::vector<int> sep;
  for (int d = 0; d < L; ++d) {
    const int64_t k0 = int64_t(1) << d;
    for (int64_t k = k0; k < 2 * k0; ++k) {
      node_lv[size_t(k)] = L - 1 - d;
      R.node_level.emplace_hint(R.node_level.end(), k, L - 1 - d);
      const auto bx = boxes[size_t(k)];
      const int x0 = bx[0], x1 = bx[1], y0 = bx[2], y1 = bx[3];
      if (d == L - 1) {
        for (int y = y0; y < y1; ++y)
          for (int x = x0; x < x1; ++x)
            if (node_of[y * nx + x] < 0) node_of[y * nx + x] = int32_t(k);
        continue;
      }
      const bool xsplit = (x1 - x0) >= (y1 - y0);
      const int lo = xsplit ? x0 : y0, hi = xsplit ? x1 : y1;
      const int mid = lo + (hi - lo) / 2;
      auto live = [&](int f) {
        return ex[f] >= x0 && ex[f] < x1 && ey[f] >= y0 && ey[f] < y1 && node_of[f] < 0;
      };
      sep.clear();
      for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) {
          const int v = y * nx + x;
          if ((xsplit ? x : y) < mid || node_of[v] >= 0) continue;
          for (int u : nbr[v]) {
            if (u >= 0 && (xsplit ? ex[u] : ey[u]) < mid && live(u)) {
              sep.push_back(v);
              break;
            }
          }
        }
      for (int v : sep) node_of[v] = int32_t(k);
      if (xsplit) {
        boxes[size_t(2 * k)] = {x0, mid, y0, y1};
        boxes[size_t(2 * k + 1)] = {mid, x1, y0, y1};
      } else {
        boxes[size_t(2 * k)] = {x0, x1, y0, mid};
        boxes[size_t(2 * k + 1)] = {x0, x1, mid, y1};
      }
      // the depth-d boxes tile the grid: box k is exactly its rectangle
      auto &bn = box_at[d + 1];
      for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x)
          bn[y * nx + x] = int32_t((xsplit ? x : y) < mid ? 2 * k : 2 * k + 1);
    }
  }
  R.node_of_elem = node_of;
  std::vector<int> lvl(K);
  for (int e = 0; e < K; ++e) lvl[e] = node_lv[size_t(node_of[e])];
  R.levels.resize(L);
  R.children.resize(L);
  // clusters of level l: live elements grouped by (node, depth-(L-1-l) box),
  // keys ascending, elements ascending.  Two stable counting sorts over the
  // ascending live elements (by box, then by node) give exactly that order.
  std::vector<int32_t> cnt(nnode + 1), byb, ord;
  std::vector<int64_t> prev_keys, keys;   // sorted cluster keys node * 2^L + box
  for (int l = 0; l < L; ++l) {
    const auto &bl = box_at[L - 1 - l];
    byb.clear();
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int e = 0; e < K; ++e)
      if (lvl[e] >= l) ++cnt[size_t(bl[e]) + 1];
    for (size_t q = 0; q < nnode; ++q) cnt[q + 1] += cnt[q];
    byb.resize(size_t(cnt[nnode]));
    for (int e = 0; e < K; ++e)
      if (lvl[e] >= l) byb[size_t(cnt[size_t(bl[e])]++)] = e;
    std::fill(cnt.begin(), cnt.end(), 0);
    for (int e : byb) ++cnt[size_t(node_of[e]) + 1];
    for (size_t q = 0; q < nnode; ++q) cnt[q + 1] += cnt[q];
    ord.resize(byb.size());
    for (int e : byb) ord[size_t(cnt[size_t(node_of[e])]++)] = e;
    std::vector<NDCluster> cl;
    keys.clear();
    for (size_t q = 0; q < ord.size();) {
      NDCluster c;
      c.node = node_of[ord[q]];
      c.box = bl[ord[q]];
      size_t r = q + 1;
      while (r < ord.size() && node_of[ord[r]] == c.node && bl[ord[r]] == c.box) ++r;
      c.elems.assign(ord.begin() + q, ord.begin() + r);
      q = r;
      c.interior = node_lv[size_t(c.node)] == l;
      keys.push_back(int64_t(c.node) * int64_t(nnode) + c.box);
      cl.push_back(std::move(c));
    }
    if (l >= 1) {
      R.children[l].resize(cl.size());
      for (size_t i = 0; i < cl.size(); ++i) {
        for (int64_t cb : {2 * int64_t(cl[i].box), 2 * int64_t(cl[i].box) + 1}) {
          const int64_t key = int64_t(cl[i].node) * int64_t(nnode) + cb;
          auto it = std::lower_bound(prev_keys.begin(), prev_keys.end(), key);
          if (it != prev_keys.end() && *it == key) R.children[l][i].push_back(int(it - prev_keys.begin()));
        }
      }
    }
    R.levels[l] = std::move(cl);
    prev_keys.swap(keys);
  }
  // elimination order: elements by (level of node, node, element); nodes
  // sorted once, elements bucketed per node in ascending order
  std::vector<std::pair<int, int64_t>> nodes;
  nodes.reserve(R.node_level.size());
  for (auto &kv : R.node_level) nodes.push_back({kv.second, kv.first});
  std::sort(nodes.begin(), nodes.end());
  std::vector<int> nidx(nnode, -1);
  for (size_t q = 0; q < nodes.size(); ++q) nidx[size_t(nodes[q].second)] = int(q);
  std::vector<int> ncount(nodes.size() + 1, 0), enode(K);
  for (int e = 0; e < K; ++e) {
    enode[e] = nidx[size_t(node_of[e])];
    ++ncount[enode[e] + 1];
  }
  for (size_t q = 0; q < nodes.size(); ++q) ncount[q + 1] += ncount[q];
  R.perm.assign(K, 0);
  for (int e = 0; e < K; ++e) R.perm[ncount[enode[e]]++] = e;
  return R;
}

// Disjoint union of the orderings of several grids whose elements are
// numbered one grid after the other (grid g from elem_off[g]): level l holds
// the level-l clusters of every grid, grid by grid, each with its own order;
// grids with fewer levels have no clusters above their top.  Node ids are
// shifted by 2^L per grid so that they stay distinct.
NDResult nd_union(const std::vector<NDResult> &parts, const std::vector<int64_t> &elem_off) {
  NDResult R;
  for (const auto &p : parts) R.L = std::max(R.L, p.L);
  R.levels.resize(size_t(R.L));
  R.children.resize(size_t(R.L));
  int64_t node_base = 0;
  std::vector<int> cbase(size_t(R.L), 0);      // clusters of each level so far
  for (size_t g = 0; g < parts.size(); ++g) {
    const NDResult &p = parts[g];
    const int32_t eo = int32_t(elem_off[g]);
    for (int32_t v : p.node_of_elem) R.node_of_elem.push_back(int32_t(v + node_base));
    for (int32_t v : p.perm) R.perm.push_back(v + eo);
    for (const auto &kv : p.node_level) R.node_level.emplace(kv.first + node_base, kv.second);
    for (int l = 0; l < p.L; ++l) {
      if (l >= 1)
        for (const auto &kids : p.children[size_t(l)]) {
          std::vector<int> k2;
          for (int c : kids) k2.push_back(c + cbase[size_t(l - 1)]);
          R.children[size_t(l)].push_back(std::move(k2));
        }
      for (const auto &c : p.levels[size_t(l)]) {
        NDCluster d = c;
        d.node = int32_t(c.node + node_base);
        for (auto &e : d.elems) e += eo;
        R.levels[size_t(l)].push_back(std::move(d));
      }
    }
    for (int l = 0; l < p.L; ++l) cbase[size_t(l)] += int(p.levels[size_t(l)].size());
    node_base += int64_t(1) << p.L;
  }
  return R;
}

}  // namespace spand
