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
#include <deque>
#include <tuple>

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
  std::vector<int32_t> node_of(K, -1);
  std::vector<std::vector<int64_t>> box_at(L, std::vector<int64_t>(K, 0));
  for (int e = 0; e < K; ++e) box_at[0][e] = 1;
  std::map<int64_t, std::array<int, 4>> boxes;
  boxes[1] = {0, nx, 0, ny};
  struct Work {
    int64_t k;
    int d;
    std::vector<int> V;
  };
  std::deque<Work> work;
  {
    Work w{1, 0, std::vector<int>(K)};
    for (int e = 0; e < K; ++e) w.V[e] = e;
    work.push_back(std::move(w));
  }
  std::vector<char> inV(K, 0), insep(K, 0);
  while (!work.empty()) {
    Work w = std::move(work.front());
    work.pop_front();
    const int64_t k = w.k;
    const int d = w.d;
    R.node_level[k] = L - 1 - d;
    auto bx = boxes[k];
    int x0 = bx[0], x1 = bx[1], y0 = bx[2], y1 = bx[3];
    if (d == L - 1) {
      for (int v : w.V) node_of[v] = int32_t(k);
      continue;
    }
    bool xsplit = (x1 - x0) >= (y1 - y0);
    int lo = xsplit ? x0 : y0, hi = xsplit ? x1 : y1;
    const std::vector<int> &coord = xsplit ? ex : ey;
    int mid = lo + (hi - lo) / 2;
    std::array<int, 4> lbox, rbox;
    if (xsplit) {
      lbox = {x0, mid, y0, y1};
      rbox = {mid, x1, y0, y1};
    } else {
      lbox = {x0, x1, y0, mid};
      rbox = {x0, x1, mid, y1};
    }
    for (int v : w.V) inV[v] = 1;
    std::vector<int> sep;
    for (int v : w.V) {
      if (coord[v] < mid) continue;
      int nb[4], cnt;
      grid_neighbours(nx, ny, px, py, ex[v], ey[v], nb, cnt);
      for (int q = 0; q < cnt; ++q) {
        int u = nb[q];
        if (inV[u] && coord[u] < mid) {
          sep.push_back(v);
          break;
        }
      }
    }
    std::sort(sep.begin(), sep.end());
    for (int v : sep) {
      node_of[v] = int32_t(k);
      insep[v] = 1;
    }
    Work wl{2 * k, d + 1, {}}, wr{2 * k + 1, d + 1, {}};
    for (int v : w.V) {
      if (coord[v] < mid)
        wl.V.push_back(v);
      else if (!insep[v])
        wr.V.push_back(v);
    }
    for (int v : w.V) inV[v] = 0;
    for (int v : sep) insep[v] = 0;
    boxes[2 * k] = lbox;
    boxes[2 * k + 1] = rbox;
    // the depth-d boxes tile the grid: box k is exactly its rectangle
    for (int y = y0; y < y1; ++y)
      for (int x = x0; x < x1; ++x) {
        const int e = y * nx + x;
        box_at[d + 1][e] = coord[e] < mid ? 2 * k : 2 * k + 1;
      }
    work.push_back(std::move(wl));
    work.push_back(std::move(wr));
  }
  R.node_of_elem = node_of;
  // node ids are below 2^L <= 2K: dense tables instead of map lookups
  std::vector<int> node_lv(size_t(1) << L, -1);
  for (auto &kv : R.node_level) node_lv[size_t(kv.first)] = kv.second;
  std::vector<int> lvl(K);
  for (int e = 0; e < K; ++e) lvl[e] = node_lv[size_t(node_of[e])];
  R.levels.resize(L);
  R.children.resize(L);
  // clusters of level l: live elements grouped by (node, depth-(L-1-l) box),
  // keys ascending, elements ascending; one sort per level of (node, box,
  // element) triples, packed into one word when they fit (node and box ids
  // are below 2^L <= 2K)
  const int ebits = [&] { int b = 1; while ((int64_t(1) << b) < K) ++b; return b; }();
  const int kbits = ebits + 1;
  const bool packed = 2 * kbits + ebits <= 64;
  std::map<std::pair<int64_t, int64_t>, int> prev_index;
  std::vector<std::array<int64_t, 3>> kt;
  std::vector<uint64_t> kw;
  for (int l = 0; l < L; ++l) {
    kt.clear();
    const auto &bl = box_at[L - 1 - l];
    if (packed) {
      kw.clear();
      for (int e = 0; e < K; ++e)
        if (lvl[e] >= l)
          kw.push_back((((uint64_t(node_of[e]) << kbits) | uint64_t(bl[e])) << ebits) | uint64_t(e));
      std::sort(kw.begin(), kw.end());
      const uint64_t emask = (uint64_t(1) << ebits) - 1, bmask = (uint64_t(1) << kbits) - 1;
      kt.resize(kw.size());
      for (size_t q = 0; q < kw.size(); ++q)
        kt[q] = {int64_t(kw[q] >> (ebits + kbits)), int64_t((kw[q] >> ebits) & bmask),
                 int64_t(kw[q] & emask)};
    } else {
      for (int e = 0; e < K; ++e)
        if (lvl[e] >= l) kt.push_back({int64_t(node_of[e]), bl[e], int64_t(e)});
      std::sort(kt.begin(), kt.end());
    }
    std::vector<NDCluster> cl;
    std::map<std::pair<int64_t, int64_t>, int> index;
    for (size_t q = 0; q < kt.size();) {
      NDCluster c;
      c.node = int32_t(kt[q][0]);
      c.box = int32_t(kt[q][1]);
      while (q < kt.size() && kt[q][0] == c.node && kt[q][1] == c.box) c.elems.push_back(int32_t(kt[q++][2]));
      c.interior = node_lv[size_t(c.node)] == l;
      index[{int64_t(c.node), int64_t(c.box)}] = int(cl.size());
      cl.push_back(std::move(c));
    }
    if (l >= 1) {
      R.children[l].resize(cl.size());
      for (size_t i = 0; i < cl.size(); ++i) {
        for (int64_t cb : {2 * int64_t(cl[i].box), 2 * int64_t(cl[i].box) + 1}) {
          auto it = prev_index.find({int64_t(cl[i].node), cb});
          if (it != prev_index.end()) R.children[l][i].push_back(it->second);
        }
      }
    }
    R.levels[l] = std::move(cl);
    prev_index = std::move(index);
  }
  // elimination order: elements by (level of node, node, element); nodes
  // sorted once, elements bucketed per node in ascending order
  std::vector<std::pair<int, int64_t>> nodes;
  nodes.reserve(R.node_level.size());
  for (auto &kv : R.node_level) nodes.push_back({kv.second, kv.first});
  std::sort(nodes.begin(), nodes.end());
  std::vector<int> nidx(size_t(1) << L, -1);
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

}  // namespace spand
