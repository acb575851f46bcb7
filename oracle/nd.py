"""Oracle (test infrastructure only): geometric nested dissection of the grid.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may use
anything under oracle/; the product path never does.

Follows the paper's spaND description (Sec. "Sparsified Nested Dissection
algorithm"): an ND ordering defines interiors, separators and interfaces at
each level 0 <= l < lmax, level 0 being the leaves; elements get integer
coordinates (i, j) and are partitioned by standard recursive bisection
(Sec. "Scalability study of spaND"); interfaces are the parts of a separator
next to a pair of interiors, and clusters are merged from one level to the
next.  The paper leaves the exact bisection rule open; the reading used here:

* graph: 4-neighbour element adjacency, wrap edges in periodic directions;
* tree: heap numbering (root 1, children 2k, 2k+1); a node at depth d has
  level L-1-d; leaves are at depth L-1;
* split of a node with box [x0,x1) x [y0,y1) and vertex set V: axis x if
  x1-x0 >= y1-y0 else y; mid = lo + (hi-lo)//2; left box coord < mid,
  right box coord >= mid; separator = {v in V: coord(v) >= mid and v has a
  neighbour u in V with coord(u) < mid}; V_left = V in left box,
  V_right = (V in right box) minus the separator;
* level-l clusters: every element v not yet eliminated (its node has level
  >= l) gets key (node(v), id of the depth-(L-1-l) box containing v);
  equal keys form one cluster; a cluster is an interior when its node has
  level l, an interface otherwise;  clusters are ordered by key, elements
  inside a cluster ascending;
* merge: cluster (S, B) at level l+1 is the union of (S, 2B), (S, 2B+1) at
  level l, in that order;
* elimination permutation: elements sorted by (level(node), node, e).
"""
from __future__ import annotations

import dataclasses

import numpy as np


def default_levels(K: int) -> int:
    """Leaf boxes of about 32 elements: L = log2(K/32) + 1 (Tables 1 and 2)."""
    return max(1, int(round(np.log2(K / 32.0))) + 1)


@dataclasses.dataclass
class Cluster:
    node: int            # heap id of the separator / leaf owning the elements
    box: int             # heap id of the level box containing them
    elems: np.ndarray    # ascending element ids
    interior: bool


@dataclasses.dataclass
class NDResult:
    nx: int
    ny: int
    L: int
    node_of_elem: np.ndarray       # int32 [K]
    node_level: dict               # node id -> level
    levels: list                   # list (per level) of list[Cluster]
    children: list                 # per level l>=1: list of child cluster ids at l-1
    perm: np.ndarray               # int32 [K]


def neighbours(nx, ny, px, py):
    """Adjacency lists (duplicates removed) of the element grid."""
    K = nx * ny
    adj = []
    for e in range(K):
        i, j = e % nx, e // nx
        s = set()
        for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
            ii, jj = i + di, j + dj
            if px:
                ii %= nx
            if py:
                jj %= ny
            if 0 <= ii < nx and 0 <= jj < ny:
                f = jj * nx + ii
                if f != e:
                    s.add(f)
        adj.append(sorted(s))
    return adj


def nested_dissection(nx: int, ny: int, periodic_x: bool, periodic_y: bool,
                      L: int) -> NDResult:
    K = nx * ny
    adj = neighbours(nx, ny, periodic_x, periodic_y)
    ex = np.arange(K) % nx
    ey = np.arange(K) // nx
    node_of = np.full(K, -1, dtype=np.int64)
    node_level = {}
    # box containing each element at each depth (geometry only)
    box_at = np.zeros((L, K), dtype=np.int64)
    box_at[0, :] = 1
    boxes = {1: (0, nx, 0, ny)}
    # the root's vertex set is every element
    work = [(1, 0, np.arange(K))]
    while work:
        k, d, V = work.pop(0)
        lvl = L - 1 - d
        node_level[k] = lvl
        x0, x1, y0, y1 = boxes[k]
        if d == L - 1:
            node_of[V] = k
            continue
        if (x1 - x0) >= (y1 - y0):
            lo, hi, coord = x0, x1, ex
            lbox = (x0, x0 + (x1 - x0) // 2, y0, y1)
            rbox = (x0 + (x1 - x0) // 2, x1, y0, y1)
        else:
            lo, hi, coord = y0, y1, ey
            lbox = (x0, x1, y0, y0 + (y1 - y0) // 2)
            rbox = (x0, x1, y0 + (y1 - y0) // 2, y1)
        mid = lo + (hi - lo) // 2
        inV = np.zeros(K, dtype=bool)
        inV[V] = True
        sep = []
        for v in V:
            if coord[v] >= mid and any(inV[u] and coord[u] < mid for u in adj[v]):
                sep.append(v)
        sep = np.array(sorted(sep), dtype=np.int64)
        node_of[sep] = k
        insep = np.zeros(K, dtype=bool)
        insep[sep] = True
        Vl = np.array([v for v in V if coord[v] < mid], dtype=np.int64)
        Vr = np.array([v for v in V if coord[v] >= mid and not insep[v]], dtype=np.int64)
        boxes[2 * k] = lbox
        boxes[2 * k + 1] = rbox
        # geometry: children boxes for all elements of this box
        inbox = box_at[d] == k
        box_at[d + 1, inbox & (coord < mid)] = 2 * k
        box_at[d + 1, inbox & (coord >= mid)] = 2 * k + 1
        work.append((2 * k, d + 1, Vl))
        work.append((2 * k + 1, d + 1, Vr))
    assert (node_of >= 0).all()
    lvl_of_elem = np.array([node_level[int(k)] for k in node_of])
    levels = []
    children = [None]
    prev_index = None
    for l in range(L):
        alive = np.nonzero(lvl_of_elem >= l)[0]
        keys = {}
        for v in alive:
            key = (int(node_of[v]), int(box_at[L - 1 - l, v]))
            keys.setdefault(key, []).append(int(v))
        cl = []
        for key in sorted(keys):
            S, B = key
            cl.append(Cluster(S, B, np.array(sorted(keys[key]), dtype=np.int64),
                              node_level[S] == l))
        levels.append(cl)
        index = {(c.node, c.box): i for i, c in enumerate(cl)}
        if l >= 1:
            ch = []
            for c in cl:
                kids = []
                for cb in (2 * c.box, 2 * c.box + 1):
                    if (c.node, cb) in prev_index:
                        kids.append(prev_index[(c.node, cb)])
                ch.append(kids)
            children.append(ch)
        prev_index = index
    order = sorted(range(K), key=lambda e: (node_level[int(node_of[e])], int(node_of[e]), e))
    perm = np.array(order, dtype=np.int32)
    return NDResult(nx, ny, L, node_of.astype(np.int32), node_level, levels, children, perm)


def flatten(nd: NDResult):
    """Integer arrays describing the clusters, for exact comparison.

    Returns dict with 'node_of_elem', 'perm' and, per level l,
    'ptr_l' (cluster -> element range), 'elems_l', 'key_l' ([ncl,2] node,box),
    'interior_l'.
    """
    out = {"node_of_elem": nd.node_of_elem.astype(np.int32),
           "perm": nd.perm.astype(np.int32)}
    for l, cl in enumerate(nd.levels):
        ptr = np.zeros(len(cl) + 1, dtype=np.int32)
        for i, c in enumerate(cl):
            ptr[i + 1] = ptr[i] + len(c.elems)
        out[f"ptr_{l}"] = ptr
        out[f"elems_{l}"] = (np.concatenate([c.elems for c in cl]) if cl
                             else np.zeros(0, np.int64)).astype(np.int32)
        out[f"key_{l}"] = np.array([[c.node, c.box] for c in cl], dtype=np.int32).reshape(-1, 2)
        out[f"interior_{l}"] = np.array([c.interior for c in cl], dtype=np.int32)
    return out
