"""Pins of the nested-dissection oracle (bit-exact integer contract)."""
import collections
import os

import numpy as np
import pytest

from oracle.nd import default_levels, flatten, neighbours, nested_dissection

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read(name):
    out = {}
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, *v = line.split()
            out[k] = v
    return out


def test_hand_worked_4x4():
    g = _read("nd_4x4_px_L3.txt")
    nd = nested_dissection(4, 4, True, False, 3)
    assert nd.node_of_elem.tolist() == [int(t) for t in g["node_of_elem"]]
    assert nd.perm.tolist() == [int(t) for t in g["perm"]]
    for l in range(3):
        want = []
        for item in g[f"level{l}"]:
            head, el = item.split(":")
            node, box, inter = (int(t) for t in head.split(","))
            want.append((node, box, bool(inter), [int(t) for t in el.split(",")]))
        got = [(c.node, c.box, c.interior, c.elems.tolist()) for c in nd.levels[l]]
        assert got == want
    assert nd.children[1] == [[int(t) for t in s.split(",")] for s in g["children1"]]
    assert nd.children[2] == [[int(t) for t in s.split(",")] for s in g["children2"]]


def test_separator_counts_c1():
    with open(os.path.join(GOLD, "nd_counts.txt")) as f:
        rows = [l.split() for l in f if not l.startswith("#") and l.strip()]
    for r in rows:
        nx, ny, px, py, L = (int(t) for t in r[:5])
        want = [int(t) for t in r[5:]]
        nd = nested_dissection(nx, ny, bool(px), bool(py), L)
        cnt = collections.Counter(nd.node_level[int(k)] for k in nd.node_of_elem)
        assert [cnt.get(l, 0) for l in range(L)] == want


def test_default_levels_table_rule():
    # Tables 1 and 2: K -> lmax with 32-element leaf boxes
    for K, L in [(16384, 10), (65536, 12), (262144, 14), (1048576, 16), (4194304, 18)]:
        assert default_levels(K) == L
    assert default_levels(256) == 4


@pytest.mark.parametrize("nx,ny,px,py,L", [(16, 16, 1, 0, 4), (12, 7, 1, 1, 3), (9, 13, 0, 0, 4),
                                            (5, 5, 1, 0, 2), (32, 32, 1, 0, 6), (3, 2, 1, 1, 2)])
def test_invariants(nx, ny, px, py, L):
    nd = nested_dissection(nx, ny, bool(px), bool(py), L)
    K = nx * ny
    assert sorted(nd.perm.tolist()) == list(range(K))
    adj = neighbours(nx, ny, bool(px), bool(py))
    lvl = np.array([nd.node_level[int(k)] for k in nd.node_of_elem])
    # no edge joins two different level-l interiors (ND separation)
    for e in range(K):
        for f in adj[e]:
            if lvl[e] == lvl[f] and nd.node_of_elem[e] != nd.node_of_elem[f]:
                pytest.fail(f"edge {e}-{f} joins interiors of the same level")
    for l in range(L):
        seen = np.concatenate([c.elems for c in nd.levels[l]]) if nd.levels[l] else np.zeros(0)
        assert sorted(seen.tolist()) == sorted(np.nonzero(lvl >= l)[0].tolist())
        for c in nd.levels[l]:
            assert c.interior == (nd.node_level[c.node] == l)
            assert np.all(np.diff(c.elems) > 0)
    # merge: every level-(l+1) cluster is the union of its children, in order
    for l in range(1, L):
        prev = nd.levels[l - 1]
        for c, kids in zip(nd.levels[l], nd.children[l]):
            u = np.sort(np.concatenate([prev[k].elems for k in kids]))
            assert np.array_equal(u, c.elems)
    assert len(nd.levels[L - 1]) == 1


def test_c2_leaf_sizes():
    nd = nested_dissection(128, 128, True, False, 10)
    cnt = collections.Counter(nd.node_level[int(k)] for k in nd.node_of_elem)
    assert 16384 - cnt[0] == 5536
    sizes = collections.Counter(len(c.elems) for c in nd.levels[0] if c.interior)
    assert sizes.most_common(1)[0][0] == 21


def test_flatten_roundtrip():
    nd = nested_dissection(8, 8, True, False, 3)
    f = flatten(nd)
    for l in range(3):
        ptr = f[f"ptr_{l}"]
        assert ptr[-1] == len(f[f"elems_{l}"])
        assert len(f[f"key_{l}"]) == len(ptr) - 1
