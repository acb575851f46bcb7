"""Pins of the spaND oracle: Eqs. (10)-(13) identities, eps=0 / L=1 special
cases, adjointness and the O(eps) quality trend."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle import direct, spand
from oracle.nd import nested_dissection
from synth.dg_euler import DGConfig, make_problem


def _setup(n=16, p=1, L=4, seed=0):
    cfg = DGConfig(n=n, p=p, seed=seed)
    A, xs, b, _ = make_problem(cfg)
    As = A.to_scipy().tocsr()
    nd = nested_dissection(n, n, True, False, L)
    return cfg, As, xs, b, nd


@pytest.mark.parametrize("n,p,L", [(16, 1, 4), (8, 2, 3), (12, 1, 5)])
def test_eps0_reproduces_direct_solve(n, p, L):
    cfg, As, xs, b, nd = _setup(n, p, L)
    F = spand.factor(As, nd, cfg.b, 0.0)
    y = spand.apply(F, b)
    xd = direct.solve(As, b)
    kappa = np.linalg.cond(As.toarray())
    assert kappa * 1.1e-16 <= 1e-13
    assert np.linalg.norm(y - xd) <= 1e-12 * np.linalg.norm(xd)
    # manufactured solution
    assert np.linalg.norm(xd - xs) <= 10 * kappa * 1.1e-16 * np.linalg.norm(xs)


def test_single_level_is_dense_lu():
    cfg, As, xs, b, _ = _setup(8, 1, 1)
    nd = nested_dissection(8, 8, True, False, 1)
    F = spand.factor(As, nd, cfg.b, 1e-2)
    assert len(F.ops) == 1 and isinstance(F.ops[0], spand.Elim)
    np.testing.assert_allclose(spand.apply(F, b), np.linalg.solve(As.toarray(), b),
                               rtol=0, atol=1e-13 * np.abs(xs).max() * 10)


def test_elimination_gives_schur_complement():
    # Eq. (10): after eliminating the level-0 interiors the trailing matrix is
    # A_nn - A_nS A_SS^{-1} A_Sn (S = all leaves, n = all separators)
    cfg, As, xs, b, nd = _setup(8, 1, 3)
    Ad = As.toarray()
    got = {}

    def hook(stage, lvl, blocks, dofs, extra):
        if stage == "elim" and lvl == 0:
            got["blocks"] = {k: v.copy() for k, v in blocks.items()}
            got["dofs"] = [d.copy() for d in dofs]

    spand.factor(As, nd, cfg.b, 1e-2, hook=hook)
    leaf = np.concatenate([got["dofs"][i] for i, c in enumerate(nd.levels[0]) if c.interior])
    sep = np.setdiff1d(np.arange(cfg.N), leaf)
    S = Ad[np.ix_(sep, sep)] - Ad[np.ix_(sep, leaf)] @ np.linalg.solve(Ad[np.ix_(leaf, leaf)],
                                                                      Ad[np.ix_(leaf, sep)])
    pos = {d: i for i, d in enumerate(sep)}
    T = np.zeros_like(S)
    for (i, j), B in got["blocks"].items():
        ri = [pos[d] for d in got["dofs"][i]]
        rj = [pos[d] for d in got["dofs"][j]]
        T[np.ix_(ri, rj)] = B
    assert np.abs(T - S).max() <= 1e-12 * np.abs(S).max()


def test_scaling_invariants():
    cfg, As, xs, b, nd = _setup(8, 1, 3)
    before = {}

    def hook(stage, lvl, blocks, dofs, extra):
        if stage == "elim" and lvl == 0:
            before.update({k: v.copy() for k, v in blocks.items() if k[0] == k[1]})

    F = spand.factor(As, nd, cfg.b, 1e-2, hook=hook)
    sc = [op for op in F.ops if isinstance(op, spand.Scale) and op.level == 0]
    assert sc
    cl0 = nd.levels[0]
    for op in sc:
        # the cluster whose dofs this op scaled
        s = next(i for i, c in enumerate(cl0) if not c.interior and
                 np.array_equal(np.sort((c.elems[:, None] * cfg.b + np.arange(cfg.b)).ravel()),
                                np.sort(op.dofs)))
        Ass = before[(s, s)]
        Xl = sla.solve_triangular(op.Lh, Ass[op.P], lower=True)          # Lh^-1 P^T A
        Z = sla.solve_triangular(op.Uh, Xl.T, lower=False, trans="T").T   # ... Uh^-1
        np.testing.assert_allclose(Z, np.eye(len(op.dofs)), atol=1e-11)
        np.testing.assert_allclose(np.diag(op.Lh), np.abs(np.diag(op.Uh)), rtol=1e-14)


def test_rrqr_bound_and_orthogonality():
    cfg, As, xs, b, nd = _setup(8, 1, 3)
    eps = 1e-2
    seen = []

    def hook(stage, lvl, blocks, dofs, extra):
        if stage == "rrqr":
            s, W, Q, R, k = extra
            m = Q.shape[0]
            np.testing.assert_allclose(Q.T @ Q, np.eye(m), atol=1e-13)
            if W.shape[1]:
                Qc = Q[:, :k]
                resid = np.linalg.norm(W - Qc @ (Qc.T @ W), 2)
                assert resid <= np.sqrt(W.shape[1]) * eps * abs(R[0, 0]) * (1 + 1e-12)
                if k < min(W.shape):
                    assert abs(R[k, k]) <= eps * abs(R[0, 0])
                assert np.all(np.abs(np.diag(R))[:k] > eps * abs(R[0, 0]))
            seen.append(k)

    spand.factor(As, nd, cfg.b, eps, hook=hook)
    assert len(seen) > 0 and 0 < sum(seen) < 10 ** 6


def test_apply_T_is_transpose_dense():
    cfg, As, xs, b, nd = _setup(6, 1, 3)
    F = spand.factor(As, nd, cfg.b, 1e-1)
    I = np.eye(cfg.N)
    Mi = np.stack([spand.apply(F, I[:, i]) for i in range(cfg.N)], axis=1)
    MiT = np.stack([spand.apply_T(F, I[:, i]) for i in range(cfg.N)], axis=1)
    assert np.abs(Mi.T - MiT).max() <= 1e-13 * np.abs(Mi).max()


def test_quality_improves_with_eps():
    cfg, As, xs, b, nd = _setup(8, 1, 3)
    Ad = As.toarray()
    errs = []
    for eps in [1e-1, 1e-2, 1e-3, 1e-4]:
        F = spand.factor(As, nd, cfg.b, eps)
        I = np.eye(cfg.N)
        Mi = np.stack([spand.apply(F, I[:, i]) for i in range(cfg.N)], axis=1)
        errs.append(np.linalg.norm(np.eye(cfg.N) - Ad @ Mi, 2))
    assert all(errs[i + 1] < errs[i] for i in range(3)), errs
    assert errs[-1] < 1e-2


def test_rank_statistics_shape():
    cfg, As, xs, b, nd = _setup(16, 1, 4)
    F = spand.factor(As, nd, cfg.b, 1e-2)
    st = spand.rank_stats(F)
    assert len(st) == 3
    for (mn, av, mx, kept, tot) in st:
        assert 0 <= mn <= av <= mx and kept <= tot


def test_rank_statistics_values():
    """rank_stats fields, hand-computed: per level (min k, mean k, max k,
    sum k, sum |s|) over the interfaces' (|s|, k) pairs."""
    F = spand.Factor(0, [], [[(32, 5), (16, 9)], [(8, 0)], []], 1e-2, 4)
    assert spand.rank_stats(F) == [(5, 7.0, 9, 14, 48), (0, 0.0, 0, 0, 8), (0, 0.0, 0, 0, 0)]


def test_rank_statistics_eps0_sizes():
    """At eps = 0 every unknown is kept: k = |s| for each interface, and the
    level-0 total is the level-0 interface elements of the ND times b."""
    cfg, As, xs, b, nd = _setup(8, 1, 3)
    F = spand.factor(As, nd, cfg.b, 0.0)
    st = spand.rank_stats(F)
    ifs0 = [len(c.elems) * cfg.b for c in nd.levels[0] if not c.interior]
    assert st[0] == (min(ifs0), float(np.mean(ifs0)), max(ifs0), sum(ifs0), sum(ifs0))
    for lv in st:
        assert lv[3] == lv[4]
