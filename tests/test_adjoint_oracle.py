"""Pins of the reference gradient of L = g^T x (x = A^{-1} b)."""
import numpy as np

from oracle import adjoint, direct
from synth.dg_euler import DGConfig, make_problem


def test_dense_gradient_vs_finite_differences():
    cfg = DGConfig(n=6, p=1)
    A, xs, b, _ = make_problem(cfg)
    g = np.random.default_rng(cfg.seed + 1).standard_normal(cfg.N)
    x, lam, gb, gv = adjoint.dense_gradient(A.to_scipy().tocsr(), A.rowptr, A.colind, A.bs, b, g)
    np.testing.assert_allclose(x, xs, rtol=1e-9, atol=1e-9)

    def solve(vals, rhs):
        import scipy.sparse as sp
        M = sp.bsr_matrix((vals, A.colind, A.rowptr), shape=(cfg.N, cfg.N)).tocsr()
        return direct.solve(M, rhs)

    rng = np.random.default_rng(9)
    for _ in range(4):
        dv = rng.standard_normal(A.val.shape)
        dv *= np.linalg.norm(A.val) / np.linalg.norm(dv)
        db = rng.standard_normal(cfg.N)
        fd = adjoint.fd_directional(solve, A.val, b, g, dv, db)
        an = np.sum(gv * dv) + gb @ db
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
