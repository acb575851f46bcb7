"""Adjoint (differentiation) checks on the GPU: x = A^{-1} b through
SpandSolve (FP64 s-step GMRES, FP32 spaND preconditioner), L = g^T x.
  * 16x16, p=1 (C1 size): dL/db and dL/dA against the dense reference
    gradient (direct solves), 1e-10 relative;
  * 192x192, p=2 (C5, N = 1.33M): 32 central finite differences
    (h = 1e-6, directions on the BSR pattern scaled to ||A||_F, plus b),
    every solve at rtol 1e-13, agreement 1e-6 relative."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2101_01763_amd as sp  # noqa: E402
from oracle import adjoint  # noqa: E402
from synth.dg_euler import DGConfig, make_problem  # noqa: E402


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def test_dense_gradient_c1():
    cfg = DGConfig(n=16, p=1)
    A, xs, b, _ = make_problem(cfg)
    dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
    g = np.random.default_rng(cfg.seed + 1).standard_normal(cfg.N)
    F = sp.factor(dA, 16, 16, True, False, eps=1e-2, nlevels=4, dtype="f32")
    vals = dA.val.clone().requires_grad_(True)
    bt = _dev(b).requires_grad_(True)
    x = sp.SpandSolve.apply(vals, bt, dA, F, dict(s=4, restart=40, rtol=1e-13))
    (x * _dev(g)).sum().backward()
    _, lam, gb, gv = adjoint.dense_gradient(A.to_scipy().tocsr(), A.rowptr, A.colind, A.bs, b, g)
    torch.cuda.synchronize()
    assert np.linalg.norm(bt.grad.cpu().numpy() - gb) <= 1e-10 * np.linalg.norm(gb)
    assert np.linalg.norm(vals.grad.cpu().numpy() - gv) <= 1e-10 * np.linalg.norm(gv)


def test_fd_directions_c5():
    cfg = DGConfig(n=192, p=2)
    A, xs, b, _ = make_problem(cfg)
    dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
    db = _dev(b)
    g = _dev(np.random.default_rng(cfg.seed + 1).standard_normal(cfg.N))
    F = sp.factor(dA, 192, 192, True, False, eps=1e-2, nlevels=11, dtype="f32")
    opts = dict(s=5, restart=60, rtol=1e-13)
    vals = dA.val.clone().requires_grad_(True)
    bt = db.clone().requires_grad_(True)
    x = sp.SpandSolve.apply(vals, bt, dA, F, opts)
    (x * g).sum().backward()
    gv, gb = vals.grad.detach(), bt.grad.detach()
    nA = torch.linalg.norm(dA.val)
    gen = torch.Generator(device="cuda").manual_seed(77)
    h = 1e-6
    worst = 0.0
    for k in range(32):
        dv = torch.randn(dA.val.shape, generator=gen, device="cuda", dtype=torch.float64)
        dv *= nA / torch.linalg.norm(dv)
        dbv = torch.randn(cfg.N, generator=gen, device="cuda", dtype=torch.float64)
        dbv *= torch.linalg.norm(db) / torch.linalg.norm(dbv)
        xp, ip = sp.solve(dA, db + h * dbv, F, val=dA.val + h * dv, **opts)
        xm, im = sp.solve(dA, db - h * dbv, F, val=dA.val - h * dv, **opts)
        assert ip.converged and im.converged
        fd = float(((g * xp).sum() - (g * xm).sum()) / (2 * h))
        an = float((gv * dv).sum() + (gb * dbv).sum())
        err = abs(fd - an) / max(1.0, abs(an))
        worst = max(worst, err)
        assert err <= 1e-6, (k, fd, an)
    print(f"worst relative FD error over 32 directions: {worst:.2e}")
