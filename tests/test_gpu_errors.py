"""GPU checks of the error paths and of the batched entry points' edge cases:
  * a structurally singular interior block makes spand_factor return
    SPAND_ESINGULAR (exact zero pivot, detected on the device, reported at
    the end of the build) and no handle;
  * the batched solve after a first cycle that converged inside its s MGS
    steps (the regression case of the single-system solve, through
    sstep_gmres_solve_batched);
  * one factor handle shared by several systems of a batched solve (one
    operator, many right-hand sides) gives bit-for-bit the single solves.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2101_01763_amd as sp  # noqa: E402
from oracle.nd import nested_dissection  # noqa: E402
from synth.dg_euler import DGConfig, make_problem  # noqa: E402


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_singular_interior_block(dtype):
    """Zero block row of an element inside a leaf interior: that leaf's
    diagonal block has b zero rows, which stay exactly zero under
    elimination, so its last b pivots are exactly zero."""
    n, p, L = 8, 1, 3
    cfg = DGConfig(n=n, p=p)
    A, xs, b, _ = make_problem(cfg)
    nd = nested_dissection(n, n, True, False, L)
    leaf = next(c for c in nd.levels[0] if c.interior and len(c.elems) > 1)
    e = int(leaf.elems[len(leaf.elems) // 2])
    val = np.array(A.val, copy=True)
    val[A.rowptr[e]:A.rowptr[e + 1]] = 0.0
    dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, val)
    with pytest.raises(sp.SpandError) as ei:
        sp.factor(dA, n, n, True, False, eps=1e-2, nlevels=L, dtype=dtype)
    assert ei.value.code == sp.SPAND_ESINGULAR
    assert "zero pivot" in str(ei.value)
    # the library is still usable: the regular matrix factors afterwards
    dA0 = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
    F = sp.factor(dA0, n, n, True, False, eps=1e-2, nlevels=L, dtype=dtype)
    x, info = sp.solve(dA0, _dev(b), F, s=4, restart=40, rtol=1e-8)
    assert info.converged


def test_batched_restart_after_early_convergence():
    """An exact FP64 factor (one level, eps = 0) and tolerances near rounding
    level: the Givens estimate can meet the tolerance inside the first s
    steps while the true residual does not, so a second cycle starts with
    all-zero shifts.  Through the batched entry, every system must end at
    the solution and match its single-system solve bit for bit."""
    cfg = DGConfig(n=8, p=1)
    A, xs, b, _ = make_problem(cfg)
    dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
    db = _dev(b)
    took = 0
    for rtol in (1e-14, 1e-15, 3e-16, 1e-16):
        Fs = [sp.factor(dA, 8, 8, True, False, eps=0.0, nlevels=1, dtype="f64") for _ in range(2)]
        xb, infos = sp.solve_batched([dA, dA], [db, db], Fs, s=5, restart=60, rtol=rtol, maxit=40)
        x1, i1 = sp.solve(dA, db, Fs[0], s=5, restart=60, rtol=rtol, maxit=40)
        for x, info in zip(xb, infos):
            assert info.relres <= 1e-13, rtol
            assert np.linalg.norm(_host(x) - xs) <= 1e-10 * np.linalg.norm(xs)
            assert info.iters == i1.iters and info.restarts == i1.restarts
            assert np.array_equal(_host(x), _host(x1))
        if infos[0].restarts >= 2 and all(z == 0 for z in infos[0].shifts):
            took += 1
    assert took >= 1


@pytest.mark.parametrize("lagged", [False, True])
def test_batched_shared_factor(lagged):
    """Four right-hand sides of one operator with one factor handle, mixed
    with a system of its own, in one batched solve: each result equals its
    single-system solve bit for bit (the systems sharing the handle run one
    after another on one worker stream; concurrently they would race on the
    handle's scratch vectors)."""
    cfg = DGConfig(n=12, p=2)
    A, xs, b, _ = make_problem(cfg)
    dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
    F = sp.factor(dA, 12, 12, True, False, eps=1e-2, nlevels=4, dtype="f32")
    cfg2 = DGConfig(n=10, p=1, seed=5)
    A2, xs2, b2, _ = make_problem(cfg2)
    dA2 = sp.BSRMatrix.from_numpy(A2.rowptr, A2.colind, A2.val)
    F2 = sp.factor(dA2, 10, 10, True, False, eps=1e-2, nlevels=4, dtype="f32")
    rng = np.random.default_rng(9)
    rhs = [_dev(rng.standard_normal(cfg.N)) for _ in range(4)]
    As_ = [dA, dA2, dA, dA, dA]
    bs_ = [rhs[0], _dev(b2), rhs[1], rhs[2], rhs[3]]
    Ms = [F, F2, F, F, F]
    xb, infos = sp.solve_batched(As_, bs_, Ms, s=5, restart=60, rtol=1e-8, lagged=lagged)
    for i in range(5):
        x1, i1 = sp.solve(As_[i], bs_[i], Ms[i], s=5, restart=60, rtol=1e-8, lagged=lagged)
        assert infos[i].converged and i1.converged
        assert infos[i].iters == i1.iters, i
        assert np.array_equal(_host(xb[i]), _host(x1)), i
