"""GPU parity: every entry point of the C ABI against the CPU oracle on the
same seeded inputs (C1-sized and small ragged grids).  Tolerances:
  * SpMV / pattern outer product: 1e-14 relative (float64 sums of 5 b x b
    blocks, same data);
  * eps = 0 spaND apply vs the direct solve: 1e-12 (an exact factorization:
    only rounding separates the two);
  * eps > 0 FP64 apply vs oracle apply: 1e-10 relative, when the ranks agree
    level by level (otherwise the paths legitimately differ);
  * s-step GMRES FP64: same iteration count, x within 1e-10 of the oracle's.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2101_01763_amd as sp  # noqa: E402
from oracle import direct, krylov, spand  # noqa: E402
from oracle.nd import nested_dissection  # noqa: E402
from synth.dg_euler import DGConfig, make_problem  # noqa: E402


def _problem(n, p, seed=0, **kw):
    cfg = DGConfig(n=n, p=p, seed=seed, **kw)
    A, xs, b, _ = make_problem(cfg)
    dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
    return cfg, A, A.to_scipy().tocsr(), xs, b, dA


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n,p", [(16, 1), (7, 2), (5, 3)])
def test_spmv(n, p):
    cfg, A, As, xs, b, dA = _problem(n, p)
    x = np.random.default_rng(3).standard_normal(cfg.N)
    y = _host(sp.spmv(dA, _dev(x)))
    ref = As @ x
    assert np.abs(y - ref).max() <= 1e-14 * np.abs(ref).max() * 10
    yt = _host(sp.spmv(dA, _dev(x), transpose=True))
    reft = As.T @ x
    assert np.abs(yt - reft).max() <= 1e-14 * np.abs(reft).max() * 10


def test_pattern_outer():
    cfg, A, As, xs, b, dA = _problem(6, 1)
    rng = np.random.default_rng(4)
    u, v = rng.standard_normal(cfg.N), rng.standard_normal(cfg.N)
    got = _host(sp.pattern_outer(dA, _dev(u), _dev(v), alpha=-1.0))
    bs = cfg.b
    for I in range(cfg.K):
        for t in range(A.rowptr[I], A.rowptr[I + 1]):
            J = A.colind[t]
            np.testing.assert_array_equal(got[t], -np.outer(u[I * bs:(I + 1) * bs], v[J * bs:(J + 1) * bs]))


# FP64 matrices of 513-1024 rows take fused blocks of 32 columns: 8x8 p = 3
# with 3 levels (leaves and the last interface of up to 1024 unknowns: the
# Gauss-Jordan inverses and the LU scaling), 14x14 p = 2 with 4 levels
# (leaves up to 756, interfaces up to 1008); with 3 levels its leaves span
# 180-1764 unknowns, so one elimination splits into the 64- and 32-column
# fused paths and the panel path (on the side stream)
@pytest.mark.parametrize("n,p,L", [(16, 1, 4), (8, 2, 3), (12, 1, 5), (6, 3, 2), (8, 1, 1),
                                   (8, 3, 3), (14, 2, 4), (14, 2, 3)])
def test_eps0_direct(n, p, L):
    cfg, A, As, xs, b, dA = _problem(n, p)
    F = sp.factor(dA, n, n, True, False, eps=0.0, nlevels=L, dtype="f64")
    y = _host(F.apply(_dev(b)))
    xd = direct.solve(As, b)
    assert np.linalg.norm(y - xd) <= 1e-12 * np.linalg.norm(xd)
    yt = _host(F.apply_T(_dev(b)))
    xdt = direct.solve(As, b, transpose=True)
    assert np.linalg.norm(yt - xdt) <= 1e-12 * np.linalg.norm(xdt)


@pytest.mark.parametrize("n,p,L,eps", [(16, 1, 4, 1e-2), (16, 1, 4, 1e-1), (10, 2, 3, 1e-2),
                                       (13, 1, 4, 1e-3), (16, 3, 5, 1e-2)])
def test_apply_parity_fp64(n, p, L, eps):
    cfg, A, As, xs, b, dA = _problem(n, p)
    F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f64")
    Fo = spand.factor(As, nested_dissection(n, n, True, False, L), cfg.b, eps)
    st = F.stats()
    ro = spand.rank_stats(Fo)
    ranks_gpu = [(a, c) for a, c in zip(st["size_before"], st["size_after"])]
    ranks_ora = [(r[4], r[3]) for r in ro]
    r = np.random.default_rng(7).standard_normal(cfg.N)
    if ranks_gpu != ranks_ora:
        # one interface whose |R_kk| ties the threshold to rounding changes
        # one level's kept count by one (and the later levels' sizes by it);
        # anything else is a failure, not a tie
        diff = [(g, o) for g, o in zip(ranks_gpu, ranks_ora) if g != o]
        first = diff[0]
        assert len(ranks_gpu) == len(ranks_ora)
        assert first[0][0] == first[1][0] and abs(first[0][1] - first[1][1]) == 1, diff
        pytest.skip(f"one rank tie at the threshold: gpu {ranks_gpu} oracle {ranks_ora}")
    y = _host(F.apply(_dev(r)))
    yo = spand.apply(Fo, r)
    assert np.linalg.norm(y - yo) <= 1e-10 * np.linalg.norm(yo)
    yt = _host(F.apply_T(_dev(r)))
    yto = spand.apply_T(Fo, r)
    assert np.linalg.norm(yt - yto) <= 1e-10 * np.linalg.norm(yto)


def test_apply_adjointness_and_determinism():
    cfg, A, As, xs, b, dA = _problem(16, 1)
    F = sp.factor(dA, 16, 16, True, False, eps=1e-1, nlevels=4, dtype="f64")
    rng = np.random.default_rng(11)
    u, v = rng.standard_normal(cfg.N), rng.standard_normal(cfg.N)
    Mu = _host(F.apply(_dev(u)))
    MTv = _host(F.apply_T(_dev(v)))
    assert abs(Mu @ v - u @ MTv) <= 1e-12 * abs(Mu @ v)
    a1 = _host(F.apply(_dev(u)))
    assert np.array_equal(Mu, a1)
    du = _dev(u)
    F.apply(du, out=du)                      # in place
    assert np.array_equal(_host(du), Mu)


def test_sstep_unpreconditioned():
    cfg, A, As, xs, b, dA = _problem(8, 1)
    x, info = sp.solve(dA, _dev(b), None, s=4, restart=40, rtol=1e-8, maxit=400)
    xo, io = krylov.sstep_gmres(lambda v: As @ v, b, None, s=4, rtol=1e-8, restart=40, maxit=400)
    assert info.converged and io.converged
    assert abs(info.iters - io.iters) <= 1
    n = min(len(info.history), len(io.history), 20)
    h, ho = np.array(info.history[:n]), np.array(io.history[:n])
    assert np.max(np.abs(h - ho) / ho) <= 1e-6


def test_sstep_restart_after_early_convergence():
    """With an exact (single-level FP64) factor the Givens estimate can meet
    a tolerance near rounding level inside the first s (MGS) steps while the
    true residual does not, so another cycle starts.  As in the oracle the
    shifts are then all zero (monomial basis) and that cycle runs its blocks.
    Over a few tolerances at least one must take this path; none may fail."""
    cfg, A, As, xs, b, dA = _problem(8, 1)
    F = sp.factor(dA, 8, 8, True, False, eps=0.0, nlevels=1, dtype="f64")
    took = 0
    for rtol in (1e-14, 1e-15, 3e-16, 1e-16):
        x, info = sp.solve(dA, _dev(b), F, s=5, restart=60, rtol=rtol, maxit=40)
        assert info.relres <= 1e-13, rtol
        assert np.linalg.norm(_host(x) - xs) <= 1e-10 * np.linalg.norm(xs)
        if info.restarts >= 2 and all(z == 0 for z in info.shifts):
            took += 1
    assert took >= 1


@pytest.mark.parametrize("s,eps", [(4, 1e-2), (5, 1e-1), (1, 1e-1), (2, 1e-2)])
def test_sstep_parity_fp64(s, eps):
    n, p, L = 16, 1, 4
    cfg, A, As, xs, b, dA = _problem(n, p)
    F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f64")
    m = 40 if 40 % s == 0 else 40 - 40 % s
    x, info = sp.solve(dA, _dev(b), F, s=s, restart=m, rtol=1e-8)
    Fo = spand.factor(As, nested_dissection(n, n, True, False, L), cfg.b, eps)
    xo, io = krylov.sstep_gmres(lambda v: As @ v, b, lambda v: spand.apply(Fo, v), s=s,
                                rtol=1e-8, restart=m)
    xg = _host(x)
    assert info.converged and info.relres <= 1e-8
    assert info.iters == io.iters
    assert np.linalg.norm(xg - xo) <= 1e-10 * np.linalg.norm(xo)
    np.testing.assert_allclose(info.history, io.history, rtol=1e-6)


def test_fp32_factor_iterations_within_10pct():
    n, p, L = 16, 2, 4
    cfg, A, As, xs, b, dA = _problem(n, p)
    res = {}
    for dt in ("f64", "f32"):
        F = sp.factor(dA, n, n, True, False, eps=1e-2, nlevels=L, dtype=dt)
        x, info = sp.solve(dA, _dev(b), F, s=5, restart=60, rtol=1e-8)
        assert info.converged
        res[dt] = (info.iters, np.linalg.norm(_host(x) - xs) / np.linalg.norm(xs))
    assert res["f32"][0] <= int(np.ceil(1.1 * res["f64"][0]))
    assert res["f32"][1] < 1e-6


def test_adjoint_gradient_dense():
    from oracle import adjoint
    n, p = 6, 1
    cfg, A, As, xs, b, dA = _problem(n, p)
    g = np.random.default_rng(cfg.seed + 1).standard_normal(cfg.N)
    F = sp.factor(dA, n, n, True, False, eps=1e-2, nlevels=3, dtype="f32")
    vals = dA.val.clone().requires_grad_(True)
    bt = _dev(b).requires_grad_(True)
    x = sp.SpandSolve.apply(vals, bt, dA, F, dict(s=4, restart=40, rtol=1e-13))
    L = (x * _dev(g)).sum()
    L.backward()
    _, lam, gb, gv = adjoint.dense_gradient(As, A.rowptr, A.colind, A.bs, b, g)
    assert np.linalg.norm(_host(bt.grad) - gb) <= 1e-10 * np.linalg.norm(gb)
    assert np.linalg.norm(_host(vals.grad) - gv) <= 1e-10 * np.linalg.norm(gv)


def test_graph_replay_matches_eager():
    """Captured sweeps replayed many times, with eager work and syncs between
    replays, give exactly the eager results (apply and apply_T)."""
    cfg, A, As, xs, b, dA = _problem(16, 2)
    Fg = sp.factor(dA, 16, 16, True, False, eps=1e-2, nlevels=4, dtype="f32", graphs=True)
    Fe = sp.factor(dA, 16, 16, True, False, eps=1e-2, nlevels=4, dtype="f32", graphs=False)
    rng = np.random.default_rng(12)
    for rep in range(5):
        r = _dev(rng.standard_normal(cfg.N))
        ye = _host(Fe.apply(r))
        _ = sp.spmv(dA, r)                       # unrelated eager work in between
        torch.cuda.synchronize()
        yg = _host(Fg.apply(r))
        assert np.array_equal(ye, yg), rep
        assert np.array_equal(_host(Fe.apply_T(r)), _host(Fg.apply_T(r))), rep


@pytest.mark.parametrize("lagged", [False, True])
def test_batched_matches_individual(lagged):
    from synth.dg_euler import batch_configs
    cfgs = batch_configs(6, seed=3, nmin=8, nmax=14)
    systems, rhs, sols = [], [], []
    for c in cfgs:
        A, xs, b, _ = make_problem(c)
        systems.append((sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val), c.n, c.n, True, False))
        rhs.append(_dev(b))
        sols.append(xs)
    Ls = [sp.levels_for(c.N) for c in cfgs]
    Fs = sp.factor_batched(systems, eps=1e-2, nlevels=Ls, dtype="f32")
    xs_b, infos = sp.solve_batched([s[0] for s in systems], rhs, Fs, s=5, restart=60, rtol=1e-8,
                                   lagged=lagged)
    for i, (sysd, b, xstar) in enumerate(zip(systems, rhs, sols)):
        F = sp.factor(sysd[0], sysd[1], sysd[2], True, False, eps=1e-2, nlevels=Ls[i], dtype="f32")
        x1, i1 = sp.solve(sysd[0], b, F, s=5, restart=60, rtol=1e-8, lagged=lagged)
        assert infos[i].converged and i1.converged
        assert infos[i].iters == i1.iters
        assert np.array_equal(_host(x1), _host(xs_b[i])), i


@pytest.mark.parametrize("monomial,passes", [(True, 1), (True, 2), (False, 1), (False, 2)])
def test_sstep_stability_variants(monomial, passes):
    """Basis (Newton / monomial) x orthogonalisation passes (1 / 2) with the
    loss of orthogonality recorded after every block, against the oracle:
    same iterations, residual histories to 1e-6 (1e-2 with one pass, whose
    basis is only orthogonal to the recorded loss), losses within a factor
    of 10 where they are above rounding level."""
    n, p, L, eps, s = 16, 1, 4, 1e-1, 5
    cfg, A, As, xs, b, dA = _problem(n, p)
    F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f64")
    x, info = sp.solve(dA, _dev(b), F, s=s, restart=40, rtol=1e-8, monomial=monomial,
                       passes=passes, orth_loss=True)
    Fo = spand.factor(As, nested_dissection(n, n, True, False, L), cfg.b, eps)
    xo, io = krylov.sstep_gmres(lambda v: As @ v, b, lambda v: spand.apply(Fo, v), s=s,
                                rtol=1e-8, restart=40, shifts=[0.0] * s if monomial else None,
                                record_Q=True, passes=passes)
    assert info.converged and io.converged and info.relres <= 1e-8
    assert info.iters == io.iters
    np.testing.assert_allclose(info.history, io.history, rtol=1e-6 if passes == 2 else 1e-2)
    if monomial:
        assert all(z == 0 for z in info.shifts)
    cols = [c for c, _ in info.orth_loss]
    g = np.array([v for _, v in info.orth_loss])
    o = np.array(io.orth_err)
    assert len(g) == len(o) > 0
    assert cols == sorted(cols) and all((c - 1) % s == 0 for c in cols)
    big = o > 1e-10
    assert np.all(np.abs(np.log10(g[big] / o[big])) <= 1.0)
    assert np.all(g[~big] <= 1e-10)


def test_classical_gmres_parity():
    """SSTEP_FLAG_CLASSICAL (every column an Arnoldi step with modified
    Gram-Schmidt) against the oracle's classical GMRES (Algorithm 1), with
    and without restarts: same iterations, histories to 1e-6, x to 1e-10."""
    n, p, L, eps = 16, 1, 4, 1e-1
    cfg, A, As, xs, b, dA = _problem(n, p)
    F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f64")
    Fo = spand.factor(As, nested_dissection(n, n, True, False, L), cfg.b, eps)
    for m in (40, 10):
        x, info = sp.solve(dA, _dev(b), F, s=5, restart=m, rtol=1e-8, classical=True)
        xo, io = krylov.gmres(lambda v: As @ v, b, lambda v: spand.apply(Fo, v), rtol=1e-8,
                              restart=m)
        assert info.converged and io.converged and info.relres <= 1e-8
        assert info.iters == io.iters, m
        np.testing.assert_allclose(info.history, io.history, rtol=1e-6)
        assert np.linalg.norm(_host(x) - xo) <= 1e-10 * np.linalg.norm(xo)


@pytest.mark.gpu
@pytest.mark.parametrize("n,s,m,monomial", [(16, 5, 40, False), (10, 4, 12, False),
                                            (16, 5, 40, True), (10, 3, 9, False)])
def test_lagged_schedule_parity(n, s, m, monomial):
    """SSTEP_FLAG_LAGGED (Algorithm 2's single-reduce schedule) against the
    oracle's lagged schedule and against the default two-pass schedule on
    the GPU: same iterations, residual histories to 1e-6, x to 1e-8, the
    final basis orthonormal after every block, and far fewer reductions.
    n = 10 gives a row count that is not a multiple of the Gram chunk;
    m = 12 and 9 restart, so each cycle's last block gets a step of its own."""
    p, L, eps = 1, 4, 1e-1
    cfg, A, As, xs, b, dA = _problem(n, p)
    F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f64")
    x, info = sp.solve(dA, _dev(b), F, s=s, restart=m, rtol=1e-8, monomial=monomial,
                       lagged=True, orth_loss=True)
    x2, info2 = sp.solve(dA, _dev(b), F, s=s, restart=m, rtol=1e-8, monomial=monomial)
    Fo = spand.factor(As, nested_dissection(n, n, True, False, L), cfg.b, eps)
    xo, io = krylov.sstep_gmres(lambda v: As @ v, b, lambda v: spand.apply(Fo, v), s=s,
                                rtol=1e-8, restart=m, shifts=[0.0] * s if monomial else None,
                                lagged=True, record_Q=True)
    assert info.converged and io.converged and info.relres <= 1e-8
    assert info.iters == io.iters == info2.iters
    assert info.restarts == io.restarts
    np.testing.assert_allclose(info.history, io.history, rtol=1e-6)
    np.testing.assert_allclose(info.history, info2.history, rtol=1e-6)
    assert np.linalg.norm(_host(x) - xo) <= 1e-8 * np.linalg.norm(xo)
    g = np.array([v for _, v in info.orth_loss])
    assert len(g) > 0 and np.all(g <= 1e-10)
    assert all((c - 1) % s == 0 for c, _ in info.orth_loss)
    # four Gram matrices per block against one per step (the dot products of
    # the first cycle's Ritz steps are common to both)
    assert info.n_reduce < info2.n_reduce
    if info.restarts == 1 and not monomial:
        assert info2.n_reduce - info.n_reduce >= 2 * ((io.iters - s) // s)


@pytest.mark.gpu
def test_lagged_transpose_solve():
    """The single-reduce schedule on the adjoint system A^T x = b (M^-T):
    same iterations and histories as the two-pass schedule, x to 1e-8, and
    A^T x = b to the tolerance."""
    n, p, L, eps = 12, 1, 4, 1e-1
    cfg, A, As, xs, b, dA = _problem(n, p)
    F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f64")
    x1, i1 = sp.solve(dA, _dev(b), F, s=5, restart=40, rtol=1e-8, transpose=True, lagged=True)
    x2, i2 = sp.solve(dA, _dev(b), F, s=5, restart=40, rtol=1e-8, transpose=True)
    assert i1.converged and i2.converged and i1.iters == i2.iters
    np.testing.assert_allclose(i1.history, i2.history, rtol=1e-6)
    xa, xb = _host(x1), _host(x2)
    assert np.linalg.norm(xa - xb) <= 1e-8 * np.linalg.norm(xb)
    assert np.linalg.norm(As.T @ xa - b) <= 1e-8 * np.linalg.norm(b)


@pytest.mark.gpu
def test_lagged_rejects_one_pass():
    cfg, A, As, xs, b, dA = _problem(8, 1)
    with pytest.raises(RuntimeError):
        sp.solve(dA, _dev(b), None, s=4, restart=8, rtol=1e-8, lagged=True, passes=1)


@pytest.mark.gpu
@pytest.mark.parametrize("case", ["restart_eq_s", "maxit", "widest"])
def test_lagged_edge_cases(case):
    """Edge cases of the single-reduce schedule against the oracle's and the
    two-pass schedule: restart = s (every block is the last of its cycle),
    maxit ending a cycle early (not converged, the pending block finished
    before the budget), and the largest shape, s = 8 and m = 128 without a
    preconditioner (Gram matrices of 16 columns over up to 129 basis
    vectors)."""
    n, p, L, eps = 10, 1, 4, 1e-1
    cfg, A, As, xs, b, dA = _problem(n, p)
    kw = dict(s=5, restart=40, rtol=1e-8, maxit=1000)
    F, Mo = None, None
    if case != "widest":
        F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f64")
        Fo = spand.factor(As, nested_dissection(n, n, True, False, L), cfg.b, eps)
        Mo = lambda v: spand.apply(Fo, v)
    if case == "restart_eq_s":
        kw.update(s=4, restart=4)
    elif case == "maxit":
        kw.update(maxit=13)
    else:
        kw.update(s=8, restart=128, rtol=1e-10, maxit=400)
    x, info = sp.solve(dA, _dev(b), F, lagged=True, **kw)
    x2, info2 = sp.solve(dA, _dev(b), F, **kw)
    xo, io = krylov.sstep_gmres(lambda v: As @ v, b, Mo, s=kw["s"], rtol=kw["rtol"],
                                restart=kw["restart"], maxit=kw["maxit"], lagged=True)
    assert info.iters == info2.iters == io.iters
    assert info.converged == info2.converged == io.converged
    assert info.restarts == io.restarts
    rt = 1e-6 if case != "widest" else 1e-4
    np.testing.assert_allclose(info.history, io.history, rtol=rt)
    np.testing.assert_allclose(info.history, info2.history, rtol=rt)
    if case == "maxit":
        assert info.iters == 13 and not info.converged
        assert info.status == sp.SPAND_ENOTCONV
    else:
        assert info.converged and info.relres <= kw["rtol"]
    if case == "widest":
        assert info.iters > 128        # a full cycle: the 129-column basis was reached


def test_full_size_c3_schedules():
    """The benchmark's full configuration (256 x 256 grid, p = 3, N = 4,194,304;
    FP32 spaND eps = 1e-2, L = 13; s = 5, m = 60, rtol 1e-8), as bench.py
    launches it: the single-reduce and two-pass schedules reach the same
    iteration count and residual history, and the residual b - A x of the
    result, evaluated in float64 on the host from the host copy of A on 256
    sampled rows, is within the tolerance's scale; the error against the
    generated x* matches the benchmark's order."""
    n, p, eps, L = 256, 3, 1e-2, 13
    cfg = DGConfig(n=n, p=p)
    A, xs, b, _ = make_problem(cfg)
    dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
    db = _dev(b)
    F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f32")
    x1, i1 = sp.solve(dA, db, F, s=5, restart=60, rtol=1e-8, lagged=True)
    x2, i2 = sp.solve(dA, db, F, s=5, restart=60, rtol=1e-8)
    assert i1.converged and i2.converged and i1.iters == i2.iters
    assert i1.relres <= 1e-8 and i2.relres <= 1e-8
    np.testing.assert_allclose(i1.history, i2.history, rtol=1e-6)
    assert i1.n_reduce < i2.n_reduce
    xh = _host(x1)
    bs = cfg.b
    rows = np.random.default_rng(7).choice(cfg.N, 256, replace=False)
    val = np.asarray(A.val).reshape(-1, bs, bs)
    res = []
    for R in rows:
        I, r = divmod(int(R), bs)
        acc = 0.0
        for t in range(A.rowptr[I], A.rowptr[I + 1]):
            J = int(A.colind[t])
            acc += float(val[t, r, :] @ xh[J * bs:(J + 1) * bs])
        res.append(b[R] - acc)
    # per-row residuals of a vector whose full residual norm is 1e-8 ||b||
    assert np.sqrt(np.mean(np.square(res))) <= 1e-8 * np.linalg.norm(b) / np.sqrt(cfg.N) * 10
    err = np.linalg.norm(xh - xs) / np.linalg.norm(xs)
    assert err <= 1e-6
    del F
