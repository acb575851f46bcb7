"""GPU parity of the FP32 spaND factor (the matrix-core path: FP32 storage,
FP32 products with FP32 accumulation, FP64 vectors) against the FP64
oracle, entry by entry.

Tolerance (derived from FP32 rounding, not fitted to the kernels):
the FP32 path starts by rounding A to FP32 (a relative perturbation of at
most u32 = 2^-24 per entry); every later step (Gauss-Jordan inverses, LU
with partial pivoting, Gram-Schmidt QR, the compressions) is backward
stable, i.e. equivalent to a further perturbation of the blocks it works on
of about sqrt(n) u32 relative (statistical rounding model, n = the block
order; Higham, Accuracy and Stability of Numerical Algorithms, Sec. 2.8
and Ch. 9).  The oracle measures the sensitivity of its own result to the
first of these perturbations, delta_in = |y(fl32(A)) - y(A)| / |y(A)|
(FP64 arithmetic on the FP32-rounded input, same ranks required).  A row
of M^-1 r passes through up to 4 stored operators per level (elimination,
scaling, the two sides of the compression) in each of the 2 sweeps, over
L levels, each adding about sqrt(n_max) rounding steps of that size, so

    |y_gpu - y_oracle| <= tau |y_oracle|,
    tau = 8 L sqrt(n_max) max(delta_in, u32),

with n_max the largest cluster of the factorization.  The same bound is
applied element-wise against the largest entry
(|y_gpu - y_oracle|_inf <= tau |y_oracle|_inf).  Measured errors are 10-100
times delta_in, i.e. 5-30 times below tau; a wrong term, sign or index
gives errors of 1e-3 or more.  Ranks are compared first:
every level's kept and total unknowns must equal the oracle's (the chosen
grids keep every |R_kk| at least 4e-5 relative away from the threshold,
which the FP32 rounding of |R_kk|, about 1e-6 relative, cannot cross).

Grids: 16x16 p=1 and 10x10 p=2 (C1-sized), and 16x16 p=3 with 5 levels
(N = 16,384), whose 16 leaf interiors of 384-1024 unknowns reach every
64-row size class of the fused block elimination up to its 1024-row limit,
whose level-0 Schur updates run on the 64x64 element blocks of the FP32
matrix-core kernel, and whose interfaces' W matrices (up to 256 x ~4,000,
most columns of the interior-side blocks zero) are pruned and packed by the
QRCP in the first candidate block.  eps = 0 at 28x28 p=1 and 14x14 p=2
takes the panel elimination path (leaves of 1040-1764 unknowns, beyond the
fused limit) and completes nearly full-rank Q's (the Gram-Schmidt stops at
the FP32 floor 1e-4 |R_00|, the completion supplies the rest).
"""
import math

import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2101_01763_amd as sp  # noqa: E402
from oracle import direct, krylov, spand  # noqa: E402
from oracle.nd import nested_dissection  # noqa: E402
from synth.dg_euler import DGConfig, make_problem  # noqa: E402

U32 = 2.0 ** -24


def _dev(x):
    return torch.as_tensor(np.ascontiguousarray(x), device="cuda")


def _host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _round32(A):
    """The same matrix with every entry rounded to FP32 (then held in FP64)."""
    B = A.copy()
    B.data = B.data.astype(np.float32).astype(np.float64)
    return B


def _levels(F):
    return [(sum(m for m, _ in lr), sum(k for _, k in lr)) for lr in F.ranks]


def _nmax(nd, b):
    return max(len(c.elems) for lv in nd.levels for c in lv) * b


def _check(y, yo, tau, what):
    err2 = np.linalg.norm(y - yo) / np.linalg.norm(yo)
    errinf = np.abs(y - yo).max() / np.abs(yo).max()
    print(f"{what}: |dy|/|y| = {err2:.3e}, |dy|_inf/|y|_inf = {errinf:.3e}, tau = {tau:.3e}")
    assert err2 <= tau, (what, err2, tau)
    assert errinf <= tau, (what, errinf, tau)


@pytest.mark.parametrize("n,p,L,eps", [(16, 1, 4, 1e-1), (16, 1, 4, 1e-2), (10, 2, 3, 1e-1),
                                       (10, 2, 3, 1e-2), (16, 3, 5, 1e-1), (16, 3, 5, 1e-2)])
def test_fp32_apply_vs_oracle(n, p, L, eps):
    cfg = DGConfig(n=n, p=p)
    A, xs, b, _ = make_problem(cfg)
    As = A.to_scipy().tocsr()
    dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
    nd = nested_dissection(n, n, True, False, L)
    F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f32")
    Fo = spand.factor(As, nd, cfg.b, eps)
    Fp = spand.factor(_round32(As), nd, cfg.b, eps)
    st = F.stats()
    gpu = [(int(a), int(c)) for a, c in zip(st["size_before"], st["size_after"])]
    assert gpu == _levels(Fo), (gpu, _levels(Fo))
    assert _levels(Fp) == _levels(Fo)
    tau_base = 8.0 * L * math.sqrt(_nmax(nd, cfg.b))
    r = np.random.default_rng(7).standard_normal(cfg.N)
    for name, f_gpu, f_or in (("apply", F.apply, spand.apply), ("apply_T", F.apply_T, spand.apply_T)):
        yo = f_or(Fo, r)
        d_in = np.linalg.norm(f_or(Fp, r) - yo) / np.linalg.norm(yo)
        y = _host(f_gpu(_dev(r)))
        _check(y, yo, tau_base * max(d_in, U32), f"{name} n={n} p={p} eps={eps} d_in={d_in:.2e}")


@pytest.mark.parametrize("n,p,L", [(16, 1, 4), (8, 2, 3), (28, 1, 4), (14, 2, 3)])
def test_fp32_eps0_vs_direct(n, p, L):
    """eps = 0 keeps every unknown: the FP32 factor is an FP32 direct solver,
    compared with the exact solution A^{-1} b (and A^{-T} b)."""
    cfg = DGConfig(n=n, p=p)
    A, xs, b, _ = make_problem(cfg)
    As = A.to_scipy().tocsr()
    dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
    nd = nested_dissection(n, n, True, False, L)
    F = sp.factor(dA, n, n, True, False, eps=0.0, nlevels=L, dtype="f32")
    tau_base = 8.0 * L * math.sqrt(_nmax(nd, cfg.b))
    Ap = _round32(As)
    for tr, f_gpu in ((False, F.apply), (True, F.apply_T)):
        xd = direct.solve(As, b, transpose=tr)
        d_in = np.linalg.norm(direct.solve(Ap, b, transpose=tr) - xd) / np.linalg.norm(xd)
        y = _host(f_gpu(_dev(b)))
        _check(y, xd, tau_base * max(d_in, U32), f"eps0 n={n} p={p} T={tr} d_in={d_in:.2e}")


def test_fp32_solve_vs_oracle_c1():
    """The headline precision pattern at the C1 operator: FP64 s-step GMRES
    preconditioned by the FP32 factor against the FP64 oracle's solve.
    Both stop at |b - A x| <= 1e-8 |b|, so their solutions may differ by
    kappa(A) 2e-8 relative (kappa_1 estimated by the oracle's sparse LU);
    iterations within 10% of the oracle's FP64 count."""
    import scipy.sparse.linalg as spl
    n, p, L, eps = 16, 1, 4, 1e-2
    cfg = DGConfig(n=n, p=p)
    A, xs, b, _ = make_problem(cfg)
    As = A.to_scipy().tocsr()
    dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
    F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f32")
    x, info = sp.solve(dA, _dev(b), F, s=4, restart=40, rtol=1e-8)
    Fo = spand.factor(As, nested_dissection(n, n, True, False, L), cfg.b, eps)
    xo, io = krylov.sstep_gmres(lambda v: As @ v, b, lambda v: spand.apply(Fo, v), s=4,
                                rtol=1e-8, restart=40)
    lu = spl.splu(As.tocsc())
    Ainv = spl.LinearOperator(As.shape, matvec=lu.solve, rmatvec=lambda v: lu.solve(v, trans="T"))
    kappa = spl.onenormest(Ainv) * spl.norm(As, 1)
    err = np.linalg.norm(_host(x) - xo) / np.linalg.norm(xo)
    print(f"C1 FP32-spaND solve: iters {info.iters} (oracle FP64 {io.iters}), "
          f"|x - x_oracle|/|x_oracle| = {err:.3e}, kappa_1 = {kappa:.3e}")
    assert info.converged and io.converged and info.relres <= 1e-8
    assert info.iters <= math.ceil(1.1 * io.iters)
    assert err <= 2e-8 * kappa


def test_fp32_batched_vs_oracle():
    """Every system of an uneven FP32 batch (factor_batched, solve_batched)
    against the oracle: per-level ranks equal, M^-1 r within the FP32 bound,
    the batched solution within kappa(A) 2e-8 of the oracle's solve and its
    iterations within 10% of the oracle's FP64 count."""
    import scipy.sparse.linalg as spl
    from synth.dg_euler import batch_configs
    cfgs = batch_configs(6, seed=3, nmin=8, nmax=14)
    systems, rhs, probs = [], [], []
    for c in cfgs:
        A, xs, b, _ = make_problem(c)
        systems.append((sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val), c.n, c.n, True, False))
        rhs.append(_dev(b))
        probs.append((A.to_scipy().tocsr(), b))
    Ls = [sp.levels_for(c.N) for c in cfgs]
    Fs = sp.factor_batched(systems, eps=1e-2, nlevels=Ls, dtype="f32")
    xs_b, infos = sp.solve_batched([s[0] for s in systems], rhs, Fs, s=5, restart=60, rtol=1e-8)
    for i, (c, (As, b)) in enumerate(zip(cfgs, probs)):
        nd = nested_dissection(c.n, c.n, True, False, Ls[i])
        Fo = spand.factor(As, nd, c.b, 1e-2)
        st = Fs[i].stats()
        gpu = [(int(a), int(k)) for a, k in zip(st["size_before"], st["size_after"])]
        assert gpu == _levels(Fo), (i, gpu, _levels(Fo))
        Fp = spand.factor(_round32(As), nd, c.b, 1e-2)
        assert _levels(Fp) == _levels(Fo), i
        r = np.random.default_rng(100 + i).standard_normal(c.N)
        yo = spand.apply(Fo, r)
        d_in = np.linalg.norm(spand.apply(Fp, r) - yo) / np.linalg.norm(yo)
        _check(_host(Fs[i].apply(_dev(r))), yo,
               8.0 * Ls[i] * math.sqrt(_nmax(nd, c.b)) * max(d_in, U32),
               f"batched system {i} (n={c.n}, p={c.p})")
        xo, io = krylov.sstep_gmres(lambda v: As @ v, b, lambda v: spand.apply(Fo, v), s=5,
                                    rtol=1e-8, restart=60)
        lu = spl.splu(As.tocsc())
        Ainv = spl.LinearOperator(As.shape, matvec=lu.solve, rmatvec=lambda v: lu.solve(v, trans="T"))
        kappa = spl.onenormest(Ainv) * spl.norm(As, 1)
        err = np.linalg.norm(_host(xs_b[i]) - xo) / np.linalg.norm(xo)
        print(f"batched system {i}: iters {infos[i].iters} (oracle {io.iters}), err {err:.3e}, "
              f"kappa_1 {kappa:.3e}")
        assert infos[i].converged and infos[i].relres <= 1e-8
        assert infos[i].iters <= math.ceil(1.1 * io.iters), i
        assert err <= 2e-8 * kappa, i
