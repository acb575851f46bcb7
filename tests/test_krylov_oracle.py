"""Pins of the GMRES / s-step GMRES oracle (Algorithms 1 and 2)."""
import os

import numpy as np
import pytest

from oracle import krylov, spand
from oracle.nd import nested_dissection
from synth.dg_euler import DGConfig, make_problem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_full_gmres_exact_on_tiny():
    rng = np.random.default_rng(0)
    n = 12
    A = rng.standard_normal((n, n)) + 4 * np.eye(n)
    b = rng.standard_normal(n)
    x, info = krylov.gmres(lambda v: A @ v, b, rtol=1e-14, restart=n)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10)
    assert info.iters <= n


def test_diagonal_k_distinct_eigs_converges_in_k():
    d = np.repeat([1.0, 2.0, 5.0, 9.0], 10)
    b = np.random.default_rng(1).standard_normal(d.size)
    x, info = krylov.gmres(lambda v: d * v, b, rtol=1e-12, restart=20)
    assert info.iters == 4 and info.converged


def test_givens_estimate_equals_true_residual():
    rng = np.random.default_rng(2)
    n = 30
    A = rng.standard_normal((n, n)) + 6 * np.eye(n)
    b = rng.standard_normal(n)
    for k in range(1, 8):
        x, info = krylov.gmres(lambda v: A @ v, b, rtol=1e-300, restart=k, maxit=k)
        assert abs(info.history[-1] - np.linalg.norm(b - A @ x)) <= 1e-12 * np.linalg.norm(b)


def test_leja_hand_example():
    with open(os.path.join(GOLD, "leja_4321.txt")) as f:
        g = {l.split()[0]: [float(t) for t in l.split()[1:]] for l in f if not l.startswith("#")}
    assert krylov.leja_order(g["input"]) == g["order"]


def test_leja_complex_pair_and_split():
    sh = krylov.leja_order([1 + 2j, 1 - 2j, 0.5])
    assert sh[0] == ("pair", 1.0, 2.0) and sh[1] == 0.5
    sh = krylov.leja_order([0.1, 1 + 2j, 1 - 2j], s=2)
    # largest modulus first = the pair (Im>0 member), which fills both slots
    assert sh == [("pair", 1.0, 2.0)]
    sh = krylov.leja_order([3.0, 1 + 1j, 1 - 1j], s=2)
    assert sh == [3.0, 1.0]            # last slot would split a pair: real part


def test_zero_shifts_give_monomial_basis():
    rng = np.random.default_rng(3)
    A = rng.standard_normal((10, 10))
    q = rng.standard_normal(10)
    W, Bb = krylov.newton_basis(lambda v: A @ v, q, krylov.shift_slots([0.0, 0.0, 0.0]))
    np.testing.assert_allclose(W, np.stack([A @ q, A @ A @ q, A @ A @ A @ q], 1), rtol=1e-13)


def test_newton_basis_change_of_basis():
    rng = np.random.default_rng(4)
    A = rng.standard_normal((12, 12))
    q = rng.standard_normal(12)
    slots = krylov.shift_slots([0.7, ("pair", 0.2, 0.9), -0.4])
    W, Bb = krylov.newton_basis(lambda v: A @ v, q, slots)
    W0 = np.column_stack([q, W])
    np.testing.assert_allclose(A @ W0[:, :4], W0 @ Bb, atol=1e-12)


def test_hessenberg_reconstruction_matches_explicit():
    rng = np.random.default_rng(5)
    n = 60
    A = rng.standard_normal((n, n)) / np.sqrt(n) + np.eye(n)
    b = rng.standard_normal(n)
    s = 4
    Q = np.zeros((n, 13)); H = np.zeros((13, 12))
    Q[:, 0] = b / np.linalg.norm(b)
    for j in range(s):                        # MGS steps
        v = A @ Q[:, j]
        for i in range(j + 1):
            H[i, j] = v @ Q[:, i]; v -= H[i, j] * Q[:, i]
        H[j + 1, j] = np.linalg.norm(v); Q[:, j + 1] = v / H[j + 1, j]
    slots = krylov.shift_slots([0.9, ("pair", 1.0, 0.2), 1.1])
    for j in (4, 8):
        W, Bb = krylov.newton_basis(lambda v: A @ v, Q[:, j], slots)
        Wn, Ra, Rb = krylov.bcgs2_cholqr2(Q[:, :j + 1], W)
        Q[:, j + 1:j + s + 1] = Wn
        H[:j + s + 1, j:j + s] = krylov.hessenberg_block(H, j, s, Ra, Rb, Bb)
    Hx = Q.T @ A @ Q[:, :12]
    np.testing.assert_allclose(H, Hx, atol=1e-12)
    assert np.abs(np.tril(H, -2)).max() < 1e-12
    assert np.linalg.norm(Q.T @ Q - np.eye(13)) < 1e-12


def _dg_problem(eps=1e-2):
    cfg = DGConfig(n=16, p=1)
    A, xs, b, _ = make_problem(cfg)
    As = A.to_scipy().tocsr()
    F = spand.factor(As, nested_dissection(16, 16, True, False, 4), cfg.b, eps)
    return As, xs, b, F


def test_s1_reproduces_classical_history():
    As, xs, b, F = _dg_problem(1e-1)
    Af = lambda v: As @ v
    Mf = lambda v: spand.apply(F, v)
    _, i1 = krylov.gmres(Af, b, Mf, rtol=1e-8, restart=40)
    _, i3 = krylov.sstep_gmres(Af, b, Mf, s=1, rtol=1e-8, restart=40)
    h1, h3 = np.array(i1.history), np.array(i3.history)
    assert len(h1) == len(h3)
    m = h1 > 1e-12 * np.linalg.norm(b)
    assert np.max(np.abs(h1[m] - h3[m]) / h1[m]) <= 1e-8


@pytest.mark.parametrize("s", [2, 4, 5])
def test_sstep_converges_like_classical(s):
    As, xs, b, F = _dg_problem(1e-1)
    Af = lambda v: As @ v
    Mf = lambda v: spand.apply(F, v)
    x1, i1 = krylov.gmres(Af, b, Mf, rtol=1e-8, restart=40)
    x2, i2 = krylov.sstep_gmres(Af, b, Mf, s=s, rtol=1e-8, restart=40)
    assert i2.converged and abs(i2.iters - i1.iters) <= 1
    assert np.linalg.norm(b - As @ x2) <= 1e-8 * np.linalg.norm(b)


def test_sstep_restarts_unpreconditioned():
    As, xs, b, F = _dg_problem()
    x, info = krylov.sstep_gmres(lambda v: As @ v, b, None, s=4, rtol=1e-8, restart=40)
    assert info.converged and info.restarts > 1
    assert np.linalg.norm(b - As @ x) <= 1e-8 * np.linalg.norm(b)


# ---- stability-study variants (monomial basis, one orthogonalisation pass)

def test_one_pass_decomposition_identity():
    """One block CGS + CholQR pass: W = Q R_a + Wnew R_b exactly (up to
    rounding), Wnew orthonormal, R_b upper triangular."""
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((200, 7)))
    W = rng.standard_normal((200, 4))
    Wn, Ra, Rb = krylov.bcgs_cholqr(Q, W)
    assert np.linalg.norm(Q @ Ra + Wn @ Rb - W) <= 1e-12 * np.linalg.norm(W)
    assert np.linalg.norm(Wn.T @ Wn - np.eye(4)) <= 1e-12
    assert np.allclose(Rb, np.triu(Rb))


def test_two_passes_keep_orthogonality_one_pass_loses_it():
    """The study's claim in small: on an ill-conditioned monomial basis one
    CGS + CholQR pass leaves orders of magnitude more loss of orthogonality
    than two; both still converge on this well-conditioned system."""
    As, xs, b, F = _dg_problem(1e-1)
    Af = lambda v: As @ v
    Mf = lambda v: spand.apply(F, v)
    zs = [0.0] * 5
    x2, i2 = krylov.sstep_gmres(Af, b, Mf, s=5, rtol=1e-8, restart=40, shifts=zs, record_Q=True)
    x1, i1 = krylov.sstep_gmres(Af, b, Mf, s=5, rtol=1e-8, restart=40, shifts=zs, record_Q=True,
                                passes=1)
    assert i2.converged and i1.converged
    assert max(i2.orth_err) <= 1e-12
    assert max(i1.orth_err) >= 100 * max(i2.orth_err)
    for x in (x1, x2):
        assert np.linalg.norm(b - As @ x) <= 1e-8 * np.linalg.norm(b)


# ---- single-reduce schedule (Algorithm 2, second pass lagged by one block)

def test_lagged_step_identities():
    """One single-reduce step, checked by rebuilding its inputs from its
    outputs: P = Q_old R1 + Phat T, W = [Q_old, Phat] C + What RV, the whole
    basis orthonormal, T and RV upper triangular."""
    rng = np.random.default_rng(11)
    n, a, s = 300, 9, 4
    Qo, _ = np.linalg.qr(rng.standard_normal((n, a)))
    # a previous block after one pass: orthonormal, slightly off Q_old
    P, _ = np.linalg.qr(rng.standard_normal((n, s)) - Qo @ (Qo.T @ rng.standard_normal((n, s))))
    P = P + 1e-6 * Qo @ rng.standard_normal((a, s))
    W = rng.standard_normal((n, s))
    Q = np.hstack([Qo, P, W])
    P0, W0 = P.copy(), W.copy()
    st = krylov.lagged_reduce_step(Q, a, s, s)
    assert st.T is not None and st.RV is not None
    assert np.linalg.norm(Qo @ st.R1 + Q[:, a:a + s] @ st.T - P0) <= 1e-13 * np.linalg.norm(P0)
    assert np.linalg.norm(Q[:, :a + s] @ st.C + Q[:, a + s:] @ st.RV - W0) \
        <= 1e-12 * np.linalg.norm(W0)
    assert np.linalg.norm(Q.T @ Q - np.eye(a + 2 * s)) <= 1e-12
    assert np.allclose(st.T, np.triu(st.T)) and np.allclose(st.RV, np.triu(st.RV))
    # the end-of-cycle step (no new block) and the first step (no previous one)
    Q2 = np.hstack([Qo, P0])
    st2 = krylov.lagged_reduce_step(Q2, a, s, 0)
    assert st2.C is None and np.allclose(st2.T, st.T, rtol=1e-12, atol=1e-14)
    Q3 = np.hstack([Qo, W0])
    st3 = krylov.lagged_reduce_step(Q3, a, 0, s)
    assert np.linalg.norm(Qo @ st3.C + Q3[:, a:] @ st3.RV - W0) <= 1e-12 * np.linalg.norm(W0)
    assert np.linalg.norm(Q3.T @ Q3 - np.eye(a + s)) <= 1e-12


@pytest.mark.parametrize("s", [2, 4, 5])
def test_lagged_history_matches_two_pass_and_classical(s):
    """In exact arithmetic the lagged schedule yields the basis, Hessenberg
    matrix and residual history of the non-lagged one, and s-step GMRES
    those of classical GMRES."""
    As, xs, b, F = _dg_problem(1e-1)
    Af = lambda v: As @ v
    Mf = lambda v: spand.apply(F, v)
    _, i1 = krylov.gmres(Af, b, Mf, rtol=1e-8, restart=40)
    _, i2 = krylov.sstep_gmres(Af, b, Mf, s=s, rtol=1e-8, restart=40)
    x3, i3 = krylov.sstep_gmres(Af, b, Mf, s=s, rtol=1e-8, restart=40, lagged=True,
                                record_Q=True)
    assert i3.converged and i3.iters == i2.iters and abs(i3.iters - i1.iters) <= 1
    h1, h2, h3 = (np.array(i.history) for i in (i1, i2, i3))
    nn = min(len(h1), len(h3))
    assert np.max(np.abs(h3 - h2) / h2) <= 1e-7
    assert np.max(np.abs(h3[:nn] - h1[:nn]) / h1[:nn]) <= 1e-6
    assert max(i3.orth_err) <= 1e-12
    assert np.linalg.norm(b - As @ x3) <= 1e-8 * np.linalg.norm(b)


def test_lagged_restarts_and_monomial():
    """Restarted cycles (the last block of each gets its own second pass) and
    the monomial basis under the lagged schedule."""
    As, xs, b, F = _dg_problem()
    x, info = krylov.sstep_gmres(lambda v: As @ v, b, None, s=4, rtol=1e-8, restart=40,
                                 lagged=True)
    _, ref = krylov.sstep_gmres(lambda v: As @ v, b, None, s=4, rtol=1e-8, restart=40)
    assert info.converged and info.restarts > 1 and info.restarts == ref.restarts
    assert abs(info.iters - ref.iters) <= 1
    assert np.linalg.norm(b - As @ x) <= 1e-8 * np.linalg.norm(b)
    As2, xs2, b2, F2 = _dg_problem(1e-1)
    Mf = lambda v: spand.apply(F2, v)
    zs = [0.0] * 5
    x2, i2 = krylov.sstep_gmres(lambda v: As2 @ v, b2, Mf, s=5, rtol=1e-8, restart=40,
                                shifts=zs, lagged=True, record_Q=True)
    assert i2.converged and max(i2.orth_err) <= 1e-12
    assert np.linalg.norm(b2 - As2 @ x2) <= 1e-8 * np.linalg.norm(b2)
