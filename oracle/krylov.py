"""Oracle (test infrastructure only): classical GMRES and s-step GMRES.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may use
anything under oracle/; the product path never does.  Plain FP64 numpy.

Classical GMRES follows the paper's Algorithm 1 (SpMV, modified
Gram-Schmidt, Givens rotations, convergence check, least squares, update).
s-step GMRES follows Algorithm 2 and the stability measures of the paper's
CAGMRES section: s basis vectors per block from s operator applications
in a Newton basis whose shifts are Ritz values of s steps of standard
GMRES in Leja order for real arithmetic, block classical Gram-Schmidt
against the previous basis and Cholesky QR, each done twice ("two CGS
and two CholQR"), then Hessenberg assembly, Givens rotations and the
convergence check.

Readings where the paper is silent:
  * right preconditioning, A_hat = A M^{-1}; x0 = 0 unless given; converged
    when ||b - A x|| <= rtol ||b|| (the estimate |g_{k+1}| is checked after
    every column, the true residual at the end of every cycle);
  * iteration count = number of Krylov vectors used (A_hat applications
    whose column enters the least-squares problem);
  * Ritz values from the first s MGS steps of the first cycle (these steps
    count as iterations and give the first s basis vectors); the shifts are
    reused for every later block and restart;
  * Leja order: largest modulus first, then the maximiser of the sum of
    log-distances to the chosen values; ties -> larger real part, then
    larger imaginary part; a value with Im > 0 is followed by its
    conjugate; if the last slot would split a pair its real part is used;
  * by default the two passes are not lagged (block CGS2 + CholQR2); the
    Hessenberg columns of a block are recovered from the change-of-basis
    matrix and the orthogonalisation coefficients:
      H[:, j:j+s] = (Rhat Bbar - [H[0:j+1, 0:j] Rhat[0:j, 0:s]; 0]) T^{-1},
    Rhat = [[rho, R_a], [0, R_b]], T = Rhat[j:j+s, 0:s], where rho holds
    the coefficients of the block's starting vector on Q[:, 0:j+1] (e_j
    when it is the final basis vector q_j);
  * lagged=True is Algorithm 2's single-reduce schedule: the operator
    applications of a block start from the last vector of the previous
    block after its first pass only; one Gram matrix
    Q[:, 0:j+s+1]^T [P, W] then gives the second pass of the previous block
    P (re-orthogonalisation and re-normalisation), its Hessenberg columns,
    the Givens rotations and the convergence check, and the first pass of
    the new block W against the re-orthogonalised basis (the coefficients
    on the new P are T^{-T}(P^T W - R_1^T Q_old^T W), its Gram matrix
    W^T W - C^T C); the last block of a cycle gets its second pass from a
    reduction of its own.  In exact arithmetic the basis, the Hessenberg
    matrix and the residual history are those of the non-lagged schedule.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass
class SolveInfo:
    iters: int = 0
    restarts: int = 0
    converged: bool = False
    history: list = dataclasses.field(default_factory=list)   # |g| after each column
    relres: float = float("nan")
    shifts: list = dataclasses.field(default_factory=list)
    breakdown: bool = False


def _givens(a, b):
    if b == 0.0:
        return 1.0, 0.0, a
    r = math.hypot(a, b)
    return a / r, b / r, r


class _LSQ:
    """Incremental Givens QR of the Hessenberg matrix (Alg. 1 lines 10-14)."""

    def __init__(self, m, beta):
        self.cs = np.zeros(m)
        self.sn = np.zeros(m)
        self.g = np.zeros(m + 1)
        self.g[0] = beta
        self.Rm = np.zeros((m + 1, m))

    def add_column(self, j, h):
        h = np.array(h[:j + 2], dtype=np.float64, copy=True)
        for i in range(j):
            t = self.cs[i] * h[i] + self.sn[i] * h[i + 1]
            h[i + 1] = -self.sn[i] * h[i] + self.cs[i] * h[i + 1]
            h[i] = t
        c, s, r = _givens(h[j], h[j + 1])
        self.cs[j], self.sn[j] = c, s
        h[j], h[j + 1] = r, 0.0
        self.Rm[:j + 2, j] = h
        self.g[j + 1] = -s * self.g[j]
        self.g[j] = c * self.g[j]
        return abs(self.g[j + 1])

    def solve(self, k):
        """y solving the k x k triangular system."""
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):
            y[i] = (self.g[i] - self.Rm[i, i + 1:k] @ y[i + 1:k]) / self.Rm[i, i]
        return y


def gmres(A, b, M=None, x0=None, rtol=1e-8, restart=40, maxit=1000):
    """Classical restarted GMRES, right preconditioned.  A, M: callables."""
    Mf = M if M is not None else (lambda v: v)
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    info = SolveInfo()
    if bnorm == 0.0:
        info.converged, info.relres = True, 0.0
        return np.zeros(n), info
    tol = rtol * bnorm
    while True:
        r = b - A(x)
        beta = np.linalg.norm(r)
        info.relres = beta / bnorm
        if beta <= tol:
            info.converged = True
            return x, info
        if info.iters >= maxit:
            return x, info
        Q = np.zeros((n, restart + 1))
        Q[:, 0] = r / beta
        lsq = _LSQ(restart, beta)
        k = 0
        for j in range(restart):
            v = A(Mf(Q[:, j]))
            h = np.zeros(j + 2)
            for i in range(j + 1):                      # MGS
                h[i] = v @ Q[:, i]
                v = v - h[i] * Q[:, i]
            h[j + 1] = np.linalg.norm(v)
            info.iters += 1
            est = lsq.add_column(j, h)
            info.history.append(est)
            k = j + 1
            if h[j + 1] == 0.0 or est <= tol or info.iters >= maxit:
                break
            Q[:, j + 1] = v / h[j + 1]
        y = lsq.solve(k)
        x = x + Mf(Q[:, :k] @ y)
        info.restarts += 1


# ------------------------------------------------------------ s-step pieces

def _tie_key(z):
    return (z.real, z.imag)


def leja_order(vals, s=None, rtol=1e-12):
    """Leja ordering of Ritz values for real arithmetic.

    Returns a list of s shifts, each a real float or a tuple ('pair', a, b)
    standing for the two slots a +- ib.
    """
    vals = [complex(v) for v in vals]
    s = len(vals) if s is None else s
    remaining = list(vals)
    chosen = []

    def better(score, z, best_score, best_z):
        if best_z is None:
            return True
        if score > best_score + rtol * max(1.0, abs(best_score)):
            return True
        if score < best_score - rtol * max(1.0, abs(best_score)):
            return False
        return _tie_key(z) > _tie_key(best_z)

    while remaining and len(chosen) < s:
        best, best_score = None, None
        for z in remaining:
            if not chosen:
                score = abs(z)
            else:
                d = [abs(z - c) for c in chosen]
                score = -math.inf if min(d) == 0.0 else sum(math.log(t) for t in d)
            if better(score, z, best_score, best):
                best, best_score = z, score
        if best.imag != 0.0:
            zp = complex(best.real, abs(best.imag))
            zm = zp.conjugate()
            remaining.remove(min(remaining, key=lambda t: abs(t - zp)))
            remaining.remove(min(remaining, key=lambda t: abs(t - zm)))
            chosen += [zp, zm]
        else:
            remaining.remove(best)
            chosen.append(best)
    chosen = chosen[:s]
    out = []
    i = 0
    while i < len(chosen):
        z = chosen[i]
        if z.imag > 0.0:
            if i + 1 < len(chosen):
                out.append(("pair", z.real, z.imag))
                i += 2
                continue
            out.append(z.real)      # last slot would split a pair
        else:
            out.append(z.real)
        i += 1
    return out


def shift_slots(shifts):
    """Flatten shifts into per-slot (kind, a, b): kind 0 real, 1/2 pair slots."""
    slots = []
    for sh in shifts:
        if isinstance(sh, tuple):
            slots.append((1, sh[1], sh[2]))
            slots.append((2, sh[1], sh[2]))
        else:
            slots.append((0, float(sh), 0.0))
    return slots


def newton_basis(Ahat, w0, slots):
    """w_k = (A_hat - theta_k) w_{k-1}; pairs a+-ib in real arithmetic.
    Returns W [n, s] and the change-of-basis matrix Bbar [(s+1), s]."""
    s = len(slots)
    n = w0.shape[0]
    W = np.zeros((n, s + 1))
    W[:, 0] = w0
    Bb = np.zeros((s + 1, s))
    for k in range(1, s + 1):
        kind, a, b = slots[k - 1]
        v = Ahat(W[:, k - 1])
        if kind == 0:
            W[:, k] = v - a * W[:, k - 1]
            Bb[k - 1, k - 1] = a
            Bb[k, k - 1] = 1.0
        elif kind == 1:
            W[:, k] = v - a * W[:, k - 1]
            Bb[k - 1, k - 1] = a
            Bb[k, k - 1] = 1.0
        else:
            W[:, k] = v - a * W[:, k - 1] + b * b * W[:, k - 2]
            Bb[k - 2, k - 1] = -b * b
            Bb[k - 1, k - 1] = a
            Bb[k, k - 1] = 1.0
    return W[:, 1:], Bb


def _chol_upper(G):
    """Upper Cholesky factor T with G = T^T T, or None if G is not SPD."""
    try:
        Lc = np.linalg.cholesky(G)
    except np.linalg.LinAlgError:
        return None
    return Lc.T


def bcgs2_cholqr2(Q, W):
    """Two passes of block CGS + CholQR.  Returns (Wnew, R_a, R_b) with
    W = Q R_a + Wnew R_b, or None on breakdown (Gram not SPD)."""
    R1 = Q.T @ W
    W1 = W - Q @ R1
    T1 = _chol_upper(W1.T @ W1)
    if T1 is None:
        return None
    W1 = np.linalg.solve(T1.T, W1.T).T          # W1 T1^{-1}
    R2 = Q.T @ W1
    W2 = W1 - Q @ R2
    T2 = _chol_upper(W2.T @ W2)
    if T2 is None:
        return None
    W2 = np.linalg.solve(T2.T, W2.T).T
    return W2, R1 + R2 @ T1, T2 @ T1


def bcgs_cholqr(Q, W):
    """One pass of block CGS + CholQR (the single-pass variant of the
    stability study).  Returns (Wnew, R_a, R_b) with W = Q R_a + Wnew R_b, or
    None on breakdown."""
    R1 = Q.T @ W
    W1 = W - Q @ R1
    T1 = _chol_upper(W1.T @ W1)
    if T1 is None:
        return None
    W1 = np.linalg.solve(T1.T, W1.T).T
    return W1, R1, T1


def hessenberg_block(H, j, s, Ra, Rb, Bb, rho=None):
    """Columns j..j+s-1 of the Hessenberg matrix of A_hat in the basis Q.
    rho: coefficients of the block's starting vector on Q[:, 0:j+1]
    (default e_j, the starting vector is q_j itself)."""
    nr = j + 1 + s
    Rhat = np.zeros((nr, s + 1))
    if rho is None:
        Rhat[j, 0] = 1.0
    else:
        Rhat[:j + 1, 0] = rho
    Rhat[:j + 1, 1:] = Ra
    Rhat[j + 1:, 1:] = Rb
    RB = Rhat @ Bb
    if j > 0:
        RB[:j + 1] -= H[:j + 1, :j] @ Rhat[:j, :s]
    T = Rhat[j:j + s, :s]
    return np.linalg.solve(T.T, RB.T).T          # RB T^{-1}


class LagStep:
    """Coefficients of one single-reduce step: P = Q_old R1 + Phat T (second
    pass of the previous block) and W = Q[:, 0:a+sp] C + What RV (first pass
    of the new block).  Any of them is None when absent or on breakdown."""

    def __init__(self):
        self.R1 = self.T = self.C = self.RV = None


def lagged_reduce_step(Q, a, sp, sw):
    """One step of Algorithm 2's single-reduce orthogonalisation, in place.

    Q[:, 0:a] is final and orthonormal, Q[:, a:a+sp] the previous block after
    its first pass (sp = 0 in the first block of a cycle) and Q[:, a+sp:a+sp+sw]
    the new block from the operator applications (sw = 0 for the second pass
    of the last block of a cycle).  The only inner products taken are the
    single Gram matrix G = Q[:, 0:a+sp+sw]^T Q[:, a:a+sp+sw]; everything else
    follows from it.  Breakdown (a Gram matrix that is not positive definite)
    leaves the corresponding coefficients None."""
    st = LagStep()
    G = Q[:, :a + sp + sw].T @ Q[:, a:a + sp + sw]          # the single reduction
    if sp:
        R1 = G[:a, :sp]
        T = _chol_upper(G[a:a + sp, :sp] - R1.T @ R1)       # Gram of P - Q_old R1
        if T is None:
            return st
        st.R1, st.T = R1, T
        P1 = Q[:, a:a + sp] - Q[:, :a] @ R1                 # re-orthogonalise
        Q[:, a:a + sp] = np.linalg.solve(T.T, P1.T).T       # re-normalise
    if sw:
        C = G[:a, sp:]
        if sp:
            # coefficients on the re-orthogonalised P from the same Gram matrix
            CP = np.linalg.solve(st.T.T, G[a:a + sp, sp:] - st.R1.T @ C)
            C = np.vstack([C, CP])
        RV = _chol_upper(G[a + sp:, sp:] - C.T @ C)
        if RV is None:
            return st
        st.C, st.RV = C, RV
        W1 = Q[:, a + sp:a + sp + sw] - Q[:, :a + sp] @ C   # orthogonalise (one pass)
        Q[:, a + sp:a + sp + sw] = np.linalg.solve(RV.T, W1.T).T
    return st


def sstep_gmres(A, b, M=None, x0=None, s=4, rtol=1e-8, restart=40, maxit=1000,
                shifts=None, record_Q=False, passes=2, lagged=False):
    """s-step GMRES, right preconditioned; restart must be a multiple of s.
    shifts = zeros gives the monomial basis; passes = 1 orthogonalises each
    block once (block CGS + CholQR) instead of twice; lagged = True uses the
    single-reduce schedule (second pass lagged by one block); record_Q keeps
    ||Q^T Q - I||_F of the final basis after every block in info.orth_err."""
    assert restart % s == 0 and restart >= s
    assert passes in (1, 2)
    assert not (lagged and passes == 1)
    Mf = M if M is not None else (lambda v: v)
    Ahat = lambda v: A(Mf(v))
    n = b.shape[0]
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    info = SolveInfo()
    if bnorm == 0.0:
        info.converged, info.relres = True, 0.0
        return np.zeros(n), info
    tol = rtol * bnorm
    m = restart
    first = True
    slots = None if shifts is None else shift_slots(shifts)
    info.shifts = shifts
    orth_err = []
    while True:
        r = b - A(x)
        beta = np.linalg.norm(r)
        info.relres = beta / bnorm
        if beta <= tol:
            info.converged = True
            break
        if info.iters >= maxit:
            break
        Q = np.zeros((n, m + 1))
        H = np.zeros((m + 1, m))
        Q[:, 0] = r / beta
        lsq = _LSQ(m, beta)
        k = 0
        done = False
        j = 0
        if first and slots is None:
            # s classical steps: Ritz values for the Newton shifts
            for jj in range(s):
                v = Ahat(Q[:, jj])
                h = np.zeros(jj + 2)
                for i in range(jj + 1):
                    h[i] = v @ Q[:, i]
                    v = v - h[i] * Q[:, i]
                h[jj + 1] = np.linalg.norm(v)
                H[:jj + 2, jj] = h
                info.iters += 1
                est = lsq.add_column(jj, h)
                info.history.append(est)
                k = jj + 1
                if h[jj + 1] == 0.0 or est <= tol or info.iters >= maxit:
                    done = True
                    break
                Q[:, jj + 1] = v / h[jj + 1]
            theta = np.linalg.eigvals(H[:s, :s]) if not done else np.zeros(s)
            shifts = leja_order(theta, s)
            info.shifts = shifts
            slots = shift_slots(shifts)
            j = s
        first = False
        pend = None      # (j0, R_a, R_b, rho) of the block in Q[:, j0+1:j0+s+1]
        while lagged and not done:
            sw = s if j < m else 0
            if pend is None and sw == 0:
                break
            if sw:
                W, Bb = newton_basis(Ahat, Q[:, j], slots)
                Q[:, j + 1:j + s + 1] = W
            sp = s if pend is not None else 0
            st = lagged_reduce_step(Q, j + 1 - sp, sp, sw)
            if sp:
                if st.T is None:
                    info.breakdown = True
                    k = pend[0]
                    break
                j0, Ra0, Rb0, rho0 = pend
                H[:j0 + s + 1, j0:j0 + s] = hessenberg_block(
                    H, j0, s, Ra0 + st.R1 @ Rb0, st.T @ Rb0, Bb, rho0)
                if record_Q:
                    nq = j0 + s + 1
                    orth_err.append(np.linalg.norm(Q[:, :nq].T @ Q[:, :nq] - np.eye(nq)))
                for c in range(j0, j0 + s):
                    info.iters += 1
                    est = lsq.add_column(c, H[:c + 2, c])
                    info.history.append(est)
                    k = c + 1
                    if est <= tol or info.iters >= maxit:
                        done = True
                        break
            if done or not sw:
                pend = None
                continue
            if st.RV is None:
                info.breakdown = True
                break
            if sp:
                rho = np.concatenate([st.R1[:, -1], st.T[:, -1]])
            else:
                rho = np.zeros(j + 1)
                rho[j] = 1.0
            pend = (j, st.C, st.RV, rho)
            j += s
        while not lagged and not done and j < m:
            W, Bb = newton_basis(Ahat, Q[:, j], slots)
            res = (bcgs2_cholqr2 if passes == 2 else bcgs_cholqr)(Q[:, :j + 1], W)
            if res is None:
                info.breakdown = True
                done = True
                break
            Wn, Ra, Rb = res
            Q[:, j + 1:j + s + 1] = Wn
            H[:j + s + 1, j:j + s] = hessenberg_block(H, j, s, Ra, Rb, Bb)
            if record_Q:
                orth_err.append(np.linalg.norm(Q[:, :j + s + 1].T @ Q[:, :j + s + 1]
                                               - np.eye(j + s + 1)))
            for c in range(j, j + s):
                info.iters += 1
                est = lsq.add_column(c, H[:c + 2, c])
                info.history.append(est)
                k = c + 1
                if est <= tol or info.iters >= maxit:
                    done = True
                    break
            j += s
        if k > 0:
            y = lsq.solve(k)
            x = x + Mf(Q[:, :k] @ y)
        info.restarts += 1
        if info.breakdown:
            r = b - A(x)
            info.relres = np.linalg.norm(r) / bnorm
            info.converged = info.relres <= rtol
            break
    if record_Q:
        info.orth_err = orth_err
    return x, info
