"""Oracle (test infrastructure only): spaND factorization, apply and apply^T.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may use
anything under oracle/; the product path never does.  Plain FP64
numpy/scipy, no blocking or fusion beyond what the method states.

Follows the paper, Sec. "Sparsified Nested Dissection algorithm":
  for every level l = 0 .. lmax-2:
    1. eliminate each level-l interior s with a row-pivoted LU A_ss = P L U
       and the Schur update A_nm -= A_ns A_ss^{-1} A_sm   (Eq. 10);
    2. scale every remaining interface with its own P L U, the diagonal of
       U split evenly between L and U (Eq. 11);
    3. compute, for every interface s, a rank-revealing QR of
       [A_sn  A_ns^T] (all neighbours n)                      (Eq. 12);
    4. only after all Q are known, compress every block
       A_ij <- Q_ic^T A_ij Q_jc and drop the f unknowns        (Eq. 13);
    5. merge clusters and go to the next level.
  The top separator is eliminated last.  The result is A ~ prod F_i used
  as a preconditioner.

Readings where the paper is silent (all listed in the design notes):
  * pivot = first index of max |a| (LAPACK getrf semantics);
  * scaling: S = diag(sqrt|u_ii|), Lh = L S, Uh = S^-1 U (sign stays in Uh);
  * W columns: neighbours in ascending cluster id, first all A_sn then all
    A_ns^T;  QRCP = LAPACK geqp3 (scipy);
  * rank k = first i with |R_ii| <= eps |R_00| (all of min(m, ncols) if
    none); eps = 0 keeps every unknown (k = |s|) with the same Q;
  * interfaces are sparsified at every level below the top.

Apply y = M^{-1} r follows from (prod L_op) A (prod R_op) ~ I:
forward over the op list applies L_op, backward in reverse applies R_op;
apply^T applies R_op^T forward and L_op^T backward.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .nd import NDResult


@dataclasses.dataclass
class Elim:
    dofs: np.ndarray
    P: np.ndarray          # permutation vector: A_ss = P L U with P = I[:, perm]
    L: np.ndarray
    U: np.ndarray
    nbr_dofs: list         # list of dof arrays of neighbours n
    A_ns: list             # |n| x |s|
    A_sn: list             # |s| x |n|
    level: int


@dataclasses.dataclass
class Scale:
    dofs: np.ndarray
    P: np.ndarray
    Lh: np.ndarray
    Uh: np.ndarray
    level: int


@dataclasses.dataclass
class Spars:
    dofs: np.ndarray
    Q: np.ndarray
    k: int
    level: int


@dataclasses.dataclass
class Factor:
    N: int
    ops: list
    ranks: list            # per level: list of (|s| before, k)
    eps: float
    L: int


def _lu(A):
    """A = P L U (getrf).  Returns perm vector p with (P^T x) = x[p]."""
    P, L, U = sla.lu(A)
    p = np.argmax(P, axis=0)      # P[:, i] = e_{p[i]}  -> (P^T x)_i = x[p[i]]
    return p, L, U


def _level0(A: sp.spmatrix, nd: NDResult, bs: int):
    cl = nd.levels[0]
    K = nd.nx * nd.ny
    which = np.empty(K, dtype=np.int64)
    dofs = []
    for ci, c in enumerate(cl):
        which[c.elems] = ci
        dofs.append((c.elems[:, None] * bs + np.arange(bs)[None, :]).reshape(-1))
    Ab = A.tocsr()
    # structural cluster adjacency from the block pattern
    B = sp.csr_matrix((np.ones(A.nnz), A.tocsr().indices, A.tocsr().indptr), shape=A.shape)
    coo = B.tocoo()
    er = coo.row // bs
    ec = coo.col // bs
    pairs = set(zip(which[er].tolist(), which[ec].tolist()))
    blocks = {}
    for (i, j) in sorted(pairs):
        blocks[(i, j)] = Ab[dofs[i]][:, dofs[j]].toarray()
    return dofs, blocks


def factor(A: sp.spmatrix, nd: NDResult, bs: int, eps: float, hook=None) -> Factor:
    """spaND factorization.  ``hook(stage, level, blocks, dofs, extra)`` is
    called after each stage (tests use it to check the Eq. (10)-(13)
    identities on the trailing matrix)."""
    N = A.shape[0]
    hook = hook or (lambda *a: None)
    L = nd.L
    dofs, blocks = _level0(A, nd, bs)
    ops = []
    ranks = []
    for lvl in range(L):
        cl = nd.levels[lvl]
        ncl = len(cl)
        alive = [len(dofs[i]) > 0 for i in range(ncl)]
        nbrs = [set() for _ in range(ncl)]
        for (i, j) in blocks:
            if i != j:
                nbrs[i].add(j)
                nbrs[j].add(i)
        # ---- 1. eliminate interiors (ascending cluster id)
        for s in range(ncl):
            if not cl[s].interior or not alive[s]:
                continue
            p, Lf, Uf = _lu(blocks[(s, s)])
            ns = sorted(n for n in nbrs[s] if alive[n])
            A_sn = [blocks[(s, n)] for n in ns]
            A_ns = [blocks[(n, s)] for n in ns]
            # X_m = A_ss^{-1} A_sm
            X = []
            for Asm in A_sn:
                y = sla.solve_triangular(Lf, Asm[p], lower=True, unit_diagonal=True)
                X.append(sla.solve_triangular(Uf, y, lower=False))
            for a, n in enumerate(ns):
                for c, m in enumerate(ns):
                    upd = A_ns[a] @ X[c]
                    if (n, m) in blocks:
                        blocks[(n, m)] = blocks[(n, m)] - upd
                    else:
                        blocks[(n, m)] = -upd
                        nbrs[n].add(m)
                        nbrs[m].add(n)
            ops.append(Elim(dofs[s].copy(), p, Lf, Uf, [dofs[n].copy() for n in ns],
                            A_ns, A_sn, lvl))
            for n in ns:
                del blocks[(s, n)], blocks[(n, s)]
                nbrs[n].discard(s)
            del blocks[(s, s)]
            alive[s] = False
            nbrs[s] = set()
        hook("elim", lvl, blocks, dofs, None)
        if lvl == L - 1:
            break
        remaining = [s for s in range(ncl) if alive[s]]
        # ---- 2. scale every remaining interface
        for s in remaining:
            p, Lf, Uf = _lu(blocks[(s, s)])
            d = np.sqrt(np.abs(np.diag(Uf)))
            Lh = Lf * d[None, :]
            Uh = Uf / d[:, None]
            for n in sorted(nbrs[s]):
                if not alive[n]:
                    continue
                blocks[(s, n)] = sla.solve_triangular(Lh, blocks[(s, n)][p], lower=True)
                blocks[(n, s)] = sla.solve_triangular(Uh, blocks[(n, s)].T, lower=False,
                                                      trans="T").T
            blocks[(s, s)] = np.eye(len(dofs[s]))
            ops.append(Scale(dofs[s].copy(), p, Lh, Uh, lvl))
        hook("scale", lvl, blocks, dofs, None)
        # ---- 3. rank-revealing QR of [A_sn  A_ns^T] for every interface
        Qs = {}
        lvl_ranks = []
        for s in remaining:
            m = len(dofs[s])
            ns = sorted(n for n in nbrs[s] if alive[n])
            cols = [blocks[(s, n)] for n in ns] + [blocks[(n, s)].T for n in ns]
            W = np.hstack(cols) if cols else np.zeros((m, 0))
            if W.shape[1] > 0:
                Q, R, _ = sla.qr(W, mode="full", pivoting=True)
            else:
                Q, R = np.eye(m), np.zeros((m, 0))
            if eps == 0.0:
                k = m
            else:
                dr = np.abs(np.diag(R))
                if dr.size == 0 or dr[0] == 0.0:
                    k = 0
                else:
                    small = np.nonzero(dr <= eps * dr[0])[0]
                    k = int(small[0]) if small.size else int(dr.size)
            Qs[s] = (Q, k)
            lvl_ranks.append((m, k))
            hook("rrqr", lvl, blocks, dofs, (s, W, Q, R, k))
        ranks.append(lvl_ranks)
        # ---- 4. compress every block with the coarse bases
        for (i, j) in list(blocks):
            Qi, ki = Qs[i]
            Qj, kj = Qs[j]
            if i == j:
                blocks[(i, j)] = np.eye(ki)
            else:
                blocks[(i, j)] = Qi[:, :ki].T @ blocks[(i, j)] @ Qj[:, :kj]
        for s in remaining:
            Q, k = Qs[s]
            ops.append(Spars(dofs[s].copy(), Q, k, lvl))
            dofs[s] = dofs[s][:k]
        # ---- 5. merge into the level-(l+1) clusters
        kids = nd.children[lvl + 1]
        ncl1 = len(nd.levels[lvl + 1])
        new_dofs = []
        parent = {}
        offs = {}
        for I in range(ncl1):
            o = 0
            parts = []
            for c in kids[I]:
                parent[c] = I
                offs[c] = o
                o += len(dofs[c])
                parts.append(dofs[c])
            new_dofs.append(np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64))
        new_blocks = {}
        for (i, j), B in blocks.items():
            if i not in parent or j not in parent:
                continue
            I, J = parent[i], parent[j]
            if (I, J) not in new_blocks:
                new_blocks[(I, J)] = np.zeros((len(new_dofs[I]), len(new_dofs[J])))
            new_blocks[(I, J)][offs[i]:offs[i] + B.shape[0], offs[j]:offs[j] + B.shape[1]] = B
        # drop empty clusters' blocks
        blocks = {k: v for k, v in new_blocks.items() if v.size > 0 or k[0] == k[1]}
        dofs = new_dofs
    return Factor(N, ops, ranks, eps, L)


# ---------------------------------------------------------------- apply

def apply(F: Factor, r: np.ndarray) -> np.ndarray:
    """y = M^{-1} r."""
    x = np.array(r, dtype=np.float64, copy=True)
    for op in F.ops:                          # forward: L_op
        if isinstance(op, Elim):
            xs = x[op.dofs]
            y = sla.solve_triangular(op.L, xs[op.P], lower=True, unit_diagonal=True)
            t = sla.solve_triangular(op.U, y, lower=False)
            x[op.dofs] = y
            for dn, Ans in zip(op.nbr_dofs, op.A_ns):
                x[dn] -= Ans @ t
        elif isinstance(op, Scale):
            x[op.dofs] = sla.solve_triangular(op.Lh, x[op.dofs][op.P], lower=True)
        else:
            x[op.dofs] = op.Q.T @ x[op.dofs]
    for op in reversed(F.ops):                # backward: R_op
        if isinstance(op, Elim):
            acc = np.zeros(len(op.dofs))
            for dn, Asn in zip(op.nbr_dofs, op.A_sn):
                acc += Asn @ x[dn]
            z = sla.solve_triangular(op.L, acc[op.P], lower=True, unit_diagonal=True)
            x[op.dofs] = sla.solve_triangular(op.U, x[op.dofs] - z, lower=False)
        elif isinstance(op, Scale):
            x[op.dofs] = sla.solve_triangular(op.Uh, x[op.dofs], lower=False)
        else:
            x[op.dofs] = op.Q @ x[op.dofs]
    return x


def _unpermute(v, p):
    """P v for the permutation vector p ((P^T x) = x[p])."""
    out = np.empty_like(v)
    out[p] = v
    return out


def apply_T(F: Factor, r: np.ndarray) -> np.ndarray:
    """y = M^{-T} r (exact transpose of ``apply``)."""
    x = np.array(r, dtype=np.float64, copy=True)
    for op in F.ops:                          # forward: R_op^T
        if isinstance(op, Elim):
            y = sla.solve_triangular(op.U, x[op.dofs], lower=False, trans="T")
            x[op.dofs] = y
            w = _unpermute(sla.solve_triangular(op.L, y, lower=True, unit_diagonal=True,
                                                trans="T"), op.P)
            for dn, Asn in zip(op.nbr_dofs, op.A_sn):
                x[dn] -= Asn.T @ w
        elif isinstance(op, Scale):
            x[op.dofs] = sla.solve_triangular(op.Uh, x[op.dofs], lower=False, trans="T")
        else:
            x[op.dofs] = op.Q.T @ x[op.dofs]
    for op in reversed(F.ops):                # backward: L_op^T
        if isinstance(op, Elim):
            acc = np.zeros(len(op.dofs))
            for dn, Ans in zip(op.nbr_dofs, op.A_ns):
                acc += Ans.T @ x[dn]
            z = sla.solve_triangular(op.U, acc, lower=False, trans="T")
            v = sla.solve_triangular(op.L, x[op.dofs] - z, lower=True, unit_diagonal=True,
                                     trans="T")
            x[op.dofs] = _unpermute(v, op.P)
        elif isinstance(op, Scale):
            v = sla.solve_triangular(op.Lh, x[op.dofs], lower=True, trans="T")
            x[op.dofs] = _unpermute(v, op.P)
        else:
            x[op.dofs] = op.Q @ x[op.dofs]
    return x


def rank_stats(F: Factor):
    """Per level (min, mean, max) of the kept ranks and total kept/size."""
    out = []
    for lr in F.ranks:
        ks = [k for _, k in lr]
        ms = [m for m, _ in lr]
        if ks:
            out.append((min(ks), float(np.mean(ks)), max(ks), sum(ks), sum(ms)))
        else:
            out.append((0, 0.0, 0, 0, 0))
    return out
