"""Oracle (test infrastructure only): reference gradients of L = g^T x.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may use
anything under oracle/; the product path never does.

With A x = b and L = g^T x: lambda = A^{-T} g, dL/db = lambda and
dL/dA = -lambda x^T; restricted to the stored blocks of the block-sparse
pattern this is dL/dA(I,J) = -lambda_I x_J^T for every stored block (I,J).
(Standard adjoint of a linear solve; the paper's Eq. (5) defines A.)
"""
from __future__ import annotations

import numpy as np

from . import direct


def dense_gradient(A, rowptr, colind, bs, b, g):
    """(x, lambda, dL/db, dL/dvals[nnzb, bs, bs]) by direct solves."""
    x = direct.solve(A, b)
    lam = direct.solve(A, g, transpose=True)
    nb = len(rowptr) - 1
    gv = np.zeros((len(colind), bs, bs))
    for I in range(nb):
        for t in range(rowptr[I], rowptr[I + 1]):
            J = colind[t]
            gv[t] = -np.outer(lam[I * bs:(I + 1) * bs], x[J * bs:(J + 1) * bs])
    return x, lam, lam.copy(), gv


def fd_directional(solve_fn, vals, b, g, dvals, db, h=1e-6):
    """Central difference of L(vals + t dvals, b + t db) at t = 0."""
    Lp = g @ solve_fn(vals + h * dvals, b + h * db)
    Lm = g @ solve_fn(vals - h * dvals, b - h * db)
    return (Lp - Lm) / (2.0 * h)
