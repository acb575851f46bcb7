"""Pseudo-transient continuation on the GPU solver (paper Sec. "Flow Solver").

Every pseudo-time step n solves the backward-Euler system of Eq. (5),
(M/dtau^n + dR/du) du = -R^n, with dtau^n = min_k CFL^n / lambda_k (Eq. (8))
and CFL^n = min(CFL^0 |R^0| / |R^{n-1}|, CFL^inf) (Eq. (9)), until the
density residual has dropped by `orders` orders of magnitude.

The residual, the Jacobian values and lambda_k come from the caller's
assembly on the host, evaluated at the current state; their values are
streamed to the device every step.  The linear system is factored with spaND
on the device: the first step by spand_factor, every later step by
spand_refactor, which reuses the first step's symbolic phase (block pattern
and nested dissection; the paper partitions once, in pre-processing, and
factors at every nonlinear step).  It is solved by s-step GMRES with that
preconditioner to the relative tolerance `rtol` (the paper's experiments
solve to 1e-3).  The state lives on the host, where the assembly needs it.
"""
from __future__ import annotations

import dataclasses
import time

import numpy as np

from . import BSRMatrix, factor, solve


@dataclasses.dataclass
class PTCResult:
    steps: int = 0
    converged: bool = False
    res_norm: list = dataclasses.field(default_factory=list)    # |R^n|, n = 0, 1, ...
    rho_norm: list = dataclasses.field(default_factory=list)    # density components
    cfl: list = dataclasses.field(default_factory=list)         # CFL^n, n = 1, ...
    dtau: list = dataclasses.field(default_factory=list)
    lin_iters: list = dataclasses.field(default_factory=list)
    t_assemble_s: float = 0.0      # host residual + Jacobian + lambda
    t_upload_s: float = 0.0        # host -> device Jacobian values and right-hand side
    t_factor_s: float = 0.0        # spand_factor / spand_refactor
    t_solve_s: float = 0.0         # s-step GMRES


def _rho(R):
    return float(np.linalg.norm(R.reshape(-1, 4)[:, 0]))


def ptc_solve(grid, residual, jacobian, lambdas, u0, cfl0=1000.0, cfl_inf=1e8, orders=8.0,
              max_steps=100, eps=1e-2, nlevels=0, dtype="f32", s=5, restart=60, rtol=1e-3,
              maxit=1000, lagged=True):
    """grid = (nx, ny, periodic_x, periodic_y); residual(u) -> R (numpy);
    jacobian(u, dtau) -> (rowptr, colind, val [nnzb, b, b]) of M/dtau + dR/du;
    lambdas(u) -> lambda_k per element; u0 numpy vector.  Returns (u, PTCResult)."""
    import torch
    nx, ny, px, py = grid
    u = np.array(u0, dtype=np.float64, copy=True)
    res = PTCResult()
    t = time.perf_counter()
    R = residual(u)
    res.t_assemble_s += time.perf_counter() - t
    r0 = float(np.linalg.norm(R))
    d0 = _rho(R)
    res.res_norm.append(r0)
    res.rho_norm.append(d0)
    if d0 == 0.0:
        res.converged = True
        return u, res
    dA, F, rprev = None, None, r0
    for n in range(1, max_steps + 1):
        cfl = min(cfl0 * r0 / rprev, cfl_inf)
        t = time.perf_counter()
        dtau = float(np.min(cfl / lambdas(u)))
        rowptr, colind, val = jacobian(u, dtau)
        t1 = time.perf_counter()
        if dA is None:
            dA = BSRMatrix.from_numpy(rowptr, colind, val)
        else:
            dA.val.copy_(torch.from_numpy(np.ascontiguousarray(val, dtype=np.float64)))
        rhs = torch.as_tensor(-R, device="cuda")
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if F is None:
            F = factor(dA, nx, ny, px, py, eps=eps, nlevels=nlevels, dtype=dtype)
        else:
            F.refactor(dA)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        du, info = solve(dA, rhs, F, s=s, restart=restart, rtol=rtol, maxit=maxit, lagged=lagged)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        u += du.cpu().numpy()
        t5 = time.perf_counter()
        R = residual(u)
        t6 = time.perf_counter()
        rprev = float(np.linalg.norm(R))
        res.t_assemble_s += (t1 - t) + (t6 - t5)
        res.t_upload_s += (t2 - t1) + (t5 - t4)
        res.t_factor_s += t3 - t2
        res.t_solve_s += t4 - t3
        res.steps = n
        res.cfl.append(cfl)
        res.dtau.append(dtau)
        res.lin_iters.append(info.iters)
        res.res_norm.append(rprev)
        res.rho_norm.append(_rho(R))
        if res.rho_norm[-1] <= 10.0 ** (-orders) * d0:
            res.converged = True
            break
    return u, res
