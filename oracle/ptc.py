"""Oracle (test infrastructure only): the pseudo-transient nonlinear loop.

Only tests/, the smoke check and the benchmark's CPU-baseline leg may use
anything under oracle/; the product path never does.  Plain FP64 numpy.

Follows the paper, Sec. "Flow Solver": every pseudo-time step n solves the
backward-Euler system of Eq. (5),
    (M / dtau^n + dR/du|^n) du = -R^n,   u^{n+1} = u^n + du,
with the time step of Eq. (8), dtau = min_k CFL / lambda_k, and the CFL
number of Eq. (9),
    CFL^n = min(CFL^0 |R^0| / |R^{n-1}|, CFL^inf),
until the density residual has dropped by the requested number of orders
(8 in the paper's experiments, Sec. "Numerical results").  The residual,
Jacobian and lambda_k come from the caller (the shared input generator);
the linear solve is a callable (exact, or spaND-preconditioned s-step
GMRES as the paper does).

Readings where the paper is silent (listed in the design notes):
  * |R| in Eq. (9) is the Euclidean norm of the whole residual vector; the
    stopping test uses the density components (variable 0 of every mode);
  * the first step (n = 1) uses CFL^1 = CFL^0 (|R^0| / |R^0| = 1);
  * the LF spectral radius of the residual and of its Jacobian is frozen at
    the element means of the current state; lambda_k of Eq. (8) is taken at
    the same element means;
  * CFL^inf is a parameter (the paper gives none).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class PTCInfo:
    steps: int = 0
    converged: bool = False
    res_norm: list = dataclasses.field(default_factory=list)     # |R^n|, n = 0, 1, ...
    rho_norm: list = dataclasses.field(default_factory=list)     # density part
    cfl: list = dataclasses.field(default_factory=list)          # CFL^n, n = 1, ...
    dtau: list = dataclasses.field(default_factory=list)
    lin_iters: list = dataclasses.field(default_factory=list)


def density_norm(R: np.ndarray) -> float:
    """Norm of the density components (local dof index 4m + 0)."""
    return float(np.linalg.norm(R.reshape(-1, 4)[:, 0]))


def ptc(u0, residual, jacobian, lambdas, linear_solve, cfl0=1000.0, cfl_inf=1e8, orders=8.0,
        max_steps=100):
    """Pseudo-transient continuation from u0 (a vector of modal coefficients).

    residual(u) -> R (vector), jacobian(u, dtau) -> sparse A = M/dtau + dR/du,
    lambdas(u) -> lambda_k per element, linear_solve(A, rhs) -> (du, iters).
    Returns (u, PTCInfo)."""
    u = np.array(u0, dtype=np.float64, copy=True)
    info = PTCInfo()
    R = residual(u)
    r0 = float(np.linalg.norm(R))
    d0 = density_norm(R)
    info.res_norm.append(r0)
    info.rho_norm.append(d0)
    if d0 == 0.0:
        info.converged = True
        return u, info
    rprev = r0
    for n in range(1, max_steps + 1):
        cfl = min(cfl0 * r0 / rprev, cfl_inf)                  # Eq. (9)
        dtau = float(np.min(cfl / lambdas(u)))                 # Eq. (8)
        A = jacobian(u, dtau)                                  # Eq. (5), left side
        du, it = linear_solve(A, -R)
        u = u + du
        R = residual(u)
        rprev = float(np.linalg.norm(R))
        info.steps = n
        info.cfl.append(cfl)
        info.dtau.append(dtau)
        info.lin_iters.append(it)
        info.res_norm.append(rprev)
        info.rho_norm.append(density_norm(R))
        if info.rho_norm[-1] <= 10.0 ** (-orders) * d0:
            info.converged = True
            break
    return u, info
