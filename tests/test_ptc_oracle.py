"""Pins of the pseudo-transient loop's oracle (oracle/ptc.py) and of the
generator's Jacobian at a general state (synth.dg_euler.jacobian), CPU only:
  * the Jacobian is the derivative of the quadrature residual (central
    finite differences) and reduces to the closed-form operator of
    ``assemble`` at element-constant states;
  * a free-stream start is already steady (R = 0, no step);
  * with exact linear solves and CFL growing to infinity the loop is Newton's
    method: quadratic convergence of the residual;
  * a tiny CFL makes the first step explicit Euler in pseudo time,
    du = -dtau M^-1 R + O(dtau^2) with M = (h/2)^2 I;
  * Eq. (8): dtau is CFL over the largest lambda_k; Eq. (9): CFL^n grows by
    the residual reduction and stops at CFL^inf.
"""
import numpy as np
import pytest

from oracle import direct, ptc
from synth.dg_euler import (DGConfig, assemble, element_means, freestream, initial_state,
                            jacobian, local_lambda, residual, state_to_modal)


def _callables(cfg):
    def res(u):
        uh = u.reshape(cfg.K, -1, 4)
        return residual(cfg, uh, element_means(cfg, uh)).reshape(-1)

    def jac(u, dtau):
        uh = u.reshape(cfg.K, -1, 4)
        return jacobian(cfg, uh, element_means(cfg, uh), dtau).to_scipy().tocsr()

    def lam(u):
        return local_lambda(cfg, element_means(cfg, u.reshape(cfg.K, -1, 4)))

    return res, jac, lam


def _exact(A, b):
    return direct.solve(A, b), 0


@pytest.mark.parametrize("p", [1, 2])
def test_jacobian_is_residual_derivative(p):
    cfg = DGConfig(n=3, p=p)
    uh = initial_state(cfg)
    uh = uh + 0.01 * np.random.default_rng(1).standard_normal(uh.shape) * np.abs(uh).max()
    lam = element_means(cfg, uh)
    J = jacobian(cfg, uh, lam, None).to_scipy().toarray()
    x0 = uh.reshape(-1)

    def fd(h):
        Jfd = np.empty_like(J)
        for i in range(x0.size):
            e = np.zeros(x0.size)
            e[i] = h
            Jfd[:, i] = (residual(cfg, (x0 + e).reshape(uh.shape), lam).reshape(-1)
                         - residual(cfg, (x0 - e).reshape(uh.shape), lam).reshape(-1)) / (2 * h)
        return np.abs(J - Jfd).max() / np.abs(J).max()

    # central differences converge to J at second order in h
    e1, e2 = fd(1e-5), fd(1e-6)
    assert e2 <= 1e-6
    assert e1 <= 1e-8 or 50.0 <= e1 / e2 <= 200.0   # (at p = 1 both are at rounding level)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_jacobian_matches_closed_form_at_constant_states(p):
    cfg = DGConfig(n=5, p=p)
    A, info = assemble(cfg, include_mass=True)
    U = info["U"]
    J = jacobian(cfg, state_to_modal(cfg, U), U, info["dtau"])
    assert np.array_equal(J.rowptr, A.rowptr) and np.array_equal(J.colind, A.colind)
    assert np.abs(J.val - A.val).max() <= 1e-13 * np.abs(A.val).max()


def test_freestream_is_steady():
    cfg = DGConfig(n=6, p=1)
    res, jac, lam = _callables(cfg)
    u0 = state_to_modal(cfg, np.broadcast_to(freestream(cfg), (cfg.K, 4))).reshape(-1)
    assert np.abs(res(u0)).max() <= 1e-13
    u, info = ptc.ptc(u0 + 0.0, lambda u: np.zeros_like(u), jac, lam, _exact)
    assert info.steps == 0 and info.converged


def test_newton_limit_converges_quadratically():
    """With the LF spectral radius held fixed the Jacobian is exact, and with
    exact solves at CFL -> infinity each step is a Newton step.  (The density
    residual is linear in u for a fixed spectral radius, so it vanishes after
    the first step; the full residual shows the quadratic rate.)"""
    cfg = DGConfig(n=8, p=1)
    u0 = initial_state(cfg).reshape(-1)
    lam0 = element_means(cfg, u0.reshape(cfg.K, -1, 4))
    res = lambda u: residual(cfg, u.reshape(cfg.K, -1, 4), lam0).reshape(-1)
    jac = lambda u, dt: jacobian(cfg, u.reshape(cfg.K, -1, 4), lam0, dt).to_scipy().tocsr()
    lam = lambda u: local_lambda(cfg, element_means(cfg, u.reshape(cfg.K, -1, 4)))
    u, info = ptc.ptc(u0, res, jac, lam, _exact, cfl0=1e15, cfl_inf=1e15, orders=40, max_steps=3)
    r = np.array(info.res_norm)
    assert info.steps == 3
    assert info.rho_norm[1] <= 1e-12 * info.rho_norm[0]
    # quadratic: r_{n+1} <= C r_n^2 with about one constant over the first
    # steps (the last one is limited by the conditioning of dR/du alone)
    C = r[1:3] / r[:2] ** 2
    assert C[1] <= 10 * C[0]
    assert r[3] <= 1e-8 * r[0]


def test_small_cfl_step_is_explicit_euler():
    cfg = DGConfig(n=6, p=1)
    res, jac, lam = _callables(cfg)
    u0 = initial_state(cfg).reshape(-1)
    R0 = res(u0)
    steps = {}
    for cfl in (1e-4, 2e-4):
        u, info = ptc.ptc(u0, res, jac, lam, _exact, cfl0=cfl, cfl_inf=cfl, max_steps=1)
        dtau = info.dtau[0]
        assert dtau == pytest.approx(cfl / lam(u0).max(), rel=1e-15)
        hh = 0.5 / cfg.n
        steps[cfl] = (u - u0, -dtau / (hh * hh) * R0)
    # the difference to explicit Euler is second order in dtau
    e1 = np.linalg.norm(steps[1e-4][0] - steps[1e-4][1])
    e2 = np.linalg.norm(steps[2e-4][0] - steps[2e-4][1])
    assert e1 <= 1e-3 * np.linalg.norm(steps[1e-4][1])
    assert 3.0 <= e2 / e1 <= 5.0


def test_cfl_ramp_and_cap():
    cfg = DGConfig(n=8, p=1)
    res, jac, lam = _callables(cfg)
    u, info = ptc.ptc(initial_state(cfg).reshape(-1), res, jac, lam, _exact, cfl0=10.0,
                      cfl_inf=2000.0)
    assert info.converged and info.rho_norm[-1] <= 1e-8 * info.rho_norm[0]
    assert info.cfl[0] == 10.0
    # while the residual falls the CFL number grows, and never beyond the cap
    assert all(b >= a for a, b in zip(info.cfl, info.cfl[1:]))
    assert max(info.cfl) == 2000.0
