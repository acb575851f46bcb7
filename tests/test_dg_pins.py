"""Pins of the synthetic DG Jacobian generator (paper Eqs. (1)-(8))."""
import math

import numpy as np
import pytest

from synth.dg_euler import (DGConfig, assemble, base_state, conserved_to_primitive,
                            draw_phases, flux_jacobians, freestream, make_problem,
                            residual, sound_speed, state_to_modal, stiffness_1d,
                            vector_to_modal, _legendre_vals, _gauss)


def test_flux_jacobian_eigenvalues():
    # closed form: eig(n_x A + n_y B) = v_n - c, v_n, v_n, v_n + c
    rng = np.random.default_rng(3)
    for _ in range(20):
        rho = rng.uniform(0.5, 2); u, v = rng.normal(size=2); p = rng.uniform(0.5, 3)
        from synth.dg_euler import primitive_to_conserved
        U = primitive_to_conserved(np.float64(rho), np.float64(u), np.float64(v), np.float64(p))
        A, B = flux_jacobians(U)
        th = rng.uniform(0, 2 * math.pi); nx, ny = math.cos(th), math.sin(th)
        ev = np.sort(np.linalg.eigvals(nx * A + ny * B).real)
        vn = u * nx + v * ny; c = math.sqrt(1.4 * p / rho)
        np.testing.assert_allclose(ev, np.sort([vn - c, vn, vn, vn + c]), rtol=1e-12, atol=1e-12)


def test_flux_jacobian_is_derivative():
    from synth.dg_euler import euler_flux, primitive_to_conserved
    U = primitive_to_conserved(np.float64(1.2), np.float64(0.3), np.float64(-0.4), np.float64(2.0))
    A, B = flux_jacobians(U)
    h = 1e-7
    for k in range(4):
        d = np.zeros(4); d[k] = h
        Fp, Gp = euler_flux(U + d); Fm, Gm = euler_flux(U - d)
        np.testing.assert_allclose((Fp - Fm) / (2 * h), A[:, k], atol=1e-7)
        np.testing.assert_allclose((Gp - Gm) / (2 * h), B[:, k], atol=1e-7)


@pytest.mark.parametrize("p", [1, 2, 3])
def test_stiffness_closed_form_vs_quadrature(p):
    x, w = _gauss(p + 2)
    V, D = _legendre_vals(p, x)
    Sq = np.einsum("cr,ar,r->ca", V, D, w)
    np.testing.assert_allclose(stiffness_1d(p), Sq, atol=1e-13)
    # orthonormality (Eq. 6 with an orthonormal basis gives M = (h/2)^2 I)
    np.testing.assert_allclose(np.einsum("ar,cr,r->ac", V, V, w), np.eye(p + 1), atol=1e-13)


@pytest.mark.parametrize("p", [1, 2])
def test_jacobian_matches_fd_of_quadrature_residual(p):
    cfg = DGConfig(n=6, p=p)
    A0, info = assemble(cfg, include_mass=False)
    U = info["U"]
    uh0 = state_to_modal(cfg, U)
    d = np.random.default_rng(5).standard_normal(cfg.N)
    h = 1e-6
    Rp = residual(cfg, uh0 + h * vector_to_modal(cfg, d), U).reshape(-1)
    Rm = residual(cfg, uh0 - h * vector_to_modal(cfg, d), U).reshape(-1)
    fd = (Rp - Rm) / (2 * h)
    Jd = A0.matvec(d)
    assert np.linalg.norm(fd - Jd) <= 1e-8 * np.linalg.norm(Jd)


def test_free_stream_preservation():
    cfg = DGConfig(n=5, p=2)
    _, info = assemble(cfg, include_mass=False)
    Uinf = np.broadcast_to(freestream(cfg), (cfg.K, 4)).copy()
    R = residual(cfg, state_to_modal(cfg, Uinf), info["U"])
    assert np.abs(R).max() < 1e-13


def test_uniform_perturbation_zero_in_interior_rows():
    cfg = DGConfig(n=6, p=1)
    J, _ = assemble(cfg, include_mass=False, amp=0.0)
    du = np.zeros((cfg.K, (cfg.p + 1) ** 2, 4))
    du[:, 0, :] = np.array([0.3, -0.2, 0.5, 1.1])
    r = J.matvec(du.reshape(-1)).reshape(cfg.K, -1)
    j = np.arange(cfg.K) // cfg.n
    interior = (j > 0) & (j < cfg.n - 1)
    assert np.abs(r[interior]).max() < 1e-13 * np.abs(J.val).max()
    assert np.abs(r[~interior]).max() > 1e-6        # far-field rows do respond


def test_conservation_fully_periodic():
    cfg = DGConfig(n=5, p=2, periodic_y=True)
    J, _ = assemble(cfg, include_mass=False)
    Jd = J.to_scipy().toarray()
    rows = (np.arange(cfg.K)[:, None] * cfg.b + np.arange(4)[None, :]).reshape(-1)
    cs = Jd[rows].reshape(cfg.K, 4, -1).sum(axis=0)
    assert np.abs(cs).max() < 1e-13 * np.abs(Jd).max()


def test_pattern_and_mass():
    cfg = DGConfig(n=16, p=1)
    A, info = assemble(cfg)
    assert A.nnzb == 5 * cfg.K - 2 * cfg.n == 1248
    assert A.bs == 16 and A.N == 4096
    J, _ = assemble(cfg, include_mass=False)
    h = 1.0 / cfg.n
    diff = A.val - J.val
    diag_slots = [A.rowptr[e] + list(A.colind[A.rowptr[e]:A.rowptr[e + 1]]).index(e)
                  for e in range(cfg.K)]
    mass = (h / 2) ** 2 / info["dtau"]
    for s in diag_slots:
        np.testing.assert_allclose(diff[s], mass * np.eye(cfg.b), atol=1e-14 * mass)
    # dtau = CFL / max_k (2p+1)(|v_k|+c_k)/h
    rho, u, v, p = conserved_to_primitive(info["U"])
    lam = 3 * (np.hypot(u, v) + sound_speed(info["U"])) / h
    assert abs(info["dtau"] - 10.0 / lam.max()) < 1e-15


def test_manufactured_rhs_seeded():
    cfg = DGConfig(n=8, p=1, seed=7)
    A, xs, b, _ = make_problem(cfg)
    A2, xs2, b2, _ = make_problem(cfg)
    assert np.array_equal(xs, xs2) and np.array_equal(b, b2)
    np.testing.assert_allclose(A.matvec(xs), b, rtol=0, atol=0)
