"""GPU checks of the pseudo-transient loop and of spand_refactor.

  * spand_refactor on new values of the same block pattern gives the factor
    that spand_factor builds from scratch, bit for bit (same kernels, same
    plan), and rejects a different pattern before any launch;
  * the GPU loop (paper_2101_01763_amd.ptc: spaND factor, then refactor at
    every later step, s-step GMRES to 1e-3 as in the paper's experiments)
    against the oracle's loop (oracle/ptc.py with the oracle's spaND and
    s-step GMRES) on the 16x16, p = 1 problem from the seeded smooth state,
    FP64 factor: same number of steps and of GMRES iterations per step,
    residual history within 1e-6 (down to 1e-12 of the first residual, the
    rounding level of its evaluation), final state within 1e-8 (the linear
    solves agree to ~1e-10 on the same Krylov path);
  * with the FP32 factor the loop reaches the same 8 orders in at most one
    more step.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2101_01763_amd as sp  # noqa: E402
from paper_2101_01763_amd.ptc import ptc_solve  # noqa: E402
from oracle import krylov, ptc, spand  # noqa: E402
from oracle.nd import nested_dissection  # noqa: E402
from synth.dg_euler import (DGConfig, element_means, initial_state, jacobian,  # noqa: E402
                            local_lambda, make_problem, residual)


def _callables(cfg):
    def res(u):
        uh = u.reshape(cfg.K, -1, 4)
        return residual(cfg, uh, element_means(cfg, uh)).reshape(-1)

    def jac(u, dtau):
        uh = u.reshape(cfg.K, -1, 4)
        return jacobian(cfg, uh, element_means(cfg, uh), dtau)

    def lam(u):
        return local_lambda(cfg, element_means(cfg, u.reshape(cfg.K, -1, 4)))

    return res, jac, lam


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_refactor_matches_fresh_factor(dtype):
    n, p, L = 12, 2, 4
    cfg = DGConfig(n=n, p=p)
    A1, xs, b, info = make_problem(cfg)
    u = initial_state(cfg)
    A2 = jacobian(cfg, u, element_means(cfg, u), 0.5 * info["dtau"])
    d1 = sp.BSRMatrix.from_numpy(A1.rowptr, A1.colind, A1.val)
    d2 = sp.BSRMatrix.from_numpy(A2.rowptr, A2.colind, A2.val)
    F = sp.factor(d1, n, n, True, False, eps=1e-2, nlevels=L, dtype=dtype)
    F.refactor(d2)
    G = sp.factor(d2, n, n, True, False, eps=1e-2, nlevels=L, dtype=dtype)
    r = torch.as_tensor(np.random.default_rng(3).standard_normal(cfg.N), device="cuda")
    assert torch.equal(F.apply(r), G.apply(r))
    assert torch.equal(F.apply_T(r), G.apply_T(r))
    sf, sg = F.stats(), G.stats()
    assert sf["size_after"] == sg["size_after"] and sf["factor_bytes"] == sg["factor_bytes"]
    # a different block pattern (one column index changed) is rejected
    ci = A2.colind.copy()
    row = 5
    a, e = A2.rowptr[row], A2.rowptr[row + 1]
    ci[a:e] = np.sort(np.where(ci[a:e] == row, (row + 2) % cfg.K, ci[a:e]))
    if len(set(ci[a:e])) == e - a:
        d3 = sp.BSRMatrix.from_numpy(A2.rowptr, ci, A2.val)
        with pytest.raises(sp.SpandError) as ei:
            F.refactor(d3)
        assert ei.value.code == sp.SPAND_EINVAL
        assert torch.equal(F.apply(r), G.apply(r))      # the factor is unchanged


def _oracle_ptc(cfg, L, eps, s, m, rtol, cfl0, cfl_inf):
    res, jac, lam = _callables(cfg)
    nd = nested_dissection(cfg.n, cfg.n, True, False, L)

    def lin(A, rhs):
        F = spand.factor(A, nd, cfg.b, eps)
        x, io = krylov.sstep_gmres(lambda v: A @ v, rhs, lambda v: spand.apply(F, v), s=s,
                                   rtol=rtol, restart=m)
        return x, io.iters

    return ptc.ptc(initial_state(cfg).reshape(-1), res, lambda u, dt: jac(u, dt).to_scipy().tocsr(),
                   lam, lin, cfl0=cfl0, cfl_inf=cfl_inf)


def test_ptc_parity_c1():
    cfg = DGConfig(n=16, p=1)
    L, eps, s, m, rtol, cfl0, cfl_inf = 4, 1e-2, 4, 40, 1e-3, 10.0, 1e8
    res, jac, lam = _callables(cfg)
    jv = lambda u, dt: (lambda B: (B.rowptr, B.colind, B.val))(jac(u, dt))
    u, r = ptc_solve((cfg.n, cfg.n, True, False), res, jv, lam, initial_state(cfg).reshape(-1),
                     cfl0=cfl0, cfl_inf=cfl_inf, eps=eps, nlevels=L, dtype="f64", s=s,
                     restart=m, rtol=rtol, lagged=False)
    uo, io = _oracle_ptc(cfg, L, eps, s, m, rtol, cfl0, cfl_inf)
    print(f"PTC C1 FP64: steps {r.steps} (oracle {io.steps}), GMRES iterations {r.lin_iters} "
          f"(oracle {io.lin_iters}), density residual {r.rho_norm[-1] / r.rho_norm[0]:.2e}")
    assert r.converged and io.converged
    assert r.steps == io.steps
    assert r.lin_iters == io.lin_iters
    # residual norms within 1e-6, down to the rounding level of the residual
    # evaluation itself (sums of O(1) fluxes: 1e-12 of the initial residual)
    np.testing.assert_allclose(r.res_norm, io.res_norm, rtol=1e-6, atol=1e-12 * io.res_norm[0])
    np.testing.assert_allclose(r.cfl, io.cfl, rtol=1e-6)
    assert np.linalg.norm(u - uo) <= 1e-8 * np.linalg.norm(uo)


def test_ptc_fp32_factor():
    cfg = DGConfig(n=16, p=1)
    res, jac, lam = _callables(cfg)
    jv = lambda u, dt: (lambda B: (B.rowptr, B.colind, B.val))(jac(u, dt))
    out = {}
    for dt in ("f64", "f32"):
        u, r = ptc_solve((cfg.n, cfg.n, True, False), res, jv, lam,
                         initial_state(cfg).reshape(-1), cfl0=10.0, eps=1e-2, nlevels=4,
                         dtype=dt, s=4, restart=40, rtol=1e-3)
        assert r.converged and r.rho_norm[-1] <= 1e-8 * r.rho_norm[0]
        out[dt] = (u, r.steps)
    assert out["f32"][1] <= out["f64"][1] + 1
    # both reach the same steady state
    assert np.linalg.norm(out["f32"][0] - out["f64"][0]) <= 1e-7 * np.linalg.norm(out["f64"][0])
