"""sstep_gmres_solve_noalloc (workspace in the library's per-device scratch
array, no device allocation inside the call) against sstep_gmres_solve on
the same inputs: two no-allocation calls in a row, the second with a
smaller system (a transposed solve with M^-T), each equal bit for bit to
the allocating entry point's result (same kernels in the same order; the
allocating calls run first so that both use the tuned SpMV lanes)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2101_01763_amd as sp  # noqa: E402
from synth.dg_euler import DGConfig, make_problem  # noqa: E402


def _case(n, p, L):
    cfg = DGConfig(n=n, p=p)
    A, xs, b, _ = make_problem(cfg)
    dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
    F = sp.factor(dA, n, n, True, False, eps=1e-2, nlevels=L, dtype="f32")
    return cfg, xs, dA, torch.as_tensor(b, device="cuda"), F


def test_noalloc_matches_solve():
    big = _case(16, 2, 4)        # N = 9,216
    small = _case(8, 1, 3)       # N = 1,024
    kw_big = dict(s=5, restart=60, rtol=1e-8)
    kw_small = dict(s=4, restart=40, rtol=1e-8, transpose=True, lagged=True)
    ref = [sp.solve(big[2], big[3], big[4], **kw_big),
           sp.solve(small[2], small[3], small[4], **kw_small)]
    got = [sp.solve_noalloc(big[2], big[3], big[4], **kw_big),
           sp.solve_noalloc(small[2], small[3], small[4], **kw_small)]
    torch.cuda.synchronize()
    for (x1, i1), (x2, i2), case in zip(ref, got, (big, small)):
        assert i1.converged and i2.converged and i2.relres <= 1e-8
        assert i2.iters == i1.iters and i2.restarts == i1.restarts
        assert i2.history == i1.history
        assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
        assert i2.t_total_ms == 0.0          # no phase timers inside the call
    # the transposed solve reached A^T x = b
    cfg, xs, dA, db, F = small
    r = sp.spmv(dA, got[1][0], transpose=True) - db
    assert torch.linalg.norm(r) <= 1e-8 * torch.linalg.norm(db)
