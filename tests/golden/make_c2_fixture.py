"""Writes tests/golden/c2_fp64.json: the oracle's result on the 128 x 128,
p = 2 operator (N = 589,824; spaND eps = 1e-2 with 10 levels, s-step GMRES
s = 5, restart 60, rtol 1e-8, FP64 throughout), the "plain method on GPU"
workload.  Calls only oracle/ (and the shared input generator), so every
stored value is the oracle's.

Stored: the per-level rank statistics (interfaces, min/max rank, kept and
total unknowns: Eq. (12) with the relative threshold), the smallest relative
distance of any |R_kk| from the threshold eps |R_00| (how far the rank
decisions are from a tie), the iteration count, the residual estimates
after every column (Algorithm 2), the true relative residual, the norm of x
and x on 4096 seeded indices.

Usage: python tests/golden/make_c2_fixture.py   (several minutes, ~20 GB)
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import krylov, spand  # noqa: E402
from oracle.nd import nested_dissection  # noqa: E402
from synth.dg_euler import DGConfig, make_problem  # noqa: E402

N_SAMPLE = 4096
SAMPLE_SEED = 20210105


def main(out=os.path.join(os.path.dirname(os.path.abspath(__file__)), "c2_fp64.json")):
    n, p, eps, L, s, m, rtol = 128, 2, 1e-2, 10, 5, 60, 1e-8
    cfg = DGConfig(n=n, p=p)
    t0 = time.perf_counter()
    A, xs, b, _ = make_problem(cfg)
    As = A.to_scipy().tocsr()
    t1 = time.perf_counter()
    margins = []

    def hook(stage, level, blocks, dofs, extra):
        if stage != "rrqr":
            return
        _, W, Q, R, k = extra
        d = np.abs(np.diag(R))
        if d.size == 0 or d[0] == 0.0:
            return
        thr = eps * d[0]
        margins.append(float(np.min(np.abs(d / thr - 1.0))))

    nd = nested_dissection(n, n, True, False, L)
    F = spand.factor(As, nd, cfg.b, eps, hook=hook)
    t2 = time.perf_counter()
    x, info = krylov.sstep_gmres(lambda v: As @ v, b, lambda v: spand.apply(F, v), s=s,
                                 rtol=rtol, restart=m)
    t3 = time.perf_counter()
    idx = np.sort(np.random.default_rng(SAMPLE_SEED).choice(cfg.N, N_SAMPLE, replace=False))
    levels = []
    for lr in F.ranks:
        ks = [k for _, k in lr]
        ms = [mm for mm, _ in lr]
        levels.append({"interfaces": len(lr), "rank_min": min(ks) if ks else 0,
                       "rank_max": max(ks) if ks else 0, "kept": int(sum(ks)),
                       "size": int(sum(ms))})
    rec = {
        "workload": "128x128 grid, p = 2, N = 589,824; FP64 spaND eps 1e-2, 10 levels; "
                    "s-step GMRES s 5, restart 60, rtol 1e-8; seed 0",
        "n": n, "p": p, "eps": eps, "levels": L, "s": s, "restart": m, "rtol": rtol,
        "N": cfg.N, "rank_levels": levels,
        "min_threshold_margin": min(margins) if margins else None,
        "iters": info.iters, "restarts": info.restarts, "converged": bool(info.converged),
        "relres": info.relres, "history": [float(h) for h in info.history],
        "x_norm": float(np.linalg.norm(x)),
        "err_vs_xstar": float(np.linalg.norm(x - xs) / np.linalg.norm(xs)),
        "sample_seed": SAMPLE_SEED, "sample_idx": idx.tolist(),
        "sample_x": [float(v) for v in x[idx]],
        "oracle_seconds": {"assemble": t1 - t0, "factor": t2 - t1, "solve": t3 - t2},
    }
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
    print(f"wrote {out}: iters {info.iters}, relres {info.relres:.3e}, "
          f"factor {t2 - t1:.1f} s, solve {t3 - t2:.1f} s, margin {rec['min_threshold_margin']}")


if __name__ == "__main__":
    main()
