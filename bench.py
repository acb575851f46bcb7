"""Benchmark: spaND factor + s-step GMRES to rtol 1e-8 on one MI355X.

One step = one pass of the whole hot path on the synthetic 2D-Euler DG
Jacobian: host nested dissection + plan, spaND factorization (elimination,
scaling, RRQR sparsification, merge; FP32 or FP64 factor), and the s-step
GMRES solve (FP64 SpMV / Gram / CholQR / Hessenberg) to rtol 1e-8.
value = N / (t_factor + t_solve) in DOF/s, inputs resident in HBM.

Prints ONE JSON line.  Extra fields: the roofline of the dominant kernel
(the rank-revealing QR, ALU-bound: algorithmic flops and bytes per launch from
the factor's counters, duration from HIP events around every launch in the
timed region; HBM traffic from the committed PMC measurement while its kernel
source is unchanged), the SpMV roofline, a one-step comparison with the other factor
precision, and the CPU oracle timed on a bounded sample of the same operator
family.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    # name: (n, p, eps, L, s, restart).  C3 uses L = 13: leaves of 3x3
    # elements = 576 unknowns, the closest to the paper's ~512-unknown leaves
    # (32 elements x 16 at p = 1); the Table 1/2 element rule would give L = 12.
    "c1": (16, 1, 1e-2, 4, 4, 40),
    "c2": (128, 2, 1e-2, 10, 5, 60),
    "c3": (256, 3, 1e-2, 13, 5, 60),
    "c5": (192, 2, 1e-2, 11, 5, 60),
}
HBM_PEAK_GBS = 8000.0
# FP32 vector peak: 256 CUs x 4 SIMDs x 16 lanes x 2 (dual issue) x 2 (FMA)
# x 2.4 GHz = 157.3 TFLOP/s
ALU_F32_PEAK_TFS = 157.3


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(p, eps, s, restart, budget_s=30.0):
    """Oracle (plain FP64 numpy/scipy) on a bounded sample: a smaller grid of
    the same operator family (same p, eps, s, restart), factor + solve."""
    from threadpoolctl import threadpool_info

    from oracle import krylov, spand
    from oracle.nd import default_levels, nested_dissection
    from synth.dg_euler import DGConfig, make_problem
    n = 32 if p >= 3 else 48
    cfg = DGConfig(n=n, p=p)
    A, xs, b, _ = make_problem(cfg)
    As = A.to_scipy().tocsr()
    L = default_levels(cfg.K)
    t0 = time.perf_counter()
    F = spand.factor(As, nested_dissection(n, n, True, False, L), cfg.b, eps)
    t1 = time.perf_counter()
    x, info = krylov.sstep_gmres(lambda v: As @ v, b, lambda v: spand.apply(F, v), s=s,
                                 rtol=1e-8, restart=restart)
    t2 = time.perf_counter()
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {"value": cfg.N / (t2 - t0), "unit": "DOF/s", "cores": int(threads),
            "kind": "oracle",
            "sample": f"{n}x{n} grid, p={p} (N={cfg.N}), eps={eps}, L={L}, s={s}, m={restart}: "
                      f"factor {t1 - t0:.2f} s + solve {t2 - t1:.2f} s, {info.iters} iterations",
            "t_factor_s": t1 - t0, "t_solve_s": t2 - t1}


def pmc_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed PMC measurement
    (profiles/pmc_traffic.json), or None if the kernel source changed since."""
    import hashlib
    try:
        rec = json.load(open(os.path.join(ROOT, "profiles", "pmc_traffic.json")))
        src = open(os.path.join(ROOT, rec["source"]), "rb").read()
        if rec["kernel"] == kernel and hashlib.sha256(src).hexdigest() == rec["source_sha256"]:
            return rec["traffic_bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    return None


def bench_batch(args):
    """C4: 64 uneven seeded systems (n ~ U{32..96}, p ~ U{1,2,3},
    M ~ U[0.3,0.7], alpha ~ U[-4,4] deg), FP32 spaND eps=1e-2, s=5, m=60,
    rtol 1e-8; factored and solved concurrently (batched entry points,
    graph-replayed sweeps, autotuned SpMV/GEMV shapes).  value = total DOF /
    wall time of one batched factor+solve; the same batch on one stream is
    timed beside it."""
    import torch

    import paper_2101_01763_amd as sp
    from synth.dg_euler import batch_configs, make_problem
    cfgs = batch_configs(64, seed=0)
    t = time.time()
    systems, rhs, Ls = [], [], []
    for c in cfgs:
        A, xs, b, _ = make_problem(c)
        systems.append((sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val), c.n, c.n, True, False))
        rhs.append(torch.as_tensor(b, device="cuda"))
        Ls.append(sp.levels_for(c.N))
    ntot = sum(c.N for c in cfgs)
    log(f"generated 64 systems, {ntot} DOF in {time.time() - t:.1f} s")
    torch.cuda.synchronize()

    def run(streams):
        os.environ["SPAND_BATCH_STREAMS"] = str(streams)
        t0 = time.perf_counter()
        Fs = sp.factor_batched(systems, eps=1e-2, nlevels=Ls, dtype="f32")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        xs, infos = sp.solve_batched([q[0] for q in systems], rhs, Fs, s=5, restart=60, rtol=1e-8,
                                     lagged=args.schedule == "lagged")
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        for F in Fs:
            F.destroy()
        return t1 - t0, t2 - t1, infos

    for _ in range(args.warmup):
        run(8)
    res = [run(8) for _ in range(args.steps)]
    tf = float(np.median([r[0] for r in res]))
    ts = float(np.median([r[1] for r in res]))
    infos = res[-1][2]
    seq = run(1)
    out = {
        "metric": "batched spaND factor + s-step GMRES (64 uneven systems); DOF/s",
        "value": ntot / (tf + ts), "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * (tf + ts), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (spaND) + f64 (Krylov)",
        "data": "synthetic (64 seeded DG-Euler systems)",
        "config": {"workload": f"C4 batch: 64 systems, {ntot} DOF total, n in 32..96, p in 1..3, "
                               f"FP32 spaND eps=1e-2, s=5, m=60, rtol=1e-8 ({args.schedule}), "
                               f"8 streams", "schedule": args.schedule},
        "t_factor_ms": 1e3 * tf, "t_solve_ms": 1e3 * ts,
        "all_converged": all(i.converged for i in infos),
        "iters_min_max": [min(i.iters for i in infos), max(i.iters for i in infos)],
        "one_stream": {"t_factor_ms": 1e3 * seq[0], "t_solve_ms": 1e3 * seq[1],
                       "dof_per_s": ntot / (seq[0] + seq[1])},
    }
    print(json.dumps(out), flush=True)


def bench_basis_study(args):
    """Stability of the s-step basis (the paper's CAGMRES study) and the
    classical-GMRES baseline: FP32-spaND preconditioned GMRES (rtol 1e-8) on
    the 128x128, p = 2 operator with s = 5, m = 60 and {Newton, monomial}
    basis x {1, 2} passes of block CGS + CholQR (||Q^T Q - I||_F after every
    block), then s-step against classical GMRES (modified Gram-Schmidt) with
    the phase times on that operator and on the 256x256, p = 3 one."""
    import torch
    import paper_2101_01763_amd as sp
    from synth.dg_euler import DGConfig, make_problem

    def run(name, cfg, dA, db, dxs, F, s, m, **kw):
        sp.solve(dA, db, F, s=s, restart=m, rtol=1e-8, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = sp.solve(dA, db, F, s=s, restart=m, rtol=1e-8, **kw)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rec = {"sweep": "basis", "workload": name, "N": cfg.N, "s": s, "restart": m,
               "variant": kw, "iters": info.iters, "converged": info.converged,
               "n_reduce": info.n_reduce,
               "relres": info.relres, "t_solve_ms": 1e3 * (t1 - t0),
               "phases_ms": {"spmv": info.t_spmv_ms, "apply": info.t_apply_ms,
                             "orth": info.t_orth_ms, "other": info.t_other_ms},
               "rel_err_vs_xstar": float(torch.linalg.norm(x - dxs) / torch.linalg.norm(dxs))}
        if not kw.get("classical"):
            # the losses from a separate run (the Gram matrices are diagnostics)
            _, info2 = sp.solve(dA, db, F, s=s, restart=m, rtol=1e-8, orth_loss=True, **kw)
            rec["orth_loss"] = info2.orth_loss
        print(json.dumps(rec), flush=True)

    for name in ("c2", "c3"):
        n, p, eps, L, s, m = WORKLOADS[name]
        cfg = DGConfig(n=n, p=p)
        A, xs, b, _ = make_problem(cfg)
        dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
        del A
        db = torch.as_tensor(b, device="cuda")
        dxs = torch.as_tensor(xs, device="cuda")
        F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f32")
        variants = [{}, {"lagged": True}, {"classical": True}]
        if name == "c2":
            variants = [{}, {"passes": 1}, {"monomial": True}, {"monomial": True, "passes": 1},
                        {"lagged": True}, {"monomial": True, "lagged": True}, {"classical": True}]
        for kw in variants:
            run(name, cfg, dA, db, dxs, F, s, m, **kw)
        del F, dA


def bench_sweep(args):
    """FP32-spaND + s-step GMRES (s = 5, m = 60, rtol 1e-8) on the 256x256
    grid over one parameter; per case one untimed and one timed build."""
    import torch
    import paper_2101_01763_amd as sp
    from synth.dg_euler import DGConfig, make_problem

    if args.sweep == "basis":
        return bench_basis_study(args)
    n = 256
    # leaves of about 600 unknowns: L = 11, 12, 13 at p = 1, 2, 3
    lp = {1: 11, 2: 12, 3: 13}
    if args.sweep == "eps":
        cases = [(3, e, 13) for e in (1e-1, 1e-2, 1e-3, 1e-4)]
    elif args.sweep == "levels":
        cases = [(3, 1e-2, L) for L in (12, 13, 14)]   # L = 11: 4096-unknown leaves
    else:
        cases = [(p, 1e-2, lp[p]) for p in (1, 2, 3)]
    probs = {}
    for p, eps, L in cases:
        if p not in probs:
            cfg = DGConfig(n=n, p=p)
            A, xs, b, _ = make_problem(cfg)
            probs[p] = (cfg, sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val),
                        torch.as_tensor(b, device="cuda"), torch.as_tensor(xs, device="cuda"))
            del A
            log(f"generated p={p}: N={cfg.N}")
        cfg, dA, db, dxs = probs[p]
        try:
            F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f32")
        except sp.SpandError as ex:      # e.g. a cluster beyond the kernel limits
            print(json.dumps({"sweep": args.sweep, "p": p, "eps": eps, "levels": L,
                              "error": str(ex)}), flush=True)
            continue
        del F
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype="f32")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, info = sp.solve(dA, db, F, s=5, restart=60, rtol=1e-8)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        st = F.stats()
        print(json.dumps({
            "sweep": args.sweep, "p": p, "N": cfg.N, "eps": eps, "levels": L,
            "t_factor_ms": 1e3 * (t1 - t0), "t_solve_ms": 1e3 * (t2 - t1),
            "dof_per_s": cfg.N / (t2 - t0), "iters": info.iters, "relres": info.relres,
            "rel_err_vs_xstar": float(torch.linalg.norm(x - dxs) / torch.linalg.norm(dxs)),
            "resident_GiB": st["resident_bytes"] / 2**30, "factor_GB": st["factor_bytes"] / 1e9,
            "rank_avg": st["rank_avg"], "rank_max": st["rank_max"]}), flush=True)
        del F, x


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS) + ["c4"])
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--levels", type=int, default=0)
    ap.add_argument("--eps", type=float, default=None)
    ap.add_argument("--schedule", default="lagged", choices=["two-pass", "lagged"],
                    help="s-step orthogonalisation: two passes per block, or the "
                         "single-reduce schedule with the second pass lagged")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the one-step FP64-factor comparison run")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 1 GiB device copy (PMC byte-counter calibration)")
    ap.add_argument("--sweep", choices=["eps", "levels", "p", "basis"], default=None,
                    help="256x256 grid: ranks, iterations, times and memory over eps "
                         "(1e-1..1e-4), the number of levels, or p = 1..3; 'basis': the "
                         "128x128 p=2 operator, Newton/monomial basis x 1/2 orthogonalisation "
                         "passes with the loss of orthogonality per block (one JSON line each)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import torch

    if args.calibrate_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")    # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration": "device copy", "bytes_read": a.numel() * 8,
                          "bytes_written": b.numel() * 8, "launches": 3}))
        return

    import paper_2101_01763_amd as sp
    from synth.dg_euler import DGConfig, make_problem

    if args.sweep:
        return bench_sweep(args)
    if args.workload == "c4":
        return bench_batch(args)
    n, p, eps, L, s, m = WORKLOADS[args.workload]
    if args.eps is not None:
        eps = args.eps
    if args.levels:
        L = args.levels
    cfg = DGConfig(n=n, p=p)
    t = time.time()
    A, xs, b, _ = make_problem(cfg)
    log(f"generated {args.workload}: N={cfg.N} nnzb={A.nnzb} in {time.time() - t:.1f} s")
    dA = sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val)
    db = torch.as_tensor(b, device="cuda")
    dxs = torch.as_tensor(xs, device="cuda")
    del A
    torch.cuda.synchronize()

    def step():
        t0 = time.perf_counter()
        F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype=args.dtype)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, info = sp.solve(dA, db, F, s=s, restart=m, rtol=1e-8,
                           lagged=args.schedule == "lagged")
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return F, x, info, t1 - t0, t2 - t1

    for w in range(args.warmup):
        F, x, info, tf, ts = step()
        log(f"warmup {w}: factor {tf * 1e3:.1f} ms solve {ts * 1e3:.1f} ms iters {info.iters}")
        del F
    torch.cuda.synchronize()
    tfs, tss, infos = [], [], []
    spmv_ms, spmv_n = 0.0, 0
    qrcp_ms, qrcp_n, qrcp_bytes, qrcp_flops = 0.0, 0, 0.0, 0.0
    t_start = time.perf_counter()
    for k in range(args.steps):
        F, x, info, tf, ts = step()
        tfs.append(tf)
        tss.append(ts)
        infos.append(info)
        spmv_ms += info.t_spmv_ms
        spmv_n += info.n_spmv
        st = F.stats()
        qrcp_ms += st["t_qrcp_ms"]
        qrcp_n += st["n_qrcp"]
        qrcp_bytes += st["qrcp_bytes"]
        qrcp_flops += st["qrcp_flops"]
        log(f"step {k}: factor {tf * 1e3:.1f} ms solve {ts * 1e3:.1f} ms iters {info.iters} "
            f"relres {info.relres:.2e} | lu {st['t_lu_ms']:.0f} schur {st['t_schur_ms']:.0f} "
            f"scale {st['t_scale_ms']:.0f} rrqr {st['t_rrqr_ms']:.0f} (qrcp {st['t_qrcp_ms']:.0f}) "
            f"compress {st['t_compress_ms']:.0f} host {st['t_host_ms']:.0f} "
            f"alloc {st['t_alloc_ms']:.0f} ms, resident {st['resident_bytes'] / 2**30:.1f} GiB | "
            f"host plan ms " + " ".join(f"{v:.0f}" for v in st['t_plan_ms']))
        del F
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    err = float(torch.linalg.norm(x - dxs) / torch.linalg.norm(dxs))
    ms_per_step = 1e3 * t_total / args.steps
    value = cfg.N * args.steps / t_total
    nnzb = int(dA.colind.numel())
    bsz = cfg.b
    # SpMV algorithmic bytes per launch: values, indices, x read once, y written;
    # the fused Newton terms read up to two more vectors (counted as 8N each when used:
    # here we count the base contract 16N for x and y).
    spmv_bytes = 8 * nnzb * bsz * bsz + 4 * nnzb + 4 * (cfg.K + 1) + 16 * cfg.N
    spmv_avg_ms = spmv_ms / max(spmv_n, 1)
    achieved = spmv_bytes / (spmv_avg_ms * 1e-3) / 1e9 if spmv_n else 0.0
    # dominant kernel of the step: the rank-revealing QR (one launch per level)
    q_avg_ms = qrcp_ms / max(qrcp_n, 1)
    q_bytes_launch = qrcp_bytes / max(qrcp_n, 1)
    q_ach = q_bytes_launch / (q_avg_ms * 1e-3) / 1e9 if qrcp_n else 0.0
    q_flops_launch = qrcp_flops / max(qrcp_n, 1)
    q_tfs = q_flops_launch / (q_avg_ms * 1e-3) / 1e12 if qrcp_n else 0.0
    traffic = pmc_traffic("k_qrcp")
    out = {
        "metric": "spaND factor+s-step GMRES time to rtol 1e-8, FP32- vs FP64-spaND; DOF/s",
        "value": value,
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": f"{args.dtype} (spaND factor/apply) + f64 (SpMV, Gram, CholQR, Hessenberg)",
        "data": "synthetic (seeded DG-Euler Jacobian, x* ~ N(0,1), b = A x*)",
        "config": {
            "workload": f"DG-Euler {n}x{n} p={p} (b={bsz}, N={cfg.N}, nnzb={nnzb}); "
                        f"spaND eps={eps} L={L} {args.dtype}; s-step GMRES s={s} m={m} rtol=1e-8"
                        f" ({args.schedule})",
            "n": n, "p": p, "N": cfg.N, "eps": eps, "levels": L, "s": s, "restart": m,
            "factor_dtype": args.dtype, "schedule": args.schedule,
        },
        "t_factor_ms": 1e3 * float(np.median(tfs)),
        "t_solve_ms": 1e3 * float(np.median(tss)),
        "iters": infos[-1].iters,
        "relres": infos[-1].relres,
        "rel_err_vs_xstar": err,
        "factor_stats": {k: v for k, v in st.items() if k.startswith("t_") or k in
                         ("top_size", "factor_bytes", "factor_flops", "rank_avg", "rank_max")},
        "solve_phases_ms": {"spmv": infos[-1].t_spmv_ms, "apply": infos[-1].t_apply_ms,
                            "orth": infos[-1].t_orth_ms, "other": infos[-1].t_other_ms},
        "solve_reductions": infos[-1].n_reduce,
        # Arithmetic intensity of the QR (algorithmic flops over algorithmic
        # bytes, about 60 flop/B) is above the FP32 ridge point (157.3 / 8 =
        # 20 flop/B): the binding roof is the vector ALU, not HBM.
        "roofline": {"kernel": "k_qrcp (column-pivoted QR of [A_sn A_ns^T], all interfaces "
                               "of one level per launch)", "bound": "alu",
                     "achieved": q_tfs, "peak": ALU_F32_PEAK_TFS, "unit": "TFLOP/s",
                     "frac": q_tfs / ALU_F32_PEAK_TFS, "traffic": traffic,
                     "flops_per_launch": q_flops_launch, "avg_launch_ms": q_avg_ms,
                     "launches": qrcp_n,
                     "algorithmic_flops": "sum over interfaces of 4mck - 2k^2(m+c) + 4k^3/3 "
                                          "(k Householder-equivalent steps on m x c)",
                     "bytes_per_launch": q_bytes_launch, "hbm_achieved_GBs": q_ach,
                     "algorithmic_bytes": "each W (m x ncols) read once + each Q (m x m) "
                                          "written once, factor precision"},
        "roofline_spmv": {"kernel": "k_spmv (BSR SpMV, FP64)", "bound": "hbm",
                          "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                          "frac": achieved / HBM_PEAK_GBS, "bytes_per_launch": spmv_bytes,
                          "avg_launch_ms": spmv_avg_ms, "launches": spmv_n},
    }
    if not args.no_compare:
        # The other precision, one warm-up and one timed step, in a child
        # process: a fresh device allocator, as in a run of its own (in this
        # process the block cache and the driver hold the first precision's
        # blocks, whose sizes the other precision never asks for).
        import subprocess
        other = "f64" if args.dtype == "f32" else "f32"
        sp.pool_trim()
        torch.cuda.empty_cache()
        cmd = [sys.executable, os.path.abspath(__file__), "--workload", args.workload,
               "--dtype", other, "--steps", "1", "--warmup", "1", "--no-compare",
               "--no-cpu-baseline", "--levels", str(L), "--eps", str(eps),
               "--schedule", args.schedule]
        log(f"comparison: {other} factor in a child process")
        try:
            r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
            lines = [q for q in r.stdout.strip().splitlines() if q.startswith("{")]
            if r.returncode != 0 or not lines:
                raise RuntimeError(f"exit {r.returncode}: {r.stderr[-500:]}")
            c = json.loads(lines[-1])
            out[f"compare_{other}_factor"] = {
                "t_factor_ms": c["t_factor_ms"], "t_solve_ms": c["t_solve_ms"],
                "iters": c["iters"], "relres": c["relres"],
                "rel_err_vs_xstar": c["rel_err_vs_xstar"], "dof_per_s": c["value"],
                "run": "child process, 1 warm-up + 1 timed step"}
        except (RuntimeError, subprocess.TimeoutExpired, ValueError, KeyError) as ex:
            # the comparison is context; the measured line stands without it
            log(f"comparison run failed: {ex}")
            out[f"compare_{other}_factor"] = {"error": str(ex)[-500:]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, eps, s, m)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
