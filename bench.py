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
source is unchanged), the HBM rooflines of the SpMV and of the preconditioner
apply, the matrix-core roofline of the factorization's products, the
achievable copy and matrix-core ceilings measured on the device, the
other 256x256 p = 3 points (L = 12; eps = 0.1), the other factor precision
(median of three steps in a child process), and the CPU oracle timed on a
bounded sample of the same operator family.
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
# x 2.4 GHz = 157.3 TFLOP/s; FP64 vector: half of it, 78.6 TFLOP/s
ALU_F32_PEAK_TFS = 157.3
ALU_F64_PEAK_TFS = 78.6
MFMA_F32_PEAK_TFS = 157.3   # dense FP32 matrix
MFMA_F64_PEAK_TFS = 78.6    # dense FP64 matrix


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cores():
    """(logical CPUs this process may run on, physical cores behind them)."""
    try:
        cpus = sorted(os.sched_getaffinity(0))
    except AttributeError:
        cpus = list(range(os.cpu_count() or 1))
    phys = set()
    try:
        core, pkg, cur = {}, {}, None
        for line in open("/proc/cpuinfo"):
            k, _, v = line.partition(":")
            k, v = k.strip(), v.strip()
            if k == "processor":
                cur = int(v)
            elif k == "core id" and cur is not None:
                core[cur] = v
            elif k == "physical id" and cur is not None:
                pkg[cur] = v
        phys = {(pkg.get(c), core.get(c)) for c in cpus if c in core}
    except OSError:
        pass
    return len(cpus), (len(phys) if phys else None)


def cpu_baseline(p, eps, s, restart, budget_s=30.0):
    """Oracle (plain FP64 numpy/scipy) on a bounded sample: a smaller grid of
    the same operator family (same p, eps, s, restart, leaves of about 1024
    unknowns as on the GPU), factor + solve, BLAS threads on every physical
    core."""
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import krylov, spand
    from oracle.nd import nested_dissection
    from synth.dg_euler import DGConfig, make_problem
    import paper_2101_01763_amd as sp
    n = 32 if p >= 3 else 48
    cfg = DGConfig(n=n, p=p)
    A, xs, b, _ = make_problem(cfg)
    As = A.to_scipy().tocsr()
    L = sp.levels_for(cfg.N)
    nproc, nphys = host_cores()
    with threadpool_limits(limits=nphys or nproc):
        t0 = time.perf_counter()
        F = spand.factor(As, nested_dissection(n, n, True, False, L), cfg.b, eps)
        t1 = time.perf_counter()
        x, info = krylov.sstep_gmres(lambda v: As @ v, b, lambda v: spand.apply(F, v), s=s,
                                     rtol=1e-8, restart=restart)
        t2 = time.perf_counter()
        threads = max([d.get("num_threads", 1) for d in threadpool_info()] + [1])
    return {"value": cfg.N / (t2 - t0), "unit": "DOF/s", "cores": int(threads),
            "kind": "oracle", "nproc": nproc, "physical_cores": nphys,
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
    graph-replayed sweeps, autotuned SpMV/GEMV shapes).  The systems of one
    block size are factored together (one set of launches per phase for a
    group of up to 4M unknowns); each is solved on its own worker stream.
    value = total DOF / wall time of one batched factor+solve; the same batch
    with every system factored on its own (8 streams, then 1) is timed
    beside it."""
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

    extra = {}

    def run(streams, separate=False, probe=False):
        os.environ["SPAND_BATCH_STREAMS"] = str(streams)
        os.environ["SPAND_BATCH_SEPARATE"] = "1" if separate else "0"
        t0 = time.perf_counter()
        Fs = sp.factor_batched(systems, eps=1e-2, nlevels=Ls, dtype="f32")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        xs, infos = sp.solve_batched([q[0] for q in systems], rhs, Fs, s=5, restart=60, rtol=1e-8,
                                     lagged=args.schedule == "lagged")
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if probe:
            # the shared factorizations, and one apply of every system: one
            # replay per shared sweep graph against one apply per handle
            extra["shared_factorizations"] = int(round(sum(1.0 / F.stats()["batch_systems"]
                                                           for F in Fs)))
            outs = [torch.empty_like(b) for b in rhs]
            sp.apply_batched(Fs, rhs, outs)
            torch.cuda.synchronize()
            tb = []
            for _ in range(5):
                t3 = time.perf_counter()
                sp.apply_batched(Fs, rhs, outs)
                torch.cuda.synchronize()
                tb.append(time.perf_counter() - t3)
            t3 = time.perf_counter()
            for F, b, o in zip(Fs, rhs, outs):
                F.apply(b, out=o)
            torch.cuda.synchronize()
            extra["apply_all_ms"] = {"batched_graphs": 1e3 * float(np.median(tb)),
                                     "per_handle": 1e3 * (time.perf_counter() - t3)}
        for F in Fs:
            F.destroy()
        return t1 - t0, t2 - t1, infos

    nst = args.batch_streams
    for _ in range(args.warmup):
        run(nst)
    res = [run(nst, probe=(k == 0)) for k in range(args.steps)]
    tf = float(np.median([r[0] for r in res]))
    ts = float(np.median([r[1] for r in res]))
    infos = res[-1][2]
    sep = run(nst, separate=True)
    seq = run(1, separate=True)
    out = {
        "metric": "batched spaND factor + s-step GMRES (64 uneven systems); DOF/s",
        "value": ntot / (tf + ts), "unit": "DOF/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": 1e3 * (tf + ts), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32 (spaND) + f64 (Krylov)",
        "data": "synthetic (64 seeded DG-Euler systems)",
        "config": {"workload": f"C4 batch: 64 systems, {ntot} DOF total, n in 32..96, p in 1..3, "
                               f"FP32 spaND eps=1e-2, s=5, m=60, rtol=1e-8 ({args.schedule}); "
                               f"systems of one block size factored together (groups of up to 4M "
                               f"unknowns, 2 at a time), solves on {nst} streams",
                   "schedule": args.schedule},
        "t_factor_ms": 1e3 * tf, "t_solve_ms": 1e3 * ts,
        "all_converged": all(i.converged for i in infos),
        "iters_min_max": [min(i.iters for i in infos), max(i.iters for i in infos)],
        "shared_factorizations": extra.get("shared_factorizations"),
        "apply_all_ms": extra.get("apply_all_ms"),
        "separate_factorizations": {"t_factor_ms": 1e3 * sep[0], "t_solve_ms": 1e3 * sep[1],
                                    "dof_per_s": ntot / (sep[0] + sep[1])},
        "one_stream": {"t_factor_ms": 1e3 * seq[0], "t_solve_ms": 1e3 * seq[1],
                       "dof_per_s": ntot / (seq[0] + seq[1])},
    }
    print(json.dumps(out), flush=True)


def bench_ptc(args):
    """The pseudo-transient nonlinear loop (paper Sec. "Flow Solver", Eqs. (5),
    (8), (9)) on the 128x128, p = 2 operator family from the seeded smooth
    state: CFL^0 = 1000 (the paper's), CFL^inf = 1e8, until the density
    residual has dropped 8 orders; each step factors (then refactors, reusing
    the symbolic phase) with FP32 spaND eps = 1e-2, L = 10, and solves with
    s-step GMRES (s = 5, m = 60) to 1e-3 or at most 20 iterations, as in the
    paper's experiments.  The
    residual and the exact Jacobian are assembled on the host (numpy) and
    streamed to the device every step; their time is reported apart from the
    device's factor and solve time."""
    import torch
    from paper_2101_01763_amd.ptc import ptc_solve
    from synth.dg_euler import (DGConfig, element_means, initial_state, jacobian, local_lambda,
                                residual)
    cfg = DGConfig(n=128, p=2)

    def res(u):
        uh = u.reshape(cfg.K, -1, 4)
        return residual(cfg, uh, element_means(cfg, uh)).reshape(-1)

    def jac(u, dtau):
        uh = u.reshape(cfg.K, -1, 4)
        B = jacobian(cfg, uh, element_means(cfg, uh), dtau)
        return B.rowptr, B.colind, B.val

    def lam(u):
        return local_lambda(cfg, element_means(cfg, u.reshape(cfg.K, -1, 4)))

    t0 = time.perf_counter()
    u, r = ptc_solve((cfg.n, cfg.n, True, False), res, jac, lam, initial_state(cfg).reshape(-1),
                     cfl0=1000.0, cfl_inf=args.ptc_cfl_inf, eps=args.ptc_eps, nlevels=10,
                     dtype=args.dtype, s=5, restart=60, rtol=1e-3, maxit=args.ptc_maxit)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    dev = r.t_factor_s + r.t_solve_s
    print(json.dumps({
        "metric": "pseudo-transient loop to 8 orders of density residual; device factor+solve "
                  "time per nonlinear step",
        "value": 1e3 * dev / max(r.steps, 1), "unit": "ms/step", "higher_is_better": False,
        "n_gpus": 1, "dtype": f"{args.dtype} (spaND) + f64 (Krylov, residual, Jacobian)",
        "data": "synthetic (seeded smooth DG-Euler state)",
        "config": {"workload": f"DG-Euler 128x128 p=2 (N={cfg.N}); CFL0 1000, "
                               f"CFLinf {args.ptc_cfl_inf:g}; spaND eps {args.ptc_eps:g} L 10; "
                               f"s-step GMRES "
                               f"s 5 m 60 rtol 1e-3, at most {args.ptc_maxit} iterations per "
                               f"step"},
        "steps": r.steps, "converged": r.converged,
        "density_residual_drop": r.rho_norm[-1] / r.rho_norm[0],
        "res_norm": r.res_norm, "cfl": r.cfl, "gmres_iters": r.lin_iters,
        "t_factor_ms": 1e3 * r.t_factor_s, "t_solve_ms": 1e3 * r.t_solve_s,
        "t_host_assembly_s": r.t_assemble_s, "t_transfer_s": r.t_upload_s, "wall_s": wall}),
        flush=True)


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
    ap.add_argument("--workload", default="c3", choices=sorted(WORKLOADS) + ["c4", "ptc"])
    ap.add_argument("--dtype", default="f32", choices=["f32", "f64"])
    ap.add_argument("--levels", type=int, default=0)
    ap.add_argument("--eps", type=float, default=None)
    ap.add_argument("--schedule", default="lagged", choices=["two-pass", "lagged"],
                    help="s-step orthogonalisation: two passes per block, or the "
                         "single-reduce schedule with the second pass lagged")
    ap.add_argument("--ptc-cfl-inf", type=float, default=1e8,
                    help="pseudo-transient loop: largest CFL number (Eq. (9))")
    ap.add_argument("--ptc-eps", type=float, default=1e-3,
                    help="pseudo-transient loop: spaND tolerance (the paper's: 1e-3)")
    ap.add_argument("--ptc-maxit", type=int, default=20,
                    help="pseudo-transient loop: GMRES iterations per step (the paper's: 20)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the FP64-factor comparison run (child process)")
    ap.add_argument("--no-secondary", action="store_true",
                    help="skip the secondary C3 points (L = 12; eps = 0.1)")
    ap.add_argument("--batch-streams", type=int, default=8,
                    help="C4: worker streams of the batched calls")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the measured copy / matrix-core ceilings")
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
    if args.workload == "ptc":
        return bench_ptc(args)
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
    nnzb = int(dA.colind.numel())
    bsz = cfg.b
    ceil = None
    if not args.no_ceilings:
        # achievable ceilings of this device, measured by the library's own
        # kernels before the timed region
        ceil = {"copy_GBs": sp.measure_bandwidth("copy", 4 << 30, 5),
                "read_GBs": sp.measure_bandwidth("read", 4 << 30, 5),
                "mfma_f32_TFs": sp.measure_mfma("f32", 5), "mfma_f64_TFs": sp.measure_mfma("f64", 5),
                "kernels": "streaming copy and streaming read of 4 GiB (16-byte non-temporal "
                           "loads/stores); loops of independent v_mfma_f32_32x32x2f32 / "
                           "v_mfma_f64_16x16x4f64 on every CU"}
        log(f"ceilings: copy {ceil['copy_GBs']:.0f} GB/s, read {ceil['read_GBs']:.0f} GB/s, FP32 "
            f"MFMA {ceil['mfma_f32_TFs']:.1f} TFLOP/s, FP64 MFMA {ceil['mfma_f64_TFs']:.1f} TFLOP/s")

    r = run_steps(sp, torch, dA, db, dxs, cfg, eps, L, args.dtype, s, m, args.schedule,
                  args.steps, args.warmup, label="")
    mfma_peak = MFMA_F32_PEAK_TFS if args.dtype == "f32" else MFMA_F64_PEAK_TFS
    out = {
        "metric": "spaND factor+s-step GMRES time to rtol 1e-8, FP32- vs FP64-spaND; DOF/s",
        "value": r["value"],
        "unit": "DOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
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
    }
    out.update(r["summary"])
    # dominant factorization kernel: the rank-revealing QR (one launch per
    # level).  Its arithmetic is FP64 on the vector units (the factor's FP32
    # W is widened to double for every dot product, norm and coordinate), so
    # its roof is the FP64 vector peak; its arithmetic intensity (algorithmic
    # flops over algorithmic bytes, about 60 flop/B) is above that ridge
    # point (78.6 / 8 = 10 flop/B): the binding roof is the ALU, not HBM.
    q = r["qrcp"]
    out["roofline"] = {
        "kernel": "k_qrcp (column-pivoted QR of [A_sn A_ns^T], all interfaces of one level per "
                  "launch)", "bound": "alu",
        "achieved": q["tflops"], "peak": ALU_F64_PEAK_TFS, "unit": "TFLOP/s",
        "frac": q["tflops"] / ALU_F64_PEAK_TFS, "traffic": pmc_traffic("k_qrcp"),
        "arithmetic": "FP64 vector (FP32 operands widened)",
        "flops_per_launch": q["flops_per_launch"], "avg_launch_ms": q["avg_ms"],
        "launches": q["launches"],
        "algorithmic_flops": "sum over interfaces of 4mck - 2k^2(m+c) + 4k^3/3 "
                             "(k Householder-equivalent steps on m x c)",
        "bytes_per_launch": q["bytes_per_launch"], "hbm_achieved_GBs": q["GBs"],
        "algorithmic_bytes": "each W (m x ncols) read once + each Q (m x m) written once, "
                             "factor precision"}
    sv = r["spmv"]
    out["roofline_spmv"] = {
        "kernel": "k_spmv (BSR SpMV, FP64)", "bound": "hbm", "achieved": sv["GBs"],
        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": sv["GBs"] / HBM_PEAK_GBS,
        "bytes_per_launch": sv["bytes"], "avg_launch_ms": sv["avg_ms"], "launches": sv["launches"],
        "algorithmic_bytes": "8 nnzb b^2 + 4 nnzb + 4 (K+1) + 16 N"}
    ap_ = r["apply"]
    out["roofline_apply"] = {
        "kernel": "M^-1 r sweeps (k_gemv, k_pull, k_slot_copy replayed from a hipGraph)",
        "bound": "hbm", "achieved": ap_["GBs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
        "frac": ap_["GBs"] / HBM_PEAK_GBS, "bytes_per_apply": ap_["bytes"],
        "avg_apply_ms": ap_["avg_ms"], "applies": ap_["n"],
        "algorithmic_bytes": "every stored factor entry once per apply (A_ss^-1 in both sweeps) "
                             "in factor precision + 16 N for the FP64 vector in and out"}
    g = r["mfma"]
    out["roofline_factor_mfma"] = {
        "kernel": "factorization products on the matrix cores (k_gemm_f32_mfma / "
                  "k_gemm_f64_mfma batched GEMMs, k_schur_elem_mfma level-0 Schur)",
        "bound": "mfma", "achieved": g["tflops"], "peak": mfma_peak, "unit": "TFLOP/s",
        "frac": g["tflops"] / mfma_peak, "flops_per_step": g["flops"], "ms_per_step": g["ms"],
        "launches_per_step": g["launches"], "hbm_GBs": g["GBs"],
        "gemm": g["gemm"], "schur_elem": g["schur"],
        "algorithmic_flops": "2MNK per product (zero half of triangular operands excluded), "
                             "4 b^3 per level-0 Schur coupling pair"}
    if ceil:
        out["ceilings_measured"] = ceil
        out["roofline"]["frac_of_measured"] = None          # ALU roof: no matrix-core loop
        # the SpMV and the sweeps read almost all of their bytes: against the
        # measured streaming-read bandwidth
        out["roofline_spmv"]["frac_of_measured"] = sv["GBs"] / ceil["read_GBs"]
        out["roofline_apply"]["frac_of_measured"] = ap_["GBs"] / ceil["read_GBs"]
        out["roofline_factor_mfma"]["frac_of_measured"] = g["tflops"] / (
            ceil["mfma_f32_TFs"] if args.dtype == "f32" else ceil["mfma_f64_TFs"])
    if not args.no_secondary and args.workload == "c3":
        # the other 256x256 p = 3 points, same process and precision: the
        # element rule's L = 12, and the paper's other tolerance eps = 0.1
        sec = []
        for e2, L2 in ((eps, 12), (1e-1, L)):
            if (e2, L2) == (eps, L):
                continue
            r2 = run_steps(sp, torch, dA, db, dxs, cfg, e2, L2, args.dtype, s, m, args.schedule,
                           3, 1, label=f"eps={e2} L={L2} ")
            d = {"eps": e2, "levels": L2, "dof_per_s": r2["value"],
                 "ms_per_step": r2["ms_per_step"], "steps": 3, "warmup": 1}
            d.update(r2["summary"])
            d["roofline_apply_GBs"] = r2["apply"]["GBs"]
            sec.append(d)
        out["secondary"] = sec
    if not args.no_compare:
        # The other precision, one warm-up and three timed steps, in a child
        # process: a fresh device allocator, as in a run of its own (in this
        # process the block cache and the driver hold the first precision's
        # blocks, whose sizes the other precision never asks for).  With the
        # secondary points, also at the paper's other tolerance eps = 0.1.
        import subprocess
        other = "f64" if args.dtype == "f32" else "f32"
        sp.pool_trim()
        torch.cuda.empty_cache()
        cmp_eps = [eps]
        if args.workload == "c3" and not args.no_secondary and eps != 1e-1:
            cmp_eps.append(1e-1)
        for ce in cmp_eps:
            key = f"compare_{other}_factor" + ("" if ce == eps else f"_eps{ce:g}")
            cmd = [sys.executable, os.path.abspath(__file__), "--workload", args.workload,
                   "--dtype", other, "--steps", "3", "--warmup", "1", "--no-compare",
                   "--no-cpu-baseline", "--no-secondary", "--no-ceilings", "--levels", str(L),
                   "--eps", str(ce), "--schedule", args.schedule]
            log(f"comparison: {other} factor, eps {ce:g}, in a child process")
            try:
                rr = subprocess.run(cmd, capture_output=True, text=True, timeout=900)
                lines = [q_ for q_ in rr.stdout.strip().splitlines() if q_.startswith("{")]
                if rr.returncode != 0 or not lines:
                    raise RuntimeError(f"exit {rr.returncode}: {rr.stderr[-500:]}")
                c = json.loads(lines[-1])
                keep = ("t_factor_ms", "t_solve_ms", "iters", "relres", "rel_err_vs_xstar",
                        "factor_phases_ms", "solve_phases_ms", "t_factor_ms_min", "t_solve_ms_min")
                d = {"eps": ce, "levels": L}
                d.update({k: c[k] for k in keep if k in c})
                d["dof_per_s"] = c["value"]
                d["roofline_apply_GBs"] = c["roofline_apply"]["achieved"]
                d["roofline_factor_mfma"] = {k: c["roofline_factor_mfma"][k] for k in
                                             ("achieved", "peak", "frac", "unit")}
                d["run"] = "child process, 1 warm-up + 3 timed steps (medians)"
                out[key] = d
            except (RuntimeError, subprocess.TimeoutExpired, ValueError, KeyError) as ex:
                # the comparison is context; the measured line stands without it
                log(f"comparison run failed: {ex}")
                out[key] = {"error": str(ex)[-500:]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(p, eps, s, m)
    print(json.dumps(out), flush=True)


def run_steps(sp, torch, dA, db, dxs, cfg, eps, L, dtype, s, m, schedule, steps, warmup,
              label=""):
    """`warmup` untimed and `steps` timed steps of (factor, solve); returns the
    rate, per-step medians, phase times and the per-kernel rooflines over the
    timed steps."""
    n = cfg.n

    def step():
        t0 = time.perf_counter()
        F = sp.factor(dA, n, n, True, False, eps=eps, nlevels=L, dtype=dtype)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, info = sp.solve(dA, db, F, s=s, restart=m, rtol=1e-8, lagged=schedule == "lagged")
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        return F, x, info, t1 - t0, t2 - t1

    for w in range(warmup):
        F, x, info, tf, ts = step()
        log(f"{label}warmup {w}: factor {tf * 1e3:.1f} ms solve {ts * 1e3:.1f} ms iters {info.iters}")
        del F
    torch.cuda.synchronize()
    tfs, tss, infos, sts = [], [], [], []
    t_start = time.perf_counter()
    for k in range(steps):
        F, x, info, tf, ts = step()
        st = F.stats()
        tfs.append(tf)
        tss.append(ts)
        infos.append(info)
        sts.append(st)
        log(f"{label}step {k}: factor {tf * 1e3:.1f} ms solve {ts * 1e3:.1f} ms iters {info.iters} "
            f"relres {info.relres:.2e} | lu {st['t_lu_ms']:.0f} schur {st['t_schur_ms']:.0f} "
            f"scale {st['t_scale_ms']:.0f} rrqr {st['t_rrqr_ms']:.0f} (qrcp {st['t_qrcp_ms']:.0f}) "
            f"compress {st['t_compress_ms']:.0f} host {st['t_host_ms']:.0f} "
            f"alloc {st['t_alloc_ms']:.0f} ms | gemm {st['t_gemm_ms']:.0f} ms "
            f"schur-mfma {st['t_schur_elem_ms']:.0f} ms | apply {info.t_apply_ms:.0f} ms "
            f"spmv {info.t_spmv_ms:.0f} ms")
        del F
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t_start
    err = float(torch.linalg.norm(x - dxs) / torch.linalg.norm(dxs))
    N, nnzb, bsz = cfg.N, int(dA.colind.numel()), cfg.b
    tot = lambda key: sum(q[key] for q in sts)
    # SpMV: values, indices, x read once, y written
    spmv_bytes = 8 * nnzb * bsz * bsz + 4 * nnzb + 4 * (cfg.K + 1) + 16 * N
    spmv_ms = sum(i.t_spmv_ms for i in infos)
    spmv_n = sum(i.n_spmv for i in infos)
    spmv_avg = spmv_ms / max(spmv_n, 1)
    # apply: every stored factor entry once per application + FP64 vector in/out
    app_bytes = float(sts[-1]["factor_bytes"]) + 16.0 * N
    app_ms = sum(i.t_apply_ms for i in infos)
    app_n = sum(i.n_apply for i in infos)
    app_avg = app_ms / max(app_n, 1)
    q_ms, q_n = tot("t_qrcp_ms"), tot("n_qrcp")
    q_avg = q_ms / max(q_n, 1)
    q_fl = tot("qrcp_flops") / max(q_n, 1)
    q_by = tot("qrcp_bytes") / max(q_n, 1)
    g_ms, g_fl, g_by = tot("t_gemm_ms"), tot("gemm_flops"), tot("gemm_bytes")
    c_ms, c_fl, c_by = tot("t_schur_elem_ms"), tot("schur_elem_flops"), tot("schur_elem_bytes")
    mf_ms = g_ms + c_ms
    med = lambda v: float(np.median(v))
    last = sts[-1]
    return {
        "value": N * steps / t_total, "ms_per_step": 1e3 * t_total / steps,
        "summary": {
            "t_factor_ms": 1e3 * med(tfs), "t_solve_ms": 1e3 * med(tss),
            "t_factor_ms_min": 1e3 * min(tfs), "t_solve_ms_min": 1e3 * min(tss),
            "iters": infos[-1].iters, "relres": infos[-1].relres, "rel_err_vs_xstar": err,
            "factor_phases_ms": {k: med([q[k] for q in sts]) for k in
                                 ("t_host_ms", "t_lu_ms", "t_schur_ms", "t_scale_ms", "t_rrqr_ms",
                                  "t_compress_ms", "t_qrcp_ms", "t_gemm_ms", "t_schur_elem_ms",
                                  "t_alloc_ms")},
            "factor_stats": {k: last[k] for k in ("top_size", "factor_bytes", "factor_flops",
                                                  "rank_avg", "rank_max", "resident_bytes")},
            "solve_phases_ms": {"spmv": med([i.t_spmv_ms for i in infos]),
                                "apply": med([i.t_apply_ms for i in infos]),
                                "orth": med([i.t_orth_ms for i in infos]),
                                "other": med([i.t_other_ms for i in infos])},
            "solve_reductions": infos[-1].n_reduce,
        },
        "spmv": {"bytes": spmv_bytes, "avg_ms": spmv_avg, "launches": spmv_n,
                 "GBs": spmv_bytes / (spmv_avg * 1e-3) / 1e9 if spmv_n else 0.0},
        "apply": {"bytes": app_bytes, "avg_ms": app_avg, "n": app_n,
                  "GBs": app_bytes / (app_avg * 1e-3) / 1e9 if app_n else 0.0},
        "qrcp": {"avg_ms": q_avg, "launches": q_n, "flops_per_launch": q_fl,
                 "bytes_per_launch": q_by,
                 "tflops": q_fl / (q_avg * 1e-3) / 1e12 if q_n else 0.0,
                 "GBs": q_by / (q_avg * 1e-3) / 1e9 if q_n else 0.0},
        "mfma": {"flops": (g_fl + c_fl) / steps, "ms": mf_ms / steps,
                 "launches": (tot("n_gemm") + tot("n_schur_elem")) / steps,
                 "tflops": (g_fl + c_fl) / (mf_ms * 1e-3) / 1e12 if mf_ms else 0.0,
                 "GBs": (g_by + c_by) / (mf_ms * 1e-3) / 1e9 if mf_ms else 0.0,
                 "gemm": {"ms_per_step": g_ms / steps, "flops_per_step": g_fl / steps,
                          "tflops": g_fl / (g_ms * 1e-3) / 1e12 if g_ms else 0.0,
                          "GBs": g_by / (g_ms * 1e-3) / 1e9 if g_ms else 0.0},
                 "schur": {"ms_per_step": c_ms / steps, "flops_per_step": c_fl / steps,
                           "tflops": c_fl / (c_ms * 1e-3) / 1e12 if c_ms else 0.0,
                           "GBs": c_by / (c_ms * 1e-3) / 1e9 if c_ms else 0.0}},
    }


if __name__ == "__main__":
    main()
