"""Python binding of libspand (spaND-preconditioned s-step GMRES on MI355X).

Argument marshalling only: every step of the solver runs in the HIP
kernels of libspand.so (built in-tree by ``paper_2101_01763_amd.build``).
PyTorch supplies device memory (tensors) and the current HIP stream.
There is no fallback: if the library is missing, importing the binding's
functions raises.

Entry points mirror include/spand.h:
    factor(A, grid, eps, nlevels, dtype) -> Factor
    Factor.apply(r), Factor.apply_T(r), Factor.stats()
    solve(A, b, M=None, s=5, restart=60, rtol=1e-8, maxit=1000, transpose=False, x0=None)
    spmv(A, x, transpose=False), pattern_outer(A, u, v, alpha)
    nd(nx, ny, periodic_x, periodic_y, L)     (host only, no GPU)
    SpandSolve.apply(vals, b, A_pattern, M, opts)  (autograd: adjoint solve)
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspand.so")

SPAND_OK, SPAND_EINVAL, SPAND_ENOMEM, SPAND_ESINGULAR, SPAND_EHIP = 0, -1, -2, -3, -4
SPAND_ENOTCONV, SPAND_EBREAKDOWN = 1, 2
SPAND_F64, SPAND_F32 = 0, 1
SSTEP_MAX_HIST = 1024
SPAND_MAX_LEVELS = 32


class spand_bsr_t(C.Structure):
    _fields_ = [("n_brows", C.c_int32), ("bs", C.c_int32), ("nnzb", C.c_int64),
                ("d_rowptr", C.c_void_p), ("d_colind", C.c_void_p), ("d_val", C.c_void_p)]


class spand_grid_t(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("periodic_x", C.c_int32),
                ("periodic_y", C.c_int32)]


class spand_opts_t(C.Structure):
    _fields_ = [("eps", C.c_double), ("nlevels", C.c_int32), ("factor_dtype", C.c_int32),
                ("flags", C.c_int32)]


SSTEP_FLAG_MONOMIAL, SSTEP_FLAG_ONE_PASS, SSTEP_FLAG_ORTH_LOSS, SSTEP_FLAG_CLASSICAL = 1, 2, 4, 8
SSTEP_FLAG_LAGGED = 16


class sstep_opts_t(C.Structure):
    _fields_ = [("s", C.c_int32), ("restart", C.c_int32), ("maxit", C.c_int32),
                ("transpose", C.c_int32), ("rtol", C.c_double), ("flags", C.c_int32),
                ("pad", C.c_int32)]


class sstep_stats_t(C.Structure):
    _fields_ = [("iters", C.c_int32), ("restarts", C.c_int32), ("converged", C.c_int32),
                ("n_hist", C.c_int32), ("relres", C.c_double),
                ("hist", C.c_double * SSTEP_MAX_HIST), ("n_shifts", C.c_int32),
                ("shift_re", C.c_double * 8), ("shift_im", C.c_double * 8),
                ("t_total_ms", C.c_double), ("t_spmv_ms", C.c_double),
                ("t_apply_ms", C.c_double), ("t_orth_ms", C.c_double),
                ("t_other_ms", C.c_double), ("n_spmv", C.c_int32), ("n_apply", C.c_int32),
                ("n_orth", C.c_int32), ("n_reduce", C.c_int32),
                ("orth_loss", C.c_double * SSTEP_MAX_HIST),
                ("orth_cols", C.c_int32 * SSTEP_MAX_HIST)]


class spand_factor_stats_t(C.Structure):
    L = SPAND_MAX_LEVELS
    _fields_ = [("nlevels", C.c_int32), ("n_clusters", C.c_int32 * L),
                ("rank_min", C.c_int32 * L), ("rank_max", C.c_int32 * L),
                ("rank_avg", C.c_double * L), ("size_before", C.c_int64 * L),
                ("size_after", C.c_int64 * L), ("top_size", C.c_int32),
                ("factor_bytes", C.c_int64), ("factor_flops", C.c_double),
                ("t_host_ms", C.c_double), ("t_device_ms", C.c_double),
                ("t_lu_ms", C.c_double), ("t_schur_ms", C.c_double),
                ("t_scale_ms", C.c_double), ("t_rrqr_ms", C.c_double),
                ("t_compress_ms", C.c_double), ("t_qrcp_ms", C.c_double),
                ("n_qrcp", C.c_int32), ("pad0", C.c_int32), ("qrcp_bytes", C.c_double),
                ("qrcp_flops", C.c_double), ("t_alloc_ms", C.c_double),
                ("resident_bytes", C.c_int64), ("t_plan_ms", C.c_double * 6),
                ("t_gemm_ms", C.c_double), ("gemm_flops", C.c_double),
                ("gemm_bytes", C.c_double), ("n_gemm", C.c_int32), ("n_schur_elem", C.c_int32),
                ("t_schur_elem_ms", C.c_double), ("schur_elem_flops", C.c_double),
                ("schur_elem_bytes", C.c_double), ("batch_systems", C.c_int32),
                ("pad1", C.c_int32)]


EXPORTS = ["spand_factor", "spand_apply", "spand_apply_T", "sstep_gmres_solve",
           "spand_bsr_spmv", "spand_bsr_pattern_outer", "spand_factor_stats",
           "spand_destroy", "spand_nd", "spand_status_string", "spand_last_error",
           "spand_factor_batched", "sstep_gmres_solve_batched", "spand_pool_trim",
           "sstep_gmres_solve_noalloc", "spand_measure_bandwidth", "spand_measure_mfma",
           "spand_refactor", "spand_apply_batched"]
SPAND_NOALLOC_SCRATCH_BYTES = 64 << 20
SPAND_FLAG_NO_GRAPH = 1

_lib = None


class SpandError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{msg} (status {code})")
        self.code = code


def lib():
    """Load libspand.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: run `python -m paper_2101_01763_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp, i32, dbl = C.c_void_p, C.c_int32, C.c_double
        L.spand_factor.argtypes = [C.POINTER(spand_bsr_t), C.POINTER(spand_grid_t),
                                   C.POINTER(spand_opts_t), vp, C.POINTER(vp)]
        L.spand_apply.argtypes = [vp, vp, vp, vp]
        L.spand_refactor.argtypes = [vp, C.POINTER(spand_bsr_t), vp]
        L.spand_apply_T.argtypes = [vp, vp, vp, vp]
        L.sstep_gmres_solve.argtypes = [C.POINTER(spand_bsr_t), vp, vp, vp,
                                        C.POINTER(sstep_opts_t), C.POINTER(sstep_stats_t), vp]
        L.sstep_gmres_solve_noalloc.argtypes = L.sstep_gmres_solve.argtypes
        L.spand_measure_bandwidth.argtypes = [i32, C.c_size_t, C.c_int, vp, C.POINTER(dbl)]
        L.spand_measure_mfma.argtypes = [i32, C.c_int, vp, C.POINTER(dbl)]
        L.spand_bsr_spmv.argtypes = [C.POINTER(spand_bsr_t), C.c_int, dbl, vp, dbl, vp, vp]
        L.spand_bsr_pattern_outer.argtypes = [C.POINTER(spand_bsr_t), vp, vp, dbl, vp, vp]
        L.spand_factor_stats.argtypes = [vp, C.POINTER(spand_factor_stats_t)]
        L.spand_destroy.argtypes = [vp]
        L.spand_nd.argtypes = [C.POINTER(spand_grid_t), i32, C.POINTER(i32)] + [vp] * 7
        L.spand_factor_batched.argtypes = [i32, C.POINTER(spand_bsr_t), C.POINTER(spand_grid_t),
                                           C.POINTER(spand_opts_t), vp, C.POINTER(vp)]
        L.sstep_gmres_solve_batched.argtypes = [i32, C.POINTER(spand_bsr_t), C.POINTER(vp),
                                                C.POINTER(vp), C.POINTER(vp),
                                                C.POINTER(sstep_opts_t), C.POINTER(sstep_stats_t), vp]
        L.spand_apply_batched.argtypes = [i32, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), i32,
                                          vp]
        L.spand_pool_trim.argtypes = []
        L.spand_status_string.restype = C.c_char_p
        L.spand_status_string.argtypes = [C.c_int]
        L.spand_last_error.restype = C.c_char_p
        for f in EXPORTS:
            if f not in ("spand_status_string", "spand_last_error"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def _check(code, allow=(SPAND_OK,)):
    if code in allow:
        return code
    L = lib()
    raise SpandError(code, f"{L.spand_status_string(code).decode()}: "
                           f"{L.spand_last_error().decode()}")


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _vec(t, n, name, dtype=None, shape=None, check_device=True):
    """Device pointer of a tensor the kernels read or write, after checking
    that it is a contiguous float64 (or `dtype`) CUDA tensor of n elements
    (or of `shape`): a wrong dtype, size or device would make the kernels
    read or write out of bounds, so it is rejected before any launch."""
    import torch
    dtype = torch.float64 if dtype is None else dtype
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name}: expected a torch.Tensor, got {type(t).__name__}")
    if t.dtype != dtype:
        raise ValueError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name}: shape {tuple(t.shape)}, expected {tuple(shape)}")
    if t.numel() != n:
        raise ValueError(f"{name}: {t.numel()} elements, expected {n}")
    if check_device and not t.is_cuda:
        raise ValueError(f"{name}: must be a CUDA (HIP) device tensor")
    return C.c_void_p(t.data_ptr())


@dataclasses.dataclass
class BSRMatrix:
    """Device BSR matrix (torch tensors): rowptr/colind int32, val float64 [nnzb, bs, bs]."""
    rowptr: object
    colind: object
    val: object

    @property
    def n_brows(self):
        return int(self.rowptr.numel()) - 1

    @property
    def bs(self):
        return int(self.val.shape[-1])

    @property
    def N(self):
        return self.n_brows * self.bs

    def c(self, val=None):
        import torch
        v = self.val if val is None else val
        nb, bs = self.n_brows, self.bs
        nnzb = int(self.colind.numel())
        _vec(self.rowptr, nb + 1, "rowptr", dtype=torch.int32, check_device=False)
        _vec(self.colind, nnzb, "colind", dtype=torch.int32, check_device=False)
        _vec(v, nnzb * bs * bs, "val", shape=(nnzb, bs, bs), check_device=False)
        for name, t in (("rowptr", self.rowptr), ("colind", self.colind), ("val", v)):
            if not t.is_cuda:
                raise ValueError(f"{name}: must be a CUDA (HIP) device tensor")
        return spand_bsr_t(nb, bs, nnzb, self.rowptr.data_ptr(), self.colind.data_ptr(),
                           v.data_ptr())

    @staticmethod
    def from_numpy(rowptr, colind, val, device="cuda"):
        import torch
        return BSRMatrix(torch.as_tensor(np.asarray(rowptr, dtype=np.int32), device=device),
                         torch.as_tensor(np.asarray(colind, dtype=np.int32), device=device),
                         torch.as_tensor(np.ascontiguousarray(val, dtype=np.float64), device=device))


class Factor:
    """Handle of a spaND factorization (library-owned device memory)."""

    def __init__(self, handle, N):
        self._h = handle
        self.N = N

    def __del__(self):
        try:
            if self._h:
                lib().spand_destroy(self._h)
                self._h = None
        except Exception:
            pass

    def destroy(self):
        if self._h:
            lib().spand_destroy(self._h)
            self._h = None

    def refactor(self, A, val=None):
        """Rebuild this factorization for new values of a matrix with the
        same block pattern (reuses the nested dissection and the pattern)."""
        Ac = A.c(val)
        if A.N != self.N:
            raise ValueError(f"A has {A.N} unknowns, the factor {self.N}")
        _check(lib().spand_refactor(self._h, C.byref(Ac), _stream()))
        return self

    def apply(self, r, out=None):
        import torch
        pr = _vec(r, self.N, "r")
        out = torch.empty_like(r) if out is None else out
        _check(lib().spand_apply(self._h, pr, _vec(out, self.N, "out"), _stream()))
        return out

    def apply_T(self, r, out=None):
        import torch
        pr = _vec(r, self.N, "r")
        out = torch.empty_like(r) if out is None else out
        _check(lib().spand_apply_T(self._h, pr, _vec(out, self.N, "out"), _stream()))
        return out

    def stats(self):
        st = spand_factor_stats_t()
        _check(lib().spand_factor_stats(self._h, C.byref(st)))
        L = st.nlevels
        return {
            "nlevels": L,
            "n_clusters": list(st.n_clusters[:L - 1]),
            "rank_min": list(st.rank_min[:L - 1]),
            "rank_avg": list(st.rank_avg[:L - 1]),
            "rank_max": list(st.rank_max[:L - 1]),
            "size_before": list(st.size_before[:L - 1]),
            "size_after": list(st.size_after[:L - 1]),
            "top_size": st.top_size,
            "factor_bytes": st.factor_bytes,
            "factor_flops": st.factor_flops,
            "t_host_ms": st.t_host_ms, "t_device_ms": st.t_device_ms,
            "t_lu_ms": st.t_lu_ms, "t_schur_ms": st.t_schur_ms, "t_scale_ms": st.t_scale_ms,
            "t_rrqr_ms": st.t_rrqr_ms, "t_compress_ms": st.t_compress_ms,
            "t_qrcp_ms": st.t_qrcp_ms, "n_qrcp": st.n_qrcp, "qrcp_bytes": st.qrcp_bytes,
            "qrcp_flops": st.qrcp_flops,
            "t_alloc_ms": st.t_alloc_ms, "resident_bytes": st.resident_bytes,
            "t_plan_ms": list(st.t_plan_ms),
            "t_gemm_ms": st.t_gemm_ms, "gemm_flops": st.gemm_flops, "gemm_bytes": st.gemm_bytes,
            "n_gemm": st.n_gemm, "t_schur_elem_ms": st.t_schur_elem_ms,
            "schur_elem_flops": st.schur_elem_flops, "schur_elem_bytes": st.schur_elem_bytes,
            "n_schur_elem": st.n_schur_elem, "batch_systems": st.batch_systems,
        }


def factor(A: BSRMatrix, nx, ny, periodic_x=True, periodic_y=False, eps=1e-2, nlevels=0,
           dtype="f64", val=None, graphs=True) -> Factor:
    g = spand_grid_t(nx, ny, int(periodic_x), int(periodic_y))
    o = spand_opts_t(float(eps), int(nlevels), SPAND_F32 if dtype == "f32" else SPAND_F64,
                     0 if graphs else SPAND_FLAG_NO_GRAPH)
    h = C.c_void_p()
    Ac = A.c(val)
    _check(lib().spand_factor(C.byref(Ac), C.byref(g), C.byref(o), _stream(), C.byref(h)))
    return Factor(h, A.N)


@dataclasses.dataclass
class SolveInfo:
    status: int
    iters: int
    restarts: int
    converged: bool
    relres: float
    history: list
    shifts: list
    t_total_ms: float
    t_spmv_ms: float
    t_apply_ms: float
    t_orth_ms: float
    t_other_ms: float
    n_spmv: int
    n_apply: int
    orth_loss: list = None      # [(basis columns, ||Q^T Q - I||_F)] with orth_loss=True
    n_reduce: int = 0           # inner-product reductions (dots and Gram matrices)


def solve(A: BSRMatrix, b, M: Factor | None = None, s=5, restart=60, rtol=1e-8, maxit=1000,
          transpose=False, x0=None, val=None, monomial=False, passes=2, orth_loss=False,
          classical=False, lagged=False, _entry="sstep_gmres_solve"):
    """s-step GMRES; returns (x, SolveInfo).  ENOTCONV/EBREAKDOWN do not raise.
    monomial / passes=1 / orth_loss: the basis and orthogonalisation variants
    of the stability study; classical: GMRES with modified Gram-Schmidt
    Arnoldi steps (the baseline; s is then unused); lagged: the single-reduce
    schedule of Algorithm 2 (SSTEP_FLAG_*)."""
    import torch
    if passes not in (1, 2):
        raise ValueError("passes must be 1 or 2")
    Ac = A.c(val)
    pb = _vec(b, A.N, "b")
    if x0 is not None:
        _vec(x0, A.N, "x0")
    x = torch.zeros_like(b) if x0 is None else x0.clone(memory_format=torch.contiguous_format)
    flags = ((SSTEP_FLAG_MONOMIAL if monomial else 0) | (SSTEP_FLAG_ONE_PASS if passes == 1 else 0)
             | (SSTEP_FLAG_ORTH_LOSS if orth_loss else 0) | (SSTEP_FLAG_CLASSICAL if classical else 0)
             | (SSTEP_FLAG_LAGGED if lagged else 0))
    o = sstep_opts_t(int(s), int(restart), int(maxit), int(bool(transpose)), float(rtol), flags, 0)
    st = sstep_stats_t()
    if M is not None and M.N != A.N:
        raise ValueError(f"M: factor of {M.N} unknowns for a system of {A.N}")
    code = getattr(lib(), _entry)(C.byref(Ac), M._h if M is not None else None, pb,
                                  _vec(x, A.N, "x"), C.byref(o), C.byref(st), _stream())
    _check(code, allow=(SPAND_OK, SPAND_ENOTCONV, SPAND_EBREAKDOWN))
    info = SolveInfo(code, st.iters, st.restarts, bool(st.converged), st.relres,
                     list(st.hist[:st.n_hist]),
                     [complex(st.shift_re[i], st.shift_im[i]) for i in range(st.n_shifts)],
                     st.t_total_ms, st.t_spmv_ms, st.t_apply_ms, st.t_orth_ms, st.t_other_ms,
                     st.n_spmv, st.n_apply,
                     [(st.orth_cols[i], st.orth_loss[i]) for i in range(st.n_orth)],
                     st.n_reduce)
    return x, info


def solve_noalloc(A: BSRMatrix, b, M: Factor | None = None, **kw):
    """solve() through sstep_gmres_solve_noalloc: no device allocation inside
    the call (the workspace is the library's per-device scratch array of
    SPAND_NOALLOC_SCRATCH_BYTES); same arguments and results."""
    return solve(A, b, M, _entry="sstep_gmres_solve_noalloc", **kw)


def _info(code, st):
    return SolveInfo(code, st.iters, st.restarts, bool(st.converged), st.relres,
                     list(st.hist[:st.n_hist]),
                     [complex(st.shift_re[i], st.shift_im[i]) for i in range(st.n_shifts)],
                     st.t_total_ms, st.t_spmv_ms, st.t_apply_ms, st.t_orth_ms, st.t_other_ms,
                     st.n_spmv, st.n_apply)


def levels_for(N, box_unknowns=1024):
    """Number of ND levels whose leaf boxes hold about `box_unknowns`
    unknowns: round(log2(N / box_unknowns)) + 1 (C2 -> 10, C3 -> 13, C5 -> 11)."""
    import math
    return max(1, int(round(math.log2(max(N, 1) / box_unknowns))) + 1)


def factor_batched(systems, eps=1e-2, nlevels=0, dtype="f32", graphs=True):
    """Factor several systems concurrently.  systems: list of
    (BSRMatrix, nx, ny, periodic_x, periodic_y).  Returns a list of Factor."""
    n = len(systems)
    As = (spand_bsr_t * n)(*[s[0].c() for s in systems])
    gs = (spand_grid_t * n)(*[spand_grid_t(s[1], s[2], int(s[3]), int(s[4])) for s in systems])
    nl = nlevels if isinstance(nlevels, (list, tuple)) else [nlevels] * n
    os_ = (spand_opts_t * n)(*[spand_opts_t(float(eps), int(nl[i]),
                                            SPAND_F32 if dtype == "f32" else SPAND_F64,
                                            0 if graphs else SPAND_FLAG_NO_GRAPH) for i in range(n)])
    hs = (C.c_void_p * n)()
    code = lib().spand_factor_batched(n, As, gs, os_, _stream(), hs)
    fs = [Factor(C.c_void_p(hs[i]), systems[i][0].N) if hs[i] else None for i in range(n)]
    _check(code)
    return fs


def apply_batched(Fs, rs, outs=None, transpose=False):
    """outs[i] = M_i^-1 rs[i] (M_i^-T with transpose) for every factor of Fs;
    the factors of one factor_batched group are applied together by one
    replay of their shared sweep graph."""
    import torch
    n = len(Fs)
    if len(rs) != n or (outs is not None and len(outs) != n):
        raise ValueError("Fs, rs and outs must have the same length")
    outs = [torch.empty_like(r) for r in rs] if outs is None else outs
    pin = [_vec(r, F.N, f"rs[{i}]") for i, (F, r) in enumerate(zip(Fs, rs))]
    pout = [_vec(o, F.N, f"outs[{i}]") for i, (F, o) in enumerate(zip(Fs, outs))]
    hs = (C.c_void_p * n)(*[F._h.value for F in Fs])
    pi = (C.c_void_p * n)(*[p.value for p in pin])
    po = (C.c_void_p * n)(*[p.value for p in pout])
    _check(lib().spand_apply_batched(n, hs, pi, po, 1 if transpose else 0, _stream()))
    return outs


def solve_batched(As, bs, Ms=None, s=5, restart=60, rtol=1e-8, maxit=1000, lagged=False):
    """Concurrent s-step GMRES solves; returns (list of x, list of SolveInfo).
    lagged: the single-reduce schedule of Algorithm 2 for every system."""
    import torch
    n = len(As)
    if len(bs) != n or (Ms is not None and len(Ms) != n):
        raise ValueError("As, bs and Ms must have the same length")
    Ac = (spand_bsr_t * n)(*[A.c() for A in As])
    pbl = [_vec(b, A.N, f"bs[{i}]") for i, (A, b) in enumerate(zip(As, bs))]
    for i, m in enumerate(Ms or []):
        if m is not None and m.N != As[i].N:
            raise ValueError(f"Ms[{i}]: factor of {m.N} unknowns for a system of {As[i].N}")
    xs = [torch.zeros_like(b) for b in bs]
    Mh = (C.c_void_p * n)(*[(m._h.value if m is not None else None) for m in (Ms or [None] * n)])
    pb = (C.c_void_p * n)(*[p.value for p in pbl])
    px = (C.c_void_p * n)(*[x.data_ptr() for x in xs])
    fl = SSTEP_FLAG_LAGGED if lagged else 0
    o = (sstep_opts_t * n)(*[sstep_opts_t(int(s), int(restart), int(maxit), 0, float(rtol), fl, 0)
                             for _ in range(n)])
    st = (sstep_stats_t * n)()
    code = lib().sstep_gmres_solve_batched(n, Ac, Mh, pb, px, o, st, _stream())
    _check(code, allow=(SPAND_OK, SPAND_ENOTCONV, SPAND_EBREAKDOWN))
    return xs, [_info(code, st[i]) for i in range(n)]


def measure_bandwidth(mode="copy", nbytes=4 << 30, reps=5):
    """Streaming bandwidth of the device in GB/s: "copy" (read + write bytes)
    or "read"."""
    v = C.c_double()
    _check(lib().spand_measure_bandwidth(0 if mode == "copy" else 1, int(nbytes), int(reps),
                                         _stream(), C.byref(v)))
    return v.value


def measure_mfma(dtype="f32", reps=5):
    """Matrix-core throughput in TFLOP/s from loops of the factorization's
    MFMA instructions (FP32 32x32x2 or FP64 16x16x4)."""
    v = C.c_double()
    _check(lib().spand_measure_mfma(SPAND_F32 if dtype == "f32" else SPAND_F64, int(reps),
                                    _stream(), C.byref(v)))
    return v.value


def pool_trim():
    """Return the library's cached device blocks to the driver."""
    _check(lib().spand_pool_trim())


def spmv(A: BSRMatrix, x, transpose=False, alpha=1.0, beta=0.0, y=None, val=None):
    import torch
    Ac = A.c(val)
    px = _vec(x, A.N, "x")
    y = torch.zeros_like(x) if y is None else y
    _check(lib().spand_bsr_spmv(C.byref(Ac), int(bool(transpose)), float(alpha), px,
                                float(beta), _vec(y, A.N, "y"), _stream()))
    return y


def pattern_outer(A: BSRMatrix, u, v, alpha=1.0):
    import torch
    Ac = A.c()
    pu, pv = _vec(u, A.N, "u"), _vec(v, A.N, "v")
    out = torch.empty_like(A.val)
    _check(lib().spand_bsr_pattern_outer(C.byref(Ac), pu, pv, float(alpha),
                                         _vec(out, out.numel(), "out"), _stream()))
    return out


def nd(nx, ny, periodic_x=True, periodic_y=False, L=0):
    """Host-only nested dissection (no GPU use).  Returns a dict of int32 arrays
    with the same layout as oracle.nd.flatten."""
    K = nx * ny
    g = spand_grid_t(nx, ny, int(periodic_x), int(periodic_y))
    Lo = C.c_int32()
    node = np.zeros(K, np.int32)
    perm = np.zeros(K, np.int32)
    ncl = np.zeros(SPAND_MAX_LEVELS, np.int32)
    vp = lambda a: a.ctypes.data_as(C.c_void_p)
    _check(lib().spand_nd(C.byref(g), int(L), C.byref(Lo), vp(node), vp(perm), vp(ncl),
                          None, None, None, None))
    L = Lo.value
    tot = int(ncl[:L].sum())
    ptr = np.zeros(tot + L, np.int32)
    elems = np.zeros(L * K, np.int32)
    key = np.zeros(2 * tot, np.int32)
    inter = np.zeros(tot, np.int32)
    _check(lib().spand_nd(C.byref(g), int(L), C.byref(Lo), vp(node), vp(perm), vp(ncl),
                          vp(ptr), vp(elems), vp(key), vp(inter)))
    out = {"L": L, "node_of_elem": node, "perm": perm}
    pb = cb = 0
    for l in range(L):
        n = int(ncl[l])
        p = ptr[pb:pb + n + 1].copy()
        out[f"ptr_{l}"] = p
        out[f"elems_{l}"] = elems[l * K:l * K + p[-1]].copy()
        out[f"key_{l}"] = key[2 * cb:2 * (cb + n)].reshape(-1, 2).copy()
        out[f"interior_{l}"] = inter[cb:cb + n].copy()
        pb += n + 1
        cb += n
    return out


class SpandSolve:
    """Differentiable x = A^{-1} b (A given by its BSR values on a fixed
    pattern), solved with spaND-preconditioned s-step GMRES.  Backward solves
    A^T lambda = g with the transposed operator and M^{-T} (spand_apply_T) and
    returns dL/db = lambda, dL/dvals = -lambda_I x_J^T on the stored blocks."""

    @staticmethod
    def apply(vals, b, A: BSRMatrix, M: Factor, opts: dict):
        import torch

        class _Fn(torch.autograd.Function):
            @staticmethod
            def forward(ctx, vals_, b_):
                x, info = solve(A, b_, M, val=vals_, **opts)
                if not info.converged:
                    raise SpandError(info.status, f"forward solve did not converge: {info}")
                ctx.save_for_backward(vals_, x)
                return x

            @staticmethod
            def backward(ctx, g):
                vals_, x = ctx.saved_tensors
                lam, info = solve(A, g.contiguous(), M, transpose=True, val=vals_, **opts)
                if not info.converged:
                    raise SpandError(info.status, f"adjoint solve did not converge: {info}")
                gv = pattern_outer(BSRMatrix(A.rowptr, A.colind, vals_), lam, x, alpha=-1.0)
                return gv, lam

        return _Fn.apply(vals, b)
