"""Host-side checks of the C ABI: the library loads, exports every entry
point of include/spand.h, the host ND is bit-exact with the oracle ND, and
argument validation fails before any launch (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import paper_2101_01763_amd as sp
from oracle.nd import flatten, nested_dissection

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_match_header():
    hdr = open(os.path.join(ROOT, "include", "spand.h")).read()
    declared = set(re.findall(r"^\s*(?:int|const char \*)\s*(\w+)\s*\(", hdr, re.M))
    L = sp.lib()
    for name in declared:
        assert hasattr(L, name), name
    assert set(sp.EXPORTS) <= declared


@pytest.mark.parametrize("nx,ny,px,py,L", [(16, 16, 1, 0, 4), (4, 4, 1, 0, 3), (12, 7, 1, 1, 3),
                                            (9, 13, 0, 0, 4), (32, 32, 1, 0, 6), (3, 2, 1, 1, 2),
                                            (128, 128, 1, 0, 10), (20, 36, 1, 0, 0)])
def test_nd_bit_exact_with_oracle(nx, ny, px, py, L):
    from oracle.nd import default_levels
    Lr = L if L > 0 else default_levels(nx * ny)
    ref = flatten(nested_dissection(nx, ny, bool(px), bool(py), Lr))
    got = sp.nd(nx, ny, bool(px), bool(py), L)
    assert got["L"] == Lr
    for k, v in ref.items():
        assert np.array_equal(np.asarray(got[k]), v), k


def test_status_strings():
    L = sp.lib()
    assert L.spand_status_string(0) == b"SPAND_OK"
    assert L.spand_status_string(-3) == b"SPAND_ESINGULAR"
    assert L.spand_status_string(2) == b"SPAND_EBREAKDOWN"


def test_validation_before_launch():
    L = sp.lib()
    A = sp.spand_bsr_t(0, 16, 0, None, None, None)
    g = sp.spand_grid_t(4, 4, 1, 0)
    o = sp.spand_opts_t(1e-2, 0, 0, 0)
    h = C.c_void_p()
    assert L.spand_factor(C.byref(A), C.byref(g), C.byref(o), None, C.byref(h)) == sp.SPAND_EINVAL
    assert b"bad BSR" in L.spand_last_error()
    # grid / size mismatch and bad eps are rejected on the host
    A = sp.spand_bsr_t(16, 16, 64, 1, 1, 1)     # dummy non-null pointers, never dereferenced
    g = sp.spand_grid_t(5, 4, 1, 0)
    assert L.spand_factor(C.byref(A), C.byref(g), C.byref(o), None, C.byref(h)) == sp.SPAND_EINVAL
    g = sp.spand_grid_t(4, 4, 1, 0)
    o = sp.spand_opts_t(-1.0, 0, 0, 0)
    assert L.spand_factor(C.byref(A), C.byref(g), C.byref(o), None, C.byref(h)) == sp.SPAND_EINVAL
    o = sp.spand_opts_t(1e-2, 0, 7, 0)
    assert L.spand_factor(C.byref(A), C.byref(g), C.byref(o), None, C.byref(h)) == sp.SPAND_EINVAL
    so = sp.sstep_opts_t(4, 42, 100, 0, 1e-8)   # restart not a multiple of s
    assert L.sstep_gmres_solve(C.byref(A), None, 1, 1, C.byref(so), None, None) == sp.SPAND_EINVAL
    so = sp.sstep_opts_t(9, 45, 100, 0, 1e-8)   # s too large
    assert L.sstep_gmres_solve(C.byref(A), None, 1, 1, C.byref(so), None, None) == sp.SPAND_EINVAL
    assert L.spand_nd(C.byref(sp.spand_grid_t(0, 4, 1, 0)), 2, None, *([None] * 7)) == sp.SPAND_EINVAL


def test_noalloc_rejects_oversize_before_launch():
    """A solve whose workspace exceeds the no-allocation scratch is rejected
    on the host, before any device call (dummy pointers, never used)."""
    L = sp.lib()
    N_brows = 200_000                       # N = 3.2M unknowns at b = 16
    A = sp.spand_bsr_t(N_brows, 16, N_brows, 1, 1, 1)
    so = sp.sstep_opts_t(5, 60, 100, 0, 1e-8)
    r = L.sstep_gmres_solve_noalloc(C.byref(A), None, 1, 1, C.byref(so), None, None)
    assert r == sp.SPAND_EINVAL
    assert b"no-allocation scratch" in L.spand_last_error()
    so = sp.sstep_opts_t(4, 42, 100, 0, 1e-8)  # the usual argument checks come first
    assert L.sstep_gmres_solve_noalloc(C.byref(A), None, 1, 1, C.byref(so), None, None) == sp.SPAND_EINVAL
    assert b"restart" in L.spand_last_error()
