"""The Python binding rejects tensors the kernels cannot take (wrong dtype,
size, layout or device) with ValueError before any library call, so these
run without a GPU: a float32 right-hand side would otherwise make the solver
read 8N bytes from a 4N-byte buffer, a host tensor would hand a host
pointer to the kernels, and a strided x0 would be read as if contiguous."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2101_01763_amd as sp  # noqa: E402


def _bsr(n=4, bs=2, device="cpu", vdtype=torch.float64):
    rowptr = torch.arange(n + 1, dtype=torch.int32, device=device)
    colind = torch.arange(n, dtype=torch.int32, device=device)
    val = torch.ones(n, bs, bs, dtype=vdtype, device=device)
    return sp.BSRMatrix(rowptr, colind, val)


def test_vec_checks_dtype_layout_size_device():
    t = torch.zeros(8, dtype=torch.float64)
    with pytest.raises(ValueError, match="dtype"):
        sp._vec(t.float(), 8, "b")
    with pytest.raises(ValueError, match="contiguous"):
        sp._vec(torch.zeros(16, dtype=torch.float64)[::2], 8, "b")
    with pytest.raises(ValueError, match="elements"):
        sp._vec(torch.zeros(7, dtype=torch.float64), 8, "b")
    with pytest.raises(ValueError, match="device"):
        sp._vec(t, 8, "b")
    with pytest.raises(ValueError, match="Tensor"):
        sp._vec(np.zeros(8), 8, "b")
    with pytest.raises(ValueError, match="shape"):
        sp._vec(torch.zeros(2, 4, dtype=torch.float64), 8, "val", shape=(4, 2))


def test_bsr_checks():
    with pytest.raises(ValueError, match="val: dtype"):
        _bsr(vdtype=torch.float32).c()
    A = _bsr()
    with pytest.raises(ValueError, match="val: shape"):
        A.c(torch.ones(4, 4, dtype=torch.float64))
    A = sp.BSRMatrix(A.rowptr.long(), A.colind, A.val)
    with pytest.raises(ValueError, match="rowptr: dtype"):
        A.c()
    with pytest.raises(ValueError, match="device"):
        _bsr().c()


def test_apply_and_solve_reject_bad_vectors():
    F = sp.Factor(None, 8)
    with pytest.raises(ValueError, match="dtype"):
        F.apply(torch.zeros(8, dtype=torch.float32))
    with pytest.raises(ValueError, match="elements"):
        F.apply_T(torch.zeros(9, dtype=torch.float64))
    with pytest.raises(ValueError, match="contiguous"):
        F.apply(torch.zeros(16, dtype=torch.float64)[::2])
    with pytest.raises(ValueError):
        sp.solve(_bsr(), torch.zeros(8, dtype=torch.float32))
    with pytest.raises(ValueError):
        sp.spmv(_bsr(), torch.zeros(8, dtype=torch.float64))
    with pytest.raises(ValueError):
        sp.pattern_outer(_bsr(), torch.zeros(8), torch.zeros(8))
