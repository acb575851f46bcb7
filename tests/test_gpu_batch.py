"""GPU checks of the batched factorization (systems of one block size,
precision and eps factored together, one set of launches per phase):

  * every system's factor equals the one spand_factor computes for it alone,
    bit for bit (per-level ranks, top size, stored bytes, M^-1 r and M^-T r),
    in a batch that mixes block sizes (p = 1, 2: two groups), grid sizes and
    numbers of levels inside one group;
  * spand_apply_batched (one replay of a group's shared sweep graph for all
    its systems) equals the per-handle applies, also for a partial set of a
    group's handles (applied one by one) and in place;
  * the handles of a group stay valid when other handles of the group are
    destroyed; a handle that shares a factorization cannot be refactored;
  * a call mixing whole groups, a partial group, an FP64 group and a factor
    of its own; empty and one-system batches.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2101_01763_amd as sp  # noqa: E402
from synth.dg_euler import DGConfig, make_problem  # noqa: E402

# (n, p, L): two p = 1 systems with 3 and 5 levels, three p = 2 systems with
# 3, 4 and 4 levels (grids of different sizes share a group)
CASES = [(8, 1, 3), (14, 2, 3), (12, 1, 5), (10, 2, 4), (16, 2, 4)]


def _batch(dtype, eps=1e-2):
    systems, cfgs = [], []
    for i, (n, p, L) in enumerate(CASES):
        c = DGConfig(n=n, p=p, seed=40 + i)
        A, xs, b, _ = make_problem(c)
        systems.append((sp.BSRMatrix.from_numpy(A.rowptr, A.colind, A.val), n, n, True, False))
        cfgs.append(c)
    Ls = [L for (_, _, L) in CASES]
    Fs = sp.factor_batched(systems, eps=eps, nlevels=Ls, dtype=dtype)
    return systems, cfgs, Ls, Fs


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_batched_factor_equals_individual(dtype):
    systems, cfgs, Ls, Fs = _batch(dtype)
    groups = {}
    for i, c in enumerate(cfgs):
        groups.setdefault(c.b, []).append(i)
    for i, (sysd, c) in enumerate(zip(systems, cfgs)):
        F1 = sp.factor(sysd[0], sysd[1], sysd[2], True, False, eps=1e-2, nlevels=Ls[i], dtype=dtype)
        sb, s1 = Fs[i].stats(), F1.stats()
        assert sb["batch_systems"] == len(groups[c.b]) and s1["batch_systems"] == 1
        for key in ("nlevels", "n_clusters", "rank_min", "rank_max", "size_before", "size_after",
                    "top_size", "factor_bytes", "factor_flops"):
            assert sb[key] == s1[key], (i, key, sb[key], s1[key])
        r = torch.as_tensor(np.random.default_rng(7 + i).standard_normal(c.N), device="cuda")
        assert torch.equal(Fs[i].apply(r), F1.apply(r)), i
        assert torch.equal(Fs[i].apply_T(r), F1.apply_T(r)), i
        F1.destroy()


def test_apply_batched():
    systems, cfgs, Ls, Fs = _batch("f32")
    rng = np.random.default_rng(11)
    rs = [torch.as_tensor(rng.standard_normal(c.N), device="cuda") for c in cfgs]
    for tr in (False, True):
        ref = [F.apply_T(r) if tr else F.apply(r) for F, r in zip(Fs, rs)]
        out = sp.apply_batched(Fs, rs, transpose=tr)
        for i in range(len(Fs)):
            assert torch.equal(out[i], ref[i]), (tr, i)
        # a partial set of a group (not every system): applied one by one
        sub = [0, 1, 3]
        out = sp.apply_batched([Fs[i] for i in sub], [rs[i] for i in sub], transpose=tr)
        for k, i in enumerate(sub):
            assert torch.equal(out[k], ref[i]), (tr, i)
        # in place
        cp = [r.clone() for r in rs]
        sp.apply_batched(Fs, cp, outs=cp, transpose=tr)
        for i in range(len(Fs)):
            assert torch.equal(cp[i], ref[i]), (tr, i)


def test_batched_handles_lifetime_and_refactor():
    systems, cfgs, Ls, Fs = _batch("f32")
    rng = np.random.default_rng(5)
    rs = [torch.as_tensor(rng.standard_normal(c.N), device="cuda") for c in cfgs]
    ref = [F.apply(r) for F, r in zip(Fs, rs)]
    with pytest.raises(sp.SpandError) as ei:
        Fs[2].refactor(systems[2][0])
    assert ei.value.code == sp.SPAND_EINVAL
    # destroy two handles of the p = 2 group; the third still applies
    Fs[1].destroy()
    Fs[3].destroy()
    torch.cuda.synchronize()
    assert torch.equal(Fs[4].apply(rs[4]), ref[4])
    x, info = sp.solve(systems[4][0], rs[4], Fs[4], s=5, restart=60, rtol=1e-8)
    assert info.converged and info.relres <= 1e-8


def test_apply_batched_mixed_handles():
    """A call mixing whole groups, a partial group, a factor of its own and
    FP64 handles (a group of their own): every result equals that handle's
    own apply; an empty call does nothing."""
    systems, cfgs, Ls, Fs = _batch("f32")
    sysd = systems[0]
    F1 = sp.factor(sysd[0], sysd[1], sysd[2], True, False, eps=1e-2, nlevels=Ls[0], dtype="f32")
    sys64 = [systems[1], systems[3]]
    F64 = sp.factor_batched(sys64, eps=1e-2, nlevels=[Ls[1], Ls[3]], dtype="f64")
    assert all(F.stats()["batch_systems"] == 2 for F in F64)
    # whole groups: p = 1 (Fs[0], Fs[2]) and FP64 (F64); partial: p = 2
    # (Fs[1], Fs[3] without Fs[4]); F1 a factor of its own
    hs = [Fs[0], Fs[2], F1, F64[1], Fs[1], Fs[3], F64[0]]
    ns = [cfgs[0].N, cfgs[2].N, cfgs[0].N, cfgs[3].N, cfgs[1].N, cfgs[3].N, cfgs[1].N]
    rng = np.random.default_rng(21)
    rs = [torch.as_tensor(rng.standard_normal(n), device="cuda") for n in ns]
    for tr in (False, True):
        out = sp.apply_batched(hs, rs, transpose=tr)
        for i, (F, r) in enumerate(zip(hs, rs)):
            ref = F.apply_T(r) if tr else F.apply(r)
            assert torch.equal(out[i], ref), (tr, i)
    assert sp.apply_batched([], []) == []
    with pytest.raises(ValueError):
        sp.apply_batched([Fs[0]], [rs[1]])          # wrong length for the handle


def test_factor_batched_empty_and_single():
    assert sp.factor_batched([], eps=1e-2) == []
    systems, cfgs, Ls, Fs = _batch("f32")
    one = sp.factor_batched([systems[2]], eps=1e-2, nlevels=[Ls[2]], dtype="f32")
    assert one[0].stats()["batch_systems"] == 1
    r = torch.as_tensor(np.random.default_rng(2).standard_normal(cfgs[2].N), device="cuda")
    assert torch.equal(one[0].apply(r), Fs[2].apply(r))
