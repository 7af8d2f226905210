"""End-to-end parity of the GPU construction (Alg. 2) with the oracle."""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import butterfly as obf
from oracle import metrics as om
from oracle import operators as ops
from tests.bfconv import canonical_to_oracle, oracle_to_canonical

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bf():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2002_03400_amd as m
    m.lib()
    return m


def _t(x):
    import torch
    return torch.from_numpy(np.asarray(x, np.complex64)).cuda()


def _err(AOm, FOm):
    return float(np.linalg.norm(AOm - FOm) / np.linalg.norm(AOm))


def _exported(bf, H):
    kU, kV = H.ranks()
    return canonical_to_oracle(H.m, H.n, H.L, kU, kV, H.export())


@pytest.fixture(scope="module")
def c1(bf):
    """n = m = 1024, 8 points per wavelength, leaf 32, tol 1e-6, seed 1."""
    g = wl.segment_pair(1024, ppw=8.0)
    op_o = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    Fo = obf.construct(op_o, 1e-6, 32, seed=1)
    say("construct C1 on GPU")
    op = bf.segkernel(g.targets, g.sources, g.k)
    H = bf.construct(op, 1e-6, 32, seed=1)
    return g, op_o, Fo, op, H


def test_c1_error_parity(bf, c1):
    g, op_o, Fo, op, H = c1
    Om = wl.test_columns(1024, 16, 1001)
    AOm = op_o.matvec(Om)
    e_or = _err(AOm, obf.apply(Fo, Om))
    e_gpu = _err(AOm, H.apply(_t(Om)).cpu().numpy())
    say("C1 errors oracle", e_or, "gpu", e_gpu)
    assert e_gpu <= 2 * e_or
    assert e_gpu <= math.sqrt(1.25 * (H.L + 2)) * 1e-6 * 1.2


def test_c1_ranks_and_exported_factors(bf, c1):
    g, op_o, Fo, op, H = c1
    kU, kV = H.ranks()
    ko_U, ko_V, _ = oracle_to_canonical(Fo)
    assert np.abs(kU.astype(int) - ko_U).max() <= 2
    assert np.abs(kV.astype(int) - ko_V).max() <= 2
    Fg = _exported(bf, H)
    A = op_o.dense()
    D = obf.dense(Fg)       # the oracle's independent assembly of the GPU factors
    rel = np.linalg.norm(A - D) / np.linalg.norm(A)
    say("C1 dense reconstruction of GPU factors", rel)
    assert rel <= math.sqrt(1.25 * (H.L + 2)) * 1e-6 * 1.2
    # orthonormal bases
    for U in Fg.U:
        np.testing.assert_allclose(U.conj().T @ U, np.eye(U.shape[1]), atol=1e-12)
    for d in Fg.R.values():
        for Rb in d.values():
            np.testing.assert_allclose(Rb.conj().T @ Rb, np.eye(Rb.shape[1]), atol=1e-12)
    info = H.stats()
    assert info.max_rank == max(kU.max(), kV.max())
    assert info.factor_entries == sum(x.size for x in [*Fg.U, *Fg.V]) + sum(
        b.size for b in Fg.B.values()) + sum(x.size for d in Fg.R.values() for x in d.values()) + sum(
        x.size for d in Fg.W.values() for x in d.values())


def test_c1_apply_adjoint(bf, c1):
    g, op_o, Fo, op, H = c1
    Fg = _exported(bf, H)
    X = wl.test_columns(1024, 5, 3)
    np.testing.assert_allclose(H.apply(_t(X), trans=True).cpu().numpy(),
                               obf.apply_adjoint(Fg, X), atol=2e-6 * np.abs(obf.apply_adjoint(Fg, X)).max())


def test_deterministic(bf):
    g = wl.segment_pair(512, ppw=8.0)
    op = bf.segkernel(g.targets, g.sources, g.k)
    say("determinism n=512")
    a = bf.construct(op, 1e-6, 32, seed=3).export()
    b = bf.construct(op, 1e-6, 32, seed=3).export()
    c = bf.construct(op, 1e-6, 32, seed=4).export()
    assert np.array_equal(a, b)
    assert not (a.shape == c.shape and np.array_equal(a, c))


@pytest.mark.parametrize("L,r", [(3, 2), (4, 4), (5, 8), (6, 8)])
def test_exact_butterfly_recovery(bf, L, r):
    """Sec. 6.1: the GPU recovers an exact butterfly (black box = GPU apply of
    the imported factors, complex64) to single-precision level, all ranks r."""
    fx = wl.exact_butterfly_factors(L, r, seed=L * 10 + r)
    F0 = obf.from_exact(fx)
    kU, kV, data = oracle_to_canonical(F0)
    say("exact butterfly", L, r)
    src = bf.import_factors(fx.n, fx.n, 8, kU, kV, data)
    op = bf.from_factors(src)
    H = bf.construct(op, 1e-5, 8, seed=5)
    gU, gV = H.ranks()
    assert set(np.unique(gU)) == {r} and set(np.unique(gV)) == {r}
    Om = wl.test_columns(fx.n, 16, 2)
    e = _err(obf.apply(F0, Om), H.apply(_t(Om)).cpu().numpy())
    say("exact err", e)
    assert e < 5e-6


@pytest.mark.parametrize("m,n,leaf", [(300, 257, 16), (100, 1000, 40), (24, 24, 32), (50, 20, 8)])
def test_ragged_and_degenerate_shapes(bf, m, n, leaf):
    g = wl.segment_pair(n, ppw=10.0, m=m)
    op_o = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    say("ragged", m, n, leaf)
    op = bf.segkernel(g.targets, g.sources, g.k)
    H = bf.construct(op, 1e-6, leaf, seed=4)
    Fo = obf.construct(op_o, 1e-6, leaf, seed=4)
    Om = wl.test_columns(n, 16, 9)
    AOm = op_o.matvec(Om)
    e_gpu = _err(AOm, H.apply(_t(Om)).cpu().numpy())
    e_or = _err(AOm, obf.apply(Fo, Om))
    say("ragged errors", e_or, e_gpu)
    assert e_gpu <= 2 * e_or


def test_rank_cap_error(bf):
    g = wl.segment_pair(256, ppw=8.0)
    op = bf.segkernel(g.targets, g.sources, g.k)
    say("rank cap")
    with pytest.raises(bf.BFError) as ei:
        bf.construct(op, 1e-6, 64, seed=1, max_rank=4)
    assert ei.value.code == -4


@pytest.mark.parametrize("m,n,leaf", [(2048, 2048, 16), (1500, 1100, 20)])
def test_sample_groups(bf, m, n, leaf):
    """Sweep levels processed one sample at a time (workspace bound of one
    byte) give the factorization of the unbounded run: same ranks, same error
    to rounding, and the error of the oracle's construction."""
    g = wl.segment_pair(n, ppw=8.0, m=m)
    op = bf.segkernel(g.targets, g.sources, g.k)
    say("sample groups", m, n, leaf)
    A = bf.construct(op, 1e-6, leaf, seed=12)
    B = bf.construct(op, 1e-6, leaf, seed=12, work_bytes=1)
    ua, va = A.ranks()
    ub, vb = B.ranks()
    assert np.abs(ua.astype(int) - ub).max() <= 1 and np.abs(va.astype(int) - vb).max() <= 1
    assert (ua != ub).mean() < 0.01 and (va != vb).mean() < 0.01
    ref = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    Om = wl.test_columns(n, 16, 5)
    AOm = ref.matvec(Om)
    ea = _err(AOm, A.apply(_t(Om)).cpu().numpy())
    eb = _err(AOm, B.apply(_t(Om)).cpu().numpy())
    Fo = obf.construct(ref, 1e-6, leaf, seed=12)
    eo = _err(AOm, obf.apply(Fo, Om))
    say("groups errors", ea, eb, "oracle", eo)
    assert abs(ea - eb) <= 0.05 * ea + 1e-8
    assert eb <= 2 * eo
    with pytest.raises(bf.BFError):
        bf.construct(op, 1e-6, leaf, seed=12, work_bytes=-1)


def test_exact_butterfly_at_scale(bf):
    """Sec. 6.1 at L = 12 (n = 32768, leaf 8, r = 8, random factors drawn level
    by level): recovered through the butterfly black box with every rank 8 and
    complex64-level error; factor storage is that of the source (O(n log n))."""
    L, r, leaf = 12, 8, 8
    n = leaf << L
    kU, kV, data = wl.exact_butterfly_canonical(L, r, seed=5)
    say("exact at scale", L)
    src = bf.import_factors(n, n, leaf, kU, kV, data)
    H = bf.construct(bf.from_factors(src), 1e-5, leaf, seed=6)
    gU, gV = H.ranks()
    assert set(np.unique(gU)) == {r} and set(np.unique(gV)) == {r}
    assert H.stats().factor_entries == src.stats().factor_entries
    Om = _t(wl.test_columns(n, 16, 3))
    ref = src.apply(Om)
    e = float((H.apply(Om) - ref).norm() / ref.norm())
    say("exact at scale err", e)
    assert e < 2e-6
    H.close()
    src.close()


@pytest.mark.parametrize("center,lm", [("column", 0), (1, 1), ("row", 5)])
def test_centre_level_variants(bf, center, lm):
    """Column-wise (Sec. 3.3.1), an intermediate level, and row-wise (Sec. 3.3.2)
    factorizations of C1 against the oracle's, with the black-box column
    counts of the two sides equal."""
    g = wl.segment_pair(1024, ppw=8.0)
    op_o = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    Fo = obf.construct(op_o, 1e-6, 32, seed=1, lm=lm)
    say("centre level", center, lm)
    op = bf.segkernel(g.targets, g.sources, g.k)
    H = bf.construct(op, 1e-6, 32, seed=1, center=center)
    assert (H.L, H.lm) == (5, lm)
    Om = wl.test_columns(1024, 16, 1001)
    AOm = op_o.matvec(Om)
    e_or = _err(AOm, obf.apply(Fo, Om))
    e_gpu = _err(AOm, H.apply(_t(Om)).cpu().numpy())
    say("variant errors oracle", e_or, "gpu", e_gpu)
    assert e_gpu <= 2 * e_or
    kU, kV = H.ranks()
    ko_U, ko_V, _ = oracle_to_canonical(Fo)
    assert np.abs(kU.astype(int) - ko_U).max() <= 2
    assert np.abs(kV.astype(int) - ko_V).max() <= 2
    Fg = canonical_to_oracle(H.m, H.n, H.L, kU, kV, H.export(), lm=lm)
    A = op_o.dense()
    assert np.linalg.norm(A - obf.dense(Fg)) / np.linalg.norm(A) <= 2 * e_or
    # adjoint of the variant's own factors
    X = wl.test_columns(1024, 5, 3)
    ref = obf.apply_adjoint(Fg, X)
    np.testing.assert_allclose(H.apply(_t(X), trans=True).cpu().numpy(), ref,
                               atol=2e-6 * np.abs(ref).max())
    # black-box columns: equal up to the widths' dependence on ranks (+-2) and
    # the merged leaf passes the loop did not reach (at most 10 + 18 + 34
    # columns after the first pass of r0 = 4, p = 2)
    info = H.stats()
    for got, ref in ((info.matvec_cols, Fo.stats["matvec"]), (info.rmatvec_cols, Fo.stats["rmatvec"])):
        assert 0.95 * ref <= got <= 1.05 * ref + 62


@pytest.mark.parametrize("center", ["column", "row"])
def test_centre_level_exact_recovery(bf, center):
    """An exact rank-4 butterfly (L = 5) has rank 4 at every level, so the
    column- and row-wise constructions recover it like the hybrid."""
    fx = wl.exact_butterfly_factors(5, 4, seed=54)
    F0 = obf.from_exact(fx)
    kU, kV, data = oracle_to_canonical(F0)
    src = bf.import_factors(fx.n, fx.n, 8, kU, kV, data)
    op = bf.from_factors(src)
    H = bf.construct(op, 1e-5, 8, seed=5, center=center)
    gU, gV = H.ranks()
    assert set(np.unique(gU)) == {4} and set(np.unique(gV)) == {4}
    Om = wl.test_columns(fx.n, 16, 2)
    e = _err(obf.apply(F0, Om), H.apply(_t(Om)).cpu().numpy())
    say("exact variant", center, e)
    assert e < 5e-6
    with pytest.raises(bf.BFError):
        bf.construct(op, 1e-5, 8, seed=5, center=6)


def test_reused_device_blocks_do_not_change_results(bf):
    """Device blocks and pinned staging are recycled across requests (their
    old contents are never cleared): a construction repeated after others of
    different sizes, precisions and operators, whose factors were freed in
    between, gives bitwise the same factors, applies and ranks."""
    g = wl.segment_pair(3000, ppw=8.0, m=2500)
    op = bf.segkernel(g.targets, g.sources, g.k)
    say("block reuse: reference")
    first = bf.construct(op, 1e-6, 48, seed=11)
    ref = first.export()
    X = _t(np.random.default_rng(5).standard_normal((3000, 7)) + 0j)
    Yref = first.apply(X).cpu().numpy()
    first.close()
    held = []
    for n, tol, prec in ((6000, 1e-4, "bf16x3"), (1024, 1e-7, "fp64"), (4096, 1e-6, "bf16x3")):
        gg = wl.segment_pair(n, ppw=6.0)
        o = bf.segkernel(gg.targets, gg.sources, gg.k)
        o.set_precision(prec)
        H = bf.construct(o, tol, 32, seed=n)
        H.apply(_t(np.ones((n, 3), complex)))
        held.append(H)
    for H in held[:2]:
        H.close()
    say("block reuse: repeat")
    again = bf.construct(op, 1e-6, 48, seed=11)
    assert np.array_equal(again.export(), ref)
    assert np.array_equal(again.apply(X).cpu().numpy(), Yref)
    again.close()
    held[2].close()
    # giving the kept memory back returns it to the device; later requests
    # allocate afresh and still agree bitwise
    import torch
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    bf.release_cached_memory()
    free1 = torch.cuda.mem_get_info()[0]
    say("release cached memory: free", free0 >> 20, "->", free1 >> 20, "MiB")
    assert free1 > free0
    once_more = bf.construct(op, 1e-6, 48, seed=11)
    assert np.array_equal(once_more.export(), ref)
    once_more.close()


@pytest.mark.parametrize("geom,n,tol,p", [("segments", 16384, 1e-6, 2), ("segments", 8192, 1e-4, 2),
                                          ("hemispheres", 4096, 1e-2, 4)])
def test_merged_sweep_levels(bf, geom, n, tol, p):
    """Consecutive sweep levels sharing one black-box call (the default for
    the built-in operators that evaluate their entries on the fly) against one
    call per level: the same ranks (within 1 where a level's guessed width
    proved too small and the next level made its own call), an apply error on
    16 Gaussian columns within 5% of the level-by-level construction's, fewer
    black-box launches, and bitwise repeatable."""
    import torch
    if geom == "segments":
        g = wl.segment_pair(n, ppw=8.0)
        op = bf.segkernel(g.targets, g.sources, g.k)
        ref64 = bf.segkernel(g.targets, g.sources, g.k).set_precision("fp64")
    else:
        g = wl.hemisphere_pair(n, seed=1)
        op = bf.helmholtz3d(g.targets, g.sources, g.k)
        ref64 = bf.helmholtz3d(g.targets, g.sources, g.k).set_precision("fp64")
    say("merged sweep levels", geom, n, tol)
    runs = {}
    bf.set_autotune(False)    # launch counts without the tuner's timing runs
    try:
        for merge in (True, False):
            bf.profile_start()
            H = bf.construct(op, tol, 64, p=p, seed=9, merge_sweeps=merge)
            torch.cuda.synchronize()
            calls = bf.profile_stop()["matfree"]["launches"]
            runs[merge] = (H, calls)
    finally:
        bf.set_autotune(True)
    (Hm, cm), (Hs, cs) = runs[True], runs[False]
    im, is_ = Hm.stats(), Hs.stats()
    say("black-box launches merged", cm, "level by level", cs, "merged levels", im.merged_levels,
        "misses", im.merge_misses)
    assert im.merged_levels > 0 and is_.merged_levels == 0 and is_.merge_misses == 0
    assert cm < cs
    for a, b in zip(Hm.ranks(), Hs.ranks()):
        if im.merge_misses == 0:
            assert np.array_equal(a, b)
        else:
            assert np.abs(a.astype(int) - b.astype(int)).max() <= 1
    # reference products from the FP64 black box (checked against the oracle
    # by test_gpu_kernels and test_gpu_3d)
    Om = wl.test_columns(n, 16, 77)
    ref = ref64.matvec(_t(Om)).cpu().numpy()
    em = _err(ref, Hm.apply(_t(Om)).cpu().numpy())
    es = _err(ref, Hs.apply(_t(Om)).cpu().numpy())
    say("errors merged", em, "level by level", es)
    assert em <= 1.05 * es
    # bitwise repeatable (tuned launch shapes give the same bits)
    again = bf.construct(op, tol, 64, p=p, seed=9)
    assert np.array_equal(again.export(), Hm.export())
    again.close()
    Hm.close()
    Hs.close()
    ref64.close()
    op.close()


def test_merged_leaf_passes_same_result(bf):
    """Leaf-loop passes merged into one black-box call give bitwise the same
    factors as one call per pass; only the call count differs."""
    g = wl.segment_pair(2048, ppw=8.0)
    op = bf.segkernel(g.targets, g.sources, g.k)
    calls = {}
    for merge in (True, False):
        H = bf.construct(op, 1e-6, 64, seed=7, merge_leaf=merge)
        calls[merge] = (H.export(), H.stats())
    (a, ia), (b, ib) = calls[True], calls[False]
    say("merged leaf passes", ia.v_iters, ia.u_iters, ia.matvec_cols, ib.matvec_cols)
    assert np.array_equal(a, b)
    assert (ia.v_iters, ia.u_iters) == (ib.v_iters, ib.u_iters) and ia.v_iters >= 3
    assert ia.matvec_cols >= ib.matvec_cols and ia.rmatvec_cols >= ib.rmatvec_cols


def test_unknown_option_flags_rejected(bf):
    """bf_opts.flags bits the library does not know are an argument error, not
    silently ignored."""
    import ctypes as C
    g = wl.segment_pair(256, ppw=8.0)
    op = bf.segkernel(g.targets, g.sources, g.k)
    o = bf.bf_opts(2, 4, 0, 16, 0, 0)
    h = C.c_void_p()
    rc = bf.lib().bf_construct(op._op.matvec, op._op.rmatvec, op._op.user, op.m, op.n, 1e-6, 32,
                               C.byref(o), None, None, C.byref(h))
    assert rc == -1 and not h.value


def _two_sides_case(bf, kind):
    if kind == "segment":
        g = wl.segment_pair(8192, ppw=8.0)
        return bf.segkernel(g.targets, g.sources, g.k), 1e-6, 64, []
    if kind == "fio":
        return bf.fio(4096), 1e-6, 16, []
    if kind == "ragged":
        g = wl.segment_pair(3000, ppw=6.0, m=2100)
        return bf.segkernel(g.targets, g.sources, g.k), 1e-5, 40, []
    # recompression: the product of two butterflies as the black box
    g01, g12 = wl.segment_triple(2048, ppw=8.0)
    B1 = bf.construct(bf.segkernel(g01.targets, g01.sources, g01.k), 1e-6, 32, seed=21)
    B2 = bf.construct(bf.segkernel(g12.targets, g12.sources, g12.k), 1e-6, 32, seed=22)
    return bf.compose(bf.from_factors(B1), bf.from_factors(B2)), 1e-6, 32, [B1, B2]


@pytest.mark.parametrize("kind", ["segment", "fio", "ragged", "compose"])
@pytest.mark.parametrize("allocator", ["torch", None])
def test_two_sides_give_the_same_factors(bf, kind, allocator):
    """The row side on its own stream and host thread beside the column side
    (the default for built-in operators) enqueues the same work as the
    one-stream run: bitwise the same factors, ranks and column counts."""
    op, tol, leaf, keep = _two_sides_case(bf, kind)
    say("two sides", kind, allocator)
    A = bf.construct(op, tol, leaf, seed=5, allocator=allocator)
    B = bf.construct(op, tol, leaf, seed=5, allocator=allocator, two_sides=False)
    a, b = A.stats(), B.stats()
    assert a.L >= 2
    for f in ("max_rank", "v_iters", "u_iters", "matvec_cols", "rmatvec_cols", "merged_levels",
              "merge_misses", "factor_entries"):
        assert getattr(a, f) == getattr(b, f), f
    assert np.array_equal(A.export(), B.export())
    X = _t(wl.test_columns(op.n, 3, 4))
    assert bool((A.apply(X) == B.apply(X)).all())
    for H in (A, B, *keep):
        H.close()


def test_rank_cap_with_two_sides(bf):
    """A rank-cap failure with the sides on two threads: the row side stops in
    its leaf loop (leaves of 64 sources need r above 8), the column side
    (leaves of 4 targets) later at an R level; the call raises BF_ERANK as in
    the one-stream run whichever thread fails first, and the next
    constructions are unaffected."""
    g = wl.segment_pair(2048, ppw=8.0, m=128)
    op = bf.segkernel(g.targets, g.sources, g.k)
    say("row-side error")
    for two in (True, False):
        with pytest.raises(bf.BFError) as ei:
            bf.construct(op, 1e-6, 64, seed=1, max_rank=8, two_sides=two)
        assert ei.value.code == -4
    H = bf.construct(op, 1e-6, 64, seed=1)
    H2 = bf.construct(op, 1e-6, 64, seed=1, two_sides=False)
    assert np.array_equal(H.export(), H2.export())
    H.close()
    H2.close()
