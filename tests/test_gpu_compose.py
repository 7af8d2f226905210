"""Recompression of a product of two butterflies (category (ii) of Sec. 1):
the GPU builds B1 ~ A(X0, X1) and B2 ~ A(X1, X2), then recompresses the
composition B1 B2 with Alg. 2 using the butterfly applies as the black box."""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import butterfly as obf
from oracle import operators as ops

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


@pytest.mark.parametrize("n,leaf", [(1024, 32), (2000, 40)])
def test_recompress_product(bf, n, leaf):
    g01, g12 = wl.segment_triple(n, ppw=8.0)
    tol = 1e-6
    say("compose", n, leaf)
    o1 = bf.segkernel(g01.targets, g01.sources, g01.k)
    o2 = bf.segkernel(g12.targets, g12.sources, g12.k)
    B1 = bf.construct(o1, tol, leaf, seed=21)
    B2 = bf.construct(o2, tol, leaf, seed=22)
    prod = bf.compose(bf.from_factors(B1), bf.from_factors(B2))
    F = bf.construct(prod, tol, leaf, seed=23)
    # oracle: the same pipeline in FP64
    r1 = ops.SegmentKernelOp(g01.targets, g01.sources, g01.k)
    r2 = ops.SegmentKernelOp(g12.targets, g12.sources, g12.k)
    P1 = obf.construct(r1, tol, leaf, seed=21)
    P2 = obf.construct(r2, tol, leaf, seed=22)
    Fo = obf.construct(ops.ComposeOp(obf.FactorsOp(P1), obf.FactorsOp(P2)), tol, leaf, seed=23)
    Om = wl.test_columns(n, 16, 1001)
    exact = r1.matvec(r2.matvec(Om))          # the FP64 composition of the kernels
    e_gpu = np.linalg.norm(F.apply(_t(Om)).cpu().numpy() - exact) / np.linalg.norm(exact)
    e_or = np.linalg.norm(obf.apply(Fo, Om) - exact) / np.linalg.norm(exact)
    say("compose errors oracle", e_or, "gpu", e_gpu, "ranks", F.stats().max_rank)
    assert e_gpu <= 2 * e_or
    # the product's adjoint through the recompressed factors
    Z = wl.test_columns(n, 3, 7)
    exactH = r2.rmatvec(r1.rmatvec(Z))
    e_h = np.linalg.norm(F.apply(_t(Z), trans=True).cpu().numpy() - exactH) / np.linalg.norm(exactH)
    assert e_h <= 2 * e_or


@pytest.mark.parametrize("n,leaf", [(2048, 16), (3000, 24)])
def test_fio_construction_and_recompression(bf, n, leaf):
    """1D FIO (low-dimensional Fourier operator, Sec. 4.4.1) built matrix-free
    with both black-box precisions (split-BF16 matrix cores and FP64 matrix
    cores), then recompressed with its own butterfly as the black box; each
    against the oracle's construction of the same operator (FP64 entries)."""
    if n % 2:
        n += 1
    tol = 1e-6
    x, xi = wl.fio_params(n)
    ref = ops.FIOOp(x, xi)
    say("fio", n, leaf)
    Fo = obf.construct(ref, tol, leaf, seed=31)
    Om = wl.test_columns(n, 16, 1003)
    AOm = ref.matvec(Om)
    e_or = np.linalg.norm(obf.apply(Fo, Om) - AOm) / np.linalg.norm(AOm)
    op = bf.fio(n)
    errs = {}
    for prec in ("bf16x3", "fp64"):
        op.set_precision(prec)
        F = bf.construct(op, tol, leaf, seed=31)
        errs[prec] = np.linalg.norm(F.apply(_t(Om)).cpu().numpy() - AOm) / np.linalg.norm(AOm)
        if prec == "bf16x3":
            Fk = F
        else:
            F.close()
    say("fio errors oracle", e_or, "gpu", errs)
    for e in errs.values():
        assert e <= 2 * e_or
    # the two black-box precisions agree to the tolerance's order
    assert abs(errs["bf16x3"] - errs["fp64"]) <= 0.5 * e_or
    G = bf.construct(bf.from_factors(Fk), tol, leaf, seed=32)
    e_re = np.linalg.norm(G.apply(_t(Om)).cpu().numpy() - AOm) / np.linalg.norm(AOm)
    say("fio recompressed", e_re)
    # recompressing a tol-accurate butterfly at tol: errors add at most
    assert e_re <= errs["bf16x3"] + 2 * e_or
    G.close()
    Fk.close()


@pytest.mark.parametrize("trans", [False, True])
def test_structured_samples_through_factors(bf, trans):
    """A butterfly as the black box of structured samples (Sec. 4.1): the
    product for row segments that are nodes of one tree level (all of them, or
    a run of consecutive ones, as a level split into sample groups gives) runs
    the stages that keep the segments apart once on the sample itself, and for
    whole levels the next merging stages on per-node windows of the segments
    below each node.  It must equal the definition of the callback: the
    factors applied to the block-diagonal expansion of the sample -- bitwise
    at 5 or more columns (the same matrix-core arithmetic per column), to
    complex64 rounding at fewer (vector-ALU stages on the sample, matrix-core
    ones on the expansion).  Segments that are not tree nodes take the
    expansion path."""
    import torch
    n, leaf = 4096, 32
    g = wl.segment_pair(n, ppw=8.0, m=3000)
    F = bf.construct(bf.segkernel(g.targets, g.sources, g.k), 1e-6, leaf, seed=41)
    L = F.L
    op = bf.from_factors(F)
    rows_in = F.m if trans else F.n
    lo = lambda l, i: (i * rows_in) >> l
    cases = [[lo(1, i) for i in range(3)], [lo(3, i) for i in range(9)],
             [lo(5, i) for i in range(33)], [lo(L, i) for i in range((1 << L) + 1)],
             [lo(5, i) for i in range(3, 13)], [lo(L, i) for i in range(40, 57)],
             [0, 100, 1000, rows_in]]   # not tree nodes
    rng = np.random.default_rng(8)
    for seg in cases:
        for s in (3, 6, 20):
            X = (rng.standard_normal((rows_in, s)) + 1j * rng.standard_normal((rows_in, s))).astype(np.complex64)
            Xd = torch.from_numpy(X).cuda()
            got = (op.rmatvec if trans else op.matvec)(Xd, seg=seg)
            E = torch.zeros((rows_in, (len(seg) - 1) * s), dtype=torch.complex64, device="cuda")
            for q in range(len(seg) - 1):
                E[seg[q]:seg[q + 1], q * s:(q + 1) * s] = Xd[seg[q]:seg[q + 1]]
            ref = F.apply(E, trans=trans)
            say("structured", trans, len(seg) - 1, s)
            if s >= 5:
                assert bool((got == ref).all()), (seg[:3], s)
            else:
                err = float((got - ref).norm() / ref.norm())
                assert err <= 1e-6, (seg[:3], s, err)
    F.close()
