"""GPU parity of the batched building blocks against the oracle (through the
C ABI).  Each test prints the case it runs before touching the device."""
import math
import os
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import butterfly as obf
from oracle import cpqr as ocpqr
from oracle import operators as ops
from oracle import philox
from tests.bfconv import bf16_exact, canonical_to_oracle, oracle_to_canonical

pytestmark = pytest.mark.gpu


def _same_bits(a, b):
    """Bitwise equality of two complex64 device tensors (any strides)."""
    x = np.ascontiguousarray(a.cpu().numpy()).view(np.uint32)
    y = np.ascontiguousarray(b.cpu().numpy()).view(np.uint32)
    return x.shape == y.shape and np.array_equal(x, y)


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


def _cg(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2)


def _t(x):
    import torch
    return torch.from_numpy(np.asarray(x, np.complex64)).cuda()


# ---------------------------------------------------------------- RNG -------
@pytest.mark.parametrize("seed,phase,level,node,row0,rows,cols",
                         [(1, 1, 0, 0, 0, 1000, 6), (7, 4, 3, 5, 12345, 300, 40),
                          (2**63 + 5, 3, 9, 511, 65000, 536, 3)])
def test_gauss_matches_oracle(bf, seed, phase, level, node, row0, rows, cols):
    tg = philox.tag(phase, level, node)
    say("gauss", seed, tg, row0, rows, cols)
    g = bf.gauss(seed, tg, row0, rows, cols).cpu().numpy()
    ref = philox.gaussian_block(seed, tg, row0, rows, cols)
    # same Philox bits; FP64 log / sincospi on the device vs the host libm
    np.testing.assert_allclose(g, ref, rtol=0, atol=4e-15 * np.abs(ref).max())


# ---------------------------------------------------------------- CPQR ------
def _cpqr_cases():
    rng = np.random.default_rng(11)
    cases = []
    for (M, N) in [(24, 26), (36, 40), (64, 34), (72, 74), (5, 9), (9, 5), (1, 1), (130, 70),
                   (200, 200), (64, 6)]:
        cases.append(_cg(rng, M, N) * rng.uniform(0.3, 3.0, N)[None, :])
    cases.append(_cg(rng, 40, 6) @ _cg(rng, 6, 30))              # exact rank 6
    U = np.linalg.qr(_cg(rng, 50, 30))[0]
    cases.append((U * 0.5 ** np.arange(30)) @ _cg(rng, 30, 32))  # geometric spectrum
    cases.append(np.zeros((10, 7), complex))                     # zero block
    cases.append(np.zeros((0, 5), complex))                      # empty
    return cases


@pytest.mark.parametrize("tol", [1e-6, 1e-3])
def test_cpqr_matches_oracle(bf, tol):
    blocks = _cpqr_cases()
    say("cpqr batch", [b.shape for b in blocks], tol)
    Qs, ranks = bf.cpqr_batched(blocks, tol)
    for b, Q, k in zip(blocks, Qs, ranks):
        Qo, ko = ocpqr.range_basis(b, tol)
        assert k == ko, (b.shape, k, ko)
        if k:
            np.testing.assert_allclose(Q, Qo, atol=1e-10)
            np.testing.assert_allclose(Q.conj().T @ Q, np.eye(k), atol=1e-12)


def test_cpqr_large_blocks_in_chunks(bf):
    """Blocks far beyond the LDS (ranks of the 3D regime of Sec. 6.3): 600 x 520
    with a geometric spectrum, 200 copies (1.2 GB of scratch: two launches),
    plus single 300 x 560 and 700 x 260 blocks."""
    rng = np.random.default_rng(11)
    U = np.linalg.qr(_cg(rng, 600, 300))[0]
    big = (U * 0.93 ** np.arange(300)) @ _cg(rng, 300, 520)
    odd = [_cg(rng, 300, 560) * rng.uniform(0.3, 3.0, 560)[None, :],
           (np.linalg.qr(_cg(rng, 700, 200))[0] * 0.9 ** np.arange(200)) @ _cg(rng, 200, 260)]
    tol = 1e-6
    Qo, ko = ocpqr.range_basis(big, tol)
    say("cpqr large", big.shape, "x200, oracle rank", ko)
    Qs, ranks = bf.cpqr_batched([big] * 200 + odd, tol)
    for t in range(200):
        assert ranks[t] == ko
        np.testing.assert_allclose(Qs[t], Qo, atol=1e-10)
    for b, Q, k in zip(odd, Qs[200:], ranks[200:]):
        Qb, kb = ocpqr.range_basis(b, tol)
        assert k == kb, (b.shape, k, kb)
        np.testing.assert_allclose(Q, Qb, atol=1e-10)
        np.testing.assert_allclose(Q.conj().T @ Q, np.eye(k), atol=1e-12)


# ---------------------------------------------------------------- LS --------
def test_lsq_matches_oracle(bf):
    rng = np.random.default_rng(5)
    shapes = [(13, 13, 20), (20, 18, 40), (1, 1, 3), (35, 33, 72), (7, 12, 12),
              (150, 140, 300), (260, 250, 256)]   # the last two: device-scratch path
    Cs = [_cg(rng, ku, s) for ku, kv, s in shapes]
    Xs = [_cg(rng, kv, s) for ku, kv, s in shapes]
    say("lsq", shapes)
    Bs = bf.lsq_batched(Cs, Xs)
    for C, X, B in zip(Cs, Xs, Bs):
        ref = obf._lstsq_right(C, X)
        np.testing.assert_allclose(B, ref, atol=1e-10 * max(1, np.abs(ref).max()))


# ------------------------------------------------------- black boxes -------
def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("m,n,ppw", [(1024, 1024, 8.0), (700, 1500, 5.0)])
def test_segkernel_products(bf, m, n, ppw):
    g = wl.segment_pair(n, ppw=ppw, m=m)
    say("segkernel", m, n, ppw)
    op = bf.segkernel(g.targets, g.sources, g.k)
    ref = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    rng = np.random.default_rng(1)
    X = _cg(rng, n, 7)
    Y = op.matvec(_t(X)).cpu().numpy()
    assert _rel(Y, ref.matvec(X)) < 2e-6
    Xt = _cg(rng, m, 5)
    Yt = op.rmatvec(_t(Xt)).cpu().numpy()
    assert _rel(Yt, ref.rmatvec(Xt)) < 2e-6
    # structured samples: ragged segments, per-segment products
    seg = np.array([0, 3, 400, 401, n], np.int64)
    Ys = op.matvec(_t(X), seg=seg).cpu().numpy()
    for q in range(4):
        Xq = np.zeros_like(X)
        Xq[seg[q]:seg[q + 1]] = X[seg[q]:seg[q + 1]]
        exp = ref.matvec(Xq)
        got = Ys[:, q * 7:(q + 1) * 7]
        assert np.linalg.norm(got - exp) <= 2e-6 * max(np.linalg.norm(exp), 1e-30) + 1e-12


def test_segkernel_wide_and_split(bf):
    """65 columns (two column chunks) and a long inner range (split-K path)."""
    n = 20000
    g = wl.segment_pair(n, ppw=8.0, m=300)
    say("segkernel wide", n)
    op = bf.segkernel(g.targets, g.sources, g.k)
    ref = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    X = _cg(np.random.default_rng(2), n, 65)
    Y = op.matvec(_t(X)).cpu().numpy()
    assert _rel(Y, ref.matvec(X)) < 3e-6


def test_autotuned_tile_widths_do_not_change_products(bf):
    """The autotuner times candidate column chunkings on the first product of a
    shape class and reuses the fastest; every candidate gives bitwise the same
    product, so tuned, cached and untuned products agree exactly, and so do
    constructions."""
    n = 6000
    g = wl.segment_pair(n, ppw=8.0, m=3000)
    op = bf.segkernel(g.targets, g.sources, g.k)
    say("autotune")
    X = _cg(np.random.default_rng(9), n, 70)
    Xb = bf16_exact(X)
    gg = wl.segment_pair(2048, ppw=8.0)
    opc = bf.segkernel(gg.targets, gg.sources, gg.k)
    bf.set_autotune(False)
    try:
        ref = op.matvec(_t(Xb)).cpu().numpy()
        ref_g = op.matvec(_t(X)).cpu().numpy()
        fa = bf.construct(opc, 1e-6, 32, seed=21).export()
        bf.autotune_clear()
        bf.set_autotune(True)
        n0 = bf.autotune_entries()
        tuned = op.matvec(_t(Xb)).cpu().numpy()
        n1 = bf.autotune_entries()
        cached = op.matvec(_t(Xb)).cpu().numpy()
        tuned_g = op.matvec(_t(X)).cpu().numpy()
        fb = bf.construct(opc, 1e-6, 32, seed=21).export()
        fc = bf.construct(opc, 1e-6, 32, seed=21).export()
    finally:
        bf.set_autotune(True)
    assert n1 == n0 + 1
    assert np.array_equal(tuned, ref) and np.array_equal(cached, ref)
    assert np.array_equal(tuned_g, ref_g)
    assert np.array_equal(fa, fb) and np.array_equal(fa, fc)


# candidates of each tuned family (include/bf.h, bf_set_autotune)
TUNE_CANDIDATES = {"matfree_width": [48, 64, 80], "chain_rows": [8, 16, 20, 24, 32, 40, 48, 64],
                   "cpqr_threads": [256, 512], "apply_fused": [1, 0],
                   "apply_rows": [1, 0, 2, 4, 9, 10, 17, 49, 25, 57],
                   "apply_mfma": [1, 2, 0]}


def _tune_rows(path):
    rows = []
    for line in open(path):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows.append((f[0], [int(x) for x in f[1:-1]], int(f[-1])))
    return rows


def _valid(fam, fields, c):
    if fam == "chain_rows":      # tile heights at least the launch's largest block
        m = fields[1]
        return c >= m if m <= 64 else c in (32, 64)
    if fam == "apply_mfma":      # column tiles per wave, at most the apply's tiles
        return c <= max(1, fields[0] // 16)
    if fam == "apply_rows":      # record kernel, or row groups (+ 8: inputs in LDS,
        ncl, it = fields[0], fields[1]   # + 16 / 48: 2 / 4 waves per block)
        ok = ((4, 2, 1, 0) if it == 1 else (1, 2, 0)) if ncl <= 2 else \
             ((2, 1, 9, 10, 0) if it == 1 else (1, 9, 10, 0))
        if fields[2] < 4096:
            ok += (17, 49) if ncl <= 2 else (17, 49, 25, 57)
        return c in ok
    return True


def test_every_autotuner_candidate_gives_the_same_bits(bf, tmp_path):
    """Every family the tuner covers -- black-box column tile, chain tile
    height, CPQR workgroup, fused or staged few-column apply, block or record
    few-column kernel, wave or workgroup matrix-core apply -- and every one of
    its candidates gives the bits of the untuned rule: the table is saved,
    rewritten with each candidate in turn for every class, loaded, and the
    construction and applies repeated against the untuned reference."""
    import torch
    g = wl.segment_pair(4096, ppw=8.0)
    op = bf.segkernel(g.targets, g.sources, g.k)
    # applies of an exact rank-8 butterfly with L = 10 (1024 blocks a stage,
    # enough groups for fused launches)
    kU, kV, data = wl.exact_butterfly_canonical(10, 8, seed=5, leaf=8)
    E = bf.import_factors(8192, 8192, 8, kU, kV, data)
    X = _t(_cg(np.random.default_rng(3), 8192, 3))
    # 20 columns through the matrix-core stages of the constructed factors
    # (blocks of 17 to 64 rows)
    X20 = _t(_cg(np.random.default_rng(4), 4096, 20))

    def run():
        F = bf.construct(op, 1e-6, 64, seed=31)
        out = [F.export()]
        for trans in (False, True):
            out.append(np.ascontiguousarray(F.apply(X20, trans=trans).cpu().numpy()))
        F.close()
        for c in (1, 2, 3):
            for trans in (False, True):
                out.append(np.ascontiguousarray(E.apply(X[:, :c], trans=trans).cpu().numpy()))
        torch.cuda.synchronize()
        return out

    bf.set_autotune(False)
    try:
        ref = run()
        bf.autotune_clear()
        bf.set_autotune(True)
        tuned = run()
        path = str(tmp_path / "tune.tsv")
        bf.autotune_save(path)
        rows = _tune_rows(path)
        say("tuned classes", len(rows), sorted({r[0] for r in rows}))
        assert {r[0] for r in rows} == set(TUNE_CANDIDATES)
        for a, b in zip(ref, tuned):
            assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
        for trial in range(max(len(v) for v in TUNE_CANDIDATES.values())):
            forced = str(tmp_path / f"forced{trial}.tsv")
            with open(forced, "w") as f:
                for fam, fields, _ in rows:
                    ok = [c for c in TUNE_CANDIDATES[fam] if _valid(fam, fields, c)]
                    f.write(" ".join([fam] + [str(x) for x in fields] +
                                     [str(ok[trial % len(ok)])]) + "\n")
            bf.autotune_clear()
            bf.autotune_load(forced)
            say("forced candidates, trial", trial)
            got = run()
            for a, b in zip(ref, got):
                assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), trial
        # a saved table restores every class
        bf.autotune_clear()
        bf.autotune_load(path)
        assert bf.autotune_entries() == len(rows)
    finally:
        bf.set_autotune(True)
        E.close()


@pytest.mark.parametrize("L,r,leaf", [(10, 8, 8), (9, 20, 24), (8, 40, 40)])
def test_block_and_record_kernels_give_the_same_bits(bf, tmp_path, L, r, leaf):
    """Stage-by-stage applies of 1 to 4 columns: the block kernel (rows of up
    to 32, 64 or 96 terms -- here 16, 40 and 80 -- with 1, 2 or 4 groups of 8
    rows loaded together, inputs in registers or, for 3 and 4 columns, in
    LDS, one, two or four waves per block) and the row-record kernel, each
    variant forced through the autotuner's table, give the same bits, forward
    and adjoint; all are within 2e-6 of the oracle's FP64 apply in every
    column."""
    import torch
    n = leaf << L
    kU, kV, data = wl.exact_butterfly_canonical(L, r, seed=L + r, leaf=leaf)
    F = canonical_to_oracle(n, n, L, kU, kV, data)
    H = bf.import_factors(n, n, leaf, kU, kV, data)
    H.set_fusion(False)
    say("block vs record kernel", L, r, leaf)
    rng = np.random.default_rng(L)
    cases = [(s, _cg(rng, n, s)) for s in (1, 2, 3, 4)]
    path = str(tmp_path / "tune.tsv")
    try:
        bf.set_autotune(True)
        bf.autotune_clear()
        got = {}
        rows = None
        for choice in (None, 0, 1, 2, 4, 9, 10, 17, 49, 25, 57):
            if choice is not None:
                if rows is None:
                    rows = _tune_rows(path)
                    assert any(fam == "apply_rows" for fam, _, _ in rows)
                with open(path, "w") as f:
                    for fam, fields, c in rows:
                        if fam == "apply_rows" and _valid(fam, fields, choice):
                            c = choice
                        f.write(" ".join([fam] + [str(x) for x in fields] + [str(c)]) + "\n")
                bf.autotune_clear()
                bf.autotune_load(path)
            out = []
            for s, X in cases:
                for trans in (False, True):
                    out.append(np.ascontiguousarray(H.apply(_t(X), trans=trans).cpu().numpy()))
            torch.cuda.synchronize()
            if choice is None:
                bf.autotune_save(path)
            got[choice] = out
        for choice, out in got.items():
            for a, b in zip(got[None], out):
                assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), choice
        i = 0
        for s, X in cases:
            for ref in (obf.apply(F, X), obf.apply_adjoint(F, X)):
                y = got[1][i]
                i += 1
                for col in range(s):
                    assert np.linalg.norm(y[:, col] - ref[:, col]) <= 2e-6 * np.linalg.norm(ref[:, col])
    finally:
        bf.autotune_clear()
        saved = os.path.join(os.path.dirname(bf.__file__), "tune_gfx950.tsv")
        if os.path.exists(saved):   # the table saved beside the library
            bf.autotune_load(saved)
        bf.set_autotune(True)
        H.close()


@pytest.mark.parametrize("L,r,leaf", [(9, 20, 24), (8, 40, 40), (7, 30, 64)])
def test_mfma_wave_and_workgroup_kernels_give_the_same_bits(bf, tmp_path, L, r, leaf):
    """Stage-by-stage split-BF16 applies of 5 to 100 columns on blocks of 17
    to 64 rows: one workgroup per block and 64 columns, and one wave per
    block with 1, 2, ... or all of its 16-column tiles, each forced through
    the autotuner's table, give the same bits, forward and adjoint, and are
    within 2e-6 of the oracle's FP64 apply in every column."""
    import torch
    n = leaf << L
    kU, kV, data = wl.exact_butterfly_canonical(L, r, seed=L + r, leaf=leaf)
    F = canonical_to_oracle(n, n, L, kU, kV, data)
    H = bf.import_factors(n, n, leaf, kU, kV, data)
    say("mfma wave vs workgroup", L, r, leaf)
    rng = np.random.default_rng(L + 1)
    cases = [(s, _cg(rng, n, s)) for s in (5, 16, 20, 64, 100)]
    path = str(tmp_path / "tune.tsv")

    def run():
        out = []
        for s, X in cases:
            for trans in (False, True):
                out.append(np.ascontiguousarray(H.apply(_t(X), trans=trans).cpu().numpy()))
        torch.cuda.synchronize()
        return out

    try:
        bf.set_autotune(True)
        bf.autotune_clear()
        ref = run()
        bf.autotune_save(path)
        rows = _tune_rows(path)
        assert any(fam == "apply_mfma" for fam, _, _ in rows)
        for pick in ("workgroup", "one", "all"):
            with open(path, "w") as f:
                for fam, fields, c in rows:
                    if fam == "apply_mfma":
                        c = {"workgroup": 0, "one": 1, "all": max(1, fields[0] // 16)}[pick]
                    f.write(" ".join([fam] + [str(x) for x in fields] + [str(c)]) + "\n")
            bf.autotune_clear()
            bf.autotune_load(path)
            say("forced", pick)
            for a, b in zip(ref, run()):
                assert np.array_equal(a.view(np.uint64), b.view(np.uint64)), pick
        i = 0
        for s, X in cases:
            for want in (obf.apply(F, X), obf.apply_adjoint(F, X)):
                y = ref[i]
                i += 1
                for col in range(s):
                    assert np.linalg.norm(y[:, col] - want[:, col]) <= 2e-6 * np.linalg.norm(want[:, col])
    finally:
        bf.autotune_clear()
        saved = os.path.join(os.path.dirname(bf.__file__), "tune_gfx950.tsv")
        if os.path.exists(saved):
            bf.autotune_load(saved)
        bf.set_autotune(True)
        H.close()


@pytest.mark.parametrize("prec", ["bf16x3", "fp64"])
def test_helmholtz3d_products(bf, prec):
    """eq. 3dkernel between the two semi-spheres: plain and structured
    products, both directions, both arithmetic modes."""
    n = 3000
    g = wl.hemisphere_pair(n, seed=4, m=2500)
    say("helmholtz3d", prec)
    op = bf.helmholtz3d(g.targets, g.sources, g.k)
    op.set_precision(prec)
    ref = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    rng = np.random.default_rng(3)
    X = _cg(rng, n, 9)
    assert _rel(op.matvec(_t(X)).cpu().numpy(), ref.matvec(X)) < 3e-6
    Xt = _cg(rng, 2500, 40)
    assert _rel(op.rmatvec(_t(Xt)).cpu().numpy(), ref.rmatvec(Xt)) < 3e-6
    seg = np.array([0, 700, 701, 2500], np.int64)
    Ys = op.rmatvec(_t(Xt[:, :6]), seg=seg).cpu().numpy()
    for q in range(3):
        Xq = np.zeros_like(Xt[:, :6])
        Xq[seg[q]:seg[q + 1]] = Xt[seg[q]:seg[q + 1], :6]
        exp = ref.rmatvec(Xq)
        assert np.linalg.norm(Ys[:, 6 * q:6 * q + 6] - exp) <= 3e-6 * np.linalg.norm(exp)
    with pytest.raises(ValueError):
        bf.helmholtz3d(g.targets[:, :2], g.sources, g.k)


@pytest.mark.parametrize("ncols", [5, 23, 40, 64])
def test_segkernel_bf16_exact_inputs(bf, ncols):
    """Inputs exact in BF16 (the construction's random blocks) take the
    three-product path, general inputs the six-product path, a mix the general
    one; all agree with the FP64 products (ragged chunks, split-K, every tile
    width)."""
    m, n = 517, 9000
    g = wl.segment_pair(n, ppw=8.0, m=m)
    say("segkernel exact inputs", ncols)
    op = bf.segkernel(g.targets, g.sources, g.k)
    ref = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    X = _cg(np.random.default_rng(ncols), n, ncols)
    Xb = bf16_exact(X)
    Xm = Xb.copy()
    Xm[1234, ncols - 1] = X[1234, ncols - 1]
    for Z in (Xb, X, Xm):
        Y = op.matvec(_t(Z)).cpu().numpy()
        E = ref.matvec(Z)
        assert _rel(Y, E) < 5e-7
        # column by column: no column is computed on a stale or wrong path
        for c in range(ncols):
            assert np.linalg.norm(Y[:, c] - E[:, c]) <= 1e-6 * np.linalg.norm(E[:, c])
    Ys = op.rmatvec(_t(Xb[:m]), seg=np.array([0, 17, 300, m], np.int64)).cpu().numpy()
    for q, (lo, hi) in enumerate([(0, 17), (17, 300), (300, m)]):
        Zq = np.zeros((m, ncols), complex)
        Zq[lo:hi] = Xb[lo:hi]
        exp = ref.rmatvec(Zq)
        assert _rel(Ys[:, q * ncols:(q + 1) * ncols], exp) < 5e-7


def test_fio_products(bf):
    n = 2048
    x, xi = wl.fio_params(n)
    say("fio", n)
    op = bf.fio(n)
    ref = ops.FIOOp(x, xi)
    X = _cg(np.random.default_rng(3), n, 4)
    assert _rel(op.matvec(_t(X)).cpu().numpy(), ref.matvec(X)) < 2e-6
    assert _rel(op.rmatvec(_t(X)).cpu().numpy(), ref.rmatvec(X)) < 2e-6


def test_dense_products(bf):
    import torch
    rng = np.random.default_rng(4)
    A = _cg(rng, 300, 200)
    say("dense", A.shape)
    op = bf.dense(torch.from_numpy(A.astype(np.complex64)).cuda())
    X = _cg(rng, 200, 3)
    Z = _cg(rng, 300, 3)
    assert _rel(op.matvec(_t(X)).cpu().numpy(), A @ X) < 1e-6
    assert _rel(op.rmatvec(_t(Z)).cpu().numpy(), A.conj().T @ Z) < 1e-6


# ---------------------------------------------------------------- apply -----
@pytest.mark.parametrize("n,leaf", [(1024, 32), (600, 40), (20, 32)])
def test_apply_of_oracle_factors(bf, n, leaf):
    g = wl.segment_pair(n, ppw=8.0)
    op = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    F = obf.construct(op, 1e-6, leaf, seed=1)
    kU, kV, data = oracle_to_canonical(F)
    say("apply import", n, leaf, F.L)
    H = bf.import_factors(n, n, leaf, kU, kV, data)
    X = _cg(np.random.default_rng(6), n, 9)
    Y = H.apply(_t(X)).cpu().numpy()
    assert _rel(Y, obf.apply(F, X)) < 1e-6
    Yh = H.apply(_t(X), trans=True).cpu().numpy()
    assert _rel(Yh, obf.apply_adjoint(F, X)) < 1e-6
    back = H.export()
    np.testing.assert_array_equal(back, data)
    H.close()


@pytest.mark.parametrize("n,leaf", [(2000, 40), (4096, 16)])
def test_apply_precisions(bf, n, leaf):
    """Applies of imported oracle factors with FP32 vector arithmetic and
    with the default arithmetic (split-BF16 matrix cores from 5 right-hand
    sides, the FP32 vector path below), forward and adjoint, against the
    oracle's FP64 apply; the default is at least as accurate."""
    g = wl.segment_pair(n, ppw=6.0)
    op = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    F = obf.construct(op, 1e-6, leaf, seed=2)
    kU, kV, data = oracle_to_canonical(F)
    say("apply precisions", n, leaf, F.L)
    H = bf.import_factors(n, n, leaf, kU, kV, data)
    rng = np.random.default_rng(7)
    for s in (1, 3, 6, 16, 40, 100):
        X = _cg(rng, n, s)
        ref = obf.apply(F, X)
        refh = obf.apply_adjoint(F, X)
        out = {}
        for prec in ("fp32", "bf16x3"):
            H.set_precision(prec)
            out[prec] = (H.apply(_t(X)).cpu().numpy(), H.apply(_t(X), trans=True).cpu().numpy())
            say("apply", prec, s, "forward", _rel(out[prec][0], ref), "adjoint",
                _rel(out[prec][1], refh))
            assert _rel(out[prec][0], ref) < 1e-6, (s, prec)
            assert _rel(out[prec][1], refh) < 1e-6, (s, prec)
            for c in range(s):    # every column, so no tile or chunk is skipped
                assert np.linalg.norm(out[prec][0][:, c] - ref[:, c]) <= 2e-6 * np.linalg.norm(ref[:, c])
        e32, e16 = _rel(out["fp32"][0], ref), _rel(out["bf16x3"][0], ref)
        assert e16 <= 1.2 * e32 + 1e-8, (s, e16, e32)
    with pytest.raises(bf.BFError):
        lib_rc = bf.lib().bf_set_apply_precision(H._h, 0)
        bf._check(lib_rc, "bf_set_apply_precision")
    H.close()


@pytest.mark.parametrize("L,r,leaf", [(10, 8, 8), (11, 6, 6)])
def test_fused_apply_matches_staged(bf, L, r, leaf):
    """Applies of 1 to 4 columns run several stages per launch
    (bf_set_apply_fusion) when every launch keeps 256 groups (here exact
    butterflies of Sec. 6.1 with 1024 and 2048 blocks a level): bitwise the
    stage-by-stage results (same slots and summation order) and within the
    apply tolerance of the oracle's FP64 apply of the same factors, forward
    and adjoint, in both apply precisions; 5 to 16 columns (stage by stage
    whatever the switch) within the same tolerance."""
    n = leaf << L
    kU, kV, data = wl.exact_butterfly_canonical(L, r, seed=L, leaf=leaf)
    F = canonical_to_oracle(n, n, L, kU, kV, data)
    say("fused apply", n, leaf, L)
    H = bf.import_factors(n, n, leaf, kU, kV, data)
    assert H.stats().fused_launches >= 2
    rng = np.random.default_rng(11)
    cases = []
    for s in (1, 2, 3, 4, 5, 8, 11, 16):
        X = _cg(rng, n, s)
        cases.append((s, X, obf.apply(F, X), obf.apply_adjoint(F, X)))
    for prec in ("bf16x3", "fp32"):
        H.set_precision(prec)
        for s, X, ref, refh in cases:
            got = {}
            for fuse in (True, False):
                H.set_fusion(fuse)
                got[fuse] = (H.apply(_t(X)).cpu().numpy(), H.apply(_t(X), trans=True).cpu().numpy())
            H.set_fusion(True)
            say("fused", prec, s, _rel(got[True][0], ref), _rel(got[True][1], refh))
            if s <= 4:
                for d in (0, 1):
                    assert np.array_equal(got[True][d].view(np.uint64),
                                          got[False][d].view(np.uint64)), (prec, s, d)
            for d, r in ((0, ref), (1, refh)):
                assert _rel(got[True][d], r) < 1e-6, (prec, s, d)
                for c in range(s):
                    assert np.linalg.norm(got[True][d][:, c] - r[:, c]) <= 2e-6 * np.linalg.norm(r[:, c])
    H.close()


def test_fused_apply_ragged_shapes(bf):
    """Fused applies of GPU-built factors with m != n, uneven node sizes and
    uneven ranks (L = 10, leaves of 12 to 16 points) agree with the
    stage-by-stage apply (bitwise up to 4 columns)."""
    import torch
    g = wl.segment_pair(15000, ppw=8.0, m=11000)
    op = bf.segkernel(g.targets, g.sources, g.k)
    H = bf.construct(op, 1e-4, 16, seed=4)
    assert H.L == 10 and H.stats().fused_launches >= 2
    rng = np.random.default_rng(12)
    for s in (1, 3, 7, 16):
        for trans, rows in ((False, 15000), (True, 11000)):
            X = _t(_cg(rng, rows, s))
            H.set_fusion(True)
            a = H.apply(X, trans=trans)
            H.set_fusion(False)
            b = H.apply(X, trans=trans)
            torch.cuda.synchronize()
            if s <= 4:
                assert _same_bits(a, b), (s, trans)
            else:
                assert float((a - b).norm() / b.norm()) < 1e-6, (s, trans)
    H.set_fusion(True)
    H.close()


def test_apply_graphs_replay_bitwise(bf):
    """Applies run as captured HIP graphs (bf_set_apply_graph_cols) give the
    bits of the directly launched stages, on every replay, with direct applies
    and host synchronizations between the replays, for both directions, both
    apply precisions, few-column and matrix-core widths, and above the limit."""
    import torch
    n, leaf = 2000, 40
    g = wl.segment_pair(n, ppw=6.0)
    op = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    F = obf.construct(op, 1e-6, leaf, seed=2)
    kU, kV, data = oracle_to_canonical(F)
    H = bf.import_factors(n, n, leaf, kU, kV, data)
    rng = np.random.default_rng(11)
    cases = [(s, trans, prec) for s in (1, 4, 8, 12) for trans in (False, True)
             for prec in ("bf16x3", "fp32")]
    Xs = {s: _t(_cg(rng, n, s)) for s in (1, 4, 8, 12)}
    ref = {}
    for s, trans, prec in cases:
        H.set_precision(prec)
        ref[(s, trans, prec)] = H.apply(Xs[s], trans=trans).cpu().numpy()
    H.set_graph_cols(8)
    say("apply graphs")
    for rep in range(3):
        for s, trans, prec in cases:
            H.set_precision(prec)
            got = H.apply(Xs[s], trans=trans).cpu().numpy()
            assert np.array_equal(got, ref[(s, trans, prec)]), (rep, s, trans, prec)
            # direct work between replays on the same stream
            H.set_graph_cols(0)
            H.apply(Xs[4], trans=not trans)
            H.set_graph_cols(8)
            torch.cuda.synchronize()
    # one graph per (width <= 8, direction, precision) on this stream; 12 columns ran directly
    assert H.stats().apply_graphs == 12
    H.set_graph_cols(0)
    H.close()
