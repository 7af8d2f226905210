"""Pins of the oracle's Alg. 2, apply and dense assembly."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import butterfly as bf
from oracle import cpqr, metrics, operators as ops


def _seg_op(n, ppw=8.0, m=None):
    g = wl.segment_pair(n, ppw=ppw, m=m)
    return ops.SegmentKernelOp(g.targets, g.sources, g.k)


@pytest.fixture(scope="module")
def c1():
    """n = m = 1024, 8 points per wavelength, leaf 32, tol 1e-6, seed 1."""
    op = _seg_op(1024)
    F = bf.construct(op, 1e-6, 32, seed=1)
    return op, op.dense(), F


def test_apply_matches_dense_assembly(c1):
    _, _, F = c1
    D = bf.dense(F)
    X = wl.test_columns(1024, 4, 3)
    np.testing.assert_allclose(bf.apply(F, X), D @ X, atol=1e-12 * np.linalg.norm(D @ X))
    np.testing.assert_allclose(bf.apply_adjoint(F, X), D.conj().T @ X,
                               atol=1e-12 * np.linalg.norm(D.conj().T @ X))


@pytest.mark.parametrize("m,n,leaf", [(300, 257, 16), (100, 1000, 40), (64, 64, 64), (50, 20, 8)])
def test_ragged_shapes_apply_dense_and_error(m, n, leaf):
    op = _seg_op(n, ppw=10.0, m=m)
    F = bf.construct(op, 1e-6, leaf, seed=4)
    D = bf.dense(F)
    X = wl.test_columns(n, 3, 8)
    np.testing.assert_allclose(bf.apply(F, X), D @ X, atol=1e-12 * np.linalg.norm(D @ X))
    A = op.dense()
    # The adaptive loop may stop with little oversampling (e.g. s = 18 columns
    # for a rank-14 leaf); Alg. 1 then meets eps on the sample but only a few
    # eps on the block, so the bound gets a factor 10 here.
    assert np.linalg.norm(A - D) / np.linalg.norm(A) <= 10 * math.sqrt(F.L + 2) * 1e-6


@pytest.mark.parametrize("L,r", [(3, 2), (4, 4), (5, 8), (6, 8), (4, 3)])
def test_exact_butterfly_recovered(L, r):
    """Sec. 6.1: Alg. 2 recovers a random exact butterfly to rounding level,
    with every recovered rank equal to the generator's r."""
    fx = wl.exact_butterfly_factors(L, r, seed=L * 10 + r)
    op = bf.FactorsOp(bf.from_exact(fx))
    F = bf.construct(op, 1e-6, 8, p=2, r0=4, seed=5)
    A = bf.dense(op.F)
    assert np.linalg.norm(A - bf.dense(F)) <= 1e-12 * np.linalg.norm(A)
    ks = {k for d in F.kU.values() for k in d.values()} | {k for d in F.kV.values() for k in d.values()}
    assert ks == {r}


def test_error_bounds_c1(c1):
    """Thms 4.1-4.3 and eq. (error) at n=1024.  Alg. 1 meets its tolerance on
    the random sample, not on the block itself, so the theorems' assumption
    holds only approximately; 25% slack is allowed on each bound."""
    op, A, F = c1
    eps, L = 1e-6, F.L
    slack = 1.25
    assert metrics.thm43_sum(A, F) <= slack * (L + 2) * eps ** 2
    for l in range(F.lm, L + 1):
        assert metrics.thm41_sum(A, F, l) <= slack * (L - l + 1) * eps ** 2
    for l in range(0, F.lm + 1):
        assert metrics.thm42_sum(A, F, l) <= slack * (l + 1) * eps ** 2
    full = np.linalg.norm(A - bf.dense(F)) / np.linalg.norm(A)
    assert full <= math.sqrt(slack * (L + 2)) * eps
    Om = wl.test_columns(1024, 16, 1001)
    err = metrics.rel_error(A @ Om, bf.apply(F, Om))
    assert 0.2 * eps < err <= math.sqrt(slack * (L + 2)) * eps


def test_ranks_match_brute_force_svd(c1):
    """Complementary low rank (Sec. 3.2): every recovered rank lies within
    [svd_rank(eps) - 1, svd_rank(eps / 100)] of the block's own SVD."""
    _, A, F = c1
    for side in (F.kU, F.kV):
        for l, d in side.items():
            for (i, j), k in d.items():
                K = metrics._block(A, F, l, i, j)
                assert metrics.svd_rank(K, 1e-6) - 1 <= k <= metrics.svd_rank(K, 1e-8)
    # ranks are flat across levels (the constant-r regime of Sec. 4.4.1)
    maxes = [max(d.values()) for d in list(F.kU.values()) + list(F.kV.values())]
    assert max(maxes) - min(maxes) <= 2


def test_error_tracks_tolerance():
    op = _seg_op(512)
    X = wl.test_columns(512, 16, 2)
    AX = op.matvec(X)
    errs = [metrics.rel_error(AX, bf.apply(bf.construct(op, t, 32, seed=3), X)) for t in (1e-3, 1e-5, 1e-7)]
    for e, t in zip(errs, (1e-3, 1e-5, 1e-7)):
        assert 0.1 * t < e < 4 * t
    assert errs[0] > errs[1] > errs[2]


def test_deterministic_and_seeded():
    op = _seg_op(256)
    F1 = bf.construct(op, 1e-5, 16, seed=9)
    F2 = bf.construct(op, 1e-5, 16, seed=9)
    F3 = bf.construct(op, 1e-5, 16, seed=10)
    X = wl.test_columns(256, 2, 1)
    assert np.array_equal(bf.apply(F1, X), bf.apply(F2, X))
    assert not np.array_equal(bf.apply(F1, X), bf.apply(F3, X))


def test_single_block_and_zero_operator():
    """L = 0 (n <= leaf) is one low-rank block U B V^H; the zero operator has
    every rank 1 and applies to zero."""
    op = _seg_op(24)
    F = bf.construct(op, 1e-6, 32, seed=1)
    assert F.L == 0
    A = op.dense()
    assert np.linalg.norm(A - bf.dense(F)) <= 2 * 1e-6 * np.linalg.norm(A)
    Z = ops.DenseOp(np.zeros((40, 40)))
    Fz = bf.construct(Z, 1e-6, 8, seed=1)
    assert {k for d in Fz.kU.values() for k in d.values()} == {1}
    assert np.all(bf.apply(Fz, np.ones((40, 1))) == 0)


def test_rank_cap():
    op = _seg_op(256)
    with pytest.raises(bf.RankCapExceeded):
        bf.construct(op, 1e-6, 64, seed=1, max_rank=4)


# ---- planted mistakes: each must be caught by one of the pins above -------

def test_planted_missing_conjugate_is_caught(monkeypatch):
    fx = wl.exact_butterfly_factors(4, 4, seed=1)
    F0 = bf.from_exact(fx)
    X = wl.test_columns(fx.n, 2, 1)
    good = bf.dense(F0) @ X
    monkeypatch.setattr(bf, "_H", lambda a: a.T)
    assert np.linalg.norm(bf.apply(F0, X) - good) > 1e-3 * np.linalg.norm(good)


def test_planted_wrong_child_index_is_caught(monkeypatch):
    """Feeding the W stage its children in swapped order breaks exact recovery."""
    fx = wl.exact_butterfly_factors(4, 4, seed=2)
    op = bf.FactorsOp(bf.from_exact(fx))
    A = bf.dense(op.F)
    orig_vstack = np.vstack

    def swapped(parts):
        if isinstance(parts, list) and len(parts) == 2:
            return orig_vstack([parts[1], parts[0]])
        return orig_vstack(parts)

    F = bf.construct(op, 1e-6, 8, seed=5)
    assert np.linalg.norm(A - bf.dense(F)) <= 1e-12 * np.linalg.norm(A)
    monkeypatch.setattr(bf.np, "vstack", swapped)
    Fbad = bf.construct(op, 1e-6, 8, seed=5)
    monkeypatch.setattr(bf.np, "vstack", orig_vstack)
    assert np.linalg.norm(A - bf.dense(Fbad)) > 1e-3 * np.linalg.norm(A)


def test_planted_pivot_rule_is_caught(monkeypatch):
    """Pivoting on the smallest column norm disagrees with LAPACK's geqp3."""
    import scipy.linalg as sla
    rng = np.random.default_rng(0)
    W = rng.standard_normal((20, 10)) * rng.uniform(0.2, 5, 10)
    monkeypatch.setattr(cpqr.np, "argmax", np.argmin)
    _, _, perm, _ = cpqr.cpqr_truncated(W, 1e-300)
    assert not np.array_equal(perm, sla.qr(W, pivoting=True, mode="economic")[2])


@pytest.mark.parametrize("L,r", [(4, 3), (5, 4)])
def test_centre_level_variants_exact(L, r):
    """The column-wise (lm = 0, Sec. 3.3.1), row-wise (lm = L, Sec. 3.3.2) and
    intermediate factorizations recover an exact butterfly (the complementary
    low-rank property gives rank r at every level), and their black-box
    column counts follow the sweep structure: an R level l costs 2^(L-l)
    samples and a W level 2^l, each 2r + p wide, so the hybrid lm = L/2 needs
    the fewest."""
    fx = wl.exact_butterfly_factors(L, r, seed=L * 10 + r)
    op = bf.FactorsOp(bf.from_exact(fx))
    A = bf.dense(op.F)
    p = 2
    leaf_cols, rr = 0, 4            # adaptive leaf loop from r0 = 4: doubles until r > rank
    while True:
        leaf_cols += rr + p
        if rr > r:
            break
        rr *= 2
    counts = {}
    for lm in range(L + 1):
        F = bf.construct(op, 1e-6, 8, p=p, r0=4, seed=5, lm=lm)
        assert F.lm == lm
        assert np.linalg.norm(A - bf.dense(F)) <= 1e-12 * np.linalg.norm(A)
        ks = {k for d in F.kU.values() for k in d.values()} | {k for d in F.kV.values() for k in d.values()}
        assert ks == {r}
        s = 2 * r + p
        mv = leaf_cols + sum(2 ** (L - l) * s for l in range(lm, L)) + (r + p if lm == L else 0)
        rmv = leaf_cols + sum(2 ** l * s for l in range(1, lm + 1))
        assert (F.stats["matvec"], F.stats["rmatvec"]) == (mv, rmv)
        counts[lm] = mv + rmv
    assert min(counts, key=counts.get) == L // 2
    assert bf.construct(op, 1e-6, 8, seed=5, lm=-1).lm == L
    with pytest.raises(ValueError):
        bf.construct(op, 1e-6, 8, seed=5, lm=L + 1)


@pytest.mark.parametrize("lm", [0, 2, 5])
def test_centre_level_variants_error(lm):
    """Thm 4.3 bounds the error of the level-l factorization for any l: the
    column- and row-wise variants of an oscillatory operator meet the same
    tolerance model as the hybrid."""
    op = _seg_op(512)
    F = bf.construct(op, 1e-6, 16, seed=2, lm=lm)
    assert F.L == 5 and F.lm == lm
    A = op.dense()
    assert np.linalg.norm(A - bf.dense(F)) / np.linalg.norm(A) <= 10 * math.sqrt(F.L + 2) * 1e-6
