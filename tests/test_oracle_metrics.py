"""Pins of the oracle's accuracy measures (eq. error of Sec. 6, the sums of
Thms 4.1-4.3, brute-force SVD ranks) and of the diagnostic truncation rule,
each against a value fixed by the mathematics of a constructed case: an exact
butterfly has zero projection residual at every level, and a perturbation
orthogonal to a block's basis adds exactly its own squared norm."""
import math

import numpy as np
import pytest

import workloads as wl
from oracle import butterfly as obf
from oracle import cpqr, metrics


def _unitary(rng, n):
    q, r = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
    return q * (np.diag(r) / np.abs(np.diag(r)))


def _with_singular_values(s, rows, cols, seed):
    rng = np.random.default_rng(seed)
    U = _unitary(rng, rows)[:, :len(s)]
    V = _unitary(rng, cols)[:, :len(s)]
    return (U * np.asarray(s)) @ V.conj().T


# s = (1, 0.5, 0.1, 0.01, 0.001): ||K||_F^2 = 1.260101, and the tails
# ||s[k:]|| / ||K||_F are 0.454, 0.0895, 0.00895, 0.000891 for k = 1..4.
@pytest.mark.parametrize("eps,k", [(0.5, 1), (0.4, 2), (0.05, 3), (1e-3, 4), (5e-4, 5)])
def test_svd_rank_prescribed_singular_values(eps, k):
    K = _with_singular_values([1.0, 0.5, 0.1, 0.01, 0.001], 9, 7, seed=int(eps * 1e6))
    assert metrics.svd_rank(K, eps) == k


def test_svd_rank_exact_low_rank_and_empty():
    K = _with_singular_values([2.0, 1.0], 12, 10, seed=3)
    assert metrics.svd_rank(K, 1e-10) == 2
    assert metrics.svd_rank(np.zeros((0, 4)), 1e-6) == 0
    # identity of order 3: the tails of one and two unit values are
    # 1/sqrt(3) = 0.577 and sqrt(2/3) = 0.816 of ||I||_F
    assert metrics.svd_rank(np.eye(3), 0.5) == 3
    assert metrics.svd_rank(np.eye(3), 0.58) == 2
    assert metrics.svd_rank(np.eye(3), 0.82) == 1


def test_rel_error_closed_form():
    a = np.ones((4, 3), complex)
    assert metrics.rel_error(a, 1.25 * a) == pytest.approx(0.25, rel=1e-15)
    assert metrics.rel_error(a, a) == 0.0


@pytest.fixture(scope="module")
def exact():
    """An exact hybrid butterfly (Sec. 6.1, every rank 3, L = 4, leaves of 8)
    and its dense matrix."""
    fx = wl.exact_butterfly_factors(4, 3, seed=17)
    F = obf.from_exact(fx)
    return F, obf.dense(F)


def test_nested_bases_are_orthonormal(exact):
    F, _ = exact
    for d in list(obf.column_bases(F).values()) + list(obf.row_bases(F).values()):
        for Q in d.values():
            assert np.allclose(Q.conj().T @ Q, np.eye(Q.shape[1]), atol=1e-12)


def test_theorem_sums_vanish_on_exact_butterfly(exact):
    F, A = exact
    for l in range(F.lm, F.L + 1):
        assert metrics.thm41_sum(A, F, l) < 1e-26
    for l in range(0, F.lm + 1):
        assert metrics.thm42_sum(A, F, l) < 1e-26
    assert metrics.thm43_sum(A, F) < 1e-26


def _block_slices(F, l, i, j):
    t0, t1 = F.trange(l, i)
    s0, s1 = F.srange(F.L - l, j)
    return slice(t0, t1), slice(s0, s1)


def _perturb(F, A, l, blocks, side, seed):
    """A + E, E nonzero only on the given blocks of level l and orthogonal to
    the block's column basis (side "U": E = (I - U U^H) G) or row basis
    (side "V": E = G (I - V V^H)); returns the perturbed matrix and sum ||E||^2."""
    rng = np.random.default_rng(seed)
    Ap = A.copy()
    tot = 0.0
    bases = obf.column_bases(F)[l] if side == "U" else obf.row_bases(F)[l]
    for (i, j) in blocks:
        rs, cs = _block_slices(F, l, i, j)
        shape = Ap[rs, cs].shape
        G = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        Q = bases[(i, j)]
        E = G - Q @ (Q.conj().T @ G) if side == "U" else G - (G @ Q) @ Q.conj().T
        Ap[rs, cs] += E
        tot += np.linalg.norm(E) ** 2
    return Ap, tot


@pytest.mark.parametrize("l", [2, 3, 4])
def test_thm41_sum_counts_every_perturbed_block(exact, l):
    """Column-basis residual at level l: exactly ||E||^2 / ||A + E||^2 when E
    lies outside range(U) on two blocks of the level (a sum that skipped a
    block or a level would miss half of it)."""
    F, A = exact
    nT, nS = 1 << l, 1 << (F.L - l)
    blocks = [(0, 0), (nT - 1, nS - 1)]
    Ap, e2 = _perturb(F, A, l, blocks, "U", seed=l)
    assert metrics.thm41_sum(Ap, F, l) == pytest.approx(e2 / np.linalg.norm(Ap) ** 2, rel=1e-9)


@pytest.mark.parametrize("l", [0, 1, 2])
def test_thm42_sum_counts_every_perturbed_block(exact, l):
    F, A = exact
    nT, nS = 1 << l, 1 << (F.L - l)
    blocks = [(0, nS - 1), (nT - 1, 0)] if (nT, nS) != (1, 1) else [(0, 0)]
    Ap, e2 = _perturb(F, A, l, blocks, "V", seed=10 + l)
    assert metrics.thm42_sum(Ap, F, l) == pytest.approx(e2 / np.linalg.norm(Ap) ** 2, rel=1e-9)


def test_thm43_sum_two_sided_projection(exact):
    """Centre level: a perturbation outside range(U) on one block and outside
    range(V) on another both survive the two-sided projection in full; a
    general perturbation G keeps ||G||^2 - ||U^H G V||^2 (Pythagoras)."""
    F, A = exact
    l = F.lm
    Ap, e2u = _perturb(F, A, l, [(0, 0)], "U", seed=21)
    Ap, e2v = _perturb(F, Ap, l, [(1, 2)], "V", seed=22)
    assert metrics.thm43_sum(Ap, F) == pytest.approx((e2u + e2v) / np.linalg.norm(Ap) ** 2, rel=1e-9)
    rng = np.random.default_rng(23)
    rs, cs = _block_slices(F, l, 2, 1)
    Ag = A.copy()
    G = rng.standard_normal(Ag[rs, cs].shape) + 1j * rng.standard_normal(Ag[rs, cs].shape)
    Ag[rs, cs] += G
    U = obf.column_bases(F)[l][(2, 1)]
    V = obf.row_bases(F)[l][(2, 1)]
    keep = np.linalg.norm(G) ** 2 - np.linalg.norm(U.conj().T @ G @ V) ** 2
    assert metrics.thm43_sum(Ag, F) == pytest.approx(keep / np.linalg.norm(Ag) ** 2, rel=1e-9)


def test_truncation_rules_differ_as_defined():
    """diag(1, .1, .1, .1, .1) at eps = 0.15: the pivot rule stops at k = 1
    (|R_11| = 0.1 <= 0.15), the Frobenius-tail rule at k = 3 (tails 0.2, 0.173,
    0.141 against 0.15 ||W||_F = 0.153)."""
    W = np.diag([1.0, 0.1, 0.1, 0.1, 0.1]).astype(complex)
    assert cpqr.range_basis(W, 0.15, "diag")[1] == 1
    assert cpqr.range_basis(W, 0.15, "fro")[1] == 3
    with pytest.raises(ValueError):
        cpqr.range_basis(W, 0.15, "other")


def test_error_to_tolerance_under_both_rules():
    """Diagnostic of the tolerance reading at n = 1024 (leaf 32, seed 1):
    error / eps of eq. (error) under the Frobenius-tail rule (the reading
    used) and under the pivot rule |R_kk| <= eps |R_11|, at eps = 1e-4 and
    1e-6.  The pivot rule keeps more columns (its threshold is on one column,
    not on the whole tail), so its ranks are at least those of the tail
    rule and its error no larger up to the sampling noise; both stay within
    Thm 4.3's sqrt(L + 2) eps."""
    from oracle import operators as ops
    g = wl.segment_pair(1024, ppw=8.0)
    op = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    Om = wl.test_columns(1024, 16, 1001)
    AOm = op.matvec(Om)
    for eps in (1e-4, 1e-6):
        res = {}
        for rule in ("fro", "diag"):
            F = obf.construct(op, eps, 32, seed=1, rule=rule)
            res[rule] = (metrics.rel_error(AOm, obf.apply(F, Om)) / eps, F.max_rank())
        print(f"eps={eps:g}: error/eps (max rank) fro {res['fro'][0]:.2f} ({res['fro'][1]}), "
              f"diag {res['diag'][0]:.2f} ({res['diag'][1]})")
        assert res["diag"][1] >= res["fro"][1]
        for ratio, _ in res.values():
            assert ratio <= math.sqrt(F.L + 2)
