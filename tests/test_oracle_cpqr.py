"""Pins of the oracle's truncated column-pivoted QR (Alg. 1 step 3) against
LAPACK's geqp3 (scipy) and against closed-form special cases."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.cpqr import cpqr_truncated, range_basis


def _cgauss(rng, *shape):
    return (rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / np.sqrt(2)


@pytest.mark.parametrize("M,N", [(30, 20), (20, 30), (64, 34), (24, 26), (1, 5), (5, 1)])
def test_full_rank_matches_geqp3(M, N):
    rng = np.random.default_rng(M * 100 + N)
    W = _cgauss(rng, M, N) * rng.uniform(0.2, 5.0, N)[None, :]
    Q, k, perm, R = cpqr_truncated(W, 1e-300)
    Rs, Ps = sla.qr(W, mode="r", pivoting=True)[0], sla.qr(W, pivoting=True, mode="economic")[2]
    Qs = sla.qr(W, pivoting=True, mode="economic")[0]
    assert k == min(M, N)
    assert np.array_equal(perm, Ps)
    np.testing.assert_allclose(np.abs(np.diag(R)), np.abs(np.diag(Rs[:k])), rtol=1e-12, atol=1e-13)
    # same column space, orthonormal columns, W P = Q R
    np.testing.assert_allclose(Q @ Q.conj().T, Qs[:, :k] @ Qs[:, :k].conj().T, atol=1e-12)
    np.testing.assert_allclose(Q.conj().T @ Q, np.eye(k), atol=1e-13)
    np.testing.assert_allclose(W[:, perm], Q @ R, atol=1e-12 * np.linalg.norm(W))
    assert np.allclose(np.tril(R, -1), 0)


@pytest.mark.parametrize("eps", [1e-2, 1e-4, 1e-6, 1e-9])
def test_truncation_rule(eps):
    """Rank k is the first k>=1 with ||R[k:,k:]||_F <= eps ||W||_F, measured on
    LAPACK's R with the same pivots; the projection error equals that tail."""
    rng = np.random.default_rng(7)
    M, N = 60, 40
    # geometric spectrum so that every tolerance cuts somewhere inside
    U = np.linalg.qr(_cgauss(rng, M, N))[0]
    V = np.linalg.qr(_cgauss(rng, N, N))[0]
    W = (U * (0.6 ** np.arange(N))) @ V.conj().T
    Q, k, perm, _ = cpqr_truncated(W, eps)
    Rs, Ps = sla.qr(W, mode="r", pivoting=True)[0], sla.qr(W, pivoting=True, mode="economic")[2]
    nW = np.linalg.norm(W)
    tails = [np.linalg.norm(Rs[j:, j:]) for j in range(N)]
    expect = next((j for j in range(1, N) if tails[j] <= eps * nW), N)
    assert np.array_equal(perm[:k], Ps[:k])
    assert k == expect
    err = np.linalg.norm(W - Q @ (Q.conj().T @ W))
    assert err <= eps * nW * (1 + 1e-9)
    np.testing.assert_allclose(err, tails[k] if k < N else 0.0, rtol=1e-6, atol=1e-14 * nW)


@pytest.mark.parametrize("r", [1, 3, 8, 17])
def test_exact_rank_recovered(r):
    """Alg. 1 on an exact rank-r sample: k = r, residual at rounding level."""
    rng = np.random.default_rng(r)
    W = _cgauss(rng, 50, r) @ _cgauss(rng, r, 30)
    Q, k = range_basis(W, 1e-10)
    assert k == r
    assert np.linalg.norm(W - Q @ (Q.conj().T @ W)) < 1e-13 * np.linalg.norm(W)


def test_degenerate_blocks():
    Q, k = range_basis(np.zeros((6, 4), complex), 1e-6)
    assert k == 1 and Q.shape == (6, 1) and abs(np.linalg.norm(Q) - 1) < 1e-15
    Q, k = range_basis(np.zeros((0, 4), complex), 1e-6)
    assert k == 0 and Q.shape == (0, 0)
    Q, k = range_basis(np.zeros((5, 0), complex), 1e-6)
    assert k == 0 and Q.shape == (5, 0)
    Q, k = range_basis(np.array([[3 - 4j]]), 1e-6)
    assert k == 1 and np.isclose(abs(Q[0, 0]), 1.0)


def test_zero_padding_columns_neutral():
    """Zero columns appended to a sample change neither the rank nor the basis."""
    rng = np.random.default_rng(2)
    W = _cgauss(rng, 40, 5) @ _cgauss(rng, 5, 12) + 1e-9 * _cgauss(rng, 40, 12)
    Q1, k1 = range_basis(W, 1e-6)
    Q2, k2 = range_basis(np.hstack([W, np.zeros((40, 7))]), 1e-6)
    assert k1 == k2 == 5
    np.testing.assert_allclose(Q1, Q2, atol=1e-14)


def test_pivot_ties_take_lowest_index():
    W = np.eye(4, dtype=complex)
    _, k, perm, _ = cpqr_truncated(W, 1e-300)
    assert k == 4 and list(perm) == [0, 1, 2, 3]
