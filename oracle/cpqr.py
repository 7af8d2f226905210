"""Column-pivoted Householder QR with a truncation tolerance (Alg. 1 step 3).

Alg. 1 returns U = Q from W P = Q R computed "with truncation tolerance eps".
The paper leaves the tolerance's meaning open; its error analysis (Sec. 4,
first paragraph) assumes a relative Frobenius bound ||A - U U^T A||_F <=
eps ||A||_F.  The reading used here is the same relative Frobenius tail on
the sample W itself: stop at the first k >= 1 with ||R[k:, k:]||_F <=
eps ||W||_F (or at k = min(rows, cols)); an empty block has rank 0.

Pivoting is Businger-Golub: at step k the trailing column of largest
Euclidean norm (lowest index on ties) is swapped into position k.  Column
norms are recomputed from the trailing submatrix at every step, never
downdated.  Reflectors are complex Householder H = I - 2 v v^H / (v^H v) with
v = x - alpha e_1, alpha = -exp(i arg x_0) ||x||, so H x = alpha e_1 and the
diagonal of R is alpha (no cancellation when forming v_0).

``rule="diag"`` selects the other reading of the tolerance, kept only as a
diagnostic: stop at the first k >= 1 whose pivot |R[k, k]| (the largest
trailing column norm, which pivoting brings to the diagonal) is at most
eps |R[0, 0]|.
"""
from __future__ import annotations

import numpy as np


def cpqr_truncated(W: np.ndarray, eps: float, rule: str = "fro"):
    """Return (Q_k, k, perm, R_k) with W[:, perm] ~= Q_k R_k, Q_k (M x k)."""
    if rule not in ("fro", "diag"):
        raise ValueError(f"unknown truncation rule {rule!r}")
    A = np.array(W, dtype=np.complex128, copy=True)
    M, N = A.shape
    perm = np.arange(N)
    if M == 0 or N == 0:
        return np.zeros((M, 0), np.complex128), 0, perm, np.zeros((0, N), np.complex128)
    total = np.linalg.norm(A)
    kmax = min(M, N)
    refl = []
    rank = kmax
    r00 = 0.0
    for k in range(kmax):
        norms = np.sum(np.abs(A[k:, k:]) ** 2, axis=0)
        if k >= 1:
            if rule == "fro":
                stop = np.linalg.norm(A[k:, k:]) <= eps * total
            else:
                stop = np.sqrt(norms.max()) <= eps * r00
            if stop:
                rank = k
                break
        p = k + int(np.argmax(norms))          # first maximum: lowest index
        if p != k:
            A[:, [k, p]] = A[:, [p, k]]
            perm[[k, p]] = perm[[p, k]]
        x = A[k:, k]
        xn = np.linalg.norm(x)
        if k == 0:
            r00 = xn
        phase = x[0] / abs(x[0]) if x[0] != 0 else 1.0
        alpha = -phase * xn
        v = x.copy()
        v[0] -= alpha
        vn2 = np.real(np.vdot(v, v))
        if vn2 > 0.0:
            A[k:, k:] -= (2.0 / vn2) * np.outer(v, v.conj() @ A[k:, k:])
        refl.append((v, vn2))
    Q = np.zeros((M, rank), np.complex128)
    Q[np.arange(rank), np.arange(rank)] = 1.0
    for k in reversed(range(rank)):
        v, vn2 = refl[k]
        if vn2 > 0.0:
            Q[k:, :] -= (2.0 / vn2) * np.outer(v, v.conj() @ Q[k:, :])
    R = np.triu(A[:rank, :])
    return Q, rank, perm, R


def range_basis(W: np.ndarray, eps: float, rule: str = "fro"):
    """Alg. 1 step 3 on a sample W = A Omega: orthonormal basis Q_k and rank k."""
    Q, k, _, _ = cpqr_truncated(W, eps, rule)
    return Q, k
