"""Accuracy measures of Secs. 4 and 6.

* ``rel_error``: eq. (error), ||A Om - F Om||_F / ||A Om||_F with a random
  test matrix Om of 16 columns.
* ``thm41_sum`` / ``thm42_sum`` / ``thm43_sum``: the left-hand sides of
  eqs. (thm_column), (thm_row), (thm_hybrid) divided by ||K||_F^2, so that the
  theorems read  <= (L-l+1) eps^2,  <= (l+1) eps^2  and  <= (L+2) eps^2.
* ``svd_rank``: numerical rank with the same relative Frobenius tail as the
  truncation rule of Alg. 1, from a full SVD (brute force, small blocks).
"""
from __future__ import annotations

import numpy as np

from .butterfly import column_bases, row_bases


def rel_error(AOm: np.ndarray, FOm: np.ndarray) -> float:
    return float(np.linalg.norm(AOm - FOm) / np.linalg.norm(AOm))


def _block(A, F, l, i, j):
    t0, t1 = F.trange(l, i)
    s0, s1 = F.srange(F.L - l, j)
    return A[t0:t1, s0:s1]


def thm41_sum(A, F, l):
    U = column_bases(F)[l]
    tot = 0.0
    for (i, j), Ub in U.items():
        K = _block(A, F, l, i, j)
        tot += np.linalg.norm(K - Ub @ (Ub.conj().T @ K)) ** 2
    return tot / np.linalg.norm(A) ** 2


def thm42_sum(A, F, l):
    V = row_bases(F)[l]
    tot = 0.0
    for (i, j), Vb in V.items():
        K = _block(A, F, l, i, j)
        tot += np.linalg.norm(K - (K @ Vb) @ Vb.conj().T) ** 2
    return tot / np.linalg.norm(A) ** 2


def thm43_sum(A, F):
    l = F.lm
    U = column_bases(F)[l]
    V = row_bases(F)[l]
    tot = 0.0
    for (i, j), Ub in U.items():
        Vb = V[(i, j)]
        K = _block(A, F, l, i, j)
        P = Ub @ (Ub.conj().T @ K @ Vb) @ Vb.conj().T
        tot += np.linalg.norm(K - P) ** 2
    return tot / np.linalg.norm(A) ** 2


def svd_rank(K: np.ndarray, eps: float) -> int:
    """Smallest k >= 1 with sqrt(sum_{q>=k} s_q^2) <= eps ||K||_F."""
    if K.size == 0:
        return 0
    s = np.linalg.svd(K, compute_uv=False)
    tail = np.sqrt(np.cumsum((s ** 2)[::-1])[::-1])   # tail[k] = ||s[k:]||
    tot = tail[0]
    for k in range(1, len(s)):
        if tail[k] <= eps * tot:
            return k
    return len(s)


def level_svd_ranks(A, F, l, eps):
    """Brute-force eps-ranks of all 2^L blocks at level l (complementary low rank)."""
    out = {}
    for i in range(1 << l):
        for j in range(1 << (F.L - l)):
            out[(i, j)] = svd_rank(_block(A, F, l, i, j), eps)
    return out
