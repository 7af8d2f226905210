"""FP64 black-box operators for Alg. 2 (Alg. 2, input: products of A and of
A^H with any block of columns the algorithm chooses).

Complex data: every transpose of the paper becomes the conjugate transpose
(Sec. 2.1 extends the real algorithms to complex matrices), so the second
routine is ``rmatvec(X) = A^H X``.

``matvec(X, support)`` may be told that X vanishes outside rows
[support[0], support[1]); the structured random matrices of Sec. 4.1 are zero
outside one tree node, and an operator may skip the zero rows.  This is only a
saving, never a change of result.
"""
from __future__ import annotations

import math

import numpy as np


class DenseOp:
    """Explicit matrix as the black box."""

    def __init__(self, A: np.ndarray):
        self.A = np.asarray(A, dtype=np.complex128)
        self.m, self.n = self.A.shape

    def matvec(self, X, support=None):
        if support is None:
            return self.A @ X
        lo, hi = support
        return self.A[:, lo:hi] @ X[lo:hi]

    def rmatvec(self, X, support=None):
        if support is None:
            return self.A.conj().T @ X
        lo, hi = support
        return self.A[lo:hi].conj().T @ X[lo:hi]


def segment_kernel_entries(targets, sources, k, rows=slice(None), cols=slice(None)):
    """A_ij = exp(i k r_ij) / r_ij with r_ij = |x_i - y_j| (2D or 3D points), FP64.

    The Helmholtz kernel of Sec. 3 (written there as exp(i 2 pi kappa r)/r):
    on the parallel-line geometry of Sec. 6.2 (2D points) and on the two
    semi-spheres of Sec. 6.3, eq. 3dkernel (3D points).
    """
    x = np.asarray(targets)[rows]
    y = np.asarray(sources)[cols]
    r2 = np.zeros((len(x), len(y)))
    for d in range(x.shape[1]):
        dd = x[:, None, d] - y[None, :, d]
        r2 += dd * dd
    r = np.sqrt(r2)
    return np.exp(1j * k * r) / r


class SegmentKernelOp:
    """exp(i k r)/r evaluated on the fly in row chunks (never stored)."""

    def __init__(self, targets, sources, k, chunk_entries=1 << 22):
        self.t = np.asarray(targets, dtype=np.float64)
        self.s = np.asarray(sources, dtype=np.float64)
        self.k = float(k)
        self.m, self.n = len(self.t), len(self.s)
        self.chunk = chunk_entries

    def dense(self):
        return segment_kernel_entries(self.t, self.s, self.k)

    def matvec(self, X, support=None):
        lo, hi = (0, self.n) if support is None else support
        Y = np.zeros((self.m, X.shape[1]), np.complex128)
        step = max(1, self.chunk // max(1, hi - lo))
        for r0 in range(0, self.m, step):
            r1 = min(self.m, r0 + step)
            Y[r0:r1] = segment_kernel_entries(self.t, self.s, self.k,
                                              slice(r0, r1), slice(lo, hi)) @ X[lo:hi]
        return Y

    def rmatvec(self, X, support=None):
        lo, hi = (0, self.m) if support is None else support
        Y = np.zeros((self.n, X.shape[1]), np.complex128)
        step = max(1, self.chunk // max(1, hi - lo))
        for c0 in range(0, self.n, step):
            c1 = min(self.n, c0 + step)
            blk = segment_kernel_entries(self.t, self.s, self.k, slice(lo, hi), slice(c0, c1))
            Y[c0:c1] = blk.conj().T @ X[lo:hi]
        return Y


def fio_entries(x, xi, rows=slice(None), cols=slice(None)):
    """A_jk = exp(2 pi i (x_j xi_k + c(x_j) |xi_k|)), c(x) = (2 + sin 2 pi x)/16.

    x_j = j/n, so x_j xi_k = j xi_k / n; its fractional part is taken exactly
    in integers before adding the smooth term c(x_j)|xi_k|.
    """
    n = len(x)
    j = np.arange(n, dtype=np.int64)[rows][:, None]
    xk = np.asarray(xi, dtype=np.int64)[cols][None, :]
    lin = np.mod(j * xk, n).astype(np.float64) / n
    c = (2.0 + np.sin(2.0 * math.pi * np.asarray(x)[rows])) / 16.0
    ph = lin + c[:, None] * np.abs(xk).astype(np.float64)
    return np.exp(2j * math.pi * ph)


class FIOOp:
    """1D Fourier integral operator evaluated on the fly in row chunks."""

    def __init__(self, x, xi, chunk_entries=1 << 22):
        self.x = np.asarray(x, np.float64)
        self.xi = np.asarray(xi, np.int64)
        self.m = self.n = len(self.x)
        self.chunk = chunk_entries

    def dense(self):
        return fio_entries(self.x, self.xi)

    def matvec(self, X, support=None):
        lo, hi = (0, self.n) if support is None else support
        Y = np.zeros((self.m, X.shape[1]), np.complex128)
        step = max(1, self.chunk // max(1, hi - lo))
        for r0 in range(0, self.m, step):
            r1 = min(self.m, r0 + step)
            Y[r0:r1] = fio_entries(self.x, self.xi, slice(r0, r1), slice(lo, hi)) @ X[lo:hi]
        return Y

    def rmatvec(self, X, support=None):
        lo, hi = (0, self.m) if support is None else support
        Y = np.zeros((self.n, X.shape[1]), np.complex128)
        step = max(1, self.chunk // max(1, hi - lo))
        for c0 in range(0, self.n, step):
            c1 = min(self.n, c0 + step)
            blk = fio_entries(self.x, self.xi, slice(lo, hi), slice(c0, c1))
            Y[c0:c1] = blk.conj().T @ X[lo:hi]
        return Y


class ComposeOp:
    """Product A1 A2 of two black boxes (category (ii) of Sec. 1)."""

    def __init__(self, op1, op2):
        if op1.n != op2.m:
            raise ValueError("inner dimensions differ")
        self.op1, self.op2 = op1, op2
        self.m, self.n = op1.m, op2.n

    def matvec(self, X, support=None):
        return self.op1.matvec(self.op2.matvec(X, support))

    def rmatvec(self, X, support=None):
        return self.op2.rmatvec(self.op1.rmatvec(X, support))
