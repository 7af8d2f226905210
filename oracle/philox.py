"""Philox4x64-10 and the complex Gaussian drawn from it.

Alg. 1 step 1 and Alg. 2 (the lines that form Gamma_t, Omega_s, Gamma_tau and
Omega_nu) draw i.i.d. normal random matrices.  To make the draw reproducible
and independent of the order in which samples are generated, every entry is a
pure function of (seed, tag, row, col):

    o = Philox4x64-10(counter = (row, col, tag, 0), key = (seed, 0))
    u_q = ((o_q >> 12) + 1/2) * 2^-52            q = 0, 1     (u in (0, 1))
    g = sqrt(-2 ln u_0) * (cos 2 pi u_1 + i sin 2 pi u_1) / sqrt(2)

Philox4x64-10 is the counter-based generator of Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of
two 64x64->128-bit multiplications with the published multipliers, with a
Weyl-sequence key schedule.  The complex normal has E|g|^2 = 1 (real and
imaginary parts N(0, 1/2)); complex data are the paper's "trivial extension"
of its real algorithms (Sec. 2.1).

The construction's random matrices (``gaussian_block``) are these draws
themselves: i.i.d. complex normal entries, as Alg. 1 step 1 and Sec. 4.1 ask.
How a device stores or rounds them is its own choice and not the oracle's.

Tags: ``tag(phase, level, node) = phase << 56 | level << 40 | node``.
"""
from __future__ import annotations

import math

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
_MASK64 = (1 << 64) - 1

PHASE_V0 = 1   # adaptive loop for the leaf row bases V (level-0 blocks)
PHASE_U0 = 2   # adaptive loop for the leaf column bases U (level-L blocks)
PHASE_W = 3    # structured samples Gamma_tau of the W sweep
PHASE_R = 4    # structured samples Omega_nu of the R sweep


def tag(phase: int, level: int, node: int) -> int:
    return (phase << 56) | (level << 40) | node


def philox4x64_10_scalar(ctr, key):
    """Reference Philox4x64-10 on Python integers (one block)."""
    c = [int(x) & _MASK64 for x in ctr]
    k = [int(x) & _MASK64 for x in key]
    for rnd in range(10):
        if rnd:
            k = [(k[0] + W0) & _MASK64, (k[1] + W1) & _MASK64]
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [(p1 >> 64) ^ c[1] ^ k[0], p1 & _MASK64,
             (p0 >> 64) ^ c[3] ^ k[1], p0 & _MASK64]
    return c


def _mulhilo(a: np.ndarray, b: int):
    """128-bit product of uint64 array ``a`` and constant ``b``: (hi, lo)."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    bl = np.uint64(b & 0xFFFFFFFF)
    bh = np.uint64(b >> 32)
    al = a & m32
    ah = a >> s32
    ll = al * bl
    hl = ah * bl
    lh = al * bh
    hh = ah * bh
    cross = (ll >> s32) + (hl & m32) + (lh & m32)
    hi = hh + (hl >> s32) + (lh >> s32) + (cross >> s32)
    lo = a * np.uint64(b)
    return hi, lo


def philox4x64_10(c0, c1, c2, c3, key0: int, key1: int = 0):
    """Vectorised Philox4x64-10 over uint64 arrays of counters."""
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.broadcast_to(np.asarray(c1, dtype=np.uint64), c0.shape).copy()
    c2 = np.broadcast_to(np.asarray(c2, dtype=np.uint64), c0.shape).copy()
    c3 = np.broadcast_to(np.asarray(c3, dtype=np.uint64), c0.shape).copy()
    c0 = c0.copy()
    k0, k1 = key0 & _MASK64, key1 & _MASK64
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd:
                k0 = (k0 + W0) & _MASK64
                k1 = (k1 + W1) & _MASK64
            hi0, lo0 = _mulhilo(c0, M0)
            hi1, lo1 = _mulhilo(c2, M1)
            n0 = hi1 ^ c1 ^ np.uint64(k0)
            n2 = hi0 ^ c3 ^ np.uint64(k1)
            c0, c1, c2, c3 = n0, lo1, n2, lo0
    return c0, c1, c2, c3


def uniform52(o: np.ndarray) -> np.ndarray:
    """Map 64 random bits to the open interval (0, 1): ((o >> 12) + 1/2) 2^-52.

    Every value is exact in binary64 and lies in [2^-53, 1 - 2^-53]."""
    return ((o >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)


def gaussian_block(seed: int, tg: int, row0: int, nrows: int, ncols: int) -> np.ndarray:
    """Complex Gaussian entries for global rows [row0, row0+nrows), cols [0, ncols)."""
    rows = np.arange(row0, row0 + nrows, dtype=np.uint64)[:, None]
    cols = np.arange(ncols, dtype=np.uint64)[None, :]
    r = np.broadcast_to(rows, (nrows, ncols))
    c = np.broadcast_to(cols, (nrows, ncols))
    o0, o1, _, _ = philox4x64_10(r, c, np.uint64(tg & _MASK64), 0, seed)
    u0 = uniform52(o0)
    u1 = uniform52(o1)
    rad = np.sqrt(-2.0 * np.log(u0)) / math.sqrt(2.0)
    ang = 2.0 * math.pi * u1
    return (rad * np.cos(ang) + 1j * (rad * np.sin(ang))).astype(np.complex128)
