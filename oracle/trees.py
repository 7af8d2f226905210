"""Bisection cluster trees T_T and T_S (Sec. 3.1).

Points are already sorted along their curve, so bisection of a node is a split
of its index range.  Node (l, i), 0 <= i < 2^l, of a tree over N points covers
[floor(i N / 2^l), floor((i+1) N / 2^l)); its children are (l+1, 2i) and
(l+1, 2i+1) and they partition it exactly for every N (the paper assumes
complete trees, which this floor rule gives for any N).  Both trees have the
same depth L: the smallest L with ceil(max(m, n) / 2^L) <= n0 (leaf size).
The centre level is l_m = floor(L / 2) (Sec. 3.3.3).
"""
from __future__ import annotations


def num_levels(m: int, n: int, leaf: int) -> int:
    if leaf < 1:
        raise ValueError("leaf size must be >= 1")
    big = max(m, n)
    L = 0
    while -(-big // (1 << L)) > leaf:
        L += 1
    return L


def center_level(L: int) -> int:
    return L // 2


def node_range(npts: int, level: int, idx: int) -> tuple[int, int]:
    return (idx * npts) // (1 << level), ((idx + 1) * npts) // (1 << level)


def node_size(npts: int, level: int, idx: int) -> int:
    lo, hi = node_range(npts, level, idx)
    return hi - lo
