"""Pins of the bisection trees (Sec. 3.1)."""
import pytest

from oracle import trees


@pytest.mark.parametrize("N", [1, 7, 64, 1000, 1024, 2049, 65536])
def test_children_partition_parent(N):
    L = 6
    for l in range(L):
        for i in range(1 << l):
            lo, hi = trees.node_range(N, l, i)
            a = trees.node_range(N, l + 1, 2 * i)
            b = trees.node_range(N, l + 1, 2 * i + 1)
            assert a[0] == lo and a[1] == b[0] and b[1] == hi
    assert trees.node_range(N, 0, 0) == (0, N)
    # sizes differ by at most one within a level
    for l in range(L + 1):
        sz = [trees.node_size(N, l, i) for i in range(1 << l)]
        assert max(sz) - min(sz) <= 1 and sum(sz) == N


@pytest.mark.parametrize("m,n,leaf,L", [(1024, 1024, 32, 5), (16384, 16384, 64, 8),
                                        (65536, 65536, 64, 10), (262144, 262144, 16, 14),
                                        (20, 20, 32, 0), (33, 10, 32, 1), (3000, 2048, 64, 6)])
def test_num_levels_closed_form(m, n, leaf, L):
    assert trees.num_levels(m, n, leaf) == L
    assert -(-max(m, n) // (1 << L)) <= leaf
    if L:
        assert -(-max(m, n) // (1 << (L - 1))) > leaf


def test_center_level():
    assert [trees.center_level(L) for L in range(6)] == [0, 0, 1, 1, 2, 2]
