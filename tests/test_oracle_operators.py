"""Pins of the FP64 black-box operators."""
import cmath
import math

import numpy as np
import pytest

import workloads as wl
from oracle import operators as ops


def test_segment_kernel_closed_form_points():
    g = wl.segment_pair(64, ppw=8.0)
    A = ops.segment_kernel_entries(g.targets, g.sources, g.k)
    # x_i = ((i+1/2)/64, 0), y_j = ((j+1/2)/64, 1): same index -> r = 1
    assert np.allclose(np.diag(A), cmath.exp(1j * g.k))
    i, j = 5, 40
    r = math.hypot((i - j) / 64.0, 1.0)
    assert abs(A[i, j] - cmath.exp(1j * g.k * r) / r) < 1e-13
    # modulus 1/r, Toeplitz in i - j on equispaced lines, reciprocity K(x,y)=K(y,x)
    R = np.hypot((np.arange(64)[:, None] - np.arange(64)[None, :]) / 64.0, 1.0)
    np.testing.assert_allclose(np.abs(A), 1.0 / R, rtol=1e-14)
    np.testing.assert_allclose(A[1:, 1:], A[:-1, :-1], atol=1e-13)
    At = ops.segment_kernel_entries(g.sources, g.targets, g.k)
    np.testing.assert_allclose(At, A.T, atol=1e-14)
    # eight points per wavelength: phase advances by 2 pi over 8 index steps far away
    assert abs(g.k * 8 / 64 - 2 * math.pi) < 1e-12


@pytest.mark.parametrize("opname", ["seg", "fio"])
def test_matvec_rmatvec_chunks_and_adjoint(opname):
    n = 96
    if opname == "seg":
        g = wl.segment_pair(n, ppw=6.0, m=80)
        op = ops.SegmentKernelOp(g.targets, g.sources, g.k, chunk_entries=700)
    else:
        x, xi = wl.fio_params(n)
        op = ops.FIOOp(x, xi, chunk_entries=700)
    A = op.dense()
    rng = np.random.default_rng(0)
    X = rng.standard_normal((op.n, 3)) + 1j * rng.standard_normal((op.n, 3))
    Yv = rng.standard_normal((op.m, 3)) + 1j * rng.standard_normal((op.m, 3))
    np.testing.assert_allclose(op.matvec(X), A @ X, atol=1e-11)
    np.testing.assert_allclose(op.rmatvec(Yv), A.conj().T @ Yv, atol=1e-11)
    # <A x, y> = <x, A^H y>
    lhs = np.vdot(Yv, op.matvec(X))
    rhs = np.vdot(op.rmatvec(Yv), X)
    assert abs(lhs - rhs) < 1e-10 * abs(lhs)
    # structured (supported) input gives the same result as the zero-padded one
    Xs = np.zeros_like(X)
    Xs[10:40] = X[10:40]
    np.testing.assert_allclose(op.matvec(Xs, support=(10, 40)), A @ Xs, atol=1e-11)
    Ys = np.zeros_like(Yv)
    Ys[5:33] = Yv[5:33]
    np.testing.assert_allclose(op.rmatvec(Ys, support=(5, 33)), A.conj().T @ Ys, atol=1e-11)


def test_fio_linear_part_is_a_dft():
    """Removing the smooth phase c(x)|xi| leaves exp(2 pi i j xi / n): a DFT,
    checked against numpy.fft."""
    n = 128
    x, xi = wl.fio_params(n)
    A = ops.fio_entries(x, xi)
    c = (2 + np.sin(2 * np.pi * x)) / 16
    D = A * np.exp(-2j * np.pi * c[:, None] * np.abs(xi)[None, :])
    v = np.random.default_rng(1).standard_normal(n) + 0j
    # sum_k exp(2 pi i j (k - n/2)/n) v_k = (-1)^j * n * ifft(v)_j
    ref = ((-1.0) ** np.arange(n)) * n * np.fft.ifft(v)
    np.testing.assert_allclose(D @ v, ref, atol=1e-9)
    assert np.allclose(np.abs(A), 1.0)


def test_fio_integer_phase_exact_at_large_index():
    """j*xi mod n in integers keeps the phase exact where a float product
    would lose digits."""
    n = 262144
    x, xi = wl.fio_params(n)
    j, k = n - 3, n - 1
    e = ops.fio_entries(x, xi, slice(j, j + 1), slice(k, k + 1))[0, 0]
    lin = ((j * int(xi[k])) % n) / n
    c = (2 + math.sin(2 * math.pi * j / n)) / 16
    ref = cmath.exp(2j * math.pi * (lin + c * abs(int(xi[k]))))
    assert abs(e - ref) < 1e-10


def test_compose_op():
    g01, g12 = wl.segment_triple(40, ppw=5.0)
    o1 = ops.SegmentKernelOp(g01.targets, g01.sources, g01.k)
    o2 = ops.SegmentKernelOp(g12.targets, g12.sources, g12.k)
    c = ops.ComposeOp(o1, o2)
    X = np.random.default_rng(2).standard_normal((40, 2)) + 0j
    np.testing.assert_allclose(c.matvec(X), o1.dense() @ (o2.dense() @ X), atol=1e-10)
    np.testing.assert_allclose(c.rmatvec(X), (o1.dense() @ o2.dense()).conj().T @ X, atol=1e-10)


def test_serving_streams_are_seeded_and_well_formed():
    a = wl.mixed_stream(200, rate=10.0, seed=3)
    b = wl.mixed_stream(200, rate=10.0, seed=3)
    assert a == b
    ts = [r.t for r in a]
    assert ts == sorted(ts) and ts[0] > 0
    cons = [i for i, r in enumerate(a) if r.kind == "construct"]
    assert 0.55 < len(cons) / len(a) < 0.85
    for i, r in enumerate(a):
        if r.kind == "construct":
            assert 2048 <= r.n <= 65536 and 4.0 <= r.ppw <= 16.0 and r.tol in (1e-4, 1e-6)
        else:
            assert 1 <= r.nrhs <= 64 and a[r.target].kind == "construct" and r.target < i
    p = wl.poisson_stream(50, rate=2.0, seed=1)
    gaps = np.diff([0.0] + [r.t for r in p])
    assert abs(gaps.mean() - 0.5) < 0.2 and len({r.seed for r in p}) == 50


def test_helmholtz3d_entries_closed_form():
    """eq. 3dkernel on hand-placed 3D points: a 3-4-5 offset and a unit one."""
    t = np.array([[0.0, 0.0, 0.0], [1.0, 2.0, 2.0]])
    s = np.array([[0.0, 3.0, 4.0], [1.0, 2.0, 3.0]])
    k = 2.5
    A = ops.segment_kernel_entries(t, s, k)
    assert abs(A[0, 0] - cmath.exp(5j * k) / 5.0) < 1e-15
    assert abs(A[1, 1] - cmath.exp(1j * k)) < 1e-15
    r01 = math.sqrt(1.0 + 4.0 + 9.0)
    assert abs(A[0, 1] - cmath.exp(1j * k * r01) / r01) < 1e-15
    # reciprocity and |A| = 1/r on the semi-sphere pair
    g = wl.hemisphere_pair(300, seed=3)
    A = ops.segment_kernel_entries(g.targets, g.sources, g.k)
    At = ops.segment_kernel_entries(g.sources, g.targets, g.k)
    np.testing.assert_allclose(At, A.T, atol=1e-13)
    R = np.linalg.norm(g.targets[:, None, :] - g.sources[None, :, :], axis=-1)
    np.testing.assert_allclose(np.abs(A), 1.0 / R, rtol=1e-13)


def test_hemisphere_pair_geometry():
    n = 2000
    g = wl.hemisphere_pair(n, seed=1)
    h = math.sqrt(2 * math.pi / n)
    assert g.targets.shape == (n, 3) and g.sources.shape == (n, 3)
    np.testing.assert_allclose(np.linalg.norm(g.targets, axis=1), 1.0, atol=1e-14)
    np.testing.assert_allclose(np.linalg.norm(g.sources - [0, 0, -h / 2], axis=1), 1.0, atol=1e-14)
    assert g.targets[:, 2].min() > 0 and g.sources[:, 2].max() < -h / 2
    # n = 50 k^2 / pi: ten points per wavelength
    assert abs(50 * g.k ** 2 / math.pi - n) < 1e-9 * n
    # adjacent but disjoint: closest pair at about the point spacing
    R = np.linalg.norm(g.targets[:, None, :] - g.sources[None, :, :], axis=-1)
    assert 0.5 * h < R.min() < 2 * h
    # equal-area spiral: the heights are a permutation of (i + 1/2) / n
    np.testing.assert_allclose(np.sort(g.targets[:, 2]), (np.arange(n) + 0.5) / n, atol=1e-15)


def test_bisection_order_clusters():
    """Every node range of the bisection tree splits into two children that
    are separated along one coordinate axis (a spatial cluster tree)."""
    g = wl.hemisphere_pair(1000, seed=2, depth=6)
    for pts in (g.targets, g.sources):
        N = len(pts)
        for l in range(6):
            for i in range(1 << l):
                a, c, b = (i * N) >> l, ((2 * i + 1) * N) >> (l + 1), ((i + 1) * N) >> l
                lo, hi = pts[a:c], pts[c:b]
                assert any(lo[:, ax].max() <= hi[:, ax].min() for ax in range(3))
    # a permutation: no point lost or duplicated
    p = wl.bisection_order(np.random.default_rng(0).random((513, 3)), 5)
    assert sorted(p.tolist()) == list(range(513))
