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
