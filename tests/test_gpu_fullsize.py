"""The benchmark's own configuration (segment kernel, n = m = 65536, 8 points
per wavelength, leaf 64, p = 2, r0 = 4, tol 2e-7, seed 3: the launch shapes
bench.py times), checked on sampled outputs the oracle computes one by one,
and through properties that hold at any size."""
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import operators as ops

pytestmark = pytest.mark.gpu

N, LEAF, TOL = 65536, 64, 2e-7


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def full(request):
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2002_03400_amd as bf
    g = wl.segment_pair(N, ppw=8.0)
    op = bf.segkernel(g.targets, g.sources, g.k)
    say("full-size construction n =", N)
    F = bf.construct(op, TOL, LEAF, seed=3)
    return bf, g, op, F


def _t(x):
    import torch
    return torch.from_numpy(np.asarray(x, np.complex64)).cuda()


def test_sampled_rows_against_oracle(full):
    """eq. error on 16 test columns, restricted to 128 sampled rows whose FP64
    entries the oracle evaluates directly: within the metric's 1e-6, and the
    black-box product itself FP32-accurate on the same rows."""
    bf, g, op, F = full
    Om = wl.test_columns(N, 16, 1001)
    rows = np.sort(np.random.default_rng(5).choice(N, 128, replace=False))
    ref = ops.segment_kernel_entries(g.targets, g.sources, g.k, rows=rows) @ Om
    got = F.apply(_t(Om)).cpu().numpy()[rows]
    err = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    bb = op.matvec(_t(Om)).cpu().numpy()[rows]
    err_bb = np.linalg.norm(bb - ref) / np.linalg.norm(ref)
    say("full size: factorization err", err, "black box err", err_bb)
    assert err <= 1e-6
    assert err_bb <= 5e-7


def test_adjoint_and_ranks(full):
    """<F x, y> = <x, F^H y> to single precision; the leaf loops needed r = 32
    (max rank between 16 and 32) and every block of every level is ranked."""
    bf, g, op, F = full
    rng = np.random.default_rng(9)
    x = (rng.standard_normal((N, 3)) + 1j * rng.standard_normal((N, 3))).astype(np.complex64)
    y = (rng.standard_normal((N, 3)) + 1j * rng.standard_normal((N, 3))).astype(np.complex64)
    Fx = F.apply(_t(x)).cpu().numpy().astype(np.complex128)
    Fhy = F.apply(_t(y), trans=True).cpu().numpy().astype(np.complex128)
    lhs = np.vdot(y.astype(np.complex128), Fx)
    rhs = np.vdot(Fhy, x.astype(np.complex128))
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)
    info = F.stats()
    kU, kV = F.ranks()
    assert (info.L, info.lm) == (10, 5)
    assert 16 < info.max_rank <= 32 and info.v_iters == 4 and info.u_iters == 4
    assert kU.min() >= 1 and kV.min() >= 1 and max(kU.max(), kV.max()) == info.max_rank


def test_deterministic_at_full_size(full):
    bf, g, op, F = full
    F2 = bf.construct(op, TOL, LEAF, seed=3)
    assert np.array_equal(F.export(), F2.export())
