"""The 3D weak-admissibility regime (Sec. 6.3, eq. 3dkernel): the two adjacent
unit semi-spheres, p = 4, GPU construction against the oracle's."""
import math
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import butterfly as obf
from oracle import operators as ops
from tests.bfconv import canonical_to_oracle, oracle_to_canonical

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def bf():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2002_03400_amd as m
    m.lib()
    return m


def _t(x):
    import torch
    return torch.from_numpy(np.asarray(x, np.complex64)).cuda()


def _err(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(a))


# (n, leaf, tol, r0): L = 5 and 6; the second has Z blocks of more than 100 rows
# (QR and least squares in device scratch) and starts the leaf loop at r0 = 64
@pytest.mark.parametrize("n,leaf,tol,r0", [(2048, 64, 1e-3, 16), (4096, 64, 1e-4, 64)])
def test_hemispheres_parity(bf, n, leaf, tol, r0):
    g = wl.hemisphere_pair(n, seed=1)
    op_o = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    say("oracle 3D construction", n, tol)
    Fo = obf.construct(op_o, tol, leaf, p=4, r0=r0, seed=2)
    say("GPU 3D construction", n, tol)
    op = bf.helmholtz3d(g.targets, g.sources, g.k)
    H = bf.construct(op, tol, leaf, p=4, r0=r0, seed=2)
    Om = wl.test_columns(n, 16, 1001)
    AOm = op_o.matvec(Om)
    e_or = _err(AOm, obf.apply(Fo, Om))
    e_gpu = _err(AOm, H.apply(_t(Om)).cpu().numpy())
    kU, kV = H.ranks()
    ko_U, ko_V, _ = oracle_to_canonical(Fo)
    say("3D errors oracle", e_or, "gpu", e_gpu, "max rank", int(max(kU.max(), kV.max())),
        "oracle", int(max(ko_U.max(), ko_V.max())))
    assert e_gpu <= 1.5 * e_or
    assert np.abs(kU.astype(int) - ko_U).max() <= 2
    assert np.abs(kV.astype(int) - ko_V).max() <= 2
    # the exported GPU factors, assembled densely by the oracle
    kU2, kV2 = H.ranks()
    Fg = canonical_to_oracle(H.m, H.n, H.L, kU2, kV2, H.export())
    D = obf.dense(Fg)
    A = op_o.dense()
    rel = np.linalg.norm(A - D) / np.linalg.norm(A)
    say("3D dense reconstruction", rel)
    assert rel <= 2.0 * e_or


def test_progress_reports(bf):
    """The construction reports every leaf-loop iteration and sweep level,
    in order: leaf V and leaf U iterations, W levels 1..lm, R levels L-1..lm."""
    g = wl.hemisphere_pair(1024, seed=5)
    op = bf.helmholtz3d(g.targets, g.sources, g.k)
    seen = []
    H = bf.construct(op, 1e-3, 32, p=4, r0=8, seed=1,
                     progress=lambda ph, lv: seen.append((ph, lv)))
    info = H.stats()
    L, lm = H.L, H.lm
    say("progress", seen)
    expect = ([("leaf V", i) for i in range(1, info.v_iters + 1)] +
              [("leaf U", i) for i in range(1, info.u_iters + 1)] +
              [("W", l) for l in range(1, lm + 1)] + [("R", l) for l in range(L - 1, lm - 1, -1)])
    assert seen == expect
    assert info.v_iters >= 2 and info.u_iters >= 2   # r0 = 8 is below the leaf ranks
