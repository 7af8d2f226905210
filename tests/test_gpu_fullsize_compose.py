"""Category (ii) of Sec. 1 at its full size: three parallel unit segments at
y = 0, 1, 2 with n = 65536 points each (8 points per wavelength), B1 ~ A01 and
B2 ~ A12 built matrix-free on the GPU (leaf 64, tol 1e-6), and the composition
B1 B2 recompressed into one butterfly with the two butterflies' applies as the
black box.  The FP64 reference A01 (A12 Omega) on 128 sampled rows is
tests/golden/c3_rows_n65536.json, written by tests/golden/make_c3_rows.py
(oracle/ only).  Bounds: each construction's eq. error within
2 sqrt(L + 2) eps (Thm 4.3's bound on the level projections, with the factor 2
the parity tests allow over the oracle for the randomized range finder), and
the recompression's error against A01 A12 within the triangle inequality's
||F - B1 B2|| + ||B1 B2 - A01 A12||."""
import json
import math
import os
import sys

import numpy as np
import pytest

import workloads as wl
from oracle import operators as ops

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c3_rows_n65536.json")
LEAF, TOL = 64, 1e-6


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rel(got, ref):
    return float(np.linalg.norm(got - ref) / np.linalg.norm(ref))


def _bound(L):
    return 2.0 * math.sqrt(L + 2) * TOL


@pytest.fixture(scope="module")
def c3():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible")
    import paper_2002_03400_amd as bf
    gold = json.load(open(GOLDEN))
    n = gold["n"]
    rows = np.asarray(gold["rows"], np.int64)
    ref = np.asarray(gold["re"]) + 1j * np.asarray(gold["im"])
    g01, g12 = wl.segment_triple(n, ppw=gold["ppw"])
    Om = wl.test_columns(n, 16, gold["test_seed"])
    o1 = bf.segkernel(g01.targets, g01.sources, g01.k)
    o2 = bf.segkernel(g12.targets, g12.sources, g12.k)
    say(f"C3: B1, B2 at n={n}")
    B1 = bf.construct(o1, TOL, LEAF, seed=21)
    B2 = bf.construct(o2, TOL, LEAF, seed=22)
    say("C3: recompression of B1 B2")
    F = bf.construct(bf.compose(bf.from_factors(B1), bf.from_factors(B2)), TOL, LEAF, seed=23)
    OmD = torch.from_numpy(Om.astype(np.complex64)).cuda()
    yield bf, g01, g12, Om, OmD, rows, ref, B1, B2, F
    for H in (F, B1, B2):
        H.close()


def test_input_butterflies_against_oracle_rows(c3):
    """B1 and B2 each on the same 128 rows of the oracle's FP64 kernel entries."""
    bf, g01, g12, Om, OmD, rows, ref, B1, B2, F = c3
    for name, B, g in (("B1", B1, g01), ("B2", B2, g12)):
        exact = ops.segment_kernel_entries(g.targets, g.sources, g.k, rows=rows) @ Om
        e = _rel(B.apply(OmD).cpu().numpy()[rows], exact)
        say(f"C3 {name}: err {e:.3e}, L {B.L}, max rank {B.stats().max_rank}")
        assert e <= _bound(B.L)


def test_recompression_against_fp64_product(c3):
    bf, g01, g12, Om, OmD, rows, ref, B1, B2, F = c3
    BB = B1.apply(B2.apply(OmD))
    FO = F.apply(OmD)
    e_fb = float((FO - BB).norm() / BB.norm())
    e_bb = _rel(BB.cpu().numpy()[rows], ref)
    e_f = _rel(FO.cpu().numpy()[rows], ref)
    st = F.stats()
    say(f"C3 recompressed: err {e_f:.3e} vs FP64 A01 A12 (B1 B2 itself {e_bb:.3e}), "
        f"{e_fb:.3e} vs B1 B2, L {st.L}, max rank {st.max_rank}")
    assert st.L == 10
    assert e_fb <= _bound(st.L)
    assert e_f <= e_bb + _bound(st.L)


def test_recompression_adjoint(c3):
    """F^H Z against B2^H (B1^H Z): the recompressed factors' adjoint apply."""
    bf, g01, g12, Om, OmD, rows, ref, B1, B2, F = c3
    import torch
    Z = torch.from_numpy(wl.test_columns(len(g01.targets), 3, 7).astype(np.complex64)).cuda()
    exp = B2.apply(B1.apply(Z, trans=True), trans=True)
    e = float((F.apply(Z, trans=True) - exp).norm() / exp.norm())
    say(f"C3 adjoint: {e:.3e}")
    assert e <= _bound(F.L)
