"""The plain method on the GPU at n = m = 16384 (segment pair, 8 points per
wavelength, leaf 64, matrix-free black box, complex64 products, FP64 block
solves) at tol 1e-4 and 1e-6, against the FP64 oracle's construction of the
same problem with the same seed: error of eq. (error) on 16 Gaussian test
columns within 2x the oracle's, same L, largest rank within 2 of the
oracle's.  The oracle figures are tests/golden/c2_oracle.json, written by
tests/golden/make_c2_oracle.py (oracle/ only)."""
import json
import os
import sys

import numpy as np
import pytest

import workloads as wl
from tests.fp64ref import kernel_times

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "c2_oracle.json")


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


@pytest.fixture(scope="module")
def c2():
    ref = json.load(open(GOLDEN))
    g = wl.segment_pair(ref["n"], ppw=ref["ppw"])
    Om = wl.test_columns(ref["n"], 16, ref["test_seed"])
    say("C2: FP64 A Omega on the host")
    AOm = kernel_times(g.targets, g.sources, g.k, Om)
    return ref, g, Om, AOm


@pytest.mark.parametrize("tol", ["0.0001", "1e-06"])
def test_c2_construction_parity(bf, c2, tol):
    import torch
    ref, g, Om, AOm = c2
    case = ref["cases"][tol]
    op = bf.segkernel(g.targets, g.sources, g.k)
    say(f"C2: GPU construction n={ref['n']} tol={tol}")
    F = bf.construct(op, case["tol"], ref["leaf"], p=ref["p"], r0=ref["r0"], seed=ref["seed"])
    got = F.apply(torch.from_numpy(Om.astype(np.complex64)).cuda()).cpu().numpy()
    err = float(np.linalg.norm(got - AOm) / np.linalg.norm(AOm))
    st = F.stats()
    say(f"C2 tol {tol}: gpu err {err:.3e} (oracle {case['err']:.3e}), max rank {st.max_rank} "
        f"(oracle {case['max_rank']}), L {st.L}")
    assert st.L == case["L"]
    assert err <= 2.0 * case["err"]
    assert abs(st.max_rank - case["max_rank"]) <= 2
    F.close()
