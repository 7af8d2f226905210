"""Writes tests/golden/c3_rows_n65536.json: the FP64 product A01 (A12 Omega) of
the category (ii) workload of Sec. 1 at n = 65536 (three parallel unit
segments at y = 0, 1, 2, 8 points per wavelength; A01 maps the y = 1 points to
the y = 0 points, A12 the y = 2 points to the y = 1 points), on 128 sampled
rows, for 16 Gaussian test columns Omega (seed 1001).  A12 Omega is formed in
full from the oracle's kernel entries, then the sampled rows of A01 multiply
it.  Calls only oracle/ (through tests/fp64ref.py's process pool) and the
input generators in workloads/; run from the repository root:

    python tests/golden/make_c3_rows.py

(a few minutes on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import operators as ops  # noqa: E402
from tests.fp64ref import kernel_times  # noqa: E402

N, PPW, TEST_SEED, ROW_SEED, NROWS = 65536, 8.0, 1001, 0, 128


def main():
    g01, g12 = wl.segment_triple(N, ppw=PPW)
    Om = wl.test_columns(N, 16, TEST_SEED)
    t0 = time.perf_counter()
    A12Om = kernel_times(g12.targets, g12.sources, g12.k, Om, workers=os.cpu_count() or 8)
    print(f"A12 Omega in {time.perf_counter() - t0:.1f} s", flush=True)
    rows = np.sort(np.random.default_rng(ROW_SEED).choice(N, NROWS, replace=False))
    ref = ops.segment_kernel_entries(g01.targets, g01.sources, g01.k, rows=rows) @ A12Om
    out = {"n": N, "ppw": PPW, "test_seed": TEST_SEED, "row_seed": ROW_SEED,
           "rows": [int(r) for r in rows],
           "re": [[float(v) for v in r] for r in ref.real],
           "im": [[float(v) for v in r] for r in ref.imag]}
    path = os.path.join(ROOT, "tests", "golden", "c3_rows_n65536.json")
    with open(path, "w") as f:
        json.dump(out, f)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
