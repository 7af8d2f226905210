"""Writes tests/golden/c2_oracle.json: the FP64 oracle's Alg. 2 at n = m = 16384
(segment pair of Sec. 6.2's geometry, 8 points per wavelength, leaf 64, p = 2,
r0 = 4, seed 2) for tol 1e-4 and 1e-6, with the eq. error of Sec. 6 on 16
Gaussian test columns (seed 1002) against the oracle's exact product A Omega,
and the ranks.  Calls only oracle/ and the input generators in workloads/;
run from the repository root:

    python tests/golden/make_c2_oracle.py

(about 10 minutes on 8 cores).
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as wl  # noqa: E402
from oracle import butterfly as obf  # noqa: E402
from oracle import operators as ops  # noqa: E402

N, LEAF, PPW, SEED, TEST_SEED = 16384, 64, 8.0, 2, 1002


def main():
    g = wl.segment_pair(N, ppw=PPW)
    op = ops.SegmentKernelOp(g.targets, g.sources, g.k)
    Om = wl.test_columns(N, 16, TEST_SEED)
    t0 = time.perf_counter()
    AOm = op.matvec(Om)
    print(f"A Omega in {time.perf_counter() - t0:.1f} s", flush=True)
    out = {"n": N, "leaf": LEAF, "ppw": PPW, "seed": SEED, "test_seed": TEST_SEED, "p": 2, "r0": 4,
           "cases": {}}
    for tol in (1e-4, 1e-6):
        t0 = time.perf_counter()
        F = obf.construct(op, tol, LEAF, seed=SEED)
        dt = time.perf_counter() - t0
        err = float(np.linalg.norm(obf.apply(F, Om) - AOm) / np.linalg.norm(AOm))
        ku = [k for lv in F.kU.values() for k in lv.values()]
        kv = [k for lv in F.kV.values() for k in lv.values()]
        out["cases"][f"{tol:g}"] = {"tol": tol, "err": err, "L": F.L, "lm": F.lm,
                                    "max_rank": int(max(ku + kv)), "seconds": dt}
        print(f"tol {tol:g}: L={F.L} max rank {max(ku + kv)} err {err:.3e} ({dt:.0f} s)", flush=True)
    path = os.path.join(ROOT, "tests", "golden", "c2_oracle.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
