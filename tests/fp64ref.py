"""FP64 products of the oracle's kernel entries over a process pool (tests
only): row blocks of exp(i k r)/r times a block of columns, each worker in a
fresh interpreter that never touches the GPU."""
import multiprocessing as mp

import numpy as np


def _rows_times(args):
    from oracle import operators as ops
    t, s, k, r0, r1, X = args
    return ops.segment_kernel_entries(t, s, k, rows=slice(r0, r1)) @ X


def kernel_times(targets, sources, k, X, workers=12):
    m, n = len(targets), len(sources)
    step = max(1, (1 << 22) // n)
    jobs = [(targets, sources, k, r0, min(m, r0 + step), X) for r0 in range(0, m, step)]
    with mp.get_context("spawn").Pool(workers) as pool:
        return np.concatenate(pool.map(_rows_times, jobs), axis=0)
