"""Plain, slow, obviously-correct CPU oracle of the randomized butterfly
construction (Liu et al., "Butterfly factorization via randomized
matrix-vector multiplications", arXiv:2002.03400).

TEST INFRASTRUCTURE ONLY.  This package exists to check the HIP path.  Only
the test suite, the smoke check and the benchmark's CPU-baseline leg may
import it; the library path never does, and it shares no code with the HIP
path (the only common module is ``workloads``, which builds inputs and holds
none of the method's arithmetic).

Everything is numpy complex128 / float64.  Each function cites the passage of
the paper it follows:

* ``philox``    counter-based Philox4x64-10 (Salmon et al., SC'11) and the
                Box-Muller complex Gaussian that feeds the random matrices of
                Alg. 1 step 1 and of Alg. 2.
* ``trees``     bisection cluster trees (Sec. 3.1).
* ``cpqr``      column-pivoted Householder QR with truncation tolerance
                (Alg. 1 step 3).
* ``operators`` the dense / on-the-fly FP64 operators used as black boxes.
* ``butterfly`` Alg. 2 (adaptive randomized hybrid butterfly construction),
                the hybrid butterfly apply (eq. hybrid_butterfly_mat) and an
                independent explicit dense assembly of the factors.
* ``metrics``   eq. (error) of Sec. 6, the bounds of Thms 4.1-4.3, SVD ranks.
"""
