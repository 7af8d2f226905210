"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only builds inputs: point geometries, wavenumbers, the random
test columns of the error metric, and the random factors of an exactly
butterfly-structured matrix.  It holds none of the factorization's arithmetic
(no range finder, no pivoted QR, no butterfly apply); both the oracle and the
HIP path receive what it builds as plain arrays.

Workload recipes (the paper's own operators are not available, so these
synthetic operators of the same geometry class stand in for them):

* Segment pair (the 2D parallel-line geometry of Sec. 6.2: two parallel lines
  of unit length at unit distance).  Targets x_i = ((i+1/2)/m, 0), sources
  y_j = ((j+1/2)/n, 1), kernel exp(i k r)/r with r = |x_i - y_j|.  The
  wavenumber gives ``ppw`` points per wavelength at spacing 1/n:
  k = 2 pi n / ppw.
* Three parallel segments at y = 0, 1, 2 for the composition of two
  oscillatory operators (category (ii) of Sec. 1).
* 1D Fourier integral operator A_jk = exp(2 pi i (x_j xi_k + c(x_j)|xi_k|)),
  x_j = j/n, xi_k = k - n/2, c(x) = (2 + sin 2 pi x)/16 ("low-dimensional
  Fourier operators", Sec. 4.4.1).
* Exact butterfly (Sec. 6.1): random unitary leaf bases and transfer blocks
  and Gaussian centre blocks, all ranks r, leaves of 8 points, n = 2^(L+3).
* Two adjacent unit semi-spheres (the 3D weak-admissibility geometry of
  Sec. 6.3, whose Nystrom meshes are not available): n targets on the upper
  unit hemisphere and n sources on a lower unit hemisphere whose rim lies
  half a point spacing below the first one's.  Points follow an equal-area
  golden-angle spiral (height uniform in (0, 1), azimuth advancing by the
  golden angle from a seeded offset), then are reordered by recursive
  bisection so that the index ranges of the butterfly's binary trees are
  spatial clusters.  Kernel exp(i k r)/r with k = sqrt(pi n / 50), i.e.
  n = 50 k^2 / pi: ten points per wavelength on the hemisphere's area 2 pi.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "SegmentGeometry", "segment_pair", "segment_triple", "fio_params",
    "test_columns", "ExactButterflyFactors", "exact_butterfly_factors",
    "node_range_host", "Request", "poisson_stream", "mixed_stream", "exact_butterfly_canonical",
    "hemisphere_pair", "bisection_order",
]


@dataclass(frozen=True)
class SegmentGeometry:
    """Target points (rows) and source points (columns) of exp(i k r)/r."""
    targets: np.ndarray   # (m, 2) or (m, 3) float64
    sources: np.ndarray   # (n, 2) or (n, 3) float64
    k: float              # wavenumber of exp(i k r)/r
    ppw: float            # points per wavelength at the source spacing


def _line(npts: int, y: float) -> np.ndarray:
    x = (np.arange(npts, dtype=np.float64) + 0.5) / npts
    return np.stack([x, np.full(npts, float(y))], axis=1)


def segment_pair(n: int, ppw: float = 8.0, m: int | None = None,
                 y_target: float = 0.0, y_source: float = 1.0) -> SegmentGeometry:
    """Two parallel unit segments at distance |y_source - y_target|.

    ``k = 2 pi n / ppw`` puts ``ppw`` source points in one wavelength.
    """
    m = n if m is None else m
    k = 2.0 * math.pi * n / ppw
    return SegmentGeometry(_line(m, y_target), _line(n, y_source), k, ppw)


def segment_triple(n: int, ppw: float = 8.0):
    """Three parallel unit segments at y = 0, 1, 2 (same n and wavenumber).

    Returns (A(X0, X1) geometry, A(X1, X2) geometry): the product of the two
    kernels maps sources on y=2 to targets on y=0 through y=1.
    """
    g01 = segment_pair(n, ppw, y_target=0.0, y_source=1.0)
    g12 = segment_pair(n, ppw, y_target=1.0, y_source=2.0)
    return g01, g12


def bisection_order(pts: np.ndarray, depth: int) -> np.ndarray:
    """Permutation that makes every node range [floor(i N / 2^l),
    floor((i+1) N / 2^l)), l <= depth, a spatial cluster: each node is split
    at its children's boundary floor((2i+1) N / 2^(l+1)) along the axis of
    its largest extent (stable sort, so the order is deterministic)."""
    N = len(pts)
    perm = np.arange(N)
    for l in range(depth):
        for i in range(1 << l):
            a, b = (i * N) >> l, ((i + 1) * N) >> l
            if b - a < 2:
                continue
            idx = perm[a:b]
            p = pts[idx]
            ax = int(np.argmax(p.max(axis=0) - p.min(axis=0)))
            perm[a:b] = idx[np.argsort(p[:, ax], kind="stable")]
    return perm


def _hemisphere(n: int, phase: float, sign: float, dz: float) -> np.ndarray:
    z = (np.arange(n, dtype=np.float64) + 0.5) / n
    phi = phase + np.arange(n, dtype=np.float64) * (math.pi * (3.0 - math.sqrt(5.0)))
    rho = np.sqrt(1.0 - z * z)
    return np.stack([rho * np.cos(phi), rho * np.sin(phi), sign * z + dz], axis=1)


def hemisphere_pair(n: int, seed: int = 0, ppw: float = 10.0, depth: int | None = None,
                    m: int | None = None) -> SegmentGeometry:
    """Two adjacent unit semi-spheres (3D, weak admissibility), see the module
    docstring.  ``depth`` bisection levels (default: down to about 8 points
    per node); ``ppw`` points per wavelength (10 gives k = sqrt(pi n / 50))."""
    m = n if m is None else m
    rng = np.random.default_rng(seed)
    ph = rng.uniform(0.0, 2.0 * math.pi, 2)
    h = math.sqrt(2.0 * math.pi / n)                 # mean spacing of the sources
    t = _hemisphere(m, ph[0], +1.0, 0.0)
    s = _hemisphere(n, ph[1], -1.0, -0.5 * h)
    if depth is None:
        depth = max(0, int(math.ceil(math.log2(max(m, n) / 8.0))))
    t = t[bisection_order(t, depth)]
    s = s[bisection_order(s, depth)]
    k = 2.0 * math.pi / (ppw * h)
    return SegmentGeometry(np.ascontiguousarray(t), np.ascontiguousarray(s), k, ppw)


def fio_params(n: int):
    """Sample points x_j = j/n and frequencies xi_k = k - n/2 (integers)."""
    if n % 2:
        raise ValueError("FIO workload needs even n")
    x = np.arange(n, dtype=np.float64) / n
    xi = np.arange(n, dtype=np.int64) - n // 2
    return x, xi


def test_columns(n: int, ncols: int = 16, seed: int = 1001) -> np.ndarray:
    """Gaussian complex test matrix of the error metric (Sec. 6, 16 columns)."""
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, ncols)) + 1j * rng.standard_normal((n, ncols))
    return (z / math.sqrt(2.0)).astype(np.complex128)


def node_range_host(npts: int, level: int, idx: int) -> tuple[int, int]:
    """Index range of node ``idx`` at ``level`` of a bisection tree over
    ``npts`` sorted points: [floor(idx*N/2^l), floor((idx+1)*N/2^l))."""
    return (idx * npts) >> level, ((idx + 1) * npts) >> level


@dataclass
class ExactButterflyFactors:
    """Random factors of an L-level hybrid butterfly with all ranks r.

    Block (l, i, j): T-node i at T-level l, S-node j at S-level L-l.
    U[i]: (leaf, r) for leaves of the T-tree; V[j]: (leaf, r) for leaves of
    the S-tree; R[l][(i, j)] (l_m <= l < L): (2r, r); W[l][(i, j)]
    (1 <= l <= l_m): (2r, r); B[(i, j)] at l_m: (r, r).
    """
    L: int
    r: int
    n: int
    U: list
    V: list
    R: dict
    W: dict
    B: dict


def _unitary(rng, rows, cols):
    z = rng.standard_normal((rows, cols)) + 1j * rng.standard_normal((rows, cols))
    q, _ = np.linalg.qr(z)
    return q[:, :cols]


def exact_butterfly_factors(L: int, r: int, seed: int = 7, leaf: int = 8) -> ExactButterflyFactors:
    """Random exact butterfly of Sec. 6.1 (n = leaf * 2^L, every rank = r)."""
    if r > leaf:
        raise ValueError("rank cannot exceed the leaf size")
    rng = np.random.default_rng(seed)
    n = leaf << L
    lm = L // 2
    U = [_unitary(rng, leaf, r) for _ in range(1 << L)]
    V = [_unitary(rng, leaf, r) for _ in range(1 << L)]
    R = {l: {(i, j): _unitary(rng, 2 * r, r)
             for i in range(1 << l) for j in range(1 << (L - l))}
         for l in range(lm, L)}
    W = {l: {(i, j): _unitary(rng, 2 * r, r)
             for i in range(1 << l) for j in range(1 << (L - l))}
         for l in range(1, lm + 1)}
    B = {(i, j): (rng.standard_normal((r, r)) + 1j * rng.standard_normal((r, r))) / math.sqrt(2)
         for i in range(1 << lm) for j in range(1 << (L - lm))}
    return ExactButterflyFactors(L, r, n, U, V, R, W, B)


def _unitary_batch(rng, count, rows, cols):
    z = rng.standard_normal((count, rows, cols)) + 1j * rng.standard_normal((count, rows, cols))
    q, _ = np.linalg.qr(z)
    return q[:, :, :cols]


def exact_butterfly_canonical(L: int, r: int, seed: int = 7, leaf: int = 8):
    """Random exact butterfly of Sec. 6.1 at scale (n = leaf * 2^L, every rank
    r), drawn level by level with batched QR and laid out directly in the
    library's canonical factor order: U (leaf x r per leaf), R^{L-1..lm}
    (2r x r), B (r x r), W^{lm..1} (2r x r), V (leaf x r), each block column-
    major, blocks of a level in the order i * 2^(L-l) + j.  Returns (kU, kV,
    data) with kU of shape (L - lm + 1, 2^L) and kV of shape (lm + 1, 2^L).
    A different draw than exact_butterfly_factors (batched), same law."""
    if r > leaf:
        raise ValueError("rank cannot exceed the leaf size")
    rng = np.random.default_rng(seed)
    nb = 1 << L
    lm = L // 2
    parts = []
    colmajor = lambda a: np.ascontiguousarray(np.transpose(a, (0, 2, 1))).ravel()
    parts.append(colmajor(_unitary_batch(rng, nb, leaf, r)))                 # U
    for _ in range(L - 1, lm - 1, -1):
        parts.append(colmajor(_unitary_batch(rng, nb, 2 * r, r)))            # R^l
    b = (rng.standard_normal((nb, r, r)) + 1j * rng.standard_normal((nb, r, r))) / math.sqrt(2)
    parts.append(colmajor(b))                                                # B
    for _ in range(lm, 0, -1):
        parts.append(colmajor(_unitary_batch(rng, nb, 2 * r, r)))            # W^l
    parts.append(colmajor(_unitary_batch(rng, nb, leaf, r)))                 # V
    kU = np.full((L - lm + 1, nb), r, np.int32)
    kV = np.full((lm + 1, nb), r, np.int32)
    return kU, kV, np.concatenate(parts).astype(np.complex128)


@dataclass
class Request:
    """One request of a synthetic serving stream."""
    t: float            # arrival time (s) after the stream starts
    kind: str           # "construct" or "apply"
    n: int = 0          # construct: problem size (m = n)
    ppw: float = 8.0    # construct: points per wavelength
    tol: float = 1e-6   # construct: truncation tolerance
    seed: int = 0       # construct: key of its random matrices
    nrhs: int = 0       # apply: right-hand sides
    target: int = -1    # apply: index (in the stream) of the construction it uses


def poisson_stream(nreq: int, rate: float, seed: int = 4242, n: int = 65536, ppw: float = 8.0,
                   tol: float = 2e-7) -> list:
    """Constructions of one fixed size arriving as a Poisson process."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, nreq))
    return [Request(float(t[i]), "construct", n, ppw, tol, 3 + i) for i in range(nreq)]


def mixed_stream(nreq: int = 256, rate: float = 20.0, seed: int = 4242, nmin: int = 2048,
                 nmax: int = 65536, tols=(1e-4, 1e-6), frac_construct: float = 0.7) -> list:
    """Serving mix: Poisson arrivals; 70% constructions with n log-uniform in
    [nmin, nmax], 4..16 points per wavelength and a tolerance drawn from
    `tols`; 30% applies of 1..64 right-hand sides against a construction that
    arrived earlier (uniformly chosen)."""
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, nreq))
    out, built = [], []
    for i in range(nreq):
        if not built or rng.uniform() < frac_construct:
            n = int(round(math.exp(rng.uniform(math.log(nmin), math.log(nmax)))))
            out.append(Request(float(t[i]), "construct", n, float(rng.uniform(4.0, 16.0)),
                               float(tols[int(rng.integers(len(tols)))]), 100 + i))
            built.append(i)
        else:
            out.append(Request(float(t[i]), "apply", nrhs=int(rng.integers(1, 65)),
                               target=int(built[int(rng.integers(len(built)))])))
    return out
