"""Conversion between the oracle's Factors and the library's canonical factor
layout (pure data reshuffling; used by the parity tests only), and test inputs
that are exact in BF16."""
import numpy as np

from oracle import butterfly as obf


def oracle_to_canonical(F):
    L, lm = F.L, F.lm
    nb = 1 << L
    kU = np.zeros((L - lm + 1, nb), np.int32)
    kV = np.zeros((lm + 1, nb), np.int32)
    for l, d in F.kU.items():
        for (i, j), k in d.items():
            kU[l - lm, (i << (L - l)) + j] = k
    for l, d in F.kV.items():
        for (i, j), k in d.items():
            kV[l, (i << (L - l)) + j] = k
    parts = [u.ravel(order="F") for u in F.U]
    for l in range(L - 1, lm - 1, -1):
        parts += [F.R[l][(i, j)].ravel(order="F") for i in range(1 << l) for j in range(1 << (L - l))]
    parts += [F.B[(i, j)].ravel(order="F") for i in range(1 << lm) for j in range(1 << (L - lm))]
    for l in range(lm, 0, -1):
        parts += [F.W[l][(i, j)].ravel(order="F") for i in range(1 << l) for j in range(1 << (L - l))]
    parts += [v.ravel(order="F") for v in F.V]
    data = np.concatenate(parts) if parts else np.zeros(0, np.complex128)
    return kU, kV, data


def canonical_to_oracle(m, n, L, kU, kV, data, lm=None):
    lm = L // 2 if lm is None else lm
    F = obf.Factors(m, n, L, lm)
    ku = lambda l, i, j: int(kU[l - lm, (i << (L - l)) + j])
    kv = lambda l, i, j: int(kV[l, (i << (L - l)) + j])
    F.kU = {l: {(i, j): ku(l, i, j) for i in range(1 << l) for j in range(1 << (L - l))} for l in range(lm, L + 1)}
    F.kV = {l: {(i, j): kv(l, i, j) for i in range(1 << l) for j in range(1 << (L - l))} for l in range(0, lm + 1)}
    off = 0

    def take(r, c):
        nonlocal off
        blk = data[off:off + r * c].reshape((r, c), order="F")
        off += r * c
        return blk

    F.U = [take(F.trange(L, i)[1] - F.trange(L, i)[0], ku(L, i, 0)) for i in range(1 << L)]
    F.R = {}
    for l in range(L - 1, lm - 1, -1):
        F.R[l] = {(i, j): take(ku(l + 1, 2 * i, j >> 1) + ku(l + 1, 2 * i + 1, j >> 1), ku(l, i, j))
                  for i in range(1 << l) for j in range(1 << (L - l))}
    F.B = {(i, j): take(ku(lm, i, j), kv(lm, i, j)) for i in range(1 << lm) for j in range(1 << (L - lm))}
    F.W = {}
    for l in range(lm, 0, -1):
        F.W[l] = {(i, j): take(kv(l - 1, i >> 1, 2 * j) + kv(l - 1, i >> 1, 2 * j + 1), kv(l, i, j))
                  for i in range(1 << l) for j in range(1 << (L - l))}
    F.V = [take(F.srange(L, j)[1] - F.srange(L, j)[0], kv(0, 0, j)) for j in range(1 << L)]
    assert off == len(data)
    return F


def bf16_exact(X):
    """X with the real and imaginary parts rounded to BF16 by torch's
    float32 -> bfloat16 conversion (round to nearest even): test inputs that
    the split-BF16 products take on their exact-input path."""
    import torch
    re = torch.from_numpy(np.ascontiguousarray(X.real, np.float32)).to(torch.bfloat16).double().numpy()
    im = torch.from_numpy(np.ascontiguousarray(X.imag, np.float32)).to(torch.bfloat16).double().numpy()
    return re + 1j * im
