"""Alg. 2 (adaptive randomized hybrid butterfly), its apply, and an explicit
dense assembly of the factors.  numpy complex128, one Python loop per sample
and per block.

Notation (Sec. 3): A = K(T, S) is m x n; rows are the targets T (tree T_T),
columns the sources S (tree T_S); both trees have depth L and l_m = floor(L/2).
A block at level l is (tau, nu) = (T-node (l, i), S-node (L-l, j)), written
(l, i, j); the 2^L blocks of a level tile A (Sec. 3.3.3).

Factors of eq. (hybrid_butterfly_mat), A ~ (U^L R^{L-1} .. R^{l_m}) B^{l_m}
(W^{l_m} .. W^1 V^0):

* U[i]            leaf column basis U_{tau,s} of block (L, i, 0), m_i x kU
* R[l][(i, j)]    transfer of eq. (nested_basis), l_m <= l < L:
                  rows kU(l+1, 2i, j>>1) + kU(l+1, 2i+1, j>>1), cols kU(l, i, j)
* B[(i, j)]       centre block at l_m, kU(l_m, i, j) x kV(l_m, i, j)
* W[l][(i, j)]    transfer of eq. (nested_basis_col), 1 <= l <= l_m:
                  rows kV(l-1, i>>1, 2j) + kV(l-1, i>>1, 2j+1), cols kV(l, i, j)
* V[j]            leaf row basis V_{t,nu} of block (0, 0, j), n_j x kV

Readings of the paper taken here (each also binds the HIP path):
* transposes become conjugate transposes and the second black box is A^H;
* Alg. 1's tolerance is the relative Frobenius tail on the sample;
* adaptive loops (Alg. 2, first two loops): draw a fresh random matrix each
  pass, stop without doubling once r > max rank, and restart the U loop from
  r = r0;
* the R-sweep comment "tau at level L-l" is read as tau at level l;
* the printed formula eq. (Bij) is read from its argmin:
  B = (U^H K Omega) (V^H Omega)^+, with U^H K Omega = R^H Z;
* at l = l_m the sample width also covers the V-side ranks so that V^H Omega
  has full row rank: s = max(max_i(kU1 + kU2), max_i kV) + p;
* sample widths are per sample (the r of each Gamma_tau / Omega_nu).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import philox
from .cpqr import range_basis
from .trees import center_level, node_range, num_levels


class RankCapExceeded(RuntimeError):
    pass


@dataclass
class Factors:
    m: int
    n: int
    L: int
    lm: int
    U: list = field(default_factory=list)
    R: dict = field(default_factory=dict)
    B: dict = field(default_factory=dict)
    W: dict = field(default_factory=dict)
    V: list = field(default_factory=list)
    kU: dict = field(default_factory=dict)   # kU[l][(i, j)], l_m <= l <= L
    kV: dict = field(default_factory=dict)   # kV[l][(i, j)], 0 <= l <= l_m
    stats: dict = field(default_factory=dict)

    def trange(self, l, i):
        return node_range(self.m, l, i)

    def srange(self, l, j):
        return node_range(self.n, l, j)

    def max_rank(self):
        ks = [k for d in self.kU.values() for k in d.values()]
        ks += [k for d in self.kV.values() for k in d.values()]
        return max(ks) if ks else 0

    def num_entries(self):
        tot = sum(u.size for u in self.U) + sum(v.size for v in self.V)
        tot += sum(b.size for b in self.B.values())
        tot += sum(x.size for d in self.R.values() for x in d.values())
        tot += sum(x.size for d in self.W.values() for x in d.values())
        return tot


def _H(a):
    return a.conj().T


# ---------------------------------------------------------------- Alg. 2 --

def construct(op, tol, leaf, p=2, r0=4, seed=0, max_rank=None, lm=None, rule="fro") -> Factors:
    """Alg. 2.  ``op`` has ``m, n, matvec(X, support), rmatvec(X, support)``.

    ``lm`` is the level of the centre factor B (eq. hybrid_butterfly_mat);
    default floor(L/2), the hybrid factorization of Sec. 3.3.3.  lm = 0 gives
    the column-wise factorization of Sec. 3.3.1 (E^0 = B^0 V^0) and lm = L
    the row-wise one of Sec. 3.3.2 (F^L = U^L B^L), the variants Sec. 4 says
    the same algorithm builds at a higher cost.  Negative lm counts from
    L + 1 (-1 is L).

    ``rule`` is the truncation rule of Alg. 1 (``cpqr.cpqr_truncated``):
    "fro", the relative Frobenius tail of the sample (the reading used
    throughout), or "diag", |R_kk| <= eps |R_11|, a diagnostic only."""
    m, n = op.m, op.n
    if m <= 0 or n <= 0:
        raise ValueError("empty operator")
    if not (0.0 < tol < 1.0):
        raise ValueError("tol must lie in (0, 1)")
    L = num_levels(m, n, leaf)
    if lm is None:
        lm = center_level(L)
    elif lm < 0:
        lm += L + 1
    if not 0 <= lm <= L:
        raise ValueError(f"centre level {lm} outside [0, {L}]")
    F = Factors(m, n, L, lm)
    F.kU = {l: {} for l in range(lm, L + 1)}
    F.kV = {l: {} for l in range(0, lm + 1)}
    F.R = {l: {} for l in range(lm, L)}
    F.W = {l: {} for l in range(1, lm + 1)}
    cols = {"matvec": 0, "rmatvec": 0, "v_iters": 0, "u_iters": 0}

    def cap(r):
        if max_rank is not None and r > max_rank:
            raise RankCapExceeded(f"rank estimate {r} exceeds cap {max_rank}")

    # -- adaptive leaf row bases V_{t,nu}: loop "Adaptive computation of V" --
    r, it = r0, 0
    while True:
        cap(r)
        s = r + p
        G = philox.gaussian_block(seed, philox.tag(philox.PHASE_V0, it, 0), 0, m, s)
        Yp = op.rmatvec(G)
        cols["rmatvec"] += s
        F.V = []
        for j in range(1 << L):
            lo, hi = F.srange(L, j)
            Q, k = range_basis(Yp[lo:hi], tol, rule)
            F.V.append(Q)
            F.kV[0][(0, j)] = k
        cols["v_iters"] += 1
        if r > max(F.kV[0].values()):
            break
        r *= 2
        it += 1

    # -- adaptive leaf column bases U_{tau,s}: loop "Adaptive computation of U"
    r, it = r0, 0
    while True:
        cap(r)
        s = r + p
        Om = philox.gaussian_block(seed, philox.tag(philox.PHASE_U0, it, 0), 0, n, s)
        Y = op.matvec(Om)
        cols["matvec"] += s
        F.U = []
        for i in range(1 << L):
            lo, hi = F.trange(L, i)
            Q, k = range_basis(Y[lo:hi], tol, rule)
            F.U.append(Q)
            F.kU[L][(i, 0)] = k
        cols["u_iters"] += 1
        if r > max(F.kU[L].values()):
            break
        r *= 2
        it += 1

    # -- W sweep, l = 1 .. l_m (Sec. 4.3) --
    for l in range(1, lm + 1):
        for i in range(1 << l):
            s = max(F.kV[l - 1][(i >> 1, 2 * j)] + F.kV[l - 1][(i >> 1, 2 * j + 1)]
                    for j in range(1 << (L - l))) + p
            lo, hi = F.trange(l, i)
            G = np.zeros((m, s), np.complex128)
            G[lo:hi] = philox.gaussian_block(seed, philox.tag(philox.PHASE_W, l, i), lo, hi - lo, s)
            Yp = op.rmatvec(G, support=(lo, hi))
            cols["rmatvec"] += s
            # V-chain^H: V^0 then W^1 .. W^{l-1} on the T-ancestors of tau
            P = [_H(F.V[jj]) @ Yp[slice(*F.srange(L, jj))] for jj in range(1 << L)]
            for lp in range(1, l):
                ip = i >> (l - lp)
                P = [_H(F.W[lp][(ip, jj)]) @ np.vstack([P[2 * jj], P[2 * jj + 1]])
                     for jj in range(1 << (L - lp))]
            for j in range(1 << (L - l)):
                Z = np.vstack([P[2 * j], P[2 * j + 1]])
                Q, k = range_basis(Z, tol, rule)
                F.W[l][(i, j)] = Q
                F.kV[l][(i, j)] = k

    # -- R sweep, l = L-1 .. l_m, and B at l_m (Secs. 4.2, 4.4) --
    for l in range(L - 1, lm - 1, -1):
        for j in range(1 << (L - l)):
            s = max(F.kU[l + 1][(2 * i, j >> 1)] + F.kU[l + 1][(2 * i + 1, j >> 1)]
                    for i in range(1 << l))
            if l == lm:
                s = max(s, max(F.kV[lm][(i, j)] for i in range(1 << lm)))
            s += p
            lo, hi = F.srange(L - l, j)
            Om = np.zeros((n, s), np.complex128)
            Om[lo:hi] = philox.gaussian_block(seed, philox.tag(philox.PHASE_R, l, j), lo, hi - lo, s)
            Y = op.matvec(Om, support=(lo, hi))
            cols["matvec"] += s
            # U-chain^H: U^L then R^{L-1} .. R^{l+1} on the S-ancestors of nu
            P = [_H(F.U[ii]) @ Y[slice(*F.trange(L, ii))] for ii in range(1 << L)]
            for lp in range(L - 1, l, -1):
                jp = j >> (lp - l)
                P = [_H(F.R[lp][(ii, jp)]) @ np.vstack([P[2 * ii], P[2 * ii + 1]])
                     for ii in range(1 << lp)]
            Zs = []
            for i in range(1 << l):
                Z = np.vstack([P[2 * i], P[2 * i + 1]])
                Q, k = range_basis(Z, tol, rule)
                F.R[l][(i, j)] = Q
                F.kU[l][(i, j)] = k
                Zs.append(Z)
            if l == lm:
                X = _x_chain(F, Om, j)
                for i in range(1 << lm):
                    C = _H(F.R[lm][(i, j)]) @ Zs[i]
                    F.B[(i, j)] = _lstsq_right(C, X[i])

    if lm == L:
        # centre at the row leaves (the row-wise factorization, and L = 0):
        # B_{i,0} = (U_i^H A Omega)(V_{i,0}^H Omega)^+ with the leaf column
        # bases themselves (no R level) and the full-height row bases
        s = max(max(F.kU[L][(i, 0)], F.kV[L][(i, 0)]) for i in range(1 << L)) + p
        Om = philox.gaussian_block(seed, philox.tag(philox.PHASE_R, L, 0), 0, n, s)
        Y = op.matvec(Om)
        cols["matvec"] += s
        X = _x_chain(F, Om, 0)
        for i in range(1 << L):
            C = _H(F.U[i]) @ Y[slice(*F.trange(L, i))]
            F.B[(i, 0)] = _lstsq_right(C, X[i])

    F.stats = cols
    return F


def _x_chain(F: Factors, Om, j):
    """X_{l_m,i,j} = V_{tau,nu}^H Omega_nu for every tau at l_m (line
    "Compute V^T Omega if l = l_m"), by the nested row bases: V^0 on the
    leaves under nu, then W^1 .. W^{l_m} restricted to nu's subtree."""
    L, lm = F.L, F.lm
    Q = {}
    for jj in range(j << lm, (j + 1) << lm):
        Q[(0, jj)] = _H(F.V[jj]) @ Om[slice(*F.srange(L, jj))]
    for lp in range(1, lm + 1):
        Qn = {}
        for ii in range(1 << lp):
            for jj in range(j << (lm - lp), (j + 1) << (lm - lp)):
                inp = np.vstack([Q[(ii >> 1, 2 * jj)], Q[(ii >> 1, 2 * jj + 1)]])
                Qn[(ii, jj)] = _H(F.W[lp][(ii, jj)]) @ inp
        Q = Qn
    return [Q[(i, j)] for i in range(1 << lm)]


def _lstsq_right(C, X):
    """argmin_B ||C - B X||_F (eq. Bij read from its argmin), via lstsq on X^H."""
    if C.shape[0] == 0 or X.shape[0] == 0:
        return np.zeros((C.shape[0], X.shape[0]), np.complex128)
    sol = np.linalg.lstsq(_H(X), _H(C), rcond=None)[0]
    return _H(sol)


# ---------------------------------------------------------------- apply --

def apply(F: Factors, X: np.ndarray) -> np.ndarray:
    """Y = F X through the factors of eq. (hybrid_butterfly_mat), right to left."""
    L, lm = F.L, F.lm
    X = np.asarray(X, np.complex128)
    c = X.shape[1]
    t = {(0, j): _H(F.V[j]) @ X[slice(*F.srange(L, j))] for j in range(1 << L)}
    for l in range(1, lm + 1):
        t = {(i, j): _H(F.W[l][(i, j)]) @ np.vstack([t[(i >> 1, 2 * j)], t[(i >> 1, 2 * j + 1)]])
             for i in range(1 << l) for j in range(1 << (L - l))}
    u = {key: F.B[key] @ t[key] for key in t}
    for l in range(lm, L):
        un = {(i, j): np.zeros((F.kU[l + 1][(i, j)], c), np.complex128)
              for i in range(1 << (l + 1)) for j in range(1 << (L - l - 1))}
        for (i, j), v in u.items():
            k1 = F.kU[l + 1][(2 * i, j >> 1)]
            w = F.R[l][(i, j)] @ v
            un[(2 * i, j >> 1)] += w[:k1]
            un[(2 * i + 1, j >> 1)] += w[k1:]
        u = un
    Y = np.zeros((F.m, c), np.complex128)
    for i in range(1 << L):
        Y[slice(*F.trange(L, i))] = F.U[i] @ u[(i, 0)]
    return Y


def apply_adjoint(F: Factors, X: np.ndarray) -> np.ndarray:
    """Y = F^H X: the conjugate-transposed stages in reverse order."""
    L, lm = F.L, F.lm
    X = np.asarray(X, np.complex128)
    c = X.shape[1]
    u = {(i, 0): _H(F.U[i]) @ X[slice(*F.trange(L, i))] for i in range(1 << L)}
    for l in range(L - 1, lm - 1, -1):
        u = {(i, j): _H(F.R[l][(i, j)]) @ np.vstack([u[(2 * i, j >> 1)], u[(2 * i + 1, j >> 1)]])
             for i in range(1 << l) for j in range(1 << (L - l))}
    t = {key: _H(F.B[key]) @ u[key] for key in u}
    for l in range(lm, 0, -1):
        tn = {(i, j): np.zeros((F.kV[l - 1][(i, j)], c), np.complex128)
              for i in range(1 << (l - 1)) for j in range(1 << (L - l + 1))}
        for (i, j), v in t.items():
            ka = F.kV[l - 1][(i >> 1, 2 * j)]
            w = F.W[l][(i, j)] @ v
            tn[(i >> 1, 2 * j)] += w[:ka]
            tn[(i >> 1, 2 * j + 1)] += w[ka:]
        t = tn
    Y = np.zeros((F.n, c), np.complex128)
    for j in range(1 << L):
        Y[slice(*F.srange(L, j))] = F.V[j] @ t[(0, j)]
    return Y


# ------------------------------------------------------- dense assembly --

def _offsets(kd, keys):
    off, o = {}, 0
    for key in keys:
        off[key] = o
        o += kd[key]
    return off, o


def factor_matrices(F: Factors):
    """The sparse factors of eq. (hybrid_butterfly_mat) as explicit dense
    matrices, in product order [U^L, R^{L-1}, .., R^{l_m}, B, W^{l_m}, .., W^1, V^0].
    Built block by block from the index maps, without the apply's loops."""
    L, lm = F.L, F.lm
    keysU = {l: [(i, j) for i in range(1 << l) for j in range(1 << (L - l))] for l in F.kU}
    keysV = {l: [(i, j) for i in range(1 << l) for j in range(1 << (L - l))] for l in F.kV}
    offU = {l: _offsets(F.kU[l], keysU[l]) for l in F.kU}
    offV = {l: _offsets(F.kV[l], keysV[l]) for l in F.kV}
    mats = []
    o, tot = offU[L]
    UL = np.zeros((F.m, tot), np.complex128)
    for i in range(1 << L):
        lo, hi = F.trange(L, i)
        UL[lo:hi, o[(i, 0)]:o[(i, 0)] + F.kU[L][(i, 0)]] = F.U[i]
    mats.append(UL)
    for l in range(L - 1, lm - 1, -1):
        orow, nrow = offU[l + 1]
        ocol, ncol = offU[l]
        M = np.zeros((nrow, ncol), np.complex128)
        for (i, j) in keysU[l]:
            Rb = F.R[l][(i, j)]
            k1 = F.kU[l + 1][(2 * i, j >> 1)]
            c0 = ocol[(i, j)]
            r1 = orow[(2 * i, j >> 1)]
            r2 = orow[(2 * i + 1, j >> 1)]
            M[r1:r1 + k1, c0:c0 + Rb.shape[1]] = Rb[:k1]
            M[r2:r2 + Rb.shape[0] - k1, c0:c0 + Rb.shape[1]] = Rb[k1:]
        mats.append(M)
    orow, nrow = offU[lm]
    ocol, ncol = offV[lm]
    Bm = np.zeros((nrow, ncol), np.complex128)
    for key in keysU[lm]:
        b = F.B[key]
        Bm[orow[key]:orow[key] + b.shape[0], ocol[key]:ocol[key] + b.shape[1]] = b
    mats.append(Bm)
    for l in range(lm, 0, -1):
        orow, nrow = offV[l]
        ocol, ncol = offV[l - 1]
        M = np.zeros((nrow, ncol), np.complex128)
        for (i, j) in keysV[l]:
            Wh = _H(F.W[l][(i, j)])
            ka = F.kV[l - 1][(i >> 1, 2 * j)]
            r0 = orow[(i, j)]
            ca = ocol[(i >> 1, 2 * j)]
            cb = ocol[(i >> 1, 2 * j + 1)]
            M[r0:r0 + Wh.shape[0], ca:ca + ka] = Wh[:, :ka]
            M[r0:r0 + Wh.shape[0], cb:cb + Wh.shape[1] - ka] = Wh[:, ka:]
        mats.append(M)
    o, tot = offV[0]
    V0 = np.zeros((tot, F.n), np.complex128)
    for j in range(1 << L):
        lo, hi = F.srange(L, j)
        V0[o[(0, j)]:o[(0, j)] + F.kV[0][(0, j)], lo:hi] = _H(F.V[j])
    mats.append(V0)
    return mats


def dense(F: Factors) -> np.ndarray:
    mats = factor_matrices(F)
    out = mats[0]
    for Mx in mats[1:]:
        out = out @ Mx
    return out


# ------------------------------------------------- explicit nested bases --

def column_bases(F: Factors):
    """U_{tau,nu} of every block at levels l_m..L, expanded by eq. (nested_basis)."""
    L, lm = F.L, F.lm
    U = {L: {(i, 0): F.U[i] for i in range(1 << L)}}
    for l in range(L - 1, lm - 1, -1):
        U[l] = {}
        for i in range(1 << l):
            for j in range(1 << (L - l)):
                a = U[l + 1][(2 * i, j >> 1)]
                b = U[l + 1][(2 * i + 1, j >> 1)]
                D = np.zeros((a.shape[0] + b.shape[0], a.shape[1] + b.shape[1]), np.complex128)
                D[:a.shape[0], :a.shape[1]] = a
                D[a.shape[0]:, a.shape[1]:] = b
                U[l][(i, j)] = D @ F.R[l][(i, j)]
    return U


def row_bases(F: Factors):
    """V_{tau,nu} of every block at levels 0..l_m, expanded by eq. (nested_basis_col)."""
    L, lm = F.L, F.lm
    V = {0: {(0, j): F.V[j] for j in range(1 << L)}}
    for l in range(1, lm + 1):
        V[l] = {}
        for i in range(1 << l):
            for j in range(1 << (L - l)):
                a = V[l - 1][(i >> 1, 2 * j)]
                b = V[l - 1][(i >> 1, 2 * j + 1)]
                D = np.zeros((a.shape[0] + b.shape[0], a.shape[1] + b.shape[1]), np.complex128)
                D[:a.shape[0], :a.shape[1]] = a
                D[a.shape[0]:, a.shape[1]:] = b
                V[l][(i, j)] = D @ F.W[l][(i, j)]
    return V


def from_exact(fx, m=None, n=None) -> Factors:
    """Wrap the random factors of an exact butterfly (workloads) as Factors."""
    L = fx.L
    lm = L // 2
    m = fx.n if m is None else m
    n = fx.n if n is None else n
    F = Factors(m, n, L, lm)
    F.U, F.V = list(fx.U), list(fx.V)
    F.R = {l: dict(d) for l, d in fx.R.items()}
    F.W = {l: dict(d) for l, d in fx.W.items()}
    F.B = dict(fx.B)
    F.kU = {l: {(i, j): fx.r for i in range(1 << l) for j in range(1 << (L - l))}
            for l in range(lm, L + 1)}
    F.kV = {l: {(i, j): fx.r for i in range(1 << l) for j in range(1 << (L - l))}
            for l in range(0, lm + 1)}
    return F


class FactorsOp:
    """A built butterfly used as a black box (e.g. the exact butterfly of
    Sec. 6.1, or a factor of a composition)."""

    def __init__(self, F: Factors):
        self.F = F
        self.m, self.n = F.m, F.n

    def matvec(self, X, support=None):
        return apply(self.F, X)

    def rmatvec(self, X, support=None):
        return apply_adjoint(self.F, X)
