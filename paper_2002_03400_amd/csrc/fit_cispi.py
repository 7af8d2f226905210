"""Coefficients of the FP32 sin/cos polynomials in matfree.hip (cis_pi).

sin(pi y) = y (s1 + s3 y^2 + ... + s9 y^8) and
cos(pi y) = 1 + y^2 (c2 + c4 y^2 + ... + c10 y^8) on |y| <= 1/2: minimax fits
(relative error for sin, absolute for cos) solved as linear programs on a
dense grid, rounded to FP32 one coefficient at a time from the lowest order,
each rounding compensated by refitting the higher-order ones.

``python fit_cispi.py`` prints the coefficients as C hex-float literals and
the error of the FP32 evaluation (emulated in numpy, one rounding per FP32
operation) against exp(i theta) in FP64.  ``parse_kernel`` reads the
constants back from matfree.hip so that a test can recheck them.
"""
from __future__ import annotations

import os
import re

import numpy as np

F32 = np.float32
HERE = os.path.dirname(os.path.abspath(__file__))
ROUND = 1.5 * 2.0**52


def _lp_minimax(cols: np.ndarray, f: np.ndarray, wt: np.ndarray) -> tuple[np.ndarray, float]:
    from scipy.optimize import linprog
    sc = np.max(np.abs(cols), 0)
    a = cols / sc * wt[:, None]
    b = f * wt
    n = a.shape[1]
    ones = np.ones((len(b), 1))
    g = np.vstack([np.hstack([a, -ones]), np.hstack([-a, -ones])])
    h = np.concatenate([b, -b])
    c = np.zeros(n + 1)
    c[-1] = 1.0
    r = linprog(c, A_ub=g, b_ub=h, bounds=[(None, None)] * n + [(0, None)], method="highs",
                options={"primal_feasibility_tolerance": 1e-10,
                         "dual_feasibility_tolerance": 1e-10})
    return r.x[:n] / sc, float(r.x[-1])


def _sequential(cols: list[np.ndarray], f: np.ndarray, wt: np.ndarray) -> list[float]:
    out, resid, cols = [], f.copy(), list(cols)
    while cols:
        c, _ = _lp_minimax(np.stack(cols, 1), resid, wt)
        c0 = float(F32(c[0]))
        out.append(c0)
        resid = resid - c0 * cols.pop(0)
    return out


def fit(npts: int = 8000) -> tuple[list[float], list[float]]:
    """(s1, s3, s5, s7, s9), (c2, c4, c6, c8, c10), each exactly an FP32 value."""
    y = np.linspace(1e-7, 0.5, npts)
    w = y * y
    s = np.sin(np.pi * y)
    sin_c = _sequential([y, y**3, y**5, y**7, y**9], s, 1.0 / s)
    cos_c = _sequential([w, w**2, w**3, w**4, w**5], np.cos(np.pi * y) - 1.0, np.ones_like(y))
    return sin_c, cos_c


def parse_kernel(path: str | None = None) -> tuple[list[float], list[float]]:
    """The coefficients as written in cis_pi of matfree.hip."""
    src = open(path or os.path.join(HERE, "matfree.hip")).read()
    body = src[src.index("cf cis_pi("):]
    body = body[:body.index("\n}\n")]
    # the first sp line carries (s9, s7), the others one coefficient each
    sin_lines = re.findall(r"sp = fmaf\(y2, ([^,]+), ([^)]+)\)", body)
    cos_lines = re.findall(r"cp = fmaf\(y2, ([^,]+), ([^)]+)\)", body)

    def coefs(lines):
        vals = []
        for a, b in lines:
            for x in (a, b):
                x = x.strip()
                if x not in ("sp", "cp"):
                    vals.append(float.fromhex(x.rstrip("f")))
        return vals[::-1]   # lowest order first

    return coefs(sin_lines), coefs(cos_lines)


def _fma32(a, b, c):
    return (np.asarray(a, np.float64) * np.asarray(b, np.float64)
            + np.asarray(c, np.float64)).astype(F32)


def emulate(t: np.ndarray, sin_c, cos_c) -> tuple[np.ndarray, np.ndarray]:
    """(cos, sin) of pi t as cis_pi computes them (amp = 1), t in FP64."""
    v = t + ROUND
    y = (t + (ROUND - v)).astype(F32)
    odd = (v.view(np.int64) & 1).astype(bool)
    y2 = (y * y).astype(F32)
    sp = _fma32(y2, F32(sin_c[4]), F32(sin_c[3]))
    for c in sin_c[2::-1]:
        sp = _fma32(y2, sp, F32(c))
    cp = _fma32(y2, F32(cos_c[4]), F32(cos_c[3]))
    for c in cos_c[2::-1]:
        cp = _fma32(y2, cp, F32(c))
    co = _fma32(y2, cp, F32(1.0)).astype(np.float64)
    si = (y * sp).astype(F32).astype(np.float64)
    sg = np.where(odd, -1.0, 1.0)
    return co * sg, si * sg


def errors(sin_c, cos_c, n: int = 2_000_000, theta_max: float = 2e4, seed: int = 1):
    """max and rms of |(cos, sin) - exp(i theta)| over uniform random phases."""
    theta = np.random.default_rng(seed).uniform(0.0, theta_max, n)
    co, si = emulate(theta / np.pi, sin_c, cos_c)
    e = np.hypot(co - np.cos(theta), si - np.sin(theta))
    return float(e.max()), float(np.sqrt(np.mean(e * e)))


def _hex32(x: float) -> str:
    m = float(F32(x)).hex()          # e.g. -0x1.4abbd00000000p+2
    mant, exp = m.split("p")
    mant = mant.rstrip("0")
    if mant.endswith("."):
        mant = mant[:-1]
    return f"{mant}p{exp}f"


if __name__ == "__main__":
    s_c, c_c = fit()
    print("sin s1..s9:", ", ".join(_hex32(x) for x in s_c))
    print("cos c2..c10:", ", ".join(_hex32(x) for x in c_c))
    print("FP32 evaluation error (max, rms): %.3g %.3g" % errors(s_c, c_c))
    ks, kc = parse_kernel()
    print("kernel constants equal the fit:", ks == s_c and kc == c_c)
    print("kernel FP32 evaluation error (max, rms): %.3g %.3g" % errors(ks, kc))
