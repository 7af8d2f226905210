"""The FP32 sin/cos polynomials of the matrix-free entry evaluation (cis_pi
in csrc/matfree.hip): the constants written in the kernel are the ones the
committed fit produces, and their FP32 evaluation (emulated with one rounding
per operation) stays within the error the kernel's comment states."""
import importlib.util
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_spec = importlib.util.spec_from_file_location(
    "fit_cispi", os.path.join(HERE, "..", "paper_2002_03400_amd", "csrc", "fit_cispi.py"))
fit_cispi = importlib.util.module_from_spec(_spec)
_spec.loader.exec_module(fit_cispi)


def test_kernel_constants_are_the_fit():
    s, c = fit_cispi.parse_kernel()
    assert len(s) == 5 and len(c) == 5
    assert (s, c) == fit_cispi.fit()
    # leading terms: pi and -pi^2 / 2 rounded to FP32
    assert s[0] == float(np.float32(np.pi))
    assert abs(c[0] + np.pi**2 / 2) < 1e-6


def test_fp32_evaluation_error():
    s, c = fit_cispi.parse_kernel()
    emax, erms = fit_cispi.errors(s, c, n=500_000)
    assert emax < 2e-7 and erms < 5e-8


def test_exact_points_and_symmetry():
    s, c = fit_cispi.parse_kernel()
    # integer half revolutions give exactly (+-1, 0); quarter turns (0, +-1) up to the fit
    t = np.array([0.0, 1.0, 2.0, -3.0, 1e6 + 1.0])
    co, si = fit_cispi.emulate(t, s, c)
    assert np.array_equal(co, [1.0, -1.0, 1.0, -1.0, -1.0]) and np.all(si == 0.0)
    co, si = fit_cispi.emulate(np.array([0.5, -0.5, 1.5]), s, c)
    assert np.allclose(si, [1.0, -1.0, -1.0], atol=1e-7) and np.all(np.abs(co) < 1e-7)
    # the negated phase is exactly the conjugate (ties to even on both sides)
    t = np.random.default_rng(0).uniform(-1e4, 1e4, 100_000)
    t[:4] = [0.5, 2.5, -0.5, 7.5]
    co1, si1 = fit_cispi.emulate(t, s, c)
    co2, si2 = fit_cispi.emulate(-t, s, c)
    assert np.array_equal(co1, co2) and np.array_equal(si1, -si2)
