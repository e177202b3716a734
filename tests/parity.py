"""Comparison helpers of the GPU parity tests.

rel() is the norm-wise metric of the coefficient agreement (reading R20:
||x_gpu - x_ref||_2 / ||x_ref||_2).  assert_coef_close() adds element-wise bounds
beside it, so that a few large coefficients cannot hide a small one that is far
off: every coordinate within tol * ||x_ref||_inf, and every coordinate of the
reference of at least 1 % of ||x_ref||_inf within 10 tol of itself, relative.
(Rounding in FP32 streaming is an absolute error on the scale of the whole
vector, so coordinates far below 1 % of the largest are held by the first bound.)
"""
import numpy as np


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def coef_errors(got, ref):
    """(norm-wise, max-abs / ||ref||_inf, max relative error over the ref entries of at
    least 1 % of ||ref||_inf)."""
    g = np.asarray(got, dtype=np.float64).ravel()
    r = np.asarray(ref, dtype=np.float64).ravel()
    d = np.abs(g - r)
    inf = float(np.max(np.abs(r))) if r.size else 0.0
    nz = (np.abs(r) >= 0.01 * inf) & (r != 0)
    per = float(np.max(d[nz] / np.abs(r[nz]))) if nz.any() else 0.0
    return rel(g, r), (float(np.max(d)) / inf if inf > 0 else float(np.max(d, initial=0.0))), per


def assert_coef_close(got, ref, tol, what="coefficients"):
    nrm, mx, per = coef_errors(got, ref)
    assert nrm <= tol, "%s: norm-wise %.3e > %.1e" % (what, nrm, tol)
    assert mx <= tol, "%s: max |d| / ||ref||_inf %.3e > %.1e" % (what, mx, tol)
    assert per <= 10 * tol, "%s: per-coordinate %.3e > %.1e" % (what, per, 10 * tol)
