"""Element-wise parity check of two fields, shared by the GPU tests.

A relative L2 bound alone averages a defect on a few entries (one wrong grid
line or Nyquist plane) over millions of values; the element-wise bound beside
it, |got - ref| <= 2 tol max|ref| at every entry, catches such a defect."""
import numpy as np


def field_errors(got, ref):
    got = np.ravel(np.asarray(got, dtype=np.float64))
    ref = np.ravel(np.asarray(ref, dtype=np.float64))
    d = got - ref
    scale = max(float(np.max(np.abs(ref))), 1e-300)
    return float(np.linalg.norm(d) / max(np.linalg.norm(ref), 1e-300)), float(np.max(np.abs(d)) / scale)


def assert_fields_close(got, ref, tol, what=""):
    l2, mx = field_errors(got, ref)
    assert l2 <= tol, ("relative L2", l2, tol, what)
    assert mx <= 2 * tol, ("element-wise, relative to max |ref|", mx, 2 * tol, what)
