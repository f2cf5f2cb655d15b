"""Parity checks shared by the GPU tests: a GPU field against the FP64 oracle's.

Two bounds, both stated against the oracle's field `want`:
  - relative L2:   ||got - want||_2 / ||want||_2 <= tol      (the stated FP32 tolerance, 1e-5);
  - per element:   max |got - want| <= elem * max |want|     (localises an error that a global norm
                                                               averages away, e.g. one ragged tile).
FP32 accumulation of at most a few thousand terms per coefficient keeps each element within a few
1e-7 of the field's peak, so elem = 1e-5 leaves a wide margin while any misplaced or dropped
coefficient (of order the peak / sqrt(points)) fails it.
"""
import numpy as np

TOL = 1e-5
ELEM = 1e-5


def rel_l2(got, want):
    want = np.asarray(want, np.complex128)
    got = np.asarray(got, np.complex128)
    return float(np.linalg.norm((got - want).ravel()) / max(np.linalg.norm(want.ravel()), 1e-300))


def max_elem(got, want):
    """max |got - want| / max |want|."""
    want = np.asarray(want, np.complex128)
    got = np.asarray(got, np.complex128)
    return float(np.max(np.abs(got - want)) / max(np.max(np.abs(want)), 1e-300))


def assert_field(got, want, tol=TOL, elem=ELEM, what=""):
    got = np.asarray(got)
    want = np.asarray(want)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    r, e = rel_l2(got, want), max_elem(got, want)
    assert r <= tol and e <= elem, "%s: rel-L2 %.3e (<= %.0e), max element %.3e of peak (<= %.0e)" % (
        what, r, tol, e, elem)
    return r, e
