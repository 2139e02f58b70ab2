"""The parity bar of the GPU tests, shared by every test file.

A float32 result passes against the float64 oracle when
  - its relative L2 error ||got - ref|| / ||ref|| is at most `tol` (1e-5 by default), and
  - no single output is off by more than 20 tol rms(ref), so that a handful of wrong outputs
    (an edge, a tile seam, an exact sample instant) cannot hide under a long pulse's norm.
An all-zero reference must be matched exactly.
"""
import numpy as np

TOL = 1e-5
ELEMENT_FACTOR = 20.0


def rel_l2(a, b):
    a = np.asarray(a, np.complex128)
    b = np.asarray(b, np.complex128)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def check(got, ref, tol=TOL, what=None):
    """Assert the parity bar; return the relative L2 error."""
    got = np.asarray(got, np.complex128)
    ref = np.asarray(ref, np.complex128)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.isfinite(got).all(), (what, "non-finite output")
    err = rel_l2(got, ref)
    assert err <= tol, (what, err)
    if ref.size:
        rms = float(np.sqrt(np.mean(np.abs(ref) ** 2)))
        emax = float(np.max(np.abs(got - ref)))
        assert emax <= ELEMENT_FACTOR * tol * rms, (what, "element-wise", emax, rms)
    return err
