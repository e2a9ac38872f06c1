"""Parity measures between a GPU result and the oracle's (test
infrastructure: the tests, the package smoke check and the benchmark's
CPU-baseline leg use them).

Both measures are taken over a whole template at once, all channels (or
links, or gradient rows) together:

  rel_err  ||got - ref||_2 / ||ref||_2
  max_err  max|got - ref| / max|ref|

The joint normalisation handles T: its norm is ~(omega L)^2 below A and E, so
a per-channel bar on T would be set by the rounding of the orbit splines, not
by the kernels.  max_err catches a single wrong element that the L2 norm
would dilute by the square root of the number of compared values.
"""
from __future__ import annotations

import numpy as np


def _pair(got, ref):
    got = np.atleast_2d(np.asarray(got, dtype=np.float64))
    ref = np.atleast_2d(np.asarray(ref, dtype=np.float64))
    if got.shape != ref.shape:
        raise ValueError("shapes differ: %s vs %s" % (got.shape, ref.shape))
    return got, ref


def rel_err(got, ref):
    """||got - ref||_F / ||ref||_F (NaN anywhere gives NaN)."""
    got, ref = _pair(got, ref)
    return float(np.linalg.norm(got - ref) / max(np.linalg.norm(ref), 1e-300))


def max_err(got, ref):
    """max|got - ref| / max|ref| (NaN anywhere gives NaN)."""
    got, ref = _pair(got, ref)
    d = np.abs(got - ref)
    if not (np.all(np.isfinite(d)) and np.all(np.isfinite(ref))):
        return float("nan")
    return float(d.max(initial=0.0) / max(np.abs(ref).max(initial=0.0), 1e-300))


def errors(got, ref):
    """(rel_err, max_err)."""
    return rel_err(got, ref), max_err(got, ref)


def check(got, ref, tol, what=""):
    """Assert rel_err <= tol and max_err <= tol; returns (rel_err, max_err)."""
    e2, em = errors(got, ref)
    assert e2 <= tol and em <= tol, "%s rel_err %.3e, max_err %.3e > %.1e" % (what, e2, em, tol)
    return e2, em
