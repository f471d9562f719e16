"""Tolerance gates for binary32 GPU results against the FP64 oracle.

The method's floating-point result is the FP64 sum of Algorithm 1; a binary32
sum in any channel order differs from it by rounding only.  Outputs cross
zero, so an element-by-element relative error is ill-posed; the gates are

  normwise        max|y - r| / max|r|                      <= 1e-5
  componentwise   |y - r| <= 1e-5 * sum_ch |x[ch][t + delay]|   for every output

(1e-5 is the stated maximum relative error for binary32 input.  A
sequential binary32 sum of C terms errs by at most (C-1) * 2^-24 * sum|x|
in the worst case and by ~sqrt(C) * 2^-24 * sum|x| typically, i.e. ~2e-6 at
C = 1,024.)  Integer-valued inputs are summed exactly in binary32 and must
match bit for bit.

Passing ``report="<configuration>"`` also records the measured errors (see
tests/errors.py) for the per-configuration error table.
"""
from __future__ import annotations

import numpy as np

from tests import errors

REL = 1e-5


def measure(y, ref, abs_ref):
    """(normwise, componentwise, elementwise) errors of y against ref:
    max|y-r|/max|r|, max |y-r|/sum|x| over outputs with a nonzero bound, and
    max |y-r|/|r| over outputs with |r| >= 1e-3 max|r|."""
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    abs_ref = np.asarray(abs_ref, dtype=np.float64)
    err = np.abs(y - ref)
    if err.size == 0:
        return 0.0, 0.0, 0.0
    rmax = float(np.max(np.abs(ref)))
    normwise = float(err.max()) / max(rmax, 1e-300)
    nz = abs_ref > 0
    comp = float((err[nz] / abs_ref[nz]).max()) if np.any(nz) else 0.0
    big = np.abs(ref) >= 1e-3 * rmax
    elem = float((err[big] / np.abs(ref[big])).max()) if rmax > 0 and np.any(big) else 0.0
    return normwise, comp, elem


def gate(y, ref, abs_ref, rel=REL, what="", report=None):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    abs_ref = np.asarray(abs_ref, dtype=np.float64)
    assert y.shape == ref.shape == abs_ref.shape, (what, y.shape, ref.shape)
    assert np.all(np.isfinite(y)), (what, "non-finite output")
    normwise, comp, elem = measure(y, ref, abs_ref)
    if report:
        errors.record(report, normwise, comp, elem, y.size, gated=True)
    assert normwise <= rel, (what, "normwise", normwise)
    err = np.abs(y - ref)
    bad = err > rel * abs_ref + 1e-30
    assert not np.any(bad), (what, "componentwise", int(bad.sum()),
                             float((err / np.maximum(abs_ref, 1e-300)).max()))
    return normwise


def exact(y, ref, what="", report=None):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert y.shape == ref.shape, (what, y.shape, ref.shape)
    diff = np.flatnonzero(y != ref)
    if report:
        errors.record(report, *measure(y, ref, np.abs(ref)), y.size, gated=True, exact=diff.size == 0)
    assert diff.size == 0, (what, "mismatches", int(diff.size), diff[:5].tolist())
