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
"""
from __future__ import annotations

import numpy as np

REL = 1e-5


def gate(y, ref, abs_ref, rel=REL, what=""):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    abs_ref = np.asarray(abs_ref, dtype=np.float64)
    assert y.shape == ref.shape == abs_ref.shape, (what, y.shape, ref.shape)
    assert np.all(np.isfinite(y)), (what, "non-finite output")
    err = np.abs(y - ref)
    scale = max(float(np.max(np.abs(ref))), 1e-300)
    normwise = float(err.max()) / scale if err.size else 0.0
    assert normwise <= rel, (what, "normwise", normwise)
    bad = err > rel * abs_ref + 1e-30
    assert not np.any(bad), (what, "componentwise", int(bad.sum()),
                             float((err / np.maximum(abs_ref, 1e-300)).max()))
    return normwise


def exact(y, ref, what=""):
    y = np.asarray(y, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert y.shape == ref.shape, (what, y.shape, ref.shape)
    diff = np.flatnonzero(y != ref)
    assert diff.size == 0, (what, "mismatches", int(diff.size), diff[:5].tolist())
