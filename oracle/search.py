"""FP64 oracle of the boxcar candidate search over dedispersed rows.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper states that the dedispersed time-series are analysed further to find
pulses (Sec. I) but does not define that step; this module fixes the plain
definition the library's search computes, in FP64:

  mu, sigma  mean and population standard deviation of the row y[0:S]
  B_w(t)     = sum_{i < w} (y[t + i] - mu),   0 <= t <= S - w
  snr_w(t)   = B_w(t) / (sigma * sqrt(w))           (0 where sigma == 0)

for widths w = 1, 2, 4, ..., 2^(n_widths - 1) (those <= S).  Per row the result
is the largest snr over all (w, t), with one (t, w) that reaches it.
"""
from __future__ import annotations

import numpy as np


def widths(n_widths: int, n_samples: int):
    return [1 << k for k in range(n_widths) if (1 << k) <= n_samples]


def row_stats(y: np.ndarray):
    y = np.asarray(y, dtype=np.float64)
    mu = y.mean()
    return mu, np.sqrt(np.mean((y - mu) ** 2))


def snr(y: np.ndarray, t: int, w: int) -> float:
    """snr_w(t) of one row, by the definition."""
    y = np.asarray(y, dtype=np.float64)
    mu, sigma = row_stats(y)
    if sigma == 0.0:
        return 0.0
    return float(np.sum(y[t:t + w] - mu) / (sigma * np.sqrt(w)))


def search_row(y: np.ndarray, n_widths: int):
    """(max snr, t, w) of one row; t, w the first maximum (smallest w, then t)."""
    y = np.asarray(y, dtype=np.float64)
    S = y.shape[0]
    mu, sigma = row_stats(y)
    if sigma == 0.0:
        return 0.0, 0, 1
    c = np.concatenate([[0.0], np.cumsum(y - mu)])
    best = (-np.inf, 0, 1)
    for w in widths(n_widths, S):
        s = (c[w:] - c[:-w]) / (sigma * np.sqrt(w))
        t = int(np.argmax(s))
        if s[t] > best[0]:
            best = (float(s[t]), t, w)
    return best


def search(y: np.ndarray, n_widths: int):
    """Rows of y [D][S]: arrays (snr [D], t [D], w [D])."""
    out = [search_row(row, n_widths) for row in np.asarray(y)]
    return (np.array([o[0] for o in out]), np.array([o[1] for o in out], dtype=np.int64),
            np.array([o[2] for o in out], dtype=np.int64))
