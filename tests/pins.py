"""Pins for the FP64 oracle: checks against what the paper and the mathematics
fix, independent of the oracle's own code.

Each ``check_*`` takes an oracle object (``oracle.COracle``) and raises
AssertionError on the first violation.  The planted-mistake tests run the
same checks on deliberately broken copies of the oracle and require that at
least one of them fails.

What pins what:
* delay table   -- exact rational arithmetic of Eq. (1) (fractions.Fraction),
                   rounded half-to-even, plus the invariants the law implies
                   (top channel 0, zero at DM 0, monotone in DM and frequency);
* forward       -- unit-impulse response (one 1 per DM row at t = tau - delay),
                   the dispersed pulse summing to exactly C, the zero-DM row
                   equal to the plain channel sum (the identical-rows case of
                   the paper's 0-DM experiment), linearity, and brute force
                   (Algorithm 1 in pure Python) on tiny inputs;
* adjoint       -- the dot-product identity <Ax, y> = <x, A^T y> (exact on
                   integers), its impulse response, and the gather form of the
                   transpose's definition in pure Python.
"""
from __future__ import annotations

import math
from fractions import Fraction

import numpy as np

from oracle import alg1


# ------------------------------------------------------------------ delays

def exact_delay_samples(n_channels, f_min, df, t_samp, dm_first, dm_step, i, ch) -> Fraction:
    """Eq. (1) divided by the sampling time, in exact rational arithmetic on
    the binary64 values of the parameters."""
    F = Fraction
    f_h = F(f_min) + (n_channels - 1) * F(df)
    f = F(f_min) + ch * F(df)
    dm = F(dm_first) + i * F(dm_step)
    return 4150 * dm * (1 / (f * f) - 1 / (f_h * f_h)) / F(t_samp)


def _sample_indices(D, C, n, rng):
    if D * C <= n:
        return [(i, c) for i in range(D) for c in range(C)]
    pts = {(0, 0), (D - 1, 0), (0, C - 1), (D - 1, C - 1), (D // 2, C // 2)}
    ii = rng.integers(0, D, size=n)
    cc = rng.integers(0, C, size=n)
    pts.update(zip(ii.tolist(), cc.tolist()))
    return sorted(pts)


def check_delay_table(orc, args, n_check=1500, seed=0):
    """args = (C, f_min, df, t_samp, dm_first, dm_step, D)."""
    C, f_min, df, t_samp, dm_first, dm_step, D = args
    table = orc.delay_table(*args)
    assert table.shape == (D, C) and table.dtype == np.int32
    rng = np.random.default_rng(seed)
    for i, ch in _sample_indices(D, C, n_check, rng):
        ex = exact_delay_samples(C, f_min, df, t_samp, dm_first, dm_step, i, ch)
        frac = ex - math.floor(ex)
        # FP64 evaluation can only disagree with exact rounding near a tie.
        assert abs(frac - Fraction(1, 2)) > Fraction(1, 10**7), (i, ch, float(ex))
        assert int(table[i, ch]) == round(ex), (i, ch, int(table[i, ch]), float(ex))
    check_delay_invariants(table, dm_first)


def check_alg1_delays(delays_fn, seed=0):
    """The pure-Python delay law (``alg1.delays``) against exact rational
    rounding of Eq. (1) on the small plans and the tiny and FD-slice
    workloads, every entry."""
    plans = DELAY_ARGS + [(64, 1400.0, 1.5625, 5e-5, 0.0, 0.5, 128),
                          (16, 1420.0, 64 * 300.0 / 1024, 1.0 / 20000, 0.0, 0.25, 32)]
    for args in plans:
        C, f_min, df, t_samp, dm_first, dm_step, D = args
        table = np.array(delays_fn(*args), dtype=np.int64)
        assert table.shape == (D, C), (args, table.shape)
        for i in range(D):
            for ch in range(C):
                ex = exact_delay_samples(C, f_min, df, t_samp, dm_first, dm_step, i, ch)
                assert int(table[i, ch]) == round(ex), (args, i, ch, int(table[i, ch]), float(ex))
        check_delay_invariants(table, dm_first)


def check_delay_invariants(table, dm_first):
    assert np.all(table[:, -1] == 0), "top channel must have zero delay"
    if dm_first == 0:
        assert np.all(table[0] == 0), "DM 0 must have zero delay"
    assert np.all(np.diff(table.astype(np.int64), axis=0) >= 0), "delay must not decrease with DM"
    assert np.all(np.diff(table.astype(np.int64), axis=1) <= 0), "delay must not increase with frequency"
    assert np.all(table >= 0)


# ------------------------------------------------------------------ forward

SMALL_PLANS = [
    # (C, f_min, df, t_samp, dm_first, dm_step, D, S)
    (8, 1400.0, 12.5, 5e-5, 0.0, 2.0, 6, 40),
    (5, 150.0, 0.75, 1e-4, 0.0, 0.5, 9, 33),
    (16, 1420.0, 18.75, 5e-5, 0.0, 0.25, 32, 64),
    (3, 300.0, 20.0, 2e-4, 1.0, 3.0, 4, 17),
]


def _plan(orc, p):
    C, f_min, df, t_samp, dm_first, dm_step, D, S = p
    table = orc.delay_table(C, f_min, df, t_samp, dm_first, dm_step, D)
    return table, S, S + int(table.max())


def check_impulse(orc, p, seed=0):
    """A single unit sample at (ch0, tau) reaches DM row i exactly once, at
    t = tau - delay[i][ch0] (when that lies in [0, S)), and nowhere else."""
    table, S, T = _plan(orc, p)
    D, C = table.shape
    rng = np.random.default_rng(seed)
    for _ in range(4):
        ch0 = int(rng.integers(0, C))
        tau = int(rng.integers(0, T))
        x = np.zeros((C, T))
        x[ch0, tau] = 1.0
        y = orc.dedisperse(x, table, S)
        for i in range(D):
            t = tau - int(table[i, ch0])
            expect = np.zeros(S)
            if 0 <= t < S:
                expect[t] = 1.0
            assert np.array_equal(y[i], expect), ("impulse", i, ch0, tau)


def check_dispersed_pulse(orc, p):
    """Unit samples placed on DM i0's delay track sum to exactly C at (i0, t0)."""
    table, S, T = _plan(orc, p)
    D, C = table.shape
    for i0 in (0, D // 2, D - 1):
        t0 = S // 3
        x = np.zeros((C, T))
        for ch in range(C):
            x[ch, t0 + table[i0, ch]] = 1.0
        y = orc.dedisperse(x, table, S)
        assert y[i0, t0] == C
        assert y.max() == C and y.min() >= 0.0
        # every DM row holds each of the C unit samples at most once
        assert np.all(y.sum(axis=1) <= C)


def check_channel_sum(orc, p, seed=0):
    """With DM 0 first, row 0 is the plain channel sum; with every DM 0 (the
    paper's 0-DM experiment) all rows equal that sum."""
    C, f_min, df, t_samp, dm_first, dm_step, D, S = p
    rng = np.random.default_rng(seed)
    zero = orc.delay_table(C, f_min, df, t_samp, 0.0, 0.0, D)
    T = S + 5
    x = rng.integers(-50, 50, size=(C, T)).astype(np.float64)
    y = orc.dedisperse(x, zero, S)
    s = x[:, :S].sum(axis=0)
    for i in range(D):
        assert np.array_equal(y[i], s), ("zero-DM row", i)
    table = orc.delay_table(C, f_min, df, t_samp, 0.0, dm_step, D)
    T = S + int(table.max())
    x = rng.integers(-50, 50, size=(C, T)).astype(np.float64)
    y = orc.dedisperse(x, table, S)
    assert np.array_equal(y[0], x[:, :S].sum(axis=0))


def check_linearity(orc, p, seed=0):
    table, S, T = _plan(orc, p)
    D, C = table.shape
    rng = np.random.default_rng(seed)
    x = rng.integers(-100, 100, size=(C, T)).astype(np.float64)
    z = rng.integers(-100, 100, size=(C, T)).astype(np.float64)
    a, b = 3.0, -0.5
    lhs = orc.dedisperse(a * x + b * z, table, S)
    rhs = a * orc.dedisperse(x, table, S) + b * orc.dedisperse(z, table, S)
    assert np.array_equal(lhs, rhs)


def check_brute_force(orc, p, seed=0):
    """Algorithm 1 in pure Python on the same (independently pinned) delays."""
    table, S, T = _plan(orc, p)
    C = table.shape[1]
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((C, T))
    y = orc.dedisperse(x, table, S)
    ref = np.array(alg1.dedisperse(x.tolist(), table.tolist(), S))
    assert np.array_equal(y, ref)
    i = rng.integers(0, table.shape[0], size=20)
    t = rng.integers(0, S, size=20)
    assert np.array_equal(orc.dedisperse_points(x, table, i, t), ref[i, t])


# ------------------------------------------------------------------ adjoint

def check_dot_product(orc, p, seed=0):
    """<A x, y> == <x, A^T y>, exact for integer data."""
    table, S, T = _plan(orc, p)
    D, C = table.shape
    rng = np.random.default_rng(seed)
    x = rng.integers(-20, 20, size=(C, T)).astype(np.float64)
    gy = rng.integers(-20, 20, size=(D, S)).astype(np.float64)
    ax = orc.dedisperse(x, table, S)
    aty = orc.adjoint(gy, table, T)
    assert aty.shape == (C, T)
    assert float(np.sum(ax * gy)) == float(np.sum(x * aty))


def check_adjoint_impulse(orc, p):
    """A unit at output (i0, t0) goes back to x[ch][t0 + delay[i0][ch]] only."""
    table, S, T = _plan(orc, p)
    D, C = table.shape
    for i0, t0 in ((0, 0), (D - 1, S - 1), (D // 2, S // 2)):
        gy = np.zeros((D, S))
        gy[i0, t0] = 1.0
        gx = orc.adjoint(gy, table, T)
        expect = np.zeros((C, T))
        for ch in range(C):
            expect[ch, t0 + table[i0, ch]] = 1.0
        assert np.array_equal(gx, expect), (i0, t0)


def check_adjoint_gather(orc, p, seed=0):
    """Gather form of the transpose's definition, in pure Python."""
    table, S, T = _plan(orc, p)
    D, C = table.shape
    rng = np.random.default_rng(seed)
    gy = rng.standard_normal((D, S))
    gx = orc.adjoint(gy, table, T)
    ref = np.array(alg1.adjoint(gy.tolist(), table.tolist(), T))
    assert np.array_equal(gx, ref)


FORWARD_CHECKS = (check_impulse, check_dispersed_pulse, check_channel_sum, check_linearity,
                  check_brute_force)
ADJOINT_CHECKS = (check_dot_product, check_adjoint_impulse, check_adjoint_gather)
DELAY_ARGS = [p[:7] for p in SMALL_PLANS]


def run_all(orc):
    """Every pin on the small plans; raises AssertionError on the first failure."""
    for args in DELAY_ARGS:
        check_delay_table(orc, args)
    for p in SMALL_PLANS:
        for chk in FORWARD_CHECKS + ADJOINT_CHECKS:
            chk(orc, p)


# ---------------------------------------------------------------- candidate search
#
# The boxcar search over dedispersed rows (oracle.search) is pinned by closed
# forms of noise-free rows, an invariance of its definition, its degenerate
# case and explicit loops on tiny rows.

def search_brute(y, n_widths):
    """(max snr, t, w) by explicit loops over every width and start (tiny rows)."""
    y = [float(v) for v in np.asarray(y, dtype=np.float64)]
    S = len(y)
    mu = math.fsum(y) / S
    sigma = math.sqrt(math.fsum((v - mu) ** 2 for v in y) / S)
    if sigma == 0.0:
        return 0.0, 0, 1
    best = (-math.inf, 0, 1)
    w = 1
    for _ in range(n_widths):
        if w > S:
            break
        for t in range(S - w + 1):
            s = math.fsum(y[t + i] - mu for i in range(w)) / (sigma * math.sqrt(w))
            if s > best[0]:
                best = (s, t, w)
        w *= 2
    return best


def check_search_spike(search_row):
    """A single spike of any height in S samples: the best boxcar is the spike
    alone, with S/N sqrt(S - 1) (mean A/S, standard deviation A sqrt(S-1)/S)."""
    for S, A, t0 in ((100, 3.0, 17), (4096, 250.0, 4000), (7, 1.0, 0)):
        y = np.zeros(S)
        y[t0] = A
        snr, t, w = search_row(y, 7)
        assert math.isclose(snr, math.sqrt(S - 1), rel_tol=1e-12), (S, snr)
        assert (t, w) == (t0, 1), (t, w)


def check_search_boxcar_pulse(search_row):
    """A noise-free boxcar of width 8 and height A: the best window is the
    pulse itself, S/N = 8 (A - mu) / (sigma sqrt(8))."""
    S, A, t0 = 1000, 2.5, 311
    y = np.zeros(S)
    y[t0:t0 + 8] = A
    mu = 8 * A / S
    sigma = math.sqrt((8 * (A - mu) ** 2 + (S - 8) * mu ** 2) / S)
    snr, t, w = search_row(y, 6)
    assert math.isclose(snr, 8 * (A - mu) / (sigma * math.sqrt(8)), rel_tol=1e-12), snr
    assert (t, w) == (t0, 8), (t, w)


def check_search_affine_invariance(search_row, seed=0):
    """S/N is unchanged when a row is scaled by a > 0 and shifted."""
    rng = np.random.default_rng(seed)
    y = rng.standard_normal(500)
    y[200:204] += 3.0
    base = search_row(y, 5)
    for a, b in ((3.0, 0.0), (0.25, 1e3), (7.0, -40.0)):
        got = search_row(a * y + b, 5)
        assert math.isclose(got[0], base[0], rel_tol=1e-9), (a, b, got, base)
        assert got[1:] == base[1:], (a, b, got, base)


def check_search_constant_row(search_row):
    """A constant row has no spread: S/N 0 at (0, 1) by definition."""
    assert search_row(np.full(64, 5.0), 4) == (0.0, 0, 1)


def check_search_brute(search_row, seed=0):
    rng = np.random.default_rng(seed)
    for S, nw in ((1, 3), (5, 4), (33, 6), (64, 7)):
        y = rng.standard_normal(S)
        got, ref = search_row(y, nw), search_brute(y, nw)
        assert math.isclose(got[0], ref[0], rel_tol=1e-12, abs_tol=1e-12), (S, got, ref)
        assert got[1:] == ref[1:], (S, got, ref)


def check_search_ties(search_row):
    """The tie rule of the definition: among equal S/N, the smaller width, then
    the earlier start.  Integer centred values keep every boxcar sum exact, so
    the ties below are exact in binary64.

    * Two identical spikes (mean 1, centred values 31 and -1): the first wins.
    * A width-4 boxcar of 3s starting at 5 and a width-1 spike of 6 at 20 (mean
      0): 12 / (2 sigma) and 6 / sigma are the same binary64 number, and the
      smaller width wins although it starts later."""
    y = np.zeros(64)
    y[12] = y[40] = 32.0
    snr, t, w = search_row(y, 6)
    assert (t, w) == (12, 1), (t, w)
    y = np.zeros(64)
    y[5:9] = 3.0
    y[20] = 6.0
    y[40:58] = -1.0
    sigma = math.sqrt(90.0 / 64.0)
    snr, t, w = search_row(y, 6)
    assert snr == 6.0 / sigma, (snr, 6.0 / sigma)
    assert (t, w) == (20, 1), (t, w)


def run_search(search_row):
    check_search_spike(search_row)
    check_search_boxcar_pulse(search_row)
    check_search_affine_invariance(search_row)
    check_search_constant_row(search_row)
    check_search_brute(search_row)
    check_search_ties(search_row)
