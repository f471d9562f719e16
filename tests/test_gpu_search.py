"""Boxcar candidate search (dd_search_boxcar) on the GPU against the FP64
oracle (oracle/search.py).

The maximum S/N is unique and is compared within a tolerance: the kernel
forms mean and standard deviation in binary64 and the centred samples in
binary64 rounded to binary32, so each boxcar sum of w centred samples is a
binary32 pairwise sum (relative error below log2(w) * 2^-24 of the sum of
magnitudes, about sqrt(w) * sigma), and the S/N is one more binary32 product:
|snr - ref| <= 1e-4 * (1 + |ref|) holds with a wide margin for w <= 2048.
The (t, w) reaching it need not be unique at that precision; the test checks
that the oracle's S/N at the kernel's (t, w) is within the same tolerance of
the maximum."""
import numpy as np
import pytest

import oracle
import synth
from oracle import search as osearch
from paper_1601_05052_amd import Plan, dedisperse, search_boxcar
from tests.gpu_util import oracle_delays, to_dev, to_host, torch_mod, workload_input

pytestmark = pytest.mark.gpu

TOL = 1e-4


def check_rows(y: np.ndarray, S: int, n_widths: int, snr, t, w, rows=None):
    rows = range(y.shape[0]) if rows is None else rows
    for r in rows:
        ref, _, _ = osearch.search_row(y[r, :S], n_widths)
        tol = TOL * (1.0 + abs(ref))
        assert abs(float(snr[r]) - ref) <= tol, (r, float(snr[r]), ref)
        assert int(w[r]) in osearch.widths(n_widths, S) and 0 <= int(t[r]) <= S - int(w[r]), (r, t[r], w[r])
        at = osearch.snr(y[r, :S], int(t[r]), int(w[r]))
        assert at >= ref - 2 * tol, (r, at, ref)


def run(y: np.ndarray, S: int, n_widths: int):
    snr, t, w = search_boxcar(to_dev(y), n_samples=S, n_widths=n_widths)
    return to_host(snr), to_host(t), to_host(w)


def test_random_rows_with_planted_pulses():
    rng = np.random.default_rng(5)
    y = synth.noise_f32(48, 9000, seed=71)
    for r in range(48):
        width = 1 << (r % 9)
        t0 = int(rng.integers(0, 9000 - width))
        y[r, t0:t0 + width] += np.float32(6.0 / np.sqrt(width))
    snr, t, w = run(y, 9000, 11)
    check_rows(y, 9000, 11, snr, t, w)


@pytest.mark.parametrize("S,n_widths", [(1, 1), (2, 3), (5, 12), (4096, 12), (4097, 12), (10000, 1), (8193, 5)])
def test_shapes_and_width_counts(S, n_widths):
    """Ragged chunks (the search stages 4096 boxcar starts per step), rows
    shorter than the widest boxcar, a single width."""
    y = synth.noise_f32(7, S, seed=S + n_widths)
    snr, t, w = run(y, S, n_widths)
    if S == 1:
        assert np.all(snr == 0) and np.all(t == 0) and np.all(w == 1)
        return
    check_rows(y, S, n_widths, snr, t, w)


def test_constant_rows_and_stride_padding():
    """sigma == 0 gives (0, 0, 1); samples past n_samples are never read."""
    torch = torch_mod()
    y = np.full((3, 700), 4.0, dtype=np.float32)
    y[1, :] = -2.0
    y[2, 5] = 9.0
    buf = torch.full((3, 711), float("nan"), device="cuda")
    buf[:, :700] = to_dev(y)
    snr, t, w = search_boxcar(buf, n_samples=700, n_widths=8)
    snr, t, w = to_host(snr), to_host(t), to_host(w)
    assert snr[0] == 0 and t[0] == 0 and w[0] == 1
    assert snr[1] == 0 and t[1] == 0 and w[1] == 1
    check_rows(y, 700, 8, snr, t, w, rows=[2])
    assert int(t[2]) == 5 and int(w[2]) == 1


def test_large_offset_rows():
    """Rows with a large common offset (u8 input summed over 1,024 channels)."""
    y = (np.float32(131072.0) + np.float32(512.0) * synth.noise_f32(16, 20000, seed=81)).astype(np.float32)
    y[3, 1000:1064] += np.float32(400.0)
    snr, t, w = run(y, 20000, 12)
    check_rows(y, 20000, 12, snr, t, w)
    assert abs(int(t[3]) - 1000) < 64


def test_tiny_workload_pulse_found_at_its_dm():
    """Dedisperse the tiny workload, then search: every row agrees with the
    oracle's search of the oracle's output, the best row is the oracle's best
    row, and it lies next to the pulse's DM (a neighbouring trial DM can win
    with a wider boxcar, the pulse being smeared there)."""
    s = synth.TINY
    x, table, T = workload_input(s)
    plan = Plan.from_setup(s)
    y = dedisperse(to_dev(x), plan)
    snr, t, w = search_boxcar(y, n_widths=8)
    snr, t, w = to_host(snr), to_host(t), to_host(w)
    ref_rows = oracle.dedisperse(x.astype(np.float64), table, s.n_samples)
    check_rows(ref_rows, s.n_samples, 8, snr, t, w)
    ref_snr = np.array([osearch.search_row(r, 8)[0] for r in ref_rows])
    assert int(np.argmax(snr)) == int(np.argmax(ref_snr))
    assert abs(int(np.argmax(snr)) - synth.TINY_PULSE_DM_INDEX) <= 1


def test_apertif_beam_sampled_rows():
    """Full-size Apertif beam: dedisperse on the GPU, search all 2048 rows,
    compare 48 rows (the pulses' DMs among them) with the oracle's search of
    the same GPU rows."""
    s = synth.APERTIF
    x, table, T = workload_input(s)
    plan = Plan.from_setup(s)
    yd = dedisperse(to_dev(x), plan)
    snr, t, w = search_boxcar(yd, n_widths=11)
    snr, t, w = to_host(snr), to_host(t), to_host(w)
    y = to_host(yd)
    pulse_rows = [i for i, _ in synth.pulse_sites(s)]
    rows = sorted(set(pulse_rows) | set(np.random.default_rng(3).integers(0, s.n_dm, 44).tolist()))
    check_rows(y, s.n_samples, 11, snr, t, w, rows=rows)
    for i in pulse_rows:
        assert snr[i] > np.median(snr) + 5, (i, snr[i])


def test_tie_rule_smaller_width_then_earlier_start():
    """Exact ties (every sum below is exact in binary32 and binary64): two
    identical spikes give the earlier start; a width-4 boxcar of 3s and a later
    width-1 spike of 6 (mean 0) have the same S/N and the smaller width wins."""
    y = np.zeros((2, 64), dtype=np.float32)
    y[0, 12] = y[0, 40] = 32.0
    y[1, 5:9] = 3.0
    y[1, 20] = 6.0
    y[1, 40:58] = -1.0
    snr, t, w = run(y, 64, 6)
    assert (int(t[0]), int(w[0])) == (12, 1), (t[0], w[0])
    assert (int(t[1]), int(w[1])) == (20, 1), (t[1], w[1])
    for r in range(2):
        ref = osearch.search_row(y[r], 6)
        assert (int(t[r]), int(w[r])) == ref[1:], (r, ref)
    check_rows(y, 64, 6, snr, t, w)
