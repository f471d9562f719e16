"""The FP64 oracle against its pins (CPU only)."""
import os

import numpy as np
import pytest

import oracle
import synth
from tests import pins

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_numbers.txt")


def paper_numbers():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                k, v = (s.strip() for s in line.split("="))
                vals[k] = float(v)
    return vals


def test_pins_on_small_plans():
    pins.run_all(oracle.default())


def test_alg1_delays_exact_rational_and_equal_to_c_oracle():
    """The pure-Python delay law against exact rational rounding, and against
    the C oracle's table (two independent codings of Eq. (1))."""
    from oracle import alg1
    pins.check_alg1_delays(alg1.delays)
    for args in pins.DELAY_ARGS + [synth.TINY.plan_args()[:7], synth.FD_SLICE.plan_args()[:7]]:
        assert np.array_equal(np.array(alg1.delays(*args), dtype=np.int32), oracle.delay_table(*args)), args


@pytest.mark.parametrize("setup", [synth.TINY, synth.APERTIF, synth.LOFAR, synth.FD_SLICE],
                         ids=lambda s: s.name)
def test_delay_table_exact_rational(setup):
    pins.check_delay_table(oracle.default(), setup.plan_args()[:7], n_check=1200, seed=setup.seed)


def test_delay_table_batched_beams():
    for beam in synth.batched_beams()[:6]:
        pins.check_delay_table(oracle.default(), beam.plan_args()[:7], n_check=300, seed=beam.seed)


def test_delay_table_is_fp64_only():
    """Evaluating Eq. (1) in binary32 changes entries of the Apertif table:
    the table is defined by the FP64 evaluation (pinned above), not FP32."""
    s = synth.APERTIF
    table = oracle.delay_table(*s.plan_args()[:7])
    f32 = np.float32
    f = (f32(s.f_min) + np.arange(s.n_channels, dtype=f32) * f32(s.df)).astype(f32)
    fh = f[-1]
    dm = (np.arange(s.n_dm, dtype=f32) * f32(s.dm_step)).astype(f32)
    k = (f32(1) / (f * f) - f32(1) / (fh * fh)).astype(f32)
    t32 = np.rint(((f32(4150) * dm)[:, None] * k[None, :]) / f32(s.t_samp)).astype(np.int64)
    assert np.count_nonzero(t32 != table) > 0


def test_max_delay_values():
    """maxDelay = delay[last DM][lowest channel] for the monotone tables."""
    for s in (synth.TINY, synth.APERTIF, synth.LOFAR):
        t = oracle.delay_table(*s.plan_args()[:7])
        assert t.max() == t[-1, 0]
        ex = pins.exact_delay_samples(*s.plan_args()[:6], s.n_dm - 1, 0)
        assert t[-1, 0] == round(ex)


def test_workloads_follow_paper_setups():
    g = paper_numbers()
    a, l = synth.APERTIF, synth.LOFAR
    assert round(1 / a.t_samp) == g["apertif_samples_per_s"]
    assert a.n_channels == g["apertif_channels"]
    assert abs(a.df - g["apertif_channel_mhz"]) < 0.005
    assert a.f_min == g["apertif_f_low_mhz"]
    assert a.f_min + a.n_channels * a.df == g["apertif_f_high_mhz"]
    assert round(1 / l.t_samp) == g["lofar_samples_per_s"]
    assert l.n_channels == g["lofar_channels"]
    assert abs(l.df - g["lofar_channel_mhz"]) < 0.005
    assert l.f_min == g["lofar_f_low_mhz"]
    assert l.n_channels * l.df == g["lofar_bandwidth_mhz"]
    assert a.dm_first == g["first_dm"] and a.dm_step == g["dm_step"]


def test_flop_and_byte_accounting_matches_paper():
    """One add per (DM, sample, channel): C*S per DM gives the paper's 20 and 6
    MFLOP per DM (printed rounded); the Apertif system's 36 GB/s in and 72 GB/s
    out follow from 4-byte samples."""
    g = paper_numbers()
    a, l = synth.APERTIF, synth.LOFAR
    assert round(a.adds / a.n_dm / 1e6) == g["apertif_mflop_per_dm"]
    assert round(l.adds / l.n_dm / 1e6) == g["lofar_mflop_per_dm"]
    b = g["bytes_per_element"]
    rate = 1 / a.t_samp
    gb_in = g["apertif_beams"] * a.n_channels * rate * b / 1e9
    gb_out = g["apertif_beams"] * g["apertif_dms"] * rate * b / 1e9
    assert int(gb_in) == g["apertif_input_gb_per_s"]
    assert round(gb_out) == g["apertif_output_gb_per_s"]


def test_tiny_pulse_lands_at_its_dm_and_time():
    s = synth.TINY
    table = oracle.delay_table(*s.plan_args()[:7])
    T = s.n_samples + int(table.max())
    x = synth.make_input(s, T, "f32", arrivals={synth.TINY_PULSE_DM_INDEX: table[synth.TINY_PULSE_DM_INDEX]})
    y = oracle.dedisperse(x, table, s.n_samples)
    i, t = np.unravel_index(np.argmax(y), y.shape)
    (dm_i, t0), = synth.pulse_sites(s)
    assert i == dm_i and t0 <= t < t0 + synth.PULSE_WIDTH


def test_points_match_full():
    s = synth.TINY
    table = oracle.delay_table(*s.plan_args()[:7])
    T = s.n_samples + int(table.max())
    x = synth.noise_f32(s.n_channels, T, 11)
    y = oracle.dedisperse(x, table, s.n_samples)
    rng = np.random.default_rng(0)
    i = rng.integers(0, s.n_dm, 500)
    t = rng.integers(0, s.n_samples, 500)
    assert np.array_equal(oracle.dedisperse_points(x, table, i, t), y[i, t])


def test_oracle_rejects_bad_plans():
    with pytest.raises(ValueError):
        oracle.delay_table(0, 1400.0, 1.0, 5e-5, 0.0, 0.5, 4)
    with pytest.raises(ValueError):
        oracle.delay_table(4, 1400.0, -1.0, 5e-5, 0.0, 0.5, 4)
    with pytest.raises(ValueError):
        oracle.delay_table(4, 10.0, 1.0, 1e-12, 0.0, 1e6, 4)   # delay beyond int32


def test_stream_windows_tile_the_output():
    """Streaming semantics (one chunk of S samples per step, Sec. III-A): the
    dedispersion of the window of stream times [k*S - max_delay, (k+1)*S), with
    zeros before time 0, is the slice [k*S - max_delay, k*S - max_delay + S) of
    the dedispersion of the whole zero-padded stream, for chunks shorter and
    longer than the largest delay."""
    for S in (4096, 100):
        args = (64, 1400.0, 1.5625, 5e-5, 0.0, 0.5, 128)
        table = oracle.delay_table(*args)
        M = int(table.max())
        K = 3 if S > M else 9
        x = synth.integers_f32(64, K * S, seed=7).astype(np.float64)
        padded = np.concatenate([np.zeros((64, M)), x], axis=1)
        full = oracle.dedisperse(padded, table, K * S)
        for k in range(K):
            w = padded[:, k * S:k * S + S + M]
            assert np.array_equal(oracle.dedisperse(w, table, S), full[:, k * S:(k + 1) * S])
        # stream time -max_delay reads channel ch at stream time delay - max_delay
        ch = np.arange(64)
        assert np.array_equal(full[:, 0], np.array([padded[ch, table[i]].sum() for i in range(128)]))


def test_search_oracle_pins():
    """Boxcar candidate search: closed forms of noise-free rows, affine
    invariance, the constant row, explicit loops on tiny rows."""
    from oracle import search
    pins.run_search(search.search_row)
