"""Forward dedispersion on the GPU against the FP64 oracle (element by element
on small cases, sampled outputs at full size)."""
import numpy as np
import pytest

import oracle
import synth
from paper_1601_05052_amd import DD_F16, DD_F32, DD_U8, DedispError, Plan, dedisperse, tile_variants
from paper_1601_05052_amd._lib import DD_EUNSUPPORTED
from tests import errors, gates
from tests.gpu_util import (oracle_delays, ref_and_abs, sample_points, to_dev, to_host, torch_mod,
                            workload_input)

pytestmark = pytest.mark.gpu


def test_tiny_workload_f32():
    s = synth.TINY
    x, table, T = workload_input(s)
    plan = Plan.from_setup(s)
    y = to_host(dedisperse(to_dev(x), plan))
    ref, absref = ref_and_abs(x, table, s.n_samples)
    gates.gate(y, ref, absref, what="tiny", report="tiny f32 forward")
    i, t = np.unravel_index(np.argmax(y), y.shape)
    assert i == synth.TINY_PULSE_DM_INDEX


RAGGED = [
    # (C, f_min, df, t_samp, dm_first, dm_step, D, S): tails in every tile dimension
    (37, 1400.0, 2.5, 5e-5, 0.0, 0.75, 77, 1001),
    (5, 140.0, 0.2, 5e-6, 0.0, 0.02, 9, 3333),
    (1, 1400.0, 1.0, 5e-5, 0.0, 1.0, 1, 1),
    (3, 1400.0, 1.0, 5e-5, 2.0, 0.0, 5, 65),
    (130, 1420.0, 300.0 / 130, 5e-5, 10.0, 0.25, 33, 515),
]
# Variants that must fit each ragged shape (counted on the host when the list
# was last changed: 39, 31, 46, 46 and 45 of 46; small delay spreads fit nearly
# every variant, the LOFAR-band shape only the wider forms).
MIN_VARIANTS = {37: 37, 5: 28, 1: 46, 3: 46, 130: 42}


def set_tile_or_skip(plan, vid, **kw):
    """Force a variant; False if it cannot serve the plan (DD_EUNSUPPORTED).
    Any other failure is an error."""
    try:
        plan.set_tile(vid, **kw)
        return True
    except DedispError as e:
        if e.code != DD_EUNSUPPORTED:
            raise
        return False


@pytest.mark.parametrize("dtype", ["f32", "u8", "f16"])
@pytest.mark.parametrize("args", RAGGED, ids=lambda a: "C%d_D%d_S%d" % (a[0], a[6], a[7]))
def test_every_tile_variant_integer_exact(args, dtype):
    """Integer-valued inputs are summed exactly in binary32 in any order, so
    every tile variant must reproduce the oracle bit for bit, including ragged
    tiles.  Rows of T_in + 3 samples, and for u8 / f16 a view starting one
    element in: row starts at every byte alignment."""
    torch = torch_mod()
    C, D, S = args[0], args[6], args[7]
    plan = Plan(*args)
    table = oracle.delay_table(*args[:7])
    assert np.array_equal(plan.delays(), table)
    T = plan.input_samples
    lo, hi = (0, 255) if dtype == "u8" else (-8, 8)
    x = synth.integers_f32(C, T + 4, seed=C * 7 + D, lo=lo, hi=hi)
    ref = oracle.dedisperse(x[:, 1:], table, S) if dtype != "f32" else oracle.dedisperse(x, table, S)
    np_t = {"f32": np.float32, "u8": np.uint8, "f16": np.float16}[dtype]
    code = {"f32": DD_F32, "u8": DD_U8, "f16": DD_F16}[dtype]
    full = to_dev(x.astype(np_t))
    xd = full if dtype == "f32" else full[:, 1:]   # odd element offset: misaligned rows
    ran = 0
    for vid, *_ in tile_variants():
        if not set_tile_or_skip(plan, vid, dtype=code):
            continue  # window does not fit LDS for this variant
        out = torch.full((D, S), float("nan"), device="cuda")
        y = to_host(dedisperse(xd, plan, out=out))
        gates.exact(y, ref, what="%s variant %d" % (dtype, vid))
        ran += 1
    plan.set_tile(-1, dtype=code)
    assert ran >= MIN_VARIANTS[C], (ran, MIN_VARIANTS[C])


def test_nan_canaries_and_stride_padding():
    """Only columns [0, S) of each output row are written."""
    torch = torch_mod()
    s = synth.TINY
    x, table, T = workload_input(s, stride_pad=5)
    plan = Plan.from_setup(s)
    out = torch.full((s.n_dm, s.n_samples + 7), float("nan"), device="cuda")
    dedisperse(to_dev(x), plan, out=out)
    o = to_host(out)
    assert np.all(np.isfinite(o[:, :s.n_samples]))
    assert np.all(np.isnan(o[:, s.n_samples:]))
    ref, absref = ref_and_abs(x[:, :T], table, s.n_samples)
    gates.gate(o[:, :s.n_samples], ref, absref, what="strided")


def test_deterministic():
    s = synth.TINY
    x, _, _ = workload_input(s)
    plan = Plan.from_setup(s)
    xd = to_dev(x)
    a = to_host(dedisperse(xd, plan))
    b = to_host(dedisperse(xd, plan))
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


def test_zero_dm_rows_are_identical_channel_sums():
    """All trial DMs 0 (the paper's perfect-reuse experiment): every row is
    the plain channel sum."""
    plan = Plan(64, 1400.0, 1.5625, 5e-5, 0.0, 0.0, 96, 3000)
    assert plan.max_delay == 0
    x = synth.integers_f32(64, 3000, seed=9)
    y = to_host(dedisperse(to_dev(x), plan))
    s = x.astype(np.float64).sum(axis=0)
    for i in range(96):
        assert np.array_equal(y[i], s)


def test_single_impulse_lands_on_its_delay_track():
    s = synth.TINY
    plan = Plan.from_setup(s)
    table = plan.delays()
    T = plan.input_samples
    x = np.zeros((s.n_channels, T), dtype=np.float32)
    ch0, tau = 17, 2000
    x[ch0, tau] = 1.0
    y = to_host(dedisperse(to_dev(x), plan))
    for i in range(s.n_dm):
        expect = np.zeros(s.n_samples, dtype=np.float32)
        expect[tau - table[i, ch0]] = 1.0
        assert np.array_equal(y[i], expect)


def test_linearity():
    s = synth.TINY
    plan = Plan.from_setup(s)
    T = plan.input_samples
    x = synth.integers_f32(s.n_channels, T, seed=1)
    z = synth.integers_f32(s.n_channels, T, seed=2)
    a = to_host(dedisperse(to_dev(3 * x - 2 * z), plan))
    b = 3 * to_host(dedisperse(to_dev(x), plan)) - 2 * to_host(dedisperse(to_dev(z), plan))
    assert np.array_equal(a, b)


def test_u8_bit_exact():
    s = synth.TINY
    x, table, _ = workload_input(s, dtype="u8")
    plan = Plan.from_setup(s)
    y = to_host(dedisperse(to_dev(x), plan))
    gates.exact(y, oracle.dedisperse(x, table, s.n_samples), what="u8", report="tiny u8 forward")


def test_f16_gate_and_quantisation_error_reported():
    """f16 storage: gated against the oracle on the stored f16 values; the
    error against the float32 data the f16 values were rounded from (storage
    quantisation plus summation) is reported, not gated."""
    s = synth.TINY
    x16, table, T = workload_input(s, dtype="f16")
    x32, _, _ = workload_input(s, dtype="f32")
    plan = Plan.from_setup(s)
    y = to_host(dedisperse(to_dev(x16), plan))
    ref, absref = ref_and_abs(x16.astype(np.float64), table, s.n_samples)
    gates.gate(y, ref, absref, what="f16 vs oracle on f16 values", report="tiny f16 forward (vs f16 values)")
    ref32, absref32 = ref_and_abs(x32, table, s.n_samples)
    q = gates.measure(y, ref32, absref32)
    errors.record("tiny f16 storage vs float32 original", *q, y.size, gated=False)
    print("tiny f16 storage error vs float32 original: normwise %.2e componentwise %.2e" % q[:2])
    assert q[0] < 1e-2  # f16 keeps 11 significant bits


@pytest.mark.parametrize("setup", [synth.APERTIF, synth.LOFAR], ids=lambda s: s.name)
def test_full_size_sampled(setup):
    """Full-size run in the launch configuration the benchmark times; outputs
    checked at sampled (DM, t) points plus whole rows at both DM ends."""
    x, table, T = workload_input(setup)
    plan = Plan.from_setup(setup)
    y = to_host(dedisperse(to_dev(x), plan))
    assert y.shape == (setup.n_dm, setup.n_samples)
    assert np.all(np.isfinite(y))
    i, t = sample_points(setup.n_dm, setup.n_samples, 20000, setup.seed)
    ref = oracle.dedisperse_points(x, table, i, t)
    absref = oracle.dedisperse_points(np.abs(x), table, i, t)
    cfg = "%s f32 forward (plan's variant)" % setup.name
    gates.gate(y[i, t], ref, absref, what=setup.name, report=cfg)
    for row in (0, setup.n_dm - 1):
        ri = np.full(setup.n_samples, row, dtype=np.int32)
        rt = np.arange(setup.n_samples, dtype=np.int64)
        gates.gate(y[row], oracle.dedisperse_points(x, table, ri, rt),
                   oracle.dedisperse_points(np.abs(x), table, ri, rt), what="%s row %d" % (setup.name, row),
                   report=cfg)


@pytest.mark.parametrize("setup,dtype", [(synth.APERTIF, "f32"), (synth.LOFAR, "f32"), (synth.APERTIF, "u8"),
                                          (synth.APERTIF, "f16")], ids=lambda a: getattr(a, "name", a))
def test_full_size_every_fitting_variant(setup, dtype):
    """The benchmark tunes the forward and times whichever variant wins, so
    every variant that fits the full-size workload is checked: 20,000 sampled
    outputs (gathered on the device) against the oracle on the same stored
    values (u8 bit for bit)."""
    torch = torch_mod()
    x, table, T = workload_input(setup, dtype=dtype)
    code = {"f32": DD_F32, "u8": DD_U8, "f16": DD_F16}[dtype]
    plan = Plan.from_setup(setup)
    i, t = sample_points(setup.n_dm, setup.n_samples, 20000, setup.seed + 1)
    x64 = x.astype(np.float64)
    ref = oracle.dedisperse_points(x64, table, i, t)
    absref = oracle.dedisperse_points(np.abs(x64), table, i, t)
    if dtype == "f16":
        x32, _, _ = workload_input(setup, dtype="f32")
        ref32 = oracle.dedisperse_points(x32, table, i, t)
        absref32 = oracle.dedisperse_points(np.abs(x32), table, i, t)
        del x32
    xd = to_dev(x)
    y = torch.empty((setup.n_dm, setup.n_samples), device="cuda")
    it, tt = torch.from_numpy(i.astype(np.int64)).cuda(), torch.from_numpy(t).cuda()
    checked = 0
    cfg = "%s %s forward (every fitting variant)" % (setup.name, dtype)
    if dtype == "f16":
        cfg += " vs f16 values"
    for vid, *_ in tile_variants():
        if not set_tile_or_skip(plan, vid, dtype=code):
            continue  # window does not fit LDS for this variant
        y.fill_(float("nan"))
        dedisperse(xd, plan, out=y)
        got = to_host(y[it, tt])
        what = "%s %s variant %d" % (setup.name, dtype, vid)
        if dtype == "u8":
            gates.exact(got, ref, what=what, report=cfg)
        else:
            gates.gate(got, ref, absref, what=what, report=cfg)
        if dtype == "f16":
            errors.record("%s f16 storage vs float32 original (every fitting variant)" % setup.name,
                          *gates.measure(got, ref32, absref32), got.size, gated=False)
        checked += 1
    plan.set_tile(-1, dtype=code)
    assert checked >= 10


def test_apertif_integer_exact_sampled():
    s = synth.APERTIF
    plan = Plan.from_setup(s)
    table = oracle_delays(s)
    x = synth.integers_f32(s.n_channels, plan.input_samples, seed=77)
    y = to_host(dedisperse(to_dev(x), plan))
    i, t = sample_points(s.n_dm, s.n_samples, 20000, 78)
    gates.exact(y[i, t], oracle.dedisperse_points(x, table, i, t), what="apertif int",
                report="apertif integer-valued f32 forward")


@pytest.mark.parametrize("dtype,code", [("u8", DD_U8), ("f16", DD_F16)])
def test_apertif_low_precision_sampled(dtype, code):
    s = synth.APERTIF
    x, table, T = workload_input(s, dtype=dtype)
    plan = Plan.from_setup(s)
    y = to_host(dedisperse(to_dev(x), plan))
    i, t = sample_points(s.n_dm, s.n_samples, 20000, 5)
    ref = oracle.dedisperse_points(x, table, i, t)
    cfg = "apertif %s forward (plan's variant)" % dtype
    if dtype == "u8":
        gates.exact(y[i, t], ref, what="apertif u8", report=cfg)
    else:
        absref = oracle.dedisperse_points(np.abs(x.astype(np.float64)), table, i, t)
        gates.gate(y[i, t], ref, absref, what="apertif f16", report=cfg + " vs f16 values")


def test_non_default_stream():
    torch = torch_mod()
    s = synth.TINY
    x, table, T = workload_input(s)
    plan = Plan.from_setup(s)
    xd = to_dev(x)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        y = dedisperse(xd, plan)
    st.synchronize()
    ref, absref = ref_and_abs(x, table, s.n_samples)
    gates.gate(y.cpu().numpy(), ref, absref, what="stream")


def test_autotune_picks_a_working_variant(tmp_path):
    s = synth.TINY
    plan = Plan.from_setup(s)
    cache = str(tmp_path / "tune.txt")
    v, ms = plan.autotune(cache_path=cache, reps=2)
    assert v >= 0 and ms > 0
    assert plan.get_tile() == v
    v2, ms2 = Plan.from_setup(s).autotune(cache_path=cache)
    assert v2 == v and abs(ms2 - ms) < 1e-6 * max(1.0, ms)  # served from the cache
    x, table, _ = workload_input(s)
    y = to_host(dedisperse(to_dev(x), plan))
    ref, absref = ref_and_abs(x, table, s.n_samples)
    gates.gate(y, ref, absref, what="tuned")
