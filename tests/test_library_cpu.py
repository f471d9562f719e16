"""libdedisp on the CPU: it loads, exports what include/dedisp.h declares,
builds delay tables bit-identical to the oracle's, and rejects bad arguments
before touching any GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth
from paper_1601_05052_amd import _lib
from paper_1601_05052_amd import Plan, DedispError, tile_variants

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dedisp.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dd_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_api():
    names = declared_functions()
    for must in ("dd_plan_create", "dd_dedisperse", "dd_dedisperse_adjoint", "dd_autotune",
                 "dd_batch_create", "dd_batch_run", "dd_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = _lib.lib()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert set(declared_functions()) == set(_lib.SIGNATURES), "binding and header disagree"


def test_version_string():
    assert b"gfx950" in _lib.lib().dd_version()


@pytest.mark.parametrize("setup", [synth.TINY, synth.APERTIF, synth.LOFAR, synth.FD_SLICE],
                         ids=lambda s: s.name)
def test_delay_table_bit_exact_vs_oracle(setup):
    p = Plan.from_setup(setup)
    mine = p.delays()
    ref = oracle.delay_table(*setup.plan_args()[:7])
    assert mine.dtype == np.int32 and mine.shape == ref.shape
    assert np.array_equal(mine, ref)
    assert p.max_delay == int(ref.max())
    assert p.input_samples == setup.n_samples + int(ref.max())


def test_delay_table_bit_exact_batched_and_random():
    for beam in synth.batched_beams():
        p = Plan.from_setup(beam)
        assert np.array_equal(p.delays(), oracle.delay_table(*beam.plan_args()[:7])), beam.name
    rng = np.random.default_rng(123)
    for _ in range(40):
        C = int(rng.integers(1, 300))
        f_min = float(rng.uniform(50, 2000))
        df = float(rng.uniform(0.001, 5.0))
        t_samp = float(rng.uniform(1e-6, 1e-3))
        dm_first = float(rng.uniform(0, 100))
        dm_step = float(rng.uniform(0, 3))
        D = int(rng.integers(1, 200))
        args = (C, f_min, df, t_samp, dm_first, dm_step, D)
        p = Plan(*args, 1000)
        assert np.array_equal(p.delays(), oracle.delay_table(*args)), args


def test_plan_dims():
    p = Plan.from_setup(synth.TINY)
    c, d, s = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _lib.check(_lib.lib().dd_plan_dims(p.handle, ctypes.byref(c), ctypes.byref(d), ctypes.byref(s)))
    assert (c.value, d.value, s.value) == (64, 128, 4096)


BAD_PLANS = [
    dict(n_channels=0), dict(n_dm=0), dict(n_samples=0), dict(f_min=0.0), dict(f_min=-5.0),
    dict(df=0.0), dict(df=-1.0), dict(t_samp=0.0), dict(dm_first=-1.0), dict(dm_step=-0.25),
    dict(f_min=float("nan")), dict(df=float("inf")), dict(t_samp=float("nan")),
    dict(dm_step=float("inf")),
    dict(f_min=10.0, t_samp=1e-12, dm_step=1e6),   # delays beyond int32
]


@pytest.mark.parametrize("bad", BAD_PLANS, ids=lambda b: ",".join("%s=%s" % kv for kv in b.items()))
def test_plan_rejects_invalid(bad):
    args = dict(n_channels=8, f_min=1400.0, df=1.0, t_samp=5e-5, dm_first=0.0, dm_step=0.5, n_dm=4,
                n_samples=64)
    args.update(bad)
    with pytest.raises(DedispError) as e:
        Plan(**args)
    assert e.value.code == _lib.DD_EINVAL
    assert _lib.lib().dd_last_error()


def test_plan_size_limit():
    """Input rows (n_samples + max delay) must stay below 2^29 samples: the
    largest such plan is accepted, one sample more is refused."""
    args = (4, 1400.0, 1.0, 5e-5, 0.0, 80.0, 4)
    md = int(oracle.delay_table(*args).max())
    assert md > 0
    assert Plan(*args, (1 << 29) - 1 - md).input_samples == (1 << 29) - 1
    with pytest.raises(DedispError) as e:
        Plan(*args, (1 << 29) - md)
    assert e.value.code == _lib.DD_EINVAL


def _fake(addr):
    return ctypes.c_void_p(addr)


def test_compute_calls_reject_bad_arguments_before_gpu_work():
    """Shape / stride / pointer errors return before any HIP call, so they can
    be exercised without a GPU using fake (never dereferenced) pointers."""
    L = _lib.lib()
    p = Plan.from_setup(synth.TINY)
    h, T, S = p.handle, p.input_samples, p.n_samples
    IN, OUT = 0x100000, 0x90000000
    cases = [
        (L.dd_dedisperse(None, _fake(IN), 0, T, _fake(OUT), S, None), _lib.DD_EINVAL),
        (L.dd_dedisperse(h, None, 0, T, _fake(OUT), S, None), _lib.DD_EINVAL),
        (L.dd_dedisperse(h, _fake(IN), 0, T, None, S, None), _lib.DD_EINVAL),
        (L.dd_dedisperse(h, _fake(IN), 7, T, _fake(OUT), S, None), _lib.DD_EINVAL),
        (L.dd_dedisperse(h, _fake(IN), 0, T - 1, _fake(OUT), S, None), _lib.DD_ESHAPE),
        (L.dd_dedisperse(h, _fake(IN), 0, T, _fake(OUT), S - 1, None), _lib.DD_ESHAPE),
        (L.dd_dedisperse(h, _fake(IN + 2), 0, T, _fake(OUT), S, None), _lib.DD_ESHAPE),
        (L.dd_dedisperse(h, _fake(IN), 0, T, _fake(IN + 64), S, None), _lib.DD_ESHAPE),  # overlap
        (L.dd_dedisperse_adjoint(h, _fake(OUT), S - 1, _fake(IN), T, None), _lib.DD_ESHAPE),
        (L.dd_dedisperse_adjoint(h, _fake(OUT), S, _fake(IN), T - 1, None), _lib.DD_ESHAPE),
        (L.dd_dedisperse_adjoint(h, _fake(OUT), S, _fake(OUT + 4), T, None), _lib.DD_ESHAPE),
        (L.dd_dedisperse_adjoint(h, None, S, _fake(IN), T, None), _lib.DD_EINVAL),
        (L.dd_plan_set_tile(h, 0, 0, 999), _lib.DD_EINVAL),
        (L.dd_plan_set_tile(h, 5, 0, 0), _lib.DD_EINVAL),
        (L.dd_autotune(h, 1, 2, 3, None, None, None, None), _lib.DD_EINVAL),
        (L.dd_autotune(h, 0, 0, 0, None, None, None, None), _lib.DD_EINVAL),
    ]
    for got, want in cases:
        assert got == want
        assert L.dd_last_error()


def test_null_plan_queries():
    L = _lib.lib()
    v = ctypes.c_int32()
    assert L.dd_plan_max_delay(None, ctypes.byref(v)) == _lib.DD_EINVAL
    assert L.dd_plan_destroy(None) == _lib.DD_OK
    assert L.dd_batch_destroy(None) == _lib.DD_OK
    assert L.dd_batch_create(None, None, 0, 0) == _lib.DD_EINVAL
    tiny = Plan.from_setup(synth.TINY)
    many = (ctypes.c_void_p * 97)(*([tiny.handle.value] * 97))
    b = ctypes.c_void_p()
    assert L.dd_batch_create(ctypes.byref(b), many, 97, 0) == _lib.DD_EINVAL   # at most 96 beams
    assert L.dd_batch_create(ctypes.byref(b), many, 0, 0) == _lib.DD_EINVAL
    assert not b.value
    assert L.dd_batch_autotune(None, 0, 0, 1, None, None) == _lib.DD_EINVAL
    p = Plan.from_setup(synth.TINY)
    arr = (ctypes.c_void_p * 1)(p.handle.value)
    assert L.dd_batch_autotune(arr, 1, 2, 0, None, None) == _lib.DD_EINVAL    # reps 0
    assert L.dd_batch_autotune(arr, 1, 9, 1, None, None) == _lib.DD_EINVAL    # dtype


def test_realtime_rejects_bad_arguments_before_gpu_work():
    L = _lib.lib()
    p = Plan.from_setup(synth.TINY)
    h = ctypes.c_void_p()
    assert L.dd_realtime_create(None, p.handle, 0, None) == _lib.DD_EINVAL
    assert L.dd_realtime_create(ctypes.byref(h), None, 0, None) == _lib.DD_EINVAL
    assert L.dd_realtime_create(ctypes.byref(h), p.handle, 9, None) == _lib.DD_EINVAL
    assert not h.value
    assert L.dd_realtime_push(None, _fake(0x1000), p.n_samples, _fake(0x9000), p.n_samples) == _lib.DD_EINVAL
    n = ctypes.c_int64()
    assert L.dd_realtime_pushed(None, ctypes.byref(n)) == _lib.DD_EINVAL
    assert L.dd_realtime_destroy(None) == _lib.DD_OK


def test_search_rejects_bad_arguments_before_gpu_work():
    L = _lib.lib()
    R, O = _fake(0x100000), _fake(0x200000)
    ok = (R, 100, 4, 100, 8, O, O, O, None)
    def call(i, v):
        a = list(ok)
        a[i] = v
        return L.dd_search_boxcar(*a)
    assert call(0, None) == _lib.DD_EINVAL
    assert call(5, None) == _lib.DD_EINVAL
    assert call(2, 0) == _lib.DD_EINVAL          # no rows
    assert call(3, 0) == _lib.DD_EINVAL          # no samples
    assert call(4, 0) == _lib.DD_EINVAL          # widths
    assert call(4, 13) == _lib.DD_EINVAL
    assert call(1, 99) == _lib.DD_ESHAPE         # stride < samples
    assert call(0, _fake(0x100002)) == _lib.DD_ESHAPE
    assert L.dd_last_error()


def test_tile_variants_cover_paper_parameters():
    """Sec. III-B: work-items and elements per work-item, in time and in DM."""
    vs = tile_variants()
    assert len(vs) >= 8
    for i, (vid, it, ia, waves, kind) in enumerate(vs):
        assert vid == i
        assert it >= 1 and ia >= 1 and 1 <= waves <= 16 and kind in (0, 1, 2)
    assert {v[4] for v in vs} == {0, 1, 2}, "LDS, register-window and direct kernels are all compiled"


def test_set_tile_rejects_window_too_large():
    """A register-window tile of 64 channels cannot serve the LOFAR-like
    adjoint (neighbouring channels' delays differ by thousands of samples
    there, far beyond a register window, skewed tiles or not); the 1-row
    variant always fits."""
    p = Plan.from_setup(synth.LOFAR)
    wide = [v[0] for v in tile_variants() if v[2] * v[3] == 64 and v[4] == 1]
    with pytest.raises(DedispError):
        p.set_tile(wide[0], direction=_lib.DD_ADJOINT)
    one = [v[0] for v in tile_variants() if v[2] * v[3] == 1][0]
    p.set_tile(one, direction=_lib.DD_ADJOINT)
    assert p.get_tile(direction=_lib.DD_ADJOINT) == one
    p.set_tile(-1, direction=_lib.DD_ADJOINT)


def test_fault_injection_alloc(monkeypatch):
    """DD_FAULT_INJECT=alloc makes table allocation fail with DD_ENOMEM (the
    failure happens before any device call)."""
    monkeypatch.setenv("DD_FAULT_INJECT", "alloc")
    p = Plan.from_setup(synth.TINY)
    rc = _lib.lib().dd_plan_prepare(p.handle, 0, 0)
    # Without a GPU, hipGetDevice may fail first (DD_EHIP); with one, DD_ENOMEM.
    assert rc in (_lib.DD_ENOMEM, _lib.DD_EHIP)


def test_generated_asm_header_is_current():
    """regwin_asm.h is generated; the committed copy must match its generator."""
    import importlib.util
    gen = os.path.join(ROOT, "paper_1601_05052_amd", "csrc", "gen_regwin_asm.py")
    spec = importlib.util.spec_from_file_location("gen_regwin_asm", gen)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    with open(os.path.join(ROOT, "paper_1601_05052_amd", "csrc", "regwin_asm.h")) as f:
        assert f.read() == mod.render()


def test_one_hip_runtime_in_process():
    """libdedisp binds to the HIP runtime PyTorch loaded (one libamdhip64 and
    one HSA runtime mapped), so torch streams are valid library handles."""
    _lib.lib()
    import torch  # noqa: F401
    with open("/proc/self/maps") as f:
        maps = f.read().splitlines()
    hip = {l.split()[-1] for l in maps if "libamdhip64" in l}
    hsa = {l.split()[-1] for l in maps if "libhsa-runtime64" in l}
    assert len(hip) == 1, hip
    assert len(hsa) == 1, hsa


def test_output_checks_reject_bad_outs_on_the_host():
    """The binding checks every caller-supplied output (dtype, shape, strides,
    device) before it hands pointers to the library; shown here on host
    tensors, where no launch can happen."""
    import torch
    from paper_1601_05052_amd import _check_output
    p = Plan(4, 1400.0, 1.0, 1e-4, 0.0, 1.0, 3, 10)
    cpu = torch.device("cpu")
    _check_output(torch.empty((3, 10)), p, cpu)
    _check_output(torch.empty((3, 16))[:, :12], p, cpu)
    bad = [torch.empty((3, 10), dtype=torch.float16),   # wrong dtype
           torch.empty((2, 10)),                         # too few rows
           torch.empty((3, 9)),                          # rows too short
           torch.empty((10, 3)).t(),                     # non-unit column stride
           torch.empty((3, 10, 1)),                      # not 2-D
           torch.empty(30).as_strided((3, 10), (5, 1))]  # overlapping rows
    for o in bad:
        with pytest.raises(ValueError):
            _check_output(o, p, cpu)
    with pytest.raises(ValueError):
        _check_output(torch.empty((3, 10)), p, torch.device("meta"))
    with pytest.raises(TypeError):
        _check_output(np.zeros((3, 10), np.float32), p, cpu)


def test_noalloc_entry_refuses_unprepared_plan_before_gpu_work():
    """dd_dedisperse_noalloc stages the plan's host tables; a plan whose tables
    were never built is refused (DD_EINVAL) before any GPU call, as are the
    forward's argument errors."""
    L = _lib.lib()
    p = Plan(4, 1400.0, 1.0, 1e-4, 0.0, 1.0, 3, 10)
    T = p.input_samples
    buf_in = ctypes.create_string_buffer(4 * 4 * T)
    buf_out = ctypes.create_string_buffer(4 * 3 * 10)
    rc = L.dd_dedisperse_noalloc(p.handle, ctypes.addressof(buf_in), 0, T, ctypes.addressof(buf_out), 10, None)
    assert rc == _lib.DD_EINVAL
    assert b"dd_plan_prepare" in L.dd_last_error()
    assert L.dd_dedisperse_noalloc(p.handle, ctypes.addressof(buf_in), 0, T - 1, ctypes.addressof(buf_out), 10,
                                   None) == _lib.DD_ESHAPE
    assert L.dd_dedisperse_noalloc(None, ctypes.addressof(buf_in), 0, T, ctypes.addressof(buf_out), 10,
                                   None) == _lib.DD_EINVAL


def test_row_split_arguments_checked_on_the_host():
    """dd_plan_set_blocks validates starts, ids and fit on the host; get_blocks
    reports one block without a split and the split after one is set."""
    from paper_1601_05052_amd import DD_ADJOINT, DD_FORWARD
    p = Plan(64, 1400.0, 1.5625, 5e-5, 0.0, 0.5, 128, 4096)
    kinds = {v[0]: v[4] for v in tile_variants()}
    assert len(p.get_blocks()) == 1 and p.get_blocks()[0][0] == 0
    p.set_blocks([0, 32], [9, 0])
    assert p.get_blocks() == [(0, 9), (32, 0)]
    assert p.get_tile() in (9, 0)
    for starts, vs in (([16, 32], [9, 9]),      # must start at row 0
                       ([0, 32, 16], [9, 9, 9]),  # must increase
                       ([0, 64], [9, 9]),       # past the last row (64 channels)
                       ([0, 32], [9, 10 ** 6])):  # unknown variant
        with pytest.raises(DedispError) as e:
            p.set_blocks(starts, vs)
        assert e.value.code == _lib.DD_EINVAL, (starts, vs)
    direct = next(v for v, k in kinds.items() if k == 2)
    with pytest.raises(DedispError) as e:
        p.set_blocks([0, 32], [9, direct])
    assert e.value.code == _lib.DD_EUNSUPPORTED
    regwin = next(v for v, k in kinds.items() if k == 1)
    with pytest.raises(DedispError) as e:   # a block start off its chunk of rows
        p.set_blocks([0, 1], [9, regwin])
    assert e.value.code == _lib.DD_EUNSUPPORTED
    p.set_tile(0)                         # a forced single variant replaces the split
    assert p.get_blocks() == [(0, 0)]
    p.set_blocks([0, 64], [9, 9], direction=DD_ADJOINT)   # adjoint rows are the 128 DMs
    assert p.get_blocks(direction=DD_ADJOINT) == [(0, 9), (64, 9)]
    n = _lib.DD_MAX_BLOCKS
    with open(os.path.join(ROOT, "include", "dedisp.h")) as f:
        assert "#define DD_MAX_BLOCKS %d\n" % n in f.read()
    p.set_blocks([4 * k for k in range(n)], [9] * n, direction=DD_ADJOINT)
    assert p.get_blocks(direction=DD_ADJOINT) == [(4 * k, 9) for k in range(n)]
    with pytest.raises(DedispError) as e:      # one block more than the arrays hold
        p.set_blocks([2 * k for k in range(n + 1)], [9] * (n + 1), direction=DD_ADJOINT)
    assert e.value.code == _lib.DD_EINVAL
    assert p.get_blocks(direction=DD_FORWARD) == [(0, 0)]
    from paper_1601_05052_amd import DD_U8
    for call in (lambda: p.set_blocks([0, 64], [9, 9], direction=DD_ADJOINT, dtype=DD_U8),
                 lambda: p.set_tile(9, direction=DD_ADJOINT, dtype=DD_U8)):
        with pytest.raises(DedispError) as e:   # the adjoint works on float32 rows only
            call()
        assert e.value.code == _lib.DD_EINVAL


def test_skewed_tiles_fit_narrower_windows_per_block():
    """Skewed tiles: within a block of input rows each accumulator row's tiles
    follow the average delay curve of the block, so the window a tile needs
    shrinks with the block.  The Apertif adjoint's fan-out across 8 channels
    reaches 61 samples at the top DM: the 40-register window of variant 31
    cannot serve all DMs at once, but serves each half; the LOFAR adjoint fits
    the prefetched LDS tile of variant 46 in 16 blocks of 128 DMs, not in 8."""
    from paper_1601_05052_amd import DD_ADJOINT
    p = Plan.from_setup(synth.APERTIF)
    with pytest.raises(DedispError) as e:
        p.set_tile(31, direction=DD_ADJOINT)
    assert e.value.code == _lib.DD_EUNSUPPORTED
    p.set_blocks([0, 1024], [31, 31], direction=DD_ADJOINT)
    assert p.get_blocks(direction=DD_ADJOINT) == [(0, 31), (1024, 31)]
    q = Plan.from_setup(synth.LOFAR)
    q.set_blocks([128 * k for k in range(16)], [46] * 16, direction=DD_ADJOINT)
    with pytest.raises(DedispError) as e:
        q.set_blocks([256 * k for k in range(8)], [46] * 8, direction=DD_ADJOINT)
    assert e.value.code == _lib.DD_EUNSUPPORTED
