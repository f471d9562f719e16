"""dd_dedisperse_noalloc (the allocation-free forward) through the C ABI,
against dd_dedisperse on the same plan and input: two calls in a row, the
second on a smaller plan, each bit-identical to dd_dedisperse (same kernels,
same tables) and within the binary32 gates of the FP64 oracle; u8 storage
bit-exact; tables beyond the array's capacity refused."""
import ctypes

import numpy as np
import pytest

import oracle
import synth
from paper_1601_05052_amd import (DD_F32, DD_FORWARD, DD_U8, DedispError, Plan, _lib, dedisperse,
                                  dedisperse_noalloc)
from tests import gates
from tests.gpu_util import sample_points, to_dev, to_host, torch_mod

pytestmark = pytest.mark.gpu


def _noalloc_c_abi(plan, x, out, code):
    """One call through the C ABI (ctypes), on torch's current stream."""
    torch = torch_mod()
    rc = _lib.lib().dd_dedisperse_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()), code, x.stride(0),
                                          ctypes.c_void_p(out.data_ptr()), out.stride(0),
                                          ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    _lib.check(rc)


BIG = synth.Setup("na_big", 1024, 1420.0, 300.0 / 1024, 1.0 / 20000, 0.0, 0.25, 512, 6000, seed=61)
SMALL = synth.Setup("na_small", 64, 1400.0, 1.5625, 5e-5, 0.0, 0.5, 96, 1500, seed=62)


def test_noalloc_matches_dedisperse_two_calls_second_smaller():
    torch = torch_mod()
    for s in (BIG, SMALL):
        plan = Plan.from_setup(s)
        plan.prepare(DD_FORWARD, DD_F32)
        table = oracle.delay_table(*s.plan_args()[:7])
        x = synth.noise_f32(s.n_channels, plan.input_samples, s.seed)
        xd = to_dev(x)
        ref_dev = to_host(dedisperse(xd, plan))
        out = torch.full((s.n_dm, s.n_samples + 3), float("nan"), device="cuda")
        _noalloc_c_abi(plan, xd, out, DD_F32)
        got = to_host(out)
        assert np.all(np.isnan(got[:, s.n_samples:])), "stride padding written"
        got = got[:, :s.n_samples]
        assert np.array_equal(got.view(np.uint32), ref_dev.view(np.uint32)), s.name
        i, t = sample_points(s.n_dm, s.n_samples, 3000, s.seed)
        gates.gate(got[i, t], oracle.dedisperse_points(x, table, i, t),
                   oracle.dedisperse_points(np.abs(x), table, i, t), what=s.name)


def test_noalloc_u8_and_binding():
    torch = torch_mod()
    s = SMALL
    plan = Plan.from_setup(s)
    plan.prepare(DD_FORWARD, DD_U8)
    table = oracle.delay_table(*s.plan_args()[:7])
    x = synth.noise_u8(s.n_channels, plan.input_samples + 1, s.seed)
    xd = to_dev(x)[:, 1:]   # rows starting at odd byte addresses
    out = torch.empty((s.n_dm, s.n_samples), device="cuda")
    dedisperse_noalloc(xd, plan, out)
    gates.exact(to_host(out), oracle.dedisperse(x[:, 1:], table, s.n_samples), what="noalloc u8")


def test_noalloc_refuses_tables_beyond_capacity():
    """An LDS-form tile of one accumulator row keeps one offset per delay-table
    entry: 4,500 DMs x 1,000 channels need 18 MB of tables, more than the
    16 MiB array."""
    torch = torch_mod()
    plan = Plan(1000, 1420.0, 0.3, 1.0 / 20000, 0.0, 0.25, 4500, 64)
    plan.set_tile(9)
    plan.prepare(DD_FORWARD, DD_F32)
    x = torch.zeros((1000, plan.input_samples), device="cuda")
    out = torch.empty((4500, 64), device="cuda")
    with pytest.raises(DedispError) as e:
        _noalloc_c_abi(plan, x, out, DD_F32)
    assert "at most" in str(e.value)
