"""Row splits (dd_plan_set_blocks): the input rows cut into blocks, each summed
by its own tile variant in its own launch, later blocks continuing the partial
sums in the output.  Every output still adds its rows in ascending order, so a
split must equal one variant for all rows bit for bit, and the oracle exactly on
integer data."""
import numpy as np
import pytest

import oracle
import synth
from paper_1601_05052_amd import (DD_ADJOINT, DD_F32, DD_FORWARD, DD_U8, DedispError, Plan, dedisperse,
                                  dedisperse_adjoint, dedisperse_noalloc, tile_variants)
from tests import gates
from tests.gpu_util import oracle_delays, to_dev, to_host, torch_mod

pytestmark = pytest.mark.gpu

KIND = {v[0]: v[4] for v in tile_variants()}
FILLER = 9   # LDS form, one row per tile: fits every block


def fitting(plan, starts, block, direction):
    """Variants (LDS and register-window kinds) that can serve block `block` of
    the split `starts`, the other blocks on the filler variant."""
    out = []
    for v in KIND:
        if KIND[v] == 2:
            continue
        vs = [FILLER] * len(starts)
        vs[block] = v
        try:
            plan.set_blocks(starts, vs, direction=direction)
            out.append(v)
        except DedispError:
            pass
    plan.set_tile(-1, direction=direction)
    return out


def run(plan, x, direction):
    return to_host(dedisperse(x, plan) if direction == DD_FORWARD else dedisperse_adjoint(x, plan))


CASES = [
    # (plan args, direction, row starts)
    ((37, 1400.0, 2.5, 5e-5, 0.0, 0.75, 77, 1001), DD_ADJOINT, [0, 32, 64]),
    ((130, 1420.0, 300.0 / 130, 5e-5, 10.0, 0.25, 33, 515), DD_ADJOINT, [0, 16]),
    ((130, 1420.0, 300.0 / 130, 5e-5, 10.0, 0.25, 33, 515), DD_FORWARD, [0, 48, 96, 112]),
    ((64, 1400.0, 1.5625, 5e-5, 0.0, 0.5, 128, 4096), DD_FORWARD, [0, 32]),
]


@pytest.mark.parametrize("args,direction,starts", CASES, ids=lambda c: str(c)[:24])
def test_splits_integer_exact(args, direction, starts):
    """Each block cycles through every variant that fits it; every split is
    exact against the oracle on integer-valued data."""
    C, D, S = args[0], args[6], args[7]
    plan = Plan(*args)
    table = oracle.delay_table(*args[:7])
    T = plan.input_samples
    if direction == DD_FORWARD:
        x = synth.integers_f32(C, T, seed=C + D)
        ref = oracle.dedisperse(x, table, S)
    else:
        x = synth.integers_f32(D, S, seed=C + D)
        ref = oracle.adjoint(x, table, T)
    xd = to_dev(x)
    fits = [fitting(plan, starts, b, direction) for b in range(len(starts))]
    assert all(fits), fits
    n = max(len(f) for f in fits)
    for k in range(n):
        vs = [f[k % len(f)] for f in fits]
        plan.set_blocks(starts, vs, direction=direction)
        assert plan.get_blocks(direction=direction) == list(zip(starts, vs))
        gates.exact(run(plan, xd, direction), ref, what="split %s %s" % (starts, vs))
    plan.set_tile(-1, direction=direction)


def test_split_bit_identical_to_one_variant_apertif_adjoint():
    """Full-size Apertif adjoint on N(0,1) data: low DMs on a narrow register
    window, higher DMs on wider ones, against the wide window for every row."""
    s = synth.APERTIF
    plan = Plan.from_setup(s)
    gy = to_dev(synth.noise_f32(s.n_dm, s.n_samples, seed=91))
    plan.set_tile(40, direction=DD_ADJOINT)
    one = run(plan, gy, DD_ADJOINT)
    plan.set_blocks([0, 512, 1024], [31, 34, 40], direction=DD_ADJOINT)
    split = run(plan, gy, DD_ADJOINT)
    assert np.array_equal(one.view(np.uint32), split.view(np.uint32))


def test_autotuned_adjoint_exact_on_channel_rows():
    """dd_autotune may pick a split for the Apertif adjoint; whatever it picks
    is exact on integer data (whole channel rows against the oracle)."""
    s = synth.APERTIF
    plan = Plan.from_setup(s)
    table = oracle_delays(s)
    T = plan.input_samples
    v, ms = plan.autotune(direction=DD_ADJOINT, reps=2)
    blocks = plan.get_blocks(direction=DD_ADJOINT)
    print("autotuned Apertif adjoint: %s, %.3f ms" % (blocks, ms))
    assert plan.get_tile(direction=DD_ADJOINT) == v
    gy = synth.integers_f32(s.n_dm, s.n_samples, seed=92, lo=-3, hi=3)
    gx = run(plan, to_dev(gy), DD_ADJOINT)
    for ch in (0, 511, 1023):
        ref = oracle.adjoint(gy, np.ascontiguousarray(table[:, ch:ch + 1]), T)[0]
        gates.exact(gx[ch], ref, what="tuned adjoint ch %d" % ch)


def test_noalloc_with_split():
    """The allocation-free forward stages every block's tables and runs the
    blocks in order: bit-identical to dd_dedisperse with the same split."""
    torch = torch_mod()
    s = synth.TINY
    plan = Plan.from_setup(s)
    starts = [0, 32]
    fits = [fitting(plan, starts, b, DD_FORWARD) for b in range(2)]
    plan.set_blocks(starts, [fits[0][-1], fits[1][0]], direction=DD_FORWARD, dtype=DD_U8)
    plan.prepare(DD_FORWARD, DD_U8)
    x = to_dev(synth.noise_u8(s.n_channels, plan.input_samples, seed=93))
    ref = to_host(dedisperse(x, plan))
    out = torch.empty((s.n_dm, s.n_samples), device="cuda")
    got = to_host(dedisperse_noalloc(x, plan, out))
    assert np.array_equal(got, ref)
    table = oracle.delay_table(*s.plan_args()[:7])
    gates.exact(got, oracle.dedisperse(to_host(x), table, s.n_samples), what="noalloc split u8")


def test_lofar_adjoint_in_dm_blocks_bit_identical_to_direct():
    """Full-size LOFAR adjoint on N(0,1) data: sixteen blocks of 128 DMs, or
    thirty-two of 64, each on a prefetched LDS tile of 8 channels (skewed
    tiles, row spans), against the direct kind over all DMs at once: the same
    rows in the same order, so bit-identical; and exact against the oracle on
    integer data for three channels."""
    s = synth.LOFAR
    plan = Plan.from_setup(s)
    gy = to_dev(synth.noise_f32(s.n_dm, s.n_samples, seed=94))
    plan.set_tile(45, direction=DD_ADJOINT)
    one = run(plan, gy, DD_ADJOINT)
    for nb, v in ((16, 46), (16, 25), (32, 37)):
        plan.set_blocks([(s.n_dm // nb) * k for k in range(nb)], [v] * nb, direction=DD_ADJOINT)
        split = run(plan, gy, DD_ADJOINT)
        assert np.array_equal(one.view(np.uint32), split.view(np.uint32)), (nb, v)
    table = oracle_delays(s)
    gi = synth.integers_f32(s.n_dm, s.n_samples, seed=95, lo=-3, hi=3)
    gx = run(plan, to_dev(gi), DD_ADJOINT)
    for ch in (0, 16, 31):
        ref = oracle.adjoint(gi, np.ascontiguousarray(table[:, ch:ch + 1]), plan.input_samples)[0]
        gates.exact(gx[ch], ref, what="LOFAR adjoint in DM blocks ch %d" % ch)


@pytest.mark.parametrize("dtype", [DD_F32, DD_U8])
def test_split_bit_identical_to_one_variant_apertif_forward(dtype):
    """Full-size Apertif forward: channels [0, 512) on variant 17 and [512,
    1024) on variant 31 (each block with its own skews) against variant 31
    for all channels, bit for bit (N(0,1) float32, or u8)."""
    s = synth.APERTIF
    plan = Plan.from_setup(s)
    if dtype == DD_F32:
        x = to_dev(synth.noise_f32(s.n_channels, plan.input_samples, seed=96))
    else:
        x = to_dev(synth.noise_u8(s.n_channels, plan.input_samples, seed=96))
    plan.set_tile(31, dtype=dtype)
    one = to_host(dedisperse(x, plan))
    plan.set_blocks([0, 512], [17, 31], dtype=dtype)
    split = to_host(dedisperse(x, plan))
    assert np.array_equal(one.view(np.uint32), split.view(np.uint32))
