"""Batched graph launch: every beam equals the oracle and, bit for bit, its
own single-beam run (same tile variant, same summation order); graph replays
pick up new inputs and pointers."""
import numpy as np
import pytest

import oracle
import synth
from paper_1601_05052_amd import DD_F16, DD_F32, DD_U8, Batch, DedispError, Plan, dedisperse, tile_variants
from tests import gates
from tests.gpu_util import sample_points, to_dev, to_host, torch_mod

pytestmark = pytest.mark.gpu


def small_beams():
    """Uneven beams small enough for full oracle checks."""
    out = []
    rng = np.random.default_rng(99)
    for b in range(7):
        c = int(rng.choice([16, 32, 64, 100]))
        d = int(rng.integers(20, 200))
        s = int(rng.integers(300, 3000))
        out.append(synth.Setup("sb%d" % b, c, 1420.0, 300.0 / c, 1.0 / 20000, 0.0, 0.25 * (b + 1), d, s,
                               seed=900 + b))
    return out


@pytest.mark.parametrize("dtype,code", [("f32", DD_F32), ("u8", DD_U8), ("f16", DD_F16)])
def test_batch_matches_oracle_and_single_beam(dtype, code):
    beams = small_beams()
    plans = [Plan.from_setup(b) for b in beams]
    xs_h = []
    for b, p in zip(beams, plans):
        x = {"f32": synth.noise_f32, "u8": synth.noise_u8, "f16": synth.noise_f16}[dtype](
            b.n_channels, p.input_samples + 3, b.seed)
        xs_h.append(x)
    xs = [to_dev(x) for x in xs_h]
    batch = Batch(plans, dtype=code)
    assert batch.variants() == [p.get_tile(dtype=code) for p in plans]
    outs = batch.run(xs)
    for b, p, x, y in zip(beams, plans, xs_h, outs):
        table = oracle.delay_table(*b.plan_args()[:7])
        yh = to_host(y)
        ref = oracle.dedisperse(x, table, b.n_samples)
        if dtype == "u8":
            gates.exact(yh, ref, what=b.name, report="batched small beams u8")
        else:
            absref = oracle.dedisperse(np.abs(x.astype(np.float64)), table, b.n_samples)
            gates.gate(yh, ref, absref, what=b.name, report="batched small beams %s" % dtype)
        single = to_host(dedisperse(to_dev(x), p))
        assert np.array_equal(single, yh), b.name


def test_batch_mixed_forced_variants_exact():
    """Beams forced onto different kinds (register window, LDS, prefetched
    LDS, direct) run as separate groups of one graph; each is exact."""
    beams = small_beams()[:5]
    plans = [Plan.from_setup(b) for b in beams]
    kinds = {v[0]: v[4] for v in tile_variants()}
    wanted = [17, 21, 27, 9, 19]
    for p, v in zip(plans, wanted):
        try:
            p.set_tile(v)
        except DedispError:
            pass  # variant does not fit this beam: keep the automatic choice
    batch = Batch(plans)
    got = batch.variants()
    assert got == [p.get_tile() for p in plans]
    assert len({kinds[v] for v in got}) >= 2
    xs_h = [synth.integers_f32(b.n_channels, p.input_samples, seed=50 + i) for i, (b, p) in enumerate(zip(beams, plans))]
    outs = batch.run([to_dev(x) for x in xs_h])
    for b, x, y in zip(beams, xs_h, outs):
        table = oracle.delay_table(*b.plan_args()[:7])
        gates.exact(to_host(y), oracle.dedisperse(x, table, b.n_samples), what=b.name)


def test_batch_of_the_most_beams_exact():
    """The largest batch (96 beams) of uneven small beams, degenerate ones
    included (one channel, one DM, one sample), u8 storage: one graph launch,
    every beam bit-exact against the oracle and against its single-beam run."""
    rng = np.random.default_rng(96)
    beams = [synth.Setup("one", 1, 1400.0, 1.0, 5e-5, 0.0, 1.0, 1, 1, seed=1000)]
    for b in range(1, 96):
        c = int(rng.choice([1, 3, 16, 64, 130]))
        d = int(rng.choice([1, 7, 40, 129]))
        s = int(rng.choice([1, 65, 513, 2000]))
        beams.append(synth.Setup("mb%d" % b, c, 1420.0, 300.0 / c, 1.0 / 20000, 0.0, 0.25 * (1 + b % 5), d, s,
                                 seed=1000 + b))
    plans = [Plan.from_setup(b) for b in beams]
    xs_h = [synth.noise_u8(b.n_channels, p.input_samples, b.seed) for b, p in zip(beams, plans)]
    batch = Batch(plans, dtype=DD_U8)
    assert len(batch.variants()) == 96
    outs = batch.run([to_dev(x) for x in xs_h])
    for b, p, x, y in zip(beams, plans, xs_h, outs):
        yh = to_host(y)
        table = oracle.delay_table(*b.plan_args()[:7])
        gates.exact(yh, oracle.dedisperse(x, table, b.n_samples), what=b.name)
        assert np.array_equal(to_host(dedisperse(to_dev(x), p)), yh), b.name


def test_batch_replay_new_data_and_pointers():
    torch = torch_mod()
    beams = small_beams()[:4]
    plans = [Plan.from_setup(b) for b in beams]
    batch = Batch(plans)
    for rep in range(3):
        xs_h = [synth.integers_f32(b.n_channels, p.input_samples, seed=rep * 10 + i)
                for i, (b, p) in enumerate(zip(beams, plans))]
        xs = [to_dev(x) for x in xs_h]
        outs = [torch.full((p.n_dm, p.n_samples + 4), float("nan"), device="cuda") for p in plans]
        batch.run(xs, outs)
        torch.cuda.synchronize()
        for b, x, o in zip(beams, xs_h, outs):
            oh = to_host(o)
            table = oracle.delay_table(*b.plan_args()[:7])
            gates.exact(oh[:, :b.n_samples], oracle.dedisperse(x, table, b.n_samples), what="rep%d" % rep)
            assert np.all(np.isnan(oh[:, b.n_samples:]))


def test_batched_workload_sampled_u8():
    """The 64-beam Apertif-band batch (u8 storage) in one launch: every beam's
    sampled outputs are bit-exact against the oracle."""
    torch = torch_mod()
    beams = synth.batched_beams()
    plans = [Plan.from_setup(b) for b in beams]
    xs_h = [synth.noise_u8(b.n_channels, p.input_samples, b.seed) for b, p in zip(beams, plans)]
    xs = [to_dev(x) for x in xs_h]
    batch = Batch(plans, dtype=DD_U8)
    outs = batch.run(xs)
    torch.cuda.synchronize()
    for b, x, y in zip(beams, xs_h, outs):
        table = oracle.delay_table(*b.plan_args()[:7])
        i, t = sample_points(b.n_dm, b.n_samples, 400, b.seed)
        yh = y[torch.from_numpy(i).long().cuda(), torch.from_numpy(t).long().cuda()].cpu().numpy()
        gates.exact(yh, oracle.dedisperse_points(x, table, i, t), what=b.name,
                    report="batched 64 beams u8, cost-model tiles (per-beam sampled outputs)")


@pytest.mark.parametrize("dtype,code", [("u8", DD_U8), ("f16", DD_F16)])
def test_batched_workload_tuned_sampled(dtype, code):
    """The configuration the benchmark times: the 64-beam batch built with
    per-beam tuning (Batch(..., tune=True, reps=1)) for u8 and f16 storage.
    Every beam's sampled outputs against the oracle on the stored values: u8
    bit for bit, f16 within the binary32 gates; errors reported per beam."""
    torch = torch_mod()
    beams = synth.batched_beams()
    plans = [Plan.from_setup(b) for b in beams]
    gen = {"u8": synth.noise_u8, "f16": synth.noise_f16}[dtype]
    xs_h = [gen(b.n_channels, p.input_samples, b.seed) for b, p in zip(beams, plans)]
    xs = [to_dev(x) for x in xs_h]
    batch = Batch(plans, dtype=code, tune=True, reps=1)
    assert batch.variants() == [p.get_tile(dtype=code) for p in plans]
    outs = [torch.full((b.n_dm, b.n_samples), float("nan"), device="cuda") for b in beams]
    batch.run(xs, outs)
    torch.cuda.synchronize()
    cfg = "batched 64 beams %s, tuned (per-beam sampled outputs)" % dtype
    for b, x, y in zip(beams, xs_h, outs):
        table = oracle.delay_table(*b.plan_args()[:7])
        i, t = sample_points(b.n_dm, b.n_samples, 400, b.seed + 1)
        yh = y[torch.from_numpy(i).long().cuda(), torch.from_numpy(t).long().cuda()].cpu().numpy()
        ref = oracle.dedisperse_points(x, table, i, t)
        if dtype == "u8":
            gates.exact(yh, ref, what=b.name, report=cfg)
        else:
            absref = oracle.dedisperse_points(np.abs(x.astype(np.float64)), table, i, t)
            gates.gate(yh, ref, absref, what=b.name, report=cfg + " vs f16 values")
    del xs, outs, batch
    torch.cuda.empty_cache()


def test_batch_run_rejects_bad_outputs_before_launch():
    """Outputs of the wrong dtype, shape, stride or count raise before any
    launch, and the caller's buffers are left untouched."""
    torch = torch_mod()
    beams = small_beams()[:2]
    plans = [Plan.from_setup(b) for b in beams]
    batch = Batch(plans)
    xs = [to_dev(synth.integers_f32(b.n_channels, p.input_samples, seed=3)) for b, p in zip(beams, plans)]
    good = [torch.full((b.n_dm, b.n_samples), float("nan"), device="cuda") for b in beams]
    bad_sets = [
        [good[0], torch.full((beams[1].n_dm, beams[1].n_samples), float("nan"), device="cuda",
                             dtype=torch.float16)],
        [good[0], torch.full((beams[1].n_dm - 1, beams[1].n_samples), float("nan"), device="cuda")],
        [good[0], torch.full((beams[1].n_dm, beams[1].n_samples - 1), float("nan"), device="cuda")],
        [good[0], torch.full((beams[1].n_samples, beams[1].n_dm), float("nan"), device="cuda").t()],
        [good[0]],
        [good[0], torch.full((beams[1].n_dm, beams[1].n_samples), float("nan"))],   # host tensor
    ]
    for outs in bad_sets:
        with pytest.raises((ValueError, TypeError)):
            batch.run(xs, outs)
    torch.cuda.synchronize()
    assert all(bool(torch.isnan(o).all()) for o in good)
    with pytest.raises((ValueError, TypeError)):
        batch.run([xs[0], xs[1].cpu()], good)


def test_batch_autotune_uses_tuned_tiles_and_stays_exact():
    """Per-beam tuning (dd_batch_autotune) stores each plan's fastest tile;
    the batch runs with exactly those tiles and still reproduces the oracle
    bit for bit on integer data."""
    torch = torch_mod()
    beams = small_beams()[:5]
    plans = [Plan.from_setup(b) for b in beams]
    batch = Batch(plans, tune=True, reps=1)
    assert batch.variants() == [p.get_tile() for p in plans]
    xs_h = [synth.integers_f32(b.n_channels, p.input_samples, seed=70 + i) for i, (b, p) in enumerate(zip(beams, plans))]
    outs = batch.run([to_dev(x) for x in xs_h])
    torch.cuda.synchronize()
    for b, x, y in zip(beams, xs_h, outs):
        table = oracle.delay_table(*b.plan_args()[:7])
        gates.exact(to_host(y), oracle.dedisperse(x, table, b.n_samples), what=b.name)
