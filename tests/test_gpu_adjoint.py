"""Adjoint kernel and the autograd wrapper against the FP64 oracle."""
import numpy as np
import pytest

import oracle
import synth
from paper_1601_05052_amd import DD_ADJOINT, Dedisperse, Plan, dedisperse, dedisperse_adjoint, tile_variants
from tests import gates
from tests.test_gpu_forward import set_tile_or_skip
from tests.gpu_util import oracle_delays, sample_points, to_dev, to_host, torch_mod

pytestmark = pytest.mark.gpu


def test_adjoint_tiny_vs_oracle():
    s = synth.TINY
    plan = Plan.from_setup(s)
    table = oracle_delays(s)
    T = plan.input_samples
    gy = synth.noise_f32(s.n_dm, s.n_samples, seed=21)
    gx = to_host(dedisperse_adjoint(to_dev(gy), plan))
    assert gx.shape == (s.n_channels, T)
    ref = oracle.adjoint(gy, table, T)
    absref = oracle.adjoint(np.abs(gy.astype(np.float64)), table, T)
    gates.gate(gx, ref, absref, what="adjoint tiny", report="tiny adjoint")


RAGGED = [
    (37, 1400.0, 2.5, 5e-5, 0.0, 0.75, 77, 1001),
    (5, 140.0, 0.2, 5e-6, 0.0, 0.02, 9, 3333),
    (1, 1400.0, 1.0, 5e-5, 0.0, 1.0, 1, 1),
    (130, 1420.0, 300.0 / 130, 5e-5, 10.0, 0.25, 33, 515),
]
# Variants that must fit each shape's adjoint (host count when the list was
# last changed: 31, 28, 46 and 46 of 46).
MIN_ADJ_VARIANTS = {37: 28, 5: 25, 1: 46, 130: 42}


@pytest.mark.parametrize("args", RAGGED, ids=lambda a: "C%d_D%d_S%d" % (a[0], a[6], a[7]))
def test_adjoint_every_variant_integer_exact(args):
    C, D, S = args[0], args[6], args[7]
    plan = Plan(*args)
    table = oracle.delay_table(*args[:7])
    T = plan.input_samples
    gy = synth.integers_f32(D, S + 2, seed=D)
    ref = oracle.adjoint(gy[:, :S], table, T)
    gyd = to_dev(gy)
    ran = 0
    for vid, *_ in tile_variants():
        if not set_tile_or_skip(plan, vid, direction=DD_ADJOINT):
            continue
        gx = to_host(dedisperse_adjoint(gyd, plan))
        gates.exact(gx, ref, what="adjoint variant %d" % vid)
        ran += 1
    assert ran >= MIN_ADJ_VARIANTS[C], (ran, MIN_ADJ_VARIANTS[C])


def test_adjoint_writes_zeros_and_keeps_padding():
    torch = torch_mod()
    s = synth.TINY
    plan = Plan.from_setup(s)
    T = plan.input_samples
    gy = torch.zeros((s.n_dm, s.n_samples), device="cuda")
    out = torch.full((s.n_channels, T + 9), float("nan"), device="cuda")
    dedisperse_adjoint(gy, plan, out=out)
    o = to_host(out)
    assert np.all(o[:, :T] == 0.0)
    assert np.all(np.isnan(o[:, T:]))


@pytest.mark.parametrize("setup", [synth.APERTIF, synth.LOFAR], ids=lambda s: s.name)
def test_dot_product_full_size(setup):
    """<A x, y> = <x, A^T y> with GPU A and A^T, inner products in FP64."""
    plan = Plan.from_setup(setup)
    T = plan.input_samples
    x = synth.noise_f32(setup.n_channels, T, seed=31)
    gy = synth.noise_f32(setup.n_dm, setup.n_samples, seed=32)
    ax = to_host(dedisperse(to_dev(x), plan)).astype(np.float64)
    aty = to_host(dedisperse_adjoint(to_dev(gy), plan)).astype(np.float64)
    lhs = float(np.dot(ax.ravel(), gy.astype(np.float64).ravel()))
    rhs = float(np.dot(x.astype(np.float64).ravel(), aty.ravel()))
    scale = float(np.dot(np.abs(ax).ravel(), np.abs(gy).astype(np.float64).ravel()))
    assert abs(lhs - rhs) <= 1e-6 * scale, (lhs, rhs, scale)


@pytest.mark.parametrize("s", [synth.APERTIF, synth.LOFAR], ids=lambda s: s.name)
def test_adjoint_whole_channel_rows(s):
    """Full-size adjoint (the plan's own variant: rows outside each tile's span
    skipped; on LOFAR rows summed in blocks over launches) checked on whole
    channel rows against the oracle, bit for bit on integer values."""
    plan = Plan.from_setup(s)
    table = oracle_delays(s)
    T = plan.input_samples
    gy = synth.integers_f32(s.n_dm, s.n_samples, seed=41, lo=-3, hi=3)
    gx = to_host(dedisperse_adjoint(to_dev(gy), plan))
    for ch in (0, s.n_channels // 2 - 1, s.n_channels - 1):
        sub = table[:, ch:ch + 1]
        ref = oracle.adjoint(gy, np.ascontiguousarray(sub), T)[0]
        gates.exact(gx[ch], ref, what="adjoint ch %d" % ch)


@pytest.mark.parametrize("s", [synth.APERTIF, synth.LOFAR], ids=lambda s: s.name)
def test_adjoint_full_size_float_rows(s):
    """Full-size adjoint of N(0,1) gradient rows with the plan's variant (the
    configuration the benchmark's adjoint extras time after tuning picks the
    same kind): whole channel rows against the FP64 oracle, gated and
    reported."""
    plan = Plan.from_setup(s)
    table = oracle_delays(s)
    T = plan.input_samples
    gy = synth.noise_f32(s.n_dm, s.n_samples, seed=44)
    gx = to_host(dedisperse_adjoint(to_dev(gy), plan))
    chans = [0, s.n_channels // 3, s.n_channels - 1]
    sub = np.ascontiguousarray(table[:, chans])
    ref = oracle.adjoint(gy, sub, T)
    absref = oracle.adjoint(np.abs(gy.astype(np.float64)), sub, T)
    for k, ch in enumerate(chans):
        gates.gate(gx[ch], ref[k], absref[k], what="%s adjoint ch %d" % (s.name, ch),
                   report="%s adjoint (plan's variant, whole channel rows)" % s.name)


@pytest.mark.parametrize("s", [synth.APERTIF, synth.LOFAR], ids=lambda s: s.name)
def test_adjoint_full_size_every_fitting_variant(s):
    """The benchmark tunes the adjoint and times whichever variant wins, so
    every variant that fits the full-size adjoint is checked, bit for bit on
    integer values, on three whole channel rows."""
    plan = Plan.from_setup(s)
    table = oracle_delays(s)
    T = plan.input_samples
    gy = synth.integers_f32(s.n_dm, s.n_samples, seed=43, lo=-3, hi=3)
    chans = (0, s.n_channels // 2, s.n_channels - 1)
    refs = {ch: oracle.adjoint(gy, np.ascontiguousarray(table[:, ch:ch + 1]), T)[0] for ch in chans}
    gyd = to_dev(gy)
    checked = 0
    for vid, *_ in tile_variants():
        if not set_tile_or_skip(plan, vid, direction=DD_ADJOINT):
            continue
        gx = dedisperse_adjoint(gyd, plan)
        for ch in chans:
            gates.exact(to_host(gx[ch]), refs[ch], what="%s adjoint variant %d ch %d" % (s.name, vid, ch))
        checked += 1
    plan.set_tile(-1, direction=DD_ADJOINT)
    assert checked >= 5


def _loss_grad_reference(x, w, table, S):
    """Gradient of sum w * (A x)^2 is 2 A^T (w * A x), all in FP64."""
    y = oracle.dedisperse(x, table, S)
    return y, oracle.adjoint(2.0 * w * y, table, x.shape[1])


def test_autograd_fd_slice():
    """16-ch x 32-DM x 256-sample slice: the autograd gradient matches the
    FP64 gradient, and central finite differences of the FP64 loss (exact for
    this quadratic loss with integer x, dyadic w, h = 1) match it too."""
    torch = torch_mod()
    s = synth.FD_SLICE
    plan = Plan.from_setup(s)
    table = oracle_delays(s)
    T = plan.input_samples
    x = synth.integers_f32(s.n_channels, T, seed=51, lo=-4, hi=4)
    w = (np.random.default_rng(52).integers(0, 16, size=(s.n_dm, s.n_samples)) / 16.0).astype(np.float32)
    xt = to_dev(x).requires_grad_(True)
    wt = to_dev(w)
    out = Dedisperse.apply(xt, plan)
    loss = (wt * out * out).sum()
    loss.backward()
    g = to_host(xt.grad)
    _, gref = _loss_grad_reference(x.astype(np.float64), w.astype(np.float64), table, s.n_samples)
    gates.exact(g, gref, what="autograd gradient")

    def loss64(xx):
        y = oracle.dedisperse(xx, table, s.n_samples)
        return float(np.sum(w.astype(np.float64) * y * y))

    def loss_gpu(xx):
        """The differentiated function itself: the GPU forward of xx, then the
        loss summed in binary64 on the device (every output is an integer and
        w has four fractional bits, so every partial sum is exact)."""
        y = dedisperse(to_dev(xx.astype(np.float32)), plan).double()
        return float((wt.double() * y * y).sum().item())

    rng = np.random.default_rng(53)
    x64 = x.astype(np.float64)
    for _ in range(24):
        ch, tau = int(rng.integers(0, s.n_channels)), int(rng.integers(0, T))
        xp, xm = x64.copy(), x64.copy()
        xp[ch, tau] += 1.0
        xm[ch, tau] -= 1.0
        fd = (loss64(xp) - loss64(xm)) / 2.0
        fd_gpu = (loss_gpu(xp) - loss_gpu(xm)) / 2.0
        assert fd == fd_gpu == gref[ch, tau] == g[ch, tau], (ch, tau, fd, fd_gpu, gref[ch, tau], g[ch, tau])


def test_autograd_apertif_beam_vs_oracle_sampled():
    """One Apertif-shaped beam of the fwd+bwd workload: the gradient of
    sum w * out^2 against the FP64 chain 2 A^T (w * A x) on whole channel
    rows.  The componentwise bound uses the magnitude of every term the GPU
    rounds: |2 w| * (|A x| + A|x|) pushed through A^T."""
    s = synth.fwd_bwd_beams(1)[0]
    plan = Plan.from_setup(s)
    table = oracle_delays(s)
    T = plan.input_samples
    x = synth.noise_f32(s.n_channels, T, seed=s.seed)
    w = synth.uniform_f32(s.n_dm, s.n_samples, seed=s.seed + 1000)
    xt = to_dev(x).requires_grad_(True)
    out = Dedisperse.apply(xt, plan)
    (to_dev(w) * out * out).sum().backward()
    g = to_host(xt.grad)
    chans = [0, 700, 1023]
    sub = np.ascontiguousarray(table[:, chans])
    w64 = w.astype(np.float64)
    yref = oracle.dedisperse(x, table, s.n_samples)
    yabs = oracle.dedisperse(np.abs(x.astype(np.float64)), table, s.n_samples)
    gref = oracle.adjoint(2.0 * w64 * yref, sub, T)
    bound = oracle.adjoint(2.0 * w64 * (np.abs(yref) + yabs), sub, T)
    for k, ch in enumerate(chans):
        gates.gate(g[ch], gref[k], bound[k], what="grad ch %d" % ch,
                   report="fwd+bwd gradient of sum w*out^2 (Apertif beam, whole channel rows)")


def test_row_blocked_direct_variants_bit_identical():
    """The direct kind summing rows in blocks over successive launches (partial
    sums carried in the output), with strided or consecutive (16-byte load)
    ownership, adds the rows in the same order as the single-launch form:
    bit-identical results on float data, several blocks."""
    args = (32, 138.0, 0.1875, 5e-6, 0.0, 0.01, 600, 5000)
    plan = Plan(*args)
    table = oracle.delay_table(*args[:7])
    T = plan.input_samples
    gy = synth.noise_f32(600, 5000, seed=17)
    gyd = to_dev(gy)
    outs = {}
    for vid, it, acc, waves, kind in tile_variants():
        if kind != 2:
            continue
        plan.set_tile(vid, direction=DD_ADJOINT)
        outs[vid] = to_host(dedisperse_adjoint(gyd, plan))
    assert {41, 43, 44, 45} <= set(outs)
    for vid in outs:  # every direct variant adds the rows in the same order
        assert np.array_equal(outs[vid], outs[41]), vid
    ref = oracle.adjoint(gy, table, T)
    absref = oracle.adjoint(np.abs(gy.astype(np.float64)), table, T)
    gates.gate(outs[43], ref, absref, what="blocked direct adjoint")
