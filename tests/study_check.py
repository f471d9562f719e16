"""Every tile variant of the auto-tuning study's library, bit for bit against
the oracle on integer-valued inputs (run by tests/test_gpu_study.py in a
process of its own, with DEDISP_LIBRARY naming the study library).

Shapes: the ragged forward and adjoint shapes of the main tests, and a
256-DM Apertif-band and a 64-DM LOFAR-band instance of one second of data
(sampled outputs), the study's own instance shapes.  Prints one line per shape
and the number of variants run; exits non-zero on the first mismatch."""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402
from paper_1601_05052_amd import DD_ADJOINT, DD_FORWARD, Plan, dedisperse, dedisperse_adjoint, tile_variants  # noqa: E402
from tests import gates  # noqa: E402
from tests.gpu_util import sample_points, to_dev, to_host, torch_mod  # noqa: E402
from tests.test_gpu_forward import RAGGED, set_tile_or_skip  # noqa: E402


def main():
    torch = torch_mod()
    variants = [v[0] for v in tile_variants()]
    assert len(variants) > 100, "not the study library: %d variants" % len(variants)
    total = 0
    for args in RAGGED:
        C, D, S = args[0], args[6], args[7]
        plan = Plan(*args)
        table = oracle.delay_table(*args[:7])
        T = plan.input_samples
        x = synth.integers_f32(C, T + 3, seed=C * 7 + D)
        ref = oracle.dedisperse(x, table, S)
        gy = synth.integers_f32(D, S + 2, seed=D)
        aref = oracle.adjoint(gy[:, :S], table, T)
        xd, gyd = to_dev(x), to_dev(gy)
        ran = [0, 0]
        for vid in variants:
            if set_tile_or_skip(plan, vid):
                gates.exact(to_host(dedisperse(xd, plan)), ref, what="fwd C%d variant %d" % (C, vid))
                ran[0] += 1
            if set_tile_or_skip(plan, vid, direction=DD_ADJOINT):
                gates.exact(to_host(dedisperse_adjoint(gyd, plan)), aref, what="adj C%d variant %d" % (C, vid))
                ran[1] += 1
        print("C=%d D=%d S=%d: forward %d variants, adjoint %d variants exact" % (C, D, S, ran[0], ran[1]),
              flush=True)
        total += sum(ran)
    import dataclasses
    for base, n_dm in ((synth.APERTIF, 256), (synth.LOFAR, 64)):
        st = dataclasses.replace(base, n_dm=n_dm)
        plan = Plan.from_setup(st)
        table = oracle.delay_table(*st.plan_args()[:7])
        x = synth.integers_f32(st.n_channels, plan.input_samples, seed=11)
        i, t = sample_points(st.n_dm, st.n_samples, 4000, 12)
        ref = oracle.dedisperse_points(x, table, i, t)
        xd = to_dev(x)
        out = torch.empty((st.n_dm, st.n_samples), device="cuda")
        it, tt = torch.from_numpy(i.astype(np.int64)).cuda(), torch.from_numpy(t).cuda()
        ran = 0
        for vid in variants:
            if not set_tile_or_skip(plan, vid):
                continue
            out.fill_(float("nan"))
            dedisperse(xd, plan, out=out)
            gates.exact(to_host(out[it, tt]), ref, what="%s %d DMs variant %d" % (st.name, n_dm, vid))
            ran += 1
        print("%s %d DMs: %d variants exact on %d sampled outputs" % (st.name, n_dm, ran, i.size), flush=True)
        total += ran
    print("study library: %d variants, %d variant-shape checks exact" % (len(variants), total), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
