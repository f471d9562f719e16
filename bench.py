"""Benchmark: brute-force dedispersion throughput on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload apertif|lofar]
                    [--no-extra] [--no-cpu-baseline]

A step is one forward dedispersion of one beam (Sclocco et al., Algorithm 1)
with the input already resident in HBM: one launch of the library's kernel.
The headline workload is the Apertif-shaped beam (1,024 channels over
1,420-1,720 MHz, 20,000 samples/s, 20,000 output samples, 2,048 trial DMs
0-511.75 step 0.25, float32 N(0,1) noise + 4 pulses).  Throughput is GFLOP/s
with one FLOP per (DM, sample, channel) addition, the paper's convention.

Printed: ONE JSON line with the headline figure, the roofline of the kernel,
the CPU oracle's throughput on a bounded sample, and (unless --no-extra)
secondary same-GPU measurements: LOFAR-shaped beam, u8/f16 storage, the
adjoint and fwd+bwd step, and the 64-beam batched launch.
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import re
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import synth  # noqa: E402

HBM_PEAK_GBPS = 8000.0
# binary32 adds: 256 CUs x 128 lanes/clk x 2.4 GHz (the published 157.3
# TFLOP/s vector FP32 figure counts a fused multiply-add as two FLOPs).
ADD_PEAK_TFLOPS = 256 * 128 * 2.4e9 / 1e12


PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["paper_1601_05052_amd/csrc/" + n for n in (
    "srs_regwin.h", "regwin_asm.h", "srs_tile.h", "srs_dims.h", "srs_launch.h", "srs_inst.inc", "srs_kernels_f32.hip",
    "variants.cpp", "plan.cpp")]
VARIANT_LIST = "paper_1601_05052_amd/csrc/srs_variants.def"


_T0 = time.monotonic()


def log(msg):
    """Progress line on stderr, prefixed by the seconds since start."""
    print("[%6.1fs] %s" % (time.monotonic() - _T0, msg), file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the sources that determine the kernels' code and tables (the
    variant list enters per variant, see variant_entry)."""
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def variant_entry(variant):
    """The variant's entry in the variant list, without its cost-model rate and
    comments (which do not change its code); None if there is no such entry."""
    with open(os.path.join(ROOT, VARIANT_LIST)) as f:
        text = re.sub(r"/\*.*?\*/|//[^\n]*", "", f.read(), flags=re.S)
    for m in re.finditer(r"X_\w+\(\s*(\d+)\s*,[^)]*\)", text):
        if int(m.group(1)) == variant:
            return re.sub(r"\s+", "", re.sub(r",\s*[0-9.]+f\)", ")", m.group(0)))
    return None


def measured_traffic(workload, variant):
    """HBM-side bytes per launch from the committed counter summary, only if it
    was taken on the current kernel sources and the same variant entry."""
    path = os.path.join(PROFILES, "traffic_%s_fwd.json" % workload)
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_hash") != kernel_source_hash():
        return None
    rec = t.get("by_variant", {}).get(str(variant))
    if not rec or rec.get("entry") != variant_entry(variant):
        return None
    return rec.get("bytes")


def vdesc(r):
    """The tile variant of a measurement, or its row split [(first row, variant)]."""
    b = r.get("blocks") or []
    return "variant %d" % r["tile"] if len(b) <= 1 else "row blocks %s" % b


def compulsory_bytes(setup, in_bytes_per_sample, plan):
    """Each input sample read once, each output written once (Eq. (3)'s
    reuse limit), plus the delay table."""
    return (setup.n_channels * plan.input_samples * in_bytes_per_sample
            + setup.n_dm * setup.n_samples * 4 + setup.n_dm * setup.n_channels * 4)


def timed(torch, fn, steps, warmup, stream):
    """Back-to-back launches: mean ms per call over `steps` calls between two
    HIP events on `stream` (caches stay warm between calls), and wall seconds."""
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(steps):
        fn()
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return e0.elapsed_time(e1) / steps, wall


FLUSH_BYTES = 1 << 30   # > the 256 MiB MALL: every timed call starts with cold caches
_FLUSH = []


def flush_caches(torch, stream):
    """Write a 1 GiB scratch buffer on `stream` (evicts the MALL and L2)."""
    if not _FLUSH:
        _FLUSH.append(torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device="cuda"))
    with torch.cuda.stream(stream):
        _FLUSH[0].fill_(float(len(_FLUSH)))


def timed_protocol(torch, fn, steps, warmup, stream):
    """The measurement protocol: `warmup` untimed calls, `steps` back-to-back
    calls (warm caches; their mean is reported as a second figure), then
    `steps` timed calls, each after a 1 GiB scratch write and between its own
    pair of HIP events on `stream` (the stream the library launches on).
    Returns mean, min and standard deviation of those per-call times."""
    warm, _ = timed(torch, fn, steps, warmup, stream)   # warm-up calls, then the back-to-back figure
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    t0 = time.perf_counter()
    for e0, e1 in ev:
        flush_caches(torch, stream)
        e0.record(stream)
        fn()
        e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    return dict(ms=float(per.mean()), ms_min=float(per.min()), ms_std=float(per.std()), ms_warm=warm,
                wall_s=wall, reps=steps)


def gpu_input(torch, setup, T, dtype, seed):
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    z = torch.randn((setup.n_channels, T), generator=g, device="cuda", dtype=torch.float32)
    if dtype == "f32":
        return z
    if dtype == "f16":
        return z.half()
    return torch.clamp(torch.round(z * 16 + 128), 0, 255).to(torch.uint8)


def measure_forward(torch, dd, setup, dtype, steps, warmup, stream, numpy_input=None, tune=True, tune_cache=None):
    plan = dd.Plan.from_setup(setup)
    T = plan.input_samples
    if numpy_input is not None:
        x = torch.from_numpy(numpy_input).to("cuda")
    else:
        x = gpu_input(torch, setup, T, dtype, setup.seed)
    out = torch.empty((setup.n_dm, setup.n_samples), dtype=torch.float32, device="cuda")
    code = {"f32": dd.DD_F32, "f16": dd.DD_F16, "u8": dd.DD_U8}[dtype]
    if tune:
        plan.autotune(dd.DD_FORWARD, code, reps=3, cache_path=tune_cache)   # Sec. IV-A: tune, then measure
    plan.prepare(dd.DD_FORWARD, code)
    t = timed_protocol(torch, lambda: dd.dedisperse(x, plan, out=out), steps, warmup, stream)
    bpe = {"f32": 4, "f16": 2, "u8": 1}[dtype]
    return dict(t, gflops=setup.adds / (t["ms"] * 1e-3) / 1e9,
                compulsory_bytes=compulsory_bytes(setup, bpe, plan), tile=plan.get_tile(dtype=code),
                blocks=plan.get_blocks(dtype=code)), plan


def measure_adjoint(torch, dd, setup, steps, warmup, stream, tune_cache=None):
    """Tuned adjoint of one beam: gradient rows [D][S] -> [C][T_in]."""
    plan = dd.Plan.from_setup(setup)
    plan.autotune(dd.DD_ADJOINT, dd.DD_F32, reps=3, cache_path=tune_cache)
    plan.prepare(dd.DD_ADJOINT, dd.DD_F32)
    g = torch.Generator(device="cuda")
    g.manual_seed(setup.seed)
    gy = torch.randn((setup.n_dm, setup.n_samples), generator=g, device="cuda")
    gx = torch.empty((setup.n_channels, plan.input_samples), device="cuda")
    t = timed_protocol(torch, lambda: dd.dedisperse_adjoint(gy, plan, out=gx), steps, warmup, stream)
    return dict(t, gflops=setup.adds / (t["ms"] * 1e-3) / 1e9,
                compulsory_bytes=compulsory_bytes(setup, 4, plan), tile=plan.get_tile(direction=dd.DD_ADJOINT),
                blocks=plan.get_blocks(direction=dd.DD_ADJOINT))


def cpu_baseline(setup, budget_s=12.0):
    """The FP64 oracle on a bounded sample of the workload: the full input,
    the first n trial DMs, n chosen so the timed run takes ~budget_s."""
    import oracle
    table = oracle.delay_table(*setup.plan_args()[:7])
    T = setup.n_samples + int(table.max())
    arrivals = {i: table[i] for i, _ in synth.pulse_sites(setup)}
    x = synth.make_input(setup, T, "f32", arrivals=arrivals).astype(np.float64)
    n = 4
    t0 = time.perf_counter()
    oracle.dedisperse(x, table[:n], setup.n_samples)
    probe = time.perf_counter() - t0
    n_dm = int(min(setup.n_dm, max(n, budget_s / max(probe, 1e-6) * n)))
    reps, dt = 0, 0.0
    while reps == 0 or (dt < budget_s and reps < 50):
        t0 = time.perf_counter()
        oracle.dedisperse(x, table[:n_dm], setup.n_samples)
        dt += time.perf_counter() - t0
        reps += 1
    adds = reps * n_dm * setup.n_samples * setup.n_channels
    return {"value": adds / dt / 1e9, "unit": "GFLOP/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": cpu_model(), "nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0)),
            "sample": "%s input, first %d of %d trial DMs, all %d channels x %d samples, %d run(s) "
                      "(%.2e adds in %.1f s)" % (setup.name, n_dm, setup.n_dm, setup.n_channels,
                                                 setup.n_samples, reps, adds, dt)}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_bandwidth(torch, stream, n_bytes=256 << 20, reps=10):
    """Device-to-device copy of n_bytes (read + write 2 * n_bytes per copy):
    the achievable HBM rate the kernels' traffic is compared with, and the
    reference dispatch for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    src = torch.empty(n_bytes // 4, dtype=torch.float32, device="cuda").normal_()
    dst = torch.empty_like(src)
    t = timed_protocol(torch, lambda: dst.copy_(src), reps, 2, stream)
    del src, dst
    return dict(bytes_moved=2 * n_bytes, ms=t["ms"], GBps=2 * n_bytes / (t["ms"] * 1e-3) / 1e9,
                ms_warm=t["ms_warm"])


def realtime(torch, dd, stream, n_chunks):
    """Real-time check (Sec. V, V-D): one-second u8 chunks of an Apertif-shaped
    beam pushed from pinned host memory; the host-to-device copy of each chunk
    overlaps the previous chunk's kernels.  Beams per GPU = one second of data
    over the time per pushed second (copies included)."""
    s = synth.APERTIF
    plan = dd.Plan.from_setup(s)
    plan.autotune(dd.DD_FORWARD, dd.DD_U8, reps=3)
    rt = dd.Realtime(plan, torch.uint8)
    g = torch.Generator().manual_seed(s.seed)
    chunks = [torch.randint(0, 256, (s.n_channels, s.n_samples), dtype=torch.uint8, generator=g).pin_memory()
              for _ in range(2)]
    outs = [torch.empty((s.n_dm, s.n_samples), device="cuda") for _ in range(2)]
    k = [0]

    def push():
        rt.push(chunks[k[0] % 2], out=outs[k[0] % 2])
        k[0] += 1

    ms_ev, wall = timed(torch, push, n_chunks, 3, stream)
    ms = max(ms_ev, wall / n_chunks * 1e3)
    dev = torch.empty((s.n_channels, s.n_samples), dtype=torch.uint8, device="cuda")
    ms_h2d, _ = timed(torch, lambda: dev.copy_(chunks[0], non_blocking=True), n_chunks, 2, stream)
    chunk_s = s.n_samples * s.t_samp
    rt.close()
    r = dict(ms_per_chunk=ms, chunk_seconds=chunk_s, realtime_beams_per_gpu=chunk_s / (ms * 1e-3),
             gflops_incl_copies=s.adds / (ms * 1e-3) / 1e9, h2d_ms=ms_h2d,
             h2d_GBps=s.n_channels * s.n_samples / (ms_h2d * 1e-3) / 1e9, tile=plan.get_tile(dtype=dd.DD_U8),
             note="pinned u8 chunks, copy stream + compute stream, wall clock per pushed second")
    log("realtime apertif u8: %.3f ms per 1 s chunk (H2D alone %.3f ms, %.1f GB/s): %.0f beams in real time"
        % (ms, ms_h2d, r["h2d_GBps"], r["realtime_beams_per_gpu"]))
    return r


EXTRAS = ("lofar_f32", "lofar_adjoint", "apertif_u8", "apertif_f16", "apertif_0dm", "lofar_0dm", "search_apertif",
          "realtime_apertif_u8", "apertif_adjoint", "fwd_bwd_8beams", "batched64_u8", "batched64_f16")


def extras(torch, dd, stream, steps, only=None):
    """Secondary same-GPU measurements (names in EXTRAS; `only`: a subset)."""
    want = (lambda name: True) if not only else (lambda name: name in only)
    res = {}
    # LOFAR-shaped beam, float32
    if want("lofar_f32"):
        r, _ = measure_forward(torch, dd, synth.LOFAR, "f32", steps, 2, stream)
        r["hbm_GBps"] = r["compulsory_bytes"] / (r["ms"] * 1e-3) / 1e9
        res["lofar_f32"] = r
        log("lofar f32: %.3f ms %.1f GFLOP/s (%s)" % (r["ms"], r["gflops"], vdesc(r)))
    if want("lofar_adjoint"):
        r = measure_adjoint(torch, dd, synth.LOFAR, steps, 2, stream)
        res["lofar_adjoint"] = r
        log("lofar adjoint: %.3f ms (%s)" % (r["ms"], vdesc(r)))
    # low precision storage, Apertif
    for dt in ("u8", "f16"):
        if want("apertif_" + dt):
            r, _ = measure_forward(torch, dd, synth.APERTIF, dt, steps, 2, stream)
            res["apertif_" + dt] = r
            log("apertif %s: %.3f ms %.1f GFLOP/s (%s)" % (dt, r["ms"], r["gflops"], vdesc(r)))
    # perfect-reuse limit (Sec. IV-C / V-C): every trial DM is 0, tuned again
    for base in (synth.APERTIF, synth.LOFAR):
        z = dataclasses.replace(base, name=base.name + "_0dm", dm_step=0.0)
        if want(z.name):
            r, _ = measure_forward(torch, dd, z, "f32", steps, 2, stream)
            res[z.name] = r
            log("%s: %.3f ms %.1f GFLOP/s (%s)" % (z.name, r["ms"], r["gflops"], vdesc(r)))
    # candidate search over the dedispersed Apertif rows (boxcars of 1 .. 1,024 samples)
    if want("search_apertif"):
        sp = dd.Plan.from_setup(synth.APERTIF)
        sy = dd.dedisperse(gpu_input(torch, synth.APERTIF, sp.input_samples, "f32", synth.APERTIF.seed), sp)
        t = timed_protocol(torch, lambda: dd.search_boxcar(sy, n_widths=11), steps, 2, stream)
        ms_s = t["ms"]
        res["search_apertif"] = dict(t, n_widths=11, rows_bytes=sy.numel() * 4,
                                     rows_GBps=sy.numel() * 4 / (ms_s * 1e-3) / 1e9)
        log("search apertif (11 widths): %.3f ms, %.0f GB/s of rows" % (ms_s, res["search_apertif"]["rows_GBps"]))
        del sy
    # streaming: one Apertif beam fed second by second from pinned host memory
    if want("realtime_apertif_u8"):
        res["realtime_apertif_u8"] = realtime(torch, dd, stream, max(10, steps // 2))
    # adjoint and fwd+bwd (8 Apertif-shaped beams through autograd)
    if want("apertif_adjoint") or want("fwd_bwd_8beams"):
        res.update(fwd_bwd(torch, dd, stream, steps, want))
    # batched: 64 uneven beams, one graph launch (one kernel per tile variant in use)
    for dt, code in (("u8", dd.DD_U8), ("f16", dd.DD_F16)):
        if not want("batched64_" + dt):
            continue
        beams = synth.batched_beams()
        plans = [dd.Plan.from_setup(b) for b in beams]
        xs = [gpu_input(torch, b, p.input_samples, dt, b.seed) for b, p in zip(beams, plans)]
        outs = [torch.empty((b.n_dm, b.n_samples), device="cuda") for b in beams]
        batch = dd.Batch(plans, dtype=code, tune=True, reps=1)
        ms_b, _ = timed(torch, lambda: batch.run(xs, outs), max(2, steps // 4), 1, stream)

        # same beams one plain launch each (same storage type)
        def singles():
            for x, p, o in zip(xs, plans, outs):
                dd.dedisperse(x, p, out=o)
        ms_s, _ = timed(torch, singles, max(2, steps // 4), 1, stream)
        res["batched64_" + dt] = dict(ms=ms_b, gflops=batch.adds / (ms_b * 1e-3) / 1e9,
                                      per_beam_launches_ms=ms_s, speedup_over_per_beam=ms_s / ms_b,
                                      adds=batch.adds, variants=sorted(set(batch.variants())),
                                      kernels_in_graph=len(set(batch.variants())),
                                      note="back-to-back graph launches (each writes 14.5 GB of outputs)")
        log("batched %s: %.3f ms (%.1f GFLOP/s), per-beam launches %.3f ms, variants %s"
            % (dt, ms_b, batch.adds / (ms_b * 1e-3) / 1e9, ms_s, sorted(set(batch.variants()))))
        del xs, outs, batch
        torch.cuda.empty_cache()
    return res


def fwd_bwd(torch, dd, stream, steps, want):
    """The Apertif adjoint alone, and fwd+bwd of 8 Apertif-shaped beams
    through autograd (loss sum w * out^2)."""
    res = {}
    beams = synth.fwd_bwd_beams()
    plans = [dd.Plan.from_setup(b) for b in beams]
    import tempfile
    with tempfile.TemporaryDirectory() as tmp:
        cache = os.path.join(tmp, "tune.txt")   # the 8 beams share one shape: tune once
        for p in plans:
            p.autotune(dd.DD_FORWARD, dd.DD_F32, reps=3, cache_path=cache)
            p.autotune(dd.DD_ADJOINT, dd.DD_F32, reps=3, cache_path=cache)
            p.prepare(dd.DD_FORWARD, dd.DD_F32)
            p.prepare(dd.DD_ADJOINT, dd.DD_F32)
    if want("apertif_adjoint"):
        gy = torch.randn((beams[0].n_dm, beams[0].n_samples), device="cuda")
        gx0 = torch.empty((beams[0].n_channels, plans[0].input_samples), device="cuda")
        t = timed_protocol(torch, lambda: dd.dedisperse_adjoint(gy, plans[0], out=gx0), steps, 2, stream)
        ms_adj = t["ms"]
        res["apertif_adjoint"] = dict(t, gflops=beams[0].adds / (ms_adj * 1e-3) / 1e9,
                                      tile=plans[0].get_tile(direction=dd.DD_ADJOINT),
                                      blocks=plans[0].get_blocks(direction=dd.DD_ADJOINT))
        del gx0, gy
        log("apertif adjoint: %.3f ms (%s)" % (ms_adj, vdesc(res["apertif_adjoint"])))
    if not want("fwd_bwd_8beams"):
        return res
    xs = [gpu_input(torch, b, p.input_samples, "f32", b.seed).requires_grad_(True) for b, p in zip(beams, plans)]
    ws = [torch.rand((b.n_dm, b.n_samples), device="cuda",
                     generator=torch.Generator(device="cuda").manual_seed(b.seed + 1)) for b in beams]

    def step():
        for x, p, w in zip(xs, plans, ws):
            x.grad = None
            y = dd.Dedisperse.apply(x, p)
            (w * y * y).sum().backward()

    ms_fb, _ = timed(torch, step, max(2, steps // 4), 1, stream)
    with torch.no_grad():
        ms_f8, _ = timed(torch, lambda: [dd.dedisperse(x, p) for x, p in zip(xs, plans)], max(2, steps // 4), 1,
                         stream)
    adds_fb = 2 * sum(b.adds for b in beams)
    res["fwd_bwd_8beams"] = dict(ms=ms_fb, gflops=adds_fb / (ms_fb * 1e-3) / 1e9, forward_only_ms=ms_f8,
                                 over_forward_only=ms_fb / ms_f8,
                                 note="forward + adjoint adds of 8 beams per step, autograd incl. loss ops; "
                                      "forward_only_ms: the same 8 forwards without autograd; back-to-back "
                                      "steps (each step moves ~4 GB, far more than the caches hold)")
    log("fwd+bwd 8 beams: %.3f ms (forward only %.3f ms, x%.2f)" % (ms_fb, ms_f8, ms_fb / ms_f8))
    del xs, ws
    torch.cuda.empty_cache()
    return res


def tune_study(torch, dd, stream, reps=5):
    """Auto-tuning study (Sec. IV-A / IV-B, V-A / V-B): for each setup and each
    instance of 2^1 .. 2^12 trial DMs (one second of data), time every tile
    variant that fits, and report the optimum, the mean and spread over the
    optimisation space, the optimum's signal-to-noise ratio with its Chebyshev
    bound, the best single fixed variant per setup, and the cost model's
    untuned choice."""
    variants = [v[0] for v in dd.tile_variants()]
    study = []
    for base in (synth.APERTIF, synth.LOFAR):
        rows = []
        for e in range(1, 13):
            st = dataclasses.replace(base, name="%s_%d" % (base.name, 2 ** e), n_dm=2 ** e)
            plan = dd.Plan.from_setup(st)
            x = gpu_input(torch, st, plan.input_samples, "f32", st.seed)
            out = torch.empty((st.n_dm, st.n_samples), device="cuda")
            gf = {}
            for vid in variants:
                try:
                    plan.set_tile(vid)
                    ms, _ = timed(torch, lambda: dd.dedisperse(x, plan, out=out), reps, 2, stream)
                except dd.DedispError:
                    continue   # the tile's window does not fit this instance
                gf[vid] = st.adds / (ms * 1e-3) / 1e9
            plan.set_tile(-1)
            model = plan.get_tile()
            vals = np.array(list(gf.values()))
            best = max(gf, key=gf.get)
            snr = (gf[best] - vals.mean()) / vals.std() if vals.std() > 0 else float("inf")
            rows.append(dict(setup=base.name, n_dm=st.n_dm, n_variants=len(gf), best=best,
                             best_gflops=gf[best], mean_gflops=float(vals.mean()), std_gflops=float(vals.std()),
                             snr=snr, chebyshev_bound=min(1.0, 1.0 / snr ** 2) if snr > 0 else 1.0,
                             model_variant=model, model_gflops=gf.get(model),
                             realtime=st.adds / (gf[best] * 1e9) < st.n_samples * st.t_samp,
                             gflops={str(k): round(v, 1) for k, v in gf.items()}))
            log("%s %4d DMs: %d variants, best %d at %.0f GFLOP/s, mean %.0f, SNR %.2f, model %d"
                % (base.name, st.n_dm, len(gf), best, gf[best], vals.mean(), snr, model))
            del x, out
            torch.cuda.empty_cache()
        # best single fixed variant: fits every instance, highest geometric-mean rate
        common = set.intersection(*[set(int(k) for k in r["gflops"]) for r in rows])
        fixed = max(common, key=lambda v: sum(np.log(r["gflops"][str(v)]) for r in rows))
        for r in rows:
            r["fixed_variant"] = fixed
            r["tuned_over_fixed"] = r["best_gflops"] / r["gflops"][str(fixed)]
        study += rows
    return study


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="apertif", choices=["apertif", "lofar"])
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--extras", metavar="NAMES",
                    help="comma-separated subset of the extras (%s)" % ", ".join(EXTRAS))
    ap.add_argument("--adjoint", action="store_true",
                    help="time the adjoint of the workload in the headline slot (for its profile)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune-cache", default=None,
                    help="autotuner cache file for the headline slot (profiling runs reuse the choice a run "
                         "without counters made: counter collection slows short launches and skews the tuner)")
    ap.add_argument("--realtime", action="store_true",
                    help="only the streaming measurement (Apertif u8 chunks from pinned host memory), one JSON line")
    ap.add_argument("--tune-study", metavar="JSON",
                    help="run the auto-tuning study over 2..4096 DMs for both setups, write it here, exit "
                         "(over the study library's grid when DEDISP_LIBRARY names it)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="accepted for older profile commands: the 256 MiB copy always runs")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: beams are independent, so several GPUs would each run their own "
              "beams with no exchange; multi-GPU runs are not implemented (--gpus %d)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1601_05052_amd as dd
    assert torch.cuda.is_available(), "bench needs a GPU"
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    setup = synth.WORKLOADS[args.workload]
    if args.realtime:
        print(json.dumps(realtime(torch, dd, stream, args.steps)), flush=True)
        return
    if args.tune_study:
        study = tune_study(torch, dd, stream)
        with open(args.tune_study, "w") as f:
            with open(os.path.join(ROOT, VARIANT_LIST)) as vl:
                curated = len(re.findall(r"X_\w+\(\s*\d+\s*,", re.sub(r"/\*.*?\*/|//[^\n]*", "", vl.read(),
                                                                        flags=re.S)))
            json.dump({"library": os.path.basename(os.environ.get("DEDISP_LIBRARY") or "libdedisp.so"),
                       "curated": curated, "variants": [list(v) for v in dd.tile_variants()], "instances": study},
                      f, indent=1)
        return

    # Headline input: the seeded workload with its pulses (arrivals from the
    # library's own plan; the timing does not depend on the values).
    plan0 = dd.Plan.from_setup(setup)
    table = plan0.delays()
    arrivals = {i: table[i] for i, _ in synth.pulse_sites(setup)}
    x = synth.make_input(setup, plan0.input_samples, "f32", arrivals=arrivals)
    log("workload %s: C=%d D=%d S=%d T_in=%d" % (setup.name, setup.n_channels, setup.n_dm, setup.n_samples,
                                                  plan0.input_samples))
    if args.adjoint:
        r = measure_adjoint(torch, dd, setup, args.steps, args.warmup, stream, tune_cache=args.tune_cache)
    else:
        r, plan = measure_forward(torch, dd, setup, "f32", args.steps, args.warmup, stream, numpy_input=x,
                                  tune_cache=args.tune_cache)
    ms = r["ms"]
    log("%s f32: %.4f ms/step, %.1f GFLOP/s, %s" % ("adjoint" if args.adjoint else "forward", ms, r["gflops"],
                                                     vdesc(r)))
    achieved_tflops = setup.adds / (ms * 1e-3) / 1e12
    hbm_gbps = r["compulsory_bytes"] / (ms * 1e-3) / 1e9
    line = {
        "metric": "dedispersion%s GFLOP/s (one FLOP per channel addition), %s-shaped beam, FP32"
                  % (" adjoint" if args.adjoint else "", {"apertif": "Apertif", "lofar": "LOFAR"}[args.workload]),
        "value": round(r["gflops"], 2),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "%s: %d channels %.0f-%.0f MHz, %d samples/s, %d output samples, %d trial DMs "
                               "%.2f-%.2f step %.2f, float32 N(0,1) + pulses" % (
                                   setup.name, setup.n_channels, setup.f_min,
                                   setup.f_min + setup.n_channels * setup.df, round(1 / setup.t_samp),
                                   setup.n_samples, setup.n_dm, setup.dm_first,
                                   setup.dm_first + (setup.n_dm - 1) * setup.dm_step, setup.dm_step),
                   "tile_variant": r["tile"], "row_blocks": r["blocks"]},
        "roofline": {"bound": "alu", "achieved": round(achieved_tflops, 3), "peak": round(ADD_PEAK_TFLOPS, 1),
                     "unit": "TFLOP/s", "frac": round(achieved_tflops / ADD_PEAK_TFLOPS, 4),
                     "traffic": None if args.adjoint or len(r["blocks"]) > 1 else measured_traffic(setup.name,
                                                                                                    r["tile"])},
        "hbm": {"compulsory_bytes": r["compulsory_bytes"], "achieved_GBps": round(hbm_gbps, 1),
                "peak_GBps": HBM_PEAK_GBPS, "frac": round(hbm_gbps / HBM_PEAK_GBPS, 4)},
        "paper_context": {"hd7970_2000dms_s": 0.106, "hd7970_GFLOPs": round(2000 * 1024 * 20000 / 0.106 / 1e9, 1),
                          "note": "AMD HD7970, OpenCL, 2,000 DMs x 1 s Apertif (Sec. V-D); other hardware"},
    }
    line["timing"] = {"protocol": "%d untimed calls, %d back-to-back calls (ms_warm_back_to_back), then %d timed "
                                  "calls, each after a 1 GiB scratch write, between its own HIP events on the "
                                  "launch stream" % (args.warmup, args.steps, args.steps),
                      "ms_mean": round(ms, 5), "ms_min": round(r["ms_min"], 5), "ms_std": round(r["ms_std"], 5),
                      "ms_warm_back_to_back": round(r["ms_warm"], 5)}
    cb = copy_bandwidth(torch, stream)
    line["hbm"].update(measured_copy_GBps=round(cb["GBps"], 1),
                       frac_of_measured_copy=round(hbm_gbps / cb["GBps"], 4),
                       copy_note="256 MiB device-to-device copy, 512 MiB moved per copy, same protocol")
    log("copy: %.1f GB/s" % cb["GBps"])
    if not args.no_extra:
        only = set(args.extras.split(",")) if args.extras else None
        if only and not only <= set(EXTRAS):
            raise SystemExit("unknown extras: %s" % sorted(only - set(EXTRAS)))
        line["extras"] = extras(torch, dd, stream, max(5, args.steps // 5), only)
    if not args.no_cpu_baseline:
        log("cpu baseline (FP64 oracle) ...")
        line["cpu_baseline"] = cpu_baseline(setup)
        log("cpu baseline: %.2f GFLOP/s on %d threads" % (line["cpu_baseline"]["value"], line["cpu_baseline"]["cores"]))
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
