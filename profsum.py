"""Text summaries of rocprofv3 CSV output, for the files under profiles/.

    python3 profsum.py trace DIR KERNEL [--calls-after FLUSH]
        Kernel-trace statistics (rocprofv3 --kernel-trace --output-format csv,
        written under DIR) of the kernels whose name contains KERNEL: all
        dispatches, and the timed calls only.  bench.py writes a 1 GiB scratch
        buffer (a fill kernel whose name contains FLUSH, default "Fill")
        before every timed call, so a timed call is the run of matching
        dispatches that directly follows such a write; its duration is the
        sum of those dispatches (kernels that split rows over several launches
        have several per call).

    python3 profsum.py counters FETCH_DIR WRITE_DIR KERNEL [--copy-bytes N]
        FETCH_SIZE and WRITE_SIZE (KiB per dispatch, two rocprofv3 --pmc runs)
        of the matching kernels, over all dispatches and over the timed calls
        only (dispatches right after the 1 GiB scratch write), scaled by what
        the same counters read for the device-to-device copy of N bytes
        (default 256 MiB) in the same run, whose kernel name contains
        "copyBuffer".

    python3 profsum.py traffic FETCH_DIR WRITE_DIR WORKLOAD VARIANT [--copy-bytes N]
        JSON on stdout for profiles/traffic_<workload>_fwd.json: the calibrated
        HBM-side bytes per launch of every tile variant whose kernel ran in the
        two counter runs (the timed calls where there are any, else the first
        pass of the autotuner, which times the variants in id order over all
        rows before it tries row splits), keyed by
        variant id, with the variant's entry in the variant list and the hash
        of the kernel sources (bench.py uses the bytes only while both match).
        Variants whose kernel name another variant shares are left out.

    python3 profsum.py sq DIR KERNEL [--calls-after FLUSH]
        Every counter of one rocprofv3 --pmc run (DIR) for the matching
        kernel: the mean over its timed calls (the dispatches right after the
        1 GiB scratch write), per call (summed over a call's dispatches).

    python3 profsum.py variants TRACE_DIR TRAFFIC_JSON
        Per tile variant the autotuner timed over all rows in the traced
        program (its first pass, variants in id order): the mean dispatch
        duration, and the bytes per launch from TRAFFIC_JSON.

    python3 profsum.py study JSON [--curated N]   (N: curated variants; default from the JSON)
        The auto-tuning study (bench.py --tune-study): per instance the
        optimum, mean and spread over the variants that fit, the optimum's
        signal-to-noise ratio and Chebyshev bound, the best fixed variant, the
        best of the first N (curated) variants against the optimum, the kind
        and tile of each optimum, and rate histograms.

Reads only the CSV / JSON files; prints Markdown on stdout.
"""
from __future__ import annotations

import argparse
import csv
import glob
import os
import statistics
import sys


def _rows(directory, suffix):
    paths = sorted(glob.glob(os.path.join(directory, "**", "*" + suffix), recursive=True))
    if not paths:
        raise SystemExit("no *%s under %s" % (suffix, directory))
    out = []
    for p in paths:
        with open(p, newline="") as f:
            out.extend(csv.DictReader(f))
    return out


def _dispatches(directory):
    """Kernel dispatches in start order: (name, start_ns, end_ns)."""
    d = []
    for r in _rows(directory, "kernel_trace.csv"):
        d.append((r["Kernel_Name"], int(r["Start_Timestamp"]), int(r["End_Timestamp"])))
    d.sort(key=lambda x: x[1])
    return d


def _stats(v):
    return (len(v), statistics.mean(v), min(v), max(v), statistics.pstdev(v) if len(v) > 1 else 0.0)


def trace(directory, kernel, flush):
    d = _dispatches(directory)
    names = sorted({n for n, _, _ in d if kernel in n})
    if not names:
        raise SystemExit("no kernel matching %r" % kernel)
    print("| kernel | dispatches | average ns | min ns | max ns |")
    print("|---|---|---|---|---|")
    for n in names:
        v = [e - s for m, s, e in d if m == n]
        c, avg, lo, hi, _ = _stats(v)
        print("| `%s` | %d | %.0f | %d | %d |" % (n, c, avg, lo, hi))
    # timed calls: matching dispatches right after a flush write
    calls, cur, prev_flush = [], None, False
    for n, s, e in d:
        if kernel in n:
            if prev_flush:
                cur = [e - s, 1]
                calls.append(cur)
            elif cur is not None:
                cur[0] += e - s
                cur[1] += 1
            prev_flush = False
        else:
            cur = None
            prev_flush = flush in n
    print()
    if not calls:
        print("No timed calls found (no matching dispatch directly after a %r kernel)." % flush)
        return
    v = [c[0] for c in calls]
    c, avg, lo, hi, sd = _stats(v)
    per = sorted({c[1] for c in calls})
    print("Timed calls (each right after the 1 GiB scratch write): %d calls of %s dispatch(es); "
          "per call average %.0f ns, min %d, max %d, std %.0f." % (c, "/".join(map(str, per)), avg, lo, hi, sd))


def _counter_seq(directory, name):
    """[(kernel name, value)] of one counter, one entry per dispatch, in
    dispatch order (a counter summed over its dimensions)."""
    vals = {}
    for r in _rows(directory, "counter_collection.csv"):
        if r.get("Counter_Name") != name:
            continue
        d = int(r["Dispatch_Id"])
        k, v = vals.get(d, (r["Kernel_Name"], 0.0))
        vals[d] = (k, v + float(r["Counter_Value"]))
    return [vals[d] for d in sorted(vals)]


def _counter(directory, name):
    """{kernel name: [value per dispatch]} of one counter."""
    out = {}
    for k, v in _counter_seq(directory, name):
        out.setdefault(k, []).append(v)
    return out


def _after_flush(seq, kernel, flush):
    """Per timed call, the sum over the run of dispatches of `kernel` that
    directly follows a dispatch whose name contains `flush` (bench.py's timed
    calls; a call on a row split makes one dispatch per block)."""
    out, cur, prev_flush = [], None, False
    for k, v in seq:
        if k == kernel:
            if prev_flush:
                cur = [v]
                out.append(cur)
            elif cur is not None:
                cur.append(v)
            prev_flush = False
        else:
            cur = None
            prev_flush = flush in k
    return [sum(c) for c in out]


def _tuning_runs(seq, owners):
    """{variant id: [values]} of the autotuner's first pass: it times the
    variants in id order, each over all rows, before it tries row splits, so
    the pass ends where a kernel of a lower id than the previous one runs.
    `owners` maps a kernel key to the variant ids that instantiate it; kernels
    shared by several variants are skipped."""
    out, last = {}, -1
    for name, v in seq:
        key = _kernel_key(name)
        if key is None or "<float," not in name or len(owners.get(key, [])) != 1:
            continue
        vid = owners[key][0]
        if vid < last:
            break
        last = vid
        out.setdefault(vid, []).append(v)
    return out


def _owners(here):
    sys.path.insert(0, here)
    import bench  # the variant list bench.py and the library use
    owners = {}
    for vid, key in _variant_kernels(os.path.join(here, bench.VARIANT_LIST)).items():
        owners.setdefault(key, []).append(vid)
    return owners


def _copies(tab):
    """Counter values of the calibration copies: the copyBuffer dispatches of
    at least half the largest one's count (the program may make small copies
    too)."""
    v = [x for k, vals in tab.items() if "copyBuffer" in k for x in vals]
    if not v:
        raise SystemExit("no copyBuffer dispatches to calibrate against")
    return [x for x in v if x >= 0.5 * max(v)]


def counters(fetch_dir, write_dir, kernel, copy_bytes, flush):
    fseq, wseq = _counter_seq(fetch_dir, "FETCH_SIZE"), _counter_seq(write_dir, "WRITE_SIZE")
    fetch, write = _counter(fetch_dir, "FETCH_SIZE"), _counter(write_dir, "WRITE_SIZE")
    copy_kib = copy_bytes / 1024.0

    cf, cw = _copies(fetch), _copies(write)
    f_scale = copy_kib / statistics.median(cf)
    w_scale = copy_kib / statistics.median(cw)
    names = sorted({k for k in list(fetch) + list(write) if kernel in k})
    if not names:
        raise SystemExit("no kernel matching %r" % kernel)
    print("| kernel | dispatches | FETCH_SIZE KiB | WRITE_SIZE KiB | timed calls | FETCH_SIZE KiB per call "
          "| WRITE_SIZE KiB per call |")
    print("|---|---|---|---|---|---|---|")
    mean = lambda v: statistics.mean(v) if v else float("nan")  # noqa: E731
    for n in names:
        f, w = fetch.get(n, []), write.get(n, [])
        tf, tw = _after_flush(fseq, n, flush), _after_flush(wseq, n, flush)
        print("| `%s` | %d / %d | %.1f | %.1f | %d / %d | %.1f | %.1f |" % (
            n, len(f), len(w), mean(f), mean(w), len(tf), len(tw), mean(tf), mean(tw)))
    print("| copy of %d MiB (`copyBuffer`) | %d / %d | %.1f | %.1f | | | |" % (
        copy_bytes >> 20, len(cf), len(cw), statistics.median(cf), statistics.median(cw)))
    print()
    print("All dispatches include the autotuner's (whole rows, and blocks of rows while it tries row "
          "splits); timed calls are the dispatches right after bench.py's 1 GiB scratch write.")
    print("Calibration: the copy reads and writes %.0f KiB per dispatch, so FETCH_SIZE is scaled by %.3f and "
          "WRITE_SIZE by %.3f." % (copy_kib, f_scale, w_scale))
    for n in names:
        tf, tw = _after_flush(fseq, n, flush), _after_flush(wseq, n, flush)
        if tf and tw:
            b = (statistics.mean(tf) * f_scale + statistics.mean(tw) * w_scale) * 1024
            print("`%s`: %.4g bytes per timed call from HBM-side counters." % (n, b))


def sq(directory, kernel, flush):
    names = set()
    counters = set()
    for r in _rows(directory, "counter_collection.csv"):
        counters.add(r["Counter_Name"])
        if kernel in r["Kernel_Name"]:
            names.add(r["Kernel_Name"])
    if len(names) != 1:
        raise SystemExit("need exactly one kernel matching %r, found %d" % (kernel, len(names)))
    name = names.pop()
    print("| counter | timed calls | mean per call |")
    print("|---|---|---|")
    for c in sorted(counters):
        v = _after_flush(_counter_seq(directory, c), name, flush)
        print("| `%s` | %d | %s |" % (c, len(v), "%.4g" % statistics.mean(v) if v else "-"))


def _variant_kernels(def_path):
    """{variant id: (kernel base name, template arguments after the input
    type)} from the X-macro variant list, as srs_inst.inc instantiates them."""
    import re
    with open(def_path) as f:
        text = re.sub(r"/\*.*?\*/|//[^\n]*", "", f.read(), flags=re.S)
    out = {}
    for m in re.finditer(r"(X_\w+)\(([^)]*)\)", text):
        kind, args = m.group(1), [a.strip() for a in m.group(2).split(",")]
        if kind == "X_LDS":
            out[int(args[0])] = ("srs_lds_kernel", tuple(args[1:4]))
        elif kind == "X_LDSP":
            out[int(args[0])] = ("srs_ldsp_kernel", tuple(args[1:6]))
        elif kind == "X_RW":
            out[int(args[0])] = ("srs_regwin_kernel", tuple(args[1:7]) + ("1",))
        elif kind == "X_RWO":
            out[int(args[0])] = ("srs_regwin_kernel", tuple(args[1:8]))
        elif kind == "X_DIRECT":
            rb, v = int(args[4]), int(args[5])
            out[int(args[0])] = ("srs_direct_kernel", tuple(args[1:4]) + (
                "true" if rb > 0 else "false", "true" if v else "false"))
    return out


def _kernel_key(name):
    """(base name, template arguments after the input type) of a kernel name."""
    import re
    m = re.search(r"(srs_\w+_kernel)<([^>]*)>", name)
    if not m:
        return None
    args = [a.strip() for a in m.group(2).split(",")]
    return m.group(1), tuple(args[1:])


def traffic(fetch_dir, write_dir, workload, variant, copy_bytes, flush):
    import json
    here = os.path.dirname(os.path.abspath(__file__))
    sys.path.insert(0, here)
    import bench  # the source hash and variant entries bench.py compares against
    fetch, write = _counter(fetch_dir, "FETCH_SIZE"), _counter(write_dir, "WRITE_SIZE")
    copy_kib = copy_bytes / 1024.0
    cf, cw = _copies(fetch), _copies(write)
    f_scale, w_scale = copy_kib / statistics.median(cf), copy_kib / statistics.median(cw)
    owners = _owners(here)
    fseq, wseq = _counter_seq(fetch_dir, "FETCH_SIZE"), _counter_seq(write_dir, "WRITE_SIZE")
    ftune, wtune = _tuning_runs(fseq, owners), _tuning_runs(wseq, owners)
    by_variant = {}
    for name in sorted(set(fetch) & set(write)):
        key = _kernel_key(name)
        if key is None or "<float," not in name or len(owners.get(key, [])) != 1:
            continue
        vid = owners[key][0]
        f, w = _after_flush(fseq, name, flush), _after_flush(wseq, name, flush)
        if not f or not w:
            f, w = ftune.get(vid), wtune.get(vid)
        if not f or not w:
            continue
        b = (statistics.mean(f) * f_scale + statistics.mean(w) * w_scale) * 1024
        by_variant[str(vid)] = {"bytes": round(b), "entry": bench.variant_entry(vid)}
    if str(variant) not in by_variant:
        raise SystemExit("variant %d did not run in the counter runs" % variant)
    json.dump({"workload": workload, "variant": variant, "source_hash": bench.kernel_source_hash(),
               "by_variant": dict(sorted(by_variant.items(), key=lambda kv: int(kv[0])))}, sys.stdout, indent=1)
    print()


def variants(trace_dir, traffic_json):
    import json
    owners = _owners(os.path.dirname(os.path.abspath(__file__)))
    with open(traffic_json) as f:
        tr = json.load(f).get("by_variant", {})
    seq = [(n, e - s) for n, s, e in _dispatches(trace_dir)]
    names = {}
    for n, _ in seq:
        key = _kernel_key(n)
        if key is not None and len(owners.get(key, [])) == 1:
            names[owners[key][0]] = n
    print("| variant | kernel | dispatches | average ns | HBM-side bytes per launch |")
    print("|---|---|---|---|---|")
    for vid, run in sorted(_tuning_runs(seq, owners).items()):
        short = names[vid].split("(")[0].replace("void dd::kern::", "")
        b = tr.get(str(vid), {}).get("bytes")
        print("| %d | `%s` | %d | %.0f | %s |" % (vid, short, len(run), statistics.mean(run),
                                                "-" if b is None else "%.3g" % b))


KINDS = {0: "LDS", 1: "register window", 2: "direct"}


def study(path, curated):
    import json
    with open(path) as f:
        d = json.load(f)
    if curated is None:  # the product list's length when the study ran (46 before it was recorded)
        curated = d.get("curated", 46)
    var = {v[0]: v for v in d["variants"]}
    rows = d["instances"]

    def desc(vid):
        _, it, acc, waves, kind = var[vid]
        return "%s %dx%d, %d waves (%d samples x %d rows)" % (KINDS[kind], it, acc, waves, 64 * it, acc * waves)

    print("Library: `%s`, %d tile variants (ids below %d: the product library's curated list)."
          % (d.get("library"), len(var), curated))
    print()
    print("| setup | DMs | variants | optimum | GFLOP/s | mean | std | SNR | Chebyshev | fixed | tuned / fixed "
          "| best curated | optimum / best curated | model | model / optimum | real time |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|---|")
    ratios = []
    for r in rows:
        g = {int(k): v for k, v in r["gflops"].items()}
        cur = {k: v for k, v in g.items() if k < curated}
        bc = max(cur, key=cur.get) if cur else None
        mg = r.get("model_gflops")
        if mg:
            ratios.append(mg / r["best_gflops"])
        print("| %s | %d | %d | %d | %.0f | %.0f | %.0f | %.2f | %.2f | %d | %.2f | %s | %s | %s | %s | %s |" % (
            r["setup"], r["n_dm"], r["n_variants"], r["best"], r["best_gflops"], r["mean_gflops"], r["std_gflops"],
            r["snr"], r["chebyshev_bound"], r["fixed_variant"], r["tuned_over_fixed"],
            "-" if bc is None else "%d" % bc, "-" if bc is None else "%.2f" % (r["best_gflops"] / cur[bc]),
            r.get("model_variant", "-"), "%.2f" % (mg / r["best_gflops"]) if mg else "-",
            "yes" if r["realtime"] else "no"))
    if ratios:
        print()
        print("Untuned cost model (the library's choice without tuning), rated by the measured rate of the "
              "variant it picks: %.2f-%.2f of the optimum, %.2f on average." % (min(ratios), max(ratios),
                                                                               sum(ratios) / len(ratios)))
    print()
    print("Optima and fixed variants:")
    print()
    for vid in sorted({r["best"] for r in rows} | {r["fixed_variant"] for r in rows}):
        print("* %d: %s" % (vid, desc(vid)))
    for setup in sorted({r["setup"] for r in rows}):
        sel = [r for r in rows if r["setup"] == setup]
        r = max(sel, key=lambda x: x["n_dm"] if x["n_dm"] <= 2048 else -1)
        vals = sorted(r["gflops"].values())
        lo, hi = 0.0, max(vals)
        nb = 12
        w = (hi - lo) / nb
        print()
        print("Rate histogram, %s, %d DMs (%d variants):" % (setup, r["n_dm"], len(vals)))
        print()
        print("| GFLOP/s | variants |")
        print("|---|---|")
        for b in range(nb):
            a0, a1 = lo + b * w, lo + (b + 1) * w
            n = sum(1 for v in vals if a0 <= v < a1 or (b == nb - 1 and v == hi))
            print("| %.0f-%.0f | %s |" % (a0, a1, "#" * n if n else "0"))
        # best per kind at this instance
        print()
        print("Best per kind at %d DMs:" % r["n_dm"])
        print()
        for kind in sorted(KINDS):
            ks = {int(k): v for k, v in r["gflops"].items() if var[int(k)][4] == kind}
            if ks:
                b = max(ks, key=ks.get)
                print("* %s: variant %d, %.0f GFLOP/s (%s); %d variants of this kind fit"
                      % (KINDS[kind], b, ks[b], desc(b), len(ks)))


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("dir")
    t.add_argument("kernel")
    t.add_argument("--calls-after", default="Fill")
    c = sub.add_parser("counters")
    c.add_argument("fetch_dir")
    c.add_argument("write_dir")
    c.add_argument("kernel")
    c.add_argument("--copy-bytes", type=int, default=256 << 20)
    c.add_argument("--calls-after", default="Fill")
    tr = sub.add_parser("traffic")
    tr.add_argument("fetch_dir")
    tr.add_argument("write_dir")
    tr.add_argument("workload")
    tr.add_argument("variant", type=int)
    tr.add_argument("--copy-bytes", type=int, default=256 << 20)
    tr.add_argument("--calls-after", default="Fill")
    q = sub.add_parser("sq")
    q.add_argument("dir")
    q.add_argument("kernel")
    q.add_argument("--calls-after", default="Fill")
    va = sub.add_parser("variants")
    va.add_argument("trace_dir")
    va.add_argument("traffic_json")
    st = sub.add_parser("study")
    st.add_argument("json")
    st.add_argument("--curated", type=int, default=None)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        trace(a.dir, a.kernel, a.calls_after)
    elif a.cmd == "traffic":
        traffic(a.fetch_dir, a.write_dir, a.workload, a.variant, a.copy_bytes, a.calls_after)
    elif a.cmd == "sq":
        sq(a.dir, a.kernel, a.calls_after)
    elif a.cmd == "variants":
        variants(a.trace_dir, a.traffic_json)
    elif a.cmd == "study":
        study(a.json, a.curated)
    else:
        counters(a.fetch_dir, a.write_dir, a.kernel, a.copy_bytes, a.calls_after)


if __name__ == "__main__":
    sys.exit(main())
