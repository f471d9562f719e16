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
        of the matching kernels, scaled by what the same counters read for the
        device-to-device copy of N bytes (default 256 MiB) in the same run,
        whose kernel name contains "copyBuffer".

    python3 profsum.py study JSON [--curated N]
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


def _counter(directory, name):
    """{kernel name: [value per dispatch]} of one counter."""
    vals = {}
    for r in _rows(directory, "counter_collection.csv"):
        if r.get("Counter_Name") != name:
            continue
        vals.setdefault(r["Kernel_Name"], {}).setdefault(r.get("Dispatch_Id", len(vals)), 0.0)
        vals[r["Kernel_Name"]][r.get("Dispatch_Id")] += float(r["Counter_Value"])
    return {k: list(v.values()) for k, v in vals.items()}


def counters(fetch_dir, write_dir, kernel, copy_bytes):
    fetch, write = _counter(fetch_dir, "FETCH_SIZE"), _counter(write_dir, "WRITE_SIZE")
    copy_kib = copy_bytes / 1024.0

    def pick(tab, key):
        ks = [k for k in tab if key in k]
        return ks, [x for k in ks for x in tab[k]]

    _, cf = pick(fetch, "copyBuffer")
    _, cw = pick(write, "copyBuffer")
    if not cf or not cw:
        raise SystemExit("no copyBuffer dispatches to calibrate against")
    f_scale = copy_kib / statistics.median(cf)
    w_scale = copy_kib / statistics.median(cw)
    print("| kernel | FETCH_SIZE KiB | WRITE_SIZE KiB | dispatches (fetch / write) |")
    print("|---|---|---|---|")
    names = sorted({k for k in list(fetch) + list(write) if kernel in k})
    if not names:
        raise SystemExit("no kernel matching %r" % kernel)
    for n in names:
        f, w = fetch.get(n, []), write.get(n, [])
        print("| `%s` | %.1f | %.1f | %d / %d |" % (n, statistics.mean(f) if f else float("nan"),
                                                    statistics.mean(w) if w else float("nan"), len(f), len(w)))
    print("| copy of %d MiB (`copyBuffer`) | %.1f | %.1f | %d / %d |" % (
        copy_bytes >> 20, statistics.median(cf), statistics.median(cw), len(cf), len(cw)))
    print()
    print("Calibration: the copy reads and writes %.0f KiB per dispatch, so FETCH_SIZE is scaled by %.3f and "
          "WRITE_SIZE by %.3f." % (copy_kib, f_scale, w_scale))
    for n in names:
        f, w = fetch.get(n, []), write.get(n, [])
        if f and w:
            b = (statistics.mean(f) * f_scale + statistics.mean(w) * w_scale) * 1024
            print("`%s`: %.4g bytes per dispatch from HBM-side counters." % (n, b))


KINDS = {0: "LDS", 1: "register window", 2: "direct"}


def study(path, curated):
    import json
    with open(path) as f:
        d = json.load(f)
    var = {v[0]: v for v in d["variants"]}
    rows = d["instances"]

    def desc(vid):
        _, it, acc, waves, kind = var[vid]
        return "%s %dx%d, %d waves (%d samples x %d rows)" % (KINDS[kind], it, acc, waves, 64 * it, acc * waves)

    print("Library: `%s`, %d tile variants (ids below %d: the product library's curated list)."
          % (d.get("library"), len(var), curated))
    print()
    print("| setup | DMs | variants | optimum | GFLOP/s | mean | std | SNR | Chebyshev | fixed | tuned / fixed "
          "| best curated | optimum / best curated | real time |")
    print("|---|---|---|---|---|---|---|---|---|---|---|---|---|---|")
    for r in rows:
        g = {int(k): v for k, v in r["gflops"].items()}
        cur = {k: v for k, v in g.items() if k < curated}
        bc = max(cur, key=cur.get) if cur else None
        print("| %s | %d | %d | %d | %.0f | %.0f | %.0f | %.2f | %.2f | %d | %.2f | %s | %s | %s |" % (
            r["setup"], r["n_dm"], r["n_variants"], r["best"], r["best_gflops"], r["mean_gflops"], r["std_gflops"],
            r["snr"], r["chebyshev_bound"], r["fixed_variant"], r["tuned_over_fixed"],
            "-" if bc is None else "%d" % bc, "-" if bc is None else "%.2f" % (r["best_gflops"] / cur[bc]),
            "yes" if r["realtime"] else "no"))
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
    st = sub.add_parser("study")
    st.add_argument("json")
    st.add_argument("--curated", type=int, default=46)
    a = ap.parse_args(argv)
    if a.cmd == "trace":
        trace(a.dir, a.kernel, a.calls_after)
    elif a.cmd == "study":
        study(a.json, a.curated)
    else:
        counters(a.fetch_dir, a.write_dir, a.kernel, a.copy_bytes)


if __name__ == "__main__":
    sys.exit(main())
