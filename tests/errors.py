"""Per-configuration error of the GPU results against the FP64 oracle.

Tests call ``record`` (through ``gates.gate(..., report=...)`` or directly for
reported-only figures such as the f16 storage error against the original
float32 data).  When the environment variable DD_ERROR_REPORT names a file,
the session's records are written there at the end of the run: a JSON list
and, next to it, a Markdown table (same name, ``.md``) with, per
configuration, the largest normwise, componentwise and elementwise errors over
every check of that configuration."""
from __future__ import annotations

import json
import os

RECORDS = []


def record(config, normwise, componentwise, elementwise, n_outputs, gated=True, exact=None):
    RECORDS.append(dict(config=config, normwise=float(normwise), componentwise=float(componentwise),
                        elementwise=float(elementwise), n_outputs=int(n_outputs), gated=bool(gated),
                        exact=exact))


def summary():
    by = {}
    for r in RECORDS:
        s = by.setdefault(r["config"], dict(config=r["config"], checks=0, n_outputs=0, normwise=0.0,
                                            componentwise=0.0, elementwise=0.0, gated=r["gated"],
                                            exact=r["exact"]))
        s["checks"] += 1
        s["n_outputs"] += r["n_outputs"]
        for k in ("normwise", "componentwise", "elementwise"):
            s[k] = max(s[k], r[k])
        if r["exact"] is not None:
            s["exact"] = bool(s["exact"]) and r["exact"]
    return [by[k] for k in sorted(by)]


def write(path):
    rows = summary()
    with open(path, "w") as f:
        json.dump(dict(records=RECORDS, summary=rows), f, indent=1)
    md = os.path.splitext(path)[0] + ".md"
    with open(md, "w") as f:
        f.write("| configuration | checks | outputs compared | normwise max|y-r|/max|r| | "
                "componentwise max |y-r|/sum|x| | elementwise (|r| >= 1e-3 max|r|) | gate |\n")
        f.write("|---|---|---|---|---|---|---|\n")
        for s in rows:
            gate = ("bit-exact" if s["exact"] else "MISMATCH") if s["exact"] is not None else (
                "<= 1e-5" if s["gated"] else "reported only")
            f.write("| %s | %d | %d | %.2e | %.2e | %.2e | %s |\n" % (
                s["config"], s["checks"], s["n_outputs"], s["normwise"], s["componentwise"], s["elementwise"], gate))
