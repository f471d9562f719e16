"""profsum.py (the rocprofv3 summary behind profiles/) on small synthetic CSVs."""
import csv
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _write(path, header, rows):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(header)
        w.writerows(rows)


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "profsum.py")] + list(args), check=True,
                          capture_output=True, text=True).stdout


def test_trace_timed_calls_follow_the_flush(tmp_path):
    rows, t = [], 0
    seq = ["srs_k"] * 3 + ["FillFunctor"] + ["srs_k", "srs_k"] + ["FillFunctor", "srs_k", "srs_k", "other", "srs_k"]
    for i, n in enumerate(seq):
        dur = 100 if n == "srs_k" else 50
        rows.append([n, t, t + dur, i])
        t += 1000
    _write(str(tmp_path / "host" / "1" / "x_kernel_trace.csv"),
           ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Dispatch_Id"], rows)
    out = _run("trace", str(tmp_path), "srs_k")
    assert "| `srs_k` | 8 | 100 | 100 | 100 |" in out
    assert "2 calls of 2 dispatch(es); per call average 200 ns" in out


def test_counters_scaled_by_the_copy(tmp_path):
    """Timed calls are the dispatches right after the flush write; the bytes
    line uses them only (the first, untimed dispatch reads less)."""
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    _write(str(tmp_path / "f" / "a_counter_collection.csv"), hdr,
           [[1, "k", "FETCH_SIZE", 10.0], [2, "FillFunctor", "FETCH_SIZE", 1.0], [3, "k", "FETCH_SIZE", 1000.0],
            [4, "copyBuffer", "FETCH_SIZE", 512.0]])
    _write(str(tmp_path / "w" / "a_counter_collection.csv"), hdr,
           [[1, "k", "WRITE_SIZE", 30.0], [2, "FillFunctor", "WRITE_SIZE", 1.0], [3, "k", "WRITE_SIZE", 300.0],
            [4, "copyBuffer", "WRITE_SIZE", 1024.0]])
    out = _run("counters", str(tmp_path / "f"), str(tmp_path / "w"), "k", "--copy-bytes", str(1 << 20))
    assert "FETCH_SIZE is scaled by 2.000 and WRITE_SIZE by 1.000" in out
    assert "| `k` | 2 / 2 | 505.0 | 165.0 | 1 / 1 | 1000.0 | 300.0 |" in out
    assert "`k`: 2.355e+06 bytes per timed call" in out  # (1000 * 2 + 300) KiB


def test_traffic_maps_kernels_to_variants(tmp_path):
    """traffic keys each kernel's bytes by the variant whose template arguments
    it carries (variant 31: register window 8x8, 40 registers, 8 waves)."""
    import json
    name = "void dd::kern::srs_regwin_kernel<float, 8, 8, 40, 8, 1, 12, 4>(float const*)"
    v17 = "void dd::kern::srs_regwin_kernel<float, 8, 8, 40, 4, 1, 12, 4>(float const*)"
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    # the tuner's pass over whole rows (variant 31), then a row-split attempt
    # (variant 17 on a block, variant 31 on the next): only the pass counts
    _write(str(tmp_path / "f" / "a_counter_collection.csv"), hdr,
           [[1, name, "FETCH_SIZE", 100.0], [2, name, "FETCH_SIZE", 100.0], [3, v17, "FETCH_SIZE", 1.0],
            [4, name, "FETCH_SIZE", 7.0], [5, "copyBuffer", "FETCH_SIZE", 512.0]])
    _write(str(tmp_path / "w" / "a_counter_collection.csv"), hdr,
           [[1, name, "WRITE_SIZE", 50.0], [2, name, "WRITE_SIZE", 50.0], [3, v17, "WRITE_SIZE", 1.0],
            [4, name, "WRITE_SIZE", 7.0], [5, "copyBuffer", "WRITE_SIZE", 1024.0]])
    out = _run("traffic", str(tmp_path / "f"), str(tmp_path / "w"), "apertif", "31", "--copy-bytes", str(1 << 20))
    d = json.loads(out)
    assert d["variant"] == 31 and list(d["by_variant"]) == ["31"]
    assert d["by_variant"]["31"]["bytes"] == (100 * 2 + 50) * 1024   # the tuner's pass; no flush in this trace
    assert d["by_variant"]["31"]["entry"] == "X_RWO(31,8,8,40,8,1,12,4)"
