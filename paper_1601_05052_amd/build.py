"""Build libdedisp.so in-tree for gfx950 with hipcc.

    python -m paper_1601_05052_amd.build [-v]
    python -m paper_1601_05052_amd.build --study [-v]   # auto-tuning study library
    python -m paper_1601_05052_amd.build --ceilings     # in-core ceilings microbenchmark

Flags:
  --offload-arch=gfx950        CDNA4 only; no other targets, no CUDA path
  -Xclang -target-feature -Xclang -packed-fp32-ops
                               no v_pk_*_f32 instructions in device code
  -ffp-contract=off            the host's FP64 delay table is evaluated one
                               IEEE operation at a time (no FMA contraction)
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB_NAME = "libdedisp.so"


def library_path() -> str:
    return os.path.join(PKG, LIB_NAME)


def hipcc() -> str:
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if c and os.path.exists(c):
            return c
    return "hipcc"


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")) + glob.glob(os.path.join(CSRC, "*.cpp")))


def compile_flags():
    return ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-ffp-contract=off", "-fno-fast-math",
            "-Wall", "-Wno-unused-function",
            "-I", INCLUDE, "-I", CSRC]


# Kernel units compiled with -save-temps=obj: their device assembly stays in
# _build/ (<stem>-hip-amdgcn-amd-amdhsa-gfx950.s), so tests can inspect the
# register use of the inline-assembly kernels.
LISTED = ("srs_kernels_f32.hip", "srs_kernels_f16.hip", "srs_kernels_u8.hip")


def listing_paths():
    return [os.path.join(PKG, "_build", os.path.splitext(n)[0] + "-hip-amdgcn-amd-amdhsa-gfx950.s") for n in LISTED]


def build(verbose: bool = False, jobs: int = 8) -> str:
    """Compile every source to an object in _build/ (in parallel) and link."""
    out_dir = os.path.join(PKG, "_build")
    os.makedirs(out_dir, exist_ok=True)
    objs, procs = [], []
    # Largest units first so they start early.
    for src in sorted(sources(), key=lambda p: os.path.basename(p) not in LISTED):
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        objs.append(obj)
        temps = ["-save-temps=obj"] if os.path.basename(src) in LISTED else []
        cmd = [hipcc(), "-c", "-x", "hip"] + compile_flags() + temps + ["-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0), verbose)
    for p in procs:
        _wait(p, verbose)
    lib = library_path()
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [hipcc(), "-shared", "--offload-arch=gfx950", "-o", tmp] + objs
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


STUDY_LIB_NAME = "libdedisp_study.so"


def study_library_path() -> str:
    return os.path.join(PKG, STUDY_LIB_NAME)


def build_study(verbose: bool = False, jobs: int = 8) -> str:
    """The auto-tuning study's library (Sec. IV-A): the same sources compiled
    with -DDD_STUDY over the generated variant grid (csrc/gen_study.py),
    float32 single-beam kernels only.  Not part of the product build."""
    out_dir = os.path.join(PKG, "_build", "study")
    sys.path.insert(0, CSRC)
    import gen_study
    n = gen_study.write(out_dir)
    srcs = [p for p in sources() if not os.path.basename(p).startswith("srs_kernels_")]
    srcs = sorted(glob.glob(os.path.join(out_dir, "study_kernels_*.hip"))) + srcs
    objs, procs = [], []
    for src in srcs:
        obj = os.path.join(out_dir, os.path.basename(src) + ".o")
        objs.append(obj)
        cmd = [hipcc(), "-c", "-x", "hip"] + compile_flags() + ["-DDD_STUDY", "-I", out_dir, "-o", obj, src]
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append((src, subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT)))
        if len(procs) >= jobs:
            _wait(procs.pop(0), verbose)
    for p in procs:
        _wait(p, verbose)
    lib = study_library_path()
    tmp = lib + ".tmp%d" % os.getpid()
    subprocess.run([hipcc(), "-shared", "--offload-arch=gfx950", "-o", tmp] + objs, check=True)
    os.replace(tmp, lib)
    if verbose:
        print("%d study variants" % n)
    return lib


def ceilings_path() -> str:
    return os.path.join(PKG, "ceilings")


def build_ceilings() -> str:
    """The in-core ceilings microbenchmark (ceilings.hip), an executable."""
    exe = ceilings_path()
    tmp = exe + ".tmp"
    proc = subprocess.Popen([hipcc()] + compile_flags() + ["-o", tmp, os.path.join(PKG, "ceilings.hip")],
                            stdout=subprocess.PIPE, stderr=subprocess.STDOUT)
    _wait((exe, proc), False)
    os.replace(tmp, exe)
    return exe


def _wait(item, verbose):
    src, proc = item
    out, _ = proc.communicate()
    text = out.decode(errors="replace")
    # hipcc's host pass does not know the packed-fp32 feature; harmless.
    lines = [l for l in text.splitlines() if "packed-fp32-ops" not in l]
    if proc.returncode != 0:
        sys.stderr.write("\n".join(lines) + "\n")
        raise RuntimeError("hipcc failed on %s" % src)
    if verbose and lines:
        print("\n".join(lines))


if __name__ == "__main__":
    if "--study" in sys.argv:
        print(build_study(verbose="-v" in sys.argv))
    elif "--ceilings" in sys.argv:
        print(build_ceilings())
    else:
        print(build(verbose="-v" in sys.argv))
