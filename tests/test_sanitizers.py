"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds the library's host sources (plans, tile layouts, variant table, tile
choice, the C-ABI argument checks) and the C oracle with g++/gcc and
-fsanitize=address,undefined, links them into tests/sanitize_driver.cpp and
runs it.  The HIP kernel units are left out (nothing here launches work); a
compute call with valid arguments fails on the missing device, after every
host-side check has run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1601_05052_amd", "csrc")
HOST_SOURCES = ["plan.cpp", "select.cpp", "api.cpp", "variants.cpp"]  # noalloc.hip needs device code
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


@pytest.mark.skipif(not shutil.which("g++") or not os.path.isdir("/opt/rocm/include"),
                    reason="needs g++ and the ROCm headers")
def test_host_code_clean_under_asan_ubsan(tmp_path):
    objs = []
    for src in HOST_SOURCES + [os.path.join(ROOT, "tests", "sanitize_driver.cpp")]:
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run(["g++", "-std=c++17", "-c", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
                        "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-ffp-contract=off"] + SAN +
                       [os.path.join(CSRC, src), "-o", obj], check=True)
        objs.append(obj)
    obj = str(tmp_path / "dd_oracle.o")
    subprocess.run(["gcc", "-std=c11", "-c", "-ffp-contract=off"] + SAN +
                   [os.path.join(ROOT, "oracle", "dd_oracle.c"), "-o", obj], check=True)
    objs.append(obj)
    exe = str(tmp_path / "sanitize_driver")
    subprocess.run(["g++"] + SAN + objs + ["-o", exe, "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib",
                                           "-lamdhip64", "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized host checks ok" in r.stdout
