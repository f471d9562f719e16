"""The auto-tuning study's library (every grid variant, float32): each
variant bit for bit against the oracle on integer-valued inputs.  Runs
tests/study_check.py in a process of its own (the library is chosen when the
binding loads).  Skipped when the study library is not built
(python -m paper_1601_05052_amd.build --study)."""
import os
import subprocess
import sys

import pytest

from paper_1601_05052_amd import build

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(not os.path.exists(build.study_library_path()), reason="study library not built")
def test_every_study_variant_integer_exact():
    env = dict(os.environ, DEDISP_LIBRARY=build.study_library_path())
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "study_check.py")], env=env,
                       capture_output=True, text=True, timeout=900)
    print(r.stdout)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "variant-shape checks exact" in r.stdout
