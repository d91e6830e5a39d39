"""The oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc), driven through its 1D and 2D entry points on small seeded states
(every degree, post-stage operator and boundary type, the positivity limiter
and both 2D spaces): no memory error, no undefined behaviour, no
unexpected return code."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_under_asan_and_ubsan():
    od = os.path.join(ROOT, "oracle")
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "driver")
        cmd = ["gcc", "-O1", "-g", "-std=c11", "-D_DEFAULT_SOURCE", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", od,
               os.path.join(ROOT, "tests", "oracle_sanitize_driver.c"),
               *(os.path.join(od, f) for f in ("dgref.c", "dgref2d.c", "dgref_hll.c")),
               "-lm", "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert "0 unexpected return codes" in r.stdout
