"""The C-ABI tests (tests/test_abi.py: argument validation, the host planner over a
sweep of shapes, tuning entries, the JSON cache loader and its fuzzing) against
the host-sanitizer build of the library (AddressSanitizer and
UndefinedBehaviorSanitizer on the CPU code; built by __graft_entry__.build()).
A sanitizer finding aborts the run and leaves a report: the test fails on either."""
import glob
import os
import subprocess
import sys

import pytest

from paper_2012_11430_amd import build as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(not os.path.exists(B.SANITIZED_LIB), reason="sanitizer build missing (run __graft_entry__.build())")
def test_abi_suite_under_host_sanitizers(tmp_path):
    runtime = B.asan_runtime()
    assert os.path.exists(runtime), runtime
    log = str(tmp_path / "san")
    env = dict(os.environ)
    env.update(PRONY_LIB=B.SANITIZED_LIB, LD_PRELOAD=runtime,
               ASAN_OPTIONS=f"detect_leaks=0:abort_on_error=1:log_path={log}",
               UBSAN_OPTIONS=f"print_stacktrace=1:halt_on_error=1:log_path={log}")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    reports = glob.glob(log + "*")
    text = "".join(open(p).read()[:4000] for p in reports)
    assert r.returncode == 0 and not reports, (r.stdout[-3000:], r.stderr[-3000:], text)
    assert " passed" in r.stdout
