"""The host set-up code (colouring, internal numbering, validation) under
AddressSanitizer and UndefinedBehaviorSanitizer, on the CPU: a copy of the library
with those files instrumented, loaded into a Python process with the ASan runtime
preloaded. Any report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_host_setup_paths_clean_under_asan_ubsan():
    from paper_1903_08243_amd import build as b
    try:
        lib = b.build_host_sanitized()
        rt = b.asan_runtime()
    except (RuntimeError, OSError, subprocess.CalledProcessError) as ex:
        pytest.skip(f"sanitized build unavailable: {ex}")
    if not os.path.exists(rt):
        pytest.skip("ASan runtime not found")
    env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "host_sanitize_driver.py"), lib], env=env,
                       capture_output=True, text=True, timeout=600)
    report = r.stdout[-3000:] + r.stderr[-6000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, report
    assert "host paths ok" in r.stdout
