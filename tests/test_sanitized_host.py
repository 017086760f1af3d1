"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer: a build
with both (device code unchanged) runs the C-ABI tests that need no GPU (argument
validation of every entry point, server and statistics calls, error strings) in a child
process with the sanitizer runtime preloaded; any report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_is_clean_under_asan_and_ubsan():
    from paper_1412_4080_amd import build
    try:
        hipcc = build.hipcc()
        runtime = build.sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(str(e))
    assert hipcc
    lib = build.build_sanitized()
    env = dict(os.environ)
    env["DS_LIBRARY"] = lib
    env["LD_PRELOAD"] = runtime
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    # the plain C client links the product library by name; it is covered by the product run
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
                        "-k", "not plain_c_client", os.path.join(ROOT, "tests", "test_capi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
