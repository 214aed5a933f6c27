"""The host side of the library (geometry validation, FP64 plan tables, the C
ABI's argument checks, the PAT_FAULT hook) under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU: a host-only build of the same
sources, driven by tests/host_checks.py in a child process with the ASan
runtime preloaded.  Any sanitizer report fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("hipcc") is None and not os.path.exists("/opt/rocm/bin/hipcc"),
                    reason="needs hipcc")
def test_host_code_under_asan_and_ubsan():
    from paper_0808_3510_amd import build
    srcs = [os.path.join(build.CSRC, f) for f in os.listdir(build.CSRC)] + [os.path.join(ROOT, "include", "pat.h")]
    lib = build.SAN_LIB
    if not os.path.exists(lib) or os.path.getmtime(lib) < max(os.path.getmtime(f) for f in srcs):
        lib = build.build_host_sanitized()
    env = dict(os.environ)
    env["LD_PRELOAD"] = build.asan_runtime()
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=66"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1:exitcode=67"
    env.pop("PAT_FAULT", None)
    res = subprocess.run([sys.executable, os.path.join(ROOT, "tests", "host_checks.py"), lib], env=env,
                         capture_output=True, text=True, timeout=300)
    out = res.stdout + res.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert res.returncode == 0, out[-4000:]
    assert "host checks passed" in res.stdout
