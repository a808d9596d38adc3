"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The FP64 oracle (oracle/kc_oracle.c) is built with gcc and driven through every
entry point on degenerate and ragged grids (tests/sanitize/oracle_driver.c);
the library's autotune-cache parser (csrc/kc_tune.hip, host code only) is
built for the host alone and fed malformed, truncated, overlong and
out-of-range lines (tests/sanitize/cache_driver.cpp).  Any out-of-bounds
access or undefined operation aborts the driver, and the test fails.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    return r.returncode, r.stdout + r.stderr


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    src = [os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "kc_oracle.c")]
    flags = ["-std=c99", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
             "-fno-sanitize-recover=all", "-fsanitize=address,undefined"]
    rc, out = _run(["gcc"] + flags + src + ["-o", exe, "-lm"])
    assert rc == 0, out
    rc, out = _run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=1"))
    print(out)
    assert rc == 0 and "0 failures" in out, out
    assert "AddressSanitizer" not in out and "runtime error" not in out


def _hipcc():
    for c in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if c and os.path.exists(c):
            return c
    return None


@pytest.mark.skipif(_hipcc() is None, reason="hipcc not available")
def test_autotune_cache_parser_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "cache_driver")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1301_5058_amd", "csrc")]
    src = [os.path.join(ROOT, "paper_1301_5058_amd", "csrc", "kc_tune.hip"),
           os.path.join(SAN, "cache_driver.cpp")]
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    cmd = [_hipcc(), "--offload-host-only", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer"]
    rc, out = _run(cmd + host_san + inc + src + ["-o", exe])
    assert rc == 0, out
    rc, out = _run([exe, str(tmp_path / "cache.jsonl")], env=ENV)
    print(out)
    assert rc == 0 and "0 failed checks" in out, out
    assert "AddressSanitizer" not in out and "runtime error" not in out
