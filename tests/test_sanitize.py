"""Host code under the sanitizers (CPU only).

The CPU oracle (plain C) and the library's host close-encounter resolver
(C++, with its worker pool) are built with AddressSanitizer and
UndefinedBehaviorSanitizer (and the resolver once more with ThreadSanitizer)
into small driver programs under tests/sanitize/, which run their entry points
on small systems (list overflow, gas drag, big and small bodies, the full
method's groups).  Any sanitizer report or a wrong result fails the test.
Device code is not built here: the GPU has no sanitizer on this platform.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2601_19654_amd", "csrc")

ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]
TSAN = ["-fsanitize=thread", "-g", "-O1"]


def _build_and_run(cmd, exe, tmp_path):
    subprocess.check_call(cmd, cwd=tmp_path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    r = subprocess.run([str(tmp_path / exe)], capture_output=True, text=True, env=env, timeout=300)
    out = r.stdout + r.stderr
    print(out)
    assert r.returncode == 0, out
    for marker in ("runtime error", "AddressSanitizer", "LeakSanitizer", "ThreadSanitizer"):
        assert marker not in out, out
    return out


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no host C compiler")
def test_oracle_under_asan_ubsan(tmp_path):
    cmd = ["gcc", *ASAN, "-std=c99", "-ffp-contract=off", "-o", "oracle_asan",
           os.path.join(ROOT, "oracle", "nbody_oracle.c"), os.path.join(HERE, "oracle_driver.c"), "-lm"]
    out = _build_and_run(cmd, "oracle_asan", tmp_path)
    assert "full=1" in out and "cap=2" in out


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
@pytest.mark.parametrize("flags,name", [(ASAN, "resolve_asan"), (TSAN, "resolve_tsan")])
def test_host_resolver_under_sanitizers(tmp_path, flags, name):
    cmd = ["g++", *flags, "-std=c++17", "-pthread", "-I", CSRC, "-o", name,
           os.path.join(CSRC, "nb_resolve.cpp"), os.path.join(HERE, "resolve_driver.cpp")]
    out = _build_and_run(cmd, name, tmp_path)
    assert "3 groups, 9 bodies" in out and "identical" in out
