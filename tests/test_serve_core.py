"""The serving loop's scheduling core (tickets, admission, ticks, stages,
completion) against a host-only executor and clock, with clients on several
threads: built with AddressSanitizer + UndefinedBehaviorSanitizer and with
ThreadSanitizer (tests/cpp/test_serve_core.cpp lists what it checks).  The
ThreadSanitizer build uses clang's runtime: the one of this image's g++
does not intercept pthread_cond_clockwait, which libstdc++'s
condition_variable calls, and reports every wait as a race."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2212_09642_amd", "csrc")
SOURCES = [os.path.join(ROOT, "tests", "cpp", "test_serve_core.cpp"), os.path.join(CSRC, "serve_core.cpp"),
           os.path.join(CSRC, "serve_host.cpp")]


def _build_and_run(cxx, flags, exe):
    subprocess.run([cxx, "-std=c++17", "-O1", "-g", "-pthread"] + flags +
                   ["-I", os.path.join(ROOT, "include"), "-I", CSRC] + SOURCES + ["-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    return r


def test_serve_core_asan(tmp_path):
    r = _build_and_run("g++", ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"],
                       str(tmp_path / "serve_core_asan"))
    assert r.returncode == 0 and "serve core ok" in r.stdout, r.stdout + r.stderr


def _clang():
    for c in ("/opt/rocm/lib/llvm/bin/clang++", "/opt/rocm/llvm/bin/clang++", shutil.which("clang++")):
        if c and os.path.exists(c):
            return c
    return None


def test_serve_core_tsan(tmp_path):
    cxx = _clang()
    if cxx is None:
        pytest.skip("no clang++ with a ThreadSanitizer runtime")
    r = _build_and_run(cxx, ["-fsanitize=thread"], str(tmp_path / "serve_core_tsan"))
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and "serve core ok" in r.stdout, r.stdout + r.stderr[-2000:]
