"""Host C++ check of the threaded colouring (tests/cpp/test_coloring.cpp)
under AddressSanitizer + UndefinedBehaviorSanitizer and under
ThreadSanitizer: equal to a plain sequential first-fit reference for 1, 3
and 8 worker threads and for d = 1, 2, 3 from one shared search."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2212_09642_amd", "csrc")


@pytest.mark.parametrize("san", ["address,undefined", "thread"])
def test_threaded_colouring_matches_sequential_reference(tmp_path, san):
    exe = str(tmp_path / "test_coloring")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=" + san, "-pthread",
                    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                    os.path.join(ROOT, "tests", "cpp", "test_coloring.cpp"),
                    os.path.join(CSRC, "coloring.cpp"), os.path.join(CSRC, "host_graph.cpp"), "-o", exe],
                   check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0 and "colouring ok" in r.stdout, r.stdout + r.stderr[-4000:]
