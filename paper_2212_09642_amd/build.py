"""Builds libvne.so in-tree: host C++ with g++, HIP sources with hipcc for gfx950."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libvne.so")

HOST_SOURCES = ["host_graph.cpp", "coloring.cpp", "serve_host.cpp", "serve_core.cpp", "probing_host.cpp"]
HIP_SOURCES = ["kernels.hip", "runtime.hip", "server.hip", "probing.hip", "noalloc.hip", "rational.hip",
               "hutchpp_adaptive.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
HIP_FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
CXX_FLAGS = ["-O2", "-fPIC", "-std=c++17", "-Wall"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose=True, out=None, defines=(), build_dir=None):
    """Compile and link libvne.so (or `out`); `defines` adds -D flags to the
    HIP sources (used for A/B measurements of compile-time options)."""
    lib_path = out or LIB
    bdir = build_dir or BUILD
    os.makedirs(bdir, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for src in HOST_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        _run(["g++"] + CXX_FLAGS + inc + ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    for src in HIP_SOURCES:
        obj = os.path.join(bdir, src + ".o")
        _run([HIPCC] + HIP_FLAGS + ["-D" + d for d in defines] + inc +
             ["-c", os.path.join(CSRC, src), "-o", obj])
        objs.append(obj)
    tmp = lib_path + ".tmp"
    # only the C ABI is exported
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC",
          "-Wl,--version-script=" + os.path.join(CSRC, "libvne.map"), "-o", tmp] + objs)
    os.replace(tmp, lib_path)
    return lib_path


if __name__ == "__main__":
    build()
    sys.exit(0)
