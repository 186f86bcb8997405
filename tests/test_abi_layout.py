"""The ctypes mirrors of the public structs have the size and field offsets
that a C compiler gives the declarations in include/vne.h (a layout slip
would silently corrupt every call that passes the struct)."""
import ctypes
import os
import shutil
import subprocess

import pytest

import paper_2212_09642_amd as vne

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

# C struct name -> ctypes mirror
PAIRS = {
    "vne_csr": vne._Csr, "vne_probes": vne._Probes, "vne_result": vne._Result,
    "vne_stop_rule": vne._StopRule, "vne_probing_cfg": vne._ProbingCfg,
    "vne_probing_result": vne._ProbingResult, "vne_distance_choice": vne._DistanceChoice,
    "vne_server_cfg": vne._ServerCfg, "vne_query": vne._Query, "vne_query_result": vne._QueryResult,
    "vne_server_info": vne._ServerInfo, "vne_rational_cfg": vne._RationalCfg,
    "vne_rational_out": vne._RationalOut, "vne_hutchpp_cfg": vne._HutchppCfg,
    "vne_hutchpp_result": vne._HutchppResult,
}


@pytest.fixture(scope="module")
def c_layout(tmp_path_factory):
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    d = tmp_path_factory.mktemp("abi")
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "vne.h"', "int main(void) {"]
    for cname, py in PAIRS.items():
        lines.append('  printf("%s size %%zu\\n", sizeof(%s));' % (cname, cname))
        for fname, _ in py._fields_:
            lines.append('  printf("%s %s %%zu\\n", offsetof(%s, %s));' % (cname, fname, cname, fname))
    lines += ["  return 0;", "}"]
    src = d / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = d / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    table = {}
    for line in out.splitlines():
        a, b, v = line.split()
        table[(a, b)] = int(v)
    return table


@pytest.mark.parametrize("cname", sorted(PAIRS))
def test_struct_layout_matches_header(c_layout, cname):
    py = PAIRS[cname]
    assert ctypes.sizeof(py) == c_layout[(cname, "size")]
    for fname, _ in py._fields_:
        assert getattr(py, fname).offset == c_layout[(cname, fname)], fname
