"""CPU tests of libvne: exported symbols, host-side ingest and colouring
(bit-exact against the oracle), validation, and the kernel work schedule.
No GPU call is made here."""
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import synth
import paper_2212_09642_amd as vne

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "vne.h")).read()
    declared = sorted(set(re.findall(r"\b(vne_[a-z_0-9]+)\s*\(", hdr)))
    assert declared == sorted(vne.EXPORTS)
    L = vne.lib()
    for name in declared:
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", vne.LIB_PATH], capture_output=True, text=True).stdout
    for name in declared:
        assert re.search(r"\sT\s%s$" % name, out, re.M), name


GRAPHS = [lambda: synth.erdos_renyi(300, 2.0, 5), lambda: synth.erdos_renyi(2000, 8.0, 2212),
          lambda: synth.barabasi_albert(3000, 3, 1), lambda: synth.two_components(5, 12),
          lambda: synth.watts_strogatz(4000, 10, 0.1, 3), lambda: synth.star_graph(90),
          lambda: synth.complete_graph(33), lambda: synth.grid2d_graph(20, 31)]


@pytest.mark.parametrize("maker", GRAPHS)
@pytest.mark.parametrize("dtype", [np.float32, np.float64])
def test_laplacian_bit_exact_with_oracle(maker, dtype):
    n, e = maker()
    # noise the oracle must ignore in the same way: duplicates, reversed pairs, self loops
    noisy = np.concatenate([e, e[: len(e) // 3, ::-1], np.array([[0, 0], [n - 1, n - 1]])])
    a = vne.laplacian_from_edges(n, noisy, dtype)
    o = oracle.laplacian_from_edges(n, noisy)
    assert np.array_equal(a["row_ptr"], o.row_ptr)
    assert np.array_equal(a["col_idx"], o.col_idx)
    assert np.array_equal(a["values"].astype(np.float64), o.values)
    assert np.array_equal(a["node_ids"], o.node_ids)
    assert a["scale"] == o.scale


def test_laplacian_errors():
    with pytest.raises(vne.VneError):
        vne.laplacian_from_edges(1, np.zeros((0, 2)))            # no edge
    with pytest.raises(vne.VneError):
        vne.laplacian_from_edges(5, np.array([[0, 5]]))          # out of range
    with pytest.raises(vne.VneError):
        vne.laplacian_from_edges(0, np.zeros((0, 2)))
    a = vne.laplacian_from_edges(2, np.array([[0, 1]]))
    assert a["n"] == 2 and a["values"].tolist() == [1, -1, -1, 1] and a["scale"] == 0.5


@pytest.mark.parametrize("maker", GRAPHS)
@pytest.mark.parametrize("d", [1, 2, 3])
def test_coloring_bit_exact_with_oracle(maker, d):
    n, e = maker()
    a = vne.laplacian_from_edges(n, e)
    c1, s1 = vne.color_greedy(a["row_ptr"], a["col_idx"], a["values"], d)
    c2, s2 = oracle.greedy_distance_coloring(a["row_ptr"], a["col_idx"], a["n"], d)
    assert s1 == s2 and np.array_equal(c1, c2)


@pytest.mark.parametrize("maker", [lambda: synth.erdos_renyi(300, 2.0, 5), lambda: synth.grid2d_graph(20, 31),
                                   lambda: synth.watts_strogatz(600, 6, 0.1, 8), lambda: synth.path_graph(400)])
@pytest.mark.parametrize("d", [5, 8, 13])
def test_coloring_larger_distances_bit_exact_with_oracle(maker, d):
    # odd and even d split the distance between the two balls differently
    n, e = maker()
    a = vne.laplacian_from_edges(n, e)
    c1, s1 = vne.color_greedy(a["row_ptr"], a["col_idx"], a["values"], d)
    c2, s2 = oracle.greedy_distance_coloring(a["row_ptr"], a["col_idx"], a["n"], d)
    assert s1 == s2 and np.array_equal(c1, c2)


def test_coloring_distance_range():
    a = vne.laplacian_from_edges(*synth.path_graph(300))
    c, s = vne.color_greedy(a["row_ptr"], a["col_idx"], a["values"], 254)
    # nodes of a path within distance 254 of each other all differ: 255 colours
    assert s == 255
    for i in range(a["n"]):
        assert c[i] not in c[i + 1:i + 255]
    for d in (0, 255):
        with pytest.raises(vne.VneError):
            vne.color_greedy(a["row_ptr"], a["col_idx"], a["values"], d)


@pytest.mark.slow
def test_coloring_probing_workload_full_size():
    # WS n=1e6, k=10, p=0.1, distance 2: the probing configuration
    from synth import workloads
    w = workloads.probing()
    a = vne.laplacian_from_edges(w["n_nodes"], w["edges"])
    c1, s1 = vne.color_greedy(a["row_ptr"], a["col_idx"], a["values"], 2)
    c2, s2 = oracle.greedy_distance_coloring(a["row_ptr"], a["col_idx"], a["n"], 2)
    assert s1 == s2 and np.array_equal(c1, c2)
    assert 11 <= s1 <= 10 ** 2 + 1


def test_validation_rejects_bad_csr():
    a = vne.laplacian_from_edges(*synth.cycle_graph(6))
    rp, ci, va = a["row_ptr"], a["col_idx"], a["values"]
    st, _ = vne.csr_validate(rp, ci, va, a["scale"], vne.VALIDATE_SYMMETRIC | vne.VALIDATE_ZERO_ROWSUM)
    assert st == 0
    bad = ci.copy(); bad[1], bad[2] = bad[2], bad[1]          # unsorted row
    assert vne.csr_validate(rp, bad, va, 1.0)[0] == -1
    bad = ci.copy(); bad[0] = 6                              # out of range
    assert vne.csr_validate(rp, bad, va, 1.0)[0] == -1
    badv = va.copy(); badv[3] = np.nan
    assert vne.csr_validate(rp, ci, badv, 1.0)[0] == -1
    badv = va.copy(); badv[1] = -2.0                          # asymmetric, nonzero row sum
    assert vne.csr_validate(rp, ci, badv, 1.0, vne.VALIDATE_SYMMETRIC)[0] == -1
    assert vne.csr_validate(rp, ci, badv, 1.0, vne.VALIDATE_ZERO_ROWSUM)[0] == -1
    assert vne.csr_validate(rp, ci, va, 0.0)[0] == -1        # scale must be > 0
    badr = rp.copy(); badr[-1] += 1
    assert vne.csr_validate(badr, ci, va, 1.0)[0] == -1


def test_work_schedule_invariants(tmp_path):
    exe = str(tmp_path / "test_schedule")
    csrc = os.path.join(ROOT, "paper_2212_09642_amd", "csrc")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                    "-I", os.path.join(ROOT, "include"), "-I", csrc,
                    os.path.join(ROOT, "tests", "cpp", "test_schedule.cpp"),
                    os.path.join(csrc, "host_graph.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0 and "schedule ok" in r.stdout, r.stdout + r.stderr
