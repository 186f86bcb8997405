"""Host helpers of bench.py: the golden-file oracle check of a bench line
(used only when graph, probes and sizes match) and the source hash that keeps
counter traffic from being reused on other kernels."""
import json

import pytest

import bench


def test_oracle_check_matches_only_the_same_problem():
    with open(bench.os.path.join(bench.ROOT, "tests", "golden", "hutchpp_large.json")) as fh:
        g = json.load(fh)
    keys = dict(workload=g["workload"], n=g["n"], nnz=g["nnz"], n_sketch=g["n_sketch"], k=g["k"],
                probe_seed=g["probe_seed"])
    est = g["estimate"] * (1 + 2e-9)
    chk = bench.oracle_check("hutchpp_large.json", est, **keys)
    assert chk["oracle_estimate"] == g["estimate"] and chk["bar"] == 1e-5
    assert chk["rel_err"] == pytest.approx(2e-9, rel=1e-6)
    # another seed, size or step count: no check
    for k, v in (("probe_seed", g["probe_seed"] + 1), ("k", g["k"] + 1), ("n", g["n"] - 1)):
        assert bench.oracle_check("hutchpp_large.json", est, **dict(keys, **{k: v})) is None
    assert bench.oracle_check("no_such_golden.json", est, **keys) is None


def test_adaptive_golden_keys():
    with open(bench.os.path.join(bench.ROOT, "tests", "golden", "hutchpp_adaptive_large.json")) as fh:
        g = json.load(fh)
    chk = bench.oracle_check("hutchpp_adaptive_large.json", g["estimate"], rel_eps=g["rel_eps"], delta=g["delta"],
                             k=g["k"], probe_seed=g["probe_seed"], n=g["n"], nnz=g["nnz"])
    assert chk["rel_err"] == 0.0
    assert bench.oracle_check("hutchpp_adaptive_large.json", g["estimate"], rel_eps=1e-3, delta=g["delta"],
                              k=g["k"], probe_seed=g["probe_seed"], n=g["n"], nnz=g["nnz"]) is None


def test_traffic_is_dropped_for_other_sources(tmp_path, monkeypatch):
    # a traffic summary taken on other kernel sources reads as null
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "lanczos_step_w_traffic.json").write_text(json.dumps(
        {"hbm_bytes_per_launch": 123.0, "kernel_source_hash": "not-this-source"}))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "this-source")
    assert bench.load_traffic("w") is None
    (prof / "lanczos_step_w_traffic.json").write_text(json.dumps(
        {"hbm_bytes_per_launch": 123.0, "kernel_source_hash": "this-source"}))
    assert bench.load_traffic("w") == 123.0
    assert bench.load_traffic("missing") is None


def test_serve_summary_keeps_each_stopping_rule_apart():
    # the first rule's rates are the object's own; each other rule sits in a
    # sub-object of its own, with the same pool and arrivals
    rows_b, rows_e = [{"offered_per_s": 20.0, "completed_per_s": 19.0}], [{"offered_per_s": 20.0,
                                                                           "completed_per_s": 20.0}]
    sv = dict(pool=24, exact_graphs=2, rel_eps=1e-3, rows=rows_b, rows_by_rule={"bound": rows_b, "estimate": rows_e})
    out = bench.serve_summary(sv, [20.0], 200)
    assert out["stop"] == "bound" and out["rates"] is rows_b
    assert out["stop_estimate"] == {"stop": "estimate", "rates": rows_e}
    one = bench.serve_summary(dict(sv, rows_by_rule={"bound": rows_b}), [20.0], 200)
    assert "stop_estimate" not in one and one["rates"] is rows_b
