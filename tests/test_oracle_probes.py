"""Pins of the probe generators (eq. (3.1), (3.8); Remark 4.6)."""
import os

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _kat():
    seed, outs = None, []
    for line in open(os.path.join(GOLDEN, "splitmix64_kat.txt")):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        if line.startswith("seed"):
            seed = int(line.split()[1])
        else:
            outs.append(int(line))
    return seed, outs


def test_splitmix64_known_answers():
    seed, outs = _kat()
    gamma = 0x9E3779B97F4A7C15
    states = np.array([(seed + (i + 1) * gamma) % 2 ** 64 for i in range(len(outs))], np.uint64)
    got = [int(x) for x in oracle.splitmix64_mix(states)]
    assert got == outs


def test_rademacher_counter_layout():
    # entry (key r, col c) is the mix of seed + (r*2^32 + c + 1) * gamma
    seed = 77
    keys = np.array([0, 5, 2 ** 31 + 3])
    B = oracle.rademacher_block(seed, keys, np.arange(4))
    gamma = 0x9E3779B97F4A7C15
    for i, r in enumerate(keys):
        for c in range(4):
            z = (seed + ((int(r) << 32) + c + 1) * gamma) % 2 ** 64
            h = int(oracle.splitmix64_mix(np.array([z], np.uint64))[0])
            assert B[i, c] == (1.0 if h >> 63 == 0 else -1.0)


def test_rademacher_moments():
    n, m = 64, 20000
    X = oracle.rademacher_block(9642, np.arange(n), np.arange(m))
    assert set(np.unique(X)) == {-1.0, 1.0}
    assert abs(X.mean()) < 5 / np.sqrt(n * m)
    M = X @ X.T / m                                 # E[x x^T] = I
    assert np.abs(M - np.eye(n)).max() < 6 / np.sqrt(m)
    # neighbouring columns and seeds are uncorrelated
    assert abs((X[:, :-1] * X[:, 1:]).mean()) < 5 / np.sqrt(n * m)
    Y = oracle.rademacher_block(9643, np.arange(n), np.arange(m))
    assert abs((X * Y).mean()) < 5 / np.sqrt(n * m)


def test_indicator_and_desingularization():
    colors = np.array([0, 2, 1, 0, 2, 2])
    B = oracle.indicator_block(colors, 3)
    assert np.array_equal(B.sum(axis=1), np.ones(6))
    assert np.array_equal(B.sum(axis=0), [2, 1, 3])
    C = oracle.desingularize(B)
    assert np.abs(C.sum(axis=0)).max() < 1e-15
    assert np.allclose((C * C).sum(0), (B * B).sum(0) - B.sum(0) ** 2 / 6)
