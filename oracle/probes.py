"""Probe vectors for the trace estimators.

* Rademacher vectors (+-1 entries): the paper draws N(0,1) vectors for
  Hutchinson's estimator (eq. (3.8)) and Hutch++ (eq. (3.9)) and only needs
  E[x x^T] = I; Rademacher vectors satisfy the same identity and are used
  here.  Entry (row key r, column c) is +1 or -1 by the top bit of the
  SplitMix64 output mix(seed + (r * 2^32 + c + 1) * 0x9E3779B97F4A7C15)
  (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
  OOPSLA 2014; the finalizer constants are those of the published SplitMix64):
  top bit 0 gives +1.  All arithmetic is modulo 2^64.
* Probing vectors v_l = sum of e_i over the nodes of colour l (eq. (3.1)).
* Implicit desingularization (Remark 4.6): c = b - (1^T b / n) 1.

Pinned by: the published SplitMix64 known-answer sequence
(tests/golden/splitmix64_kat.txt, outputs of the generator started from a
fixed state), which fixes the mixer bit for bit; statistical properties of
the Rademacher block (mean, second moment, independence of neighbouring
counters), one-hot structure of the probing block and c being orthogonal
to 1 (tests).
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64_mix(z):
    """SplitMix64 output function on uint64 input (vectorized)."""
    z = np.asarray(z, np.uint64).copy()
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def rademacher_block(seed, keys, cols):
    """n x len(cols) float64 block of +-1 entries; keys are row keys (the
    original node ids), cols the probe column indices."""
    keys = np.asarray(keys, np.uint64)
    cols = np.asarray(cols, np.uint64)
    with np.errstate(over="ignore"):
        ctr = (keys[:, None] << np.uint64(32)) + cols[None, :] + np.uint64(1)
        z = np.uint64(seed) + ctr * _GAMMA
    h = splitmix64_mix(z)
    return np.where((h >> np.uint64(63)) == 0, 1.0, -1.0)


def indicator_block(colors, n_colors):
    """eq. (3.1): column l is the indicator vector of colour class l."""
    colors = np.asarray(colors, np.int64)
    B = np.zeros((colors.size, n_colors))
    B[np.arange(colors.size), colors] = 1.0
    return B


def desingularize(B):
    """Remark 4.6: replace each column b by c = b - (1^T b / n) 1."""
    B = np.asarray(B, np.float64)
    return B - B.mean(axis=0, keepdims=True)
