"""Pins of the oracle's k-mer steps (Section 2, k-mer counts and r_ij) against
brute force: collections.Counter for the counts and fractions.Fraction for the
exact rational r_ij = c_ij / d_ij."""
import json
import os
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def kmers_brute(x, k):
    return Counter(tuple(int(v) for v in x[t:t + k]) for t in range(len(x) - k + 1))


def tau_of(t, A):
    v = 0
    for c in t:
        v = v * A + c
    return v


@pytest.mark.parametrize("A,k", [(20, 3), (4, 8), (4, 2), (20, 1), (20, 2)])
def test_kmer_list_vs_counter(oracle_lib, A, k):
    rng = np.random.default_rng(1)
    for trial in range(20):
        L = int(rng.integers(k, 60))
        x = rng.integers(0, A if trial % 3 else 2, L).astype(np.uint8)
        taus, cnts = oracle.kmer_list(x, A, k)
        ref = kmers_brute(x, k)
        exp = sorted((tau_of(t, A), c) for t, c in ref.items())
        assert list(zip(taus.tolist(), cnts.tolist())) == exp
        assert cnts.sum() == L - k + 1


def test_common_and_fhat_vs_fraction(oracle_lib):
    rng = np.random.default_rng(2)
    for trial in range(200):
        A = 4 if trial % 2 else 20
        k = int(rng.integers(1, 5)) if A == 4 else int(rng.integers(1, 4))
        Li, Lj = int(rng.integers(k, 40)), int(rng.integers(k, 40))
        alpha = int(rng.integers(2, A + 1))
        xi = rng.integers(0, alpha, Li).astype(np.uint8)
        xj = rng.integers(0, alpha, Lj).astype(np.uint8)
        ci, cj = kmers_brute(xi, k), kmers_brute(xj, k)
        c = sum(min(ci[t], cj[t]) for t in ci)
        assert oracle.common_kmers(xi, xj, A, k) == c
        r = Fraction(c, min(Li, Lj) - k + 1)
        assert 0 <= r <= 1
        assert oracle.fhat(xi, xj, A, k) == (r * 2 ** 31).__floor__()
        assert oracle.fhat(xj, xi, A, k) == oracle.fhat(xi, xj, A, k)


def test_fhat_identical_and_short(oracle_lib):
    rng = np.random.default_rng(3)
    x = rng.integers(0, 20, 50).astype(np.uint8)
    assert oracle.fhat(x, x, 20, 3) == 2 ** 31
    # a prefix shares all its k-mers with the full sequence: r = 1 as well
    assert oracle.fhat(x[:20], x, 20, 3) == 2 ** 31
    # shorter than k: no k-mers, similarity 0
    assert oracle.fhat(x[:2], x, 20, 3) == 0


def test_golden_kmer_examples(oracle_lib):
    with open(os.path.join(GOLDEN, "kmer_examples.json")) as f:
        cases = json.load(f)["cases"]
    for cs in cases:
        A, k = cs["A"], cs["k"]
        letters = cs["letters"]
        xi = np.array([letters.index(ch) for ch in cs["x"]], np.uint8)
        xj = np.array([letters.index(ch) for ch in cs["y"]], np.uint8)
        assert oracle.common_kmers(xi, xj, A, k) == cs["c"], cs
        assert oracle.fhat(xi, xj, A, k) == cs["fhat"], cs
