"""Pins of the oracle's rank and partition steps (Sections 2, 2.3.1, 2.3.2).

The checks use an independent brute-force similarity matrix (Counter-based
k-mer counts), Python's sorted() and bisect for order statistics, and the
properties the paper states (bucket sizes add to N; keys fall between their
pivots; regular sampling keeps buckets below 2N/p)."""
import bisect
from collections import Counter

import numpy as np
import pytest

import oracle
from workloads import make_inputs


def brute_F(codes, offsets, A, k):
    n = len(offsets) - 1
    seqs = [codes[offsets[i]:offsets[i + 1]] for i in range(n)]
    cnt = [Counter(tuple(s[t:t + k]) for t in range(len(s) - k + 1)) for s in seqs]
    F = np.zeros((n, n), dtype=object)
    for i in range(n):
        for j in range(n):
            c = sum(min(v, cnt[j][t]) for t, v in cnt[i].items())
            d = min(len(seqs[i]), len(seqs[j])) - k + 1
            F[i, j] = (c << 31) // d
    return F


def chunk_bounds(n, p):
    return [(c * n // p, (c + 1) * n // p) for c in range(p)]


def random_set(rng, n, A, lo=8, hi=30, alpha=None):
    alpha = alpha or A
    lens = rng.integers(lo, hi, n)
    offs = np.zeros(n + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    codes = rng.integers(0, alpha, int(offs[-1])).astype(np.uint8)
    return codes, offs


@pytest.mark.parametrize("n,p,s_max", [(24, 3, 1024), (30, 4, 1024), (40, 5, 8), (13, 6, 1024),
                                       (10, 1, 1024), (20, 2, 1024)])
def test_rank_samples_and_keys(oracle_lib, n, p, s_max):
    rng = np.random.default_rng(n * 100 + p)
    codes, offs = random_set(rng, n, 4, alpha=3)
    k = 2
    F = brute_F(codes, offs, 4, k)
    key, samples = oracle.kmer_rank(codes, offs, 4, k, p, s_max)
    bounds = chunk_bounds(n, p)
    w_min = min(h - l for l, h in bounds)
    ks = min(p - 1, max(1, s_max // p), w_min - 1)
    assert len(samples) == p * ks
    for c, (lo, hi) in enumerate(bounds):
        w = hi - lo
        kloc = {i: sum(F[i, j] for j in range(lo, hi)) for i in range(lo, hi)}
        order = sorted(range(lo, hi), key=lambda i: (kloc[i], i))
        exp = [order[(t * w) // (ks + 1)] for t in range(1, ks + 1)]
        assert samples[c * ks:(c + 1) * ks].tolist() == exp
    for i in range(n):
        assert int(key[i]) == sum(F[i, s] for s in samples.tolist())


def test_rank_rejects_bad_inputs(oracle_lib):
    rng = np.random.default_rng(5)
    codes, offs = random_set(rng, 10, 4)
    with pytest.raises(oracle.OracleError):
        oracle.kmer_rank(codes, offs, 4, 2, 6)          # N < 2p
    bad = codes.copy()
    bad[3] = 7
    with pytest.raises(oracle.OracleError):
        oracle.kmer_rank(bad, offs, 4, 2, 2)            # code >= A
    with pytest.raises(oracle.OracleError):
        oracle.kmer_rank(codes, offs, 4, 9, 2)          # a sequence shorter than k
    with pytest.raises(oracle.OracleError):
        oracle.kmer_rank(codes, offs, 20, 4, 2)         # A^k above 2^16


def check_partition(key, p, out):
    n = len(key)
    bounds = chunk_bounds(n, p)
    Y = []
    for lo, hi in bounds:
        w = hi - lo
        order = sorted(range(lo, hi), key=lambda i: (int(key[i]), i))
        Y += [(int(key[order[(t * w) // p]]), order[(t * w) // p]) for t in range(1, p)]
    Y.sort()
    piv = [Y[p // 2 + (t - 1) * p - 1] for t in range(1, p)]
    assert [(int(a), int(b)) for a, b in zip(out["pivot_key"], out["pivot_id"])] == piv
    # bucket(i): number of pivots strictly below (K_i, i)
    for i in range(n):
        assert out["bucket"][i] == bisect.bisect_left(piv, (int(key[i]), i))
    boff = out["bucket_off"]
    assert boff[0] == 0 and boff[-1] == n and (np.diff(boff) >= 0).all()
    for b in range(p):
        mem = out["members"][boff[b]:boff[b + 1]]
        assert (np.diff(mem) > 0).all()
        assert (out["bucket"][mem] == b).all()
    return np.diff(boff)


@pytest.mark.parametrize("n,p", [(64, 4), (2000, 16), (100, 10), (21, 10), (50, 1), (9, 4)])
def test_partition_order_statistics(oracle_lib, n, p):
    rng = np.random.default_rng(n + p)
    # coarse keys force many equal K values, so the id tie-break matters
    key = rng.integers(0, max(n // 4, 2), n).astype(np.uint64) * np.uint64(1 << 33)
    out = oracle.partition(key, p)
    sizes = check_partition(key, p, out)
    assert sizes.sum() == n


@pytest.mark.parametrize("n,p", [(64, 4), (2000, 16), (1000, 8), (300, 10)])
def test_partition_regular_sampling_bound(oracle_lib, n, p):
    """Section 3: with regular sampling no bucket receives 2N/p items or more
    (asserted where every chunk holds at least p items)."""
    rng = np.random.default_rng(7 * n + p)
    for trial in range(5):
        key = rng.permutation(n).astype(np.uint64)
        out = oracle.partition(key, p)
        sizes = check_partition(key, p, out)
        assert sizes.max() < 2 * n / p


def test_partition_prot64_pipeline(oracle_lib):
    s = make_inputs("prot64")
    key, samples = oracle.kmer_rank(s.codes, s.offsets, 20, 3, 4)
    out = oracle.partition(key, 4)
    sizes = check_partition(key, 4, out)
    assert sizes.sum() == 64 and sizes.max() < 2 * 64 / 4
    assert len(samples) == 12 and len(set(samples.tolist())) == 12
