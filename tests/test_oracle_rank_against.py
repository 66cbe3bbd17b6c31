"""Pins of the oracle's rank against a given sample (Section 2.3.1): the
centralised rank (every sequence against all N) and the rank against an
explicit list, plus the host-side statistics of Table 1 / Figs. 1 and 3.

Independent checks: a Counter-based brute-force similarity matrix summed by
rows, identical sequences (every F = 2^31, so K_i = S 2^31), the globalised
rank of the oracle's own sampling step recomputed from its sample list, and
hand-computed statistics."""
from collections import Counter

import numpy as np
import pytest

import oracle
from paper_0901_2742_amd.rankstats import rank_stats


def brute_F(codes, offsets, k):
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


def random_set(rng, n, A, lo=8, hi=30):
    lens = rng.integers(lo, hi, n)
    offs = np.zeros(n + 1, np.int64)
    offs[1:] = np.cumsum(lens)
    codes = rng.integers(0, A, int(offs[-1])).astype(np.uint8)
    return codes, offs


@pytest.mark.parametrize("seed,n,A,k", [(1, 12, 20, 3), (2, 9, 4, 4), (3, 15, 4, 2)])
def test_central_rank_is_row_sum_of_brute_force_F(seed, n, A, k):
    rng = np.random.default_rng(seed)
    codes, offs = random_set(rng, n, A)
    F = brute_F(codes, offs, k)
    got = oracle.rank_against(codes, offs, A, k)
    want = [int(sum(F[i, :])) for i in range(n)]
    assert [int(v) for v in got] == want


def test_listed_sample_with_repeats_and_rows():
    rng = np.random.default_rng(7)
    codes, offs = random_set(rng, 10, 20)
    F = brute_F(codes, offs, 3)
    samples = np.array([3, 3, 0, 9], np.int32)  # a repeated id counts twice
    rows = np.array([9, 0, 4], np.int32)
    got = oracle.rank_against(codes, offs, 20, 3, samples=samples, rows=rows)
    want = [int(sum(F[i, s] for s in samples)) for i in rows]
    assert [int(v) for v in got] == want
    assert len(oracle.rank_against(codes, offs, 20, 3, samples=np.zeros(0, np.int32))) == 10
    assert not oracle.rank_against(codes, offs, 20, 3, samples=np.zeros(0, np.int32)).any()


def test_identical_sequences_closed_form():
    x = np.array([1, 5, 2, 7, 7, 3, 1, 5, 2], np.uint8)
    n = 6
    codes = np.tile(x, n)
    offs = np.arange(n + 1, dtype=np.int64) * len(x)
    got = oracle.rank_against(codes, offs, 20, 3)
    assert all(int(v) == n * (1 << 31) for v in got)


def test_globalised_rank_recomputed_from_its_sample():
    rng = np.random.default_rng(11)
    codes, offs = random_set(rng, 40, 20, 20, 60)
    key, sid = oracle.kmer_rank(codes, offs, 20, 3, 4)
    again = oracle.rank_against(codes, offs, 20, 3, samples=sid)
    assert np.array_equal(key, again)


def test_bad_ids_rejected():
    rng = np.random.default_rng(5)
    codes, offs = random_set(rng, 6, 20)
    for bad in ([0, 6], [-1]):
        with pytest.raises(oracle.OracleError) as e:
            oracle.rank_against(codes, offs, 20, 3, samples=np.array(bad, np.int32))
        assert e.value.code == oracle.E_INVAL
    with pytest.raises(oracle.OracleError):
        oracle.rank_against(codes, offs, 20, 3, rows=np.array([7], np.int32))


def test_rank_stats_hand_example():
    u = 1 << 31
    # central over S = 2: ranks 0.5, 1.0, 0.25; globalised over S = 1: 0.5, 0.5, 0.5
    c = [1 * u, 2 * u, u // 2]
    g = [u // 2, u // 2, u // 2]
    st = rank_stats(c, g, 2, 1, bins=4)
    assert st["central"] == {"max": 1.0, "min": 0.25, "mean": pytest.approx(1.75 / 3)}
    assert st["global"] == {"max": 0.5, "min": 0.5, "mean": 0.5}
    assert st["var_wrt_central"] == pytest.approx((0.0 + 0.25 + 0.0625) / 3)
    assert st["std_wrt_central"] == pytest.approx(np.sqrt(0.3125 / 3))
    assert st["hist_central"] == [0, 1, 1, 1]  # 0.25 | 0.5 | 1.0 (last bin closed)
    assert st["hist_global"] == [0, 0, 3, 0]
    with pytest.raises(ValueError):
        rank_stats([], [], 1, 1)
