"""sad_partition_noalloc (static device scratch, no allocation) against
sad_partition through the C-ABI: identical pivots, buckets, offsets and
members on consecutive calls, the second with a smaller input (so the static
scratch holds the previous call's contents), and a host-side capacity error
for a partition larger than the static scratch."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _seqs_stub(n):
    from paper_0901_2742_amd import binding as B
    # the partition reads only the count and the keys
    codes = torch.zeros(1, dtype=torch.uint8, device="cuda")
    offs = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    return B.DeviceSeqs(n, 20, codes, offs, 0, 3)


def _both(seqs, key, prm):
    from paper_0901_2742_amd import binding as B
    ref = B.sad_partition(seqs, key, prm)
    ref = {k: v.clone() for k, v in ref.items()}
    got = B.sad_partition(seqs, key, prm, noalloc=True)
    torch.cuda.synchronize()
    for k in ("pivot_key", "pivot_id", "bucket", "bucket_off", "members"):
        assert torch.equal(ref[k], got[k]), k
    return got


def _params(p):
    from paper_0901_2742_amd import binding as B
    from workloads import workload
    w = workload("prot2000")
    return B.Params(w.kmer_k, p, w.subst(), w.gap_open, w.gap_extend, w.s_max, B.SAD_BATCHED_MFMA)


def test_noalloc_partition_matches_on_consecutive_calls():
    from paper_0901_2742_amd import binding as B
    from workloads import make_inputs, workload
    # 1: the 2000-protein workload's own rank keys, 16 buckets
    w = workload("prot2000")
    s = make_inputs("prot2000")
    seqs = B.DeviceSeqs.from_numpy(s.codes, s.offsets, s.alphabet)
    prm = _params(w.p)
    key, _ = B.sad_kmer_rank(seqs, prm)
    big = _both(seqs, key, prm)
    assert int(big["bucket_off"][-1]) == s.n
    # 2: a smaller input next (fewer ids, fewer buckets, many tied keys)
    rng = np.random.default_rng(7)
    n2, p2 = 301, 5
    key2 = torch.from_numpy(rng.integers(0, 4, n2).astype(np.int64)).cuda()
    small = _both(_seqs_stub(n2), key2, _params(p2))
    assert int(small["bucket_off"][-1]) == n2
    # 3: larger again, every id in one chunk order (p = 1) and p = 2
    for n3, p3 in ((1000, 1), (999, 2)):
        key3 = torch.from_numpy(rng.integers(0, 1 << 40, n3).astype(np.int64)).cuda()
        _both(_seqs_stub(n3), key3, _params(p3))


def test_noalloc_partition_at_the_largest_bucket_count():
    """200000 ids in 1024 buckets: the largest partition of the workloads fits."""
    rng = np.random.default_rng(11)
    n, p = 200000, 1024
    key = torch.from_numpy(rng.integers(0, 1 << 50, n).astype(np.int64)).cuda()
    got = _both(_seqs_stub(n), key, _params(p))
    assert int(got["bucket_off"][-1]) == n


def test_noalloc_partition_rejects_oversized_scratch():
    from paper_0901_2742_amd import binding as B
    n, p = 3000, 1500          # 24 p (p - 1) bytes of samples alone exceed 32 MiB
    key = torch.zeros(n, dtype=torch.int64, device="cuda")
    with pytest.raises(B.SadError) as e:
        B.sad_partition(_seqs_stub(n), key, _params(p), noalloc=True)
    assert e.value.code == B.SAD_E_CAPACITY
    assert "static scratch" in str(e.value)
    # and the check is on the host: the invalid-argument path still wins first
    with pytest.raises(B.SadError) as e:
        B.sad_partition(_seqs_stub(10), torch.zeros(10, dtype=torch.int64, device="cuda"),
                        _params(6), noalloc=True)
    assert e.value.code == B.SAD_E_INVAL
