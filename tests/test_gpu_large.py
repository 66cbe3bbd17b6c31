"""Parity at the large workloads, in the launch configuration the benchmark
uses, on outputs the oracle can recompute one by one: rank keys of sampled
sequences (sum of F against the GPU's samples), the partition of the GPU's
keys, and whole buckets re-aligned by the oracle.  Plus properties that hold
at any size (degapped rows, widths, glued alignment restricted to a bucket)."""
import sys

import numpy as np
import pytest

import oracle
from workloads import make_inputs, workload

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def hip():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0901_2742_amd import binding as B
    from paper_0901_2742_amd import pipeline
    B.lib()
    return B, pipeline


def check_rows(offsets, ids, colmap, width):
    used = np.zeros(width, bool)
    for i in ids:
        c = colmap[offsets[i]:offsets[i + 1]]
        assert (np.diff(c) > 0).all() and c.min() >= 0 and c.max() < width
        used[c] = True
    assert used.all()


@pytest.mark.parametrize("name,nbuckets", [("prot20k", 3), ("dna50k", 2), ("prot200k", 2)])
def test_large_sampled(hip, name, nbuckets):
    B, pipeline = hip
    _say(f"case {name}")
    w = workload(name)
    s = make_inputs(name)
    prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, 1)
    got = pipeline.run(s.codes, s.offsets, s.alphabet, prm)
    rng = np.random.default_rng(1)
    samples = got["samples"]
    for i in rng.choice(s.n, 4, replace=False):
        ref = sum(oracle.fhat(s.seq(i), s.seq(j), s.alphabet, w.kmer_k) for j in samples)
        assert int(got["key"][i]) == ref
    part = oracle.partition(got["key"], w.p)
    boff, mem = got["part"]["bucket_off"], got["part"]["members"]
    assert np.array_equal(part["bucket_off"], boff) and np.array_equal(part["members"], mem)
    al = got["align"]
    for b in rng.choice(w.p, nbuckets, replace=False):
        ids = mem[boff[b]:boff[b + 1]]
        sub = s.subset(ids)
        ra = oracle.align_buckets(sub.codes, sub.offsets, s.alphabet,
                                  np.array([0, len(ids)], np.int32),
                                  np.arange(len(ids), dtype=np.int32), w.kmer_k, w.subst(),
                                  w.gap_open, w.gap_extend)
        gcm = np.concatenate([al["colmap"][s.offsets[i]:s.offsets[i + 1]] for i in ids])
        assert np.array_equal(gcm, ra["colmap"]), f"bucket {b}"
        assert al["width"][b] == ra["width"][0]
        sl = slice(boff[b], boff[b] + len(ids) - 1)
        assert np.array_equal(al["merge_score"][sl], ra["merge_score"][:len(ids) - 1])
        assert np.array_equal(al["merge_list"][sl], ra["merge_list"][:len(ids) - 1])
    for b in range(w.p):
        ids = mem[boff[b]:boff[b + 1]]
        if len(ids):
            check_rows(s.offsets, ids, al["colmap"], int(al["width"][b]))
    rf = got["refine"]
    check_rows(s.offsets, range(s.n), rf["colmap"], rf["width"])
    for b in rng.choice(w.p, 8, replace=False):
        ids = mem[boff[b]:boff[b + 1]]
        res = np.concatenate([np.arange(s.offsets[i], s.offsets[i + 1]) for i in ids])
        used = np.unique(rf["colmap"][res])
        assert np.array_equal(np.searchsorted(used, rf["colmap"][res]), al["colmap"][res])
