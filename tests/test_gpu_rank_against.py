"""Parity of sad_rank_against (the centralised rank and the rank against an
explicit sample, Section 2.3.1) with the oracle, bit-exact (integer keys)."""
import sys

import numpy as np
import pytest

import oracle
from workloads import generate, make_inputs

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
    return B, pipeline, torch


def _prot(n, seed):
    return generate(seed, n, 20, max(1, n // 250), {"kind": "normal", "mean": 316, "sd": 60,
                                                    "lo": 100, "hi": 600}, 0.10, 0.02, 3)


def test_central_rank_n500(hip):
    B, pipeline, torch = hip
    _say("case central rank N=500")
    s = _prot(500, 4242)
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
    got = B.sad_rank_against(seqs, 3).cpu().numpy().view(np.uint64)
    want = oracle.rank_against(s.codes, s.offsets, 20, 3)
    assert np.array_equal(got, want)


def test_central_rank_n5000_sampled_rows(hip):
    B, pipeline, torch = hip
    _say("case central rank N=5000 (sampled rows)")
    s = _prot(5000, 4243)
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
    got = B.sad_rank_against(seqs, 3).cpu().numpy().view(np.uint64)
    rows = np.unique(np.r_[0, 4999, np.random.default_rng(3).integers(0, 5000, 30)]).astype(np.int32)
    want = oracle.rank_against(s.codes, s.offsets, 20, 3, rows=rows)
    assert np.array_equal(got[rows], want)


def test_listed_sample_matches_kmer_rank(hip):
    B, pipeline, torch = hip
    _say("case rank against the globalised sample (prot2000)")
    s = make_inputs("prot2000")
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
    prm = B.Params(3, 16, np.zeros((20, 20), np.int8), 10, 1, 1024, 1)
    key, sid = B.sad_kmer_rank(seqs, prm)
    again = B.sad_rank_against(seqs, 3, sid)
    assert torch.equal(key, again)
    # a repeated id and a DNA set with k = 6 against the oracle
    d = generate(77, 300, 4, 2, {"kind": "uniform_int", "lo": 60, "hi": 200}, 0.1, 0.02, 6)
    dseqs = pipeline.to_device(d.codes, d.offsets, d.alphabet)
    smp = np.array([5, 5, 0, 299, 17], np.int32)
    got = B.sad_rank_against(dseqs, 6, torch.from_numpy(smp)).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, oracle.rank_against(d.codes, d.offsets, 4, 6, samples=smp))


def test_central_rank_dna_k8(hip):
    """k = 8 on DNA: a 4^8-entry (128 KB) histogram per row in LDS."""
    B, pipeline, torch = hip
    _say("case central rank DNA k=8")
    d = generate(8080, 240, 4, 3, {"kind": "uniform_int", "lo": 300, "hi": 700}, 0.05, 0.01, 8)
    seqs = pipeline.to_device(d.codes, d.offsets, d.alphabet)
    got = B.sad_rank_against(seqs, 8).cpu().numpy().view(np.uint64)
    assert np.array_equal(got, oracle.rank_against(d.codes, d.offsets, 4, 8))


def test_rank_against_errors(hip):
    B, pipeline, torch = hip
    _say("case rank against errors")
    s = _prot(40, 99)
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
    for bad in ([0, 40], [-3]):
        with pytest.raises(B.SadError) as e:
            B.sad_rank_against(seqs, 3, torch.tensor(bad, dtype=torch.int32))
        assert e.value.code == B.SAD_E_INVAL
    with pytest.raises(B.SadError) as e:
        B.sad_rank_against(seqs, 0)
    assert e.value.code == B.SAD_E_INVAL
    # an empty sample gives zero keys
    z = B.sad_rank_against(seqs, 3, torch.zeros(0, dtype=torch.int32))
    assert int(z.abs().sum()) == 0
