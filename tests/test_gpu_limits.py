"""The library's documented limits, through the C-ABI: profiles up to 4096
columns align bit-exactly against the oracle; a merge wider than that is a
SAD_E_CAPACITY error; sequences above 8192 residues are SAD_E_INVAL."""
import sys

import numpy as np
import pytest

import oracle
from workloads import generate, protein_matrix
from test_gpu_parity import compare, run_both

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


def test_widest_profiles(hip):
    """Three close relatives of ~4000 residues: merges of ~4000 x ~4000 columns
    (63 strips, the whole tie-byte scratch) and a refinement of the same size."""
    B, pipeline = hip
    _say("case widest profiles")
    s = generate(4096, 3, 20, 1, {"kind": "fixed", "value": 4000}, 0.02, 0.0005, 3)
    assert max(np.diff(s.offsets)) <= 4096
    got, ref = run_both(B, pipeline, s, 3, 1, protein_matrix(), 10, 1, 1)
    assert ref["refine"]["width"] <= 4096
    compare(got, ref, "widest profiles")


def test_width_beyond_limit(hip):
    B, pipeline = hip
    _say("case width beyond the limit")
    rng = np.random.default_rng(17)
    L = 5000
    codes = rng.integers(0, 20, 2 * L).astype(np.uint8)
    offsets = np.array([0, L, 2 * L], np.int64)
    prm = B.Params(3, 1, protein_matrix(), 10, 1, 1024, 1)
    with pytest.raises(B.SadError) as e:
        pipeline.run(codes, offsets, 20, prm)
    assert e.value.code == B.SAD_E_CAPACITY


def test_sequence_beyond_limit(hip):
    B, pipeline = hip
    _say("case sequence beyond the limit")
    rng = np.random.default_rng(18)
    lens = [8193, 100, 100, 100]
    offsets = np.zeros(5, np.int64)
    offsets[1:] = np.cumsum(lens)
    codes = rng.integers(0, 20, int(offsets[-1])).astype(np.uint8)
    seqs = pipeline.to_device(codes, offsets, 20)
    with pytest.raises(B.SadError) as e:
        B.sad_kmer_rank(seqs, B.Params(3, 2, protein_matrix(), 10, 1))
    assert e.value.code == B.SAD_E_INVAL
