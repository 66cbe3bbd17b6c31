"""Parity of sad_quality (the Q measure of Section 4 against homology classes)
with the oracle's counts: exact integers, on the glued alignments of the
seeded workloads and on random inputs with edge cases (no residues,
singleton classes, one class of 3000 members, an id out of range)."""
import sys

import numpy as np
import pytest

import oracle
from workloads import CONFIGS, make_inputs

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


@pytest.mark.parametrize("name", ["prot64", "prot2000"])
def test_quality_of_pipeline(hip, name):
    B, pipeline, torch = hip
    _say(f"case quality {name}")
    w = CONFIGS[name]
    s = make_inputs(name)
    prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, B.SAD_BATCHED_MFMA)
    got = pipeline.run(s.codes, s.offsets, s.alphabet, prm)
    cls, ncls = s.homology_classes()
    colmap = got["refine"]["colmap"]
    a, t = B.sad_quality(torch.tensor(colmap, dtype=torch.int32, device="cuda"),
                         torch.tensor(cls, device="cuda"), ncls)
    assert (a, t) == oracle.quality_counts(colmap, cls)
    assert 0 < a <= t


@pytest.mark.parametrize("seed,n,ncls,ncol", [(1, 1000, 300, 50), (2, 5000, 5000, 20),
                                              (3, 3000, 1, 7), (4, 20000, 4000, 400)])
def test_quality_random(hip, seed, n, ncls, ncol):
    B, _, torch = hip
    _say(f"case quality random seed={seed} n={n}")
    rng = np.random.default_rng(seed)
    cls = rng.integers(0, ncls, size=n).astype(np.int32)
    colmap = rng.integers(0, ncol, size=n).astype(np.int32)
    a, t = B.sad_quality(torch.tensor(colmap, device="cuda"), torch.tensor(cls, device="cuda"),
                         ncls)
    assert (a, t) == oracle.quality_counts(colmap, cls)


def test_quality_empty_and_errors(hip):
    B, _, torch = hip
    _say("case quality empty / errors")
    e = torch.zeros(0, dtype=torch.int32, device="cuda")
    assert B.sad_quality(e, e, 1) == (0, 0)
    cls = torch.tensor([0, 1, 5], dtype=torch.int32, device="cuda")
    col = torch.tensor([0, 0, 0], dtype=torch.int32, device="cuda")
    with pytest.raises(B.SadError) as err:
        B.sad_quality(col, cls, 3)
    assert err.value.code == B.SAD_E_INVAL
    with pytest.raises(B.SadError):
        B.sad_quality(col, cls, 0)
