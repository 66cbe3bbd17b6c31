"""Pins of the oracle's quality counts (the Q measure of Section 4: correctly
aligned residue pairs over the residue pairs of the reference) against
brute-force enumeration of residue pairs and alignments with known answers."""
import itertools

import numpy as np
import pytest

import oracle
from workloads import generate, make_inputs


def brute(colmap, cls):
    aligned = true_pairs = 0
    for a, b in itertools.combinations(range(len(cls)), 2):
        if cls[a] == cls[b]:
            true_pairs += 1
            aligned += int(colmap[a] == colmap[b])
    return aligned, true_pairs


@pytest.mark.parametrize("seed", range(6))
def test_quality_counts_brute_force(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 120))
    cls = rng.integers(0, max(1, n // 3), size=n)
    colmap = rng.integers(0, 6, size=n)
    assert oracle.quality_counts(colmap, cls) == brute(colmap, cls)


def test_quality_counts_empty():
    assert oracle.quality_counts(np.zeros(0, np.int32), np.zeros(0, np.int32)) == (0, 0)


def test_perfect_and_shifted_alignment():
    # 5 copies of one 40-residue sequence: residue t of every copy is class t
    nseq, L = 5, 40
    cls = np.tile(np.arange(L), nseq)
    colmap = np.tile(np.arange(L), nseq)
    a, t = oracle.quality_counts(colmap, cls)
    assert t == L * nseq * (nseq - 1) // 2 and a == t
    # shift one copy by one column: its pairs with the other four are lost
    shifted = colmap.copy()
    shifted[:L] += 1
    a2, t2 = oracle.quality_counts(shifted, cls)
    assert t2 == t and a2 == t - L * (nseq - 1)


def test_generator_classes_unique_within_sequences():
    s = make_inputs("prot64")
    cls, ncls = s.homology_classes()
    assert cls.min() == 0 and cls.max() == ncls - 1
    for i in range(s.n):
        c = cls[s.offsets[i]:s.offsets[i + 1]]
        assert len(np.unique(c)) == len(c)
    # residues of one class come from one family
    fam = np.repeat(s.family, np.diff(s.offsets))
    for c in np.unique(cls)[:200]:
        assert len(np.unique(fam[cls == c])) == 1


def test_pipeline_quality_in_range():
    s = generate(91, 12, 20, 2, {"kind": "fixed", "value": 60}, 0.1, 0.02, 3)
    from workloads import protein_matrix
    ref = oracle.run_pipeline(s.codes, s.offsets, s.alphabet, 3, 2, protein_matrix(), 10, 1)
    cls, _ = s.homology_classes()
    a, t = oracle.quality_counts(ref["refine"]["colmap"], cls)
    assert 0 < a <= t
