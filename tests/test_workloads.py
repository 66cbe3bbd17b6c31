"""The seeded input generator: determinism, laws, and matrix properties."""
import numpy as np
import pytest

from workloads import (CONFIGS, SplitMix64, dna_matrix, generate, make_inputs, protein_matrix)
from workloads.matrices import load_ncbi_matrix, validate_matrix
from workloads.synth import family_sizes


def test_splitmix64_reference_values():
    # First outputs of SplitMix64 seeded with 0 (Steele, Lea & Flood 2014).
    r = SplitMix64(0)
    got = [int(v) for v in r.u64(3)]
    assert got == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_generator_deterministic():
    a = make_inputs("prot64")
    b = generate(CONFIGS["prot64"].seed, 64, 20, 1, {"kind": "fixed", "value": 100}, 0.1, 0.02, 3)
    assert a.sha256() == b.sha256()
    assert a.n == 64
    assert (a.lengths >= 3).all()
    assert a.codes.max() < 20


def test_generator_laws_prot2000():
    s = make_inputs("prot2000")
    assert s.n == 2000
    fam, cnt = np.unique(s.family, return_counts=True)
    assert list(cnt) == [250] * 8
    L = s.lengths
    assert 150 < L.mean() < 450
    # substitutions are uniform: residue frequencies near 1/20
    f = np.bincount(s.codes, minlength=20) / len(s.codes)
    assert np.abs(f - 0.05).max() < 0.01


def test_homology_ids_consistent():
    s = make_inputs("prot64")
    # a homology id occurs at most once per sequence and ids increase along each sequence
    for i in range(s.n):
        h = s.homology[s.offsets[i]:s.offsets[i + 1]]
        assert len(np.unique(h)) == len(h)


def test_family_sizes_zipf():
    sz = family_sizes(20000, 64, 1.2)
    assert sz.sum() == 20000 and sz.min() >= 2 and (np.diff(sz) <= 0).all()
    eq = family_sizes(50000, 32, None)
    assert eq.sum() == 50000 and eq.max() - eq.min() <= 1


def test_matrices():
    m = protein_matrix()
    validate_matrix(m)
    assert m.shape == (20, 20)
    assert np.diag(m).min() >= 4 and np.diag(m).max() <= 11
    off = m[~np.eye(20, dtype=bool)]
    assert off.min() >= -4 and off.max() <= 3
    d = dna_matrix()
    validate_matrix(d)
    assert d[0, 0] == 2 and d[0, 1] == -3


def test_ncbi_loader(tmp_path):
    order = "ACGT"
    text = "# toy\n   A  C  G  T  N\nA  5 -4 -4 -4 -2\nC -4  5 -4 -4 -2\nG -4 -4  5 -4 -2\n" \
           "T -4 -4 -4  5 -2\nN -2 -2 -2 -2 -1\n"
    p = tmp_path / "m.txt"
    p.write_text(text)
    m = load_ncbi_matrix(str(p), order)
    assert m.dtype == np.int8 and m[0, 0] == 5 and m[1, 2] == -4
    validate_matrix(m)


def test_bad_matrix_rejected():
    m = dna_matrix().copy()
    m[0, 1] = 3
    with pytest.raises(ValueError):
        validate_matrix(m)


def test_inputs_match_frozen_manifest():
    """Every workload regenerates byte for byte as frozen in
    tests/data/manifest.json (codes, offsets and homology ids)."""
    import hashlib
    import json
    import os
    from workloads import CONFIGS, make_inputs
    with open(os.path.join(os.path.dirname(__file__), "data", "manifest.json")) as fh:
        man = json.load(fh)["workloads"]
    assert set(man) == set(CONFIGS)
    for name, exp in man.items():
        s = make_inputs(name)
        assert s.n == exp["n"] and int(s.offsets[-1]) == exp["residues"], name
        assert s.sha256() == exp["sha256"], name
        h = hashlib.sha256(np.ascontiguousarray(s.homology, dtype=np.int64).tobytes())
        assert h.hexdigest() == exp["homology_sha256"], name
    make_inputs.cache_clear()


def test_parallel_generation_is_identical():
    from workloads import generate
    kw = dict(seed=77, n=600, alphabet=20, n_families=12,
              root_len={"kind": "normal", "mean": 120, "sd": 30, "lo": 40, "hi": 200},
              p_sub=0.1, p_indel=0.02, min_len=3, zipf=1.2)
    a = generate(**kw, workers=1)
    b = generate(**kw, workers=4)
    assert a.sha256() == b.sha256()
    assert np.array_equal(a.homology, b.homology) and np.array_equal(a.family, b.family)
