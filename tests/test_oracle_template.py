"""Pins of the oracle's richer refinement template (the paper's future work
after Section 2.3.3): each bucket aligned with the ancestors' alignment as a
profile of q rows instead of GA as one row.

Independent checks: one non-empty bucket (both templates are the bucket's own
ancestor); identical ancestors (the q-row template is q times GA's one-row
profile, so every DP value scales by q: same alignments, scores times q);
and on tiny inputs the template rebuilt from the ancestors' recorded merges
and each refinement score checked against exhaustive enumeration."""
import numpy as np
import pytest

import oracle
from workloads import generate, protein_matrix, dna_matrix
from test_oracle_align import brute_best
from test_oracle_pipeline import check_rows, replay_bucket


def profile_of(codes, offsets, ids, colmap, width, A):
    C = np.zeros((width, A), np.int64)
    for i in ids:
        r = np.arange(offsets[i], offsets[i + 1])
        np.add.at(C, (colmap[r], codes[r]), 1)
    return C


def test_one_bucket_templates_agree(oracle_lib):
    s = generate(31, 14, 20, 1, {"kind": "fixed", "value": 40}, 0.1, 0.02, 3)
    ga = oracle.run_pipeline(s.codes, s.offsets, 20, 3, 1, protein_matrix(), 10, 1)
    ms = oracle.run_pipeline(s.codes, s.offsets, 20, 3, 1, protein_matrix(), 10, 1,
                             template="ga_msa")
    for key in ("colmap", "merge_score", "merge_cells", "ga"):
        assert np.array_equal(ga["refine"][key], ms["refine"][key])
    assert ga["refine"]["width"] == ms["refine"]["width"]


@pytest.mark.parametrize("q", [2, 3, 5])
def test_identical_ancestors_scale_by_q(oracle_lib, q):
    base = generate(500 + q, 6, 20, 1, {"kind": "fixed", "value": 30}, 0.15, 0.03, 3)
    m = base.n
    lens = np.diff(base.offsets)
    codes = np.tile(base.codes, q)
    offsets = np.zeros(q * m + 1, np.int64)
    offsets[1:] = np.cumsum(np.tile(lens, q))
    boff = np.arange(q + 1, dtype=np.int32) * m
    mem = np.arange(q * m, dtype=np.int32)
    S = protein_matrix()
    al = oracle.align_buckets(codes, offsets, 20, boff, mem, 3, S, 10, 1)
    ga = oracle.refine(codes, offsets, 20, boff, mem, al["colmap"], al["width"], 3, S, 10, 1)
    ms = oracle.refine(codes, offsets, 20, boff, mem, al["colmap"], al["width"], 3, S, 10, 1,
                       template="ga_msa")
    assert np.array_equal(ga["colmap"], ms["colmap"]) and ga["width"] == ms["width"]
    # ancestor merges are shared; refinement scores scale by q, cells do not change
    assert np.array_equal(ga["merge_score"][:q - 1], ms["merge_score"][:q - 1])
    assert np.array_equal(ga["merge_score"][q - 1:] * q, ms["merge_score"][q - 1:])
    assert np.array_equal(ga["merge_cells"], ms["merge_cells"])


@pytest.mark.parametrize("seed", range(4))
def test_refinement_scores_optimal_against_rebuilt_template(oracle_lib, seed):
    rng = np.random.default_rng(900 + seed)
    A, k = 4, 2
    S = dna_matrix()
    n = 6
    lens = rng.integers(3, 6, n)
    offsets = np.zeros(n + 1, np.int64)
    offsets[1:] = np.cumsum(lens)
    codes = rng.integers(0, A, int(offsets[-1])).astype(np.uint8)
    boff = np.array([0, 2, 4, 6], np.int32)
    mem = np.arange(n, dtype=np.int32)
    go, ge = 3, 1
    al = oracle.align_buckets(codes, offsets, A, boff, mem, k, S, go, ge)
    rf = oracle.refine(codes, offsets, A, boff, mem, al["colmap"], al["width"], k, S, go, ge,
                       template="ga_msa")
    check_rows(codes, offsets, range(n), rf["colmap"], rf["width"])
    # ancestors, then their alignment replayed from its recorded op strings
    q = 3
    profs, ancs = [], []
    for b in range(q):
        ids = mem[boff[b]:boff[b + 1]]
        C = profile_of(codes, offsets, ids, al["colmap"], int(al["width"][b]), A)
        profs.append((C, len(ids)))
        ancs.append(oracle.consensus(C, len(ids)))
    aoff = np.zeros(q + 1, np.int64)
    aoff[1:] = np.cumsum([len(a) for a in ancs])
    acodes = np.concatenate(ancs).astype(np.uint8)
    one = np.array([0, q], np.int32)
    amem = np.arange(q, dtype=np.int32)
    aal = oracle.align_buckets(acodes, aoff, A, one, amem, k, S, go, ge, want_ops=True)
    assert np.array_equal(aal["merge_list"][:q - 1].ravel(), rf["merge_list"][:q - 1].ravel())
    (T, tn), _ = replay_bucket(acodes, aoff, amem, A, S, go, ge, aal["merge_list"][:q - 1],
                               aal["merge_score"][:q - 1], aal["ops"], aal["ops_off"], 0)
    assert tn == q
    for b in range(q):
        C, nb = profs[b]
        best, _ = brute_best(C, nb, T, tn, S, go, ge)
        assert rf["merge_score"][q - 1 + b] == best
        assert rf["merge_cells"][q - 1 + b] == C.shape[0] * T.shape[0]
