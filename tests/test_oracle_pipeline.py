"""Whole-pipeline invariants of the oracle (Sections 2.2-2.3.3): the output is
the input with gaps inserted, rows have equal length, no column is all gaps,
every merge's score equals the score of its alignment recomputed from the
children, and refinement keeps each bucket's own alignment intact (restricting
the glued alignment to one bucket gives back that bucket's alignment)."""
import numpy as np
import pytest

import oracle
from workloads import dna_matrix, make_inputs, protein_matrix, generate
from test_oracle_align import alignment_score, brute_best

M, X, Y = 0, 1, 2


def check_rows(codes, offsets, ids, colmap, width):
    """Degapped rows reproduce the inputs: residues keep their order and land
    in distinct increasing columns below the width; every column is used."""
    used = np.zeros(width, bool)
    for i in ids:
        c = colmap[offsets[i]:offsets[i + 1]]
        assert (np.diff(c) > 0).all()
        assert c.min() >= 0 and c.max() < width
        used[c] = True
    assert used.all(), "all-gap column"


def replay_bucket(codes, offsets, mem, A, S, go, ge, merges, scores, ops, ops_off, base):
    """Rebuilds the bucket alignment from the recorded op strings: leaves are
    one-row profiles; a merge lays out P1's and P2's columns by its ops."""
    n = len(mem)
    prof = {}
    cols = {}
    for a, sid in enumerate(mem):
        x = codes[offsets[sid]:offsets[sid + 1]]
        C = np.zeros((len(x), A), np.int64)
        C[np.arange(len(x)), x] = 1
        prof[a] = (C, 1)
        cols[a] = {sid: np.arange(len(x))}
    for t, (a, b) in enumerate(merges):
        (C1, n1), (C2, n2) = prof[a], prof[b]
        op = ops[ops_off[base + t]:ops_off[base + t + 1]]
        sc = C1 @ S.astype(np.int64) @ C2.T
        assert alignment_score(op, sc, n1 * n2 * go, n1 * n2 * ge) == scores[t]
        m1 = np.zeros(C1.shape[0], np.int64)
        m2 = np.zeros(C2.shape[0], np.int64)
        C = np.zeros((len(op), A), np.int64)
        i = j = 0
        for c, o in enumerate(op):
            if o != Y:
                C[c] += C1[i]
                m1[i] = c
                i += 1
            if o != X:
                C[c] += C2[j]
                m2[j] = c
                j += 1
        assert i == C1.shape[0] and j == C2.shape[0]
        prof[n + t] = (C, n1 + n2)
        cols[n + t] = {**{s: m1[v] for s, v in cols[a].items()},
                       **{s: m2[v] for s, v in cols[b].items()}}
    root = 2 * n - 2 if n > 1 else 0
    return prof[root], cols[root]


def run_and_check(s, A, k, p, S, go, ge):
    r = oracle.run_pipeline(s.codes, s.offsets, A, k, p, S, go, ge, want_ops=True)
    part, al, rf = r["part"], r["align"], r["refine"]
    boff, mem = part["bucket_off"], part["members"]
    n = s.n
    assert np.diff(boff).sum() == n
    total_cells = 0
    for b in range(p):
        ids = mem[boff[b]:boff[b + 1]]
        if len(ids) == 0:
            assert al["width"][b] == 0
            continue
        check_rows(s.codes, s.offsets, ids, al["colmap"], int(al["width"][b]))
        nb = len(ids)
        merges = al["merge_list"][boff[b]:boff[b] + nb - 1]
        scores = al["merge_score"][boff[b]:boff[b] + nb - 1]
        (C, nrows), cols = replay_bucket(s.codes, s.offsets, ids, A, S, go, ge, merges, scores,
                                         al["ops"], al["ops_off"], boff[b])
        assert nrows == nb and C.shape[0] == al["width"][b]
        for sid, cm in cols.items():
            assert (al["colmap"][s.offsets[sid]:s.offsets[sid + 1]] == cm).all()
        total_cells += int(al["merge_cells"][boff[b]:boff[b] + nb - 1].sum())
    assert total_cells == al["cells"]
    # glued alignment
    check_rows(s.codes, s.offsets, range(n), rf["colmap"], rf["width"])
    for b in range(p):
        ids = mem[boff[b]:boff[b + 1]]
        if len(ids) == 0:
            continue
        res = np.concatenate([np.arange(s.offsets[i], s.offsets[i + 1]) for i in ids])
        g = rf["colmap"][res]
        used = np.unique(g)
        # restriction to bucket b, all-gap columns dropped, is bucket b's alignment
        assert (np.searchsorted(used, g) == al["colmap"][res]).all()
        assert len(used) == al["width"][b]
    q = int((np.diff(boff) > 0).sum())
    assert len(rf["merge_score"]) == (q - 1) + q
    return r


def test_pipeline_prot64(oracle_lib):
    s = make_inputs("prot64")
    run_and_check(s, 20, 3, 4, protein_matrix(), 10, 1)


def test_pipeline_dna_small(oracle_lib):
    s = generate(77, 48, 4, 3, {"kind": "uniform_int", "lo": 60, "hi": 90}, 0.05, 0.01, 8)
    run_and_check(s, 4, 8, 4, dna_matrix(), 5, 2)


@pytest.mark.parametrize("p", [1, 2, 3, 8])
def test_pipeline_small_p(oracle_lib, p):
    s = generate(1234 + p, 24, 20, 2, {"kind": "fixed", "value": 40}, 0.2, 0.05, 3)
    run_and_check(s, 20, 3, p, protein_matrix(), 10, 1)


def test_pipeline_p1_refine_against_own_consensus(oracle_lib):
    """p = 1: one bucket; GA is its own consensus and the glued alignment keeps
    the bucket's columns in order."""
    s = generate(99, 20, 20, 1, {"kind": "fixed", "value": 30}, 0.1, 0.02, 3)
    r = run_and_check(s, 20, 3, 1, protein_matrix(), 10, 1)
    al, rf = r["align"], r["refine"]
    assert len(rf["merge_score"]) == 1


def test_small_merges_are_optimal(oracle_lib):
    """Tiny buckets: each merge's score is the enumerated optimum."""
    s = generate(5, 12, 4, 2, {"kind": "fixed", "value": 5}, 0.3, 0.0, 2)
    S = dna_matrix()
    r = oracle.run_pipeline(s.codes, s.offsets, 4, 2, 3, S, 5, 2, want_ops=True)
    boff, mem = r["part"]["bucket_off"], r["part"]["members"]
    al = r["align"]
    for b in range(3):
        ids = mem[boff[b]:boff[b + 1]]
        nb = len(ids)
        if nb < 2:
            continue
        # first merge joins two leaves: check it against enumeration
        a, c = al["merge_list"][boff[b]]
        x1 = s.seq(ids[a])
        x2 = s.seq(ids[c])
        C1 = np.eye(4, dtype=np.int64)[x1]
        C2 = np.eye(4, dtype=np.int64)[x2]
        score, _ = brute_best(C1, 1, C2, 1, S, 5, 2)
        assert score == al["merge_score"][boff[b]]


@pytest.mark.parametrize("name,p", [("prot64", 4), ("prot64", 7)])
def test_threads_do_not_change_results(oracle_lib, name, p):
    """The oracle's loops over sequences, chunks, buckets and refinement
    alignments give the same outputs on 4 threads as on one."""
    s = make_inputs(name)
    S = protein_matrix()
    outs = []
    try:
        for t in (1, 4):
            oracle.set_threads(t)
            outs.append(oracle.run_pipeline(s.codes, s.offsets, s.alphabet, 3, p, S, 10, 1))
            outs[-1]["rank_all"] = oracle.rank_against(s.codes, s.offsets, s.alphabet, 3)
    finally:
        oracle.set_threads(1)
    a, b = outs

    def same(x, y):
        if isinstance(x, dict):
            assert x.keys() == y.keys()
            for k in x:
                same(x[k], y[k])
        else:
            assert np.array_equal(np.asarray(x), np.asarray(y))
    same(a, b)


def test_threaded_tree_scan_keeps_the_merge_order(oracle_lib):
    """The guide tree's pair scan split over threads (steps with 256 or more
    clusters) gives the single-thread merges: a 400-member matrix with many
    tied averages (values from four levels) and one of distinct values."""
    rng = np.random.default_rng(11)
    n = 400
    mats = []
    tied = (rng.integers(0, 4, (n, n)) * (1 << 29)).astype(np.uint32)
    mats.append(np.triu(tied, 1) + np.triu(tied, 1).T)
    dist = rng.integers(0, 1 << 31, (n, n)).astype(np.uint32)
    mats.append(np.triu(dist, 1) + np.triu(dist, 1).T)
    try:
        for F in mats:
            got = []
            for t in (1, 5):
                oracle.set_threads(t)
                got.append(np.asarray(oracle.upgma(F)))
            assert np.array_equal(got[0], got[1])
    finally:
        oracle.set_threads(1)
