"""Pins of the oracle's tree-dependent refinement of the glued alignment.

The main pin re-runs the whole procedure in Python on tiny inputs, written
independently: group membership from the tree, the two parts' profiles, the
score of the present alignment (alignment_score), the best alignment by
exhaustive enumeration with the library's tie rule (brute_best), acceptance,
and the new layout.  Plus: identical sequences (already optimal: nothing
changes), a converged result is a fixed point, every accepted step raised the
score, and rows stay valid on a real workload."""
import numpy as np
import pytest

import oracle
from workloads import dna_matrix, generate, make_inputs, protein_matrix
from test_oracle_align import alignment_score, brute_best
from test_oracle_pipeline import check_rows

M, X, Y = 0, 1, 2


def python_refine_tree(codes, offsets, A, boff, mem, colmap, width, tree, S, go, ge, passes):
    n = len(offsets) - 1
    nb = np.diff(boff)
    leaves = [b for b in range(len(nb)) if nb[b] > 0]
    q = len(leaves)
    seq_leaf = {}
    for u, b in enumerate(leaves):
        for sid in mem[boff[b]:boff[b + 1]]:
            seq_leaf[int(sid)] = u
    cm = np.array(colmap, np.int64)
    W = int(width)
    recs = []
    if q < 2:
        return cm, W, recs
    children = {q + t: (int(a), int(b)) for t, (a, b) in enumerate(tree)}

    def leaves_under(v):
        if v < q:
            return {v}
        a, b = children[v]
        return leaves_under(a) | leaves_under(b)

    depth = {2 * q - 2: 0}
    for v in range(2 * q - 2, q - 1, -1):
        for c in children[v]:
            depth[c] = depth[v] + 1
    skip = int(tree[q - 2][1])
    order = sorted((v for v in range(2 * q - 2) if v != skip), key=lambda v: (-depth[v], v))
    for _ in range(passes):
        changed = False
        for v in order:
            g1 = leaves_under(v)
            in1 = np.array([seq_leaf[s] in g1 for s in range(n)])
            cols = [np.zeros((W, A), np.int64), np.zeros((W, A), np.int64)]
            for s in range(n):
                g = 0 if in1[s] else 1
                for r in range(offsets[s], offsets[s + 1]):
                    cols[g][cm[r], codes[r]] += 1
            h1 = cols[0].sum(1) > 0
            h2 = cols[1].sum(1) > 0
            assert (h1 | h2).all()
            C1, C2 = cols[0][h1], cols[1][h2]
            n1, n2 = int(in1.sum()), int(n - in1.sum())
            old = [M if a and b else (X if a else Y) for a, b in zip(h1, h2)]
            sc = C1 @ S.astype(np.int64) @ C2.T
            s_old = alignment_score(old, sc, n1 * n2 * go, n1 * n2 * ge)
            s_new, ops = brute_best(C1, n1, C2, n2, S, go, ge)
            recs.append((v, s_old, s_new))
            if s_new > s_old:
                i1 = np.cumsum(h1) - 1
                i2 = np.cumsum(h2) - 1
                m1, m2 = [], []
                for t, o in enumerate(ops):
                    if o != Y:
                        m1.append(t)
                    if o != X:
                        m2.append(t)
                for s in range(n):
                    for r in range(offsets[s], offsets[s + 1]):
                        cm[r] = m1[i1[cm[r]]] if in1[s] else m2[i2[cm[r]]]
                W = len(ops)
                changed = True
        if not changed:
            break
    return cm, W, recs


def tiny_case(seed):
    rng = np.random.default_rng(seed)
    A, k = 4, 1
    n = 6
    lens = rng.integers(2, 4, n)
    offsets = np.zeros(n + 1, np.int64)
    offsets[1:] = np.cumsum(lens)
    codes = rng.integers(0, A, int(offsets[-1])).astype(np.uint8)
    boff = np.array([0, 2, 4, 6], np.int32)
    mem = rng.permutation(n).astype(np.int32)
    for b in range(3):
        mem[boff[b]:boff[b + 1]] = np.sort(mem[boff[b]:boff[b + 1]])
    return A, k, codes, offsets, boff, mem


@pytest.mark.parametrize("seed", range(6))
def test_matches_independent_python_run(oracle_lib, seed):
    A, k, codes, offsets, boff, mem = tiny_case(3000 + seed)
    S = dna_matrix()
    go, ge = 4, 1
    al = oracle.align_buckets(codes, offsets, A, boff, mem, k, S, go, ge)
    rf = oracle.refine(codes, offsets, A, boff, mem, al["colmap"], al["width"], k, S, go, ge)
    tree = rf["merge_list"][:2]
    got = oracle.refine_tree(codes, offsets, A, boff, mem, rf["colmap"], rf["width"], tree, k, S,
                             go, ge, passes=2)
    cm, W, recs = python_refine_tree(codes, offsets, A, boff, mem, rf["colmap"], rf["width"],
                                     tree, S, go, ge, 2)
    assert got["steps"] == len(recs)
    assert [(int(a), int(b), int(c)) for a, b, c in
            zip(got["rec_node"], got["rec_old"], got["rec_new"])] == recs
    assert got["width"] == W and np.array_equal(got["colmap"], cm)
    check_rows(codes, offsets, range(len(offsets) - 1), got["colmap"], got["width"])


def test_identical_sequences_unchanged(oracle_lib):
    x = np.array([3, 1, 4, 1, 5, 9, 2, 6], np.uint8)
    n = 8
    codes = np.tile(x, n)
    offsets = np.arange(n + 1, dtype=np.int64) * len(x)
    boff = np.array([0, 2, 4, 6, 8], np.int32)
    mem = np.arange(n, dtype=np.int32)
    S = protein_matrix()
    al = oracle.align_buckets(codes, offsets, 20, boff, mem, 3, S, 10, 1)
    rf = oracle.refine(codes, offsets, 20, boff, mem, al["colmap"], al["width"], 3, S, 10, 1)
    got = oracle.refine_tree(codes, offsets, 20, boff, mem, rf["colmap"], rf["width"],
                             rf["merge_list"][:3], 3, S, 10, 1, passes=3)
    assert got["accepted"] == 0 and got["steps"] == 5  # 2q - 3 splits, one pass
    assert np.array_equal(got["colmap"], rf["colmap"]) and got["width"] == rf["width"]
    assert (got["rec_new"] == got["rec_old"]).all()


def test_workload_rows_valid_and_fixed_point(oracle_lib):
    s = generate(2024, 60, 20, 3, {"kind": "uniform_int", "lo": 40, "hi": 70}, 0.2, 0.04, 3)
    S = protein_matrix()
    r = oracle.run_pipeline(s.codes, s.offsets, 20, 3, 6, S, 10, 1)
    boff, mem = r["part"]["bucket_off"], r["part"]["members"]
    q = int((np.diff(boff) > 0).sum())
    tree = r["refine"]["merge_list"][:q - 1]
    got = oracle.refine_tree(s.codes, s.offsets, 20, boff, mem, r["refine"]["colmap"],
                             r["refine"]["width"], tree, 3, S, 10, 1, passes=8)
    check_rows(s.codes, s.offsets, range(s.n), got["colmap"], got["width"])
    assert (got["rec_new"] >= got["rec_old"]).all()
    assert got["accepted"] == int((got["rec_new"] > got["rec_old"]).sum())
    # every step's parts keep their own alignment (restriction to one side)
    for b in range(len(boff) - 1):
        ids = mem[boff[b]:boff[b + 1]]
        if len(ids) == 0:
            continue
        res = np.concatenate([np.arange(s.offsets[i], s.offsets[i + 1]) for i in ids])
        g, a = got["colmap"][res], r["align"]["colmap"][res]
        assert (np.searchsorted(np.unique(g), g) == a).all()
    if got["steps"] < 8 * (2 * q - 3):
        again = oracle.refine_tree(s.codes, s.offsets, 20, boff, mem, got["colmap"],
                                   got["width"], tree, 3, S, 10, 1, passes=1)
        assert again["accepted"] == 0
        assert np.array_equal(again["colmap"], got["colmap"])


def test_bad_tree_rejected(oracle_lib):
    A, k, codes, offsets, boff, mem = tiny_case(1)
    S = dna_matrix()
    al = oracle.align_buckets(codes, offsets, A, boff, mem, k, S, 4, 1)
    rf = oracle.refine(codes, offsets, A, boff, mem, al["colmap"], al["width"], k, S, 4, 1)
    with pytest.raises(oracle.OracleError):
        oracle.refine_tree(codes, offsets, A, boff, mem, rf["colmap"], rf["width"],
                           np.array([[0, 0], [1, 3]]), k, S, 4, 1)
