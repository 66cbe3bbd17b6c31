"""Pins of the oracle's guide tree and profile-profile alignment.

* UPGMA: scipy's average linkage on d = 1 - F / 2^31 (tie-free inputs) gives
  the same merge sequence; crafted ties pin the tie rule.
* Alignment: exhaustive enumeration of every alignment of two tiny profiles
  (all op strings over M/X/Y) gives the optimal score and, among optimal ones,
  the op string that is lexicographically smallest read backwards (M < X < Y);
  column scores come from numpy's C1 @ S @ C2.T.
* One-row profiles reduce to textbook pairwise affine alignment (Gotoh), coded
  here independently with its own three matrices.
"""
import itertools
import json
import os

import numpy as np
import pytest
from scipy.cluster.hierarchy import linkage
from scipy.spatial.distance import squareform

import oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
M, X, Y = 0, 1, 2


# ----------------------------------------------------------------- UPGMA

def test_upgma_matches_scipy_average_linkage(oracle_lib):
    rng = np.random.default_rng(11)
    for trial in range(60):
        n = int(rng.integers(2, 14))
        F = rng.integers(0, 2 ** 31, (n, n)).astype(np.int64)
        F = np.triu(F, 1)
        F = F + F.T
        np.fill_diagonal(F, 2 ** 31)
        merges = oracle.upgma(F.astype(np.uint32))
        D = 1.0 - F.astype(np.float64) / 2 ** 31
        np.fill_diagonal(D, 0.0)
        Z = linkage(squareform(D, checks=False), method="average")
        # skip inputs whose linkage heights come too close for float64 averaging
        if np.min(np.diff(np.sort(Z[:, 2]))) < 1e-9 if n > 2 else False:
            continue
        ref = [tuple(sorted((int(a), int(b)))) for a, b in Z[:, :2]]
        assert [tuple(m) for m in merges.tolist()] == ref


def test_upgma_tie_rule(oracle_lib):
    # all similarities equal: every pair ties; the smallest (min id, max id) wins
    F = np.full((4, 4), 7, np.uint32)
    assert oracle.upgma(F).tolist() == [[0, 1], [2, 3], [4, 5]]
    # ties between an old and a new cluster: (0,1) merge to 3; avg(3,2) = avg
    # of F[0,2], F[1,2] = 5 = nothing else; single choice
    F = np.array([[9, 9, 4], [9, 9, 6], [4, 6, 9]], np.uint32)
    assert oracle.upgma(F).tolist() == [[0, 1], [2, 3]]
    # exact rational comparison: 3 vs (5+1)/2 = 3 -> tie -> smaller pair key
    F = np.array([[0, 5, 1, 3], [5, 0, 0, 0], [1, 0, 0, 0], [3, 0, 0, 0]], np.uint32)
    # step 0: best pair (0,1) with 5; new id 4 = {0,1}; avg(4,3) = (3+0)/2,
    # avg(4,2) = (1+0)/2, avg(2,3) = 0 -> (3,4)
    assert oracle.upgma(F).tolist() == [[0, 1], [3, 4], [2, 5]]


def test_upgma_trivial(oracle_lib):
    assert oracle.upgma(np.zeros((1, 1), np.uint32)).shape == (0, 2)


# ------------------------------------------------------- alignment, brute force

def enumerate_alignments(W1, W2):
    out = []

    def rec(i, j, acc):
        if i == W1 and j == W2:
            out.append(tuple(acc))
            return
        if i < W1 and j < W2:
            rec(i + 1, j + 1, acc + [M])
        if i < W1:
            rec(i + 1, j, acc + [X])
        if j < W2:
            rec(i, j + 1, acc + [Y])

    rec(0, 0, [])
    return out


def alignment_score(ops, sc, o, e):
    """Score of an op string: column scores of M ops minus g(l) = o + (l-1) e
    per maximal run of X, and per maximal run of Y."""
    i = j = 0
    total = 0
    prev = None
    for op in ops:
        if op == M:
            total += int(sc[i, j])
            i += 1
            j += 1
        elif op == X:
            total -= e if prev == X else o
            i += 1
        else:
            total -= e if prev == Y else o
            j += 1
        prev = op
    return total


def brute_best(C1, n1, C2, n2, S, go, ge):
    sc = C1.astype(np.int64) @ S.astype(np.int64) @ C2.astype(np.int64).T
    G = n1 * n2
    best = None
    for ops in enumerate_alignments(C1.shape[0], C2.shape[0]):
        s = alignment_score(ops, sc, G * go, G * ge)
        key = (-s, tuple(reversed(ops)))
        if best is None or key < best:
            best = key
    return -best[0], list(reversed(best[1]))


def random_profile(rng, W, n, A, alpha):
    C = np.zeros((W, A), np.int64)
    for c in range(W):
        for r in range(n):
            if rng.random() < 0.8:
                C[c, rng.integers(0, alpha)] += 1
    return C


@pytest.mark.parametrize("seed", range(8))
def test_profile_align_vs_enumeration(oracle_lib, seed):
    rng = np.random.default_rng(100 + seed)
    for trial in range(60):
        A = int(rng.integers(2, 6))
        W1, W2 = int(rng.integers(0, 6)), int(rng.integers(0, 6))
        if W1 + W2 > 9:
            W2 = max(0, 9 - W1)
        n1, n2 = int(rng.integers(1, 4)), int(rng.integers(1, 4))
        S = rng.integers(-4, 6, (A, A)).astype(np.int8)   # not symmetric: catches transposes
        ge = int(rng.integers(0, 4))
        go = ge + int(rng.integers(0, 5))
        if trial % 7 == 0:
            go = ge                                         # o == e
        C1 = random_profile(rng, W1, n1, A, int(rng.integers(1, A + 1)))
        C2 = random_profile(rng, W2, n2, A, int(rng.integers(1, A + 1)))
        ops, score = oracle.profile_align(C1, n1, C2, n2, S, go, ge)
        bscore, bops = brute_best(C1, n1, C2, n2, S, go, ge)
        assert score == bscore
        assert ops.tolist() == bops, (W1, W2, A, go, ge)


def test_profile_align_all_ties(oracle_lib):
    """Zero scores and free gaps: every alignment ties, so the answer is the
    backward-lexicographic minimum among all of them."""
    S = np.zeros((2, 2), np.int8)
    C1 = np.ones((3, 2), np.int64)
    C2 = np.ones((4, 2), np.int64)
    ops, score = oracle.profile_align(C1, 1, C2, 1, S, 0, 0)
    assert score == 0
    _, bops = brute_best(C1, 1, C2, 1, S, 0, 0)
    assert ops.tolist() == bops
    # read backwards the smallest string is M M M then Y: forwards Y M M M
    assert ops.tolist() == [Y, M, M, M]


# ---------------------------------------------------- textbook pairwise Gotoh

def textbook_gotoh(a, b, S, go, ge):
    """Classic three-matrix affine global alignment score, gap of length l
    costing go + (l-1) ge, written independently of the oracle."""
    NEG = -10 ** 15
    n, m = len(a), len(b)
    Mm = [[NEG] * (m + 1) for _ in range(n + 1)]
    Ix = [[NEG] * (m + 1) for _ in range(n + 1)]
    Iy = [[NEG] * (m + 1) for _ in range(n + 1)]
    Mm[0][0] = 0
    for i in range(1, n + 1):
        Ix[i][0] = -go - (i - 1) * ge
    for j in range(1, m + 1):
        Iy[0][j] = -go - (j - 1) * ge
    for i in range(1, n + 1):
        for j in range(1, m + 1):
            prev = max(Mm[i - 1][j - 1], Ix[i - 1][j - 1], Iy[i - 1][j - 1])
            Mm[i][j] = prev + int(S[a[i - 1], b[j - 1]])
            Ix[i][j] = max(Mm[i - 1][j] - go, Ix[i - 1][j] - ge, Iy[i - 1][j] - go)
            Iy[i][j] = max(Mm[i][j - 1] - go, Iy[i][j - 1] - ge, Ix[i][j - 1] - go)
    return max(Mm[n][m], Ix[n][m], Iy[n][m])


def onehot(x, A):
    C = np.zeros((len(x), A), np.int64)
    C[np.arange(len(x)), x] = 1
    return C


def test_pairwise_special_case_textbook(oracle_lib):
    from workloads import protein_matrix
    S = protein_matrix()
    rng = np.random.default_rng(21)
    for trial in range(40):
        a = rng.integers(0, 20, int(rng.integers(1, 40)))
        b = rng.integers(0, 20, int(rng.integers(1, 40)))
        go, ge = [(10, 1), (5, 2), (3, 3), (11, 0)][trial % 4]
        _, score = oracle.profile_align(onehot(a, 20), 1, onehot(b, 20), 1, S, go, ge)
        assert score == textbook_gotoh(a, b, S, go, ge)


def test_profile_align_edges(oracle_lib):
    S = np.eye(3, dtype=np.int8) * 2 + 1
    C = np.ones((4, 3), np.int64)
    ops, score = oracle.profile_align(C, 2, np.zeros((0, 3)), 3, S, 4, 1)
    assert ops.tolist() == [X] * 4 and score == -(6 * 4 + 3 * 6)
    ops, score = oracle.profile_align(np.zeros((0, 3)), 1, np.zeros((0, 3)), 1, S, 4, 1)
    assert ops.tolist() == [] and score == 0
    with pytest.raises(oracle.OracleError):
        oracle.profile_align(C, 1, C, 1, S, 1, 2)          # go < ge


def test_golden_alignment_examples(oracle_lib):
    with open(os.path.join(GOLDEN, "align_examples.json")) as f:
        cases = json.load(f)["cases"]
    for cs in cases:
        letters = cs["letters"]
        A = len(letters)
        S = np.array(cs["S"], np.int8)
        a = np.array([letters.index(ch) for ch in cs["x"]])
        b = np.array([letters.index(ch) for ch in cs["y"]])
        ops, score = oracle.profile_align(onehot(a, A), 1, onehot(b, A), 1, S, cs["go"], cs["ge"])
        assert score == cs["score"], cs
        assert "".join("MXY"[o] for o in ops) == cs["ops"], cs


# ----------------------------------------------------------------- consensus

def test_consensus_rule(oracle_lib):
    # n = 4 rows; columns: 3 residues (kept, argmax 2), 2 residues tie 1 vs 0
    # (kept, smallest code), 1 residue (dropped: 2*1 < 4)
    counts = np.array([[0, 1, 2, 0], [1, 1, 0, 0], [0, 0, 0, 1]], np.uint16)
    assert oracle.consensus(counts, 4).tolist() == [2, 0]
    # odd n: 2 of 3 is a majority, 1 of 3 is not
    counts = np.array([[0, 2], [1, 0]], np.uint16)
    assert oracle.consensus(counts, 3).tolist() == [1]
