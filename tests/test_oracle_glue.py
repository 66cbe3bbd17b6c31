"""Pins of the oracle's glue (Section 2.3.3, step 15 of the algorithm box)
and of the one-row global ancestor (steps 12-13).

The glue is checked three ways: hand-worked op strings with their laid-out
result (tests/golden/glue_examples.json); an independent Python re-run that
builds the joined alignment as an explicit list of columns from the
refinement op strings the oracle recorded; and whole refinements with 2-4
buckets (one of them empty) compared with that re-run.  GA is checked against
the majority consensus of the ancestors' alignment rebuilt from its recorded
merges, and each refinement score against exhaustive enumeration with GA as a
one-row profile."""
import json
import os

import numpy as np
import pytest

import oracle
from workloads import dna_matrix, generate, protein_matrix
from test_oracle_align import alignment_score, brute_best
from test_oracle_pipeline import check_rows, replay_bucket
from test_oracle_template import profile_of

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
CODE = {"M": 0, "X": 1, "Y": 2}


def glue_columns(tmpl_width, ops_list, widths):
    """The joined alignment as a list of columns, each a dict bucket -> bucket
    column: for every template position the inserts of its slot (sorted by
    bucket, then by column), then the shared column; the trailing slot last;
    empty columns removed."""
    slots = [[] for _ in range(tmpl_width + 1)]
    shared = [{} for _ in range(tmpl_width)]
    for u, ops in enumerate(ops_list):
        i = j = 0
        for o in ops:
            if o == CODE["X"]:
                slots[j].append((u, i))
                i += 1
            elif o == CODE["M"]:
                shared[j][u] = i
                i += 1
                j += 1
            else:
                j += 1
        assert i == widths[u] and j == tmpl_width
    columns = []
    for j in range(tmpl_width + 1):
        columns.extend({u: c} for u, c in sorted(slots[j]))
        if j < tmpl_width:
            columns.append(shared[j])
    columns = [c for c in columns if c]
    to_g = [np.full(w, -1, np.int64) for w in widths]
    for g, col in enumerate(columns):
        for u, c in col.items():
            to_g[u][c] = g
    assert all((t >= 0).all() for t in to_g)
    return to_g, len(columns)


def majority_consensus(C, n):
    """Column kept iff at least half the rows hold a residue there; its residue
    is the most frequent one, the smallest code among equals."""
    keep = 2 * C.sum(axis=1) >= n
    return np.argmax(C[keep], axis=1).astype(np.uint8)


def load_cases():
    with open(os.path.join(GOLDEN, "glue_examples.json")) as fh:
        return json.load(fh)["cases"]


@pytest.mark.parametrize("case", load_cases(), ids=lambda c: c["name"][:40])
def test_golden_glue(oracle_lib, case):
    ops = [np.array([CODE[ch] for ch in s], np.uint8) for s in case["ops"]]
    got, width = oracle.glue(case["tmpl_width"], ops, case["widths"])
    assert width == case["width"]
    for u, exp in enumerate(case["to_g"]):
        assert got[u].tolist() == exp
    # the independent re-run agrees with the hand-worked layout too
    ref, wref = glue_columns(case["tmpl_width"], ops, case["widths"])
    assert wref == case["width"]
    assert all(r.tolist() == e for r, e in zip(ref, case["to_g"]))


def test_glue_rejects_ops_that_do_not_span(oracle_lib):
    ops = [np.array([0, 1], np.uint8)]
    with pytest.raises(oracle.OracleError):
        oracle.glue(2, ops, [2])


def random_buckets(seed, p, empty=None, A=20):
    """Tiny family-structured sequences cut into p contiguous buckets (bucket
    `empty` left without members)."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(2 * p + 2, 4 * p + 4))
    s = generate(seed, n, A, 2, {"kind": "fixed", "value": int(rng.integers(8, 16))},
                 0.2, 0.06, 3 if A == 20 else 4)
    sizes = np.ones(p, np.int64)
    if empty is not None:
        sizes[empty] = 0
    rest = n - int(sizes.sum())
    for t in rng.integers(0, p, rest):
        if t != empty:
            sizes[t] += 1
        else:
            sizes[(t + 1) % p] += 1
    boff = np.zeros(p + 1, np.int32)
    boff[1:] = np.cumsum(sizes)
    mem = rng.permutation(n).astype(np.int32)
    for b in range(p):
        mem[boff[b]:boff[b + 1]].sort()
    return s, boff, mem


@pytest.mark.parametrize("seed,p,empty,template",
                         [(1, 2, None, "ga"), (2, 3, None, "ga"), (3, 4, 1, "ga"),
                          (4, 4, None, "ga"), (5, 3, 0, "ga"), (6, 4, 3, "ga"),
                          (7, 3, None, "ga_msa"), (8, 4, 2, "ga_msa")])
def test_refine_glue_matches_rerun(oracle_lib, seed, p, empty, template):
    A = 20
    s, boff, mem = random_buckets(100 + seed, p, empty, A)
    S = protein_matrix()
    al = oracle.align_buckets(s.codes, s.offsets, A, boff, mem, 3, S, 10, 1)
    rf = oracle.refine(s.codes, s.offsets, A, boff, mem, al["colmap"], al["width"], 3, S, 10, 1,
                       template=template, want_ops=True)
    nonempty = [b for b in range(p) if boff[b + 1] > boff[b]]
    widths = [int(al["width"][b]) for b in nonempty]
    assert len(rf["ops"]) == len(nonempty)
    # every op string scores what the refinement step reported
    q = len(nonempty)
    to_g, width = glue_columns(rf["tmpl_width"], rf["ops"], widths)
    assert rf["width"] == width
    exp = np.full(len(s.codes), -1, np.int64)
    for u, b in enumerate(nonempty):
        for i in mem[boff[b]:boff[b + 1]]:
            r = np.arange(s.offsets[i], s.offsets[i + 1])
            exp[r] = to_g[u][al["colmap"][r]]
    assert np.array_equal(exp, rf["colmap"])
    check_rows(s.codes, s.offsets, range(s.n), rf["colmap"], rf["width"])
    assert len(rf["merge_score"]) == 2 * q - 1


@pytest.mark.parametrize("seed", range(5))
def test_ga_is_consensus_of_ancestor_alignment(oracle_lib, seed):
    """GA (the default template) is the majority consensus of the ancestors'
    alignment, which is rebuilt from the recorded ancestor merges; every
    refinement step's score is the enumerated optimum against GA as one row,
    and its recorded op string attains it."""
    rng = np.random.default_rng(700 + seed)
    A, k, S, go, ge = 4, 2, dna_matrix(), 3, 1
    q = int(rng.integers(2, 5))
    n = 2 * q
    lens = rng.integers(3, 7, n)
    offsets = np.zeros(n + 1, np.int64)
    offsets[1:] = np.cumsum(lens)
    codes = rng.integers(0, A, int(offsets[-1])).astype(np.uint8)
    boff = (np.arange(q + 1) * 2).astype(np.int32)
    mem = np.arange(n, dtype=np.int32)
    al = oracle.align_buckets(codes, offsets, A, boff, mem, k, S, go, ge)
    rf = oracle.refine(codes, offsets, A, boff, mem, al["colmap"], al["width"], k, S, go, ge,
                       want_ops=True)
    profs, ancs = [], []
    for b in range(q):
        ids = mem[boff[b]:boff[b + 1]]
        C = profile_of(codes, offsets, ids, al["colmap"], int(al["width"][b]), A)
        profs.append((C, len(ids)))
        ancs.append(majority_consensus(C, len(ids)))
    if len({a.tobytes() for a in ancs}) < 2:
        pytest.skip("ancestors coincide for this seed")
    aoff = np.zeros(q + 1, np.int64)
    aoff[1:] = np.cumsum([len(a) for a in ancs])
    acodes = np.concatenate(ancs).astype(np.uint8)
    one = np.array([0, q], np.int32)
    amem = np.arange(q, dtype=np.int32)
    aal = oracle.align_buckets(acodes, aoff, A, one, amem, k, S, go, ge, want_ops=True)
    assert np.array_equal(aal["merge_list"][:q - 1], rf["merge_list"][:q - 1])
    (T, tn), _ = replay_bucket(acodes, aoff, amem, A, S, go, ge, aal["merge_list"][:q - 1],
                               aal["merge_score"][:q - 1], aal["ops"], aal["ops_off"], 0)
    assert tn == q
    ga = majority_consensus(T, q)
    assert np.array_equal(rf["ga"], ga)
    assert rf["tmpl_width"] == len(ga)
    G1 = np.eye(A, dtype=np.int64)[ga]
    for u in range(q):
        C, nb = profs[u]
        best, _ = brute_best(C, nb, G1, 1, S, go, ge)
        assert rf["merge_score"][q - 1 + u] == best
        sc = C @ S.astype(np.int64) @ G1.T
        assert alignment_score(rf["ops"][u], sc, nb * go, nb * ge) == best
