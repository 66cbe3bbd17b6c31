"""Parity of the HIP library (through the C-ABI) with the CPU oracle.

Every output is integer, so the bar is bit-exact: rank keys, samples, pivots,
buckets, per-merge scores/cells/merge lists, column maps, widths, the global
ancestor and the glued column map.  Inputs are the seeded workloads (full size
for the two smaller ones) plus small edge cases (p = 1, empty buckets,
DNA with k = 8, tiny buckets)."""
import os
import sys

import numpy as np
import pytest

import oracle
from workloads import CONFIGS, dna_matrix, generate, make_inputs, protein_matrix

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


def compare(got, ref, what=""):
    assert np.array_equal(got["key"], ref["key"]), f"{what}: keys"
    assert np.array_equal(got["samples"], ref["samples"]), f"{what}: samples"
    for k in ("pivot_key", "pivot_id", "bucket", "bucket_off", "members"):
        assert np.array_equal(np.asarray(got["part"][k]), np.asarray(ref["part"][k])), f"{what}: {k}"
    boff = ref["part"]["bucket_off"]
    ga, ra = got["align"], ref["align"]
    assert np.array_equal(ga["width"], ra["width"]), f"{what}: widths"
    p = len(boff) - 1
    for b in range(p):
        lo, nb = boff[b], boff[b + 1] - boff[b]
        sl = slice(lo, lo + max(nb - 1, 0))
        assert np.array_equal(ga["merge_list"][sl], ra["merge_list"][sl]), f"{what}: merges {b}"
        assert np.array_equal(ga["merge_score"][sl], ra["merge_score"][sl]), f"{what}: scores {b}"
        assert np.array_equal(ga["merge_cells"][sl], ra["merge_cells"][sl]), f"{what}: cells {b}"
    assert ga["cells"] == ra["cells"], f"{what}: total cells"
    assert np.array_equal(ga["colmap"], ra["colmap"]), f"{what}: bucket column maps"
    gr, rr = got["refine"], ref["refine"]
    assert np.array_equal(gr["ga"], rr["ga"]), f"{what}: global ancestor"
    assert np.array_equal(gr["merge_list"], rr["merge_list"]), f"{what}: ancestor merges"
    assert np.array_equal(gr["merge_score"], rr["merge_score"]), f"{what}: refine scores"
    assert np.array_equal(gr["merge_cells"], rr["merge_cells"]), f"{what}: refine cells"
    assert gr["cells"] == rr["cells"]
    assert gr["width"] == rr["width"], f"{what}: glued width"
    assert np.array_equal(gr["colmap"], rr["colmap"]), f"{what}: glued column map"


def run_both(B, pipeline, s, k, p, S, go, ge, mode, s_max=1024):
    prm = B.Params(k, p, S, go, ge, s_max, mode)
    got = pipeline.run(s.codes, s.offsets, s.alphabet, prm)
    ref = oracle.run_pipeline(s.codes, s.offsets, s.alphabet, k, p, S, go, ge, s_max)
    return got, ref


@pytest.mark.parametrize("mode", [0, 1])
def test_prot64_full(hip, mode):
    B, pipeline = hip
    w = CONFIGS["prot64"]
    _say(f"case prot64 mode={mode}")
    s = make_inputs("prot64")
    got, ref = run_both(B, pipeline, s, w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, mode)
    compare(got, ref, "prot64")


@pytest.mark.parametrize("sched", ["0,0,1,1", "0,0,0,0", "0,0,1,1,16", "0,1,1,1,16"])
@pytest.mark.parametrize("p", [3, 15])
def test_small_sets_separate_trees(hip, monkeypatch, p, sched):
    """Guide trees by the separate kernel (the ready merges ordered on the
    device), MFMA or vector-ALU scores, on 30 proteins in 3 buckets and in 15
    (two of them of a single member, so without merges); the MFMA strips also
    in 16-step chunks, with separate trees and with the trees in the launch."""
    B, pipeline = hip
    _say(f"case small protein p={p} schedule {sched}")
    monkeypatch.setenv("SAD_SCHEDULE", sched)
    s = generate(4245, 30, 20, 3, {"kind": "fixed", "value": 70}, 0.15, 0.04, 3)
    got, ref = run_both(B, pipeline, s, 3, p, protein_matrix(), 10, 1, 1)
    compare(got, ref, f"p={p} {sched}")


@pytest.mark.parametrize("p", [1, 2, 3, 7])
def test_small_protein_sets(hip, p):
    B, pipeline = hip
    _say(f"case small protein p={p}")
    s = generate(4242 + p, 30, 20, 3, {"kind": "fixed", "value": 70}, 0.15, 0.04, 3)
    got, ref = run_both(B, pipeline, s, 3, p, protein_matrix(), 10, 1, 1)
    compare(got, ref, f"p={p}")


@pytest.mark.parametrize("sched", [None, "0,-1,1,1,16"])
def test_small_dna_k8(hip, monkeypatch, sched):
    B, pipeline = hip
    _say(f"case small dna k=8 schedule {sched}")
    if sched:
        monkeypatch.setenv("SAD_SCHEDULE", sched)
    s = generate(808, 40, 4, 4, {"kind": "uniform_int", "lo": 90, "hi": 140}, 0.05, 0.01, 8)
    got, ref = run_both(B, pipeline, s, 8, 4, dna_matrix(), 5, 2, 1)
    compare(got, ref, "dna")


@pytest.mark.parametrize("sched", [None, "0,-1,1,1,16", "0,-1,0,1,16"])
def test_long_sequences_multi_strip(hip, monkeypatch, sched):
    """Profiles wider than several 64-row strips and the 256-column ring; the
    MFMA strips also in 16-step chunks, with and without cooperative merges."""
    B, pipeline = hip
    _say(f"case long sequences schedule {sched}")
    if sched:
        monkeypatch.setenv("SAD_SCHEDULE", sched)
    s = generate(31, 12, 20, 2, {"kind": "fixed", "value": 700}, 0.1, 0.02, 3)
    got, ref = run_both(B, pipeline, s, 3, 2, protein_matrix(), 10, 1, 1)
    compare(got, ref, "long")


@pytest.mark.parametrize("sched", [None, "0,-1,1,1,16"])
def test_gap_models(hip, monkeypatch, sched):
    """o == e and free extension: many tied optima exercise the tie rule."""
    B, pipeline = hip
    if sched:
        monkeypatch.setenv("SAD_SCHEDULE", sched)
    s = generate(77, 16, 20, 2, {"kind": "fixed", "value": 50}, 0.3, 0.05, 3)
    for go, ge in [(3, 3), (6, 0), (0, 0)]:
        _say(f"case gaps {go}/{ge} schedule {sched}")
        got, ref = run_both(B, pipeline, s, 3, 2, protein_matrix(), go, ge, 1)
        compare(got, ref, f"gaps {go}/{ge}")


@pytest.mark.parametrize("mode", [1, 0])
@pytest.mark.parametrize("alphabet", [20, 4])
def test_wide_dp(hip, mode, alphabet):
    """Merges whose static bound (W1 + W2 + 2) n1 n2 max(|S|, go) reaches 2^29
    run the 64-bit DP; a large gap-open cost gets there with small inputs."""
    B, pipeline = hip
    _say(f"case wide dp mode={mode} A={alphabet}")
    k = 3 if alphabet == 20 else 6
    S = protein_matrix() if alphabet == 20 else dna_matrix()
    s = generate(2027 + alphabet, 80, alphabet, 2, {"kind": "uniform_int", "lo": 90, "hi": 130},
                 0.1, 0.02, k)
    go, ge = 3000, 1
    top = 40 * 40 * 2 * 130 * go
    assert top >= 1 << 29
    got, ref = run_both(B, pipeline, s, k, 1, S, go, ge, mode)
    compare(got, ref, f"wide A={alphabet} mode {mode}")


@pytest.mark.parametrize("mode", [1, 0])
def test_large_bucket(hip, mode):
    """One bucket of 700 members: guide tree beyond the 64-bit cross-product
    range (128-bit comparisons), built outside the engine launch, and merges
    near the root whose bound (W1 + W2 + 2) n1 n2 go passes 2^29 (64-bit DP,
    64-bit strip boundary rows) from the first engine attempt."""
    B, pipeline = hip
    _say(f"case large bucket mode={mode}")
    s = generate(6007, 700, 20, 2, {"kind": "uniform_int", "lo": 24, "hi": 40}, 0.1, 0.02, 3)
    got, ref = run_both(B, pipeline, s, 3, 1, protein_matrix(), 40, 2, mode)
    compare(got, ref, f"large bucket mode {mode}")


def test_bucket_of_4200(hip):
    """One bucket of 4200 short DNA sequences (p = 1): a guide tree above 4096
    members, whose clusters keep their best pair sums in HBM rather than LDS,
    and 4199 progressive merges, all bit-exact.  The oracle's pair scans run
    on up to 16 host threads (about 20-40 s)."""
    B, pipeline = hip
    _say("case bucket of 4200")
    s = generate(7331, 4200, 4, 6, {"kind": "uniform_int", "lo": 20, "hi": 32}, 0.1, 0.02, 4)
    oracle.set_threads(min(16, os.cpu_count() or 1))
    try:
        got, ref = run_both(B, pipeline, s, 4, 1, dna_matrix(), 6, 1, 1)
    finally:
        oracle.set_threads(1)
    compare(got, ref, "bucket of 4200")


@pytest.mark.parametrize("mode", [1, 0])
def test_prot2000_full(hip, mode):
    # mode 1: one persistent launch over all trees, MFMA tile scores;
    # mode 0: one launch per tree level, VALU column scores
    B, pipeline = hip
    w = CONFIGS["prot2000"]
    _say(f"case prot2000 mode={mode}")
    s = make_inputs("prot2000")
    got, ref = run_both(B, pipeline, s, w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, mode)
    compare(got, ref, f"prot2000 mode {mode}")


def test_repeat_runs_identical(hip):
    B, pipeline = hip
    _say("case determinism")
    w = CONFIGS["prot64"]
    s = make_inputs("prot64")
    prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, 1)
    a = pipeline.run(s.codes, s.offsets, s.alphabet, prm)
    b = pipeline.run(s.codes, s.offsets, s.alphabet, prm)
    assert np.array_equal(a["refine"]["colmap"], b["refine"]["colmap"])
    assert np.array_equal(a["align"]["merge_score"], b["align"]["merge_score"])


def test_error_paths(hip):
    B, pipeline = hip
    _say("case error paths")
    s = make_inputs("prot64")
    seqs = pipeline.to_device(s.codes, s.offsets, 20)
    with pytest.raises(B.SadError) as e:
        B.sad_kmer_rank(seqs, B.Params(3, 40, protein_matrix(), 10, 1))   # N < 2p
    assert e.value.code == B.SAD_E_INVAL
    bad = s.codes.copy()
    bad[5] = 25
    seqs_bad = pipeline.to_device(bad, s.offsets, 20)
    with pytest.raises(B.SadError) as e:
        B.sad_kmer_rank(seqs_bad, B.Params(3, 4, protein_matrix(), 10, 1))
    assert e.value.code == B.SAD_E_INVAL
    with pytest.raises(B.SadError) as e:
        B.sad_kmer_rank(seqs, B.Params(4, 4, protein_matrix(), 10, 1))    # 20^4 > 2^16
    assert e.value.code == B.SAD_E_INVAL


def test_prot2000_extreme_bucket_counts(hip):
    """The bucket-count sweep's extremes, bit-exact in full: p = 1 (one bucket
    of 2000 proteins, its guide tree by the standalone kernel) and p = 256
    (buckets of about 8, k_s = 4 samples per chunk, 256 ancestors)."""
    from concurrent.futures import ThreadPoolExecutor
    B, pipeline = hip
    w = CONFIGS["prot2000"]
    s = make_inputs("prot2000")

    def ref(p):   # the oracle's C code runs outside the interpreter lock
        return oracle.run_pipeline(s.codes, s.offsets, s.alphabet, w.kmer_k, p, w.subst(),
                                   w.gap_open, w.gap_extend, w.s_max)

    with ThreadPoolExecutor(2) as ex:
        refs = dict(zip((1, 256), ex.map(ref, (1, 256))))
    for p in (1, 256):
        for mode in (1, 0):
            _say(f"case prot2000 p={p} mode={mode}")
            prm = B.Params(w.kmer_k, p, w.subst(), w.gap_open, w.gap_extend, w.s_max, mode)
            got = pipeline.run(s.codes, s.offsets, s.alphabet, prm)
            compare(got, refs[p], f"prot2000 p={p} mode={mode}")


@pytest.mark.parametrize("alphabet", [4, 20])
def test_repeat_rich_sequences(hip, alphabet):
    """Sequences with k-mers repeated more than 15 times (homopolymer and
    short tandem-repeat runs) next to ordinary ones: the pair kernels' row
    groups that hold such a row take the one-row path with full 16-bit
    counts; keys, samples, buckets and the bucket similarity matrices (through
    the guide trees and alignments) must still be the oracle's."""
    from workloads.synth import SeqSet
    B, pipeline = hip
    _say(f"case repeat-rich A={alphabet}")
    k = 8 if alphabet == 4 else 3
    s = generate(1500 + alphabet, 48, alphabet, 3, {"kind": "uniform_int", "lo": 90, "hi": 140},
                 0.1, 0.02, k)
    rng = np.random.default_rng(alphabet)
    codes = [s.codes[s.offsets[i]:s.offsets[i + 1]].copy() for i in range(s.n)]
    for t, i in enumerate(rng.choice(s.n, 9, replace=False)):
        x = codes[i]
        at = int(rng.integers(0, len(x) - 40))
        if t % 3 == 0:
            x[at:at + 40] = 0                                  # homopolymer: one k-mer 40 - k + 1 times
        elif t % 3 == 1:
            x[at:at + 40] = np.tile(np.array([1, 2], np.uint8), 20)   # period-2 repeat
        else:
            x[at:at + 40] = np.tile(np.array([3, 1, 2], np.uint8), 14)[:40]
    offs = np.zeros(s.n + 1, np.int64)
    offs[1:] = np.cumsum([len(x) for x in codes])
    rs = SeqSet(alphabet, np.concatenate(codes).astype(np.uint8), offs, s.family, s.homology)
    S = dna_matrix() if alphabet == 4 else protein_matrix()
    for mode in (1, 0):
        got, ref = run_both(B, pipeline, rs, k, 4, S, 10, 1, mode)
        compare(got, ref, f"repeat-rich A={alphabet} mode {mode}")
