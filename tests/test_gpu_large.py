"""Parity at the large workloads (20000 proteins in 128 buckets, 50000 DNA
sequences in 256, 200000 proteins in 1024), in the launch configuration the
benchmark uses, stage by stage, in both modes:

* rank: the samples of 8 chunks (first and last included) re-derived by the
  oracle from the chunk's own local ranks (Section 2.3.1), and the keys of 256
  sampled sequences recomputed against the library's sample list;
* partition: recomputed by the oracle from the library's keys, all of it;
* bucket alignment: whole buckets re-aligned by the oracle (different ones in
  the two modes), plus properties of every bucket;
* refinement and glue: the oracle's steps 12-15 run on the library's own
  stage-3 alignment, compared in full (GA, ancestor merges, refinement
  scores and cells, glued column map and width);
* plain mode: every output identical to the batched mode's.

The oracle's share of the CPU time is printed per case (about 30 s for the
three refinements and a few seconds for the rest on the machine's host)."""
import sys
import time

import numpy as np
import pytest

import oracle
from workloads import make_inputs, workload

pytestmark = pytest.mark.gpu

_INPUTS = {}
_RESULTS = {}


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


def _inputs(name):
    if name not in _INPUTS:
        _INPUTS[name] = make_inputs(name)
    return _INPUTS[name]


def check_rows(offsets, ids, colmap, width):
    used = np.zeros(width, bool)
    for i in ids:
        c = colmap[offsets[i]:offsets[i + 1]]
        assert (np.diff(c) > 0).all() and c.min() >= 0 and c.max() < width
        used[c] = True
    assert used.all()


def check_samples(s, w, samples, chunks):
    """Section 2.3.1 on one chunk: local ranks over the chunk (self included),
    order by (rank, id), k_s picks at floor(t w / (k_s + 1))."""
    n, p = s.n, w.p
    wmin = min(((c + 1) * n) // p - (c * n) // p for c in range(p))
    ks = min(p - 1, max(1, w.s_max // p), wmin - 1)
    assert len(samples) == p * ks
    for c in chunks:
        lo, hi = (c * n) // p, ((c + 1) * n) // p
        ids = np.arange(lo, hi, dtype=np.int32)
        kl = oracle.rank_against(s.codes, s.offsets, s.alphabet, w.kmer_k, samples=ids, rows=ids)
        order = np.lexsort((ids, kl))
        wc = hi - lo
        exp = [int(ids[order[(t * wc) // (ks + 1)]]) for t in range(1, ks + 1)]
        assert [int(x) for x in samples[c * ks:(c + 1) * ks]] == exp, f"chunk {c}"
    return ks


def _run(hip, name, mode):
    B, pipeline = hip
    s = _inputs(name)
    w = workload(name)
    prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, mode)
    t0 = time.time()
    got = pipeline.run(s.codes, s.offsets, s.alphabet, prm)
    _say(f"  {name} mode {mode}: library pipeline {time.time() - t0:.1f} s (incl. copies)")
    _RESULTS[(name, mode)] = got
    return s, w, got


@pytest.mark.parametrize("name", ["prot20k", "dna50k", "prot200k"])
def test_large_batched_stagewise(hip, name):
    _say(f"case {name} batched")
    s, w, got = _run(hip, name, 1)
    rng = np.random.default_rng(1)
    t_or = time.time()
    # rank: samples of 8 chunks, keys of 256 sequences
    chunks = sorted({0, w.p - 1, *rng.choice(np.arange(1, w.p - 1), 6, replace=False).tolist()})
    ks = check_samples(s, w, got["samples"], chunks)
    rows = np.sort(rng.choice(s.n, 256, replace=False)).astype(np.int32)
    kref = oracle.rank_against(s.codes, s.offsets, s.alphabet, w.kmer_k, samples=got["samples"],
                               rows=rows)
    assert np.array_equal(got["key"][rows], kref)
    # partition of the library's keys, in full
    part = oracle.partition(got["key"], w.p)
    for k in ("pivot_key", "pivot_id", "bucket", "bucket_off", "members"):
        assert np.array_equal(np.asarray(got["part"][k]), part[k]), k
    boff, mem = got["part"]["bucket_off"], got["part"]["members"]
    # bucket alignment: two or three whole buckets
    al = got["align"]
    for b in rng.choice(w.p, 3 if name == "prot20k" else 2, replace=False):
        ids = mem[boff[b]:boff[b + 1]]
        sub = s.subset(ids)
        ra = oracle.align_buckets(sub.codes, sub.offsets, s.alphabet,
                                  np.array([0, len(ids)], np.int32),
                                  np.arange(len(ids), dtype=np.int32), w.kmer_k, w.subst(),
                                  w.gap_open, w.gap_extend)
        gcm = np.concatenate([al["colmap"][s.offsets[i]:s.offsets[i + 1]] for i in ids])
        assert np.array_equal(gcm, ra["colmap"]), f"bucket {b}"
        assert al["width"][b] == ra["width"][0]
        sl = slice(boff[b], boff[b] + len(ids) - 1)
        assert np.array_equal(al["merge_score"][sl], ra["merge_score"][:len(ids) - 1])
        assert np.array_equal(al["merge_list"][sl], ra["merge_list"][:len(ids) - 1])
        assert np.array_equal(al["merge_cells"][sl], ra["merge_cells"][:len(ids) - 1])
    for b in range(w.p):
        ids = mem[boff[b]:boff[b + 1]]
        if len(ids):
            check_rows(s.offsets, ids, al["colmap"], int(al["width"][b]))
    assert al["cells"] == int(al["merge_cells"].sum())
    # refinement and glue: the oracle's steps 12-15 on the library's stage 3
    t_rf = time.time()
    rr = oracle.refine(s.codes, s.offsets, s.alphabet, boff, mem, al["colmap"], al["width"],
                       w.kmer_k, w.subst(), w.gap_open, w.gap_extend)
    t_rf = time.time() - t_rf
    rf = got["refine"]
    assert np.array_equal(rf["ga"], rr["ga"]), "global ancestor"
    assert np.array_equal(rf["merge_list"], rr["merge_list"]), "ancestor merges"
    assert np.array_equal(rf["merge_score"], rr["merge_score"]), "refinement scores"
    assert np.array_equal(rf["merge_cells"], rr["merge_cells"]), "refinement cells"
    assert rf["cells"] == rr["cells"]
    assert rf["width"] == rr["width"], "glued width"
    assert np.array_equal(rf["colmap"], rr["colmap"]), "glued column map"
    check_rows(s.offsets, range(s.n), rf["colmap"], rf["width"])
    _say(f"  {name}: k_s = {ks}, oracle checks {time.time() - t_or:.1f} s "
         f"(refinement {t_rf:.1f} s)")


@pytest.mark.parametrize("name", ["prot20k", "dna50k", "prot200k"])
def test_large_plain_matches(hip, name):
    _say(f"case {name} plain")
    s, w, got = _run(hip, name, 0)
    ref = _RESULTS.get((name, 1))
    if ref is None:
        _, _, ref = _run(hip, name, 1)
    from test_gpu_parity import compare
    compare(got, ref, f"{name} plain vs batched")
    # and two other buckets re-aligned by the oracle in plain mode
    rng = np.random.default_rng(2)
    boff, mem, al = got["part"]["bucket_off"], got["part"]["members"], got["align"]
    for b in rng.choice(w.p, 2, replace=False):
        ids = mem[boff[b]:boff[b + 1]]
        sub = s.subset(ids)
        ra = oracle.align_buckets(sub.codes, sub.offsets, s.alphabet,
                                  np.array([0, len(ids)], np.int32),
                                  np.arange(len(ids), dtype=np.int32), w.kmer_k, w.subst(),
                                  w.gap_open, w.gap_extend)
        gcm = np.concatenate([al["colmap"][s.offsets[i]:s.offsets[i + 1]] for i in ids])
        assert np.array_equal(gcm, ra["colmap"]), f"plain bucket {b}"
    _RESULTS.pop((name, 0), None)
    _RESULTS.pop((name, 1), None)
    _INPUTS.pop(name, None)
