"""Parity of sad_refine_tree (tree-dependent refinement of the glued
alignment) with the oracle: the refined column map, width, step count,
accepted steps and every step's (node, present score, new score), bit-exact,
through the C-ABI."""
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
    return B, pipeline, torch


def run_case(B, pipeline, torch, s, k, p, S, go, ge, mode, passes, template="ga"):
    prm = B.Params(k, p, S, go, ge, 1024, mode)
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
    res = pipeline.run_device(seqs, prm, template=template)
    cap = passes * 2 * p
    cm, W, steps, acc, rec = B.sad_refine_tree(seqs, res["part"]["bucket_off"],
                                               res["part"]["members"], res["refine"], prm,
                                               passes, cap)
    torch.cuda.synchronize()
    # the oracle refines its own glued alignment (no oracle input comes from
    # the library)
    r0 = oracle.run_pipeline(s.codes, s.offsets, s.alphabet, k, p, S, go, ge, template=template)
    boff, mem = r0["part"]["bucket_off"], r0["part"]["members"]
    q = int((np.diff(boff) > 0).sum())
    ref = oracle.refine_tree(s.codes, s.offsets, s.alphabet, boff, mem, r0["refine"]["colmap"],
                             r0["refine"]["width"], r0["refine"]["merge_list"][:max(q - 1, 0)],
                             k, S, go, ge, passes)
    assert steps == ref["steps"] and acc == ref["accepted"]
    assert np.array_equal(rec[:, 0], ref["rec_node"])
    assert np.array_equal(rec[:, 1], ref["rec_old"]) and np.array_equal(rec[:, 2], ref["rec_new"])
    assert W == ref["width"]
    assert np.array_equal(cm.cpu().numpy(), ref["colmap"])
    return steps, acc


@pytest.mark.parametrize("mode", [1, 0])
def test_tree_refine_prot2000(hip, mode):
    B, pipeline, torch = hip
    w = CONFIGS["prot2000"]
    _say(f"case tree refine prot2000 mode={mode}")
    steps, acc = run_case(B, pipeline, torch, make_inputs("prot2000"), w.kmer_k, w.p, w.subst(),
                          w.gap_open, w.gap_extend, mode, 1)
    assert steps == 29 and acc > 0


@pytest.mark.parametrize("p", [1, 2, 5])
def test_tree_refine_small(hip, p):
    B, pipeline, torch = hip
    _say(f"case tree refine small p={p}")
    s = generate(5100 + p, 60, 20, 3, {"kind": "uniform_int", "lo": 40, "hi": 70}, 0.2, 0.04, 3)
    run_case(B, pipeline, torch, s, 3, p, protein_matrix(), 10, 1, 1, 6)
    d = generate(5200 + p, 50, 4, 3, {"kind": "uniform_int", "lo": 60, "hi": 100}, 0.08, 0.02, 6)
    run_case(B, pipeline, torch, d, 6, p, dna_matrix(), 5, 2, 1, 3, template="ga_msa")


def test_tree_refine_errors(hip):
    B, pipeline, torch = hip
    _say("case tree refine errors")
    s = make_inputs("prot64")
    w = CONFIGS["prot64"]
    prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, 1)
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
    res = pipeline.run_device(seqs, prm)
    bad = dict(res["refine"])
    ml = bad["merge_list"].clone()
    ml[0] = ml[1]  # a node merged with itself: not a tree
    bad["merge_list"] = ml
    with pytest.raises(B.SadError) as e:
        B.sad_refine_tree(seqs, res["part"]["bucket_off"], res["part"]["members"], bad, prm, 1)
    assert e.value.code == B.SAD_E_INVAL
    with pytest.raises(B.SadError):
        B.sad_refine_tree(seqs, res["part"]["bucket_off"], res["part"]["members"], res["refine"],
                          prm, -1)
    # zero passes: the alignment comes back unchanged
    cm, W, steps, acc, _ = B.sad_refine_tree(seqs, res["part"]["bucket_off"],
                                             res["part"]["members"], res["refine"], prm, 0)
    assert steps == 0 and acc == 0 and W == int(res["refine"]["width"][0].item())
    assert torch.equal(cm, res["refine"]["colmap"][:seqs.total_len])
