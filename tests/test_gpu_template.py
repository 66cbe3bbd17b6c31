"""Parity of sad_refine_template with the ancestors' alignment as a q-row
template (SAD_TEMPLATE_GA_MSA) against the oracle, bit-exact on every
output, through the C-ABI."""
import sys

import numpy as np
import pytest

import oracle
from workloads import CONFIGS, dna_matrix, generate, make_inputs, protein_matrix
from test_gpu_parity import compare

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


def run_both(B, pipeline, s, k, p, S, go, ge, mode, s_max=1024):
    prm = B.Params(k, p, S, go, ge, s_max, mode)
    got = pipeline.run(s.codes, s.offsets, s.alphabet, prm, template="ga_msa")
    ref = oracle.run_pipeline(s.codes, s.offsets, s.alphabet, k, p, S, go, ge, s_max,
                              template="ga_msa")
    return got, ref


@pytest.mark.parametrize("mode", [1, 0])
@pytest.mark.parametrize("name", ["prot64", "prot2000"])
def test_msa_template_workloads(hip, name, mode):
    B, pipeline = hip
    w = CONFIGS[name]
    _say(f"case msa template {name} mode={mode}")
    s = make_inputs(name)
    got, ref = run_both(B, pipeline, s, w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, mode)
    compare(got, ref, f"msa template {name} mode {mode}")


@pytest.mark.parametrize("p", [1, 3, 7])
def test_msa_template_small(hip, p):
    B, pipeline = hip
    _say(f"case msa template small p={p}")
    s = generate(4100 + p, 40, 20, 3, {"kind": "uniform_int", "lo": 30, "hi": 90}, 0.15, 0.03, 3)
    got, ref = run_both(B, pipeline, s, 3, p, protein_matrix(), 10, 1, 1)
    compare(got, ref, f"msa template p={p}")
    d = generate(4200 + p, 48, 4, 3, {"kind": "uniform_int", "lo": 60, "hi": 120}, 0.05, 0.01, 8)
    got, ref = run_both(B, pipeline, d, 8, p, dna_matrix(), 5, 2, 1)
    compare(got, ref, f"msa template dna p={p}")


def test_msa_template_wide_refinement(hip):
    """G = n_b q with a large gap-open cost: the refinement alignments run the
    64-bit DP."""
    B, pipeline = hip
    _say("case msa template wide refinement")
    s = generate(4300, 80, 20, 2, {"kind": "uniform_int", "lo": 90, "hi": 130}, 0.1, 0.02, 3)
    got, ref = run_both(B, pipeline, s, 3, 8, protein_matrix(), 30000, 1, 1)
    compare(got, ref, "msa template wide")


def test_msa_template_bad_kind(hip):
    B, pipeline = hip
    import ctypes
    _say("case msa template errors")
    s = make_inputs("prot64")
    w = CONFIGS["prot64"]
    prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, 1)
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
    res = pipeline.run_device(seqs, prm)
    out = res["refine"]
    sst, pp = seqs.c_struct(), prm.c_struct()
    mb, mg = B._msa_struct(res["align"]), B._msa_struct(out)
    gl, nst = ctypes.c_int32(0), ctypes.c_int32(0)
    code = B.lib().sad_refine_template(ctypes.byref(sst), B._ptr(res["part"]["bucket_off"]),
                                       B._ptr(res["part"]["members"]), ctypes.byref(mb),
                                       ctypes.byref(pp), 7, B._ptr(out["ga"]), out["ga"].numel(),
                                       ctypes.byref(gl), ctypes.byref(mg), ctypes.byref(nst),
                                       None, 0, B._stream())
    assert code == B.SAD_E_INVAL
