"""Caller-owned workspaces of the four stage calls (through the C-ABI): each
call sized by its sad_*_workspace query and given a torch-allocated block
gives the oracle's results bit for bit; a block that is too small is
SAD_E_CAPACITY with a size that suffices in sad_workspace_needed(); a
misaligned block is SAD_E_INVAL; the library's own workspace (NULL) gives
the same results."""
import sys

import numpy as np
import pytest

import oracle
from workloads import CONFIGS, make_inputs

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


def _ref(name):
    w = CONFIGS[name]
    s = make_inputs(name)
    ref = oracle.run_pipeline(s.codes, s.offsets, s.alphabet, w.kmer_k, w.p, w.subst(),
                              w.gap_open, w.gap_extend, w.s_max)
    return w, s, ref


def _compare(pipeline, res, seqs, p, ref, what):
    from test_gpu_parity import compare
    got = pipeline.to_host(res, seqs.n, p, seqs.total_len)
    compare(got, ref, what)


@pytest.mark.parametrize("mode", [1, 0])
def test_exact_query_sizes_prot2000(hip, mode):
    """Each stage in a block of exactly the queried size (separate blocks)."""
    import torch
    B, pipeline = hip
    _say(f"case workspace prot2000 mode={mode}")
    w, s, ref = _ref("prot2000")
    prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, mode)
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)

    def block(n):
        return torch.empty(n, dtype=torch.uint8, device="cuda")

    n1 = B.sad_kmer_rank_workspace(seqs, prm)
    key, samples = B.sad_kmer_rank(seqs, prm, ws=block(n1))
    n2 = B.sad_partition_workspace(seqs, prm)
    part = B.sad_partition(seqs, key, prm, ws=block(n2))
    n3 = B.sad_align_buckets_workspace(seqs, part["bucket_off"], prm)
    al = B.sad_align_buckets(seqs, part["bucket_off"], part["members"], prm, ws=block(n3))
    n4 = B.sad_refine_workspace(seqs, part["bucket_off"], al, prm)
    rf = B.sad_refine(seqs, part["bucket_off"], part["members"], al, prm, ws=block(n4))
    torch.cuda.synchronize()
    _say(f"  workspace bytes: rank {n1}, partition {n2}, align {n3}, refine {n4}")
    assert 0 < n1 < 64 << 20 and 0 < n2 < 1 << 20
    _compare(pipeline, dict(key=key, samples=samples, part=part, align=al, refine=rf), seqs,
             w.p, ref, f"prot2000 caller workspace mode {mode}")


def test_too_small_and_misaligned(hip):
    import torch
    B, pipeline = hip
    _say("case workspace too small / misaligned")
    w, s, ref = _ref("prot64")
    prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, 1)
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
    # rank: exact size; 512 bytes less is too small and reports the exact size
    n1 = B.sad_kmer_rank_workspace(seqs, prm)
    with pytest.raises(B.SadError) as e:
        B.sad_kmer_rank(seqs, prm, ws=torch.empty(n1 - 512, dtype=torch.uint8, device="cuda"))
    assert e.value.code == B.SAD_E_CAPACITY
    assert B.sad_workspace_needed() == n1
    key, samples = B.sad_kmer_rank(seqs, prm, ws=torch.empty(n1, dtype=torch.uint8,
                                                              device="cuda"))
    big = torch.empty(n1 + 1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(B.SadError) as e:
        B.sad_kmer_rank(seqs, prm, ws=big[1:])
    assert e.value.code == B.SAD_E_INVAL
    part = B.sad_partition(seqs, key, prm, ws="library")
    # alignment: 64 KiB cannot hold the engine; the reported size suffices
    n3 = B.sad_align_buckets_workspace(seqs, part["bucket_off"], prm)
    with pytest.raises(B.SadError) as e:
        B.sad_align_buckets(seqs, part["bucket_off"], part["members"], prm,
                            ws=torch.empty(64 << 10, dtype=torch.uint8, device="cuda"))
    assert e.value.code == B.SAD_E_CAPACITY
    need = B.sad_workspace_needed()
    assert 64 << 10 < need <= n3
    al = B.sad_align_buckets(seqs, part["bucket_off"], part["members"], prm,
                             ws=torch.empty(need, dtype=torch.uint8, device="cuda"))
    # refinement: a block that holds the stage buffers but not the engine
    n4 = B.sad_refine_workspace(seqs, part["bucket_off"], al, prm)
    with pytest.raises(B.SadError) as e:
        B.sad_refine(seqs, part["bucket_off"], part["members"], al, prm,
                     ws=torch.empty(4096, dtype=torch.uint8, device="cuda"))
    assert e.value.code == B.SAD_E_CAPACITY
    assert 4096 < B.sad_workspace_needed() <= n4
    rf = B.sad_refine(seqs, part["bucket_off"], part["members"], al, prm,
                      ws=torch.empty(B.sad_workspace_needed(), dtype=torch.uint8,
                                     device="cuda"))
    torch.cuda.synchronize()
    _compare(pipeline, dict(key=key, samples=samples, part=part, align=al, refine=rf), seqs,
             w.p, ref, "prot64 after capacity retries")


def test_part_of_the_bound_and_library_workspace(hip):
    """The engine's pools take what the block leaves, so an eighth of the
    alignment bound runs prot2000; the library's own workspace agrees."""
    import torch
    B, pipeline = hip
    _say("case workspace eighth of the bound / library")
    w, s, ref = _ref("prot2000")
    prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, 1)
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
    res = pipeline.run_device(seqs, prm, ws="library")
    torch.cuda.synchronize()
    _compare(pipeline, res, seqs, w.p, ref, "prot2000 library workspace")
    part = res["part"]
    n3 = B.sad_align_buckets_workspace(seqs, part["bucket_off"], prm)
    al = B.sad_align_buckets(seqs, part["bucket_off"], part["members"], prm,
                             ws=torch.empty(n3 // 8 // 256 * 256, dtype=torch.uint8,
                                            device="cuda"))
    torch.cuda.synchronize()
    got = al["colmap"][:seqs.total_len].cpu().numpy()
    assert np.array_equal(got, ref["align"]["colmap"])
    assert np.array_equal(al["width"][:w.p].cpu().numpy(), ref["align"]["width"])
