"""Replays of the captured batched launch and the autotuner.

sad_align_buckets records its device work into a hipGraph after a successful
eager call (batched mode, guide trees built in the launch) and replays it while
the baked-in arguments are unchanged.  Every replay is checked against the
oracle, with eager work of the program (the rank and partition calls, a torch
op, synchronisations) between the replays; the autotuner's choice must not
change any result."""
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
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_0901_2742_amd import binding as B
    from paper_0901_2742_amd import pipeline
    w = CONFIGS["prot2000"]
    s = make_inputs("prot2000")
    ref = oracle.run_pipeline(s.codes, s.offsets, s.alphabet, w.kmer_k, w.p, w.subst(),
                              w.gap_open, w.gap_extend, w.s_max)
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
    prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max,
                   B.SAD_BATCHED_MFMA)
    key, _ = B.sad_kmer_rank(seqs, prm)
    part = B.sad_partition(seqs, key, prm)
    return B, torch, s, w, ref, seqs, prm, part


def check_align(torch, al, ref, s, p):
    torch.cuda.synchronize()
    ra = ref["align"]
    n = s.n
    assert np.array_equal(al["colmap"].cpu().numpy()[:len(s.codes)], ra["colmap"])
    assert np.array_equal(al["width"].cpu().numpy()[:p], ra["width"])
    assert np.array_equal(al["merge_score"].cpu().numpy()[:n], ra["merge_score"])
    assert np.array_equal(al["merge_list"].cpu().numpy()[:2 * n].reshape(-1, 2),
                          ra["merge_list"])
    assert np.array_equal(al["merge_cells"].cpu().numpy()[:n], ra["merge_cells"])
    assert int(al["cells"].cpu().numpy()[0]) == ra["cells"]


def test_graph_replays(setup):
    B, torch, s, w, ref, seqs, prm, part = setup
    out = None
    B.sad_profile_graphs(reset=True)
    for rep in range(6):
        _say(f"case graph replay {rep}")
        # engine timing on for the later calls (timed replays)
        B.sad_profile_enable(rep >= 3)
        # scribble over the outputs so that a replay that wrote nothing fails
        if out is not None:
            for t in out.values():
                if torch.is_tensor(t):
                    t.fill_(-7)
        out = B.sad_align_buckets(seqs, part["bucket_off"], part["members"], prm, out)
        check_align(torch, out, ref, s, w.p)
        # the program's own eager work between replays
        key, _ = B.sad_kmer_rank(seqs, prm)
        torch.cuda.synchronize()
        assert np.array_equal(key.cpu().numpy().view(np.uint64), ref["key"])
        _ = (torch.arange(1 << 20, device="cuda") * 3).sum().item()
    B.sad_profile_enable(False)
    ms, launches = B.sad_profile_read(reset=True)
    assert launches == 3 and ms > 0
    captured, replayed = B.sad_profile_graphs(reset=True)
    # eager, eager + capture, then replays
    assert captured == 1 and replayed == 4


def test_graphs_disabled_same_results(setup, monkeypatch):
    B, torch, s, w, ref, seqs, prm, part = setup
    _say("case graphs disabled")
    monkeypatch.setenv("SAD_GRAPHS", "0")
    al = B.sad_align_buckets(seqs, part["bucket_off"], part["members"], prm)
    check_align(torch, al, ref, s, w.p)


@pytest.mark.parametrize("mfma", [0, 1])
def test_trees_in_launch_large_buckets(setup, monkeypatch, mfma):
    """The guide trees built inside the launch with their pair sums in HBM
    (buckets above the MFMA kernel's LDS limit of 182 members: prot2000 in 8
    buckets of 232-262), with vector-ALU or MFMA column scores; the eager call,
    the one that captures the launch and a replay, each against the oracle."""
    B, torch, s, w, _, seqs, _, _ = setup
    p = 8
    _say(f"case trees in the launch, 8 buckets, mfma={mfma}")
    ref = oracle.run_pipeline(s.codes, s.offsets, s.alphabet, w.kmer_k, p, w.subst(),
                              w.gap_open, w.gap_extend, w.s_max)
    prm = B.Params(w.kmer_k, p, w.subst(), w.gap_open, w.gap_extend, w.s_max,
                   B.SAD_BATCHED_MFMA)
    key, _ = B.sad_kmer_rank(seqs, prm)
    part = B.sad_partition(seqs, key, prm)
    sizes = np.diff(part["bucket_off"].cpu().numpy())
    assert 182 < sizes.max() <= 600
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    monkeypatch.setenv("SAD_SCHEDULE", f"{cus},1,1,1" if mfma else f"{2 * cus},1,0,0")
    B.sad_profile_graphs(reset=True)
    out = None
    for rep in range(3):
        if out is not None:
            for t in out.values():
                if torch.is_tensor(t):
                    t.fill_(-7)
        out = B.sad_align_buckets(seqs, part["bucket_off"], part["members"], prm, out)
        check_align(torch, out, ref, s, p)
    captured, replayed = B.sad_profile_graphs(reset=True)
    assert captured == 1 and replayed == 1


@pytest.mark.parametrize("mode", [1, 0])
def test_autotune_keeps_results(setup, mode):
    B, torch, s, w, ref, seqs, _, part = setup
    _say(f"case autotune mode={mode}")
    prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, mode)
    grid, fuse, coop, mfma, chunk = B.sad_tune(seqs, part["bucket_off"], part["members"], prm)
    assert grid > 0 and chunk in (16, 32)
    al = B.sad_align_buckets(seqs, part["bucket_off"], part["members"], prm)
    check_align(torch, al, ref, s, w.p)
    al = B.sad_align_buckets(seqs, part["bucket_off"], part["members"], prm)
    check_align(torch, al, ref, s, w.p)


def tuner_candidates(torch, mode):
    """The schedules sad_tune measures: batched, a grid of 1, 3/4 or 1/2
    workgroup per CU, the guide trees inside the launch or by a separate
    kernel, cooperative merges on or off, or vector-ALU scores with 1-3
    workgroups per CU and the trees inside the launch or separate; plain, 1-3
    workgroups per CU.  The MFMA schedules with 32-step chunks (the tuner
    times its best one with 16-step chunks as well: here every one of them)."""
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    if mode == 1:
        return ([(cus * den // 4, fuse, coop, 1, chunk) for chunk in (32, 16) for coop in (1, 0)
                 for fuse in (1, 0) for den in (4, 3, 2)] +
                [(cus * per, fuse, 0, 0, 32) for fuse in (1, 0) for per in (1, 2, 3)])
    return [(cus * per, 0, 0, 0, 32) for per in (1, 2, 3)]


@pytest.mark.parametrize("mode", [1, 0])
def test_every_tuner_candidate_matches_the_oracle(setup, monkeypatch, mode):
    """Each schedule the autotuner can pick, imposed with SAD_SCHEDULE, gives
    the oracle's bucket alignment (results never depend on the schedule)."""
    B, torch, s, w, ref, seqs, _, part = setup
    prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, mode)
    out = None
    for grid, fuse, coop, mfma, chunk in tuner_candidates(torch, mode):
        _say(f"case tuner candidate mode={mode} grid={grid} fuse={fuse} coop={coop} mfma={mfma} "
             f"chunk={chunk}")
        monkeypatch.setenv("SAD_SCHEDULE", f"{grid},{fuse},{coop},{mfma},{chunk}")
        if out is not None:
            for t in out.values():
                if torch.is_tensor(t):
                    t.fill_(-7)
        out = B.sad_align_buckets(seqs, part["bucket_off"], part["members"], prm, out)
        check_align(torch, out, ref, s, w.p)


def test_graph_key_follows_kmer_length(setup):
    """A captured launch bakes the k-mer length into its similarity kernels: a
    call with another k on the same buffers must not replay it.  k alternates
    3, 2, 3, 3 (the last call a replay of the re-captured k = 3 launch), each
    call checked against the oracle on the same buckets."""
    B, torch, s, w, ref, seqs, _, part = setup
    boff = part["bucket_off"].cpu().numpy()
    mem = part["members"].cpu().numpy()
    refs = {}
    for k in (3, 2):
        refs[k] = oracle.align_buckets(s.codes, s.offsets, s.alphabet, boff, mem, k, w.subst(),
                                       w.gap_open, w.gap_extend)
    assert not np.array_equal(refs[3]["merge_list"], refs[2]["merge_list"])
    out = None
    B.sad_profile_graphs(reset=True)
    for rep, k in enumerate((3, 3, 2, 3, 3, 2, 2)):
        _say(f"case graph key k={k} call {rep}")
        prm = B.Params(k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, B.SAD_BATCHED_MFMA)
        if out is not None:
            for t in out.values():
                if torch.is_tensor(t):
                    t.fill_(-7)
        out = B.sad_align_buckets(seqs, part["bucket_off"], part["members"], prm, out)
        check_align(torch, out, {"align": refs[k]}, s, w.p)
    captured, replayed = B.sad_profile_graphs(reset=True)
    assert replayed >= 1
