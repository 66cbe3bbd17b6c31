#!/usr/bin/env python3
"""Benchmark of the Sample-Align-D data-parallel core on one MI355X.

One step = one pass of the whole path (k-mer rank, partition, per-bucket
alignment, ancestor refinement + glue) over the 2000-protein workload
(8 families x 250, mean root length 316, 16 buckets, k = 3, gaps 10/1), with
the inputs already resident in HBM.  Prints one JSON line:
  value      alignment GCUPS = DP cells of all alignment steps / step time
  seq_per_s  sequences aligned per second (same step time)
  roofline   the alignment engine kernel (DP + traceback + merge) against the
             int32 vector-ALU peak, timed with HIP events on its own stream
  cpu_baseline  the CPU oracle on the same workload (all host threads; one
             thread beside it), or on a bounded sample of it when the main
             workload is one of the large ones
  workloads  the other workloads (64 proteins, 20000 proteins, 50000 DNA
             sequences, 200000 proteins): batched and plain pass times,
             GCUPS, the engine's roofline, the oracle on a sample
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "alignment GCUPS + sequences/s at 2000×316 aa, batched+MFMA vs plain, bit-exact"
# int32 vector ALU peak: 256 CUs x 64 lanes x 2.4 GHz
INT32_PEAK_TOPS = 256 * 64 * 2.4e9 / 1e12
# algorithmic int32 operations per DP cell: M (1 add), X and Y (2 subtractions
# + 1 max each), H (2 max), tie information (2 for H's op code, 4 for the X/Y
# open/extend flags)
OPS_PER_CELL = 14


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="prot2000")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-tune", action="store_true",
                    help="time the default schedule without autotuning first (profiling runs)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the q-row template and tree-refinement figures (profiling runs)")
    ap.add_argument("--sweep-p", default="", metavar="P1,P2,...",
                    help="instead of the benchmark line, one line per bucket count p: step time "
                         "and alignment quality (Q) of the pipeline on the workload")
    ap.add_argument("--template", default="ga", choices=("ga", "ga_msa"),
                    help="refinement template of --sweep-p runs (the benchmark line times "
                         "\"ga\" and reports \"ga_msa\" beside it)")
    ap.add_argument("--rank-study", default="", metavar="N1,N2,...",
                    help="instead of the benchmark line, one line per set size N: the "
                         "centralised rank (all N as the sample) against the globalised rank "
                         "(p (p - 1) samples at most), their statistics and histograms")
    ap.add_argument("--rank-p", type=int, default=16,
                    help="bucket count p of the globalised rank in --rank-study")
    ap.add_argument("--workloads", default="prot64,prot20k,dna50k,prot200k",
                    help="other workloads timed beside the benchmark line (batched and plain "
                         "pass times, GCUPS, engine roofline, the oracle on a sample); "
                         "empty to skip")
    ap.add_argument("--workload-steps", type=int, default=3)
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the timed steps, copy a buffer of this many MiB once (a kernel "
                         "of known traffic for scaling hardware byte counters)")
    return ap.parse_args()


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "engine_kernel_traffic_prot2000.txt")


def engine_source_digest() -> str:
    """Digest of the engine kernel's sources: a measured traffic figure is only
    reported while the kernel is the one it was measured on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_0901_2742_amd", "csrc")
    for f in ("engine.hip", "upgma_core.h", "sad_internal.h"):
        with open(os.path.join(csrc, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str):
    """HBM bytes per engine launch from the committed counter summary (FETCH_SIZE
    + WRITE_SIZE, each scaled by the copy-kernel calibration), or None."""
    if workload != "prot2000" or not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    with open(TRAFFIC_FILE) as fh:
        for line in fh:
            if "=" in line and not line.startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    if vals.get("engine_source_digest") != engine_source_digest():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def timed_steps(run, seqs, prm, steps, warmup, B, torch, template="ga"):
    bufs = {}  # output buffers kept across passes, as a serving loop would
    for _ in range(warmup):
        run(seqs, prm, bufs, template=template)
    torch.cuda.synchronize()
    B.sad_profile_read(reset=True)
    B.sad_profile_enable(True)
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record(stream)
    res = None
    for _ in range(steps):
        res = run(seqs, prm, bufs, template=template)
    t1.record(stream)
    torch.cuda.synchronize()
    B.sad_profile_enable(False)
    eng_ms, launches = B.sad_profile_read(reset=True)
    return res, t0.elapsed_time(t1) / steps, eng_ms, launches


def extras(out, args, B, pipeline, torch, seqs, prm, s, w, res, quality):
    """The refinement variants beside the benchmark line: the same pipeline
    with the ancestors' alignment as the template, and tree-dependent
    refinement of the glued alignment (one pass; passes until nothing
    changes, at most 8)."""
    res_m, ms_m, _, _ = timed_steps(pipeline.run_device, seqs, prm, args.steps, args.warmup, B,
                                    torch, "ga_msa")
    host_m = pipeline.to_host(res_m, s.n, w.p, seqs.total_len)
    cells_m = host_m["align"]["cells"] + host_m["refine"]["cells"]
    out["template_ga_msa"] = {"ms_per_step": round(ms_m, 3),
                              "value": round(cells_m / (ms_m / 1e3) / 1e9, 3), "unit": "GCUPS",
                              "dp_cells_per_step": cells_m,
                              "quality": quality(host_m["refine"]["colmap"])}
    # tree-dependent refinement of the glued alignment: one pass over the
    # ancestor tree's edges, and passes until nothing changes (at most 8)
    tr = {}
    for passes in (1, 8):
        B.sad_refine_tree(seqs, res["part"]["bucket_off"], res["part"]["members"],
                          res["refine"], prm, passes)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        reps = 3
        for _ in range(reps):
            cm_t, w_t, st_t, acc_t, _ = B.sad_refine_tree(seqs, res["part"]["bucket_off"],
                                                          res["part"]["members"], res["refine"],
                                                          prm, passes)
        e1.record()
        torch.cuda.synchronize()
        tr[f"passes_{passes}"] = {"ms": round(e0.elapsed_time(e1) / reps, 3), "steps": st_t,
                                  "accepted": acc_t, "width": w_t,
                                  "quality": quality(cm_t.cpu().numpy())}
    out["tree_refine"] = tr


def host_threads() -> int:
    """Host cores this process may use (affinity, capped by OMP_NUM_THREADS
    when set: a machine shared by several GPUs gives each GPU's process a
    share of the host)."""
    n = len(os.sched_getaffinity(0))
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(n, 1)


def oracle_sample(s, w, host, threads):
    """The oracle on a bounded sample of a large workload, all host threads:
    the rank keys of 256 sequences against the library's samples, and the
    alignment of 16 whole buckets (spread over the bucket order)."""
    import numpy as np

    import oracle
    oracle.set_threads(threads)
    try:
        rng = np.random.default_rng(3)
        rows = np.sort(rng.choice(s.n, 256, replace=False)).astype(np.int32)
        t0 = time.perf_counter()
        kref = oracle.rank_against(s.codes, s.offsets, s.alphabet, w.kmer_k,
                                   samples=host["samples"], rows=rows)
        t_rank = time.perf_counter() - t0
        boff, mem = host["part"]["bucket_off"], host["part"]["members"]
        pick = np.linspace(0, w.p - 1, 16).round().astype(int)
        ids = np.concatenate([mem[boff[b]:boff[b + 1]] for b in pick])
        sizes = [boff[b + 1] - boff[b] for b in pick]
        sub = s.subset(ids)
        sboff = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
        t0 = time.perf_counter()
        ra = oracle.align_buckets(sub.codes, sub.offsets, s.alphabet, sboff,
                                  np.arange(len(ids), dtype=np.int32), w.kmer_k, w.subst(),
                                  w.gap_open, w.gap_extend)
        t_al = time.perf_counter() - t0
    finally:
        oracle.set_threads(1)
    same = bool(np.array_equal(kref, host["key"][rows]))
    gcm = np.concatenate([host["align"]["colmap"][s.offsets[i]:s.offsets[i + 1]] for i in ids])
    same = same and bool(np.array_equal(gcm, ra["colmap"]))
    return {"value": round(ra["cells"] / t_al / 1e9, 5), "unit": "GCUPS", "cores": threads,
            "kind": "oracle",
            "sample": f"alignment of 16 whole buckets ({int(ra['cells'])} DP cells, "
                      f"{t_al:.2f} s) and rank keys of 256 sequences ({t_rank:.2f} s)",
            "bit_exact_vs_library": same}


def workload_figures(name, args, B, pipeline, torch, threads):
    """Batched and plain pass times of one workload (each mode autotuned
    first), GCUPS, sequences/s, the engine kernel against the int32 peak,
    the caller workspace the pass used, and the oracle on a sample."""
    import numpy as np

    from workloads import make_inputs, workload
    w = workload(name)
    t0 = time.perf_counter()
    s = make_inputs(name)
    gen_s = time.perf_counter() - t0
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
    out = {"n": s.n, "alphabet": s.alphabet, "mean_len": round(float(s.lengths.mean()), 1),
           "buckets": w.p, "kmer_k": w.kmer_k, "gaps": f"{w.gap_open}/{w.gap_extend}",
           "input_generation_s": round(gen_s, 1)}
    hosts = {}
    for mode, label in ((B.SAD_BATCHED_MFMA, "batched"), (B.SAD_PLAIN, "plain")):
        print(f"workload {name}: {label}", file=sys.stderr, flush=True)
        prm = B.Params(w.kmer_k, w.p, w.subst(), w.gap_open, w.gap_extend, w.s_max, mode)
        key0, _ = B.sad_kmer_rank(seqs, prm)
        part0 = B.sad_partition(seqs, key0, prm)
        tuned = B.sad_tune(seqs, part0["bucket_off"], part0["members"], prm)
        B.sad_profile_graphs(reset=True)
        res, ms, eng_ms, launches = timed_steps(pipeline.run_device, seqs, prm,
                                                args.workload_steps, 1, B, torch)
        graphs = B.sad_profile_graphs(reset=True)
        host = pipeline.to_host(res, s.n, w.p, seqs.total_len)
        hosts[label] = host
        cells = host["align"]["cells"] + host["refine"]["cells"]
        eng_pass = eng_ms / args.workload_steps
        achieved = cells * OPS_PER_CELL / (eng_pass / 1e3) / 1e12 if eng_pass > 0 else 0.0
        out[label] = {"ms_per_pass": round(ms, 3),
                      "value": round(cells / (ms / 1e3) / 1e9, 3), "unit": "GCUPS",
                      "seq_per_s": round(s.n / (ms / 1e3), 1), "dp_cells_per_pass": cells,
                      "engine_ms_per_pass": round(eng_pass, 3),
                      "engine_launches_per_pass": launches // args.workload_steps,
                      "roofline": {"bound": "alu", "achieved": round(achieved, 4),
                                   "peak": round(INT32_PEAK_TOPS, 2), "unit": "TOP/s (int32)",
                                   "frac": round(achieved / INT32_PEAK_TOPS, 5)},
                      "schedule": {"engine_workgroups": tuned[0],
                                   "trees_in_launch": bool(tuned[1]),
                                   "cooperative_merges": bool(tuned[2]),
                                   "mfma_scores": bool(tuned[3]),
                                   "chunk_steps": tuned[4] if tuned[3] else None,
                                   "graph_replays": graphs[1]}}
    out["same_result"] = bool(
        all(np.array_equal(hosts["batched"][st]["colmap"], hosts["plain"][st]["colmap"])
            for st in ("align", "refine")))
    out["workspace_bytes"] = int(max(t.numel() for t in B._WS.values())) if B._WS else 0
    if name == "prot64":
        import oracle
        oracle.set_threads(threads)
        t0 = time.perf_counter()
        ref = oracle.run_pipeline(s.codes, s.offsets, s.alphabet, w.kmer_k, w.p, w.subst(),
                                  w.gap_open, w.gap_extend, w.s_max)
        dt = time.perf_counter() - t0
        oracle.set_threads(1)
        rc = ref["align"]["cells"] + ref["refine"]["cells"]
        out["cpu_baseline"] = {"value": round(rc / dt / 1e9, 5), "unit": "GCUPS",
                               "cores": threads, "kind": "oracle",
                               "sample": f"full pipeline, {dt:.2f} s",
                               "bit_exact_vs_library": bool(
                                   np.array_equal(ref["refine"]["colmap"],
                                                  hosts["batched"]["refine"]["colmap"]))}
    else:
        out["cpu_baseline"] = oracle_sample(s, w, hosts["batched"], threads)
    del seqs, hosts
    B.release_workspace()
    torch.cuda.empty_cache()
    return out


def rank_study(args, B, pipeline, torch):
    """Centralised vs globalised k-mer rank on synthetic proteins: families of
    250 around roots of normal length (mean 316, sd 60, within 100..600), 10%
    substitutions and 2% indels per leaf, k = 3; the centralised rank is timed
    on the GPU (HIP events over 3 calls after one warm-up)."""
    import numpy as np

    from paper_0901_2742_amd.rankstats import rank_stats
    from workloads import generate

    p = args.rank_p
    for n in [int(x) for x in args.rank_study.split(",") if x]:
        print(f"rank study: N = {n}", file=sys.stderr, flush=True)
        s = generate(5000 + n, n, 20, max(1, n // 250),
                     {"kind": "normal", "mean": 316, "sd": 60, "lo": 100, "hi": 600},
                     0.10, 0.02, 3)
        seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
        prm = B.Params(3, p, np.zeros((20, 20), np.int8), 10, 1, 1024, B.SAD_BATCHED_MFMA)
        key, sid = B.sad_kmer_rank(seqs, prm)
        central = B.sad_rank_against(seqs, 3)
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record()
        for _ in range(3):
            central = B.sad_rank_against(seqs, 3)
        t1.record()
        torch.cuda.synchronize()
        ms = t0.elapsed_time(t1) / 3
        g = key.cpu().numpy().view(np.uint64)
        c = central.cpu().numpy().view(np.uint64)
        st = rank_stats(c, g, n, int(sid.numel()))
        line = {"study": "rank", "n": n, "p": p, "global_samples": int(sid.numel()),
                "central_ms": round(ms, 3), "central_pairs": n * n}
        def sig(v):
            return float(f"{v:.6g}")

        line.update({k: (sig(v) if isinstance(v, float) else v) for k, v in st.items()
                     if k not in ("central", "global", "hist_edges")})
        line["central"] = {k: sig(v) for k, v in st["central"].items()}
        line["global"] = {k: sig(v) for k, v in st["global"].items()}
        print(json.dumps(line), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU and this benchmark measures one GPU "
              f"only (asked for --gpus {args.gpus}); sharding across GPUs is not implemented",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_0901_2742_amd import binding as B
    from paper_0901_2742_amd import pipeline
    from workloads import make_inputs, workload

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.rank_study:
        rank_study(args, B, pipeline, torch)
        return
    w = workload(args.workload)
    s = make_inputs(args.workload)
    seqs = pipeline.to_device(s.codes, s.offsets, s.alphabet)
    S = w.subst()
    cls, ncls = s.homology_classes()
    d_cls = torch.tensor(cls, device="cuda")

    def quality(colmap):
        a, t = B.sad_quality(torch.tensor(colmap, dtype=torch.int32, device="cuda"), d_cls, ncls)
        return {"Q": round(a / t, 5) if t else None, "aligned_pairs": a, "true_pairs": t}

    if args.sweep_p:
        # bucket-count sweep: time and quality of the pipeline at each p
        # (the default schedule at every p: the sweep is over p, not schedules)
        for p in [int(x) for x in args.sweep_p.split(",") if x]:
            print(f"sweep: p = {p}", file=sys.stderr, flush=True)
            prm_s = B.Params(w.kmer_k, p, S, w.gap_open, w.gap_extend, w.s_max,
                             B.SAD_BATCHED_MFMA)
            res_s, ms_s, eng_s, nl = timed_steps(pipeline.run_device, seqs, prm_s, args.steps,
                                                 args.warmup, B, torch, args.template)
            h = pipeline.to_host(res_s, s.n, p, seqs.total_len)
            cl = h["align"]["cells"] + h["refine"]["cells"]
            sizes = np.diff(h["part"]["bucket_off"])
            line = {"sweep": "buckets", "workload": w.name, "p": p, "template": args.template,
                    "ms_per_step": round(ms_s, 3),
                    "value": round(cl / (ms_s / 1e3) / 1e9, 3), "unit": "GCUPS",
                    "dp_cells_per_step": cl, "largest_bucket": int(sizes.max()),
                    "engine_ms_per_step": round(eng_s / args.steps, 3),
                    "quality": quality(h["refine"]["colmap"])}
            print(json.dumps(line), flush=True)
        return
    prm = B.Params(w.kmer_k, w.p, S, w.gap_open, w.gap_extend, w.s_max, B.SAD_BATCHED_MFMA)
    # autotune the bucket alignment's schedule on this workload (cached for
    # the process), then time the pipeline with it
    key0, _ = B.sad_kmer_rank(seqs, prm)
    part0 = B.sad_partition(seqs, key0, prm)
    tuned = (0, -1, 1, 1, 32) if args.no_tune else B.sad_tune(seqs, part0["bucket_off"],
                                                    part0["members"], prm)
    B.sad_profile_graphs(reset=True)
    res, ms, eng_ms, launches = timed_steps(pipeline.run_device, seqs, prm, args.steps,
                                            args.warmup, B, torch)
    graphs = B.sad_profile_graphs(reset=True)
    host = pipeline.to_host(res, s.n, w.p, seqs.total_len)
    if args.calibrate_copy > 0:
        src = torch.ones(args.calibrate_copy * (1 << 20) // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    cells = host["align"]["cells"] + host["refine"]["cells"]
    gcups = cells / (ms / 1e3) / 1e9
    qual = quality(host["refine"]["colmap"])
    seq_s = s.n / (ms / 1e3)
    # engine kernel: algorithmic int32 ops over its measured launch time
    eng_ops = cells * args.steps * OPS_PER_CELL
    achieved = eng_ops / (eng_ms / 1e3) / 1e12 if eng_ms > 0 else 0.0
    out = {
        "metric": METRIC, "value": round(gcups, 3), "unit": "GCUPS", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic (seeded family-structured proteins)",
        "config": {"workload": w.name, "n": s.n, "mean_len": round(float(s.lengths.mean()), 1),
                   "buckets": w.p, "kmer_k": w.kmer_k, "gaps": f"{w.gap_open}/{w.gap_extend}",
                   "matrix": ("seeded 20x20 integer stand-in (BLOSUM62 range)"
                              if s.alphabet == 20 else "+2/-3 (DNA)"),
                   "parallelism": "single GPU"},
        "seq_per_s": round(seq_s, 2),
        "dp_cells_per_step": cells,
        "quality": qual,
        "mode": "batched",
        # (untuned: the library's default, trees in the launch while buckets
        # have at most 182 members; null here)
        "schedule": {"engine_workgroups": tuned[0],
                     "trees_in_launch": bool(tuned[1]) if tuned[1] >= 0 else None,
                     "cooperative_merges": bool(tuned[2]), "mfma_scores": bool(tuned[3]),
                     "chunk_steps": tuned[4] if tuned[3] else None,
                     "graph_captures": graphs[0], "graph_replays": graphs[1]},
        "engine_kernel": {"ms_total": round(eng_ms, 3), "launches": launches,
                          "avg_launch_ms": round(eng_ms / max(launches, 1), 4),
                          "share_of_step": round(eng_ms / (ms * args.steps), 3)},
        "roofline": {"bound": "alu", "achieved": round(achieved, 4),
                     "peak": round(INT32_PEAK_TOPS, 2), "unit": "TOP/s (int32)",
                     "frac": round(achieved / INT32_PEAK_TOPS, 5),
                     "traffic": measured_traffic(w.name),
                     "ops_per_cell": OPS_PER_CELL},
    }
    if not args.no_extras:
        extras(out, args, B, pipeline, torch, seqs, prm, s, w, res, quality)
    if not args.no_plain:
        prm_p = B.Params(w.kmer_k, w.p, S, w.gap_open, w.gap_extend, w.s_max, B.SAD_PLAIN)
        tuned_p = B.sad_tune(seqs, part0["bucket_off"], part0["members"], prm_p)
        res_p, ms_p, _, _ = timed_steps(pipeline.run_device, seqs, prm_p, args.steps,
                                        args.warmup, B, torch)
        host_p = pipeline.to_host(res_p, s.n, w.p, seqs.total_len)
        out["plain"] = {"value": round(cells / (ms_p / 1e3) / 1e9, 3), "unit": "GCUPS",
                        "ms_per_step": round(ms_p, 3), "engine_workgroups": tuned_p[0],
                        "same_result": bool(np.array_equal(host_p["refine"]["colmap"],
                                                           host["refine"]["colmap"]))}
    threads = host_threads()
    if not args.no_cpu_baseline and w.name not in ("prot64", "prot2000"):
        # a large workload as the main one: the oracle on a bounded sample
        out["cpu_baseline"] = oracle_sample(s, w, host, threads)
        out["bit_exact_vs_oracle"] = out["cpu_baseline"]["bit_exact_vs_library"]
    elif not args.no_cpu_baseline:
        import oracle
        # one thread, then every host core this process may use
        t = time.perf_counter()
        ref1 = oracle.run_pipeline(s.codes, s.offsets, s.alphabet, w.kmer_k, w.p, S, w.gap_open,
                                   w.gap_extend, w.s_max)
        dt1 = time.perf_counter() - t
        oracle.set_threads(threads)
        t = time.perf_counter()
        ref = oracle.run_pipeline(s.codes, s.offsets, s.alphabet, w.kmer_k, w.p, S, w.gap_open,
                                  w.gap_extend, w.s_max)
        dt = time.perf_counter() - t
        oracle.set_threads(1)
        ref_cells = ref["align"]["cells"] + ref["refine"]["cells"]
        exact = (np.array_equal(ref["key"], host["key"])
                 and np.array_equal(ref["part"]["members"], host["part"]["members"])
                 and np.array_equal(ref["align"]["colmap"], host["align"]["colmap"])
                 and np.array_equal(ref["align"]["merge_score"][:s.n],
                                    host["align"]["merge_score"][:s.n])
                 and np.array_equal(ref["refine"]["ga"], host["refine"]["ga"])
                 and np.array_equal(ref["refine"]["colmap"], host["refine"]["colmap"])
                 and ref_cells == cells
                 and np.array_equal(ref1["refine"]["colmap"], ref["refine"]["colmap"]))
        out["cpu_baseline"] = {"value": round(ref_cells / dt / 1e9, 5), "unit": "GCUPS",
                               "cores": threads, "kind": "oracle",
                               "sample": f"full {w.name} pipeline (all four stages), one run on "
                                         f"{threads} threads ({dt:.2f} s) and one on one thread "
                                         f"({dt1:.2f} s)",
                               "seq_per_s": round(s.n / dt, 2),
                               "single_thread": {"value": round(ref_cells / dt1 / 1e9, 5),
                                                 "unit": "GCUPS", "seconds": round(dt1, 2),
                                                 "seq_per_s": round(s.n / dt1, 2)}}
        out["bit_exact_vs_oracle"] = bool(exact)
    if args.workloads:
        # the other workloads: parity cases of the test suite, timed here so
        # that the engine's roofline is reported where it is throughput-bound
        out["workloads"] = {}
        for name in [x for x in args.workloads.split(",") if x]:
            out["workloads"][name] = workload_figures(name, args, B, pipeline, torch, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
