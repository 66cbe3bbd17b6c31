"""CPU oracle for the Sample-Align-D data-parallel core -- TEST INFRASTRUCTURE.

A ctypes wrapper over ``sad_oracle.c`` (plain single-threaded C written from
the paper's definitions).  Only the tests, the smoke check and the benchmark's
CPU-baseline leg may import this package; the HIP library never calls it and
shares no code with it.

Parity status per step (what pins it, in ``tests/test_oracle_*.py``):
  k-mer lists, c_ij, F          brute force (collections.Counter, Fraction)
  local/global rank, samples    order-statistic and sum properties, sorted()
  pivots, buckets               Y order statistics, pivot ranges, paper bound
  UPGMA                         scipy average linkage (tie-free), crafted ties
  profile alignment             exhaustive enumeration of alignments (score
                                and tie-broken path), textbook pairwise Gotoh,
                                numpy column scores, score recomputation
  progressive / refine / glue   replay invariants (degapped rows, restriction,
                                no all-gap columns, recomputed merge scores)
  quality counts (Q)            brute-force enumeration of residue pairs,
                                perfect and shifted alignments
  rank against a sample         Counter-built F summed by rows, identical
                                sequences, the globalised rank recomputed
  q-row refinement template     one bucket, identical ancestors (scores x q),
                                enumeration against the rebuilt template
  tree-dependent refinement     an independent Python re-run of every step
                                with exhaustive enumeration on tiny inputs;
                                converged and optimal inputs unchanged
The whole pipeline has no printed example in the paper: end to end it is pinned
only through those invariants.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sad_oracle.c")
# SADREF_LIB names another build of the same source to load instead (the
# sanitizer test runs the pin suite against an ASan/UBSan build)
_LIB = os.environ.get("SADREF_LIB") or os.path.join(_HERE, "libsad_oracle.so")

OP_M, OP_X, OP_Y = 0, 1, 2
OK, E_INVAL, E_CAPACITY, E_OVERFLOW = 0, -1, -2, -3


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: status {code}")
        self.code = code


def build(force: bool = False) -> str:
    """Compiles the oracle with gcc (plain -O2, portable code)."""
    if os.environ.get("SADREF_LIB"):
        return _LIB
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-Wall",
                               "-Wno-unused-function", _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


P = ctypes.c_void_p
I32, I64 = ctypes.c_int32, ctypes.c_int64


def _declare(L):
    L.sadref_set_threads.argtypes = [I32]
    L.sadref_set_threads.restype = None
    L.sadref_kmer_list.argtypes = [P, I64, ctypes.c_int, ctypes.c_int, P, P, P]
    L.sadref_common_kmers.argtypes = [P, I64, P, I64, ctypes.c_int, ctypes.c_int]
    L.sadref_common_kmers.restype = I64
    L.sadref_fhat.argtypes = [P, I64, P, I64, ctypes.c_int, ctypes.c_int]
    L.sadref_fhat.restype = ctypes.c_uint32
    L.sadref_kmer_rank.argtypes = [I32, I32, P, P, I32, I32, I32, P, P, I32, P]
    L.sadref_rank_against.argtypes = [I32, I32, P, P, I32, P, I32, P, I32, P]
    L.sadref_partition.argtypes = [I32, P, I32, P, P, P, P, P]
    L.sadref_upgma.argtypes = [I32, P, P]
    L.sadref_profile_align.argtypes = [P, I32, I32, P, I32, I32, I32, P, I32, I32, P, P, P]
    L.sadref_align_buckets.argtypes = [I32, I32, P, P, I32, P, P, I32, P, I32, I32,
                                       P, P, P, P, P, P, P, I64, P]
    L.sadref_consensus.argtypes = [P, I32, I32, I32, P, P]
    L.sadref_refine.argtypes = [I32, I32, P, P, I32, P, P, P, P, I32, P, I32, I32,
                                P, I32, P, P, P, P, P, P, P, P]
    L.sadref_refine_template.argtypes = [I32, I32, P, P, I32, P, P, P, P, I32, P, I32, I32, I32,
                                         P, I32, P, P, P, P, P, P, P, P]
    L.sadref_refine_template_ops.argtypes = [I32, I32, P, P, I32, P, P, P, P, I32, P, I32, I32,
                                             I32, P, I32, P, P, P, P, P, P, P, P, P, I64, P, P]
    L.sadref_glue.argtypes = [I32, I32, P, P, P, P, P]
    L.sadref_refine_tree.argtypes = [I32, I32, P, P, I32, P, P, P, I32, P, I32, P, I32, I32, I32,
                                     P, P, P, P, P, P, I32, P]
    for f in ("sadref_refine_tree", "sadref_kmer_list", "sadref_kmer_rank", "sadref_rank_against", "sadref_partition",
              "sadref_upgma",
              "sadref_profile_align", "sadref_align_buckets", "sadref_consensus",
              "sadref_refine", "sadref_refine_template", "sadref_refine_template_ops",
              "sadref_glue"):
        getattr(L, f).restype = ctypes.c_int


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


def _check(st, what):
    if st != OK:
        raise OracleError(st, what)


# --------------------------------------------------------------------------
# k-mers
# --------------------------------------------------------------------------

def kmer_list(x, A: int, k: int):
    x = _c(x, np.uint8)
    m = max(len(x) - k + 1, 1)
    taus = np.zeros(m, np.int32)
    cnts = np.zeros(m, np.int32)
    nu = np.zeros(1, np.int64)
    _check(lib().sadref_kmer_list(_p(x), len(x), A, k, _p(taus), _p(cnts), _p(nu)), "kmer_list")
    u = int(nu[0])
    return taus[:u].copy(), cnts[:u].copy()


def common_kmers(xi, xj, A: int, k: int) -> int:
    xi, xj = _c(xi, np.uint8), _c(xj, np.uint8)
    return int(lib().sadref_common_kmers(_p(xi), len(xi), _p(xj), len(xj), A, k))


def fhat(xi, xj, A: int, k: int) -> int:
    xi, xj = _c(xi, np.uint8), _c(xj, np.uint8)
    return int(lib().sadref_fhat(_p(xi), len(xi), _p(xj), len(xj), A, k))


# --------------------------------------------------------------------------
# rank and partition
# --------------------------------------------------------------------------

def set_threads(threads: int) -> None:
    """Threads of the oracle's loops over independent items (1: the calling
    thread only, the default); results do not depend on it."""
    lib().sadref_set_threads(int(threads))


def kmer_rank(codes, offsets, A: int, k: int, p: int, s_max: int = 1024):
    codes, offsets = _c(codes, np.uint8), _c(offsets, np.int64)
    n = len(offsets) - 1
    key = np.zeros(max(n, 1), np.uint64)
    cap = max(s_max, p) + p
    sid = np.zeros(cap, np.int32)
    ns = np.zeros(1, np.int32)
    st = lib().sadref_kmer_rank(n, A, _p(codes), _p(offsets), k, p, s_max, _p(key), _p(sid),
                                cap, _p(ns))
    _check(st, "kmer_rank")
    return key[:n].copy(), sid[:int(ns[0])].copy()


def rank_against(codes, offsets, A: int, k: int, samples=None, rows=None):
    """K_i = sum over the samples s of F(i, s) for the listed rows (Section
    2.3.1).  samples=None: all N sequences, i.e. the centralised rank that the
    globalised rank (against the k p samples) approximates; rows=None: all."""
    codes, offsets = _c(codes, np.uint8), _c(offsets, np.int64)
    n = len(offsets) - 1
    sp = None if samples is None else _c(samples, np.int32)
    rp = None if rows is None else _c(rows, np.int32)
    nr = n if rp is None else len(rp)
    key = np.zeros(max(nr, 1), np.uint64)
    st = lib().sadref_rank_against(n, A, _p(codes), _p(offsets), k,
                                   None if sp is None else _p(sp), 0 if sp is None else len(sp),
                                   None if rp is None else _p(rp), nr, _p(key))
    _check(st, "rank_against")
    return key[:nr].copy()


def partition(key, p: int):
    key = _c(key, np.uint64)
    n = len(key)
    pk = np.zeros(max(p - 1, 1), np.uint64)
    pid = np.zeros(max(p - 1, 1), np.int32)
    bucket = np.zeros(max(n, 1), np.int32)
    boff = np.zeros(p + 1, np.int32)
    mem = np.zeros(max(n, 1), np.int32)
    st = lib().sadref_partition(n, _p(key), p, _p(pk), _p(pid), _p(bucket), _p(boff), _p(mem))
    _check(st, "partition")
    return dict(pivot_key=pk[:p - 1].copy(), pivot_id=pid[:p - 1].copy(),
                bucket=bucket[:n].copy(), bucket_off=boff, members=mem[:n].copy())


# --------------------------------------------------------------------------
# alignment pieces
# --------------------------------------------------------------------------

def upgma(F):
    F = _c(F, np.uint32)
    n = F.shape[0]
    merges = np.zeros(max(2 * (n - 1), 2), np.int32)
    _check(lib().sadref_upgma(n, _p(F), _p(merges)), "upgma")
    return merges[:2 * max(n - 1, 0)].reshape(-1, 2).copy()


def profile_align(C1, n1: int, C2, n2: int, S, go: int, ge: int):
    """Returns (ops, score); C1: W1 x A, C2: W2 x A counts."""
    S = _c(S, np.int8)
    A = S.shape[0]
    C1 = _c(np.asarray(C1).reshape(-1, A), np.uint16)
    C2 = _c(np.asarray(C2).reshape(-1, A), np.uint16)
    W1, W2 = C1.shape[0], C2.shape[0]
    ops = np.zeros(max(W1 + W2, 1), np.uint8)
    nops = np.zeros(1, np.int32)
    score = np.zeros(1, np.int64)
    st = lib().sadref_profile_align(_p(C1), W1, n1, _p(C2), W2, n2, A, _p(S), go, ge,
                                    _p(ops), _p(nops), _p(score))
    _check(st, "profile_align")
    return ops[:int(nops[0])].copy(), int(score[0])


def consensus(counts, n: int):
    counts = _c(counts, np.uint16)
    W, A = counts.shape
    out = np.zeros(max(W, 1), np.uint8)
    ln = np.zeros(1, np.int32)
    _check(lib().sadref_consensus(_p(counts), W, n, A, _p(out), _p(ln)), "consensus")
    return out[:int(ln[0])].copy()


def align_buckets(codes, offsets, A: int, bucket_off, members, k: int, S, go: int, ge: int,
                  want_ops: bool = False):
    codes, offsets = _c(codes, np.uint8), _c(offsets, np.int64)
    boff, mem, S = _c(bucket_off, np.int32), _c(members, np.int32), _c(S, np.int8)
    n = len(offsets) - 1
    p = len(boff) - 1
    colmap = np.zeros(max(len(codes), 1), np.int32)
    width = np.zeros(p, np.int32)
    mscore = np.zeros(max(n, 1), np.int64)
    mlist = np.full(max(2 * n, 2), -1, np.int32)
    mcells = np.zeros(max(n, 1), np.int64)
    cells = np.zeros(1, np.int64)
    if want_ops:
        cap = int(2 * len(codes) * max(1, int(np.log2(max(n, 2)))) + 16)
        while True:
            ops = np.zeros(cap, np.uint8)
            ops_off = np.zeros(n + 1, np.int64)
            st = lib().sadref_align_buckets(n, A, _p(codes), _p(offsets), p, _p(boff), _p(mem),
                                            k, _p(S), go, ge, _p(colmap), _p(width), _p(mscore),
                                            _p(mlist), _p(mcells), _p(cells), _p(ops), cap,
                                            _p(ops_off))
            if st == E_CAPACITY:
                cap *= 4
                continue
            break
    else:
        ops = ops_off = None
        st = lib().sadref_align_buckets(n, A, _p(codes), _p(offsets), p, _p(boff), _p(mem),
                                        k, _p(S), go, ge, _p(colmap), _p(width), _p(mscore),
                                        _p(mlist), _p(mcells), _p(cells), None, 0, None)
    _check(st, "align_buckets")
    out = dict(colmap=colmap[:len(codes)].copy(), width=width, merge_score=mscore[:n].copy(),
               merge_list=mlist[:2 * n].reshape(-1, 2).copy(), merge_cells=mcells[:n].copy(),
               cells=int(cells[0]))
    if want_ops:
        out["ops"] = ops
        out["ops_off"] = ops_off
    return out


TEMPLATES = {"ga": 0, "ga_msa": 1}


def glue(TW: int, ops_list, widths):
    """Step 15 on its own: bucket op strings (one per non-empty bucket, in
    bucket order, over M/X/Y = 0/1/2) against a template of TW columns ->
    (list of per-bucket arrays: glued column of each bucket column, width)."""
    q = len(ops_list)
    ops = np.concatenate([_c(o, np.uint8) for o in ops_list]) if q else np.zeros(1, np.uint8)
    if len(ops) == 0:
        ops = np.zeros(1, np.uint8)
    off = np.zeros(q + 1, np.int64)
    off[1:] = np.cumsum([len(o) for o in ops_list])
    wu = _c(widths, np.int32) if q else np.zeros(1, np.int32)
    to_g = np.zeros(max(int(np.sum(widths)) if q else 0, 1), np.int32)
    wg = np.zeros(1, np.int32)
    _check(lib().sadref_glue(q, TW, _p(ops), _p(off), _p(wu), _p(to_g), _p(wg)), "glue")
    out, base = [], 0
    for w in widths:
        out.append(to_g[base:base + w].copy())
        base += w
    return out, int(wg[0])


def refine(codes, offsets, A: int, bucket_off, members, colmap_b, width_b, k: int, S,
           go: int, ge: int, template: str = "ga", want_ops: bool = False):
    """Steps 12-15: ancestors, GA, each bucket against the template, glue.
    template "ga": GA as a one-row profile; "ga_msa": the ancestors' alignment
    as a profile of q rows (the paper's future-work template).  want_ops: also
    return the refinement op strings ("ops": one array per non-empty bucket)
    and the template's width ("tmpl_width")."""
    codes, offsets = _c(codes, np.uint8), _c(offsets, np.int64)
    boff, mem, S = _c(bucket_off, np.int32), _c(members, np.int32), _c(S, np.int8)
    cb, wb = _c(colmap_b, np.int32), _c(width_b, np.int32)
    n = len(offsets) - 1
    p = len(boff) - 1
    # the ancestors' alignment is at most as wide as all ancestors together
    ga_cap = max(int(wb.astype(np.int64).sum()), 1)
    ga = np.zeros(ga_cap, np.uint8)
    ga_len = np.zeros(1, np.int32)
    cg = np.zeros(max(len(codes), 1), np.int32)
    wg = np.zeros(1, np.int32)
    ms = np.zeros(2 * p, np.int64)
    ml = np.zeros(4 * p, np.int32)
    mc = np.zeros(2 * p, np.int64)
    nm = np.zeros(1, np.int32)
    cells = np.zeros(1, np.int64)
    # the refinement op strings: each at most W_b + template width <= 2 sum W
    ops_cap = max(4 * int(wb.astype(np.int64).sum()) + 16, 16) if want_ops else 0
    rops = np.zeros(max(ops_cap, 1), np.uint8)
    roff = np.zeros(p + 1, np.int64)
    tw = np.zeros(1, np.int32)
    st = lib().sadref_refine_template_ops(
        n, A, _p(codes), _p(offsets), p, _p(boff), _p(mem), _p(cb), _p(wb), k, _p(S), go, ge,
        TEMPLATES[template], _p(ga), ga_cap, _p(ga_len), _p(cg), _p(wg), _p(ms), _p(ml), _p(mc),
        _p(nm), _p(cells), _p(rops) if want_ops else None, ops_cap,
        _p(roff) if want_ops else None, _p(tw) if want_ops else None)
    _check(st, "refine")
    m = int(nm[0])
    out = dict(ga=ga[:int(ga_len[0])].copy(), colmap=cg[:len(codes)].copy(), width=int(wg[0]),
               merge_score=ms[:m].copy(), merge_list=ml[:2 * m].reshape(-1, 2).copy(),
               merge_cells=mc[:m].copy(), cells=int(cells[0]))
    if want_ops:
        q = int(np.count_nonzero(np.diff(boff)))
        out["ops"] = [rops[roff[u]:roff[u + 1]].copy() for u in range(q)]
        out["tmpl_width"] = int(tw[0])
    return out


def refine_tree(codes, offsets, A: int, bucket_off, members, colmap, width: int, tree, k: int,
                S, go: int, ge: int, passes: int = 1):
    """Tree-dependent refinement of a glued alignment: for every edge of the
    ancestors' guide tree (``tree``: its q - 1 merges as (a, b) pairs over
    leaves 0..q-1 = the non-empty buckets in bucket order), deepest first, the
    two sides' parts are re-aligned as profiles and kept iff the profile score
    rises; up to ``passes`` passes, stopping after one that changes nothing."""
    codes, offsets = _c(codes, np.uint8), _c(offsets, np.int64)
    boff, mem, S = _c(bucket_off, np.int32), _c(members, np.int32), _c(S, np.int8)
    cm = _c(colmap, np.int32)
    tr = _c(np.asarray(tree).reshape(-1), np.int32)
    n = len(offsets) - 1
    p = len(boff) - 1
    out = np.zeros(max(len(codes), 1), np.int32)
    wout = np.zeros(1, np.int32)
    nst = np.zeros(1, np.int32)
    nacc = np.zeros(1, np.int32)
    cap = max(1, passes * max(1, 2 * p))
    rn = np.zeros(cap, np.int32)
    ro = np.zeros(cap, np.int64)
    rw = np.zeros(cap, np.int64)
    st = lib().sadref_refine_tree(n, A, _p(codes), _p(offsets), p, _p(boff), _p(mem), _p(cm),
                                  int(width), _p(tr) if len(tr) else None, k, _p(S), go, ge,
                                  passes, _p(out), _p(wout), _p(nst), _p(rn), _p(ro), _p(rw), cap,
                                  _p(nacc))
    _check(st, "refine_tree")
    m = min(int(nst[0]), cap)
    return dict(colmap=out[:len(codes)].copy(), width=int(wout[0]), steps=int(nst[0]),
                accepted=int(nacc[0]), rec_node=rn[:m].copy(), rec_old=ro[:m].copy(),
                rec_new=rw[:m].copy())


def run_pipeline(codes, offsets, A: int, k: int, p: int, S, go: int, ge: int,
                 s_max: int = 1024, want_ops: bool = False, template: str = "ga"):
    """All four steps in order, as the HIP library's calls chain them."""
    key, samples = kmer_rank(codes, offsets, A, k, p, s_max)
    part = partition(key, p)
    al = align_buckets(codes, offsets, A, part["bucket_off"], part["members"], k, S, go, ge,
                       want_ops=want_ops)
    rf = refine(codes, offsets, A, part["bucket_off"], part["members"], al["colmap"],
                al["width"], k, S, go, ge, template=template)
    return dict(key=key, samples=samples, part=part, align=al, refine=rf)


def quality_counts(colmap, cls):
    """Q measure of Section 4 against homology classes: (aligned pairs, true
    pairs).  A true pair is two residues of one class; it is aligned when the
    alignment puts both in one column.  Counted per class and per (class,
    column) group: a group of m residues holds m (m - 1) / 2 pairs."""
    colmap = np.asarray(colmap, dtype=np.int64)
    cls = np.asarray(cls, dtype=np.int64)
    if colmap.shape != cls.shape:
        raise ValueError("colmap and classes differ in length")
    if colmap.size == 0:
        return 0, 0
    _, m = np.unique(cls, return_counts=True)
    true_pairs = int((m * (m - 1) // 2).sum())
    _, g = np.unique(np.stack([cls, colmap], axis=1), axis=0, return_counts=True)
    aligned = int((g * (g - 1) // 2).sum())
    return aligned, true_pairs
