"""ctypes binding of libsad.so (include/sad.h).

Argument marshalling only: torch tensors provide device memory and the HIP
stream; every step of the method runs in the library's gfx950 kernels.  If the
library is not built this module raises -- there is no fallback path.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsad.so")

SAD_OK = 0
SAD_E_INVAL = -1
SAD_E_CAPACITY = -2
SAD_E_OVERFLOW = -3
SAD_E_DEVICE = -4
SAD_E_UNIMPLEMENTED = -5
SAD_PLAIN = 0
SAD_BATCHED_MFMA = 1

# the functions include/sad.h declares
EXPORTS = ("sad_kmer_rank", "sad_kmer_rank_workspace", "sad_rank_against", "sad_partition",
           "sad_partition_workspace", "sad_partition_noalloc", "sad_align_buckets_workspace",
           "sad_refine_workspace", "sad_workspace_needed", "sad_align_buckets", "sad_refine", "sad_refine_template", "sad_refine_tree", "sad_tune",
           "sad_quality",
           "sad_profile_enable", "sad_profile_read", "sad_profile_phases", "sad_profile_jobs", "sad_profile_graphs",
           "sad_last_error",
           "sad_release",
           "sad_version")


class SadError(RuntimeError):
    def __init__(self, code: int, call: str, msg: str):
        super().__init__(f"{call} failed with status {code}: {msg}")
        self.code = code


class SadSeqs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("alphabet", ctypes.c_int32),
                ("d_codes", ctypes.c_void_p), ("d_offsets", ctypes.c_void_p),
                ("total_len", ctypes.c_int64), ("max_len", ctypes.c_int32)]


class SadParams(ctypes.Structure):
    _fields_ = [("kmer_k", ctypes.c_int32), ("p", ctypes.c_int32), ("s_max", ctypes.c_int32),
                ("subst", ctypes.c_void_p), ("gap_open", ctypes.c_int32),
                ("gap_extend", ctypes.c_int32), ("mode", ctypes.c_uint32)]


class SadMsa(ctypes.Structure):
    _fields_ = [("d_colmap", ctypes.c_void_p), ("d_width", ctypes.c_void_p),
                ("d_merge_score", ctypes.c_void_p), ("d_merge_list", ctypes.c_void_p),
                ("d_merge_cells", ctypes.c_void_p), ("d_cells", ctypes.c_void_p)]


_lib = None


def lib():
    """Loads libsad.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_0901_2742_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I32 = ctypes.c_int32
        SZ = ctypes.c_size_t
        L.sad_kmer_rank.argtypes = [P, P, P, P, I32, P, P, SZ, P]
        L.sad_rank_against.argtypes = [P, I32, P, I32, P, P]
        L.sad_partition.argtypes = [P, P, P, P, P, P, P, P, P, SZ, P]
        L.sad_partition_noalloc.argtypes = [P, P, P, P, P, P, P, P, P]
        L.sad_align_buckets.argtypes = [P, P, P, P, P, P, SZ, P]
        L.sad_refine.argtypes = [P, P, P, P, P, P, I32, P, P, P, P, SZ, P]
        L.sad_refine_template.argtypes = [P, P, P, P, P, I32, P, I32, P, P, P, P, SZ, P]
        L.sad_kmer_rank_workspace.argtypes = [P, P, P]
        L.sad_partition_workspace.argtypes = [P, P, P]
        L.sad_align_buckets_workspace.argtypes = [P, P, P, P, P]
        L.sad_refine_workspace.argtypes = [P, P, P, P, P, P]
        for f in ("sad_kmer_rank_workspace", "sad_partition_workspace",
                  "sad_align_buckets_workspace", "sad_refine_workspace"):
            getattr(L, f).restype = I32
        L.sad_workspace_needed.argtypes = []
        L.sad_workspace_needed.restype = SZ
        L.sad_refine_tree.argtypes = [P, P, P, P, P, I32, P, P, P, P, I32, P]
        for f in ("sad_kmer_rank", "sad_rank_against", "sad_partition", "sad_partition_noalloc",
                  "sad_align_buckets",
                  "sad_refine", "sad_refine_template", "sad_refine_tree"):
            getattr(L, f).restype = I32
        L.sad_profile_enable.argtypes = [I32]
        L.sad_profile_enable.restype = I32
        L.sad_profile_read.argtypes = [P, P, I32]
        L.sad_profile_read.restype = I32
        L.sad_profile_phases.argtypes = [P, P, I32]
        L.sad_profile_phases.restype = I32
        L.sad_profile_jobs.argtypes = [P, ctypes.c_int64, P]
        L.sad_profile_jobs.restype = I32
        L.sad_tune.argtypes = [P, P, P, P, P, P, P, P, P]
        L.sad_tune.restype = I32
        L.sad_profile_graphs.argtypes = [P, P, I32]
        L.sad_profile_graphs.restype = I32
        L.sad_quality.argtypes = [P, P, ctypes.c_int64, I32, P, P, P]
        L.sad_quality.restype = I32
        L.sad_last_error.restype = ctypes.c_char_p
        L.sad_version.restype = ctypes.c_char_p
        L.sad_release.restype = None
        _lib = L
    return _lib


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check(code: int, call: str):
    if code != SAD_OK:
        raise SadError(code, call, lib().sad_last_error().decode(errors="replace"))


# Device workspace of the four stage calls: caller-owned (a torch uint8
# tensor per device, grown on demand and shared by the calls, which run one
# after another on the current stream).  ws="library" passes NULL, letting the
# library use its own workspace; a tensor is used as given.
_WS: dict = {}


def _ws_tensor(dev, nbytes: int) -> torch.Tensor:
    idx = dev.index if dev.index is not None else torch.cuda.current_device()
    t = _WS.get(idx)
    if t is None or t.numel() < nbytes:
        _WS.pop(idx, None)
        # whole 2 MiB pages; torch's blocks are 512-byte aligned
        size = max((nbytes + (2 << 20) - 1) // (2 << 20) * (2 << 20), 2 << 20)
        t = torch.empty(size, dtype=torch.uint8, device=dev)
        _WS[idx] = t
    return t


def release_workspace() -> None:
    """Drops the binding's cached workspaces."""
    _WS.clear()


def _query(fn, *args, stream: bool = False) -> int:
    """Calls a workspace query: (args..., size_t* ws_bytes[, stream])."""
    n = ctypes.c_size_t(0)
    tail = (ctypes.byref(n), _stream()) if stream else (ctypes.byref(n),)
    _check(getattr(lib(), fn)(*args, *tail), fn)
    return n.value


def _with_ws(name: str, dev, ws, query, call):
    """Runs call(ptr, nbytes) with the workspace choice `ws`; with the
    binding's own workspace, sizes it by `query()` on first use and grows it
    to sad_workspace_needed() after a capacity failure."""
    if isinstance(ws, str):
        if ws != "library":
            raise ValueError("ws must be a tensor, None or 'library'")
        code = call(None, 0)
    elif ws is not None:
        if ws.dtype != torch.uint8 or not ws.is_contiguous():
            raise ValueError("workspace must be a contiguous uint8 tensor")
        code = call(_ptr(ws), ws.numel())
    else:
        idx = dev.index if dev.index is not None else torch.cuda.current_device()
        t = _WS.get(idx)
        if t is None:
            t = _ws_tensor(dev, query())
        code = call(_ptr(t), t.numel())
        need = lib().sad_workspace_needed()
        if code == SAD_E_CAPACITY and need > t.numel():
            t = _ws_tensor(dev, need)
            code = call(_ptr(t), t.numel())
    _check(code, name)


@dataclasses.dataclass
class DeviceSeqs:
    """Sequences resident in HBM (uint8 codes, int64 offsets)."""
    n: int
    alphabet: int
    codes: torch.Tensor
    offsets: torch.Tensor
    total_len: int
    max_len: int

    @classmethod
    def from_numpy(cls, codes: np.ndarray, offsets: np.ndarray, alphabet: int,
                   device: str = "cuda") -> "DeviceSeqs":
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        n = len(offsets) - 1
        lens = np.diff(offsets)
        c = torch.from_numpy(codes if len(codes) else np.zeros(1, np.uint8)).to(device)
        o = torch.from_numpy(offsets).to(device)
        return cls(n, alphabet, c, o, int(offsets[-1]), int(lens.max()) if n else 0)

    def c_struct(self) -> SadSeqs:
        return SadSeqs(self.n, self.alphabet, self.codes.data_ptr(), self.offsets.data_ptr(),
                       self.total_len, self.max_len)


@dataclasses.dataclass
class Params:
    kmer_k: int
    p: int
    subst: np.ndarray
    gap_open: int
    gap_extend: int
    s_max: int = 1024
    mode: int = SAD_BATCHED_MFMA

    def c_struct(self) -> SadParams:
        self._s = np.ascontiguousarray(self.subst, dtype=np.int8)  # keep alive
        return SadParams(self.kmer_k, self.p, self.s_max,
                         self._s.ctypes.data_as(ctypes.c_void_p).value, self.gap_open,
                         self.gap_extend, self.mode)


def sad_kmer_rank_workspace(seqs: DeviceSeqs, prm: Params) -> int:
    s, p = seqs.c_struct(), prm.c_struct()
    return _query("sad_kmer_rank_workspace", ctypes.byref(s), ctypes.byref(p))


def sad_partition_workspace(seqs: DeviceSeqs, prm: Params) -> int:
    s, p = seqs.c_struct(), prm.c_struct()
    return _query("sad_partition_workspace", ctypes.byref(s), ctypes.byref(p))


def sad_align_buckets_workspace(seqs: DeviceSeqs, bucket_off: torch.Tensor, prm: Params) -> int:
    s, p = seqs.c_struct(), prm.c_struct()
    return _query("sad_align_buckets_workspace", ctypes.byref(s), _ptr(bucket_off),
                  ctypes.byref(p), stream=True)


def sad_refine_workspace(seqs: DeviceSeqs, bucket_off: torch.Tensor, buckets: dict,
                         prm: Params) -> int:
    s, p, mb = seqs.c_struct(), prm.c_struct(), _msa_struct(buckets)
    return _query("sad_refine_workspace", ctypes.byref(s), _ptr(bucket_off), ctypes.byref(mb),
                  ctypes.byref(p), stream=True)


def sad_workspace_needed() -> int:
    return int(lib().sad_workspace_needed())


def sad_kmer_rank(seqs: DeviceSeqs, prm: Params, out: dict | None = None, ws=None):
    """Stage 1: globalised k-mer rank.  Returns (key[n] uint64 as int64 tensor,
    sample_ids int32 tensor).  `out` (a dict, filled on first use) keeps the
    output buffers across calls; `ws` chooses the workspace (see _with_ws)."""
    dev = seqs.codes.device
    cap = max(prm.s_max, prm.p) + prm.p
    if out is None:
        out = {}
    if "key" not in out:
        out["key"] = torch.empty(max(seqs.n, 1), dtype=torch.int64, device=dev)
        out["sid"] = torch.empty(cap, dtype=torch.int32, device=dev)
    key, sid = out["key"], out["sid"]
    ns = ctypes.c_int32(0)
    s, p = seqs.c_struct(), prm.c_struct()
    _with_ws("sad_kmer_rank", dev, ws, lambda: sad_kmer_rank_workspace(seqs, prm),
             lambda w, nb: lib().sad_kmer_rank(ctypes.byref(s), ctypes.byref(p), _ptr(key),
                                               _ptr(sid), cap, ctypes.byref(ns), w, nb,
                                               _stream()))
    return key[:seqs.n], sid[:ns.value]


def sad_rank_against(seqs: DeviceSeqs, kmer_k: int, samples: torch.Tensor | None = None):
    """K_i against the listed samples (int32 device tensor of ids) or, with
    samples=None, against all n sequences (the centralised rank).  Returns
    key[n] (uint64 as an int64 tensor)."""
    dev = seqs.codes.device
    key = torch.empty(max(seqs.n, 1), dtype=torch.int64, device=dev)
    s = seqs.c_struct()
    ns = 0
    if samples is not None:
        ns = samples.numel()
        # an empty list still needs a non-null pointer (null means all n)
        samples = samples.to(device=dev, dtype=torch.int32).contiguous() if ns else \
            torch.zeros(1, dtype=torch.int32, device=dev)
    code = lib().sad_rank_against(ctypes.byref(s), int(kmer_k),
                                  None if samples is None else _ptr(samples), ns, _ptr(key),
                                  _stream())
    _check(code, "sad_rank_against")
    return key[:seqs.n]


def sad_partition(seqs: DeviceSeqs, key: torch.Tensor, prm: Params, bufs: dict | None = None,
                  noalloc: bool = False, ws=None):
    """Stage 2: pivots and buckets.  Returns a dict of device tensors; `bufs`
    (a dict, filled on first use) keeps the buffers across calls.  noalloc:
    call sad_partition_noalloc (static device scratch, no synchronisation)."""
    dev = key.device
    n, p = seqs.n, prm.p
    if bufs is None:
        bufs = {}
    if "bucket_off" not in bufs:
        bufs.update(pivot_key=torch.empty(max(p - 1, 1), dtype=torch.int64, device=dev),
                    pivot_id=torch.empty(max(p - 1, 1), dtype=torch.int32, device=dev),
                    bucket=torch.empty(max(n, 1), dtype=torch.int32, device=dev),
                    bucket_off=torch.empty(p + 1, dtype=torch.int32, device=dev),
                    members=torch.empty(max(n, 1), dtype=torch.int32, device=dev))
    s, pp = seqs.c_struct(), prm.c_struct()
    args = (ctypes.byref(s), _ptr(key), ctypes.byref(pp), _ptr(bufs["pivot_key"]),
            _ptr(bufs["pivot_id"]), _ptr(bufs["bucket"]), _ptr(bufs["bucket_off"]),
            _ptr(bufs["members"]))
    if noalloc:
        _check(lib().sad_partition_noalloc(*args, _stream()), "sad_partition_noalloc")
    else:
        _with_ws("sad_partition", dev, ws, lambda: sad_partition_workspace(seqs, prm),
                 lambda w, nb: lib().sad_partition(*args, w, nb, _stream()))
    return dict(pivot_key=bufs["pivot_key"][:p - 1], pivot_id=bufs["pivot_id"][:p - 1],
                bucket=bufs["bucket"][:n], bucket_off=bufs["bucket_off"],
                members=bufs["members"][:n])


def _msa_tensors(n_res: int, n_width: int, n_steps: int, dev):
    return dict(colmap=torch.empty(max(n_res, 1), dtype=torch.int32, device=dev),
                width=torch.empty(max(n_width, 1), dtype=torch.int32, device=dev),
                merge_score=torch.empty(max(n_steps, 1), dtype=torch.int64, device=dev),
                merge_list=torch.empty(max(2 * n_steps, 2), dtype=torch.int32, device=dev),
                merge_cells=torch.empty(max(n_steps, 1), dtype=torch.int64, device=dev),
                cells=torch.empty(1, dtype=torch.int64, device=dev))


def _msa_struct(m: dict) -> SadMsa:
    def ptr(key):
        t = m.get(key)
        return t.data_ptr() if t is not None else None

    return SadMsa(ptr("colmap"), ptr("width"), ptr("merge_score"), ptr("merge_list"),
                  ptr("merge_cells"), ptr("cells"))


def sad_align_buckets(seqs: DeviceSeqs, bucket_off: torch.Tensor, members: torch.Tensor,
                      prm: Params, out: dict | None = None, ws=None):
    """Stage 3: align every bucket.  Returns a dict of device tensors."""
    dev = seqs.codes.device
    if out is None:
        out = _msa_tensors(seqs.total_len, prm.p, seqs.n, dev)
    s, pp, m = seqs.c_struct(), prm.c_struct(), _msa_struct(out)
    _with_ws("sad_align_buckets", dev, ws,
             lambda: sad_align_buckets_workspace(seqs, bucket_off, prm),
             lambda w, nb: lib().sad_align_buckets(ctypes.byref(s), _ptr(bucket_off),
                                                   _ptr(members), ctypes.byref(pp),
                                                   ctypes.byref(m), w, nb, _stream()))
    return out


SAD_TEMPLATE_GA = 0
SAD_TEMPLATE_GA_MSA = 1
TEMPLATES = {"ga": SAD_TEMPLATE_GA, "ga_msa": SAD_TEMPLATE_GA_MSA}


def sad_refine(seqs: DeviceSeqs, bucket_off: torch.Tensor, members: torch.Tensor, buckets: dict,
               prm: Params, out: dict | None = None, ga_cap: int | None = None,
               template: str = "ga", ws=None):
    """Stage 4: global ancestor, refinement and glue.  Returns a dict of device
    tensors plus ``ga_len`` and ``n_steps``.  template "ga" (sad_refine: GA as
    one row) or "ga_msa" (sad_refine_template: the ancestors' alignment)."""
    dev = seqs.codes.device
    if out is None:
        out = _msa_tensors(seqs.total_len, 1, 2 * prm.p, dev)
    if ga_cap is None:
        # GA is no longer than the sum of the ancestors, each no longer than its
        # bucket's width, which is at most the bucket's residue count
        ga_cap = max(seqs.total_len, 1)
    ga = out.get("ga")
    if ga is None or ga.numel() < ga_cap:
        ga = torch.empty(max(ga_cap, 1), dtype=torch.uint8, device=dev)
        out["ga"] = ga
    gl = ctypes.c_int32(0)
    nst = ctypes.c_int32(0)
    s, pp = seqs.c_struct(), prm.c_struct()
    mb, mg = _msa_struct(buckets), _msa_struct(out)
    query = lambda: sad_refine_workspace(seqs, bucket_off, buckets, prm)  # noqa: E731
    if template == "ga":
        _with_ws("sad_refine", dev, ws, query,
                 lambda w, nb: lib().sad_refine(ctypes.byref(s), _ptr(bucket_off), _ptr(members),
                                                ctypes.byref(mb), ctypes.byref(pp), _ptr(ga),
                                                ga_cap, ctypes.byref(gl), ctypes.byref(mg),
                                                ctypes.byref(nst), w, nb, _stream()))
    else:
        _with_ws("sad_refine_template", dev, ws, query,
                 lambda w, nb: lib().sad_refine_template(
                     ctypes.byref(s), _ptr(bucket_off), _ptr(members), ctypes.byref(mb),
                     ctypes.byref(pp), TEMPLATES[template], _ptr(ga), ga_cap, ctypes.byref(gl),
                     ctypes.byref(mg), ctypes.byref(nst), w, nb, _stream()))
    out["ga_len"] = gl.value
    out["n_steps"] = nst.value
    return out


def sad_refine_tree(seqs: DeviceSeqs, bucket_off: torch.Tensor, members: torch.Tensor,
                    glued: dict, prm: Params, passes: int = 1, rec_cap: int = 0):
    """Tree-dependent refinement of a glued alignment (the dict sad_refine
    returns).  Returns (colmap tensor, width, steps, accepted, records) with
    records an int64 array of (tree node, present score, new score) rows."""
    dev = seqs.codes.device
    colmap = torch.empty(max(seqs.total_len, 1), dtype=torch.int32, device=dev)
    width = torch.zeros(1, dtype=torch.int32, device=dev)
    out = {"colmap": colmap, "width": width}
    mg, mo = _msa_struct(glued), _msa_struct(out)
    rec = np.zeros((max(rec_cap, 1), 3), np.int64)
    nst, nacc = ctypes.c_int32(0), ctypes.c_int32(0)
    s, pp = seqs.c_struct(), prm.c_struct()
    code = lib().sad_refine_tree(ctypes.byref(s), _ptr(bucket_off), _ptr(members),
                                 ctypes.byref(mg), ctypes.byref(pp), int(passes), ctypes.byref(mo),
                                 ctypes.byref(nst), ctypes.byref(nacc),
                                 rec.ctypes.data_as(ctypes.c_void_p), int(rec_cap), _stream())
    _check(code, "sad_refine_tree")
    return (colmap[:seqs.total_len], int(width.item()), nst.value, nacc.value,
            rec[:min(nst.value, rec_cap)].copy())


def sad_profile_enable(on: bool, phases: bool = False) -> None:
    """Engine kernel timing; with phases=True also per-job phase records."""
    lib().sad_profile_enable((1 if on else 0) | (2 if on and phases else 0))


def sad_profile_read(reset: bool = False):
    """(engine kernel milliseconds, engine launches) accumulated while enabled."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    lib().sad_profile_read(ctypes.byref(ms), ctypes.byref(n), 1 if reset else 0)
    return ms.value, n.value


def sad_profile_phases(reset: bool = False):
    """Engine job phases (ms summed over jobs): wait, dp, traceback, merge, publish;
    and the number of jobs."""
    out = (ctypes.c_double * 5)()
    n = ctypes.c_int64(0)
    lib().sad_profile_phases(out, ctypes.byref(n), 1 if reset else 0)
    return dict(wait=out[0], dp=out[1], traceback=out[2], merge=out[3], publish=out[4],
                jobs=n.value)


def sad_tune(seqs: DeviceSeqs, bucket_off: torch.Tensor, members: torch.Tensor, prm: Params,
             out: dict | None = None):
    """Autotunes the schedule of sad_align_buckets for these buckets (cached for
    later calls with the same workload shape).  Returns (grid, fuse, coop,
    mfma, chunk): workgroups, trees in the launch, cooperative merges, MFMA
    column scores, steps per chunk of the MFMA kernel's DP strips."""
    dev = seqs.codes.device
    if out is None:
        out = _msa_tensors(seqs.total_len, prm.p, seqs.n, dev)
    s, pp, m = seqs.c_struct(), prm.c_struct(), _msa_struct(out)
    g, f, c = ctypes.c_int32(0), ctypes.c_int32(0), ctypes.c_int32(0)
    code = lib().sad_tune(ctypes.byref(s), _ptr(bucket_off), _ptr(members), ctypes.byref(pp),
                          ctypes.byref(m), ctypes.byref(g), ctypes.byref(f), ctypes.byref(c),
                          _stream())
    _check(code, "sad_tune")
    return g.value, f.value, c.value & 1, (c.value >> 1) & 1, 16 if c.value & 4 else 32


def sad_profile_graphs(reset: bool = False):
    """(captures, replays) of the bucket-alignment graph since the last reset."""
    c, r = ctypes.c_int64(0), ctypes.c_int64(0)
    lib().sad_profile_graphs(ctypes.byref(c), ctypes.byref(r), 1 if reset else 0)
    return c.value, r.value


def sad_quality(colmap, cls, nclass: int):
    """Alignment quality against homology classes (include/sad.h): returns
    (aligned_pairs, true_pairs) for device int32 tensors colmap and cls of one
    length; Q = aligned / true."""
    total = int(colmap.numel())
    if int(cls.numel()) != total:
        raise ValueError("colmap and class ids differ in length")
    if colmap.dtype != torch.int32 or cls.dtype != torch.int32:
        raise ValueError("colmap and class ids must be int32")
    a, t = ctypes.c_uint64(0), ctypes.c_uint64(0)
    code = lib().sad_quality(_ptr(colmap.contiguous()) if total else None,
                             _ptr(cls.contiguous()) if total else None, total, int(nclass),
                             ctypes.byref(a), ctypes.byref(t), _stream())
    _check(code, "sad_quality")
    return a.value, t.value


def sad_profile_jobs():
    """Per-job records of the last profiled engine launch, an (n, 8) int64
    array: W1, W2, ops, fetch, start, DP end, traceback end, merge end (ns)."""
    import numpy as np
    n = ctypes.c_int64(0)
    lib().sad_profile_jobs(None, 0, ctypes.byref(n))
    out = np.zeros((n.value, 8), np.int64)
    if n.value:
        lib().sad_profile_jobs(out.ctypes.data_as(ctypes.c_void_p), n.value, ctypes.byref(n))
    return out


def sad_version() -> str:
    return lib().sad_version().decode()


def sad_release() -> None:
    lib().sad_release()
