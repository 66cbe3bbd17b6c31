"""Family-structured synthetic sequence sets.

Model (stands in for the ROSE sets and the *M. acetivorans* proteins of the
paper's Section 4, which are not available):

* root: i.i.d. uniform residues over the alphabet;
* tree: a Yule process per family (repeatedly pick a current leaf uniformly and
  replace it by two children, each evolved independently from it) until the
  family has its requested number of leaves;
* one branch: each site is substituted with probability ``p_sub`` by a uniform
  residue (which may equal the old one); then each site draws an indel event
  with probability ``p_indel`` -- insertion or deletion with probability 1/2
  each, length Geometric(mean 2) on {1, 2, ...}.  Events are applied from the
  last site to the first: an insertion adds uniform residues after the site,
  a deletion removes residues starting at the site (clipped at the end);
* a leaf shorter than ``min_len`` is re-drawn from its parent with fresh draws;
* families are concatenated, then shuffled by a seeded permutation.

Every residue carries a homology id (family, root-or-insertion site), so two
residues in the output are truly homologous iff their ids are equal.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

from .rng import SplitMix64


@dataclasses.dataclass
class SeqSet:
    """N sequences as concatenated residue codes plus offsets (N+1)."""
    alphabet: int
    codes: np.ndarray      # uint8 [sum L]
    offsets: np.ndarray    # int64 [N+1]
    family: np.ndarray     # int32 [N]
    homology: np.ndarray   # int64 [sum L]; equal ids = truly homologous residues

    @property
    def n(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def seq(self, i: int) -> np.ndarray:
        return self.codes[self.offsets[i]:self.offsets[i + 1]]

    def homology_classes(self):
        """The homology ids renumbered 0..nclass-1 (int32), and nclass."""
        _, inv = np.unique(self.homology, return_inverse=True)
        inv = inv.astype(np.int32).reshape(-1)
        return inv, int(inv.max()) + 1 if inv.size else 1

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.alphabet).tobytes())
        h.update(np.ascontiguousarray(self.offsets, dtype=np.int64).tobytes())
        h.update(np.ascontiguousarray(self.codes, dtype=np.uint8).tobytes())
        return h.hexdigest()

    def subset(self, ids) -> "SeqSet":
        ids = np.asarray(ids, dtype=np.int64)
        lens = self.lengths[ids]
        offs = np.zeros(len(ids) + 1, dtype=np.int64)
        np.cumsum(lens, out=offs[1:])
        idx = np.concatenate([np.arange(self.offsets[i], self.offsets[i + 1]) for i in ids]) \
            if len(ids) else np.zeros(0, dtype=np.int64)
        return SeqSet(self.alphabet, self.codes[idx].copy(), offs, self.family[ids].copy(),
                      self.homology[idx].copy())

    def to_fasta(self, path: str, letters: str) -> None:
        with open(path, "w", encoding="ascii") as f:
            for i in range(self.n):
                f.write(f">s{i} family={int(self.family[i])}\n")
                s = "".join(letters[c] for c in self.seq(i))
                for k in range(0, len(s), 60):
                    f.write(s[k:k + 60] + "\n")


def _evolve(rng: SplitMix64, seq: np.ndarray, hom: np.ndarray, alphabet: int,
            p_sub: float, p_indel: float, next_id: list) -> tuple:
    """One branch of the mutation model on (residues, homology ids)."""
    L = seq.shape[0]
    seq = seq.copy()
    if L:
        sub = rng.uniform(L) < p_sub
        ns = int(sub.sum())
        if ns:
            seq[sub] = rng.integers(ns, alphabet).astype(np.uint8)
        ev = np.nonzero(rng.uniform(L) < p_indel)[0]
    else:
        ev = np.zeros(0, dtype=np.int64)
    if ev.shape[0] == 0:
        return seq, hom.copy()
    kinds = rng.uniform(ev.shape[0]) < 0.5          # True: insertion
    lens = rng.geometric(ev.shape[0], 2.0)
    pieces_s = []
    pieces_h = []
    end = L
    # apply from the last site to the first, building the result right to left
    for e in range(ev.shape[0] - 1, -1, -1):
        site = int(ev[e])
        ln = int(lens[e])
        if site >= end:
            # a later deletion already removed this site
            continue
        if kinds[e]:
            pieces_s.append(seq[site + 1:end])
            pieces_h.append(hom[site + 1:end])
            ins = rng.integers(ln, alphabet).astype(np.uint8)
            ids = np.arange(next_id[0], next_id[0] + ln, dtype=np.int64)
            next_id[0] += ln
            pieces_s.append(ins)
            pieces_h.append(ids)
            end = site + 1
        else:
            stop = min(end, site + ln)
            pieces_s.append(seq[stop:end])
            pieces_h.append(hom[stop:end])
            end = site
    pieces_s.append(seq[:end])
    pieces_h.append(hom[:end])
    return np.concatenate(pieces_s[::-1]), np.concatenate(pieces_h[::-1])


def evolve_family(rng: SplitMix64, root_len: int, n_leaves: int, alphabet: int,
                  p_sub: float, p_indel: float, min_len: int, fam_id: int):
    """Yule-tree family: returns lists of leaf residue arrays and homology ids."""
    root = rng.integers(root_len, alphabet).astype(np.uint8)
    base = np.int64(fam_id) << np.int64(32)
    hom = base + np.arange(root_len, dtype=np.int64)
    next_id = [int(base) + root_len]
    leaves = [(root, hom)]
    if n_leaves <= 1:
        return [root], [hom]

    def child(par):
        for _ in range(1000):
            s, h = _evolve(rng, par[0], par[1], alphabet, p_sub, p_indel, next_id)
            if s.shape[0] >= min_len:
                return s, h
        raise RuntimeError("could not evolve a leaf of the minimum length")

    while len(leaves) < n_leaves:
        k = rng.integer(len(leaves))
        par = leaves[k]
        leaves[k] = child(par)
        leaves.append(child(par))
    return [l[0] for l in leaves], [l[1] for l in leaves]


def _clip_round(x: np.ndarray, lo: int, hi: int) -> np.ndarray:
    return np.clip(np.rint(x), lo, hi).astype(np.int64)


def root_lengths(rng: SplitMix64, n: int, spec: dict) -> np.ndarray:
    kind = spec["kind"]
    if kind == "fixed":
        return np.full(n, int(spec["value"]), dtype=np.int64)
    if kind == "normal":
        return _clip_round(spec["mean"] + spec["sd"] * rng.normal(n), spec["lo"], spec["hi"])
    if kind == "lognormal":
        return _clip_round(np.exp(np.log(spec["median"]) + spec["sigma"] * rng.normal(n)),
                           spec["lo"], spec["hi"])
    if kind == "uniform_int":
        return spec["lo"] + rng.integers(n, spec["hi"] - spec["lo"] + 1)
    raise ValueError(f"unknown length law {kind}")


def family_sizes(n_total: int, n_fam: int, zipf: float | None, min_size: int = 2) -> np.ndarray:
    """Family sizes summing to n_total: equal split, or Zipf(s) weights with
    largest-remainder rounding and a floor of ``min_size`` per family."""
    if zipf is None:
        w = np.ones(n_fam)
    else:
        w = 1.0 / np.arange(1, n_fam + 1, dtype=np.float64) ** zipf
    free = n_total - min_size * n_fam if zipf is not None else n_total
    floor_ = min_size if zipf is not None else 0
    q = w / w.sum() * free
    base = np.floor(q).astype(np.int64)
    rem = free - int(base.sum())
    order = np.argsort(-(q - base), kind="stable")
    base[order[:rem]] += 1
    return base + floor_


def _family_job(args):
    """One family from its own stream (a worker's unit of work)."""
    seed, f, root_len, size, alphabet, p_sub, p_indel, min_len = args
    frng = SplitMix64(seed).split(1000 + f)
    return evolve_family(frng, root_len, size, alphabet, p_sub, p_indel, min_len, f)


def default_workers() -> int:
    """Worker processes for generating large sets: the host's cores, at most 16
    (SAD_GEN_WORKERS overrides; 1 generates in this process)."""
    import os
    v = os.environ.get("SAD_GEN_WORKERS")
    if v:
        return max(1, int(v))
    return max(1, min(16, os.cpu_count() or 1))


def generate(seed: int, n: int, alphabet: int, n_families: int, root_len: dict,
             p_sub: float, p_indel: float, min_len: int, zipf: float | None = None,
             workers: int | None = None) -> SeqSet:
    """Generates a shuffled family-structured SeqSet (see module docstring).
    Every family draws from a stream of its own, so the result does not depend
    on ``workers`` (families are evolved in that many forked processes when the
    set is large; None: default_workers())."""
    rng = SplitMix64(seed)
    sizes = family_sizes(n, n_families, zipf)
    rl = root_lengths(rng.split(1), n_families, root_len)
    jobs = [(seed, f, int(rl[f]), int(sizes[f]), alphabet, p_sub, p_indel, min_len)
            for f in range(n_families)]
    if workers is None:
        workers = default_workers() if n >= 10000 and n_families > 1 else 1
    workers = min(workers, n_families)
    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers) as pool:
            fam_out = pool.map(_family_job, jobs, chunksize=max(1, n_families // (4 * workers)))
    else:
        fam_out = [_family_job(j) for j in jobs]
    seqs, homs, fams = [], [], []
    for f, (s, h) in enumerate(fam_out):
        seqs.extend(s)
        homs.extend(h)
        fams.extend([f] * len(s))
    perm = rng.split(2).permutation(len(seqs))
    seqs = [seqs[i] for i in perm]
    homs = [homs[i] for i in perm]
    fam = np.asarray(fams, dtype=np.int32)[perm]
    lens = np.array([s.shape[0] for s in seqs], dtype=np.int64)
    offs = np.zeros(len(seqs) + 1, dtype=np.int64)
    np.cumsum(lens, out=offs[1:])
    codes = np.concatenate(seqs).astype(np.uint8) if seqs else np.zeros(0, np.uint8)
    hom = np.concatenate(homs).astype(np.int64) if homs else np.zeros(0, np.int64)
    return SeqSet(alphabet, codes, offs, fam, hom)
