"""The five synthetic workloads (sizes, mutation laws, k-mer length, bucket
count and scoring) and a helper that materialises their inputs.

Names describe the workload; ``index`` is only used to derive the seed.
"""
from __future__ import annotations

import dataclasses
import functools

import numpy as np

from .matrices import dna_matrix, protein_matrix
from .synth import SeqSet, generate

SEED_BASE = 0x09012742


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    index: int
    n: int
    alphabet: int
    n_families: int
    root_len: dict
    p_sub: float
    p_indel: float
    kmer_k: int
    p: int
    gap_open: int
    gap_extend: int
    zipf: float | None = None
    s_max: int = 1024
    description: str = ""

    @property
    def seed(self) -> int:
        return SEED_BASE + self.index

    def subst(self) -> np.ndarray:
        return protein_matrix() if self.alphabet == 20 else dna_matrix()


CONFIGS = {
    "prot64": Workload(
        name="prot64", index=0, n=64, alphabet=20, n_families=1,
        root_len={"kind": "fixed", "value": 100}, p_sub=0.10, p_indel=0.02,
        kmer_k=3, p=4, gap_open=10, gap_extend=1,
        description="64 proteins, one family, root length 100, 4 buckets"),
    "prot2000": Workload(
        name="prot2000", index=1, n=2000, alphabet=20, n_families=8,
        root_len={"kind": "normal", "mean": 316, "sd": 60, "lo": 100, "hi": 600},
        p_sub=0.10, p_indel=0.02, kmer_k=3, p=16, gap_open=10, gap_extend=1,
        description="2000 proteins (8 families x 250), mean root length 316, 16 buckets"),
    "prot20k": Workload(
        name="prot20k", index=2, n=20000, alphabet=20, n_families=64,
        root_len={"kind": "lognormal", "median": 300, "sigma": 0.4, "lo": 50, "hi": 1500},
        p_sub=0.10, p_indel=0.02, kmer_k=3, p=128, gap_open=10, gap_extend=1, zipf=1.2,
        description="20000 proteins, 64 Zipf(1.2)-sized families, 128 buckets"),
    "dna50k": Workload(
        name="dna50k", index=3, n=50000, alphabet=4, n_families=32,
        root_len={"kind": "uniform_int", "lo": 800, "hi": 1200},
        p_sub=0.05, p_indel=0.01, kmer_k=8, p=256, gap_open=5, gap_extend=2,
        description="50000 DNA sequences (32 families), lengths 800-1200, k=8, 256 buckets"),
    "prot200k": Workload(
        name="prot200k", index=4, n=200000, alphabet=20, n_families=512,
        root_len={"kind": "normal", "mean": 316, "sd": 80, "lo": 60, "hi": 1000},
        p_sub=0.15, p_indel=0.02, kmer_k=3, p=1024, gap_open=10, gap_extend=1,
        description="200000 proteins (512 families), 1024 buckets"),
}


def workload(name: str) -> Workload:
    return CONFIGS[name]


@functools.lru_cache(maxsize=8)
def make_inputs(name: str, n: int | None = None) -> SeqSet:
    """Generates the workload's sequence set (optionally its first ``n`` after
    shuffling, for bounded samples)."""
    w = CONFIGS[name]
    s = generate(w.seed, w.n, w.alphabet, w.n_families, w.root_len, w.p_sub, w.p_indel,
                 min_len=w.kmer_k, zipf=w.zipf)
    if n is not None and n < s.n:
        s = s.subset(np.arange(n))
    return s
