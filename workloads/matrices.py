"""Integer substitution matrices for the synthetic workloads.

* DNA: match +2 / mismatch -3 over ACGT (fully specified by the nucleotide
  workload).
* Protein: the BLOSUM62 table is not shipped with this repository (no copy is
  available offline, and it is not reproduced from memory).  The protein
  workloads therefore use ``protein_matrix()``: a seeded, symmetric 20x20
  integer matrix with BLOSUM62's shape and value range (diagonal 4..11,
  off-diagonal -4..3, every row's maximum on its diagonal).  The generated
  sequences evolve with uniform substitutions, so no biological matrix is
  "right" for them; the kernels take the matrix as an input and are exact for
  any int8 matrix.  A real NCBI-format matrix file (e.g. BLOSUM62) can be
  loaded with ``load_ncbi_matrix`` and passed instead.
"""
from __future__ import annotations

import hashlib

import numpy as np

from .rng import SplitMix64

# Conventional one-letter residue order of NCBI matrix files; codes 0..19 index it.
PROTEIN_ORDER = "ARNDCQEGHILKMFPSTWYV"
DNA_ORDER = "ACGT"

_PROTEIN_SEED = 0x62B105E
# Off-diagonal value distribution (value, weight): mostly mildly negative.
_OFFDIAG = [(-4, 5), (-3, 22), (-2, 26), (-1, 22), (0, 13), (1, 8), (2, 3), (3, 1)]


def protein_matrix() -> np.ndarray:
    """Seeded symmetric int8 20x20 stand-in matrix (see module docstring)."""
    rng = SplitMix64(_PROTEIN_SEED)
    a = 20
    m = np.zeros((a, a), dtype=np.int64)
    diag = 4 + rng.integers(a, 8)  # 4..11
    vals = np.array([v for v, _ in _OFFDIAG], dtype=np.int64)
    cw = np.cumsum([w for _, w in _OFFDIAG])
    iu = np.triu_indices(a, 1)
    u = rng.integers(len(iu[0]), int(cw[-1]))
    off = vals[np.searchsorted(cw, u, side="right")]
    m[iu] = off
    m = m + m.T
    m[np.arange(a), np.arange(a)] = diag
    out = m.astype(np.int8)
    validate_matrix(out)
    return out


def dna_matrix(match: int = 2, mismatch: int = -3) -> np.ndarray:
    m = np.full((4, 4), mismatch, dtype=np.int8)
    np.fill_diagonal(m, match)
    return m


def validate_matrix(m: np.ndarray) -> None:
    """Checks the properties the method relies on: square, symmetric, int8,
    positive diagonal that holds each row's maximum."""
    m = np.asarray(m)
    if m.ndim != 2 or m.shape[0] != m.shape[1]:
        raise ValueError("substitution matrix must be square")
    if m.dtype != np.int8:
        raise ValueError("substitution matrix must be int8")
    if not np.array_equal(m, m.T):
        raise ValueError("substitution matrix must be symmetric")
    d = np.diag(m).astype(np.int64)
    if (d <= 0).any():
        raise ValueError("diagonal entries must be positive")
    if (m.astype(np.int64).max(axis=1) != d).any():
        raise ValueError("each row's maximum must be on the diagonal")


def load_ncbi_matrix(path: str, order: str = PROTEIN_ORDER) -> np.ndarray:
    """Parses an NCBI-format matrix file (header row of letters, then one row per
    letter) and returns the int8 sub-matrix restricted to ``order``."""
    rows = {}
    header = None
    with open(path, "r", encoding="ascii") as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            parts = line.split()
            if header is None:
                header = parts
                continue
            rows[parts[0]] = [int(v) for v in parts[1:]]
    if header is None:
        raise ValueError("empty matrix file")
    col = {c: k for k, c in enumerate(header)}
    out = np.zeros((len(order), len(order)), dtype=np.int64)
    for i, a in enumerate(order):
        for j, b in enumerate(order):
            out[i, j] = rows[a][col[b]]
    res = out.astype(np.int8)
    if not np.array_equal(res.astype(np.int64), out):
        raise ValueError("matrix entries exceed int8")
    return res


def matrix_sha256(m: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(m, dtype=np.int8).tobytes()).hexdigest()
