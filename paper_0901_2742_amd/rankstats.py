"""Centralised vs globalised k-mer rank (Section 2.3.1, Table 1, Figs. 1 and 3).

Host-side statistics over two rank vectors that the library computed on the
GPU (``sad_rank_against`` with all N sequences as the sample, and
``sad_kmer_rank`` against its k p samples).  Each rank is taken as the mean F
over its samples, K / (S 2^31), which lies in [0, 1]; the paper does not say
how its printed values were scaled."""
from __future__ import annotations

import numpy as np


def rank_stats(central, globalised, n_samples_central: int, n_samples_global: int,
               bins: int = 20) -> dict:
    """Maximum, minimum and mean of each rank, the mean squared difference of
    the globalised rank from the centralised one and its square root (the
    "variance / standard deviation w.r.t. centralised" rows of Table 1), and
    both histograms over ``bins`` equal bins of [0, 1]."""
    if n_samples_central <= 0 or n_samples_global <= 0:
        raise ValueError("sample counts must be positive")
    c = np.asarray(central, np.float64) / (float(n_samples_central) * 2.0 ** 31)
    g = np.asarray(globalised, np.float64) / (float(n_samples_global) * 2.0 ** 31)
    if c.shape != g.shape or c.size == 0:
        raise ValueError("need two non-empty rank vectors of one length")
    edges = np.linspace(0.0, 1.0, bins + 1)
    var = float(np.mean((g - c) ** 2))
    return {
        "central": {"max": float(c.max()), "min": float(c.min()), "mean": float(c.mean())},
        "global": {"max": float(g.max()), "min": float(g.min()), "mean": float(g.mean())},
        "var_wrt_central": var,
        "std_wrt_central": float(np.sqrt(var)),
        "hist_edges": edges.tolist(),
        "hist_central": np.histogram(c, edges)[0].tolist(),
        "hist_global": np.histogram(g, edges)[0].tolist(),
    }
