"""Seeded synthetic inputs for the Sample-Align-D data-parallel core.

This package only *generates inputs* (sequence sets, scoring matrices and the
five workload descriptions).  It contains none of the method's arithmetic, and
it is the only code shared by the CPU oracle's tests and the HIP path's tests
and benchmark.

The paper (Section 4) measured on 2000 *M. acetivorans* proteins and on ROSE
synthetic sets; neither is available here, so family-structured sets evolved
along random trees stand in for them (see ``synth``).
"""
from .rng import SplitMix64
from .matrices import protein_matrix, dna_matrix, load_ncbi_matrix, PROTEIN_ORDER, DNA_ORDER
from .synth import SeqSet, generate, evolve_family
from .configs import CONFIGS, Workload, workload, make_inputs

__all__ = [
    "SplitMix64", "protein_matrix", "dna_matrix", "load_ncbi_matrix",
    "PROTEIN_ORDER", "DNA_ORDER", "SeqSet", "generate", "evolve_family",
    "CONFIGS", "Workload", "workload", "make_inputs",
]
