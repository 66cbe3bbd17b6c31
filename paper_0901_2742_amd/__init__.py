"""Sample-Align-D data-parallel core on MI355X (gfx950).

The four stages of the method (k-mer rank, regular-sampling partition,
independent bucket alignment, ancestor refinement + glue) run in hand-written
HIP kernels behind the C-ABI in ``include/sad.h``; ``binding`` marshals torch
device tensors into it and ``pipeline`` chains the four calls.
"""
__all__ = ["binding", "pipeline", "build"]
