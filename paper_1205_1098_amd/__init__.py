"""Fused FP64 BLAS-1/2 sequences (the Build to Order BLAS kernels) on MI355X.

Submodules:
  bto    -- Python binding of the C entry points in libbto.so
  synth  -- seeded synthetic inputs (SplitMix64)
Importing the package itself loads nothing; ``paper_1205_1098_amd.bto``
loads the HIP library and fails loudly if it has not been built.
"""

__all__ = ["bto", "synth"]
