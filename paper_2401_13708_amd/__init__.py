"""MI355X-native hyperbolic t-SNE gradient (Poincare disk).

The compute path is the C-ABI library ``libhts.so`` (hand-written HIP for
gfx950) declared in ``include/hts.h``; ``paper_2401_13708_amd.hts`` is its
thin Python binding.  Importing the package does not load the library.
"""
__all__ = ["hts", "synth"]
