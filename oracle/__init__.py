"""CPU oracle — TEST INFRASTRUCTURE ONLY.

Plain, slow, float64 NumPy definitions of what the SVD-decomposed spatial-aware LUT
method computes, written from the paper (arXiv 2508.16121).  Only ``tests/``, the smoke
check in ``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it.  It
shares no code with the HIP library (``paper_2508_16121_amd``) and never imports it.

Modules:
  lut        2D-LUT reconstruction, decode, bilinear lookup, map upsample, fusion,
             trilinear 3D-LUT lookup, backward, losses
  generator  the factor/map generator (downsample, convolutions, pooling, FC), its
             backward and Adam
  pairs      degrade->restore training pairs for the generator
"""
from . import lut, generator, pairs  # noqa: F401
