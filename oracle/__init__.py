"""FP64 CPU oracle for the 2D-surfel sensor renderer.

TEST INFRASTRUCTURE ONLY: a plain, slow, obviously-correct reference of what
the renderer computes.  Only tests, the smoke check and the benchmark's CPU
baseline leg may import it.  The product path (paper_2503_11731_amd) never
imports, calls or links anything here, and this package shares no code with
it: the two meet only through the seeded input generators in gen/.

Modules:
  spec32  FP32 binning specification (visibility, rectangles, depth key)
  sh      real spherical-harmonic basis (FP64, differentiable)
  raster  per-ray FP64 compositing for pinhole and LiDAR, gradients by autograd
  decode  neural-Gaussian MLP decode (FP64 on bf16 operands)
"""
from . import spec32, sh, raster  # noqa: F401
