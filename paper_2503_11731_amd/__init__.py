"""MI355X-native 2D Gaussian surfel sensor renderer (camera + LiDAR).

Hot path of "Industrial-Grade Sensor Simulation via Gaussian Splatting"
(arXiv 2503.11731), Sec. III-A: neural-Gaussian decode, unified two-plane
projection (Eq. 1-5), tile binning, depth sort, front-to-back compositing and
its adjoint, and the inpainting patch affinity of Sec. III-B (Eq. 6), as
hand-written HIP kernels for gfx950 behind the C-ABI in include/gs2d.h.  This package is the thin Python binding.
"""
from . import _lib  # noqa: F401
from .render import PRODUCTION, STRICT, Renderer, SceneShape, poses_tensor, render, scene_tensors  # noqa: F401
from .decode import Decoder  # noqa: F401
from .inpaint import affinity  # noqa: F401
