"""Inpainting patch affinity (Sec. III-B, Eq. 6): thin binding of gs_affinity."""
from __future__ import annotations

import torch

from . import _lib as L


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def affinity(xt: torch.Tensor, xs: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
    """Row softmax of X_T X_S^T over the source anchors, per patch pair.

    xt: [B][P][d] and xs: [B][Q][d] bf16 bit patterns (int16 or uint16 device
    tensors, contiguous); returns FP32 [B][P][Q] (into `out` when given).
    """
    if xt.dim() != 3 or xs.dim() != 3 or xt.shape[0] != xs.shape[0] or xt.shape[2] != xs.shape[2]:
        raise ValueError("affinity expects xt [B][P][d] and xs [B][Q][d]")
    if xt.element_size() != 2 or xs.element_size() != 2:
        raise ValueError("affinity inputs are bf16 bit patterns (16-bit tensors)")
    xt = xt.contiguous()
    xs = xs.contiguous()
    b, p, d = xt.shape
    q = xs.shape[1]
    if out is None:
        out = torch.empty((b, p, q), dtype=torch.float32, device=xt.device)
    elif out.shape != (b, p, q) or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous FP32 [B][P][Q] tensor")
    lib = L.load()
    L.check(lib.gs_affinity(xt.data_ptr(), xs.data_ptr(), b, p, q, d, out.data_ptr(), _stream()))
    return out
