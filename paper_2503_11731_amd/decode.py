"""Python binding of the neural-Gaussian decode (MFMA) and its adjoint.

Sec. III-A: each anchor's feature passes through the scene's MLP to give the
2D-Gaussian attributes of its K offsets.  Argument marshalling only; the
decode runs in libgs2d.so.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib as L


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


class Decoder:
    """Anchors + per-group MLPs on the device.

    Tensors: xyz [3,A] f32, scaling [A] f32, offsets [3,K,A] f32,
    feat [A,32] bf16, w1 [G,32,35] bf16, b1 [G,32] f32, w2 [G,K*J,32] bf16,
    b2 [G,K*J] f32.
    """

    def __init__(self, xyz, scaling, offsets, feat, w1, b1, w2, b2, group_offsets, lidar: bool, plain_fp32=False):
        self.lib = L.load()
        self.xyz, self.scaling, self.offsets, self.feat = xyz, scaling, offsets, feat
        self.w1, self.b1, self.w2, self.b2 = w1, b1, w2, b2
        self.group_offsets = [int(x) for x in group_offsets]
        self.lidar = bool(lidar)
        self.K = int(offsets.shape[1])
        self.A = int(xyz.shape[1])
        self.J = 9 if lidar else 10
        self._off = (ctypes.c_int32 * len(self.group_offsets))(*self.group_offsets)
        self.flags = L.GS_DECODE_VALU_FP32 if plain_fp32 else 0

    @classmethod
    def from_gen(cls, sc, device="cuda", feat_bits=None, plain_fp32=False):
        """Build from a gen.scenes.AnchorScene (bf16 features/weights as raw bits)."""
        def bf(bits):
            return torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).view(torch.bfloat16).to(device)

        def bf_from_f32(a):
            u = np.ascontiguousarray(a, np.float32).view(np.uint32)
            return bf((u >> 16).astype(np.uint16))

        t = lambda a: torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(device)
        w1 = torch.stack([bf_from_f32(m["w1"]) for m in sc.mlps])
        w2 = torch.stack([bf_from_f32(m["w2"]) for m in sc.mlps])
        b1 = torch.stack([t(m["b1"]) for m in sc.mlps])
        b2 = torch.stack([t(m["b2"]) for m in sc.mlps])
        fb = sc.feat_bf16 if feat_bits is None else feat_bits
        return cls(t(sc.xyz), t(sc.scaling), t(sc.offsets), bf(fb), w1.contiguous(), b1, w2.contiguous(), b2,
                   sc.group_offsets, sc.sensor_kind != "pinhole", plain_fp32=plain_fp32)

    def _struct(self):
        return L.AnchorSet(self.A, self.K, int(self.lidar), len(self.group_offsets) - 1, self._off,
                           self.xyz.data_ptr(), self.scaling.data_ptr(), self.offsets.data_ptr(),
                           self.feat.data_ptr(), self.w1.data_ptr(), self.b1.data_ptr(), self.w2.data_ptr(),
                           self.b2.data_ptr(), self.flags)

    def new_decoded(self):
        n = self.A * self.K
        dev = self.xyz.device
        e = lambda c: torch.empty((c, n), dtype=torch.float32, device=dev)
        out = dict(mean=e(3), quat=e(4), scale=e(2), opacity=torch.empty(n, dtype=torch.float32, device=dev))
        if self.lidar:
            out["intensity"] = torch.empty(n, dtype=torch.float32, device=dev)
            out["drop"] = torch.empty(n, dtype=torch.float32, device=dev)
        else:
            out["rgb"] = e(3)
        return out

    def forward(self, sensor_pose: torch.Tensor, group_poses: torch.Tensor, out=None) -> dict:
        """Decode for one sensor pose into `out` (new buffers if None).  out["mean"] may be None: the
        centres do not depend on the sensor, and are then not written."""
        out = out or self.new_decoded()
        p = lambda k: L.ptr(out.get(k))
        d = L.Decoded(p("mean"), p("quat"), p("scale"), p("opacity"), p("rgb"), p("intensity"), p("drop"))
        s = self._struct()
        L.check(self.lib.gs_decode_forward(ctypes.byref(s), sensor_pose.data_ptr(), group_poses.data_ptr(),
                                           ctypes.byref(d), _stream()))
        return out

    def scratch_bytes(self) -> int:
        """Bytes of the scratch buffer gs_decode_backward needs (weight-gradient partials)."""
        s = self._struct()
        nb = ctypes.c_size_t()
        L.check(self.lib.gs_decode_scratch_size(ctypes.byref(s), ctypes.byref(nb)))
        return max(int(nb.value), 256)

    def backward(self, sensor_pose, group_poses, grad_in: dict, grads: dict | None = None,
                 noalloc: bool = False, scratch: torch.Tensor | None = None) -> dict:
        """Adjoint (+= into grads).  noalloc: use gs_decode_backward_noalloc, which
        needs no scratch buffer (the library's own per-GPU array holds the
        weight-gradient partials); scratch: a caller buffer of scratch_bytes()
        for gs_decode_backward.  Either way nothing is allocated when grads is
        given."""
        dev = self.xyz.device
        if grads is None:
            z = lambda t: torch.zeros(t.shape, dtype=torch.float32, device=dev)
            grads = dict(xyz=z(self.xyz), scaling=z(self.scaling), offsets=z(self.offsets), feat=z(self.feat),
                         w1=z(self.w1), b1=z(self.b1), w2=z(self.w2), b2=z(self.b2))
        gi = {k: (v.contiguous() if v is not None else None) for k, v in grad_in.items()}
        p = lambda k: L.ptr(gi.get(k))
        d = L.Decoded(p("mean"), p("quat"), p("scale"), p("opacity"), p("rgb"), p("intensity"), p("drop"))
        g = lambda k: L.ptr(grads.get(k))
        ag = L.AnchorGrads(g("xyz"), g("scaling"), g("offsets"), g("feat"), g("w1"), g("b1"), g("w2"), g("b2"))
        s = self._struct()
        if noalloc:
            L.check(self.lib.gs_decode_backward_noalloc(ctypes.byref(s), sensor_pose.data_ptr(),
                                                        group_poses.data_ptr(), ctypes.byref(d), ctypes.byref(ag),
                                                        _stream()))
            return grads
        if scratch is None:
            scratch = torch.empty(self.scratch_bytes(), dtype=torch.uint8, device=dev)
        elif scratch.numel() * scratch.element_size() < self.scratch_bytes():
            raise ValueError("decode scratch buffer too small")
        L.check(self.lib.gs_decode_backward(ctypes.byref(s), sensor_pose.data_ptr(), group_poses.data_ptr(),
                                            ctypes.byref(d), ctypes.byref(ag), scratch.data_ptr(), _stream()))
        return grads
