"""Neural-Gaussian MLP decode in FP64 -- TEST INFRASTRUCTURE ONLY.

Sec. III-A: surfel attributes are inferred by passing each anchor's feature
through the scene's MLP (anchors organised as in Scaffold-GS; the camera and
LiDAR scenes have different MLPs).  The paper does not size the network; this
reading takes the benchmark's 2-layer MLP, input = [feature (32); unit view
direction from the sensor centre to the anchor, in the anchor group's frame
(3)], hidden 32 with ReLU, output K offsets x J attributes:

  camera  J = 10: opacity, r, g, b, s_u, s_v, q_w, q_x, q_y, q_z
  LiDAR   J = 9 : opacity, intensity, s_u, s_v, q_w, q_x, q_y, q_z, ray-drop

Heads: opacity, colour, intensity = sigmoid(y); scale = l_a * sigmoid(y);
rotation = the raw 4-vector (the renderer normalises quaternions); centre
mu_k = x_a + l_a * O_k.  Surfel n = a * K + k.

Quantisation: features and weights are bfloat16 parameters (exact bf16 values
held in FP32/FP64 here); every other quantity is FP64.
"""
from __future__ import annotations

import numpy as np
import torch

DT = torch.float64


def _t(x, grad=False):
    return torch.as_tensor(np.asarray(x, np.float64), dtype=DT).requires_grad_(grad)


def decode(anchors: dict, mlps: list, group_poses_s: np.ndarray, kind: str, params=None):
    """Decode anchors into an explicit surfel parameter set (FP64 torch tensors).

    anchors: dict with xyz [3,A], scaling [A], offsets [3,K,A], feat [A,32]
    (float values of the bf16 features), group_offsets [G+1].
    mlps: list per group of dict(w1 [H,35], b1 [H], w2 [K*J,H], b2 [K*J]).
    group_poses_s: FP32 sensor<-object poses per group [G,3,4] (the composed
    poses of the binning spec).
    params: optional dict of FP64 leaf tensors replacing the numpy inputs
    (keys xyz, scaling, offsets, feat, and w1_g/b1_g/w2_g/b2_g per group).
    Returns dict mean [3,N], quat [4,N], scale [2,N], opacity [N] and rgb [3,N]
    or intensity [N], with N = A*K.
    """
    p = params or {}
    xyz = p.get("xyz", _t(anchors["xyz"]))
    scaling = p.get("scaling", _t(anchors["scaling"]))
    offsets = p.get("offsets", _t(anchors["offsets"]))
    feat = p.get("feat", _t(anchors["feat"]))
    go = np.asarray(anchors["group_offsets"], np.int64)
    K = offsets.shape[1]
    J = 10 if kind == "pinhole" else 9
    ys = []
    for g in range(len(go) - 1):
        sl = slice(int(go[g]), int(go[g + 1]))
        P = torch.as_tensor(np.asarray(group_poses_s[g], np.float64))
        Rm, t = P[:, :3], P[:, 3]
        cam = -(Rm.T @ t)  # sensor centre in the group's frame
        d = xyz[:, sl] - cam[:, None]
        d = d / torch.linalg.norm(d, dim=0, keepdim=True)
        x = torch.cat([feat[sl].T, d], 0)  # [35, A_g]
        w1 = p.get(f"w1_{g}", _t(mlps[g]["w1"]))
        b1 = p.get(f"b1_{g}", _t(mlps[g]["b1"]))
        w2 = p.get(f"w2_{g}", _t(mlps[g]["w2"]))
        b2 = p.get(f"b2_{g}", _t(mlps[g]["b2"]))
        h = torch.relu(w1 @ x + b1[:, None])
        ys.append(w2 @ h + b2[:, None])  # [K*J, A_g]
    y = torch.cat(ys, 1).reshape(K, J, -1)  # [K, J, A]
    A = y.shape[2]
    sig = torch.sigmoid

    def per_surfel(v):  # [K, A] -> [A*K] with n = a*K + k
        return v.T.reshape(-1)

    out = {}
    out["opacity"] = per_surfel(sig(y[:, 0]))
    if kind == "pinhole":
        out["rgb"] = torch.stack([per_surfel(sig(y[:, 1 + c])) for c in range(3)])
        so = 4
    else:
        out["intensity"] = per_surfel(sig(y[:, 1]))
        so = 2
    out["scale"] = torch.stack([per_surfel(scaling[None, :] * sig(y[:, so + c])) for c in range(2)])
    out["quat"] = torch.stack([per_surfel(y[:, so + 2 + c]) for c in range(4)])
    if kind != "pinhole":
        out["drop"] = per_surfel(sig(y[:, 8]))  # ray-drop probability
    mean = xyz[:, None, :] + scaling[None, None, :] * offsets  # [3, K, A]
    out["mean"] = mean.permute(0, 2, 1).reshape(3, A * K)
    return out
