"""Scene builders shared by the tests (plain numpy; no renderer arithmetic)."""
import numpy as np
from scipy.spatial.transform import Rotation

F32 = np.float32


def quat_wxyz(rot: Rotation) -> np.ndarray:
    x, y, z, w = rot.as_quat().T
    return np.stack([w, x, y, z]).astype(F32).reshape(4, -1)


def surfels(mean, quat, scale, opacity, rgb=None, intensity=None, sh=None, sh_degree=-1, drop=None):
    mean = np.asarray(mean, F32).reshape(-1, 3).T.copy()
    n = mean.shape[1]
    sc = dict(mean=mean, quat=np.asarray(quat, F32).reshape(4, n).copy(),
              scale=np.asarray(scale, F32).reshape(-1, 2).T.copy(),
              opacity=np.asarray(opacity, F32).reshape(n).copy(),
              group_offsets=np.array([0, n], np.int32), group_poses=identity_poses(1))
    if rgb is not None:
        sc["rgb"] = np.asarray(rgb, F32).reshape(-1, 3).T.copy()
    if intensity is not None:
        sc["intensity"] = np.asarray(intensity, F32).reshape(n).copy()
    if drop is not None:
        sc["drop"] = np.asarray(drop, F32).reshape(n).copy()
    if sh is not None:
        sc["sh"] = np.asarray(sh, F32).copy()
        sc["sh_degree"] = sh_degree
    return sc


def identity_poses(g):
    p = np.zeros((g, 3, 4), F32)
    p[:, 0, 0] = p[:, 1, 1] = p[:, 2, 2] = 1
    return p


def from_gen(sc):
    """Scene dict from a gen.scenes.SurfelScene."""
    d = dict(mean=sc.mean, quat=sc.quat, scale=sc.scale, opacity=sc.opacity,
             group_offsets=sc.group_offsets, group_poses=sc.group_poses)
    if sc.sh is not None:
        d["sh"] = sc.sh
        d["sh_degree"] = sc.sh_degree
    if sc.rgb is not None:
        d["rgb"] = sc.rgb
    if sc.intensity is not None:
        d["intensity"] = sc.intensity
    if getattr(sc, "drop", None) is not None:
        d["drop"] = sc.drop
    return d


def subset(scene, idx):
    idx = np.asarray(idx)
    out = dict(scene)
    for k in ("mean", "quat", "scale", "rgb", "sh"):
        if k in scene and scene[k] is not None:
            out[k] = np.ascontiguousarray(scene[k][:, idx])
    for k in ("opacity", "intensity", "drop"):
        if k in scene and scene[k] is not None:
            out[k] = np.ascontiguousarray(scene[k][idx])
    out["group_offsets"] = np.array([0, idx.size], np.int32)
    out["group_poses"] = identity_poses(1)
    return out
