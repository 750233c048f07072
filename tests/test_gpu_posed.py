"""Posed actor groups (scene assembly, Sec. III-B "Gaussian Inplacing": each
inserted actor carries its own model matrix) rendered on the GPU vs the FP64
oracle.

The scene holds a static group at the identity pose and three actor groups
with full 3D rotations and translations; the camera itself is posed.  This
covers the composition V_s G_g of every group (not only group 0), the group
lookup of every surfel, and view-dependent SH colour evaluated in the actor's
own frame.  Pair lists are compared bit for bit; floats per pixel (with the
near-threshold alternatives of the oracle); gradients at 1e-3 of the largest
reference entry per tensor.
"""
import sys

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

pytestmark = pytest.mark.gpu

from gen import scenes as S  # noqa: E402
from oracle import raster  # noqa: E402
from tests.gpu_common import (ALT_TOL, assert_verified, check_integer_parity, gmap_of, gpu_render, oracle_opts,  # noqa: E402
                              quiet_median,
                              verify)
from tests.helpers import F32  # noqa: E402

import paper_2503_11731_amd as gs  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def posed_scene(seed, n_static=1500, n_actor=500, sh_degree=3, lidar=False):
    """A static cloud plus three actor clouds, each in its own frame, placed by rotations and translations."""
    rng = np.random.default_rng(seed)
    parts, poses = [], []
    static = S.random_cloud(seed=seed, n=n_static, lo=(-3, -2, 4), hi=(3, 2, 12), log_scale=(-2.7, 0.4),
                            with_intensity=lidar)
    parts.append(static)
    poses.append(np.concatenate([np.eye(3), np.zeros((3, 1))], 1))
    for k in range(3):
        a = S.random_cloud(seed=seed + 1 + k, n=n_actor, lo=(-0.8, -0.5, -0.8), hi=(0.8, 0.5, 0.8),
                           log_scale=(-3.0, 0.3), with_intensity=lidar)
        parts.append(a)
        R = Rotation.from_euler("xyz", rng.uniform(-180, 180, 3), degrees=True).as_matrix()
        t = np.array([rng.uniform(-1.5, 1.5), rng.uniform(-0.8, 0.8), rng.uniform(4.0, 7.0)])
        poses.append(np.concatenate([R, t[:, None]], 1))
    n = sum(p.n for p in parts)
    scene = dict(mean=np.concatenate([p.mean for p in parts], 1), quat=np.concatenate([p.quat for p in parts], 1),
                 scale=np.concatenate([p.scale for p in parts], 1),
                 opacity=np.concatenate([p.opacity for p in parts]),
                 group_offsets=np.cumsum([0] + [p.n for p in parts]).astype(np.int32),
                 group_poses=np.stack(poses).astype(F32))
    if lidar:
        scene["intensity"] = np.concatenate([p.intensity for p in parts])
    elif sh_degree >= 0:
        scene["sh"] = (0.3 * rng.standard_normal(((sh_degree + 1) ** 2 * 3, n))).astype(F32)
        scene["sh_degree"] = sh_degree
    else:
        scene["rgb"] = np.concatenate([p.rgb for p in parts], 1)
    return scene


def _camera():
    pose = S.camera_yaw_pose(12.0).astype(np.float64)
    pose[:, 3] = [0.2, -0.1, 0.4]
    return S.pinhole(192, 128, 140.0, pose=pose)


@pytest.mark.parametrize("mode", ["production", "strict"])
@pytest.mark.parametrize("sh_degree", [3, -1])
def test_posed_groups_forward_parity(mode, sh_degree):
    _say(f"posed groups forward {mode} sh {sh_degree}")
    scene = posed_scene(21, sh_degree=sh_degree)
    cam = _camera()
    opts = gs.PRODUCTION if mode == "production" else gs.STRICT
    tile = (32, 8)
    r, st, sp, gp, outs = gpu_render(scene, [cam], opts, tiles=tile)
    o = oracle_opts(opts, tile)
    n_pairs = check_integer_parity(r, scene, cam, o)
    ref = raster.render(scene, cam, o, alternatives=ALT_TOL)
    v = verify(outs[0].cpu().numpy(), ref, "pinhole")
    # every actor group is seen
    g = np.repeat(np.arange(4), np.diff(scene["group_offsets"]))
    seen = np.unique(g[ref["bins"]["touch"]])
    _say(f"  pairs {n_pairs} groups seen {seen.tolist()} {v}")
    assert seen.tolist() == [0, 1, 2, 3]
    assert_verified(v)


def test_posed_groups_lidar_forward_parity():
    _say("posed groups lidar")
    scene = posed_scene(23, lidar=True)
    L = S.lidar_spinning(n_beams=32, n_az=360, pose=np.concatenate([np.eye(3), np.zeros((3, 1))], 1))
    # LiDAR frame (x forward, z up): tip the scene so that the actors sit in front of the sensor
    Rz = np.array([[0, 0, 1], [-1, 0, 0], [0, -1, 0]], np.float64)
    L["pose"] = np.concatenate([Rz, np.zeros((3, 1))], 1).astype(F32)
    r, st, sp, gp, outs = gpu_render(scene, [L], gs.PRODUCTION, tiles=(32, 8))
    o = oracle_opts(gs.PRODUCTION, (32, 8))
    check_integer_parity(r, scene, L, o)
    ref = raster.render(scene, L, o, alternatives=ALT_TOL)
    v = verify(outs[0].cpu().numpy(), ref, "lidar")
    _say(f"  {v}")
    assert_verified(v)


@pytest.mark.parametrize("sh_degree", [3, -1])
def test_posed_groups_backward_parity(sh_degree):
    _say(f"posed groups backward sh {sh_degree}")
    scene = posed_scene(25, n_static=300, n_actor=120, sh_degree=sh_degree)
    cam = S.pinhole(96, 72, 80.0, pose=_camera()["pose"])
    tile = (16, 16)
    r, st, sp, gp, outs = gpu_render(scene, [cam], gs.PRODUCTION, tiles=tile)
    rng = np.random.default_rng(9)
    go = rng.standard_normal(tuple(outs[0].shape)).astype(np.float32)
    quiet_median(go, scene, cam, oracle_opts(gs.PRODUCTION, tile))
    grads = r.backward([st], sp, gp, outs, [torch.from_numpy(go).to(outs[0].device)])[0]
    torch.cuda.synchronize()
    gmap = gmap_of(go, "pinhole")
    ref = raster.render(scene, cam, oracle_opts(gs.PRODUCTION, tile),
                        grad_out={k: v.astype(np.float64) for k, v in gmap.items()})
    keys = ["mean", "quat", "scale", "opacity", "sh" if sh_degree >= 0 else "rgb"]
    for k in keys:
        g = grads[k].cpu().numpy().astype(np.float64)
        gr = ref["grads"][k]
        err, scale = float(np.abs(g - gr).max()), float(np.abs(gr).max())
        _say(f"  {k}: err {err:.3e} scale {scale:.3e}")
        assert err <= 1e-3 * scale + 1e-6, (k, err, scale)
    # actor surfels receive gradient (their group's pose was used)
    off = scene["group_offsets"]
    gm = grads["mean"].abs().sum(0).cpu().numpy()
    for gi in range(1, 4):
        assert gm[off[gi]:off[gi + 1]].max() > 0
