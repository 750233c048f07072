"""Seeded synthetic inputs for the 2D-surfel sensor renderer.

This module only *draws* inputs: surfel clouds, neural-Gaussian anchors, MLP
weights, sensor rigs and object poses.  It contains none of the renderer's
arithmetic (no projection, binning, compositing or decoding), so the FP64
oracle and the HIP path can both consume it without sharing method code.

Every array is numpy, C-contiguous, in the structure-of-arrays layout the
renderer reads:

  surfels  mean [3,N] f32 (object frame of its group), quat [4,N] f32 (w,x,y,z),
           scale [2,N] f32 (linear metres), opacity [N] f32 in (0,1),
           rgb [3,N] f32  or  sh [16*3,N] f32 (coefficient-major: row k*3+c),
           group_offsets [G+1] i32, group_poses [G,3,4] f32 (object->world)
  anchors  xyz [3,A] f32, scaling [A] f32, offsets [3,K,A] f32,
           feat_bf16 [A,32] u16 (raw bfloat16 bits), group_offsets [G+1] i32
  mlp      w1 [H,35] f32 (bf16-representable), b1 [H] f32,
           w2 [K*J,H] f32 (bf16-representable), b2 [K*J] f32

The workloads stand in for the paper's driving clips (Para-Lane, Sec. IV),
which are not available: shapes and distributions follow the five benchmark
configurations (256^2 random cloud; 1080p road corridor with SH3 colour;
neural anchors at 720p; 128x1800 LiDAR; 6 cameras + LiDAR with 20 inserted
assets).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

F32 = np.float32

# ----------------------------------------------------------------------------
# small helpers (input preparation only)
# ----------------------------------------------------------------------------


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def bf16_round_bits(x: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round-to-nearest-even); raw u16 bits."""
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16).astype(np.uint16)
    return r


def bf16_bits_to_f32(u: np.ndarray) -> np.ndarray:
    return (np.ascontiguousarray(u, dtype=np.uint16).astype(np.uint32) << 16).view(np.float32)


def bf16_representable(x: np.ndarray) -> np.ndarray:
    return bf16_bits_to_f32(bf16_round_bits(x))


def _quat_from_frames(tu: np.ndarray, tv: np.ndarray, n: np.ndarray) -> np.ndarray:
    """Unit quaternion (w,x,y,z) [4,N] of the rotation whose columns are tu, tv, n.

    Input preparation: the generator builds surfel frames from face geometry and
    stores them as quaternions (Shepperd's branch-on-largest-diagonal method).
    """
    m = np.stack([tu, tv, n], axis=-1).astype(np.float64)  # [N,3,3] columns
    tr = m[:, 0, 0] + m[:, 1, 1] + m[:, 2, 2]
    q = np.empty((m.shape[0], 4))
    c0 = tr > 0
    s = np.sqrt(np.maximum(tr + 1.0, 1e-300)) * 2
    q[c0, 0] = 0.25 * s[c0]
    q[c0, 1] = (m[c0, 2, 1] - m[c0, 1, 2]) / s[c0]
    q[c0, 2] = (m[c0, 0, 2] - m[c0, 2, 0]) / s[c0]
    q[c0, 3] = (m[c0, 1, 0] - m[c0, 0, 1]) / s[c0]
    rest = ~c0
    i1 = rest & (m[:, 0, 0] > m[:, 1, 1]) & (m[:, 0, 0] > m[:, 2, 2])
    s1 = np.sqrt(np.maximum(1.0 + m[:, 0, 0] - m[:, 1, 1] - m[:, 2, 2], 1e-300)) * 2
    q[i1, 0] = (m[i1, 2, 1] - m[i1, 1, 2]) / s1[i1]
    q[i1, 1] = 0.25 * s1[i1]
    q[i1, 2] = (m[i1, 0, 1] + m[i1, 1, 0]) / s1[i1]
    q[i1, 3] = (m[i1, 0, 2] + m[i1, 2, 0]) / s1[i1]
    i2 = rest & ~i1 & (m[:, 1, 1] > m[:, 2, 2])
    s2 = np.sqrt(np.maximum(1.0 + m[:, 1, 1] - m[:, 0, 0] - m[:, 2, 2], 1e-300)) * 2
    q[i2, 0] = (m[i2, 0, 2] - m[i2, 2, 0]) / s2[i2]
    q[i2, 1] = (m[i2, 0, 1] + m[i2, 1, 0]) / s2[i2]
    q[i2, 2] = 0.25 * s2[i2]
    q[i2, 3] = (m[i2, 1, 2] + m[i2, 2, 1]) / s2[i2]
    i3 = rest & ~i1 & ~i2
    s3 = np.sqrt(np.maximum(1.0 + m[:, 2, 2] - m[:, 0, 0] - m[:, 1, 1], 1e-300)) * 2
    q[i3, 0] = (m[i3, 1, 0] - m[i3, 0, 1]) / s3[i3]
    q[i3, 1] = (m[i3, 0, 2] + m[i3, 2, 0]) / s3[i3]
    q[i3, 2] = (m[i3, 1, 2] + m[i3, 2, 1]) / s3[i3]
    q[i3, 3] = 0.25 * s3[i3]
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.T.astype(F32)


def _sigmoid(x):
    return 1.0 / (1.0 + np.exp(-x))


# ----------------------------------------------------------------------------
# sensors and poses
# ----------------------------------------------------------------------------


def pinhole(width: int, height: int, f: float, pose=None, cx=None, cy=None, z_near=0.2) -> dict:
    """Pinhole camera: x right, y down, z forward; pose is world->camera [3,4]."""
    if pose is None:
        pose = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    return dict(kind="pinhole", width=int(width), height=int(height),
                fx=float(f), fy=float(f),
                cx=float(width / 2 if cx is None else cx),
                cy=float(height / 2 if cy is None else cy),
                z_near=float(z_near), pose=np.asarray(pose, dtype=F32).reshape(3, 4).copy())


def cylindrical(width: int, height: int, hfov_deg: float, pose=None, z_near=0.2) -> dict:
    """Cylindrical (fisheye) camera: columns span hfov_deg about the camera's y
    axis (f_x pixels per radian), rows are heights on the unit cylinder with
    f_y = f_x; x right, y down, z forward; pose is world->camera [3,4]."""
    if pose is None:
        pose = np.concatenate([np.eye(3), np.zeros((3, 1))], axis=1)
    f = float(width) / math.radians(hfov_deg)
    return dict(kind="cylindrical", width=int(width), height=int(height), fx=f, fy=f,
                cx=float(width / 2), cy=float(height / 2), z_near=float(z_near),
                pose=np.asarray(pose, dtype=F32).reshape(3, 4).copy())


def lidar_spinning(n_beams=128, n_az=1800, el_min_deg=-25.0, el_max_deg=15.0, pose=None,
                   z_near=0.5) -> dict:
    """Spinning LiDAR: x forward, y left, z up; beams uniform in elevation.

    Rows of the range image are beams (ascending elevation), columns are
    azimuth steps az_i = az0 + 2*pi*i/n_az (counter-clockwise about +z).
    """
    el = np.deg2rad(np.linspace(el_min_deg, el_max_deg, n_beams, dtype=np.float64))
    if pose is None:
        pose = lidar_rig_pose()
    return dict(kind="lidar", width=int(n_az), height=int(n_beams), elevations=el, az0=0.0,
                z_near=float(z_near), pose=np.asarray(pose, dtype=F32).reshape(3, 4).copy())


def lidar_rig_pose() -> np.ndarray:
    """world->LiDAR: LiDAR at world (0,-0.3,0); LiDAR x=world +z, y=world -x, z=world -y."""
    r = np.array([[0, 0, 1], [-1, 0, 0], [0, -1, 0]], dtype=np.float64)
    o = np.array([0.0, -0.3, 0.0])
    t = -r @ o
    return np.concatenate([r, t[:, None]], axis=1).astype(F32)


def camera_yaw_pose(yaw_deg: float) -> np.ndarray:
    """world->camera for a camera at the origin turned by yaw about world -y (up).

    Positive yaw turns the optical axis towards world -x (to the left).
    """
    a = math.radians(yaw_deg)
    # camera axes expressed in world coordinates
    fwd = np.array([-math.sin(a), 0.0, math.cos(a)])
    right = np.array([math.cos(a), 0.0, math.sin(a)])
    down = np.array([0.0, 1.0, 0.0])
    r = np.stack([right, down, fwd])  # rows: world->camera
    return np.concatenate([r, np.zeros((3, 1))], axis=1).astype(F32)


def yaw_translate_pose(yaw: float, tx: float, ty: float, tz: float) -> np.ndarray:
    """object->world: rotation about world y by yaw, then translation."""
    c, s = math.cos(yaw), math.sin(yaw)
    r = np.array([[c, 0, s], [0, 1, 0], [-s, 0, c]])
    return np.concatenate([r, np.array([[tx], [ty], [tz]])], axis=1).astype(F32)


# ----------------------------------------------------------------------------
# corridor geometry: rectangles (origin, e1, e2) with area-proportional sampling
# ----------------------------------------------------------------------------

GROUND_Y = 1.6  # world y is down; the ground plane sits 1.6 m below the cameras


def _box_faces(x0, x1, y0, y1, z0, z1, bottom=False):
    """Faces of an axis-aligned box as (origin, e1, e2) rectangles."""
    o = np.array
    faces = [
        (o([x0, y0, z0]), o([0, y1 - y0, 0]), o([0, 0, z1 - z0])),  # x = x0
        (o([x1, y0, z0]), o([0, y1 - y0, 0]), o([0, 0, z1 - z0])),  # x = x1
        (o([x0, y0, z0]), o([x1 - x0, 0, 0]), o([0, 0, z1 - z0])),  # y = y0 (top, y down)
        (o([x0, y0, z0]), o([x1 - x0, 0, 0]), o([0, y1 - y0, 0])),  # z = z0
        (o([x0, y0, z1]), o([x1 - x0, 0, 0]), o([0, y1 - y0, 0])),  # z = z1
    ]
    if bottom:
        faces.append((o([x0, y1, z0]), o([x1 - x0, 0, 0]), o([0, 0, z1 - z0])))
    return faces


def _corridor_faces(rng, z_lo, z_hi, n_vehicles=40):
    ground = [(np.array([-12.0, GROUND_Y, z_lo]), np.array([24.0, 0, 0]), np.array([0, 0, z_hi - z_lo]))]
    facades = []
    span = z_hi - z_lo
    n_b = 10 if span <= 130 else int(round(10 * span / 120))
    blen = span / n_b
    for side in (-1, 1):
        for i in range(n_b):
            za = z_lo + i * blen + 1.0
            zb = z_lo + (i + 1) * blen - 1.0
            xa, xb = (12.0, 14.0) if side > 0 else (-14.0, -12.0)
            facades += _box_faces(xa, xb, GROUND_Y - 10.0, GROUND_Y, za, zb)
    vehicles = []
    lanes = [-7.0, -3.5, 3.5, 7.0]
    per_lane = [[] for _ in lanes]
    placed = 0
    tries = 0
    while placed < n_vehicles and tries < 10000:
        tries += 1
        li = int(rng.integers(0, len(lanes)))
        zc = float(rng.uniform(z_lo + 5.0, z_hi - 5.0))
        if any(abs(zc - z) < 6.0 for z in per_lane[li]):
            continue
        per_lane[li].append(zc)
        x = lanes[li]
        vehicles += _box_faces(x - 0.9, x + 0.9, GROUND_Y - 1.5, GROUND_Y, zc - 2.25, zc + 2.25)
        placed += 1
    return ground, facades, vehicles


def _sample_faces(rng, faces, n):
    """Area-proportional points on rectangles; returns pos, unit normal, unit e1-direction."""
    if n == 0:
        z = np.zeros((0, 3))
        return z, z, z
    areas = np.array([np.linalg.norm(np.cross(e1, e2)) for _, e1, e2 in faces])
    idx = rng.choice(len(faces), size=n, p=areas / areas.sum())
    org = np.stack([f[0] for f in faces])[idx]
    e1 = np.stack([f[1] for f in faces])[idx]
    e2 = np.stack([f[2] for f in faces])[idx]
    st = rng.uniform(0.0, 1.0, size=(n, 2))
    pos = org + st[:, :1] * e1 + st[:, 1:] * e2
    nrm = np.cross(e1, e2)
    nrm /= np.linalg.norm(nrm, axis=1, keepdims=True)
    d1 = e1 / np.linalg.norm(e1, axis=1, keepdims=True)
    return pos, nrm, d1


def _frames(rng, nrm, d1, tilt_deg=5.0):
    """Tilt the face normal by N(0, tilt) and spin the tangent frame uniformly."""
    n = nrm.shape[0]
    d2 = np.cross(nrm, d1)
    ang = np.deg2rad(tilt_deg) * rng.standard_normal(n)
    phi = rng.uniform(0, 2 * np.pi, n)
    axis = np.cos(phi)[:, None] * d1 + np.sin(phi)[:, None] * d2
    # Rodrigues rotation of the normal about axis (axis is perpendicular to it)
    nt = np.cos(ang)[:, None] * nrm + np.sin(ang)[:, None] * np.cross(axis, nrm)
    nt /= np.linalg.norm(nt, axis=1, keepdims=True)
    a = d1 - np.sum(d1 * nt, axis=1, keepdims=True) * nt
    a /= np.linalg.norm(a, axis=1, keepdims=True)
    b = np.cross(nt, a)
    th = rng.uniform(0, 2 * np.pi, n)
    tu = np.cos(th)[:, None] * a + np.sin(th)[:, None] * b
    tv = np.cross(nt, tu)
    return tu, tv, nt


def corridor_points(rng, n, z_lo=0.0, z_hi=120.0, n_vehicles=40, jitter=0.02):
    """Points on a road corridor: ground 60 %, facades 30 %, vehicles 10 %.

    Returns pos [n,3], tu [n,3], tv [n,3], normal [n,3] (world frame: x right,
    y down, z forward).
    """
    ground, facades, vehicles = _corridor_faces(rng, z_lo, z_hi, n_vehicles)
    n_g = int(round(0.6 * n))
    n_f = int(round(0.3 * n))
    n_v = n - n_g - n_f
    parts = [_sample_faces(rng, ground, n_g), _sample_faces(rng, facades, n_f),
             _sample_faces(rng, vehicles, n_v)]
    pos = np.concatenate([p[0] for p in parts])
    nrm = np.concatenate([p[1] for p in parts])
    d1 = np.concatenate([p[2] for p in parts])
    perm = rng.permutation(n)
    pos, nrm, d1 = pos[perm], nrm[perm], d1[perm]
    tu, tv, nt = _frames(rng, nrm, d1)
    pos = pos + jitter * rng.standard_normal((n, 1)) * nt
    return pos, tu, tv, nt


def vehicle_asset_points(rng, n):
    """Points on a 4.5 x 1.5 x 1.8 m box in its own frame (origin at the ground centre)."""
    faces = _box_faces(-0.9, 0.9, -1.5, 0.0, -2.25, 2.25)
    pos, nrm, d1 = _sample_faces(rng, faces, n)
    tu, tv, nt = _frames(rng, nrm, d1)
    pos = pos + 0.01 * rng.standard_normal((n, 1)) * nt
    return pos, tu, tv, nt


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------


@dataclass
class SurfelScene:
    mean: np.ndarray
    quat: np.ndarray
    scale: np.ndarray
    opacity: np.ndarray
    rgb: np.ndarray | None = None
    sh: np.ndarray | None = None
    sh_degree: int = -1
    intensity: np.ndarray | None = None
    drop: np.ndarray | None = None      # LiDAR ray-drop probability per surfel
    group_offsets: np.ndarray = field(default_factory=lambda: np.zeros(2, np.int32))
    group_poses: np.ndarray = field(default_factory=lambda: np.zeros((1, 3, 4), F32))

    @property
    def n(self) -> int:
        return int(self.mean.shape[1])


def _identity_poses(g=1):
    p = np.zeros((g, 3, 4), F32)
    p[:, 0, 0] = p[:, 1, 1] = p[:, 2, 2] = 1
    return p


def random_cloud(seed=1, n=4096, lo=(-2, -2, 3), hi=(2, 2, 8), log_scale=(-3.0, 0.5),
                 opacity_logit=(0.0, 1.0), with_intensity=False) -> SurfelScene:
    """Uniform random surfels in a box with random orientations and RGB colour."""
    rng = _rng(seed)
    mean = rng.uniform(lo, hi, size=(n, 3)).T.astype(F32)
    ls = rng.normal(log_scale[0], log_scale[1], size=(2, n))
    q = rng.standard_normal((4, n))
    q /= np.linalg.norm(q, axis=0, keepdims=True)
    op = _sigmoid(rng.normal(opacity_logit[0], opacity_logit[1], size=n))
    rgb = rng.uniform(0, 1, size=(3, n))
    sc = SurfelScene(mean=np.ascontiguousarray(mean), quat=q.astype(F32),
                     scale=np.exp(ls).astype(F32), opacity=op.astype(F32), rgb=rgb.astype(F32),
                     sh_degree=-1, group_offsets=np.array([0, n], np.int32),
                     group_poses=_identity_poses(1))
    if with_intensity:
        sc.intensity = rng.uniform(0, 1, size=n).astype(F32)
        # ray drop: most surfels return, a few (dark, specular, far) mostly do not
        sc.drop = (rng.uniform(0, 1, size=n) ** 3).astype(F32)
    return sc


def corridor_surfels(seed=2, n=1_000_000, sh_degree=3, z_lo=0.0, z_hi=120.0,
                     log_scale=(-2.5, 0.4), opacity_logit=(2.0, 1.0), sh_std=0.2,
                     with_intensity=False) -> SurfelScene:
    """Explicit surfels on the synthetic road corridor with SH colour."""
    rng = _rng(seed)
    pos, tu, tv, nt = corridor_points(rng, n, z_lo, z_hi)
    q = _quat_from_frames(tu, tv, nt)
    ls = rng.normal(log_scale[0], log_scale[1], size=(2, n))
    op = _sigmoid(rng.normal(opacity_logit[0], opacity_logit[1], size=n))
    sc = SurfelScene(mean=np.ascontiguousarray(pos.T.astype(F32)), quat=q,
                     scale=np.exp(ls).astype(F32), opacity=op.astype(F32),
                     group_offsets=np.array([0, n], np.int32), group_poses=_identity_poses(1))
    if sh_degree >= 0:
        nb = (sh_degree + 1) ** 2
        sc.sh = rng.standard_normal(size=(nb * 3, n), dtype=np.float32)
        sc.sh *= F32(sh_std)
        sc.sh_degree = sh_degree
    else:
        sc.rgb = rng.uniform(0, 1, size=(3, n)).astype(F32)
    if with_intensity:
        sc.intensity = rng.uniform(0, 1, size=n).astype(F32)
        # ray drop: most surfels return, a few (dark, specular, far) mostly do not
        sc.drop = (rng.uniform(0, 1, size=n) ** 3).astype(F32)
    return sc


@dataclass
class AnchorScene:
    xyz: np.ndarray          # [3,A]
    scaling: np.ndarray      # [A]
    offsets: np.ndarray      # [3,K,A]
    feat_bf16: np.ndarray    # [A,32] u16
    group_offsets: np.ndarray
    group_poses: np.ndarray
    mlps: list               # one dict per group: w1,b1,w2,b2 (f32; w bf16-representable)
    sensor_kind: str = "pinhole"

    @property
    def n_anchors(self) -> int:
        return int(self.xyz.shape[1])

    @property
    def k(self) -> int:
        return int(self.offsets.shape[1])


FEAT_DIM = 32
HIDDEN = 32
K_OFFSETS = 10
ATTRS_CAMERA = 10   # opacity, r, g, b, s_u, s_v, qw, qx, qy, qz
ATTRS_LIDAR = 9     # opacity, intensity, s_u, s_v, qw, qx, qy, qz, ray-drop


def mlp_params(rng, n_out, n_in=FEAT_DIM + 3, hidden=HIDDEN) -> dict:
    """Two-layer MLP with torch.nn.Linear's default (Kaiming-uniform, a=sqrt 5) init.

    Weights are rounded to bfloat16 so that they are exact bf16 parameters.
    """
    b1 = 1.0 / math.sqrt(n_in)
    b2 = 1.0 / math.sqrt(hidden)
    w1 = bf16_representable(rng.uniform(-b1, b1, size=(hidden, n_in)).astype(F32))
    bias1 = rng.uniform(-b1, b1, size=hidden).astype(F32)
    w2 = bf16_representable(rng.uniform(-b2, b2, size=(n_out, hidden)).astype(F32))
    bias2 = rng.uniform(-b2, b2, size=n_out).astype(F32)
    return dict(w1=np.ascontiguousarray(w1), b1=bias1, w2=np.ascontiguousarray(w2), b2=bias2)


def _anchor_block(rng, pos, tu, tv, k, scale_log_std=0.2, base=0.1):
    a = pos.shape[0]
    l = (base * np.exp(rng.normal(0.0, scale_log_std, size=a))).astype(F32)
    c = rng.standard_normal((a, k, 2))
    off = c[..., :1] * tu[:, None, :] + c[..., 1:] * tv[:, None, :]  # [A,K,3]
    feat = rng.standard_normal((a, FEAT_DIM)).astype(F32)
    return l, np.ascontiguousarray(off.transpose(2, 1, 0).astype(F32)), bf16_round_bits(feat)


def corridor_anchors(seed=3, n_anchors=50_000, k=K_OFFSETS, sensor_kind="pinhole",
                     z_lo=0.0, z_hi=120.0, n_assets=0, asset_anchors=2_000) -> AnchorScene:
    """Neural-Gaussian anchors on the corridor, plus optional vehicle assets.

    Group 0 is the static scene (identity pose); groups 1..n_assets are
    vehicle-box assets, each with its own MLP and an object->world pose drawn
    as yaw ~ U[0, 2pi), x ~ U[-9, 9], z ~ U[5, 100], standing on the ground.
    """
    rng = _rng(seed)
    n_attr = ATTRS_CAMERA if sensor_kind == "pinhole" else ATTRS_LIDAR
    pos, tu, tv, _ = corridor_points(rng, n_anchors, z_lo, z_hi)
    l, off, feat = _anchor_block(rng, pos, tu, tv, k)
    xyz = [pos.T.astype(F32)]
    ls, offs, feats = [l], [off], [feat]
    mlps = [mlp_params(rng, k * n_attr)]
    poses = [_identity_poses(1)[0]]
    offsets = [0, n_anchors]
    for _ in range(n_assets):
        p, a_tu, a_tv, _ = vehicle_asset_points(rng, asset_anchors)
        la, oa, fa = _anchor_block(rng, p, a_tu, a_tv, k, base=0.03)
        xyz.append(p.T.astype(F32))
        ls.append(la)
        offs.append(oa)
        feats.append(fa)
        mlps.append(mlp_params(rng, k * n_attr))
        poses.append(yaw_translate_pose(rng.uniform(0, 2 * np.pi), rng.uniform(-9, 9), GROUND_Y,
                                        rng.uniform(5, 100)))
        offsets.append(offsets[-1] + asset_anchors)
    return AnchorScene(xyz=np.ascontiguousarray(np.concatenate(xyz, axis=1)),
                       scaling=np.concatenate(ls), offsets=np.ascontiguousarray(np.concatenate(offs, axis=2)),
                       feat_bf16=np.ascontiguousarray(np.concatenate(feats, axis=0)),
                       group_offsets=np.array(offsets, np.int32), group_poses=np.stack(poses).astype(F32),
                       mlps=mlps, sensor_kind=sensor_kind)


# ----------------------------------------------------------------------------
# the five benchmark workloads
# ----------------------------------------------------------------------------


def config1():
    """256x256 pinhole (f=256, centred, identity pose), 4096 random RGB surfels."""
    return random_cloud(seed=1, n=4096), [pinhole(256, 256, 256.0)]


def config2(n=1_000_000):
    """1920x1080 pinhole (f=960), 1M corridor surfels with degree-3 SH colour."""
    return corridor_surfels(seed=2, n=n), [pinhole(1920, 1080, 960.0)]


def config3(n_anchors=50_000):
    """1280x720 pinhole (f=640), 50k anchors x 10 offsets, camera MLP."""
    return corridor_anchors(seed=3, n_anchors=n_anchors), [pinhole(1280, 720, 640.0)]


def config4(n_anchors=200_000):
    """128-beam x 1800-step LiDAR, 200k anchors x 10 on the extended corridor."""
    return (corridor_anchors(seed=4, n_anchors=n_anchors, sensor_kind="lidar", z_lo=-60.0, z_hi=120.0),
            [lidar_spinning()])


CAMERA_RIG = [("front", 0.0, 1920, 1080, 960.0), ("front_left", 55.0, 1920, 1080, 960.0),
              ("front_right", -55.0, 1920, 1080, 960.0), ("rear", 180.0, 1280, 720, 640.0),
              ("rear_left", 125.0, 1280, 720, 640.0), ("rear_right", -125.0, 1280, 720, 640.0)]


def config5(n_anchors=300_000, n_assets=20, asset_anchors=2_000):
    """Six cameras + LiDAR; corridor anchors plus 20 posed vehicle assets.

    Returns (camera anchor scene, lidar anchor scene, sensors): separate camera
    and LiDAR scenes with separate MLPs (Sec. III-A keeps a camera scene and a
    LiDAR scene).  Their static corridor anchors are the same; the vehicle
    assets and their poses are drawn after each scene's MLPs, so the two
    scenes' assets differ.
    """
    cam = corridor_anchors(seed=5, n_anchors=n_anchors, sensor_kind="pinhole", z_lo=-60.0, z_hi=120.0,
                           n_assets=n_assets, asset_anchors=asset_anchors)
    lid = corridor_anchors(seed=5, n_anchors=n_anchors, sensor_kind="lidar", z_lo=-60.0, z_hi=120.0,
                           n_assets=n_assets, asset_anchors=asset_anchors)
    sensors = [pinhole(w, h, f, pose=camera_yaw_pose(yaw)) for _, yaw, w, h, f in CAMERA_RIG]
    sensors.append(lidar_spinning())
    return cam, lid, sensors


def translate_pose(pose: np.ndarray, c) -> np.ndarray:
    """world->sensor pose of a sensor carried by a vehicle moved by c (world)."""
    p = np.asarray(pose, np.float64).reshape(3, 4)
    t = p[:, 3] - p[:, :3] @ np.asarray(c, np.float64)
    return np.concatenate([p[:, :3], t[:, None]], axis=1).astype(F32)


def zone_mlps(seed: int, n_zones: int, sensor_kind="pinhole", k=K_OFFSETS) -> list:
    """One MLP per zone (every zone of a large scene is reconstructed on its own)."""
    rng = _rng(seed)
    n_attr = ATTRS_CAMERA if sensor_kind == "pinhole" else ATTRS_LIDAR
    return [mlp_params(rng, k * n_attr) for _ in range(n_zones)]


def static_and_actors(sc: AnchorScene):
    """Split an anchor scene into its static group (group 0) and its actor groups.

    Returns (static dict(xyz, scaling, offsets, feat), actors dict or None), the
    arrays as stored in the scene (feat as bf16 bits).
    """
    s = int(sc.group_offsets[1])
    static = dict(xyz=np.ascontiguousarray(sc.xyz[:, :s]), scaling=np.ascontiguousarray(sc.scaling[:s]),
                  offsets=np.ascontiguousarray(sc.offsets[:, :, :s]), feat=np.ascontiguousarray(sc.feat_bf16[:s]))
    if len(sc.group_offsets) <= 2:
        return static, None
    actors = dict(xyz=np.ascontiguousarray(sc.xyz[:, s:]), scaling=np.ascontiguousarray(sc.scaling[s:]),
                  offsets=np.ascontiguousarray(sc.offsets[:, :, s:]), feat=np.ascontiguousarray(sc.feat_bf16[s:]),
                  group_offsets=np.asarray(sc.group_offsets[1:], np.int64) - s, mlps=list(sc.mlps[1:]),
                  group_poses=sc.group_poses[1:])
    return static, actors


def zone_scene(sc: AnchorScene, anchors, mlp: dict) -> AnchorScene:
    """The anchor scene a zone renders: the zone's static anchors (ascending ids)
    with the zone's own MLP, followed by every actor group of `sc`."""
    a = np.asarray(anchors, np.int64)
    s = int(sc.group_offsets[1])
    xyz = np.concatenate([sc.xyz[:, a], sc.xyz[:, s:]], 1)
    scaling = np.concatenate([sc.scaling[a], sc.scaling[s:]])
    offsets = np.concatenate([sc.offsets[:, :, a], sc.offsets[:, :, s:]], 2)
    feat = np.concatenate([sc.feat_bf16[a], sc.feat_bf16[s:]], 0)
    goff = np.concatenate([[0], a.size + np.asarray(sc.group_offsets[1:], np.int64) - s]).astype(np.int32)
    return AnchorScene(xyz=np.ascontiguousarray(xyz), scaling=np.ascontiguousarray(scaling),
                       offsets=np.ascontiguousarray(offsets), feat_bf16=np.ascontiguousarray(feat),
                       group_offsets=goff, group_poses=sc.group_poses.copy(), mlps=[mlp] + list(sc.mlps[1:]),
                       sensor_kind=sc.sensor_kind)


def target_features(scene: AnchorScene, seed: int, std=0.1) -> np.ndarray:
    """Perturbed anchor features (bf16 bits) for the training-step target render."""
    rng = _rng(seed)
    f = bf16_bits_to_f32(scene.feat_bf16) + std * rng.standard_normal(scene.feat_bf16.shape).astype(F32)
    return bf16_round_bits(f)
