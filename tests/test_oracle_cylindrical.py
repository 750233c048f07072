"""Pins of the cylindrical (fisheye) camera of Eq. 4 in the oracle (CPU only).

Column i looks at the horizontal angle phi = (i + 1/2 - c_x) / f_x about the
camera's y axis and row j at height y_n = (j + 1/2 - c_y) / f_y on the unit
cylinder, so its ray runs along (sin phi, y_n, cos phi).  The pins below fix,
independently of the oracle's two-plane solve:
  - both planes of Eq. 4 (as read: h_u = (cos phi, 0, -sin phi), h_v =
    (y_n sin phi, -1, y_n cos phi)) contain the ray and are orthogonal;
  - the column at phi = 0 is the pinhole column x_n = 0 (same rays, same
    depth), so it reproduces the independently pinned pinhole renderer;
  - a surfel facing the camera on a pixel's ray gives alpha = o there and
    depth = its cylindrical radius;
  - the FP32 pixel rectangle is conservative (brute force = culled), also
    for a wide field of view with surfels behind the camera;
  - the analytic gradient matches central differences;
  - moving the asset or the camera by the same rigid motion changes nothing.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import raster, spec32
from tests.helpers import F32, quat_wxyz, surfels

IDPOSE = np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(F32)


def cyl(width=96, height=40, fx=30.0, fy=30.0, cx=None, cy=None, z_near=0.2, pose=IDPOSE):
    return dict(kind="cylindrical", width=width, height=height, fx=fx, fy=fy,
                cx=width / 2 if cx is None else cx, cy=height / 2 if cy is None else cy, z_near=z_near,
                pose=np.asarray(pose, F32))


def _scene(seed, n, r=(2.5, 7.0), phi=(-1.4, 1.4), yn=(-0.5, 0.5), logs=(-2.3, 0.4), sh_degree=-1):
    rng = np.random.default_rng(seed)
    rr = rng.uniform(*r, n)
    ph = rng.uniform(*phi, n)
    mean = np.stack([rr * np.sin(ph), rr * rng.uniform(*yn, n), rr * np.cos(ph)], 1)
    q = quat_wxyz(Rotation.random(n, random_state=seed))
    s = np.exp(rng.normal(logs[0], logs[1], (n, 2)))
    o = 1 / (1 + np.exp(-rng.normal(0.5, 1.5, n)))
    if sh_degree >= 0:
        return surfels(mean, q, s, o, sh=rng.normal(0, 0.3, ((sh_degree + 1) ** 2 * 3, n)), sh_degree=sh_degree)
    return surfels(mean, q, s, o, rgb=rng.uniform(0, 1, (n, 3)))


def test_planes_contain_the_ray_and_are_orthogonal():
    C = cyl()
    rays = raster._rays(C, np.arange(C["width"] * C["height"]))
    tabs = spec32.cylindrical_tables(C)
    i = np.arange(C["width"] * C["height"]) % C["width"]
    j = np.arange(C["width"] * C["height"]) // C["width"]
    phi = (i + 0.5 - C["cx"]) / C["fx"]
    yn = (j + 0.5 - C["cy"]) / C["fy"]
    d = np.stack([np.sin(phi), yn, np.cos(phi)], 1)
    hu, hv = rays["hu"].numpy(), rays["hv"].numpy()
    for a, b in ((hu, d), (hv, d), (hu, hv)):
        assert np.abs((a * b).sum(1)).max() < 1e-13
    np.testing.assert_allclose(np.arctan2(tabs["sin_phi"], tabs["cos_phi"]),
                               (np.arange(C["width"]) + 0.5 - C["cx"]) / C["fx"], atol=1e-13)


def test_centre_column_equals_the_pinhole_column():
    # c_x = i0 + 1/2 puts phi = 0 exactly on column i0: its rays are the pinhole
    # rays (0, y_n, 1) and the cylindrical depth of their hits is z.  Depths are
    # spaced so that the two depth keys (mu_z, mu_x^2 + mu_z^2) order alike.
    n, i0 = 40, 11
    rng = np.random.default_rng(8)
    z = 2.5 + 0.1 * np.arange(n) + rng.uniform(0, 0.02, n)
    mean = np.stack([rng.uniform(-0.25, 0.25, n), rng.uniform(-0.4, 0.4, n), z], 1)
    q = quat_wxyz(Rotation.random(n, random_state=3))
    sc = surfels(mean, q, np.exp(rng.normal(-2.0, 0.3, (n, 2))), rng.uniform(0.2, 0.8, n),
                 rgb=rng.uniform(0, 1, (n, 3)))
    C = cyl(width=24, height=30, fx=32.0, fy=32.0, cx=i0 + 0.5, cy=15.0)
    P = dict(kind="pinhole", width=24, height=30, fx=32.0, fy=32.0, cx=i0 + 0.5, cy=15.0, z_near=0.2, pose=IDPOSE)
    opts = raster.make_opts(raster.STRICT, lowpass=False, tile_w=8, tile_h=8)
    a = raster.render(sc, C, opts)
    b = raster.render(sc, P, opts)
    assert a["alpha"][:, i0].max() > 0.3
    for ch in ("rgb", "normal"):
        np.testing.assert_allclose(a[ch][:, :, i0], b[ch][:, :, i0], atol=1e-12)
    for ch in ("depth", "alpha", "T_final"):
        np.testing.assert_allclose(a[ch][:, i0], b[ch][:, i0], atol=1e-12)


@pytest.mark.parametrize("i,j,r", [(70, 12, 4.0), (10, 30, 6.5), (48, 20, 3.0)])
def test_facing_surfel_on_a_pixel_ray(i, j, r):
    C = cyl()
    tabs = spec32.cylindrical_tables(C)
    d = np.array([tabs["sin_phi"][i], tabs["yn"][j], tabs["cos_phi"][i]])
    nrm = d / np.linalg.norm(d)
    tu = np.cross([0, 1.0, 0], nrm)
    tu /= np.linalg.norm(tu)
    tv = np.cross(nrm, tu)
    q = quat_wxyz(Rotation.from_matrix(np.stack([tu, tv, nrm], 1)))
    sc = surfels([r * d], q, [0.1, 0.1], [0.7], rgb=[0.2, 0.5, 0.9])
    out = raster.render(sc, C, raster.make_opts())
    mu = sc["mean"][:, 0].astype(np.float64)
    o = float(F32(0.7))
    assert out["alpha"][j, i] == pytest.approx(o, rel=1e-6)
    assert out["depth"][j, i] / out["alpha"][j, i] == pytest.approx(math.hypot(mu[0], mu[2]), rel=1e-6)
    np.testing.assert_allclose(out["rgb"][:, j, i] / out["alpha"][j, i], sc["rgb"][:, 0].astype(np.float64),
                               rtol=1e-6)


@pytest.mark.parametrize("strict", [False, True])
def test_brute_force_equals_culled(strict):
    C = cyl()
    sc = _scene(3, 150)
    opts = raster.make_opts(raster.STRICT if strict else raster.PRODUCTION, tile_w=8, tile_h=8)
    a = raster.render(sc, C, opts, mode="brute")
    b = raster.render(sc, C, opts, mode="culled")
    for ch in ("rgb", "depth", "normal", "alpha", "T_final"):
        np.testing.assert_array_equal(a[ch], b[ch])
    assert a["alpha"].max() > 0.5


def test_wide_field_of_view_with_surfels_all_around():
    # 270 degrees of columns; surfels all around the camera, some straddling
    # the back (phi = +-pi), where the rectangle takes every column
    C = cyl(width=144, height=24, fx=144 / (1.5 * math.pi), fy=20.0)
    sc = _scene(5, 200, phi=(-math.pi, math.pi), yn=(-0.4, 0.4), logs=(-1.2, 0.4))
    opts = raster.make_opts(tile_w=8, tile_h=8)
    b = raster.render(sc, C, opts, mode="culled")
    a = raster.render(sc, C, opts, mode="brute")
    for ch in ("rgb", "depth", "alpha"):
        np.testing.assert_array_equal(a[ch], b[ch])
    bins = b["bins"]
    full = bins["touch"] & (bins["i_lo"] == 0) & (bins["i_hi"] == C["width"] - 1)
    assert full.any() and a["alpha"].max() > 0.5


def test_fd_gradient():
    from tests.test_oracle_grad_sh_decode import FD_OPTS, _fd_check
    C = cyl(width=16, height=12, fx=20.0, fy=20.0)
    rng = np.random.default_rng(6)
    n = 3
    ph = rng.uniform(-0.2, 0.2, n)
    r = rng.uniform(3.0, 3.6, n)
    mean = np.stack([r * np.sin(ph), rng.uniform(-0.1, 0.1, n), r * np.cos(ph)], 1)
    q = quat_wxyz(Rotation.random(n, random_state=2)) * F32(1.2)
    sc = surfels(mean, q, np.exp(rng.normal(-2.0, 0.2, (n, 2))), rng.uniform(0.3, 0.9, n),
                 rgb=rng.uniform(0, 1, (n, 3)))
    _fd_check(sc, C, raster.make_opts(FD_OPTS, tile_w=8, tile_h=4), ["mean", "quat", "scale", "opacity", "rgb"],
              ["rgb", "depth", "normal", "alpha"])


def test_fd_gradient_with_the_lowpass_filter():
    # tiny surfels: the low-pass term decides alpha, the centre the depth
    from tests.test_oracle_grad_sh_decode import _fd_check
    C = cyl(width=16, height=12, fx=20.0, fy=20.0)
    rng = np.random.default_rng(9)
    n = 2
    ph = rng.uniform(-0.2, 0.2, n)
    r = rng.uniform(3.0, 3.6, n)
    mean = np.stack([r * np.sin(ph), rng.uniform(-0.1, 0.1, n), r * np.cos(ph)], 1)
    sc = surfels(mean, quat_wxyz(Rotation.random(n, random_state=4)), np.full((n, 2), 0.01), [0.8, 0.6],
                 rgb=rng.uniform(0, 1, (n, 3)))
    opts = raster.make_opts(raster.STRICT, cutoff2=400.0, tile_w=8, tile_h=4)
    _fd_check(sc, C, opts, ["mean", "quat", "scale", "opacity", "rgb"], ["rgb", "depth", "alpha"])


def test_rigid_invariance_group_pose_vs_sensor_pose():
    sc = _scene(6, 80, sh_degree=2)
    G = np.eye(4)
    G[:3, :3] = Rotation.from_euler("xyz", [5, -30, 20], degrees=True).as_matrix()
    G[:3, 3] = [0.2, -0.1, 0.4]
    V = np.eye(4)
    V[:3, :3] = Rotation.from_euler("y", 25, degrees=True).as_matrix()
    turned = dict(sc, group_poses=G[None, :3, :].astype(F32))
    C = cyl()
    a = raster.render(sc, dict(C, pose=V[:3, :].astype(F32)), raster.make_opts(raster.STRICT))
    b = raster.render(turned, dict(C, pose=(V @ np.linalg.inv(G))[:3, :].astype(F32)), raster.make_opts(raster.STRICT))
    assert a["alpha"].max() > 0.5
    for ch in ("rgb", "depth", "normal", "alpha"):
        np.testing.assert_allclose(a[ch], b[ch], rtol=2e-5, atol=2e-5)
