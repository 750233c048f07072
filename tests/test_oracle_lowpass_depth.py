"""Pins of the depth a pair takes under the low-pass filter (CPU only).

The filter (Sec. II, against degenerate line projections) replaces a pair's
rho = u^2 + v^2 by the screen-space term rho_lp when that is smaller.  That
happens when the surfel is seen (nearly) edge-on or is tiny: then the ray's
hit point on the surfel plane is far from the surfel, or meaningless, so the
pair takes the depth of the surfel centre (camera mu_z, LiDAR |mu|), as the
cited 2DGS filter does; a pair that uses rho keeps the depth of its hit
point.  The hit points below come from a direct ray/plane intersection
t = (n . mu) / (n . d), independent of the oracle's two-plane solve.
"""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

from oracle import raster, spec32
from tests.helpers import F32, quat_wxyz, surfels

CAM = dict(kind="pinhole", width=64, height=48, fx=64.0, fy=64.0, cx=32.0, cy=24.0, z_near=0.2,
           pose=np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(F32))
TOL = 1e-5


def _ray_point(i, j, z):
    return [(i + 0.5 - CAM["cx"]) / CAM["fx"] * z, (j + 0.5 - CAM["cy"]) / CAM["fy"] * z, z]


def _dir(i, j):
    return np.array([(i + 0.5 - CAM["cx"]) / CAM["fx"], (j + 0.5 - CAM["cy"]) / CAM["fy"], 1.0])


def _frame(q):
    """Unit tangents and normal of the FP32 quaternion q (w, x, y, z)."""
    w, x, y, z = (float(v) for v in q)
    R = Rotation.from_quat([x, y, z, w]).as_matrix()
    return R[:, 0], R[:, 1], R[:, 2]


def _hit(mu, n, d):
    t = float(n @ mu) / float(n @ d)
    return t * d


def _lp_rho(mu, i, j, lp):
    pcx = CAM["fx"] * mu[0] / mu[2] + CAM["cx"]
    pcy = CAM["fy"] * mu[1] / mu[2] + CAM["cy"]
    return lp * ((i + 0.5 - pcx) ** 2 + (j + 0.5 - pcy) ** 2)


def test_nearly_edge_on_surfel_takes_the_centre_depth():
    # The surfel's normal is 1 degree from the image x axis: the ray of the
    # next pixel meets its plane ~2 m in front of the centre, far outside the
    # surfel (rho ~ 1e3), so the low-pass term sets alpha and the centre sets
    # the depth.
    opts = raster.make_opts()
    q = quat_wxyz(Rotation.from_euler("y", 89.0, degrees=True))[:, 0]
    sc = surfels([_ray_point(32, 24, 5.0)], q, [0.05, 0.05], [0.8], rgb=[1, 1, 1])
    mu = sc["mean"][:, 0].astype(np.float64)
    tu, tv, n = _frame(q)
    x = _hit(mu, n, _dir(33, 24))
    s = float(F32(0.05))
    rho = (((x - mu) @ tu) / s) ** 2 + (((x - mu) @ tv) / s) ** 2
    rho_lp = _lp_rho(mu, 33, 24, opts["lp_inv_sigma2"])
    assert rho > 100 * rho_lp and abs(x[2] - mu[2]) > 1.0   # the two readings differ by > 1 m
    out = raster.render(sc, CAM, opts)
    a = out["alpha"][24, 33]
    assert a == pytest.approx(float(F32(0.8)) * math.exp(-0.5 * rho_lp), rel=1e-12)
    assert out["depth"][24, 33] / a == pytest.approx(mu[2], rel=1e-12)


def test_tilted_surfel_within_its_disc_keeps_the_hit_depth():
    # 45-degree tilt, large surfel: four pixels from the centre the ray meets
    # the plane inside the disc (rho < rho_lp), at depth ~4.7 instead of 5.
    opts = raster.make_opts()
    q = quat_wxyz(Rotation.from_euler("y", 45.0, degrees=True))[:, 0]
    sc = surfels([_ray_point(32, 24, 5.0)], q, [0.5, 0.5], [0.8], rgb=[1, 1, 1])
    mu = sc["mean"][:, 0].astype(np.float64)
    tu, tv, n = _frame(q)
    x = _hit(mu, n, _dir(36, 24))
    s = float(F32(0.5))
    rho = (((x - mu) @ tu) / s) ** 2 + (((x - mu) @ tv) / s) ** 2
    assert rho < _lp_rho(mu, 36, 24, opts["lp_inv_sigma2"]) and abs(x[2] - mu[2]) > 0.2
    out = raster.render(sc, CAM, opts)
    a = out["alpha"][24, 36]
    assert a == pytest.approx(float(F32(0.8)) * math.exp(-0.5 * rho), rel=1e-9)
    assert out["depth"][24, 36] / a == pytest.approx(x[2], rel=1e-9)


def test_lowpass_choice_near_a_tie_is_flagged_with_the_hit_depth_alternative():
    # A 30-degree tilt; the scale is chosen so that at the next pixel rho sits
    # just above rho_lp: nominally the low-pass term wins (centre depth), the
    # choice is flagged, and its alternative is the pair with rho and the
    # depth of its hit point.
    opts = raster.make_opts()
    q = quat_wxyz(Rotation.from_euler("y", 30.0, degrees=True))[:, 0]
    mu0 = _ray_point(32, 24, 5.0)
    mu = np.asarray(mu0, F32).astype(np.float64)
    tu, tv, n = _frame(q)
    x = _hit(mu, n, _dir(34, 24))
    dist = math.sqrt(((x - mu) @ tu) ** 2 + ((x - mu) @ tv) ** 2)
    rho_lp = _lp_rho(mu, 34, 24, opts["lp_inv_sigma2"])
    s = float(F32(dist / math.sqrt(rho_lp * (1 + 5e-6))))
    rho = (dist / s) ** 2
    rel = (rho - rho_lp) / rho
    assert 0 < rel < TOL and abs(x[2] - mu[2]) > 0.05
    o = float(F32(0.8))
    sc = surfels([mu0], q, [s, s], [o], rgb=[1, 1, 1])
    res = raster.render(sc, CAM, opts, alternatives=TOL, margins=True)
    r = 24 * CAM["width"] + 34
    a = res["alpha"][24, 34]
    assert a == pytest.approx(o * math.exp(-0.5 * rho_lp), rel=1e-12)
    assert res["depth"][24, 34] / a == pytest.approx(mu[2], rel=1e-12)
    assert res["n_flags"][r] == 1
    assert res["margin"][24, 34] == pytest.approx(rel, rel=1e-6)
    rays = list(res["alts"]["rays"])
    assert r in rays
    assert res["alts"]["kinds"][rays.index(r)] == [3]
    alt = res["alts"]["values"][rays.index(r)]
    assert alt.shape == (1, 9)  # the 8 sums and the median depth
    assert alt[0][7] == pytest.approx(o * math.exp(-0.5 * rho), rel=1e-12)
    assert alt[0][3] / alt[0][7] == pytest.approx(x[2], rel=1e-9)


def _lidar(n_beams=16, n_az=96):
    from gen.scenes import lidar_spinning
    L = lidar_spinning(n_beams=n_beams, n_az=n_az, el_min_deg=-25, el_max_deg=15,
                       pose=np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(F32))
    L["z_near"] = 0.2
    return L


def test_lidar_nearly_edge_on_surfel_takes_the_centre_range():
    # A surfel on beam (j, i) whose plane holds the beam (up to 1 degree) and
    # the vertical: the next column's beam meets the plane far from the
    # surfel, so the low-pass term (chord to the centre direction in azimuth
    # steps) sets alpha and |mu| the range.
    L = _lidar()
    tabs = spec32.lidar_tables(L)
    opts = raster.make_opts(tile_w=16, tile_h=4)
    i, j, r = 10, 7, 6.0

    def beam(c, b):  # products of the FP32 table entries, in FP64
        ce, se = float(tabs["cos_el"][b]), float(tabs["sin_el"][b])
        return np.array([ce * float(tabs["cos_az"][c]), ce * float(tabs["sin_az"][c]), se])

    d = beam(i, j)
    side = np.cross(d, [0, 0, 1.0])
    side /= np.linalg.norm(side)
    up = np.cross(side, d)
    ang = math.radians(1.0)
    n = math.cos(ang) * side + math.sin(ang) * d        # normal 89 degrees from the beam, across the columns
    tu = np.cross(up, n)
    tu /= np.linalg.norm(tu)
    R = np.stack([tu, up, n], 1)
    q = quat_wxyz(Rotation.from_matrix(R))
    sc = surfels([r * d], q, [0.05, 0.05], [0.8], intensity=[0.3])
    mu = sc["mean"][:, 0].astype(np.float64)
    rr = float(np.linalg.norm(mu))
    d2 = beam(i + 1, j)
    qf = q[:, 0]
    _, _, nf = _frame(qf)
    x = _hit(mu, nf, d2)
    assert abs(float(np.linalg.norm(x)) - rr) > 1.0      # the hit point is over a metre away
    step = 2 * math.pi / L["width"]
    chord = d2 - mu / rr
    rho_lp = opts["lp_inv_sigma2"] * float(chord @ chord) / step ** 2
    out = raster.render(sc, L, opts)
    a = out["alpha"][j, i + 1]
    assert a == pytest.approx(float(F32(0.8)) * math.exp(-0.5 * rho_lp), rel=1e-9)
    assert out["range"][j, i + 1] / a == pytest.approx(rr, rel=1e-12)
