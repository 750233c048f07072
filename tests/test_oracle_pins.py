"""Pins of the FP64 oracle against closed forms, geometry and invariants (CPU only).

Each test fixes a fact that the paper's geometry (Sec. III-A, Eq. 1-5) or
textbook front-to-back compositing determines independently of the oracle's
own code, so that a dropped term, a sign error or a transposed operand in the
oracle fails at least one of them.
"""
import math

import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation

from oracle import raster, spec32
from tests.helpers import F32, quat_wxyz, surfels

CAM = dict(kind="pinhole", width=256, height=256, fx=256.0, fy=256.0, cx=128.0, cy=128.0, z_near=0.2,
           pose=np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(F32))
IDQ = [1.0, 0.0, 0.0, 0.0]


def _ray_point(i, j, z, cam=CAM):
    """Point at depth z on the ray of pixel (i, j) (pixel centres at +0.5)."""
    return [(i + 0.5 - cam["cx"]) / cam["fx"] * z, (j + 0.5 - cam["cy"]) / cam["fy"] * z, z]


def _pix(out, ch, i, j):
    v = out[ch]
    return v[:, j, i] if v.ndim == 3 else v[j, i]


def test_single_facing_splat_centre_pixel_alpha_equals_opacity():
    # A camera-facing surfel centred on a pixel's ray: rho = rho_lp = 0 there,
    # so alpha = o, depth = o * z, normal = o * (0, 0, -1), rgb = o * c.
    z = 5.0
    sc = surfels([_ray_point(128, 128, z)], IDQ, [0.05, 0.08], [0.7], rgb=[0.2, 0.4, 0.9])
    out = raster.render(sc, CAM, raster.make_opts())
    o = float(F32(0.7))
    mu = sc["mean"][:, 0].astype(np.float64)
    assert _pix(out, "alpha", 128, 128) == pytest.approx(o, abs=1e-12)
    assert _pix(out, "depth", 128, 128) == pytest.approx(o * mu[2], abs=1e-12)
    np.testing.assert_allclose(_pix(out, "normal", 128, 128), [0, 0, -o], atol=1e-12)
    np.testing.assert_allclose(_pix(out, "rgb", 128, 128), o * sc["rgb"][:, 0].astype(np.float64), atol=1e-12)
    assert out["T_final"][128, 128] == pytest.approx(1 - o, abs=1e-12)


@pytest.mark.parametrize("delta", [1, 2, 3])
@pytest.mark.parametrize("spin", [0.0, 90.0])
def test_gaussian_falloff_along_tangent(delta, spin):
    # Plane z = const: the ray of pixel (128+delta, 128) meets it at x offset
    # delta*z/f from the centre.  With t_u along the image x axis (spin 0) the
    # offset is u*s_u; spun by 90 deg it is -v*s_v.  alpha = o exp(-rho/2).
    z, su, sv, o = 5.0, 0.05, 0.02, 0.8
    q = quat_wxyz(Rotation.from_euler("z", spin, degrees=True))
    sc = surfels([_ray_point(128, 128, z)], q, [su, sv], [o], rgb=[1, 1, 1])
    out = raster.render(sc, CAM, raster.make_opts(lowpass=False))
    mu = sc["mean"][:, 0].astype(np.float64)
    x_hit = (128 + delta + 0.5 - 128) / 256.0 * mu[2]
    off = x_hit - mu[0]
    s_eff = float(F32(su)) if spin == 0.0 else float(F32(sv))
    rho = (off / s_eff) ** 2
    expect = float(F32(o)) * math.exp(-0.5 * rho)
    if expect < 1 / 255:
        expect = 0.0
    assert _pix(out, "alpha", 128 + delta, 128) == pytest.approx(expect, rel=1e-6, abs=1e-12)


def test_lowpass_filter_dominates_for_tiny_splat():
    # A surfel far below a pixel: rho >> rho_lp, so alpha = o exp(-rho_lp/2)
    # with rho_lp = 2 |p - c|^2 (sigma = sqrt(2)/2 px).
    z, o = 5.0, 0.9
    sc = surfels([_ray_point(128, 128, z)], IDQ, [1e-4, 1e-4], [o], rgb=[1, 1, 1])
    out = raster.render(sc, CAM, raster.make_opts())
    of = float(F32(o))
    assert _pix(out, "alpha", 129, 128) == pytest.approx(of * math.exp(-1.0), rel=1e-6)
    assert _pix(out, "alpha", 129, 129) == pytest.approx(of * math.exp(-2.0), rel=1e-6)
    assert _pix(out, "alpha", 128, 128) == pytest.approx(of, rel=1e-9)


def test_two_and_three_splat_compositing_closed_form():
    z = [4.0, 6.0, 7.5]
    o = [0.6, 0.5, 0.4]
    c = [[1, 0, 0], [0, 1, 0], [0, 0, 1]]
    mus = [_ray_point(100, 60, zz) for zz in z]
    # input order deliberately not depth order
    perm = [2, 0, 1]
    sc = surfels([mus[p] for p in perm], [IDQ] * 3, [[0.1, 0.1]] * 3, [o[p] for p in perm],
                 rgb=[c[p] for p in perm])
    out = raster.render(sc, CAM, raster.make_opts())
    of = [float(F32(x)) for x in o]
    zf = [float(sc["mean"][2, perm.index(i)]) for i in range(3)]
    T = 1.0
    col = np.zeros(3)
    dep = 0.0
    for i in range(3):
        col += T * of[i] * np.asarray(c[i], float)
        dep += T * of[i] * zf[i]
        T *= 1 - of[i]
    np.testing.assert_allclose(_pix(out, "rgb", 100, 60), col, atol=1e-12)
    assert _pix(out, "depth", 100, 60) == pytest.approx(dep, abs=1e-12)
    assert _pix(out, "alpha", 100, 60) == pytest.approx(1 - T, abs=1e-12)


def test_alpha_clamp_skip_and_stop_rules():
    opts = raster.make_opts()
    # clamp: o above alpha_max -> alpha_max
    sc = surfels([_ray_point(50, 50, 5.0)], IDQ, [0.1, 0.1], [0.995], rgb=[1, 1, 1])
    out = raster.render(sc, CAM, opts)
    assert _pix(out, "alpha", 50, 50) == pytest.approx(opts["alpha_max"], abs=1e-12)
    # skip: o below alpha_min -> nothing
    sc = surfels([_ray_point(50, 50, 5.0)], IDQ, [0.1, 0.1], [0.003], rgb=[1, 1, 1])
    out = raster.render(sc, CAM, opts)
    assert _pix(out, "alpha", 50, 50) == 0.0
    # stop: three o = 0.98 layers; after two, T = 4e-4 (kept, 4e-4 >= T_min);
    # the third would take T to 8e-6 < T_min, so it is excluded.
    sc = surfels([_ray_point(50, 50, zz) for zz in (4.0, 5.0, 6.0)], [IDQ] * 3, [[0.1, 0.1]] * 3,
                 [0.98] * 3, rgb=[[1, 0, 0], [0, 1, 0], [0, 0, 1]])
    out = raster.render(sc, CAM, opts)
    a = float(F32(0.98))
    np.testing.assert_allclose(_pix(out, "rgb", 50, 50), [a, (1 - a) * a, 0.0], atol=1e-12)
    assert out["n_contrib"][50, 50] == 2


def _random_scene(seed, n, lo=(-1, -1, 2.5), hi=(1, 1, 6), logs=(-2.5, 0.5), lidar=False):
    rng = np.random.default_rng(seed)
    mean = rng.uniform(lo, hi, size=(n, 3))
    q = quat_wxyz(Rotation.random(n, random_state=seed))
    s = np.exp(rng.normal(logs[0], logs[1], size=(n, 2)))
    o = 1 / (1 + np.exp(-rng.normal(0, 1.5, size=n)))
    rgb = rng.uniform(0, 1, size=(n, 3))
    inten = rng.uniform(0, 1, size=n) if lidar else None
    return surfels(mean, q, s, o, rgb=rgb, intensity=inten)


SMALL_CAM = dict(CAM, width=48, height=40, fx=48.0, fy=48.0, cx=24.0, cy=20.0)


@pytest.mark.parametrize("strict", [False, True])
@pytest.mark.parametrize("seed", [0, 1])
def test_alpha_plus_transmittance_is_one(strict, seed):
    sc = _random_scene(seed, 120)
    opts = raster.make_opts(raster.STRICT if strict else raster.PRODUCTION)
    out = raster.render(sc, SMALL_CAM, opts)
    np.testing.assert_allclose(out["alpha"] + out["T_final"], 1.0, atol=1e-13)


def _small_lidar(n_beams=16, n_az=96):
    from gen.scenes import lidar_spinning
    L = lidar_spinning(n_beams=n_beams, n_az=n_az, el_min_deg=-25, el_max_deg=15,
                       pose=np.concatenate([np.eye(3), np.zeros((3, 1))], 1))
    return L


def _lidar_scene(seed, n):
    rng = np.random.default_rng(seed)
    r = rng.uniform(3, 9, n)
    az = rng.uniform(-np.pi, np.pi, n)
    el = np.deg2rad(rng.uniform(-30, 20, n))
    mean = np.stack([r * np.cos(el) * np.cos(az), r * np.cos(el) * np.sin(az), r * np.sin(el)], 1)
    q = quat_wxyz(Rotation.random(n, random_state=seed + 7))
    s = np.exp(rng.normal(-1.3, 0.4, size=(n, 2)))
    o = 1 / (1 + np.exp(-rng.normal(0.5, 1.5, size=n)))
    return surfels(mean, q, s, o, intensity=rng.uniform(0, 1, n))


@pytest.mark.parametrize("strict", [False, True])
def test_brute_force_equals_culled_camera(strict):
    sc = _random_scene(3, 150)
    opts = raster.make_opts(raster.STRICT if strict else raster.PRODUCTION, tile_w=8, tile_h=8)
    a = raster.render(sc, SMALL_CAM, opts, mode="brute")
    b = raster.render(sc, SMALL_CAM, opts, mode="culled")
    for ch in ("rgb", "depth", "normal", "alpha", "T_final"):
        np.testing.assert_array_equal(a[ch], b[ch])
    assert a["alpha"].max() > 0.5


@pytest.mark.parametrize("strict", [False, True])
def test_brute_force_equals_culled_lidar(strict):
    L = _small_lidar()
    sc = _lidar_scene(4, 150)
    opts = raster.make_opts(raster.STRICT if strict else raster.PRODUCTION, tile_w=16, tile_h=4)
    a = raster.render(sc, L, opts, mode="brute")
    b = raster.render(sc, L, opts, mode="culled")
    for ch in ("range", "intensity", "alpha", "T_final"):
        np.testing.assert_array_equal(a[ch], b[ch])
    assert a["alpha"].max() > 0.5
    assert b["bins"]["wrap"].any() or b["bins"]["full_cols"].any()


def test_permutation_invariance():
    sc = _random_scene(5, 100)
    perm = np.random.default_rng(0).permutation(100)
    sp = dict(sc)
    for k in ("mean", "quat", "scale", "rgb"):
        sp[k] = np.ascontiguousarray(sc[k][:, perm])
    sp["opacity"] = np.ascontiguousarray(sc["opacity"][perm])
    a = raster.render(sc, SMALL_CAM, raster.make_opts())
    b = raster.render(sp, SMALL_CAM, raster.make_opts())
    for ch in ("rgb", "depth", "normal", "alpha"):
        np.testing.assert_allclose(a[ch], b[ch], atol=1e-12)


def test_rigid_invariance_group_pose_vs_sensor_pose():
    # Placing the scene with an object->world pose G and moving the camera by
    # the same G (camera pose V*G^-1) leaves the image unchanged up to the FP32
    # rounding of the composed pose.
    sc = _random_scene(6, 80)
    G = np.eye(4)
    G[:3, :3] = Rotation.from_euler("xyz", [10, -20, 35], degrees=True).as_matrix()
    G[:3, 3] = [0.3, -0.2, 0.5]
    Gi = np.linalg.inv(G)
    sg = dict(sc, group_poses=G[None, :3, :].astype(F32))
    cam = dict(SMALL_CAM, pose=Gi[:3, :].astype(F32))
    a = raster.render(sc, SMALL_CAM, raster.make_opts(raster.STRICT))
    b = raster.render(sg, cam, raster.make_opts(raster.STRICT))
    for ch in ("rgb", "depth", "normal", "alpha"):
        np.testing.assert_allclose(a[ch], b[ch], rtol=2e-5, atol=2e-5)


def test_rigid_invariance_holds_for_sh_colour():
    # The SH colour is evaluated at the view direction in the surfel group's
    # own frame: an asset turned by G and seen by the camera equals the
    # unturned asset seen by the camera moved by G (camera pose V G), for
    # degree-3 coefficients.  A world-frame direction would break this.
    rng = np.random.default_rng(21)
    sc = _random_scene(7, 60)
    sc.pop("rgb")
    sc["sh"] = rng.normal(0.0, 0.3, (16 * 3, 60)).astype(F32)
    sc["sh_degree"] = 3
    G = np.eye(4)
    G[:3, :3] = Rotation.from_euler("xyz", [25, -40, 70], degrees=True).as_matrix()
    G[:3, 3] = [0.2, 0.1, -0.3]
    V = np.eye(4)
    V[:3, :3] = Rotation.from_euler("y", 15, degrees=True).as_matrix()
    V[:3, 3] = [0.1, 0.0, 0.4]
    Gi = np.linalg.inv(G)
    # asset turned by G in a world seen through V G^-1  ==  the plain asset seen through V
    turned = dict(sc, group_poses=G[None, :3, :].astype(F32))
    cam_t = dict(SMALL_CAM, pose=(V @ Gi)[:3, :].astype(F32))
    cam_p = dict(SMALL_CAM, pose=V[:3, :].astype(F32))
    a = raster.render(sc, cam_p, raster.make_opts(raster.STRICT))
    b = raster.render(turned, cam_t, raster.make_opts(raster.STRICT))
    assert a["alpha"].max() > 0.5
    for ch in ("rgb", "depth", "normal", "alpha"):
        np.testing.assert_allclose(a[ch], b[ch], rtol=2e-5, atol=2e-5)
    # and the colour does depend on the direction: the same scene seen through
    # the turned camera without turning the asset differs
    c = raster.render(sc, cam_t, raster.make_opts(raster.STRICT))
    assert np.abs(c["rgb"] - a["rgb"]).max() > 1e-2


def test_sh_colour_uses_the_view_direction_in_the_group_frame():
    # Degree-1 SH with only the Y_1,0 = sqrt(3 / 4 pi) z coefficients set:
    # colour = 0.5 + c sqrt(3 / 4 pi) d_z, with d the unit direction from the
    # camera centre to the surfel expressed in the group's frame.  The camera
    # (centre c_w, general rotation) sees the surfel centre on a pixel's ray,
    # where alpha = o, so rgb / alpha is the colour.  Sensor-frame or
    # world-frame directions give other values.
    c_w = np.array([0.3, -0.2, -0.5])
    Rv = Rotation.from_euler("zyx", [20, -35, 10], degrees=True).as_matrix()
    V = np.concatenate([Rv, (-Rv @ c_w)[:, None]], 1)
    Rg = Rotation.from_euler("xyz", [50, 30, -70], degrees=True).as_matrix()
    tg = np.array([0.5, 0.1, 0.2])
    G = np.concatenate([Rg, tg[:, None]], 1)
    i, j, z = 20, 15, 4.0
    p_s = np.array([(i + 0.5 - SMALL_CAM["cx"]) / SMALL_CAM["fx"] * z, (j + 0.5 - SMALL_CAM["cy"]) / SMALL_CAM["fy"] * z, z])
    p_w = Rv.T @ p_s + c_w            # on the ray of pixel (i, j)
    mu_g = Rg.T @ (p_w - tg)          # the surfel centre in its group's frame
    coef = np.array([0.6, -0.4, 0.2])
    sh = np.zeros((4 * 3, 1))
    sh[2 * 3:2 * 3 + 3, 0] = coef
    q = quat_wxyz(Rotation.from_euler("xy", [10, -20], degrees=True))
    sc = surfels([mu_g], q, [0.05, 0.05], [0.8], sh=sh, sh_degree=1)
    sc["group_poses"] = G[None].astype(F32)
    out = raster.render(sc, dict(SMALL_CAM, pose=V.astype(F32)), raster.make_opts(raster.STRICT))
    a = out["alpha"][j, i]
    assert a == pytest.approx(float(F32(0.8)), rel=1e-5)
    d = Rg.T @ (p_w - c_w)
    d /= np.linalg.norm(d)
    want = 0.5 + coef.astype(F32).astype(np.float64) * math.sqrt(3 / (4 * math.pi)) * d[2]
    np.testing.assert_allclose(out["rgb"][:, j, i] / a, want, atol=2e-6)


def test_lidar_planes_contain_beam_direction():
    # Eq. 5 read with azimuth/elevation roles such that both planes contain
    # the beam: h_u . d = h_v . d = h_u . h_v = 0.
    L = _small_lidar(32, 360)
    rays = raster._rays(L, np.arange(32 * 360))
    hu, hv, d = rays["hu"].numpy(), rays["hv"].numpy(), rays["d"].numpy()
    for a, b in ((hu, d), (hv, d), (hu, hv)):
        assert np.abs((a * b).sum(1)).max() < 1e-6
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), 1.0, atol=1e-6)


def test_lidar_single_facing_splat_range():
    L = _small_lidar(16, 96)
    tabs = spec32.lidar_tables(L)
    i, j, r = 10, 7, 6.0
    d = np.array([tabs["cos_el"][j] * tabs["cos_az"][i], tabs["cos_el"][j] * tabs["sin_az"][i],
                  tabs["sin_el"][j]], np.float64)
    tu = np.cross(d, [0, 0, 1.0])
    tu /= np.linalg.norm(tu)
    tv = np.cross(d, tu)
    q = quat_wxyz(Rotation.from_matrix(np.stack([tu, tv, d], 1)))
    sc = surfels([r * d], q, [0.2, 0.2], [0.8], intensity=[0.3])
    out = raster.render(sc, L, raster.make_opts(tile_w=16, tile_h=4))
    o = float(F32(0.8))
    rr = float(np.linalg.norm(sc["mean"][:, 0].astype(np.float64)))
    assert out["alpha"][j, i] == pytest.approx(o, abs=1e-6)
    assert out["range"][j, i] / out["alpha"][j, i] == pytest.approx(rr, rel=1e-6)
    assert out["intensity"][j, i] == pytest.approx(o * float(F32(0.3)), abs=1e-6)


def test_plane_solve_matches_direct_intersection_and_plane_choice():
    # (u, v) from Eq. 2's two-plane solve equals the direct ray/plane
    # intersection in the surfel's tangent frame, and does not depend on which
    # two planes through the ray are used.
    rng = np.random.default_rng(11)
    sc = _random_scene(12, 40, logs=(-1.0, 0.2))
    bins = raster.spec_bins(sc, SMALL_CAM, raster.make_opts())
    params = {k: torch.as_tensor(sc[k].astype(np.float64)) for k in ("mean", "quat", "scale", "opacity", "rgb")}
    sq = raster.splat_quantities(sc, SMALL_CAM, bins, params)
    ray_ids = rng.integers(0, 48 * 40, 40)
    rays = raster._rays(SMALL_CAM, ray_ids)
    rp = np.arange(40)
    sp = np.arange(40)
    sol = raster._solve(sq, rays, rp, sp, SMALL_CAM, raster.make_opts(raster.STRICT), sc)
    M = sq["M"].numpy()
    for p in range(40):
        d = np.cross(rays["hu"][p].numpy(), rays["hv"][p].numpy())
        tu, tv, mu = M[p][:, 0], M[p][:, 1], M[p][:, 2]
        n = np.cross(tu, tv)
        t = n @ mu / (n @ d)
        x = t * d - mu
        # solve x = u tu + v tv
        uv = np.linalg.lstsq(np.stack([tu, tv], 1), x, rcond=None)[0]
        assert sol["u"][p].item() == pytest.approx(uv[0], rel=1e-9, abs=1e-9)
        assert sol["v"][p].item() == pytest.approx(uv[1], rel=1e-9, abs=1e-9)
    th = 0.7
    rays2 = dict(rays)
    rays2["hu"] = rays["hu"] * math.cos(th) + rays["hv"] * math.sin(th)
    rays2["hv"] = -rays["hu"] * math.sin(th) + rays["hv"] * math.cos(th)
    sol2 = raster._solve(sq, rays2, rp, sp, SMALL_CAM, raster.make_opts(raster.STRICT), sc)
    np.testing.assert_allclose(sol2["u"].numpy(), sol["u"].numpy(), rtol=1e-9, atol=1e-9)
    np.testing.assert_allclose(sol2["v"].numpy(), sol["v"].numpy(), rtol=1e-9, atol=1e-9)


def test_dual_conic_box_of_facing_disc():
    # A disc parallel to the image plane projects to a circle of radius
    # f*sqrt(k)*s/z around f*mu_x/z + c_x; the FP32 rectangle is that box
    # padded by one pixel.
    k = raster.make_opts(lowpass=False)["cutoff2"]
    z, s = 4.0, 0.1
    mu = [0.37, -0.21, z]
    sc = surfels([mu], IDQ, [s, s], [0.9], rgb=[1, 1, 1])
    b = raster.spec_bins(sc, CAM, raster.make_opts(lowpass=False))
    m = sc["mean"][:, 0].astype(np.float64)
    rad = 256.0 * math.sqrt(k) * float(F32(s)) / m[2]
    xc = 256.0 * m[0] / m[2] + 128.0
    yc = 256.0 * m[1] / m[2] + 128.0
    assert b["i_lo"][0] == math.ceil(xc - rad - 1 - 0.5)
    assert b["i_hi"][0] == math.floor(xc + rad + 1 - 0.5)
    assert b["j_lo"][0] == math.ceil(yc - rad - 1 - 0.5)
    assert b["j_hi"][0] == math.floor(yc + rad + 1 - 0.5)
    assert b["key"][0] == F32(z)


def test_edge_on_and_behind_camera_are_invisible():
    # Behind the near plane: invisible.  A disc crossing the camera plane
    # (d >= 0 in the dual conic): invisible.
    q_side = quat_wxyz(Rotation.from_euler("y", 90, degrees=True))
    quats = np.stack([IDQ, q_side[:, 0], IDQ], 1)
    sc = surfels([[0, 0, 0.1], [0, 0, 1.0], [0, 0, 3.0]], quats, [[0.1, 0.1], [2.0, 2.0], [0.1, 0.1]],
                 [0.9] * 3, rgb=[[1, 1, 1]] * 3)
    b = raster.spec_bins(sc, CAM, raster.make_opts())
    assert list(b["visible"]) == [False, False, True]


def test_atan2_spec_within_published_error_bound():
    # A&S 4.4.49 bounds the polynomial's error by 1e-5 rad on [0,1]; with
    # FP32 evaluation we allow 1.2e-5 over the whole circle.
    ang = np.linspace(-np.pi, np.pi, 20001)
    for r in (1e-3, 1.0, 250.0):
        y = (r * np.sin(ang)).astype(F32)
        x = (r * np.cos(ang)).astype(F32)
        got = spec32.atan2_spec(y, x).astype(np.float64)
        ref = np.arctan2(y.astype(np.float64), x.astype(np.float64))
        err = np.abs(np.angle(np.exp(1j * (got - ref))))
        assert err.max() < 1.2e-5
    s = np.linspace(0, 1, 5001).astype(F32)
    err = np.abs(spec32.asin_spec(s).astype(np.float64) - np.arcsin(s.astype(np.float64)))
    assert err.max() < 1.2e-5


def test_tile_pairs_vectorised_matches_loop():
    sc = _random_scene(8, 200)
    opts = raster.make_opts(tile_w=8, tile_h=8)
    b = raster.spec_bins(sc, SMALL_CAM, opts)
    t1, s1 = spec32.tile_pairs(b)
    t2, s2 = spec32.tile_pairs_fast(b)
    np.testing.assert_array_equal(t1, t2)
    np.testing.assert_array_equal(s1, s2)
    L = _small_lidar()
    sl = _lidar_scene(9, 200)
    b = raster.spec_bins(sl, L, raster.make_opts(tile_w=16, tile_h=4))
    t1, s1 = spec32.tile_pairs(b)
    t2, s2 = spec32.tile_pairs_fast(b)
    np.testing.assert_array_equal(t1, t2)
    np.testing.assert_array_equal(s1, s2)


def test_grid_sample_matches_full_image():
    # The strided-grid candidate enumeration (used for bounded CPU samples)
    # reproduces the full-image result on the sampled rays.
    sc = _random_scene(13, 120)
    full = raster.render(sc, SMALL_CAM, raster.make_opts())
    sub = raster.render(sc, SMALL_CAM, raster.make_opts(), rays=("grid", 3))
    ids = raster.grid_rays(SMALL_CAM, 3)
    for ch in ("rgb", "depth", "alpha"):
        f = full[ch].reshape(full[ch].shape[:-2] + (-1,))
        np.testing.assert_array_equal(f[..., ids], sub[ch])


def test_lidar_grid_sample_matches_full_image():
    # Same for a LiDAR, whose column ranges wrap around the circle or span it.
    L = _small_lidar(32, 96)
    sc = _lidar_scene(14, 300)
    full = raster.render(sc, L, raster.make_opts(tile_w=16, tile_h=8))
    b = full["bins"]
    assert (b["wrap"] | b["full_cols"]).any() and b["touch"].sum() > 100
    for stride in (2, 5):
        sub = raster.render(sc, L, raster.make_opts(tile_w=16, tile_h=8), rays=("grid", stride))
        ids = raster.grid_rays(L, stride)
        for ch in ("range", "intensity", "alpha"):
            np.testing.assert_array_equal(full[ch].reshape(-1)[ids], sub[ch])
        assert sub["alpha"].max() > 0.1
