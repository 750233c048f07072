"""Pins of the oracle's near-threshold decision flags and their alternatives (CPU only).

Production-mode parity compares a float32 device path with the FP64 oracle.
Where a ray's skip, stop or support decision lies within rounding of its
threshold the two may legitimately decide differently, so the oracle flags
such decisions and also returns the outputs the definition gives with them
taken the other way.  These tests fix, against closed forms of camera-facing
surfels on a pixel's ray (alpha = opacity at the centre pixel), that:

  - a pixel whose alpha is within 1e-5 (relative) of alpha_min is flagged and
    its alternative is the pixel with that surfel skipped;
  - a pixel whose T (1 - alpha) is within 1e-5 of T_min is flagged and its
    alternative is the composite stopped before that surfel;
  - a pixel whose hit lies within 1e-5 of the support cutoff is flagged and
    its alternative includes the surfel with alpha = o exp(-rho / 2);
  - pixels far from every threshold carry no flag and no alternative, and the
    per-ray margin agrees with the flags.
"""
import math

import numpy as np
import pytest

from oracle import raster
from tests.helpers import F32, surfels

CAM = dict(kind="pinhole", width=64, height=48, fx=64.0, fy=64.0, cx=32.0, cy=24.0, z_near=0.2,
           pose=np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(F32))
IDQ = [1.0, 0.0, 0.0, 0.0]
TOL = 1e-5


def _ray_point(i, j, z):
    return [(i + 0.5 - CAM["cx"]) / CAM["fx"] * z, (j + 0.5 - CAM["cy"]) / CAM["fy"] * z, z]


def _ray(i, j):
    return j * CAM["width"] + i


def _alts(res, ray):
    rays = list(res["alts"]["rays"])
    return res["alts"]["values"][rays.index(ray)] if ray in rays else None


def test_alpha_min_flag_and_skip_alternative():
    opts = raster.make_opts()
    amin = opts["alpha_min"]
    o = float(F32(amin * (1 + 5e-6)))
    rel = (o - amin) / amin
    assert 0 < rel < TOL
    sc = surfels([_ray_point(20, 10, 5.0)], IDQ, [0.2, 0.2], [o], rgb=[0.3, 0.6, 0.9])
    res = raster.render(sc, CAM, opts, alternatives=TOL, margins=True)
    r = _ray(20, 10)
    # nominal: alpha = o >= alpha_min, composited
    assert res["alpha"][10, 20] == pytest.approx(o, abs=1e-15)
    assert res["n_flags"][r] == 1
    assert res["margin"][10, 20] == pytest.approx(rel, rel=1e-9)
    alt = _alts(res, r)
    assert alt is not None and alt.shape == (1, 9)
    np.testing.assert_allclose(alt[0], 0.0, atol=1e-15)  # the surfel skipped: nothing composited


def test_stop_flag_and_stopped_alternative():
    opts = raster.make_opts()
    tmin = opts["T_min"]
    a = float(F32(0.9))
    T3 = (1 - a) ** 3
    o4 = float(F32(1 - tmin * (1 + 5e-6) / T3))
    rel = (T3 * (1 - o4) - tmin) / tmin
    assert 0 < rel < TOL
    zs = (3.0, 4.0, 5.0, 6.0)
    cols = [[1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0]]
    sc = surfels([_ray_point(30, 20, z) for z in zs], np.repeat(np.array(IDQ)[:, None], 4, 1), [[0.3, 0.3]] * 4, [a, a, a, o4], rgb=cols)
    res = raster.render(sc, CAM, opts, alternatives=TOL)
    r = _ray(30, 20)
    ops = [a, a, a, o4]
    T = 1.0
    nominal = np.zeros(8)
    stopped = None
    for k in range(4):
        if k == 3:
            stopped = nominal.copy()
        f = np.array(cols[k] + [float(sc["mean"][2, k]), 0.0, 0.0, -1.0, 1.0])
        nominal += T * ops[k] * f
        T *= 1 - ops[k]
    got = np.concatenate([res["rgb"][:, 20, 30], [res["depth"][20, 30]], res["normal"][:, 20, 30],
                          [res["alpha"][20, 30]]])
    np.testing.assert_allclose(got, nominal, atol=1e-12)
    assert res["n_flags"][r] == 1
    alt = _alts(res, r)
    assert alt is not None and alt.shape == (1, 9)
    np.testing.assert_allclose(alt[0][:8], stopped, atol=1e-12)
    # the median depth is the first surfel's (T = 0.1 after it) either way
    assert res["median"][20, 30] == pytest.approx(zs[0], rel=1e-6) and alt[0][8] == res["median"][20, 30]


def test_support_cutoff_flag_and_included_alternative():
    # strict mode, no low-pass: the ray of pixel (21, 10) meets a facing surfel
    # centred on pixel 20's ray at u = off / s_u; s_u is chosen so that
    # rho = u^2 sits just beyond cutoff^2 = 25.
    opts = raster.make_opts(raster.STRICT, lowpass=False)
    z = 5.0
    mu = _ray_point(20, 10, z)
    mu32 = np.asarray(mu, F32).astype(np.float64)
    off = (21 + 0.5 - CAM["cx"]) / CAM["fx"] * mu32[2] - mu32[0]
    su = float(F32(off / math.sqrt(25.0 * (1 + 5e-6))))
    rho = (off / su) ** 2
    rel = (rho - 25.0) / 25.0
    assert 0 < rel < TOL
    o = 0.8
    sc = surfels([mu], IDQ, [su, su], [o], rgb=[1.0, 1.0, 1.0])
    res = raster.render(sc, CAM, opts, alternatives=TOL)
    r = _ray(21, 10)
    assert res["alpha"][10, 21] == 0.0  # outside the support
    assert res["n_flags"][r] == 1
    alt = _alts(res, r)
    assert alt is not None
    of = float(F32(o))
    assert alt[0][7] == pytest.approx(of * math.exp(-0.5 * rho), rel=1e-9)


def test_far_pixels_carry_no_flag():
    opts = raster.make_opts()
    sc = surfels([_ray_point(20, 10, 5.0)], IDQ, [0.05, 0.08], [0.7], rgb=[0.2, 0.4, 0.9])
    res = raster.render(sc, CAM, opts, alternatives=TOL, margins=True)
    r = _ray(20, 10)
    assert res["n_flags"][r] == 0
    assert _alts(res, r) is None
    assert res["margin"][10, 20] > 0.1
    # flags exactly where the margin is within the tolerance
    np.testing.assert_array_equal(res["n_flags"].reshape(CAM["height"], CAM["width"]) > 0,
                                  res["margin"] <= TOL)


def test_alternatives_of_a_random_scene_agree_with_margins():
    rng = np.random.default_rng(4)
    n = 150
    mean = np.stack([rng.uniform(-1, 1, n), rng.uniform(-0.7, 0.7, n), rng.uniform(2.5, 6, n)], 1)
    q = rng.standard_normal((n, 4))
    s = np.exp(rng.normal(-2.3, 0.4, (n, 2)))
    o = 1 / (1 + np.exp(-rng.normal(0.5, 1.5, n)))
    sc = surfels(mean, q, s, o, rgb=rng.uniform(0, 1, (n, 3)))
    res = raster.render(sc, CAM, raster.make_opts(), alternatives=1e-2, margins=True)
    nf = res["n_flags"].reshape(CAM["height"], CAM["width"])
    np.testing.assert_array_equal(nf > 0, res["margin"] <= 1e-2)
    # one alternative per non-empty subset of flags; flipping an alpha_min or a
    # stop decision always changes the ray (a support flip may not: in
    # production alpha at the cutoff is below alpha_min; nor may the low-pass
    # choice of a pair outside the support either way)
    nom = np.concatenate([res["rgb"], res["depth"][None], res["normal"], res["alpha"][None],
                          res["median"][None]]).reshape(9, -1)
    n_checked = 0
    for r, vals, kinds in zip(res["alts"]["rays"], res["alts"]["values"], res["alts"]["kinds"]):
        assert vals.shape[0] == 2 ** nf.reshape(-1)[r] - 1
        if 0 not in kinds and 3 not in kinds:
            assert (np.abs(vals - nom[:, r][None]).max(1) > 0).all()
            n_checked += 1
    assert n_checked > 0
