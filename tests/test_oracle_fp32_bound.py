"""The first-order FP32 error bound the oracle uses to widen its decision
windows (oracle.raster._fp32_uv_error) against an actual FP32 evaluation
(CPU only).

A surfel seen nearly edge-on projects to a needle: the homography of Eq. 2
from pixel offsets to (u, v) has large rows and its evaluation cancels.  The
FP32 evaluation below follows the arithmetic a single-precision solve does --
the centre in a 16-pixel tile's frame held as an FP32 value plus its FP32
residual, the offset from it, the rows' products -- and every pixel's
(u, v) error against FP64 must lie within the bound: its rho error within
drho.  A bound that is too tight (a dropped term, a wrong scale) fails here;
one that is loose by orders of magnitude fails the check that it is within
a factor 60 of the worst error seen.
"""
import numpy as np
import torch
from scipy.spatial.transform import Rotation

from oracle import raster
from tests.helpers import F32, quat_wxyz, surfels

CAM = dict(kind="pinhole", width=96, height=64, fx=80.0, fy=80.0, cx=48.0, cy=32.0, z_near=0.2,
           pose=np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(F32))


def _needles(seed, n):
    rng = np.random.default_rng(seed)
    mean = np.stack([rng.uniform(-1.5, 1.5, n), rng.uniform(-0.8, 0.8, n), rng.uniform(4.0, 9.0, n)], 1)
    # normals nearly perpendicular to the view ray: tilt 89.5-89.99 degrees
    rot = []
    for k in range(n):
        view = mean[k] / np.linalg.norm(mean[k])
        a = np.deg2rad(rng.uniform(89.5, 89.99))
        side = np.cross(view, [0.0, 1.0, 0.0])
        side /= np.linalg.norm(side)
        nrm = np.cos(a) * (-view) + np.sin(a) * side
        tu = np.cross([0.0, 1.0, 0.0], nrm)
        tu /= np.linalg.norm(tu)
        tv = np.cross(nrm, tu)
        rot.append(np.stack([tu, tv, nrm], 1))
    q = quat_wxyz(Rotation.from_matrix(np.array(rot)))
    s = np.exp(rng.normal(-1.2, 0.3, (n, 2)))
    return surfels(mean, q, s, np.full(n, 0.8), rgb=rng.uniform(0, 1, (n, 3)))


def test_fp32_solve_error_is_within_the_bound():
    sc = _needles(3, 200)
    opts = raster.make_opts(raster.STRICT, tile_w=16, tile_h=16)
    bins = raster.spec_bins(sc, CAM, opts)
    params = {k: raster._leaf(sc[k], False) for k in ("mean", "quat", "scale", "opacity", "rgb")}
    sq = raster.splat_quantities(sc, CAM, bins, params)
    rp, sp = raster._candidate_pairs(bins, CAM, np.arange(CAM["width"] * CAM["height"]), "brute", None)
    rays_t = raster._rays(CAM, np.arange(CAM["width"] * CAM["height"]))
    with torch.no_grad():
        sol = raster._solve(sq, rays_t, rp, sp, CAM, opts, sc, 1e-4)
    u64, v64 = sol["u"].numpy(), sol["v"].numpy()
    drho = raster._fp32_uv_error(sq["M"][torch.as_tensor(sp)], sq["mu_s"][torch.as_tensor(sp)], sol["u"], sol["v"], rays_t,
                                 torch.as_tensor(rp), CAM, opts).numpy()
    # the FP32 evaluation, from the FP64 homography rows
    M = sq["M"].detach().numpy()[sp]
    mu = M[:, :, 2]
    det = np.linalg.det(M)
    adj = np.linalg.inv(M) * det[:, None, None]
    muz = mu[:, 2]
    P0 = (adj[:, :, 0] * (muz / (CAM["fx"] * det))[:, None]).astype(np.float32)
    P1 = (adj[:, :, 1] * (muz / (CAM["fy"] * det))[:, None]).astype(np.float32)
    pcx = CAM["fx"] * mu[:, 0] / muz + CAM["cx"]
    pcy = CAM["fy"] * mu[:, 1] / muz + CAM["cy"]
    i, j = rays_t["i"][rp], rays_t["j"][rp]
    ox, oy = (i // 16) * 16, (j // 16) * 16
    cx, cy = pcx - ox, pcy - oy
    chx, chy = cx.astype(np.float32), cy.astype(np.float32)
    clx, cly = (cx - chx).astype(np.float32), (cy - chy).astype(np.float32)
    plx, ply = (i - ox + 0.5).astype(np.float32), (j - oy + 0.5).astype(np.float32)
    dx = (plx - chx) - clx
    dy = (ply - chy) - cly
    h = [np.float32(P0[:, r]) * dx + np.float32(P1[:, r]) * dy for r in range(3)]
    h2 = h[2] + np.float32(1.0)
    u32, v32 = (h[0] / h2).astype(np.float64), (h[1] / h2).astype(np.float64)
    # within the relevant region (rho up to the cutoff)
    m = (u64 ** 2 + v64 ** 2 <= opts["cutoff2"]) & (np.abs(h2) > 0.125)
    assert m.sum() > 200
    e_rho = np.abs((u32 ** 2 + v32 ** 2) - (u64 ** 2 + v64 ** 2))[m]
    bound = drho[m]
    assert (e_rho <= bound).all(), (e_rho / bound).max()
    # the needles make the FP32 solve visibly inexact, and the bound is not vacuous

    assert (e_rho / bound).max() > 1.0 / 60.0
    assert e_rho.max() > 2e-6  # a well-conditioned FP32 solve errs by ~1e-7
