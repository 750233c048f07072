"""Full-size parity in the launch configuration bench.py times.

Driving frame: 1920x1080 pinhole, 1M corridor surfels with degree-3 SH, one
per-sensor plan with the default 32x8 tiles and the default segment length (the horizon
tiles are split into segments and merged).  Integer outputs (visibility,
3.1M-entry pair list, tile ranges) are compared bit for bit with the oracle's
FP32 specification; float outputs on a sample the FP64 oracle computes ray by
ray: every 24th row and column plus every ray of the two heaviest tiles.

LiDAR range image: 128 x 1800, 200k anchors x 10 = 2M surfels, per-sensor plan
with the default 16x8 LiDAR tiles.  Two claims,
checked separately: (1) render parity: the oracle's FP64 decode, rounded to
FP32, is rendered by both sides (pair list bit-exact; floats on every 32nd
column of every 8th beam plus the heaviest tile, which is split into hundreds
of segments); (2) decode parity: the GPU's BF16 MFMA decode against the FP64
decode, element by element.  Chaining the two decodes into the renders is not
a parity claim: an FP32-level difference in a decoded centre can reorder two
near-equal depth keys or move a binning decision, which changes the image by
far more than the rounding (the definition is discontinuous there).

Tolerances and the near-threshold protocol as in the small parity tests:
every sampled ray must match the oracle's nominal outputs or one of the
alternatives of its near-threshold decisions; rays with too many such
decisions to verify are counted and must be at most 1e-4 of the sample.

Adjoint at full size: the 1280x720 neural-Gaussian training step (500k
surfels decoded from 50k anchors) with the L1 loss restricted to a 64x64
crop at the horizon; gradients down to the anchors and MLP weights against
the oracle's autograd through its decode and the crop's rays.
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gen import scenes as S  # noqa: E402
from oracle import decode as odec  # noqa: E402
from oracle import raster, spec32  # noqa: E402
from tests.gpu_common import ALT_TOL, DEV, assert_verified, check_integer_parity, oracle_opts, verify  # noqa: E402

import paper_2503_11731_amd as gs  # noqa: E402

def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _tile_rays(tile, n_tx, tw, th, width, height):
    tx, ty = tile % n_tx, tile // n_tx
    ids = [(ty * th + y) * width + tx * tw + x for y in range(th) for x in range(tw)
           if ty * th + y < height and tx * tw + x < width]
    return np.array(ids, np.int64)


def test_driving_1080p_full_size_parity():
    _say("driving 1080p full size: generate")
    sc, sens = S.config2()
    cam = sens[0]
    scene = dict(mean=sc.mean, quat=sc.quat, scale=sc.scale, opacity=sc.opacity, sh=sc.sh, sh_degree=3,
                 group_offsets=sc.group_offsets, group_poses=sc.group_poses)
    r = gs.Renderer([gs.SceneShape(sc.n, 3, False, (0, sc.n))], [cam], opts=gs.PRODUCTION, device=DEV)
    st = gs.scene_tensors(scene, DEV)
    sp = gs.poses_tensor([cam["pose"]], DEV)
    gp = gs.poses_tensor(sc.group_poses, DEV)
    _say("  gpu forward")
    (out,) = r.forward([st], sp, gp)
    torch.cuda.synchronize()
    status = r.status()
    assert not status["overflow"]
    assert status["segments"] > 0, "the horizon tiles should be split at this size"
    tw, th = 32, 8  # the default camera tile
    o = oracle_opts(gs.PRODUCTION, (tw, th))
    _say(f"  integer parity over {status['pairs'][0]} pairs")
    n_pairs = check_integer_parity(r, scene, cam, o)
    ranges = r.inspect(0)["ranges"].cpu().numpy().astype(np.int64)
    heavy = np.argsort(ranges[:, 1] - ranges[:, 0])[-2:]
    n_tx = (cam["width"] + tw - 1) // tw
    rays = np.concatenate([raster.grid_rays(cam, 24)] +
                          [_tile_rays(int(t), n_tx, tw, th, cam["width"], cam["height"]) for t in heavy])
    _say(f"  oracle on {rays.size} rays (heaviest tiles {heavy.tolist()}, "
         f"{(ranges[heavy, 1] - ranges[heavy, 0]).tolist()} pairs)")
    ref = raster.render(scene, cam, o, rays=rays, alternatives=ALT_TOL)
    got = out.reshape(out.shape[0], -1)[:, torch.from_numpy(rays).to(DEV)].cpu().numpy()
    v = verify(got, ref, "pinhole")
    _say(f"  pairs {n_pairs} segments {status['segments']} {v}")
    assert_verified(v)


def _lidar_fullsize():
    sc, sens = S.config4()
    lid = sens[0]
    poses_s = np.stack([spec32.compose_pose(lid["pose"], g) for g in sc.group_poses])
    anchors = dict(xyz=sc.xyz.astype(np.float64), scaling=sc.scaling.astype(np.float64),
                   offsets=sc.offsets.astype(np.float64), feat=S.bf16_bits_to_f32(sc.feat_bf16).astype(np.float64),
                   group_offsets=sc.group_offsets)
    with torch.no_grad():
        ref_dec = odec.decode(anchors, sc.mlps, poses_s, "lidar")
    return sc, lid, ref_dec


def test_lidar_full_size_render_parity():
    """The oracle's decoded 2M surfels rendered by both sides (pairs bit-exact, sampled floats)."""
    _say("lidar 128x1800, 2M surfels: oracle decode")
    sc, lid, ref_dec = _lidar_fullsize()
    n = sc.n_anchors * sc.k
    offs = tuple(int(x) * sc.k for x in sc.group_offsets)
    scene = {k: np.ascontiguousarray(v.numpy().astype(np.float32)) for k, v in ref_dec.items()}
    scene.update(group_offsets=np.array(offs, np.int32), group_poses=sc.group_poses)
    r = gs.Renderer([gs.SceneShape(n, -1, True, offs)], [lid], opts=gs.PRODUCTION, device=DEV)
    st = gs.scene_tensors(scene, DEV)
    sp = gs.poses_tensor([lid["pose"]], DEV)
    gp = gs.poses_tensor(sc.group_poses, DEV)
    _say("  gpu forward")
    (out,) = r.forward([st], sp, gp)
    torch.cuda.synchronize()
    status = r.status()
    assert not status["overflow"]
    tw, th = 16, 8  # the default tile of a LiDAR sensor in a per-sensor plan
    o = oracle_opts(gs.PRODUCTION, (tw, th))
    _say(f"  integer parity over {status['pairs'][0]} pairs")
    check_integer_parity(r, scene, lid, o)
    ranges = r.inspect(0)["ranges"].cpu().numpy().astype(np.int64)
    heavy = int(np.argmax(ranges[:, 1] - ranges[:, 0]))
    n_tx = (lid["width"] + tw - 1) // tw
    cols = np.arange(0, lid["width"], 32)
    beams = np.arange(0, lid["height"], 8)
    grid = (beams[:, None] * lid["width"] + cols[None, :]).ravel()
    rays = np.unique(np.concatenate([grid, _tile_rays(heavy, n_tx, tw, th, lid["width"], lid["height"])]))
    _say(f"  oracle render on {rays.size} rays (heaviest tile {ranges[heavy, 1] - ranges[heavy, 0]} pairs, "
         f"segments {status['segments']})")
    ref = raster.render(scene, lid, o, rays=rays, alternatives=ALT_TOL)
    got = out.reshape(out.shape[0], -1)[:, torch.from_numpy(rays).to(DEV)].cpu().numpy()
    v = verify(got, ref, "lidar")
    _say(f"  {v}")
    assert_verified(v)


def test_lidar_full_size_decode_parity():
    """BF16 MFMA decode of 200k anchors x 10 vs the FP64 oracle decode, element by element."""
    _say("lidar decode 200k anchors")
    sc, lid, ref_dec = _lidar_fullsize()
    dec = gs.Decoder.from_gen(sc, DEV)
    sp = gs.poses_tensor([lid["pose"]], DEV)
    gp = gs.poses_tensor(sc.group_poses, DEV)
    d = dec.forward(sp[0], gp)
    torch.cuda.synchronize()
    errs = {}
    for k in ("opacity", "scale", "intensity", "drop"):
        errs[k] = float(np.abs(d[k].cpu().numpy().astype(np.float64) - ref_dec[k].numpy()).max())
    for k in ("quat", "mean"):
        ref = ref_dec[k].numpy()
        errs[k] = float((np.abs(d[k].cpu().numpy().astype(np.float64) - ref) / np.maximum(1.0, np.abs(ref))).max())
    _say(f"  {errs}")
    for k, e in errs.items():
        assert e <= 1e-4, (k, e)


def test_training_720p_full_size_adjoint_on_a_crop():
    """Decode -> render -> L1 on a 64x64 crop -> adjoint render -> adjoint decode at full size
    (1280x720, 50k anchors x 10) vs the oracle's autograd chain over the crop's rays."""
    _say("720p training step adjoint, 64x64 crop")
    sc, sens = S.config3()
    cam = sens[0]
    x0, y0, cw = 608, 336, 64
    ys, xs = np.mgrid[y0:y0 + cw, x0:x0 + cw]
    rays = (ys * cam["width"] + xs).reshape(-1)
    anchors = dict(xyz=sc.xyz.astype(np.float64), scaling=sc.scaling.astype(np.float64),
                   offsets=sc.offsets.astype(np.float64), feat=S.bf16_bits_to_f32(sc.feat_bf16).astype(np.float64),
                   group_offsets=sc.group_offsets)
    leaves = {k: torch.as_tensor(v).requires_grad_(True) for k, v in anchors.items() if k != "group_offsets"}
    for name in ("w1", "b1", "w2", "b2"):
        leaves[f"{name}_0"] = torch.as_tensor(sc.mlps[0][name].astype(np.float64)).requires_grad_(True)
    poses_s = np.stack([spec32.compose_pose(cam["pose"], g) for g in sc.group_poses])
    dec = odec.decode(anchors, sc.mlps, poses_s, "pinhole", params=leaves)
    n = sc.n_anchors * sc.k
    offs = tuple(int(x) * sc.k for x in sc.group_offsets)
    sc32 = {k: np.ascontiguousarray(v.detach().numpy().astype(np.float32)) for k, v in dec.items()}
    sc32.update(group_offsets=np.array(offs, np.int32), group_poses=sc.group_poses)
    o = oracle_opts(gs.PRODUCTION, (32, 8))
    _say("  oracle forward on the crop")
    fwd = raster.render(sc32, cam, o, rays=rays, params={k: v.detach() for k, v in dec.items()})
    target = np.random.default_rng(3).uniform(0, 1, (3, rays.size))
    g_rgb = np.sign(fwd["rgb"] - target) / target.size  # dL/d(rgb) of the L1 loss, from the oracle's forward
    _say("  gpu step")
    dcd = gs.Decoder.from_gen(sc, DEV)
    sp = gs.poses_tensor([cam["pose"]], DEV)
    gp = gs.poses_tensor(sc.group_poses, DEV)
    r = gs.Renderer([gs.SceneShape(n, -1, False, offs)], [cam], opts=gs.PRODUCTION, device=DEV)
    d = dcd.forward(sp[0], gp)
    (out,) = r.forward([d], sp, gp)
    go = torch.zeros_like(out)
    gflat = go.view(go.shape[0], -1)
    gflat[:3, torch.from_numpy(rays).to(DEV)] = torch.from_numpy(g_rgb.astype(np.float32)).to(DEV)
    (gsurf,) = r.backward([d], sp, gp, [out], [go])
    ga = dcd.backward(sp[0], gp, gsurf)
    torch.cuda.synchronize()
    crop = out.view(out.shape[0], -1)[:, torch.from_numpy(rays).to(DEV)].cpu().numpy()
    assert np.abs(crop[:3] - fwd["rgb"]).max() < 1e-3
    _say("  oracle adjoint")
    res = raster.render(sc32, cam, o, rays=rays, params={k: v.detach().requires_grad_(True) for k, v in dec.items()},
                        grad_out={"rgb": g_rgb})
    tot = sum((dec[k] * torch.as_tensor(res["grads"][k])).sum() for k in res["grads"])
    keys = list(leaves.keys())
    rg = dict(zip(keys, torch.autograd.grad(tot, [leaves[k] for k in keys])))
    for k in keys:
        r_ = rg[k].numpy()
        g = ga[k.split("_")[0]].cpu().numpy().astype(np.float64).reshape(r_.shape)
        err, scale = float(np.abs(g - r_).max()), float(np.abs(r_).max())
        _say(f"  {k}: err {err:.3e} scale {scale:.3e}")
        assert scale > 0
        assert err <= 1e-3 * scale + 1e-9, (k, err, scale)
