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

Tolerances as in the small parity tests; production-mode pixels whose oracle
margin to a compositing threshold is below 1e-4 relative are excluded and
counted; every pixel outside tolerance must be one of them (camera: at most
2 % excluded; LiDAR: at most 1 % outside tolerance).
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gen import scenes as S  # noqa: E402
from oracle import decode as odec  # noqa: E402
from oracle import raster, spec32  # noqa: E402
from tests.gpu_common import (DEV, camera_bad_pixels, camera_errors, check_integer_parity,  # noqa: E402
                              lidar_bad_rays, lidar_errors, oracle_opts, within)

import paper_2503_11731_amd as gs  # noqa: E402

MARGIN = 1e-4


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
    ref = raster.render(scene, cam, o, rays=rays, margins=True)
    got = out.reshape(out.shape[0], -1)[:, torch.from_numpy(rays).to(DEV)].cpu().numpy()
    mask = ref["margin"] >= MARGIN
    errs = camera_errors(got, ref, mask)
    bad = camera_bad_pixels(got, ref)
    _say(f"  pairs {n_pairs} segments {status['segments']} near-threshold {int((~mask).sum())} "
         f"out-of-tol {int(bad.sum())} errs {errs}")
    assert within(errs), errs
    assert not (bad & mask).any()
    assert (~mask).sum() <= 0.02 * mask.size


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
    ref = raster.render(scene, lid, o, rays=rays, margins=True)
    got = out.reshape(out.shape[0], -1)[:, torch.from_numpy(rays).to(DEV)].cpu().numpy()
    mask = ref["margin"] >= MARGIN
    errs = lidar_errors(got, ref, mask)
    bad = lidar_bad_rays(got, ref)
    _say(f"  near-threshold {int((~mask).sum())} out-of-tol {int(bad.sum())} errs {errs}")
    assert within(errs), errs
    # every ray outside tolerance has some compositing decision at a threshold, and there are few;
    # a ray of the heaviest tile crosses up to ~3e5 pairs, so many rays have some near-threshold decision
    assert not (bad & mask).any()
    assert bad.sum() <= 0.01 * bad.size


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
    for k in ("opacity", "scale", "intensity"):
        errs[k] = float(np.abs(d[k].cpu().numpy().astype(np.float64) - ref_dec[k].numpy()).max())
    for k in ("quat", "mean"):
        ref = ref_dec[k].numpy()
        errs[k] = float((np.abs(d[k].cpu().numpy().astype(np.float64) - ref) / np.maximum(1.0, np.abs(ref))).max())
    _say(f"  {errs}")
    for k, e in errs.items():
        assert e <= 1e-4, (k, e)
