"""Batched multi-sensor step (one record space, one sort, one persistent launch) and HIP-graph replay.

The batched layout runs exactly the per-pair arithmetic of the per-sensor
layout in the same per-tile order, so forward outputs are bit-identical;
adjoints differ only in atomic summation order.  Graph replays are checked
against eager runs after every replay, with eager work and pose updates in
between.
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gen import scenes as S  # noqa: E402
from oracle import raster, spec32  # noqa: E402
from tests.gpu_common import DEV  # noqa: E402

import paper_2503_11731_amd as gs  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rig():
    sc = S.corridor_surfels(seed=9, n=30000, sh_degree=-1, z_lo=-25, z_hi=40, with_intensity=True)
    scene = dict(mean=sc.mean, quat=sc.quat, scale=sc.scale, opacity=sc.opacity, rgb=sc.rgb, intensity=sc.intensity,
                 group_offsets=sc.group_offsets, group_poses=sc.group_poses)
    cams = [S.pinhole(200, 120, 100.0, pose=S.camera_yaw_pose(0.0)),
            S.pinhole(160, 96, 80.0, pose=S.camera_yaw_pose(55.0)),
            S.pinhole(160, 96, 80.0, pose=S.camera_yaw_pose(180.0))]
    lid = S.lidar_spinning(n_beams=32, n_az=400)
    sensors = cams + [dict(lid, scene=1)]
    for c in cams:
        c["scene"] = 0
    return scene, sensors


def _renderer(scene, sensors, batched, tiles=None):
    n = scene["mean"].shape[1]
    shapes = [gs.SceneShape(n, -1, False, (0, n)), gs.SceneShape(n, -1, True, (0, n))]
    sens = []
    for i, s in enumerate(sensors):
        s = dict(s)
        if tiles is not None:
            s["tile"] = tiles[i]
        sens.append(s)
    return gs.Renderer(shapes, sens, opts=gs.PRODUCTION, device=DEV, batched=batched)


def _tensors(scene, sensors):
    st = gs.scene_tensors(scene, DEV)
    cam_scene = {k: st[k] for k in ("mean", "quat", "scale", "opacity", "rgb")}
    lid_scene = {k: st[k] for k in ("mean", "quat", "scale", "opacity", "intensity")}
    sp = gs.poses_tensor([s["pose"] for s in sensors], DEV)
    gp = gs.poses_tensor(np.concatenate([scene["group_poses"], scene["group_poses"]]), DEV)
    return [cam_scene, lid_scene], sp, gp


@pytest.mark.parametrize("tiles", [None, [(32, 8), (16, 16), (8, 32), (16, 16)]])
def test_batched_forward_matches_per_sensor_and_oracle(tiles):
    _say(f"batched forward tiles={tiles}")
    scene, sensors = _rig()
    scenes, sp, gp = _tensors(scene, sensors)
    # same tile shapes on both sides: the batched defaults (32x8 for every
    # sensor) differ from the per-sensor LiDAR default (16x8)
    ra = _renderer(scene, sensors, False, tiles or [(32, 8)] * len(sensors))
    rb = _renderer(scene, sensors, True, tiles)
    oa = ra.forward(scenes, sp, gp)
    ob = rb.forward(scenes, sp, gp)
    torch.cuda.synchronize()
    for a, b in zip(oa, ob):
        assert torch.equal(a, b)
    st = rb.status()
    assert not st["overflow"]
    # integer parity of the batched pair list, sensor by sensor
    v = rb.inspect(0)
    tile = v["pair_tile"].cpu().numpy().astype(np.int64)
    rec = v["pair_surfel"].cpu().numpy().astype(np.int64)
    n = scene["mean"].shape[1]
    toff = 0
    for i, s in enumerate(sensors):
        tw, th = (tiles[i] if tiles else (32, 8))
        o = raster.make_opts(gs.PRODUCTION, tile_w=tw, tile_h=th)
        bins = raster.spec_bins(scene, s, o)
        t_ref, s_ref = spec32.tile_pairs_fast(bins)
        n_t = bins["n_tx"] * bins["n_ty"]
        sel = (tile >= toff) & (tile < toff + n_t)
        np.testing.assert_array_equal(tile[sel] - toff, t_ref)
        np.testing.assert_array_equal(rec[sel] - i * n, s_ref)
        toff += n_t
    assert toff == v["n_tiles"]


def test_batched_backward_matches_per_sensor():
    _say("batched backward")
    scene, sensors = _rig()
    scenes, sp, gp = _tensors(scene, sensors)
    ra = _renderer(scene, sensors, False, [(32, 8)] * len(sensors))  # the batched default tiles
    rb = _renderer(scene, sensors, True)
    rng = np.random.default_rng(1)
    res = []
    for r in (ra, rb):
        outs = r.forward(scenes, sp, gp)
        go = [torch.from_numpy(rng.standard_normal(tuple(o.shape)).astype(np.float32)).to(DEV) for o in outs]
        rng = np.random.default_rng(1)
        res.append(r.backward(scenes, sp, gp, outs, go))
    torch.cuda.synchronize()
    for si in range(2):
        for k, ga in res[0][si].items():
            gb = res[1][si][k]
            scale = float(ga.abs().max())
            err = float((ga - gb).abs().max())
            assert err <= 1e-5 * scale + 1e-7, (si, k, err, scale)


def test_graph_replay_matches_eager_with_pose_updates():
    _say("graph replay")
    scene, sensors = _rig()
    scenes, sp, gp = _tensors(scene, sensors)
    rg = _renderer(scene, sensors, True)
    re_ = _renderer(scene, sensors, True)
    stream = torch.cuda.Stream()
    outs = rg.new_outputs()
    with torch.cuda.stream(stream):
        rg.forward(scenes, sp, gp, outputs=outs)  # warm (lazy module loading) before capture
        stream.synchronize()
        rg.capture(scenes, sp, gp, outs)
    for step in range(4):
        # move every sensor a little (in place: the graph reads the pose buffer)
        shift = torch.zeros_like(sp)
        shift[:, 3] = 0.05 * (step + 1)
        sp_new = sp + shift
        sp.copy_(sp_new)
        with torch.cuda.stream(stream):
            rg.forward(scenes, sp, gp, outputs=outs)  # replay
        stream.synchronize()
        ref = re_.forward(scenes, sp, gp)  # eager
        x = torch.randn(1000, 1000, device=DEV) @ torch.randn(1000, 1000, device=DEV)  # unrelated eager work
        torch.cuda.synchronize()
        del x
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), f"replay {step} differs"


def test_autotune_picks_valid_shapes_and_same_image():
    """The tuner returns candidates from its lists; a plan built with them renders what the default plan renders
    up to FP32 rounding order (tile shape and segment length change nothing else)."""
    from paper_2503_11731_amd import autotune as at
    _say("autotune")
    scene, sensors = _rig()
    scenes, sp, gp = _tensors(scene, sensors)
    n = scene["mean"].shape[1]
    shapes = [gs.SceneShape(n, -1, s["kind"] != "pinhole", (0, n)) for s in sensors]
    scs = [scenes[0] if s["kind"] == "pinhole" else scenes[1] for s in sensors]
    gps = [gs.poses_tensor(scene["group_poses"], DEV)] * len(sensors)
    res = at.autotune(shapes, scs, sensors, sp, gps, batched=True, segments=[256, 1024], steps=1, warmup=1,
                      cache_path=None)
    assert len(res.tiles) == len(sensors)
    assert all(t in at.TILES_256 for t in res.tiles)
    assert res.segment_pairs in (256, 1024)
    rt = _renderer(scene, sensors, True, res.tiles)
    ra = _renderer(scene, sensors, True)
    ot = rt.forward(scenes, sp, gp)
    oa = ra.forward(scenes, sp, gp)
    torch.cuda.synchronize()
    for a, b in zip(ot, oa):
        # tile origins enter the FP32 offsets, so a ray next to a skip/stop threshold may decide differently
        frac = float(((a - b).abs() > 1e-4).float().mean())
        assert frac <= 1e-3, frac
