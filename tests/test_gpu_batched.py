"""Batched multi-sensor step (one record space, one sort, one persistent launch) and HIP-graph replay.

Two rigs, each with three cameras of uneven resolution (ragged tiles) and a
LiDAR:
  - an explicit-surfel corridor (one static group): the batched layout runs
    the per-pair arithmetic of the per-sensor layout in the same per-tile
    order, so its outputs are bit-identical to the per-sensor plan, and both
    are compared with the FP64 oracle;
  - a neural-Gaussian rig with three posed vehicle actors (own MLPs, random
    yaw and position): every sensor decodes its scene (BF16 MFMA) and all
    sensors render in one batched launch; compared with the oracle's chain
    (FP64 decode of the same bf16 parameters, then the FP64 render), forward
    per pixel and adjoint down to the anchors and MLP weights.  The same
    oracle-decoded surfels rounded to FP32 and fed to the batched plan as
    explicit surfels give bit-exact pair lists.
Graph replays are compared with eager runs and with the oracle after every
replay, with pose updates and unrelated eager work in between.
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gen import scenes as S  # noqa: E402
from oracle import decode as odec  # noqa: E402
from oracle import raster, spec32  # noqa: E402
from tests.gpu_common import ALT_TOL, DEV, assert_verified, gmap_of, median_channel, verify  # noqa: E402

import paper_2503_11731_amd as gs  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cameras():
    return [S.pinhole(200, 120, 100.0, pose=S.camera_yaw_pose(0.0)),
            S.pinhole(160, 96, 80.0, pose=S.camera_yaw_pose(55.0)),
            S.pinhole(100, 60, 50.0, pose=S.camera_yaw_pose(180.0))]


def _rig():
    sc = S.corridor_surfels(seed=9, n=30000, sh_degree=-1, z_lo=-25, z_hi=40, with_intensity=True)
    scene = dict(mean=sc.mean, quat=sc.quat, scale=sc.scale, opacity=sc.opacity, rgb=sc.rgb, intensity=sc.intensity,
                 group_offsets=sc.group_offsets, group_poses=sc.group_poses)
    cams = _cameras()
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


def _check_pairs(rb, sensor_scenes, sensors, tiles, rec_bases):
    """Integer parity of a batched plan's pair list and per-sensor visible
    counts, sensor by sensor."""
    v = rb.inspect(0)
    n_vis = rb.status()["n_visible"]
    tile = v["pair_tile"].cpu().numpy().astype(np.int64)
    rec = v["pair_surfel"].cpu().numpy().astype(np.int64)
    toff = 0
    for i, s in enumerate(sensors):
        tw, th = tiles[i] if tiles else (32, 8)
        o = raster.make_opts(gs.PRODUCTION, tile_w=tw, tile_h=th)
        bins = raster.spec_bins(sensor_scenes[i], s, o)
        t_ref, s_ref = spec32.tile_pairs_fast(bins)
        n_t = bins["n_tx"] * bins["n_ty"]
        sel = (tile >= toff) & (tile < toff + n_t)
        np.testing.assert_array_equal(tile[sel] - toff, t_ref)
        np.testing.assert_array_equal(rec[sel] - rec_bases[i], s_ref)
        assert n_vis[i] == int(np.count_nonzero(bins["visible"])), (i, n_vis[i])
        toff += n_t
    assert toff == v["n_tiles"]


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
    assert not rb.status()["overflow"]
    assert ra.status()["n_visible"] == rb.status()["n_visible"]
    n = scene["mean"].shape[1]
    _check_pairs(rb, [scene] * len(sensors), sensors, tiles, [i * n for i in range(len(sensors))])
    for i, s in enumerate(sensors):
        tw, th = tiles[i] if tiles else (32, 8)
        ref = raster.render(scene, s, raster.make_opts(gs.PRODUCTION, tile_w=tw, tile_h=th), alternatives=ALT_TOL)
        v = verify(ob[i].cpu().numpy(), ref, s["kind"])
        _say(f"  sensor {i}: {v}")
        assert_verified(v, f"sensor {i}")


def test_batched_sensor_with_nothing_visible():
    """A camera turned away from the whole scene between two that see it: its
    visible count is zero, the others' match the oracle's culling, and the
    batched outputs equal the per-sensor plan's."""
    _say("batched forward with an empty sensor")
    scene, sensors = _rig()
    away = dict(sensors[1], pose=S.translate_pose(S.camera_yaw_pose(180.0), (0.0, 0.0, -1.0e4)))
    sensors = [sensors[0], away, sensors[2], sensors[3]]
    scenes, sp, gp = _tensors(scene, sensors)
    ra = _renderer(scene, sensors, False, [(32, 8)] * len(sensors))
    rb = _renderer(scene, sensors, True)
    oa = ra.forward(scenes, sp, gp)
    ob = rb.forward(scenes, sp, gp)
    torch.cuda.synchronize()
    for a, b in zip(oa, ob):
        assert torch.equal(a, b)
    st = rb.status()
    assert not st["overflow"]
    assert st["n_visible"][1] == 0
    assert ra.status()["n_visible"] == st["n_visible"]
    n = scene["mean"].shape[1]
    _check_pairs(rb, [scene] * len(sensors), sensors, None, [i * n for i in range(len(sensors))])


def _oracle_scene_grads(scene, sensors, outs_grad, scene_of):
    """Oracle gradients per scene, summed over the sensors that render it."""
    acc = {}
    for i, s in enumerate(sensors):
        go = outs_grad[i]
        gmap = gmap_of(go, s["kind"])
        sc = dict(scene)
        if s["kind"] == "pinhole":
            sc.pop("intensity", None)
        else:
            sc.pop("rgb", None)
        ref = raster.render(sc, s, raster.make_opts(gs.PRODUCTION, tile_w=32, tile_h=8),
                            grad_out={k: v.astype(np.float64) for k, v in gmap.items()})
        d = acc.setdefault(scene_of[i], {})
        for k, g in ref["grads"].items():
            d[k] = d.get(k, 0.0) + g
    return acc


def test_batched_backward_matches_per_sensor_and_oracle():
    _say("batched backward")
    scene, sensors = _rig()
    scenes, sp, gp = _tensors(scene, sensors)
    ra = _renderer(scene, sensors, False, [(32, 8)] * len(sensors))  # the batched default tiles
    rb = _renderer(scene, sensors, True)
    res = []
    gos = None
    for r in (ra, rb):
        outs = r.forward(scenes, sp, gp)
        rng = np.random.default_rng(1)
        gos = [rng.standard_normal(tuple(o.shape)).astype(np.float32) for o in outs]
        for g, s in zip(gos, sensors):
            g[median_channel(s["kind"])] = 0.0  # the median's gradient is tested per sensor
        res.append(r.backward(scenes, sp, gp, outs, [torch.from_numpy(g).to(DEV) for g in gos]))
    torch.cuda.synchronize()
    for si in range(2):
        for k, ga in res[0][si].items():
            gb = res[1][si][k]
            scale = float(ga.abs().max())
            err = float((ga - gb).abs().max())
            assert err <= 1e-5 * scale + 1e-7, (si, k, err, scale)
    ref = _oracle_scene_grads(scene, sensors, gos, [s["scene"] for s in sensors])
    for si in range(2):
        for k, gr in ref[si].items():
            g = res[1][si][k].cpu().numpy().astype(np.float64)
            err, scale = float(np.abs(g - gr).max()), float(np.abs(gr).max())
            _say(f"  scene {si} {k}: err {err:.3e} scale {scale:.3e}")
            assert err <= 1e-3 * scale + 1e-6, (si, k, err, scale)


# ----------------------------------------------------------------------------
# neural-Gaussian rig with posed actors
# ----------------------------------------------------------------------------

def _decoded_rig():
    cam_sc = S.corridor_anchors(seed=61, n_anchors=1200, sensor_kind="pinhole", z_lo=-20, z_hi=40, n_assets=3,
                                asset_anchors=120)
    lid_sc = S.corridor_anchors(seed=62, n_anchors=1200, sensor_kind="lidar", z_lo=-20, z_hi=40, n_assets=3,
                                asset_anchors=120)
    # actors ahead, ahead-left and behind the rig (random yaw), so that every camera sees one
    spots = [(-3.5, 10.0), (-7.5, 6.0), (3.5, -9.0)]
    for sc in (cam_sc, lid_sc):
        rng = np.random.default_rng(7)
        for g in range(1, len(sc.mlps)):
            x, z = spots[g - 1]
            sc.group_poses[g] = S.yaw_translate_pose(rng.uniform(0, 2 * np.pi), x, S.GROUND_Y, z)
    sensors = _cameras() + [S.lidar_spinning(n_beams=32, n_az=360)]
    for i, s in enumerate(sensors):
        s["scene"] = i
    return cam_sc, lid_sc, sensors


def _anchor_dict(sc):
    return dict(xyz=sc.xyz.astype(np.float64), scaling=sc.scaling.astype(np.float64),
                offsets=sc.offsets.astype(np.float64), feat=S.bf16_bits_to_f32(sc.feat_bf16).astype(np.float64),
                group_offsets=sc.group_offsets)


class _GpuRig:
    """Decoders of the two anchor scenes and one batched plan over all sensors (scene i = sensor i's decode)."""

    def __init__(self, cam_sc, lid_sc, sensors, tiles=None):
        self.cam_sc, self.lid_sc, self.sensors = cam_sc, lid_sc, sensors
        self.dc = gs.Decoder.from_gen(cam_sc, DEV)
        self.dl = gs.Decoder.from_gen(lid_sc, DEV)
        self.sp = gs.poses_tensor([s["pose"] for s in sensors], DEV)
        self.gp_c = gs.poses_tensor(cam_sc.group_poses, DEV)
        self.gp_l = gs.poses_tensor(lid_sc.group_poses, DEV)
        shapes, sens = [], []
        for i, s in enumerate(sensors):
            an = cam_sc if s["kind"] == "pinhole" else lid_sc
            offs = tuple(int(x) * an.k for x in an.group_offsets)
            shapes.append(gs.SceneShape(an.n_anchors * an.k, -1, s["kind"] != "pinhole", offs))
            s = dict(s)
            if tiles:
                s["tile"] = tiles[i]
            sens.append(s)
        self.r = gs.Renderer(shapes, sens, opts=gs.PRODUCTION, device=DEV, batched=True)
        self.gp_all = torch.cat([self.gp_c if s["kind"] == "pinhole" else self.gp_l for s in sensors]).contiguous()
        self.ds = [(self.dc if s["kind"] == "pinhole" else self.dl).new_decoded() for s in sensors]
        self.outs = self.r.new_outputs()

    def forward(self):
        for i, s in enumerate(self.sensors):
            if s["kind"] == "pinhole":
                self.dc.forward(self.sp[i], self.gp_c, out=self.ds[i])
            else:
                self.dl.forward(self.sp[i], self.gp_l, out=self.ds[i])
        self.r.forward(self.ds, self.sp, self.gp_all, outputs=self.outs)
        return self.outs

    def backward(self, gouts):
        gsurf = self.r.backward(self.ds, self.sp, self.gp_all, self.outs, gouts)
        agc = agl = None
        for i, s in enumerate(self.sensors):
            if s["kind"] == "pinhole":
                agc = self.dc.backward(self.sp[i], self.gp_c, gsurf[i], grads=agc)
            else:
                agl = self.dl.backward(self.sp[i], self.gp_l, gsurf[i], grads=agl)
        return agc, agl


def _oracle_decoded(an_sc, sensor, kind, leaves=None):
    poses_s = np.stack([spec32.compose_pose(sensor["pose"], g) for g in an_sc.group_poses])
    dec = odec.decode(_anchor_dict(an_sc), an_sc.mlps, poses_s, kind, params=leaves)
    n = an_sc.n_anchors * an_sc.k
    sc32 = {k: np.ascontiguousarray(v.detach().numpy().astype(np.float32)) for k, v in dec.items()}
    sc32.update(group_offsets=np.array([int(x) * an_sc.k for x in an_sc.group_offsets], np.int32),
                group_poses=an_sc.group_poses)
    assert sc32["mean"].shape[1] == n
    return dec, sc32


def _oracle_outputs(cam_sc, lid_sc, sensors):
    refs = []
    for s in sensors:
        an = cam_sc if s["kind"] == "pinhole" else lid_sc
        with torch.no_grad():
            dec, sc32 = _oracle_decoded(an, s, s["kind"])
        refs.append(raster.render(sc32, s, raster.make_opts(gs.PRODUCTION, tile_w=32, tile_h=8), params=dec,
                                  alternatives=ALT_TOL))
    return refs


def test_decoded_posed_rig_forward_matches_oracle_chain():
    """GPU decode (BF16 MFMA) -> one batched launch vs oracle decode (FP64) -> oracle render, every sensor."""
    _say("decoded posed rig forward vs oracle")
    cam_sc, lid_sc, sensors = _decoded_rig()
    rig = _GpuRig(cam_sc, lid_sc, sensors)
    outs = rig.forward()
    torch.cuda.synchronize()
    st = rig.r.status()
    assert not st["overflow"]
    refs = _oracle_outputs(cam_sc, lid_sc, sensors)
    for i, (s, ref) in enumerate(zip(sensors, refs)):
        v = verify(outs[i].cpu().numpy(), ref, s["kind"])
        an = cam_sc if s["kind"] == "pinhole" else lid_sc
        grp = np.repeat(np.arange(len(an.mlps)), np.diff(an.group_offsets) * an.k)
        seen = np.unique(grp[ref["bins"]["touch"]]).tolist()
        _say(f"  sensor {i} ({s['kind']} {s['width']}x{s['height']}): groups seen {seen} {v}")
        assert len(seen) >= 2, seen
        assert_verified(v, f"sensor {i}")


def test_decoded_posed_rig_explicit_surfels_bit_exact_pairs():
    """The oracle's decoded surfels (rounded to FP32) as explicit scenes of the batched plan: pair lists
    bit-exact per sensor, floats per pixel."""
    _say("oracle-decoded posed rig through the batched plan")
    cam_sc, lid_sc, sensors = _decoded_rig()
    scenes32, shapes = [], []
    for s in sensors:
        an = cam_sc if s["kind"] == "pinhole" else lid_sc
        with torch.no_grad():
            _, sc32 = _oracle_decoded(an, s, s["kind"])
        scenes32.append(sc32)
        shapes.append(gs.SceneShape(sc32["mean"].shape[1], -1, s["kind"] != "pinhole",
                                    tuple(int(x) for x in sc32["group_offsets"])))
    r = gs.Renderer(shapes, sensors, opts=gs.PRODUCTION, device=DEV, batched=True)
    st = [gs.scene_tensors(sc, DEV) for sc in scenes32]
    sp = gs.poses_tensor([s["pose"] for s in sensors], DEV)
    gp = gs.poses_tensor(np.concatenate([sc["group_poses"] for sc in scenes32]), DEV)
    outs = r.forward(st, sp, gp)
    torch.cuda.synchronize()
    bases = np.cumsum([0] + [sc["mean"].shape[1] for sc in scenes32])[:-1]
    _check_pairs(r, scenes32, sensors, None, bases)
    for i, s in enumerate(sensors):
        ref = raster.render(scenes32[i], s, raster.make_opts(gs.PRODUCTION, tile_w=32, tile_h=8),
                            alternatives=ALT_TOL)
        v = verify(outs[i].cpu().numpy(), ref, s["kind"])
        _say(f"  sensor {i}: {v}")
        assert_verified(v, f"sensor {i}")


def test_decoded_posed_rig_backward_matches_oracle_chain():
    """Adjoint of the whole batched step down to anchors and MLP weights vs oracle autograd through
    decode and render, summed over the sensors that share each anchor scene."""
    _say("decoded posed rig backward vs oracle")
    cam_sc, lid_sc, sensors = _decoded_rig()
    rig = _GpuRig(cam_sc, lid_sc, sensors)
    outs = rig.forward()
    rng = np.random.default_rng(12)
    gos = [rng.standard_normal(tuple(o.shape)).astype(np.float32) for o in outs]
    for g, s in zip(gos, sensors):
        g[median_channel(s["kind"])] = 0.0  # the median's gradient is tested per sensor
    agc, agl = rig.backward([torch.from_numpy(g).to(DEV) for g in gos])
    torch.cuda.synchronize()
    for kind, an, ag in (("pinhole", cam_sc, agc), ("lidar", lid_sc, agl)):
        G = len(an.mlps)
        leaves = {k: torch.as_tensor(v).requires_grad_(True) for k, v in _anchor_dict(an).items()
                  if k != "group_offsets"}
        for g in range(G):
            for name in ("w1", "b1", "w2", "b2"):
                leaves[f"{name}_{g}"] = torch.as_tensor(an.mlps[g][name].astype(np.float64)).requires_grad_(True)
        total = 0.0
        for i, s in enumerate(sensors):
            if s["kind"] != kind:
                continue
            dec, sc32 = _oracle_decoded(an, s, kind, leaves=leaves)
            go = gos[i]
            gmap = gmap_of(go, kind)
            res = raster.render(sc32, s, raster.make_opts(gs.PRODUCTION, tile_w=32, tile_h=8),
                                params={k: v.detach().requires_grad_(True) for k, v in dec.items()},
                                grad_out={k: v.astype(np.float64) for k, v in gmap.items()})
            total = total + sum((dec[k] * torch.as_tensor(res["grads"][k])).sum() for k in res["grads"])
        keys = list(leaves.keys())
        rg = dict(zip(keys, torch.autograd.grad(total, [leaves[k] for k in keys], allow_unused=True)))
        checks = {k: rg[k].numpy() for k in ("xyz", "scaling", "offsets", "feat")}
        for name in ("w1", "b1", "w2", "b2"):
            checks[name] = np.stack([rg[f"{name}_{g}"].numpy() for g in range(G)])
        for k, r_ in checks.items():
            g = ag[k].cpu().numpy().astype(np.float64).reshape(r_.shape)
            err, scale = float(np.abs(g - r_).max()), float(np.abs(r_).max())
            _say(f"  {kind} {k}: err {err:.3e} scale {scale:.3e}")
            assert err <= 1e-3 * scale + 1e-7, (kind, k, err, scale)


def test_graph_replay_of_decode_and_render_matches_eager_and_oracle():
    """The whole decoded step (four decodes + one batched render) captured in one graph; after each
    pose update the replay equals an eager run and the oracle at the new poses."""
    _say("graph replay of the decoded step")
    cam_sc, lid_sc, sensors = _decoded_rig()
    rg = _GpuRig(cam_sc, lid_sc, sensors)
    re_ = _GpuRig(cam_sc, lid_sc, sensors)
    stream = torch.cuda.Stream()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.stream(stream):
        rg.forward()  # warm (lazy module loading) before capture
        stream.synchronize()
        with torch.cuda.graph(graph, stream=stream):
            rg.forward()
    for step in range(3):
        shift = torch.zeros_like(rg.sp)
        shift[:, 3] = 0.07 * (step + 1)
        new_sp = rg.sp + shift
        rg.sp.copy_(new_sp)
        re_.sp.copy_(new_sp)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            graph.replay()
        torch.cuda.current_stream().wait_stream(stream)
        ref = re_.forward()
        x = torch.randn(512, 512, device=DEV) @ torch.randn(512, 512, device=DEV)  # unrelated eager work
        torch.cuda.synchronize()
        del x
        for a, b in zip(rg.outs, ref):
            assert torch.equal(a, b), f"replay {step} differs from eager"
        if step == 2:
            moved = [dict(s, pose=rg.sp[i].cpu().numpy().reshape(3, 4)) for i, s in enumerate(sensors)]
            refs = _oracle_outputs(cam_sc, lid_sc, moved)
            for i, (s, ref_o) in enumerate(zip(moved, refs)):
                v = verify(rg.outs[i].cpu().numpy(), ref_o, s["kind"])
                _say(f"  replay {step} sensor {i}: {v}")
                assert_verified(v, f"replay sensor {i}")


def test_step_capture_through_the_abi_replays_forward_and_backward():
    """A whole training step -- four decodes, one batched render, the adjoint render and the four decode
    adjoints (allocation-free), gradient clears in between -- captured through gs_plan_begin_capture /
    gs_plan_end_capture and replayed by gs_plan_launch: after each pose update the replay's outputs equal an
    eager step and its gradients match the eager ones (atomic summation order aside)."""
    _say("ABI step capture: forward + backward")
    cam_sc, lid_sc, sensors = _decoded_rig()
    rg = _GpuRig(cam_sc, lid_sc, sensors)
    re_ = _GpuRig(cam_sc, lid_sc, sensors)
    rng = np.random.default_rng(5)
    gouts = [torch.from_numpy(rng.standard_normal(tuple(o.shape)).astype(np.float32)).to(DEV) for o in rg.outs]
    gsurf = [{k: torch.zeros_like(v) for k, v in d.items()} for d in rg.ds]

    def zeros(dec):
        z = lambda t: torch.zeros(t.shape, dtype=torch.float32, device=DEV)
        return dict(xyz=z(dec.xyz), scaling=z(dec.scaling), offsets=z(dec.offsets), feat=z(dec.feat),
                    w1=z(dec.w1), b1=z(dec.b1), w2=z(dec.w2), b2=z(dec.b2))

    agc, agl = zeros(rg.dc), zeros(rg.dl)

    def step():
        rg.forward()
        for d in gsurf + [agc, agl]:
            for v in d.values():
                v.zero_()
        rg.r.backward(rg.ds, rg.sp, rg.gp_all, rg.outs, gouts, grads=gsurf)
        for i, s in enumerate(sensors):
            if s["kind"] == "pinhole":
                rg.dc.backward(rg.sp[i], rg.gp_c, gsurf[i], grads=agc, noalloc=True)
            else:
                rg.dl.backward(rg.sp[i], rg.gp_l, gsurf[i], grads=agl, noalloc=True)

    stream = torch.cuda.Stream()
    stream.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(stream):
        step()  # warm (lazy module loading) before capture
        stream.synchronize()
        rg.r.begin_capture()
        step()
        rg.r.end_capture()
    for it in range(3):
        shift = torch.zeros_like(rg.sp)
        shift[:, 3] = 0.06 * (it + 1)
        new_sp = rg.sp + shift
        rg.sp.copy_(new_sp)
        re_.sp.copy_(new_sp)
        stream.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(stream):
            rg.r.launch()
        torch.cuda.current_stream().wait_stream(stream)
        ref = [o.clone() for o in re_.forward()]
        rc, rl = re_.backward(gouts)
        x = torch.randn(512, 512, device=DEV) @ torch.randn(512, 512, device=DEV)  # unrelated eager work
        torch.cuda.synchronize()
        del x
        for a, b in zip(rg.outs, ref):
            assert torch.equal(a, b), f"replay {it}: outputs differ from eager"
        for got, want in ((agc, rc), (agl, rl)):
            for k in want:
                err = float((got[k] - want[k]).abs().max())
                scale = float(want[k].abs().max())
                assert scale > 0 and err <= 1e-4 * scale, (it, k, err, scale)
        _say(f"  replay {it}: outputs bit-equal, gradients within 1e-4 of eager")
    with torch.cuda.stream(stream):
        st = rg.r.status()
    assert st["step_launches"] == 3 and not st["overflow"]


def test_plan_graph_replay_matches_eager_with_pose_updates():
    _say("plan graph replay")
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
        sp.copy_(sp + shift)
        stream.wait_stream(torch.cuda.current_stream())  # the replay must see the new poses
        with torch.cuda.stream(stream):
            rg.forward(scenes, sp, gp, outputs=outs)  # replay
        stream.synchronize()
        ref = re_.forward(scenes, sp, gp)  # eager
        x = torch.randn(1000, 1000, device=DEV) @ torch.randn(1000, 1000, device=DEV)  # unrelated eager work
        torch.cuda.synchronize()
        del x
        for a, b in zip(outs, ref):
            assert torch.equal(a, b), f"replay {step} differs"
    with torch.cuda.stream(stream):
        assert rg.status()["graph_replays"] == 4
    assert re_.status()["graph_replays"] == 0


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
