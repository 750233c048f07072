"""Double-buffered zone swap-in (Sec. III-A, large-scale scenes) on the GPU.

1. Buffer contents: after every acquire, each field of the buffer equals the
   zone oracle's gather of that zone (bit for bit: anchor rows in ascending
   order, the fill value up to the capacity, columns past the capacity
   untouched, per-zone blocks whole), over a sequence of uploads that reuses
   both buffers, queues two uploads into one buffer, and streams an empty
   zone.  Error paths of the C-ABI.
2. Streamed render: zone anchors swapped into a capacity-padded buffer
   (padding anchors have zero scaling), decoded and rendered, against (a) the
   oracle decode of the zone's anchors with the zone's MLP, (b) the oracle
   render of the decoded surfels, and (c) a direct decode + render of exactly
   the zone's anchors, which it must equal bit for bit (padding changes
   nothing).
3. A drive across zone boundaries with the upload of the next zone
   overlapping the renders of the current one: every frame equals the direct
   render of its zone.
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gen import scenes as S  # noqa: E402
from oracle import decode as odec  # noqa: E402
from oracle import raster, spec32  # noqa: E402
from oracle import zones as Z  # noqa: E402
from tests.gpu_common import ALT_TOL, assert_verified, oracle_opts, verify  # noqa: E402

import paper_2503_11731_amd as gs  # noqa: E402
from paper_2503_11731_amd import _lib as L  # noqa: E402
from paper_2503_11731_amd import zones as gz  # noqa: E402

DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# ---------------------------------------------------------------------------
# 1. buffer contents
# ---------------------------------------------------------------------------

def _fields(rng, n, C, Zn):
    """Host arrays of several element sizes and their device pairs (7 resident columns past C)."""
    E = C + 7
    xyz = rng.standard_normal((3, n)).astype(np.float32)
    feat = rng.integers(0, 65535, (n, 32)).astype(np.uint16)
    code = rng.integers(0, 255, (2, n)).astype(np.uint8)
    wide = rng.standard_normal((1, n))
    block = rng.integers(0, 255, (Zn, 36)).astype(np.uint8)
    dev = lambda shape, dt, v: [torch.full(shape, v, dtype=dt, device=DEV) for _ in range(2)]
    d_xyz = dev((3, E), torch.float32, 5.0)
    d_feat = dev((E, 32), torch.int16, 3)
    d_code = dev((2, E), torch.uint8, 1)
    d_wide = dev((1, E), torch.float64, 2.0)
    d_block = dev((36,), torch.uint8, 0)
    fill_xyz = np.float32(1e9)
    fields = [
        gz.Field(xyz, d_xyz, 3, 4, n, E, fill=fill_xyz.tobytes()),
        gz.Field(feat, d_feat, 1, 64, n, E),
        gz.Field(code, d_code, 2, 1, n, E, fill=bytes([0x7F])),
        gz.Field(wide, d_wide, 1, 8, n, E, fill=np.float64(-3.5).tobytes()),
        gz.Field(block, d_block, 1, 36, per_zone=True),
    ]
    host = dict(xyz=xyz, feat=feat, code=code, wide=wide, block=block)
    dev_t = dict(xyz=d_xyz, feat=d_feat, code=d_code, wide=d_wide, block=d_block)
    return fields, host, dev_t, fill_xyz


def _check_buffer(b, zone, offs, idx, C, host, dev_t, fill_xyz):
    torch.cuda.current_stream().synchronize()
    L_ = idx[offs[zone]:offs[zone + 1]]
    exp = {
        "xyz": Z.zone_buffer(host["xyz"], L_, C, fill=fill_xyz),
        "feat": Z.zone_buffer(host["feat"][None], L_, C)[0],
        "code": Z.zone_buffer(host["code"], L_, C, fill=np.uint8(0x7F)),
        "wide": Z.zone_buffer(host["wide"], L_, C, fill=np.float64(-3.5)),
    }
    got = {k: dev_t[k][b].cpu().numpy() for k in ("xyz", "feat", "code", "wide")}
    assert np.array_equal(got["xyz"][:, :C], exp["xyz"]), ("xyz", zone, b)
    assert np.array_equal(got["feat"][:C].view(np.uint16), exp["feat"]), ("feat", zone, b)
    assert np.array_equal(got["code"][:, :C], exp["code"]), ("code", zone, b)
    assert np.array_equal(got["wide"][:, :C], exp["wide"]), ("wide", zone, b)
    # resident columns untouched
    assert np.all(got["xyz"][:, C:] == 5.0) and np.all(got["feat"][C:] == 3)
    assert np.all(got["code"][:, C:] == 1) and np.all(got["wide"][:, C:] == 2.0)
    assert np.array_equal(dev_t["block"][b].cpu().numpy(), host["block"][zone])


def test_swap_in_buffers_match_the_oracle_gather():
    _say("zone swap-in: buffer contents")
    rng = np.random.default_rng(5)
    n = 20000
    xyz_pos = np.stack([rng.uniform(-8, 8, n), rng.uniform(-1, 1, n), rng.uniform(0, 37.0, n)]).astype(np.float32)
    grid = gz.ZoneGrid(axis=(0, 2), origin=(-10.0, 0.0), size=10.0, pad=0.25, nx=1, ny=5)
    offs, idx = Z.partition(xyz_pos, grid.axis, grid.origin, grid.size, grid.pad, grid.nx, grid.ny)
    counts = np.diff(offs.astype(np.int64))
    assert counts[4] == 0 and counts[:4].min() > 0  # zone 4 (padded z >= 37.5) is empty
    C = int(counts.max()) + 3
    fields, host, dev_t, fill_xyz = _fields(rng, n, C, grid.n_zones)
    torch.cuda.synchronize()
    zs = gz.ZoneStream(offs, idx, C, n, fields, threads=3)
    with pytest.raises(L.GsError):
        zs.acquire(1)  # nothing queued yet
    for bad in ((5, 0), (-1, 0), (0, 2)):
        with pytest.raises(L.GsError):
            zs.prefetch(*bad)
    zs.prefetch(0, 0)
    assert zs.acquire(0) == (0, int(counts[0]))
    _check_buffer(0, 0, offs, idx, C, host, dev_t, fill_xyz)
    zs.prefetch(1, 1)
    assert zs.acquire(1) == (1, int(counts[1]))
    _check_buffer(1, 1, offs, idx, C, host, dev_t, fill_xyz)
    zs.release(0)
    zs.prefetch(2, 0)
    zs.prefetch(3, 0)  # queued behind it: the last upload wins
    with pytest.raises(L.GsError):
        zs.release(0)  # uploads into buffer 0 are still queued
    assert zs.acquire(0) == (3, int(counts[3]))
    _check_buffer(0, 3, offs, idx, C, host, dev_t, fill_xyz)
    zs.release(1)
    zs.prefetch(4, 1)  # the empty zone: all fill
    assert zs.acquire(1) == (4, 0)
    _check_buffer(1, 4, offs, idx, C, host, dev_t, fill_xyz)
    st = zs.stats(0)
    row_bytes = C * (3 * 4 + 64 + 2 * 1 + 8)
    assert st["zone"] == 3 and st["count"] == counts[3] and st["bytes"] == row_bytes + 36
    assert st["upload_ms"] > 0 and st["gather_ms"] >= 0
    _say(f"  stats {st}")
    zs.close()
    # create-time checks: capacity below a zone, an index beyond the anchors
    with pytest.raises(L.GsError):
        gz.ZoneStream(offs, idx, int(counts.max()) - 1, n, fields)
    bad_idx = idx.copy()
    bad_idx[0] = n
    with pytest.raises(L.GsError):
        gz.ZoneStream(offs, bad_idx, C, n, fields)


# ---------------------------------------------------------------------------
# 2. streamed decode + render
# ---------------------------------------------------------------------------

GRID = gz.ZoneGrid(axis=(0, 2), origin=(-20.0, -10.0), size=20.0, pad=0.25, nx=2, ny=3)
TILE = (32, 8)


def _scene(kind):
    return S.corridor_anchors(seed=41, n_anchors=3000, sensor_kind=kind, z_lo=-10.0, z_hi=50.0, n_assets=2,
                              asset_anchors=150)


def _anchor_dict(sc):
    return dict(xyz=sc.xyz.astype(np.float64), scaling=sc.scaling.astype(np.float64),
                offsets=sc.offsets.astype(np.float64), feat=S.bf16_bits_to_f32(sc.feat_bf16).astype(np.float64),
                group_offsets=sc.group_offsets)


def _sensor(kind, c):
    if kind == "pinhole":
        s = S.pinhole(96, 64, 60.0, pose=S.translate_pose(S.camera_yaw_pose(15.0), c))
    else:
        s = S.lidar_spinning(n_beams=16, n_az=180, pose=S.translate_pose(S.lidar_rig_pose(), c))
    s["tile"] = TILE
    return s


def _render(decoded, n_surf, goff_surf, sensor, gp, lidar):
    r = gs.Renderer([gs.SceneShape(n_surf, -1, lidar, tuple(goff_surf))], [sensor], opts=gs.PRODUCTION, device=DEV)
    sp = gs.poses_tensor(sensor["pose"], DEV)
    (o,) = r.forward([decoded], sp, gp)
    return o


def _direct(sc_zone, sensor, lidar):
    dec = gs.Decoder.from_gen(sc_zone, DEV)
    sp = gs.poses_tensor(sensor["pose"], DEV)
    gp = gs.poses_tensor(sc_zone.group_poses, DEV)
    d = dec.forward(sp[0], gp)
    n = sc_zone.n_anchors * sc_zone.k
    o = _render(d, n, [int(x) * sc_zone.k for x in sc_zone.group_offsets], sensor, gp, lidar)
    return d, o


@pytest.mark.parametrize("kind", ["pinhole", "lidar"])
def test_streamed_zone_render(kind):
    _say(f"streamed zone decode + render {kind}")
    lidar = kind == "lidar"
    sc = _scene(kind)
    static, actors = S.static_and_actors(sc)
    mlps = S.zone_mlps(7, GRID.n_zones, kind)
    za = gz.ZonedAnchors(static, mlps, GRID, lidar=lidar, device=DEV, actors=actors, threads=2)
    ro, ri = Z.partition(static["xyz"], GRID.axis, GRID.origin, GRID.size, GRID.pad, GRID.nx, GRID.ny)
    assert np.array_equal(za.offsets, ro) and np.array_equal(za.index, ri)
    zone = 3  # (i = 1, j = 1): x in [0, 20), z in [10, 30)
    c = (5.0, 0.0, 20.0)
    assert GRID.zone_of(c[0], c[2]) == zone
    sensor = _sensor(kind, c)
    za.stream.prefetch(zone, 0)
    assert za.stream.acquire(0) == (zone, int(za.counts[zone]))
    K = sc.k
    dec = za.decoders[0]
    sp = gs.poses_tensor(sensor["pose"], DEV)
    gp = gs.poses_tensor(sc.group_poses, DEV)
    d = dec.forward(sp[0], gp)
    o = _render(d, dec.A * K, [x * K for x in za.group_offsets], sensor, gp, lidar)
    torch.cuda.synchronize()
    # (a) decode of the zone's anchors (zone MLP) and of the actors, vs the oracle decode
    anchors = ri[ro[zone]:ro[zone + 1]]
    sz = S.zone_scene(sc, anchors, mlps[zone])
    poses_s = np.stack([spec32.compose_pose(sensor["pose"], g) for g in sz.group_poses])
    ref = odec.decode(_anchor_dict(sz), sz.mlps, poses_s, kind)
    nz, C = anchors.size * K, za.capacity * K
    keep = np.concatenate([np.arange(nz), C + np.arange(ref["opacity"].shape[-1] - nz)])
    errs = {}
    for k, v in d.items():
        g = v.cpu().numpy().astype(np.float64)
        rv = ref[k].numpy()
        g_real = g[..., keep]
        scale = np.maximum(1.0, np.abs(rv)) if k in ("mean", "quat") else 1.0
        errs[k] = float((np.abs(g_real - rv) / scale).max())
    _say(f"  decode errs {errs}")
    assert all(e <= 1e-4 for e in errs.values()), errs
    pad = np.arange(nz, C)
    assert np.all(d["scale"].cpu().numpy()[:, pad] == 0.0)
    # (b) render vs the oracle render of the decoded surfels (padding included)
    sc32 = {k: np.ascontiguousarray(v.cpu().numpy()) for k, v in d.items()}
    sc32.update(group_offsets=np.array([x * K for x in za.group_offsets], np.int32), group_poses=sc.group_poses)
    oref = raster.render(sc32, sensor, oracle_opts(gs.PRODUCTION, TILE),
                         alternatives=ALT_TOL)
    v = verify(o.cpu().numpy(), oref, kind)
    _say(f"  render {v}")
    assert_verified(v)
    # (c) bit for bit equal to the direct decode + render of exactly the zone's anchors
    _, od = _direct(sz, sensor, lidar)
    torch.cuda.synchronize()
    assert torch.equal(o, od)
    za.close()


# ---------------------------------------------------------------------------
# 3. a drive across zone boundaries
# ---------------------------------------------------------------------------

def test_drive_across_zone_boundaries_with_prefetch():
    _say("zone drive")
    sc = _scene("pinhole")
    static, actors = S.static_and_actors(sc)
    mlps = S.zone_mlps(8, GRID.n_zones, "pinhole")
    za = gz.ZonedAnchors(static, mlps, GRID, lidar=False, device=DEV, actors=actors, threads=2)
    K = sc.k
    gp = gs.poses_tensor(sc.group_poses, DEV)
    dec = za.decoders
    cam0 = _sensor("pinhole", (5.0, 0.0, -5.0))
    r = gs.Renderer([gs.SceneShape(dec[0].A * K, -1, False, tuple(x * K for x in za.group_offsets))], [cam0],
                    opts=gs.PRODUCTION, device=DEV)
    outs = r.new_outputs()
    d_out = [dec[b].new_decoded() for b in range(2)]
    zs = za.stream
    path = [(5.0, z) for z in np.arange(-5.0, 46.0, 3.0)]  # zones 1, 3, 5 (x in [0, 20))
    lookahead = GRID.pad * GRID.size
    cur_b, held, queued = 0, {}, {}
    z0 = GRID.zone_of(*path[0])
    zs.prefetch(z0, 0)
    held[0] = z0
    zs.acquire(0)
    frames, crossings = 0, 0
    for (x, zc) in path:
        zone = GRID.zone_of(x, zc)
        if held.get(cur_b) != zone:
            nb = 1 - cur_b
            if queued.get(nb) != zone:
                zs.release(nb)
                zs.prefetch(zone, nb)
            got = zs.acquire(nb)
            assert got[0] == zone
            zs.release(cur_b)
            held[nb], cur_b = zone, nb
            queued.pop(nb, None)
            crossings += 1
        # prefetch the zone ahead once within the lookahead of the boundary
        ahead = GRID.zone_of(x, zc + lookahead)
        nb = 1 - cur_b
        if ahead not in (-1, zone) and queued.get(nb) != ahead and held.get(nb) != ahead:
            zs.prefetch(ahead, nb)
            queued[nb] = ahead
        cam = _sensor("pinhole", (x, 0.0, zc))
        sp = gs.poses_tensor(cam["pose"], DEV)
        dd = dec[cur_b].forward(sp[0], gp, out=d_out[cur_b])
        r.forward([dd], sp, gp, outputs=outs)
        anchors = za.index[za.offsets[zone]:za.offsets[zone + 1]]
        _, od = _direct(S.zone_scene(sc, anchors, mlps[zone]), cam, False)
        torch.cuda.synchronize()
        assert torch.equal(outs[0], od), (x, zc, zone)
        frames += 1
    _say(f"  frames {frames} crossings {crossings}")
    assert crossings == 2
    za.close()
