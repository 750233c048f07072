"""Shared helpers for GPU parity tests: run the HIP path and the FP64 oracle on one input."""
import numpy as np
import torch

import paper_2503_11731_amd as gs
from oracle import raster, spec32

DEV = torch.device("cuda:0")

TOL = 1e-4           # absolute, colour / alpha / normal / intensity
TOL_DEPTH = 1e-4     # relative to max(1, |reference|), depth / range


def gpu_render(scene, sensors, opts, tiles=None, pair_capacity=0, segment_pairs=0):
    shapes = [gs.SceneShape(int(scene["mean"].shape[1]), int(scene.get("sh_degree", -1) if scene.get("sh") is not None else -1),
                            scene.get("intensity") is not None,
                            tuple(int(x) for x in scene["group_offsets"]))]
    sens = []
    for i, s in enumerate(sensors):
        s = dict(s)
        if tiles is not None:
            s["tile"] = tiles[i] if isinstance(tiles, list) else tiles
        sens.append(s)
    r = gs.Renderer(shapes, sens, opts=opts, pair_capacity=pair_capacity, device=DEV, segment_pairs=segment_pairs)
    st = gs.scene_tensors(scene, DEV)
    sp = gs.poses_tensor([s["pose"] for s in sensors], DEV)
    gp = gs.poses_tensor(scene["group_poses"], DEV)
    outs = r.forward([st], sp, gp)
    torch.cuda.synchronize()
    return r, st, sp, gp, outs


def oracle_opts(opts, tile):
    o = raster.make_opts(opts)
    o["tile_w"], o["tile_h"] = tile
    return o


def camera_errors(got, ref, mask=None):
    """Max errors per channel group; got [8,H,W] (or [8,R]) numpy, ref oracle dict."""
    g = got.astype(np.float64)
    m = np.ones(ref["alpha"].shape, bool) if mask is None else mask
    e = {}
    e["rgb"] = np.abs(g[0:3] - ref["rgb"])[:, m].max(initial=0.0)
    e["normal"] = np.abs(g[4:7] - ref["normal"])[:, m].max(initial=0.0)
    e["alpha"] = np.abs(g[7] - ref["alpha"])[m].max(initial=0.0)
    e["depth"] = (np.abs(g[3] - ref["depth"]) / np.maximum(1.0, np.abs(ref["depth"])))[m].max(initial=0.0)
    return e


def camera_bad_pixels(got, ref):
    """Pixels where any channel is outside tolerance."""
    g = got.astype(np.float64)
    bad = (np.abs(g[0:3] - ref["rgb"]) > TOL).any(0)
    bad |= (np.abs(g[4:7] - ref["normal"]) > TOL).any(0)
    bad |= np.abs(g[7] - ref["alpha"]) > TOL
    bad |= np.abs(g[3] - ref["depth"]) > TOL_DEPTH * np.maximum(1.0, np.abs(ref["depth"]))
    return bad


def lidar_errors(got, ref, mask=None):
    g = got.astype(np.float64)
    m = np.ones(ref["alpha"].shape, bool) if mask is None else mask
    e = {}
    e["range"] = (np.abs(g[0] - ref["range"]) / np.maximum(1.0, np.abs(ref["range"])))[m].max(initial=0.0)
    e["intensity"] = np.abs(g[1] - ref["intensity"])[m].max(initial=0.0)
    e["alpha"] = np.abs(g[2] - ref["alpha"])[m].max(initial=0.0)
    return e


def lidar_bad_rays(got, ref):
    """Rays where any LiDAR channel is outside tolerance."""
    g = got.astype(np.float64)
    bad = np.abs(g[0] - ref["range"]) > TOL_DEPTH * np.maximum(1.0, np.abs(ref["range"]))
    bad |= np.abs(g[1] - ref["intensity"]) > TOL
    bad |= np.abs(g[2] - ref["alpha"]) > TOL
    return bad


ALT_TOL = 1e-4      # relative distance to a threshold below which a decision is flagged and verified both ways


def oracle_vector(ref, kind):
    """Oracle outputs as [C, R] in the device channel order."""
    if kind != "lidar":
        v = np.concatenate([ref["rgb"].reshape(3, -1), ref["depth"].reshape(1, -1), ref["normal"].reshape(3, -1),
                            ref["alpha"].reshape(1, -1), ref["median"].reshape(1, -1)])
    else:
        v = np.stack([ref["range"].reshape(-1), ref["intensity"].reshape(-1), ref["alpha"].reshape(-1),
                      ref["drop"].reshape(-1), ref["drop_mask"].reshape(-1), ref["median"].reshape(-1)])
    return v


CAMERA_NAMES = ["r", "g", "b", "depth", "nx", "ny", "nz", "alpha", "median"]
LIDAR_NAMES = ["range", "intensity", "alpha", "drop", "drop_mask", "median"]


def depth_like(kind):
    """Channels compared relative to max(1 m, |value|): depth / range and the median."""
    return (3, 8) if kind != "lidar" else (0, 5)


def gmap_of(go, kind):
    """dL/d(outputs) [C, ...] as the oracle's grad_out dict (the drop mask has no gradient)."""
    if kind != "lidar":
        return {"rgb": go[0:3], "depth": go[3], "normal": go[4:7], "alpha": go[7], "median": go[8]}
    return {"range": go[0], "intensity": go[1], "alpha": go[2], "drop": go[3], "median": go[5]}


def median_channel(kind):
    return 8 if kind != "lidar" else 5


def quiet_median(go, scene, sensor, o, rays=None):
    """Zero dL/d(median) (in place) on rays with a decision within ALT_TOL of its
    threshold: the median's surfel is itself a decision (transmittance against
    1/2), which the FP32 kernel and the FP64 oracle may then take differently."""
    m = raster.render(scene, sensor, o, margins=True, rays=rays)["margin"]
    go[median_channel(sensor["kind"])][m <= ALT_TOL] = 0.0
    return go


def _tolerance(v, kind):
    """Per-entry tolerance of output vectors v [C, ...]: 1e-4 absolute, depth/range and median 1e-4 relative
    to max(1, |v|)."""
    t = np.full(v.shape, TOL)
    for d in depth_like(kind):
        t[d] = TOL_DEPTH * np.maximum(1.0, np.abs(v[d]))
    return t


def verify(got, ref, kind):
    """Per-ray verification of device outputs got [C, R] against the oracle run with
    `alternatives`: a ray passes when every channel is within tolerance of the
    oracle's nominal output or of one of the alternatives of its near-threshold
    decisions.  Returns counts and per-channel errors against the matched candidate."""
    g = got.astype(np.float64).reshape(got.shape[0], -1)
    nom = oracle_vector(ref, kind)
    err = np.abs(g - nom)
    ok = (err <= _tolerance(nom, kind)).all(0)
    best = err.copy()
    alt_only = 0
    for r, vals in zip(ref["alts"]["rays"], ref["alts"]["values"]):
        if ok[r]:
            continue
        e = np.abs(g[:, r][None] - vals)
        good = (e <= _tolerance(vals.T, kind).T).all(1)
        if good.any():
            ok[r] = True
            alt_only += 1
            best[:, r] = e[np.argmax(good)]
    unver = np.zeros(ok.shape, bool)
    unver[ref["unverified"]] = True
    bad = ~ok & ~unver
    names = CAMERA_NAMES if kind != "lidar" else LIDAR_NAMES
    rel = best.copy()
    for d in depth_like(kind):
        rel[d] = best[d] / np.maximum(1.0, np.abs(nom[d]))
    m = ~unver
    errs = {n: float(rel[c][m].max(initial=0.0)) for c, n in enumerate(names)}
    return dict(rays=int(ok.size), flagged=int(len(ref["alts"]["rays"])), alt_only=alt_only,
                unverified=int(unver.sum()), bad=int(bad.sum()), bad_rays=np.nonzero(bad)[0][:8].tolist(),
                errs=errs)


def assert_verified(v, what=""):
    """Every verifiable ray matches; rays with too many near-threshold decisions to verify are at most 1e-4 of all."""
    assert v["bad"] == 0, (what, v)
    assert v["unverified"] <= 1e-4 * v["rays"], (what, v)


def within(errs):
    return all(v <= (TOL_DEPTH if k in ("depth", "range") else TOL) for k, v in errs.items())


def gpu_pairs(r, i=0):
    v = r.inspect(i)
    return (v["pair_tile"].cpu().numpy().astype(np.int64), v["pair_surfel"].cpu().numpy().astype(np.int64),
            v["ranges"].cpu().numpy().astype(np.int64), v["visible"].cpu().numpy().astype(bool), v["pairs"])


def check_integer_parity(r, scene, sensor, o, i=0):
    bins = raster.spec_bins(scene, sensor, o)
    t_ref, s_ref = spec32.tile_pairs_fast(bins)
    t_got, s_got, ranges, vis, count = gpu_pairs(r, i)
    assert count == t_ref.size, (count, t_ref.size)
    np.testing.assert_array_equal(vis, bins["visible"])
    np.testing.assert_array_equal(t_got, t_ref)
    np.testing.assert_array_equal(s_got, s_ref)
    # ranges: [start, end) of each tile in the sorted list
    n_tiles = ranges.shape[0]
    starts = np.searchsorted(t_ref, np.arange(n_tiles), side="left")
    ends = np.searchsorted(t_ref, np.arange(n_tiles), side="right")
    nz = ends > starts
    np.testing.assert_array_equal(ranges[nz, 0], starts[nz])
    np.testing.assert_array_equal(ranges[nz, 1], ends[nz])
    return t_ref.size
