"""GPU (HIP) path vs the FP64 oracle: integer outputs bit-exact, floats within tolerance.

Tolerances: 1e-4 absolute per channel for colour, alpha, normal and
intensity; depth and range 1e-4 relative to max(1 m, reference).  Every
pixel is compared.  Where one of a ray's compositing decisions (a pair
entering or leaving the support, the alpha_min skip, the T_min stop) lies
within 1e-4 (relative) of its threshold, float32 and FP64 may decide it
differently: the oracle then also computes the outputs with those decisions
taken the other way, and the ray passes if it matches the nominal outputs or
one of these alternatives.  Rays with more than three such decisions cannot
be verified this way; they are counted and must be at most 1e-4 of the rays.
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gen import scenes as S  # noqa: E402
from oracle import raster  # noqa: E402
from tests.gpu_common import (ALT_TOL, assert_verified, check_integer_parity, gmap_of, gpu_render, oracle_opts,  # noqa: E402
                              quiet_median,
                              verify)
from tests.helpers import from_gen  # noqa: E402

import paper_2503_11731_amd as gs  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _cfg1():
    sc, sens = S.config1()
    return from_gen(sc), sens


def _forward_check(scene, sensor, opts, tile, segment_pairs=0, what=""):
    r, st, sp, gp, outs = gpu_render(scene, [sensor], opts, tiles=tile, segment_pairs=segment_pairs)
    o = oracle_opts(opts, tile)
    n_pairs = check_integer_parity(r, scene, sensor, o)
    ref = raster.render(scene, sensor, o, alternatives=ALT_TOL)
    v = verify(outs[0].cpu().numpy(), ref, sensor["kind"])
    _say(f"  {what} pairs {n_pairs} flagged {v['flagged']} alt-only {v['alt_only']} unverified {v['unverified']} "
         f"bad {v['bad']} errs {v['errs']}")
    assert_verified(v, what)
    return r, st, sp, gp, outs, v


@pytest.mark.parametrize("mode", ["production", "strict"])
@pytest.mark.parametrize("tile", [(16, 16), (8, 8), (32, 8)])
def test_config1_forward_parity(mode, tile):
    _say(f"config1 forward {mode} tile {tile}")
    scene, sens = _cfg1()
    opts = gs.PRODUCTION if mode == "production" else gs.STRICT
    _forward_check(scene, sens[0], opts, tile, what=f"config1 {mode} {tile}")


@pytest.mark.parametrize("degree", [0, 1, 2, 3])
@pytest.mark.parametrize("mode", ["production", "strict"])
def test_sh_degree_forward_parity(degree, mode):
    """View-dependent colour of every SH degree (one preprocess instantiation each)."""
    _say(f"SH degree {degree} forward {mode}")
    rng = np.random.default_rng(40 + degree)
    sc = S.random_cloud(seed=12 + degree, n=3000, lo=(-2, -1.5, 2.5), hi=(2, 1.5, 7), log_scale=(-2.9, 0.4))
    scene = from_gen(sc)
    scene.pop("rgb")
    nb = (degree + 1) ** 2
    scene["sh"] = (0.3 * rng.standard_normal((nb * 3, sc.n))).astype(np.float32)
    scene["sh_degree"] = degree
    cam = S.pinhole(160, 120, 110.0, pose=S.camera_yaw_pose(8.0))
    opts = gs.PRODUCTION if mode == "production" else gs.STRICT
    _forward_check(scene, cam, opts, (32, 8), what=f"sh{degree} {mode}")


@pytest.mark.parametrize("mode", ["production", "strict"])
def test_lidar_forward_parity(mode):
    _say(f"lidar forward {mode}")
    L = S.lidar_spinning(n_beams=32, n_az=360)
    sc = S.corridor_surfels(seed=7, n=20000, sh_degree=-1, z_lo=-30, z_hi=30, with_intensity=True)
    opts = gs.PRODUCTION if mode == "production" else gs.STRICT
    _forward_check(from_gen(sc), L, opts, (32, 8), what=f"lidar {mode}")


@pytest.mark.parametrize("mode,tile", [("production", (16, 16)), ("strict", (16, 16)), ("production", (8, 8))])
def test_split_tiles_forward_parity(mode, tile):
    """Tile lists split into 32-pair segments and merged: same oracle bar, and
    the same result as the unsplit path up to FP32 rounding order."""
    _say(f"config1 split forward {mode} tile {tile}")
    scene, sens = _cfg1()
    opts = gs.PRODUCTION if mode == "production" else gs.STRICT
    r, st, sp, gp, outs, v = _forward_check(scene, sens[0], opts, tile, segment_pairs=32, what="split")
    status = r.status()
    assert status["segments"] > 0 and status["work_items"] > status["segments"] // 2
    # the merge is deterministic
    again = r.forward([st], sp, gp)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], again[0])
    # unsplit vs split: identical up to rounding order away from near-threshold decisions
    _, _, _, _, whole = gpu_render(scene, sens, opts, tiles=tile, segment_pairs=-1)
    ref = raster.render(scene, sens[0], oracle_opts(opts, tile), alternatives=ALT_TOL)
    diff = (whole[0] - outs[0]).abs().cpu().numpy().reshape(outs[0].shape[0], -1)
    m = ref["n_flags"] == 0
    assert diff[:, m].max() <= 2e-5, diff[:, m].max()


@pytest.mark.parametrize("mode", ["production", "strict"])
def test_split_lidar_forward_parity(mode):
    _say(f"lidar split forward {mode}")
    L = S.lidar_spinning(n_beams=32, n_az=360)
    sc = S.corridor_surfels(seed=7, n=20000, sh_degree=-1, z_lo=-30, z_hi=30, with_intensity=True)
    opts = gs.PRODUCTION if mode == "production" else gs.STRICT
    r, *_ = _forward_check(from_gen(sc), L, opts, (32, 8), segment_pairs=32, what="lidar split")
    assert r.status()["segments"] > 0


def _edge_on_cloud(seed, n):
    """Surfels whose plane nearly contains the camera ray to their centre (85-89.5 deg from facing)."""
    rng = np.random.default_rng(seed)
    mean = np.stack([rng.uniform(-1.2, 1.2, n), rng.uniform(-0.9, 0.9, n), rng.uniform(3.0, 7.0, n)], 1)
    view = mean / np.linalg.norm(mean, axis=1, keepdims=True)
    side = np.cross(view, rng.standard_normal((n, 3)))
    side /= np.linalg.norm(side, axis=1, keepdims=True)
    tilt = np.deg2rad(rng.uniform(0.5, 5.0, n)) * rng.choice([-1, 1], n)
    nrm = np.cos(tilt)[:, None] * side + np.sin(tilt)[:, None] * view  # angle to the view ray: 90 deg - tilt
    tu = np.cross(nrm, view)
    tu /= np.linalg.norm(tu, axis=1, keepdims=True)
    tv = np.cross(nrm, tu)
    q = S._quat_from_frames(tu, tv, nrm)
    from tests.helpers import surfels
    sc = surfels(mean, q, np.exp(rng.normal(-2.6, 0.3, (n, 2))), rng.uniform(0.3, 0.95, n),
                 rgb=rng.uniform(0, 1, (n, 3)))
    return sc


@pytest.mark.parametrize("mode", ["strict", "production"])
def test_grazing_surfels_take_the_fp64_resolve(mode):
    """Edge-on surfels: rays near the horizon line of a surfel's plane have h'_2 near 0 and are
    re-solved in FP64; the re-solve must run and the outputs must still match the oracle."""
    _say(f"grazing {mode}")
    scene = _edge_on_cloud(17, 600)
    cam = S.pinhole(128, 96, 96.0)
    opts = gs.PRODUCTION if mode == "production" else gs.STRICT
    r, *_ = _forward_check(scene, cam, opts, (16, 16), what=f"grazing {mode}")
    st = r.status()
    _say(f"  fp64 re-solves {st['fp64_pairs']} of {st['evaluated']} evaluated pairs")
    assert st["fp64_pairs"] > 0


def test_forward_is_deterministic_and_order_invariant():
    _say("determinism / permutation")
    scene, sens = _cfg1()
    r, st, sp, gp, outs = gpu_render(scene, sens, gs.PRODUCTION)
    a = outs[0].clone()
    outs2 = r.forward([st], sp, gp)
    torch.cuda.synchronize()
    assert torch.equal(a, outs2[0])
    perm = np.random.default_rng(0).permutation(scene["mean"].shape[1])
    sp_scene = dict(scene)
    for k in ("mean", "quat", "scale", "rgb"):
        sp_scene[k] = np.ascontiguousarray(scene[k][:, perm])
    sp_scene["opacity"] = np.ascontiguousarray(scene["opacity"][perm])
    _, _, _, _, outs3 = gpu_render(sp_scene, sens, gs.PRODUCTION)
    # keys are tie-free, so the composited order and every float op are the same
    assert torch.equal(a, outs3[0])
    # the pair counters of calibration runs change no output
    r.set_counters(True)
    outs4 = r.forward([st], sp, gp)
    st4 = r.status()
    torch.cuda.synchronize()
    assert torch.equal(a, outs4[0])
    assert st4["evaluated"] >= st4["composited"] > 0 and st4["wave_pairs"] > 0
    assert st4["evaluated"] <= 64 * st4["wave_pairs"]
    r.set_counters(False)
    r.forward([st], sp, gp)
    assert r.status()["evaluated"] == 0


def grad_check(scene, sensor, opts, tile, keys, channels_seed=0, segment_pairs=0):
    """Device adjoint vs the oracle's autograd gradient for random dL/d(outputs):
    per tensor, max error and max |reference|."""
    r, st, sp, gp, outs = gpu_render(scene, [sensor], opts, tiles=tile, segment_pairs=segment_pairs)
    if segment_pairs > 0:
        assert r.status()["segments"] > 0
    rng = np.random.default_rng(channels_seed)
    go = rng.standard_normal(tuple(outs[0].shape)).astype(np.float32)
    o = oracle_opts(opts, tile)
    quiet_median(go, scene, sensor, o)
    grads = r.backward([st], sp, gp, outs, [torch.from_numpy(go).to(outs[0].device)])[0]
    torch.cuda.synchronize()
    gmap = gmap_of(go, sensor["kind"])
    ref = raster.render(scene, sensor, o, grad_out={k: v.astype(np.float64) for k, v in gmap.items()})
    res = {}
    for k in keys:
        g = grads[k].cpu().numpy().astype(np.float64)
        gr = ref["grads"][k]
        res[k] = (float(np.abs(g - gr).max()), float(np.abs(gr).max()))
    return res


@pytest.mark.parametrize("n", [4097, 32769, 50001])
def test_sort_block_boundaries_pair_lists(n):
    """Pair lists and ranges bit-exact when the radix passes span several
    4096-key blocks chained by the look-back (4097 and 32769 surfels leave a
    single key in the depth sort's last block; the pair lists span tens of
    blocks with ragged ends)."""
    _say(f"sort block boundaries n={n}")
    sc = S.random_cloud(seed=5, n=n, lo=(-3, -3, 3), hi=(3, 3, 12), log_scale=(-3.4, 0.4))
    scene = from_gen(sc)
    cam = S.pinhole(320, 240, 200.0)
    r, st, sp, gp, outs = gpu_render(scene, [cam], gs.PRODUCTION, tiles=(16, 16))
    n_pairs = check_integer_parity(r, scene, cam, oracle_opts(gs.PRODUCTION, (16, 16)))
    _say(f"  pairs {n_pairs}")
    assert n_pairs > 4096


@pytest.mark.parametrize("kind,seg", [("rgb", 0), ("sh3", 0), ("sh1", 0), ("sh2", 0), ("rgb", 32)])
def test_camera_backward_parity(kind, seg):
    _say(f"camera backward {kind} segment_pairs {seg}")
    rng = np.random.default_rng(3)
    n = 300
    sc = S.random_cloud(seed=11, n=n, lo=(-1, -1, 3), hi=(1, 1, 6), log_scale=(-2.6, 0.4))
    scene = from_gen(sc)
    if kind.startswith("sh"):
        deg = int(kind[2:])
        scene.pop("rgb")
        scene["sh"] = (0.3 * rng.standard_normal(((deg + 1) ** 2 * 3, n))).astype(np.float32)
        scene["sh_degree"] = deg
    cam = S.pinhole(96, 80, 96.0)
    keys = ["mean", "quat", "scale", "opacity", "rgb" if kind == "rgb" else "sh"]
    res = grad_check(scene, cam, gs.PRODUCTION, (16, 16), keys, segment_pairs=seg)
    _say(f"  {res}")
    for k, (err, scale) in res.items():
        assert err <= 1e-3 * scale + 1e-6, (k, err, scale)


@pytest.mark.parametrize("seg", [0, 32])
def test_lidar_backward_parity(seg):
    _say(f"lidar backward segment_pairs {seg}")
    L = S.lidar_spinning(n_beams=16, n_az=180, pose=np.concatenate([np.eye(3), np.zeros((3, 1))], 1))
    rng = np.random.default_rng(5)
    n = 300
    r_ = rng.uniform(4, 9, n)
    az = rng.uniform(-np.pi, np.pi, n)
    el = np.deg2rad(rng.uniform(-25, 15, n))
    mean = np.stack([r_ * np.cos(el) * np.cos(az), r_ * np.cos(el) * np.sin(az), r_ * np.sin(el)]).astype(np.float32)
    q = rng.standard_normal((4, n)).astype(np.float32)
    scene = dict(mean=mean, quat=q, scale=np.exp(rng.normal(-1.6, 0.3, (2, n))).astype(np.float32),
                 opacity=rng.uniform(0.2, 0.95, n).astype(np.float32), intensity=rng.uniform(0, 1, n).astype(np.float32),
                 group_offsets=np.array([0, n], np.int32), group_poses=S._identity_poses(1))
    res = grad_check(scene, L, gs.PRODUCTION, (32, 8), ["mean", "quat", "scale", "opacity", "intensity"],
                     segment_pairs=seg)
    _say(f"  {res}")
    for k, (err, scale) in res.items():
        assert err <= 1e-3 * scale + 1e-6, (k, err, scale)


def test_empty_and_offscreen_scenes():
    _say("empty / offscreen")
    cam = S.pinhole(40, 30, 40.0)
    empty = dict(mean=np.zeros((3, 0), np.float32), quat=np.zeros((4, 0), np.float32), scale=np.zeros((2, 0), np.float32),
                 opacity=np.zeros(0, np.float32), rgb=np.zeros((3, 0), np.float32),
                 group_offsets=np.array([0, 0], np.int32), group_poses=S._identity_poses(1))
    r, st, sp, gp, outs = gpu_render(empty, [cam], gs.PRODUCTION)
    assert float(outs[0].abs().max()) == 0.0
    behind = S.random_cloud(seed=2, n=500, lo=(-1, -1, -5), hi=(1, 1, -1))
    r, st, sp, gp, outs = gpu_render(from_gen(behind), [cam], gs.PRODUCTION)
    assert float(outs[0].abs().max()) == 0.0
    assert r.status()["pairs"][0] == 0
