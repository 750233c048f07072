"""Cylindrical (fisheye) camera of Eq. 4 on the GPU vs the FP64 oracle.

Same bar as the pinhole parity tests: the pair lists, tile ranges and
visibility bit for bit against the oracle's FP32 binning specification;
every ray within 1e-4 of the oracle's nominal outputs or of an alternative of
its near-threshold decisions (depth 1e-4 relative to max(1 m, depth));
gradients within 1e-3 of the largest reference entry per tensor.

Small cases: a road-corridor cloud seen by a 180-degree camera in production
and strict compositing, split tile lists, SH colour, edge-on surfels that take
the FP64 re-solve, and the adjoint.  Full size: a 1920x1080 cylindrical camera
(180 degrees) over the 1M-surfel SH3 driving corridor in production and strict
compositing (integer parity in full, floats on a ray sample plus the two
heaviest tiles), and its adjoint on a 64x64 crop.
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gen import scenes as S  # noqa: E402
from oracle import raster  # noqa: E402
from tests.gpu_common import (ALT_TOL, DEV, assert_verified, check_integer_parity, gmap_of, gpu_render, oracle_opts,  # noqa: E402
                              quiet_median,
                              verify)
from tests.helpers import from_gen, surfels  # noqa: E402

import paper_2503_11731_amd as gs  # noqa: E402


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _check(scene, cam, opts, tile, segment_pairs=0, what=""):
    r, st, sp, gp, outs = gpu_render(scene, [cam], opts, tiles=tile, segment_pairs=segment_pairs)
    assert not r.status()["overflow"]
    o = oracle_opts(opts, tile)
    n_pairs = check_integer_parity(r, scene, cam, o)
    ref = raster.render(scene, cam, o, alternatives=ALT_TOL)
    v = verify(outs[0].cpu().numpy(), ref, "cylindrical")
    _say(f"  {what}: pairs {n_pairs} {v}")
    assert_verified(v, what)
    assert float(outs[0][7].max()) > 0.5
    return r, st, sp, gp, outs


def _corridor(n=20000, sh_degree=-1, seed=17):
    return from_gen(S.corridor_surfels(seed=seed, n=n, sh_degree=sh_degree, z_lo=-25, z_hi=40))


@pytest.mark.parametrize("mode", ["production", "strict"])
@pytest.mark.parametrize("tile", [(32, 8), (16, 16)])
def test_cylindrical_forward_parity(mode, tile):
    _say(f"cylindrical forward {mode} {tile}")
    cam = S.cylindrical(320, 120, 180.0, pose=S.camera_yaw_pose(20.0))
    _check(_corridor(), cam, gs.PRODUCTION if mode == "production" else gs.STRICT, tile, what=f"cyl {mode} {tile}")


def test_cylindrical_wide_split_sh_parity():
    """270 degrees, SH2 colour, tile lists split into 64-pair segments."""
    _say("cylindrical 270 deg, SH2, split lists")
    cam = S.cylindrical(360, 96, 270.0)
    r, *_ = _check(_corridor(sh_degree=2, seed=23), cam, gs.PRODUCTION, (32, 8), segment_pairs=64,
                   what="cyl wide split sh2")
    assert r.status()["segments"] > 0


def _edge_on_ring(seed, n):
    """Surfels around the camera whose plane nearly holds the ray to their centre."""
    rng = np.random.default_rng(seed)
    r = rng.uniform(3.0, 7.0, n)
    ph = rng.uniform(-1.3, 1.3, n)
    mean = np.stack([r * np.sin(ph), rng.uniform(-0.8, 0.8, n), r * np.cos(ph)], 1)
    view = mean / np.linalg.norm(mean, axis=1, keepdims=True)
    side = np.cross(view, rng.standard_normal((n, 3)))
    side /= np.linalg.norm(side, axis=1, keepdims=True)
    tilt = np.deg2rad(rng.uniform(0.5, 5.0, n)) * rng.choice([-1, 1], n)
    nrm = np.cos(tilt)[:, None] * side + np.sin(tilt)[:, None] * view
    tu = np.cross(nrm, view)
    tu /= np.linalg.norm(tu, axis=1, keepdims=True)
    tv = np.cross(nrm, tu)
    q = S._quat_from_frames(tu, tv, nrm)
    return surfels(mean, q, np.exp(rng.normal(-2.6, 0.3, (n, 2))), rng.uniform(0.3, 0.95, n),
                   rgb=rng.uniform(0, 1, (n, 3)))


@pytest.mark.parametrize("mode", ["strict", "production"])
def test_cylindrical_grazing_surfels_take_the_fp64_resolve(mode):
    _say(f"cylindrical grazing {mode}")
    cam = S.cylindrical(192, 96, 160.0)
    r, *_ = _check(_edge_on_ring(19, 600), cam, gs.PRODUCTION if mode == "production" else gs.STRICT, (16, 16),
                   what=f"cyl grazing {mode}")
    st = r.status()
    _say(f"  fp64 re-solves {st['fp64_pairs']}")
    assert st["fp64_pairs"] > 0


@pytest.mark.parametrize("kind", ["rgb", "sh3"])
def test_cylindrical_backward_parity(kind):
    _say(f"cylindrical backward {kind}")
    rng = np.random.default_rng(4)
    n = 300
    r_ = rng.uniform(3.0, 6.0, n)
    ph = rng.uniform(-1.2, 1.2, n)
    mean = np.stack([r_ * np.sin(ph), rng.uniform(-0.6, 0.6, n) * r_, r_ * np.cos(ph)], 1)
    q = rng.standard_normal((n, 4))
    scale = np.exp(rng.normal(-2.2, 0.4, (n, 2)))
    if kind == "rgb":
        scene = surfels(mean, q.T, scale, rng.uniform(0.2, 0.95, n), rgb=rng.uniform(0, 1, (n, 3)))
    else:
        scene = surfels(mean, q.T, scale, rng.uniform(0.2, 0.95, n),
                        sh=0.3 * rng.standard_normal((48, n)), sh_degree=3)
    cam = S.cylindrical(128, 64, 170.0)
    r, st, sp, gp, outs = gpu_render(scene, [cam], gs.PRODUCTION, tiles=(16, 16))
    go = rng.standard_normal(tuple(outs[0].shape)).astype(np.float32)
    quiet_median(go, scene, cam, oracle_opts(gs.PRODUCTION, (16, 16)))
    grads = r.backward([st], sp, gp, outs, [torch.from_numpy(go).to(DEV)])[0]
    torch.cuda.synchronize()
    gmap = gmap_of(go, "cylindrical")
    ref = raster.render(scene, cam, oracle_opts(gs.PRODUCTION, (16, 16)),
                        grad_out={k: v.astype(np.float64) for k, v in gmap.items()})
    for k in ("mean", "quat", "scale", "opacity", "rgb" if kind == "rgb" else "sh"):
        g = grads[k].cpu().numpy().astype(np.float64)
        gr = ref["grads"][k]
        err, sc = float(np.abs(g - gr).max()), float(np.abs(gr).max())
        _say(f"  {k}: err {err:.3e} scale {sc:.3e}")
        assert sc > 0 and err <= 1e-3 * sc + 1e-6, (k, err, sc)


def _tile_rays(tile, n_tx, tw, th, width, height):
    tx, ty = tile % n_tx, tile // n_tx
    ids = [(ty * th + y) * width + tx * tw + x for y in range(th) for x in range(tw)
           if ty * th + y < height and tx * tw + x < width]
    return np.array(ids, np.int64)


def _fullsize_scene():
    sc, _ = S.config2()
    scene = dict(mean=sc.mean, quat=sc.quat, scale=sc.scale, opacity=sc.opacity, sh=sc.sh, sh_degree=3,
                 group_offsets=sc.group_offsets, group_poses=sc.group_poses)
    return sc, scene


@pytest.mark.parametrize("mode", ["production", "strict"])
def test_cylindrical_1080p_full_size_parity(mode):
    _say(f"cylindrical 1920x1080 full size {mode}: generate")
    sc, scene = _fullsize_scene()
    cam = S.cylindrical(1920, 1080, 180.0)
    opts = gs.PRODUCTION if mode == "production" else gs.STRICT
    r = gs.Renderer([gs.SceneShape(sc.n, 3, False, (0, sc.n))], [cam], opts=opts, device=DEV)
    st = gs.scene_tensors(scene, DEV)
    sp = gs.poses_tensor([cam["pose"]], DEV)
    gp = gs.poses_tensor(sc.group_poses, DEV)
    _say("  gpu forward")
    (out,) = r.forward([st], sp, gp)
    torch.cuda.synchronize()
    status = r.status()
    assert not status["overflow"]
    tw, th = 32, 8
    o = oracle_opts(opts, (tw, th))
    _say(f"  integer parity over {status['pairs'][0]} pairs")
    n_pairs = check_integer_parity(r, scene, cam, o)
    ranges = r.inspect(0)["ranges"].cpu().numpy().astype(np.int64)
    heavy = np.argsort(ranges[:, 1] - ranges[:, 0])[-2:]
    n_tx = (cam["width"] + tw - 1) // tw
    # a 12-pixel grid (14400 rays) and the two heaviest tiles: enough rays that
    # the bar on unverifiable rays (1e-4 of all) allows the one or two dense
    # strict-mode rays with more near-threshold decisions than are verified
    rays = np.concatenate([raster.grid_rays(cam, 12)] +
                          [_tile_rays(int(t), n_tx, tw, th, cam["width"], cam["height"]) for t in heavy])
    _say(f"  oracle on {rays.size} rays (heaviest tiles {(ranges[heavy, 1] - ranges[heavy, 0]).tolist()} pairs)")
    # strict compositing keeps every pair of a ray (no stop), so dense rays carry
    # more near-threshold decisions: up to 8 are verified both ways
    ref = raster.render(scene, cam, o, rays=rays, alternatives=ALT_TOL, max_flags=8)
    got = out.reshape(out.shape[0], -1)[:, torch.from_numpy(rays).to(DEV)].cpu().numpy()
    v = verify(got, ref, "cylindrical")
    _say(f"  pairs {n_pairs} segments {status['segments']} {v}")
    assert_verified(v)
    assert float(out[7].max()) > 0.9


def test_cylindrical_1080p_full_size_adjoint_on_a_crop():
    """Adjoint of the full 1920x1080 cylindrical frame with dL/dO nonzero on a 64x64 crop only,
    against the oracle's autograd over the crop's rays."""
    _say("cylindrical 1920x1080 adjoint, 64x64 crop")
    sc, scene = _fullsize_scene()
    cam = S.cylindrical(1920, 1080, 180.0)
    x0, y0, cw = 1240, 500, 64
    ys, xs = np.mgrid[y0:y0 + cw, x0:x0 + cw]
    rays = (ys * cam["width"] + xs).reshape(-1)
    r = gs.Renderer([gs.SceneShape(sc.n, 3, False, (0, sc.n))], [cam], opts=gs.PRODUCTION, device=DEV)
    st = gs.scene_tensors(scene, DEV)
    sp = gs.poses_tensor([cam["pose"]], DEV)
    gp = gs.poses_tensor(sc.group_poses, DEV)
    (out,) = r.forward([st], sp, gp)
    rng = np.random.default_rng(8)
    C = out.shape[0]
    g_crop = rng.standard_normal((C, rays.size))
    g_crop[8] = 0.0  # the median's gradient is tested on the small cases
    go = torch.zeros_like(out)
    go.view(C, -1)[:, torch.from_numpy(rays).to(DEV)] = torch.from_numpy(g_crop.astype(np.float32)).to(DEV)
    (grads,) = r.backward([st], sp, gp, [out], [go])
    torch.cuda.synchronize()
    o = oracle_opts(gs.PRODUCTION, (32, 8))
    gmap = gmap_of(g_crop, "cylindrical")
    _say("  oracle adjoint over the crop")
    ref = raster.render(scene, cam, o, rays=rays, grad_out=gmap)
    crop = out.view(C, -1)[:, torch.from_numpy(rays).to(DEV)].cpu().numpy()
    assert np.abs(crop[7] - ref["alpha"]).max() < 1e-3 and ref["alpha"].max() > 0.5
    for k in ("mean", "quat", "scale", "opacity", "sh"):
        g = grads[k].cpu().numpy().astype(np.float64)
        gr = ref["grads"][k]
        err, scl = float(np.abs(g - gr).max()), float(np.abs(gr).max())
        _say(f"  {k}: err {err:.3e} scale {scl:.3e}")
        assert scl > 0 and err <= 1e-3 * scl + 1e-9, (k, err, scl)
