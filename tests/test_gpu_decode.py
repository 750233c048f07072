"""Neural-Gaussian decode on MFMA vs the FP64 oracle decode, forward and adjoint.

Weights and features are bf16 parameters (exact on both sides); the oracle
computes in FP64, the GPU accumulates in FP32 with bf16 hi+lo activations.
Forward outputs within 1e-4 (absolute for sigmoid heads, relative to
max(1, |x|) for raw quaternions and centres); gradients within 1e-3 of the
largest reference entry per tensor.
"""
import sys

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

from gen import scenes as S  # noqa: E402
from oracle import decode as odec  # noqa: E402
from oracle import raster, spec32  # noqa: E402

import paper_2503_11731_amd as gs  # noqa: E402

DEV = torch.device("cuda:0")


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _anchor_dict(sc, feat_bits=None):
    fb = sc.feat_bf16 if feat_bits is None else feat_bits
    return dict(xyz=sc.xyz.astype(np.float64), scaling=sc.scaling.astype(np.float64),
                offsets=sc.offsets.astype(np.float64), feat=S.bf16_bits_to_f32(fb).astype(np.float64),
                group_offsets=sc.group_offsets)


def _setup(kind, n_anchors=3000, n_assets=2, plain=False):
    sc = S.corridor_anchors(seed=21, n_anchors=n_anchors, sensor_kind=kind, z_lo=-20, z_hi=40, n_assets=n_assets,
                            asset_anchors=200)
    if kind == "pinhole":
        sensor = S.pinhole(320, 200, 160.0, pose=S.camera_yaw_pose(10.0))
    else:
        sensor = S.lidar_spinning(n_beams=32, n_az=360)
    dec = gs.Decoder.from_gen(sc, DEV, plain_fp32=plain)
    sp = gs.poses_tensor(sensor["pose"], DEV)[0]
    gp = gs.poses_tensor(sc.group_poses, DEV)
    poses_s = np.stack([spec32.compose_pose(sensor["pose"], g) for g in sc.group_poses])
    return sc, sensor, dec, sp, gp, poses_s


def _cmp(name, got, ref, rel=False):
    g = got.detach().cpu().numpy().astype(np.float64)
    scale = np.maximum(1.0, np.abs(ref)) if rel else 1.0
    err = float((np.abs(g - ref) / scale).max())
    return err


@pytest.mark.parametrize("plain", [False, True])
@pytest.mark.parametrize("kind", ["pinhole", "lidar"])
def test_decode_forward_parity(kind, plain):
    _say(f"decode forward {kind} plain_fp32={plain}")
    sc, sensor, dec, sp, gp, poses_s = _setup(kind, plain=plain)
    out = dec.forward(sp, gp)
    torch.cuda.synchronize()
    ref = odec.decode(_anchor_dict(sc), sc.mlps, poses_s, kind)
    errs = {}
    for k in ("opacity", "scale") + (("rgb",) if kind == "pinhole" else ("intensity", "drop")):
        errs[k] = _cmp(k, out[k], ref[k].numpy())
    errs["quat"] = _cmp("quat", out["quat"], ref["quat"].numpy(), rel=True)
    errs["mean"] = _cmp("mean", out["mean"], ref["mean"].numpy(), rel=True)
    _say(f"  {errs}")
    for k, e in errs.items():
        assert e <= 1e-4, (k, e)


@pytest.mark.parametrize("plain", [False, True])
def test_decode_without_centres_writes_the_same_other_outputs(plain):
    """out.mean = NULL: the centres are not written (they do not depend on the sensor); every other
    output is bit-identical to a full decode."""
    _say(f"decode without centres plain_fp32={plain}")
    sc, sensor, dec, sp, gp, poses_s = _setup("pinhole", plain=plain)
    full = dec.forward(sp, gp)
    part = dec.new_decoded()
    part["mean"] = None
    part = dec.forward(sp, gp, out=part)
    torch.cuda.synchronize()
    for k, v in full.items():
        if k != "mean":
            assert torch.equal(v, part[k]), k
    assert part["mean"] is None


@pytest.mark.parametrize("kind", ["pinhole", "lidar"])
def test_decode_backward_parity(kind):
    _say(f"decode backward {kind}")
    sc, sensor, dec, sp, gp, poses_s = _setup(kind, n_anchors=1500, n_assets=1)
    out = dec.forward(sp, gp)
    rng = np.random.default_rng(4)
    gi = {k: torch.from_numpy(rng.standard_normal(tuple(v.shape)).astype(np.float32)).to(DEV) for k, v in out.items()}
    grads = dec.backward(sp, gp, gi)
    torch.cuda.synchronize()
    G = len(sc.mlps)
    leaves = {k: torch.as_tensor(v).requires_grad_(True) for k, v in _anchor_dict(sc).items() if k != "group_offsets"}
    for g in range(G):
        for name in ("w1", "b1", "w2", "b2"):
            leaves[f"{name}_{g}"] = torch.as_tensor(sc.mlps[g][name].astype(np.float64)).requires_grad_(True)
    ref = odec.decode(_anchor_dict(sc), sc.mlps, poses_s, kind, params=leaves)
    tot = sum((ref[k] * torch.as_tensor(gi[k].cpu().numpy().astype(np.float64))).sum() for k in ref)
    keys = list(leaves.keys())
    rg = dict(zip(keys, torch.autograd.grad(tot, [leaves[k] for k in keys], allow_unused=True)))
    res = {}
    for k in ("xyz", "scaling", "offsets", "feat"):
        r_ = rg[k].numpy()
        res[k] = (float(np.abs(grads[k].cpu().numpy() - r_).max()), float(np.abs(r_).max()))
    for name in ("w1", "b1", "w2", "b2"):
        r_ = np.stack([rg[f"{name}_{g}"].numpy() for g in range(G)])
        res[name] = (float(np.abs(grads[name].cpu().numpy() - r_).max()), float(np.abs(r_).max()))
    _say(f"  {res}")
    for k, (err, scale) in res.items():
        assert err <= 1e-3 * scale + 1e-7, (k, err, scale)


def test_training_step_gradient_chain():
    """Decode -> render -> L1 loss -> adjoint render -> adjoint decode, vs the oracle's autograd chain.

    dL/d(rgb) is the L1 gradient sign(O - target) / n of the oracle's own forward output, given to both sides."""
    _say("training step chain")
    sc = S.corridor_anchors(seed=31, n_anchors=400, sensor_kind="pinhole", z_lo=2, z_hi=14)
    cam = S.pinhole(64, 48, 48.0)
    target = np.random.default_rng(2).uniform(0, 1, (3, 48, 64))
    n = sc.n_anchors * sc.k
    # oracle chain
    poses_s = np.stack([spec32.compose_pose(cam["pose"], g) for g in sc.group_poses])
    leaves = {k: torch.as_tensor(v).requires_grad_(True) for k, v in _anchor_dict(sc).items() if k != "group_offsets"}
    ref_dec = odec.decode(_anchor_dict(sc), sc.mlps, poses_s, "pinhole", params=leaves)
    sc32 = {k: v.detach().numpy().astype(np.float32) for k, v in ref_dec.items()}
    sc32.update(group_offsets=np.array([0, n], np.int32), group_poses=sc.group_poses)
    fwd = raster.render(sc32, cam, raster.make_opts(), params={k: v.detach() for k, v in ref_dec.items()})
    g_rgb = np.sign(fwd["rgb"] - target) / target.size
    res = raster.render(sc32, cam, raster.make_opts(), params=ref_dec, grad_out={"rgb": g_rgb})
    # device chain with the same dL/d(rgb)
    dec = gs.Decoder.from_gen(sc, DEV)
    sp = gs.poses_tensor(cam["pose"], DEV)
    gp = gs.poses_tensor(sc.group_poses, DEV)
    r = gs.Renderer([gs.SceneShape(n, -1, False, (0, n))], [cam], opts=gs.PRODUCTION, device=DEV)
    d = dec.forward(sp[0], gp)
    (o,) = r.forward([d], sp, gp)
    go = torch.zeros_like(o)
    go[:3] = torch.from_numpy(g_rgb.astype(np.float32)).to(DEV)
    (gsurf,) = r.backward([d], sp, gp, [o], [go])
    ga = dec.backward(sp[0], gp, gsurf)
    torch.cuda.synchronize()
    assert np.abs(o[:3].cpu().numpy() - fwd["rgb"]).max() < 1e-4
    leaf_keys = ["xyz", "scaling", "offsets", "feat"]
    gl = torch.autograd.grad(sum((ref_dec[k] * torch.as_tensor(res["grads"][k])).sum() for k in res["grads"]),
                             [leaves[k] for k in leaf_keys])
    out = {}
    for k, g in zip(leaf_keys, gl):
        r_ = g.numpy()
        out[k] = (float(np.abs(ga[k].cpu().numpy() - r_).max()), float(np.abs(r_).max()))
    _say(f"  {out}")
    for k, (err, scale) in out.items():
        assert err <= 1e-3 * scale + 1e-7, (k, err, scale)


def test_decode_weight_gradients_are_deterministic():
    """Per-block partials summed in a fixed order: repeated adjoints agree bit for bit."""
    _say("decode backward determinism")
    sc, sensor, dec, sp, gp, poses_s = _setup("pinhole", n_anchors=3000, n_assets=2)
    out = dec.forward(sp, gp)
    rng = np.random.default_rng(8)
    gi = {k: torch.from_numpy(rng.standard_normal(tuple(v.shape)).astype(np.float32)).to(DEV) for k, v in out.items()}
    g1 = dec.backward(sp, gp, gi)
    g2 = dec.backward(sp, gp, gi)
    torch.cuda.synchronize()
    for k in ("w1", "b1", "w2", "b2"):
        assert torch.equal(g1[k], g2[k]), k
        assert float(g1[k].abs().max()) > 0.0, k
