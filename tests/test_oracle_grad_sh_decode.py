"""Pins of the oracle's gradients (central differences), SH basis (scipy) and decode (closed forms)."""
import math

import numpy as np
import pytest
import scipy.special
import torch
from scipy.spatial.transform import Rotation

from oracle import decode as odec
from oracle import raster, sh as osh, spec32
from tests.helpers import F32, quat_wxyz, surfels

# Continuous setting for finite differences: no alpha_min skip, no T_min stop,
# cutoff far out in the tail (alpha there is exp(-200)), so the program is
# smooth in every input away from measure-zero kinks.
FD_OPTS = dict(raster.STRICT, cutoff2=400.0)
FD_CAM = dict(kind="pinhole", width=16, height=16, fx=64.0, fy=64.0, cx=8.0, cy=8.0, z_near=0.2,
              pose=np.concatenate([np.eye(3), np.zeros((3, 1))], 1).astype(F32))


def _fd_check(scene, sensor, opts, keys, grad_keys, seed=0, n_probe=None, rel=2e-6):
    rng = np.random.default_rng(seed)
    ref = raster.render(scene, sensor, opts)
    go = {k: rng.standard_normal(ref[k].shape) for k in grad_keys}
    params = {k: torch.as_tensor(scene[k].astype(np.float64)).requires_grad_(True) for k in keys}
    res = raster.render(scene, sensor, opts, grad_out=go, params=params)
    g = res["grads"]

    def loss(pdict):
        out = raster.render(scene, sensor, opts, params=pdict)
        return sum(float((out[k] * go[k]).sum()) for k in grad_keys)

    for k in keys:
        base = scene[k].astype(np.float64)
        flat = base.reshape(-1)
        idxs = range(flat.size) if n_probe is None else rng.choice(flat.size, min(n_probe, flat.size), replace=False)
        gmax = np.abs(g[k]).max() + 1e-30
        for i in idxs:
            h = 1e-6 * max(1.0, abs(flat[i]))
            pp = {kk: torch.as_tensor(scene[kk].astype(np.float64)) for kk in keys}
            vp = flat.copy()
            vp[i] += h
            pp[k] = torch.as_tensor(vp.reshape(base.shape))
            lp = loss(pp)
            vm = flat.copy()
            vm[i] -= h
            pp[k] = torch.as_tensor(vm.reshape(base.shape))
            lm = loss(pp)
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[i]
            assert abs(fd - an) <= rel * max(gmax, 1.0) + 1e-7 * abs(an), (k, i, fd, an)


def _fd_scene(seed, n, sh_degree=-1):
    rng = np.random.default_rng(seed)
    mean = np.stack([rng.uniform(-0.25, 0.25, n), rng.uniform(-0.25, 0.25, n), rng.uniform(3.0, 4.0, n)], 1)
    q = quat_wxyz(Rotation.random(n, random_state=seed)) * F32(1.3)  # non-unit quaternions
    s = np.exp(rng.normal(-3.0, 0.3, size=(n, 2)))
    o = rng.uniform(0.3, 0.9, n)
    if sh_degree >= 0:
        nb = (sh_degree + 1) ** 2
        return surfels(mean, q, s, o, sh=rng.normal(0, 0.3, size=(nb * 3, n)), sh_degree=sh_degree)
    return surfels(mean, q, s, o, rgb=rng.uniform(0, 1, (n, 3)))


def test_fd_gradient_camera_rgb():
    sc = _fd_scene(1, 4)
    _fd_check(sc, FD_CAM, raster.make_opts(FD_OPTS), ["mean", "quat", "scale", "opacity", "rgb"],
              ["rgb", "depth", "normal", "alpha"])


def test_fd_gradient_camera_sh3():
    sc = _fd_scene(2, 2, sh_degree=3)
    _fd_check(sc, FD_CAM, raster.make_opts(FD_OPTS), ["mean", "quat", "scale", "opacity", "sh"],
              ["rgb", "depth", "alpha"], n_probe=24)


def test_fd_gradient_lidar():
    from gen.scenes import lidar_spinning
    L = lidar_spinning(n_beams=8, n_az=64, el_min_deg=-10, el_max_deg=10,
                       pose=np.concatenate([np.eye(3), np.zeros((3, 1))], 1))
    rng = np.random.default_rng(3)
    n = 3
    az = rng.uniform(-0.3, 0.3, n)
    el = rng.uniform(-0.1, 0.1, n)
    r = rng.uniform(4, 6, n)
    mean = np.stack([r * np.cos(el) * np.cos(az), r * np.cos(el) * np.sin(az), r * np.sin(el)], 1)
    q = quat_wxyz(Rotation.random(n, random_state=4))
    s = np.exp(rng.normal(-1.8, 0.2, size=(n, 2)))
    sc = surfels(mean, q, s, rng.uniform(0.3, 0.9, n), intensity=rng.uniform(0, 1, n))
    _fd_check(sc, L, raster.make_opts(FD_OPTS, tile_w=16, tile_h=4), ["mean", "quat", "scale", "opacity", "intensity"],
              ["range", "intensity", "alpha"])


# ----------------------------------------------------------------------------
# spherical harmonics
# ----------------------------------------------------------------------------

def _scipy_real_sh(l, m, theta, phi):
    """Real SH from scipy's complex SH (which carries the Condon-Shortley phase)."""
    if hasattr(scipy.special, "sph_harm_y"):
        Y = scipy.special.sph_harm_y(l, abs(m), theta, phi)
    else:  # older scipy: sph_harm(m, l, azimuth, polar)
        Y = scipy.special.sph_harm(abs(m), l, phi, theta)
    if m == 0:
        return Y.real
    if m > 0:
        return math.sqrt(2) * Y.real
    return math.sqrt(2) * Y.imag


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(0)
    d = rng.standard_normal((3, 500))
    d /= np.linalg.norm(d, axis=0)
    d[:, 0] = [0, 0, 1]
    d[:, 1] = [0, 0, -1]
    Y = osh.sh_basis(torch.as_tensor(d), 3).numpy()
    theta = np.arccos(np.clip(d[2], -1, 1))
    phi = np.arctan2(d[1], d[0])
    for l in range(4):
        for m in range(-l, l + 1):
            np.testing.assert_allclose(Y[l * l + l + m], _scipy_real_sh(l, m, theta, phi), atol=1e-12)


def test_sh_basis_orthonormal():
    z, wz = np.polynomial.legendre.leggauss(8)
    phi = np.arange(16) * 2 * np.pi / 16
    Z, P = np.meshgrid(z, phi, indexing="ij")
    s = np.sqrt(1 - Z ** 2)
    d = np.stack([s * np.cos(P), s * np.sin(P), Z]).reshape(3, -1)
    w = (wz[:, None] * np.full(16, 2 * np.pi / 16)[None]).reshape(-1)
    Y = osh.sh_basis(torch.as_tensor(d), 3).numpy()
    G = (Y * w) @ Y.T
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_degree0_gives_constant_colour():
    c = np.zeros((3, 5))
    c[:, :] = [[0.5], [-0.2], [1.0]]
    d = np.random.default_rng(1).standard_normal((3, 5))
    d /= np.linalg.norm(d, axis=0)
    col = osh.sh_colour(torch.as_tensor(c), torch.as_tensor(d), 0).numpy()
    y0 = 0.5 / math.sqrt(math.pi)
    np.testing.assert_allclose(col, np.maximum(0, np.array([[0.5], [-0.2], [1.0]]) * y0 + 0.5) * np.ones((1, 5)),
                               atol=1e-14)


# ----------------------------------------------------------------------------
# decode
# ----------------------------------------------------------------------------

def _anchors(A=5, K=3, seed=0):
    rng = np.random.default_rng(seed)
    return dict(xyz=rng.uniform(-3, 3, (3, A)) + np.array([[0], [0], [8]]), scaling=rng.uniform(0.05, 0.2, A),
                offsets=rng.standard_normal((3, K, A)), feat=rng.standard_normal((A, 32)),
                group_offsets=np.array([0, A]))


IDPOSE = np.concatenate([np.eye(3), np.zeros((3, 1))], 1)[None].astype(F32)


@pytest.mark.parametrize("kind", ["pinhole", "lidar"])
def test_decode_zero_second_layer_gives_bias_heads(kind):
    an = _anchors()
    K = 3
    J = 10 if kind == "pinhole" else 9
    rng = np.random.default_rng(2)
    b2 = rng.standard_normal(K * J)
    mlp = dict(w1=rng.standard_normal((32, 35)), b1=rng.standard_normal(32), w2=np.zeros((K * J, 32)), b2=b2)
    out = odec.decode(an, [mlp], IDPOSE, kind)
    sig = lambda x: 1 / (1 + np.exp(-x))
    y = b2.reshape(K, J)
    A = 5
    for a in range(A):
        for k in range(K):
            n = a * K + k
            assert out["opacity"][n].item() == pytest.approx(sig(y[k, 0]), abs=1e-14)
            if kind == "pinhole":
                np.testing.assert_allclose(out["rgb"][:, n].numpy(), sig(y[k, 1:4]), atol=1e-14)
                so = 4
            else:
                assert out["intensity"][n].item() == pytest.approx(sig(y[k, 1]), abs=1e-14)
                so = 2
            np.testing.assert_allclose(out["scale"][:, n].numpy(), an["scaling"][a] * sig(y[k, so:so + 2]), atol=1e-14)
            np.testing.assert_allclose(out["quat"][:, n].numpy(), y[k, so + 2:so + 6], atol=1e-14)
            if kind != "pinhole":  # the ray-drop head
                assert out["drop"][n].item() == pytest.approx(sig(y[k, 8]), abs=1e-14)
            np.testing.assert_allclose(out["mean"][:, n].numpy(),
                                       an["xyz"][:, a] + an["scaling"][a] * an["offsets"][:, k, a], atol=1e-14)


def test_decode_feature_relu_and_view_direction_routing():
    # W1 = [I_32 | 0]: hidden = relu(feature).  W2 row (k=1, opacity) picks
    # hidden unit 5, row (k=0, opacity) picks the view-direction x component
    # through hidden unit 0 re-routed by W1's first row.
    an = _anchors(A=4, K=2, seed=3)
    K, J = 2, 10
    w1 = np.zeros((32, 35))
    w1[1:, 1:32] = np.eye(31)
    w1[0, 32] = 1.0  # hidden 0 = relu(d_x)
    b1 = np.zeros(32)
    w2 = np.zeros((K * J, 32))
    w2[1 * J + 0, 5] = 1.0
    w2[0 * J + 0, 0] = 1.0
    mlp = dict(w1=w1, b1=b1, w2=w2, b2=np.zeros(K * J))
    # camera at world (1, -2, 0.5), identity rotation -> sensor<-world t = -c
    pose = IDPOSE.copy()
    pose[0, :, 3] = [-1.0, 2.0, -0.5]
    out = odec.decode(an, [mlp], pose, "pinhole")
    sig = lambda x: 1 / (1 + np.exp(-x))
    cam = np.array([1.0, -2.0, 0.5])
    for a in range(4):
        d = an["xyz"][:, a] - cam
        d /= np.linalg.norm(d)
        assert out["opacity"][a * K + 1].item() == pytest.approx(sig(max(an["feat"][a, 5], 0.0)), abs=1e-14)
        assert out["opacity"][a * K + 0].item() == pytest.approx(sig(max(d[0], 0.0)), abs=1e-14)


def test_decode_view_direction_with_turned_sensor_and_group():
    # Sensor at world centre c with a general rotation, group turned and moved
    # by G = [Rg | tg]: the decoder's view direction is the unit vector from
    # the sensor centre to the anchor in the group's frame, with the centre
    # there at Rg^T (c - tg).  W1 routes d_x, d_y, d_z + 2 to hidden units
    # 0-2 and W2 sends unit k to offset k's opacity, so sigmoid^-1(opacity) - 2
    # reads the direction back.
    an = _anchors(A=5, K=3, seed=6)
    K, J = 3, 10
    w1 = np.zeros((32, 35))
    b1 = np.zeros(32)
    for c in range(3):
        w1[c, 32 + c] = 1.0
        b1[c] = 2.0
    w2 = np.zeros((K * J, 32))
    for k in range(3):
        w2[k * J + 0, k] = 1.0
    mlp = dict(w1=w1, b1=b1, w2=w2, b2=np.zeros(K * J))
    from scipy.spatial.transform import Rotation
    from oracle import spec32
    c_w = np.array([1.5, -0.7, 2.0])
    Rv = Rotation.from_euler("zyx", [30, -50, 20], degrees=True).as_matrix()
    V = np.concatenate([Rv, (-Rv @ c_w)[:, None]], 1).astype(F32)
    Rg = Rotation.from_euler("xyz", [-15, 65, 40], degrees=True).as_matrix()
    tg = np.array([0.4, 0.2, -1.1])
    G = np.concatenate([Rg, tg[:, None]], 1).astype(F32)
    P = spec32.compose_pose(V, G)[None]
    out = odec.decode(an, [mlp], P, "pinhole")
    op = out["opacity"].numpy().reshape(5, K)
    d_got = np.log(op / (1 - op)) - 2.0
    c_g = Rg.T @ (c_w - tg)
    for a in range(5):
        d = an["xyz"][:, a] - c_g
        np.testing.assert_allclose(d_got[a], d / np.linalg.norm(d), atol=2e-6)


def test_decode_groups_use_their_own_mlp_and_pose():
    an = _anchors(A=6, K=2, seed=4)
    an["group_offsets"] = np.array([0, 4, 6])
    K, J = 2, 9
    m0 = dict(w1=np.zeros((32, 35)), b1=np.zeros(32), w2=np.zeros((K * J, 32)), b2=np.full(K * J, 0.3))
    m1 = dict(w1=np.zeros((32, 35)), b1=np.zeros(32), w2=np.zeros((K * J, 32)), b2=np.full(K * J, -0.7))
    poses = np.concatenate([IDPOSE, IDPOSE])
    out = odec.decode(an, [m0, m1], poses, "lidar")
    sig = lambda x: 1 / (1 + np.exp(-x))
    op = out["opacity"].numpy()
    np.testing.assert_allclose(op[:8], sig(0.3), atol=1e-14)
    np.testing.assert_allclose(op[8:], sig(-0.7), atol=1e-14)


def test_fd_gradient_through_decode_and_raster():
    # Decode (FP64) feeding the raster: autograd gradient of the composite
    # program w.r.t. features, weights and anchor geometry vs central differences.
    rng = np.random.default_rng(5)
    A, K = 2, 2
    an = dict(xyz=np.stack([rng.uniform(-0.15, 0.15, A), rng.uniform(-0.15, 0.15, A), rng.uniform(3.2, 3.6, A)]),
              scaling=rng.uniform(0.04, 0.06, A), offsets=0.5 * rng.standard_normal((3, K, A)),
              feat=rng.standard_normal((A, 32)), group_offsets=np.array([0, A]))
    J = 10
    mlp = dict(w1=rng.uniform(-0.17, 0.17, (32, 35)), b1=rng.uniform(-0.17, 0.17, 32),
               w2=rng.uniform(-0.18, 0.18, (K * J, 32)), b2=rng.uniform(-0.18, 0.18, K * J))
    opts = raster.make_opts(FD_OPTS)
    keys = ["xyz", "scaling", "offsets", "feat"]
    wkeys = ["w1_0", "b1_0", "w2_0", "b2_0"]

    def leaves(grad, over=None):
        d = {k: torch.as_tensor(np.asarray(an[k], np.float64)).requires_grad_(grad) for k in keys}
        for wk, mk in zip(wkeys, ("w1", "b1", "w2", "b2")):
            d[wk] = torch.as_tensor(np.asarray(mlp[mk], np.float64)).requires_grad_(grad)
        if over:
            d.update(over)
        return d

    def run(pd, grad_out=None):
        dec = odec.decode(an, [mlp], IDPOSE, "pinhole", params=pd)
        sc32 = {k: v.detach().numpy().astype(F32) for k, v in dec.items()}
        sc32.update(group_offsets=np.array([0, A * K], np.int32), group_poses=IDPOSE)
        return raster.render(sc32, FD_CAM, opts, params=dec, grad_out=grad_out)

    ref = run(leaves(False))
    go = {k: rng.standard_normal(ref[k].shape) for k in ("rgb", "depth", "alpha")}
    pd = leaves(True)
    dec = odec.decode(an, [mlp], IDPOSE, "pinhole", params=pd)
    sc32 = {k: v.detach().numpy().astype(F32) for k, v in dec.items()}
    sc32.update(group_offsets=np.array([0, A * K], np.int32), group_poses=IDPOSE)
    out = raster.render(sc32, FD_CAM, opts, params=dec)
    # raster.render returns numpy outputs; rebuild the scalar loss with autograd
    # by asking for gradients of the decoded leaves and chaining through decode.
    res = raster.render(sc32, FD_CAM, opts, params={k: v.detach().requires_grad_(True) for k, v in dec.items()},
                        grad_out=go)
    gdec = res["grads"]
    tot = sum((dec[k] * torch.as_tensor(gdec[k])).sum() for k in gdec)
    grads = torch.autograd.grad(tot, list(pd.values()), allow_unused=True)
    gmap = {k: (np.zeros(pd[k].shape) if g is None else g.numpy()) for k, g in zip(pd.keys(), grads)}
    del out

    def loss(over):
        o = run(leaves(False, over))
        return sum(float((o[k] * go[k]).sum()) for k in go)

    base_all = leaves(False)
    for k in keys + wkeys:
        base = base_all[k].numpy()
        flat = base.reshape(-1)
        gk = gmap[k].reshape(-1)
        gmax = np.abs(gk).max() + 1e-30
        for i in rng.choice(flat.size, min(6, flat.size), replace=False):
            h = 1e-6 * max(1.0, abs(flat[i]))
            vp, vm = flat.copy(), flat.copy()
            vp[i] += h
            vm[i] -= h
            fd = (loss({k: torch.as_tensor(vp.reshape(base.shape))}) -
                  loss({k: torch.as_tensor(vm.reshape(base.shape))})) / (2 * h)
            assert abs(fd - gk[i]) <= 2e-6 * max(gmax, 1.0), (k, i, fd, gk[i])
