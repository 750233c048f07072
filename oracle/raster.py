"""FP64 reference renderer for 2D Gaussian surfels -- TEST INFRASTRUCTURE ONLY.

Plain definition of what the renderer computes, per ray (Sec. III-A):

1. Each surfel is the sensor-frame map M = [s_u R t_u, s_v R t_v, mu_s] of
   Eq. 1 (W restricted to the rigid pose; intrinsics live in the planes).
2. A ray is the intersection of two planes h_u, h_v (Eq. 2): pinhole planes
   (Eq. 3) written in the sensor frame as h_u = (-1, 0, x_n), h_v = (0, -1, y_n)
   with x_n = (p_x - c_x)/f_x; LiDAR planes (Eq. 5) with the azimuth/elevation
   roles read so that both planes contain the beam direction:
   h_u = (sin az, -cos az, 0), h_v = (sin el cos az, sin el sin az, -cos el).
3. The hit (u, v) solves [h_u, h_v]^T M (u, v, 1)^T = 0, i.e. (u, v, 1) is
   proportional to a x b with a = h_u^T M, b = h_v^T M.
4. rho = u^2 + v^2, optionally low-pass filtered as min(rho, rho_lp) (the 2DGS
   filter against degenerate line projections, Sec. II), with rho_lp the
   squared distance to the projected centre in units of sigma (pinhole:
   pixels; LiDAR: chord to the centre direction in azimuth steps).
5. The candidate set of a ray is every visible surfel whose support contains
   it: rho_hat <= cutoff^2, depth (camera z / LiDAR range) > z_near.
   Candidates are ordered by the FP32 depth key, ties by surfel index.
   The depth of a pair is that of its hit point when rho itself is used and
   that of the surfel centre when the low-pass term is smaller (the filter's
   degenerate, edge-on case, where the hit point is not meaningful).
6. Front-to-back alpha compositing (Sec. II, splatting): alpha =
   min(alpha_max, o exp(-rho_hat/2)); skip if alpha < alpha_min; stop before a
   surfel that would take T (1 - alpha) below T_min; w = alpha T.
   Camera outputs: RGB + T_final*bg, depth (sum w z), normal (sum w n, normal
   turned to face the sensor), alpha (sum w).  LiDAR: range, intensity, alpha.

Floating point is FP64 everywhere except the integer decisions (visibility,
rectangles, key, normal sign), which follow the FP32 binning spec in
spec32.py.  Gradients are the autograd derivative of this FP64 program;
skip/stop decisions carry no gradient.  Two candidate modes: "brute" tests every
ray against every visible surfel; "culled" tests only surfels whose FP32 pixel
rectangle holds the ray.  Their equality on small scenes pins the rectangle's
conservativeness.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import sh as shmod
from . import spec32

F32 = np.float32
DT = torch.float64

PRODUCTION = dict(alpha_min=1.0 / 255.0, alpha_max=0.99, T_min=1e-4, cutoff2=2.0 * math.log(255.0),
                  lowpass=True, lp_inv_sigma2=2.0, tile_w=16, tile_h=16, bg=(0.0, 0.0, 0.0))
STRICT = dict(PRODUCTION, alpha_min=0.0, T_min=0.0, cutoff2=25.0)


def make_opts(base=PRODUCTION, **kw):
    o = dict(base)
    o.update(kw)
    # the FP32 spec reads these as float32 values; the FP64 side uses the same values
    o["cutoff2"] = float(F32(o["cutoff2"]))
    o["lp_inv_sigma2"] = float(F32(o["lp_inv_sigma2"]))
    o["alpha_min"] = float(F32(o["alpha_min"]))
    o["alpha_max"] = float(F32(o["alpha_max"]))
    o["T_min"] = float(F32(o["T_min"]))
    return o


# ----------------------------------------------------------------------------
# FP32 spec side: poses, frames, bins
# ----------------------------------------------------------------------------

def _group_of(scene) -> np.ndarray:
    go = np.asarray(scene["group_offsets"], np.int64)
    n = int(go[-1])
    g = np.zeros(n, np.int64)
    for i in range(len(go) - 1):
        g[go[i]:go[i + 1]] = i
    return g


def spec_frames(scene, sensor):
    """Per-surfel FP32 frame (concatenated over groups) and per-group composed poses."""
    go = np.asarray(scene["group_offsets"], np.int64)
    poses = [spec32.compose_pose(sensor["pose"], gp) for gp in np.asarray(scene["group_poses"], F32)]
    parts = []
    for g in range(len(go) - 1):
        sl = slice(int(go[g]), int(go[g + 1]))
        parts.append(spec32.splat_frame(poses[g], scene["mean"][:, sl], scene["quat"][:, sl],
                                        scene["scale"][:, sl]))
    fr = {}
    for key in ("mu_s", "tu_s", "tv_s", "n_s"):
        fr[key] = np.concatenate([p[key] for p in parts], axis=1)
    fr["M"] = np.concatenate([p["M"] for p in parts], axis=2)
    fr["valid"] = np.concatenate([p["valid"] for p in parts])
    return fr, np.stack(poses)


def is_lidar(sensor) -> bool:
    """LiDAR (range, intensity, alpha) rather than a camera (pinhole or cylindrical; 8 channels)."""
    return sensor["kind"] == "lidar"


def spec_bins(scene, sensor, opts):
    fr, poses = spec_frames(scene, sensor)
    if sensor["kind"] == "pinhole":
        b = spec32.pinhole_bins(fr, sensor, opts)
    elif sensor["kind"] == "cylindrical":
        b = spec32.cylindrical_bins(fr, scene["scale"], sensor, opts)
    else:
        b = spec32.lidar_bins(fr, scene["scale"], sensor, opts)
    b["normal_sign"] = spec32.normal_sign(fr["n_s"], fr["mu_s"])
    b["poses"] = poses
    b["frame"] = fr
    return b


# ----------------------------------------------------------------------------
# FP64 side
# ----------------------------------------------------------------------------

def _leaf(x, grad):
    t = torch.as_tensor(np.asarray(x, np.float64), dtype=DT)
    return t.requires_grad_(grad)


def _rays(sensor, ray_ids: np.ndarray):
    """Per-ray plane coefficients h_u, h_v [R,3], FP64, plus pixel data."""
    W = int(sensor["width"])
    i = ray_ids % W
    j = ray_ids // W
    if sensor["kind"] == "pinhole":
        px = i.astype(np.float64) + 0.5
        py = j.astype(np.float64) + 0.5
        xn = (px - sensor["cx"]) / sensor["fx"]
        yn = (py - sensor["cy"]) / sensor["fy"]
        hu = np.stack([-np.ones_like(xn), np.zeros_like(xn), xn], 1)
        hv = np.stack([np.zeros_like(yn), -np.ones_like(yn), yn], 1)
        return dict(hu=torch.as_tensor(hu), hv=torch.as_tensor(hv), px=torch.as_tensor(px),
                    py=torch.as_tensor(py), i=i, j=j)
    if sensor["kind"] == "cylindrical":
        # Eq. 4: h_u = (cos phi, 0, -sin phi); h_v = (y_n sin phi, -1, y_n cos phi),
        # the plane through the camera's x-free line at height y_n on the unit cylinder
        tabs = spec32.cylindrical_tables(sensor)
        sp = tabs["sin_phi"][i]
        cp = tabs["cos_phi"][i]
        yn = tabs["yn"][j]
        hu = np.stack([cp, np.zeros_like(cp), -sp], 1)
        hv = np.stack([yn * sp, -np.ones_like(yn), yn * cp], 1)
        hdir = np.stack([sp, np.zeros_like(sp), cp], 1)  # the column's horizontal direction
        return dict(hu=torch.as_tensor(hu), hv=torch.as_tensor(hv), hdir=torch.as_tensor(hdir),
                    px=torch.as_tensor(i.astype(np.float64) + 0.5), py=torch.as_tensor(j.astype(np.float64) + 0.5),
                    i=i, j=j)
    tabs = spec32.lidar_tables(sensor)
    ca = tabs["cos_az"][i].astype(np.float64)
    sa = tabs["sin_az"][i].astype(np.float64)
    ce = tabs["cos_el"][j].astype(np.float64)
    se = tabs["sin_el"][j].astype(np.float64)
    hu = np.stack([sa, -ca, np.zeros_like(sa)], 1)
    hv = np.stack([se * ca, se * sa, -ce], 1)
    d = np.stack([ce * ca, ce * sa, se], 1)
    return dict(hu=torch.as_tensor(hu), hv=torch.as_tensor(hv), d=torch.as_tensor(d), i=i, j=j)


def splat_quantities(scene, sensor, bins, params):
    """Differentiable FP64 per-surfel quantities in the sensor frame.

    params: dict of FP64 torch tensors mean [3,N], quat [4,N], scale [2,N],
    opacity [N], and rgb [3,N] | sh [nb*3,N] (camera) or intensity [N] (LiDAR).
    """
    g = _group_of(scene)
    P = torch.as_tensor(bins["poses"].astype(np.float64))[torch.as_tensor(g)]  # [N,3,4]
    Rm = P[:, :, :3]
    t = P[:, :, 3]
    mean, quat, scale = params["mean"], params["quat"], params["scale"]
    w, x, y, z = quat[0], quat[1], quat[2], quat[3]
    s = 2.0 / (w * w + x * x + y * y + z * z)
    tu = torch.stack([1 - s * (y * y + z * z), s * (x * y + w * z), s * (x * z - w * y)], 1)  # [N,3]
    tv = torch.stack([s * (x * y - w * z), 1 - s * (x * x + z * z), s * (y * z + w * x)], 1)
    nn = torch.stack([s * (x * z + w * y), s * (y * z - w * x), 1 - s * (x * x + y * y)], 1)
    mu_s = torch.einsum("nij,nj->ni", Rm, mean.T) + t
    tu_s = torch.einsum("nij,nj->ni", Rm, tu)
    tv_s = torch.einsum("nij,nj->ni", Rm, tv)
    n_s = torch.einsum("nij,nj->ni", Rm, nn)
    M = torch.stack([scale[0][:, None] * tu_s, scale[1][:, None] * tv_s, mu_s], 2)  # [N,3,3] (row, col)
    out = dict(M=M, mu_s=mu_s, opacity=params["opacity"])
    sign = torch.as_tensor(bins["normal_sign"].astype(np.float64))
    out["normal"] = n_s * sign[:, None]
    if not is_lidar(sensor):
        if "sh" in params and params["sh"] is not None:
            dirs = torch.einsum("nji,nj->ni", Rm, mu_s)  # R^T mu_s: object-frame ray direction
            dirs = dirs / torch.linalg.norm(dirs, dim=1, keepdim=True)
            out["colour"] = shmod.sh_colour(params["sh"], dirs.T, int(scene["sh_degree"])).T
        else:
            out["colour"] = params["rgb"].T
    else:
        out["intensity"] = params["intensity"]
        if params.get("drop") is not None:
            out["drop"] = params["drop"]
    return out


def grid_rays(sensor, stride: int) -> np.ndarray:
    """Flat ray ids of every stride-th column of every stride-th row (a regular sample)."""
    W, H = int(sensor["width"]), int(sensor["height"])
    j, i = np.meshgrid(np.arange(0, H, stride), np.arange(0, W, stride), indexing="ij")
    return (j * W + i).reshape(-1).astype(np.int64)


def _grid_pairs(bins, sensor, stride):
    """Candidate pairs for the grid_rays(sensor, stride) sample (pinhole rectangles)."""
    W, H = int(sensor["width"]), int(sensor["height"])
    nW = (W + stride - 1) // stride
    touch = np.nonzero(bins["touch"])[0]
    c_lo = -(-bins["i_lo"][touch] // stride)
    c_hi = bins["i_hi"][touch] // stride
    r_lo = -(-bins["j_lo"][touch] // stride)
    r_hi = bins["j_hi"][touch] // stride
    ncol = np.maximum(c_hi - c_lo + 1, 0)
    nrow = np.maximum(r_hi - r_lo + 1, 0)
    cnt = ncol * nrow
    sp = np.repeat(touch, cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(int(cnt.sum())) - start
    nc = np.repeat(np.maximum(ncol, 1), cnt)
    col = np.repeat(c_lo, cnt) + local % nc
    row = np.repeat(r_lo, cnt) + local // nc
    return row * nW + col, sp


def _grid_pairs_lidar(bins, sensor, stride):
    """Candidate pairs for the grid_rays(sensor, stride) sample of a LiDAR: the
    beam/column rectangles, whose columns may wrap ([i_lo, W) u [0, i_hi]) or
    span the full circle."""
    W = int(sensor["width"])
    nW = (W + stride - 1) // stride
    touch = np.nonzero(bins["touch"])[0]
    lo, hi = bins["i_lo"][touch], bins["i_hi"][touch]
    full = bins["full_cols"][touch]
    wrap = (lo > hi) & ~full
    # up to two inclusive column runs per surfel
    a1 = np.where(full, 0, lo)
    b1 = np.where(full | wrap, W - 1, hi)
    a2 = np.zeros_like(lo)
    b2 = np.where(wrap, hi, -1)
    r_lo = -(-bins["j_lo"][touch] // stride)
    r_hi = bins["j_hi"][touch] // stride
    nrow = np.maximum(r_hi - r_lo + 1, 0)
    rps, sps = [], []
    for a, b in ((a1, b1), (a2, b2)):
        c_lo = -(-a // stride)
        c_hi = np.where(b >= 0, b // stride, -1)
        ncol = np.maximum(c_hi - c_lo + 1, 0)
        cnt = ncol * nrow
        sp = np.repeat(touch, cnt)
        start = np.repeat(np.cumsum(cnt) - cnt, cnt)
        local = np.arange(int(cnt.sum())) - start
        nc = np.repeat(np.maximum(ncol, 1), cnt)
        col = np.repeat(c_lo, cnt) + local % nc
        row = np.repeat(r_lo, cnt) + local // nc
        rps.append(row * nW + col)
        sps.append(sp)
    return np.concatenate(rps), np.concatenate(sps)


def _candidate_pairs(bins, sensor, ray_ids, mode, grid_stride=None):
    """(ray position, surfel) candidate pairs before the per-pair support test."""
    if grid_stride is not None and mode != "brute":
        if not is_lidar(sensor):
            return _grid_pairs(bins, sensor, grid_stride)
        return _grid_pairs_lidar(bins, sensor, grid_stride)
    W = int(sensor["width"])
    vis = np.nonzero(bins["visible"])[0]
    R = ray_ids.size
    if mode == "brute":
        rp = np.repeat(np.arange(R), vis.size)
        sp = np.tile(vis, R)
        return rp, sp
    touch = np.nonzero(bins["touch"])[0]
    full_image = R == int(sensor["width"]) * int(sensor["height"]) and np.array_equal(ray_ids, np.arange(R))
    lidar = is_lidar(sensor)
    if full_image:
        i_lo, i_hi = bins["i_lo"][touch], bins["i_hi"][touch]
        j_lo, j_hi = bins["j_lo"][touch], bins["j_hi"][touch]
        if lidar:
            full = bins["full_cols"][touch]
            ncol = np.where(full, W, np.mod(i_hi - i_lo, W) + 1)
            i_lo = np.where(full, 0, i_lo)
        else:
            ncol = i_hi - i_lo + 1
        nrow = j_hi - j_lo + 1
        cnt = ncol * nrow
        sp = np.repeat(touch, cnt)
        start = np.repeat(np.cumsum(cnt) - cnt, cnt)
        local = np.arange(int(cnt.sum())) - start
        nc = np.repeat(ncol, cnt)
        col = (np.repeat(i_lo, cnt) + local % nc) % W
        row = np.repeat(j_lo, cnt) + local // nc
        return row * W + col, sp
    ii = ray_ids % W
    jj = ray_ids // W
    rps, sps = [], []
    il, ih = bins["i_lo"][touch], bins["i_hi"][touch]
    jl, jh = bins["j_lo"][touch], bins["j_hi"][touch]
    full = bins["full_cols"][touch] if lidar else None
    for c0 in range(0, R, 32):
        ci = ii[c0:c0 + 32, None]
        cj = jj[c0:c0 + 32, None]
        inr = (cj >= jl[None]) & (cj <= jh[None])
        if lidar:
            wrap = il > ih
            inc = np.where(wrap[None], (ci >= il[None]) | (ci <= ih[None]), (ci >= il[None]) & (ci <= ih[None]))
            inc |= full[None]
        else:
            inc = (ci >= il[None]) & (ci <= ih[None])
        r, s = np.nonzero(inr & inc)
        rps.append(r + c0)
        sps.append(touch[s])
    return np.concatenate(rps), np.concatenate(sps)


def render(scene, sensor, opts=None, *, mode="culled", rays=None, grad_out=None, margins=False,
           params=None, alternatives=None, max_flags=3):
    """Render one sensor in FP64.

    scene: dict of numpy arrays (see gen.scenes layouts; 'sh_degree' if 'sh').
    rays: None for the whole image, flat ray ids (row * width + col), or
    ("grid", stride) for the regular sample grid_rays(sensor, stride).
    grad_out: optional dict channel -> array shaped like the output; then the
    result also holds 'grads' (d(sum grad_out * out)/d inputs).
    params: optional dict of FP64 torch tensors to use as inputs (e.g. the
    output of the decode oracle); gradients then flow into them.
    margins: also return per ray the smallest relative distance of any of its
    compositing decisions to the decision's threshold ('margin'; with
    alternatives, in the measure that flags them, see _relative_distances).
    alternatives: a relative tolerance tol.  Every decision of a ray that lies
    within tol of its threshold -- a pair entering or leaving the support
    (cutoff, z_near), the alpha_min skip, the T_min stop, the choice between
    rho and the low-pass term (which sets the pair's depth) -- is flagged (a
    decision on rho also when rho lies within the first-order error bound of
    an FP32 evaluation of the solve, _fp32_uv_error), and the
    result also holds, for every ray with 1..max_flags flags, the outputs the
    definition gives when any non-empty subset of those decisions goes the
    other way ('alts': rays, values [n_alt, C] in the channel order of the
    device layout); rays with more flags are listed in 'unverified'.
    Returns dict of numpy FP64 outputs shaped [C, H, W] (or [C, R] for rays):
    camera rgb, depth, normal, alpha, median (depth); LiDAR range, intensity,
    alpha, drop (ray-drop probability), drop_mask, median (range); and
    T_final.  The alternatives' value vectors hold every channel in the
    device order (camera 9, LiDAR 6).
    """
    opts = make_opts(**(opts or {})) if not isinstance(opts, dict) or "tile_w" not in opts else opts
    W, H = int(sensor["width"]), int(sensor["height"])
    lidar = is_lidar(sensor)
    full = rays is None
    grid_stride = None
    if isinstance(rays, tuple) and rays[0] == "grid":
        grid_stride = int(rays[1])
        rays = grid_rays(sensor, grid_stride)
    ray_ids = np.arange(W * H, dtype=np.int64) if full else np.asarray(rays, np.int64)
    R = ray_ids.size
    bins = spec_bins(scene, sensor, opts)
    want_grad = grad_out is not None
    if params is None:
        params = dict(mean=_leaf(scene["mean"], want_grad), quat=_leaf(scene["quat"], want_grad),
                      scale=_leaf(scene["scale"], want_grad), opacity=_leaf(scene["opacity"], want_grad))
        if lidar:
            params["intensity"] = _leaf(scene["intensity"], want_grad)
            if scene.get("drop") is not None:
                params["drop"] = _leaf(scene["drop"], want_grad)
        elif scene.get("sh") is not None:
            params["sh"] = _leaf(scene["sh"], want_grad)
        else:
            params["rgb"] = _leaf(scene["rgb"], want_grad)
    sq = splat_quantities(scene, sensor, bins, params)
    rays_t = _rays(sensor, ray_ids)
    tol = float(alternatives) if alternatives is not None else 0.0

    rp, sp = _candidate_pairs(bins, sensor, ray_ids, mode, grid_stride)
    # ----- no-grad pass: support test on every candidate pair; pairs within
    # tol of the support boundary stay listed (not present) for the alternatives
    with torch.no_grad():
        sol = _solve(sq, rays_t, rp, sp, sensor, opts, scene, tol)
        keep = (sol["support"] | sol["near"]).numpy()
    rp, sp = rp[keep], sp[keep]
    # ----- order: ray, then FP32 key bits, then surfel index
    order = np.lexsort((sp, bins["key_bits"][sp], rp))
    rp, sp = rp[order], sp[order]
    # ----- differentiable pass on listed pairs only
    sol = _solve(sq, rays_t, rp, sp, sensor, opts, scene, tol)
    counts = np.bincount(rp, minlength=R)
    K = int(counts.max()) if counts.size and counts.max() > 0 else 1
    seg_start = np.cumsum(counts) - counts
    pos = np.arange(rp.size) - seg_start[rp]
    rp_t, pos_t = torch.as_tensor(rp), torch.as_tensor(pos)
    sp_t = torch.as_tensor(sp)

    def grid(v, fill=0.0):  # per pair [P] -> [R, K]
        z = torch.full((R, K), fill, dtype=v.dtype) if v.dtype != torch.bool else torch.zeros((R, K), dtype=torch.bool)
        return z.index_put((rp_t, pos_t), v)

    o = sq["opacity"][sp_t]
    a_raw = o * torch.exp(-0.5 * sol["rho_hat"])
    alpha = grid(torch.clamp(a_raw, max=opts["alpha_max"]))
    present = grid(sol["support"].detach())
    listed = grid(torch.ones(rp.size, dtype=torch.bool))
    # per-pair features in the device channel order
    if lidar:
        # ray-drop probability: a ray that meets nothing returns nothing (background 1)
        drop = sq["drop"][sp_t] if sq.get("drop") is not None else torch.zeros(rp.size, dtype=DT)
        feats = [sol["depth"], sq["intensity"][sp_t], torch.ones(rp.size, dtype=DT), drop]
        bg = torch.as_tensor([0.0, 0.0, 0.0, 1.0], dtype=DT)
    else:
        col = sq["colour"][sp_t]
        nrm = sq["normal"][sp_t]
        feats = [col[:, 0], col[:, 1], col[:, 2], sol["depth"], nrm[:, 0], nrm[:, 1], nrm[:, 2],
                 torch.ones(rp.size, dtype=DT)]
        bg = torch.as_tensor([opts["bg"][0], opts["bg"][1], opts["bg"][2], 0, 0, 0, 0, 0], dtype=DT)
    feat = torch.stack([grid(f) for f in feats], 2)  # [R, K, C]

    active, T_ex, test, skip, stopped = _decide(alpha.detach(), present, opts)
    dch = 0 if lidar else 3
    full_out, T_final = _compose(active, alpha, feat, bg, dch, lidar)

    outs = {}
    if lidar:
        outs["range"], outs["intensity"], outs["alpha"] = full_out[:, 0], full_out[:, 1], full_out[:, 2]
        outs["drop"], outs["drop_mask"], outs["median"] = full_out[:, 3], full_out[:, 4], full_out[:, 5]
    else:
        outs["rgb"] = full_out[:, 0:3].T
        outs["depth"] = full_out[:, 3]
        outs["normal"] = full_out[:, 4:7].T
        outs["alpha"] = full_out[:, 7]
        outs["median"] = full_out[:, 8]
    outs["T_final"] = T_final

    result = {}
    shape = (H, W) if full else (R,)
    for k_, v in outs.items():
        vv = v.detach().numpy()
        result[k_] = vv.reshape((vv.shape[0],) + shape) if vv.ndim == 2 else vv.reshape(shape)
    result["n_contrib"] = active.sum(1).numpy().reshape(shape)
    first_stop = torch.where(stopped.any(1), stopped.to(torch.int64).argmax(1), torch.full((R,), K))
    considered = listed & (torch.arange(K)[None, :] <= first_stop[:, None])
    derived = _derived_distances(active, alpha.detach(), full_out.detach(), lidar)
    if margins:
        result["margin"] = _margins(sol, rp, pos, R, K, alpha.detach(), test, skip, considered, opts,
                                    sensor, derived, tol).reshape(shape)
    if alternatives is not None:
        with torch.no_grad():
            alt = dict(alpha=grid(torch.clamp(o.detach() * torch.exp(-0.5 * sol["alt"]["rho_hat"]),
                                              max=opts["alpha_max"])),
                       present=grid(sol["alt"]["support"]), depth=grid(sol["alt"]["depth"]),
                       ch=0 if lidar else 3)
        result.update(_alternatives(sol, rp, pos, R, K, alpha.detach(), present, listed, feat.detach(), bg, test,
                                    skip, considered, opts, tol, max_flags, sensor, alt, derived))
    if want_grad:
        total = 0.0
        for k_, g in grad_out.items():
            gt = torch.as_tensor(np.asarray(g, np.float64)).reshape(outs[k_].shape)
            total = total + (outs[k_] * gt).sum()
        leaves = {k_: v for k_, v in params.items() if isinstance(v, torch.Tensor) and v.requires_grad}
        if isinstance(total, torch.Tensor) and total.requires_grad:
            gs = torch.autograd.grad(total, list(leaves.values()), allow_unused=True)
        else:
            gs = [None] * len(leaves)
        result["grads"] = {k_: (torch.zeros_like(v) if g is None else g).detach().numpy()
                           for (k_, v), g in zip(leaves.items(), gs)}
    result["bins"] = bins
    return result


def _decide(alpha, present, opts, flips=None):
    """Front-to-back skip and stop decisions on [R, K] depth-ordered pairs.

    A pair is skipped when it is not in the ray's support or its alpha is
    below alpha_min; before compositing a non-skipped pair the ray stops if
    T (1 - alpha) < T_min (the pair and everything after it are excluded).
    flips: optional (support, alpha_min, stop) [R, K] masks that toggle the
    outcome of the support test, of the alpha_min test and of the stop test at
    chosen pairs (a near-threshold decision taken the other way).
    Returns (active, T_ex, test, skip, stopped), no gradient.
    """
    with torch.no_grad():
        R = alpha.shape[0]
        pres = present
        low = alpha < opts["alpha_min"]
        if flips is not None:
            pres = pres ^ flips[0]
            low = low ^ flips[1]
        skip = (~pres) | low
        a_eff = torch.where(skip, torch.zeros_like(alpha), alpha)
        one_m = 1.0 - a_eff
        T_ex = torch.cumprod(torch.cat([torch.ones((R, 1), dtype=DT), one_m[:, :-1]], 1), 1)
        test = T_ex * one_m
        stop_ev = (~skip) & (test < opts["T_min"])
        if flips is not None:
            stop_ev = stop_ev ^ (flips[2] & ~skip)
        stopped = torch.cumsum(stop_ev.to(torch.int64), 1) > 0
        active = (~skip) & (~stopped)
    return active, T_ex, test, skip, stopped


def _accumulate(active, alpha, feat, bg):
    """Weights w_i = alpha_i T_i of the active pairs and the channel sums
    O = sum_i w_i f_i + T_final bg (front-to-back compositing)."""
    a_fin = torch.where(active, alpha, torch.zeros_like(alpha))
    om = 1.0 - a_fin
    R = alpha.shape[0]
    T = torch.cumprod(torch.cat([torch.ones((R, 1), dtype=DT), om[:, :-1]], 1), 1)
    w = a_fin * T
    T_final = T[:, -1] * om[:, -1]
    out = (w[:, :, None] * feat).sum(1) + T_final[:, None] * bg[None, :]
    return out, w, T_final


def _median_and_mask(active, alpha, feat, out, dch, lidar, med_flip=None, mask_flip=None):
    """The derived channels.  Median depth (2DGS): the depth feature of the
    first composited pair after which the transmittance is below 1/2, 0 where
    it never falls that low.  LiDAR ray drop: the composited drop probability
    P (background 1) and the drop mask P > 1/2.  med_flip [R, K] toggles the
    test T_after < 1/2 at chosen pairs, mask_flip [R] the mask (near-threshold
    decisions taken the other way).  Returns the extra channels [R, E]."""
    with torch.no_grad():
        a_fin = torch.where(active, alpha, torch.zeros_like(alpha))
        T_after = torch.cumprod(1.0 - a_fin, 1)
        b = active & (T_after < 0.5)
        if med_flip is not None:
            b = b ^ med_flip
        has = b.any(1)
        first = torch.where(has, b.to(torch.int64).argmax(1), torch.zeros_like(has, dtype=torch.int64))
    R = alpha.shape[0]
    med = torch.where(has, feat[torch.arange(R), first, dch], torch.zeros(R, dtype=DT))
    if not lidar:
        return med[:, None]
    P = out[:, 3]
    with torch.no_grad():
        mask = P > 0.5
        if mask_flip is not None:
            mask = mask ^ mask_flip
    return torch.stack([P, mask.to(DT), med], 1)


def _compose(active, alpha, feat, bg, dch, lidar, med_flip=None, mask_flip=None):
    """Every output channel in the device order ([R, C]: the camera's 8
    sums and its median depth; the LiDAR's range, intensity and alpha sums,
    drop probability, drop mask and median range) and T_final."""
    out, w, T_final = _accumulate(active, alpha, feat, bg)
    ext = _median_and_mask(active, alpha, feat, out, dch, lidar, med_flip, mask_flip)
    if lidar:
        return torch.cat([out[:, 0:3], ext], 1), T_final
    return torch.cat([out, ext], 1), T_final


def _fp32_uv_error(M, mu, u, v, rays_t, rp_t, sensor, opts):
    """First-order bound on the (u, v) error of the ray-splat solve carried
    out in FP32 (test infrastructure: it sizes the window within which a
    decision on rho is verified both ways, not any output).

    The FP32 solve evaluates the homography of Eq. 2 on pixel offsets from the
    projected centre (LiDAR: on direction offsets from the centre direction),
    h' = P d + e3 normalised so that h'_2 = 1 at the centre; a surfel seen
    nearly edge-on makes P's rows large and the evaluation cancels.  With
    kappa the largest absolute sum of the (u, v) rows of P plus 3.4 times that
    of its h'_2 row, the error is bounded by
      pinhole      (2^-22 kappa |d|_inf + 2^-20) / |h'_2|
      cylindrical  (2^-21 kappa |(X, Y)|_inf + 2^-20) / |h'_2|, X = f tan dphi,
                   Y = dy + (p_y - c_y)(sec dphi - 1) in the centre's column frame
      LiDAR        (2^-23 kappa (2 |d|_inf + |d_p|_inf + |c|_inf) + 2^-20) / |h'_2|,
                   d = ray - centre direction, c = tile reference ray - centre
                   direction, d_p = ray - tile reference ray
    (two roundings of the offsets' size, two in the products, the centre held
    to twice FP32 precision in the tile's frame)."""
    det = torch.linalg.det(M)
    adj = torch.linalg.inv(M) * det[:, None, None]
    kind = sensor["kind"]
    if kind in ("pinhole", "cylindrical"):
        if kind == "pinhole":
            muz = mu[:, 2]
            pcx = sensor["fx"] * mu[:, 0] / muz + sensor["cx"]
        else:
            muz = torch.sqrt(mu[:, 0] ** 2 + mu[:, 2] ** 2)
            c, sn = mu[:, 2] / muz, mu[:, 0] / muz
            adj = torch.stack([adj[:, :, 0] * c[:, None] - adj[:, :, 2] * sn[:, None], adj[:, :, 1],
                               adj[:, :, 0] * sn[:, None] + adj[:, :, 2] * c[:, None]], 2)
            pcx = sensor["fx"] * torch.atan2(mu[:, 0], mu[:, 2]) + sensor["cx"]
        pcy = sensor["fy"] * mu[:, 1] / muz + sensor["cy"]
        P = torch.stack([adj[:, :, 0] * (muz / (sensor["fx"] * det))[:, None],
                         adj[:, :, 1] * (muz / (sensor["fy"] * det))[:, None]], 2)  # [P, 3 rows, 2]
        dx = rays_t["px"][rp_t] - pcx
        dy = rays_t["py"][rp_t] - pcy
        if kind == "pinhole":
            X, Y, w = dx, dy, 2.0 ** -22
        else:
            ph = dx / sensor["fx"]
            X = sensor["fx"] * torch.tan(ph)
            Y = dy + (rays_t["py"][rp_t] - sensor["cy"]) * (1.0 / torch.cos(ph) - 1.0)
            w = 2.0 ** -21
        rs = P.abs().sum(2)
        kap = torch.maximum(rs[:, 0], rs[:, 1]) + 3.4 * rs[:, 2]
        h2 = 1.0 + P[:, 2, 0] * X + P[:, 2, 1] * Y
        e = (w * kap * torch.maximum(X.abs(), Y.abs()) + 2.0 ** -20) / h2.abs()
    else:
        rn = torch.linalg.norm(mu, dim=1)
        Q = adj * (rn / det)[:, None, None]
        mh = mu / rn[:, None]
        d = rays_t["d"][rp_t] - mh
        tw, th = int(opts["tile_w"]), int(opts["tile_h"])
        i, j = rays_t["i"][rp_t.numpy()], rays_t["j"][rp_t.numpy()]
        ref = (j // th) * th * int(sensor["width"]) + (i // tw) * tw
        dt = _rays(sensor, ref)["d"]
        c = dt - mh
        dp = rays_t["d"][rp_t] - dt
        rs = Q.abs().sum(2)
        kap = torch.maximum(rs[:, 0], rs[:, 1]) + 3.4 * rs[:, 2]
        h2 = 1.0 + (Q[:, 2, :] * d).sum(1)
        e = (2.0 ** -23 * kap * (2.0 * d.abs().amax(1) + dp.abs().amax(1) + c.abs().amax(1)) + 2.0 ** -20) / h2.abs()
    # rho's error: 2 |(u, v)|_1 e + 2 e^2, taken with a 20% margin
    return 2.4 * (u.abs() + v.abs()) * e + 2.0 * e * e


def _solve(sq, rays_t, rp, sp, sensor, opts, scene, tol=0.0):
    """Per-pair ray-splat solve (Eq. 2): (u, v), rho_hat, depth, support mask,
    and `near`: the support decision, or the choice between the surfel's own
    rho and the low-pass term, lies within tol (relative) of its threshold.

    Depth (camera z, LiDAR range) is that of the hit point x = M (u, v, 1)
    when rho itself is used.  When the low-pass term is smaller, the pair is
    the degenerate line projection the filter stands in for (Sec. II): the
    plane is seen (nearly) edge-on, its hit point is not meaningful and can
    lie arbitrarily far along the ray, so the pair takes the depth of the
    surfel centre (camera mu_z, LiDAR |mu|), as the cited 2DGS filter does.
    The same depth decides the z_near test.  `alt` holds the pair's rho_hat,
    depth and support under the other choice.
    """
    rp_t = torch.as_tensor(rp)
    sp_t = torch.as_tensor(sp)
    M = sq["M"][sp_t]  # [P,3,3]
    hu = rays_t["hu"][rp_t]
    hv = rays_t["hv"][rp_t]
    a = torch.einsum("pi,pij->pj", hu, M)
    b = torch.einsum("pi,pij->pj", hv, M)
    h = torch.linalg.cross(a, b, dim=1)
    h2 = h[:, 2]
    ok = h2 != 0
    h2s = torch.where(ok, h2, torch.ones_like(h2))
    u = h[:, 0] / h2s
    v = h[:, 1] / h2s
    rho = u * u + v * v
    uv1 = torch.stack([u, v, torch.ones_like(u)], 1)
    X = torch.einsum("pij,pj->pi", M, uv1)
    mu = sq["mu_s"][sp_t]
    lp = opts["lp_inv_sigma2"]
    if sensor["kind"] == "pinhole":
        depth_hit = X[:, 2]
        depth_c = mu[:, 2]
        if opts["lowpass"]:
            pcx = sensor["fx"] * mu[:, 0] / mu[:, 2] + sensor["cx"]
            pcy = sensor["fy"] * mu[:, 1] / mu[:, 2] + sensor["cy"]
            dx = rays_t["px"][rp_t] - pcx
            dy = rays_t["py"][rp_t] - pcy
            rho_lp = lp * (dx * dx + dy * dy)
    elif sensor["kind"] == "cylindrical":
        # cylindrical depth: distance from the camera's vertical axis, signed
        # along the column's horizontal direction (negative behind the camera)
        hd = rays_t["hdir"][rp_t]
        depth_hit = (hd * X).sum(1) / torch.linalg.norm(hd, dim=1)
        r_c = torch.sqrt(mu[:, 0] * mu[:, 0] + mu[:, 2] * mu[:, 2])
        depth_c = r_c
        if opts["lowpass"]:
            pcx = sensor["fx"] * torch.atan2(mu[:, 0], mu[:, 2]) + sensor["cx"]
            pcy = sensor["fy"] * mu[:, 1] / r_c + sensor["cy"]
            dx = rays_t["px"][rp_t] - pcx
            dy = rays_t["py"][rp_t] - pcy
            rho_lp = lp * (dx * dx + dy * dy)
    else:
        d = rays_t["d"][rp_t]
        depth_hit = (d * X).sum(1)
        rn = torch.linalg.norm(mu, dim=1)
        depth_c = rn
        if opts["lowpass"]:
            step = 2.0 * math.pi / int(sensor["width"])
            mh = mu / rn[:, None]
            dd = d - mh
            rho_lp = lp * (dd * dd).sum(1) / (step * step)
    c2, zn = opts["cutoff2"], sensor["z_near"]
    with torch.no_grad():
        drho = _fp32_uv_error(M.detach(), mu.detach(), u.detach(), v.detach(), rays_t, rp_t, sensor, opts)
    if opts["lowpass"]:
        use_rho = rho <= rho_lp
        rho_hat = torch.where(use_rho, rho, rho_lp)
        depth = torch.where(use_rho, depth_hit, depth_c)
    else:
        rho_hat = rho
        depth = depth_hit
    support = ok & (rho_hat <= c2) & (depth > zn)
    with torch.no_grad():
        # a window of tol relative, widened to rho's FP32 error bound where
        # rho itself is compared (not the low-pass term, which has no such error)
        wr = drho if tol > 0.0 else torch.zeros_like(drho)
        wt = torch.full_like(wr, tol * c2)
        rho_dec = use_rho if opts["lowpass"] else torch.ones_like(ok)
        wc = torch.where(rho_dec, torch.maximum(wt, wr), wt)
        near = ok & (((rho_hat - c2).abs() <= wc) | ((depth - zn).abs() <= tol * zn))
        if opts["lowpass"]:
            big = torch.maximum(rho, rho_lp)
            scale = torch.maximum(big, wr / tol) if tol > 0.0 else big
            d_lp = torch.where(big > 0, (rho - rho_lp).abs() / torch.where(big > 0, scale, torch.ones_like(scale)),
                               torch.full_like(big, math.inf))
            near_lp = ok & (d_lp <= tol)
            rho_alt = torch.where(use_rho, rho_lp, rho).detach()
            depth_alt = torch.where(use_rho, depth_c, depth_hit).detach()
            support_alt = ok & (rho_alt <= c2) & (depth_alt > zn)
            wc_alt = torch.where(use_rho, wt, torch.maximum(wt, wr))
            near = near | (near_lp & (support_alt | ((rho_alt - c2).abs() <= wc_alt) |
                                      ((depth_alt - zn).abs() <= tol * zn)))
        else:
            d_lp = torch.full_like(rho, math.inf)
            rho_alt, depth_alt, support_alt = rho_hat.detach(), depth.detach(), support.detach()
        if tol <= 0.0:
            near = torch.zeros_like(near)
    # the support and alpha_min decisions see rho's error only where rho decides
    drho_dec = torch.where(use_rho, drho, torch.zeros_like(drho)) if opts["lowpass"] else drho
    return dict(u=u, v=v, rho_hat=rho_hat, depth=depth, support=support, near=near, d_lp=d_lp, drho=drho_dec,
                alt=dict(rho_hat=rho_alt, depth=depth_alt, support=support_alt))


def _relative_distances(sol, rp, pos, R, K, alpha, test, skip, opts, sensor, tol=0.0):
    """Per listed pair [R, K]: relative distance of its support decision
    (cutoff, z_near), its alpha_min skip, (non-skipped pairs) its T_min stop
    test and its choice between rho and the low-pass term to the threshold;
    inf where the rule is off.  With tol > 0 the distances of the decisions
    on rho are scaled so that a pair whose rho lies within its FP32 error
    bound of the threshold (sol['drho']) also comes out at most tol."""
    rp_t, pos_t = torch.as_tensor(rp), torch.as_tensor(pos)
    with torch.no_grad():
        rh = sol["rho_hat"].detach()
        dep = sol["depth"].detach()
        c2, zn = opts["cutoff2"], sensor["z_near"]
        wr = sol["drho"].detach() / tol if tol > 0.0 else torch.zeros_like(rh)
        m_sup = torch.minimum((rh - c2).abs() / torch.clamp(wr, min=c2), (dep - zn).abs() / max(zn, 1e-300))
        d_sup = torch.full((R, K), math.inf, dtype=DT).index_put((rp_t, pos_t), m_sup)
        d_lp = torch.full((R, K), math.inf, dtype=DT).index_put((rp_t, pos_t), sol["d_lp"].detach())
        inf = torch.full((R, K), math.inf, dtype=DT)
        am, tm = opts["alpha_min"], opts["T_min"]
        # alpha moves by about alpha drho / 2 (0.6 with margin) when rho does by drho
        wa = torch.zeros((R, K), dtype=DT).index_put((rp_t, pos_t), wr) * alpha * 0.6
        d_amin = (alpha - am).abs() / torch.clamp(wa, min=am) if am > 0 else inf
        d_stop = torch.where(skip, inf, (test - tm).abs() / tm) if tm > 0 else inf
    return d_sup, d_amin, d_stop, d_lp


def _derived_distances(active, alpha, out_full, lidar):
    """Relative distances of the derived channels' decisions to their
    thresholds: per pair [R, K] the median crossing test T_after < 1/2 (active
    pairs), per ray [R] the LiDAR drop mask P > 1/2 (inf for cameras)."""
    with torch.no_grad():
        a_fin = torch.where(active, alpha, torch.zeros_like(alpha))
        T_after = torch.cumprod(1.0 - a_fin, 1)
        d_med = torch.where(active, (T_after - 0.5).abs() / 0.5, torch.full_like(alpha, math.inf))
        if lidar:
            d_mask = (out_full[:, 3] - 0.5).abs() / 0.5
        else:
            d_mask = torch.full((alpha.shape[0],), math.inf, dtype=DT)
    return d_med, d_mask


def _margins(sol, rp, pos, R, K, alpha, test, skip, considered, opts, sensor, derived, tol=0.0):
    """Per ray: the smallest relative distance of any decision of a considered
    pair (up to and including the stopping one) to its threshold (with
    tol > 0, in the scaled measure of _relative_distances), the derived
    channels' decisions (median crossing, drop mask) included."""
    d_sup, d_amin, d_stop, d_lp = _relative_distances(sol, rp, pos, R, K, alpha, test, skip, opts, sensor, tol)
    d_med, d_mask = derived
    m = torch.minimum(torch.minimum(d_sup, d_amin), torch.minimum(d_stop, d_lp))
    m = torch.minimum(m, d_med)
    m = torch.where(considered, m, torch.full_like(m, math.inf))
    mr = m.min(1).values if K > 0 else torch.full((R,), math.inf, dtype=DT)
    return torch.minimum(mr, d_mask).numpy()


def _alternatives(sol, rp, pos, R, K, alpha, present, listed, feat, bg, test, skip, considered, opts, tol,
                  max_flags, sensor, alt, derived):
    """Outputs of every ray under each non-empty subset of its near-threshold
    decisions taken the other way (see render's `alternatives`).  Flag kinds:
    0 support (cutoff or z_near), 1 alpha_min, 2 stop, 3 the choice between
    rho and the low-pass term (the other choice gives the pair the alpha,
    depth and support in `alt`: [R, K] grids 'alpha', 'present', 'depth', and
    the depth channel index 'ch'), 4 the median crossing test T < 1/2 at a
    pair, 5 the LiDAR drop mask P > 1/2 (listed at pair 0)."""
    d_sup, d_amin, d_stop, d_lp = _relative_distances(sol, rp, pos, R, K, alpha, test, skip, opts, sensor, tol)
    d_med, d_mask = derived
    lidar = is_lidar(sensor)
    with torch.no_grad():
        mask_col = torch.zeros((R, K), dtype=torch.bool)
        mask_col[:, 0] = d_mask <= tol
        fm = [considered & (d_sup <= tol), considered & (d_amin <= tol), considered & (d_stop <= tol),
              considered & (d_lp <= tol), considered & (d_med <= tol), mask_col]
        n_flags = sum(f.to(torch.int64) for f in fm).sum(1)
    nf = n_flags.numpy()
    rays = np.nonzero((nf >= 1) & (nf <= max_flags))[0]
    unverified = np.nonzero(nf > max_flags)[0]
    values, kinds = [], []
    for r in rays:
        r_t = torch.as_tensor([int(r)])
        flags = [(kd, int(k)) for kd in range(6) for k in torch.nonzero(fm[kd][r]).reshape(-1).tolist()]
        alts = []
        for subset in range(1, 1 << len(flags)):
            a_r, p_r, f_r = alpha[r_t].clone(), present[r_t].clone(), feat[r_t].clone()
            fl = [torch.zeros((1, K), dtype=torch.bool) for _ in range(3)]
            med_flip = torch.zeros((1, K), dtype=torch.bool)
            mask_flip = torch.zeros((1,), dtype=torch.bool)
            for b, (kd, k) in enumerate(flags):
                if (subset >> b) & 1:
                    if kd == 3:
                        a_r[0, k] = alt["alpha"][r, k]
                        p_r[0, k] = alt["present"][r, k]
                        f_r[0, k, alt["ch"]] = alt["depth"][r, k]
                    elif kd == 4:
                        med_flip[0, k] = True
                    elif kd == 5:
                        mask_flip[0] = True
                    else:
                        fl[kd][0, k] = True
            act = _decide(a_r, p_r, opts, flips=fl)[0]
            alts.append(_compose(act, a_r, f_r, bg, alt["ch"], lidar, med_flip, mask_flip)[0][0].numpy())
        values.append(np.stack(alts))
        kinds.append([kd for kd, _ in flags])
    return dict(alts=dict(rays=rays, values=values, kinds=kinds), unverified=unverified, n_flags=nf)
