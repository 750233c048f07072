"""FP32 binning specification (oracle side) -- TEST INFRASTRUCTURE ONLY.

The renderer's integer outputs (which splats are visible, which tiles each one
touches, and the depth key that orders them) are decided in single precision.
To make those decisions comparable bit for bit, they follow a written FP32
specification: IEEE-754 binary32 operations only (+ - * / sqrt, correctly
rounded, no fused multiply-add, fixed association order), evaluated here with
numpy float32 arrays.  The HIP path implements the same specification
independently.

Geometry follows Sec. III-A: a surfel is the tangent-plane map of Eq. 1,
P(u,v) = W H (u,v,1)^T with H = [s_u t_u, s_v t_v, mu; 0 0 1].  We restrict W
to the rigid world->sensor transform and move the intrinsics into the ray
planes (Eq. 3 for pinhole, Eq. 5 for LiDAR), so the surfel becomes the 3x3
sensor-frame matrix M = [s_u R t_u, s_v R t_v, R mu + t].

Nothing here is differentiated; the FP64 renderer reads only the integer
decisions (visibility, pixel/tile rectangles, key bits, normal sign) and the
FP32 composed pose.
"""
from __future__ import annotations

import math

import numpy as np

F32 = np.float32
PI_F = F32(math.pi)
HALF_PI_F = F32(math.pi / 2)

# Abramowitz & Stegun 4.4.49: atan(t) on [0,1] as an odd degree-9 polynomial,
# absolute error <= 1e-5 rad.  Used only to *guess* LiDAR angular ranges; the
# ranges are padded by a full angular step, so the guess error is harmless.
ATAN_C = (F32(0.9998660), F32(-0.3302995), F32(0.1801410), F32(-0.0851330), F32(0.0208351))


def _f(x):
    a = np.asarray(x)
    assert a.dtype == np.float32, a.dtype
    return a


# ----------------------------------------------------------------------------
# a0: pose composition
# ----------------------------------------------------------------------------

def compose_pose(sensor_pose: np.ndarray, group_pose: np.ndarray) -> np.ndarray:
    """FP32 3x4 sensor<-object transform V_s * G_g (no FMA, left-to-right sums).

    R[i][j] = (Rs[i][0]*Rg[0][j] + Rs[i][1]*Rg[1][j]) + Rs[i][2]*Rg[2][j]
    t[i]    = ((Rs[i][0]*tg[0] + Rs[i][1]*tg[1]) + Rs[i][2]*tg[2]) + ts[i]
    """
    a = _f(np.asarray(sensor_pose, F32).reshape(3, 4))
    b = _f(np.asarray(group_pose, F32).reshape(3, 4))
    out = np.zeros((3, 4), F32)
    for i in range(3):
        for j in range(3):
            out[i, j] = (a[i, 0] * b[0, j] + a[i, 1] * b[1, j]) + a[i, 2] * b[2, j]
        out[i, 3] = ((a[i, 0] * b[0, 3] + a[i, 1] * b[1, 3]) + a[i, 2] * b[2, 3]) + a[i, 3]
    return out


# ----------------------------------------------------------------------------
# a2: sensor-frame surfel matrix (shared by both sensor kinds)
# ----------------------------------------------------------------------------

def splat_frame(pose: np.ndarray, mean, quat, scale):
    """Sensor-frame quantities in FP32.

    pose: FP32 3x4 sensor<-object.  mean [3,N], quat [4,N] (w,x,y,z, any norm),
    scale [2,N].  Returns dict with mu_s [3,N], tu_s, tv_s, n_s [3,N],
    M [3,3,N] (columns s_u*tu_s, s_v*tv_s, mu_s) and valid [N] (finite, q != 0).

    Rotation of a (not necessarily unit) quaternion, with s = 2/|q|^2:
      t_u = (1 - s(yy+zz), s(xy+wz), s(xz-wy))
      t_v = (s(xy-wz), 1 - s(xx+zz), s(yz+wx))
      n   = (s(xz+wy), s(yz-wx), 1 - s(xx+yy))
    """
    p = _f(np.asarray(pose, F32))
    mean, quat, scale = _f(mean), _f(quat), _f(scale)
    one = F32(1.0)
    two = F32(2.0)

    def rot(v0, v1, v2):
        return [((p[i, 0] * v0 + p[i, 1] * v1) + p[i, 2] * v2) for i in range(3)]

    mu_s = [((p[i, 0] * mean[0] + p[i, 1] * mean[1]) + p[i, 2] * mean[2]) + p[i, 3] for i in range(3)]
    w, x, y, z = quat[0], quat[1], quat[2], quat[3]
    nq2 = ((w * w + x * x) + y * y) + z * z
    with np.errstate(divide="ignore", invalid="ignore", over="ignore"):
        s = two / nq2
        xx, yy, zz = x * x, y * y, z * z
        xy, xz, yz = x * y, x * z, y * z
        wx, wy, wz = w * x, w * y, w * z
        tu = [one - s * (yy + zz), s * (xy + wz), s * (xz - wy)]
        tv = [s * (xy - wz), one - s * (xx + zz), s * (yz + wx)]
        nn = [s * (xz + wy), s * (yz - wx), one - s * (xx + yy)]
        tu_s = rot(*tu)
        tv_s = rot(*tv)
        n_s = rot(*nn)
        M = np.stack([np.stack([scale[0] * tu_s[i], scale[1] * tv_s[i], mu_s[i]]) for i in range(3)])
    finite = np.isfinite(M).all(axis=(0, 1)) & np.isfinite(np.stack(n_s)).all(axis=0)
    valid = finite & (nq2 > 0) & (scale[0] > 0) & (scale[1] > 0)
    return dict(mu_s=np.stack(mu_s), tu_s=np.stack(tu_s), tv_s=np.stack(tv_s), n_s=np.stack(n_s),
                M=M.astype(F32), valid=valid)


def normal_sign(n_s, mu_s):
    """-1 where the sensor-frame normal points away from the sensor (n . mu_s > 0), else +1."""
    d = (n_s[0] * mu_s[0] + n_s[1] * mu_s[1]) + n_s[2] * mu_s[2]
    return np.where(d > 0, F32(-1.0), F32(1.0)).astype(F32)


# ----------------------------------------------------------------------------
# pinhole binning
# ----------------------------------------------------------------------------

def pinhole_bins(fr: dict, sensor: dict, opts: dict):
    """Visibility, pixel rectangle, tile rectangle and depth key for a pinhole camera.

    Support of a surfel (its ray set) is the union of the ellipse u^2+v^2 <= k
    (k = cutoff^2) and the low-pass disc |p - c|^2 * lp <= k around the
    projected centre c.  The ellipse's screen box comes from the dual conic of
    the circle diag(k,k,-1) mapped by T = diag(fx,fy,1) M (principal-point
    centred pixels): with d = T3 D T3^T, f_i = T_i D T3^T, g_i = T_i D T_i^T,
    centre_i = f_i / d and half-extent_i = sqrt(f_i^2 - d g_i) / (-d).
    A surfel is visible iff mu_z >= z_near and d < 0 (its disc of radius
    sqrt(k) lies wholly in front of the camera) and every bound is finite
    (tested explicitly, so that no min/max ever sees a NaN).
    """
    M = _f(fr["M"])
    mu = _f(fr["mu_s"])
    W, H = int(sensor["width"]), int(sensor["height"])
    fx, fy = F32(sensor["fx"]), F32(sensor["fy"])
    cx, cy = F32(sensor["cx"]), F32(sensor["cy"])
    z_near = F32(sensor["z_near"])
    k = F32(opts["cutoff2"])
    lp = F32(opts["lp_inv_sigma2"])
    use_lp = bool(opts["lowpass"])
    tw, th = int(opts["tile_w"]), int(opts["tile_h"])
    with np.errstate(all="ignore"):
        T1 = [fx * M[0, j] for j in range(3)]
        T2 = [fy * M[1, j] for j in range(3)]
        T3 = [M[2, j] for j in range(3)]
        d = k * (T3[0] * T3[0] + T3[1] * T3[1]) - T3[2] * T3[2]
        f1 = k * (T1[0] * T3[0] + T1[1] * T3[1]) - T1[2] * T3[2]
        g1 = k * (T1[0] * T1[0] + T1[1] * T1[1]) - T1[2] * T1[2]
        f2 = k * (T2[0] * T3[0] + T2[1] * T3[1]) - T2[2] * T3[2]
        g2 = k * (T2[0] * T2[0] + T2[1] * T2[1]) - T2[2] * T2[2]
        xc = f1 / d
        yc = f2 / d
        nd = -d
        disc_x = f1 * f1 - d * g1
        disc_y = f2 * f2 - d * g2
        ok = np.isfinite(disc_x) & np.isfinite(disc_y)
        hx = np.sqrt(np.maximum(np.where(ok, disc_x, F32(0.0)), F32(0.0))) / nd
        hy = np.sqrt(np.maximum(np.where(ok, disc_y, F32(0.0)), F32(0.0))) / nd
        xlo, xhi = xc - hx, xc + hx
        ylo, yhi = yc - hy, yc + hy
        ok &= np.isfinite(xlo) & np.isfinite(xhi) & np.isfinite(ylo) & np.isfinite(yhi)
        if use_lp:
            rl = np.sqrt(k / lp)
            pcx = (fx * mu[0]) / mu[2]
            pcy = (fy * mu[1]) / mu[2]
            ok &= np.isfinite(pcx - rl) & np.isfinite(pcx + rl) & np.isfinite(pcy - rl) & np.isfinite(pcy + rl)
            # both operands are finite wherever ok holds
            xlo = np.where(ok, np.minimum(xlo, pcx - rl), F32(0.0))
            xhi = np.where(ok, np.maximum(xhi, pcx + rl), F32(0.0))
            ylo = np.where(ok, np.minimum(ylo, pcy - rl), F32(0.0))
            yhi = np.where(ok, np.maximum(yhi, pcy + rl), F32(0.0))
        one = F32(1.0)
        half = F32(0.5)
        X_lo = ((xlo - one) + cx) - half
        X_hi = ((xhi + one) + cx) - half
        Y_lo = ((ylo - one) + cy) - half
        Y_hi = ((yhi + one) + cy) - half
        ok &= np.isfinite(X_lo) & np.isfinite(X_hi) & np.isfinite(Y_lo) & np.isfinite(Y_hi)
    vis = fr["valid"] & (mu[2] >= z_near) & (d < 0) & ok
    # clamp in float before converting (both bounds are finite after this)
    X_lo = np.minimum(np.maximum(X_lo, F32(-2.0)), F32(W + 2))
    X_hi = np.minimum(np.maximum(X_hi, F32(-2.0)), F32(W + 2))
    Y_lo = np.minimum(np.maximum(Y_lo, F32(-2.0)), F32(H + 2))
    Y_hi = np.minimum(np.maximum(Y_hi, F32(-2.0)), F32(H + 2))
    i_lo = np.maximum(np.ceil(X_lo).astype(np.int64), 0)
    i_hi = np.minimum(np.floor(X_hi).astype(np.int64), W - 1)
    j_lo = np.maximum(np.ceil(Y_lo).astype(np.int64), 0)
    j_hi = np.minimum(np.floor(Y_hi).astype(np.int64), H - 1)
    touch = vis & (i_lo <= i_hi) & (j_lo <= j_hi)
    n_tx = (W + tw - 1) // tw
    tx_lo, tx_hi = i_lo // tw, i_hi // tw
    ty_lo, ty_hi = j_lo // th, j_hi // th
    n_tiles = np.where(touch, (tx_hi - tx_lo + 1) * (ty_hi - ty_lo + 1), 0)
    key = np.where(vis, mu[2], F32(0.0)).astype(F32)
    return dict(visible=vis, touch=touch, i_lo=i_lo, i_hi=i_hi, j_lo=j_lo, j_hi=j_hi,
                tx_lo=tx_lo, tx_hi=tx_hi, ty_lo=ty_lo, ty_hi=ty_hi, n_tx=n_tx,
                n_ty=(H + th - 1) // th, n_tiles=n_tiles, key=key,
                key_bits=key.view(np.uint32).astype(np.int64), wrap=np.zeros_like(vis))


# ----------------------------------------------------------------------------
# LiDAR binning
# ----------------------------------------------------------------------------

def atan2_spec(y, x):
    """Four-quadrant arctangent from the A&S 4.4.49 polynomial (FP32 spec ops)."""
    y, x = _f(y), _f(x)
    ax, ay = np.abs(x), np.abs(y)
    mn, mx = np.minimum(ax, ay), np.maximum(ax, ay)
    with np.errstate(all="ignore"):
        t = np.where(mx > 0, mn / np.where(mx > 0, mx, F32(1.0)), F32(0.0)).astype(F32)
        s = t * t
        c1, c3, c5, c7, c9 = ATAN_C
        p = ((((c9 * s + c7) * s + c5) * s + c3) * s + c1) * t
    a = np.where(ay > ax, HALF_PI_F - p, p).astype(F32)
    a = np.where(x < 0, PI_F - a, a).astype(F32)
    a = np.where(y < 0, -a, a).astype(F32)
    return a


def asin_spec(s):
    """arcsin on [0,1] as atan2_spec(s, sqrt(1 - s*s))."""
    s = _f(s)
    return atan2_spec(s, np.sqrt(np.maximum(F32(1.0) - s * s, F32(0.0))))


def lidar_tables(sensor: dict):
    """The LiDAR sensor definition as FP32 tables (FP64 libm, rounded to nearest).

    Column i has azimuth az_i = 2*pi*i/n_az; beam j has elevation el_j (input,
    FP64 radians, ascending).  Both sides use these rounded values as the
    definition of the rays.
    """
    n_az = int(sensor["width"])
    el = np.asarray(sensor["elevations"], np.float64)
    az = [((2.0 * math.pi) * float(i)) / n_az for i in range(n_az)]
    # libm (math) rather than numpy's vectorised kernels: correctly rounded FP64
    cosf = lambda v: np.array([math.cos(t) for t in v], np.float64).astype(F32)
    sinf = lambda v: np.array([math.sin(t) for t in v], np.float64).astype(F32)
    return dict(cos_az=cosf(az), sin_az=sinf(az), cos_el=cosf(el), sin_el=sinf(el),
                el=el.astype(F32), inv_step=F32(n_az / (2.0 * math.pi)),
                step=F32(2.0 * math.pi / n_az))


def lidar_bins(fr: dict, scale, sensor: dict, opts: dict):
    """Visibility, beam/column rectangle, tile rectangle and range key for a spinning LiDAR.

    The support lies inside the sphere of radius R = sqrt(k) * max(s_u, s_v)
    around mu_s, and the low-pass cone (chord |d - mu_hat| <= c_lp =
    sqrt(k/lp) * step) lies inside the cone of a sphere of radius r * c_lp, so
    both lie inside the cone of the sphere of radius R_eff = R + r * c_lp.
    Its elevation half-angle is asin(R_eff / r) and its azimuth half-angle
    asin(R_eff / rho_xy) (all azimuths when rho_xy <= R_eff).  Ranges are
    padded by one beam and one column; columns wrap modulo n_az.
    Visible iff r^2 > (R + z_near)^2.  Key = |mu_s|^2 (monotone in range).
    """
    mu = _f(fr["mu_s"])
    scale = _f(scale)
    n_az, n_b = int(sensor["width"]), int(sensor["height"])
    tabs = lidar_tables(sensor)
    z_near = F32(sensor["z_near"])
    k = F32(opts["cutoff2"])
    lp = F32(opts["lp_inv_sigma2"])
    use_lp = bool(opts["lowpass"])
    tw, th = int(opts["tile_w"]), int(opts["tile_h"])
    with np.errstate(all="ignore"):
        rxy2 = mu[0] * mu[0] + mu[1] * mu[1]
        r2 = rxy2 + mu[2] * mu[2]
        rxy = np.sqrt(rxy2)
        r = np.sqrt(r2)
        R = np.sqrt(k) * np.maximum(scale[0], scale[1])
        Rn = R + z_near
        vis = fr["valid"] & (r2 > Rn * Rn)
        if use_lp:
            c_lp = np.sqrt(k / lp) * tabs["step"]
            Reff = R + r * c_lp
        else:
            Reff = R
        vis &= np.isfinite(r2) & np.isfinite(Reff)
        el_c = atan2_spec(mu[2], rxy)
        az_c = atan2_spec(mu[1], mu[0])
        sb = np.minimum(Reff / r, F32(1.0))
        beta = asin_spec(np.where(vis, sb, F32(0.0)).astype(F32))
        el_lo = el_c - beta
        el_hi = el_c + beta
        full_az = ~(rxy > Reff)
        sa = np.where(full_az | ~vis, F32(0.0), Reff / rxy).astype(F32)
        daz = asin_spec(sa)
        az_lo = (az_c - daz) * tabs["inv_step"]
        az_hi = (az_c + daz) * tabs["inv_step"]
    el_tab = tabs["el"]
    # first beam with el >= el_lo, last beam with el <= el_hi, then one beam of padding
    j_lo = np.searchsorted(el_tab, np.where(vis, el_lo, 0), side="left").astype(np.int64) - 1
    j_hi = np.searchsorted(el_tab, np.where(vis, el_hi, 0), side="right").astype(np.int64) - 1 + 1
    j_lo = np.maximum(j_lo, 0)
    j_hi = np.minimum(j_hi, n_b - 1)
    az_lo = np.where(vis & ~full_az, az_lo, F32(0.0)).astype(F32)
    az_hi = np.where(vis & ~full_az, az_hi, F32(0.0)).astype(F32)
    i_lo = np.floor(az_lo).astype(np.int64) - 1
    i_hi = np.ceil(az_hi).astype(np.int64) + 1
    full = full_az | (i_hi - i_lo + 1 >= n_az)
    i_lo = np.where(full, 0, i_lo)
    i_hi = np.where(full, n_az - 1, i_hi)
    c_lo = np.mod(i_lo, n_az)
    c_hi = np.mod(i_hi, n_az)
    n_tx = (n_az + tw - 1) // tw
    n_ty = (n_b + th - 1) // th
    tx_lo, tx_hi = c_lo // tw, c_hi // tw
    wrap = c_lo > c_hi
    # a wrapped column range whose two tile runs meet covers every column tile
    all_tx = wrap & (tx_hi >= tx_lo)
    wrap = wrap & ~all_tx
    tx_lo = np.where(all_tx, 0, tx_lo)
    tx_hi = np.where(all_tx, n_tx - 1, tx_hi)
    ncols = np.where(wrap, (n_tx - tx_lo) + (tx_hi + 1), tx_hi - tx_lo + 1)
    ty_lo, ty_hi = j_lo // th, j_hi // th
    touch = vis & (j_lo <= j_hi)
    n_tiles = np.where(touch, ncols * (ty_hi - ty_lo + 1), 0)
    key = np.where(vis, r2, F32(0.0)).astype(F32)
    return dict(visible=vis, touch=touch, i_lo=c_lo, i_hi=c_hi, j_lo=j_lo, j_hi=j_hi,
                tx_lo=tx_lo, tx_hi=tx_hi, ty_lo=ty_lo, ty_hi=ty_hi, n_tx=n_tx, n_ty=n_ty,
                n_tiles=n_tiles, key=key, key_bits=key.view(np.uint32).astype(np.int64),
                wrap=wrap, full_cols=full | all_tx)


# ----------------------------------------------------------------------------
# cylindrical (fisheye) camera binning
# ----------------------------------------------------------------------------

def cylindrical_tables(sensor: dict):
    """The cylindrical camera's ray definition (FP64).

    Column i looks at the horizontal angle phi_i = (i + 1/2 - c_x) / f_x about
    the camera's y axis (Eq. 4), row j at height y_n = (j + 1/2 - c_y) / f_y on
    the unit cylinder: the ray direction is (sin phi, y_n, cos phi).  These are
    exact functions of the pixel centre (no table rounding), like the pinhole's
    normalised coordinates.
    """
    W, H = int(sensor["width"]), int(sensor["height"])
    fx, fy = float(sensor["fx"]), float(sensor["fy"])
    cx, cy = float(sensor["cx"]), float(sensor["cy"])
    phi = (np.arange(W, dtype=np.float64) + 0.5 - cx) / fx
    yn = (np.arange(H, dtype=np.float64) + 0.5 - cy) / fy
    return dict(sin_phi=np.sin(phi), cos_phi=np.cos(phi), yn=yn, phi=phi)


def cylindrical_bins(fr: dict, scale, sensor: dict, opts: dict):
    """Visibility, pixel rectangle, tile rectangle and depth key for a cylindrical camera.

    Pixel (x, y) = (c_x + f_x phi, c_y + f_y y_n) for the ray of direction
    (sin phi, y_n, cos phi).  The support lies inside the ball of radius
    R = sqrt(k) max(s_u, s_v) around mu: its rays have |phi - phi_c| <=
    asin(R / r) with r = sqrt(mu_x^2 + mu_z^2) (the ball's shadow on the
    horizontal plane), and y_n = y / r' over the box y in [mu_y - R, mu_y + R],
    r' in [r - R, r + R].  The low-pass disc has radius sqrt(k / lp) pixels
    around the projected centre (c_x + f_x phi_c, c_y + f_y mu_y / r).  Angles
    come from the A&S arctangent (error <= 1e-5 rad, inside the one-pixel pad).
    Visible iff r^2 > (R + z_near)^2 (the ball is wholly outside the near
    cylinder).  A range that crosses the back of the camera (phi = +-pi) takes
    every column.  Key = r^2 (monotone in the cylindrical depth).
    """
    mu = _f(fr["mu_s"])
    scale = _f(scale)
    W, H = int(sensor["width"]), int(sensor["height"])
    fx, fy = F32(sensor["fx"]), F32(sensor["fy"])
    cx, cy = F32(sensor["cx"]), F32(sensor["cy"])
    z_near = F32(sensor["z_near"])
    k = F32(opts["cutoff2"])
    lp = F32(opts["lp_inv_sigma2"])
    use_lp = bool(opts["lowpass"])
    tw, th = int(opts["tile_w"]), int(opts["tile_h"])
    with np.errstate(all="ignore"):
        r2 = mu[0] * mu[0] + mu[2] * mu[2]
        r = np.sqrt(r2)
        R = np.sqrt(k) * np.maximum(scale[0], scale[1])
        Rn = R + z_near
        vis = fr["valid"] & (r2 > Rn * Rn) & np.isfinite(r2) & np.isfinite(R) & np.isfinite(mu[1])
        phi_c = atan2_spec(mu[0], mu[2])
        q = np.where(vis, R / r, F32(0.0)).astype(F32)
        dphi = asin_spec(np.minimum(q, F32(1.0)))
        y_lo, y_hi = mu[1] - R, mu[1] + R
        r_lo, r_hi = r - R, r + R
        yn_lo = np.minimum(y_lo / r_lo, y_lo / r_hi)
        yn_hi = np.maximum(y_hi / r_lo, y_hi / r_hi)
        a_lo, a_hi = phi_c - dphi, phi_c + dphi
        back = (a_lo < -PI_F) | (a_hi > PI_F)
        xlo, xhi = fx * a_lo, fx * a_hi
        ylo, yhi = fy * yn_lo, fy * yn_hi
        if use_lp:
            rl = np.sqrt(k / lp)
            pcx = fx * phi_c
            pcy = fy * (mu[1] / r)
            xlo = np.minimum(xlo, pcx - rl)
            xhi = np.maximum(xhi, pcx + rl)
            ylo = np.minimum(ylo, pcy - rl)
            yhi = np.maximum(yhi, pcy + rl)
        one = F32(1.0)
        half = F32(0.5)
        X_lo = ((xlo - one) + cx) - half
        X_hi = ((xhi + one) + cx) - half
        Y_lo = ((ylo - one) + cy) - half
        Y_hi = ((yhi + one) + cy) - half
        vis &= np.isfinite(X_lo) & np.isfinite(X_hi) & np.isfinite(Y_lo) & np.isfinite(Y_hi)
    X_lo = np.where(vis, X_lo, F32(0.0))
    X_hi = np.where(vis, X_hi, F32(0.0))
    Y_lo = np.where(vis, Y_lo, F32(0.0))
    Y_hi = np.where(vis, Y_hi, F32(0.0))
    X_lo = np.where(back, F32(-2.0), np.minimum(np.maximum(X_lo, F32(-2.0)), F32(W + 2)))
    X_hi = np.where(back, F32(W + 2), np.minimum(np.maximum(X_hi, F32(-2.0)), F32(W + 2)))
    Y_lo = np.minimum(np.maximum(Y_lo, F32(-2.0)), F32(H + 2))
    Y_hi = np.minimum(np.maximum(Y_hi, F32(-2.0)), F32(H + 2))
    i_lo = np.maximum(np.ceil(X_lo).astype(np.int64), 0)
    i_hi = np.minimum(np.floor(X_hi).astype(np.int64), W - 1)
    j_lo = np.maximum(np.ceil(Y_lo).astype(np.int64), 0)
    j_hi = np.minimum(np.floor(Y_hi).astype(np.int64), H - 1)
    touch = vis & (i_lo <= i_hi) & (j_lo <= j_hi)
    n_tx = (W + tw - 1) // tw
    tx_lo, tx_hi = i_lo // tw, i_hi // tw
    ty_lo, ty_hi = j_lo // th, j_hi // th
    n_tiles = np.where(touch, (tx_hi - tx_lo + 1) * (ty_hi - ty_lo + 1), 0)
    key = np.where(vis, r2, F32(0.0)).astype(F32)
    return dict(visible=vis, touch=touch, i_lo=i_lo, i_hi=i_hi, j_lo=j_lo, j_hi=j_hi,
                tx_lo=tx_lo, tx_hi=tx_hi, ty_lo=ty_lo, ty_hi=ty_hi, n_tx=n_tx,
                n_ty=(H + th - 1) // th, n_tiles=n_tiles, key=key,
                key_bits=key.view(np.uint32).astype(np.int64), wrap=np.zeros_like(vis))


def tile_pairs(bins: dict):
    """(tile id, splat index) pairs of every touched tile, in the FP32 spec's order.

    Returns (tile_ids, splat_ids) sorted by (tile, key bits, splat index): the
    reference order of the renderer's depth sort.
    """
    n_tx = bins["n_tx"]
    tiles, sids = [], []
    idx = np.nonzero(bins["touch"])[0]
    for i in idx:
        tx_lo, tx_hi = int(bins["tx_lo"][i]), int(bins["tx_hi"][i])
        if bins["wrap"][i]:
            cols = list(range(tx_lo, n_tx)) + list(range(0, tx_hi + 1))
        else:
            cols = list(range(tx_lo, tx_hi + 1))
        for ty in range(int(bins["ty_lo"][i]), int(bins["ty_hi"][i]) + 1):
            for tx in cols:
                tiles.append(ty * n_tx + tx)
                sids.append(i)
    tiles = np.asarray(tiles, np.int64)
    sids = np.asarray(sids, np.int64)
    order = np.lexsort((sids, bins["key_bits"][sids], tiles))
    return tiles[order], sids[order]


def tile_pairs_fast(bins: dict):
    """Vectorised version of tile_pairs for large scenes (same output)."""
    n_tx = int(bins["n_tx"])
    idx = np.nonzero(bins["touch"])[0]
    if idx.size == 0:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    wrap = bins["wrap"][idx]
    tx_lo = bins["tx_lo"][idx]
    tx_hi = bins["tx_hi"][idx]
    ncols = np.where(wrap, (n_tx - tx_lo) + (tx_hi + 1), tx_hi - tx_lo + 1)
    nrows = bins["ty_hi"][idx] - bins["ty_lo"][idx] + 1
    cnt = ncols * nrows
    sid = np.repeat(idx, cnt)
    start = np.repeat(np.cumsum(cnt) - cnt, cnt)
    local = np.arange(cnt.sum()) - start
    nc = np.repeat(ncols, cnt)
    row = local // nc
    col = local % nc
    tx = (np.repeat(tx_lo, cnt) + col) % n_tx
    ty = np.repeat(bins["ty_lo"][idx], cnt) + row
    tiles = ty * n_tx + tx
    order = np.lexsort((sid, bins["key_bits"][sid], tiles))
    return tiles[order].astype(np.int64), sid[order].astype(np.int64)
