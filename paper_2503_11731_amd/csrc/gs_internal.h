// Internal structures and device helpers of the gs2d HIP library (gfx950).
//
// Geometry (Sec. III-A, Eq. 1-5): a surfel is the sensor-frame map
// M = [s_u R t_u, s_v R t_v, R mu + t]; the ray of a pixel is the meet of
// two planes and hits the surfel at (u,v,1) ~ adj(M) d (the two-plane solve
// of Eq. 2 written through the adjugate: (M^T h_u) x (M^T h_v) =
// adj(M) (h_u x h_v), and h_u x h_v is the ray direction d).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gs2d.h"

namespace gs {

constexpr int kMaxGroups = GS_MAX_GROUPS;
constexpr int kRecF32 = 16;     // floats per surfel record
constexpr int kRec64 = 4;       // doubles per surfel record (camera: pc; LiDAR: unit centre)
constexpr int kGrz = 10;        // doubles per record with FP64 re-solve data
constexpr int kGradFields = 16; // per-surfel gradient accumulators
// keys per radix-sort block (256 threads x 32): on MI355X faster than 4096,
// with per-digit output runs twice as long and half the look-back chain
constexpr int kRadixItems = 8192;
// keys per radix sort (pairs, records): the look-back counts are 30-bit
constexpr uint32_t kMaxSortKeys = (1u << 30) - 1u;
constexpr uint32_t kInvalidKey = 0xFFFFFFFFu;
constexpr uint32_t kNoPair = 0xFFFFFFFFu;  // a ray whose transmittance never falls below 1/2

// record flags (stored as integer bits in float slot 14)
//  grazing: h'_2 may fall below 1/8 in the rectangle; pairs with |h'_2| < 1/8
//    are solved in FP64.
//  edge: the surfel is seen nearly edge-on, so its 2 x 2 solve is
//    ill-conditioned: the FP32 (u, v) may be off by enough to move alpha by
//    more than kEdgeTau.  The record carries FP64 re-solve data; per tile the
//    staged copy keeps the bit only where the tile's own bound still allows
//    that, and then each pair re-solves in FP64 where its alpha error could.
//  wild (staged copies only): the tile's (u, v) error bound exceeds
//    kWildErr, too large to trust the FP32 rho at all: every pair that could
//    be inside the support with that error re-solves in FP64.
constexpr uint32_t kFlagGrazing = 1u;
constexpr uint32_t kFlagEdge = 2u;
constexpr uint32_t kFlagWild = 4u;
constexpr uint32_t kFlagF64 = kFlagGrazing | kFlagEdge;  // records that carry FP64 re-solve data
// Error budget of one pair's FP32 solve: the first-order bound of its alpha
// error must stay below kEdgeTau, a tenth of the 1e-4 output bar.
constexpr float kEdgeTau = 1e-5f;
constexpr float kWildErr = 0.05f;
// The FP32 (u, v) error of a pair is bounded, to first order, by
// err = (2^-23 kappa s + 2^-20) / |h'_2|: kappa the largest absolute row sum
// of the solve's (u, v) rows plus 3.4 times that of its h'_2 row, s = 2
// |offset from the centre|_inf (the offset's own rounding and the products';
// the centre itself is held to twice FP32 precision in the tile frame).  A
// record is edge-flagged when its bound E over the pixels of the tiles its
// rectangle touches allows an alpha error above the budget (|(u, v)|_1 <= 4.7
// inside the cutoff, alpha <= 0.61 o there).
__device__ inline uint32_t conditioning_flags(double E, float o) {
  return 2.87 * (double)o * E > (double)kEdgeTau ? kFlagEdge : 0u;
}

struct GroupsK {
  int n;                     // groups in the scene
  int pose_base;             // first row of this scene in the group-pose array
  int off[kMaxGroups + 1];   // surfel (or anchor) offsets
};

struct OptsK {
  float alpha_min, alpha_max, T_min, cutoff2, lp;
  float rl;                  // sqrt(cutoff2 / lp): low-pass disc radius (pixels)
  int lowpass;
  float bg0, bg1, bg2;
};

struct SensorK {
  int kind;
  int W, H, tw, th, n_tx, n_ty;
  int tile_offset;           // first global tile id of this sensor
  float fx, fy, cx, cy, z_near;
  // LiDAR only
  float inv_step, step;      // azimuth steps per radian and its inverse (FP32 spec)
  float c_lp;                // sqrt(cutoff2 / lp) * step: low-pass chord radius
  float lp_ang;              // lp / step^2 (FP32) for the per-ray low-pass
  // LiDAR: FP32 tables, one array: elevations [H], cos and sin of elevation
  // [H] each, cos and sin of azimuth [W] each
  const float* tab;
};

// Per-sensor workspace pointers.
struct SensorWS {
  float* pose;       // [G][12] composed sensor<-group poses (FP32 spec)
  float4* rec;       // [N][4]
  double* rec64;     // [N][4]
  double* grz;       // [N][kGrz]
  int4* rect;        // [N] tile rectangle (tx_lo, tx_hi, ty_lo, ty_hi | wrap<<30)
  uint32_t* ntiles;  // [N]
  uint32_t* key[2];  // [N]
  uint32_t* val[2];  // [N]
  uint32_t* offs;    // [N+1]
  uint32_t* bsum;    // scan block sums
  uint32_t* hist;    // radix digit counts
  uint32_t* ptile[2];
  uint32_t* pval[2];
  uint2* ranges;     // [n_tiles]
  float* T_final;    // [H*W]
  uint32_t* n_last;  // [H*W]
  uint32_t* mpair;   // [H*W] pair index of the median crossing (kNoPair: none)
  uint32_t* status;  // [16]
  float* gacc;       // [kGradFields][N]
  uint32_t* visible; // [N]
};

// status word indices
enum {
  kStPairs = 0,
  kStOverflow = 1,
  kStVisible = 2,
  kStFp64 = 3,
  kStEvals = 4 /* u64 */,
  kStContrib = 6 /* u64 */,
  kStSortStall = 8 /* a sort or scan look-back wait gave up */
};
// The compositing kernel adds its pair counts to one of 8 replicas (one per
// XCD) of the four counters, words kStRep + 8 x: [0..1] evaluated (u64),
// [2..3] composited (u64), [4] FP64 re-solves, [6..7] wave pair-loop
// iterations (u64); the host sums them.  Atomics of every workgroup on the
// same words serialise across the device.
constexpr int kStRep = 16;
constexpr int kStWords = kStRep + 8 * 8;

__device__ inline int group_of(const GroupsK& g, int i) {
  int lo = 0, hi = g.n - 1;
  while (lo < hi) {  // last group whose start <= i
    int mid = (lo + hi + 1) >> 1;
    if (g.off[mid] <= i) lo = mid; else hi = mid - 1;
  }
  return lo;
}

__device__ __host__ inline bool finite_f(float x) { return __builtin_isfinite(x); }

// --------------------------------------------------------------------------
// FP32 binning specification.  Every operation below is an IEEE-754 binary32
// operation with no contraction and a fixed association order, so that the
// visibility, tile rectangle and depth key decisions are reproducible bit for
// bit by an independent implementation of the same specification.
// --------------------------------------------------------------------------

struct Frame32 {
  float mu[3], tu[3], tv[3], n[3];
  float M[3][3];
  bool valid;
};

__device__ inline void spec_frame(const float* P, float m0, float m1, float m2, float qw, float qx, float qy,
                                  float qz, float su, float sv, Frame32& f) {
#pragma clang fp contract(off)
  for (int i = 0; i < 3; ++i) f.mu[i] = ((P[4 * i] * m0 + P[4 * i + 1] * m1) + P[4 * i + 2] * m2) + P[4 * i + 3];
  float nq2 = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
  float s = 2.0f / nq2;
  float xx = qx * qx, yy = qy * qy, zz = qz * qz;
  float xy = qx * qy, xz = qx * qz, yz = qy * qz;
  float wx = qw * qx, wy = qw * qy, wz = qw * qz;
  float a[3] = {1.0f - s * (yy + zz), s * (xy + wz), s * (xz - wy)};
  float b[3] = {s * (xy - wz), 1.0f - s * (xx + zz), s * (yz + wx)};
  float c[3] = {s * (xz + wy), s * (yz - wx), 1.0f - s * (xx + yy)};
  bool fin = true;
  for (int i = 0; i < 3; ++i) {
    f.tu[i] = (P[4 * i] * a[0] + P[4 * i + 1] * a[1]) + P[4 * i + 2] * a[2];
    f.tv[i] = (P[4 * i] * b[0] + P[4 * i + 1] * b[1]) + P[4 * i + 2] * b[2];
    f.n[i] = (P[4 * i] * c[0] + P[4 * i + 1] * c[1]) + P[4 * i + 2] * c[2];
    f.M[i][0] = su * f.tu[i];
    f.M[i][1] = sv * f.tv[i];
    f.M[i][2] = f.mu[i];
    fin = fin && finite_f(f.M[i][0]) && finite_f(f.M[i][1]) && finite_f(f.M[i][2]) && finite_f(f.n[i]);
  }
  f.valid = fin && (nq2 > 0.0f) && (su > 0.0f) && (sv > 0.0f);
}

__device__ inline float spec_normal_sign(const Frame32& f) {
#pragma clang fp contract(off)
  float d = (f.n[0] * f.mu[0] + f.n[1] * f.mu[1]) + f.n[2] * f.mu[2];
  return d > 0.0f ? -1.0f : 1.0f;
}

struct Bins {
  bool vis, touch, wrap, full_cols;
  float el_c, az_c, beta;          // LiDAR: centre direction and elevation half-angle
  int tx_lo, tx_hi, ty_lo, ty_hi;  // tile rectangle
  int i_lo, i_hi, j_lo, j_hi;      // pixel/beam rectangle (columns wrap for LiDAR)
  uint32_t n_tiles;
  float key;
};

__device__ inline float fclamp_spec(float x, float lo, float hi) {
  // operands finite: plain IEEE min/max
  float y = x < lo ? lo : x;
  return y > hi ? hi : y;
}

__device__ inline void spec_pinhole_bins(const Frame32& f, const SensorK& S, const OptsK& O, Bins& b) {
#pragma clang fp contract(off)
  const float k = O.cutoff2;
  float T1[3], T2[3], T3[3];
  for (int j = 0; j < 3; ++j) {
    T1[j] = S.fx * f.M[0][j];
    T2[j] = S.fy * f.M[1][j];
    T3[j] = f.M[2][j];
  }
  float d = k * (T3[0] * T3[0] + T3[1] * T3[1]) - T3[2] * T3[2];
  float f1 = k * (T1[0] * T3[0] + T1[1] * T3[1]) - T1[2] * T3[2];
  float g1 = k * (T1[0] * T1[0] + T1[1] * T1[1]) - T1[2] * T1[2];
  float f2 = k * (T2[0] * T3[0] + T2[1] * T3[1]) - T2[2] * T3[2];
  float g2 = k * (T2[0] * T2[0] + T2[1] * T2[1]) - T2[2] * T2[2];
  float xc = f1 / d, yc = f2 / d, nd = -d;
  float disc_x = f1 * f1 - d * g1;
  float disc_y = f2 * f2 - d * g2;
  bool ok = finite_f(disc_x) && finite_f(disc_y);
  float dx0 = ok ? disc_x : 0.0f, dy0 = ok ? disc_y : 0.0f;
  float hx = sqrtf(dx0 > 0.0f ? dx0 : 0.0f) / nd;
  float hy = sqrtf(dy0 > 0.0f ? dy0 : 0.0f) / nd;
  float xlo = xc - hx, xhi = xc + hx, ylo = yc - hy, yhi = yc + hy;
  ok = ok && finite_f(xlo) && finite_f(xhi) && finite_f(ylo) && finite_f(yhi);
  if (O.lowpass) {
    float rl = O.rl;
    float pcx = (S.fx * f.mu[0]) / f.mu[2];
    float pcy = (S.fy * f.mu[1]) / f.mu[2];
    ok = ok && finite_f(pcx - rl) && finite_f(pcx + rl) && finite_f(pcy - rl) && finite_f(pcy + rl);
    if (ok) {
      float a = pcx - rl, c = pcx + rl, e = pcy - rl, g = pcy + rl;
      xlo = a < xlo ? a : xlo;
      xhi = c > xhi ? c : xhi;
      ylo = e < ylo ? e : ylo;
      yhi = g > yhi ? g : yhi;
    } else {
      xlo = xhi = ylo = yhi = 0.0f;
    }
  }
  float X_lo = ((xlo - 1.0f) + S.cx) - 0.5f;
  float X_hi = ((xhi + 1.0f) + S.cx) - 0.5f;
  float Y_lo = ((ylo - 1.0f) + S.cy) - 0.5f;
  float Y_hi = ((yhi + 1.0f) + S.cy) - 0.5f;
  ok = ok && finite_f(X_lo) && finite_f(X_hi) && finite_f(Y_lo) && finite_f(Y_hi);
  b.vis = f.valid && (f.mu[2] >= S.z_near) && (d < 0.0f) && ok;
  b.wrap = false;
  b.full_cols = false;
  b.el_c = b.az_c = b.beta = 0.0f;
  if (!b.vis) {
    b.touch = false;
    b.n_tiles = 0;
    b.key = 0.0f;
    b.tx_lo = b.tx_hi = b.ty_lo = b.ty_hi = b.i_lo = b.i_hi = b.j_lo = b.j_hi = 0;
    return;
  }
  X_lo = fclamp_spec(X_lo, -2.0f, (float)(S.W + 2));
  X_hi = fclamp_spec(X_hi, -2.0f, (float)(S.W + 2));
  Y_lo = fclamp_spec(Y_lo, -2.0f, (float)(S.H + 2));
  Y_hi = fclamp_spec(Y_hi, -2.0f, (float)(S.H + 2));
  int i_lo = max((int)ceilf(X_lo), 0);
  int i_hi = min((int)floorf(X_hi), S.W - 1);
  int j_lo = max((int)ceilf(Y_lo), 0);
  int j_hi = min((int)floorf(Y_hi), S.H - 1);
  b.i_lo = i_lo; b.i_hi = i_hi; b.j_lo = j_lo; b.j_hi = j_hi;
  b.touch = (i_lo <= i_hi) && (j_lo <= j_hi);
  b.tx_lo = i_lo / S.tw; b.tx_hi = i_hi / S.tw;
  b.ty_lo = j_lo / S.th; b.ty_hi = j_hi / S.th;
  b.n_tiles = b.touch ? (uint32_t)((b.tx_hi - b.tx_lo + 1) * (b.ty_hi - b.ty_lo + 1)) : 0u;
  b.key = f.mu[2];
}

// Four-quadrant arctangent from the odd degree-9 polynomial of Abramowitz &
// Stegun 4.4.49 (|error| <= 1e-5 rad on [0,1]), binary32 ops only.  It only
// places LiDAR angular ranges, which are padded by whole angular steps.
__device__ inline float spec_atan2(float y, float x) {
#pragma clang fp contract(off)
  const float c1 = (float)0.9998660, c3 = (float)-0.3302995, c5 = (float)0.1801410;
  const float c7 = (float)-0.0851330, c9 = (float)0.0208351;
  const float kPi = (float)3.141592653589793, kHalfPi = (float)1.5707963267948966;
  float ax = fabsf(x), ay = fabsf(y);
  float mn = ax < ay ? ax : ay;
  float mx = ax < ay ? ay : ax;
  float t = mx > 0.0f ? mn / mx : 0.0f;
  float s = t * t;
  float p = ((((c9 * s + c7) * s + c5) * s + c3) * s + c1) * t;
  float a = ay > ax ? kHalfPi - p : p;
  a = x < 0.0f ? kPi - a : a;
  return y < 0.0f ? -a : a;
}

__device__ inline float spec_asin(float s) {
#pragma clang fp contract(off)
  float c = 1.0f - s * s;
  return spec_atan2(s, sqrtf(c > 0.0f ? c : 0.0f));
}

__device__ inline int imod(int a, int n) {
  int r = a % n;
  return r < 0 ? r + n : r;
}

// first index j with el[j] >= x (n if none)
__device__ inline int lower_bound_f(const float* el, int n, float x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (el[mid] < x) lo = mid + 1; else hi = mid;
  }
  return lo;
}
// number of entries with el[j] <= x
__device__ inline int upper_bound_f(const float* el, int n, float x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    int mid = (lo + hi) >> 1;
    if (el[mid] <= x) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// Cylindrical camera (Eq. 4): pixel (c_x + f_x phi, c_y + f_y y_n) for the
// ray (sin phi, y_n, cos phi).  The support lies in the ball of radius
// R = sqrt(k) max(s_u, s_v) around mu: |phi - phi_c| <= asin(R / r),
// r = sqrt(mu_x^2 + mu_z^2), and y_n = y / r' over y in [mu_y - R, mu_y + R],
// r' in [r - R, r + R]; united with the low-pass disc around the projected
// centre (c_x + f_x phi_c, c_y + f_y mu_y / r) and padded by one pixel.  A
// range across the back of the camera (phi = +-pi) takes every column.
// Visible iff r^2 > (R + z_near)^2; key = r^2.
__device__ inline void spec_cyl_bins(const Frame32& f, float su, float sv, const SensorK& S, const OptsK& O,
                                     Bins& b) {
#pragma clang fp contract(off)
  const float k = O.cutoff2;
  const float kPi = (float)3.141592653589793;
  float r2 = f.mu[0] * f.mu[0] + f.mu[2] * f.mu[2];
  float r = sqrtf(r2);
  float R = sqrtf(k) * (su < sv ? sv : su);
  float Rn = R + S.z_near;
  bool vis = f.valid && (r2 > Rn * Rn) && finite_f(r2) && finite_f(R) && finite_f(f.mu[1]);
  float phi_c = spec_atan2(f.mu[0], f.mu[2]);
  float q = vis ? R / r : 0.0f;
  float dphi = spec_asin(q < 1.0f ? q : 1.0f);
  float y_lo = f.mu[1] - R, y_hi = f.mu[1] + R, r_lo = r - R, r_hi = r + R;
  float a1 = y_lo / r_lo, a2 = y_lo / r_hi, b1 = y_hi / r_lo, b2 = y_hi / r_hi;
  float yn_lo = a1 < a2 ? a1 : a2;
  float yn_hi = b1 < b2 ? b2 : b1;
  float a_lo = phi_c - dphi, a_hi = phi_c + dphi;
  bool back = (a_lo < -kPi) || (a_hi > kPi);
  float xlo = S.fx * a_lo, xhi = S.fx * a_hi, ylo = S.fy * yn_lo, yhi = S.fy * yn_hi;
  if (O.lowpass) {
    float rl = O.rl;
    float pcx = S.fx * phi_c;
    float pcy = S.fy * (f.mu[1] / r);
    float a = pcx - rl, c = pcx + rl, e = pcy - rl, g = pcy + rl;
    xlo = a < xlo ? a : xlo;
    xhi = c > xhi ? c : xhi;
    ylo = e < ylo ? e : ylo;
    yhi = g > yhi ? g : yhi;
  }
  float X_lo = ((xlo - 1.0f) + S.cx) - 0.5f;
  float X_hi = ((xhi + 1.0f) + S.cx) - 0.5f;
  float Y_lo = ((ylo - 1.0f) + S.cy) - 0.5f;
  float Y_hi = ((yhi + 1.0f) + S.cy) - 0.5f;
  vis = vis && finite_f(X_lo) && finite_f(X_hi) && finite_f(Y_lo) && finite_f(Y_hi);
  b.vis = vis;
  b.wrap = false;
  b.full_cols = false;
  b.el_c = b.az_c = b.beta = 0.0f;
  if (!vis) {
    b.touch = false;
    b.n_tiles = 0;
    b.key = 0.0f;
    b.tx_lo = b.tx_hi = b.ty_lo = b.ty_hi = b.i_lo = b.i_hi = b.j_lo = b.j_hi = 0;
    return;
  }
  X_lo = back ? -2.0f : fclamp_spec(X_lo, -2.0f, (float)(S.W + 2));
  X_hi = back ? (float)(S.W + 2) : fclamp_spec(X_hi, -2.0f, (float)(S.W + 2));
  Y_lo = fclamp_spec(Y_lo, -2.0f, (float)(S.H + 2));
  Y_hi = fclamp_spec(Y_hi, -2.0f, (float)(S.H + 2));
  int i_lo = max((int)ceilf(X_lo), 0);
  int i_hi = min((int)floorf(X_hi), S.W - 1);
  int j_lo = max((int)ceilf(Y_lo), 0);
  int j_hi = min((int)floorf(Y_hi), S.H - 1);
  b.i_lo = i_lo; b.i_hi = i_hi; b.j_lo = j_lo; b.j_hi = j_hi;
  b.touch = (i_lo <= i_hi) && (j_lo <= j_hi);
  b.tx_lo = i_lo / S.tw; b.tx_hi = i_hi / S.tw;
  b.ty_lo = j_lo / S.th; b.ty_hi = j_hi / S.th;
  b.n_tiles = b.touch ? (uint32_t)((b.tx_hi - b.tx_lo + 1) * (b.ty_hi - b.ty_lo + 1)) : 0u;
  b.key = r2;
}

__device__ inline void spec_lidar_bins(const Frame32& f, float su, float sv, const SensorK& S, const OptsK& O,
                                       Bins& b) {
#pragma clang fp contract(off)
  const float k = O.cutoff2;
  float rxy2 = f.mu[0] * f.mu[0] + f.mu[1] * f.mu[1];
  float r2 = rxy2 + f.mu[2] * f.mu[2];
  float rxy = sqrtf(rxy2);
  float r = sqrtf(r2);
  float R = sqrtf(k) * (su < sv ? sv : su);
  float Rn = R + S.z_near;
  bool vis = f.valid && (r2 > Rn * Rn);
  float Reff = O.lowpass ? R + r * S.c_lp : R;
  vis = vis && finite_f(r2) && finite_f(Reff);
  b.vis = vis;
  b.wrap = false;
  b.full_cols = false;
  b.el_c = b.az_c = b.beta = 0.0f;
  if (!vis) {
    b.touch = false;
    b.n_tiles = 0;
    b.key = 0.0f;
    b.tx_lo = b.tx_hi = b.ty_lo = b.ty_hi = b.i_lo = b.i_hi = b.j_lo = b.j_hi = 0;
    return;
  }
  float el_c = spec_atan2(f.mu[2], rxy);
  float az_c = spec_atan2(f.mu[1], f.mu[0]);
  float q = Reff / r;
  float sb = q < 1.0f ? q : 1.0f;
  float beta = spec_asin(sb);
  b.el_c = el_c;
  b.az_c = az_c;
  b.beta = beta;
  float el_lo = el_c - beta, el_hi = el_c + beta;
  bool full_az = !(rxy > Reff);
  float sa = full_az ? 0.0f : Reff / rxy;
  float daz = spec_asin(sa);
  float az_lo = (az_c - daz) * S.inv_step;
  float az_hi = (az_c + daz) * S.inv_step;
  int j_lo = lower_bound_f(S.tab, S.H, el_lo) - 1;
  int j_hi = upper_bound_f(S.tab, S.H, el_hi);
  j_lo = max(j_lo, 0);
  j_hi = min(j_hi, S.H - 1);
  if (full_az) { az_lo = 0.0f; az_hi = 0.0f; }
  int i_lo = (int)floorf(az_lo) - 1;
  int i_hi = (int)ceilf(az_hi) + 1;
  bool full = full_az || (i_hi - i_lo + 1 >= S.W);
  if (full) { i_lo = 0; i_hi = S.W - 1; }
  int c_lo = imod(i_lo, S.W), c_hi = imod(i_hi, S.W);
  int tx_lo = c_lo / S.tw, tx_hi = c_hi / S.tw;
  bool wrap = c_lo > c_hi;
  bool all_tx = wrap && (tx_hi >= tx_lo);
  wrap = wrap && !all_tx;
  if (all_tx) { tx_lo = 0; tx_hi = S.n_tx - 1; }
  int ncols = wrap ? (S.n_tx - tx_lo) + (tx_hi + 1) : tx_hi - tx_lo + 1;
  b.i_lo = c_lo; b.i_hi = c_hi; b.j_lo = j_lo; b.j_hi = j_hi;
  b.tx_lo = tx_lo; b.tx_hi = tx_hi;
  b.ty_lo = j_lo / S.th; b.ty_hi = j_hi / S.th;
  b.wrap = wrap;
  b.full_cols = full || all_tx;
  b.touch = j_lo <= j_hi;
  b.n_tiles = b.touch ? (uint32_t)(ncols * (b.ty_hi - b.ty_lo + 1)) : 0u;
  b.key = r2;
}

// --------------------------------------------------------------------------
// Real spherical harmonics, degree <= 3, orthonormal, Condon-Shortley phase,
// index l^2 + l + m.  Constants are K_l^m-derived values of the textbook
// definition Y_lm ~ sqrt(2) K_l^m P_l^m(cos t) (cos|sin)(m phi).
// --------------------------------------------------------------------------
struct SHC {
  static constexpr float c0 = 0.28209479177387814f;   // 1/(2 sqrt(pi))
  static constexpr float c1 = 0.4886025119029199f;    // sqrt(3/(4 pi))
  static constexpr float c2a = 1.0925484305920792f;   // sqrt(15/(4 pi))
  static constexpr float c2b = 0.31539156525252005f;  // sqrt(5/(16 pi))
  static constexpr float c2c = 0.5462742152960396f;   // sqrt(15/(16 pi))
  static constexpr float c3a = 0.5900435899266435f;   // sqrt(35/(32 pi))
  static constexpr float c3b = 2.890611442640554f;    // sqrt(105/(4 pi))
  static constexpr float c3c = 0.4570457994644658f;   // sqrt(21/(32 pi))
  static constexpr float c3d = 0.3731763325901154f;   // sqrt(7/(16 pi))
  static constexpr float c3e = 1.445305721320277f;    // sqrt(105/(16 pi))
};

// Y[0..(deg+1)^2) at unit direction (x,y,z); polynomial forms valid on the sphere.
__device__ inline void sh_eval(int deg, float x, float y, float z, float* Y) {
  Y[0] = SHC::c0;
  if (deg < 1) return;
  Y[1] = -SHC::c1 * y;
  Y[2] = SHC::c1 * z;
  Y[3] = -SHC::c1 * x;
  if (deg < 2) return;
  float xx = x * x, yy = y * y, zz = z * z;
  Y[4] = SHC::c2a * x * y;
  Y[5] = -SHC::c2a * y * z;
  Y[6] = SHC::c2b * (3.0f * zz - 1.0f);
  Y[7] = -SHC::c2a * x * z;
  Y[8] = SHC::c2c * (xx - yy);
  if (deg < 3) return;
  Y[9] = -SHC::c3a * y * (3.0f * xx - yy);
  Y[10] = SHC::c3b * x * y * z;
  Y[11] = -SHC::c3c * y * (5.0f * zz - 1.0f);
  Y[12] = SHC::c3d * z * (5.0f * zz - 3.0f);
  Y[13] = -SHC::c3c * x * (5.0f * zz - 1.0f);
  Y[14] = SHC::c3e * z * (xx - yy);
  Y[15] = -SHC::c3a * x * (xx - 3.0f * yy);
}

// Gradient of sum_k g_k Y_k(x,y,z) w.r.t. (x,y,z), treating them as free
// variables of the polynomial forms above (callers project onto the sphere).
__device__ inline void sh_grad(int deg, float x, float y, float z, const float* g, float& gx, float& gy, float& gz) {
  gx = gy = gz = 0.0f;
  if (deg < 1) return;
  gy += -SHC::c1 * g[1];
  gz += SHC::c1 * g[2];
  gx += -SHC::c1 * g[3];
  if (deg < 2) return;
  float xx = x * x, yy = y * y, zz = z * z;
  gx += SHC::c2a * y * g[4];
  gy += SHC::c2a * x * g[4];
  gy += -SHC::c2a * z * g[5];
  gz += -SHC::c2a * y * g[5];
  gz += SHC::c2b * 6.0f * z * g[6];
  gx += -SHC::c2a * z * g[7];
  gz += -SHC::c2a * x * g[7];
  gx += SHC::c2c * 2.0f * x * g[8];
  gy += -SHC::c2c * 2.0f * y * g[8];
  if (deg < 3) return;
  gx += -SHC::c3a * y * 6.0f * x * g[9];
  gy += -SHC::c3a * (3.0f * xx - 3.0f * yy) * g[9];
  gx += SHC::c3b * y * z * g[10];
  gy += SHC::c3b * x * z * g[10];
  gz += SHC::c3b * x * y * g[10];
  gy += -SHC::c3c * (5.0f * zz - 1.0f) * g[11];
  gz += -SHC::c3c * y * 10.0f * z * g[11];
  gz += SHC::c3d * (15.0f * zz - 3.0f) * g[12];
  gx += -SHC::c3c * (5.0f * zz - 1.0f) * g[13];
  gz += -SHC::c3c * x * 10.0f * z * g[13];
  gx += SHC::c3e * 2.0f * x * z * g[14];
  gy += -SHC::c3e * 2.0f * y * z * g[14];
  gz += SHC::c3e * (xx - yy) * g[14];
  gx += -SHC::c3a * (3.0f * xx - 3.0f * yy) * g[15];
  gy += SHC::c3a * 6.0f * x * y * g[15];
}

// --------------------------------------------------------------------------
// wave64 helpers
// --------------------------------------------------------------------------
template <int CTRL, int ROW_MASK>
__device__ inline float dpp_add(float v) {
  int t = __builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, ROW_MASK, 0xF, false);
  return v + __int_as_float(t);
}

// Sum over the 64 lanes; the total lands in lane 63.  All lanes must be active.
__device__ inline float wave_sum_last(float v) {
  v = dpp_add<0xB1, 0xF>(v);   // quad_perm [1,0,3,2]
  v = dpp_add<0x4E, 0xF>(v);   // quad_perm [2,3,0,1]
  v = dpp_add<0x141, 0xF>(v);  // row_half_mirror
  v = dpp_add<0x140, 0xF>(v);  // row_mirror
  v = dpp_add<0x142, 0xA>(v);  // row_bcast:15 into rows 1, 3
  v = dpp_add<0x143, 0xC>(v);  // row_bcast:31 into rows 2, 3
  return v;
}

__device__ inline uint32_t wave_sum_u32(uint32_t v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += (uint32_t)__shfl_xor((int)v, o, 64);
  return v;
}

__device__ inline uint64_t lanemask_lt() {
  uint32_t lane = __lane_id();
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// XCD-aware block -> tile map: consecutive tiles stay on one XCD (blocks are
// dealt round-robin over the 8 XCDs, each with its own L2).
__device__ inline int xcd_remap(int x, int n) {
  int q = n >> 3;
  if (x < (q << 3)) return (x & 7) * q + (x >> 3);
  return x;
}

}  // namespace gs
