// a0 + a2: pose composition and per-surfel preprocessing (pinhole, cylindrical
// camera and LiDAR).
//
// One thread per surfel.  Integer decisions (visibility, tile rectangle,
// depth key, normal orientation) follow the FP32 binning specification in
// gs_internal.h.  The blend record is built in FP64 from the FP32 inputs and
// rounded once, in the form the per-ray solve wants:
//   camera: h' = e3 + P (dx, dy) with (dx, dy) the pixel offset from the
//           projected centre, u = h'_0/h'_2, v = h'_1/h'_2, z = mu_z / h'_2
//   LiDAR : h' = e3 + Q (d - mu_hat), u, v as above, range = |mu| / h'_2
//   cylindrical: the camera form in the surfel's own column frame (the
//           sensor frame turned about y by the centre's angle phi_c, where
//           mu = (0, mu_y, r)): a ray at angle phi is the pinhole ray
//           (tan dphi, y_n sec dphi, 1), dphi = phi - phi_c, so with
//           X = f_x tan dphi, Y = f_y (y_n sec dphi - mu_y / r),
//           h' = e3 + P (X, Y) and the depth is r sec dphi / h'_2
// (h' is adj(M) d scaled so that its third entry is 1 at the surfel centre).
#include "gs_internal.h"
#include "kernels.h"

namespace gs {

__global__ void k_compose_poses(const float* __restrict__ sensor_pose, const float* __restrict__ group_poses,
                                int pose_base, int n_groups, float* __restrict__ out) {
#pragma clang fp contract(off)
  int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= n_groups) return;
  const float* a = sensor_pose;
  const float* b = group_poses + 12 * (pose_base + g);
  float* o = out + 12 * g;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) o[4 * i + j] = (a[4 * i] * b[j] + a[4 * i + 1] * b[4 + j]) + a[4 * i + 2] * b[8 + j];
    o[4 * i + 3] = ((a[4 * i] * b[3] + a[4 * i + 1] * b[7]) + a[4 * i + 2] * b[11]) + a[4 * i + 3];
  }
}

// The batched step's per-sensor set-up in one launch, one workgroup per
// sensor: its 16 status words cleared and its group poses composed.
__global__ void k_sensor_setup(const float* __restrict__ group_poses, SensorSetup s) {
#pragma clang fp contract(off)
  const int k = blockIdx.x, g = threadIdx.x;
  if (g < 16) s.status[k][g] = 0u;
  if (g >= s.n_groups[k]) return;
  const float* a = s.sensor_pose[k];
  const float* b = group_poses + 12 * (s.pose_base[k] + g);
  float* o = s.pose_out[k] + 12 * g;
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) o[4 * i + j] = (a[4 * i] * b[j] + a[4 * i + 1] * b[4 + j]) + a[4 * i + 2] * b[8 + j];
    o[4 * i + 3] = ((a[4 * i] * b[3] + a[4 * i + 1] * b[7]) + a[4 * i + 2] * b[11]) + a[4 * i + 3];
  }
}

struct Frame64 {
  double R[9], t[3];
  double tus[3], tvs[3], ns[3], mus[3];
  double M[3][3];
  double adj[3][3];  // adj[row][col]; columns are r1 x r2, r2 x r0, r0 x r1
  double det;
};

__device__ inline void frame64(const float* P, float m0, float m1, float m2, float qw, float qx, float qy, float qz,
                               float su, float sv, Frame64& F) {
  for (int i = 0; i < 3; ++i) {
    F.R[3 * i] = P[4 * i];
    F.R[3 * i + 1] = P[4 * i + 1];
    F.R[3 * i + 2] = P[4 * i + 2];
    F.t[i] = P[4 * i + 3];
  }
  double w = qw, x = qx, y = qy, z = qz;
  double s = 2.0 / (w * w + x * x + y * y + z * z);
  double a[3] = {1.0 - s * (y * y + z * z), s * (x * y + w * z), s * (x * z - w * y)};
  double b[3] = {s * (x * y - w * z), 1.0 - s * (x * x + z * z), s * (y * z + w * x)};
  double c[3] = {s * (x * z + w * y), s * (y * z - w * x), 1.0 - s * (x * x + y * y)};
  double m[3] = {m0, m1, m2};
  for (int i = 0; i < 3; ++i) {
    const double* r = F.R + 3 * i;
    F.tus[i] = r[0] * a[0] + r[1] * a[1] + r[2] * a[2];
    F.tvs[i] = r[0] * b[0] + r[1] * b[1] + r[2] * b[2];
    F.ns[i] = r[0] * c[0] + r[1] * c[1] + r[2] * c[2];
    F.mus[i] = r[0] * m[0] + r[1] * m[1] + r[2] * m[2] + F.t[i];
    F.M[i][0] = (double)su * F.tus[i];
    F.M[i][1] = (double)sv * F.tvs[i];
    F.M[i][2] = F.mus[i];
  }
  const double* r0 = F.M[0];
  const double* r1 = F.M[1];
  const double* r2 = F.M[2];
  double c0[3] = {r1[1] * r2[2] - r1[2] * r2[1], r1[2] * r2[0] - r1[0] * r2[2], r1[0] * r2[1] - r1[1] * r2[0]};
  double c1[3] = {r2[1] * r0[2] - r2[2] * r0[1], r2[2] * r0[0] - r2[0] * r0[2], r2[0] * r0[1] - r2[1] * r0[0]};
  double c2[3] = {r0[1] * r1[2] - r0[2] * r1[1], r0[2] * r1[0] - r0[0] * r1[2], r0[0] * r1[1] - r0[1] * r1[0]};
  for (int i = 0; i < 3; ++i) {
    F.adj[i][0] = c0[i];
    F.adj[i][1] = c1[i];
    F.adj[i][2] = c2[i];
  }
  F.det = r0[0] * c0[0] + r0[1] * c0[1] + r0[2] * c0[2];
}

__device__ inline void load_surfel(const PrepArgs& a, int i, float* P, float& m0, float& m1, float& m2, float& qw,
                                   float& qx, float& qy, float& qz, float& su, float& sv) {
  const int N = a.n;
  int g = group_of(a.groups, i);
  const float* pp = a.ws.pose + 12 * g;
#pragma unroll
  for (int k = 0; k < 12; ++k) P[k] = pp[k];
  m0 = a.mean[i];
  m1 = a.mean[N + i];
  m2 = a.mean[2 * N + i];
  qw = a.quat[i];
  qx = a.quat[N + i];
  qy = a.quat[2 * N + i];
  qz = a.quat[3 * N + i];
  su = a.scale[i];
  sv = a.scale[N + i];
}

// DEG: SH degree of the colour (-1: plain RGB), fixed per instantiation so
// that the coefficient loads unroll and issue together, ahead of the FP64 frame.
template <int DEG, bool CYL>
__global__ __launch_bounds__(256) void k_prep_camera(PrepArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  const int N = a.n;
  float P[12], m0, m1, m2, qw, qx, qy, qz, su, sv;
  load_surfel(a, i, P, m0, m1, m2, qw, qx, qy, qz, su, sv);
  Frame32 f;
  spec_frame(P, m0, m1, m2, qw, qx, qy, qz, su, sv, f);
  Bins b;
  if constexpr (CYL)
    spec_cyl_bins(f, su, sv, a.S, a.O, b);
  else
    spec_pinhole_bins(f, a.S, a.O, b);
  a.ws.key[0][i] = b.vis ? __float_as_uint(b.key) : kInvalidKey;
  a.ws.val[0][i] = a.rec_base + (uint32_t)i;
  a.ws.ntiles[i] = b.n_tiles;
  a.ws.visible[i] = b.vis ? 1u : 0u;
  if (!b.touch) return;
  a.ws.rect[i] = make_int4(b.tx_lo, b.tx_hi, b.ty_lo, b.ty_hi);
  constexpr int nb = DEG >= 0 ? (DEG + 1) * (DEG + 1) : 1;
  float co[3][nb];
  if constexpr (DEG >= 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int k = 0; k < nb; ++k) co[c][k] = a.sh[(size_t)(k * 3 + c) * N + i];
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c) co[c][0] = a.rgb[(size_t)c * N + i];
  }
  const float nsign = spec_normal_sign(f);

  Frame64 F;
  frame64(P, m0, m1, m2, qw, qx, qy, qz, su, sv, F);
  double muz, pcx, pcy;
  double adj[3][3];
  if constexpr (CYL) {
    // the centre's column frame: x' = c x - s z, z' = s x + c z (mu' = (0, mu_y, r));
    // adj(Ry M) = adj(M) Ry^T, det unchanged
    const double r = sqrt(F.mus[0] * F.mus[0] + F.mus[2] * F.mus[2]);
    const double phi_c = atan2(F.mus[0], F.mus[2]);
    const double c = F.mus[2] / r, sn = F.mus[0] / r;
    for (int k = 0; k < 3; ++k) {
      adj[k][0] = F.adj[k][0] * c - F.adj[k][2] * sn;
      adj[k][1] = F.adj[k][1];
      adj[k][2] = F.adj[k][0] * sn + F.adj[k][2] * c;
    }
    muz = r;
    pcx = (double)a.S.fx * phi_c + (double)a.S.cx;
    pcy = (double)a.S.fy * F.mus[1] / r + (double)a.S.cy;
  } else {
    for (int k = 0; k < 3; ++k)
      for (int c = 0; c < 3; ++c) adj[k][c] = F.adj[k][c];
    muz = F.mus[2];
    pcx = (double)a.S.fx * F.mus[0] / muz + (double)a.S.cx;
    pcy = (double)a.S.fy * F.mus[1] / muz + (double)a.S.cy;
  }
  const double k0 = muz / ((double)a.S.fx * F.det);
  const double k1 = muz / ((double)a.S.fy * F.det);
  double Pm[6] = {adj[0][0] * k0, adj[0][1] * k1, adj[1][0] * k0, adj[1][1] * k1, adj[2][0] * k0, adj[2][1] * k1};

  // colour
  float col[3];
  if constexpr (DEG >= 0) {
    // view direction in the group frame: R^T mu_s
    double dx = F.R[0] * F.mus[0] + F.R[3] * F.mus[1] + F.R[6] * F.mus[2];
    double dy = F.R[1] * F.mus[0] + F.R[4] * F.mus[1] + F.R[7] * F.mus[2];
    double dz = F.R[2] * F.mus[0] + F.R[5] * F.mus[1] + F.R[8] * F.mus[2];
    double inv = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    float Y[16];
    sh_eval(DEG, (float)(dx * inv), (float)(dy * inv), (float)(dz * inv), Y);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      float acc = 0.5f;
#pragma unroll
      for (int k = 0; k < nb; ++k) acc += co[c][k] * Y[k];
      col[c] = acc > 0.0f ? acc : 0.0f;
    }
  } else {
    col[0] = co[0][0];
    col[1] = co[1][0];
    col[2] = co[2][0];
  }
  const float o = a.opacity[i];
  const float log2o = log2f(o);

  // grazing: can h'_2 = 1 + P20 dx + P21 dy drop below 1/8 inside the rectangle?
  double mx = fmax(fabs(b.i_lo + 0.5 - pcx), fabs(b.i_hi + 0.5 - pcx));
  double my = fmax(fabs(b.j_lo + 0.5 - pcy), fabs(b.j_hi + 0.5 - pcy));
  // grazing over the rectangle; the FP32 error bound (see the record flags)
  // over the pixels of every tile the rectangle touches (up to a tile beyond
  // it): s = 2 |offset|_inf there (4 |(X, Y)|_inf for the cylindrical map)
  bool graze;
  double h2e, s;
  const double mxe = mx + a.S.tw, mye = my + a.S.th;
  if constexpr (CYL) {
    // |X| <= f tan(dphi_max), |Y| <= |dy| + |p_y - c_y| (sec dphi_max - 1); past
    // 80 degrees (only for surfels near the camera) every pair may graze
    const double dmax = mx / (double)a.S.fx;
    const double ay = fmax(fabs(b.j_lo + 0.5 - (double)a.S.cy), fabs(b.j_hi + 0.5 - (double)a.S.cy));
    const double Xm = (double)a.S.fx * tan(fmin(dmax, 1.39)), Ym = my + ay * (1.0 / cos(fmin(dmax, 1.39)) - 1.0);
    graze = dmax > 1.39 || 1.0 - (fabs(Pm[4]) * Xm + fabs(Pm[5]) * Ym) < 0.125;
    const double de = fmin(mxe / (double)a.S.fx, 1.39), aye = ay + a.S.th;
    const double Xe = (double)a.S.fx * tan(de), Ye = mye + aye * (1.0 / cos(de) - 1.0);
    h2e = 1.0 - (fabs(Pm[4]) * Xe + fabs(Pm[5]) * Ye);
    s = 4.0 * fmax(Xe, Ye);
  } else {
    graze = 1.0 - (fabs(Pm[4]) * mx + fabs(Pm[5]) * my) < 0.125;
    h2e = 1.0 - (fabs(Pm[4]) * mxe + fabs(Pm[5]) * mye);
    s = 2.0 * fmax(mxe, mye);
  }
  uint32_t flags = graze ? kFlagGrazing : 0u;
  // kappa: the (u, v) rows' largest absolute sum, plus the h'_2 row's times
  // the largest |u|, |v| inside the cutoff (its error enters as u dh'_2)
  const double kap = fmax(fabs(Pm[0]) + fabs(Pm[1]), fabs(Pm[2]) + fabs(Pm[3])) + 3.4 * (fabs(Pm[4]) + fabs(Pm[5]));
  flags |= conditioning_flags((0x1p-23 * kap * s + 0x1p-20) / fmax(h2e, 0.125), o);

  float4* r = a.ws.rec + 4 * (size_t)i;
  r[0] = make_float4((float)Pm[0], (float)Pm[1], (float)Pm[2], (float)Pm[3]);
  r[1] = make_float4((float)Pm[4], (float)Pm[5], (float)muz, log2o);
  r[2] = make_float4(col[0], col[1], col[2], (float)(nsign * F.ns[0]));
  // slot 15: the per-record factor of the pairs' FP32 error bound, 2^-23 kappa
  // times the offsets' weight in it (2, or 4 for the cylindrical map)
  r[3] = make_float4((float)(nsign * F.ns[1]), (float)(nsign * F.ns[2]), __uint_as_float(flags),
                     (float)((CYL ? 0x1p-21 : 0x1p-22) * kap));
  double* r64 = a.ws.rec64 + kRec64 * (size_t)i;
  r64[0] = pcx;
  r64[1] = pcy;
  r64[2] = muz;
  // conservative pixel rectangle (columns, rows), 16 bits per bound
  uint32_t* rr = reinterpret_cast<uint32_t*>(r64 + 3);
  rr[0] = (uint32_t)b.i_lo | ((uint32_t)b.i_hi << 16);
  rr[1] = (uint32_t)b.j_lo | ((uint32_t)b.j_hi << 16);
  if (flags & kFlagF64) {
    double* gz = a.ws.grz + kGrz * (size_t)i;
    for (int k = 0; k < 6; ++k) gz[k] = Pm[k];
    gz[6] = muz;
  }
}

__global__ __launch_bounds__(256) void k_prep_lidar(PrepArgs a) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  float P[12], m0, m1, m2, qw, qx, qy, qz, su, sv;
  load_surfel(a, i, P, m0, m1, m2, qw, qx, qy, qz, su, sv);
  Frame32 f;
  spec_frame(P, m0, m1, m2, qw, qx, qy, qz, su, sv, f);
  Bins b;
  spec_lidar_bins(f, su, sv, a.S, a.O, b);
  a.ws.key[0][i] = b.vis ? __float_as_uint(b.key) : kInvalidKey;
  a.ws.val[0][i] = a.rec_base + (uint32_t)i;
  a.ws.ntiles[i] = b.n_tiles;
  a.ws.visible[i] = b.vis ? 1u : 0u;
  if (!b.touch) return;
  a.ws.rect[i] = make_int4(b.tx_lo, b.tx_hi, b.ty_lo, b.ty_hi | (b.wrap ? (1 << 30) : 0));

  Frame64 F;
  frame64(P, m0, m1, m2, qw, qx, qy, qz, su, sv, F);
  const double rn = sqrt(F.mus[0] * F.mus[0] + F.mus[1] * F.mus[1] + F.mus[2] * F.mus[2]);
  const double kq = rn / F.det;
  double Q[9];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) Q[3 * r + c] = F.adj[r][c] * kq;
  const double mh[3] = {F.mus[0] / rn, F.mus[1] / rn, F.mus[2] / rn};
  const float o = a.opacity[i];
  const float log2o = log2f(o);
  const float inten = a.intensity ? a.intensity[i] : 0.0f;

  // grazing: bound the angle between any ray of the rectangle and the centre
  float el_lo = a.S.tab[b.j_lo], el_hi = a.S.tab[b.j_hi];
  double ang_el = fmax(fabs((double)el_lo - b.el_c), fabs((double)el_hi - b.el_c));
  double ang_az;
  if (b.full_cols) {
    ang_az = 3.2;
  } else {
    const double two_pi = 6.283185307179586;
    double step = two_pi / a.S.W;
    double d1 = fabs(remainder(b.i_lo * step - b.az_c, two_pi));
    double d2 = fabs(remainder((b.i_hi + 1) * step - b.az_c, two_pi));
    ang_az = fmax(d1, d2) + step * (double)a.S.tw;
  }
  double bound = ang_el + ang_az + 0.01;
  const double h2m = 1.0 - (fabs(Q[6]) + fabs(Q[7]) + fabs(Q[8])) * bound;
  bool graze = h2m < 0.125;
  uint32_t flags = graze ? kFlagGrazing : 0u;
  // FP32 error bound (see the record flags) over the rays of every tile the
  // rectangle touches: offsets from the centre direction and from a tile's
  // reference direction are chords of at most `bound` plus a tile's angular
  // extent (its columns' azimuth span, 0.1 rad of elevation at most)
  const double kap = fmax(fabs(Q[0]) + fabs(Q[1]) + fabs(Q[2]), fabs(Q[3]) + fabs(Q[4]) + fabs(Q[5])) +
                     3.4 * (fabs(Q[6]) + fabs(Q[7]) + fabs(Q[8]));
  const double ext = bound + 6.283185307179586 * a.S.tw / a.S.W + 0.1;
  const double h2e = 1.0 - (fabs(Q[6]) + fabs(Q[7]) + fabs(Q[8])) * ext;
  flags |= conditioning_flags((0x1p-23 * kap * 3.0 * ext + 0x1p-20) / fmax(h2e, 0.125), o);

  float4* r = a.ws.rec + 4 * (size_t)i;
  r[0] = make_float4((float)Q[0], (float)Q[1], (float)Q[2], (float)Q[3]);
  r[1] = make_float4((float)Q[4], (float)Q[5], (float)Q[6], (float)Q[7]);
  r[2] = make_float4((float)Q[8], (float)rn, log2o, inten);
  // flags; 2^-23 kappa, the per-record factor of the pairs' FP32 error bound;
  // the conservative column/beam rectangle (columns may wrap), 16 bits per bound
  r[3] = make_float4(__uint_as_float(flags), (float)(0x1p-23 * kap),
                     __uint_as_float((uint32_t)b.i_lo | ((uint32_t)b.i_hi << 16)),
                     __uint_as_float((uint32_t)b.j_lo | ((uint32_t)b.j_hi << 16)));
  double* r64 = a.ws.rec64 + kRec64 * (size_t)i;
  r64[0] = mh[0];
  r64[1] = mh[1];
  r64[2] = mh[2];
  r64[3] = a.drop ? (double)a.drop[i] : 0.0;  // ray-drop probability
  if (flags & kFlagF64) {
    double* gz = a.ws.grz + kGrz * (size_t)i;
    for (int k = 0; k < 9; ++k) gz[k] = Q[k];
    gz[9] = rn;
  }
}

void launch_compose_poses(const float* sensor_pose, const float* group_poses, int pose_base, int n_groups, float* out,
                          hipStream_t st) {
  hipLaunchKernelGGL(k_compose_poses, dim3(1), dim3(64), 0, st, sensor_pose, group_poses, pose_base, n_groups, out);
}

void launch_sensor_setup(const float* group_poses, const SensorSetup& s, hipStream_t st) {
  if (s.n <= 0) return;
  hipLaunchKernelGGL(k_sensor_setup, dim3(s.n), dim3(64), 0, st, group_poses, s);
}

void launch_prep(const PrepArgs& a, hipStream_t st) {
  if (a.n == 0) return;
  dim3 grid((a.n + 255) / 256);
  if (a.S.kind == GS_SENSOR_PINHOLE) {
    switch (a.sh_degree) {
      case 0: hipLaunchKernelGGL((k_prep_camera<0, false>), grid, dim3(256), 0, st, a); break;
      case 1: hipLaunchKernelGGL((k_prep_camera<1, false>), grid, dim3(256), 0, st, a); break;
      case 2: hipLaunchKernelGGL((k_prep_camera<2, false>), grid, dim3(256), 0, st, a); break;
      case 3: hipLaunchKernelGGL((k_prep_camera<3, false>), grid, dim3(256), 0, st, a); break;
      default: hipLaunchKernelGGL((k_prep_camera<-1, false>), grid, dim3(256), 0, st, a); break;
    }
  } else if (a.S.kind == GS_SENSOR_CYLINDRICAL) {
    switch (a.sh_degree) {
      case 0: hipLaunchKernelGGL((k_prep_camera<0, true>), grid, dim3(256), 0, st, a); break;
      case 1: hipLaunchKernelGGL((k_prep_camera<1, true>), grid, dim3(256), 0, st, a); break;
      case 2: hipLaunchKernelGGL((k_prep_camera<2, true>), grid, dim3(256), 0, st, a); break;
      case 3: hipLaunchKernelGGL((k_prep_camera<3, true>), grid, dim3(256), 0, st, a); break;
      default: hipLaunchKernelGGL((k_prep_camera<-1, true>), grid, dim3(256), 0, st, a); break;
    }
  } else
    hipLaunchKernelGGL(k_prep_lidar, grid, dim3(256), 0, st, a);
}

}  // namespace gs
