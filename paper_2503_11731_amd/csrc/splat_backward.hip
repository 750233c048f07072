// a9: per-surfel adjoint.  Maps the accumulated gradients of each surfel's
// blend record back to its parameters (centre, quaternion, scales, opacity,
// colour or SH coefficients, intensity), in FP64, one thread per surfel.
//
// Camera record: P[:,j] = adj(M)[:,j] mu_z / (f_j det M) (j = 0, 1),
//   pc = (fx mu_x / mu_z, fy mu_y / mu_z), mu_z, o, colour, normal.
// LiDAR record: Q = |mu| adj(M) / det M, mu_hat = mu / |mu|, |mu|, o, intensity.
// Cylindrical record: the camera record of M' = Ry M, the sensor frame turned
// about y by the centre's angle phi_c = atan2(mu_x, mu_z) (mu' = (0, mu_y, r)),
// with pc = (c_x + fx phi_c, c_y + fy mu_y / r) and r in place of mu_z.
// adj(M) columns are r1 x r2, r2 x r0, r0 x r1 (rows r_i of M), det = r0 . (r1 x r2),
// M = [s_u R t_u, s_v R t_v, R mu + t], (t_u, t_v, n) the columns of the
// rotation of q scaled by s = 2/|q|^2.
#include "gs_internal.h"
#include "kernels.h"

namespace gs {

namespace {

__device__ inline void cross3(const double* a, const double* b, double* c) {
  c[0] = a[1] * b[2] - a[2] * b[1];
  c[1] = a[2] * b[0] - a[0] * b[2];
  c[2] = a[0] * b[1] - a[1] * b[0];
}
__device__ inline void acc_cross(const double* a, const double* b, double* acc) {
  double c[3];
  cross3(a, b, c);
  acc[0] += c[0];
  acc[1] += c[1];
  acc[2] += c[2];
}
__device__ inline double dot3(const double* a, const double* b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

// One instantiation per sensor kind and SH degree (-1: plain colour or
// intensity): the two chain rules share little, one kernel holding both needs
// twice the registers, and a fixed degree keeps the coefficient loop unrolled
// so that each surfel's SH loads and read-modify-writes issue together.
template <int KIND, int DEG>
__global__ __launch_bounds__(256, 3) void k_splat_backward(SplatBwdArgs A) {
  const PrepArgs& a = A.p;
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= a.n) return;
  if (a.ws.ntiles[i] == 0) return;
  const int N = a.n;
  float gf[kGradFields];
  bool any = false;
#pragma unroll
  for (int f = 0; f < kGradFields; ++f) {
    gf[f] = a.ws.gacc[(size_t)f * a.gacc_stride + i];
    any = any || gf[f] != 0.0f;
  }
  if (!any) return;

  // reload and rebuild the surfel map (same arithmetic as the preprocess)
  const int g = group_of(a.groups, i);
  float P[12];
  for (int k = 0; k < 12; ++k) P[k] = a.ws.pose[12 * g + k];
  const float m0 = a.mean[i], m1 = a.mean[N + i], m2 = a.mean[2 * N + i];
  const float qwf = a.quat[i], qxf = a.quat[N + i], qyf = a.quat[2 * N + i], qzf = a.quat[3 * N + i];
  const float su = a.scale[i], sv = a.scale[N + i];
  double R[9], t[3];
  for (int r = 0; r < 3; ++r) {
    R[3 * r] = P[4 * r];
    R[3 * r + 1] = P[4 * r + 1];
    R[3 * r + 2] = P[4 * r + 2];
    t[r] = P[4 * r + 3];
  }
  const double w = qwf, x = qxf, y = qyf, z = qzf;
  const double n2 = w * w + x * x + y * y + z * z;
  const double s = 2.0 / n2;
  const double B[9] = {-(y * y + z * z), x * y - w * z, x * z + w * y,   // rows of Rq - I, over s
                       x * y + w * z,    -(x * x + z * z), y * z - w * x,
                       x * z - w * y,    y * z + w * x,  -(x * x + y * y)};
  double Rq[9];
  for (int k = 0; k < 9; ++k) Rq[k] = s * B[k] + ((k % 4) == 0 ? 1.0 : 0.0);
  // columns of Rq: t_u, t_v, n
  double tu[3] = {Rq[0], Rq[3], Rq[6]}, tv[3] = {Rq[1], Rq[4], Rq[7]}, nn[3] = {Rq[2], Rq[5], Rq[8]};
  double tus[3], tvs[3], ns[3], mus[3];
  const double mo[3] = {m0, m1, m2};
  for (int r = 0; r < 3; ++r) {
    tus[r] = dot3(R + 3 * r, tu);
    tvs[r] = dot3(R + 3 * r, tv);
    ns[r] = dot3(R + 3 * r, nn);
    mus[r] = dot3(R + 3 * r, mo) + t[r];
  }
  double Mr[3][3];
  for (int r = 0; r < 3; ++r) {
    Mr[r][0] = (double)su * tus[r];
    Mr[r][1] = (double)sv * tvs[r];
    Mr[r][2] = mus[r];
  }
  double c0[3], c1[3], c2[3];
  cross3(Mr[1], Mr[2], c0);
  cross3(Mr[2], Mr[0], c1);
  cross3(Mr[0], Mr[1], c2);
  const double det = dot3(Mr[0], c0);

  double gr0[3] = {0, 0, 0}, gr1[3] = {0, 0, 0}, gr2[3] = {0, 0, 0};  // dL/d rows of M
  double gmus_extra[3] = {0, 0, 0};                                     // direct mu_s terms
  double gns[3] = {0, 0, 0};
  double g_op = 0.0;
  double gcol[3] = {0, 0, 0};
  double g_int = 0.0;

  if constexpr (KIND == GS_SENSOR_PINHOLE) {
    const double fx = a.S.fx, fy = a.S.fy;
    const double muz = mus[2];
    const double ifx = 1.0 / fx, ify = 1.0 / fy, idet = 1.0 / det, imuz = 1.0 / muz;
    const double g0[3] = {gf[0], gf[2], gf[4]};  // dL/dP[:,0]
    const double g1[3] = {gf[1], gf[3], gf[5]};  // dL/dP[:,1]
    const double S0 = dot3(g0, c0) * ifx, S1 = dot3(g1, c1) * ify;
    const double Ssum = S0 + S1;
    const double gdet = -Ssum * muz * idet * idet;
    double ga0[3], ga1[3];
    for (int k = 0; k < 3; ++k) {
      ga0[k] = g0[k] * muz * ifx * idet;
      ga1[k] = g1[k] * muz * ify * idet;
    }
    // adj col0 = r1 x r2 ; adj col1 = r2 x r0
    acc_cross(Mr[2], ga0, gr1);
    acc_cross(ga0, Mr[1], gr2);
    acc_cross(Mr[0], ga1, gr2);
    acc_cross(ga1, Mr[2], gr0);
    for (int k = 0; k < 3; ++k) {
      gr0[k] += gdet * c0[k];
      gr1[k] += gdet * c1[k];
      gr2[k] += gdet * c2[k];
    }
    // mu_z from P's scale, from the record's mu_z, and pc
    const double gpcx = gf[6], gpcy = gf[7];
    gmus_extra[0] += gpcx * fx * imuz;
    gmus_extra[1] += gpcy * fy * imuz;
    gmus_extra[2] += Ssum * idet + (double)gf[8] - (gpcx * fx * mus[0] + gpcy * fy * mus[1]) * imuz * imuz;
    g_op = gf[9];
    gcol[0] = gf[10];
    gcol[1] = gf[11];
    gcol[2] = gf[12];
    // normal: output = sign * n_s
    Frame32 f32;
    spec_frame(P, m0, m1, m2, qwf, qxf, qyf, qzf, su, sv, f32);
    const double sgn = spec_normal_sign(f32);
    gns[0] = sgn * gf[13];
    gns[1] = sgn * gf[14];
    gns[2] = sgn * gf[15];
  } else if constexpr (KIND == GS_SENSOR_CYLINDRICAL) {
    const double fx = a.S.fx, fy = a.S.fy;
    const double r = sqrt(mus[0] * mus[0] + mus[2] * mus[2]);
    const double cc = mus[2] / r, sc = mus[0] / r;
    // rows of M' = Ry M and its adjugate columns (det unchanged)
    double Mp[3][3];
    for (int k = 0; k < 3; ++k) {
      Mp[0][k] = cc * Mr[0][k] - sc * Mr[2][k];
      Mp[1][k] = Mr[1][k];
      Mp[2][k] = sc * Mr[0][k] + cc * Mr[2][k];
    }
    double e0[3], e1[3], e2[3];
    cross3(Mp[1], Mp[2], e0);
    cross3(Mp[2], Mp[0], e1);
    cross3(Mp[0], Mp[1], e2);
    const double detp = dot3(Mp[0], e0);
    const double ifx = 1.0 / fx, ify = 1.0 / fy, idet = 1.0 / detp, ir = 1.0 / r;
    const double g0[3] = {gf[0], gf[2], gf[4]};  // dL/dP[:,0]
    const double g1[3] = {gf[1], gf[3], gf[5]};  // dL/dP[:,1]
    const double S0 = dot3(g0, e0) * ifx, S1 = dot3(g1, e1) * ify;
    const double Ssum = S0 + S1;
    const double gdet = -Ssum * r * idet * idet;
    double ga0[3], ga1[3];
    for (int k = 0; k < 3; ++k) {
      ga0[k] = g0[k] * r * ifx * idet;
      ga1[k] = g1[k] * r * ify * idet;
    }
    double hr0[3] = {0, 0, 0}, hr1[3] = {0, 0, 0}, hr2[3] = {0, 0, 0};  // dL/d rows of M'
    acc_cross(Mp[2], ga0, hr1);
    acc_cross(ga0, Mp[1], hr2);
    acc_cross(Mp[0], ga1, hr2);
    acc_cross(ga1, Mp[2], hr0);
    for (int k = 0; k < 3; ++k) {
      hr0[k] += gdet * e0[k];
      hr1[k] += gdet * e1[k];
      hr2[k] += gdet * e2[k];
    }
    // direct dependencies on mu' = (0, mu_y, r): P's scale r, the record's r, pc_y
    const double gpcx = gf[6], gpcy = gf[7];
    const double gmp[3] = {0.0, gpcy * fy * ir, Ssum * idet + (double)gf[8] - gpcy * fy * mus[1] * ir * ir};
    // phi_c: through pc_x and the turn of M' and mu'; dRy/dphi rows (-s, 0, -c), (0, 0, 0), (c, 0, -s)
    double gphi = gpcx * fx;
    for (int k = 0; k < 3; ++k)
      gphi += hr0[k] * (-sc * Mr[0][k] - cc * Mr[2][k]) + hr2[k] * (cc * Mr[0][k] - sc * Mr[2][k]);
    gphi += gmp[0] * (-sc * mus[0] - cc * mus[2]) + gmp[2] * (cc * mus[0] - sc * mus[2]);
    // back to the sensor frame (Ry^T), and phi_c = atan2(mu_x, mu_z)
    for (int k = 0; k < 3; ++k) {
      gr0[k] = cc * hr0[k] + sc * hr2[k];
      gr1[k] = hr1[k];
      gr2[k] = -sc * hr0[k] + cc * hr2[k];
    }
    gmus_extra[0] += cc * gmp[0] + sc * gmp[2] + gphi * mus[2] * ir * ir;
    gmus_extra[1] += gmp[1];
    gmus_extra[2] += -sc * gmp[0] + cc * gmp[2] - gphi * mus[0] * ir * ir;
    g_op = gf[9];
    gcol[0] = gf[10];
    gcol[1] = gf[11];
    gcol[2] = gf[12];
    Frame32 f32;
    spec_frame(P, m0, m1, m2, qwf, qxf, qyf, qzf, su, sv, f32);
    const double sgn = spec_normal_sign(f32);
    gns[0] = sgn * gf[13];
    gns[1] = sgn * gf[14];
    gns[2] = sgn * gf[15];
  } else {
    const double rn = sqrt(dot3(mus, mus));
    const double irn = 1.0 / rn, idet = 1.0 / det;
    const double mh[3] = {mus[0] * irn, mus[1] * irn, mus[2] * irn};
    const double* adjc[3] = {c0, c1, c2};
    // Q[r][c] = adj[r][c] rn / det, adj[r][c] = column c, entry r
    double gsum = 0.0;
    double gcolv[3][3];
    for (int c = 0; c < 3; ++c)
      for (int r = 0; r < 3; ++r) {
        const double gq = gf[3 * r + c];
        gcolv[c][r] = gq * rn * idet;
        gsum += gq * adjc[c][r];
      }
    const double g_rn = gsum * idet + (double)gf[12];
    const double gdet = -gsum * rn * idet * idet;
    acc_cross(Mr[2], gcolv[0], gr1);
    acc_cross(gcolv[0], Mr[1], gr2);
    acc_cross(Mr[0], gcolv[1], gr2);
    acc_cross(gcolv[1], Mr[2], gr0);
    acc_cross(Mr[1], gcolv[2], gr0);
    acc_cross(gcolv[2], Mr[0], gr1);
    for (int k = 0; k < 3; ++k) {
      gr0[k] += gdet * c0[k];
      gr1[k] += gdet * c1[k];
      gr2[k] += gdet * c2[k];
    }
    const double gmh[3] = {gf[9], gf[10], gf[11]};
    const double pr = dot3(mh, gmh);
    for (int k = 0; k < 3; ++k) gmus_extra[k] += (gmh[k] - mh[k] * pr) * irn + g_rn * mh[k];
    g_op = gf[13];
    g_int = gf[14];
  }

  // rows of M -> columns: M[r][0] = su tus[r], M[r][1] = sv tvs[r], M[r][2] = mus[r]
  const double* grow[3] = {gr0, gr1, gr2};
  double gtus[3], gtvs[3], gmus[3];
  double gsu = 0.0, gsv = 0.0;
  for (int r = 0; r < 3; ++r) {
    gtus[r] = (double)su * grow[r][0];
    gtvs[r] = (double)sv * grow[r][1];
    gmus[r] = grow[r][2] + gmus_extra[r];
    gsu += grow[r][0] * tus[r];
    gsv += grow[r][1] * tvs[r];
  }
  // back to the group frame: x_s = R x  =>  g_x = R^T g_xs
  double gtu[3], gtv[3], gn[3], gmu[3];
  for (int c = 0; c < 3; ++c) {
    gtu[c] = R[c] * gtus[0] + R[3 + c] * gtus[1] + R[6 + c] * gtus[2];
    gtv[c] = R[c] * gtvs[0] + R[3 + c] * gtvs[1] + R[6 + c] * gtvs[2];
    gn[c] = R[c] * gns[0] + R[3 + c] * gns[1] + R[6 + c] * gns[2];
    gmu[c] = R[c] * gmus[0] + R[3 + c] * gmus[1] + R[6 + c] * gmus[2];
  }

  // quaternion: Rq = I + s B(q), s = 2/|q|^2; G = dL/dRq with columns gtu, gtv, gn
  {
    const double G[9] = {gtu[0], gtv[0], gn[0], gtu[1], gtv[1], gn[1], gtu[2], gtv[2], gn[2]};
    double GB = 0.0;
    for (int k = 0; k < 9; ++k) GB += G[k] * B[k];
    const double gw = s * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
    const double gx =
        s * (y * G[1] + z * G[2] + y * G[3] - 2 * x * G[4] - w * G[5] + z * G[6] + w * G[7] - 2 * x * G[8]);
    const double gy =
        s * (-2 * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] - 2 * y * G[8]);
    const double gz =
        s * (-2 * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2 * z * G[4] + y * G[5] + x * G[6] + y * G[7]);
    const double ds = -s * s * GB;  // d s / d q_k = -s^2 q_k
    if (A.g_quat) {
      float* q = A.g_quat + i;
      const float o0 = q[0], o1 = q[N], o2 = q[2 * N], o3 = q[3 * N];
      q[0] = o0 + (float)(gw + ds * w);
      q[N] = o1 + (float)(gx + ds * x);
      q[2 * N] = o2 + (float)(gy + ds * y);
      q[3 * N] = o3 + (float)(gz + ds * z);
    }
  }
  if (A.g_scale) {
    const float o0 = A.g_scale[i], o1 = A.g_scale[N + i];
    A.g_scale[i] = o0 + (float)gsu;
    A.g_scale[N + i] = o1 + (float)gsv;
  }
  if (A.g_opacity) A.g_opacity[i] += (float)g_op;

  // colour from SH: view direction v = R^T mu_s (group frame), colour = max(0, sum c Y + 1/2)
  if constexpr (KIND != GS_SENSOR_LIDAR && DEG >= 0) {
    constexpr int nb = (DEG + 1) * (DEG + 1);
    if (gcol[0] != 0.0 || gcol[1] != 0.0 || gcol[2] != 0.0) {
      double v[3];
      for (int c = 0; c < 3; ++c) v[c] = R[c] * mus[0] + R[3 + c] * mus[1] + R[6 + c] * mus[2];
      const double vn = sqrt(dot3(v, v));
      const float dxf = (float)(v[0] / vn), dyf = (float)(v[1] / vn), dzf = (float)(v[2] / vn);
      float Y[16];
      sh_eval(DEG, dxf, dyf, dzf, Y);
      // every coefficient and every accumulator of the surfel, loaded before any store
      float co[3][nb], old[3][nb];
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int k = 0; k < nb; ++k) co[c][k] = a.sh[(size_t)(k * 3 + c) * N + i];
      if (A.g_sh) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
#pragma unroll
          for (int k = 0; k < nb; ++k) old[c][k] = A.g_sh[(size_t)(k * 3 + c) * N + i];
      }
      float gY[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) gY[k] = 0.0f;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if (gcol[c] == 0.0) continue;
        float raw = 0.5f;
#pragma unroll
        for (int k = 0; k < nb; ++k) raw += co[c][k] * Y[k];
        if (!(raw > 0.0f)) continue;
#pragma unroll
        for (int k = 0; k < nb; ++k) {
          if (A.g_sh) A.g_sh[(size_t)(k * 3 + c) * N + i] = old[c][k] + (float)(gcol[c] * Y[k]);
          gY[k] += (float)gcol[c] * co[c][k];
        }
      }
      float gxf, gyf, gzf;
      sh_grad(DEG, dxf, dyf, dzf, gY, gxf, gyf, gzf);
      const double gd[3] = {gxf, gyf, gzf};
      const double dd[3] = {v[0] / vn, v[1] / vn, v[2] / vn};
      const double pr = dot3(dd, gd);
      // v = mu - c_group, so dL/dmu gains the projected direction gradient
      for (int c = 0; c < 3; ++c) gmu[c] += (gd[c] - dd[c] * pr) / vn;
    }
  } else if constexpr (KIND != GS_SENSOR_LIDAR) {
    if (A.g_rgb) {
      const float o0 = A.g_rgb[i], o1 = A.g_rgb[N + i], o2 = A.g_rgb[2 * N + i];
      A.g_rgb[i] = o0 + (float)gcol[0];
      A.g_rgb[N + i] = o1 + (float)gcol[1];
      A.g_rgb[2 * N + i] = o2 + (float)gcol[2];
    }
  } else {
    if (A.g_intensity) A.g_intensity[i] += (float)g_int;
    if (A.g_drop) A.g_drop[i] += gf[15];  // the drop probability enters linearly
  }

  if (A.g_mean) {
    const float o0 = A.g_mean[i], o1 = A.g_mean[N + i], o2 = A.g_mean[2 * N + i];
    A.g_mean[i] = o0 + (float)gmu[0];
    A.g_mean[N + i] = o1 + (float)gmu[1];
    A.g_mean[2 * N + i] = o2 + (float)gmu[2];
  }
}

}  // namespace

template <int KIND>
void launch_kind(const SplatBwdArgs& a, hipStream_t st) {
  const dim3 grid((a.p.n + 255) / 256), block(256);
  if constexpr (KIND != GS_SENSOR_LIDAR) {
    switch (a.p.sh_degree) {
      case 0: hipLaunchKernelGGL((k_splat_backward<KIND, 0>), grid, block, 0, st, a); return;
      case 1: hipLaunchKernelGGL((k_splat_backward<KIND, 1>), grid, block, 0, st, a); return;
      case 2: hipLaunchKernelGGL((k_splat_backward<KIND, 2>), grid, block, 0, st, a); return;
      case 3: hipLaunchKernelGGL((k_splat_backward<KIND, 3>), grid, block, 0, st, a); return;
      default: break;
    }
  }
  hipLaunchKernelGGL((k_splat_backward<KIND, -1>), grid, block, 0, st, a);
}

void launch_splat_backward(const SplatBwdArgs& a, hipStream_t st) {
  if (a.p.n == 0) return;
  if (a.p.S.kind == GS_SENSOR_PINHOLE)
    launch_kind<GS_SENSOR_PINHOLE>(a, st);
  else if (a.p.S.kind == GS_SENSOR_CYLINDRICAL)
    launch_kind<GS_SENSOR_CYLINDRICAL>(a, st);
  else
    launch_kind<GS_SENSOR_LIDAR>(a, st);
}

}  // namespace gs
