// a1 / a10: neural-Gaussian decode (Sec. III-A: surfel attributes inferred
// from each anchor's feature by the scene's MLP) and its adjoint.
//
// Forward, per wave of 16 anchors of one group (MLP):
//   layer 1  H = ReLU(F W1f^T + b1 + D W1d^T)   F: bf16 features [16 x 32] on
//            MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulate); the 3-wide
//            view-direction part D W1d^T is a rank-3 FP32 update.
//   layer 2  Y = H W2^T + b2 on MFMA; H enters as a bf16 hi + lo pair
//            (H ~ hi + lo to ~2^-17 relative) so that no activation is
//            quantised to 8 mantissa bits.
//   heads    opacity / colour / intensity / ray drop = sigmoid, scale = l_a sigmoid,
//            quaternion = raw, centre = x_a + l_a O_k; surfel n = a K + k.
// Adjoint: FP32 MFMA contractions; per-block partial weight gradients summed
// in a fixed order by a second kernel.
#include <cstdint>
#include <cstring>
#include <mutex>
#include <string>

#include "gs_internal.h"
#include "kernels.h"

namespace gs {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kFeat = 32;
constexpr int kHidden = 32;
constexpr int kIn = kFeat + 3;
constexpr int kMaxKJ = 160;
constexpr int kAnchorsPerBlock = 64;

struct DecodeArgs {
  int A, K, J, lidar, n_groups;
  int goff[kMaxGroups + 1];
  int bstart[kMaxGroups + 1];
  const float* xyz;
  const float* scaling;
  const float* offsets;
  const uint16_t* feat;
  const uint16_t* w1;
  const float* b1;
  const uint16_t* w2;
  const float* b2;
  const float* sensor_pose;
  const float* group_poses;
  // forward outputs
  float* mean;
  float* quat;
  float* scale;
  float* opacity;
  float* rgb;
  float* intensity;
  float* drop;  // LiDAR ray-drop probability
  // adjoint inputs / outputs
  const float* gi_mean;
  const float* gi_quat;
  const float* gi_scale;
  const float* gi_opacity;
  const float* gi_rgb;
  const float* gi_intensity;
  const float* gi_drop;
  float* g_xyz;
  float* g_scaling;
  float* g_offsets;
  float* g_feat;
  float* g_w1;
  float* g_b1;
  float* g_w2;
  float* g_b2;
  float* part;  // per-block weight-gradient partials [blocks][w2 | b2 | w1 | b1]
};

__device__ inline uint16_t f2bf(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

union BF8 {
  uint16_t u[8];
  uint4 q;
  bf16x8 v;
};

__device__ inline float sigmoidf(float x) { return 1.0f / (1.0f + __expf(-x)); }

__device__ inline void block_group(const DecodeArgs& a, int b, int& g, int& a0) {
  int lo = 0, hi = a.n_groups - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (a.bstart[mid] <= b) lo = mid; else hi = mid - 1;
  }
  g = lo;
  a0 = a.goff[g] + (b - a.bstart[g]) * kAnchorsPerBlock;
}

// sensor centre in the group's frame from the FP32 composed pose V_s G_g
__device__ inline void group_camera(const DecodeArgs& a, int g, float* cam) {
#pragma clang fp contract(off)
  const float* A = a.sensor_pose;
  const float* B = a.group_poses + 12 * g;
  float P[12];
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) P[4 * i + j] = (A[4 * i] * B[j] + A[4 * i + 1] * B[4 + j]) + A[4 * i + 2] * B[8 + j];
    P[4 * i + 3] = ((A[4 * i] * B[3] + A[4 * i + 1] * B[7]) + A[4 * i + 2] * B[11]) + A[4 * i + 3];
  }
  for (int c = 0; c < 3; ++c)
    cam[c] = (float)(-((double)P[c] * P[3] + (double)P[4 + c] * P[7] + (double)P[8 + c] * P[11]));
}

struct WaveCtx {
  int g, abase, aend, row, kg, lane, w;
};

// Layers 1 and 2 for the wave's 16 anchors; leaves D (directions, |v|), H and
// Y (without b2) in LDS.
__device__ inline void forward_layers(const DecodeArgs& a, const WaveCtx& c, const float* cam, float (*sD)[4],
                                      float (*sH)[kHidden + 1], float (*sY)[kMaxKJ + 1]) {
  if (c.lane < 16) {
    const int ai = c.abase + c.lane;
    float d[4] = {0.f, 0.f, 0.f, 1.f};
    if (ai < c.aend) {
      const double v0 = (double)a.xyz[ai] - cam[0];
      const double v1 = (double)a.xyz[a.A + ai] - cam[1];
      const double v2 = (double)a.xyz[2 * a.A + ai] - cam[2];
      const double n = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
      d[0] = (float)(v0 / n);
      d[1] = (float)(v1 / n);
      d[2] = (float)(v2 / n);
      d[3] = (float)n;
    }
    for (int k = 0; k < 4; ++k) sD[c.lane][k] = d[k];
  }
  __syncthreads();
  const int ai = c.abase + c.row;
  BF8 A1;
  if (ai < c.aend) {
    A1.q = *reinterpret_cast<const uint4*>(a.feat + (size_t)ai * kFeat + 8 * c.kg);
  } else {
    A1.q = make_uint4(0, 0, 0, 0);
  }
  const uint16_t* W1 = a.w1 + (size_t)c.g * kHidden * kIn;
  const float* B1 = a.b1 + (size_t)c.g * kHidden;
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int j = 16 * t + c.row;
    BF8 Bf;
#pragma unroll
    for (int i = 0; i < 8; ++i) Bf.u[i] = W1[j * kIn + 8 * c.kg + i];
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A1.v, Bf.v, acc, 0, 0, 0);
    const float wd0 = bf2f(W1[j * kIn + 32]), wd1 = bf2f(W1[j * kIn + 33]), wd2 = bf2f(W1[j * kIn + 34]);
    const float bj = B1[j];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int ar = 4 * c.kg + i;
      float v = acc[i] + bj + wd0 * sD[ar][0] + wd1 * sD[ar][1] + wd2 * sD[ar][2];
      sH[ar][j] = v > 0.f ? v : 0.f;
    }
  }
  __syncthreads();
  BF8 Ahi, Alo;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const float h = sH[c.row][8 * c.kg + i];
    const uint16_t hi = f2bf(h);
    Ahi.u[i] = hi;
    Alo.u[i] = f2bf(h - bf2f(hi));
  }
  const int KJ = a.K * a.J;
  const uint16_t* W2 = a.w2 + (size_t)c.g * KJ * kHidden;
  for (int t = 0; t * 16 < KJ; ++t) {
    const int n = 16 * t + c.row;
    BF8 Bf;
    if (n < KJ) {
      Bf.q = *reinterpret_cast<const uint4*>(W2 + (size_t)n * kHidden + 8 * c.kg);
    } else {
      Bf.q = make_uint4(0, 0, 0, 0);
    }
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Ahi.v, Bf.v, acc, 0, 0, 0);
    acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Alo.v, Bf.v, acc, 0, 0, 0);
    if (n < KJ) {
#pragma unroll
      for (int i = 0; i < 4; ++i) sY[4 * c.kg + i][n] = acc[i];
    }
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_decode_fwd(DecodeArgs a) {
  __shared__ float sD[4][16][4];
  __shared__ float sH[4][16][kHidden + 1];
  __shared__ float sY[4][16][kMaxKJ + 1];
  __shared__ float sCam[3];
  int g, a0;
  block_group(a, blockIdx.x, g, a0);
  const int t = threadIdx.x;
  if (t == 0) group_camera(a, g, sCam);
  __syncthreads();
  WaveCtx c;
  c.g = g;
  c.w = t >> 6;
  c.lane = t & 63;
  c.row = c.lane & 15;
  c.kg = c.lane >> 4;
  c.abase = a0 + 16 * c.w;
  c.aend = a.goff[g + 1];
  const float cam[3] = {sCam[0], sCam[1], sCam[2]};
  forward_layers(a, c, cam, sD[c.w], sH[c.w], sY[c.w]);
  const int K = a.K, J = a.J, KJ = K * J;
  const size_t N = (size_t)a.A * K;
  const float* B2 = a.b2 + (size_t)g * KJ;
  for (int q = c.lane; q < 16 * K; q += 64) {
    const int al = q / K, k = q % K;
    const int ai = c.abase + al;
    if (ai >= c.aend) continue;
    const size_t n = (size_t)ai * K + k;
    const float* y = &sY[c.w][al][k * J];
    const float* bb = B2 + k * J;
    const float la = a.scaling[ai];
    a.opacity[n] = sigmoidf(y[0] + bb[0]);
    int so;
    if (!a.lidar) {
      a.rgb[n] = sigmoidf(y[1] + bb[1]);
      a.rgb[N + n] = sigmoidf(y[2] + bb[2]);
      a.rgb[2 * N + n] = sigmoidf(y[3] + bb[3]);
      so = 4;
    } else {
      a.intensity[n] = sigmoidf(y[1] + bb[1]);
      so = 2;
    }
    a.scale[n] = la * sigmoidf(y[so] + bb[so]);
    a.scale[N + n] = la * sigmoidf(y[so + 1] + bb[so + 1]);
#pragma unroll
    for (int e = 0; e < 4; ++e) a.quat[e * N + n] = y[so + 2 + e] + bb[so + 2 + e];
    if (a.lidar) a.drop[n] = sigmoidf(y[8] + bb[8]);
    if (a.mean) {
#pragma unroll
      for (int e = 0; e < 3; ++e)
        a.mean[e * N + n] = a.xyz[(size_t)e * a.A + ai] + la * a.offsets[((size_t)e * K + k) * a.A + ai];
    }
  }
}

// Plain FP32 decode: one thread per anchor, weights widened from bf16, every
// activation in FP32 (the comparison point for the MFMA decode).
__global__ __launch_bounds__(128) void k_decode_fwd_valu(DecodeArgs a) {
  __shared__ float sCam[kMaxGroups][3];
  if (threadIdx.x < a.n_groups) group_camera(a, threadIdx.x, sCam[threadIdx.x]);
  __syncthreads();
  const int ai = blockIdx.x * 128 + threadIdx.x;
  if (ai >= a.A) return;
  int g = 0;
  while (g + 1 < a.n_groups && a.goff[g + 1] <= ai) ++g;
  float x[kIn];
  for (int k = 0; k < kFeat; ++k) x[k] = bf2f(a.feat[(size_t)ai * kFeat + k]);
  const double v0 = (double)a.xyz[ai] - sCam[g][0];
  const double v1 = (double)a.xyz[a.A + ai] - sCam[g][1];
  const double v2 = (double)a.xyz[2 * a.A + ai] - sCam[g][2];
  const double nv = sqrt(v0 * v0 + v1 * v1 + v2 * v2);
  x[kFeat] = (float)(v0 / nv);
  x[kFeat + 1] = (float)(v1 / nv);
  x[kFeat + 2] = (float)(v2 / nv);
  const uint16_t* W1 = a.w1 + (size_t)g * kHidden * kIn;
  const float* B1 = a.b1 + (size_t)g * kHidden;
  float h[kHidden];
  for (int j = 0; j < kHidden; ++j) {
    float s = B1[j];
    for (int k = 0; k < kIn; ++k) s = fmaf(bf2f(W1[j * kIn + k]), x[k], s);
    h[j] = s > 0.f ? s : 0.f;
  }
  const int K = a.K, J = a.J, KJ = K * J;
  const uint16_t* W2 = a.w2 + (size_t)g * KJ * kHidden;
  const float* B2 = a.b2 + (size_t)g * KJ;
  const size_t N = (size_t)a.A * K;
  const float la = a.scaling[ai];
  for (int k = 0; k < K; ++k) {
    float y[10];
    for (int j = 0; j < J; ++j) {
      const int n = k * J + j;
      float s = B2[n];
      for (int q = 0; q < kHidden; ++q) s = fmaf(bf2f(W2[(size_t)n * kHidden + q]), h[q], s);
      y[j] = s;
    }
    const size_t n = (size_t)ai * K + k;
    a.opacity[n] = sigmoidf(y[0]);
    int so;
    if (!a.lidar) {
      a.rgb[n] = sigmoidf(y[1]);
      a.rgb[N + n] = sigmoidf(y[2]);
      a.rgb[2 * N + n] = sigmoidf(y[3]);
      so = 4;
    } else {
      a.intensity[n] = sigmoidf(y[1]);
      so = 2;
    }
    a.scale[n] = la * sigmoidf(y[so]);
    a.scale[N + n] = la * sigmoidf(y[so + 1]);
    for (int e = 0; e < 4; ++e) a.quat[e * N + n] = y[so + 2 + e];
    if (a.lidar) a.drop[n] = sigmoidf(y[8]);
    if (a.mean)
      for (int e = 0; e < 3; ++e)
        a.mean[e * N + n] = a.xyz[(size_t)e * a.A + ai] + la * a.offsets[((size_t)e * K + k) * a.A + ai];
  }
}

// dL/dy of one surfel's heads, written over its raw outputs y[0..J); returns
// the surfel's share of dL/d l_a through its two scale heads.
template <bool LIDAR>
__device__ inline float heads_adjoint(const DecodeArgs& a, float* y, const float* bb, size_t n, size_t N, float la) {
  constexpr int so = LIDAR ? 2 : 4;
  constexpr int J = LIDAR ? 9 : 10;
  float gy[J];
  const float s0 = sigmoidf(y[0] + bb[0]);
  gy[0] = (a.gi_opacity ? a.gi_opacity[n] : 0.f) * s0 * (1.f - s0);
  if (!LIDAR) {
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      const float s = sigmoidf(y[1 + e] + bb[1 + e]);
      gy[1 + e] = (a.gi_rgb ? a.gi_rgb[e * N + n] : 0.f) * s * (1.f - s);
    }
  } else {
    const float s = sigmoidf(y[1] + bb[1]);
    gy[1] = (a.gi_intensity ? a.gi_intensity[n] : 0.f) * s * (1.f - s);
  }
  float gla = 0.f;
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    const float s = sigmoidf(y[so + e] + bb[so + e]);
    const float gs = a.gi_scale ? a.gi_scale[e * N + n] : 0.f;
    gy[so + e] = gs * la * s * (1.f - s);
    gla += gs * s;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e) gy[so + 2 + e] = a.gi_quat ? a.gi_quat[e * N + n] : 0.f;
  if (LIDAR) {  // ray-drop head
    const float s = sigmoidf(y[8] + bb[8]);
    gy[J - 1] = (a.gi_drop ? a.gi_drop[n] : 0.f) * s * (1.f - s);
  }
#pragma unroll
  for (int j = 0; j < J; ++j) y[j] = gy[j];
  return gla;
}

__device__ inline f32x4 mfma_f32(float x, float y, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(x, y, c, 0, 0, 0);
}

constexpr int kW1Cols = 48;  // W1 row in LDS: kIn columns, zero to three whole 16-column tiles

// Adjoint, per block of 64 anchors of one group (4 waves x 16).  After the
// forward layers and the heads adjoint (dL/dy in place of y), the four
// contractions of the MLP adjoint run on FP32 MFMA (v_mfma_f32_16x16x4_f32;
// lane l holds A[l%16][l/16], B[l/16][l%16], D[4(l/16)+r][l%16]):
//   dH  = dY W2, ReLU-masked    per wave: 16 anchors x 32 hidden, over K*J
//   dX  = dH W1                 per wave: 16 anchors x 35 (features, direction)
//   dW2 = dY^T H, dW1 = dH^T X  per block: summed over its 64 anchors
// Weights are staged in LDS as bf16 bits; each block writes its weight-gradient
// partials to the scratch buffer, summed per group by k_decode_wsum.
__global__ __launch_bounds__(256) void k_decode_bwd(DecodeArgs a) {
  __shared__ float sD[4][16][4];
  __shared__ float sH[4][16][kHidden + 1];
  __shared__ float sY[4][16][kMaxKJ + 1];  // raw y, then dL/dy in place
  __shared__ float sGH[4][16][kHidden + 1];
  __shared__ float sGA[4][16][8];           // per anchor: dL/d scaling, dL/d xyz (3), dL/d dir (3)
  __shared__ float sCam[3];
  __shared__ uint16_t sW1[kHidden][kW1Cols];
  __shared__ __attribute__((aligned(16))) union {
    uint16_t w2[kMaxKJ][kHidden + 2];  // W2 rows, for dH
    uint16_t x[64][kFeat + 8];          // the block's features, for dW1
  } sU;
  int g, a0;
  block_group(a, blockIdx.x, g, a0);
  const int t = threadIdx.x;
  const int KJ = a.K * a.J;
  float* part = a.part + (size_t)blockIdx.x * (KJ * (kHidden + 1) + kHidden * (kIn + 1));
  if (t == 0) group_camera(a, g, sCam);
  for (int q = t; q < 4 * 16 * 8; q += 256) (&sGA[0][0][0])[q] = 0.f;
  const uint16_t* W2 = a.w2 + (size_t)g * KJ * kHidden;
  const uint16_t* W1 = a.w1 + (size_t)g * kHidden * kIn;
  for (int q = t; q < KJ * 4; q += 256) {
    const int n = q >> 2, p = q & 3;
    const uint4 v = *reinterpret_cast<const uint4*>(W2 + (size_t)n * kHidden + 8 * p);
    uint32_t* d = reinterpret_cast<uint32_t*>(&sU.w2[n][8 * p]);
    d[0] = v.x;
    d[1] = v.y;
    d[2] = v.z;
    d[3] = v.w;
  }
  for (int q = t; q < kHidden * kW1Cols; q += 256) {
    const int j = q / kW1Cols, k = q % kW1Cols;
    sW1[j][k] = k < kIn ? W1[j * kIn + k] : (uint16_t)0;
  }
  // one 16-byte piece of the block's features per thread, held until the W2 area is free
  uint4 xf = make_uint4(0, 0, 0, 0);
  if (a0 + (t >> 2) < a.goff[g + 1])
    xf = *reinterpret_cast<const uint4*>(a.feat + (size_t)(a0 + (t >> 2)) * kFeat + 8 * (t & 3));
  __syncthreads();
  WaveCtx c;
  c.g = g;
  c.w = t >> 6;
  c.lane = t & 63;
  c.row = c.lane & 15;
  c.kg = c.lane >> 4;
  c.abase = a0 + 16 * c.w;
  c.aend = a.goff[g + 1];
  const float cam[3] = {sCam[0], sCam[1], sCam[2]};
  forward_layers(a, c, cam, sD[c.w], sH[c.w], sY[c.w]);
  const int K = a.K, J = a.J;
  const size_t N = (size_t)a.A * K;
  const float* B2 = a.b2 + (size_t)g * KJ;
  // heads adjoint, in place: sY <- dL/dy; per-anchor sums through LDS atomics
  for (int q = c.lane; q < 16 * K; q += 64) {
    const int al = q / K, k = q % K;
    const int ai = c.abase + al;
    float* y = &sY[c.w][al][k * J];
    if (ai >= c.aend) {
      for (int j = 0; j < J; ++j) y[j] = 0.f;
      continue;
    }
    const size_t n = (size_t)ai * K + k;
    const float* bb = B2 + k * J;
    const float la = a.scaling[ai];
    float gla = a.lidar ? heads_adjoint<true>(a, y, bb, n, N, la) : heads_adjoint<false>(a, y, bb, n, N, la);
    if (a.gi_mean) {
      for (int e = 0; e < 3; ++e) {
        const float gm = a.gi_mean[e * N + n];
        const float off = a.offsets[((size_t)e * K + k) * a.A + ai];
        gla += gm * off;
        atomicAdd(&sGA[c.w][al][1 + e], gm);
        if (a.g_offsets) a.g_offsets[((size_t)e * K + k) * a.A + ai] += gm * la;
      }
    }
    atomicAdd(&sGA[c.w][al][0], gla);
  }
  __syncthreads();
  const int r16 = c.lane & 15, k4 = c.lane >> 4;
  // dL/dh = dL/dy W2, masked by the ReLU
  {
    f32x4 acc0 = {0.f, 0.f, 0.f, 0.f}, acc1 = {0.f, 0.f, 0.f, 0.f};
    for (int n0 = 0; n0 < KJ; n0 += 4) {
      const int n = n0 + k4;
      const bool ok = n < KJ;
      const int nc = ok ? n : 0;
      const float av = ok ? sY[c.w][r16][nc] : 0.f;
      const float b0 = ok ? bf2f(sU.w2[nc][r16]) : 0.f;
      const float b1 = ok ? bf2f(sU.w2[nc][16 + r16]) : 0.f;
      acc0 = mfma_f32(av, b0, acc0);
      acc1 = mfma_f32(av, b1, acc1);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int al = 4 * k4 + i;
      sGH[c.w][al][r16] = sH[c.w][al][r16] > 0.f ? acc0[i] : 0.f;
      sGH[c.w][al][16 + r16] = sH[c.w][al][16 + r16] > 0.f ? acc1[i] : 0.f;
    }
  }
  __syncthreads();
  *reinterpret_cast<uint4*>(&sU.x[t >> 2][8 * (t & 3)]) = xf;
  // dL/d features (written) and dL/d direction (to LDS): dL/dh W1
  {
    f32x4 acc[3];
#pragma unroll
    for (int ct = 0; ct < 3; ++ct) acc[ct] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int j0 = 0; j0 < kHidden; j0 += 4) {
      const int j = j0 + k4;
      const float av = sGH[c.w][r16][j];
#pragma unroll
      for (int ct = 0; ct < 3; ++ct) acc[ct] = mfma_f32(av, bf2f(sW1[j][16 * ct + r16]), acc[ct]);
    }
#pragma unroll
    for (int ct = 0; ct < 3; ++ct) {
      const int col = 16 * ct + r16;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int al = 4 * k4 + i, ai = c.abase + al;
        if (col < kFeat) {
          if (ai < c.aend && a.g_feat) a.g_feat[(size_t)ai * kFeat + col] += acc[ct][i];
        } else if (col < kIn) {
          sGA[c.w][al][4 + (col - kFeat)] = acc[ct][i];
        }
      }
    }
  }
  __syncthreads();
  if (c.lane < 16) {
    const int al = c.lane, ai = c.abase + al;
    if (ai < c.aend) {
      const float* d = sD[c.w][al];
      const float* gd = &sGA[c.w][al][4];
      const float pr = d[0] * gd[0] + d[1] * gd[1] + d[2] * gd[2];
      if (a.g_xyz)
        for (int e = 0; e < 3; ++e)
          a.g_xyz[(size_t)e * a.A + ai] += sGA[c.w][al][1 + e] + (gd[e] - d[e] * pr) / d[3];
      if (a.g_scaling) a.g_scaling[ai] += sGA[c.w][al][0];
    }
  }
  // weight gradients over the block's 64 anchors (rows of invalid anchors are
  // zero in dY and dH): 16x16 tiles of dW2 (rows n of K*J, columns j) and of
  // dW1 (rows j, columns k of features + direction), shared out over the waves
  const int nt2 = a.g_w2 ? 2 * ((KJ + 15) >> 4) : 0;
  const int nt1 = a.g_w1 ? 6 : 0;
  for (int tile = c.w; tile < nt2 + nt1; tile += 4) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    if (tile < nt2) {
      const int n0 = 16 * (tile >> 1), j0 = 16 * (tile & 1);
#pragma unroll 4
      for (int s = 0; s < 16; ++s) {
        const int an = 4 * s + k4;
        acc = mfma_f32(sY[an >> 4][an & 15][n0 + r16], sH[an >> 4][an & 15][j0 + r16], acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int n = n0 + 4 * k4 + i;
        if (n < KJ) part[n * kHidden + j0 + r16] = acc[i];
      }
    } else {
      const int u = tile - nt2;
      const int j0 = 16 * (u & 1), col = 16 * (u >> 1) + r16;
#pragma unroll 4
      for (int s = 0; s < 16; ++s) {
        const int an = 4 * s + k4;
        float bv = 0.f;
        if (col < kFeat) bv = bf2f(sU.x[an][col]);
        else if (col < kIn) bv = sD[an >> 4][an & 15][col - kFeat];
        acc = mfma_f32(sGH[an >> 4][an & 15][j0 + r16], bv, acc);
      }
      if (col < kIn) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int j = j0 + 4 * k4 + i;
          part[KJ * (kHidden + 1) + j * kIn + col] = acc[i];
        }
      }
    }
  }
  if (a.g_b2 && t < KJ) {
    float s = 0.f;
    for (int an = 0; an < 64; ++an) s += sY[an >> 4][an & 15][t];
    part[KJ * kHidden + t] = s;
  }
  if (a.g_b1 && t >= 192 && t < 192 + kHidden) {
    float s = 0.f;
    for (int an = 0; an < 64; ++an) s += sGH[an >> 4][an & 15][t - 192];
    part[KJ * (kHidden + 1) + kHidden * kIn + (t - 192)] = s;
  }
}

// Weight-gradient sums: for group g and partial entry e, the sum over the
// group's blocks of part[b][e] (16 slices of the block range per entry, then
// an LDS sum in slice order), added once to the gradient buffer.  Fixed
// order: the weight gradients are deterministic.
__global__ __launch_bounds__(1024) void k_decode_wsum(DecodeArgs a) {
  __shared__ float s_acc[16][65];
  const int g = blockIdx.y;
  const int KJ = a.K * a.J;
  const int PW = KJ * (kHidden + 1) + kHidden * (kIn + 1);
  const int le = threadIdx.x & 63, sl = threadIdx.x >> 6;
  const int e = blockIdx.x * 64 + le;
  const int b0 = a.bstart[g], b1 = a.bstart[g + 1];
  float acc = 0.f;
  if (e < PW) {
    int b = b0 + sl;
#pragma unroll 4
    for (; b < b1; b += 16) acc += a.part[(size_t)b * PW + e];
  }
  s_acc[sl][le] = acc;
  __syncthreads();
  if (sl != 0 || e >= PW) return;
  float s = 0.f;
#pragma unroll
  for (int k = 0; k < 16; ++k) s += s_acc[k][le];
  if (e < KJ * kHidden) {
    if (a.g_w2) a.g_w2[(size_t)g * KJ * kHidden + e] += s;
  } else if (e < KJ * (kHidden + 1)) {
    if (a.g_b2) a.g_b2[(size_t)g * KJ + (e - KJ * kHidden)] += s;
  } else if (e < KJ * (kHidden + 1) + kHidden * kIn) {
    if (a.g_w1) a.g_w1[(size_t)g * kHidden * kIn + (e - KJ * (kHidden + 1))] += s;
  } else {
    if (a.g_b1) a.g_b1[(size_t)g * kHidden + (e - KJ * (kHidden + 1) - kHidden * kIn)] += s;
  }
}

}  // namespace

gs_status set_error(gs_status s, const std::string& msg);

}  // namespace gs

using namespace gs;

namespace {

gs_status fill_args(const gs_anchor_set* an, const float* sensor_pose, const float* group_poses, DecodeArgs& a,
                    int& nblocks, bool need_poses = true) {
  if (!an || (need_poses && (!sensor_pose || !group_poses))) return set_error(GS_ERR_INVALID_ARG, "null decode argument");
  if (an->n_anchors < 0 || an->k < 1 || an->k > 16 || an->n_groups < 1 || an->n_groups > kMaxGroups ||
      !an->group_offsets)
    return set_error(GS_ERR_INVALID_ARG, "bad anchor set shape");
  if (an->n_anchors > 0 && (!an->xyz || !an->scaling || !an->offsets || !an->feat || !an->w1 || !an->b1 || !an->w2 ||
                            !an->b2))
    return set_error(GS_ERR_INVALID_ARG, "null anchor set array");
  if ((reinterpret_cast<uintptr_t>(an->feat) | reinterpret_cast<uintptr_t>(an->w2)) % 16 != 0)
    return set_error(GS_ERR_INVALID_ARG, "feat and w2 must be 16-byte aligned");
  memset(&a, 0, sizeof(a));
  a.A = an->n_anchors;
  a.K = an->k;
  a.lidar = an->lidar ? 1 : 0;
  a.J = a.lidar ? 9 : 10;
  a.n_groups = an->n_groups;
  int nb = 0;
  for (int g = 0; g <= an->n_groups; ++g) {
    a.goff[g] = an->group_offsets[g];
    if (g > 0 && a.goff[g] < a.goff[g - 1]) return set_error(GS_ERR_INVALID_ARG, "anchor group offsets must rise");
  }
  if (a.goff[0] != 0 || a.goff[an->n_groups] != an->n_anchors)
    return set_error(GS_ERR_INVALID_ARG, "anchor group offsets must span [0, A]");
  for (int g = 0; g < an->n_groups; ++g) {
    a.bstart[g] = nb;
    nb += (a.goff[g + 1] - a.goff[g] + kAnchorsPerBlock - 1) / kAnchorsPerBlock;
  }
  a.bstart[an->n_groups] = nb;
  nblocks = nb;
  a.xyz = an->xyz;
  a.scaling = an->scaling;
  a.offsets = an->offsets;
  a.feat = an->feat;
  a.w1 = an->w1;
  a.b1 = an->b1;
  a.w2 = an->w2;
  a.b2 = an->b2;
  a.sensor_pose = sensor_pose;
  a.group_poses = group_poses;
  return GS_OK;
}

}  // namespace

extern "C" gs_status gs_decode_forward(const gs_anchor_set* anchors, const float* sensor_pose, const float* group_poses,
                                       const gs_decoded* out, hipStream_t stream) {
  DecodeArgs a;
  int nb = 0;
  gs_status s = fill_args(anchors, sensor_pose, group_poses, a, nb);
  if (s != GS_OK) return s;
  if (!out || !out->quat || !out->scale || !out->opacity || (!a.lidar && !out->rgb) ||
      (a.lidar && (!out->intensity || !out->drop)))
    return set_error(GS_ERR_INVALID_ARG, "null decode output");
  a.mean = out->mean;
  a.quat = out->quat;
  a.scale = out->scale;
  a.opacity = out->opacity;
  a.rgb = out->rgb;
  a.intensity = out->intensity;
  a.drop = out->drop;
  if (anchors->flags & GS_DECODE_VALU_FP32) {
    if (a.A > 0) hipLaunchKernelGGL(k_decode_fwd_valu, dim3((a.A + 127) / 128), dim3(128), 0, stream, a);
  } else if (nb > 0) {
    hipLaunchKernelGGL(k_decode_fwd, dim3(nb), dim3(256), 0, stream, a);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(GS_ERR_HIP, std::string("decode launch: ") + hipGetErrorString(e));
  return set_error(GS_OK, "");
}

extern "C" gs_status gs_decode_scratch_size(const gs_anchor_set* anchors, size_t* bytes) {
  if (!anchors || !bytes) return set_error(GS_ERR_INVALID_ARG, "null argument");
  DecodeArgs a;
  int nb = 0;
  const gs_status s = fill_args(anchors, nullptr, nullptr, a, nb, false);
  if (s != GS_OK) return s;
  const size_t pw = (size_t)a.K * a.J * (kHidden + 1) + (size_t)kHidden * (kIn + 1);
  *bytes = nb > 0 ? (size_t)nb * pw * sizeof(float) : 256;
  return set_error(GS_OK, "");
}

// Scratch of the allocation-free decode adjoint: the per-block weight-gradient
// partials, in a file-scope device array (one copy per GPU, held until the
// process ends).  Host code never passes `scratch` itself to a kernel -- in
// host code the name is a stand-in, not a device address -- but the address
// hipGetSymbolAddress returns for the current device.  Every entry the sum
// kernel reads is written by the same call first, so nothing is cleared.
static __device__ __align__(256) float scratch[GS_DECODE_NOALLOC_SCRATCH_BYTES / sizeof(float)];

namespace {

gs_status decode_backward_impl(const gs_anchor_set* anchors, const float* sensor_pose, const float* group_poses,
                               const gs_decoded* grad_in, const gs_anchor_grads* grads, void* scratch,
                               size_t scratch_cap, hipStream_t stream, bool check_only = false) {
  DecodeArgs a;
  int nb = 0;
  gs_status s = fill_args(anchors, sensor_pose, group_poses, a, nb);
  if (s != GS_OK) return s;
  if (!grad_in || !grads) return set_error(GS_ERR_INVALID_ARG, "null decode gradient argument");
  a.gi_mean = grad_in->mean;
  a.gi_quat = grad_in->quat;
  a.gi_scale = grad_in->scale;
  a.gi_opacity = grad_in->opacity;
  a.gi_rgb = grad_in->rgb;
  a.gi_intensity = grad_in->intensity;
  a.gi_drop = grad_in->drop;
  a.g_xyz = grads->xyz;
  a.g_scaling = grads->scaling;
  a.g_offsets = grads->offsets;
  a.g_feat = grads->feat;
  a.g_w1 = grads->w1;
  a.g_b1 = grads->b1;
  a.g_w2 = grads->w2;
  a.g_b2 = grads->b2;
  const bool weights = a.g_w1 || a.g_b1 || a.g_w2 || a.g_b2;
  const int pw = a.K * a.J * (kHidden + 1) + kHidden * (kIn + 1);
  if (nb > 0 && weights && (size_t)nb * pw * sizeof(float) > scratch_cap)
    return set_error(GS_ERR_INVALID_ARG, "decode backward: the weight-gradient partials of " + std::to_string(nb) +
                                             " anchor blocks need " +
                                             std::to_string((size_t)nb * pw * sizeof(float)) +
                                             " bytes, more than the scratch buffer's " + std::to_string(scratch_cap));
  if (check_only) return GS_OK;
  if (nb > 0 && weights && !scratch)
    return set_error(GS_ERR_INVALID_ARG, "decode backward needs its scratch buffer for weight gradients");
  a.part = static_cast<float*>(scratch);
  if (nb > 0) hipLaunchKernelGGL(k_decode_bwd, dim3(nb), dim3(256), 0, stream, a);
  if (nb > 0 && weights)
    hipLaunchKernelGGL(k_decode_wsum, dim3((pw + 63) / 64, a.n_groups), dim3(1024), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(GS_ERR_HIP, std::string("decode backward launch: ") + hipGetErrorString(e));
  return set_error(GS_OK, "");
}

constexpr size_t kNoAllocScratchBytes = GS_DECODE_NOALLOC_SCRATCH_BYTES;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

gs_status noalloc_scratch(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(GS_ERR_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return set_error(GS_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(GS_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return GS_OK;
}

}  // namespace

extern "C" gs_status gs_decode_backward(const gs_anchor_set* anchors, const float* sensor_pose,
                                        const float* group_poses, const gs_decoded* grad_in,
                                        const gs_anchor_grads* grads, void* scratch, hipStream_t stream) {
  return decode_backward_impl(anchors, sensor_pose, group_poses, grad_in, grads, scratch, SIZE_MAX, stream);
}

extern "C" gs_status gs_decode_backward_noalloc(const gs_anchor_set* anchors, const float* sensor_pose,
                                                const float* group_poses, const gs_decoded* grad_in,
                                                const gs_anchor_grads* grads, hipStream_t stream) {
  // arguments and size first (host only), then the array's address on this device
  const gs_status v = decode_backward_impl(anchors, sensor_pose, group_poses, grad_in, grads, nullptr,
                                           kNoAllocScratchBytes, stream, /*check_only=*/true);
  if (v != GS_OK) return v;
  void* p = nullptr;
  const gs_status s = noalloc_scratch(&p);
  if (s != GS_OK) return s;
  return decode_backward_impl(anchors, sensor_pose, group_poses, grad_in, grads, p, kNoAllocScratchBytes, stream);
}
