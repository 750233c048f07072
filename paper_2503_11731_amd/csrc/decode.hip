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
//   heads    opacity / colour / intensity = sigmoid, scale = l_a sigmoid,
//            quaternion = raw, centre = x_a + l_a O_k; surfel n = a K + k.
// Adjoint: FP32 VALU with per-block partial weight gradients added by atomics.
#include <cstring>
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
  // adjoint inputs / outputs
  const float* gi_mean;
  const float* gi_quat;
  const float* gi_scale;
  const float* gi_opacity;
  const float* gi_rgb;
  const float* gi_intensity;
  float* g_xyz;
  float* g_scaling;
  float* g_offsets;
  float* g_feat;
  float* g_w1;
  float* g_b1;
  float* g_w2;
  float* g_b2;
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
#pragma unroll
    for (int e = 0; e < 3; ++e)
      a.mean[e * N + n] = a.xyz[(size_t)e * a.A + ai] + la * a.offsets[((size_t)e * K + k) * a.A + ai];
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
    for (int e = 0; e < 3; ++e)
      a.mean[e * N + n] = a.xyz[(size_t)e * a.A + ai] + la * a.offsets[((size_t)e * K + k) * a.A + ai];
  }
}

__global__ __launch_bounds__(256) void k_decode_bwd(DecodeArgs a) {
  __shared__ float sD[4][16][4];
  __shared__ float sH[4][16][kHidden + 1];
  __shared__ float sY[4][16][kMaxKJ + 1];  // raw y, then dL/dy in place
  __shared__ float sGH[4][16][kHidden + 1];
  __shared__ float sGA[4][16][8];           // per anchor: dL/d scaling, dL/d xyz (3), dL/d dir (3)
  __shared__ float sCam[3];
  int g, a0;
  block_group(a, blockIdx.x, g, a0);
  const int t = threadIdx.x;
  if (t == 0) group_camera(a, g, sCam);
  for (int q = t; q < 4 * 16 * 8; q += 256) (&sGA[0][0][0])[q] = 0.f;
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
    float gy[10];
    const float s0 = sigmoidf(y[0] + bb[0]);
    gy[0] = (a.gi_opacity ? a.gi_opacity[n] : 0.f) * s0 * (1.f - s0);
    int so;
    if (!a.lidar) {
      for (int e = 0; e < 3; ++e) {
        const float s = sigmoidf(y[1 + e] + bb[1 + e]);
        gy[1 + e] = (a.gi_rgb ? a.gi_rgb[e * N + n] : 0.f) * s * (1.f - s);
      }
      so = 4;
    } else {
      const float s = sigmoidf(y[1] + bb[1]);
      gy[1] = (a.gi_intensity ? a.gi_intensity[n] : 0.f) * s * (1.f - s);
      so = 2;
    }
    float gla = 0.f;
    for (int e = 0; e < 2; ++e) {
      const float s = sigmoidf(y[so + e] + bb[so + e]);
      const float gs = a.gi_scale ? a.gi_scale[e * N + n] : 0.f;
      gy[so + e] = gs * la * s * (1.f - s);
      gla += gs * s;
    }
    for (int e = 0; e < 4; ++e) gy[so + 2 + e] = a.gi_quat ? a.gi_quat[e * N + n] : 0.f;
    for (int j = 0; j < J; ++j) y[j] = gy[j];
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
  // dL/dh = dL/dy W2, masked by the ReLU
  const uint16_t* W2 = a.w2 + (size_t)g * KJ * kHidden;
  for (int q = c.lane; q < 16 * kHidden; q += 64) {
    const int al = q / kHidden, j = q % kHidden;
    float s = 0.f;
    if (sH[c.w][al][j] > 0.f) {
      for (int n = 0; n < KJ; ++n) s += sY[c.w][al][n] * bf2f(W2[(size_t)n * kHidden + j]);
    }
    sGH[c.w][al][j] = s;
  }
  __syncthreads();
  // dL/d features (written) and dL/d direction (to LDS)
  const uint16_t* W1 = a.w1 + (size_t)g * kHidden * kIn;
  for (int q = c.lane; q < 16 * kIn; q += 64) {
    const int al = q / kIn, k = q % kIn;
    const int ai = c.abase + al;
    float s = 0.f;
    for (int j = 0; j < kHidden; ++j) s += sGH[c.w][al][j] * bf2f(W1[j * kIn + k]);
    if (k < kFeat) {
      if (ai < c.aend && a.g_feat) a.g_feat[(size_t)ai * kFeat + k] += s;
    } else {
      sGA[c.w][al][4 + (k - kFeat)] = s;
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
  // weight gradients: partial sums over this block's anchors, one atomic per entry
  if (a.g_w2 || a.g_b2) {
    for (int q = t; q < KJ * (kHidden + 1); q += 256) {
      const int n = q / (kHidden + 1), j = q % (kHidden + 1);
      float s = 0.f;
      for (int w = 0; w < 4; ++w)
        for (int al = 0; al < 16; ++al) s += sY[w][al][n] * (j < kHidden ? sH[w][al][j] : 1.f);
      if (j < kHidden) {
        if (a.g_w2 && s != 0.f) atomicAdd(a.g_w2 + ((size_t)g * KJ + n) * kHidden + j, s);
      } else if (a.g_b2 && s != 0.f) {
        atomicAdd(a.g_b2 + (size_t)g * KJ + n, s);
      }
    }
  }
  if (a.g_w1 || a.g_b1) {
    for (int q = t; q < kHidden * (kIn + 1); q += 256) {
      const int j = q / (kIn + 1), k = q % (kIn + 1);
      float s = 0.f;
      for (int w = 0; w < 4; ++w) {
        for (int al = 0; al < 16; ++al) {
          const int ai = a0 + 16 * w + al;
          if (ai >= a.goff[g + 1]) break;
          float x;
          if (k < kFeat) x = bf2f(a.feat[(size_t)ai * kFeat + k]);
          else if (k < kIn) x = sD[w][al][k - kFeat];
          else x = 1.f;
          s += sGH[w][al][j] * x;
        }
      }
      if (k < kIn) {
        if (a.g_w1 && s != 0.f) atomicAdd(a.g_w1 + ((size_t)g * kHidden + j) * kIn + k, s);
      } else if (a.g_b1 && s != 0.f) {
        atomicAdd(a.g_b1 + (size_t)g * kHidden + j, s);
      }
    }
  }
}

}  // namespace

gs_status set_error(gs_status s, const std::string& msg);

}  // namespace gs

using namespace gs;

namespace {

gs_status fill_args(const gs_anchor_set* an, const float* sensor_pose, const float* group_poses, DecodeArgs& a,
                    int& nblocks) {
  if (!an || !sensor_pose || !group_poses) return set_error(GS_ERR_INVALID_ARG, "null decode argument");
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
  a.J = a.lidar ? 8 : 10;
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
  if (!out || !out->mean || !out->quat || !out->scale || !out->opacity || (!a.lidar && !out->rgb) ||
      (a.lidar && !out->intensity))
    return set_error(GS_ERR_INVALID_ARG, "null decode output");
  a.mean = out->mean;
  a.quat = out->quat;
  a.scale = out->scale;
  a.opacity = out->opacity;
  a.rgb = out->rgb;
  a.intensity = out->intensity;
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
  *bytes = 256;
  return set_error(GS_OK, "");
}

extern "C" gs_status gs_decode_backward(const gs_anchor_set* anchors, const float* sensor_pose,
                                        const float* group_poses, const gs_decoded* grad_in,
                                        const gs_anchor_grads* grads, void* scratch, hipStream_t stream) {
  (void)scratch;
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
  a.g_xyz = grads->xyz;
  a.g_scaling = grads->scaling;
  a.g_offsets = grads->offsets;
  a.g_feat = grads->feat;
  a.g_w1 = grads->w1;
  a.g_b1 = grads->b1;
  a.g_w2 = grads->w2;
  a.g_b2 = grads->b2;
  if (nb > 0) hipLaunchKernelGGL(k_decode_bwd, dim3(nb), dim3(256), 0, stream, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(GS_ERR_HIP, std::string("decode backward launch: ") + hipGetErrorString(e));
  return set_error(GS_OK, "");
}
