// Inpainting patch affinity (Sec. III-B, Eq. 6): for every (target, source)
// patch pair, the softmax over the source anchors of X_T X_S^T, X holding one
// encoded anchor per row (feature + positional encoding, bf16).
//
// One workgroup per 128 target rows of one pair (8 waves of 16 rows).  The
// wave keeps its 16 x d slice of X_T in registers as MFMA operands and walks
// the source anchors 64 at a time, staged in LDS once per workgroup (four
// v_mfma_f32_16x16x32_bf16 tiles, FP32 accumulate): a first sweep keeps a running
// row maximum and exponential sum per lane, the four lanes that share a row
// merge theirs, and a second sweep recomputes the logit tiles and writes
// exp(z - max) / sum, 16 bytes per lane and store.  The
// output (4 bytes per entry) dominates the traffic; recomputing the logits
// costs MFMA time that is far below the write time.
#include <cfloat>
#include <string>

#include "gs_internal.h"
#include "kernels.h"

namespace gs {

gs_status set_error(gs_status s, const std::string& msg);

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kAffWaves = 8;  // waves (16 target rows each) per workgroup

union Bf8 {
  uint4 q;
  bf16x8 v;
};

template <int KS, int NW>  // d = 32 KS; NW waves of 16 target rows
__global__ __launch_bounds__(64 * NW) void k_affinity(const uint16_t* __restrict__ xt, const uint16_t* __restrict__ xs,
                                                   int p, int q, float* __restrict__ out, bool vec) {
  constexpr int D = 32 * KS;
  constexpr int RS = D + 8;  // LDS row stride (bf16): rows 16 bytes apart in bank space
  __shared__ __attribute__((aligned(16))) uint16_t s_src[2][64 * RS];
  const int b = blockIdx.y;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  const int row0 = blockIdx.x * (16 * NW) + 16 * w;
  const uint16_t* T = xt + (size_t)b * p * D;
  const uint16_t* S = xs + (size_t)b * q * D;
  // Logit tiles are computed transposed, D = X_S X_T^T, so that a lane holds
  // four consecutive source anchors of one target row: lane l has target
  // row row0 + l % 16 and sources c + 4 (l / 16) .. + 3 of a 16-anchor tile.
  // B operand (X_T^T): lane holds target row row0 + r16, columns 32 ks + 8 kg .. + 7
  Bf8 a[KS];
  const int ra = row0 + r16;
  const bool row_ok = ra < p;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
    a[ks].q = row_ok ? *reinterpret_cast<const uint4*>(T + (size_t)ra * D + 32 * ks + 8 * kg) : make_uint4(0, 0, 0, 0);
  // The workgroup stages 64 source anchors at a time in LDS (double-buffered,
  // one barrier per step, the next chunk's loads in flight during a step), so
  // each source row is read from L2 once per workgroup rather than once per wave.
  const int ngroups = (q + 63) / 64;
  // each thread's 16-byte pieces of a 64-anchor chunk: loaded into registers
  // one chunk ahead, stored to LDS at the start of the chunk's step
  constexpr int NP = (256 * KS + 64 * NW - 1) / (64 * NW);
  uint4 pre[NP];
  auto fetch = [&](int g) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = t + 64 * NW * i;  // piece index in [0, 64 * 4 KS)
      const int row = e / (4 * KS), col = 8 * (e % (4 * KS));
      const int src = 64 * g + row;
      pre[i] = e < 256 * KS && src < q ? *reinterpret_cast<const uint4*>(S + (size_t)src * D + col)
                                       : make_uint4(0, 0, 0, 0);
    }
  };
  auto stage = [&](int g) {
    uint16_t* dst = s_src[g & 1];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      const int e = t + 64 * NW * i;
      if (e < 256 * KS) *reinterpret_cast<uint4*>(dst + (e / (4 * KS)) * RS + 8 * (e % (4 * KS))) = pre[i];
    }
  };
  // four tiles of 16 staged source anchors
  auto tiles4 = [&](int g, f32x4* z) {
    const uint16_t* src = s_src[g & 1];
    Bf8 bv[4][KS];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        bv[u][ks].q = *reinterpret_cast<const uint4*>(src + (16 * u + r16) * RS + 32 * ks + 8 * kg);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(bv[u][ks].v, a[ks].v, acc, 0, 0, 0);
      z[u] = acc;
    }
  };
  // sweep 1: running maximum and sum of exp(z - maximum) over this lane's sources
  float m = -FLT_MAX, s = 0.f;
  fetch(0);
  for (int g = 0; g < ngroups; ++g) {
    stage(g);
    if (g + 1 < ngroups) fetch(g + 1);
    __syncthreads();
    f32x4 z[4];
    tiles4(g, z);
    const int c0 = 64 * g;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        if (c0 + 16 * u + 4 * kg + r < q) {
          const float v = z[u][r];
          if (v > m) {
            s = s * __expf(m - v) + 1.f;
            m = v;
          } else {
            s += __expf(v - m);
          }
        }
      }
    }
  }
  // merge over the four lanes holding the same target row (l, l ^ 16, l ^ 32, l ^ 48)
#pragma unroll
  for (int o = 16; o < 64; o <<= 1) {
    const float mo = __shfl_xor(m, o, 64);
    const float so = __shfl_xor(s, o, 64);
    const float mm = fmaxf(m, mo);
    s = s * __expf(m - mm) + so * __expf(mo - mm);
    m = mm;
  }
  const float inv = 1.f / s;
  // sweep 2: recompute the logits and write the normalised rows, four
  // consecutive entries per lane (one 16-byte store when `vec`: q a multiple
  // of 4 and `out` 16-byte aligned).  Its first staging step may overwrite
  // the buffer that sweep 1 read last, so a barrier separates the sweeps.
  __syncthreads();
  float* O = out + (size_t)b * p * q + (size_t)ra * q;
  fetch(0);
  for (int g = 0; g < ngroups; ++g) {
    stage(g);
    if (g + 1 < ngroups) fetch(g + 1);
    __syncthreads();
    f32x4 z[4];
    tiles4(g, z);
    const int c0 = 64 * g;
    if (row_ok) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int cb = c0 + 16 * u + 4 * kg;
        float4 e;
        e.x = __expf(z[u][0] - m) * inv;
        e.y = __expf(z[u][1] - m) * inv;
        e.z = __expf(z[u][2] - m) * inv;
        e.w = __expf(z[u][3] - m) * inv;
        if (vec && cb + 3 < q) {
          *reinterpret_cast<float4*>(O + cb) = e;
        } else {
          if (cb < q) O[cb] = e.x;
          if (cb + 1 < q) O[cb + 1] = e.y;
          if (cb + 2 < q) O[cb + 2] = e.z;
          if (cb + 3 < q) O[cb + 3] = e.w;
        }
      }
    }
  }
}

}  // namespace

}  // namespace gs

using namespace gs;

extern "C" gs_status gs_affinity(const uint16_t* xt, const uint16_t* xs, int32_t batch, int32_t p, int32_t q,
                                 int32_t d, float* out, hipStream_t stream) {
  if (batch < 0 || p < 0 || q < 0) return set_error(GS_ERR_INVALID_ARG, "negative affinity size");
  if (d < 32 || d > 256 || d % 32 != 0) return set_error(GS_ERR_INVALID_ARG, "affinity row width d must be 32..256, a multiple of 32");
  if (batch > 65535) return set_error(GS_ERR_INVALID_ARG, "affinity batch above 65535");
  if (batch == 0 || p == 0 || q == 0) return set_error(GS_OK, "");
  if (!xt || !xs || !out) return set_error(GS_ERR_INVALID_ARG, "null affinity argument");
  if ((reinterpret_cast<uintptr_t>(xt) | reinterpret_cast<uintptr_t>(xs)) % 16 != 0)
    return set_error(GS_ERR_INVALID_ARG, "affinity inputs must be 16-byte aligned");
  const dim3 grid((unsigned)((p + 16 * kAffWaves - 1) / (16 * kAffWaves)), (unsigned)batch), block(64 * kAffWaves);
  const bool vec = q % 4 == 0 && reinterpret_cast<uintptr_t>(out) % 16 == 0;
  switch (d / 32) {
#define KCASE(K) \
  case K: hipLaunchKernelGGL((k_affinity<K, kAffWaves>), grid, block, 0, stream, xt, xs, p, q, out, vec); break;
    KCASE(1) KCASE(2) KCASE(3) KCASE(4) KCASE(5) KCASE(6) KCASE(7) KCASE(8)
#undef KCASE
    default: return set_error(GS_ERR_INVALID_ARG, "bad affinity row width");
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(GS_ERR_HIP, std::string("affinity launch: ") + hipGetErrorString(e));
  return set_error(GS_OK, "");
}
