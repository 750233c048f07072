// Inpainting patch affinity (Sec. III-B, Eq. 6): for every (target, source)
// patch pair, the softmax over the source anchors of X_T X_S^T, X holding one
// encoded anchor per row (feature + positional encoding, bf16).
//
// One workgroup per 64 target rows of one pair, one wave per 16 rows.  The
// wave keeps its 16 x d slice of X_T in registers as MFMA A operands and
// walks the source anchors 64 at a time (four v_mfma_f32_16x16x32_bf16
// tiles, FP32 accumulate, all their loads issued first): a first sweep keeps a running row maximum and exponential sum
// per lane, the 16 lanes that share a row merge theirs, and a second sweep
// recomputes each 16 x 16 logit tile and writes exp(z - max) / sum.  The
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

union Bf8 {
  uint4 q;
  bf16x8 v;
};

template <int KS>  // d = 32 KS
__global__ __launch_bounds__(256) void k_affinity(const uint16_t* __restrict__ xt, const uint16_t* __restrict__ xs,
                                                   int p, int q, float* __restrict__ out) {
  constexpr int D = 32 * KS;
  const int b = blockIdx.y;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r16 = lane & 15, kg = lane >> 4;
  const int row0 = blockIdx.x * 64 + 16 * w;
  if (row0 >= p) return;  // wave-uniform: every lane of the wave leaves
  const uint16_t* T = xt + (size_t)b * p * D;
  const uint16_t* S = xs + (size_t)b * q * D;
  // A operand: lane holds row row0 + r16, columns 32 ks + 8 kg .. + 7
  Bf8 a[KS];
  const int ra = row0 + r16;
#pragma unroll
  for (int ks = 0; ks < KS; ++ks)
    a[ks].q = ra < p ? *reinterpret_cast<const uint4*>(T + (size_t)ra * D + 32 * ks + 8 * kg) : make_uint4(0, 0, 0, 0);
  // logits of rows row0 + 4 kg + r (r < 4) at columns c0 + 16 u + r16 (u < 4):
  // every source load of the four tiles is issued before the first MFMA
  auto tiles4 = [&](int c0, f32x4* z) {
    Bf8 bv[4][KS];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cb = c0 + 16 * u + r16;
#pragma unroll
      for (int ks = 0; ks < KS; ++ks)
        bv[u][ks].q =
            cb < q ? *reinterpret_cast<const uint4*>(S + (size_t)cb * D + 32 * ks + 8 * kg) : make_uint4(0, 0, 0, 0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int ks = 0; ks < KS; ++ks) acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks].v, bv[u][ks].v, acc, 0, 0, 0);
      z[u] = acc;
    }
  };
  // sweep 1: running maximum and sum of exp(z - maximum) over this lane's columns
  float m[4], s[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    m[r] = -FLT_MAX;
    s[r] = 0.f;
  }
  for (int c0 = 0; c0 < q; c0 += 64) {
    f32x4 z[4];
    tiles4(c0, z);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (c0 + 16 * u + r16 < q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (z[u][r] > m[r]) {
            s[r] = s[r] * __expf(m[r] - z[u][r]) + 1.f;
            m[r] = z[u][r];
          } else {
            s[r] += __expf(z[u][r] - m[r]);
          }
        }
      }
    }
  }
  // merge over the 16 lanes holding the same rows (lanes 16 kg .. 16 kg + 15)
#pragma unroll
  for (int o = 1; o < 16; o <<= 1) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float mo = __shfl_xor(m[r], o, 64);
      const float so = __shfl_xor(s[r], o, 64);
      const float mm = fmaxf(m[r], mo);
      s[r] = s[r] * __expf(m[r] - mm) + so * __expf(mo - mm);
      m[r] = mm;
    }
  }
  float inv[4];
#pragma unroll
  for (int r = 0; r < 4; ++r) inv[r] = 1.f / s[r];
  // sweep 2: recompute the logits and write the normalised rows
  float* O = out + (size_t)b * p * q;
  for (int c0 = 0; c0 < q; c0 += 64) {
    f32x4 z[4];
    tiles4(c0, z);
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int cb = c0 + 16 * u + r16;
      if (cb < q) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = row0 + 4 * kg + r;
          if (row < p) O[(size_t)row * q + cb] = __expf(z[u][r] - m[r]) * inv[r];
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
  const dim3 grid((unsigned)((p + 63) / 64), (unsigned)batch), block(256);
  switch (d / 32) {
#define KCASE(K) \
  case K: hipLaunchKernelGGL(k_affinity<K>, grid, block, 0, stream, xt, xs, p, q, out); break;
    KCASE(1) KCASE(2) KCASE(3) KCASE(4) KCASE(5) KCASE(6) KCASE(7) KCASE(8)
#undef KCASE
    default: return set_error(GS_ERR_INVALID_ARG, "bad affinity row width");
  }
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return set_error(GS_ERR_HIP, std::string("affinity launch: ") + hipGetErrorString(e));
  return set_error(GS_OK, "");
}
