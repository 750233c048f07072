// a6 / a8: per-tile forward compositing and its adjoint.
//
// One workgroup per screen tile, one lane per ray; each wave64 owns an 8x8
// block of rays so that its lanes see nearly the same surfels.  The tile's
// depth-ordered surfel records are staged through LDS in batches of one
// record per thread; every lane then walks the batch with broadcast LDS reads.
// A wave leaves a batch as soon as a ballot shows all its rays saturated; the
// workgroup stops when a block-wide count reaches zero.
//
// Per pair (camera, Sec. III-A Eq. 2-3):  h' = e3 + P (dx, dy),
//   u = h'0/h'2, v = h'1/h'2, z = mu_z/h'2, rho = u^2 + v^2,
//   rho_lp = lp (dx^2 + dy^2), rho_hat = min(rho, rho_lp),
//   alpha = min(alpha_max, exp2(log2 o - rho_hat / (2 ln 2))).
// Per pair (LiDAR, Eq. 5): delta = d - mu_hat, h' = e3 + Q delta,
//   range = |mu| / h'2, rho_lp = lp / step^2 |delta|^2.
// Near-degenerate (grazing) pairs of flagged surfels (|h'2| < 1/8) are
// re-solved in FP64 from the FP64 record.
//
// The backward pass replays each ray front to back up to the forward's last
// contributing pair (n_last), recomputing transmittance instead of storing
// per-ray lists, and uses the forward outputs O for the suffix sums
// S_i = O - (prefix through i):  dO/dalpha_i = T_i f_i - S_i / (1 - alpha_i).
// Per-pair gradients are summed over the wave with DPP and added to per-surfel
// accumulators with one atomic per wave and field.
#include "gs_internal.h"
#include "kernels.h"

namespace gs {

namespace {

constexpr float kInv2Ln2 = 0.7213475204444817f;  // 1 / (2 ln 2)

struct PairEval {
  float alpha, u, v, z, r, dx, dy, dz3;  // dz3: LiDAR third delta component
  bool lp_used, clamped;
};

// Does the surfel's conservative rectangle (packed 16-bit bounds) miss this
// wave's 8x8 block of rays?  Pairs outside the rectangle are never in the
// support, so skipping them leaves every result unchanged.
__device__ __forceinline__ bool misses_block(uint32_t cols, uint32_t rows, int bx, int by) {
  const int c_lo = cols & 0xFFFF, c_hi = cols >> 16, r_lo = rows & 0xFFFF, r_hi = rows >> 16;
  return c_hi < bx || c_lo > bx + 7 || r_hi < by || r_lo > by + 7;
}

// LiDAR columns may wrap (c_lo > c_hi means [c_lo, W) u [0, c_hi]).
__device__ __forceinline__ bool misses_block_wrap(uint32_t cols, uint32_t rows, int bx, int by) {
  const int c_lo = cols & 0xFFFF, c_hi = cols >> 16, r_lo = rows & 0xFFFF, r_hi = rows >> 16;
  if (r_hi < by || r_lo > by + 7) return true;
  if (c_lo <= c_hi) return c_hi < bx || c_lo > bx + 7;
  return c_hi < bx && c_lo > bx + 7;
}

// ----------------------------- camera -----------------------------------
// LDS record (5 x float4):
//  [0] pcx_rel, pcy_rel, P00, P01   [1] P10, P11, P20, P21
//  [2] mu_z, log2 o, c0, c1          [3] c2, n0, n1, n2
//  [4] flags, o, pixel columns lo|hi<<16, pixel rows lo|hi<<16
__device__ __forceinline__ bool eval_pinhole(const float4* __restrict__ R, uint32_t s, float plx, float ply, int ox,
                                             int oy, const TileArgs& a, PairEval& e, uint32_t& n64) {
#pragma clang fp contract(off)
  const float4 q0 = R[0], q1 = R[1], q2 = R[2];
  const uint32_t flags = __float_as_uint(R[4].x);
  const float dx = plx - q0.x;
  const float dy = ply - q0.y;
  const float h0 = fmaf(q0.z, dx, q0.w * dy);
  const float h1 = fmaf(q1.x, dx, q1.y * dy);
  const float h2 = fmaf(q1.z, dx, fmaf(q1.w, dy, 1.0f));
  float u, v, r, z;
  if ((flags & kFlagGrazing) && fabsf(h2) < 0.125f) {
    ++n64;
    const double* G = a.grz + kGrz * (size_t)s;
    const double* r64 = a.rec64 + kRec64 * (size_t)s;
    const double ddx = ((double)ox + (double)plx) - r64[0];
    const double ddy = ((double)oy + (double)ply) - r64[1];
    const double H0 = G[0] * ddx + G[1] * ddy;
    const double H1 = G[2] * ddx + G[3] * ddy;
    const double H2 = 1.0 + G[4] * ddx + G[5] * ddy;
    if (H2 == 0.0) return false;
    const double rd = 1.0 / H2;
    u = (float)(H0 * rd);
    v = (float)(H1 * rd);
    r = (float)rd;
    z = (float)(G[6] * rd);
  } else {
    if (h2 == 0.0f) return false;
    r = __builtin_amdgcn_rcpf(h2);
    u = h0 * r;
    v = h1 * r;
    z = q2.x * r;
  }
  const float rho = fmaf(u, u, v * v);
  float rho_hat = rho;
  bool lp_used = false;
  if (a.O.lowpass) {
    const float rl = a.O.lp * fmaf(dx, dx, dy * dy);
    if (!(rho <= rl)) {
      rho_hat = rl;
      lp_used = true;
    }
  }
  if (!(rho_hat <= a.O.cutoff2) || !(z > a.S.z_near)) return false;
  float alpha = __builtin_amdgcn_exp2f(fmaf(-kInv2Ln2, rho_hat, q2.y));
  const bool clamped = alpha > a.O.alpha_max;
  if (clamped) alpha = a.O.alpha_max;
  if (alpha < a.O.alpha_min) return false;
  e.alpha = alpha;
  e.u = u;
  e.v = v;
  e.z = z;
  e.r = r;
  e.dx = dx;
  e.dy = dy;
  e.lp_used = lp_used;
  e.clamped = clamped;
  return true;
}

__device__ __forceinline__ void stage_pinhole(const TileArgs& a, uint32_t s, int ox, int oy, float4* dst) {
  const float4* r = a.rec + 4 * (size_t)s;
  const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
  const double* r64 = a.rec64 + kRec64 * (size_t)s;
  const float pcx = (float)(r64[0] - (double)ox);
  const float pcy = (float)(r64[1] - (double)oy);
  const uint2 rect = *reinterpret_cast<const uint2*>(r64 + 3);
  dst[0] = make_float4(pcx, pcy, r0.x, r0.y);
  dst[1] = make_float4(r0.z, r0.w, r1.x, r1.y);
  dst[2] = make_float4(r1.z, r1.w, r2.x, r2.y);
  dst[3] = make_float4(r2.z, r2.w, r3.x, r3.y);
  dst[4] = make_float4(r3.z, r3.w, __uint_as_float(rect.x), __uint_as_float(rect.y));
}

template <int NT>
__device__ void fwd_tile_pinhole(const TileArgs& a, int tile, float4 (*s_rec)[5], uint32_t* s_id) {
#pragma clang fp contract(off)
  const int TW = a.S.tw, TH = a.S.th, WX = TW >> 3;
  const int tx = tile % a.S.n_tx, ty = tile / a.S.n_tx;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int lx = (w % WX) * 8 + (lane & 7), ly = (w / WX) * 8 + (lane >> 3);
  const int ox = tx * TW, oy = ty * TH;
  const int bx = ox + (w % WX) * 8, by = oy + (w / WX) * 8;
  const int px = ox + lx, py = oy + ly;
  const bool inside = px < a.S.W && py < a.S.H;
  const float plx = (float)lx + 0.5f, ply = (float)ly + 0.5f;
  const uint2 rg = a.ranges[a.S.tile_offset + tile];
  float T = 1.0f;
  float acc[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) acc[c] = 0.0f;
  bool done = !inside;
  uint32_t last = rg.x, n_eval = 0, n_contrib = 0, n64 = 0;
  for (uint32_t base = rg.x; base < rg.y; base += NT) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t k = base + t;
    if (k < rg.y) {
      const uint32_t s = a.pval[k];
      stage_pinhole(a, s, ox, oy, s_rec[t]);
      s_id[t] = s;
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)NT, rg.y - base);
    for (int j = 0; j < cnt; ++j) {
      if (__ballot(!done) == 0) break;
      if (misses_block(__float_as_uint(s_rec[j][4].z), __float_as_uint(s_rec[j][4].w), bx, by)) continue;
      if (done) continue;
      PairEval e;
      ++n_eval;
      if (!eval_pinhole(s_rec[j], s_id[j], plx, ply, ox, oy, a, e, n64)) continue;
      const float Tn = T * (1.0f - e.alpha);
      if (Tn < a.O.T_min) {
        done = true;
        continue;
      }
      ++n_contrib;
      const float wgt = e.alpha * T;
      const float4 q2 = s_rec[j][2], q3 = s_rec[j][3];
      acc[0] = fmaf(wgt, q2.z, acc[0]);
      acc[1] = fmaf(wgt, q2.w, acc[1]);
      acc[2] = fmaf(wgt, q3.x, acc[2]);
      acc[3] = fmaf(wgt, e.z, acc[3]);
      acc[4] = fmaf(wgt, q3.y, acc[4]);
      acc[5] = fmaf(wgt, q3.z, acc[5]);
      acc[6] = fmaf(wgt, q3.w, acc[6]);
      acc[7] = acc[7] + wgt;
      T = Tn;
      last = base + j + 1;
    }
  }
  count_pairs(a.status, n_eval, n_contrib, n64);
  if (inside) {
    const size_t HW = (size_t)a.S.W * a.S.H;
    const size_t p = (size_t)py * a.S.W + px;
    a.out[p] = fmaf(T, a.O.bg0, acc[0]);
    a.out[HW + p] = fmaf(T, a.O.bg1, acc[1]);
    a.out[2 * HW + p] = fmaf(T, a.O.bg2, acc[2]);
#pragma unroll
    for (int c = 3; c < 8; ++c) a.out[c * HW + p] = acc[c];
    a.T_final[p] = T;
    a.n_last[p] = last;
  }
}

__device__ __forceinline__ void flush_grads(const float* g, uint32_t s, float* gacc, int N, int lane) {
#pragma unroll
  for (int f = 0; f < kGradFields; ++f) {
    const float v = wave_sum_last(g[f]);
    if (lane == 63 && v != 0.0f) atomicAdd(gacc + (size_t)f * N + s, v);
  }
}

template <int NT>
__device__ void bwd_tile_pinhole(const TileArgs& a, int tile, float4 (*s_rec)[5], uint32_t* s_id, uint32_t& s_maxlast) {
#pragma clang fp contract(off)
  const int TW = a.S.tw, TH = a.S.th, WX = TW >> 3;
  const int tx = tile % a.S.n_tx, ty = tile / a.S.n_tx;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int lx = (w % WX) * 8 + (lane & 7), ly = (w / WX) * 8 + (lane >> 3);
  const int ox = tx * TW, oy = ty * TH;
  const int bx = ox + (w % WX) * 8, by = oy + (w / WX) * 8;
  const int px = ox + lx, py = oy + ly;
  const bool inside = px < a.S.W && py < a.S.H;
  const float plx = (float)lx + 0.5f, ply = (float)ly + 0.5f;
  const uint2 rg = a.ranges[a.S.tile_offset + tile];
  const size_t HW = (size_t)a.S.W * a.S.H;
  const size_t p = inside ? (size_t)py * a.S.W + px : 0;
  float g[8], O[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) {
    g[c] = inside ? a.gout[c * HW + p] : 0.0f;
    O[c] = inside ? a.out_fwd[c * HW + p] : 0.0f;
  }
  const uint32_t last = inside ? a.n_last[p] : rg.x;
  __syncthreads();
  if (t == 0) s_maxlast = rg.x;
  __syncthreads();
  atomicMax(&s_maxlast, last);
  __syncthreads();
  const uint32_t end = s_maxlast;
  // wave-uniform end
  uint32_t wlast = last;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) wlast = max(wlast, (uint32_t)__shfl_xor((int)wlast, o, 64));
  uint32_t n64 = 0;
  float T = 1.0f;
  float A[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) A[c] = 0.0f;
  for (uint32_t base = rg.x; base < end; base += NT) {
    __syncthreads();
    const uint32_t k = base + t;
    if (k < end) {
      const uint32_t s = a.pval[k];
      stage_pinhole(a, s, ox, oy, s_rec[t]);
      s_id[t] = s;
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)NT, end - base);
    for (int j = 0; j < cnt; ++j) {
      if (base + j >= wlast) break;
      if (misses_block(__float_as_uint(s_rec[j][4].z), __float_as_uint(s_rec[j][4].w), bx, by)) continue;
      const bool active = base + j < last;
      PairEval e;
      const bool hit = active && eval_pinhole(s_rec[j], s_id[j], plx, ply, ox, oy, a, e, n64);
      float gr[kGradFields];
#pragma unroll
      for (int f = 0; f < kGradFields; ++f) gr[f] = 0.0f;
      if (hit) {
        const float4 q0 = s_rec[j][0], q1 = s_rec[j][1], q2 = s_rec[j][2], q3 = s_rec[j][3];
        const float o = s_rec[j][4].y;
        const float al = e.alpha;
        const float wgt = al * T;
        const float f[8] = {q2.z, q2.w, q3.x, e.z, q3.y, q3.z, q3.w, 1.0f};
        const float inv1m = 1.0f / (1.0f - al);
        float dal = 0.0f;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          A[c] = fmaf(wgt, f[c], A[c]);
          const float S = O[c] - A[c];
          dal += g[c] * (T * f[c] - S * inv1m);
        }
        // colour and normal
        gr[10] = g[0] * wgt;
        gr[11] = g[1] * wgt;
        gr[12] = g[2] * wgt;
        gr[13] = g[4] * wgt;
        gr[14] = g[5] * wgt;
        gr[15] = g[6] * wgt;
        const float gz = g[3] * wgt;
        float g_rhohat = 0.0f;
        if (!e.clamped) {
          gr[9] = o > 0.0f ? dal * al / o : 0.0f;
          g_rhohat = -0.5f * dal * al;
        }
        const float g_rho = e.lp_used ? 0.0f : g_rhohat;
        const float g_lp = e.lp_used ? g_rhohat : 0.0f;
        const float gu = 2.0f * e.u * g_rho, gv = 2.0f * e.v * g_rho;
        const float gh0 = gu * e.r, gh1 = gv * e.r;
        const float gh2 = -(gu * e.u + gv * e.v + gz * e.z) * e.r;
        gr[8] = gz * e.r;
        gr[0] = gh0 * e.dx;
        gr[1] = gh0 * e.dy;
        gr[2] = gh1 * e.dx;
        gr[3] = gh1 * e.dy;
        gr[4] = gh2 * e.dx;
        gr[5] = gh2 * e.dy;
        const float two_lp = 2.0f * a.O.lp * g_lp;
        const float gdx = q0.z * gh0 + q1.x * gh1 + q1.z * gh2 + two_lp * e.dx;
        const float gdy = q0.w * gh0 + q1.y * gh1 + q1.w * gh2 + two_lp * e.dy;
        gr[6] = -gdx;
        gr[7] = -gdy;
        T = T * (1.0f - al);
      }
      if (__ballot(hit) != 0) flush_grads(gr, s_id[j], a.gacc, a.gacc_stride, lane);
    }
  }
}

// ----------------------------- LiDAR -------------------------------------
// LDS record (5 x float4):
//  [0] c0, c1, c2 (= d_tile - mu_hat), Q00   [1] Q01, Q02, Q10, Q11
//  [2] Q12, Q20, Q21, Q22                    [3] |mu|, log2 o, intensity, flags
//  [4] o, columns lo|hi<<16 (may wrap), beams lo|hi<<16, -
__device__ __forceinline__ void stage_lidar(const TileArgs& a, uint32_t s, const double* dtile, float4* dst) {
  const float4* r = a.rec + 4 * (size_t)s;
  const float4 r0 = r[0], r1 = r[1], r2 = r[2], r3 = r[3];
  const double* r64 = a.rec64 + kRec64 * (size_t)s;
  const float c0 = (float)(dtile[0] - r64[0]);
  const float c1 = (float)(dtile[1] - r64[1]);
  const float c2 = (float)(dtile[2] - r64[2]);
  dst[0] = make_float4(c0, c1, c2, r0.x);
  dst[1] = make_float4(r0.y, r0.z, r0.w, r1.x);
  dst[2] = make_float4(r1.y, r1.z, r1.w, r2.x);
  dst[3] = make_float4(r2.y, r2.z, r2.w, r3.x);
  dst[4] = make_float4(r3.y, r3.z, r3.w, 0.0f);
}

__device__ __forceinline__ bool eval_lidar(const float4* __restrict__ R, uint32_t s, const float* dpix,
                                           const double* d64, const TileArgs& a, PairEval& e, uint32_t& n64) {
#pragma clang fp contract(off)
  const float4 q0 = R[0], q1 = R[1], q2 = R[2], q3 = R[3];
  const uint32_t flags = __float_as_uint(q3.w);
  const float d0 = dpix[0] + q0.x;
  const float d1 = dpix[1] + q0.y;
  const float d2 = dpix[2] + q0.z;
  const float h0 = fmaf(q0.w, d0, fmaf(q1.x, d1, q1.y * d2));
  const float h1 = fmaf(q1.z, d0, fmaf(q1.w, d1, q2.x * d2));
  const float h2 = fmaf(q2.y, d0, fmaf(q2.z, d1, fmaf(q2.w, d2, 1.0f)));
  float u, v, r, z;
  if ((flags & kFlagGrazing) && fabsf(h2) < 0.125f) {
    ++n64;
    const double* G = a.grz + kGrz * (size_t)s;
    const double* r64 = a.rec64 + kRec64 * (size_t)s;
    const double e0 = d64[0] - r64[0], e1 = d64[1] - r64[1], e2 = d64[2] - r64[2];
    const double H0 = G[0] * e0 + G[1] * e1 + G[2] * e2;
    const double H1 = G[3] * e0 + G[4] * e1 + G[5] * e2;
    const double H2 = 1.0 + G[6] * e0 + G[7] * e1 + G[8] * e2;
    if (H2 == 0.0) return false;
    const double rd = 1.0 / H2;
    u = (float)(H0 * rd);
    v = (float)(H1 * rd);
    r = (float)rd;
    z = (float)(G[9] * rd);
  } else {
    if (h2 == 0.0f) return false;
    r = __builtin_amdgcn_rcpf(h2);
    u = h0 * r;
    v = h1 * r;
    z = q3.x * r;
  }
  const float rho = fmaf(u, u, v * v);
  float rho_hat = rho;
  bool lp_used = false;
  if (a.O.lowpass) {
    const float rl = a.S.lp_ang * fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
    if (!(rho <= rl)) {
      rho_hat = rl;
      lp_used = true;
    }
  }
  if (!(rho_hat <= a.O.cutoff2) || !(z > a.S.z_near)) return false;
  float alpha = __builtin_amdgcn_exp2f(fmaf(-kInv2Ln2, rho_hat, q3.y));
  const bool clamped = alpha > a.O.alpha_max;
  if (clamped) alpha = a.O.alpha_max;
  if (alpha < a.O.alpha_min) return false;
  e.alpha = alpha;
  e.u = u;
  e.v = v;
  e.z = z;
  e.r = r;
  e.dx = d0;
  e.dy = d1;
  e.dz3 = d2;
  e.lp_used = lp_used;
  e.clamped = clamped;
  return true;
}

// Unit ray direction of LiDAR column c, beam j from the FP32 tables, in FP64.
__device__ inline void lidar_dir(const SensorK& S, int c, int j, double* d) {
  const double ce = S.cos_el[j], se = S.sin_el[j], ca = S.cos_az[c], sa = S.sin_az[c];
  d[0] = ce * ca;
  d[1] = ce * sa;
  d[2] = se;
}

template <int NT>
__device__ void fwd_tile_lidar(const TileArgs& a, int tile, float4 (*s_rec)[5], uint32_t* s_id) {
#pragma clang fp contract(off)
  const int TW = a.S.tw, TH = a.S.th, WX = TW >> 3;
  const int tx = tile % a.S.n_tx, ty = tile / a.S.n_tx;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int lx = (w % WX) * 8 + (lane & 7), ly = (w / WX) * 8 + (lane >> 3);
  const int ox = tx * TW, oy = ty * TH;
  const int bx = ox + (w % WX) * 8, by = oy + (w / WX) * 8;
  const int pc = ox + lx, pb = oy + ly;
  const bool inside = pc < a.S.W && pb < a.S.H;
  double dt[3], d64[3];
  lidar_dir(a.S, ox, oy, dt);
  lidar_dir(a.S, inside ? pc : ox, inside ? pb : oy, d64);
  const float dpix[3] = {(float)(d64[0] - dt[0]), (float)(d64[1] - dt[1]), (float)(d64[2] - dt[2])};
  const uint2 rg = a.ranges[a.S.tile_offset + tile];
  float T = 1.0f, acc0 = 0.0f, acc1 = 0.0f, acc2 = 0.0f;
  bool done = !inside;
  uint32_t last = rg.x, n_eval = 0, n_contrib = 0, n64 = 0;
  for (uint32_t base = rg.x; base < rg.y; base += NT) {
    if (__syncthreads_count(!done) == 0) break;
    const uint32_t k = base + t;
    if (k < rg.y) {
      const uint32_t s = a.pval[k];
      stage_lidar(a, s, dt, s_rec[t]);
      s_id[t] = s;
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)NT, rg.y - base);
    for (int j = 0; j < cnt; ++j) {
      if (__ballot(!done) == 0) break;
      if (misses_block_wrap(__float_as_uint(s_rec[j][4].y), __float_as_uint(s_rec[j][4].z), bx, by)) continue;
      if (done) continue;
      PairEval e;
      ++n_eval;
      if (!eval_lidar(s_rec[j], s_id[j], dpix, d64, a, e, n64)) continue;
      const float Tn = T * (1.0f - e.alpha);
      if (Tn < a.O.T_min) {
        done = true;
        continue;
      }
      ++n_contrib;
      const float wgt = e.alpha * T;
      acc0 = fmaf(wgt, e.z, acc0);
      acc1 = fmaf(wgt, s_rec[j][3].z, acc1);
      acc2 = acc2 + wgt;
      T = Tn;
      last = base + j + 1;
    }
  }
  count_pairs(a.status, n_eval, n_contrib, n64);
  if (inside) {
    const size_t HW = (size_t)a.S.W * a.S.H;
    const size_t p = (size_t)pb * a.S.W + pc;
    a.out[p] = acc0;
    a.out[HW + p] = acc1;
    a.out[2 * HW + p] = acc2;
    a.T_final[p] = T;
    a.n_last[p] = last;
  }
}

template <int NT>
__device__ void bwd_tile_lidar(const TileArgs& a, int tile, float4 (*s_rec)[5], uint32_t* s_id, uint32_t& s_maxlast) {
#pragma clang fp contract(off)
  const int TW = a.S.tw, TH = a.S.th, WX = TW >> 3;
  const int tx = tile % a.S.n_tx, ty = tile / a.S.n_tx;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int lx = (w % WX) * 8 + (lane & 7), ly = (w / WX) * 8 + (lane >> 3);
  const int ox = tx * TW, oy = ty * TH;
  const int bx = ox + (w % WX) * 8, by = oy + (w / WX) * 8;
  const int pc = ox + lx, pb = oy + ly;
  const bool inside = pc < a.S.W && pb < a.S.H;
  double dt[3], d64[3];
  lidar_dir(a.S, ox, oy, dt);
  lidar_dir(a.S, inside ? pc : ox, inside ? pb : oy, d64);
  const float dpix[3] = {(float)(d64[0] - dt[0]), (float)(d64[1] - dt[1]), (float)(d64[2] - dt[2])};
  const uint2 rg = a.ranges[a.S.tile_offset + tile];
  const size_t HW = (size_t)a.S.W * a.S.H;
  const size_t p = inside ? (size_t)pb * a.S.W + pc : 0;
  float g[3], O[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    g[c] = inside ? a.gout[c * HW + p] : 0.0f;
    O[c] = inside ? a.out_fwd[c * HW + p] : 0.0f;
  }
  const uint32_t last = inside ? a.n_last[p] : rg.x;
  __syncthreads();
  if (t == 0) s_maxlast = rg.x;
  __syncthreads();
  atomicMax(&s_maxlast, last);
  __syncthreads();
  const uint32_t end = s_maxlast;
  uint32_t wlast = last;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) wlast = max(wlast, (uint32_t)__shfl_xor((int)wlast, o, 64));
  uint32_t n64 = 0;
  float T = 1.0f, A0 = 0.0f, A1 = 0.0f, A2 = 0.0f;
  for (uint32_t base = rg.x; base < end; base += NT) {
    __syncthreads();
    const uint32_t k = base + t;
    if (k < end) {
      const uint32_t s = a.pval[k];
      stage_lidar(a, s, dt, s_rec[t]);
      s_id[t] = s;
    }
    __syncthreads();
    const int cnt = (int)min((uint32_t)NT, end - base);
    for (int j = 0; j < cnt; ++j) {
      if (base + j >= wlast) break;
      if (misses_block_wrap(__float_as_uint(s_rec[j][4].y), __float_as_uint(s_rec[j][4].z), bx, by)) continue;
      const bool active = base + j < last;
      PairEval e;
      const bool hit = active && eval_lidar(s_rec[j], s_id[j], dpix, d64, a, e, n64);
      float gr[kGradFields];
#pragma unroll
      for (int f = 0; f < kGradFields; ++f) gr[f] = 0.0f;
      if (hit) {
        const float4 q0 = s_rec[j][0], q1 = s_rec[j][1], q2 = s_rec[j][2], q3 = s_rec[j][3];
        const float o = s_rec[j][4].x;
        const float al = e.alpha;
        const float wgt = al * T;
        const float inten = q3.z;
        const float inv1m = 1.0f / (1.0f - al);
        A0 = fmaf(wgt, e.z, A0);
        A1 = fmaf(wgt, inten, A1);
        A2 = A2 + wgt;
        float dal = g[0] * (T * e.z - (O[0] - A0) * inv1m);
        dal += g[1] * (T * inten - (O[1] - A1) * inv1m);
        dal += g[2] * (T - (O[2] - A2) * inv1m);
        const float grange = g[0] * wgt;
        gr[14] = g[1] * wgt;  // intensity
        float g_rhohat = 0.0f;
        if (!e.clamped) {
          gr[13] = o > 0.0f ? dal * al / o : 0.0f;
          g_rhohat = -0.5f * dal * al;
        }
        const float g_rho = e.lp_used ? 0.0f : g_rhohat;
        const float g_lp = e.lp_used ? g_rhohat : 0.0f;
        const float gu = 2.0f * e.u * g_rho, gv = 2.0f * e.v * g_rho;
        const float gh0 = gu * e.r, gh1 = gv * e.r;
        const float gh2 = -(gu * e.u + gv * e.v + grange * e.z) * e.r;
        gr[12] = grange * e.r;  // |mu|
        const float dd[3] = {e.dx, e.dy, e.dz3};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          gr[c] = gh0 * dd[c];
          gr[3 + c] = gh1 * dd[c];
          gr[6 + c] = gh2 * dd[c];
        }
        const float two_lp = 2.0f * a.S.lp_ang * g_lp;
        const float Q[9] = {q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
        // d(delta) -> mu_hat enters with a minus sign; stored in fields 9..11
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const float gd = Q[c] * gh0 + Q[3 + c] * gh1 + Q[6 + c] * gh2 + two_lp * dd[c];
          gr[9 + c] = -gd;
        }
        T = T * (1.0f - al);
      }
      if (__ballot(hit) != 0) flush_grads(gr, s_id[j], a.gacc, a.gacc_stride, lane);
    }
  }
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_blend_fwd(TileArgs a, int n_tiles) {
  __shared__ float4 s_rec[TW * TH][5];
  __shared__ uint32_t s_id[TW * TH];
  const int tile = blockIdx.x;
  if (a.S.kind == GS_SENSOR_PINHOLE)
    fwd_tile_pinhole<TW * TH>(a, tile, s_rec, s_id);
  else
    fwd_tile_lidar<TW * TH>(a, tile, s_rec, s_id);
}

template <int TW, int TH>
__global__ __launch_bounds__(TW* TH) void k_blend_bwd(TileArgs a, int n_tiles) {
  __shared__ float4 s_rec[TW * TH][5];
  __shared__ uint32_t s_id[TW * TH];
  __shared__ uint32_t s_maxlast;
  const int tile = blockIdx.x;
  if (a.S.kind == GS_SENSOR_PINHOLE)
    bwd_tile_pinhole<TW * TH>(a, tile, s_rec, s_id, s_maxlast);
  else
    bwd_tile_lidar<TW * TH>(a, tile, s_rec, s_id, s_maxlast);
}

// Persistent compositing over every (sensor, tile) of a batched step: each
// workgroup pops work items (global tile ids, heaviest first) from a queue
// with one atomic per item until the queue is empty.  256 threads; every
// sensor's tile shape has 256 rays.
__device__ inline int sensor_of_tile(const BatchArgs& b, uint32_t gt) {
  int s = 0;
  while (s + 1 < b.n_sensors && b.tile_off[s + 1] <= (int)gt) ++s;
  return s;
}

template <bool BWD>
__global__ __launch_bounds__(256) void k_blend_persistent(BatchArgs b) {
  __shared__ float4 s_rec[256][5];
  __shared__ uint32_t s_id[256];
  __shared__ uint32_t s_maxlast;
  __shared__ int s_item;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) s_item = (int)atomicAdd(b.counter, 1u);
    __syncthreads();
    const int it = s_item;
    if (it >= b.n_items) break;
    const uint32_t gt = b.queue[it];
    const int s = sensor_of_tile(b, gt);
    const TileArgs a = b.tiles[s];
    const int tile = (int)gt - b.tile_off[s];
    if (a.S.kind == GS_SENSOR_PINHOLE) {
      if (BWD) bwd_tile_pinhole<256>(a, tile, s_rec, s_id, s_maxlast);
      else fwd_tile_pinhole<256>(a, tile, s_rec, s_id);
    } else {
      if (BWD) bwd_tile_lidar<256>(a, tile, s_rec, s_id, s_maxlast);
      else fwd_tile_lidar<256>(a, tile, s_rec, s_id);
    }
  }
}

}  // namespace

#define GS_TILE_CASES(X) X(16, 16) X(32, 8) X(8, 32) X(16, 8) X(8, 16) X(8, 8) X(32, 16) X(16, 32)

void launch_blend_forward(const TileArgs& a, int n_tiles, hipStream_t st) {
  if (n_tiles == 0) return;
  const int tw = a.S.tw, th = a.S.th;
  const dim3 grid(n_tiles);
#define CASE(W, H)                                                                 \
  if (tw == W && th == H) {                                                        \
    hipLaunchKernelGGL((k_blend_fwd<W, H>), grid, dim3(W * H), 0, st, a, n_tiles); \
    return;                                                                        \
  }
  GS_TILE_CASES(CASE)
#undef CASE
}

void launch_blend_backward(const TileArgs& a, int n_tiles, hipStream_t st) {
  if (n_tiles == 0) return;
  const int tw = a.S.tw, th = a.S.th;
  const dim3 grid(n_tiles);
#define CASE(W, H)                                                                 \
  if (tw == W && th == H) {                                                        \
    hipLaunchKernelGGL((k_blend_bwd<W, H>), grid, dim3(W * H), 0, st, a, n_tiles); \
    return;                                                                        \
  }
  GS_TILE_CASES(CASE)
#undef CASE
}

void launch_blend_persistent(const BatchArgs& b, int grid, bool backward, hipStream_t st) {
  if (b.n_items == 0) return;
  if (backward)
    hipLaunchKernelGGL((k_blend_persistent<true>), dim3(grid), dim3(256), 0, st, b);
  else
    hipLaunchKernelGGL((k_blend_persistent<false>), dim3(grid), dim3(256), 0, st, b);
}

int persistent_blocks_per_cu(bool backward) {
  int n = 0;
  hipError_t e = backward ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_blend_persistent<true>, 256, 0)
                          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_blend_persistent<false>, 256, 0);
  return e == hipSuccess ? n : 0;
}

bool tile_shape_supported(int tw, int th) {
#define CASE(W, H) \
  if (tw == W && th == H) return true;
  GS_TILE_CASES(CASE)
#undef CASE
  return false;
}

}  // namespace gs
