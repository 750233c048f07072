// a6 / a8: front-to-back compositing (Sec. III-A, Eq. 1 with the ray-splat
// solve of Eq. 2-3 / Eq. 5) and its adjoint, as one persistent work queue.
//
// Work items are (tile, segment) pairs.  A tile whose depth-ordered pair list
// is at most L pairs long is one item and is composited exactly as the
// definition reads.  A longer list is split into segments of L pairs so that
// no single workgroup walks tens of thousands of pairs while the rest of the
// chip idles (horizon tiles of a driving scene hold 100x the median list):
//  1. every segment composites its pairs for each ray starting from T = 1,
//     with the usual skip and stop rules, and stores its partial state
//     (accumulators, transmittance, last composited pair, counters);
//  2. the workgroup that finishes a tile's last segment (one atomic arrival
//     counter per tile) merges the partials front to back:
//         C <- C + T * C_seg,   T <- T * T_seg,
//     accepting a segment whole while T * T_seg stays clear of T_min; a ray
//     whose stop can fall inside segment s gets its incoming state stored in
//     slot s, the slot is marked, and (tile, s) joins a walk list;
//  3. once the main queue is drained, the same persistent workgroups walk
//     every listed segment cooperatively for its marked rays from their true
//     incoming state, so the stop rule keeps its sequential meaning (a ray
//     that then does not stop, which needs its FP32 product within rounding
//     of T_min, finishes the merge on its own); walks of tiles merged early
//     overlap the rest of the queue;
//  4. each reached segment keeps its incoming (T, prefix accumulators), so the
//     adjoint processes every segment independently.
//
// Inside an item: one lane per ray, each wave64 owns an 8x8 block of rays.
// Records are staged through LDS one per thread; lanes walk the batch with
// broadcast LDS reads; a wave skips pairs whose pixel rectangle misses its
// block and leaves as soon as a ballot shows all its rays saturated.
// Grazing pairs of flagged surfels (|h'2| < 1/8) are re-solved in FP64.
//
// The adjoint replays each ray front to back up to the forward's last
// contributing pair (n_last), recomputing transmittance, and uses the forward
// outputs O for the suffix sums S_i = O - (prefix through i):
// dO/dalpha_i = T_i f_i - S_i / (1 - alpha_i).  Per-pair gradients are summed
// over the wave with DPP and added to per-record accumulators with one atomic
// per wave and field.
#include "gs_internal.h"
#include "kernels.h"

namespace gs {

namespace {

constexpr float kInv2Ln2 = 0.7213475204444817f;  // 1 / (2 ln 2)

// Partial-state planes of one segment slot (one value per ray of the tile).
// After the merge, planes [0, C) and kPartT hold the segment's incoming state;
// a slot marked kWalk in kPartLast holds the ray's last pair so far in
// kPartCount.
enum { kPartT = 8, kPartLast = 9, kPartCount = 10 };
// A merge marks a ray whose transmittance falls below 1/2 inside a later
// segment s it takes whole with mpair = kCross | s, and lists (tile, s |
// kMedianEntry) on the walk list; the entry's replay finds the crossing pair.
constexpr uint32_t kCross = 0x80000000u;
constexpr uint32_t kMedianEntry = 0x80000000u;
constexpr uint32_t kWalk = 0xFFFFFFFFu;  // never a (last | stop bit) value: pair ids < 2^31 - 1


// Device-coherent loads of partial state published by other workgroups
// (possibly on other XCDs, after their device-scope release): these bypass
// the reader's non-coherent L2 copy, so no acquire fence (which would
// invalidate the whole L2 of the reader's XCD) is needed.
__device__ __forceinline__ float ld_coh(const float* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ld_coh(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// FP64 re-solve data of grazing-flagged records staged next to the batch:
// up to kF64Slots records per batch (more fall back to global loads); a
// staged record carries its slot + 1 in bits 8..15 of its flag word.
constexpr int kF64Slots = 64;
constexpr int kF64Doubles = kGrz + 3;  // grazing record + centre (pixel or unit direction)
typedef double F64Slot[kF64Doubles];

// Copy of a uniform value held in a vector register: the pair loop runs
// short of scalar registers, and a constant kept there would be re-fetched
// from the kernel arguments at every pair.
__device__ __forceinline__ float in_vgpr(float x) {
  float y;
  asm("v_mov_b32 %0, %1" : "=v"(y) : "v"(x));
  return y;
}

// Per-item constants of the per-pair test, loaded once per work item and
// kept in vector registers.
struct EvalK {
  float lp;         // low-pass scale (camera: 1/sigma^2 per pixel^2; LiDAR: per rad^2)
  float cutoff2, z_near, alpha_max, alpha_min, T_min;
  bool lowpass;
};

__device__ __forceinline__ EvalK eval_consts(const TileArgs& a, float lp) {
  EvalK k;
  k.lp = in_vgpr(lp);
  k.cutoff2 = in_vgpr(a.O.cutoff2);
  k.z_near = in_vgpr(a.S.z_near);
  k.alpha_max = in_vgpr(a.O.alpha_max);
  k.alpha_min = in_vgpr(a.O.alpha_min);
  k.T_min = in_vgpr(a.O.T_min);
  k.lowpass = a.O.lowpass != 0;
  return k;
}

struct PairEval {
  float alpha, u, v, z, r, dx, dy, dz3;  // dz3: LiDAR third delta component
  bool lp_used, clamped;
};

// The rest of a pair's evaluation from its solve (u, v, 1/h'_2, depth): the
// low-pass choice, the support and alpha tests and alpha itself.  rl is the
// low-pass term, zc the centre's depth (taken by pairs the low-pass term admits).
__device__ __forceinline__ bool finish_pair(float u, float v, float r, float z, bool ok, float rl, float zc,
                                            float log2o, const EvalK& K, PairEval& e) {
#pragma clang fp contract(off)
  const float rho = fmaf(u, u, v * v);
  const bool lp_used = K.lowpass && !(rho <= rl);
  const float rho_hat = lp_used ? rl : rho;
  // a pair admitted by the low-pass term (edge-on or sub-pixel surfel) takes
  // the centre's depth: its plane hit is not meaningful there
  if (lp_used) z = zc;
  ok = ok && (rho_hat <= K.cutoff2) && (z > K.z_near);
  const float alpha_raw = __builtin_amdgcn_exp2f(fmaf(-kInv2Ln2, rho_hat, log2o));
  // min(alpha_raw, alpha_max) as one median-of-three (alpha_raw >= 0); the
  // clamp flag serves the adjoint only
  const bool clamped = alpha_raw > K.alpha_max;
  const float alpha = __builtin_amdgcn_fmed3f(alpha_raw, 0.0f, K.alpha_max);
  ok = ok && !(alpha < K.alpha_min);
  e.alpha = alpha;
  e.u = u;
  e.v = v;
  e.z = z;
  e.r = r;
  e.lp_used = lp_used;
  e.clamped = clamped;
  return ok;
}

// Per-tile FP32 error bound of a staged record: Et bounds the (u, v) error of
// any of the tile's pairs to first order (see the record flags).  The edge
// bit stays only where Et still allows an alpha error above the budget, and
// the wild bit is set where Et is too large to trust the FP32 rho; Et itself
// goes to a spare slot for the block test's rounding slack.
__device__ __forceinline__ void set_tile_bound(float& flag_word, float& slot, float Et, float log2o) {
  uint32_t f = __float_as_uint(flag_word);
  if (f & kFlagEdge) {
    if (!(2.87f * __builtin_amdgcn_exp2f(log2o) * Et > kEdgeTau)) f &= ~kFlagEdge;
    if (!(Et <= kWildErr)) f |= kFlagWild;
  }
  flag_word = __uint_as_float(f);
  slot = Et;
}

// Does an edge-flagged pair need the FP64 re-solve?  err |1/h'_2| bounds its
// (u, v) error to first order, so its alpha error is at most alpha
// |(u, v)|_1 err |1/h'_2| (taken with a 30% margin) where rho decides alpha;
// a pair whose alpha comes from the low-pass term does not depend on (u, v)
// (a choice between the two that the error could flip is a near-threshold
// decision).  Where the bound exceeds kWildErr (only in wild tiles) the FP32
// rho is not trusted: the pair re-solves if rho could be inside
// min(cutoff, low-pass term) with that error.
__device__ __forceinline__ bool edge_needs_f64(const PairEval& e, float err, float rl, uint32_t flags,
                                               const EvalK& K) {
#pragma clang fp contract(off)
  const float eu = err * fabsf(e.r);
  bool r = !e.lp_used & (e.alpha * ((fabsf(e.u) + fabsf(e.v)) * eu) > kEdgeTau * (1.0f / 1.3f));
  if (flags & kFlagWild) {  // the same record for the whole wave
    const float rho = fmaf(e.u, e.u, e.v * e.v);
    const float m = K.lowpass ? fminf(K.cutoff2, rl) : K.cutoff2;
    r = r | ((eu > kWildErr) & !(rho > fmaf(eu, fmaf(2.0f, eu, 9.5f), m)));
  }
  return r;
}

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

__device__ __forceinline__ bool covers(uint32_t cols, uint32_t rows, int x, int y) {
  return (int)(cols & 0xFFFF) <= x && x <= (int)(cols >> 16) && (int)(rows & 0xFFFF) <= y && y <= (int)(rows >> 16);
}

__device__ __forceinline__ bool covers_wrap(uint32_t cols, uint32_t rows, int x, int y) {
  const int c_lo = cols & 0xFFFF, c_hi = cols >> 16;
  if (!((int)(rows & 0xFFFF) <= y && y <= (int)(rows >> 16))) return false;
  return c_lo <= c_hi ? (c_lo <= x && x <= c_hi) : (x >= c_lo || x <= c_hi);
}

// Lanes (lane = 8 y + x) of the 8x8 block at (bx, by) inside the inclusive
// column range [c0, c1] and row range [r0, r1]; wave-uniform (scalar) work.
__device__ __forceinline__ uint64_t block_lanes(int c0, int c1, int r0, int r1, int bx, int by) {
  const int x0 = max(c0 - bx, 0), x1 = min(c1 - bx, 7), y0 = max(r0 - by, 0), y1 = min(r1 - by, 7);
  if (x0 > x1 || y0 > y1) return 0ull;
  const uint64_t cols = (uint64_t)((0xFFu >> (7 - x1)) & (0xFFu << x0)) * 0x0101010101010101ull;
  const uint64_t rows = (~0ull >> (8 * (7 - y1))) & (~0ull << (8 * y0));
  return cols & rows;
}

__device__ __forceinline__ uint64_t cover_lanes_rect(uint32_t cols, uint32_t rows, int bx, int by) {
  return block_lanes((int)(cols & 0xFFFF), (int)(cols >> 16), (int)(rows & 0xFFFF), (int)(rows >> 16), bx, by);
}

// Columns may wrap (c_lo > c_hi means [c_lo, W) u [0, c_hi]).
__device__ __forceinline__ uint64_t cover_lanes_wrap(uint32_t cols, uint32_t rows, int bx, int by) {
  const int c_lo = (int)(cols & 0xFFFF), c_hi = (int)(cols >> 16), r_lo = (int)(rows & 0xFFFF),
            r_hi = (int)(rows >> 16);
  if (c_lo <= c_hi) return block_lanes(c_lo, c_hi, r_lo, r_hi, bx, by);
  return block_lanes(c_lo, 0x7FFF, r_lo, r_hi, bx, by) | block_lanes(0, c_hi, r_lo, r_hi, bx, by);
}

__device__ __forceinline__ uint32_t rfl(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// Reads a wave-uniform 32-bit word (the same LDS record for every lane) into
// a scalar register.
__device__ __forceinline__ uint32_t uniform_u32(float v) {
  return (uint32_t)__builtin_amdgcn_readfirstlane((int)__float_as_uint(v));
}

// Grazing re-solve in FP64 (the pair's h'2 is near zero, where the FP32
// solve loses accuracy): G holds the record's FP64 plane rows and depth
// numerator, c its FP64 centre.  Camera: G = P (2 x 3 rows as 6) + mu_z,
// c = projected centre; LiDAR: G = Q (9) + |mu|, c = unit centre direction.
__device__ __forceinline__ bool solve64_pinhole(const double* G, const double* c, double px, double py, float& u,
                                                float& v, float& r, float& z) {
  const double ddx = px - c[0];
  const double ddy = py - c[1];
  const double H0 = G[0] * ddx + G[1] * ddy;
  const double H1 = G[2] * ddx + G[3] * ddy;
  const double H2 = 1.0 + G[4] * ddx + G[5] * ddy;
  const double rd = 1.0 / H2;
  u = (float)(H0 * rd);
  v = (float)(H1 * rd);
  r = (float)rd;
  z = (float)(G[6] * rd);
  return H2 != 0.0;
}

__device__ __forceinline__ bool solve64_lidar(const double* G, const double* c, const double* d64, float& u, float& v,
                                              float& r, float& z) {
  const double e0 = d64[0] - c[0], e1 = d64[1] - c[1], e2 = d64[2] - c[2];
  const double H0 = G[0] * e0 + G[1] * e1 + G[2] * e2;
  const double H1 = G[3] * e0 + G[4] * e1 + G[5] * e2;
  const double H2 = 1.0 + G[6] * e0 + G[7] * e1 + G[8] * e2;
  const double rd = 1.0 / H2;
  u = (float)(H0 * rd);
  v = (float)(H1 * rd);
  r = (float)rd;
  z = (float)(G[9] * rd);
  return H2 != 0.0;
}

// A surfel's record as read from global memory: 16 floats and its 4 doubles
// (camera: projected centre, -, packed pixel rectangle; LiDAR: unit centre
// direction, -), turned into the staged form per tile by the ray kind.
struct RawRec {
  float4 r[4];
  double2 d[2];
};

__device__ __forceinline__ void load_rec(const TileArgs& a, uint32_t s, RawRec& x) {
  const float4* r = a.rec + 4 * (size_t)s;
  const double2* r64 = reinterpret_cast<const double2*>(a.rec64 + kRec64 * (size_t)s);
#pragma unroll
  for (int i = 0; i < 4; ++i) x.r[i] = r[i];
  x.d[0] = r64[0];
  x.d[1] = r64[1];
}

// The FP64 re-solve data of record s into registers: G (NG doubles: the
// solve's rows and the centre depth or range) and its FP64 centre (NC
// doubles), from the record's LDS slot when it was staged there, else from
// global memory -- every load issued before any is used.
template <int NG, int NC>
__device__ __forceinline__ void fetch64(const TileArgs& a, const F64Slot* f64, uint32_t slot, const uint32_t* sid, double* g,
                                        double* c) {
  if (slot && f64) {
    const double* d = f64[slot - 1];
#pragma unroll
    for (int k = 0; k < NG; ++k) g[k] = d[k];
#pragma unroll
    for (int k = 0; k < NC; ++k) c[k] = d[kGrz + k];
  } else {
    // the surfel id (the batch slot's word, the same for every lane) is read
    // only here: the staged FP64 data cover nearly every re-solve
    const uint32_t s = rfl(*sid);
    const double* G = a.grz + kGrz * (size_t)s;
    const double* C = a.rec64 + kRec64 * (size_t)s;
#pragma unroll
    for (int k = 0; k < NG; ++k) g[k] = G[k];
#pragma unroll
    for (int k = 0; k < NC; ++k) c[k] = C[k];
  }
}

// ----------------------------- camera -----------------------------------
// Staged record (6 x float4), the fields every pair reads first:
//  [0] pcx_rel, pcy_rel, P00, P01
//  [1] P10, P11, P20, P21
//  [2] mu_z, log2 o, the rounding residuals of pcx_rel, pcy_rel
//  [3] flags, 2^-22 kappa (2^-21 for the cylindrical map: the pairs' FP32
//      error bound factor), c0, c1
//  [4] c2, n0, n1, n2
//  [5] pixel columns lo|hi<<16, pixel rows lo|hi<<16, the tile's error bound Et, -
// The centre in the tile frame is held as an FP32 pair (value + residual),
// so that the offset dx = (p_x - pcx_rel) - residual carries only its own
// rounding, not that of a centre up to a tile away.
__device__ __forceinline__ bool eval_pinhole(const float4* __restrict__ R, const uint32_t* sid, float plx, float ply, int ox,
                                             int oy, const TileArgs& a, const EvalK& K, const F64Slot* f64,
                                             PairEval& e, uint32_t& n64) {
#pragma clang fp contract(off)
  const float4 q0 = R[0], q1 = R[1], q2 = R[2];
  const uint32_t flags = uniform_u32(R[3].x);
  const float dx = (plx - q0.x) - q2.z;
  const float dy = (ply - q0.y) - q2.w;
  const float h0 = fmaf(q0.z, dx, q0.w * dy);
  const float h1 = fmaf(q1.x, dx, q1.y * dy);
  const float h2 = fmaf(q1.z, dx, fmaf(q1.w, dy, 1.0f));
  float r = __builtin_amdgcn_rcpf(h2);
  float u = h0 * r, v = h1 * r, z = q2.x * r;
  bool ok = h2 != 0.0f;
  const float rl = K.lp * fmaf(dx, dx, dy * dy);
  e.dx = dx;
  e.dy = dy;
  bool hit = finish_pair(u, v, r, z, ok, rl, q2.x, q2.y, K, e);
  // FP64 re-solve: grazing pairs (|h'_2| < 1/8) and an edge record's pairs
  // whose error bound could matter
  const uint32_t slot = (flags >> 8) & 0xFFu;
  bool redo = false;
  if (flags & (kFlagGrazing | kFlagEdge)) {  // the same record for the whole wave
    redo = (flags & kFlagGrazing) && fabsf(h2) < 0.125f;
    // the offsets carry two roundings of their size, the products two more
    // (the record holds 2^-22 kappa)
    if (flags & kFlagEdge)
      redo = redo | edge_needs_f64(e, fmaf(R[3].y, fmaxf(fabsf(dx), fabsf(dy)), 0x1p-20f), rl, flags, K);
  }
  if (redo) {
    ++n64;
    double g[7], c[2];
    fetch64<7, 2>(a, f64, slot, sid, g, c);
    ok = solve64_pinhole(g, c, (double)ox + (double)plx, (double)oy + (double)ply, u, v, r, z);
    hit = finish_pair(u, v, r, z, ok, rl, q2.x, q2.y, K, e);
  }
  return hit;
}

__device__ __forceinline__ uint2 stage_pinhole(const RawRec& x, int ox, int oy, float4* dst) {
  const float4 r0 = x.r[0], r1 = x.r[1], r2 = x.r[2], r3 = x.r[3];
  const double cx = x.d[0].x - (double)ox, cy = x.d[0].y - (double)oy;
  const float pcx = (float)cx, pcy = (float)cy;
  const uint2 rect = make_uint2((uint32_t)__double_as_longlong(x.d[1].y),
                                (uint32_t)((unsigned long long)__double_as_longlong(x.d[1].y) >> 32));
  // global record: P (6), mu_z, log2 o, c0..c2, n0..n2, flags, 2^-23 kappa
  dst[0] = make_float4(pcx, pcy, r0.x, r0.y);
  dst[1] = make_float4(r0.z, r0.w, r1.x, r1.y);
  dst[2] = make_float4(r1.z, r1.w, (float)(cx - (double)pcx), (float)(cy - (double)pcy));
  dst[3] = make_float4(r3.z, r3.w, r2.x, r2.y);
  dst[4] = make_float4(r2.z, r2.w, r3.x, r3.y);
  dst[5] = make_float4(__uint_as_float(rect.x), __uint_as_float(rect.y), 0.0f, 0.0f);
  return rect;
}

// Largest |offset| from the centre (at c, tile frame) over the pixel centres
// of [lo - 7, hi + 7] (an image-axis range of the surfel's rectangle, widened
// to the 8-pixel blocks that evaluate it) within the tile's [0, n).
__device__ __forceinline__ float max_offset(int lo, int hi, int o, int n, float c) {
  const float a = (float)max(lo - o - 7, 0) + 0.5f, b = (float)min(hi - o + 7, n - 1) + 0.5f;
  return fmaxf(fabsf(a - c), fabsf(b - c));
}

// One camera ray of a tile: lane geometry and the per-sensor pieces of the
// compositing loop (staging, skip test, solve, features, output, adjoint).
struct CamRay {
  static constexpr int C = 8;   // accumulated: rgb, depth, normal xyz, alpha
  static constexpr int CO = 9;  // output channels: the 8 sums and the median depth
  int px, py, ox, oy, bx, by, wx;
  float plx, ply;
  int tw, th;
  bool inside;
  EvalK K;

  __device__ CamRay(const TileArgs& a, int tile) : K(eval_consts(a, a.O.lp)) {
    const int WX = a.S.tw >> 3;
    wx = WX;
    const int tx = tile % a.S.n_tx, ty = tile / a.S.n_tx;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int lx = (w % WX) * 8 + (lane & 7), ly = (w / WX) * 8 + (lane >> 3);
    ox = tx * a.S.tw;
    oy = ty * a.S.th;
    bx = __builtin_amdgcn_readfirstlane(ox + (w % WX) * 8);
    by = __builtin_amdgcn_readfirstlane(oy + (w / WX) * 8);
    px = ox + lx;
    py = oy + ly;
    inside = px < a.S.W && py < a.S.H;
    plx = (float)lx + 0.5f;
    ply = (float)ly + 0.5f;
    tw = a.S.tw;
    th = a.S.th;
  }
  __device__ size_t pix(const TileArgs& a) const { return (size_t)py * a.S.W + px; }
  // the staged record, with its FP32 error bound over this tile: the offsets
  // carry about two roundings of their own size and the products two more,
  // so s = 2 |offset|_inf at the farthest pixel of the tile that evaluates
  // the record (plus slack for the roundings relative to u, v themselves),
  // over the smallest h'_2 there
  __device__ uint2 stage(const RawRec& x, float4* dst, const float (*)[6], int) const {
    const uint2 rect = stage_pinhole(x, ox, oy, dst);
    const float cx = dst[0].x, cy = dst[0].y;
    const float mdx = max_offset(rect.x & 0xFFFF, rect.x >> 16, ox, tw, cx);
    const float mdy = max_offset(rect.y & 0xFFFF, rect.y >> 16, oy, th, cy);
    const float h2m = 1.0f - (fabsf(dst[1].z) * mdx + fabsf(dst[1].w) * mdy);
    const float Et = fmaf(dst[3].y, fmaxf(mdx, mdy), 0x1p-20f) / fmaxf(h2m, 0.125f);
    set_tile_bound(dst[3].x, dst[5].z, Et, dst[2].y);
    return rect;
  }
  // does rectangle `rect` touch the 8x8 block of wave w?
  __device__ bool touches(uint2 rect, int w) const {
    return !misses_block(rect.x, rect.y, ox + (w % wx) * 8, oy + (w / wx) * 8);
  }
  // Bit w set unless the staged record d provably has no valid hit (rho_hat
  // within the cutoff and alpha >= alpha_min) at the pixel centres of wave
  // w's 8x8 block.  rho_hat = min(rho, low-pass) <= r2 needs either the
  // low-pass disc to reach the block or the surfel's (u, v) disc to meet the
  // block's image; the block maps to a projective quadrilateral whose u and v
  // ranges are attained at its corners (u, v are linear-fractional in the
  // pixel and h'2 > 0 on it), so the test is exact up to the (u, v) bounding
  // box and a rounding margin.  Grazing records keep every block.
  template <class SH>
  __device__ void prepare(const TileArgs&, SH&) const {}
  __device__ uint32_t hit_blocks(const float4* d, int nw, const float (*)[6]) const {
#pragma clang fp contract(off)
    const uint32_t all = (1u << nw) - 1u;
    const float4 q0 = d[0], q1 = d[1], q2 = d[2];
    if (__float_as_uint(d[3].x) & kFlagGrazing) return all;
    // largest rho_hat with alpha >= alpha_min: log2 o - rho_hat / (2 ln 2) >= log2 alpha_min
    const float ra = (q2.y - __log2f(K.alpha_min)) * (1.0f / kInv2Ln2);
    float r2 = fminf(K.cutoff2, ra);
    if (!(r2 >= 0.0f)) return 0u;
    r2 = r2 * 1.001f + 1e-3f;
    // slack for the corners' own FP32 error: twice the tile's bound
    const float sl = 2.0f * d[5].z;
    uint32_t m = 0u;
    for (int w = 0; w < nw; ++w) {
      const float x0 = (float)((w % wx) * 8) + 0.5f - q0.x, x1 = x0 + 7.0f;
      const float y0 = (float)((w / wx) * 8) + 0.5f - q0.y, y1 = y0 + 7.0f;
      if (K.lowpass) {
        const float ex = x0 > 0.0f ? x0 : (x1 < 0.0f ? -x1 : 0.0f);
        const float ey = y0 > 0.0f ? y0 : (y1 < 0.0f ? -y1 : 0.0f);
        if (K.lp * (ex * ex + ey * ey) <= r2) {
          m |= 1u << w;
          continue;
        }
      }
      const float xs[2] = {x0, x1}, ys[2] = {y0, y1};
      float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
      bool front = true;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float dx = xs[c & 1], dy = ys[c >> 1];
        const float h0 = q0.z * dx + q0.w * dy;
        const float h1 = q1.x * dx + q1.y * dy;
        const float h2 = 1.0f + q1.z * dx + q1.w * dy;
        front = front && h2 > 1e-6f;
        const float r = __builtin_amdgcn_rcpf(h2);
        const float u = h0 * r, v = h1 * r;
        umin = fminf(umin, u);
        umax = fmaxf(umax, u);
        vmin = fminf(vmin, v);
        vmax = fmaxf(vmax, v);
      }
      const float eu = fmaxf((umin > 0.0f ? umin : (umax < 0.0f ? -umax : 0.0f)) - sl, 0.0f);
      const float ev = fmaxf((vmin > 0.0f ? vmin : (vmax < 0.0f ? -vmax : 0.0f)) - sl, 0.0f);
      if (!front || !(eu * eu + ev * ev > r2)) m |= 1u << w;
    }
    return m;
  }
  __device__ bool covered(const float4* R) const {
    return covers(__float_as_uint(R[5].x), __float_as_uint(R[5].y), px, py);
  }
  __device__ uint64_t cover_lanes(const float4* R) const {
    return cover_lanes_rect(uniform_u32(R[5].x), uniform_u32(R[5].y), bx, by);
  }
  __device__ bool eval(const TileArgs& a, const float4* R, const uint32_t* sid, const F64Slot* f64, PairEval& e,
                       uint32_t& n64) const {
    return eval_pinhole(R, sid, plx, ply, ox, oy, a, K, f64, e, n64);
  }
  static __device__ float& flag_word(float4* R) { return R[3].x; }
  __device__ void feat(const float4* R, const PairEval& e, float* f) const {
    f[0] = R[3].z;
    f[1] = R[3].w;
    f[2] = R[4].x;
    f[3] = e.z;
    f[4] = R[4].y;
    f[5] = R[4].z;
    f[6] = R[4].w;
    f[7] = 1.0f;
  }
  // output channels of a ray with final transmittance T and sums acc; the
  // median channel is left 0 here (the compositing pass that knows the ray's
  // incoming transmittance, or the median pass, writes it)
  static __device__ void out_values(const TileArgs& a, float T, const float* acc, float* v) {
#pragma clang fp contract(off)
    v[0] = fmaf(T, a.O.bg0, acc[0]);
    v[1] = fmaf(T, a.O.bg1, acc[1]);
    v[2] = fmaf(T, a.O.bg2, acc[2]);
#pragma unroll
    for (int c = 3; c < 8; ++c) v[c] = acc[c];
    v[8] = 0.0f;
  }
  static constexpr int kMedian = 8;  // output channel of the median depth
  // outputs of a split tile's ray that finishes after a walk (the median
  // channel and pair were written by its segment passes)
  __device__ void write(const TileArgs& a, float T, const float* acc, uint32_t last) const {
    const size_t HW = (size_t)a.S.W * a.S.H, p = pix(a);
    float v[CO];
    out_values(a, T, acc, v);
#pragma unroll
    for (int c = 0; c < CO; ++c)
      if (c != kMedian) a.out[c * HW + p] = v[c];
    a.T_final[p] = T;
    a.n_last[p] = last;
  }
  // Per-record gradient fields of one pair given dL/dalpha (dal) and the
  // pair's weight wgt = alpha T: [0..5] dP, [6..7] d(projected centre),
  // [8] d mu_z, [9] d opacity, [10..12] d colour, [13..15] d normal.
  // gzx: a further dL/d(depth) of this pair (the median depth's, at its pair)
  __device__ void grads(const TileArgs& a, const float4* R, const PairEval& e, float dal, float wgt, const float* g,
                        float gzx, float* gr) const {
#pragma clang fp contract(off)
    const float4 q0 = R[0], q1 = R[1];
    const float o = __builtin_amdgcn_exp2f(R[2].y);
    const float al = e.alpha;
    gr[10] = g[0] * wgt;
    gr[11] = g[1] * wgt;
    gr[12] = g[2] * wgt;
    gr[13] = g[4] * wgt;
    gr[14] = g[5] * wgt;
    gr[15] = g[6] * wgt;
    const float gz = fmaf(g[3], wgt, gzx);
    float g_rhohat = 0.0f;
    if (!e.clamped) {
      gr[9] = o > 0.0f ? dal * al * __builtin_amdgcn_rcpf(o) : 0.0f;
      g_rhohat = -0.5f * dal * al;
    }
    const float g_rho = e.lp_used ? 0.0f : g_rhohat;
    const float g_lp = e.lp_used ? g_rhohat : 0.0f;
    const float gu = 2.0f * e.u * g_rho, gv = 2.0f * e.v * g_rho;
    const float gh0 = gu * e.r, gh1 = gv * e.r;
    // depth = mu_z h'2^-1 at the plane hit, mu_z itself for a low-pass pair
    const float gzh = e.lp_used ? 0.0f : gz;
    const float gh2 = -(gu * e.u + gv * e.v + gzh * e.z) * e.r;
    gr[8] = e.lp_used ? gz : gz * e.r;
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
  }
};

// ------------------------- cylindrical camera ---------------------------
// A surfel's record is the camera record in its own column frame (the sensor
// frame turned about y by the centre's angle): the ray of a pixel at angle
// offset dphi = dx / f_x from the centre's column is the pinhole ray
// (tan dphi, y_n sec dphi, 1) there, so the per-pair solve is the camera's on
//   X = f_x tan dphi,   Y = dy + (p_y - c_y)(sec dphi - 1)
// (Y = f_y (y_n sec dphi - y_n,centre)), and the depth -- the distance from
// the vertical axis -- is r sec dphi / h'_2 (r = the centre's distance).

// sin and cos for the angle offsets of a cylindrical camera (|x| < 16, far
// beyond the 3 pi a full-circle camera can produce): Cody-Waite reduction by
// pi/2 in two parts, then the Taylor series of sin and cos on |r| <= pi/4
// (truncation below 2e-9 relative in FP32, 1e-19 in FP64).  Written out so
// that the pair loop carries no large-argument reduction.
__device__ __forceinline__ bool sincos_small(float x, float& s, float& c) {
#pragma clang fp contract(off)
  if (!(fabsf(x) < 16.0f)) return false;
  const float k = rintf(x * 0.63661977236758134f);
  const float r = fmaf(-k, -4.37113900018624283e-8f, fmaf(-k, 1.57079637050628662f, x));  // x - k pi/2
  const float r2 = r * r;
  float ps = fmaf(r2, 1.0f / 362880.0f, -1.0f / 5040.0f);
  ps = fmaf(r2, ps, 1.0f / 120.0f);
  ps = fmaf(r2, ps, -1.0f / 6.0f);
  const float sr = fmaf(r * r2, ps, r);
  float pc = fmaf(r2, -1.0f / 3628800.0f, 1.0f / 40320.0f);
  pc = fmaf(r2, pc, -1.0f / 720.0f);
  pc = fmaf(r2, pc, 1.0f / 24.0f);
  pc = fmaf(r2, pc, -0.5f);
  const float cr = fmaf(r2, pc, 1.0f);
  const int q = (int)k & 3;
  s = (q & 1) ? cr : sr;
  c = (q & 1) ? sr : cr;
  if (q == 1 || q == 2) c = -c;
  if (q >= 2) s = -s;
  return true;
}

__device__ __forceinline__ bool sincos_small(double x, double& s, double& c) {
  if (!(fabs(x) < 16.0)) return false;
  const double k = rint(x * 0.63661977236758134308);
  const double r = fma(-k, 6.123233995736766036e-17, fma(-k, 1.5707963267948965580, x));  // x - k pi/2
  const double r2 = r * r;
  // sin: 1/(2n+1)! through r^17; cos: 1/(2n)! through r^18
  double ps = fma(r2, 1.0 / 355687428096000.0, -1.0 / 1307674368000.0);
  ps = fma(r2, ps, 1.0 / 6227020800.0);
  ps = fma(r2, ps, -1.0 / 39916800.0);
  ps = fma(r2, ps, 1.0 / 362880.0);
  ps = fma(r2, ps, -1.0 / 5040.0);
  ps = fma(r2, ps, 1.0 / 120.0);
  ps = fma(r2, ps, -1.0 / 6.0);
  const double sr = fma(r * r2, ps, r);
  double pc = fma(r2, -1.0 / 6402373705728000.0, 1.0 / 20922789888000.0);
  pc = fma(r2, pc, -1.0 / 87178291200.0);
  pc = fma(r2, pc, 1.0 / 479001600.0);
  pc = fma(r2, pc, -1.0 / 3628800.0);
  pc = fma(r2, pc, 1.0 / 40320.0);
  pc = fma(r2, pc, -1.0 / 720.0);
  pc = fma(r2, pc, 1.0 / 24.0);
  pc = fma(r2, pc, -0.5);
  const double cr = fma(r2, pc, 1.0);
  const int q = (int)k & 3;
  s = (q & 1) ? cr : sr;
  c = (q & 1) ? sr : cr;
  if (q == 1 || q == 2) c = -c;
  if (q >= 2) s = -s;
  return true;
}

// tan x and sec x - 1.  |x| <= 1/4: their Taylor series through x^11 and x^10
// (relative error < 1e-8 there); beyond, from sin and cos.  Returns false
// where cos x <= 0: such a ray looks away from the surfel's column by more
// than 90 degrees, so it cannot meet a visible surfel's support (the rays
// that do are within asin(R / r) < 90 degrees of it).
__device__ __forceinline__ bool tan_secm1(float x, float& t, float& sm1) {
#pragma clang fp contract(off)
  if (fabsf(x) <= 0.25f) {
    const float x2 = x * x;
    // tan: 1, 1/3, 2/15, 17/315, 62/2835, 1382/155925
    float p = fmaf(x2, 1382.0f / 155925.0f, 62.0f / 2835.0f);
    p = fmaf(x2, p, 17.0f / 315.0f);
    p = fmaf(x2, p, 2.0f / 15.0f);
    p = fmaf(x2, p, 1.0f / 3.0f);
    t = fmaf(x * x2, p, x);
    // sec - 1: 1/2, 5/24, 61/720, 277/8064, 50521/3628800
    float q = fmaf(x2, 50521.0f / 3628800.0f, 277.0f / 8064.0f);
    q = fmaf(x2, q, 61.0f / 720.0f);
    q = fmaf(x2, q, 5.0f / 24.0f);
    q = fmaf(x2, q, 0.5f);
    sm1 = x2 * q;
    return true;
  }
  float sn = 0.0f, cs = 0.0f;
  if (!sincos_small(x, sn, cs) || !(cs > 0.0f)) {
    t = 0.0f;
    sm1 = 0.0f;
    return false;
  }
  const float rc = 1.0f / cs;
  t = sn * rc;
  sm1 = (sn * sn) * rc / (1.0f + cs);
  return true;
}

// Per-sensor constants of the cylindrical mapping, in vector registers.
struct CylK {
  float fx, ifx;  // f_x and 1 / f_x
};

// Grazing re-solve in FP64: the pixel's ray turned into the record's column
// frame is (tan dphi, y_n sec dphi, 1), dphi = (p_x - pc_x) / f_x exactly.
// G = P (6) + r, c = projected centre.
__device__ __forceinline__ bool solve64_cyl(const double* G, const double* c, const SensorK& S, int col, int row,
                                            float& u, float& v, float& r, float& z) {
  const double dphi = ((double)col + 0.5 - c[0]) / (double)S.fx;
  double sn, cs;
  if (!sincos_small(dphi, sn, cs) || !(cs > 0.0)) return false;
  const double sec = 1.0 / cs;
  const double X = (double)S.fx * (sn * sec);
  const double Y = ((double)row + 0.5 - (double)S.cy) * sec - (c[1] - (double)S.cy);
  const double H0 = G[0] * X + G[1] * Y;
  const double H1 = G[2] * X + G[3] * Y;
  const double H2 = 1.0 + G[4] * X + G[5] * Y;
  const double rd = 1.0 / H2;
  u = (float)(H0 * rd);
  v = (float)(H1 * rd);
  r = (float)rd;
  z = (float)(G[6] * rd * sec);
  return H2 != 0.0;
}

__device__ __forceinline__ bool eval_cyl(const float4* __restrict__ R, const uint32_t* sid, float plx, float ply, float Ay,
                                         int px, int py, const TileArgs& a, const EvalK& K, const CylK& Y0,
                                         const F64Slot* f64, PairEval& e, uint32_t& n64) {
#pragma clang fp contract(off)
  const float4 q0 = R[0], q1 = R[1], q2 = R[2];
  const uint32_t flags = uniform_u32(R[3].x);
  const float dx = (plx - q0.x) - q2.z;
  const float dy = (ply - q0.y) - q2.w;
  float tn, sm1;
  bool ok = tan_secm1(dx * Y0.ifx, tn, sm1);
  const float X = Y0.fx * tn;
  const float Y = fmaf(Ay, sm1, dy);
  const float h0 = fmaf(q0.z, X, q0.w * Y);
  const float h1 = fmaf(q1.x, X, q1.y * Y);
  const float h2 = fmaf(q1.z, X, fmaf(q1.w, Y, 1.0f));
  float r = __builtin_amdgcn_rcpf(h2);
  float u = h0 * r, v = h1 * r, z = (q2.x * r) * (1.0f + sm1);
  ok = ok && h2 != 0.0f;
  const float rl = K.lp * fmaf(dx, dx, dy * dy);
  e.dx = dx;
  e.dy = dy;
  bool hit = finish_pair(u, v, r, z, ok, rl, q2.x, q2.y, K, e);
  // FP64 re-solve as for the pinhole camera
  const uint32_t slot = (flags >> 8) & 0xFFu;
  bool redo = false;
  if (flags & (kFlagGrazing | kFlagEdge)) {
    redo = (flags & kFlagGrazing) && fabsf(h2) < 0.125f;
    // X = f tan and Y = dy + A (sec - 1) take about twice the pinhole's
    // roundings (the record holds 2^-21 kappa)
    if (flags & kFlagEdge)
      redo = redo | edge_needs_f64(e, fmaf(R[3].y, fmaxf(fabsf(X), fabsf(Y)), 0x1p-20f), rl, flags, K);
  }
  if (redo) {
    ++n64;
    double g[7], c[2];
    fetch64<7, 2>(a, f64, slot, sid, g, c);
    ok = solve64_cyl(g, c, a.S, px, py, u, v, r, z);
    hit = finish_pair(u, v, r, z, ok, rl, q2.x, q2.y, K, e);
  }
  return hit;
}

// One cylindrical-camera ray of a tile: the camera ray with the column-frame
// mapping (see above); records, features and outputs are the camera's.
struct CylRay {
  static constexpr int C = 8;   // accumulated: rgb, depth, normal xyz, alpha
  static constexpr int CO = 9;  // output channels: the 8 sums and the median depth
  static constexpr int kMedian = 8;
  int px, py, ox, oy, bx, by, wx;
  int tc, tr;               // pixel column and row of the ray (inside the image for every lane)
  float plx, ply, Ay, ay0;  // Ay: p_y - c_y of this ray; ay0: of the tile's first row
  int tw, th;
  bool inside;
  EvalK K;
  CylK Y0;

  __device__ CylRay(const TileArgs& a, int tile) : K(eval_consts(a, a.O.lp)) {
    const int WX = a.S.tw >> 3;
    wx = WX;
    const int tx = tile % a.S.n_tx, ty = tile / a.S.n_tx;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int lx = (w % WX) * 8 + (lane & 7), ly = (w / WX) * 8 + (lane >> 3);
    ox = tx * a.S.tw;
    oy = ty * a.S.th;
    bx = __builtin_amdgcn_readfirstlane(ox + (w % WX) * 8);
    by = __builtin_amdgcn_readfirstlane(oy + (w / WX) * 8);
    px = ox + lx;
    py = oy + ly;
    inside = px < a.S.W && py < a.S.H;
    tc = px < a.S.W ? px : ox;
    tr = py < a.S.H ? py : oy;
    plx = (float)lx + 0.5f;
    ply = (float)ly + 0.5f;
    Ay = ((float)py + 0.5f) - a.S.cy;
    ay0 = ((float)oy + 0.5f) - a.S.cy;
    Y0.fx = in_vgpr(a.S.fx);
    Y0.ifx = in_vgpr(1.0f / a.S.fx);
    tw = a.S.tw;
    th = a.S.th;
  }
  __device__ size_t pix(const TileArgs& a) const { return (size_t)py * a.S.W + px; }
  // the staged record, with its FP32 error bound over this tile: as the
  // pinhole camera's on the (X, Y) box of the tile's pixels (columns up to 80
  // degrees from the centre's; a tile reaching beyond is wild), doubled for
  // the extra rounding steps of X = f tan and Y = dy + A (sec - 1)
  __device__ uint2 stage(const RawRec& x, float4* dst, const float (*)[6], int) const {
#pragma clang fp contract(off)
    const uint2 rect = stage_pinhole(x, ox, oy, dst);
    const float cx = dst[0].x, cy = dst[0].y;
    const float mdx = max_offset(rect.x & 0xFFFF, rect.x >> 16, ox, tw, cx);
    const float mdy = max_offset(rect.y & 0xFFFF, rect.y >> 16, oy, th, cy);
    const float ang = mdx * Y0.ifx;
    float Et = INFINITY;
    float tn, sm1;
    if (ang <= 1.39f && tan_secm1(ang, tn, sm1)) {
      const float Aym = fmaxf(fabsf(ay0), fabsf(ay0 + (float)(th - 1)));
      const float Xm = Y0.fx * tn, Ym = mdy + Aym * sm1;
      const float h2m = 1.0f - (fabsf(dst[1].z) * Xm + fabsf(dst[1].w) * Ym);
      Et = fmaf(dst[3].y, fmaxf(Xm, Ym), 0x1p-20f) / fmaxf(h2m, 0.125f);
    }
    set_tile_bound(dst[3].x, dst[5].z, Et, dst[2].y);
    return rect;
  }
  __device__ bool touches(uint2 rect, int w) const {
    return !misses_block(rect.x, rect.y, ox + (w % wx) * 8, oy + (w / wx) * 8);
  }
  template <class SH>
  __device__ void prepare(const TileArgs&, SH&) const {}
  // The camera's block test on the box of (X, Y) over the block: X = f tan
  // is monotone in the pixel offset, sec - 1 is even and grows with |dphi|,
  // and Y = dy + (p_y - c_y)(sec - 1) is bounded by the interval products;
  // u and v, linear-fractional in (X, Y), take their ranges at the box's
  // corners.  Blocks that reach 90 degrees from the centre's column are kept.
  __device__ uint32_t hit_blocks(const float4* d, int nw, const float (*)[6]) const {
#pragma clang fp contract(off)
    const uint32_t all = (1u << nw) - 1u;
    const float4 q0 = d[0], q1 = d[1], q2 = d[2];
    if (__float_as_uint(d[3].x) & kFlagGrazing) return all;
    const float ra = (q2.y - __log2f(K.alpha_min)) * (1.0f / kInv2Ln2);
    float r2 = fminf(K.cutoff2, ra);
    if (!(r2 >= 0.0f)) return 0u;
    r2 = r2 * 1.001f + 1e-3f;
    // slack for the corners' own FP32 error: twice the tile's bound
    const float sl = 2.0f * d[5].z;
    uint32_t m = 0u;
    for (int w = 0; w < nw; ++w) {
      const float x0 = (float)((w % wx) * 8) + 0.5f - q0.x, x1 = x0 + 7.0f;
      const float y0 = (float)((w / wx) * 8) + 0.5f - q0.y, y1 = y0 + 7.0f;
      if (K.lowpass) {
        const float ex = x0 > 0.0f ? x0 : (x1 < 0.0f ? -x1 : 0.0f);
        const float ey = y0 > 0.0f ? y0 : (y1 < 0.0f ? -y1 : 0.0f);
        if (K.lp * (ex * ex + ey * ey) <= r2) {
          m |= 1u << w;
          continue;
        }
      }
      float t0, s0, t1, s1;
      if (!tan_secm1(x0 * Y0.ifx, t0, s0) || !tan_secm1(x1 * Y0.ifx, t1, s1)) {
        m |= 1u << w;
        continue;
      }
      const float smin = (x0 <= 0.0f && x1 >= 0.0f) ? 0.0f : fminf(s0, s1), smax = fmaxf(s0, s1);
      const float A0 = ay0 + (float)((w / wx) * 8), A1 = A0 + 7.0f;
      const float pa = A0 * smin, pb = A0 * smax, pc = A1 * smin, pd = A1 * smax;
      float Xlo = Y0.fx * t0, Xhi = Y0.fx * t1;
      float Ylo = y0 + fminf(fminf(pa, pb), fminf(pc, pd)), Yhi = y1 + fmaxf(fmaxf(pa, pb), fmaxf(pc, pd));
      // rounding margins: the per-pair X, Y are FP32 values of the same maps
      const float mX = 1e-5f * fmaxf(fabsf(Xlo), fabsf(Xhi)) + 1e-4f;
      const float mY = 1e-5f * (fmaxf(fabsf(Ylo), fabsf(Yhi)) + fmaxf(fabsf(A0), fabsf(A1))) + 1e-4f;
      Xlo -= mX;
      Xhi += mX;
      Ylo -= mY;
      Yhi += mY;
      const float xs[2] = {Xlo, Xhi}, ys[2] = {Ylo, Yhi};
      float umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
      bool front = true;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const float X = xs[c & 1], Y = ys[c >> 1];
        const float h0 = q0.z * X + q0.w * Y;
        const float h1 = q1.x * X + q1.y * Y;
        const float h2 = 1.0f + q1.z * X + q1.w * Y;
        front = front && h2 > 1e-6f;
        const float r = __builtin_amdgcn_rcpf(h2);
        const float u = h0 * r, v = h1 * r;
        umin = fminf(umin, u);
        umax = fmaxf(umax, u);
        vmin = fminf(vmin, v);
        vmax = fmaxf(vmax, v);
      }
      const float eu = fmaxf((umin > 0.0f ? umin : (umax < 0.0f ? -umax : 0.0f)) - sl, 0.0f);
      const float ev = fmaxf((vmin > 0.0f ? vmin : (vmax < 0.0f ? -vmax : 0.0f)) - sl, 0.0f);
      if (!front || !(eu * eu + ev * ev > r2)) m |= 1u << w;
    }
    return m;
  }
  __device__ bool covered(const float4* R) const {
    return covers(__float_as_uint(R[5].x), __float_as_uint(R[5].y), px, py);
  }
  __device__ uint64_t cover_lanes(const float4* R) const {
    return cover_lanes_rect(uniform_u32(R[5].x), uniform_u32(R[5].y), bx, by);
  }
  __device__ bool eval(const TileArgs& a, const float4* R, const uint32_t* sid, const F64Slot* f64, PairEval& e,
                       uint32_t& n64) const {
    return eval_cyl(R, sid, plx, ply, Ay, tc, tr, a, K, Y0, f64, e, n64);
  }
  static __device__ float& flag_word(float4* R) { return R[3].x; }
  __device__ void feat(const float4* R, const PairEval& e, float* f) const {
    f[0] = R[3].z;
    f[1] = R[3].w;
    f[2] = R[4].x;
    f[3] = e.z;
    f[4] = R[4].y;
    f[5] = R[4].z;
    f[6] = R[4].w;
    f[7] = 1.0f;
  }
  static __device__ void out_values(const TileArgs& a, float T, const float* acc, float* v) {
    CamRay::out_values(a, T, acc, v);
  }
  __device__ void write(const TileArgs& a, float T, const float* acc, uint32_t last) const {
    const size_t HW = (size_t)a.S.W * a.S.H, p = pix(a);
    float v[CO];
    out_values(a, T, acc, v);
#pragma unroll
    for (int c = 0; c < CO; ++c)
      if (c != kMedian) a.out[c * HW + p] = v[c];
    a.T_final[p] = T;
    a.n_last[p] = last;
  }
  // The camera's fields: [0..5] dP, [6..7] d(projected centre), [8] d r (the
  // record's centre distance), [9] d opacity, [10..12] d colour, [13..15]
  // d normal; the offsets enter through X, Y and the depth's sec factor.
  __device__ void grads(const TileArgs& a, const float4* R, const PairEval& e, float dal, float wgt, const float* g,
                        float gzx, float* gr) const {
#pragma clang fp contract(off)
    const float4 q0 = R[0], q1 = R[1], q2 = R[2];
    const float o = __builtin_amdgcn_exp2f(q2.y);
    const float al = e.alpha;
    gr[10] = g[0] * wgt;
    gr[11] = g[1] * wgt;
    gr[12] = g[2] * wgt;
    gr[13] = g[4] * wgt;
    gr[14] = g[5] * wgt;
    gr[15] = g[6] * wgt;
    const float gz = fmaf(g[3], wgt, gzx);
    float g_rhohat = 0.0f;
    if (!e.clamped) {
      gr[9] = o > 0.0f ? dal * al * __builtin_amdgcn_rcpf(o) : 0.0f;
      g_rhohat = -0.5f * dal * al;
    }
    const float g_rho = e.lp_used ? 0.0f : g_rhohat;
    const float g_lp = e.lp_used ? g_rhohat : 0.0f;
    float tn, sm1;
    (void)tan_secm1(e.dx * Y0.ifx, tn, sm1);
    const float sec = 1.0f + sm1;
    const float X = Y0.fx * tn;
    const float Y = fmaf(Ay, sm1, e.dy);
    const float gu = 2.0f * e.u * g_rho, gv = 2.0f * e.v * g_rho;
    const float gh0 = gu * e.r, gh1 = gv * e.r;
    // depth = r sec / h'_2 at the plane hit, r itself for a low-pass pair
    const float gzh = e.lp_used ? 0.0f : gz;
    const float gh2 = -(gu * e.u + gv * e.v + gzh * e.z) * e.r;
    gr[8] = e.lp_used ? gz : gz * e.r * sec;
    gr[0] = gh0 * X;
    gr[1] = gh0 * Y;
    gr[2] = gh1 * X;
    gr[3] = gh1 * Y;
    gr[4] = gh2 * X;
    gr[5] = gh2 * Y;
    const float gX = q0.z * gh0 + q1.x * gh1 + q1.z * gh2;
    const float gY = q0.w * gh0 + q1.y * gh1 + q1.w * gh2;
    // d/d dx: X' = sec^2, Y' = (p_y - c_y) sec tan / f_x, depth' = depth tan / f_x
    const float st = sec * tn * Y0.ifx;
    const float two_lp = 2.0f * a.O.lp * g_lp;
    const float gdx = gX * (sec * sec) + gY * (Ay * st) + gzh * e.z * tn * Y0.ifx + two_lp * e.dx;
    const float gdy = gY + two_lp * e.dy;
    gr[6] = -gdx;
    gr[7] = -gdy;
    (void)q2;
  }
};

// ----------------------------- LiDAR -------------------------------------
// Staged record (6 x float4), the fields every pair reads first:
//  [0] c0, c1, c2 (= d_tile - mu_hat), Q00   [1] Q01, Q02, Q10, Q11
//  [2] Q12, Q20, Q21, Q22                    [3] |mu|, log2 o, 2^-23 kappa, flags
//  [4] intensity, columns lo|hi<<16 (may wrap), beams lo|hi<<16, the tile's error bound Et
//  [5] ray-drop probability, -, -, -
__device__ __forceinline__ uint2 stage_lidar(const RawRec& x, const double* dtile, float4* dst) {
  // global record: Q (9), |mu|, log2 o, intensity, flags, 2^-23 kappa, columns,
  // beams; FP64 record: unit centre direction, ray-drop probability
  const float4 r0 = x.r[0], r1 = x.r[1], r2 = x.r[2], r3 = x.r[3];
  const float c0 = (float)(dtile[0] - x.d[0].x);
  const float c1 = (float)(dtile[1] - x.d[0].y);
  const float c2 = (float)(dtile[2] - x.d[1].x);
  dst[0] = make_float4(c0, c1, c2, r0.x);
  dst[1] = make_float4(r0.y, r0.z, r0.w, r1.x);
  dst[2] = make_float4(r1.y, r1.z, r1.w, r2.x);
  dst[3] = make_float4(r2.y, r2.z, r3.y, r3.x);
  dst[4] = make_float4(r2.w, r3.z, r3.w, 0.0f);
  dst[5] = make_float4((float)x.d[1].y, 0.0f, 0.0f, 0.0f);
  return make_uint2(__float_as_uint(r3.z), __float_as_uint(r3.w));
}

__device__ __forceinline__ bool eval_lidar(const float4* __restrict__ R, const uint32_t* sid, const float* dpix, float dpm,
                                           const double* d64, const TileArgs& a, const EvalK& K, const F64Slot* f64,
                                           PairEval& e, uint32_t& n64) {
#pragma clang fp contract(off)
  const float4 q0 = R[0], q1 = R[1], q2 = R[2], q3 = R[3];
  const uint32_t flags = uniform_u32(q3.w);
  const float d0 = dpix[0] + q0.x;
  const float d1 = dpix[1] + q0.y;
  const float d2 = dpix[2] + q0.z;
  const float h0 = fmaf(q0.w, d0, fmaf(q1.x, d1, q1.y * d2));
  const float h1 = fmaf(q1.z, d0, fmaf(q1.w, d1, q2.x * d2));
  const float h2 = fmaf(q2.y, d0, fmaf(q2.z, d1, fmaf(q2.w, d2, 1.0f)));
  float r = __builtin_amdgcn_rcpf(h2);
  float u = h0 * r, v = h1 * r, z = q3.x * r;
  bool ok = h2 != 0.0f;
  const float rl = K.lp * fmaf(d0, d0, fmaf(d1, d1, d2 * d2));
  e.dx = d0;
  e.dy = d1;
  e.dz3 = d2;
  // the centre's range |mu| for low-pass pairs (see eval_pinhole)
  bool hit = finish_pair(u, v, r, z, ok, rl, q3.x, q3.y, K, e);
  // FP64 re-solve as for the pinhole camera
  const uint32_t slot = (flags >> 8) & 0xFFu;
  bool redo = false;
  if (flags & (kFlagGrazing | kFlagEdge)) {
    redo = (flags & kFlagGrazing) && fabsf(h2) < 0.125f;
    if (flags & kFlagEdge) {
      // the roundings of dpix and of c, then two of d's size and two in the
      // products (the record holds 2^-23 kappa)
      const float dm = fmaxf(fmaxf(fabsf(d0), fabsf(d1)), fabsf(d2));
      const float cm = fmaxf(fmaxf(fabsf(q0.x), fabsf(q0.y)), fabsf(q0.z));
      redo = redo | edge_needs_f64(e, fmaf(q3.z, fmaf(2.0f, dm, dpm + cm), 0x1p-20f), rl, flags, K);
    }
  }
  if (redo) {
    ++n64;
    double g[10], c[3];
    fetch64<10, 3>(a, f64, slot, sid, g, c);
    ok = solve64_lidar(g, c, d64, u, v, r, z);
    hit = finish_pair(u, v, r, z, ok, rl, q3.x, q3.y, K, e);
  }
  return hit;
}

// Ray direction of LiDAR column c, beam j, in FP64: the line where the two
// planes of Eq. 5 built from the FP32 tables meet, h_u x h_v =
// (ce ca, ce sa, se (ca^2 + sa^2)).  The rounded tables make ca^2 + sa^2
// differ from 1 by ~1e-7; a surfel met nearly edge-on (the low-pass filter
// admits such pairs) amplifies that into its hit range by 1/h'2, so the
// solve must use the planes' own line, not the nominal unit beam.
__device__ inline void lidar_dir(const SensorK& S, int c, int j, double* d) {
  const float* t = S.tab;
  const double ce = t[S.H + j], se = t[2 * S.H + j], ca = t[3 * S.H + c], sa = t[3 * S.H + S.W + c];
  d[0] = ce * ca;
  d[1] = ce * sa;
  d[2] = se * (ca * ca + sa * sa);
}

struct LidarRay {
  static constexpr int C = 4;   // accumulated: range, intensity, alpha, ray drop
  static constexpr int CO = 6;  // output channels: range, intensity, alpha, drop probability,
                                // drop mask, median range
  static constexpr int kMedian = 5;
  int pc, pb, bx, by, ox, oy, wx;
  bool inside;
  EvalK K;
  double dt[3], d64[3];
  float dpix[3], dpm;  // dpm: max |dpix|

  __device__ LidarRay(const TileArgs& a, int tile) : K(eval_consts(a, a.S.lp_ang)) {
    const int WX = a.S.tw >> 3;
    const int tx = tile % a.S.n_tx, ty = tile / a.S.n_tx;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int lx = (w % WX) * 8 + (lane & 7), ly = (w / WX) * 8 + (lane >> 3);
    ox = tx * a.S.tw;
    oy = ty * a.S.th;
    wx = WX;
    bx = __builtin_amdgcn_readfirstlane(ox + (w % WX) * 8);
    by = __builtin_amdgcn_readfirstlane(oy + (w / WX) * 8);
    pc = ox + lx;
    pb = oy + ly;
    inside = pc < a.S.W && pb < a.S.H;
    lidar_dir(a.S, ox, oy, dt);
    lidar_dir(a.S, inside ? pc : ox, inside ? pb : oy, d64);
    dpix[0] = (float)(d64[0] - dt[0]);
    dpix[1] = (float)(d64[1] - dt[1]);
    dpix[2] = (float)(d64[2] - dt[2]);
    dpm = fmaxf(fmaxf(fabsf(dpix[0]), fabsf(dpix[1])), fabsf(dpix[2]));
  }
  __device__ size_t pix(const TileArgs& a) const { return (size_t)pb * a.S.W + pc; }
  // the staged record, with its FP32 error bound over this tile: as the
  // camera's, with the offset d = dpix + c bounded by |c| plus the largest
  // |dpix| of the blocks that evaluate the record (their direction boxes),
  // |dpix| and |c| counted once more for their own roundings
  __device__ uint2 stage(const RawRec& x, float4* dst, const float (*box)[6], int nw) const {
#pragma clang fp contract(off)
    const uint2 rect = stage_lidar(x, dt, dst);
    float m[3] = {0.0f, 0.0f, 0.0f};
    for (int w = 0; w < nw; ++w) {
      if (!touches(rect, w)) continue;  // no pair of this block is evaluated
#pragma unroll
      for (int k = 0; k < 3; ++k) m[k] = fmaxf(m[k], fmaxf(fabsf(box[w][2 * k]), fabsf(box[w][2 * k + 1])));
    }
    const float c0 = fabsf(dst[0].x), c1 = fabsf(dst[0].y), c2 = fabsf(dst[0].z);
    const float h2m = 1.0f - (fabsf(dst[2].y) * (c0 + m[0]) + fabsf(dst[2].z) * (c1 + m[1]) + fabsf(dst[2].w) * (c2 + m[2]));
    const float mi = fmaxf(fmaxf(c0 + m[0], c1 + m[1]), c2 + m[2]), mp = fmaxf(fmaxf(m[0], m[1]), m[2]);
    const float mc = fmaxf(fmaxf(c0, c1), c2);
    const float Et = fmaf(dst[3].z, 2.0f * mi + mp + mc, 0x1p-20f) / fmaxf(h2m, 0.125f);
    set_tile_bound(dst[3].w, dst[4].w, Et, dst[3].y);
    return rect;
  }
  __device__ bool touches(uint2 rect, int w) const {
    return !misses_block_wrap(rect.x, rect.y, ox + (w % wx) * 8, oy + (w / wx) * 8);
  }
  // Box of the ray directions of wave w's 8x8 block, relative to the tile's
  // reference direction (dpix range per component), into LDS (threads
  // w < nw).  The directions are products of the elevation and azimuth table
  // entries, so each component's range is an interval product.
  template <class SH>
  __device__ void prepare(const TileArgs& a, SH& sh) const {
    const int w = threadIdx.x;
    if (w >= (int)(sizeof(sh.lbox) / sizeof(sh.lbox[0])) || w >= (int)(blockDim.x >> 6)) return;
    const float* tb = a.S.tab;
    const int c0 = ox + (w % wx) * 8, j0 = oy + (w / wx) * 8;
    const int c1 = min(c0 + 7, a.S.W - 1), j1 = min(j0 + 7, a.S.H - 1);
    float ce_lo = INFINITY, ce_hi = -INFINITY, se_lo = INFINITY, se_hi = -INFINITY;
    float ca_lo = INFINITY, ca_hi = -INFINITY, sa_lo = INFINITY, sa_hi = -INFINITY;
    for (int j = j0; j <= min(j1, j0 + 7); ++j) {
      const float ce = tb[a.S.H + j], se = tb[2 * a.S.H + j];
      ce_lo = fminf(ce_lo, ce);
      ce_hi = fmaxf(ce_hi, ce);
      se_lo = fminf(se_lo, se);
      se_hi = fmaxf(se_hi, se);
    }
    for (int c = c0; c <= min(c1, c0 + 7); ++c) {
      const float ca = tb[3 * a.S.H + c], sa = tb[3 * a.S.H + a.S.W + c];
      ca_lo = fminf(ca_lo, ca);
      ca_hi = fmaxf(ca_hi, ca);
      sa_lo = fminf(sa_lo, sa);
      sa_hi = fmaxf(sa_hi, sa);
    }
    float* b = sh.lbox[w];
    if (c0 >= a.S.W || j0 >= a.S.H) {  // no ray of the image in this block
      for (int k = 0; k < 6; ++k) b[k] = 0.0f;
      return;
    }
    const float px[4] = {ce_lo * ca_lo, ce_lo * ca_hi, ce_hi * ca_lo, ce_hi * ca_hi};
    const float py[4] = {ce_lo * sa_lo, ce_lo * sa_hi, ce_hi * sa_lo, ce_hi * sa_hi};
    // relative to the tile direction dt, widened by a rounding margin
    const float m = 1e-6f;
    b[0] = fminf(fminf(px[0], px[1]), fminf(px[2], px[3])) - (float)dt[0] - m;
    b[1] = fmaxf(fmaxf(px[0], px[1]), fmaxf(px[2], px[3])) - (float)dt[0] + m;
    b[2] = fminf(fminf(py[0], py[1]), fminf(py[2], py[3])) - (float)dt[1] - m;
    b[3] = fmaxf(fmaxf(py[0], py[1]), fmaxf(py[2], py[3])) - (float)dt[1] + m;
    b[4] = se_lo - (float)dt[2] - m;
    b[5] = se_hi - (float)dt[2] + m;
  }
  // As the camera's test, with the block's direction box: d = dpix + c lies
  // in a box, h = Q d + e3 in an interval box, u = h0 / h2 and v = h1 / h2 in
  // the interval quotients (h2 > 0 on the block).
  __device__ uint32_t hit_blocks(const float4* d, int nw, const float (*box)[6]) const {
#pragma clang fp contract(off)
    const uint32_t all = (1u << nw) - 1u;
    const float4 q0 = d[0], q1 = d[1], q2 = d[2], q3 = d[3];
    if (__float_as_uint(q3.w) & kFlagGrazing) return all;
    const float ra = (q3.y - __log2f(K.alpha_min)) * (1.0f / kInv2Ln2);
    float r2 = fminf(K.cutoff2, ra);
    if (!(r2 >= 0.0f)) return 0u;
    r2 = r2 * 1.001f + 1e-3f;
    const float Q[9] = {q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
    const float cc[3] = {q0.x, q0.y, q0.z};
    const float sl = 2.0f * d[4].w;  // slack: twice the tile's FP32 error bound
    uint32_t m = 0u;
    for (int w = 0; w < nw; ++w) {
      float mid[3], rad[3], dist2 = 0.0f;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float lo = box[w][2 * k] + cc[k], hi = box[w][2 * k + 1] + cc[k];
        mid[k] = 0.5f * (lo + hi);
        rad[k] = 0.5f * (hi - lo);
        const float e = lo > 0.0f ? lo : (hi < 0.0f ? -hi : 0.0f);
        dist2 += e * e;
      }
      if (K.lowpass && K.lp * dist2 <= r2) {
        m |= 1u << w;
        continue;
      }
      float hm[3], hr[3];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        hm[i] = Q[3 * i] * mid[0] + Q[3 * i + 1] * mid[1] + Q[3 * i + 2] * mid[2];
        hr[i] = fabsf(Q[3 * i]) * rad[0] + fabsf(Q[3 * i + 1]) * rad[1] + fabsf(Q[3 * i + 2]) * rad[2];
        hr[i] = hr[i] * 1.0001f + 1e-7f;
      }
      const float h2lo = 1.0f + hm[2] - hr[2], h2hi = 1.0f + hm[2] + hr[2];
      if (!(h2lo > 1e-6f)) {
        m |= 1u << w;
        continue;
      }
      const float i_lo = __builtin_amdgcn_rcpf(h2lo), i_hi = __builtin_amdgcn_rcpf(h2hi);
      float ev[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const float a0 = hm[i] - hr[i], a1 = hm[i] + hr[i];
        const float x0 = a0 * i_lo, x1 = a0 * i_hi, x2 = a1 * i_lo, x3 = a1 * i_hi;
        const float lo = fminf(fminf(x0, x1), fminf(x2, x3)), hi = fmaxf(fmaxf(x0, x1), fmaxf(x2, x3));
        ev[i] = fmaxf((lo > 0.0f ? lo : (hi < 0.0f ? -hi : 0.0f)) - sl, 0.0f);
      }
      if (!(ev[0] * ev[0] + ev[1] * ev[1] > r2)) m |= 1u << w;
    }
    return m;
  }
  __device__ bool covered(const float4* R) const {
    return covers_wrap(__float_as_uint(R[4].y), __float_as_uint(R[4].z), pc, pb);
  }
  __device__ uint64_t cover_lanes(const float4* R) const {
    return cover_lanes_wrap(uniform_u32(R[4].y), uniform_u32(R[4].z), bx, by);
  }
  __device__ bool eval(const TileArgs& a, const float4* R, const uint32_t* sid, const F64Slot* f64, PairEval& e,
                       uint32_t& n64) const {
    return eval_lidar(R, sid, dpix, dpm, d64, a, K, f64, e, n64);
  }
  static __device__ float& flag_word(float4* R) { return R[3].w; }
  __device__ void feat(const float4* R, const PairEval& e, float* f) const {
    f[0] = e.z;
    f[1] = R[4].x;
    f[2] = 1.0f;
    f[3] = R[5].x;  // the surfel's ray-drop probability
  }
  // drop probability P = sum w rho + T (a ray that meets nothing returns
  // nothing), the drop mask P > 1/2; the median range comes from the median pass
  static __device__ void out_values(const TileArgs&, float T, const float* acc, float* v) {
#pragma clang fp contract(off)
    v[0] = acc[0];
    v[1] = acc[1];
    v[2] = acc[2];
    v[3] = acc[3] + T;
    v[4] = v[3] > 0.5f ? 1.0f : 0.0f;
    v[5] = 0.0f;
  }
  __device__ void write(const TileArgs& a, float T, const float* acc, uint32_t last) const {
    const size_t HW = (size_t)a.S.W * a.S.H, p = pix(a);
    float v[CO];
    out_values(a, T, acc, v);
#pragma unroll
    for (int c = 0; c < CO; ++c)
      if (c != kMedian) a.out[c * HW + p] = v[c];
    a.T_final[p] = T;
    a.n_last[p] = last;
  }
  // [0..8] dQ (row-major), [9..11] d mu_hat, [12] d|mu|, [13] d opacity,
  // [14] d intensity, [15] d ray drop.
  __device__ void grads(const TileArgs& a, const float4* R, const PairEval& e, float dal, float wgt, const float* g,
                        float gzx, float* gr) const {
#pragma clang fp contract(off)
    const float4 q0 = R[0], q1 = R[1], q2 = R[2];
    const float o = __builtin_amdgcn_exp2f(R[3].y);
    const float al = e.alpha;
    const float grange = fmaf(g[0], wgt, gzx);
    gr[14] = g[1] * wgt;
    gr[15] = g[3] * wgt;
    float g_rhohat = 0.0f;
    if (!e.clamped) {
      gr[13] = o > 0.0f ? dal * al * __builtin_amdgcn_rcpf(o) : 0.0f;
      g_rhohat = -0.5f * dal * al;
    }
    const float g_rho = e.lp_used ? 0.0f : g_rhohat;
    const float g_lp = e.lp_used ? g_rhohat : 0.0f;
    const float gu = 2.0f * e.u * g_rho, gv = 2.0f * e.v * g_rho;
    const float gh0 = gu * e.r, gh1 = gv * e.r;
    const float grh = e.lp_used ? 0.0f : grange;
    const float gh2 = -(gu * e.u + gv * e.v + grh * e.z) * e.r;
    gr[12] = e.lp_used ? grange : grange * e.r;
    const float dd[3] = {e.dx, e.dy, e.dz3};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      gr[c] = gh0 * dd[c];
      gr[3 + c] = gh1 * dd[c];
      gr[6 + c] = gh2 * dd[c];
    }
    const float two_lp = 2.0f * a.S.lp_ang * g_lp;
    const float Q[9] = {q0.w, q1.x, q1.y, q1.z, q1.w, q2.x, q2.y, q2.z, q2.w};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const float gd = Q[c] * gh0 + Q[3 + c] * gh1 + Q[6 + c] * gh2 + two_lp * dd[c];
      gr[9 + c] = -gd;
    }
  }
};

// ------------------------- generic compositing ---------------------------

__device__ __forceinline__ float dpp_xor1(float v) {  // quad_perm [1,0,3,2]
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0xB1, 0xF, 0xF, false));
}
__device__ __forceinline__ float dpp_xor2(float v) {  // quad_perm [2,3,0,1]
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x4E, 0xF, 0xF, false));
}
// ds_swizzle bit-mask mode inside 32-lane halves: lane -> lane ^ X
template <int X>
__device__ __forceinline__ float swz_xor(float v) {
  return __int_as_float(__builtin_amdgcn_ds_swizzle(__float_as_int(v), 0x1F | (X << 10)));
}

// Sums the 16 per-lane gradient fields over the wave and adds each total to
// the record's accumulator, as a butterfly transpose-reduction: every
// exchange step halves the fields a lane holds and doubles the lanes each of
// them is summed over (xor 1, 2 by DPP; xor 4, 8, 16 by swizzle; xor 32 by a
// permute), leaving lane l < 16 with the wave total of field
// 8 b0 + 4 b1 + 2 b2 + b3 (b_i = bit i of l), which it adds with one atomic.
// All lanes must be active.
// Wave sums of the 16 gradient fields of one pair, added to the batch's LDS
// sums of its record j (the batch's record sums go to memory once, so a
// record hit by several waves of the tile costs one global atomic per field).
template <int NT>
__device__ __forceinline__ void flush_grads(const float* g, float (*gs)[NT], uint32_t j, int lane) {
  const bool b0 = lane & 1, b1 = lane & 2, b2 = lane & 4, b3 = lane & 8;
  float x8[8], x4[4], x2[2];
#pragma unroll
  for (int i = 0; i < 8; ++i) x8[i] = (b0 ? g[i + 8] : g[i]) + dpp_xor1(b0 ? g[i] : g[i + 8]);
#pragma unroll
  for (int i = 0; i < 4; ++i) x4[i] = (b1 ? x8[i + 4] : x8[i]) + dpp_xor2(b1 ? x8[i] : x8[i + 4]);
#pragma unroll
  for (int i = 0; i < 2; ++i) x2[i] = (b2 ? x4[i + 2] : x4[i]) + swz_xor<4>(b2 ? x4[i] : x4[i + 2]);
  float x = (b3 ? x2[1] : x2[0]) + swz_xor<8>(b3 ? x2[0] : x2[1]);
  x += swz_xor<16>(x);
  x += __shfl_xor(x, 32, 64);
  const int f = (b0 ? 8 : 0) + (b1 ? 4 : 0) + (b2 ? 2 : 0) + (b3 ? 1 : 0);
  if (lane < 16 && x != 0.0f) atomicAdd(&gs[f][j], x);
}

// Per-batch gradient sums of the adjoint: [field][record of the batch].
template <int NT, bool BWD>
struct GradArea {
  float g[kGradFields][NT];
};
template <int NT>
struct GradArea<NT, false> {};

// Shared-memory state of one compositing workgroup.
template <int NT, bool BWD = false>
struct BlendShared {
  float4 rec[NT][6];
  uint32_t id[NT];
  uint64_t mask[NT / 64][NT / 64];
  F64Slot f64[kF64Slots];
  uint32_t u[8];  // [0] item, [1] flag / max last, [2] FP64 slot counter, [3] action, [4..5] walk entry,
                  // [6] next segment to walk
  // per-sensor pair counts (evaluated, composited, FP64 re-solves) of this
  // workgroup, added to the status words once at exit: per-item global
  // atomics on the same few words serialise across the whole device
  unsigned long long cnt[GS_MAX_SENSORS][4];
  float lbox[NT / 64][6];  // LiDAR: direction box of each wave's block
  // forward: each ray's median crossing (depth, pair index; kNoPair: none
  // yet), kept here rather than in registers (it is written once per ray)
  float med[NT];
  uint32_t mp[NT];
  uint32_t mbits[9];  // merge: segments holding some ray's median crossing ([8]: any from 256 on)
  GradArea<NT, BWD> ga;
};

// Writes this thread's record (pair `valid`, surfel s, raw record x) into
// batch slot threadIdx.x, staging a grazing record's FP64 re-solve data in an
// LDS slot when one is free, and stores the per-wave rectangle masks.
template <int NT, class Ray, class SH>
__device__ __forceinline__ void commit_batch(const TileArgs& a, const Ray& ray, bool valid, uint32_t s,
                                             const RawRec& x, SH& sh) {
  const int t = threadIdx.x, lane = t & 63;
  uint2 rect = make_uint2(0u, 0u);
  if (valid) {
    float4* dst = sh.rec[t];
    rect = ray.stage(x, dst, sh.lbox, NT / 64);
    sh.id[t] = s;
    float& fw = Ray::flag_word(dst);
    const uint32_t flags = __float_as_uint(fw);
    if (flags & kFlagGrazing) {
      const uint32_t slot = atomicAdd(&sh.u[2], 1u);
      if (slot < (uint32_t)kF64Slots) {
        // all loads in flight at once: one memory round trip
        const double2* G = reinterpret_cast<const double2*>(a.grz + kGrz * (size_t)s);
        double2 g[kGrz / 2];
#pragma unroll
        for (int i = 0; i < kGrz / 2; ++i) g[i] = G[i];
        double* d = sh.f64[slot];
#pragma unroll
        for (int i = 0; i < kGrz / 2; ++i) {
          d[2 * i] = g[i].x;
          d[2 * i + 1] = g[i].y;
        }
        d[kGrz] = x.d[0].x;
        d[kGrz + 1] = x.d[0].y;
        d[kGrz + 2] = x.d[1].x;
        fw = __uint_as_float(flags | ((slot + 1u) << 8));
      }
    }
  }
  const uint32_t hb = valid ? ray.hit_blocks(sh.rec[t], NT / 64, sh.lbox) : 0u;
#pragma unroll
  for (int w = 0; w < NT / 64; ++w) {
    const uint64_t m = __ballot(valid && ((hb >> w) & 1u) && ray.touches(rect, w));
    if (lane == 0) sh.mask[t >> 6][w] = m;
  }
  __syncthreads();
}

// Stages pair records [base, min(base + NT, b1)) through LDS, one per thread,
// and for every 64-record chunk c and wave w stores in mask[c][w] the bit
// mask of the chunk's records whose rectangle touches wave w's 8x8 block.
// A wave then walks only the set bits, in order.
template <int NT, class Ray, class SH>
__device__ __forceinline__ void stage_batch(const TileArgs& a, const Ray& ray, uint32_t base, uint32_t b1, SH& sh) {
  const uint32_t k = base + threadIdx.x;
  const bool valid = k < b1;
  uint32_t s = 0;
  RawRec x;
  if (valid) {
    s = a.pval[k];
    load_rec(a, s, x);
  }
  commit_batch<NT>(a, ray, valid, s, x, sh);
}

// Wave-uniform copy of a mask word from LDS.
__device__ __forceinline__ uint64_t uniform_mask(const uint64_t* p) {
  const uint64_t m = *p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)m);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(m >> 32));
  return ((uint64_t)hi << 32) | lo;
}

// Composites pairs [b0, b1) of the tile onto the running state (T, acc, last)
// of every ray not `done`; a ray whose stop rule fires becomes done.  With
// COUNT (calibration runs): n_eval counts the pixel-covered pairs up to the
// stop -- per ray with lane_counts (wave-uniform), else as a wave total held
// by every lane (counted with scalar instructions from the rectangle's lane
// mask) -- n_contrib the composited pairs per ray and n_iter the wave's pair
// iterations; without it they are left alone (the counting is a sizeable
// part of the pair loop's scalar work).  n64 always counts FP64 re-solves.
//
// With `track` (the caller's T is the ray's true transmittance: a whole tile,
// the first segment of a split one, or a walk from the merged state), the
// composited pair that takes T from at least 1/2 to below it is recorded: its
// depth in sh.med and its pair index in sh.mp (the ray's own entries).
template <int NT, bool COUNT, class Ray>
__device__ void composite(const TileArgs& a, const Ray& ray, uint32_t b0, uint32_t b1, BlendShared<NT>& sh,
                          bool lane_counts, bool& done, float& T, float* acc, uint32_t& last, uint32_t& n_eval, uint32_t& n_contrib,
                          uint32_t& n64, uint32_t& n_iter, bool track) {
#pragma clang fp contract(off)
  constexpr int C = Ray::C;
  const int t = threadIdx.x;
  const int w = t >> 6;
  // Inside the loop a stopped ray is marked by the sign bit of its
  // transmittance (never negative itself, and +0 only in strict mode), one
  // compare per pair instead of a flag turned into a lane mask.
  float Ts = done ? -T : T;
  // Software pipeline over batches: this thread's record of the next batch
  // is loaded while the current batch is composited, and the pair id of the
  // batch after it one step earlier still (the record load depends on it).
  uint32_t s_cur = 0, s_nxt = 0;
  RawRec x;
  if (b0 + t < b1) {
    s_cur = a.pval[b0 + t];
    load_rec(a, s_cur, x);
  }
  if (b0 + NT + t < b1) s_nxt = a.pval[b0 + NT + t];
  for (uint32_t base = b0; base < b1; base += NT) {
    if (t == 0) sh.u[2] = 0u;
    if (__syncthreads_count(__float_as_int(Ts) >= 0) == 0) break;
    commit_batch<NT>(a, ray, base + t < b1, s_cur, x, sh);
    bool pending = base + NT < b1;
    const int nch = (int)((min((uint32_t)NT, b1 - base) + 63) / 64);
    uint64_t live = __ballot(__float_as_int(Ts) >= 0);  // wave-uniform: rays still compositing
    for (int c = 0; c < nch && live != 0; ++c) {
      uint64_t m = uniform_mask(&sh.mask[c][w]);
      const uint32_t cb = (uint32_t)__builtin_amdgcn_readfirstlane(c) << 6;
      while (m) {
        const uint32_t j = cb + (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        // the solve's fields (the first four) into registers; the rest
        // (features, rectangle) is read where needed
        const float4* Rl = sh.rec[j];
        float4 R[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) R[i] = Rl[i];
        if constexpr (COUNT) {
          ++n_iter;
          if (lane_counts)
            n_eval += (ray.covered(Rl) && __float_as_int(Ts) >= 0) ? 1u : 0u;
          else
            n_eval += (uint32_t)__popcll(live & ray.cover_lanes(Rl));
        }
        PairEval e;
        const bool hit = ray.eval(a, R, &sh.id[j], sh.f64, e, n64) && __float_as_int(Ts) >= 0;
        const float Tn = fmaf(-e.alpha, Ts, Ts);  // T (1 - alpha), one rounding
        const bool stop = hit && Tn < ray.K.T_min;
        if (hit && !stop) {
          if constexpr (COUNT) ++n_contrib;
          const float wgt = e.alpha * Ts;
          float f[C];
          ray.feat(Rl, e, f);
#pragma unroll
          for (int c2 = 0; c2 < C; ++c2) acc[c2] = fmaf(wgt, f[c2], acc[c2]);
          if (track && Ts >= 0.5f && Tn < 0.5f) {
            sh.med[t] = e.z;
            sh.mp[t] = base + j;
          }
          Ts = Tn;
          last = base + j + 1;
        }
        if (__ballot(stop) != 0) {
          if (stop) Ts = -Ts;
          live = __ballot(__float_as_int(Ts) >= 0);
          if (live == 0) break;
        }
      }
      if (pending) {  // after the first chunk: issue the next batch's loads
        pending = false;
        s_cur = s_nxt;
        if (base + NT + t < b1) load_rec(a, s_cur, x);
        s_nxt = base + 2 * NT + t < b1 ? a.pval[base + 2 * NT + t] : 0u;
      }
    }
    if (pending) {
      s_cur = s_nxt;
      if (base + NT + t < b1) load_rec(a, s_cur, x);
      s_nxt = base + 2 * NT + t < b1 ? a.pval[base + 2 * NT + t] : 0u;
    }
  }
  done = __float_as_int(Ts) < 0;
  T = fabsf(Ts);
}

// Wave total held by every lane -> held by lane 0 only (before a wave sum).
__device__ __forceinline__ uint32_t lane0_only(uint32_t v) { return (threadIdx.x & 63) == 0 ? v : 0u; }

// Writes the outputs of the tile's rays with `wr` set, through LDS: the rays
// of a wave form an 8x8 block, so direct stores would write 32-byte pieces of
// each image row; staged, every store instruction writes whole tile rows.
// All threads call it; it reuses the record staging area (no batch is live).
// with_median: the median channel and pair index are written too (from med
// and mp of a whole tile's pass); else they are left to the segment passes.
template <int NT, class Ray>
__device__ void write_tile(const TileArgs& a, const Ray& ray, bool wr, float T, const float* acc, uint32_t last,
                           bool with_median, float med, uint32_t mp, BlendShared<NT>& sh) {
  constexpr int C = Ray::CO;
  constexpr int M = Ray::kMedian;
  static_assert((C + 4) * NT * 4 <= sizeof(sh.rec), "staging area too small");
  float* st = reinterpret_cast<float*>(&sh.rec[0][0]);
  uint32_t* su = reinterpret_cast<uint32_t*>(st);
  const int t = threadIdx.x;
  float v[C];
  Ray::out_values(a, T, acc, v);
  v[M] = mp != kNoPair ? med : 0.0f;
  __syncthreads();  // every wave is past its last read of the batch records
#pragma unroll
  for (int c = 0; c < C; ++c) st[c * NT + t] = v[c];
  st[C * NT + t] = T;
  su[(C + 1) * NT + t] = last;
  su[(C + 2) * NT + t] = wr ? 1u : 0u;
  su[(C + 3) * NT + t] = mp;
  __syncthreads();
  const int tw = a.S.tw, row = t / tw, col = t - row * tw;
  const int src = ((row >> 3) * (tw >> 3) + (col >> 3)) * 64 + (row & 7) * 8 + (col & 7);
  const int px = ray.ox + col, py = ray.oy + row;
  if (px < a.S.W && py < a.S.H && su[(C + 2) * NT + src]) {
    const size_t HW = (size_t)a.S.W * a.S.H, p = (size_t)py * a.S.W + px;
#pragma unroll
    for (int c = 0; c < C; ++c)
      if (c != M || with_median) a.out[c * HW + p] = st[c * NT + src];
    a.T_final[p] = st[C * NT + src];
    a.n_last[p] = su[(C + 1) * NT + src];
    if (with_median) a.mpair[p] = su[(C + 3) * NT + src];
  }
  __syncthreads();  // the staging area is free again
}

// Adds the wave's counts to the workgroup's counters of sensor si;
// `iters`: the wave's pair-loop iterations (wave-uniform).
template <int NT>
__device__ __forceinline__ void count_wg(BlendShared<NT>& sh, int si, uint32_t evals, uint32_t contribs,
                                         uint32_t fp64, uint32_t iters = 0u) {
  evals = wave_sum_u32(evals);
  contribs = wave_sum_u32(contribs);
  fp64 = wave_sum_u32(fp64);
  if ((threadIdx.x & 63) == 0) {
    if (evals) atomicAdd(&sh.cnt[si][0], (unsigned long long)evals);
    if (contribs) atomicAdd(&sh.cnt[si][1], (unsigned long long)contribs);
    if (fp64) atomicAdd(&sh.cnt[si][2], (unsigned long long)fp64);
    if (iters) atomicAdd(&sh.cnt[si][3], (unsigned long long)iters);
  }
}

// Can a segment with local transmittance Ts and (last | stop bit) ls be
// composited as a whole onto transmittance T?  Only with no local stop and
// either nothing composited (every pair skipped, so none can stop the ray)
// or T * Ts clear of T_min by the accumulated rounding (T_accept).
__device__ __forceinline__ bool accept_segment(float T, float Ts, uint32_t ls, float T_accept) {
  return !(ls >> 31) && (Ts == 1.0f || T * Ts >= T_accept);
}

// Front-to-back merge of a split tile's segment partials from slot sg0 with
// the ray's running state.  Every reached slot keeps the segment's incoming
// (T, prefix) for the adjoint.  Returns the first segment that cannot be
// taken whole (the ray's stop lies in it, or may), or n_seg when every
// remaining segment was taken.  With mbits (the tile's merge), a later
// segment (s >= 1) taken whole in which T falls from at least 1/2 to below
// it gets the ray's median crossing: s goes to *mark (the ray's LDS entry)
// and the segment to the LDS mask, bit s of mbits[0..8) when s < 256, else
// mbits[8] (every segment from 256 on is then listed; the replay takes only
// the rays marked for it).
template <int NT, class Ray>
__device__ uint32_t merge_from(uint32_t n_seg, uint32_t pbase, uint32_t sg0, float* part, size_t ps,
                               float T_accept, float& T, float* acc, uint32_t& last, uint32_t& n_eval,
                               uint32_t& n_contrib, uint32_t* mbits, uint32_t* mark) {
#pragma clang fp contract(off)
  constexpr int C = Ray::C;
  uint32_t* pu = reinterpret_cast<uint32_t*>(part);
  for (uint32_t sg = sg0; sg < n_seg; ++sg) {
    const size_t pe = (size_t)(pbase + sg) * NT + threadIdx.x;
    const float Ts = ld_coh(part + kPartT * ps + pe);
    const uint32_t ls = ld_coh(pu + kPartLast * ps + pe);
    const uint32_t cnt = ld_coh(pu + kPartCount * ps + pe);
    float as[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
      as[c] = ld_coh(part + c * ps + pe);
      part[c * ps + pe] = acc[c];
    }
    part[kPartT * ps + pe] = T;
    if (!accept_segment(T, Ts, ls, T_accept)) return sg;
#pragma unroll
    for (int c = 0; c < C; ++c) acc[c] = fmaf(T, as[c], acc[c]);
    const float Tn = T * Ts;
    if (mbits && sg > 0 && T >= 0.5f && Tn < 0.5f) {
      atomicOr(&mbits[min(sg >> 5, 8u)], sg < 256u ? 1u << (sg & 31u) : 1u);
      *mark = sg;
    }
    T = Tn;
    if (ls) last = ls;
    n_eval += cnt & 0xFFFFu;
    n_contrib += cnt >> 16;
  }
  return n_seg;
}

// Merge run by the workgroup that completes a split tile; queues the
// segments that hold some ray's stop for the cooperative walk.
//
// Walk-list protocol: the merged state is published (device-scope release)
// before any walk entry of the tile is listed; an entry is listed by
// reserving an index (hdr[3]) and then storing the packed (tile, segment)
// over the cleared sentinel; the tile then leaves the pending-merge count
// (hdr[5], release).  Consumers pop indices below hdr[3] and wait for the
// entry to appear.
template <int NT, class Ray>
__device__ void merge_tile(const QueueArgs& q, const TileArgs& a, const Ray& ray, uint32_t gt, uint2 rg,
                           uint32_t n_seg, uint32_t pbase, int si, BlendShared<NT>& sh) {
#pragma clang fp contract(off)
  constexpr int C = Ray::C;
  uint32_t n_eval = 0, n_contrib = 0, n64 = 0, marked = 0;
  float T = 1.0f;
  float acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0f;
  uint32_t last = rg.x;
  bool wr = false;
  if (threadIdx.x < 9) sh.mbits[threadIdx.x] = 0u;
  sh.mp[threadIdx.x] = kNoPair;  // this ray's crossing segment, if a later one
  __syncthreads();
  if (ray.inside) {
    const uint32_t sg = merge_from<NT, Ray>(n_seg, pbase, 0, q.part, q.part_stride, q.T_accept, T, acc, last, n_eval,
                                            n_contrib, sh.mbits, &sh.mp[threadIdx.x]);
    const uint32_t ms = sh.mp[threadIdx.x];
    if (ms != kNoPair) a.mpair[ray.pix(a)] = kCross | ms;
    if (sg == n_seg) {
      wr = true;
    } else {
      // the stop lies in segment sg (or may): keep the incoming state there
      // (stored by the merge), mark the slot and list a walk of it
      const size_t pe = (size_t)(pbase + sg) * NT + threadIdx.x;
      uint32_t* pu = reinterpret_cast<uint32_t*>(q.part);
      pu[kPartLast * q.part_stride + pe] = kWalk;
      pu[kPartCount * q.part_stride + pe] = last;
      marked = sg + 1;
    }
  }
  write_tile<NT>(a, ray, wr, T, acc, last, false, 0.0f, kNoPair, sh);
  count_wg(sh, si, n_eval, n_contrib, n64);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  auto list = [&](uint32_t seg) {
    const uint32_t w = atomicAdd(q.hdr + 3, 1u);
    if (w < q.walk_cap)
      __hip_atomic_store(q.walk + w, ((unsigned long long)gt << 32) | seg, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
  };
  if (marked) {
    const uint32_t slot = pbase + marked - 1;
    if (atomicCAS(q.slot_flag + slot, 0u, 1u) == 0u) list(marked - 1);
  }
  // median entries: one per segment holding some ray's crossing
  const uint32_t n_list = sh.mbits[8] ? n_seg : min(n_seg, 256u);
  for (uint32_t k = threadIdx.x; k < n_list; k += NT)
    if (k < 256u ? (sh.mbits[k >> 5] >> (k & 31u)) & 1u : 1u) list(k | kMedianEntry);
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(q.hdr + 5, 0xFFFFFFFFu, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// Adjoint over pairs [b0, b1); the incoming state is (1, 0) for a whole tile
// or the merge's (T_in, prefix) for a segment.
template <int NT, class Ray>
__device__ void bwd_range(const TileArgs& a, const Ray& ray, uint32_t b0, uint32_t b1, const float* part, size_t ps,
                          size_t pe, BlendShared<NT, true>& sh) {
#pragma clang fp contract(off)
  uint32_t& s_max = sh.u[1];
  constexpr int C = Ray::C;
  const int t = threadIdx.x, lane = t & 63;
  const size_t HW = (size_t)a.S.W * a.S.H;
  const size_t p = ray.inside ? ray.pix(a) : 0;
  float g[C], O[C], A[C];
  float T = 1.0f;
#pragma unroll
  for (int c = 0; c < C; ++c) {
    g[c] = ray.inside ? a.gout[c * HW + p] : 0.0f;
    O[c] = ray.inside ? a.out_fwd[c * HW + p] : 0.0f;
    A[c] = 0.0f;
  }
  if (part && ray.inside) {
#pragma unroll
    for (int c = 0; c < C; ++c) A[c] = part[c * ps + pe];
    T = part[kPartT * ps + pe];
  }
  // the median depth's gradient goes to the depth of its crossing pair
  const float gmed = ray.inside ? a.gout[Ray::kMedian * HW + p] : 0.0f;
  const uint32_t mp = ray.inside ? a.mpair[p] : kNoPair;
  const uint32_t last = ray.inside ? a.n_last[p] : b0;
  __syncthreads();
  if (t == 0) s_max = b0;
  __syncthreads();
  atomicMax(&s_max, last);
  __syncthreads();
  const uint32_t end = min(s_max, b1);
  uint32_t wlast = last;
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) wlast = max(wlast, (uint32_t)__shfl_xor((int)wlast, o, 64));
  wlast = rfl(wlast);
  uint32_t n64 = 0;
  const int w = t >> 6;
  for (uint32_t base = b0; base < end; base += NT) {
    if (t == 0) sh.u[2] = 0u;
#pragma unroll
    for (int f = 0; f < kGradFields; ++f) sh.ga.g[f][t] = 0.0f;
    __syncthreads();
    stage_batch<NT>(a, ray, base, end, sh);
    const int nch = (int)((min((uint32_t)NT, end - base) + 63) / 64);
    bool past = false;  // wave-uniform: every later pair is past the wave's last contribution
    for (int c = 0; c < nch && !past; ++c) {
      uint64_t m = uniform_mask(&sh.mask[c][w]);
      const uint32_t cb = (uint32_t)__builtin_amdgcn_readfirstlane(c) << 6;
      while (m) {
      const uint32_t j = cb + (uint32_t)__builtin_ctzll(m);
      m &= m - 1;
      if (base + j >= wlast) {
        past = true;
        break;
      }
      const bool active = base + j < last;
      PairEval e;
      const bool hit = ray.eval(a, sh.rec[j], &sh.id[j], sh.f64, e, n64) && active;
      float gr[kGradFields];
#pragma unroll
      for (int f = 0; f < kGradFields; ++f) gr[f] = 0.0f;
      if (hit) {
        const float al = e.alpha;
        const float wgt = al * T;
        float f[C];
        ray.feat(sh.rec[j], e, f);
        const float inv1m = __builtin_amdgcn_rcpf(1.0f - al);
        float dal = 0.0f;
#pragma unroll
        for (int c = 0; c < C; ++c) {
          A[c] = fmaf(wgt, f[c], A[c]);
          const float S = O[c] - A[c];
          dal += g[c] * (T * f[c] - S * inv1m);
        }
        ray.grads(a, sh.rec[j], e, dal, wgt, g, base + j == mp ? gmed : 0.0f, gr);
        T = fmaf(-al, T, T);  // as the forward pass
      }
      if (__ballot(hit) != 0) flush_grads<NT>(gr, sh.ga.g, j, lane);
      }
    }
    __syncthreads();
    // the batch's gradient sums, thread t for record t
    if (base + t < end) {
      const uint32_t sid = sh.id[t];
#pragma unroll
      for (int f = 0; f < kGradFields; ++f) {
        const float v = sh.ga.g[f][t];
        if (v != 0.0f) atomicAdd(a.gacc + (size_t)f * a.gacc_stride + sid, v);
      }
    }
  }
}

__device__ inline int sensor_of_tile(const QueueArgs& q, uint32_t gt) {
  int s = 0;
  while (s + 1 < q.n_sensors && q.tile_off[s + 1] <= (int)gt) ++s;
  return s;
}

// Adjoint of one work item (a whole tile, or one segment of a split tile
// from the incoming state its slot holds).
template <int NT, class Ray>
__device__ void bwd_item(const QueueArgs& q, const TileArgs& a, int tile, uint32_t gt, uint32_t sg, uint2 rg,
                         BlendShared<NT, true>& sh) {
  const Ray ray(a, tile);
  ray.prepare(a, sh);
  const uint32_t len = rg.y - rg.x;
  const uint32_t L = q.seg_len;
  const uint32_t n_seg = len > L ? (len - 1) / L + 1 : 1u;
  if (n_seg == 1) {
    bwd_range<NT>(a, ray, rg.x, rg.y, nullptr, 0, 0, sh);
    return;
  }
  const uint32_t pbase = q.pslot_base[gt];
  if (pbase + n_seg > q.pslot_cap) return;  // unreachable: slots are sized for the pair capacity
  const uint32_t b0 = rg.x + sg * L;
  const size_t pe = (size_t)(pbase + sg) * NT + threadIdx.x;
  bwd_range<NT>(a, ray, b0, min(b0 + L, rg.y), q.part, q.part_stride, pe, sh);
}

// One forward work item, through a single compositing call site:
//  - a whole tile (from T = 1; writes the outputs);
//  - a segment of a split tile (from T = 1; writes the segment's partial
//    state to its slot, and the tile's last arrival merges);
//  - (walk) a listed stop segment, for the rays the merge marked there, from
//    the incoming state it left in the slot.  A marked ray whose stop does
//    not come in that segment (T * T_seg fell between T_min and T_accept)
//    carries on: later segments are taken whole from their partials where
//    the accept test allows, and the first one that it does not is walked by
//    the workgroup again, for every ray that waits at it.
template <int NT, bool COUNT, class Ray>
__device__ void fwd_item(const QueueArgs& q, const TileArgs& a, int si, int tile, uint32_t gt, uint32_t sg,
                         uint2 rg, bool walk, BlendShared<NT>& sh) {
#pragma clang fp contract(off)
  constexpr int C = Ray::C;
  constexpr uint32_t kNone = 0xFFFFFFFFu;
  const Ray ray(a, tile);
  ray.prepare(a, sh);
  const uint32_t len = rg.y - rg.x;
  const uint32_t L = q.seg_len;
  const uint32_t n_seg = len > L ? (len - 1) / L + 1 : 1u;
  const bool split = n_seg > 1;
  const uint32_t pbase = split ? q.pslot_base[gt] : 0u;
  if (split && pbase + n_seg > q.pslot_cap) return;  // unreachable: slots are sized for the pair capacity
  const bool partial = split && !walk;
  float* part = q.part;
  const size_t ps = q.part_stride;
  uint32_t* pu = reinterpret_cast<uint32_t*>(part);
  const size_t pe = (size_t)(pbase + sg) * NT + threadIdx.x;
  float T = 1.0f;
  float acc[C];
#pragma unroll
  for (int c = 0; c < C; ++c) acc[c] = 0.0f;
  uint32_t last = partial ? 0u : rg.x, n_eval_w = 0, n_eval = 0, n_contrib = 0, n64 = 0, n_iter = 0;
  // the ray composites segment `need` next (kNone: nothing left for it here)
  uint32_t need = ray.inside ? sg : kNone;
  if (walk) {
    if (need != kNone && ld_coh(pu + kPartLast * ps + pe) == kWalk) {
      T = ld_coh(part + kPartT * ps + pe);
#pragma unroll
      for (int c = 0; c < C; ++c) acc[c] = ld_coh(part + c * ps + pe);
      last = ld_coh(pu + kPartCount * ps + pe);
      // complete these loads here: left in flight, they would make the pair
      // loop wait for every outstanding load (the next batch's prefetch
      // included) wherever it updates the running state
      asm volatile("" ::"v"(T), "v"(last));
#pragma unroll
      for (int c = 0; c < C; ++c) asm volatile("" ::"v"(acc[c]));
    } else {
      need = kNone;
    }
  }
  bool done = false;
  // the median crossing is found here where the incoming transmittance is
  // the ray's true one: a whole tile, the first segment of a split tile (1),
  // a walk (the merged state); a crossing in a later segment taken whole by a
  // merge is left to the median pass
  const bool track = walk || sg == 0;
  sh.mp[threadIdx.x] = kNoPair;  // this thread's own entry: no barrier needed
  for (uint32_t cur = sg;;) {
    const bool active = need == cur;
    done = !active;
    const uint32_t b0 = rg.x + cur * L;
    // a segment keeps per-ray counts: the merge takes them ray by ray
    composite<NT, COUNT>(a, ray, b0, split ? min(b0 + L, rg.y) : rg.y, sh, partial, done, T, acc, last,
                  partial ? n_eval : n_eval_w, n_contrib, n64, n_iter, track);
    if (!walk) break;
    if (active) {
      // a walked ray's transmittance is near T_min: no later segment can hold
      // its median crossing (nothing to mark)
      need = done ? kNone
                  : merge_from<NT, Ray>(n_seg, pbase, cur + 1, part, ps, q.T_accept, T, acc, last, n_eval, n_contrib,
                                        nullptr, nullptr);
      if (need == n_seg) need = kNone;
      if (need == kNone) ray.write(a, T, acc, last);
    }
    __syncthreads();
    if (threadIdx.x == 0) sh.u[6] = kNone;
    __syncthreads();
    if (need != kNone) atomicMin(&sh.u[6], need);
    __syncthreads();
    const uint32_t nxt = sh.u[6];
    if (nxt == kNone) break;
    cur = nxt;
  }
  const uint32_t mp = sh.mp[threadIdx.x];
  if (walk) {
    if (ray.inside && mp != kNoPair) {  // a crossing inside a walked segment
      const size_t HW = (size_t)a.S.W * a.S.H, p = ray.pix(a);
      a.out[Ray::kMedian * HW + p] = sh.med[threadIdx.x];
      a.mpair[p] = mp;
    }
    count_wg(sh, si, lane0_only(n_eval_w) + n_eval, n_contrib, n64, n_iter);
    return;
  }
  if (!partial) {
    count_wg(sh, si, lane0_only(n_eval_w), n_contrib, n64, n_iter);
    write_tile<NT>(a, ray, ray.inside, T, acc, last, true, sh.med[threadIdx.x], mp, sh);
    return;
  }
  count_wg(sh, si, 0u, 0u, n64, n_iter);
  if (ray.inside && sg == 0) {
    const size_t HW = (size_t)a.S.W * a.S.H, p = ray.pix(a);
    a.out[Ray::kMedian * HW + p] = mp != kNoPair ? sh.med[threadIdx.x] : 0.0f;
    a.mpair[p] = mp;
  }
  if (ray.inside) {
#pragma unroll
    for (int c = 0; c < C; ++c) part[c * ps + pe] = acc[c];
    part[kPartT * ps + pe] = T;
    pu[kPartLast * ps + pe] = last | (done ? 0x80000000u : 0u);
    pu[kPartCount * ps + pe] = n_eval | (n_contrib << 16);
  }
  // publish this segment (device-scope release: written back from this XCD's
  // L2), then let the tile's last arrival merge
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
  __syncthreads();
  if (threadIdx.x == 0) sh.u[1] = (atomicAdd(q.arrive + gt, 1u) + 1u == n_seg) ? 1u : 0u;
  __syncthreads();
  if (sh.u[1]) merge_tile<NT>(q, a, ray, gt, rg, n_seg, pbase, si, sh);  // partials are read device-coherently
}

// Median depth (2DGS: the depth where the accumulated opacity reaches 1/2)
// of the rays whose transmittance falls below 1/2 inside a later segment
// (s >= 1) of a split tile, which the merge took whole (whole tiles, first
// segments and walks composite from the ray's true transmittance and record
// the crossing themselves).  The merge marked those rays (mpair = kCross | s)
// and listed the segment; the rays replay its pairs from the incoming
// transmittance the merge left in the slot and take the depth of the pair
// after which it falls below 1/2.  Should the replay's rounding not cross
// inside the segment, its last composited pair stands for it.  The crossing
// comes before any stop (T_min < 1/2), so the replay needs no stop rule.
// Runs as a walk-list entry: slot state and marks are read device-coherently.
template <int NT, class Ray>
__device__ void median_item(const QueueArgs& q, const TileArgs& a, int tile, uint32_t gt, uint32_t sg, uint2 rg,
                            BlendShared<NT>& sh) {
#pragma clang fp contract(off)
  const uint32_t len = rg.y - rg.x, L = q.seg_len;
  const uint32_t n_seg = len > L ? (len - 1) / L + 1 : 1u;
  if (n_seg == 1 || sg == 0 || sg >= n_seg) return;  // unreachable: merges list later segments only
  const uint32_t pbase = q.pslot_base[gt];
  if (pbase + n_seg > q.pslot_cap) return;  // unreachable: slots are sized for the pair capacity
  const Ray ray(a, tile);
  ray.prepare(a, sh);
  const uint32_t b0 = rg.x + sg * L;
  const uint32_t b1 = min(b0 + L, rg.y);
  const int t = threadIdx.x;
  const size_t HW = (size_t)a.S.W * a.S.H, p = ray.inside ? ray.pix(a) : 0;
  const bool mine = ray.inside && ld_coh(a.mpair + p) == (kCross | sg);
  float T = mine ? ld_coh(q.part + kPartT * q.part_stride + (size_t)(pbase + sg) * NT + t) : 1.0f;
  bool active = mine;
  float med = 0.0f, zl = 0.0f;
  uint32_t mp = kNoPair, pl = kNoPair, n64 = 0;
  const int w = t >> 6;
  for (uint32_t base = b0; base < b1; base += NT) {
    if (t == 0) sh.u[2] = 0u;
    if (__syncthreads_count(active) == 0) break;
    stage_batch<NT>(a, ray, base, b1, sh);
    const int nch = (int)((min((uint32_t)NT, b1 - base) + 63) / 64);
    for (int c = 0; c < nch; ++c) {
      uint64_t m = uniform_mask(&sh.mask[c][w]);
      const uint32_t cb = (uint32_t)__builtin_amdgcn_readfirstlane(c) << 6;
      while (m && __ballot(active) != 0) {
        const uint32_t j = cb + (uint32_t)__builtin_ctzll(m);
        m &= m - 1;
        PairEval e;
        const bool hit = ray.eval(a, sh.rec[j], &sh.id[j], sh.f64, e, n64) && active;
        if (hit) {
          const float Tn = fmaf(-e.alpha, T, T);  // as the compositing pass
          zl = e.z;
          pl = base + j;
          if (Tn < 0.5f) {
            med = e.z;
            mp = base + j;
            active = false;
          }
          T = Tn;
        }
      }
    }
  }
  if (mine) {
    a.out[Ray::kMedian * HW + p] = mp != kNoPair ? med : zl;
    a.mpair[p] = mp != kNoPair ? mp : pl;
  }
}

// Sensor kinds a launch may meet (bit 0 camera, bit 1 LiDAR): single-kind
// launches leave the other kind's code and registers out.
constexpr int kKindCam = 1, kKindLidar = 2, kKindBoth = 3, kKindCyl = 4;

__device__ __forceinline__ uint32_t load_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Bound on every wait of the walk queue (polls of ~128 cycles): far above
// any drain time, so a stall can only come from a broken invariant; it is
// then reported (hdr[6]) instead of hanging.
constexpr uint32_t kSpinLimit = 1u << 21;
constexpr uint64_t kNoWalk = ~0ull;

enum { kActExit = 0, kActItem = 1, kActWalk = 2 };

// Waits (bounded) for walk entry `idx` to be stored after its reservation.
__device__ bool take_walk(const QueueArgs& q, uint32_t idx, uint32_t* u) {
  for (uint32_t w = 0; w < kSpinLimit; ++w) {
    const uint64_t e = __hip_atomic_load(q.walk + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (e != kNoWalk) {
      u[4] = (uint32_t)(e >> 32);
      u[5] = (uint32_t)e;
      return true;
    }
    __builtin_amdgcn_s_sleep(2);
  }
  return false;
}

// Thread 0 picks the workgroup's next action.  Listed walks come first (each
// completes a split tile): one compare-and-swap attempt on the walk counter,
// which on failure simply falls through.  Then a main-queue item (heaviest
// first, one atomic per item).  With the main queue drained, the workgroup
// takes a walk ticket (one atomic) and waits until that index is listed, or
// leaves once no split tile is left to merge and the ticket lies past the
// list (forward pass only; the adjoint has no walks).
__device__ uint32_t next_action(const QueueArgs& q, bool& main_left, uint32_t& drained, uint32_t xcc,
                                uint32_t n_items, bool walks, uint32_t* u) {
  if (walks) {
    const uint32_t cnt = min(load_agent(q.hdr + 3), q.walk_cap);
    const uint32_t pop = load_agent(q.hdr + 4);
    if (pop < cnt && atomicCAS(q.hdr + 4, pop, pop + 1) == pop) {
      if (take_walk(q, pop, u)) return kActWalk;
      atomicOr(q.hdr + 6, 1u);
      return kActExit;
    }
  }
  if (main_left) {
    // this XCD's sub-queue first, then the others (drained: bit per sub-queue)
    for (uint32_t r = 0; r < (uint32_t)kQueues; ++r) {
      const uint32_t x = (xcc + r) % kQueues;
      if ((drained >> x) & 1u) continue;
      const uint32_t k = atomicAdd(q.counter + kQCntStride * x, 1u);
      const uint32_t it = k * kQueues + x;
      if (k < n_items && it < n_items) {
        u[0] = it;
        return kActItem;
      }
      drained |= 1u << x;
    }
    main_left = false;
  }
  if (!walks) return kActExit;
  const uint32_t ticket = atomicAdd(q.hdr + 4, 1u);
  for (uint32_t spin = 0; spin < kSpinLimit; ++spin) {
    if (ticket < min(load_agent(q.hdr + 3), q.walk_cap)) {
      if (take_walk(q, ticket, u)) return kActWalk;
      break;
    }
    // no split tile left to merge (confirmed with an acquire, so every walk
    // its merge listed is counted) and the ticket is past the list: done
    if (load_agent(q.hdr + 5) == 0 &&
        __hip_atomic_load(q.hdr + 5, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == 0 &&
        ticket >= min(load_agent(q.hdr + 3), q.walk_cap))
      return kActExit;
    __builtin_amdgcn_s_sleep(8);
  }
  atomicOr(q.hdr + 6, 1u);
  return kActExit;
}

// Persistent compositing over (tile, segment) items and, in the forward pass,
// the walk entries the merges list.
template <int NT, bool BWD, int KINDS, bool COUNT>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(BWD || COUNT || (KINDS & kKindCyl) ? 1 : 4))) void k_blend_queue(QueueArgs q) {
  __shared__ BlendShared<NT, BWD> sh;
  uint32_t* s_u = sh.u;
  const uint32_t n_items = min(*q.n_items, q.cap_items);
  bool main_left = true;  // thread 0 only
  uint32_t drained = 0, xcc = 0;
  asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
  for (int i = threadIdx.x; i < GS_MAX_SENSORS * 4; i += NT) (&sh.cnt[0][0])[i] = 0ull;
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0)
      s_u[3] = next_action(q, main_left, drained, xcc & 7u, n_items, !BWD && q.pslot_cap > 0, s_u);
    __syncthreads();
    // the action and its item are workgroup-uniform: scalar registers
    const uint32_t act = rfl(s_u[3]);
    if (act == kActExit) break;
    uint32_t gt, sg;
    uint2 rg;
    if (act == kActItem) {
      const uint4 e = q.items[q.queue[rfl(s_u[0])]];
      gt = rfl(e.x);
      sg = rfl(e.y);
      rg = make_uint2(rfl(e.z), rfl(e.w));
    } else {
      gt = rfl(s_u[4]);  // its slot state is read device-coherently
      sg = rfl(s_u[5]);
    }
    const int si = sensor_of_tile(q, gt);
    const TileArgs& a = q.tiles[si];
    const int tile = (int)gt - q.tile_off[si];
    if (act != kActItem) rg = a.ranges[gt];
    // the sensor's kind, decided statically where the launch serves one kind
    const bool cam = (KINDS & kKindCam) && (KINDS == kKindCam || a.S.kind == GS_SENSOR_PINHOLE);
    const bool cyl = (KINDS & kKindCyl) && (KINDS == kKindCyl || a.S.kind == GS_SENSOR_CYLINDRICAL);
    if constexpr (BWD) {
      if (cam)
        bwd_item<NT, CamRay>(q, a, tile, gt, sg, rg, sh);
      else if (cyl)
        bwd_item<NT, CylRay>(q, a, tile, gt, sg, rg, sh);
      else if (KINDS & kKindLidar)
        bwd_item<NT, LidarRay>(q, a, tile, gt, sg, rg, sh);
    } else {
      const bool walk = act == kActWalk;
      if (walk && (sg & kMedianEntry)) {
        if (cam)
          median_item<NT, CamRay>(q, a, tile, gt, sg & ~kMedianEntry, rg, sh);
        else if (cyl)
          median_item<NT, CylRay>(q, a, tile, gt, sg & ~kMedianEntry, rg, sh);
        else if (KINDS & kKindLidar)
          median_item<NT, LidarRay>(q, a, tile, gt, sg & ~kMedianEntry, rg, sh);
      } else if (cam)
        fwd_item<NT, COUNT, CamRay>(q, a, si, tile, gt, sg, rg, walk, sh);
      else if (cyl)
        fwd_item<NT, COUNT, CylRay>(q, a, si, tile, gt, sg, rg, walk, sh);
      else if (KINDS & kKindLidar)
        fwd_item<NT, COUNT, LidarRay>(q, a, si, tile, gt, sg, rg, walk, sh);
    }
  }
  // the workgroup's counts, once per sensor and counter
  __syncthreads();
  const int i = threadIdx.x;
  if (!BWD && i < q.n_sensors * 4) {
    const unsigned long long v = (&sh.cnt[0][0])[i];
    uint32_t xcc;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_XCC_ID)" : "=s"(xcc));
    uint32_t* st = q.tiles[i / 4].status + kStRep + 8 * (xcc & 7u);
    if (v) {
      if (i % 4 == 0) atomicAdd(reinterpret_cast<unsigned long long*>(st), v);
      else if (i % 4 == 1) atomicAdd(reinterpret_cast<unsigned long long*>(st + 2), v);
      else if (i % 4 == 2) atomicAdd(st + 4, (uint32_t)v);
      else atomicAdd(reinterpret_cast<unsigned long long*>(st + 6), v);
    }
  }
}

}  // namespace

// Launch variants: every tile size for pinhole / LiDAR mixes; kinds with the
// cylindrical camera (bit 2) at 256-ray tiles only (plans enforce it).
#define GS_VARIANTS(X) \
  X(64, 1) X(64, 2) X(64, 3) X(128, 1) X(128, 2) X(128, 3) X(256, 1) X(256, 2) X(256, 3) X(512, 1) X(512, 2) \
  X(512, 3) X(256, 4) X(256, 5) X(256, 6) X(256, 7)

void launch_blend_queue(const QueueArgs& q, int rays, int kinds, int grid, bool backward, bool count,
                        hipStream_t st) {
#define KCASE(NT, K)                                                                              \
  if (rays == NT && kinds == K) {                                                                 \
    if (backward)                                                                                 \
      hipLaunchKernelGGL((k_blend_queue<NT, true, K, false>), dim3(grid), dim3(NT), 0, st, q);    \
    else if (count)                                                                               \
      hipLaunchKernelGGL((k_blend_queue<NT, false, K, true>), dim3(grid), dim3(NT), 0, st, q);    \
    else                                                                                          \
      hipLaunchKernelGGL((k_blend_queue<NT, false, K, false>), dim3(grid), dim3(NT), 0, st, q);   \
    return;                                                                                       \
  }
  GS_VARIANTS(KCASE)
#undef KCASE
}

int blend_blocks_per_cu(int rays, int kinds, bool backward) {
  int n = 0;
  hipError_t e = hipErrorInvalidValue;
#define KCASE(NT, K)                                                                                         \
  if (rays == NT && kinds == K)                                                                              \
    e = backward ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_blend_queue<NT, true, K, false>, NT, 0) \
                 : hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k_blend_queue<NT, false, K, false>, NT, 0);
  GS_VARIANTS(KCASE)
#undef KCASE
  return e == hipSuccess ? n : 0;
}

bool tile_shape_supported(int tw, int th) {
  if (tw % 8 != 0 || th % 8 != 0 || tw <= 0 || th <= 0) return false;
  const int rays = tw * th;
  return rays == 64 || rays == 128 || rays == 256 || rays == 512;
}

}  // namespace gs
