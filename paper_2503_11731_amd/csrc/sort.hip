// a3-a5: tile-count scan, (tile, surfel) pair emission, stable LSD radix sort
// and per-tile ranges.
//
// The depth order within a tile is obtained without sorting 64-bit
// (tile, depth) keys over all pairs: all pairs of one surfel share its depth
// key, so the low 32 key bits are sorted once over the N surfels (stable, so
// ties keep the surfel index order), pairs are then emitted in that order,
// and a stable sort on the tile id alone (ceil(log2 tiles) bits) yields
// exactly the order of a stable sort of (tile << 32 | depth) keys.
//
// Radix passes use 8-bit digits over blocks of kRadixItems keys.  One histogram kernel
// counts every digit of every pass over all keys (totals do not depend on the
// key order); each pass is then one scatter launch whose blocks take
// sequential tickets, rank their keys with wavefront ballots (match mask of
// equal digits), publish their digit counts and obtain the counts of all
// earlier blocks by a decoupled look-back over per-block status words, then
// write their keys through LDS in contiguous runs per digit.  A block only
// waits on blocks holding smaller tickets, which are already running, and
// every wait is bounded (a give-up raises a status flag instead of hanging).
#include <cstring>

#include "gs_internal.h"
#include "kernels.h"

namespace gs {

namespace {

__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  const int lane = __lane_id();
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint32_t t = __shfl_up(v, o, 64);
    if (lane >= o) v += t;
  }
  return v;
}

// Exclusive scan over NT threads; *total receives the block sum.
template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t v, uint32_t* s_w, uint32_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint32_t inc = wave_incl_scan(v);
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < NT / 64; ++k) {
    uint32_t x = s_w[k];
    off += (k < w) ? x : 0u;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// 64-bit exclusive scan over 256 threads; *total receives the block sum.
__device__ inline uint64_t block_excl_scan64(uint64_t v, uint64_t* s_w, uint64_t* total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  uint64_t inc = v;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint64_t y = __shfl_up(inc, o, 64);
    if (lane >= o) inc += y;
  }
  if (lane == 63) s_w[w] = inc;
  __syncthreads();
  uint64_t off = 0, tot = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    const uint64_t x = s_w[k];
    off += (k < w) ? x : 0ull;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

__device__ inline uint32_t sat32(uint64_t x) { return x > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)x; }

struct RadixArgs {
  const uint32_t* kin;
  const uint32_t* vin;
  uint32_t* kout;
  uint32_t* vout;
  const uint32_t* count;
  uint32_t count_const;
  uint32_t cap;
  int shift;            // first bit of this pass's digit
  int passes;           // histogram kernel: digits counted per key
  uint32_t* gcount;     // [pass][256] digit totals over all keys
  uint32_t* ticket;     // this pass's block ticket counter
  uint32_t* look;       // [block][256] status words of this pass
  uint32_t* look_next;  // the same for the next pass, cleared here
  uint32_t* err;        // set to 1 when a look-back wait gives up
};

__device__ inline uint32_t radix_n(const RadixArgs& a) {
  uint32_t n = a.count ? *a.count : a.count_const;
  return n < a.cap ? n : a.cap;
}

// status word: bits 31/30 = inclusive prefix / block aggregate available, the
// low 30 bits the count (keys per sort < 2^30)
constexpr uint32_t kLookInc = 1u << 31;
constexpr uint32_t kLookAgg = 1u << 30;
constexpr uint32_t kLookVal = kLookAgg - 1u;
constexpr uint32_t kLookSpins = 1u << 20;
constexpr int kLookWin = 16;  // earlier blocks read per look-back round trip

__device__ inline uint32_t ld_agent(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_agent(uint32_t* p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Digit totals of every pass, one read of the keys.  Few, wide blocks: the
// per-block totals meet in one global add per (pass, digit), and those adds
// to the same word serialise, so their number is kept to the grid size.
__global__ __launch_bounds__(1024) void k_rs_ghist(RadixArgs a) {
  const uint32_t n = radix_n(a);
  __shared__ uint32_t h[4][256];
  const int t = threadIdx.x;
  (&h[0][0])[t] = 0;
  __syncthreads();
  for (uint32_t i = blockIdx.x * 1024 + t; i < n; i += gridDim.x * 1024) {
    const uint32_t k = a.kin[i];
    for (int p = 0; p < a.passes; ++p) atomicAdd(&h[p][(k >> (a.shift + 8 * p)) & 255u], 1u);
  }
  __syncthreads();
  const int p = t >> 8;
  const uint32_t c = (&h[0][0])[t];
  if (p < a.passes && c != 0u) atomicAdd(&a.gcount[t], c);
}

// One pass: stable scatter of kRadixItems-key blocks in ticket order.  Each wave
// ranks its own contiguous quarter of the block (match masks from 8 ballots
// per 64 keys, per-wave digit counters in LDS that only that wave touches);
// the block then publishes its digit counts, looks back for the counts of all
// earlier blocks, groups its keys by digit in LDS and writes them out in order.
__global__ __launch_bounds__(256) void k_rs_onesweep(RadixArgs a) {
  const uint32_t n = radix_n(a);
  const uint32_t nb = (n + kRadixItems - 1) / kRadixItems;
  __shared__ uint32_t s_key[kRadixItems];
  __shared__ uint32_t s_val[kRadixItems];
  __shared__ uint32_t s_wcnt[4][256];
  __shared__ uint32_t s_start[256];
  __shared__ uint32_t s_gbase[256];
  __shared__ uint32_t s_gstart[256];
  __shared__ uint32_t s_w[4];
  __shared__ uint32_t s_ticket;
  const int t = threadIdx.x, w = t >> 6, lane = t & 63;
  const uint64_t lt = lanemask_lt();
  constexpr int R = kRadixItems / 256;  // keys per lane
  {
    uint32_t tot;
    s_gstart[t] = block_excl_scan<256>(a.gcount[t], s_w, &tot);
  }
  for (;;) {
    if (t == 0) s_ticket = atomicAdd(a.ticket, 1u);
#pragma unroll
    for (int k = 0; k < 4; ++k) s_wcnt[k][t] = 0;
    __syncthreads();
    const uint32_t b = s_ticket;
    if (b >= nb) break;
    if (a.look_next) a.look_next[(size_t)b * 256 + t] = 0u;
    const uint32_t wbase = b * kRadixItems + (uint32_t)w * (kRadixItems / 4);
    uint32_t my_key[R], my_val[R], my_rank[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t idx = wbase + r * 64 + lane;
      my_key[r] = idx < n ? a.kin[idx] : 0u;
      my_val[r] = idx < n ? a.vin[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const uint32_t idx = wbase + r * 64 + lane;
      const bool valid = idx < n;
      const uint32_t d = (my_key[r] >> a.shift) & 255u;
      uint64_t m = __ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const bool on = (d >> bit) & 1u;
        const uint64_t bb = __ballot(on);
        m &= on ? bb : ~bb;
      }
      const uint32_t below = (uint32_t)__popcll(m & lt);
      // every lane of the digit reads the count before its first lane adds
      // the digit's keys of this round (one wave, LDS in program order)
      const uint32_t pre = valid ? s_wcnt[w][d] : 0u;
      my_rank[r] = valid ? pre + below : 0xFFFFFFFFu;
      if (valid && below == 0) s_wcnt[w][d] = pre + (uint32_t)__popcll(m);
    }
    __syncthreads();
    const uint32_t c0 = s_wcnt[0][t], c1 = s_wcnt[1][t], c2 = s_wcnt[2][t], c3 = s_wcnt[3][t];
    const uint32_t cd = c0 + c1 + c2 + c3;
    // digit t: publish this block's count, then add the counts of all
    // earlier blocks (an inclusive prefix ends the walk)
    uint32_t* mine = a.look + (size_t)b * 256 + t;
    st_agent(mine, (b == 0 ? kLookInc : kLookAgg) | cd);
    uint32_t excl = 0;
    if (b > 0) {
      // walk back kLookWin blocks per round trip, nearest first; a block that
      // has published nothing yet stops the round and is read again
      uint32_t spins = 0;
      for (uint32_t k = b; k > 0;) {
        uint32_t v[kLookWin];
#pragma unroll
        for (int j = 0; j < kLookWin; ++j) v[j] = (uint32_t)j < k ? ld_agent(a.look + (size_t)(k - 1 - j) * 256 + t) : kLookInc;
        bool ended = false, inclusive = false;
        uint32_t used = 0;
#pragma unroll
        for (int j = 0; j < kLookWin; ++j) {
          if (ended || (v[j] & (kLookInc | kLookAgg)) == 0u) {
            ended = true;
          } else {
            excl += v[j] & kLookVal;
            ++used;
            inclusive = (v[j] & kLookInc) != 0u;
            ended = inclusive;
          }
        }
        k -= used < k ? used : k;
        if (inclusive) break;
        if (used == 0) {
          if (++spins > kLookSpins) {
            if (a.err) atomicOr(a.err, 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      st_agent(mine, kLookInc | (excl + cd));
    }
    uint32_t tot;
    const uint32_t st = block_excl_scan<256>(cd, s_w, &tot);
    s_start[t] = st;
    s_wcnt[0][t] = st;
    s_wcnt[1][t] = st + c0;
    s_wcnt[2][t] = st + c0 + c1;
    s_wcnt[3][t] = st + c0 + c1 + c2;
    s_gbase[t] = s_gstart[t] + excl;
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (my_rank[r] != 0xFFFFFFFFu) {
        const uint32_t d = (my_key[r] >> a.shift) & 255u;
        const uint32_t pos = s_wcnt[w][d] + my_rank[r];
        s_key[pos] = my_key[r];
        s_val[pos] = my_val[r];
      }
    }
    __syncthreads();
    const uint32_t cnt = min((uint32_t)kRadixItems, n - b * kRadixItems);
    for (uint32_t i = t; i < cnt; i += 256) {
      const uint32_t k = s_key[i];
      const uint32_t d = (k >> a.shift) & 255u;
      const uint32_t g = s_gbase[d] + (i - s_start[d]);
      a.kout[g] = k;
      a.vout[g] = s_val[i];
    }
    __syncthreads();
  }
}

// ---------------- pair offsets and emission, one pass ----------------
//
// The first pair of sorted record j is the sum of ntiles[val[i]] over i < j:
// 4096-item blocks in ticket order, each publishing its sum and reading the sums of earlier
// blocks by a bounded look-back (64 blocks per round trip, one per lane of
// the first wave), with 64-bit status words (high half: 1 = block sum, 2 = inclusive prefix; low half the
// value).  The ticket and status words are cleared with the frame's status.
// Sums are formed in 64 bits and saturate at 2^32 - 1, so a frame whose
// pairs exceed any capacity is always reported as an overflow (a wrapped
// 32-bit total could pass for a small one).

constexpr int kScanItems = 4096;
constexpr uint64_t kScanAgg = 1ull << 32;
constexpr uint64_t kScanInc = 2ull << 32;

// Pair emission of one wave's 64 consecutive surfels of the depth order (lane
// l: surfel s with cnt pairs from pair o): the wave writes the union of their
// pairs as consecutive 64-pair runs, each lane finding its surfel with a
// binary search over the wave's first pairs, so every store instruction
// writes 256 contiguous bytes.  Within a surfel the tiles go row by row (the
// order the tile sort keeps for equal tile ids).  Pairs from cap on are not
// written (the frame then reports an overflow).
__device__ __forceinline__ void emit_wave(uint32_t s, uint32_t cnt, uint64_t o, const int4* __restrict__ rect,
                                          const EmitTable& E, uint32_t cap, uint32_t* __restrict__ ptile,
                                          uint32_t* __restrict__ pval) {
  const int lane = threadIdx.x & 63;
  const uint64_t start64 = __shfl(o, 0, 64);
  if (start64 >= cap) return;  // wave-uniform
  uint64_t end64 = o + cnt;     // lanes past the list hold cnt 0
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    const uint64_t y = __shfl_xor(end64, d, 64);
    end64 = y > end64 ? y : end64;
  }
  const uint32_t start = (uint32_t)start64;
  const uint32_t end = (uint32_t)(end64 < cap ? end64 : cap);
  // local first pair (a surfel's tile count is far below 2^26, so 64 of them fit)
  const uint32_t lo = (uint32_t)(o - start64);
  int4 r = make_int4(0, 0, 0, 0);
  int n_tx = 1, toff = 0;
  if (cnt) {
    r = rect[s];
    int se = 0;
    while (se + 1 < E.n && E.rec_base[se + 1] <= s) ++se;
    n_tx = E.n_tx[se];
    toff = E.tile_off[se];
  }
  const bool wrap = (r.w >> 30) & 1;
  const int ncol = cnt == 0 ? 1 : (wrap ? (n_tx - r.x) + (r.y + 1) : (r.y - r.x + 1));
  const int row0 = toff + r.z * n_tx;  // tile id of column 0 in the first row
  for (uint32_t b = 0; start + b < end; b += 64) {
    const uint32_t k = b + (uint32_t)lane;
    // highest lane whose first pair is <= k (that lane has a pair at k: a
    // lane without pairs shares its first pair with the next lane)
    int src = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
      const uint32_t l = (uint32_t)__shfl((int)lo, src + step, 64);
      if (src + step < 64 && l <= k) src += step;
    }
    const uint32_t ls = (uint32_t)__shfl((int)lo, src, 64);
    const uint32_t ss = (uint32_t)__shfl((int)s, src, 64);
    const int nc = __shfl(ncol, src, 64);
    const int x0 = __shfl(r.x, src, 64);
    const int ntx = __shfl(n_tx, src, 64);
    const int rb = __shfl(row0, src, 64);
    const uint32_t q = start + k;
    if (q < end) {
      const uint32_t loc = k - ls;
      const uint32_t ty = loc / (uint32_t)nc;
      int tx = x0 + (int)(loc - ty * (uint32_t)nc);
      if (tx >= ntx) tx -= ntx;
      ptile[q] = (uint32_t)(rb + (int)ty * ntx + tx);
      pval[q] = ss;
    }
  }
}

__global__ __launch_bounds__(256) void k_offsets_emit(const uint32_t* __restrict__ val,
                                                      const uint32_t* __restrict__ ntiles,
                                                      const int4* __restrict__ rect, int n_max, const uint32_t* count,
                                                      uint32_t* bsum, uint32_t* status, EmitTable E, uint32_t cap,
                                                      uint32_t* __restrict__ ptile, uint32_t* __restrict__ pval) {
  __shared__ uint64_t s_w64[4];
  __shared__ uint32_t s_ticket;
  __shared__ uint64_t s_excl;
  const int t = threadIdx.x;
  // the first *count sorted records (the visible ones) when a count is given
  const int n = count ? (int)min((uint32_t)n_max, *count) : n_max;
  const int nblk = (n + kScanItems - 1) / kScanItems;
  if (n == 0) return;
  uint32_t* ticket = bsum;
  uint64_t* look = reinterpret_cast<uint64_t*>(bsum + 2);
  if (t == 0) s_ticket = atomicAdd(ticket, 1u);
  __syncthreads();
  const int b = (int)s_ticket;
  if (b >= nblk) return;
  // wave w takes the w-th quarter of the block in rounds of 64 consecutive
  // items (one per lane): index loads and offset stores are contiguous runs,
  // and each round's offsets come from a wave scan
  constexpr int PER = kScanItems / 256;
  const int w = t >> 6, lane = t & 63;
  const int base = b * kScanItems + w * (kScanItems / 4) + lane;
  uint32_t v[PER], idx[PER];
#pragma unroll
  for (int r = 0; r < PER; ++r) idx[r] = base + r * 64 < n ? val[base + r * 64] : 0u;
#pragma unroll
  for (int r = 0; r < PER; ++r) v[r] = base + r * 64 < n ? ntiles[idx[r]] : 0u;
  uint64_t sum = 0;
#pragma unroll
  for (int r = 0; r < PER; ++r) sum += v[r];
  uint64_t tot;
  // lane 0's exclusive prefix is the sum over the earlier waves' quarters
  const uint64_t wave_off = __shfl(block_excl_scan64(sum, s_w64, &tot), 0, 64);
  const uint32_t tot32 = sat32(tot);
  if (t < 64) {
    // wave 0: publish this block's sum, then read 64 earlier blocks per
    // round trip (lane i: block k - 1 - i), nearest first, up to the nearest
    // inclusive prefix; a block with nothing published yet ends the round
    uint64_t* mine = look + b;
    if (lane == 0)
      __hip_atomic_store(mine, (b == 0 ? kScanInc : kScanAgg) | tot32, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    if (b > 0) {
      uint32_t spins = 0;
      for (int k = b; k > 0;) {
        const int idx = k - 1 - lane;
        const uint64_t v = idx >= 0 ? __hip_atomic_load(look + idx, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : kScanInc;
        const uint64_t inc = __ballot((v & kScanInc) != 0u);
        const uint64_t none = __ballot((v >> 32) == 0u);
        const int fi = inc ? __builtin_ctzll(inc) : 64;    // nearest inclusive prefix
        const int fn = none ? __builtin_ctzll(none) : 64;  // nearest block not yet published
        const int used = fn <= fi ? fn : fi + 1;           // lanes [0, used) are added
        uint64_t x = lane < used ? (uint64_t)(uint32_t)v : 0ull;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) x += __shfl_xor(x, o, 64);
        excl += x;
        k -= used;
        if (fi < fn) break;  // reached an inclusive prefix
        if (used == 0) {
          if (++spins > kLookSpins) {
            if (lane == 0) atomicOr(&status[kStSortStall], 1u);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        }
      }
      if (lane == 0)
        __hip_atomic_store(mine, kScanInc | sat32(excl + tot), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      s_excl = excl;
      if (b == nblk - 1) {
        const uint32_t total = sat32(excl + tot);
        status[kStPairs] = total;
        if (total > cap) status[kStOverflow] = 1u;
      }
    }
  }
  __syncthreads();
  uint64_t off = s_excl + wave_off;
#pragma unroll
  for (int r = 0; r < PER; ++r) {
    if (base - lane + r * 64 < n) {  // wave-uniform: the round holds part of the list
      uint64_t inc = v[r];
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const uint64_t y = __shfl_up(inc, o, 64);
        if (lane >= o) inc += y;
      }
      emit_wave(idx[r], v[r], off + inc - v[r], rect, E, cap, ptile, pval);
      off += __shfl(inc, 63, 64);
    }
  }
}

// ---------------- compositing work items ----------------

// (items, partial slots) of one tile: a list longer than L splits into
// ceil(len / L) segments, each with its own partial-state slot.
// tiles per block of the work-item scans (one per thread)
constexpr int kSegItems = 256;

__device__ inline uint2 seg_counts(uint2 rg, uint32_t L) {
  const uint32_t len = rg.y - rg.x;
  const uint32_t n = len > L ? (len - 1) / L + 1 : 1u;
  return make_uint2(n, n > 1 ? n : 0u);
}

__global__ __launch_bounds__(256) void k_seg_reduce(SegScanArgs a) {
  __shared__ uint32_t s_w[4];
  const int t = blockIdx.x * kSegItems + threadIdx.x;
  uint32_t sx = 0, sy = 0;
  if (t < a.n_tiles) {
    const uint2 c = seg_counts(a.ranges[t], a.seg_len);
    sx = c.x;
    sy = c.y;
  }
  uint32_t tx, ty;
  block_excl_scan<256>(sx, s_w, &tx);
  block_excl_scan<256>(sy, s_w, &ty);
  if (threadIdx.x == 0) a.bsum[blockIdx.x] = make_uint2(tx, ty);
}

__global__ __launch_bounds__(1024) void k_seg_top(SegScanArgs a, int nblk) {
  __shared__ uint32_t s_w[16];
  const int per = (nblk + 1023) / 1024;
  const int beg = threadIdx.x * per;
  const int end = min(beg + per, nblk);
  uint32_t sx = 0, sy = 0;
  for (int i = beg; i < end; ++i) {
    sx += a.bsum[i].x;
    sy += a.bsum[i].y;
  }
  uint32_t tx, ty;
  uint32_t ox = block_excl_scan<1024>(sx, s_w, &tx);
  uint32_t oy = block_excl_scan<1024>(sy, s_w, &ty);
  for (int i = beg; i < end; ++i) {
    const uint2 b = a.bsum[i];
    a.bsum[i] = make_uint2(ox, oy);
    ox += b.x;
    oy += b.y;
  }
  if (threadIdx.x == 0) {
    a.hdr[0] = tx;
    a.hdr[1] = ty;
    a.hdr[2] = 0u;
    a.hdr[3] = 0u;
    a.hdr[4] = 0u;
    a.hdr[5] = 0u;
    a.hdr[6] = 0u;
    if (tx > a.cap_items || ty > a.pslot_cap) a.status[kStOverflow] = 1u;
  }
  if (threadIdx.x < kQueues) a.qcnt[kQCntStride * threadIdx.x] = 0u;
}

__global__ __launch_bounds__(256) void k_seg_down(SegScanArgs a) {
  __shared__ uint32_t s_w[4];
  const int t = blockIdx.x * kSegItems + threadIdx.x;
  const uint2 rg = t < a.n_tiles ? a.ranges[t] : make_uint2(0u, 0u);
  const uint2 c = t < a.n_tiles ? seg_counts(rg, a.seg_len) : make_uint2(0u, 0u);
  uint32_t tx, ty, tsplit;
  const uint32_t ix = block_excl_scan<256>(c.x, s_w, &tx) + a.bsum[blockIdx.x].x;
  const uint32_t iy = block_excl_scan<256>(c.y, s_w, &ty) + a.bsum[blockIdx.x].y;
  const bool split = t < a.n_tiles && c.y && iy + c.y <= a.pslot_cap;
  (void)block_excl_scan<256>(split ? 1u : 0u, s_w, &tsplit);
  // the block's split tiles join the count of tiles left to merge at once
  if (threadIdx.x == 0 && tsplit) atomicAdd(a.hdr + 5, tsplit);
  if (t >= a.n_tiles) return;
  const uint32_t kmax = a.key_bits >= 32 ? 0xFFFFFFFFu : ((1u << a.key_bits) - 1u);
  a.pslot_base[t] = iy;
  a.arrive[t] = 0u;
  if (split) {
    // a split tile: clear its slots' walk flags and twice as many walk-list
    // entries (a slot can be listed as a stop walk and as a median entry)
    for (uint32_t k = 0; k < c.y; ++k) {
      a.slot_flag[iy + k] = 0u;
      a.walk[2 * (iy + k)] = ~0ull;
      a.walk[2 * (iy + k) + 1] = ~0ull;
    }
  }
  const uint32_t len = rg.y - rg.x;
  for (uint32_t sg = 0; sg < c.x; ++sg) {
    const uint32_t item = ix + sg;
    if (item >= a.cap_items) break;
    // every segment of a split tile (its short last one included) weighs
    // two full segments: the tile's merge waits for all of them, and the
    // stop-segment walks follow the merge on the critical path
    const uint32_t cost = c.x == 1 ? len : 2u * a.seg_len;
    a.key[item] = kmax - (cost < kmax ? cost : kmax);
    a.val[item] = item;
    a.items[item] = make_uint4((uint32_t)t, sg, rg.x, rg.y);
  }
}

__global__ __launch_bounds__(256) void k_ranges(const uint32_t* __restrict__ ptile, const uint32_t* __restrict__ count,
                                                uint32_t cap, uint2* __restrict__ ranges, uint32_t n_tiles) {
  uint32_t n = *count;
  n = n < cap ? n : cap;
  for (uint32_t i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) {
    const uint32_t t = ptile[i];
    if (t >= n_tiles) continue;  // only a pair slot no emission wrote can hold such an id
    if (i == 0 || ptile[i - 1] != t) ranges[t].x = i;
    if (i + 1 == n || ptile[i + 1] != t) ranges[t].y = i + 1;
  }
}

__global__ void k_fill_u32(uint32_t* p, uint32_t v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}
__global__ void k_fill_f32(float* p, float v, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) p[i] = v;
}

// ---------------- compaction of the visible records ----------------
// Order-preserving: the records whose key is not kInvalidKey (the visible
// ones), in record order, so that the stable depth sort that follows ranks
// equal keys exactly as a sort of every record would.  Blocks of 4096
// records: per-block counts, one scan of those counts, then each block writes
// its records at its offset.  Inside a block wave w takes the w-th quarter in
// 16 rounds of 64 consecutive records (one per lane), so every load reads and
// every store writes one contiguous run; a round's visible records are ranked
// by a ballot.
constexpr int kCompactItems = 4096;
constexpr int kCompactRounds = kCompactItems / 256;

__global__ __launch_bounds__(256) void k_compact_count(const uint32_t* __restrict__ key, int n,
                                                       uint32_t* __restrict__ bcnt) {
  __shared__ uint32_t s_c[4];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t base = (uint32_t)blockIdx.x * kCompactItems + (uint32_t)w * (kCompactItems / 4) + (uint32_t)lane;
  uint32_t k[kCompactRounds];
#pragma unroll
  for (int r = 0; r < kCompactRounds; ++r) k[r] = base + r * 64 < (uint32_t)n ? key[base + r * 64] : kInvalidKey;
  uint32_t c = 0;
#pragma unroll
  for (int r = 0; r < kCompactRounds; ++r) c += (uint32_t)__popcll(__ballot(k[r] != kInvalidKey));
  if (lane == 0) s_c[w] = c;
  __syncthreads();
  if (threadIdx.x == 0) bcnt[blockIdx.x] = s_c[0] + s_c[1] + s_c[2] + s_c[3];
}

// exclusive scan of nblk block counts in place, one workgroup; *count = the total
__global__ __launch_bounds__(1024) void k_compact_scan(uint32_t* __restrict__ bcnt, int nblk,
                                                       uint32_t* __restrict__ count) {
  __shared__ uint32_t s_w[16];
  const int per = (nblk + 1023) / 1024;
  const int beg = threadIdx.x * per, end = min(beg + per, nblk);
  uint32_t s = 0;
  for (int i = beg; i < end; ++i) s += bcnt[i];
  uint32_t tot;
  uint32_t off = block_excl_scan<1024>(s, s_w, &tot);
  for (int i = beg; i < end; ++i) {
    const uint32_t c = bcnt[i];
    bcnt[i] = off;
    off += c;
  }
  if (threadIdx.x == 0) *count = tot;
}

// First index j < n with v[j] >= x in the ascending v[0, n) (n if none), by
// the whole workgroup: each round samples 256 evenly spaced positions of the
// open range and keeps the gap between the last sample below x and the next,
// so a range of m shrinks below m / 256 per round (4 rounds for 2^32).
__device__ uint32_t block_lower_bound(const uint32_t* __restrict__ v, uint32_t n, uint32_t x) {
  uint32_t lo = 0, hi = n;
  while (lo < hi) {
    const uint32_t step = (hi - lo + 255) / 256;
    const uint32_t m = (hi - lo + step - 1) / step;  // samples lo + t * step, t < m
    const uint32_t q = lo + threadIdx.x * step;
    const uint32_t c = (uint32_t)__syncthreads_count(threadIdx.x < m && v[q] < x);
    const uint32_t nlo = c ? lo + (c - 1) * step + 1 : lo;
    hi = c < m ? lo + c * step : hi;
    lo = nlo;
  }
  return lo;
}

// Per-sensor visible counts of a batched record space: the compacted record
// ids ascend and sensor k owns ids [rec_base[k], rec_base[k + 1]), so its
// count is the difference of two lower bounds.  One workgroup per sensor.
__global__ __launch_bounds__(256) void k_visible_split(const uint32_t* __restrict__ ids,
                                                       const uint32_t* __restrict__ count, VisibleSplit s) {
  const int k = blockIdx.x;
  const uint32_t n = *count;
  const uint32_t a = k == 0 ? 0u : block_lower_bound(ids, n, s.rec_base[k]);
  const uint32_t b = k + 1 == s.n ? n : block_lower_bound(ids, n, s.rec_base[k + 1]);
  if (threadIdx.x == 0) s.status[k][kStVisible] = b - a;
}

__global__ __launch_bounds__(256) void k_compact_scatter(const uint32_t* __restrict__ kin,
                                                         const uint32_t* __restrict__ vin, int n,
                                                         const uint32_t* __restrict__ boff,
                                                         uint32_t* __restrict__ kout, uint32_t* __restrict__ vout) {
  __shared__ uint32_t s_c[4];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint32_t base = (uint32_t)blockIdx.x * kCompactItems + (uint32_t)w * (kCompactItems / 4) + (uint32_t)lane;
  const uint64_t lt = lanemask_lt();
  uint32_t k[kCompactRounds], v[kCompactRounds];
  uint64_t m[kCompactRounds];
#pragma unroll
  for (int r = 0; r < kCompactRounds; ++r) {
    const uint32_t i = base + r * 64;
    k[r] = i < (uint32_t)n ? kin[i] : kInvalidKey;
    v[r] = i < (uint32_t)n ? vin[i] : 0u;
  }
  uint32_t c = 0;
#pragma unroll
  for (int r = 0; r < kCompactRounds; ++r) {
    m[r] = __ballot(k[r] != kInvalidKey);
    c += (uint32_t)__popcll(m[r]);
  }
  if (lane == 0) s_c[w] = c;
  __syncthreads();
  uint32_t o = boff[blockIdx.x];
  for (int q = 0; q < w; ++q) o += s_c[q];
#pragma unroll
  for (int r = 0; r < kCompactRounds; ++r) {
    if (k[r] != kInvalidKey) {
      const uint32_t pos = o + (uint32_t)__popcll(m[r] & lt);
      kout[pos] = k[r];
      vout[pos] = v[r];
    }
    o += (uint32_t)__popcll(m[r]);
  }
}

inline unsigned grid_for(size_t n, unsigned block, unsigned cap_blocks) {
  size_t g = (n + block - 1) / block;
  if (g < 1) g = 1;
  return (unsigned)(g < cap_blocks ? g : cap_blocks);
}

}  // namespace

void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, v, n);
}
void launch_fill_f32(float* p, float v, size_t n, hipStream_t st) {
  if (n == 0) return;
  hipLaunchKernelGGL(k_fill_f32, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, p, v, n);
}

static size_t radix_nb(uint32_t cap) { return (cap + kRadixItems - 1) / kRadixItems; }

// [4][256] digit totals | 16 tickets | two look-back areas of [blocks][256]
size_t radix_hist_words(uint32_t cap) { return 4 * 256 + 16 + 2 * 256 * radix_nb(cap); }

int radix_sort(uint32_t* key[2], uint32_t* val[2], const uint32_t* count, uint32_t count_const, uint32_t cap,
               int bits, uint32_t* hist, uint32_t* err, hipStream_t st) {
  const int passes = (bits + 7) / 8;
  if (passes <= 0) return 0;
  const size_t nb_max = radix_nb(cap);
  uint32_t* gcount = hist;
  uint32_t* ticket = hist + 4 * 256;
  uint32_t* area[2] = {ticket + 16, ticket + 16 + 256 * nb_max};
  launch_fill_u32(hist, 0u, 4 * 256 + 16 + 256 * nb_max, st);
  RadixArgs a;
  memset(&a, 0, sizeof(a));
  a.count = count;
  a.count_const = count_const;
  a.cap = cap;
  a.err = err;
  a.kin = key[0];
  a.passes = passes;
  a.gcount = gcount;
  hipLaunchKernelGGL(k_rs_ghist, dim3(grid_for(cap, 1024 * 8, 256)), dim3(1024), 0, st, a);
  const unsigned grid = nb_max < 1 ? 1u : (nb_max < 1024 ? (unsigned)nb_max : 1024u);
  int cur = 0;
  for (int p = 0; p < passes; ++p) {
    a.kin = key[cur];
    a.vin = val[cur];
    a.kout = key[cur ^ 1];
    a.vout = val[cur ^ 1];
    a.shift = 8 * p;
    a.gcount = gcount + 256 * p;
    a.ticket = ticket + p;
    a.look = area[p & 1];
    a.look_next = p + 1 < passes ? area[(p + 1) & 1] : nullptr;
    hipLaunchKernelGGL(k_rs_onesweep, dim3(grid), dim3(256), 0, st, a);
    cur ^= 1;
  }
  return cur;
}

// ticket (two words, keeping the status words 8-byte aligned) + one 64-bit
// look-back status word per 4096-item block
size_t scan_bsum_words(int n) { return 2 + 2 * (size_t)((n + kScanItems - 1) / kScanItems); }

void launch_offsets_emit(const uint32_t* val, const uint32_t* ntiles, const int4* rect, int n, const uint32_t* count,
                         const EmitTable& E, uint32_t* bsum, uint32_t* status, uint32_t cap, uint32_t* ptile,
                         uint32_t* pval, hipStream_t st) {
  const int nblk = (n + kScanItems - 1) / kScanItems;
  hipLaunchKernelGGL(k_offsets_emit, dim3(nblk > 0 ? nblk : 1), dim3(256), 0, st, val, ntiles, rect, n, count, bsum,
                     status, E, cap, ptile, pval);
}

size_t seg_bsum_words(int n_tiles) { return 2 * ((size_t)((n_tiles + kSegItems - 1) / kSegItems) + 1); }

void launch_build_items(const SegScanArgs& a, hipStream_t st) {
  const int nblk = (a.n_tiles + kSegItems - 1) / kSegItems;
  if (nblk > 0) hipLaunchKernelGGL(k_seg_reduce, dim3(nblk), dim3(256), 0, st, a);
  hipLaunchKernelGGL(k_seg_top, dim3(1), dim3(1024), 0, st, a, nblk);
  if (nblk > 0) hipLaunchKernelGGL(k_seg_down, dim3(nblk), dim3(256), 0, st, a);
}


void launch_ranges(const uint32_t* ptile, const uint32_t* count, uint32_t cap, uint2* ranges, int n_tiles,
                   hipStream_t st) {
  launch_fill_u32(reinterpret_cast<uint32_t*>(ranges), 0u, 2ull * n_tiles, st);
  hipLaunchKernelGGL(k_ranges, dim3(grid_for(cap, 256, 2048)), dim3(256), 0, st, ptile, count, cap, ranges,
                     (uint32_t)n_tiles);
}

void launch_compact_visible(const uint32_t* kin, const uint32_t* vin, int n, uint32_t* scratch, uint32_t* kout,
                            uint32_t* vout, uint32_t* count, hipStream_t st) {
  if (n == 0) return;  // the caller's zeroed count stands
  const int nblk = (n + kCompactItems - 1) / kCompactItems;
  hipLaunchKernelGGL(k_compact_count, dim3(nblk), dim3(256), 0, st, kin, n, scratch);
  hipLaunchKernelGGL(k_compact_scan, dim3(1), dim3(1024), 0, st, scratch, nblk, count);
  hipLaunchKernelGGL(k_compact_scatter, dim3(nblk), dim3(256), 0, st, kin, vin, n, scratch, kout, vout);
}

void launch_visible_split(const uint32_t* ids, const uint32_t* count, const VisibleSplit& s, hipStream_t st) {
  if (s.n <= 0) return;
  hipLaunchKernelGGL(k_visible_split, dim3(s.n), dim3(256), 0, st, ids, count, s);
}

}  // namespace gs
