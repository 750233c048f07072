// Kernel launch interface shared by the library's translation units.
#pragma once

#include "gs_internal.h"

namespace gs {

struct PrepArgs {
  int n;
  const float* mean;
  const float* quat;
  const float* scale;
  const float* opacity;
  const float* rgb;
  const float* sh;
  const float* intensity;
  const float* drop;      // LiDAR ray-drop probability [N] (nullptr: 0)
  int sh_degree;
  GroupsK groups;
  SensorK S;
  OptsK O;
  SensorWS ws;            // per-surfel arrays already offset to this sensor's records
  uint32_t rec_base;      // record id of surfel 0 (pair values are rec_base + i)
  size_t gacc_stride;     // plane stride of ws.gacc
};

// Per-sensor data the pair emission needs (record ranges and tile grids).
struct EmitTable {
  int n;
  uint32_t rec_base[GS_MAX_SENSORS + 1];
  int n_tx[GS_MAX_SENSORS];
  int tile_off[GS_MAX_SENSORS];
};

// One sensor's view of the blend state (per-sensor or batched layout).
struct TileArgs {
  SensorK S;              // S.tile_offset indexes `ranges`
  OptsK O;
  const float4* rec;      // records, indexed by the pair value
  const double* rec64;
  const double* grz;
  const uint2* ranges;    // [global tiles]
  const uint32_t* pval;   // sorted pair record ids
  float* out;             // forward outputs [C][H][W]
  const float* out_fwd;   // backward: forward outputs
  const float* gout;      // backward: dL/d outputs
  float* T_final;         // [H*W]
  uint32_t* n_last;       // [H*W]
  uint32_t* mpair;        // [H*W] pair index of the median crossing (kNoPair: none)
  uint32_t* status;       // counters
  float* gacc;            // [kGradFields][gacc_stride]
  size_t gacc_stride;
};

// The sorted work items are dealt round-robin to 8 sub-queues (one per XCD,
// item i to sub-queue i mod 8) with one counter each, 64 bytes apart: one
// counter popped by every workgroup of the device serialises the pops.
constexpr int kQueues = 8;
constexpr int kQCntStride = 16;

// Persistent compositing queue over (tile, segment) work items of one record
// space (one sensor, or every sensor of a batched step).
//
// The TileArgs table travels by value in the kernel arguments: pointers read
// from there are known to be global, so every access compiles to global_*
// instructions (pointers read from a table in device memory would be generic
// and compile to flat ones, which also wait on LDS traffic).
struct QueueArgs {
  TileArgs tiles[GS_MAX_SENSORS];
  int n_sensors;
  int tile_off[GS_MAX_SENSORS + 1];
  const uint32_t* queue;     // item ids, heaviest first
  const uint4* items;        // item id -> (record-space tile id, segment, tile range)
  const uint32_t* n_items;   // device count (hdr[0])
  uint32_t* hdr;             // [0] items [1] slots [2] queue counter [3] walks listed [4] walks taken
                             // [5] split tiles left to merge [6] queue stalled
  uint32_t cap_items;
  uint32_t* counter;         // 8 sub-queue counters, kQCntStride words apart; zeroed before each launch
  uint32_t* arrive;          // per tile: segments finished (forward)
  const uint32_t* pslot_base;  // per tile: first partial-state slot
  float* part;               // [11][pslot_cap * rays per tile]
  uint32_t* slot_flag;       // per slot: listed for the cooperative walk
  unsigned long long* walk;  // walk list: tile << 32 | segment (| 1 << 31: a median entry); cleared to
                             // ~0 per forward; walk_cap entries (a slot is listed at most once as a
                             // stop walk and once as a median entry)
  uint32_t walk_cap;
  size_t part_stride;        // elements per plane
  uint32_t pslot_cap;
  uint32_t seg_len;          // segment length L (pairs)
  float T_accept;            // T_min scaled by the product-rounding margin
};

struct SplatBwdArgs {
  PrepArgs p;             // scene + sensor (ws.gacc holds the per-record gradients)
  float* g_mean;
  float* g_quat;
  float* g_scale;
  float* g_opacity;
  float* g_rgb;
  float* g_sh;
  float* g_intensity;
  float* g_drop;
};

// preprocess.hip
void launch_compose_poses(const float* sensor_pose, const float* group_poses, int pose_base, int n_groups, float* out,
                          hipStream_t st);
// Batched step: for every sensor k, status[k][0..16) = 0 and its n_groups[k]
// (<= 64) composed poses (sensor_pose[k] o group pose pose_base[k] + g) to
// pose_out[k], in one launch.
struct SensorSetup {
  int n;
  const float* sensor_pose[GS_MAX_SENSORS];
  int pose_base[GS_MAX_SENSORS];
  int n_groups[GS_MAX_SENSORS];
  float* pose_out[GS_MAX_SENSORS];
  uint32_t* status[GS_MAX_SENSORS];
};
void launch_sensor_setup(const float* group_poses, const SensorSetup& s, hipStream_t st);
void launch_prep(const PrepArgs& a, hipStream_t st);

// sort.hip
void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st);
void launch_fill_f32(float* p, float v, size_t n, hipStream_t st);
// Stable LSD radix sort of (key, value) pairs over bits [0, bits); the count
// is *count (device) when count != nullptr, else count_const; at most cap
// items.  Ping-pongs between buffers 0 and 1; returns the buffer holding the
// result.
int radix_sort(uint32_t* key[2], uint32_t* val[2], const uint32_t* count, uint32_t count_const, uint32_t cap,
               int bits, uint32_t* hist, uint32_t* err, hipStream_t st);
size_t radix_hist_words(uint32_t cap);
// The (tile, surfel) pairs of the sorted records, in one pass: record j's
// pairs start at the exclusive scan of ntiles[val[j]] (total ->
// status[kStPairs], overflow flag when above cap) and are written in depth
// order, each surfel's tiles row by row.  With count (device): only the first
// min(n, *count) sorted records (the visible ones).
void launch_offsets_emit(const uint32_t* val, const uint32_t* ntiles, const int4* rect, int n, const uint32_t* count,
                         const EmitTable& E, uint32_t* bsum, uint32_t* status, uint32_t cap, uint32_t* ptile,
                         uint32_t* pval, hipStream_t st);
size_t scan_bsum_words(int n);
// Work items of a record space: per tile n_seg = ceil(len / L) (1 when
// len <= L); item_base / pslot_base by exclusive scans; items written with
// keys (cost, heaviest first) and ids for the radix sort; arrival counters and
// the queue counter cleared.  hdr[0] = items, hdr[1] = partial slots,
// hdr[2] unused (the sub-queue counters are cleared here too).
struct SegScanArgs {
  const uint2* ranges;
  int n_tiles;
  uint32_t seg_len;
  int key_bits;
  uint2* bsum;
  uint32_t* hdr;
  uint32_t* pslot_base;
  uint32_t* arrive;
  uint32_t* slot_flag;
  unsigned long long* walk;
  uint32_t* key;
  uint32_t* val;
  uint4* items;
  uint32_t cap_items, pslot_cap;
  uint32_t* status;
  uint32_t* qcnt;  // the 8 sub-queue counters (kQCntStride words apart)
};
void launch_build_items(const SegScanArgs& a, hipStream_t st);
size_t seg_bsum_words(int n_tiles);
void launch_ranges(const uint32_t* ptile, const uint32_t* count, uint32_t cap, uint2* ranges, int n_tiles,
                   hipStream_t st);
// The records whose key is not kInvalidKey, in record order, to kout / vout
// (n records in; scratch: ceil(n / 4096) words); their number to *count.
void launch_compact_visible(const uint32_t* kin, const uint32_t* vin, int n, uint32_t* scratch, uint32_t* kout,
                            uint32_t* vout, uint32_t* count, hipStream_t st);
// Sensor k of a batched record space owns record ids [rec_base[k],
// rec_base[k + 1]); its visible count goes to status[k][kStVisible].
struct VisibleSplit {
  int n;
  uint32_t rec_base[GS_MAX_SENSORS + 1];
  uint32_t* status[GS_MAX_SENSORS];
};
// ids: the *count compacted record ids (ascending), before the depth sort
void launch_visible_split(const uint32_t* ids, const uint32_t* count, const VisibleSplit& s, hipStream_t st);

// blend.hip
// kinds: bit 0 camera, bit 1 LiDAR (the sensor kinds the launch serves)
// count: the forward also counts evaluated / composited pairs and pair-loop
// iterations into the status words (calibration runs).
void launch_blend_queue(const QueueArgs& q, int rays, int kinds, int grid, bool backward, bool count,
                        hipStream_t st);
int blend_blocks_per_cu(int rays, int kinds, bool backward);
bool tile_shape_supported(int tw, int th);

// splat_backward.hip
void launch_splat_backward(const SplatBwdArgs& a, hipStream_t st);

}  // namespace gs
