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
  uint32_t* status;       // counters
  float* gacc;            // [kGradFields][gacc_stride]
  size_t gacc_stride;
};

struct BatchArgs {
  const TileArgs* tiles;  // device table [n_sensors]
  int n_sensors;
  int tile_off[GS_MAX_SENSORS + 1];
  const uint32_t* queue;  // global tile ids, heaviest first
  int n_items;
  uint32_t* counter;      // zeroed before the launch
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
};

// preprocess.hip
void launch_compose_poses(const float* sensor_pose, const float* group_poses, int pose_base, int n_groups, float* out,
                          hipStream_t st);
void launch_prep(const PrepArgs& a, hipStream_t st);

// sort.hip
void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t st);
void launch_fill_f32(float* p, float v, size_t n, hipStream_t st);
// Stable LSD radix sort of (key, value) pairs over bits [0, bits); the count
// is *count (device) when count != nullptr, else count_const; at most cap
// items.  Ping-pongs between buffers 0 and 1; returns the buffer holding the
// result.
int radix_sort(uint32_t* key[2], uint32_t* val[2], const uint32_t* count, uint32_t count_const, uint32_t cap,
               int bits, uint32_t* hist, hipStream_t st);
size_t radix_hist_words(uint32_t cap);
// offs[j] = exclusive scan of ntiles[val[j]]; total -> status[kStPairs] and offs[n]
void launch_pair_offsets(const uint32_t* val, const uint32_t* ntiles, int n, uint32_t* offs, uint32_t* bsum,
                         uint32_t* status, uint32_t cap, hipStream_t st);
size_t scan_bsum_words(int n);
void launch_emit(const uint32_t* val, const uint32_t* ntiles, const int4* rect, const uint32_t* offs, int n,
                 const EmitTable& E, uint32_t cap, uint32_t* ptile, uint32_t* pval, hipStream_t st);
// work queue keys: heaviest tiles first
void launch_queue_keys(const uint2* ranges, int n_tiles, uint32_t* key, uint32_t* val, hipStream_t st);
void launch_store_tile_args(const TileArgs& a, TileArgs* dst, hipStream_t st);
void launch_ranges(const uint32_t* ptile, const uint32_t* count, uint32_t cap, uint2* ranges, int n_tiles,
                   hipStream_t st);
void launch_count_visible(const uint32_t* visible, int n, uint32_t* status, hipStream_t st);

// blend.hip
void launch_blend_forward(const TileArgs& a, int n_tiles, hipStream_t st);
void launch_blend_backward(const TileArgs& a, int n_tiles, hipStream_t st);
void launch_blend_persistent(const BatchArgs& b, int grid, bool backward, hipStream_t st);
bool tile_shape_supported(int tw, int th);

// splat_backward.hip
void launch_splat_backward(const SplatBwdArgs& a, hipStream_t st);

}  // namespace gs
