// C-ABI of the gs2d library: plan creation, workspace layout and the
// forward / adjoint render orchestration (declarations in include/gs2d.h).
//
// Two execution layouts:
//  - per sensor: each sensor runs its own preprocess -> depth sort -> pair
//    emission -> tile sort -> ranges -> compositing chain in its own
//    workspace region;
//  - batched (one simulation step): every sensor's surfel records live in one
//    record space (record id = sensor's record base + surfel index), one depth
//    sort orders all of them, one emission and one stable tile sort build the
//    pair list over a global tile-id space (sensor tile offset + tile), and
//    one persistent compositing launch serves every sensor.  A whole step can
//    be captured into one HIP graph.
// Either way compositing drains a heaviest-first queue of (tile, segment)
// work items: tile lists longer than the segment length are split and merged
// (see blend.hip).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gs_internal.h"
#include "kernels.h"

using namespace gs;

namespace {

thread_local std::string g_last_msg;
thread_local gs_status g_last_status = GS_OK;

gs_status fail(gs_status s, const std::string& msg) {
  g_last_status = s;
  g_last_msg = msg;
  return s;
}

gs_status ok() {
  g_last_status = GS_OK;
  return GS_OK;
}

#define GS_HIP_TRY(expr)                                                                                \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess) return fail(GS_ERR_HIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
  } while (0)

struct Layout {
  size_t off = 0;
  size_t take(size_t bytes) {
    size_t o = off;
    off += (bytes + 255) & ~size_t(255);
    return o;
  }
};

// Offsets of the per-surfel and pair arrays of one record space.
struct RecordArrays {
  size_t o_rec = 0, o_rec64 = 0, o_grz = 0, o_rect = 0, o_ntiles = 0, o_visible = 0, o_key0 = 0, o_key1 = 0,
         o_val0 = 0, o_val1 = 0, o_offs = 0, o_bsum = 0, o_hist = 0, o_ptile0 = 0, o_ptile1 = 0, o_pval0 = 0,
         o_pval1 = 0, o_ranges = 0, o_status = 0, o_gacc = 0;
  // compositing work queue
  size_t o_pslot = 0, o_arrive = 0, o_qhdr = 0, o_sbsum = 0, o_qkey0 = 0, o_qkey1 = 0, o_qval0 = 0, o_qval1 = 0,
         o_items = 0, o_part = 0, part_stride = 0, o_flag = 0, o_walk = 0, o_qcnt = 0;
  uint32_t n_rec = 0, cap = 0;
  uint32_t status_words = kStWords;  // words cleared at the start of a frame
  uint32_t seg_len = 0, cap_items = 0, pslot_cap = 0;
  int n_tiles = 0, tile_bits = 0, rays = 256, key_bits = 16;
  int pair_buf = 0;   // buffer holding the sorted pairs
  int queue_buf = 0;  // buffer holding the sorted work items
  int grid_fwd = 0, grid_bwd = 0;
  int kinds = 0;  // sensor kinds served (bit 0 pinhole, bit 1 LiDAR, bit 2 cylindrical)

  void layout(Layout& L, uint32_t n, uint32_t cap_, int tiles, int rays_, uint32_t seg) {
    n_rec = n;
    cap = cap_;
    n_tiles = tiles;
    rays = rays_;
    seg_len = seg;
    const bool split = seg != 0xFFFFFFFFu;
    cap_items = (uint32_t)tiles + (split ? cap_ / seg : 0u) + 1u;
    pslot_cap = split ? 2u * (cap_ / seg) + 2u : 0u;
    key_bits = seg <= 0xFFFFu ? 16 : 24;
    queue_buf = (key_bits / 8) % 2;
    tile_bits = 0;
    while ((1 << tile_bits) < tiles) ++tile_bits;
    pair_buf = ((tile_bits + 7) / 8) % 2;
    const size_t N = n;
    o_status = L.take(kStWords * 4);
    // the pair-offset scan's ticket and look-back words sit right after the
    // status words, so that the frame's one status fill clears them too
    o_bsum = L.take(scan_bsum_words((int)N) * 4);
    status_words = (uint32_t)((o_bsum - o_status) / 4 + scan_bsum_words((int)N));
    o_rec = L.take(N * 64);
    o_rec64 = L.take(N * 8 * kRec64);
    o_grz = L.take(N * 8 * kGrz);
    o_rect = L.take(N * 16);
    o_ntiles = L.take(N * 4);
    o_visible = L.take(N * 4);
    o_key0 = L.take(N * 4);
    o_key1 = L.take(N * 4);
    o_val0 = L.take(N * 4);
    o_val1 = L.take(N * 4);
    o_offs = L.take((N + 1) * 4);
    size_t hw = radix_hist_words(cap);
    const size_t hw2 = radix_hist_words(n);
    const size_t hw3 = radix_hist_words((uint32_t)tiles);
    const size_t hw4 = radix_hist_words(cap_items);
    hw = hw > hw2 ? hw : hw2;
    hw = hw > hw3 ? hw : hw3;
    hw = hw > hw4 ? hw : hw4;
    o_hist = L.take(hw * 4);
    o_ptile0 = L.take((size_t)cap * 4);
    o_ptile1 = L.take((size_t)cap * 4);
    o_pval0 = L.take((size_t)cap * 4);
    o_pval1 = L.take((size_t)cap * 4);
    o_ranges = L.take((size_t)tiles * 8);
    o_gacc = L.take(N * 4 * kGradFields);
    o_pslot = L.take((size_t)tiles * 4);
    o_arrive = L.take((size_t)tiles * 4);
    o_qhdr = L.take(256);
    o_qcnt = L.take(kQueues * kQCntStride * 4);
    o_sbsum = L.take(seg_bsum_words(tiles) * 4);
    o_qkey0 = L.take((size_t)cap_items * 4);
    o_qkey1 = L.take((size_t)cap_items * 4);
    o_qval0 = L.take((size_t)cap_items * 4);
    o_qval1 = L.take((size_t)cap_items * 4);
    o_items = L.take((size_t)cap_items * 16);
    part_stride = (size_t)pslot_cap * (size_t)rays;
    o_part = L.take(11 * part_stride * 4);
    o_flag = L.take((size_t)pslot_cap * 4);
    o_walk = L.take((size_t)pslot_cap * 2 * 8);
  }
};

struct SensorPlan {
  gs_sensor_desc desc;
  SensorK K;
  int scene = 0;
  int n_tiles = 0;
  size_t base = 0;  // workspace byte offset of this sensor's region
  size_t o_pose = 0, o_Tfinal = 0, o_nlast = 0, o_mpair = 0, o_status = 0;
  RecordArrays R;          // per-sensor layout only
  uint32_t rec_base = 0;   // batched layout: first record id
  float* d_tabs = nullptr; // LiDAR / cylindrical tables (device, owned by the plan)
};

struct ScenePlan {
  gs_scene_desc desc;
  std::vector<int32_t> offsets;
  int pose_base = 0;
};

}  // namespace

struct gs_plan {
  int device = 0;
  std::vector<ScenePlan> scenes;
  std::vector<SensorPlan> sensors;
  OptsK O;
  gs_render_opts opts;
  int batched = 0;
  size_t ws_bytes = 0;
  // batched record space
  size_t gbase = 0;
  RecordArrays G;
  int tile_off[GS_MAX_SENSORS + 1] = {0};
  float T_accept = 0.0f;
  // stage timing
  struct Interval {
    int stage;
    hipEvent_t e0, e1;
  };
  std::vector<hipEvent_t> pool;
  std::vector<Interval> intervals;
  size_t next_event = 0;
  bool capturing = false;
  // captured forward
  hipGraphExec_t graph_exec = nullptr;
  std::vector<gs_scene> g_scenes;
  std::vector<float*> g_outputs;
  const float* g_sensor_poses = nullptr;
  const float* g_group_poses = nullptr;
  void* g_workspace = nullptr;
  hipStream_t g_stream = nullptr;
  int64_t replays = 0;
  // captured step (any work enqueued between begin and end capture)
  hipGraphExec_t step_exec = nullptr;
  hipStream_t step_stream = nullptr;
  bool step_capturing = false;
  int64_t step_launches = 0;
  bool count_pairs = false;  // forward compositing counts pairs (calibration)
};

namespace {

GroupsK groups_of(const ScenePlan& sp) {
  GroupsK g;
  memset(&g, 0, sizeof(g));
  g.n = sp.desc.n_groups;
  g.pose_base = sp.pose_base;
  for (int i = 0; i <= sp.desc.n_groups; ++i) g.off[i] = sp.offsets[i];
  return g;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(static_cast<char*>(ws) + off);
}

// SensorWS view of a record space starting at byte `base`, shifted to records [rb, ...).
SensorWS record_ws(const RecordArrays& R, void* ws, size_t base, uint32_t rb) {
  char* b = static_cast<char*>(ws) + base;
  SensorWS w;
  memset(&w, 0, sizeof(w));
  w.rec = reinterpret_cast<float4*>(b + R.o_rec) + 4 * (size_t)rb;
  w.rec64 = reinterpret_cast<double*>(b + R.o_rec64) + kRec64 * (size_t)rb;
  w.grz = reinterpret_cast<double*>(b + R.o_grz) + kGrz * (size_t)rb;
  w.rect = reinterpret_cast<int4*>(b + R.o_rect) + rb;
  w.ntiles = reinterpret_cast<uint32_t*>(b + R.o_ntiles) + rb;
  w.visible = reinterpret_cast<uint32_t*>(b + R.o_visible) + rb;
  w.key[0] = reinterpret_cast<uint32_t*>(b + R.o_key0) + rb;
  w.key[1] = reinterpret_cast<uint32_t*>(b + R.o_key1) + rb;
  w.val[0] = reinterpret_cast<uint32_t*>(b + R.o_val0) + rb;
  w.val[1] = reinterpret_cast<uint32_t*>(b + R.o_val1) + rb;
  w.offs = reinterpret_cast<uint32_t*>(b + R.o_offs);
  w.bsum = reinterpret_cast<uint32_t*>(b + R.o_bsum);
  w.hist = reinterpret_cast<uint32_t*>(b + R.o_hist);
  w.ptile[0] = reinterpret_cast<uint32_t*>(b + R.o_ptile0);
  w.ptile[1] = reinterpret_cast<uint32_t*>(b + R.o_ptile1);
  w.pval[0] = reinterpret_cast<uint32_t*>(b + R.o_pval0);
  w.pval[1] = reinterpret_cast<uint32_t*>(b + R.o_pval1);
  w.ranges = reinterpret_cast<uint2*>(b + R.o_ranges);
  w.status = reinterpret_cast<uint32_t*>(b + R.o_status);
  w.gacc = reinterpret_cast<float*>(b + R.o_gacc) + rb;
  return w;
}

const RecordArrays& records_of(const gs_plan* p, const SensorPlan& s) { return p->batched ? p->G : s.R; }
size_t records_base(const gs_plan* p, const SensorPlan& s) { return p->batched ? p->gbase : s.base; }

SensorWS sensor_ws(const gs_plan* p, const SensorPlan& s, void* ws) {
  SensorWS w = record_ws(records_of(p, s), ws, records_base(p, s), p->batched ? s.rec_base : 0);
  w.pose = at<float>(ws, s.base + s.o_pose);
  w.T_final = at<float>(ws, s.base + s.o_Tfinal);
  w.n_last = at<uint32_t>(ws, s.base + s.o_nlast);
  w.mpair = at<uint32_t>(ws, s.base + s.o_mpair);
  return w;
}

PrepArgs prep_args(const gs_plan* p, const SensorPlan& s, const gs_scene& sc, const SensorWS& ws) {
  const ScenePlan& sp = p->scenes[s.scene];
  PrepArgs a;
  memset(&a, 0, sizeof(a));
  a.n = sp.desc.n_splats;
  a.mean = sc.mean;
  a.quat = sc.quat;
  a.scale = sc.scale;
  a.opacity = sc.opacity;
  a.rgb = sc.rgb;
  a.sh = sc.sh;
  a.intensity = sc.intensity;
  a.drop = sc.drop;
  a.sh_degree = sp.desc.sh_degree;
  a.groups = groups_of(sp);
  a.S = s.K;
  a.O = p->O;
  a.ws = ws;
  a.rec_base = p->batched ? s.rec_base : 0;
  a.gacc_stride = records_of(p, s).n_rec;
  return a;
}

TileArgs tile_args(const gs_plan* p, const SensorPlan& s, void* ws) {
  const RecordArrays& R = records_of(p, s);
  const SensorWS full = record_ws(R, ws, records_base(p, s), 0);
  TileArgs t;
  memset(&t, 0, sizeof(t));
  t.S = s.K;
  t.O = p->O;
  t.rec = full.rec;
  t.rec64 = full.rec64;
  t.grz = full.grz;
  t.ranges = full.ranges;
  t.pval = full.pval[R.pair_buf];
  t.T_final = at<float>(ws, s.base + s.o_Tfinal);
  t.n_last = at<uint32_t>(ws, s.base + s.o_nlast);
  t.mpair = at<uint32_t>(ws, s.base + s.o_mpair);
  t.status = full.status;
  t.gacc = full.gacc;
  t.gacc_stride = R.n_rec;
  return t;
}

EmitTable emit_table(const gs_plan* p, const std::vector<int>& sensors) {
  EmitTable E;
  memset(&E, 0, sizeof(E));
  E.n = (int)sensors.size();
  for (int k = 0; k < E.n; ++k) {
    const SensorPlan& s = p->sensors[sensors[k]];
    E.rec_base[k] = p->batched ? s.rec_base : 0;
    E.n_tx[k] = s.K.n_tx;
    E.tile_off[k] = s.K.tile_offset;
  }
  E.rec_base[E.n] = 0xFFFFFFFFu;
  return E;
}

// Kind bit of a sensor for the compositing kernels' variants.
int kind_bit(int kind) { return kind == GS_SENSOR_PINHOLE ? 1 : kind == GS_SENSOR_LIDAR ? 2 : 4; }

gs_status check_scene(const gs_plan* p, int si, const gs_scene& sc, bool need_colour, bool need_intensity) {
  const gs_scene_desc& d = p->scenes[si].desc;
  if (d.n_splats == 0) return GS_OK;
  if (!sc.mean || !sc.quat || !sc.scale || !sc.opacity)
    return fail(GS_ERR_INVALID_ARG, "scene " + std::to_string(si) + ": mean/quat/scale/opacity must be non-null");
  if (need_colour) {
    if (d.sh_degree >= 0 && !sc.sh) return fail(GS_ERR_INVALID_ARG, "scene needs SH coefficients");
    if (d.sh_degree < 0 && !sc.rgb) return fail(GS_ERR_INVALID_ARG, "scene needs rgb");
  }
  if (need_intensity && !sc.intensity) return fail(GS_ERR_INVALID_ARG, "LiDAR scene needs intensity");
  return GS_OK;
}

// Marks the start of a stage: returns the start event or nullptr when timing
// is off, the event pool is exhausted or a graph is being captured.
hipEvent_t stage_begin(gs_plan* p, hipStream_t st) {
  if (p->capturing || p->next_event + 2 > p->pool.size()) return nullptr;
  hipEvent_t e = p->pool[p->next_event++];
  (void)hipEventRecord(e, st);
  return e;
}

void stage_end(gs_plan* p, hipStream_t st, int stage, hipEvent_t e0) {
  if (!e0) return;
  hipEvent_t e1 = p->pool[p->next_event++];
  (void)hipEventRecord(e1, st);
  p->intervals.push_back({stage, e0, e1});
}

gs_status validate_call(const gs_plan* p, const gs_scene* scenes, const float* sensor_poses,
                        const float* group_poses, const void* outputs, void* workspace) {
  if (!p || !scenes || !sensor_poses || !group_poses || !outputs || !workspace)
    return fail(GS_ERR_INVALID_ARG, "null argument to the render call");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
    return fail(GS_ERR_INVALID_ARG, "workspace must be 256-B aligned");
  for (size_t si = 0; si < p->sensors.size(); ++si) {
    const SensorPlan& s = p->sensors[si];
    gs_status cs = check_scene(p, s.scene, scenes[s.scene], s.K.kind != GS_SENSOR_LIDAR, s.K.kind == GS_SENSOR_LIDAR);
    if (cs != GS_OK) return cs;
  }
  return GS_OK;
}

// Depth sort, emission, tile sort and ranges over one record space.
void sort_and_bin(gs_plan* p, const RecordArrays& R, size_t rbase, const std::vector<int>& sensors, void* workspace,
                  hipStream_t st) {
  SensorWS w = record_ws(R, workspace, rbase, 0);
  hipEvent_t ev = stage_begin(p, st);
  // only the visible records are sorted: compacted in record order into the
  // second buffers (offs serves as the block-count scratch; their number to
  // kStVisible), then the stable depth sort over the first kStVisible of them
  launch_compact_visible(w.key[0], w.val[0], (int)R.n_rec, w.offs, w.key[1], w.val[1], w.status + kStVisible, st);
  if (p->batched) {
    VisibleSplit vs;
    memset(&vs, 0, sizeof(vs));
    vs.n = (int)sensors.size();
    for (int k = 0; k < vs.n; ++k) {
      const SensorPlan& s = p->sensors[sensors[k]];
      vs.rec_base[k] = s.rec_base;
      vs.status[k] = at<uint32_t>(workspace, s.base + s.o_status);
    }
    vs.rec_base[vs.n] = (uint32_t)R.n_rec;
    launch_visible_split(w.val[1], w.status + kStVisible, vs, st);
  }
  uint32_t* ks[2] = {w.key[1], w.key[0]};
  uint32_t* vs[2] = {w.val[1], w.val[0]};
  const uint32_t* n_vis = w.status + kStVisible;
  const int kb = radix_sort(ks, vs, n_vis, 0, R.n_rec, 32, w.hist, w.status + kStSortStall, st);
  stage_end(p, st, GS_STAGE_DEPTH_SORT, ev);
  ev = stage_begin(p, st);
  launch_offsets_emit(vs[kb], w.ntiles, w.rect, (int)R.n_rec, n_vis, emit_table(p, sensors), w.bsum, w.status, R.cap,
                      w.ptile[0], w.pval[0], st);
  stage_end(p, st, GS_STAGE_EMIT, ev);
  ev = stage_begin(p, st);
  (void)radix_sort(w.ptile, w.pval, w.status + kStPairs, 0, R.cap, R.tile_bits, w.hist, w.status + kStSortStall, st);
  stage_end(p, st, GS_STAGE_TILE_SORT, ev);
  ev = stage_begin(p, st);
  launch_ranges(w.ptile[R.pair_buf], w.status + kStPairs, R.cap, w.ranges, R.n_tiles, st);
  stage_end(p, st, GS_STAGE_RANGES, ev);
}

// Work items of one record space: segment counts, scans, keys, sort.
void build_queue(gs_plan* p, RecordArrays& R, size_t rbase, void* workspace, hipStream_t st) {
  char* b = static_cast<char*>(workspace) + rbase;
  SegScanArgs a;
  memset(&a, 0, sizeof(a));
  a.ranges = reinterpret_cast<const uint2*>(b + R.o_ranges);
  a.n_tiles = R.n_tiles;
  a.seg_len = R.seg_len;
  a.key_bits = R.key_bits;
  a.bsum = reinterpret_cast<uint2*>(b + R.o_sbsum);
  a.hdr = reinterpret_cast<uint32_t*>(b + R.o_qhdr);
  a.pslot_base = reinterpret_cast<uint32_t*>(b + R.o_pslot);
  a.arrive = reinterpret_cast<uint32_t*>(b + R.o_arrive);
  a.slot_flag = reinterpret_cast<uint32_t*>(b + R.o_flag);
  a.walk = reinterpret_cast<unsigned long long*>(b + R.o_walk);
  a.key = reinterpret_cast<uint32_t*>(b + R.o_qkey0);
  a.val = reinterpret_cast<uint32_t*>(b + R.o_qval0);
  a.items = reinterpret_cast<uint4*>(b + R.o_items);
  a.cap_items = R.cap_items;
  a.pslot_cap = R.pslot_cap;
  a.status = reinterpret_cast<uint32_t*>(b + R.o_status);
  a.qcnt = reinterpret_cast<uint32_t*>(b + R.o_qcnt);
  launch_build_items(a, st);
  uint32_t* qk[2] = {reinterpret_cast<uint32_t*>(b + R.o_qkey0), reinterpret_cast<uint32_t*>(b + R.o_qkey1)};
  uint32_t* qv[2] = {reinterpret_cast<uint32_t*>(b + R.o_qval0), reinterpret_cast<uint32_t*>(b + R.o_qval1)};
  (void)radix_sort(qk, qv, a.hdr, 0, R.cap_items, R.key_bits, reinterpret_cast<uint32_t*>(b + R.o_hist),
                   a.status + kStSortStall, st);
}

// Queue view over sensors [s0, s1) sharing record space R at byte rbase;
// out / out_fwd / gout hold the per-sensor output pointers of this call.
QueueArgs queue_args(const gs_plan* p, const RecordArrays& R, size_t rbase, int s0, int s1, void* workspace,
                     float* const* out, const float* const* out_fwd, const float* const* gout) {
  char* b = static_cast<char*>(workspace) + rbase;
  QueueArgs q;
  memset(&q, 0, sizeof(q));
  for (int i = s0; i < s1; ++i) {
    TileArgs t = tile_args(p, p->sensors[i], workspace);
    if (out) t.out = out[i];
    if (out_fwd) t.out_fwd = out_fwd[i];
    if (gout) t.gout = gout[i];
    q.tiles[i - s0] = t;
  }
  q.n_sensors = s1 - s0;
  for (int i = 0; i <= q.n_sensors; ++i) q.tile_off[i] = p->batched ? p->tile_off[s0 + i] : (i ? R.n_tiles : 0);
  q.queue = reinterpret_cast<const uint32_t*>(b + (R.queue_buf ? R.o_qval1 : R.o_qval0));
  q.items = reinterpret_cast<const uint4*>(b + R.o_items);
  q.n_items = reinterpret_cast<const uint32_t*>(b + R.o_qhdr);
  q.hdr = reinterpret_cast<uint32_t*>(b + R.o_qhdr);
  q.slot_flag = reinterpret_cast<uint32_t*>(b + R.o_flag);
  q.walk = reinterpret_cast<unsigned long long*>(b + R.o_walk);
  q.walk_cap = 2 * R.pslot_cap;
  q.cap_items = R.cap_items;
  q.counter = reinterpret_cast<uint32_t*>(b + R.o_qcnt);
  q.arrive = reinterpret_cast<uint32_t*>(b + R.o_arrive);
  q.pslot_base = reinterpret_cast<const uint32_t*>(b + R.o_pslot);
  q.part = reinterpret_cast<float*>(b + R.o_part);
  q.part_stride = R.part_stride;
  q.pslot_cap = R.pslot_cap;
  q.seg_len = R.seg_len;
  q.T_accept = p->T_accept;
  return q;
}

void enqueue_forward(gs_plan* p, const gs_scene* scenes, const float* sensor_poses, const float* group_poses,
                     float* const* outputs, void* workspace, hipStream_t st) {
  if (!p->batched) {
    for (size_t si = 0; si < p->sensors.size(); ++si) {
      SensorPlan& s = p->sensors[si];
      const ScenePlan& sp = p->scenes[s.scene];
      SensorWS ws = sensor_ws(p, s, workspace);
      hipEvent_t ev = stage_begin(p, st);
      launch_fill_u32(ws.status, 0u, s.R.status_words, st);
      launch_compose_poses(sensor_poses + 12 * si, group_poses, sp.pose_base, sp.desc.n_groups, ws.pose, st);
      launch_prep(prep_args(p, s, scenes[s.scene], ws), st);
      stage_end(p, st, GS_STAGE_PREPROCESS, ev);
      sort_and_bin(p, s.R, s.base, std::vector<int>{(int)si}, workspace, st);
      ev = stage_begin(p, st);
      build_queue(p, s.R, s.base, workspace, st);
      stage_end(p, st, GS_STAGE_RANGES, ev);
      ev = stage_begin(p, st);
      QueueArgs q = queue_args(p, s.R, s.base, (int)si, (int)si + 1, workspace, outputs, nullptr, nullptr);
      launch_blend_queue(q, s.R.rays, s.R.kinds, s.R.grid_fwd, false, p->count_pairs, st);
      stage_end(p, st, GS_STAGE_BLEND, ev);
    }
    return;
  }
  // batched step
  SensorWS g = record_ws(p->G, workspace, p->gbase, 0);
  hipEvent_t ev = stage_begin(p, st);
  launch_fill_u32(g.status, 0u, p->G.status_words, st);
  SensorSetup setup;
  memset(&setup, 0, sizeof(setup));
  setup.n = (int)p->sensors.size();
  for (size_t si = 0; si < p->sensors.size(); ++si) {
    const SensorPlan& s = p->sensors[si];
    const ScenePlan& sp = p->scenes[s.scene];
    setup.sensor_pose[si] = sensor_poses + 12 * si;
    setup.pose_base[si] = sp.pose_base;
    setup.n_groups[si] = sp.desc.n_groups;
    setup.pose_out[si] = sensor_ws(p, s, workspace).pose;
    setup.status[si] = at<uint32_t>(workspace, s.base + s.o_status);
  }
  launch_sensor_setup(group_poses, setup, st);
  for (size_t si = 0; si < p->sensors.size(); ++si) {
    SensorPlan& s = p->sensors[si];
    launch_prep(prep_args(p, s, scenes[s.scene], sensor_ws(p, s, workspace)), st);
  }
  stage_end(p, st, GS_STAGE_PREPROCESS, ev);
  std::vector<int> all(p->sensors.size());
  for (size_t i = 0; i < all.size(); ++i) all[i] = (int)i;
  sort_and_bin(p, p->G, p->gbase, all, workspace, st);
  (void)g;
  ev = stage_begin(p, st);
  build_queue(p, p->G, p->gbase, workspace, st);
  stage_end(p, st, GS_STAGE_RANGES, ev);
  ev = stage_begin(p, st);
  QueueArgs q = queue_args(p, p->G, p->gbase, 0, (int)p->sensors.size(), workspace, outputs, nullptr, nullptr);
  launch_blend_queue(q, p->G.rays, p->G.kinds, p->G.grid_fwd, false, p->count_pairs, st);
  stage_end(p, st, GS_STAGE_BLEND, ev);
}

}  // namespace

namespace gs {
gs_status set_error(gs_status s, const std::string& msg) {
  g_last_status = s;
  g_last_msg = msg;
  return s;
}
}  // namespace gs

extern "C" {

const char* gs_version(void) { return "gs2d 0.3 (gfx950)"; }

const char* gs_status_string(gs_status s) {
  switch (s) {
    case GS_OK: return "ok";
    case GS_ERR_INVALID_ARG: return "invalid argument";
    case GS_ERR_CAPACITY: return "pair capacity exceeded";
    case GS_ERR_HIP: return "HIP runtime error";
    case GS_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

gs_status gs_last_error(char* buf, size_t n) {
  if (buf && n > 0) {
    size_t m = g_last_msg.size() < n - 1 ? g_last_msg.size() : n - 1;
    memcpy(buf, g_last_msg.data(), m);
    buf[m] = 0;
  }
  return g_last_status;
}

void gs_plan_destroy(gs_plan* p) {
  if (!p) return;
  if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
  if (p->step_exec) (void)hipGraphExecDestroy(p->step_exec);
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  for (auto& s : p->sensors)
    if (s.d_tabs) (void)hipFree(s.d_tabs);
  delete p;
}

gs_status gs_plan_create(const gs_plan_desc* desc, gs_plan** out) {
  if (!desc || !out) return fail(GS_ERR_INVALID_ARG, "null descriptor or output");
  *out = nullptr;
  if (desc->n_scenes < 1 || desc->n_scenes > GS_MAX_SENSORS || !desc->scenes)
    return fail(GS_ERR_INVALID_ARG, "n_scenes must be in [1, GS_MAX_SENSORS]");
  if (desc->n_sensors < 1 || desc->n_sensors > GS_MAX_SENSORS || !desc->sensors)
    return fail(GS_ERR_INVALID_ARG, "n_sensors must be in [1, GS_MAX_SENSORS]");
  const gs_render_opts& o = desc->opts;
  if (!(o.alpha_max > 0.0f && o.alpha_max < 1.0f) || !(o.alpha_min >= 0.0f) || !(o.T_min >= 0.0f) ||
      !(o.cutoff2 > 0.0f) || !(o.lp_inv_sigma2 > 0.0f) || !std::isfinite(o.cutoff2))
    return fail(GS_ERR_INVALID_ARG, "render options out of range");
  gs_plan* p = new gs_plan();
  (void)hipGetDevice(&p->device);
  p->opts = o;
  p->batched = desc->batched ? 1 : 0;
  p->O.alpha_min = o.alpha_min;
  p->O.alpha_max = o.alpha_max;
  p->O.T_min = o.T_min;
  p->O.cutoff2 = o.cutoff2;
  p->O.lp = o.lp_inv_sigma2;
  p->O.rl = sqrtf(o.cutoff2 / o.lp_inv_sigma2);
  p->O.lowpass = o.lowpass ? 1 : 0;
  p->O.bg0 = o.bg[0];
  p->O.bg1 = o.bg[1];
  p->O.bg2 = o.bg[2];
  // segment length of the compositing queue: 0 = default, < 0 = never split
  uint32_t seg_len = 1024u;
  if (desc->segment_pairs < 0) {
    seg_len = 0xFFFFFFFFu;
  } else if (desc->segment_pairs > 0) {
    if (desc->segment_pairs < 32 || desc->segment_pairs > 32768) {
      delete p;
      return fail(GS_ERR_INVALID_ARG, "segment_pairs must be 0, negative, or in [32, 32768]");
    }
    seg_len = (uint32_t)desc->segment_pairs;
  }
  // A split segment is accepted whole by the merge while T * T_seg >= T_accept;
  // the margin covers the relative rounding of products of up to L factors.
  p->T_accept = o.T_min * (1.0f + (float)(seg_len > 65536u ? 65536u : seg_len) * 0x1p-22f);
  int cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, p->device) != hipSuccess || cus <= 0)
    cus = 256;
  auto grid_for = [&](int rays, int kinds, bool bwd) {
    const int per = blend_blocks_per_cu(rays, kinds, bwd);
    return cus * (per > 0 ? per : 2);
  };
  int all_kinds = 0;
  int pose_base = 0;
  for (int i = 0; i < desc->n_scenes; ++i) {
    const gs_scene_desc& d = desc->scenes[i];
    ScenePlan sp;
    sp.desc = d;
    if (d.n_splats < 0 || d.n_groups < 1 || d.n_groups > GS_MAX_GROUPS || !d.group_offsets || d.sh_degree > 3) {
      gs_plan_destroy(p);
      return fail(GS_ERR_INVALID_ARG, "scene " + std::to_string(i) + ": bad shape");
    }
    if ((uint32_t)d.n_splats > kMaxSortKeys) {
      gs_plan_destroy(p);
      return fail(GS_ERR_UNSUPPORTED, "scene " + std::to_string(i) + ": more than 2^30 - 1 surfels");
    }
    sp.offsets.assign(d.group_offsets, d.group_offsets + d.n_groups + 1);
    bool okoff = sp.offsets[0] == 0 && sp.offsets[d.n_groups] == d.n_splats;
    for (int g = 0; g < d.n_groups; ++g) okoff = okoff && sp.offsets[g] <= sp.offsets[g + 1];
    if (!okoff) {
      gs_plan_destroy(p);
      return fail(GS_ERR_INVALID_ARG, "scene " + std::to_string(i) + ": group offsets must rise from 0 to N");
    }
    sp.desc.group_offsets = nullptr;
    sp.pose_base = pose_base;
    pose_base += d.n_groups;
    p->scenes.push_back(sp);
  }
  Layout L;
  uint64_t total_rec = 0, total_cap = 0;
  int total_tiles = 0;
  for (int si = 0; si < desc->n_sensors; ++si) {
    const gs_sensor_desc& d = desc->sensors[si];
    SensorPlan s;
    s.desc = d;
    s.desc.elevations = nullptr;
    if (d.scene < 0 || d.scene >= desc->n_scenes || d.width <= 0 || d.height <= 0 || !(d.z_near > 0.0f)) {
      gs_plan_destroy(p);
      return fail(GS_ERR_INVALID_ARG, "sensor " + std::to_string(si) + ": bad size, scene or z_near");
    }
    s.scene = d.scene;
    const ScenePlan& sp = p->scenes[d.scene];
    const int N = sp.desc.n_splats;
    SensorK& K = s.K;
    memset(&K, 0, sizeof(K));
    K.kind = d.kind;
    K.W = d.width;
    K.H = d.height;
    K.z_near = d.z_near;
    if (d.kind == GS_SENSOR_PINHOLE) {
      if (!(d.fx > 0.0f && d.fy > 0.0f)) {
        gs_plan_destroy(p);
        return fail(GS_ERR_INVALID_ARG, "sensor " + std::to_string(si) + ": focal lengths must be > 0");
      }
      // 32x8: a tile's four 8x8 ray blocks side by side (measured fastest on
      // the driving frame, whose ground and facade footprints are wide)
      K.tw = d.tile_w ? d.tile_w : 32;
      K.th = d.tile_h ? d.tile_h : 8;
      K.fx = d.fx;
      K.fy = d.fy;
      K.cx = d.cx;
      K.cy = d.cy;
    } else if (d.kind == GS_SENSOR_LIDAR) {
      if (!d.elevations) {
        gs_plan_destroy(p);
        return fail(GS_ERR_INVALID_ARG, "sensor " + std::to_string(si) + ": LiDAR needs elevations");
      }
      for (int j = 0; j + 1 < d.height; ++j)
        if (!(d.elevations[j] < d.elevations[j + 1])) {
          gs_plan_destroy(p);
          return fail(GS_ERR_INVALID_ARG, "sensor " + std::to_string(si) + ": elevations must ascend");
        }
      if (!sp.desc.has_intensity) {
        gs_plan_destroy(p);
        return fail(GS_ERR_INVALID_ARG, "sensor " + std::to_string(si) + ": LiDAR scene needs intensity");
      }
      // 16x8 by default: two waves per workgroup balance the sparse LiDAR
      // lists best (measured); a batched plan needs 256-ray tiles
      K.tw = d.tile_w ? d.tile_w : (desc->batched ? 32 : 16);
      K.th = d.tile_h ? d.tile_h : 8;
      const double two_pi = 2.0 * M_PI;
      K.inv_step = (float)((double)d.width / two_pi);
      K.step = (float)(two_pi / (double)d.width);
      K.c_lp = sqrtf(o.cutoff2 / o.lp_inv_sigma2) * K.step;
      K.lp_ang = (float)((double)o.lp_inv_sigma2 / ((double)K.step * (double)K.step));
      // sensor tables: FP64 libm values rounded to FP32
      std::vector<float> tab(3 * d.height + 2 * d.width);
      for (int j = 0; j < d.height; ++j) {
        tab[j] = (float)d.elevations[j];
        tab[d.height + j] = (float)cos(d.elevations[j]);
        tab[2 * d.height + j] = (float)sin(d.elevations[j]);
      }
      for (int i = 0; i < d.width; ++i) {
        const double az = (two_pi * (double)i) / (double)d.width;
        tab[3 * d.height + i] = (float)cos(az);
        tab[3 * d.height + d.width + i] = (float)sin(az);
      }
      hipError_t e = hipMalloc(&s.d_tabs, tab.size() * sizeof(float));
      if (e == hipSuccess) e = hipMemcpy(s.d_tabs, tab.data(), tab.size() * sizeof(float), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        p->sensors.push_back(s);
        gs_plan_destroy(p);
        return fail(GS_ERR_HIP, std::string("LiDAR tables: ") + hipGetErrorString(e));
      }
      K.tab = s.d_tabs;
    } else if (d.kind == GS_SENSOR_CYLINDRICAL) {
      if (!(d.fx > 0.0f && d.fy > 0.0f)) {
        gs_plan_destroy(p);
        return fail(GS_ERR_INVALID_ARG, "sensor " + std::to_string(si) + ": focal lengths must be > 0");
      }
      K.tw = d.tile_w ? d.tile_w : 32;
      K.th = d.tile_h ? d.tile_h : 8;
      K.fx = d.fx;
      K.fy = d.fy;
      K.cx = d.cx;
      K.cy = d.cy;
    } else {
      gs_plan_destroy(p);
      return fail(GS_ERR_INVALID_ARG, "sensor " + std::to_string(si) + ": unknown kind");
    }
    // batched plans and cylindrical cameras composite 256-ray tiles
    const bool shape_ok = tile_shape_supported(K.tw, K.th) &&
                          ((!p->batched && K.kind != GS_SENSOR_CYLINDRICAL) || K.tw * K.th == 256);
    if (!shape_ok) {
      p->sensors.push_back(s);
      gs_plan_destroy(p);
      return fail(GS_ERR_UNSUPPORTED, "sensor " + std::to_string(si) + ": unsupported tile shape");
    }
    K.n_tx = (K.W + K.tw - 1) / K.tw;
    K.n_ty = (K.H + K.th - 1) / K.th;
    s.n_tiles = K.n_tx * K.n_ty;
    int64_t cap = desc->pair_capacity > 0 ? desc->pair_capacity : 16ll * N + 4096;
    if (cap > kMaxSortKeys) cap = kMaxSortKeys;
    // per-sensor region
    Layout R;
    const size_t HW = (size_t)K.W * K.H;
    s.o_status = R.take(kStWords * 4);
    s.o_pose = R.take(12 * 4 * (size_t)sp.desc.n_groups);
    s.o_Tfinal = R.take(HW * 4);
    s.o_nlast = R.take(HW * 4);
    s.o_mpair = R.take(HW * 4);
    if (p->batched) {
      K.tile_offset = total_tiles;
      s.rec_base = (uint32_t)total_rec;
      p->tile_off[si] = total_tiles;
    } else {
      K.tile_offset = 0;
      s.R.layout(R, (uint32_t)N, (uint32_t)cap, s.n_tiles, K.tw * K.th, seg_len);
      s.R.kinds = kind_bit(K.kind);
      s.R.grid_fwd = grid_for(K.tw * K.th, s.R.kinds, false);
      s.R.grid_bwd = grid_for(K.tw * K.th, s.R.kinds, true);
    }
    all_kinds |= kind_bit(K.kind);
    total_rec += (uint64_t)N;
    total_cap += (uint64_t)cap;
    total_tiles += s.n_tiles;
    s.base = L.take(R.off);
    p->sensors.push_back(s);
  }
  if (p->batched) {
    if (total_rec > (uint64_t)kMaxSortKeys) {
      gs_plan_destroy(p);
      return fail(GS_ERR_UNSUPPORTED, "batched plan exceeds 2^30 - 1 surfel records");
    }
    if (total_cap > (uint64_t)kMaxSortKeys) total_cap = kMaxSortKeys;
    p->tile_off[desc->n_sensors] = total_tiles;
    Layout R;
    p->G.layout(R, (uint32_t)total_rec, (uint32_t)total_cap, total_tiles, 256, seg_len);
    p->G.kinds = all_kinds;
    p->G.grid_fwd = grid_for(256, all_kinds, false);
    p->G.grid_bwd = grid_for(256, all_kinds, true);
    p->gbase = L.take(R.off);
  }
  p->ws_bytes = L.off;
  *out = p;
  return ok();
}

gs_status gs_plan_set_timing(gs_plan* p, int32_t max_records) {
  if (!p || max_records < 0) return fail(GS_ERR_INVALID_ARG, "bad timing arguments");
  for (hipEvent_t e : p->pool) (void)hipEventDestroy(e);
  p->pool.clear();
  p->intervals.clear();
  p->next_event = 0;
  for (int i = 0; i < 2 * max_records; ++i) {
    hipEvent_t e;
    GS_HIP_TRY(hipEventCreate(&e));
    p->pool.push_back(e);
  }
  return ok();
}

gs_status gs_plan_stage_times(gs_plan* p, hipStream_t st, int32_t reset, gs_stage_times* out) {
  if (!p || !out) return fail(GS_ERR_INVALID_ARG, "null argument to gs_plan_stage_times");
  GS_HIP_TRY(hipStreamSynchronize(st));
  memset(out, 0, sizeof(*out));
  for (const auto& iv : p->intervals) {
    float ms = 0.0f;
    GS_HIP_TRY(hipEventElapsedTime(&ms, iv.e0, iv.e1));
    out->ms[iv.stage] += ms;
    out->launches[iv.stage] += 1;
    out->records += 1;
  }
  if (reset) {
    p->intervals.clear();
    p->next_event = 0;
  }
  return ok();
}

gs_status gs_plan_set_counters(gs_plan* p, int32_t on) {
  if (!p) return fail(GS_ERR_INVALID_ARG, "null plan");
  p->count_pairs = on != 0;
  return ok();
}

gs_status gs_plan_workspace_size(const gs_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(GS_ERR_INVALID_ARG, "null plan or output");
  *bytes = p->ws_bytes;
  return ok();
}

gs_status gs_plan_inspect(const gs_plan* p, int32_t sensor, gs_workspace_view* out) {
  if (!p || !out || sensor < 0 || sensor >= (int)p->sensors.size()) return fail(GS_ERR_INVALID_ARG, "bad inspect args");
  const SensorPlan& s = p->sensors[sensor];
  const RecordArrays& R = records_of(p, s);
  const size_t b = records_base(p, s);
  out->pair_surfel = b + (R.pair_buf ? R.o_pval1 : R.o_pval0);
  out->pair_tile = b + (R.pair_buf ? R.o_ptile1 : R.o_ptile0);
  out->tile_ranges = b + R.o_ranges;
  out->visible = b + R.o_visible + 4ull * (p->batched ? s.rec_base : 0);
  out->pair_count = b + R.o_status + 4 * kStPairs;
  out->n_tiles = p->batched ? R.n_tiles : s.n_tiles;
  out->tile_offset = s.K.tile_offset;
  return ok();
}

gs_status gs_render_forward(gs_plan* p, const gs_scene* scenes, const float* sensor_poses, const float* group_poses,
                            float* const* outputs, void* workspace, hipStream_t st) {
  gs_status v = validate_call(p, scenes, sensor_poses, group_poses, outputs, workspace);
  if (v != GS_OK) return v;
  for (size_t si = 0; si < p->sensors.size(); ++si)
    if (!outputs[si]) return fail(GS_ERR_INVALID_ARG, "null output for sensor " + std::to_string(si));
  bool replay = !p->step_capturing && p->graph_exec && workspace == p->g_workspace &&
                sensor_poses == p->g_sensor_poses &&
                group_poses == p->g_group_poses && st == p->g_stream;
  for (size_t i = 0; replay && i < p->scenes.size(); ++i)
    replay = memcmp(&scenes[i], &p->g_scenes[i], sizeof(gs_scene)) == 0;
  for (size_t i = 0; replay && i < p->sensors.size(); ++i) replay = outputs[i] == p->g_outputs[i];
  if (replay) {
    GS_HIP_TRY(hipGraphLaunch(p->graph_exec, st));
    ++p->replays;
    return ok();
  }
  enqueue_forward(p, scenes, sensor_poses, group_poses, outputs, workspace, st);
  GS_HIP_TRY(hipGetLastError());
  return ok();
}

gs_status gs_plan_capture(gs_plan* p, const gs_scene* scenes, const float* sensor_poses, const float* group_poses,
                          float* const* outputs, void* workspace, hipStream_t st) {
  gs_status v = validate_call(p, scenes, sensor_poses, group_poses, outputs, workspace);
  if (v != GS_OK) return v;
  for (size_t si = 0; si < p->sensors.size(); ++si)
    if (!outputs[si]) return fail(GS_ERR_INVALID_ARG, "null output for sensor " + std::to_string(si));
  if (!st) return fail(GS_ERR_INVALID_ARG, "graph capture needs a non-default stream");
  if (p->graph_exec) {
    (void)hipGraphExecDestroy(p->graph_exec);
    p->graph_exec = nullptr;
  }
  GS_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  p->capturing = true;
  enqueue_forward(p, scenes, sensor_poses, group_poses, outputs, workspace, st);
  p->capturing = false;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(st, &graph);
  if (e != hipSuccess) return fail(GS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  e = hipGraphInstantiate(&p->graph_exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    p->graph_exec = nullptr;
    return fail(GS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  p->g_scenes.assign(scenes, scenes + p->scenes.size());
  p->g_outputs.assign(outputs, outputs + p->sensors.size());
  p->g_sensor_poses = sensor_poses;
  p->g_group_poses = group_poses;
  p->g_workspace = workspace;
  p->g_stream = st;
  return ok();
}

gs_status gs_plan_begin_capture(gs_plan* p, hipStream_t st) {
  if (!p) return fail(GS_ERR_INVALID_ARG, "null plan");
  if (!st) return fail(GS_ERR_INVALID_ARG, "step capture needs a non-default stream");
  if (p->step_capturing) return fail(GS_ERR_INVALID_ARG, "a step capture of this plan is already open");
  GS_HIP_TRY(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
  p->step_capturing = true;
  p->capturing = true;
  p->step_stream = st;
  return ok();
}

gs_status gs_plan_end_capture(gs_plan* p, hipStream_t st) {
  if (!p) return fail(GS_ERR_INVALID_ARG, "null plan");
  if (!p->step_capturing || st != p->step_stream)
    return fail(GS_ERR_INVALID_ARG, "no step capture of this plan is open on this stream");
  p->step_capturing = false;
  p->capturing = false;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(st, &graph);
  if (e != hipSuccess) return fail(GS_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
  if (p->step_exec) {
    (void)hipGraphExecDestroy(p->step_exec);
    p->step_exec = nullptr;
  }
  e = hipGraphInstantiate(&p->step_exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) {
    p->step_exec = nullptr;
    return fail(GS_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  return ok();
}

gs_status gs_plan_launch(gs_plan* p, hipStream_t st) {
  if (!p) return fail(GS_ERR_INVALID_ARG, "null plan");
  if (!p->step_exec) return fail(GS_ERR_INVALID_ARG, "no captured step to launch");
  if (p->step_capturing) return fail(GS_ERR_INVALID_ARG, "cannot launch while capturing");
  GS_HIP_TRY(hipGraphLaunch(p->step_exec, st));
  ++p->step_launches;
  return ok();
}

gs_status gs_render_backward(gs_plan* p, const gs_scene* scenes, const float* sensor_poses, const float* group_poses,
                             const float* const* outputs, const float* const* grad_outputs, void* workspace,
                             const gs_scene_grads* grads, hipStream_t st) {
  gs_status v = validate_call(p, scenes, sensor_poses, group_poses, outputs, workspace);
  if (v != GS_OK) return v;
  if (!grad_outputs || !grads) return fail(GS_ERR_INVALID_ARG, "null argument to gs_render_backward");
  for (size_t si = 0; si < p->sensors.size(); ++si)
    if (!outputs[si] || !grad_outputs[si])
      return fail(GS_ERR_INVALID_ARG, "null output/grad for sensor " + std::to_string(si));
  if (p->batched) {
    SensorWS g = record_ws(p->G, workspace, p->gbase, 0);
    hipEvent_t ev = stage_begin(p, st);
    launch_fill_f32(g.gacc, 0.0f, (size_t)p->G.n_rec * kGradFields, st);
    QueueArgs q = queue_args(p, p->G, p->gbase, 0, (int)p->sensors.size(), workspace, nullptr, outputs,
                             grad_outputs);
    launch_fill_u32(q.counter, 0u, kQueues * kQCntStride, st);
    launch_blend_queue(q, p->G.rays, p->G.kinds, p->G.grid_bwd, true, false, st);
    stage_end(p, st, GS_STAGE_BLEND_BWD, ev);
  }
  for (size_t si = 0; si < p->sensors.size(); ++si) {
    SensorPlan& s = p->sensors[si];
    SensorWS ws = sensor_ws(p, s, workspace);
    if (!p->batched) {
      const int N = p->scenes[s.scene].desc.n_splats;
      hipEvent_t ev = stage_begin(p, st);
      launch_fill_f32(ws.gacc, 0.0f, (size_t)N * kGradFields, st);
      QueueArgs q = queue_args(p, s.R, s.base, (int)si, (int)si + 1, workspace, nullptr, outputs, grad_outputs);
      launch_fill_u32(q.counter, 0u, kQueues * kQCntStride, st);
      launch_blend_queue(q, s.R.rays, s.R.kinds, s.R.grid_bwd, true, false, st);
      stage_end(p, st, GS_STAGE_BLEND_BWD, ev);
    }
    SplatBwdArgs sb;
    memset(&sb, 0, sizeof(sb));
    sb.p = prep_args(p, s, scenes[s.scene], ws);
    const gs_scene_grads& g = grads[s.scene];
    sb.g_mean = g.mean;
    sb.g_quat = g.quat;
    sb.g_scale = g.scale;
    sb.g_opacity = g.opacity;
    sb.g_rgb = g.rgb;
    sb.g_sh = g.sh;
    sb.g_intensity = g.intensity;
    sb.g_drop = g.drop;
    hipEvent_t ev = stage_begin(p, st);
    launch_splat_backward(sb, st);
    stage_end(p, st, GS_STAGE_SPLAT_BWD, ev);
  }
  GS_HIP_TRY(hipGetLastError());
  return ok();
}

gs_status gs_query_status(const gs_plan* p, const void* workspace, hipStream_t st, gs_run_status* out) {
  if (!p || !workspace || !out) return fail(GS_ERR_INVALID_ARG, "null argument to gs_query_status");
  GS_HIP_TRY(hipStreamSynchronize(st));
  memset(out, 0, sizeof(*out));
  bool over = false, stalled = false, sort_stall = false;
  auto read = [&](size_t off, uint32_t* w) {
    return hipMemcpy(w, static_cast<const char*>(workspace) + off, kStWords * 4, hipMemcpyDeviceToHost);
  };
  // pair counts: the base words plus the per-XCD replicas
  auto u64at = [](const uint32_t* w, int i) { return (int64_t)w[i] | ((int64_t)w[i + 1] << 32); };
  auto add_counts = [&](const uint32_t* w) {
    sort_stall = sort_stall || w[kStSortStall] != 0;
    out->fp64_pairs += w[kStFp64];
    out->evaluated += u64at(w, kStEvals);
    out->composited += u64at(w, kStContrib);
    for (int x = 0; x < 8; ++x) {
      const uint32_t* r = w + kStRep + 8 * x;
      out->evaluated += u64at(r, 0);
      out->composited += u64at(r, 2);
      out->fp64_pairs += r[4];
      out->wave_pairs += u64at(r, 6);
    }
  };
  auto read_queue = [&](const RecordArrays& R, size_t base) -> hipError_t {
    uint32_t h[16];
    hipError_t e = read(base + R.o_qhdr, h);
    if (e == hipSuccess) {
      out->work_items += h[0];
      out->segments += h[1];
      stalled = stalled || h[6] != 0;
    }
    return e;
  };
  if (p->batched) {
    uint32_t w[kStWords];
    GS_HIP_TRY(read(p->gbase + p->G.o_status, w));
    out->pairs[0] = w[kStPairs];
    add_counts(w);
    over = w[kStOverflow] != 0;
    GS_HIP_TRY(read_queue(p->G, p->gbase));
    for (size_t si = 0; si < p->sensors.size(); ++si) {
      uint32_t ws[kStWords];
      GS_HIP_TRY(read(p->sensors[si].base + p->sensors[si].o_status, ws));
      out->n_visible[si] = (int32_t)ws[kStVisible];
    }
  } else {
    for (size_t si = 0; si < p->sensors.size(); ++si) {
      const SensorPlan& s = p->sensors[si];
      uint32_t w[kStWords];
      GS_HIP_TRY(read(s.base + s.R.o_status, w));
      out->pairs[si] = w[kStPairs];
      out->n_visible[si] = (int32_t)w[kStVisible];
      add_counts(w);
      over = over || w[kStOverflow] != 0;
      GS_HIP_TRY(read_queue(s.R, s.base));
    }
  }
  out->overflow = over ? 1 : 0;
  out->graph_replays = p->replays;
  out->step_launches = p->step_launches;
  if (over) return fail(GS_ERR_CAPACITY, "pair capacity exceeded; re-plan with a larger pair_capacity");
  if (stalled) return fail(GS_ERR_HIP, "compositing work queue stalled (walk list inconsistent)");
  if (sort_stall) return fail(GS_ERR_HIP, "sort or scan look-back wait gave up (block statuses inconsistent)");
  return ok();
}

}  // extern "C"
