// C-ABI of the gs2d library: plan creation, workspace layout and the
// forward / adjoint render orchestration (see include/gs2d.h).
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "gs_internal.h"
#include "kernels.h"

namespace gs {
bool tile_shape_supported(int tw, int th);
}

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

#define GS_HIP_TRY(expr)                                                                      \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
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

struct SensorPlan {
  gs_sensor_desc desc;
  SensorK K;
  int scene;
  uint32_t cap;
  int n_tiles;
  int tile_bits;
  size_t base;  // workspace byte offset of this sensor's region
  // region offsets (relative to base)
  size_t o_pose, o_rec, o_rec64, o_grz, o_rect, o_ntiles, o_key0, o_key1, o_val0, o_val1, o_offs, o_bsum, o_hist,
      o_ptile0, o_ptile1, o_pval0, o_pval1, o_ranges, o_Tfinal, o_nlast, o_status, o_gacc, o_visible;
  int pair_buf;  // buffer holding the sorted pairs
  // device tables (LiDAR)
  float* d_tabs = nullptr;
};

struct ScenePlan {
  gs_scene_desc desc;
  std::vector<int32_t> offsets;
  int pose_base;
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

SensorWS ws_of(const SensorPlan& s, void* workspace) {
  char* b = static_cast<char*>(workspace) + s.base;
  SensorWS w;
  w.pose = reinterpret_cast<float*>(b + s.o_pose);
  w.rec = reinterpret_cast<float4*>(b + s.o_rec);
  w.rec64 = reinterpret_cast<double*>(b + s.o_rec64);
  w.grz = reinterpret_cast<double*>(b + s.o_grz);
  w.rect = reinterpret_cast<int4*>(b + s.o_rect);
  w.ntiles = reinterpret_cast<uint32_t*>(b + s.o_ntiles);
  w.key[0] = reinterpret_cast<uint32_t*>(b + s.o_key0);
  w.key[1] = reinterpret_cast<uint32_t*>(b + s.o_key1);
  w.val[0] = reinterpret_cast<uint32_t*>(b + s.o_val0);
  w.val[1] = reinterpret_cast<uint32_t*>(b + s.o_val1);
  w.offs = reinterpret_cast<uint32_t*>(b + s.o_offs);
  w.bsum = reinterpret_cast<uint32_t*>(b + s.o_bsum);
  w.hist = reinterpret_cast<uint32_t*>(b + s.o_hist);
  w.ptile[0] = reinterpret_cast<uint32_t*>(b + s.o_ptile0);
  w.ptile[1] = reinterpret_cast<uint32_t*>(b + s.o_ptile1);
  w.pval[0] = reinterpret_cast<uint32_t*>(b + s.o_pval0);
  w.pval[1] = reinterpret_cast<uint32_t*>(b + s.o_pval1);
  w.ranges = reinterpret_cast<uint2*>(b + s.o_ranges);
  w.T_final = reinterpret_cast<float*>(b + s.o_Tfinal);
  w.n_last = reinterpret_cast<uint32_t*>(b + s.o_nlast);
  w.status = reinterpret_cast<uint32_t*>(b + s.o_status);
  w.gacc = reinterpret_cast<float*>(b + s.o_gacc);
  w.visible = reinterpret_cast<uint32_t*>(b + s.o_visible);
  return w;
}

int ceil_log2(int n) {
  int b = 0;
  while ((1 << b) < n) ++b;
  return b;
}

PrepArgs prep_args(const gs_plan* p, const SensorPlan& s, const gs_scene& sc, SensorWS ws) {
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
  a.sh_degree = sp.desc.sh_degree;
  a.groups = groups_of(sp);
  a.S = s.K;
  a.O = p->O;
  a.ws = ws;
  return a;
}

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

}  // namespace

namespace gs {
gs_status set_error(gs_status s, const std::string& msg) {
  g_last_status = s;
  g_last_msg = msg;
  return s;
}
}  // namespace gs

extern "C" {

const char* gs_version(void) { return "gs2d 0.1 (gfx950)"; }

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

gs_status gs_plan_create(const gs_plan_desc* desc, gs_plan** out) {
  if (!desc || !out) return fail(GS_ERR_INVALID_ARG, "null descriptor or output");
  *out = nullptr;
  if (desc->n_scenes < 1 || desc->n_scenes > 2 || !desc->scenes)
    return fail(GS_ERR_INVALID_ARG, "n_scenes must be 1 or 2");
  if (desc->n_sensors < 1 || desc->n_sensors > GS_MAX_SENSORS || !desc->sensors)
    return fail(GS_ERR_INVALID_ARG, "n_sensors must be in [1, GS_MAX_SENSORS]");
  const gs_render_opts& o = desc->opts;
  if (!(o.alpha_max > 0.0f && o.alpha_max < 1.0f) || !(o.alpha_min >= 0.0f) || !(o.T_min >= 0.0f) ||
      !(o.cutoff2 > 0.0f) || !(o.lp_inv_sigma2 > 0.0f) || !std::isfinite(o.cutoff2))
    return fail(GS_ERR_INVALID_ARG, "render options out of range");
  if (desc->batched) return fail(GS_ERR_UNSUPPORTED, "batched plans are not available in this build");
  gs_plan* p = new gs_plan();
  hipGetDevice(&p->device);
  p->opts = o;
  p->batched = desc->batched;
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
  int pose_base = 0;
  for (int i = 0; i < desc->n_scenes; ++i) {
    const gs_scene_desc& d = desc->scenes[i];
    ScenePlan sp;
    sp.desc = d;
    if (d.n_splats < 0 || d.n_groups < 1 || d.n_groups > GS_MAX_GROUPS || !d.group_offsets || d.sh_degree > 3) {
      delete p;
      return fail(GS_ERR_INVALID_ARG, "scene " + std::to_string(i) + ": bad shape");
    }
    sp.offsets.assign(d.group_offsets, d.group_offsets + d.n_groups + 1);
    bool okoff = sp.offsets[0] == 0 && sp.offsets[d.n_groups] == d.n_splats;
    for (int g = 0; g < d.n_groups; ++g) okoff = okoff && sp.offsets[g] <= sp.offsets[g + 1];
    if (!okoff) {
      delete p;
      return fail(GS_ERR_INVALID_ARG, "scene " + std::to_string(i) + ": group offsets must rise from 0 to N");
    }
    sp.desc.group_offsets = nullptr;
    sp.pose_base = pose_base;
    pose_base += d.n_groups;
    p->scenes.push_back(sp);
  }
  Layout L;
  for (int si = 0; si < desc->n_sensors; ++si) {
    const gs_sensor_desc& d = desc->sensors[si];
    SensorPlan s;
    memset(&s, 0, sizeof(s));
    s.desc = d;
    s.desc.elevations = nullptr;
    if (d.scene < 0 || d.scene >= desc->n_scenes || d.width <= 0 || d.height <= 0 || !(d.z_near > 0.0f)) {
      delete p;
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
        delete p;
        return fail(GS_ERR_INVALID_ARG, "sensor " + std::to_string(si) + ": focal lengths must be > 0");
      }
      K.tw = d.tile_w ? d.tile_w : 16;
      K.th = d.tile_h ? d.tile_h : 16;
      K.fx = d.fx;
      K.fy = d.fy;
      K.cx = d.cx;
      K.cy = d.cy;
    } else if (d.kind == GS_SENSOR_LIDAR) {
      if (!d.elevations) {
        delete p;
        return fail(GS_ERR_INVALID_ARG, "sensor " + std::to_string(si) + ": LiDAR needs elevations");
      }
      for (int j = 0; j + 1 < d.height; ++j)
        if (!(d.elevations[j] < d.elevations[j + 1])) {
          delete p;
          return fail(GS_ERR_INVALID_ARG, "sensor " + std::to_string(si) + ": elevations must ascend");
        }
      if (!sp.desc.has_intensity) {
        delete p;
        return fail(GS_ERR_INVALID_ARG, "sensor " + std::to_string(si) + ": LiDAR scene needs intensity");
      }
      K.tw = d.tile_w ? d.tile_w : 32;
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
        delete p;
        return fail(GS_ERR_HIP, std::string("LiDAR tables: ") + hipGetErrorString(e));
      }
      K.el = s.d_tabs;
      K.cos_el = s.d_tabs + d.height;
      K.sin_el = s.d_tabs + 2 * d.height;
      K.cos_az = s.d_tabs + 3 * d.height;
      K.sin_az = s.d_tabs + 3 * d.height + d.width;
    } else {
      delete p;
      return fail(GS_ERR_INVALID_ARG, "sensor " + std::to_string(si) + ": unknown kind");
    }
    if (!tile_shape_supported(K.tw, K.th)) {
      p->sensors.push_back(s);
      gs_plan_destroy(p);
      return fail(GS_ERR_UNSUPPORTED, "sensor " + std::to_string(si) + ": unsupported tile shape");
    }
    K.n_tx = (K.W + K.tw - 1) / K.tw;
    K.n_ty = (K.H + K.th - 1) / K.th;
    K.tile_offset = 0;
    s.n_tiles = K.n_tx * K.n_ty;
    s.tile_bits = ceil_log2(s.n_tiles);
    int64_t cap = desc->pair_capacity > 0 ? desc->pair_capacity : 16ll * N + 4096;
    if (cap > 0x7FFFFFFFll) cap = 0x7FFFFFFFll;
    s.cap = (uint32_t)cap;
    // workspace region
    Layout R;
    const size_t n = (size_t)N;
    const size_t HW = (size_t)K.W * K.H;
    s.o_status = R.take(16 * 4);
    s.o_pose = R.take(12 * 4 * (size_t)sp.desc.n_groups);
    s.o_rec = R.take(n * 64);
    s.o_rec64 = R.take(n * 8 * kRec64);
    s.o_grz = R.take(n * 8 * kGrz);
    s.o_rect = R.take(n * 16);
    s.o_ntiles = R.take(n * 4);
    s.o_visible = R.take(n * 4);
    s.o_key0 = R.take(n * 4);
    s.o_key1 = R.take(n * 4);
    s.o_val0 = R.take(n * 4);
    s.o_val1 = R.take(n * 4);
    s.o_offs = R.take((n + 1) * 4);
    s.o_bsum = R.take(scan_bsum_words(N) * 4);
    size_t hw = radix_hist_words(s.cap);
    size_t hw2 = radix_hist_words((uint32_t)N);
    s.o_hist = R.take((hw > hw2 ? hw : hw2) * 4);
    s.o_ptile0 = R.take((size_t)s.cap * 4);
    s.o_ptile1 = R.take((size_t)s.cap * 4);
    s.o_pval0 = R.take((size_t)s.cap * 4);
    s.o_pval1 = R.take((size_t)s.cap * 4);
    s.o_ranges = R.take((size_t)s.n_tiles * 8);
    s.o_Tfinal = R.take(HW * 4);
    s.o_nlast = R.take(HW * 4);
    s.o_gacc = R.take(n * 4 * kGradFields);
    s.base = L.take(R.off);
    s.pair_buf = (s.tile_bits + 7) / 8 % 2;
    p->sensors.push_back(s);
  }
  p->ws_bytes = L.off;
  *out = p;
  return ok();
}

void gs_plan_destroy(gs_plan* p) {
  if (!p) return;
  for (auto& s : p->sensors)
    if (s.d_tabs) hipFree(s.d_tabs);
  delete p;
}

gs_status gs_plan_workspace_size(const gs_plan* p, size_t* bytes) {
  if (!p || !bytes) return fail(GS_ERR_INVALID_ARG, "null plan or output");
  *bytes = p->ws_bytes;
  return ok();
}

gs_status gs_plan_inspect(const gs_plan* p, int32_t sensor, gs_workspace_view* out) {
  if (!p || !out || sensor < 0 || sensor >= (int)p->sensors.size()) return fail(GS_ERR_INVALID_ARG, "bad inspect args");
  const SensorPlan& s = p->sensors[sensor];
  out->pair_surfel = s.base + (s.pair_buf ? s.o_pval1 : s.o_pval0);
  out->pair_tile = s.base + (s.pair_buf ? s.o_ptile1 : s.o_ptile0);
  out->tile_ranges = s.base + s.o_ranges;
  out->visible = s.base + s.o_visible;
  out->pair_count = s.base + s.o_status + 4 * kStPairs;
  out->n_tiles = s.n_tiles;
  out->tile_offset = s.K.tile_offset;
  return ok();
}

gs_status gs_render_forward(gs_plan* p, const gs_scene* scenes, const float* sensor_poses, const float* group_poses,
                            float* const* outputs, void* workspace, hipStream_t st) {
  if (!p || !scenes || !sensor_poses || !group_poses || !outputs || !workspace)
    return fail(GS_ERR_INVALID_ARG, "null argument to gs_render_forward");
  if (reinterpret_cast<uintptr_t>(workspace) % 256 != 0) return fail(GS_ERR_INVALID_ARG, "workspace must be 256-B aligned");
  for (size_t si = 0; si < p->sensors.size(); ++si) {
    const SensorPlan& s = p->sensors[si];
    if (!outputs[si]) return fail(GS_ERR_INVALID_ARG, "null output for sensor " + std::to_string(si));
    gs_status cs = check_scene(p, s.scene, scenes[s.scene], s.K.kind == GS_SENSOR_PINHOLE, s.K.kind == GS_SENSOR_LIDAR);
    if (cs != GS_OK) return cs;
  }
  for (size_t si = 0; si < p->sensors.size(); ++si) {
    const SensorPlan& s = p->sensors[si];
    const ScenePlan& sp = p->scenes[s.scene];
    const int N = sp.desc.n_splats;
    SensorWS ws = ws_of(s, workspace);
    launch_fill_u32(ws.status, 0u, 16, st);
    launch_compose_poses(sensor_poses + 12 * si, group_poses, sp.pose_base, sp.desc.n_groups, ws.pose, st);
    PrepArgs a = prep_args(p, s, scenes[s.scene], ws);
    launch_prep(a, st);
    launch_count_visible(ws.visible, N, ws.status, st);
    int kb = radix_sort(ws.key, ws.val, nullptr, (uint32_t)N, (uint32_t)N, 32, ws.hist, st);
    launch_pair_offsets(ws.val[kb], ws.ntiles, N, ws.offs, ws.bsum, ws.status, s.cap, st);
    launch_emit(ws.val[kb], ws.ntiles, ws.rect, ws.offs, N, s.K, s.cap, ws.ptile[0], ws.pval[0], st);
    int pb = radix_sort(ws.ptile, ws.pval, ws.status + kStPairs, 0, s.cap, s.tile_bits, ws.hist, st);
    launch_ranges(ws.ptile[pb], ws.status + kStPairs, s.cap, ws.ranges, s.n_tiles, st);
    BlendArgs b;
    memset(&b, 0, sizeof(b));
    b.S = s.K;
    b.O = p->O;
    b.ws = ws;
    b.pval = ws.pval[pb];
    b.n_tiles = s.n_tiles;
    b.n_splats = N;
    b.out = outputs[si];
    launch_blend_forward(b, st);
  }
  GS_HIP_TRY(hipGetLastError());
  return ok();
}

gs_status gs_render_backward(gs_plan* p, const gs_scene* scenes, const float* sensor_poses, const float* group_poses,
                             const float* const* outputs, const float* const* grad_outputs, void* workspace,
                             const gs_scene_grads* grads, hipStream_t st) {
  (void)sensor_poses;
  (void)group_poses;
  if (!p || !scenes || !outputs || !grad_outputs || !workspace || !grads)
    return fail(GS_ERR_INVALID_ARG, "null argument to gs_render_backward");
  for (size_t si = 0; si < p->sensors.size(); ++si) {
    if (!outputs[si] || !grad_outputs[si]) return fail(GS_ERR_INVALID_ARG, "null output/grad for sensor " + std::to_string(si));
    const SensorPlan& s = p->sensors[si];
    gs_status cs = check_scene(p, s.scene, scenes[s.scene], s.K.kind == GS_SENSOR_PINHOLE, s.K.kind == GS_SENSOR_LIDAR);
    if (cs != GS_OK) return cs;
  }
  for (size_t si = 0; si < p->sensors.size(); ++si) {
    const SensorPlan& s = p->sensors[si];
    const ScenePlan& sp = p->scenes[s.scene];
    const int N = sp.desc.n_splats;
    SensorWS ws = ws_of(s, workspace);
    launch_fill_f32(ws.gacc, 0.0f, (size_t)N * kGradFields, st);
    BlendArgs b;
    memset(&b, 0, sizeof(b));
    b.S = s.K;
    b.O = p->O;
    b.ws = ws;
    b.pval = s.pair_buf ? ws.pval[1] : ws.pval[0];
    b.n_tiles = s.n_tiles;
    b.n_splats = N;
    b.out_fwd = outputs[si];
    b.gout = grad_outputs[si];
    launch_blend_backward(b, st);
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
    launch_splat_backward(sb, st);
  }
  GS_HIP_TRY(hipGetLastError());
  return ok();
}

gs_status gs_query_status(const gs_plan* p, const void* workspace, hipStream_t st, gs_run_status* out) {
  if (!p || !workspace || !out) return fail(GS_ERR_INVALID_ARG, "null argument to gs_query_status");
  GS_HIP_TRY(hipStreamSynchronize(st));
  memset(out, 0, sizeof(*out));
  bool over = false;
  for (size_t si = 0; si < p->sensors.size(); ++si) {
    const SensorPlan& s = p->sensors[si];
    uint32_t w[16];
    GS_HIP_TRY(hipMemcpy(w, static_cast<const char*>(workspace) + s.base + s.o_status, sizeof(w), hipMemcpyDeviceToHost));
    out->pairs[si] = w[kStPairs];
    out->n_visible[si] = (int32_t)w[kStVisible];
    out->fp64_pairs += w[kStFp64];
    over = over || w[kStOverflow] != 0;
  }
  out->overflow = over ? 1 : 0;
  if (over) return fail(GS_ERR_CAPACITY, "pair capacity exceeded; re-plan with a larger pair_capacity");
  return ok();
}

}  // extern "C"
