// Scene zones and the double-buffered swap-in of a zone's Gaussians (Sec.
// III-A, large-scale scenes: square ground-plane zones with a relative
// padding on each side; two buffers at render time, the next zone's
// Gaussians brought in while the current one is rendered).
//
// gs_zone_partition is host code: a two-pass count / fill over the anchors,
// split over host threads by anchor ranges so that each zone's list stays in
// ascending anchor order.
//
// gs_zone_stream: a swap-in thread per stream.  For an upload of zone z into
// buffer b it
//   1. waits for the previous copy out of b's pinned staging to finish,
//   2. gathers every field's rows at the zone's anchor list into the staging
//      (padding up to the buffer capacity with the field's fill value),
//   3. makes the copy stream wait for the last release of b (the renderer's
//      final reads of the old contents), and
//   4. enqueues one 2D copy per field and records b's upload event.
// acquire() makes the renderer's stream wait for that event, so a renderer
// never blocks on the host for more than the gather of a zone it has not yet
// prefetched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/gs2d.h"

namespace gs {
gs_status set_error(gs_status s, const std::string& msg);
}

using gs::set_error;

namespace {

constexpr int64_t kMaxZones = int64_t(1) << 20;
constexpr int64_t kMaxAnchors = int64_t(0xFFFFFFFFu);

bool grid_ok(const gs_zone_grid& g, std::string* why) {
  auto bad = [&](const char* m) {
    *why = m;
    return false;
  };
  for (int k = 0; k < 2; ++k)
    if (g.axis[k] < 0 || g.axis[k] > 2) return bad("zone grid axis must be 0, 1 or 2");
  if (g.axis[0] == g.axis[1]) return bad("zone grid axes must differ");
  if (!std::isfinite(g.origin[0]) || !std::isfinite(g.origin[1])) return bad("zone grid origin must be finite");
  if (!std::isfinite(g.size) || !(g.size > 0.0)) return bad("zone size must be finite and > 0");
  if (!std::isfinite(g.pad) || g.pad < 0.0 || g.pad > 1.0) return bad("zone padding must be in [0, 1]");
  if (g.nx < 1 || g.ny < 1 || (int64_t)g.nx * g.ny > kMaxZones) return bad("zone counts must be >= 1, nx*ny <= 2^20");
  return true;
}

// Zones [lo, hi] along one axis whose padded interval may hold coordinate a
// (a superset: every candidate is tested exactly by `inside`).
bool candidates(double a, double origin, double size, double pad, int n, int* lo, int* hi) {
  if (!std::isfinite(a)) return false;
  const double t = (a - origin) / size;
  if (!(t > -pad - 3.0) || !(t < (double)n + pad + 3.0)) return false;
  const double l = std::floor(t - 1.0 - pad) - 1.0, h = std::floor(t + pad) + 1.0;
  *lo = (int)std::max(l, 0.0);
  *hi = (int)std::min(h, (double)(n - 1));
  return *lo <= *hi;
}

inline bool inside(double a, double origin, double size, double pad, int i) {
  const double di = (double)i;
  const double lo = origin + (di - pad) * size;
  const double hi = origin + ((di + 1.0) + pad) * size;
  return lo <= a && a < hi;
}

// Calls f(zone) for every zone holding point p, in ascending zone id.
template <class F>
inline void for_zones(const gs_zone_grid& g, const float* xyz, int64_t n, int64_t p, F&& f) {
  const double a = (double)xyz[(size_t)g.axis[0] * n + p];
  const double b = (double)xyz[(size_t)g.axis[1] * n + p];
  int i0, i1, j0, j1;
  if (!candidates(a, g.origin[0], g.size, g.pad, g.nx, &i0, &i1)) return;
  if (!candidates(b, g.origin[1], g.size, g.pad, g.ny, &j0, &j1)) return;
  for (int j = j0; j <= j1; ++j) {
    if (!inside(b, g.origin[1], g.size, g.pad, j)) continue;
    for (int i = i0; i <= i1; ++i)
      if (inside(a, g.origin[0], g.size, g.pad, i)) f((int64_t)j * g.nx + i);
  }
}

int host_threads(int64_t work, int64_t per_thread, int cap) {
  const unsigned hc = std::max(1u, std::thread::hardware_concurrency());
  const int64_t t = std::min<int64_t>({(int64_t)hc, (int64_t)cap, work / per_thread + 1});
  return (int)std::max<int64_t>(t, 1);
}

// Runs f(t) for t in [0, T) on T threads (t = 0 on the calling thread).
template <class F>
void parallel(int T, F&& f) {
  std::vector<std::thread> th;
  th.reserve(T > 1 ? T - 1 : 0);
  for (int t = 1; t < T; ++t) th.emplace_back([&f, t] { f(t); });
  f(0);
  for (auto& x : th) x.join();
}

// ---------------------------------------------------------------------------
// swap-in stream
// ---------------------------------------------------------------------------

struct Field {
  gs_zone_field f;
  std::vector<unsigned char> fill;  // elem_bytes (per_zone = 0)
  size_t staging_off = 0;           // byte offset in a buffer's staging
  size_t staging_bytes = 0;         // rows * capacity * elem_bytes, or elem_bytes per zone
};

struct Request {
  int zone, buffer;
  uint64_t seq;
};

}  // namespace

struct gs_zone_stream {
  int device = 0;
  int n_zones = 0;
  std::vector<uint32_t> offs, index;
  int64_t capacity = 0;
  int threads = 1;
  std::vector<Field> fields;
  size_t staging_bytes = 0;
  unsigned char* staging[2] = {nullptr, nullptr};
  hipStream_t copy = nullptr;
  hipEvent_t uploaded[2] = {nullptr, nullptr};  // end of the last upload into the buffer
  hipEvent_t released[2] = {nullptr, nullptr};  // last reads of the buffer's contents
  hipEvent_t t0[2] = {nullptr, nullptr}, t1[2] = {nullptr, nullptr};  // timing of the last upload

  std::thread worker;
  std::mutex mu;
  std::condition_variable cv_req, cv_done;
  std::deque<Request> queue;
  bool stop = false;
  uint64_t requested[2] = {0, 0}, enqueued[2] = {0, 0}, acquired[2] = {0, 0};
  int zone_in[2] = {-1, -1};
  int64_t count_in[2] = {0, 0}, bytes_in[2] = {0, 0};
  double gather_ms[2] = {0.0, 0.0};
  bool hip_failed = false;
  std::string hip_msg;

  void gather(int zone, unsigned char* dst) const;
  bool upload(int buffer, const unsigned char* src, int zone, std::string* msg);
  void run();
};

namespace {

// Copies `n` elements of `e` bytes from src[idx[k]] to dst[k].
inline void gather_row(unsigned char* dst, const unsigned char* src, const uint32_t* idx, int64_t n, int e) {
  switch (e) {
    case 2: {
      auto* d = reinterpret_cast<uint16_t*>(dst);
      auto* s = reinterpret_cast<const uint16_t*>(src);
      for (int64_t k = 0; k < n; ++k) d[k] = s[idx[k]];
      break;
    }
    case 4: {
      auto* d = reinterpret_cast<uint32_t*>(dst);
      auto* s = reinterpret_cast<const uint32_t*>(src);
      for (int64_t k = 0; k < n; ++k) d[k] = s[idx[k]];
      break;
    }
    case 8: {
      auto* d = reinterpret_cast<uint64_t*>(dst);
      auto* s = reinterpret_cast<const uint64_t*>(src);
      for (int64_t k = 0; k < n; ++k) d[k] = s[idx[k]];
      break;
    }
    default:
      for (int64_t k = 0; k < n; ++k) std::memcpy(dst + (size_t)k * e, src + (size_t)idx[k] * e, e);
  }
}

inline void fill_row(unsigned char* dst, const unsigned char* v, int64_t n, int e) {
  bool zero = true;
  for (int i = 0; i < e; ++i) zero = zero && v[i] == 0;
  if (zero) {
    std::memset(dst, 0, (size_t)n * e);
    return;
  }
  for (int64_t k = 0; k < n; ++k) std::memcpy(dst + (size_t)k * e, v, e);
}

}  // namespace

void gs_zone_stream::gather(int zone, unsigned char* dst) const {
  const uint32_t* L = index.data() + offs[zone];
  const int64_t n = (int64_t)offs[zone + 1] - offs[zone];
  // every thread takes one range of k (the same anchors in every row)
  const int T = std::max(1, std::min<int>(threads, (int)(capacity / 4096) + 1));
  parallel(T, [&](int t) {
    const int64_t k0 = capacity * t / T, k1 = capacity * (t + 1) / T;
    for (const Field& F : fields) {
      const int e = F.f.elem_bytes;
      if (F.f.per_zone) {
        if (t == 0)
          std::memcpy(dst + F.staging_off, static_cast<const unsigned char*>(F.f.host) + (size_t)zone * e, e);
        continue;
      }
      const auto* host = static_cast<const unsigned char*>(F.f.host);
      const int64_t g0 = std::min(k0, n), g1 = std::min(k1, n);
      for (int r = 0; r < F.f.rows; ++r) {
        unsigned char* row = dst + F.staging_off + ((size_t)r * capacity) * e;
        const unsigned char* src = host + ((size_t)r * F.f.host_stride) * e;
        if (g1 > g0) gather_row(row + (size_t)g0 * e, src, L + g0, g1 - g0, e);
        const int64_t f0 = std::max(k0, n);
        if (k1 > f0) fill_row(row + (size_t)f0 * e, F.fill.data(), k1 - f0, e);
      }
    }
  });
}

bool gs_zone_stream::upload(int b, const unsigned char* src, int zone, std::string* msg) {
  auto ck = [&](hipError_t e, const char* what) {
    if (e != hipSuccess) *msg = std::string(what) + ": " + hipGetErrorString(e);
    return e == hipSuccess;
  };
  if (!ck(hipStreamWaitEvent(copy, released[b], 0), "hipStreamWaitEvent")) return false;
  if (!ck(hipEventRecord(t0[b], copy), "hipEventRecord")) return false;
  int64_t bytes = 0;
  for (const Field& F : fields) {
    const size_t e = (size_t)F.f.elem_bytes;
    if (F.f.per_zone) {
      if (!ck(hipMemcpyAsync(F.f.device[b], src + F.staging_off, e, hipMemcpyHostToDevice, copy), "hipMemcpyAsync"))
        return false;
      bytes += (int64_t)e;
      continue;
    }
    const size_t w = (size_t)capacity * e;
    if (!ck(hipMemcpy2DAsync(F.f.device[b], (size_t)F.f.device_stride * e, src + F.staging_off, w, w,
                             (size_t)F.f.rows, hipMemcpyHostToDevice, copy),
            "hipMemcpy2DAsync"))
      return false;
    bytes += (int64_t)(w * F.f.rows);
  }
  if (!ck(hipEventRecord(t1[b], copy), "hipEventRecord")) return false;
  if (!ck(hipEventRecord(uploaded[b], copy), "hipEventRecord")) return false;
  bytes_in[b] = bytes;
  (void)zone;
  return true;
}

void gs_zone_stream::run() {
  const bool dev_ok = hipSetDevice(device) == hipSuccess;
  for (;;) {
    Request r;
    {
      std::unique_lock<std::mutex> lk(mu);
      cv_req.wait(lk, [&] { return stop || !queue.empty(); });
      if (queue.empty()) return;  // stop with nothing left
      r = queue.front();
      queue.pop_front();
    }
    std::string msg;
    bool ok = dev_ok;
    if (!dev_ok) msg = "hipSetDevice failed in the swap-in thread";
    double ms = 0.0;
    if (ok) {
      // the previous copy out of this staging buffer must be done before it is overwritten
      hipError_t e = hipEventSynchronize(uploaded[r.buffer]);
      if (e != hipSuccess) {
        ok = false;
        msg = std::string("hipEventSynchronize: ") + hipGetErrorString(e);
      }
    }
    if (ok) {
      const auto c0 = std::chrono::steady_clock::now();
      gather(r.zone, staging[r.buffer]);
      ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - c0).count();
      ok = upload(r.buffer, staging[r.buffer], r.zone, &msg);
    }
    {
      std::lock_guard<std::mutex> lk(mu);
      if (!ok && !hip_failed) {
        hip_failed = true;
        hip_msg = msg;
      }
      enqueued[r.buffer] = r.seq;
      zone_in[r.buffer] = r.zone;
      count_in[r.buffer] = (int64_t)offs[r.zone + 1] - offs[r.zone];
      gather_ms[r.buffer] = ms;
    }
    cv_done.notify_all();
  }
}

namespace {

void destroy_stream(gs_zone_stream* zs) {
  if (!zs) return;
  if (zs->worker.joinable()) {
    {
      std::lock_guard<std::mutex> lk(zs->mu);
      zs->stop = true;
    }
    zs->cv_req.notify_all();
    zs->worker.join();
  }
  if (zs->copy) (void)hipStreamSynchronize(zs->copy);
  for (int b = 0; b < 2; ++b) {
    if (zs->staging[b]) (void)hipHostFree(zs->staging[b]);
    for (hipEvent_t ev : {zs->uploaded[b], zs->released[b], zs->t0[b], zs->t1[b]})
      if (ev) (void)hipEventDestroy(ev);
  }
  if (zs->copy) (void)hipStreamDestroy(zs->copy);
  delete zs;
}

}  // namespace

extern "C" {

gs_status gs_zone_partition(const gs_zone_grid* grid, const float* xyz, int64_t n, uint32_t* zone_offsets,
                            uint32_t* index, int64_t cap, int64_t* total) {
  if (!grid || !zone_offsets || !total) return set_error(GS_ERR_INVALID_ARG, "null zone grid, offsets or total");
  std::string why;
  if (!grid_ok(*grid, &why)) return set_error(GS_ERR_INVALID_ARG, why);
  if (n < 0 || n > kMaxAnchors) return set_error(GS_ERR_INVALID_ARG, "anchor count must be in [0, 2^32 - 1]");
  if (n > 0 && !xyz) return set_error(GS_ERR_INVALID_ARG, "null xyz");
  if (cap < 0 || (cap > 0 && !index)) return set_error(GS_ERR_INVALID_ARG, "bad index capacity");
  const gs_zone_grid g = *grid;
  const int64_t Z = (int64_t)g.nx * g.ny;
  // per-thread tables are T x Z words: keep them under 2^24 entries
  const int T = host_threads(n, 1 << 16, (int)std::max<int64_t>(1, std::min<int64_t>(32, (int64_t(1) << 24) / Z)));
  // pass 1: per-thread counts over contiguous anchor ranges
  std::vector<std::vector<uint32_t>> cnt(T, std::vector<uint32_t>(Z, 0));
  parallel(T, [&](int t) {
    const int64_t p0 = n * t / T, p1 = n * (t + 1) / T;
    auto& c = cnt[t];
    for (int64_t p = p0; p < p1; ++p) for_zones(g, xyz, n, p, [&](int64_t z) { ++c[z]; });
  });
  // offsets: zone-major, thread order inside a zone (keeps anchors ascending)
  std::vector<std::vector<uint64_t>> start(T, std::vector<uint64_t>(Z, 0));
  uint64_t run = 0;
  for (int64_t z = 0; z < Z; ++z) {
    if (run > 0xFFFFFFFFull) break;
    zone_offsets[z] = (uint32_t)run;
    for (int t = 0; t < T; ++t) {
      start[t][z] = run;
      run += cnt[t][z];
    }
  }
  *total = (int64_t)run;
  if (run > 0xFFFFFFFFull) return set_error(GS_ERR_CAPACITY, "more than 2^32 - 1 zone memberships");
  zone_offsets[Z] = (uint32_t)run;
  if ((int64_t)run > cap) {
    if (index == nullptr && cap == 0) return set_error(GS_OK, "");
    return set_error(GS_ERR_CAPACITY, "zone index capacity " + std::to_string(cap) + " below the " +
                                          std::to_string(run) + " memberships");
  }
  // pass 2: fill
  parallel(T, [&](int t) {
    const int64_t p0 = n * t / T, p1 = n * (t + 1) / T;
    auto& s = start[t];
    for (int64_t p = p0; p < p1; ++p) for_zones(g, xyz, n, p, [&](int64_t z) { index[s[z]++] = (uint32_t)p; });
  });
  return set_error(GS_OK, "");
}

gs_status gs_zone_stream_create(const gs_zone_stream_desc* d, gs_zone_stream** out) {
  if (!d || !out) return set_error(GS_ERR_INVALID_ARG, "null zone stream descriptor or output");
  *out = nullptr;
  if (d->n_zones < 1 || d->n_zones > kMaxZones || !d->zone_offsets)
    return set_error(GS_ERR_INVALID_ARG, "zone stream needs 1..2^20 zones and their offsets");
  if (d->capacity < 1 || d->capacity > kMaxAnchors) return set_error(GS_ERR_INVALID_ARG, "bad zone buffer capacity");
  if (d->n_anchors < 0 || d->n_anchors > kMaxAnchors) return set_error(GS_ERR_INVALID_ARG, "bad anchor count");
  if (d->n_fields < 1 || d->n_fields > 64 || !d->fields) return set_error(GS_ERR_INVALID_ARG, "zone stream needs 1..64 fields");
  if (d->threads < 1 || d->threads > 64) return set_error(GS_ERR_INVALID_ARG, "zone stream threads must be 1..64");
  const uint32_t* o = d->zone_offsets;
  if (o[0] != 0) return set_error(GS_ERR_INVALID_ARG, "zone offsets must start at 0");
  for (int z = 0; z < d->n_zones; ++z) {
    if (o[z + 1] < o[z]) return set_error(GS_ERR_INVALID_ARG, "zone offsets must be non-decreasing");
    if ((int64_t)(o[z + 1] - o[z]) > d->capacity)
      return set_error(GS_ERR_INVALID_ARG, "zone " + std::to_string(z) + " holds " + std::to_string(o[z + 1] - o[z]) +
                                               " anchors, above the buffer capacity " + std::to_string(d->capacity));
  }
  const uint32_t m = o[d->n_zones];
  if (m > 0 && !d->index) return set_error(GS_ERR_INVALID_ARG, "null zone index");
  for (uint32_t k = 0; k < m; ++k)
    if ((int64_t)d->index[k] >= d->n_anchors) return set_error(GS_ERR_INVALID_ARG, "zone index beyond the anchors");

  auto* zs = new gs_zone_stream();
  zs->n_zones = d->n_zones;
  zs->offs.assign(o, o + d->n_zones + 1);
  zs->index.assign(d->index, d->index + m);
  zs->capacity = d->capacity;
  zs->threads = d->threads;
  size_t off = 0;
  for (int i = 0; i < d->n_fields; ++i) {
    const gs_zone_field& f = d->fields[i];
    std::string bad;
    if (!f.host || !f.device[0] || !f.device[1]) bad = "null field pointer";
    else if (f.elem_bytes < 1 || f.elem_bytes > 65536) bad = "field element size must be 1..65536 bytes";
    else if (f.per_zone != 0 && f.per_zone != 1) bad = "field per_zone must be 0 or 1";
    else if (f.per_zone && f.rows != 1) bad = "a per-zone field has one row";
    else if (!f.per_zone && (f.rows < 1 || f.host_stride < d->n_anchors || f.device_stride < d->capacity))
      bad = "anchor field needs rows >= 1, host_stride >= n_anchors and device_stride >= capacity";
    if (!bad.empty()) {
      destroy_stream(zs);
      return set_error(GS_ERR_INVALID_ARG, "field " + std::to_string(i) + ": " + bad);
    }
    Field F;
    F.f = f;
    if (!f.per_zone) {
      F.fill.assign((size_t)f.elem_bytes, 0);
      if (f.fill) std::memcpy(F.fill.data(), f.fill, (size_t)f.elem_bytes);
      F.staging_bytes = (size_t)f.rows * (size_t)d->capacity * (size_t)f.elem_bytes;
    } else {
      F.staging_bytes = (size_t)f.elem_bytes;
    }
    F.staging_off = off;
    off += (F.staging_bytes + 255) & ~size_t(255);
    zs->fields.push_back(std::move(F));
  }
  zs->staging_bytes = off;

  auto hip_fail = [&](hipError_t e, const char* what) {
    destroy_stream(zs);
    return set_error(GS_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
  };
  hipError_t e = hipGetDevice(&zs->device);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  for (int b = 0; b < 2; ++b) {
    e = hipHostMalloc(reinterpret_cast<void**>(&zs->staging[b]), zs->staging_bytes, hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "hipHostMalloc");
  }
  e = hipStreamCreateWithFlags(&zs->copy, hipStreamNonBlocking);
  if (e != hipSuccess) return hip_fail(e, "hipStreamCreateWithFlags");
  for (int b = 0; b < 2; ++b) {
    for (hipEvent_t* ev : {&zs->uploaded[b], &zs->released[b]}) {
      e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreateWithFlags");
      e = hipEventRecord(*ev, zs->copy);  // recorded once, so that every wait has a record to wait for
      if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
    }
    for (hipEvent_t* ev : {&zs->t0[b], &zs->t1[b]}) {
      e = hipEventCreate(ev);
      if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
  }
  e = hipStreamSynchronize(zs->copy);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  zs->worker = std::thread([zs] { zs->run(); });
  *out = zs;
  return set_error(GS_OK, "");
}

gs_status gs_zone_stream_prefetch(gs_zone_stream* zs, int32_t zone, int32_t buffer) {
  if (!zs) return set_error(GS_ERR_INVALID_ARG, "null zone stream");
  if (buffer < 0 || buffer > 1) return set_error(GS_ERR_INVALID_ARG, "buffer must be 0 or 1");
  if (zone < 0 || zone >= zs->n_zones) return set_error(GS_ERR_INVALID_ARG, "zone out of range");
  {
    std::lock_guard<std::mutex> lk(zs->mu);
    if (zs->hip_failed) return set_error(GS_ERR_HIP, "swap-in thread: " + zs->hip_msg);
    zs->queue.push_back({zone, buffer, ++zs->requested[buffer]});
  }
  zs->cv_req.notify_one();
  return set_error(GS_OK, "");
}

gs_status gs_zone_stream_acquire(gs_zone_stream* zs, int32_t buffer, hipStream_t stream, int32_t* zone,
                                 int64_t* count) {
  if (!zs) return set_error(GS_ERR_INVALID_ARG, "null zone stream");
  if (buffer < 0 || buffer > 1) return set_error(GS_ERR_INVALID_ARG, "buffer must be 0 or 1");
  int z;
  int64_t c;
  {
    std::unique_lock<std::mutex> lk(zs->mu);
    if (zs->requested[buffer] == 0) return set_error(GS_ERR_INVALID_ARG, "nothing was queued into this buffer");
    zs->cv_done.wait(lk, [&] { return zs->enqueued[buffer] == zs->requested[buffer]; });
    if (zs->hip_failed) return set_error(GS_ERR_HIP, "swap-in thread: " + zs->hip_msg);
    z = zs->zone_in[buffer];
    c = zs->count_in[buffer];
    zs->acquired[buffer] = zs->requested[buffer];
  }
  hipError_t e = hipStreamWaitEvent(stream, zs->uploaded[buffer], 0);
  if (e != hipSuccess) return set_error(GS_ERR_HIP, std::string("hipStreamWaitEvent: ") + hipGetErrorString(e));
  if (zone) *zone = z;
  if (count) *count = c;
  return set_error(GS_OK, "");
}

gs_status gs_zone_stream_release(gs_zone_stream* zs, int32_t buffer, hipStream_t stream) {
  if (!zs) return set_error(GS_ERR_INVALID_ARG, "null zone stream");
  if (buffer < 0 || buffer > 1) return set_error(GS_ERR_INVALID_ARG, "buffer must be 0 or 1");
  // An upload waits for the release recorded last before the swap-in thread
  // enqueues it; a release between queueing an upload and acquiring it could
  // thus order that upload after work which waits for a later upload (a
  // cycle), and is refused.
  std::lock_guard<std::mutex> lk(zs->mu);
  if (zs->acquired[buffer] != zs->requested[buffer])
    return set_error(GS_ERR_INVALID_ARG, "an upload into this buffer was queued since its last acquire");
  hipError_t e = hipEventRecord(zs->released[buffer], stream);
  if (e != hipSuccess) return set_error(GS_ERR_HIP, std::string("hipEventRecord: ") + hipGetErrorString(e));
  return set_error(GS_OK, "");
}

gs_status gs_zone_stream_stats(gs_zone_stream* zs, int32_t buffer, gs_zone_swap_stats* out) {
  if (!zs || !out) return set_error(GS_ERR_INVALID_ARG, "null zone stream or output");
  if (buffer < 0 || buffer > 1) return set_error(GS_ERR_INVALID_ARG, "buffer must be 0 or 1");
  {
    std::unique_lock<std::mutex> lk(zs->mu);
    zs->cv_done.wait(lk, [&] { return zs->enqueued[buffer] == zs->requested[buffer]; });
    if (zs->hip_failed) return set_error(GS_ERR_HIP, "swap-in thread: " + zs->hip_msg);
    out->zone = zs->zone_in[buffer];
    out->count = zs->count_in[buffer];
    out->bytes = zs->bytes_in[buffer];
    out->gather_ms = zs->gather_ms[buffer];
  }
  out->upload_ms = 0.0;
  if (out->zone >= 0) {
    hipError_t e = hipEventSynchronize(zs->t1[buffer]);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, zs->t0[buffer], zs->t1[buffer]);
    if (e != hipSuccess) return set_error(GS_ERR_HIP, std::string("zone upload timing: ") + hipGetErrorString(e));
    out->upload_ms = ms;
  }
  return set_error(GS_OK, "");
}

void gs_zone_stream_destroy(gs_zone_stream* zs) { destroy_stream(zs); }

}  // extern "C"
