/*
 * gs2d.h -- C-ABI of the MI355X 2D-Gaussian-surfel sensor renderer.
 *
 * The library renders 2D Gaussian surfels (2DGS) for pinhole cameras and
 * spinning LiDARs and computes the adjoint of that rendering, following the
 * unified projection scheme of Sec. III-A of "Industrial-Grade Sensor
 * Simulation via Gaussian Splatting" (arXiv 2503.11731):
 *
 *   - a surfel is the tangent-plane map P(u,v) = W H (u,v,1)^T of Eq. 1,
 *     H = [s_u t_u, s_v t_v, mu; 0 0 1];
 *   - a ray is the intersection of two planes h_u, h_v and meets the surfel
 *     where [h_u, h_v]^T P(u,v) = 0 (Eq. 2);
 *   - pinhole planes follow Eq. 3, LiDAR planes Eq. 5;
 *   - the surfels a ray meets are alpha-composited front to back (the
 *     splatting of Sec. II), with the 2DGS low-pass filter.
 *
 * Problem statement (the boundary): render(surfels, sensor models, poses) ->
 * image or range buffers, and its adjoint.  The neural-Gaussian decode of
 * Sec. III-A (anchor feature -> MLP -> surfel attributes) is a separate pair
 * of calls that writes/reads the same surfel layout.
 *
 * Conventions shared by every call
 *   - All array arguments named "device" are HIP device pointers; everything
 *     else is host memory that the call reads before it returns.
 *   - Layout is structure-of-arrays, FP32, plane-major: an attribute with C
 *     components over N surfels is C planes of N floats ([C][N]).
 *   - Image outputs are planar FP32 [C][H][W] (row y, column x).  For a LiDAR,
 *     W = azimuth steps (column i has azimuth 2*pi*i/W, counter-clockwise
 *     about the sensor's +z, x forward, y left) and H = beams (row j is
 *     elevations[j], ascending).
 *   - Poses are row-major 3x4 FP32 rigid transforms: sensor poses map world
 *     to sensor, group poses map a surfel group's own frame to world.
 *     Camera frame: x right, y down, z forward.
 *   - The caller owns every buffer (inputs, outputs, workspace, gradients),
 *     allocated on the plan's device.  Calls enqueue work on the given stream
 *     and never synchronise it, except gs_query_status.  No call allocates
 *     device memory after gs_plan_create.
 *   - Errors: every call returns gs_status; nothing throws or aborts across
 *     the ABI.  Argument errors are detected on the host before any launch
 *     (GS_ERR_INVALID_ARG).  Data-dependent overflow of the (tile, surfel)
 *     pair capacity is detected on the device, recorded in the workspace's
 *     status words and reported by gs_query_status (GS_ERR_CAPACITY); the
 *     outputs of such a run are undefined but no memory outside the given
 *     buffers is touched.  gs_last_error() returns a message for the calling
 *     thread's last failure.
 *   - A plan is not re-entrant: calls that share a plan and a workspace must
 *     be ordered on one stream.
 */
#ifndef GS2D_H
#define GS2D_H

#include <stddef.h>
#include <stdint.h>

#ifndef __HIP_INCLUDE_HIP_HIP_RUNTIME_API_H__
/* Same declaration as the HIP runtime's, so this header needs no HIP include. */
typedef struct ihipStream_t* hipStream_t;
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum gs_status {
  GS_OK = 0,
  GS_ERR_INVALID_ARG = 1,   /* bad argument, detected before any launch        */
  GS_ERR_CAPACITY = 2,      /* pair capacity exceeded (device-detected)         */
  GS_ERR_HIP = 3,           /* a HIP runtime call failed                        */
  GS_ERR_UNSUPPORTED = 4    /* valid but unsupported combination of options     */
} gs_status;

/* Sensor kinds: pinhole camera (Eq. 3), spinning LiDAR (Eq. 5) and
 * cylindrical (fisheye) camera (Eq. 4: column i looks at the angle
 * phi = (i + 1/2 - cx) / fx about the camera's y axis, row j at height
 * y_n = (j + 1/2 - cy) / fy on the unit cylinder, ray (sin phi, y_n, cos phi);
 * its depth channel is the distance from the camera's vertical axis). */
enum gs_sensor_kind { GS_SENSOR_PINHOLE = 0, GS_SENSOR_LIDAR = 1, GS_SENSOR_CYLINDRICAL = 2 };

/* Maximum number of surfel groups (static scene + posed objects) per scene. */
#define GS_MAX_GROUPS 64
/* Maximum number of sensors per plan. */
#define GS_MAX_SENSORS 16

/* Sensor model (Eq. 3 pinhole, Eq. 5 spinning LiDAR). */
typedef struct gs_sensor_desc {
  int32_t kind;              /* gs_sensor_kind                                     */
  int32_t width, height;     /* cameras: pixels; LiDAR: azimuth steps x beams        */
  float fx, fy, cx, cy;      /* camera intrinsics; pixel (i,j) centre = (i+.5,j+.5);
                                cylindrical: fx in pixels per radian              */
  const double* elevations;  /* LiDAR: host array of `height` ascending angles (rad) */
  float z_near;              /* camera: min depth (cylindrical: min distance from the
                                vertical axis); LiDAR: min range                  */
  int32_t scene;             /* index of the scene this sensor renders              */
  int32_t tile_w, tile_h;    /* screen tile; 0 = default: 32x8, except 16x8 for a
                                LiDAR sensor of a per-sensor (not batched) plan */
} gs_sensor_desc;

/* Compositing rules (front-to-back alpha blending with the 2DGS low-pass
 * filter): alpha = min(alpha_max, o * exp(-rho_hat / 2)) with
 * rho_hat = min(u^2 + v^2, rho_lp) when `lowpass` is set; a ray-surfel pair
 * contributes iff rho_hat <= cutoff2, its depth (range) > z_near and
 * alpha >= alpha_min; a ray stops before the surfel that would take its
 * transmittance T (1 - alpha) below T_min.  rho_lp is lp_inv_sigma2 times
 * the squared distance to the projected centre in pixels (camera) or the
 * squared chord to the centre direction in azimuth steps (LiDAR).  A pair's
 * depth is that of the ray's hit point on the surfel plane when u^2 + v^2 is
 * used, and that of the surfel centre (camera mu_z, LiDAR |mu|) when rho_lp
 * is smaller (the filter's degenerate, edge-on case). */
typedef struct gs_render_opts {
  float alpha_min;       /* e.g. 1/255; 0 disables the skip test          */
  float alpha_max;       /* e.g. 0.99                                     */
  float T_min;           /* e.g. 1e-4; 0 disables early stopping          */
  float cutoff2;         /* squared support radius in sigma, e.g. 2 ln 255 */
  float lp_inv_sigma2;   /* low-pass 1/sigma^2, e.g. 2 (sigma = sqrt(2)/2)  */
  int32_t lowpass;       /* 1: apply the low-pass filter                  */
  float bg[3];           /* camera background colour added as T_final*bg  */
} gs_render_opts;

/* Static shape of one scene. */
typedef struct gs_scene_desc {
  int32_t n_splats;             /* N >= 0                                      */
  int32_t sh_degree;            /* 0..3: colour from SH; -1: plain RGB         */
  int32_t has_intensity;        /* 1 if a LiDAR renders this scene             */
  int32_t n_groups;             /* 1..GS_MAX_GROUPS                            */
  const int32_t* group_offsets; /* host, n_groups+1 non-decreasing, [0]=0, [G]=N */
} gs_scene_desc;

/* Per-call surfel data (device pointers, FP32 SoA).  Unused channels may be NULL. */
typedef struct gs_scene {
  const float* mean;       /* [3][N] centre mu, in the group's frame              */
  const float* quat;       /* [4][N] rotation (w,x,y,z), any non-zero norm        */
  const float* scale;      /* [2][N] s_u, s_v > 0 (metres)                         */
  const float* opacity;    /* [N] in (0,1]                                         */
  const float* rgb;        /* [3][N] when sh_degree < 0                            */
  const float* sh;         /* [(deg+1)^2*3][N], row k*3+channel, when sh_degree>=0 */
  const float* intensity;  /* [N] when has_intensity                              */
  const float* drop;       /* [N] LiDAR ray-drop probability in [0,1] (Sec. III-A's
                              attribute rho, read as the probability that a beam
                              meeting the surfel returns nothing); NULL = 0     */
} gs_scene;

/* Gradient buffers (device pointers), same layouts as gs_scene.  The adjoint
 * ACCUMULATES into them (+=); the caller zeroes them.  NULL entries skip. */
typedef struct gs_scene_grads {
  float* mean;
  float* quat;
  float* scale;
  float* opacity;
  float* rgb;
  float* sh;
  float* intensity;
  float* drop;
} gs_scene_grads;

typedef struct gs_plan_desc {
  int32_t n_scenes;              /* 1..GS_MAX_SENSORS (e.g. one decoded scene
                                    per sensor, or camera + LiDAR scenes)      */
  const gs_scene_desc* scenes;   /* host array [n_scenes]                      */
  int32_t n_sensors;             /* 1..GS_MAX_SENSORS                          */
  const gs_sensor_desc* sensors; /* host array [n_sensors]                     */
  gs_render_opts opts;
  int64_t pair_capacity;         /* (tile, surfel) pairs per sensor; 0 = 16*N+4096;
                                    clamped to 2^30 - 1 (sort key limit)     */
  int32_t batched;               /* 1: all sensors of the plan form one step:
                                    one record space, one depth sort, one pair
                                    list over a global tile space and one
                                    persistent compositing launch for all of
                                    them; every tile shape must then hold 256
                                    rays                                       */
  int32_t segment_pairs;         /* compositing work-item size L: a tile whose
                                    depth-ordered list holds more than L pairs
                                    is composited as ceil(len/L) segments in
                                    parallel and merged front to back (same
                                    results up to FP32 rounding order).
                                    0 = default (1024), < 0 = never split,
                                    else 32..32768                             */
} gs_plan_desc;

typedef struct gs_plan gs_plan; /* opaque, owned by the library */

/* Output channel counts: camera (pinhole or cylindrical) [9][H][W] = rgb(3),
 * depth, normal(3), alpha, median depth;
 * LiDAR [6][H][W] = range, intensity, alpha, ray-drop probability, drop
 * mask, median range.  Depth/range and normal are unnormalised sums (divide
 * by alpha for the expected value).  The median depth (range) is the depth
 * of the first composited surfel after which the transmittance is below 1/2
 * (the 2DGS median), 0 where it never falls that low.  The drop probability
 * is P = sum_i w_i rho_i + T_final (a beam that meets nothing returns
 * nothing) and the mask is 1 where P > 1/2, else 0.  The adjoint takes
 * gradients of every channel but the mask; the median's goes to the depth
 * of its surfel. */
#define GS_CAMERA_CHANNELS 9
#define GS_LIDAR_CHANNELS 6

/* Status of the last run on a workspace (filled by gs_query_status). */
typedef struct gs_run_status {
  int64_t pairs[GS_MAX_SENSORS];  /* (tile, surfel) pairs emitted per sensor */
  int32_t overflow;               /* 1 if any sensor exceeded pair_capacity  */
  int32_t n_visible[GS_MAX_SENSORS];
  int64_t fp64_pairs;             /* pairs re-solved in FP64 (grazing rays)  */
  int64_t evaluated;              /* (with gs_plan_set_counters) ray-surfel pairs the
                                     forward evaluates: per ray,
                                     the pairs of its tile list whose pixel
                                     rectangle holds the ray, up to its stop,
                                     except pairs proven to have no valid hit
                                     (cutoff and alpha >= alpha_min) on any pixel
                                     centre of the ray's 8x8 block             */
  int64_t composited;             /* (with gs_plan_set_counters) ray-surfel pairs
                                     that contributed                              */
  int64_t work_items;             /* compositing work items (tiles + extra segments) */
  int64_t segments;               /* segments of split tiles                       */
  int64_t graph_replays;          /* forward calls of this plan that replayed a
                                     captured graph (host count, since creation) */
  int64_t step_launches;          /* gs_plan_launch calls of this plan (host count) */
  int64_t wave_pairs;             /* (with gs_plan_set_counters) forward pair-loop
                                     iterations of all wavefronts:
                                     each evaluates one pair for the wave's 64 rays,
                                     so evaluated / (64 wave_pairs) is the lane
                                     utilisation of the compositing kernel     */
} gs_run_status;

/* Pipeline stages, for per-stage timing. */
enum gs_stage {
  GS_STAGE_PREPROCESS = 0, /* pose composition, projection, binning, records */
  GS_STAGE_DEPTH_SORT,     /* radix sort of surfels by depth key             */
  GS_STAGE_EMIT,           /* tile-count scan and pair emission              */
  GS_STAGE_TILE_SORT,      /* stable radix sort of pairs by tile             */
  GS_STAGE_RANGES,         /* per-tile ranges and compositing work items     */
  GS_STAGE_BLEND,          /* forward compositing (one persistent launch per
                              record space)                                  */
  GS_STAGE_BLEND_BWD,      /* adjoint compositing                            */
  GS_STAGE_SPLAT_BWD,      /* per-surfel adjoint                             */
  GS_N_STAGES
};

typedef struct gs_stage_times {
  int32_t records;                  /* stage intervals summed              */
  int32_t launches[GS_N_STAGES];    /* intervals per stage                 */
  double ms[GS_N_STAGES];           /* summed elapsed milliseconds         */
} gs_stage_times;

/* Enables (max_records > 0) or disables (0) HIP-event timing of every stage
 * of subsequent forward/backward calls, keeping up to max_records stage
 * intervals.  Creates the events now; the render calls then only record. */
gs_status gs_plan_set_timing(gs_plan* plan, int32_t max_records);
/* Synchronises `stream` and sums the recorded intervals per stage; clears
 * them when `reset` is non-zero. */
gs_status gs_plan_stage_times(gs_plan* plan, hipStream_t stream, int32_t reset, gs_stage_times* out);

/* Enables (on != 0) or disables (0, the default) the pair counters of later
 * forward calls: evaluated and composited ray-surfel pairs and wavefront
 * pair-loop iterations (gs_run_status).  Counting costs the compositing loop
 * scalar work, so it is meant for calibration runs; FP64 re-solves are always
 * counted. */
gs_status gs_plan_set_counters(gs_plan* plan, int32_t on);

/* Library version string and status text. */
const char* gs_version(void);
const char* gs_status_string(gs_status s);
/* Copies the calling thread's last error message into buf (always
 * NUL-terminated when n > 0) and returns the last status. */
gs_status gs_last_error(char* buf, size_t n);

/* Creates a plan on the current HIP device: validates the descriptor,
 * uploads sensor tables and fixes the workspace layout.  Host-only
 * descriptor memory may be freed after the call.  *out receives the plan. */
gs_status gs_plan_create(const gs_plan_desc* desc, gs_plan** out);
void gs_plan_destroy(gs_plan* plan);

/* Bytes of device workspace a forward+backward pair needs (256-B aligned
 * base required).  The forward leaves in it the state the backward reads
 * (per-surfel records, sorted pair lists, tile ranges, final transmittance),
 * so one workspace must be passed unchanged from a forward to its backward. */
gs_status gs_plan_workspace_size(const gs_plan* plan, size_t* bytes);

/* Forward render of every sensor of the plan.
 *   scenes        host array [n_scenes] of device surfel data
 *   sensor_poses  device [n_sensors][12] world->sensor
 *   group_poses   device [sum of n_groups over scenes][12] group->world,
 *                 scene 0's groups first
 *   outputs       host array [n_sensors] of device output planes (see above)
 *   workspace     device, gs_plan_workspace_size bytes
 * Integer work (visibility, tile lists, depth order) follows a fixed FP32
 * specification; per-ray compositing is FP32 with an FP64 re-solve of
 * near-degenerate (grazing) ray-surfel intersections. */
gs_status gs_render_forward(gs_plan* plan, const gs_scene* scenes, const float* sensor_poses,
                            const float* group_poses, float* const* outputs, void* workspace,
                            hipStream_t stream);

/* Adjoint of gs_render_forward: given the forward's outputs and dL/d(outputs)
 * (same layout), accumulates dL/d(surfel attributes) into `grads` (host array
 * [n_scenes]).  Uses the forward's workspace state; transmittance is
 * recomputed front to back rather than stored per pixel list. */
gs_status gs_render_backward(gs_plan* plan, const gs_scene* scenes, const float* sensor_poses,
                             const float* group_poses, const float* const* outputs,
                             const float* const* grad_outputs, void* workspace,
                             const gs_scene_grads* grads, hipStream_t stream);

/* Captures the forward of this plan with these exact arguments into a HIP
 * graph on `stream` (which must not be the legacy default stream).  Later
 * gs_render_forward calls with identical pointers and stream replay the
 * graph (one graph launch per step); other calls run uncaptured.  Stage
 * timing is not recorded inside the graph. */
gs_status gs_plan_capture(gs_plan* plan, const gs_scene* scenes, const float* sensor_poses,
                          const float* group_poses, float* const* outputs, void* workspace,
                          hipStream_t stream);

/* Step capture: everything enqueued on `stream` by the calling thread between
 * gs_plan_begin_capture and gs_plan_end_capture -- this plan's forward and
 * backward, decode calls, and the caller's own kernels on that stream (a
 * loss gradient, gradient clears) -- becomes one HIP graph held by the plan,
 * and gs_plan_launch replays it as one graph launch: a whole simulation or
 * training step (decode, batched render, loss, adjoint render, adjoint decode)
 * for the pointers used while capturing.  Inside the capture the calls only
 * enqueue (no stage timing, no forward-graph replay); the caller must not
 * allocate device memory or synchronise the stream in between (allocation-
 * free calls such as gs_decode_backward_noalloc suit it), and must keep every
 * buffer the graph uses alive while it may be launched.  `stream` must not be
 * the legacy default stream.  A new capture replaces the previous step. */
gs_status gs_plan_begin_capture(gs_plan* plan, hipStream_t stream);
gs_status gs_plan_end_capture(gs_plan* plan, hipStream_t stream);
gs_status gs_plan_launch(gs_plan* plan, hipStream_t stream);

/* Synchronises `stream`, then reads the workspace's status words. Returns
 * GS_ERR_CAPACITY when a sensor overflowed its pair capacity, and GS_ERR_HIP
 * when a device-side bounded wait gave up (the compositing work queue, or the
 * look-back of a sort or scan: the outputs of that run are not valid). */
gs_status gs_query_status(const gs_plan* plan, const void* workspace, hipStream_t stream,
                          gs_run_status* out);

/* Byte offsets of internal arrays inside the workspace, for inspection by
 * tests: sorted pair surfel indices (uint32 [capacity]), sorted pair tile ids
 * (uint32 [capacity]), tile ranges (uint32 [n_tiles][2]), per-surfel visible
 * flag (uint32 [N]) and the device pair counter (uint32). */
typedef struct gs_workspace_view {
  size_t pair_surfel, pair_tile, tile_ranges, visible, pair_count;
  int32_t n_tiles, tile_offset;
} gs_workspace_view;
gs_status gs_plan_inspect(const gs_plan* plan, int32_t sensor, gs_workspace_view* out);

/* ---------------------------------------------------------------------
 * Neural-Gaussian decode (Sec. III-A: attributes inferred from each
 * anchor's feature by the scene's MLP).  Per anchor a: input
 * x = [f_a (F, bf16); unit(x_a - sensor centre) in the group frame (3)],
 * h = ReLU(W1 x + b1) (H wide), y = W2 h + b2 with K offsets x J attributes:
 *   camera J = 10: opacity, r, g, b, s_u, s_v, q (4)
 *   LiDAR  J = 9 : opacity, intensity, s_u, s_v, q (4), ray drop
 * Heads: opacity/colour/intensity/ray drop = sigmoid, scale = l_a * sigmoid,
 * rotation = raw 4-vector, centre = x_a + l_a * O_k.  Surfel n = a*K + k.
 * The contractions run on MFMA with bf16 weights and features and FP32
 * accumulation; activations keep ~16 mantissa bits (hi+lo bf16 split).
 * ------------------------------------------------------------------- */
typedef struct gs_anchor_set {
  int32_t n_anchors;            /* A                                       */
  int32_t k;                    /* offsets per anchor (K <= 16)            */
  int32_t lidar;                /* 0: camera heads (J=10), 1: LiDAR (J=9)  */
  int32_t n_groups;             /* groups, each with its own MLP           */
  const int32_t* group_offsets; /* host [n_groups+1] over anchors          */
  const float* xyz;             /* device [3][A]                           */
  const float* scaling;         /* device [A]                              */
  const float* offsets;         /* device [3][K][A]                        */
  const uint16_t* feat;         /* device [A][32] bf16                     */
  const uint16_t* w1;           /* device [G][32][35] bf16 (out x in)      */
  const float* b1;              /* device [G][32]                          */
  const uint16_t* w2;           /* device [G][K*J][32] bf16                */
  const float* b2;              /* device [G][K*J]                         */
  int32_t flags;                /* GS_DECODE_* bits                        */
} gs_anchor_set;

/* Decode the MLP with plain FP32 vector arithmetic (one thread per anchor,
 * FP32 hidden activations) instead of bf16 MFMA: the reference "plain"
 * decode the MFMA path is compared against. */
#define GS_DECODE_VALU_FP32 1

/* Decoded surfel buffers (device, [C][A*K]).  rgb for camera, intensity and
 * drop (ray-drop probability) for LiDAR. */
typedef struct gs_decoded {
  float* mean;
  float* quat;
  float* scale;
  float* opacity;
  float* rgb;
  float* intensity;
  float* drop;
} gs_decoded;

/* Decodes every anchor for one sensor pose.  sensor_pose: device [12]
 * world->sensor; group_poses: device [n_groups][12] group->world.  Writes
 * A*K surfels; anchors of group g become surfels [K*off[g], K*off[g+1]).
 * out->mean may be NULL: the centres x_a + l_a O_k do not depend on the
 * sensor, so a caller decoding one anchor set for several sensors writes
 * them once (every other output is required). */
gs_status gs_decode_forward(const gs_anchor_set* anchors, const float* sensor_pose,
                            const float* group_poses, const gs_decoded* out, hipStream_t stream);

/* Adjoint of gs_decode_forward.  grad_in holds dL/d(decoded surfels) (same
 * layout as `out`, read only); accumulates (+=) into the FP32 gradient
 * buffers (device, NULL to skip): xyz [3][A], scaling [A], offsets [3][K][A],
 * feat [A][32], w1 [G][32][35], b1 [G][32], w2 [G][K*J][32], b2 [G][K*J].
 * scratch: device, gs_decode_scratch_size bytes (per-block partials of the
 * weight gradients, summed in a fixed order: weight gradients are
 * deterministic); may be NULL only when w1, b1, w2 and b2 are all NULL. */
typedef struct gs_anchor_grads {
  float* xyz;
  float* scaling;
  float* offsets;
  float* feat;
  float* w1;
  float* b1;
  float* w2;
  float* b2;
} gs_anchor_grads;
gs_status gs_decode_scratch_size(const gs_anchor_set* anchors, size_t* bytes);
gs_status gs_decode_backward(const gs_anchor_set* anchors, const float* sensor_pose,
                             const float* group_poses, const gs_decoded* grad_in,
                             const gs_anchor_grads* grads, void* scratch, hipStream_t stream);

/* Allocation-free variant of gs_decode_backward, for callers that cannot
 * allocate device memory or pass a workspace (code under HIP graph capture,
 * serving loops, harnesses that forbid allocation): same arguments and
 * results, without `scratch`.  The weight-gradient partials live in a
 * library-owned device array of GS_DECODE_NOALLOC_SCRATCH_BYTES per GPU
 * (allocated when the library is loaded, held until the process ends; its
 * address is looked up once per device on the first call there).  Inputs
 * whose partials need more (gs_decode_scratch_size) are rejected with
 * GS_ERR_INVALID_ARG before any launch: with K = 10 offsets that is about
 * 120k camera (J = 10) or 140k LiDAR (J = 8) anchors in one group (64 per
 * block, blocks rounded up per group) when weight gradients are requested;
 * without them there is no limit.  Every call on a GPU shares
 * that GPU's array: calls that may overlap on one GPU (other streams, other
 * host threads) race and must be ordered by the caller.  Calls no allocating
 * routine. */
#define GS_DECODE_NOALLOC_SCRATCH_BYTES ((size_t)32 << 20)
gs_status gs_decode_backward_noalloc(const gs_anchor_set* anchors, const float* sensor_pose,
                                     const float* group_poses, const gs_decoded* grad_in,
                                     const gs_anchor_grads* grads, hipStream_t stream);

/* Inpainting patch affinity (Sec. III-B, Eq. 6).  For each of `batch` pairs
 * of a target patch (p anchors) and a candidate source patch (q anchors):
 *   out[b][i][j] = exp(z_ij - max_k z_ik) / sum_k exp(z_ik - max_k z_ik),
 *   z = X_T X_S^T,
 * the softmax over the source anchors of the product of the encoded anchor
 * matrices (one anchor per row: its feature followed by the positional
 * encoding of its location, built and rounded to bf16 by the caller).
 * xt: device bf16 bits [batch][p][d] row-major; xs: device bf16 bits
 * [batch][q][d]; both 16-byte aligned; d a multiple of 32 in [32, 256]
 * (zero-pad the rows).  out: device FP32 [batch][p][q], written whole.
 * Products are bf16 x bf16 on MFMA with FP32 accumulation; exponentials FP32.
 * batch, p or q = 0: nothing is launched.  Errors (before any launch):
 * GS_ERR_INVALID_ARG for negative sizes, batch > 65535, a bad d, null or
 * misaligned pointers; GS_ERR_HIP if the launch fails.  Asynchronous on
 * `stream`; no memory is allocated. */
gs_status gs_affinity(const uint16_t* xt, const uint16_t* xs, int32_t batch, int32_t p, int32_t q, int32_t d,
                      float* out, hipStream_t stream);

/* ---------------------------------------------------------------------
 * Scene zones and double-buffered swap-in (Sec. III-A, large-scale scenes:
 * the scene is cut by ground-plane position into square zones, 40 m on a
 * side in the paper, each widened on every side by a fixed fraction of its
 * side, 25 % in the paper; at render time two buffers are used, and the
 * Gaussians of the zone the vehicle is about to enter are brought into one
 * while the other is rendered).
 *
 * Zone (i, j) of a grid covers, in ground coordinates (a, b) =
 * (x[axis[0]], x[axis[1]]) converted to double,
 *   origin[0] + (i - pad) * size <= a < origin[0] + ((i + 1) + pad) * size
 *   origin[1] + (j - pad) * size <= b < origin[1] + ((j + 1) + pad) * size,
 * each bound evaluated in IEEE double exactly as written (i, j converted to
 * double).  Zone id = j * nx + i.  With pad > 0 neighbouring zones overlap,
 * so a point belongs to up to four zones; points outside every zone (or
 * with a NaN coordinate) belong to none.
 * ------------------------------------------------------------------- */
typedef struct gs_zone_grid {
  int32_t axis[2];   /* world axes spanning the ground plane (0 x, 1 y, 2 z), distinct */
  double origin[2];  /* ground coordinates of the low corner of zone (0, 0)            */
  double size;       /* zone side, finite and > 0 (metres)                              */
  double pad;        /* padding on each side as a fraction of `size`, finite, in [0, 1] */
  int32_t nx, ny;    /* zones along axis[0] and axis[1], >= 1, nx * ny <= 2^20          */
} gs_zone_grid;

/* Lists the anchors (points) of every zone.  xyz: host [3][n] FP32.
 * zone_offsets: host [nx*ny + 1], always written (CSR offsets).  index: host
 * [cap]; the anchors of zone z are index[zone_offsets[z] ..
 * zone_offsets[z+1]) in ascending order.  *total: number of (zone, anchor)
 * memberships, always written.  index may be NULL with cap = 0 to query
 * *total.  Errors: GS_ERR_INVALID_ARG (bad grid, n outside [0, 2^32 - 1],
 * null pointers); GS_ERR_CAPACITY when *total > cap (index is then left
 * unspecified).  Host only: no HIP call is made. */
gs_status gs_zone_partition(const gs_zone_grid* grid, const float* xyz, int64_t n, uint32_t* zone_offsets,
                            uint32_t* index, int64_t cap, int64_t* total);

/* One array that moves with a zone.
 *   per_zone = 0: an anchor attribute.  host is [rows][host_stride]
 *     elements of elem_bytes bytes over every anchor of the scene; an upload
 *     of zone z into buffer b writes, for every row r and k < capacity,
 *       device[b][r * device_stride + k] = host[r * host_stride + L[k]]
 *     for the zone's anchor list L (k < |L|), and `fill` (elem_bytes bytes;
 *     NULL: zero bytes) for |L| <= k < capacity.  Elements of a device row
 *     at or beyond `capacity` (e.g. resident actors) are not touched.
 *   per_zone = 1: a per-zone block (e.g. the zone's MLP weights).  host is
 *     [n_zones][elem_bytes] bytes; an upload writes the zone's block to
 *     device[b] (rows must be 1; strides and fill unused).
 * host is read by the swap-in thread while the stream exists and must not
 * change meanwhile; device[0] and device[1] are device memory of the
 * stream's device. */
typedef struct gs_zone_field {
  const void* host;
  int64_t host_stride;     /* elements per host row (per_zone = 0)          */
  void* device[2];         /* destination in buffer 0 and buffer 1          */
  int64_t device_stride;   /* elements per device row, >= capacity           */
  int32_t rows;            /* >= 1                                           */
  int32_t elem_bytes;      /* 1..65536                                        */
  int32_t per_zone;        /* 0 or 1                                         */
  const void* fill;        /* host, elem_bytes bytes, or NULL                 */
} gs_zone_field;

typedef struct gs_zone_stream_desc {
  int32_t n_zones;               /* >= 1                                         */
  const uint32_t* zone_offsets;  /* host [n_zones + 1] (gs_zone_partition)       */
  const uint32_t* index;         /* host [zone_offsets[n_zones]]                 */
  int64_t capacity;              /* anchors per buffer, >= the largest zone       */
  int64_t n_anchors;             /* anchors of the scene (every index below it)  */
  int32_t n_fields;              /* 1..64                                        */
  const gs_zone_field* fields;   /* host [n_fields]                              */
  int32_t threads;               /* host threads that gather one zone, 1..64      */
} gs_zone_stream_desc;

typedef struct gs_zone_stream gs_zone_stream; /* opaque, owned by the library */

/* The calls on one zone stream are made from one host thread (the swap-in
 * thread is the library's own). */

/* Creates a swap-in stream on the current device: pinned host staging for
 * both buffers (the bytes of one zone at full capacity, per buffer), a copy
 * stream of its own, and one swap-in thread.  The descriptor's arrays are
 * copied; `host` arrays are not.  Errors: GS_ERR_INVALID_ARG (bad sizes or
 * pointers, an index at or beyond n_anchors, capacity below a zone's
 * count), GS_ERR_HIP. */
gs_status gs_zone_stream_create(const gs_zone_stream_desc* desc, gs_zone_stream** out);

/* Queues an upload of `zone` into `buffer` (0 or 1) and returns at once.  The
 * swap-in thread waits until the previous upload from that buffer's staging
 * has finished, gathers the zone into the staging, and enqueues the copies
 * on the copy stream behind the last gs_zone_stream_release of the buffer.
 * Uploads are processed in the order they are queued. */
gs_status gs_zone_stream_prefetch(gs_zone_stream* zs, int32_t zone, int32_t buffer);

/* Waits on the host until every upload queued into `buffer` has been
 * enqueued, then makes `stream` wait on the device for the last of them:
 * work enqueued on `stream` afterwards sees the buffer's new contents.
 * Writes the zone the buffer holds and its anchor count (NULL to skip).
 * GS_ERR_INVALID_ARG if nothing was ever queued into the buffer; GS_ERR_HIP
 * if the swap-in thread met a HIP error (sticky). */
gs_status gs_zone_stream_acquire(gs_zone_stream* zs, int32_t buffer, hipStream_t stream, int32_t* zone,
                                 int64_t* count);

/* Marks the end of the reads of `buffer` by the work enqueued on `stream` so
 * far: the next upload into the buffer starts on the device only after that
 * work.  Call it after enqueuing the last use of the buffer's contents and
 * before queueing an upload into it.  GS_ERR_INVALID_ARG if an upload was
 * queued into the buffer since its last acquire (that upload could
 * otherwise be ordered behind work that waits for a later upload). */
gs_status gs_zone_stream_release(gs_zone_stream* zs, int32_t buffer, hipStream_t stream);

typedef struct gs_zone_swap_stats {
  int32_t zone;       /* zone of the last upload into the buffer (-1: none)   */
  int64_t count;      /* its anchors                                          */
  int64_t bytes;      /* bytes copied host to device                          */
  double gather_ms;   /* host time of the gather into pinned staging          */
  double upload_ms;   /* device time of the copies on the copy stream         */
} gs_zone_swap_stats;

/* Statistics of the last upload into `buffer`; waits for that upload to
 * complete. */
gs_status gs_zone_stream_stats(gs_zone_stream* zs, int32_t buffer, gs_zone_swap_stats* out);

/* Waits for queued uploads, stops the swap-in thread and frees the staging,
 * stream and events.  NULL is a no-op. */
void gs_zone_stream_destroy(gs_zone_stream* zs);

#ifdef __cplusplus
}
#endif

#endif /* GS2D_H */
