"""ctypes declarations of the gs2d C-ABI (include/gs2d.h) and library loading.

Argument marshalling only: every step of rendering runs in the HIP library.
Loading fails loudly when the built library is missing.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_size_t, c_uint16, c_void_p

PKG_DIR = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG_DIR, "libgs2d.so")

GS_OK, GS_ERR_INVALID_ARG, GS_ERR_CAPACITY, GS_ERR_HIP, GS_ERR_UNSUPPORTED = range(5)
GS_SENSOR_PINHOLE, GS_SENSOR_LIDAR, GS_SENSOR_CYLINDRICAL = 0, 1, 2
GS_MAX_GROUPS = 64
GS_MAX_SENSORS = 16
GS_CAMERA_CHANNELS = 9
GS_LIDAR_CHANNELS = 6


class SensorDesc(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("width", c_int32), ("height", c_int32), ("fx", c_float), ("fy", c_float),
                ("cx", c_float), ("cy", c_float), ("elevations", POINTER(c_double)), ("z_near", c_float),
                ("scene", c_int32), ("tile_w", c_int32), ("tile_h", c_int32)]


class RenderOpts(ctypes.Structure):
    _fields_ = [("alpha_min", c_float), ("alpha_max", c_float), ("T_min", c_float), ("cutoff2", c_float),
                ("lp_inv_sigma2", c_float), ("lowpass", c_int32), ("bg", c_float * 3)]


class SceneDesc(ctypes.Structure):
    _fields_ = [("n_splats", c_int32), ("sh_degree", c_int32), ("has_intensity", c_int32), ("n_groups", c_int32),
                ("group_offsets", POINTER(c_int32))]


class Scene(ctypes.Structure):
    _fields_ = [("mean", c_void_p), ("quat", c_void_p), ("scale", c_void_p), ("opacity", c_void_p),
                ("rgb", c_void_p), ("sh", c_void_p), ("intensity", c_void_p), ("drop", c_void_p)]


class SceneGrads(ctypes.Structure):
    _fields_ = [("mean", c_void_p), ("quat", c_void_p), ("scale", c_void_p), ("opacity", c_void_p),
                ("rgb", c_void_p), ("sh", c_void_p), ("intensity", c_void_p), ("drop", c_void_p)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("n_scenes", c_int32), ("scenes", POINTER(SceneDesc)), ("n_sensors", c_int32),
                ("sensors", POINTER(SensorDesc)), ("opts", RenderOpts), ("pair_capacity", c_int64),
                ("batched", c_int32), ("segment_pairs", c_int32)]


class RunStatus(ctypes.Structure):
    _fields_ = [("pairs", c_int64 * GS_MAX_SENSORS), ("overflow", c_int32), ("n_visible", c_int32 * GS_MAX_SENSORS),
                ("fp64_pairs", c_int64), ("evaluated", c_int64), ("composited", c_int64),
                ("work_items", c_int64), ("segments", c_int64), ("graph_replays", c_int64),
                ("step_launches", c_int64), ("wave_pairs", c_int64)]


STAGES = ("preprocess", "depth_sort", "emit", "tile_sort", "ranges", "blend", "blend_bwd", "splat_bwd")


class StageTimes(ctypes.Structure):
    _fields_ = [("records", c_int32), ("launches", c_int32 * len(STAGES)), ("ms", c_double * len(STAGES))]


class WorkspaceView(ctypes.Structure):
    _fields_ = [("pair_surfel", c_size_t), ("pair_tile", c_size_t), ("tile_ranges", c_size_t), ("visible", c_size_t),
                ("pair_count", c_size_t), ("n_tiles", c_int32), ("tile_offset", c_int32)]


class AnchorSet(ctypes.Structure):
    _fields_ = [("n_anchors", c_int32), ("k", c_int32), ("lidar", c_int32), ("n_groups", c_int32),
                ("group_offsets", POINTER(c_int32)), ("xyz", c_void_p), ("scaling", c_void_p), ("offsets", c_void_p),
                ("feat", c_void_p), ("w1", c_void_p), ("b1", c_void_p), ("w2", c_void_p), ("b2", c_void_p),
                ("flags", c_int32)]


GS_DECODE_VALU_FP32 = 1
GS_DECODE_NOALLOC_SCRATCH_BYTES = 32 << 20


class Decoded(ctypes.Structure):
    _fields_ = [("mean", c_void_p), ("quat", c_void_p), ("scale", c_void_p), ("opacity", c_void_p),
                ("rgb", c_void_p), ("intensity", c_void_p), ("drop", c_void_p)]


class AnchorGrads(ctypes.Structure):
    _fields_ = [("xyz", c_void_p), ("scaling", c_void_p), ("offsets", c_void_p), ("feat", c_void_p),
                ("w1", c_void_p), ("b1", c_void_p), ("w2", c_void_p), ("b2", c_void_p)]


class ZoneGrid(ctypes.Structure):
    _fields_ = [("axis", c_int32 * 2), ("origin", c_double * 2), ("size", c_double), ("pad", c_double),
                ("nx", c_int32), ("ny", c_int32)]


class ZoneField(ctypes.Structure):
    _fields_ = [("host", c_void_p), ("host_stride", c_int64), ("device", c_void_p * 2), ("device_stride", c_int64),
                ("rows", c_int32), ("elem_bytes", c_int32), ("per_zone", c_int32), ("fill", c_void_p)]


class ZoneStreamDesc(ctypes.Structure):
    _fields_ = [("n_zones", c_int32), ("zone_offsets", c_void_p), ("index", c_void_p), ("capacity", c_int64),
                ("n_anchors", c_int64), ("n_fields", c_int32), ("fields", POINTER(ZoneField)), ("threads", c_int32)]


class ZoneSwapStats(ctypes.Structure):
    _fields_ = [("zone", c_int32), ("count", c_int64), ("bytes", c_int64), ("gather_ms", c_double),
                ("upload_ms", c_double)]


# (name, restype, argtypes) of every exported function of include/gs2d.h
SIGNATURES = [
    ("gs_version", c_char_p, []),
    ("gs_status_string", c_char_p, [c_int32]),
    ("gs_last_error", c_int32, [c_char_p, c_size_t]),
    ("gs_plan_create", c_int32, [POINTER(PlanDesc), POINTER(c_void_p)]),
    ("gs_plan_destroy", None, [c_void_p]),
    ("gs_plan_workspace_size", c_int32, [c_void_p, POINTER(c_size_t)]),
    ("gs_render_forward", c_int32, [c_void_p, POINTER(Scene), c_void_p, c_void_p, POINTER(c_void_p), c_void_p,
                                    c_void_p]),
    ("gs_render_backward", c_int32, [c_void_p, POINTER(Scene), c_void_p, c_void_p, POINTER(c_void_p),
                                     POINTER(c_void_p), c_void_p, POINTER(SceneGrads), c_void_p]),
    ("gs_plan_set_counters", c_int32, [c_void_p, c_int32]),
    ("gs_plan_begin_capture", c_int32, [c_void_p, c_void_p]),
    ("gs_plan_end_capture", c_int32, [c_void_p, c_void_p]),
    ("gs_plan_launch", c_int32, [c_void_p, c_void_p]),
    ("gs_plan_capture", c_int32, [c_void_p, POINTER(Scene), c_void_p, c_void_p, POINTER(c_void_p), c_void_p,
                                  c_void_p]),
    ("gs_query_status", c_int32, [c_void_p, c_void_p, c_void_p, POINTER(RunStatus)]),
    ("gs_plan_inspect", c_int32, [c_void_p, c_int32, POINTER(WorkspaceView)]),
    ("gs_plan_set_timing", c_int32, [c_void_p, c_int32]),
    ("gs_plan_stage_times", c_int32, [c_void_p, c_void_p, c_int32, POINTER(StageTimes)]),
    ("gs_decode_forward", c_int32, [POINTER(AnchorSet), c_void_p, c_void_p, POINTER(Decoded), c_void_p]),
    ("gs_decode_scratch_size", c_int32, [POINTER(AnchorSet), POINTER(c_size_t)]),
    ("gs_decode_backward", c_int32, [POINTER(AnchorSet), c_void_p, c_void_p, POINTER(Decoded),
                                     POINTER(AnchorGrads), c_void_p, c_void_p]),
    ("gs_decode_backward_noalloc", c_int32, [POINTER(AnchorSet), c_void_p, c_void_p, POINTER(Decoded),
                                             POINTER(AnchorGrads), c_void_p]),
    ("gs_affinity", c_int32, [c_void_p, c_void_p, c_int32, c_int32, c_int32, c_int32, c_void_p, c_void_p]),
    ("gs_zone_partition", c_int32, [POINTER(ZoneGrid), c_void_p, c_int64, c_void_p, c_void_p, c_int64,
                                    POINTER(c_int64)]),
    ("gs_zone_stream_create", c_int32, [POINTER(ZoneStreamDesc), POINTER(c_void_p)]),
    ("gs_zone_stream_prefetch", c_int32, [c_void_p, c_int32, c_int32]),
    ("gs_zone_stream_acquire", c_int32, [c_void_p, c_int32, c_void_p, POINTER(c_int32), POINTER(c_int64)]),
    ("gs_zone_stream_release", c_int32, [c_void_p, c_int32, c_void_p]),
    ("gs_zone_stream_stats", c_int32, [c_void_p, c_int32, POINTER(ZoneSwapStats)]),
    ("gs_zone_stream_destroy", None, [c_void_p]),
]

_lib = None


class GsError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"gs2d status {status}: {message}")
        self.status = status


def load(path: str | None = None) -> ctypes.CDLL:
    """Load the built HIP library (raises if it has not been built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"gs2d HIP library not found at {p}; build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    lib = ctypes.CDLL(p)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = lib
    return lib


def check(status: int):
    if status != GS_OK:
        buf = ctypes.create_string_buffer(1024)
        load().gs_last_error(buf, 1024)
        raise GsError(status, buf.value.decode(errors="replace"))


def ptr(t) -> int | None:
    """Device pointer of a tensor (None for None)."""
    if t is None:
        return None
    return t.data_ptr()
