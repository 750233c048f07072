"""Python binding of the gs2d renderer: plans, workspaces and autograd.

Argument marshalling only -- every rendering step runs in the HIP library
(libgs2d.so); PyTorch supplies device memory and the stream.  Render
semantics: Sec. III-A of the paper (Eq. 1 surfels, Eq. 2 two-plane ray-splat
solve, Eq. 3 pinhole and Eq. 5 LiDAR planes) with front-to-back compositing.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L

PRODUCTION = dict(alpha_min=1.0 / 255.0, alpha_max=0.99, T_min=1e-4, cutoff2=2.0 * math.log(255.0),
                  lowpass=True, lp_inv_sigma2=2.0, bg=(0.0, 0.0, 0.0))
STRICT = dict(PRODUCTION, alpha_min=0.0, T_min=0.0, cutoff2=25.0)

CAMERA_CHANNELS = ("r", "g", "b", "depth", "nx", "ny", "nz", "alpha", "median")
LIDAR_CHANNELS = ("range", "intensity", "alpha", "drop", "drop_mask", "median")


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _f32(t: torch.Tensor | None, name: str) -> torch.Tensor | None:
    if t is None:
        return None
    if t.dtype != torch.float32 or not t.is_cuda or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    return t


@dataclass
class SceneShape:
    n_splats: int
    sh_degree: int = -1
    has_intensity: bool = False
    group_offsets: tuple = ()

    def offsets(self):
        return list(self.group_offsets) if self.group_offsets else [0, self.n_splats]


class Renderer:
    """A render plan for a fixed set of scenes (shapes) and sensors.

    scenes:  list of SceneShape (1 or 2 scenes, e.g. camera and LiDAR)
    sensors: list of dicts (gen.scenes.pinhole / lidar_spinning layout) with an
             optional 'scene' index and 'tile' (tw, th)
    opts:    compositing options (PRODUCTION / STRICT or overrides)
    """

    def __init__(self, scenes, sensors, opts=None, pair_capacity: int = 0, device="cuda", batched=False,
                 segment_pairs: int = 0):
        self.lib = L.load()
        self.device = torch.device(device)
        self.scenes = [s if isinstance(s, SceneShape) else SceneShape(**s) for s in scenes]
        self.sensors = list(sensors)
        o = dict(PRODUCTION)
        o.update(opts or {})
        self.opts = o
        self._keep = []
        sd = (L.SceneDesc * len(self.scenes))()
        for i, s in enumerate(self.scenes):
            off = (ctypes.c_int32 * len(s.offsets()))(*s.offsets())
            self._keep.append(off)
            sd[i] = L.SceneDesc(s.n_splats, s.sh_degree, int(s.has_intensity), len(s.offsets()) - 1, off)
        sens = (L.SensorDesc * len(self.sensors))()
        for i, s in enumerate(self.sensors):
            tw, th = s.get("tile", (0, 0))
            if s["kind"] in ("pinhole", "cylindrical"):
                kind = L.GS_SENSOR_PINHOLE if s["kind"] == "pinhole" else L.GS_SENSOR_CYLINDRICAL
                sens[i] = L.SensorDesc(kind, s["width"], s["height"], s["fx"], s["fy"], s["cx"],
                                       s["cy"], None, s["z_near"], s.get("scene", 0), tw, th)
            else:
                el = np.ascontiguousarray(s["elevations"], np.float64)
                self._keep.append(el)
                sens[i] = L.SensorDesc(L.GS_SENSOR_LIDAR, s["width"], s["height"], 0, 0, 0, 0,
                                       el.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), s["z_near"],
                                       s.get("scene", 0), tw, th)
        ro = L.RenderOpts(o["alpha_min"], o["alpha_max"], o["T_min"], o["cutoff2"], o["lp_inv_sigma2"],
                          int(bool(o["lowpass"])), (ctypes.c_float * 3)(*o["bg"]))
        desc = L.PlanDesc(len(self.scenes), sd, len(self.sensors), sens, ro, int(pair_capacity), int(batched),
                          int(segment_pairs))
        plan = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.gs_plan_create(ctypes.byref(desc), ctypes.byref(plan)))
        self.plan = plan
        nb = ctypes.c_size_t()
        L.check(self.lib.gs_plan_workspace_size(self.plan, ctypes.byref(nb)))
        self.workspace = torch.empty(max(int(nb.value), 256), dtype=torch.uint8, device=self.device)
        self.batched = bool(batched)
        assert self.workspace.data_ptr() % 256 == 0
        self.generation = 0

    def __del__(self):
        plan = getattr(self, "plan", None)
        if plan is not None and plan.value:
            try:
                self.lib.gs_plan_destroy(plan)
            except Exception:
                pass
            self.plan = None

    # ------------------------------------------------------------------
    def channels(self, i: int) -> int:
        return L.GS_LIDAR_CHANNELS if self.sensors[i]["kind"] == "lidar" else L.GS_CAMERA_CHANNELS

    def _scene_structs(self, scenes):
        arr = (L.Scene * len(self.scenes))()
        for i, (shape, sc) in enumerate(zip(self.scenes, scenes)):
            p = lambda k: L.ptr(_f32(sc.get(k), k))
            if sc["mean"].shape[-1] != shape.n_splats:
                raise ValueError(f"scene {i}: expected {shape.n_splats} surfels, got {sc['mean'].shape[-1]}")
            arr[i] = L.Scene(p("mean"), p("quat"), p("scale"), p("opacity"), p("rgb"), p("sh"), p("intensity"),
                             p("drop"))
        return arr

    def new_outputs(self):
        return [torch.empty((self.channels(i), s["height"], s["width"]), dtype=torch.float32, device=self.device)
                for i, s in enumerate(self.sensors)]

    def forward(self, scenes, sensor_poses: torch.Tensor, group_poses: torch.Tensor, outputs=None):
        """Render every sensor; returns a list of [C, H, W] tensors."""
        _f32(sensor_poses, "sensor_poses")
        _f32(group_poses, "group_poses")
        outs = outputs if outputs is not None else self.new_outputs()
        optr = (ctypes.c_void_p * len(outs))(*[o.data_ptr() for o in outs])
        sc = self._scene_structs(scenes)
        L.check(self.lib.gs_render_forward(self.plan, sc, sensor_poses.data_ptr(), group_poses.data_ptr(), optr,
                                           self.workspace.data_ptr(), _stream()))
        self.generation += 1
        return outs

    def capture(self, scenes, sensor_poses, group_poses, outputs):
        """Capture the forward into a HIP graph on the current (non-default) stream.

        Later forward() calls with the same tensors replay the graph.
        """
        optr = (ctypes.c_void_p * len(outputs))(*[o.data_ptr() for o in outputs])
        sc = self._scene_structs(scenes)
        L.check(self.lib.gs_plan_capture(self.plan, sc, sensor_poses.data_ptr(), group_poses.data_ptr(), optr,
                                         self.workspace.data_ptr(), _stream()))

    def begin_capture(self):
        """Start capturing everything enqueued on the current (non-default) stream
        into this plan's step graph (see gs_plan_begin_capture)."""
        L.check(self.lib.gs_plan_begin_capture(self.plan, _stream()))

    def end_capture(self):
        L.check(self.lib.gs_plan_end_capture(self.plan, _stream()))

    def launch(self):
        """Replay the captured step on the current stream (one graph launch)."""
        L.check(self.lib.gs_plan_launch(self.plan, _stream()))

    def backward(self, scenes, sensor_poses, group_poses, outputs, grad_outputs, grads=None):
        """Adjoint of forward (uses the workspace state of the last forward).

        Returns (or accumulates into) one dict of gradient tensors per scene.
        """
        if grads is None:
            grads = []
            for shape, sc in zip(self.scenes, scenes):
                grads.append({k: torch.zeros_like(v) for k, v in sc.items() if isinstance(v, torch.Tensor)})
        gptr = (L.SceneGrads * len(self.scenes))()
        for i, g in enumerate(grads):
            p = lambda k: L.ptr(g.get(k))
            gptr[i] = L.SceneGrads(p("mean"), p("quat"), p("scale"), p("opacity"), p("rgb"), p("sh"), p("intensity"),
                                   p("drop"))
        grad_outputs = [g.contiguous() for g in grad_outputs]
        optr = (ctypes.c_void_p * len(outputs))(*[o.data_ptr() for o in outputs])
        gop = (ctypes.c_void_p * len(grad_outputs))(*[g.data_ptr() for g in grad_outputs])
        sc = self._scene_structs(scenes)
        L.check(self.lib.gs_render_backward(self.plan, sc, sensor_poses.data_ptr(), group_poses.data_ptr(), optr, gop,
                                            self.workspace.data_ptr(), gptr, _stream()))
        return grads

    def status(self) -> dict:
        st = L.RunStatus()
        rc = self.lib.gs_query_status(self.plan, self.workspace.data_ptr(), _stream(), ctypes.byref(st))
        n = len(self.sensors)
        out = dict(pairs=list(st.pairs[:n]), overflow=bool(st.overflow), n_visible=list(st.n_visible[:n]),
                   fp64_pairs=int(st.fp64_pairs), evaluated=int(st.evaluated), composited=int(st.composited),
                   work_items=int(st.work_items), segments=int(st.segments),
                   graph_replays=int(st.graph_replays), step_launches=int(st.step_launches), wave_pairs=int(st.wave_pairs), rc=rc)
        return out

    def set_counters(self, on: bool):
        """Count evaluated / composited pairs and pair-loop iterations in later forwards (calibration)."""
        L.check(self.lib.gs_plan_set_counters(self.plan, int(bool(on))))

    def set_timing(self, max_records: int):
        """Record HIP events around every stage of the next calls (0 disables)."""
        L.check(self.lib.gs_plan_set_timing(self.plan, int(max_records)))

    def stage_times(self, reset=True) -> dict:
        """Summed milliseconds and interval counts per stage since the last reset (syncs)."""
        t = L.StageTimes()
        L.check(self.lib.gs_plan_stage_times(self.plan, _stream(), int(reset), ctypes.byref(t)))
        return {name: (float(t.ms[i]), int(t.launches[i])) for i, name in enumerate(L.STAGES)}

    def inspect(self, i: int) -> dict:
        """Views of sensor i's sorted pair list, tile ranges and visibility (tests)."""
        v = L.WorkspaceView()
        L.check(self.lib.gs_plan_inspect(self.plan, i, ctypes.byref(v)))
        ws = self.workspace
        n = self.scenes[self.sensors[i].get("scene", 0)].n_splats

        def u32(off, count):
            return ws[off:off + 4 * count].view(torch.int32)

        count = int(u32(v.pair_count, 1).item())
        cap = (ws.numel() - v.pair_surfel) // 4
        count_c = min(count, cap)
        return dict(pairs=count, pair_surfel=u32(v.pair_surfel, count_c), pair_tile=u32(v.pair_tile, count_c),
                    ranges=u32(v.tile_ranges, 2 * v.n_tiles).view(v.n_tiles, 2), visible=u32(v.visible, n),
                    n_tiles=v.n_tiles)


def poses_tensor(poses, device="cuda") -> torch.Tensor:
    a = np.ascontiguousarray(np.asarray(poses, np.float32).reshape(-1, 12))
    return torch.from_numpy(a).to(device)


def scene_tensors(scene: dict, device="cuda") -> dict:
    """numpy scene dict (gen / tests layout) -> dict of CUDA float32 tensors."""
    out = {}
    for k in ("mean", "quat", "scale", "opacity", "rgb", "sh", "intensity", "drop"):
        v = scene.get(k)
        if v is not None:
            out[k] = torch.from_numpy(np.ascontiguousarray(v, np.float32)).to(device)
    return out


class _RenderFn(torch.autograd.Function):
    @staticmethod
    def forward(ctx, renderer, sensor_poses, group_poses, keys, *flat):
        scenes = _unflatten(keys, flat)
        outs = renderer.forward(scenes, sensor_poses, group_poses)
        ctx.renderer = renderer
        ctx.generation = renderer.generation
        ctx.keys = keys
        ctx.poses = (sensor_poses, group_poses)
        ctx.save_for_backward(*flat, *outs)
        ctx.n_flat = len(flat)
        return tuple(outs)

    @staticmethod
    def backward(ctx, *gouts):
        r = ctx.renderer
        if r.generation != ctx.generation:
            raise RuntimeError("renderer workspace was reused by a later forward before this backward")
        saved = ctx.saved_tensors
        flat, outs = saved[:ctx.n_flat], saved[ctx.n_flat:]
        scenes = _unflatten(ctx.keys, flat)
        gouts = [g if g is not None else torch.zeros_like(o) for g, o in zip(gouts, outs)]
        grads = r.backward(scenes, ctx.poses[0], ctx.poses[1], list(outs), gouts)
        flat_g = []
        for si, ks in enumerate(ctx.keys):
            for k in ks:
                flat_g.append(grads[si].get(k))
        return (None, None, None, None, *flat_g)


def _flatten(scenes):
    keys = tuple(tuple(sorted(k for k, v in sc.items() if isinstance(v, torch.Tensor))) for sc in scenes)
    flat = [sc[k] for sc, ks in zip(scenes, keys) for k in ks]
    return keys, flat


def _unflatten(keys, flat):
    out, i = [], 0
    for ks in keys:
        d = {}
        for k in ks:
            d[k] = flat[i]
            i += 1
        out.append(d)
    return out


def render(renderer: Renderer, scenes, sensor_poses, group_poses):
    """Differentiable render: list of [C, H, W] outputs, gradients flow to scene tensors."""
    keys, flat = _flatten(scenes)
    return list(_RenderFn.apply(renderer, sensor_poses, group_poses, keys, *flat))
