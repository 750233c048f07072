"""Tile-shape and segment-length autotuner for the compositing queue.

The best tile shape depends on the sensor: a 1080p camera looking down a road
corridor has a few horizon tiles with 100x the median list, a 128 x 1800
LiDAR range image has long thin features along the azimuth.  The segment
length L trades the critical path of the heaviest tile (long L) against the
extra partial-state traffic and re-evaluation of split tiles (short L).

`autotune` times the forward render of every candidate (tile shape x L) on a
calibration scene, one sensor at a time, and picks per sensor the fastest
tile shape and per plan the L with the smallest summed time.  Results are
cached by (GPU architecture, sensor kind, W x H, surfel-count bucket) in a
JSON file, so that later plans for the same class of sensor skip the timing.
Batched plans need 256-ray tiles, so only those shapes are tried for them.

Choices keep a preferred candidate (the kind's usual tile shape, L = 2048)
unless another is faster by more than a margin (3 %): candidates within
timing noise of each other would otherwise flip from run to run, and a
plan's counters and profiles would describe a different configuration than
its timed run.  For the same reason the package ships the timings measured
on MI355X (gfx950) for its benchmark sensors (`tuned/autotune_seed.json`):
their entries take precedence over the user cache, so every machine of that
kind runs the configuration the profiles describe (GS2D_AUTOTUNE_SEED=""
turns the seed off).
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import torch

from .render import Renderer

TILES_ANY = [(8, 8), (16, 8), (8, 16), (16, 16), (32, 8), (8, 32), (32, 16), (16, 32), (64, 8)]
TILES_256 = [(16, 16), (32, 8), (8, 32)]
SEGMENTS = [256, 512, 1024, 2048, 4096]
# preferred candidates (kept unless another is faster by more than MARGIN)
PREFER_TILE = {"pinhole": (32, 8), "cylindrical": (32, 8), "lidar": (16, 16)}
PREFER_TILE_SINGLE = {"pinhole": (32, 8), "cylindrical": (32, 8), "lidar": (16, 8)}
PREFER_SEG = 2048
MARGIN = 0.03


def pick(ms: dict, prefer, margin: float = MARGIN):
    """The key of the smallest value of ms, except that `prefer` (a key of ms)
    is kept unless the smallest is below it by more than `margin`."""
    best = min(ms, key=lambda k: ms[k])
    if prefer is not None and prefer in ms and ms[prefer] <= (1.0 + margin) * ms[best]:
        return prefer
    return best


SEED_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned", "autotune_seed.json")


def seed_path() -> str:
    return os.environ.get("GS2D_AUTOTUNE_SEED", SEED_PATH)


def default_cache_path() -> str:
    return os.environ.get("GS2D_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "gs2d", "autotune.json"))


def n_bucket(n: int) -> int:
    """Power of two nearest to n (in log scale)."""
    return 1 << max(0, int(round(math.log2(max(n, 1)))))


def cache_key(arch: str, kind: str, width: int, height: int, n: int, batched: bool) -> str:
    return f"{arch}|{kind}|{width}x{height}|n{n_bucket(n)}|{'b' if batched else 's'}"


@dataclass
class TuneResult:
    tiles: list                       # per sensor (tw, th)
    segment_pairs: int
    timings: dict = field(default_factory=dict)  # key -> {"tile,seg": ms}
    from_cache: list = field(default_factory=list)


class TuneCache:
    """JSON map cache_key -> {"ms": {"tw x th / L": ms}} (all candidates kept)."""

    def __init__(self, path: str | None, seed: str | None = None):
        self.path = path
        self.data = self._read(path)
        self.data.update(self._read(seed_path() if seed is None else seed))  # shipped timings win

    @staticmethod
    def _read(path):
        if not path or not os.path.exists(path):
            return {}
        try:
            with open(path) as f:
                d = json.load(f)
            return d if isinstance(d, dict) else {}
        except (OSError, ValueError):
            return {}

    def get(self, key):
        return self.data.get(key)

    def put(self, key, value):
        self.data[key] = value

    def save(self):
        if not self.path:
            return
        os.makedirs(os.path.dirname(self.path) or ".", exist_ok=True)
        tmp = self.path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(self.data, f, indent=1, sort_keys=True)
        os.replace(tmp, self.path)


def _fmt(tile, seg):
    return f"{tile[0]}x{tile[1]}/{seg}"


def _parse(s):
    t, seg = s.split("/")
    tw, th = t.split("x")
    return (int(tw), int(th)), int(seg)


def _time_forward(shape, scene, sensor, pose, group_poses, tile, seg, opts, pair_capacity, steps, warmup, device):
    s = dict(sensor)
    s["scene"] = 0
    s["tile"] = tile
    r = Renderer([shape], [s], opts=opts, pair_capacity=pair_capacity, device=device, segment_pairs=seg)
    outs = r.new_outputs()
    sp = pose.reshape(1, 12).contiguous()
    for _ in range(warmup):
        r.forward([scene], sp, group_poses, outputs=outs)
    if r.status()["overflow"]:
        raise RuntimeError("pair capacity overflow while autotuning")
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        r.forward([scene], sp, group_poses, outputs=outs)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def autotune(shapes, scenes, sensors, sensor_poses, group_poses_per_sensor, *, batched=False, opts=None,
             tiles=None, segments=None, pair_capacity=0, steps=5, warmup=2, cache_path="default",
             device="cuda", margin=MARGIN) -> TuneResult:
    """Choose tile shapes (per sensor) and the segment length (per plan).

    shapes / scenes: per sensor, the SceneShape and the scene tensors it renders;
    sensor_poses: [S, 12] tensor; group_poses_per_sensor: list of [G, 12]
    tensors (the groups of each sensor's scene).  Timing runs use one
    single-sensor plan per candidate on the caller's current stream.
    """
    cands = tiles or (TILES_256 if batched else TILES_ANY)
    if batched:
        cands = [t for t in cands if t[0] * t[1] == 256]
    segs = segments or SEGMENTS
    path = default_cache_path() if cache_path == "default" else cache_path
    cache = TuneCache(path)
    arch = torch.cuda.get_device_properties(torch.device(device)).gcnArchName.split(":")[0]
    per_sensor = []
    from_cache = []
    timings = {}
    for i, s in enumerate(sensors):
        key = cache_key(arch, s["kind"], s["width"], s["height"], shapes[i].n_splats, batched)
        hit = cache.get(key)
        wanted = {_fmt(t, g) for t in cands for g in segs}
        if hit and wanted.issubset(hit["ms"].keys()):
            ms = {k: v for k, v in hit["ms"].items() if k in wanted}
            from_cache.append(True)
        else:
            ms = {}
            for t in cands:
                for g in segs:
                    ms[_fmt(t, g)] = _time_forward(shapes[i], scenes[i], s, sensor_poses[i], group_poses_per_sensor[i],
                                                   t, g, opts, pair_capacity, steps, warmup, device)
            merged = dict(hit["ms"]) if hit else {}
            merged.update(ms)
            cache.put(key, {"ms": merged})
            from_cache.append(False)
        timings[key] = ms
        per_sensor.append(ms)
    cache.save()
    # plan-wide segment length: smallest sum over sensors of each sensor's best tile at that L
    totals = {g: sum(min(ms[_fmt(t, g)] for t in cands) for ms in per_sensor) for g in segs}
    best_seg = pick(totals, PREFER_SEG, margin)
    prefer = PREFER_TILE if batched else PREFER_TILE_SINGLE
    chosen = []
    for s, ms in zip(sensors, per_sensor):
        at_seg = {t: ms[_fmt(t, best_seg)] for t in cands}
        chosen.append(pick(at_seg, prefer.get(s["kind"]), margin))
    return TuneResult(tiles=chosen, segment_pairs=best_seg, timings=timings, from_cache=from_cache)
