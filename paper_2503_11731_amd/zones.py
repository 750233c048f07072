"""Python binding of the scene zones and their double-buffered swap-in.

Sec. III-A (large-scale scenes): anchors are grouped by ground-plane position
into square zones (40 m, padded by 25 % of the side on every side); at render
time two device buffers hold zones, and the zone the vehicle is about to
enter is gathered and copied into one while the other is rendered.  The
partition, the gather into pinned staging and the host-to-device copies run
in libgs2d.so (a swap-in thread of its own); this module marshals arguments
and lays out the two device anchor sets.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib as L
from .decode import Decoder


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


@dataclass(frozen=True)
class ZoneGrid:
    """Square zones of side `size` over the ground plane spanned by world axes
    `axis`, zone (i, j) with its low corner at origin + (i, j) * size, widened
    on every side by pad * size.  Zone id = j * nx + i."""
    axis: tuple = (0, 2)
    origin: tuple = (0.0, 0.0)
    size: float = 40.0
    pad: float = 0.25
    nx: int = 1
    ny: int = 1

    def _c(self):
        return L.ZoneGrid((ctypes.c_int32 * 2)(*self.axis), (ctypes.c_double * 2)(*self.origin), float(self.size),
                          float(self.pad), int(self.nx), int(self.ny))

    @property
    def n_zones(self) -> int:
        return self.nx * self.ny

    def zone_of(self, a: float, b: float) -> int:
        """Zone whose unpadded square holds ground point (a, b) (-1 outside the grid)."""
        i = int(np.floor((a - self.origin[0]) / self.size))
        j = int(np.floor((b - self.origin[1]) / self.size))
        if 0 <= i < self.nx and 0 <= j < self.ny:
            return j * self.nx + i
        return -1


def partition(xyz: np.ndarray, grid: ZoneGrid):
    """Anchor lists of every zone: (offsets [Z+1] u32, index [total] u32), via gs_zone_partition."""
    lib = L.load()
    xyz = np.ascontiguousarray(xyz, dtype=np.float32)
    if xyz.ndim != 2 or xyz.shape[0] != 3:
        raise ValueError("xyz must be [3, n]")
    n = int(xyz.shape[1])
    g = grid._c()
    offs = np.zeros(grid.n_zones + 1, np.uint32)
    total = ctypes.c_int64()
    L.check(lib.gs_zone_partition(ctypes.byref(g), xyz.ctypes.data, n, offs.ctypes.data, None, 0,
                                  ctypes.byref(total)))
    index = np.zeros(max(int(total.value), 1), np.uint32)
    L.check(lib.gs_zone_partition(ctypes.byref(g), xyz.ctypes.data, n, offs.ctypes.data, index.ctypes.data,
                                  index.size, ctypes.byref(total)))
    return offs, index[:int(total.value)]


@dataclass
class Field:
    """One array that moves with a zone (gs_zone_field).  host: a C-contiguous
    numpy array kept alive by the stream; device: the two destination tensors."""
    host: np.ndarray
    device: tuple
    rows: int
    elem_bytes: int
    host_stride: int = 0
    device_stride: int = 0
    per_zone: bool = False
    fill: bytes | None = None


class ZoneStream:
    """gs_zone_stream: two device buffers filled by the library's swap-in thread."""

    def __init__(self, offsets: np.ndarray, index: np.ndarray, capacity: int, n_anchors: int, fields: list,
                 threads: int = 4):
        self.lib = L.load()
        self._offs = np.ascontiguousarray(offsets, np.uint32)
        self._index = np.ascontiguousarray(index, np.uint32)
        self._fields = fields
        self._fills = []
        cf = (L.ZoneField * len(fields))()
        for i, f in enumerate(fields):
            if not f.host.flags.c_contiguous:
                raise ValueError("zone field host arrays must be C-contiguous")
            for t in f.device:
                if not t.is_contiguous():
                    raise ValueError("zone field device tensors must be contiguous")
            fill = None
            if f.fill is not None:
                if len(f.fill) != f.elem_bytes:
                    raise ValueError("fill must hold elem_bytes bytes")
                fill = ctypes.create_string_buffer(bytes(f.fill), len(f.fill))
                self._fills.append(fill)
            cf[i] = L.ZoneField(f.host.ctypes.data, int(f.host_stride), (ctypes.c_void_p * 2)(
                f.device[0].data_ptr(), f.device[1].data_ptr()), int(f.device_stride), int(f.rows),
                int(f.elem_bytes), int(bool(f.per_zone)), ctypes.addressof(fill) if fill is not None else None)
        self._cf = cf
        d = L.ZoneStreamDesc(len(self._offs) - 1, self._offs.ctypes.data, self._index.ctypes.data if self._index.size
                             else None, int(capacity), int(n_anchors), len(fields), cf, int(threads))
        h = ctypes.c_void_p()
        L.check(self.lib.gs_zone_stream_create(ctypes.byref(d), ctypes.byref(h)))
        self.h = h
        self.capacity = int(capacity)

    def prefetch(self, zone: int, buffer: int):
        L.check(self.lib.gs_zone_stream_prefetch(self.h, int(zone), int(buffer)))

    def acquire(self, buffer: int):
        """Orders the current stream after the buffer's last upload; returns (zone, anchor count)."""
        z, c = ctypes.c_int32(), ctypes.c_int64()
        L.check(self.lib.gs_zone_stream_acquire(self.h, int(buffer), _stream(), ctypes.byref(z), ctypes.byref(c)))
        return int(z.value), int(c.value)

    def release(self, buffer: int):
        """The buffer's current contents are no longer read after the work enqueued so far."""
        L.check(self.lib.gs_zone_stream_release(self.h, int(buffer), _stream()))

    def stats(self, buffer: int) -> dict:
        s = L.ZoneSwapStats()
        L.check(self.lib.gs_zone_stream_stats(self.h, int(buffer), ctypes.byref(s)))
        return dict(zone=s.zone, count=s.count, bytes=s.bytes, gather_ms=s.gather_ms, upload_ms=s.upload_ms)

    def close(self):
        if getattr(self, "h", None):
            self.lib.gs_zone_stream_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# padding anchors: zero scaling (their surfels have zero extent and are culled), parked far away
PAD_XYZ = np.float32(1.0e9).tobytes()


class ZonedAnchors:
    """Two device anchor sets for one sensor kind, streamed zone by zone.

    Buffer layout (per buffer, A = capacity + resident anchors):
      anchors [0, capacity)      the zone's static anchors, then padding
      anchors [capacity, A)      resident actor groups (never swapped)
      MLP group 0                the zone's own MLP; groups 1.. the actors'
    static: dict of host arrays over all static anchors (xyz [3,S] f32,
    scaling [S] f32, offsets [3,K,S] f32, feat [S,32] bf16 bits u16);
    zone_mlps: per zone dict(w1, b1, w2, b2) (f32, w bf16-representable);
    actors: None or dict(xyz, scaling, offsets, feat, group_offsets (from 0),
    mlps).
    """

    def __init__(self, static: dict, zone_mlps: list, grid: ZoneGrid, lidar: bool, device="cuda",
                 actors: dict | None = None, capacity: int | None = None, threads: int = 4, offsets=None, index=None):
        def c(a, dt):
            return np.ascontiguousarray(a, dtype=dt)

        self.grid = grid
        self.lidar = bool(lidar)
        xyz, scaling = c(static["xyz"], np.float32), c(static["scaling"], np.float32)
        offs3, feat = c(static["offsets"], np.float32), c(static["feat"], np.uint16)
        S, K = int(xyz.shape[1]), int(offs3.shape[1])
        if offsets is None:
            offsets, index = partition(xyz, grid)
        counts = np.diff(offsets.astype(np.int64))
        C = int(capacity if capacity is not None else max(int(counts.max()), 1))
        na = 0 if actors is None else int(actors["xyz"].shape[1])
        A = C + na
        J = 9 if lidar else 10
        G = 1 + (0 if actors is None else len(actors["mlps"]))
        self.counts, self.capacity, self.K, self.J = counts, C, K, J
        dev = torch.device(device)

        def bf16_bits(w):
            return (np.ascontiguousarray(w, np.float32).view(np.uint32) >> 16).astype(np.uint16)

        def dbuf():
            z = lambda *shape: torch.zeros(shape, dtype=torch.float32, device=dev)
            bz = lambda *shape: torch.zeros(shape, dtype=torch.bfloat16, device=dev)
            return dict(xyz=z(3, A), scaling=z(A), offsets=z(3, K, A), feat=bz(A, 32), w1=bz(G, 32, 35), b1=z(G, 32),
                        w2=bz(G, K * J, 32), b2=z(G, K * J))

        self.buf = [dbuf(), dbuf()]
        goff = [0, C]
        if actors is not None:
            ag = [int(x) for x in actors["group_offsets"]]
            goff += [C + x for x in ag[1:]]
            for b in self.buf:
                b["xyz"][:, C:] = torch.from_numpy(c(actors["xyz"], np.float32))
                b["scaling"][C:] = torch.from_numpy(c(actors["scaling"], np.float32))
                b["offsets"][:, :, C:] = torch.from_numpy(c(actors["offsets"], np.float32))
                b["feat"][C:] = torch.from_numpy(c(actors["feat"], np.uint16).view(np.int16)).view(torch.bfloat16)
                for g, m in enumerate(actors["mlps"]):
                    b["w1"][1 + g] = torch.from_numpy(bf16_bits(m["w1"]).view(np.int16)).view(torch.bfloat16)
                    b["w2"][1 + g] = torch.from_numpy(bf16_bits(m["w2"]).view(np.int16)).view(torch.bfloat16)
                    b["b1"][1 + g] = torch.from_numpy(c(m["b1"], np.float32))
                    b["b2"][1 + g] = torch.from_numpy(c(m["b2"], np.float32))
        self.group_offsets = goff
        self.decoders = [Decoder(b["xyz"], b["scaling"], b["offsets"], b["feat"], b["w1"], b["b1"], b["w2"], b["b2"],
                                 goff, lidar) for b in self.buf]
        # per-zone MLP blocks (group 0 of a buffer)
        self._w1 = np.stack([bf16_bits(m["w1"]) for m in zone_mlps])
        self._b1 = np.stack([c(m["b1"], np.float32) for m in zone_mlps])
        self._w2 = np.stack([bf16_bits(m["w2"]) for m in zone_mlps])
        self._b2 = np.stack([c(m["b2"], np.float32) for m in zone_mlps])
        if len(zone_mlps) != grid.n_zones:
            raise ValueError("one MLP per zone")
        self._host = (xyz, scaling, offs3, feat)
        pair = lambda k: (self.buf[0][k], self.buf[1][k])
        fields = [
            Field(xyz, pair("xyz"), 3, 4, S, A, fill=PAD_XYZ),
            Field(scaling, pair("scaling"), 1, 4, S, A),
            Field(offs3, pair("offsets"), 3 * K, 4, S, A),
            Field(feat, pair("feat"), 1, 64, S, A),
            Field(self._w1, pair("w1"), 1, self._w1[0].nbytes, per_zone=True),
            Field(self._b1, pair("b1"), 1, self._b1[0].nbytes, per_zone=True),
            Field(self._w2, pair("w2"), 1, self._w2[0].nbytes, per_zone=True),
            Field(self._b2, pair("b2"), 1, self._b2[0].nbytes, per_zone=True),
        ]
        torch.cuda.synchronize(dev)
        self.stream = ZoneStream(offsets, index, C, S, fields, threads=threads)
        self.offsets, self.index = offsets, index

    @property
    def n_surfels(self) -> int:
        return self.decoders[0].A * self.K

    def close(self):
        self.stream.close()
