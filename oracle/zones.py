"""Scene zones and the contents of a zone buffer -- TEST INFRASTRUCTURE ONLY.

Sec. III-A (large-scale scenes) cuts the scene by ground-plane (XOY)
position into square zones of 40 m and widens each by a relative padding of
25 %; at render time the Gaussians of the zone the vehicle moves into are
swapped into a second buffer.

Readings (the paper is silent on the details):
  - the ground plane is spanned by two chosen world axes (with y pointing
    down, the ground axes are x and z);
  - "25 % relative padding" widens every side of a zone by 25 % of the side
    (a 40 m zone covers a 60 m square);
  - a zone's Gaussians are the anchors whose centre lies in its padded square
    (the paper groups sensor frames, and a zone is reconstructed from its
    frames; with no training here, anchor position stands in for that);
  - intervals are half-open, [lo, hi), with
        lo = origin + (i - pad) * size,  hi = origin + ((i + 1) + pad) * size
    evaluated in IEEE double from the FP32 coordinate converted to double;
    zone id = j * nx + i;
  - a buffer of `capacity` anchors holds the zone's anchors in ascending
    order followed by padding elements of a fill value.

Plain numpy, one zone at a time, straight from these definitions.  Used only
by the tests.
"""
from __future__ import annotations

import numpy as np


def zone_bounds(origin, size, pad, i):
    """[lo, hi) of zone i along one axis (doubles, evaluated as defined above)."""
    di = float(i)
    return float(origin) + (di - float(pad)) * float(size), float(origin) + ((di + 1.0) + float(pad)) * float(size)


def members(xyz, axis, origin, size, pad, nx, ny, i, j):
    """Ascending anchor indices of zone (i, j)."""
    a = np.asarray(xyz[axis[0]], np.float32).astype(np.float64)
    b = np.asarray(xyz[axis[1]], np.float32).astype(np.float64)
    alo, ahi = zone_bounds(origin[0], size, pad, i)
    blo, bhi = zone_bounds(origin[1], size, pad, j)
    inside = (alo <= a) & (a < ahi) & (blo <= b) & (b < bhi)
    return np.nonzero(inside)[0].astype(np.uint32)


def partition(xyz, axis, origin, size, pad, nx, ny):
    """CSR lists of every zone: (offsets [nx*ny + 1] uint32, index uint32)."""
    lists = []
    for j in range(ny):
        for i in range(nx):
            lists.append(members(xyz, axis, origin, size, pad, nx, ny, i, j))
    offsets = np.zeros(nx * ny + 1, np.int64)
    offsets[1:] = np.cumsum([len(x) for x in lists])
    index = np.concatenate(lists) if lists else np.zeros(0, np.uint32)
    return offsets.astype(np.uint32), index.astype(np.uint32)


def zone_buffer(host_rows, anchors, capacity, fill=None):
    """Contents of one field in a zone buffer: host_rows [rows, n, ...] gathered at
    `anchors` into the first len(anchors) slots, `fill` (default zeros) after."""
    host_rows = np.asarray(host_rows)
    anchors = np.asarray(anchors, np.int64)
    if anchors.size > capacity:
        raise ValueError("zone larger than the buffer")
    out_shape = (host_rows.shape[0], capacity) + host_rows.shape[2:]
    out = np.zeros(out_shape, host_rows.dtype)
    if fill is not None:
        out[:, anchors.size:] = fill
    out[:, :anchors.size] = host_rows[:, anchors]
    return out
