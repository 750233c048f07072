"""Pins of the zone oracle (oracle/zones.py) against facts fixed by the
definition of padded square zones (Sec. III-A, large-scale scenes: 40 m zones
with 25 % relative padding), independent of the oracle's own arithmetic:

  - exact rational membership (fractions.Fraction) on random and boundary
    points: the oracle's double evaluation agrees;
  - with no padding the zones tile the grid: every point inside it lies in
    exactly the zone floor((a - origin) / size), points outside in none;
  - closed-form membership counts with 25 % padding: 1 zone in a zone's core,
    2 within 10 m of one interior edge, 4 near an interior corner;
  - half-open intervals: a point on a low bound is in, on a high bound out;
  - zone ids run j * nx + i (an asymmetric grid and swapped axes);
  - a buffer holds the zone's anchors in ascending order, then the fill.
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import zones as Z


def exact_members(xyz, axis, origin, size, pad, nx, ny):
    """Brute force with exact rationals: zone lists of every zone."""
    out = [[] for _ in range(nx * ny)]
    a_all = np.asarray(xyz[axis[0]], np.float32)
    b_all = np.asarray(xyz[axis[1]], np.float32)
    o0, o1, s, p = Fraction(origin[0]), Fraction(origin[1]), Fraction(size), Fraction(pad)
    for n in range(a_all.size):
        a, b = Fraction(float(a_all[n])), Fraction(float(b_all[n]))
        for j in range(ny):
            if not (o1 + (j - p) * s <= b < o1 + (j + 1 + p) * s):
                continue
            for i in range(nx):
                if o0 + (i - p) * s <= a < o0 + (i + 1 + p) * s:
                    out[j * nx + i].append(n)
    return out


def lists_of(offsets, index):
    return [index[offsets[z]:offsets[z + 1]].tolist() for z in range(len(offsets) - 1)]


def _cloud(rng, n, lo, hi):
    xyz = np.zeros((3, n), np.float32)
    xyz[0] = rng.uniform(lo[0], hi[0], n)
    xyz[1] = rng.uniform(-3, 3, n)
    xyz[2] = rng.uniform(lo[1], hi[1], n)
    return xyz


def test_double_evaluation_matches_exact_rationals_on_random_and_boundary_points():
    rng = np.random.default_rng(0)
    grid = dict(axis=(0, 2), origin=(-20.0, -20.0), size=40.0, pad=0.25, nx=2, ny=4)
    xyz = _cloud(rng, 3000, (-40, -40), (80, 160))
    # points on and next to every padded bound (-30, 30, 10, 70, ... along both axes)
    bounds = [-20 + 40 * i - 10 for i in range(6)] + [-20 + 40 * (i + 1) + 10 for i in range(6)]
    extra = []
    for v in bounds:
        for w in (np.float32(v), np.nextafter(np.float32(v), np.float32(-1e9)),
                  np.nextafter(np.float32(v), np.float32(1e9))):
            extra.append((w, 0.0, 5.0))
            extra.append((5.0, 0.0, w))
    xyz = np.concatenate([xyz, np.array(extra, np.float32).T], 1)
    offs, idx = Z.partition(xyz, **grid)
    assert lists_of(offs, idx) == exact_members(xyz, **grid)


def test_without_padding_zones_tile_the_grid():
    rng = np.random.default_rng(1)
    nx, ny, size, o = 3, 2, 40.0, (-60.0, 0.0)
    xyz = _cloud(rng, 4000, (-100, -30), (100, 110))
    offs, idx = Z.partition(xyz, (0, 2), o, size, 0.0, nx, ny)
    count = np.bincount(idx, minlength=xyz.shape[1])
    ia = np.floor((xyz[0].astype(np.float64) - o[0]) / size).astype(int)
    jb = np.floor((xyz[2].astype(np.float64) - o[1]) / size).astype(int)
    in_grid = (ia >= 0) & (ia < nx) & (jb >= 0) & (jb < ny)
    assert np.all(count[in_grid] == 1)
    assert np.all(count[~in_grid] == 0)
    zone = np.full(xyz.shape[1], -1)
    for z in range(nx * ny):
        zone[idx[offs[z]:offs[z + 1]]] = z
    assert np.array_equal(zone[in_grid], (jb * nx + ia)[in_grid])


@pytest.mark.parametrize("a,b,count", [
    (20.0, 20.0, 1),     # core of zone (0, 0) of a 2 x 2 grid with origin (0, 0)
    (35.0, 20.0, 2),     # 5 m before the interior edge a = 40: zones (0,0), (1,0)
    (45.0, 20.0, 2),     # 5 m after it
    (49.9, 20.0, 2),     # just inside zone (0,0)'s padded edge at 50
    (50.0, 20.0, 1),     # on it: out of zone (0,0), in zone (1,0) only
    (29.99, 20.0, 1),    # zone (1,0)'s padded low edge is 30
    (30.0, 20.0, 2),     # on it: in
    (38.0, 42.0, 4),     # near the interior corner (40, 40)
    (-9.0, 20.0, 1),     # outer padding of zone (0,0) (its low edge is -10)
    (-10.0, 20.0, 1),    # on the outer low edge: in
    (-10.01, 20.0, 0),   # beyond: outside every zone
    (90.0, 20.0, 0),     # high edge of zone (1,0) is 90 (half-open): out
])
def test_closed_form_membership_counts_with_25_percent_padding(a, b, count):
    xyz = np.array([[a], [0.0], [b]], np.float32)
    offs, idx = Z.partition(xyz, (0, 2), (0.0, 0.0), 40.0, 0.25, 2, 2)
    assert idx.size == count


def test_zone_ids_and_axis_order():
    # 3 x 2 grid; a point in the core of zone (i=2, j=1) has id 1 * 3 + 2 = 5
    xyz = np.array([[100.0], [7.0], [60.0]], np.float32)
    offs, idx = Z.partition(xyz, (0, 2), (0.0, 0.0), 40.0, 0.25, 3, 2)
    assert [z for z in range(6) if offs[z + 1] > offs[z]] == [5]
    # swapping the axes swaps the roles of the coordinates: (60, 100) is zone (i=1, j=2) of a 2 x 3 grid = 2 * 2 + 1
    offs, idx = Z.partition(xyz, (2, 0), (0.0, 0.0), 40.0, 0.25, 2, 3)
    assert [z for z in range(6) if offs[z + 1] > offs[z]] == [5]
    # the vertical axis (y) as a ground axis moves the point out of the grid
    offs, idx = Z.partition(xyz, (0, 1), (0.0, 0.0), 40.0, 0.25, 3, 2)
    assert [z for z in range(6) if offs[z + 1] > offs[z]] == [2]


def test_padded_square_side_is_one_and_a_half_zones():
    # 25 % per side: zone (1, 1) of a 3x3 grid with origin 0 covers [30, 90) on both axes
    g = np.linspace(0.0, 120.0, 1201, dtype=np.float32)
    A, B = np.meshgrid(g, g)
    xyz = np.stack([A.ravel(), np.zeros(A.size, np.float32), B.ravel()])
    offs, idx = Z.partition(xyz, (0, 2), (0.0, 0.0), 40.0, 0.25, 3, 3)
    m = idx[offs[4]:offs[5]]
    a, b = xyz[0, m], xyz[2, m]
    assert a.min() == 30.0 and b.min() == 30.0
    assert a.max() == np.float32(89.9) and b.max() == np.float32(89.9)


def test_buffer_contents():
    rng = np.random.default_rng(2)
    host = rng.standard_normal((3, 50)).astype(np.float32)
    anchors = np.array([3, 7, 8, 41], np.uint32)
    buf = Z.zone_buffer(host, anchors, 6, fill=np.float32(9.0))
    assert buf.shape == (3, 6)
    assert np.array_equal(buf[:, :4], host[:, [3, 7, 8, 41]])
    assert np.all(buf[:, 4:] == 9.0)
    # 64-byte elements (rows of a [n, 32] u16 array): gathered whole
    feat = rng.integers(0, 65535, (1, 50, 32)).astype(np.uint16)
    fb = Z.zone_buffer(feat, anchors, 5)
    assert np.array_equal(fb[0, :4], feat[0, anchors]) and np.all(fb[0, 4] == 0)
    # without padding, the zones' buffers are a permutation of the whole scene
    xyz = _cloud(rng, 500, (0, 0), (80, 80))
    offs, idx = Z.partition(xyz, (0, 2), (0.0, 0.0), 40.0, 0.0, 2, 2)
    parts = [Z.zone_buffer(xyz, idx[offs[z]:offs[z + 1]], int(offs[z + 1] - offs[z])) for z in range(4)]
    assert np.array_equal(np.concatenate(parts, 1)[:, np.argsort(idx, kind="stable")], xyz)
