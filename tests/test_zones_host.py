"""Host-side zone partition of the C-ABI (gs_zone_partition: host code, no HIP
call) against the zone oracle, bit for bit: same lists, same order.  Covers
random clouds over several grids, points on and next to every padded bound,
a cloud large enough to split over host threads, NaN coordinates, the size
query and the error paths."""
import ctypes

import numpy as np
import pytest

from oracle import zones as Z
from paper_2503_11731_amd import _lib as L
from paper_2503_11731_amd import zones as gz


def _cloud(rng, n, lo, hi):
    xyz = np.zeros((3, n), np.float32)
    xyz[0] = rng.uniform(lo[0], hi[0], n)
    xyz[1] = rng.uniform(-3, 3, n)
    xyz[2] = rng.uniform(lo[1], hi[1], n)
    return xyz


GRIDS = [
    gz.ZoneGrid(axis=(0, 2), origin=(-20.0, -20.0), size=40.0, pad=0.25, nx=1, ny=5),
    gz.ZoneGrid(axis=(0, 2), origin=(-50.0, 3.5), size=40.0, pad=0.25, nx=3, ny=4),
    gz.ZoneGrid(axis=(2, 0), origin=(0.1, -7.3), size=13.7, pad=0.37, nx=5, ny=2),
    gz.ZoneGrid(axis=(0, 1), origin=(0.0, 0.0), size=1.0, pad=0.0, nx=7, ny=3),
    gz.ZoneGrid(axis=(1, 2), origin=(-1.0, -1.0), size=0.5, pad=1.0, nx=2, ny=2),
]


def _oracle(xyz, g):
    return Z.partition(xyz, g.axis, g.origin, g.size, g.pad, g.nx, g.ny)


@pytest.mark.parametrize("gi", range(len(GRIDS)))
def test_partition_matches_oracle(gi):
    g = GRIDS[gi]
    rng = np.random.default_rng(10 + gi)
    xyz = rng.uniform(-80, 200, (3, 5000)).astype(np.float32)
    # points on and next to padded bounds along both ground axes
    ext = []
    for k in range(2):
        for i in range(-1, max(g.nx, g.ny) + 2):
            for v in Z.zone_bounds(g.origin[k], g.size, g.pad, i):
                f = np.float32(v)
                for w in (f, np.nextafter(f, np.float32(-np.inf)), np.nextafter(f, np.float32(np.inf))):
                    p = np.float32(rng.uniform(-5, 5, 3))
                    p[g.axis[k]] = w
                    ext.append(p)
    xyz = np.concatenate([xyz, np.array(ext, np.float32).T], 1)
    offs, idx = gz.partition(xyz, g)
    ro, ri = _oracle(xyz, g)
    assert np.array_equal(offs, ro)
    assert np.array_equal(idx, ri)


def test_partition_large_cloud_split_over_threads():
    g = GRIDS[0]
    rng = np.random.default_rng(3)
    xyz = _cloud(rng, 400_000, (-14, -20), (14, 180))
    offs, idx = gz.partition(xyz, g)
    ro, ri = _oracle(xyz, g)
    assert np.array_equal(offs, ro) and np.array_equal(idx, ri)
    # every zone list ascending; padded zones overlap
    for z in range(g.n_zones):
        lst = idx[offs[z]:offs[z + 1]]
        assert np.all(np.diff(lst.astype(np.int64)) > 0)
    assert idx.size > xyz.shape[1]


def test_partition_nan_and_empty():
    g = GRIDS[1]
    xyz = np.array([[np.nan, 0.0, 1.0], [0, 0, 0], [5.0, np.nan, 10.0]], np.float32)
    offs, idx = gz.partition(xyz, g)
    ro, ri = _oracle(xyz, g)
    assert np.array_equal(offs, ro) and np.array_equal(idx, ri)
    assert 0 not in idx.tolist() and 1 not in idx.tolist()
    offs, idx = gz.partition(np.zeros((3, 0), np.float32), g)
    assert idx.size == 0 and np.all(offs == 0)


def _call(grid, xyz, n, offs, index, cap):
    lib = L.load()
    total = ctypes.c_int64(-1)
    st = lib.gs_zone_partition(ctypes.byref(grid) if grid is not None else None,
                               xyz.ctypes.data if xyz is not None else None, n,
                               offs.ctypes.data if offs is not None else None,
                               index.ctypes.data if index is not None else None, cap, ctypes.byref(total))
    return st, total.value


def test_partition_errors():
    xyz = np.zeros((3, 4), np.float32)
    offs = np.zeros(6, np.uint32)
    ok = gz.ZoneGrid(nx=5, ny=1)._c()
    # size query
    st, total = _call(ok, xyz, 4, offs, None, 0)
    assert st == L.GS_OK and total == 4
    # capacity too small: total still reported
    idx = np.zeros(2, np.uint32)
    st, total = _call(ok, xyz, 4, offs, idx, 2)
    assert st == L.GS_ERR_CAPACITY and total == 4
    bad = [gz.ZoneGrid(axis=(0, 0)), gz.ZoneGrid(axis=(0, 3)), gz.ZoneGrid(size=0.0), gz.ZoneGrid(size=float("nan")),
           gz.ZoneGrid(pad=-0.1), gz.ZoneGrid(pad=1.5), gz.ZoneGrid(nx=0), gz.ZoneGrid(nx=2048, ny=1024),
           gz.ZoneGrid(origin=(float("inf"), 0.0))]
    for g in bad:
        st, _ = _call(g._c(), xyz, 4, offs, None, 0)
        assert st == L.GS_ERR_INVALID_ARG, g
    assert _call(None, xyz, 4, offs, None, 0)[0] == L.GS_ERR_INVALID_ARG
    assert _call(ok, None, 4, offs, None, 0)[0] == L.GS_ERR_INVALID_ARG
    assert _call(ok, xyz, -1, offs, None, 0)[0] == L.GS_ERR_INVALID_ARG
    assert _call(ok, xyz, 4, None, None, 0)[0] == L.GS_ERR_INVALID_ARG
    assert _call(ok, xyz, 4, offs, None, 5)[0] == L.GS_ERR_INVALID_ARG
