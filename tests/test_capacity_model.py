"""Host-side bounds model of the pair pipeline under capacity overflow (CPU only).

The pair emission, the tile sort, the tile ranges and the compositing queue
index the pair arrays (capacity `cap` entries each) as follows:

  tile-count scan  offs[j] = saturating (2^32 - 1) exclusive prefix of the
                   per-surfel tile counts in depth order, formed in 64 bits;
                   total = saturating sum, overflow flagged when total > cap
  emission         wave w (surfels j0 .. j0 + 63) writes pair slots
                   q in [offs[j0], min(max_j(offs[j] + cnt[j]), cap)), the
                   slot's surfel being the last lane whose offset is <= q
  tile sort        n = min(total, cap) keys
  ranges           slots [0, n); a tile id >= n_tiles is skipped
  queue            per tile [start, end) inside [0, n)

This model runs that arithmetic on adversarial tile counts (totals far above
the capacity, 32-bit wrap-around of the true total) and checks that every
written slot is below the capacity, that every slot below min(total, cap) is
written exactly once by the surfel whose pairs it holds (so the sort and the
ranges only read written slots), and that overflow is always reported.
"""
import numpy as np
import pytest

U32 = (1 << 32) - 1


def scan(counts):
    """offs (saturating uint32), total (saturating) as the device scan forms them."""
    c = counts.astype(np.uint64)
    incl = np.cumsum(c, dtype=np.uint64)  # exact: inputs < 2^32, at most 2^20 of them
    excl = incl - c
    offs = np.minimum(excl, U32).astype(np.uint64)
    total = int(min(int(incl[-1]) if incl.size else 0, U32))
    return offs, total


def emit_model(counts, cap):
    """Slots written per wave and the surfel each slot is attributed to."""
    n = counts.size
    offs, total = scan(counts)
    written = np.zeros(cap, np.int64)
    owner = np.full(cap, -1, np.int64)
    for j0 in range(0, n, 64):
        js = np.arange(j0, min(j0 + 64, n))
        o = offs[js]
        cnt = counts[js].astype(np.uint64)
        start = int(o[0])
        end = min(int((o + cnt).max()), cap)
        lo = o - o[0]
        for q in range(start, end):
            k = q - start
            src = int(np.nonzero(lo <= k)[0].max())  # last lane whose first pair is <= k
            assert q < cap
            written[q] += 1
            owner[q] = js[src]
    return offs, total, written, owner


@pytest.mark.parametrize("seed,n,mean_tiles,cap", [(0, 500, 3, 1000), (1, 300, 40, 5000), (2, 64, 2, 100),
                                                     (3, 1000, 1, 100000), (4, 129, 7, 1)])
def test_emission_stays_inside_the_capacity(seed, n, mean_tiles, cap):
    rng = np.random.default_rng(seed)
    counts = rng.poisson(mean_tiles, n).astype(np.uint32)
    counts[rng.random(n) < 0.2] = 0  # invisible surfels
    offs, total, written, owner = emit_model(counts, cap)
    true_total = int(counts.astype(np.uint64).sum())
    assert total == min(true_total, U32)
    assert (total > cap) == (true_total > cap)  # the overflow flag
    m = min(true_total, cap)
    assert (written[:m] == 1).all() and (written[m:] == 0).all()
    # a slot holds one of its surfel's pairs
    o = offs[owner[:m]].astype(np.int64)
    q = np.arange(m)
    assert ((o <= q) & (q < o + counts[owner[:m]].astype(np.int64))).all()


def test_wrapped_32_bit_total_is_still_an_overflow():
    # true total 2^32 + 5: a 32-bit sum would wrap to 5 and pass for a tiny frame
    counts = np.array([U32 - 10, 7, 8, 0, 1], np.uint64).astype(np.uint32)
    cap = 64
    offs, total, written, owner = emit_model(counts, cap)
    assert total == U32 and total > cap
    assert (written == 1).all()
    assert (owner == 0).all()  # the first surfel's pairs fill the capacity


def test_ranges_and_queue_read_only_written_slots():
    rng = np.random.default_rng(7)
    n_tiles = 37
    counts = rng.poisson(5, 400).astype(np.uint32)
    cap = 900
    offs, total, written, owner = emit_model(counts, cap)
    n = min(total, cap)
    assert written[:n].all()
    # ranges over slots [0, n) of tile ids in [0, n_tiles): every range lies inside [0, n)
    tiles = np.sort(rng.integers(0, n_tiles, n))
    starts = np.searchsorted(tiles, np.arange(n_tiles), "left")
    ends = np.searchsorted(tiles, np.arange(n_tiles), "right")
    assert (starts >= 0).all() and (ends <= n).all()
