"""The block-wavefront schedule of the sweep (art_schedule, host only): the
properties that make it correct without atomics or cross-workgroup waits
(Sect. 3.1 single writers, Sect. 3.3 wave-front order).

* Every (bucket, block) pair is one work item, once: in one sweep each
  (bucket, cell) accumulator copy has exactly one writer.
* The blocks of a dominant axis tile the mesh: no cell is in two blocks, none
  is left out.
* Along every axis, the block downstream in the bucket's direction of travel
  is on the next wavefront, so every ray hand-off (rays leave a block only
  through its downstream faces, since no direction moves more than one
  column per slab) goes to a strictly later launch on the same stream.
"""
import itertools

import numpy as np
import pytest

from paper_1410_0763_amd import art


def _blocks(shape_xyz, a, depth):
    b, c = (1, 2) if a == 0 else ((0, 2) if a == 1 else (0, 1))
    N = list(shape_xyz)
    nblk = [0, 0, 0]
    nblk[a] = -(-N[a] // depth)
    nblk[b] = -(-N[b] // 8)
    nblk[c] = -(-N[c] // 8)
    return b, c, nblk


def _decode(block, a, nblk):
    b, c = (1, 2) if a == 0 else ((0, 2) if a == 1 else (0, 1))
    nbb, nbc = nblk[b], nblk[c]
    pb = block % nbb
    pc = (block // nbb) % nbc
    pa = block // (nbb * nbc)
    p = [0, 0, 0]
    p[a], p[b], p[c] = pa, pb, pc
    return tuple(p)


CASES = [((20, 13, 9), 5, 2), ((16, 16, 16), 6, 1), ((7, 31, 12), 3, 3), ((33, 9, 17), 8, 1),
         ((1, 1, 1), 6, 1), ((64, 40, 24), 6, 2)]


@pytest.mark.parametrize("shape,depth,subsets", CASES)
def test_schedule_single_writers_and_wavefront_order(shape, depth, subsets):
    items, nwave = art.schedule(shape, depth=depth, subsets=subsets)
    assert items.shape[1] == 3 and len(items) > 0
    w_of = {}
    for w, blk, bk in items:
        key = (int(bk), int(blk))
        assert key not in w_of, f"bucket {bk} block {blk} scheduled twice"
        w_of[key] = int(w)
    assert items[:, 0].max() == nwave - 1 and np.all(np.diff(items[:, 0]) >= 0)
    for a in range(3):
        b, c, nblk = _blocks(shape, a, depth)
        nall = nblk[0] * nblk[1] * nblk[2]
        for octant in range(8):
            for s in range(subsets):
                bk = (a * 8 + octant) * subsets + s
                got = sorted(blk for (kb, blk) in w_of if kb == bk)
                assert got == list(range(nall)), f"bucket {bk}: blocks missing or extra"
                for blk in range(nall):
                    p = _decode(blk, a, nblk)
                    w = w_of[(bk, blk)]
                    for ax in range(3):
                        step = -1 if (octant >> ax) & 1 else 1          # direction of travel
                        q = list(p)
                        q[ax] += step
                        if 0 <= q[ax] < nblk[ax]:
                            qb = (q[a] * nblk[c] + q[c]) * nblk[b] + q[b]
                            assert w_of[(bk, qb)] == w + 1, (bk, p, ax)
        # the blocks of axis a tile the mesh: count the cells each block covers
        cover = np.zeros(shape[::-1], dtype=np.int32)                   # [z][y][x]
        for blk in range(nall):
            p = _decode(blk, a, nblk)
            lo = [p[ax] * (depth if ax == a else 8) for ax in range(3)]
            hi = [min(shape[ax], lo[ax] + (depth if ax == a else 8)) for ax in range(3)]
            cover[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] += 1
        assert np.all(cover == 1), f"axis {a}: cells not covered exactly once"


@pytest.mark.parametrize("nside", [1, 2, 4, 8])
def test_directions_move_at_most_one_column_downstream(oracle_mod, nside):
    """Every HEALPix direction has |t_b|, |t_c| <= 1 for its dominant axis, so
    per slab a ray crosses at most one plane of each transverse axis, in the
    direction of its octant: hand-offs only cross downstream faces."""
    O = oracle_mod
    n = O.directions(nside)
    for d in range(len(n)):
        g = O.dir_geom(nside, d)
        assert abs(g["tb"]) <= 1.0 + 1e-12 and abs(g["tc"]) <= 1.0 + 1e-12
        assert g["tb"] == 0.0 or np.sign(g["tb"]) == np.sign(n[d, g["b"]])
        assert g["tc"] == 0.0 or np.sign(g["tc"]) == np.sign(n[d, g["c"]])
        assert np.sign(n[d, g["a"]]) == g["sig"]


def test_schedule_rejects_bad_arguments():
    with pytest.raises(art.ArtError):
        art.schedule((0, 4, 4))
    with pytest.raises(art.ArtError):
        art.schedule((8, 8, 8), depth=0)
    with pytest.raises(art.ArtError):
        art.schedule((8, 8, 8), interleave=5)
