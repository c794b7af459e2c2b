"""Pins of the oracle's ROI-with-holes rectangles (thesis Section 5.3: the
framebuffer analysis can detect holes). Independent facts: hand-worked
grids (tests/golden/roi_rects.txt); on random grids, properties that fix
the decomposition without restating it (disjoint rectangles whose union is
exactly the occupied cells, every rectangle row a maximal run of its grid
row, no rectangle extendable up or down by an equal run, start order, the
bounding-box fallback); and the compositing identity: compositing the
rectangles' pixels as contributors gives the composite of the full frames,
since everything left out is clear."""
import numpy as np
import pytest

import oracle
from conftest import read_golden

F = 0xFFFFFFFF


def _sec(name):
    return [[int(t) for t in row] for row in read_golden("roi_rects.txt")[name]]


def test_hand_worked_grids():
    a = np.array(_sec("a_grid"), np.uint8)
    assert oracle.roi_rects(a, (4, 4), 16, 15) == [tuple(r) for r in _sec("a_rects")]
    b = np.array(_sec("b_grid"), np.uint8)
    assert oracle.roi_rects(b, (10, 10), 30, 30) == [tuple(r) for r in _sec("b_rects")]
    assert oracle.roi_rects(b, (10, 10), 30, 30, max_rects=3) == [tuple(r) for r in _sec("b_bbox")]
    assert oracle.roi_rects(b, (10, 10), 30, 30, max_rects=4) == [tuple(r) for r in _sec("b_rects")]


def _runs(row):
    """Maximal runs of ones of a 0/1 row as (first, end)."""
    out, c = [], 0
    while c < len(row):
        if row[c]:
            e = c
            while e < len(row) and row[e]:
                e += 1
            out.append((c, e))
            c = e
        else:
            c += 1
    return out


@pytest.mark.parametrize("seed", range(40))
def test_random_grids_properties(seed):
    rng = np.random.default_rng(seed)
    gh, gw = int(rng.integers(1, 12)), int(rng.integers(1, 12))
    p = rng.uniform(0.2, 0.9)
    g = (rng.random((gh, gw)) < p).astype(np.uint8)
    if seed % 5 == 0:   # blocky grids: runs that repeat over several rows
        g = np.repeat(np.repeat((rng.random((max(1, gh // 3), max(1, gw // 2))) < 0.6), 3, 0), 2, 1)[:gh, :gw].astype(np.uint8)
        gh, gw = g.shape
    cw, ch = int(rng.integers(1, 9)), int(rng.integers(1, 9))
    w = gw * cw - int(rng.integers(0, cw))
    h = gh * ch - int(rng.integers(0, ch))
    rects = oracle.roi_rects(g, (cw, ch), w, h, max_rects=10_000)
    cov = np.zeros((gh, gw), np.int32)
    cells = []
    for x, y, rw, rh in rects:
        assert rw > 0 and rh > 0 and x % cw == 0 and y % ch == 0
        c0, r0 = x // cw, y // ch
        c1 = min(gw, -(-(x + rw) // cw)) if x + rw < w else gw
        r1 = min(gh, -(-(y + rh) // ch)) if y + rh < h else gh
        # clipped to the image, whole cells otherwise
        assert x + rw == min(c1 * cw, w) and y + rh == min(r1 * ch, h)
        cov[r0:r1, c0:c1] += 1
        cells.append((c0, r0, c1, r1))
    assert (cov == g).all()                    # disjoint, exactly the occupied cells
    for c0, r0, c1, r1 in cells:
        for r in range(r0, r1):
            assert (c0, c1) in _runs(g[r])     # each rectangle row is a maximal run
        assert r0 == 0 or (c0, c1) not in _runs(g[r0 - 1])
        assert r1 == gh or (c0, c1) not in _runs(g[r1])
    assert cells == sorted(cells, key=lambda t: (t[1], t[0]))   # numbered as they start
    # fallback: fewer allowed rectangles than there are -> the bounding box
    if len(rects) > 1:
        bb = oracle.roi_rects(g, (cw, ch), w, h, max_rects=len(rects) - 1)
        ys, xs = np.nonzero(g)
        x0, y0 = xs.min() * cw, ys.min() * ch
        assert bb == [(x0, y0, min((xs.max() + 1) * cw, w) - x0, min((ys.max() + 1) * ch, h) - y0)]
    if not g.any():
        assert rects == []


def test_rect_pieces_composite_like_full_frames():
    """Depth compositing of each image's rectangles as separate contributors
    (in image order) equals compositing the full frames: the cells left out
    hold only clear pixels, which never win."""
    rng = np.random.default_rng(7)
    H, W, cell = 40, 56, (8, 8)
    cols, deps, pieces_c, pieces_d, pieces_roi = [], [], [], [], []
    for i in range(4):
        d = np.full((H, W), F, np.uint32)
        c = np.zeros((H, W), np.uint32)
        for _ in range(3):   # separate blobs: a ROI with holes
            y0, x0 = int(rng.integers(0, H - 6)), int(rng.integers(0, W - 6))
            hh, ww = int(rng.integers(2, 12)), int(rng.integers(2, 14))
            d[y0:y0 + hh, x0:x0 + ww] = rng.integers(0, 50, (min(hh, H - y0), min(ww, W - x0)))
            c[y0:y0 + hh, x0:x0 + ww] = rng.integers(1, 2 ** 32, (min(hh, H - y0), min(ww, W - x0)), dtype=np.uint64)
        cols.append(c)
        deps.append(d)
        g = oracle.roi_grid(d, cell)
        for x, y, rw, rh in oracle.roi_rects(g, cell, W, H):
            pieces_c.append(np.ascontiguousarray(c[y:y + rh, x:x + rw]))
            pieces_d.append(np.ascontiguousarray(d[y:y + rh, x:x + rw]))
            pieces_roi.append((x, y, rw, rh))
        # nothing with data lies outside the rectangles
        inside = np.zeros((H, W), bool)
        for x, y, rw, rh in oracle.roi_rects(g, cell, W, H):
            inside[y:y + rh, x:x + rw] = True
        assert (d[~inside] == F).all()
    ref = oracle.composite_depth(cols, deps, [(0, 0, W, H)] * 4, (0, 0, W, H))
    got = oracle.composite_depth(pieces_c, pieces_d, pieces_roi, (0, 0, W, H))
    assert (got[0] == ref[0]).all() and (got[1] == ref[1]).all()
