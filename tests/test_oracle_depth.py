"""Pins of the oracle's depth compositing against facts that do not come from
the oracle itself: the hand-worked 4x4 example, a brute-force lexicographic
argmin written with numpy, and the invariants the thesis implies (arrival order
does not matter, Section 5.6; blank areas may be omitted, Section 5.3; a failed
source's contribution is simply missing, Section 3.8)."""
import numpy as np
import pytest

import oracle
from conftest import read_golden

F = 0xFFFFFFFF
A_COL, B_COL = 0xFF332211, 0xFF665544


def _grid(rows):
    return np.array([[F if t == "F" else int(t) for t in r] for r in rows], dtype=np.uint32)


def test_worked_example_4x4():
    g = read_golden("depth_4x4.txt")
    da, db = _grid(g["A_depth"]), _grid(g["B_depth"])
    ca = np.where(da != F, A_COL, 0).astype(np.uint32)
    cb = np.where(db != F, B_COL, 0).astype(np.uint32)
    oc, od = oracle.composite_depth([ca, cb], [da, db], [(0, 0, 4, 4)] * 2, (0, 0, 4, 4))
    assert (od == _grid(g["out_depth"])).all()
    win = {"A": A_COL, "B": B_COL, "-": 0}
    exp = np.array([[win[t] for t in r] for r in g["out_winner"]], dtype=np.uint32)
    assert (oc == exp).all()
    rois = {r[0]: tuple(int(v) for v in r[1:]) for r in g["roi"]}
    assert oracle.roi_detect_depth(da) == rois["A"]
    assert oracle.roi_detect_depth(db) == rois["B"]
    assert oracle.roi_detect_depth(od) == rois["out"]
    # cropping A to its ROI changes nothing (Section 5.3)
    x, y, w, h = rois["A"]
    oc2, od2 = oracle.composite_depth([ca[y:y + h, x:x + w], cb], [da[y:y + h, x:x + w], db],
                                      [rois["A"], (0, 0, 4, 4)], (0, 0, 4, 4))
    assert (oc2 == oc).all() and (od2 == od).all()


def _random_case(rng, n, W, H, depth_range, pitch_extra=3):
    cols, deps, rois = [], [], []
    for _ in range(n):
        w = int(rng.integers(0, W + 1))
        h = int(rng.integers(0, H + 1))
        x = int(rng.integers(-2, W + 2))
        y = int(rng.integers(-2, H + 2))
        P = w + int(rng.integers(0, pitch_extra + 1))
        d = rng.integers(0, depth_range, size=(h, P), dtype=np.uint64).astype(np.uint32)
        d[rng.random((h, P)) < 0.2] = F
        c = rng.integers(0, 2 ** 32, size=(h, P), dtype=np.uint64).astype(np.uint32)
        cols.append(c)
        deps.append(d)
        rois.append((x, y, w, h))
    vp = (int(rng.integers(-1, 2)), int(rng.integers(-1, 2)), W, H)
    return cols, deps, rois, vp


def _brute(cols, deps, rois, vp):
    """Per pixel, the (depth, index)-lexicographic minimum; numpy's argmin
    returns the first (lowest-index) minimum."""
    X0, Y0, W, H = vp
    n = len(cols)
    D = np.full((n + 1, H, W), F, dtype=np.uint64)
    C = np.zeros((n + 1, H, W), dtype=np.uint64)
    for i, (c, d, (x, y, w, h)) in enumerate(zip(cols, deps, rois)):
        for v in range(H):
            for u in range(W):
                X, Y = X0 + u, Y0 + v
                if x <= X < x + w and y <= Y < y + h:
                    D[i, v, u] = d[Y - y, X - x]
                    C[i, v, u] = c[Y - y, X - x]
    # the clear depth never wins: a slot with depth F is a non-candidate, and
    # the extra last slot (F, 0) is the background
    key = np.where(D == F, np.uint64(2 ** 40), D)
    key[n] = 2 ** 40
    win = np.argmin(key, axis=0)
    best = np.take_along_axis(key, win[None], 0)[0]
    win = np.where(best == 2 ** 40, n, win)
    oc = np.take_along_axis(C, win[None], 0)[0].astype(np.uint32)
    od = np.take_along_axis(D, win[None], 0)[0].astype(np.uint32)
    return oc, od


@pytest.mark.parametrize("seed", range(12))
def test_brute_force_argmin(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(1, 7))
    # a tiny depth range forces many ties
    cols, deps, rois, vp = _random_case(rng, n, 9, 7, depth_range=4 if seed % 2 else 2 ** 32 - 1)
    oc, od = oracle.composite_depth(cols, deps, rois, vp)
    bc, bd = _brute(cols, deps, rois, vp)
    assert (oc == bc).all() and (od == bd).all()


def _merge(a, b):
    """Merge two partial composites; on equal depth the left (lower-index)
    partial wins, which is what keeps any merge tree equal to index order."""
    (ca, da), (cb, db) = a, b
    take_b = db < da
    return np.where(take_b, cb, ca), np.where(take_b, db, da)


@pytest.mark.parametrize("seed", range(6))
def test_any_merge_tree_equals_sequential(seed):
    """Binary-swap style trees over contiguous index ranges (Section 5.2.2)
    give the same bits as the sequential composite under the tie rule."""
    rng = np.random.default_rng(100 + seed)
    n = 8
    cols, deps, rois, vp = _random_case(rng, n, 11, 6, depth_range=3)
    full = oracle.composite_depth(cols, deps, rois, vp)
    parts = [oracle.composite_depth([cols[i]], [deps[i]], [rois[i]], vp) for i in range(n)]
    while len(parts) > 1:  # balanced pairwise tree
        parts = [_merge(parts[i], parts[i + 1]) for i in range(0, len(parts), 2)]
    assert (parts[0][0] == full[0]).all() and (parts[0][1] == full[1]).all()
    # an unbalanced left-deep tree over a random split
    k = int(rng.integers(1, n))
    left = oracle.composite_depth(cols[:k], deps[:k], rois[:k], vp)
    right = oracle.composite_depth(cols[k:], deps[k:], rois[k:], vp)
    m = _merge(left, right)
    assert (m[0] == full[0]).all() and (m[1] == full[1]).all()


def test_permutation_invariant_without_ties():
    """Arrival order does not matter (Section 5.6) when depths are distinct."""
    rng = np.random.default_rng(7)
    n, W, H = 5, 10, 8
    cols, deps, rois, vp = _random_case(rng, n, W, H, depth_range=2 ** 32 - 1)
    # make all depths distinct across contributors
    vals = rng.permutation(2 ** 20)[: sum(d.size for d in deps)].astype(np.uint32)
    o = 0
    for d in deps:
        keep = d == F
        d[...] = vals[o:o + d.size].reshape(d.shape)
        d[keep] = F
        o += d.size
    full = oracle.composite_depth(cols, deps, rois, vp)
    p = rng.permutation(n)
    perm = oracle.composite_depth([cols[i] for i in p], [deps[i] for i in p], [rois[i] for i in p], vp)
    assert (perm[0] == full[0]).all() and (perm[1] == full[1]).all()


def test_crop_to_detected_roi_is_lossless():
    rng = np.random.default_rng(3)
    cols, deps, rois = [], [], []
    W, H = 12, 9
    for i in range(4):
        d = np.full((H, W), F, np.uint32)
        x0, y0 = rng.integers(0, 6, 2)
        d[y0:y0 + 3, x0:x0 + 4] = rng.integers(0, 5, (min(3, H - y0), min(4, W - x0)))
        c = rng.integers(0, 2 ** 32, (H, W), dtype=np.uint64).astype(np.uint32)
        cols.append(c); deps.append(d); rois.append((0, 0, W, H))
    full = oracle.composite_depth(cols, deps, rois, (0, 0, W, H))
    cc, cd, cr = [], [], []
    for c, d in zip(cols, deps):
        x, y, w, h = oracle.roi_detect_depth(d)
        cc.append(c[y:y + h, x:x + w]); cd.append(d[y:y + h, x:x + w]); cr.append((x, y, w, h))
    crop = oracle.composite_depth(cc, cd, cr, (0, 0, W, H))
    assert (crop[0] == full[0]).all() and (crop[1] == full[1]).all()


def test_empty_contributor_equals_absent():
    """A source with nothing to show (empty ROI, e.g. a failed node whose
    contribution goes missing, Section 3.8) changes nothing."""
    rng = np.random.default_rng(11)
    cols, deps, rois, vp = _random_case(rng, 3, 8, 8, depth_range=6)
    base = oracle.composite_depth(cols, deps, rois, vp)
    e = np.zeros((0, 0), np.uint32)
    for pos in range(4):
        c2 = cols[:pos] + [e] + cols[pos:]
        d2 = deps[:pos] + [e] + deps[pos:]
        r2 = rois[:pos] + [(0, 0, 0, 0)] + rois[pos:]
        out = oracle.composite_depth(c2, d2, r2, vp)
        assert (out[0] == base[0]).all() and (out[1] == base[1]).all()


def test_no_contributors_gives_background():
    oc, od = oracle.composite_depth([], [], [], (0, 0, 5, 3))
    assert (oc == 0).all() and (od == F).all()


def test_clear_depth_never_wins():
    d = np.full((2, 2), F, np.uint32)
    c = np.full((2, 2), 0xDEADBEEF, np.uint32)
    oc, od = oracle.composite_depth([c], [d], [(0, 0, 2, 2)], (0, 0, 2, 2))
    assert (oc == 0).all() and (od == F).all()
