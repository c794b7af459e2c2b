"""GPU parity of ROI with holes (thesis Section 5.3): the rectangles that
cover each image's occupied cells, against the oracle's, and the pipeline
that compresses, decompresses and composites those rectangles instead of
bounding boxes: streams byte-identical to the oracle's RLE of each
rectangle, and a composite equal to the oracle's composite of the full
frames."""
import numpy as np
import pytest
import torch

import oracle
import paper_1902_08755_amd as cmp
import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
F = 0xFFFFFFFF


def note(msg):
    print(f"[gpu case] {msg}", flush=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(DEV)


def _blobs(rng, H, W, nblobs, depth_range=1 << 20):
    """A clear frame with a few separate rectangles of data (holes between)."""
    d = np.full((H, W), F, np.uint32)
    c = np.zeros((H, W), np.uint32)
    for _ in range(nblobs):
        hh, ww = int(rng.integers(1, max(2, H // 3))), int(rng.integers(1, max(2, W // 3)))
        y0, x0 = int(rng.integers(0, H - hh + 1)), int(rng.integers(0, W - ww + 1))
        d[y0:y0 + hh, x0:x0 + ww] = rng.integers(0, depth_range, (hh, ww))
        c[y0:y0 + hh, x0:x0 + ww] = rng.integers(1, 2 ** 32, (hh, ww), dtype=np.uint64)
    return c, d


@pytest.mark.parametrize("max_rects", [1, 3, 8, 64])
def test_roi_rects_random_grids(max_rects):
    """Random blob frames of many shapes and cell sizes (grid rows of one and
    of several 64-cell words, partial last cells, empty frames), each
    image's rectangles and count equal to the oracle's (the bounding box
    when there are more than max_rects)."""
    rng = np.random.default_rng(100 + max_rects)
    shapes = [(1, 1), (7, 5), (64, 64), (100, 700), (33, 1030), (480, 640), (20, 4000), (5, 5)]
    imgs, host = [], []
    for k, (H, W) in enumerate(shapes):
        c, d = _blobs(rng, H, W, 0 if k == 7 else int(rng.integers(1, 6)))
        imgs.append(cmp.Image(_dev(c), _dev(d), (0, 0, W, H)))
        host.append(d)
    for cell in [(1, 1), (8, 8), (16, 4), (64, 64), (13, 7)]:
        note(f"roi rects cell={cell} max_rects={max_rects}")
        grids = cmp.roi_grid(imgs, cell)
        rects, counts = cmp.roi_rects(imgs, cell, grids, max_rects=max_rects)
        torch.cuda.synchronize()
        rects, counts = rects.cpu().numpy(), counts.cpu().numpy()
        for k, d in enumerate(host):
            H, W = d.shape
            g = oracle.roi_grid(d, cell)
            assert (grids[k].cpu().numpy() == g).all()
            ref = oracle.roi_rects(g, cell, W, H, max_rects=max_rects)
            assert int(counts[k]) == len(ref), (cell, k)
            assert [tuple(r) for r in rects[k, :len(ref)].tolist()] == ref, (cell, k)
            assert (rects[k, len(ref):] == 0).all()


def test_roi_rects_pipeline():
    """16 frames of 640x480, each with a few separate blobs: occupancy grid
    (32x32 cells) -> rectangles (4 per frame) -> RLE of every rectangle in
    one call (each frame listed 4 times, unused rectangles empty ROIs) ->
    decompression -> depth compositing of the 64 pieces placed by their
    decoded ROIs (binary swap over 16 owners). Streams equal the oracle's RLE
    of each rectangle; the composite equals the oracle's composite of the
    full frames; the rectangles hold fewer pixels than the bounding boxes."""
    rng = np.random.default_rng(5)
    H, W, cell, R = 480, 640, (32, 32), 4
    imgs, host = [], []
    for i in range(16):
        c, d = _blobs(rng, H, W, int(rng.integers(1, 4)))
        imgs.append(cmp.Image(_dev(c), _dev(d), (0, 0, W, H)))
        host.append((c, d))
    note("roi rects pipeline 16 x 640x480")
    grids = cmp.roi_grid(imgs, cell)
    rects, counts = cmp.roi_rects(imgs, cell, grids, max_rects=R)
    pieces = [imgs[i] for i in range(16) for _ in range(R)]
    roi_dev = rects.view(16 * R, 4)
    batch = cmp.RleBatch(pieces, roi_dev=roi_dev)
    streams, sizes, _ = batch.run()
    blocks = [cmp.Image(torch.zeros((H, W), dtype=torch.int32, device=DEV),
                        torch.zeros((H, W), dtype=torch.int32, device=DEV), (0, 0, W, H))
              for _ in pieces]
    ro, st = cmp.rle_decompress(streams, blocks)
    oc, od = cmp.composite_depth(blocks, (0, 0, W, H), roi_dev=ro, schedule=("binary_swap", 16))
    torch.cuda.synchronize()
    assert int(batch.status.abs().sum()) == 0 and (st == 0).all()
    rects_h = rects.cpu().numpy()
    rect_px = box_px = 0
    for i, (c, d) in enumerate(host):
        g = oracle.roi_grid(d, cell)
        ref = oracle.roi_rects(g, cell, W, H, max_rects=R)
        assert [tuple(r) for r in rects_h[i, :len(ref)].tolist()] == ref
        for k in range(R):
            r = tuple(rects_h[i, k].tolist()) if k < len(ref) else (0, 0, 0, 0)
            s = oracle.rle_compress(c, d, r)
            n = int(sizes[i * R + k])
            assert n == s.size and (streams[i * R + k][:n].cpu().numpy() == s).all(), (i, k)
            rect_px += r[2] * r[3]
        x, y, w, h = oracle.roi_detect_depth(d)
        box_px += w * h
    ref_c, ref_d = oracle.composite_depth([c for c, _ in host], [d for _, d in host],
                                          [(0, 0, W, H)] * 16, (0, 0, W, H))
    assert (synth.as_u32(oc) == ref_c).all() and (synth.as_u32(od) == ref_d).all()
    print(f"[roi rects] rectangles {rect_px} px vs bounding boxes {box_px} px", flush=True)
    assert rect_px < box_px
