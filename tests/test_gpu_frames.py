"""GPU parity of the frame-placed forms (thesis Section 5.3: the input frame
places the pixel data at the ROI's position): decompression into frames at
the ROI (cmp_rle_decompress_at_roi) and depth compositing of placed frames
cropped to device rectangles (cmp_composite_depth_crop), against the oracle."""
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


def test_pipeline_into_frames_full_size():
    """16 x 1920x1080: ROI detection -> RLE -> decompression into 16 frames at
    the ROIs -> compositing of the frames cropped to the decoded ROIs (binary
    swap over 16 owners): the oracle's composite of the full frames; each
    frame holds its ROI block in place and nothing elsewhere."""
    note("pipeline into frames 16x1920x1080")
    wl = synth.depth_ramps_full(seed=2, n=16, W=1920, H=1080, device=DEV)
    roi = cmp.roi_detect(wl.images)
    streams, sizes, cst = cmp.rle_compress(wl.images, roi_dev=roi)
    frames = [cmp.Image(torch.zeros((1080, 1920), dtype=torch.int32, device=DEV),
                        torch.zeros((1080, 1920), dtype=torch.int32, device=DEV), (0, 0, 1920, 1080))
              for _ in range(16)]
    ro, st = cmp.rle_decompress(streams, frames, at_roi=True)
    oc, od = cmp.composite_depth(frames, wl.viewport, roi_dev=ro, schedule=("binary_swap", 16),
                                 crop=True)
    torch.cuda.synchronize()
    assert int(cst.abs().sum()) == 0 and (st == 0).all()
    assert torch.equal(ro, roi)
    ref_c, ref_d = oracle.composite_depth([synth.as_u32(i.color) for i in wl.images],
                                          [synth.as_u32(i.depth) for i in wl.images],
                                          [i.roi for i in wl.images], wl.viewport)
    assert (synth.as_u32(oc) == ref_c).all() and (synth.as_u32(od) == ref_d).all()
    for im, fr, (x, y, w, h) in zip(wl.images, frames, roi.cpu().tolist()):
        inside = torch.zeros((1080, 1920), dtype=torch.bool, device=DEV)
        inside[y:y + h, x:x + w] = True
        assert torch.equal(fr.color[inside], im.color[inside])
        assert torch.equal(fr.depth[inside], im.depth[inside])
        assert int(fr.color[~inside].abs().sum()) == 0 and int(fr.depth[~inside].abs().sum()) == 0


def test_decompress_at_roi_outside_the_frame():
    """A ROI that does not lie inside the destination frame: CMP_ENOSPC, and
    the same stream decodes into a frame large enough."""
    rng = np.random.default_rng(3)
    d = np.full((40, 50), F, np.uint32)
    d[10:30, 20:45] = rng.integers(0, 99, (20, 25))
    c = np.where(d != F, 0x11223344, 0).astype(np.uint32)
    s = torch.from_numpy(oracle.rle_compress(c, d, (20, 10, 25, 20))).to(DEV)
    outs = [cmp.Image(torch.zeros((40, 50), dtype=torch.int32, device=DEV),
                      torch.zeros((40, 50), dtype=torch.int32, device=DEV), (0, 0, 50, 40)),
            cmp.Image(torch.zeros((40, 44), dtype=torch.int32, device=DEV),
                      torch.zeros((40, 44), dtype=torch.int32, device=DEV), (0, 0, 44, 40)),
            cmp.Image(torch.zeros((29, 50), dtype=torch.int32, device=DEV),
                      torch.zeros((29, 50), dtype=torch.int32, device=DEV), (0, 0, 50, 29))]
    note("decompress at roi, outside the frame")
    _, st = cmp.rle_decompress([s, s, s], outs, at_roi=True)
    torch.cuda.synchronize()
    assert st.cpu().tolist() == [0, cmp.CMP_ENOSPC, cmp.CMP_ENOSPC]
    assert (synth.as_u32(outs[0].depth) == np.where(d != F, d, 0)).all()


@pytest.mark.parametrize("seed", range(4))
def test_depth_crop_random(seed):
    """Placed frames (some off the viewport's origin, with wide pitches)
    cropped to device rectangles that reach past the frames, are empty or
    negative: the oracle's composite of the cropped parts."""
    rng = np.random.default_rng(700 + seed)
    W, H = int(rng.integers(30, 200)), int(rng.integers(20, 120))
    n = [3, 16, 49, 64][seed]
    imgs, crops, pc, pd, pr = [], [], [], [], []
    for i in range(n):
        fw, fh = int(rng.integers(1, W + 10)), int(rng.integers(1, H + 10))
        fx, fy = int(rng.integers(-5, W)), int(rng.integers(-5, H))
        P = fw + int(rng.integers(0, 5))
        d = rng.integers(0, 40, (fh, P)).astype(np.uint32)
        d[rng.random((fh, P)) < 0.3] = F
        c = rng.integers(0, 2 ** 32, (fh, P), dtype=np.uint64).astype(np.uint32)
        imgs.append(cmp.Image(_dev(c), _dev(d), (fx, fy, fw, fh)))
        cx, cy = int(rng.integers(fx - 10, fx + fw)), int(rng.integers(fy - 10, fy + fh))
        cw, ch = int(rng.integers(-3, fw + 15)), int(rng.integers(-3, fh + 15))
        crops.append((cx, cy, cw, ch))
        # the oracle's piece: the frame's part inside the crop rectangle
        x0, y0 = max(cx, fx), max(cy, fy)
        x1, y1 = min(cx + max(cw, 0), fx + fw), min(cy + max(ch, 0), fy + fh)
        if x1 > x0 and y1 > y0:
            pc.append(np.ascontiguousarray(c[y0 - fy:y1 - fy, x0 - fx:x1 - fx]))
            pd.append(np.ascontiguousarray(d[y0 - fy:y1 - fy, x0 - fx:x1 - fx]))
            pr.append((x0, y0, x1 - x0, y1 - y0))
        else:
            pc.append(np.zeros((1, 1), np.uint32))
            pd.append(np.full((1, 1), F, np.uint32))
            pr.append((0, 0, 0, 0))
    rd = torch.tensor(crops, dtype=torch.int32, device=DEV)
    vp = (int(rng.integers(-3, 4)), int(rng.integers(-3, 4)), W, H)
    note(f"depth crop seed={seed} n={n}")
    oc, od = cmp.composite_depth(imgs, vp, roi_dev=rd, schedule=("binary_swap", 4), crop=True)
    torch.cuda.synchronize()
    ref_c, ref_d = oracle.composite_depth(pc, pd, pr, vp)
    assert (synth.as_u32(oc) == ref_c).all() and (synth.as_u32(od) == ref_d).all()
