"""GPU parity: every entry point of the HIP library against the oracle on the
same seeded inputs. Integer work (depth compositing, ROI, RLE) must match bit
for bit; float work within the stated tolerances:
  over forward:  |x - ref| <= 2e-6 |ref| + 1e-30 per channel, ref = FP64 oracle
  over backward: |g - ref| <= 2e-6 g_abs + 1e-30, g_abs = the oracle's
                 componentwise condition scale (G can cancel in the alpha term)
"""
import sys

import os

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
    sys.stdout.flush()


def u32(t):
    return synth.as_u32(t)


def _oracle_depth(images, viewport):
    return oracle.composite_depth([u32(i.color) for i in images], [u32(i.depth) for i in images],
                                  [i.roi for i in images], viewport)


def _close(got, ref, rtol=2e-6):
    got = np.asarray(got, dtype=np.float64)
    return np.abs(got - ref) <= rtol * np.abs(ref) + 1e-30


# ------------------------------------------------------------------ depth
SCHEDS = [("seq", 1), ("direct_send", 4), ("direct_send", 7), ("binary_swap", 4),
          ("binary_swap", 16), ("binary_swap", 64)]


def test_depth_rect_workload_all_schedules():
    """4 x 640x480 contributors with 20 random rectangles each."""
    note("depth rects 4x640x480")
    wl = synth.depth_rects(seed=1, n=4, W=640, H=480, device=DEV)
    ref_c, ref_d = _oracle_depth(wl.images, wl.viewport)
    for sched in SCHEDS:
        for tile in [(0, 0), (128, 8), (32, 32), (4, 1)]:
            oc, od = cmp.composite_depth(wl.images, wl.viewport, schedule=sched, tile=tile)
            torch.cuda.synchronize()
            assert (u32(oc) == ref_c).all(), (sched, tile)
            assert (u32(od) == ref_d).all(), (sched, tile)


def _random_depth_images(rng, n, W, H, depth_range, device=DEV):
    imgs = []
    for i in range(n):
        w, h = int(rng.integers(0, W + 3)), int(rng.integers(0, H + 3))
        x, y = int(rng.integers(-3, W + 2)), int(rng.integers(-3, H + 2))
        P = w + int(rng.integers(0, 5))
        d = rng.integers(0, depth_range, size=(h, P), dtype=np.uint64).astype(np.uint32)
        d[rng.random((h, P)) < 0.15] = F
        c = rng.integers(0, 2 ** 32, size=(h, P), dtype=np.uint64).astype(np.uint32)
        imgs.append(cmp.Image(torch.from_numpy(c.view(np.int32)).to(device),
                              torch.from_numpy(d.view(np.int32)).to(device), (x, y, w, h)))
    return imgs


@pytest.mark.parametrize("seed", range(12))
def test_depth_random_ragged(seed):
    """Random placements (partly outside), pitches, ties, ragged tiles and
    viewport offsets; 0..150 contributors (more than one pass above 48: up
    to four)."""
    rng = np.random.default_rng(seed)
    n = [3, 5, 9, 17, 33, 49, 60, 2, 1, 0, 97, 150][seed]
    W, H = int(rng.integers(1, 300)), int(rng.integers(1, 130))
    imgs = _random_depth_images(rng, n, W, H, depth_range=5 if seed % 2 else 2 ** 32 - 1)
    vp = (int(rng.integers(-5, 6)), int(rng.integers(-5, 6)), W, H)
    note(f"depth random seed={seed} n={n} vp={vp}")
    ref_c, ref_d = _oracle_depth(imgs, vp)
    for sched in [("seq", 1), ("direct_send", 3), ("binary_swap", 8)]:
        # a wider output pitch
        oc = torch.full((H, W + 7), -1, dtype=torch.int32, device=DEV)
        od = torch.full((H, W + 7), -1, dtype=torch.int32, device=DEV)
        cmp.composite_depth(imgs, vp, out_color=oc, out_depth=od, schedule=sched, tile=(8, 3))
        torch.cuda.synchronize()
        assert (u32(oc[:, :W]) == ref_c).all(), sched
        assert (u32(od[:, :W]) == ref_d).all(), sched
        assert (oc[:, W:] == -1).all() and (od[:, W:] == -1).all()   # no write past the row


def test_depth_device_roi_override_and_colour_only():
    rng = np.random.default_rng(77)
    imgs = _random_depth_images(rng, 6, 90, 50, depth_range=100)
    # device placements: shifted, shrunk, one negative (empty), one larger than the buffer
    rois = []
    for k, im in enumerate(imgs):
        x, y, w, h = im.roi
        rois.append([(x + 3, y - 2, w - 1, h, ), (x, y, -4, h), (x, y, w + 10, h + 10)][k % 3])
    rd = torch.tensor(rois, dtype=torch.int32, device=DEV)
    eff = [(x, y, max(0, min(w, im.roi[2])), max(0, min(h, im.roi[3])))
           for (x, y, w, h), im in zip(rois, imgs)]
    note("depth device roi override")
    vp = (0, 0, 90, 50)
    ref_c, ref_d = oracle.composite_depth([u32(i.color) for i in imgs], [u32(i.depth) for i in imgs],
                                          eff, vp)
    oc, od = cmp.composite_depth(imgs, vp, roi_dev=rd)
    oc2, _ = cmp.composite_depth(imgs, vp, roi_dev=rd, want_depth=False)
    torch.cuda.synchronize()
    assert (u32(oc) == ref_c).all() and (u32(od) == ref_d).all()
    assert (u32(oc2) == ref_c).all()


def test_depth_repeat_runs_bitwise_equal():
    """Race canary: repeated launches give identical bits."""
    wl = synth.depth_ramps_roi(seed=2, n=16, W=1920, H=1080, device=DEV)
    note("depth repeat 16x1920x1080")
    first = [t.clone() for t in cmp.composite_depth(wl.images, wl.viewport,
                                                    schedule=("binary_swap", 16))]
    for _ in range(3):
        oc, od = cmp.composite_depth(wl.images, wl.viewport, schedule=("binary_swap", 16))
        assert torch.equal(oc, first[0]) and torch.equal(od, first[1])


# -------------------------------------------------------------------- ROI
def test_roi_detect_ramp_images_exact():
    """16 full-frame 1920x1080 contributors; the generator knows each ROI."""
    wl = synth.depth_ramps_full(seed=2, n=16, W=1920, H=1080, device=DEV)
    note("roi 16x1920x1080")
    roi = cmp.roi_detect(wl.images)
    torch.cuda.synchronize()
    got = [tuple(r) for r in roi.cpu().tolist()]
    assert got == [im.true_roi for im in wl.images]
    # and the oracle on two of them
    for k in (0, 7):
        assert got[k] == oracle.roi_detect_depth(u32(wl.images[k].depth))
    # repeated calls reuse the workspace (it is left zeroed)
    for _ in range(3):
        assert [tuple(r) for r in cmp.roi_detect(wl.images).cpu().tolist()] == got


@pytest.mark.parametrize("fmt", ["depth", "rgba8", "f32", "f16"])
def test_roi_detect_random_formats(fmt):
    rng = np.random.default_rng({"depth": 1, "rgba8": 2, "f32": 3, "f16": 4}[fmt])
    imgs, refs = [], []
    shapes = [(1, 1), (3, 5), (17, 64), (130, 257), (64, 1), (9, 1000), (50, 50), (50, 50)]
    for k, (h, w) in enumerate(shapes):
        P = w + (k % 3) * 4
        m = rng.random((h, P)) < [0.0, 0.5, 0.01, 0.0005, 0.2, 0.001, 1.0, 0.0][k]
        if k == 3:
            m[h - 1, w - 1] = True     # a single corner pixel
        if fmt in ("depth", "rgba8"):
            v = np.where(m, rng.integers(0, F - 1, (h, P), dtype=np.uint64), F if fmt == "depth" else 0)
            a = v.astype(np.uint32)
            t = torch.from_numpy(a.view(np.int32)).to(DEV)
            img = cmp.Image(t, t if fmt == "depth" else None, (0, 0, w, h))
            refs.append(oracle.roi_detect_depth(a, w, h) if fmt == "depth" else oracle.roi_detect_rgba8(a, w, h))
        else:
            L = np.zeros((h, P, 4), np.float32)
            L[m, k % 4] = rng.random(m.sum()).astype(np.float32) + 0.25
            L[~m, 0] = -0.0          # negative zero is empty
            if k == 5:
                L[0, 0, 2] = np.nan  # NaN is data
            L = L.astype(np.float16 if fmt == "f16" else np.float32)
            img = cmp.Image(torch.from_numpy(L).to(DEV), None, (0, 0, w, h))
            refs.append(oracle.roi_detect_rgbaf(L, w, h))
        imgs.append(img)
    note(f"roi formats {fmt}")
    f = {"depth": cmp.RGBA8, "rgba8": cmp.RGBA8, "f32": cmp.RGBA32F, "f16": cmp.RGBA16F}[fmt]
    roi = cmp.roi_detect(imgs, fmt=f)
    torch.cuda.synchronize()
    assert [tuple(r) for r in roi.cpu().tolist()] == refs


def test_roi_detect_tall_images_many_bands():
    """Images tall enough that their bands hit the per-image limit of 1024
    workgroups (the last workgroup folds 1024 partial boxes): data only in
    the first and last bands, only in the last band, and none."""
    h, w = 1_100_000, 32
    a = np.full((h, w), F, np.uint32)
    a[5, 31] = 7
    a[h - 1, 0] = 9
    a[h // 2, 10] = 1
    b = np.full((h, w), F, np.uint32)
    b[h - 3, 17] = 0
    c = np.full((h, w), F, np.uint32)
    imgs = [cmp.Image(*(2 * [torch.from_numpy(x.view(np.int32)).to(DEV)]), (0, 0, w, h))
            for x in (a, b, c)]
    note("roi tall images")
    roi = cmp.roi_detect(imgs)
    torch.cuda.synchronize()
    assert [tuple(r) for r in roi.cpu().tolist()] == [oracle.roi_detect_depth(x) for x in (a, b, c)]
    assert [tuple(r) for r in roi.cpu().tolist()] == [(0, 5, 32, h - 5), (17, h - 3, 1, 1), (0, 0, 0, 0)]


# -------------------------------------------------------------------- RLE
def _check_streams(imgs, rois, streams, sizes):
    for k, im in enumerate(imgs):
        c, d = u32(im.color), (u32(im.depth) if im.depth is not None else None)
        ref = oracle.rle_compress(c, d, rois[k])
        n = int(sizes[k])
        assert n == ref.size, (k, n, ref.size)
        assert (streams[k][:n].cpu().numpy() == ref).all(), k


def _run_images(rng, n, H, W, max_run):
    """n images of H x W (colour and depth) made of runs of 1..max_run pixels."""
    imgs = []
    for _ in range(n):
        planes = []
        for _ in range(2):
            lens = rng.integers(1, max_run + 1, H * W)
            vals = rng.integers(0, 2 ** 32, H * W, dtype=np.uint64).astype(np.uint32)
            planes.append(np.repeat(vals, lens)[:H * W].reshape(H, W))
        imgs.append(cmp.Image(torch.from_numpy(planes[0].view(np.int32)).to(DEV),
                              torch.from_numpy(planes[1].view(np.int32)).to(DEV), (0, 0, W, H)))
    return imgs


def test_rle_call_counter_wrap_clears_flags():
    """The compression workspace's 30-bit call counter wraps after 2^30 calls.
    Forced from the host (the counter word set to 2^30 - 1), the wrapping call
    zeroes the look-back flags of every earlier call, so that the next call,
    which runs under counter 0 as the workspace's first call did, cannot take
    a flag of that first call (same layout, other sizes) for its own."""
    rng = np.random.default_rng(11)
    a = _run_images(rng, 4, 480, 640, 12)     # the first call: 4 x 75 blocks
    a2 = _run_images(rng, 4, 480, 640, 3)     # same block layout, other stream sizes
    c = _run_images(rng, 1, 64, 64, 5)        # the wrapping call: one block
    ba, ba2, bc = cmp.RleBatch(a), cmp.RleBatch(a2), cmp.RleBatch(c)
    ws = ba.ws
    ba2.ws = bc.ws = ws
    ctl = 8192 // 4                           # word index of the counter (after the tickets)
    hwm_word, flags0, nflags = ctl + 33, 8192 + 256, 4 * 75
    words = ws.view(torch.int32)
    note("rle call counter wrap: first call")
    streams, sizes, _ = ba.run()
    torch.cuda.synchronize()
    assert int(ba.status.abs().sum()) == 0
    assert int(words[ctl]) == 1 and int(words[hwm_word]) == nflags
    _check_streams(a, [im.roi for im in a], streams, sizes)
    flags = ws[flags0:flags0 + 8 * nflags].view(torch.int64)
    assert int((flags != 0).sum()) == nflags   # every block published a flag under counter 0
    words[ctl] = (1 << 30) - 1
    note("rle call counter wrap: the wrapping call")
    streams, sizes, _ = bc.run()
    torch.cuda.synchronize()
    assert int(bc.status.abs().sum()) == 0
    _check_streams(c, [im.roi for im in c], streams, sizes)
    assert int(words[ctl]) == 0 and int(words[hwm_word]) == nflags
    assert int((ws[flags0:flags0 + 8 * nflags] != 0).sum()) == 0
    note("rle call counter wrap: the call after it, under counter 0 again")
    for rep in range(2):
        streams, sizes, _ = ba2.run()
        torch.cuda.synchronize()
        assert int(ba2.status.abs().sum()) == 0
        _check_streams(a2, [im.roi for im in a2], streams, sizes)
    assert int(words[ctl]) == 2


def test_rle_rect_composite_round_trip():
    """RLE of the composite of the 640x480 rectangle workload, ROI from the GPU."""
    wl = synth.depth_rects(seed=1, n=4, W=640, H=480, device=DEV)
    oc, od = cmp.composite_depth(wl.images, wl.viewport)
    full = cmp.Image(oc, od, (0, 0, 640, 480))
    roi = cmp.roi_detect([full])
    note("rle rect composite")
    streams, sizes, cst = cmp.rle_compress([full], roi_dev=roi)
    torch.cuda.synchronize()
    assert int(cst[0]) == 0
    r = tuple(roi[0].tolist())
    _check_streams([full], [r], streams, sizes)
    outc = torch.zeros((480, 640), dtype=torch.int32, device=DEV)
    outd = torch.zeros((480, 640), dtype=torch.int32, device=DEV)
    ro, st = cmp.rle_decompress([streams[0]], [cmp.Image(outc, outd, (0, 0, 640, 480))])
    torch.cuda.synchronize()
    assert int(st[0]) == 0 and tuple(ro[0].tolist()) == r
    x, y, w, h = r
    # the ROI block lands at the top left of the destination, in its pitch
    assert torch.equal(outc[:h, :w], oc[y:y + h, x:x + w])
    assert torch.equal(outd[:h, :w], od[y:y + h, x:x + w])


def test_rle_adversarial_images():
    """Runs of 255/256/257, noise, single pixels, one-block and block+1 ROIs,
    empty ROIs, 4-plane (colour-only) images, several images per launch."""
    rng = np.random.default_rng(5)
    specs = [((1, 1), (0, 0, 1, 1)), ((130, 150), (7, 3, 129, 101)), ((64, 128), (0, 0, 128, 32)),
             ((65, 64), (0, 0, 64, 65)), ((20, 30), (5, 5, 0, 7)), ((300, 301), (0, 0, 301, 300)),
             ((40, 4100), (1, 2, 4097, 3)), ((33, 33), (32, 32, 1, 1))]
    imgs, rois, mk = [], [], []
    for k, ((H, W), roi) in enumerate(specs):
        c = np.zeros((H, W), np.uint32)
        d = np.full((H, W), F, np.uint32)
        flat, dflat = c.reshape(-1), d.reshape(-1)
        pos = 0
        for run in [255, 256, 257, 1, 1, 2, 511, 513, 4095, 4096, 4097]:
            if pos >= flat.size:
                break
            flat[pos:pos + run] = rng.integers(0, 2 ** 32, dtype=np.uint64)
            dflat[pos:pos + run] = rng.integers(0, 2 ** 32, dtype=np.uint64)
            pos = min(flat.size, pos + run)
        k2 = min(flat.size, pos + 3000)
        flat[pos:k2] = rng.integers(0, 2 ** 32, k2 - pos, dtype=np.uint64).astype(np.uint32)
        tc = torch.from_numpy(c.view(np.int32)).to(DEV)
        td = torch.from_numpy(d.view(np.int32)).to(DEV)
        imgs.append(cmp.Image(tc, td if k % 3 else None, (0, 0, W, H)))
        rois.append(roi)
    rd = torch.tensor(rois, dtype=torch.int32, device=DEV)
    note("rle adversarial")
    batch = cmp.RleBatch(imgs, roi_dev=rd)
    for rep in range(3):          # the workspace is reused: epochs, tickets
        streams, sizes, _ = batch.run()
        torch.cuda.synchronize()
        assert int(batch.status.abs().sum()) == 0
        _check_streams(imgs, [r if r[2] * r[3] else (0, 0, 0, 0) for r in rois], streams, sizes)
    # decode all at once into full-size buffers
    outs = [cmp.Image(torch.zeros_like(im.color), None if im.depth is None else torch.zeros_like(im.depth),
                      im.roi) for im in imgs]
    ro, st = cmp.rle_decompress(streams, outs)
    torch.cuda.synchronize()
    assert (st == 0).all()
    for im, o, (x, y, w, h) in zip(imgs, outs, rois):
        if w * h == 0:
            continue
        assert torch.equal(o.color[:h, :w], im.color[y:y + h, x:x + w])
        if im.depth is not None:
            assert torch.equal(o.depth[:h, :w], im.depth[y:y + h, x:x + w])


def test_roi_rle_sixty_four_images():
    """The per-call maximum of 64 images: ROI detection on the device, then
    compression with those ROIs and decompression, against the oracle; sizes
    from 1x1 to 90x70, some images empty, colour-only and depth images."""
    rng = np.random.default_rng(64)
    imgs, refs = [], []
    for k in range(64):
        H, W = int(rng.integers(1, 71)), int(rng.integers(1, 91))
        d = np.full((H, W), F, np.uint32)
        c = np.zeros((H, W), np.uint32)
        if k % 9 != 4:   # every ninth image holds no data
            y0, x0 = int(rng.integers(0, H)), int(rng.integers(0, W))
            y1, x1 = int(rng.integers(y0, H)) + 1, int(rng.integers(x0, W)) + 1
            d[y0:y1, x0:x1] = rng.integers(0, 4, (y1 - y0, x1 - x0)) + 1000 * k
            c[y0:y1, x0:x1] = rng.integers(0, 3, (y1 - y0, x1 - x0)).astype(np.uint32) * 0x01020304 + 1
        has_depth = k % 5 != 1
        tc = torch.from_numpy(c.view(np.int32)).to(DEV)
        td = torch.from_numpy(d.view(np.int32)).to(DEV)
        imgs.append(cmp.Image(tc, td if has_depth else None, (0, 0, W, H)))
        refs.append(oracle.roi_detect_depth(d) if has_depth else oracle.roi_detect_rgba8(c))
    note("roi + rle, 64 images")
    # ROI per image kind (the depth test for images with depth, the colour test otherwise)
    with_d = [k for k in range(64) if imgs[k].depth is not None]
    without = [k for k in range(64) if imgs[k].depth is None]
    roi = torch.zeros((64, 4), dtype=torch.int32, device=DEV)
    roi[with_d] = cmp.roi_detect([imgs[k] for k in with_d])
    roi[without] = cmp.roi_detect([imgs[k] for k in without])
    torch.cuda.synchronize()
    got = [tuple(r) for r in roi.cpu().tolist()]
    assert got == refs
    batch = cmp.RleBatch(imgs, roi_dev=roi)
    streams, sizes, _ = batch.run()
    torch.cuda.synchronize()
    assert int(batch.status.abs().sum()) == 0
    _check_streams(imgs, got, streams, sizes)
    outs = [cmp.Image(torch.zeros_like(im.color), None if im.depth is None else torch.zeros_like(im.depth),
                      im.roi) for im in imgs]
    ro, st = cmp.rle_decompress(streams, outs)
    torch.cuda.synchronize()
    assert (st == 0).all()
    assert [tuple(r) for r in ro.cpu().tolist()] == got
    for im, o, (x, y, w, h) in zip(imgs, outs, got):
        if w * h == 0:
            continue
        assert torch.equal(o.color[:h, :w], im.color[y:y + h, x:x + w])
        if im.depth is not None:
            assert torch.equal(o.depth[:h, :w], im.depth[y:y + h, x:x + w])


def test_rle_decompress_rejects_corrupt_streams():
    depth = np.array([[5, 5, F], [5, 3, F], [F, F, F], [F, F, 7]], np.uint32)
    color = np.where(depth != F, 0xFF332211, 0).astype(np.uint32)
    good = oracle.rle_compress(color, depth, (0, 0, 3, 4))
    cases = {"magic": (0, 0x53), "nplanes": (20, 5), "block": (25, 0x20), "nblocks": (28, 2),
             "boff": (32, 16), "odd": (36, 11), "toolong": (36, 13), "overflow": (80, 5),
             "short": (80, 0)}
    streams, names = [], []
    for name, (pos, val) in cases.items():
        s = good.copy()
        s[pos] = val
        streams.append(torch.from_numpy(s).to(DEV))
        names.append(name)
    streams.append(torch.from_numpy(good).to(DEV))
    names.append("good")
    outs = [cmp.Image(torch.zeros((4, 3), dtype=torch.int32, device=DEV),
                      torch.zeros((4, 3), dtype=torch.int32, device=DEV), (0, 0, 3, 4))
            for _ in streams]
    # a too-small destination and a missing depth buffer: CMP_ENOSPC
    streams += [torch.from_numpy(good).to(DEV)] * 2
    names += ["small", "nodepth"]
    outs.append(cmp.Image(torch.zeros((4, 3), dtype=torch.int32, device=DEV),
                          torch.zeros((4, 3), dtype=torch.int32, device=DEV), (0, 0, 2, 4)))
    outs.append(cmp.Image(torch.zeros((4, 3), dtype=torch.int32, device=DEV), None, (0, 0, 3, 4)))
    note("rle corrupt")
    _, st = cmp.rle_decompress(streams, outs)
    torch.cuda.synchronize()
    st = st.cpu().tolist()
    for name, s in zip(names, st):
        if name == "good":
            assert s == 0
        elif name in ("small", "nodepth"):
            assert s == cmp.CMP_ENOSPC, name
        else:
            assert s == cmp.CMP_ECORRUPT, name
    assert (u32(outs[names.index("good")].color) == color).all()


def test_rle_decompress_rejects_runs_across_segments():
    """A run that crosses a multiple of 256 pixels is malformed (the oracle
    rejects it too); the unmodified stream decodes."""
    color = np.full((1, 300), 0x7E7E7E7E, np.uint32)
    good = oracle.rle_compress(color, color.copy(), (0, 0, 300, 1))
    bad1, bad2 = good.copy(), good.copy()
    bad1[80], bad1[82] = 199, 99
    bad2[84], bad2[86] = 254, 44          # plane 1
    for b in (bad1, bad2):
        with pytest.raises(oracle.CorruptStream):
            oracle.rle_decompress(b)
    streams = [torch.from_numpy(x).to(DEV) for x in (good, bad1, bad2)]
    outs = [cmp.Image(torch.zeros((1, 300), dtype=torch.int32, device=DEV),
                      torch.zeros((1, 300), dtype=torch.int32, device=DEV), (0, 0, 300, 1))
            for _ in streams]
    note("rle run across segment")
    _, st = cmp.rle_decompress(streams, outs)
    torch.cuda.synchronize()
    assert st.cpu().tolist() == [0, cmp.CMP_ECORRUPT, cmp.CMP_ECORRUPT]
    assert (u32(outs[0].color) == color).all() and (u32(outs[0].depth) == color).all()


# ------------------------------------------------------------------- over
def _over_layers(rng, n, W, H, dtype, full=False):
    layers = []
    for _ in range(n):
        if full:
            x, y, w, h = 0, 0, W, H
        else:
            w, h = int(rng.integers(1, W + 1)), int(rng.integers(1, H + 1))
            x, y = int(rng.integers(-2, W)), int(rng.integers(-2, H))
        P = w + int(rng.integers(0, 3))
        a = rng.beta(2, 5, size=(h, P))
        L = np.empty((h, P, 4))
        L[..., :3] = rng.random((h, P, 3)) * a[..., None]
        L[..., 3] = a
        layers.append(cmp.Image(torch.from_numpy(L.astype(dtype)).to(DEV), None, (x, y, w, h)))
    return layers


def _np(l):
    return l.color.cpu().numpy()


@pytest.mark.parametrize("dtype", [np.float32, np.float16])
@pytest.mark.parametrize("seed", range(4))
def test_over_random(dtype, seed):
    rng = np.random.default_rng(200 + seed)
    n = [1, 7, 13, 70][seed]
    W, H = int(rng.integers(1, 200)), int(rng.integers(1, 90))
    layers = _over_layers(rng, n, W, H, dtype)
    order = list(rng.permutation(n))
    vp = (int(rng.integers(-2, 3)), int(rng.integers(-2, 3)), W, H)
    note(f"over random seed={seed} n={n} dtype={dtype.__name__}")
    ref = oracle.composite_over([_np(l) for l in layers], [l.roi for l in layers], order, vp)
    seq = cmp.composite_over(layers, order, vp, tile=(16, 4))
    ds = cmp.composite_over(layers, order, vp, schedule=("direct_send", 5), tile=(64, 1))
    torch.cuda.synchronize()
    assert _close(seq.cpu().numpy(), ref).all()
    assert torch.equal(seq, ds)               # same per-pixel chain, same bits
    if n <= 64:
        for P in (2, 4, 16):
            bs = cmp.composite_over(layers, order, vp, schedule=("binary_swap", P))
            tref = oracle.composite_over([_np(l) for l in layers], [l.roi for l in layers], order,
                                         vp, groups=P)
            torch.cuda.synchronize()
            assert _close(bs.cpu().numpy(), tref).all(), P
            # tree and sequential agree within 1e-6 in FP32
            s = seq.cpu().numpy().astype(np.float64)
            assert (np.abs(bs.cpu().numpy() - s) <= 1e-6 * np.abs(s) + 1e-30).all()


def _over_frame_vs_oracle(layers, order, out, band_rows=136):
    """Compares a full-viewport over composite of full-frame layers with the
    FP64 oracle, band of rows by band of rows (every element). Returns the
    number of elements, the maximum relative error and the 99.99th
    percentile of the relative error over all channels."""
    H, W = out.shape[0], out.shape[1]
    n = len(layers)
    total, worst, tails = 0, 0.0, []
    for y0 in range(0, H, band_rows):
        y1 = min(H, y0 + band_rows)
        band = [l.rgba[y0:y1].detach().cpu().numpy() for l in layers]
        ref = oracle.composite_over(band, [(0, 0, W, y1 - y0)] * n, order, (0, 0, W, y1 - y0))
        got = out[y0:y1].cpu().numpy().astype(np.float64)
        ok = _close(got, ref)
        assert ok.all(), (y0, np.abs(got - ref)[~ok].max())
        nz = ref != 0
        rel = np.abs(got[nz] - ref[nz]) / np.abs(ref[nz])
        assert (got[~nz] == 0).all()
        total += ref.size
        worst = max(worst, float(rel.max(initial=0.0)))
        k = max(1, rel.size // 10_000 + 1)
        tails.append(np.partition(rel, rel.size - k)[rel.size - k:] if rel.size > k else rel)
        del band, ref, got
    tail = np.sort(np.concatenate(tails))[::-1]
    p9999 = float(tail[min(len(tail) - 1, total // 10_000)])
    return total, worst, p9999


@pytest.mark.parametrize("dtype", [torch.float32, torch.float16])
def test_over_bricks_full_frame(dtype):
    """64 layers at 3840x2160 (the brick workload): every element of the
    frame against the FP64 oracle, in bands of rows; prints the relative
    error distribution (maximum and 99.99th percentile)."""
    note(f"over bricks 64x3840x2160 {dtype}")
    ow = synth.over_bricks(seed=3, n=64, W=3840, H=2160, device=DEV, dtype=dtype)
    out = cmp.composite_over(ow.layers, ow.order, ow.viewport)
    torch.cuda.synchronize()
    total, worst, p9999 = _over_frame_vs_oracle(ow.layers, ow.order, out)
    print(f"[over error] 64x3840x2160 {dtype}: {total} elements, max rel {worst:.3e}, "
          f"p99.99 rel {p9999:.3e}", flush=True)
    assert worst <= 2e-6


# --------------------------------------------------------------- backward
def _bwd_check(layers, order, vp, G):
    grads = cmp.composite_over_backward(layers, order, vp, torch.from_numpy(G.astype(np.float32)).to(DEV))
    torch.cuda.synchronize()
    ref, scale = oracle.composite_over_backward([_np(l) for l in layers], [l.roi for l in layers],
                                                order, vp, G.astype(np.float32).astype(np.float64),
                                                want_scale=True)
    for k, (g, r, s) in enumerate(zip(grads, ref, scale)):
        w = layers[k].roi[2]
        got = g.cpu().numpy().astype(np.float64)
        bad = np.abs(got - r[:, :w]) > 2e-6 * s[:, :w] + 1e-30
        assert not bad.any(), (k, np.abs(got - r[:, :w]).max())


@pytest.mark.parametrize("seed", range(7))
def test_over_backward_random(seed):
    """Random layers, partial placements and orders; 33..64 layers take two
    chunks, 100 and 256 layers (the maximum) take 4 and 8 with transmittance
    checkpoints and descriptors in a workspace."""
    rng = np.random.default_rng(300 + seed)
    n = [1, 5, 32, 50, 64, 100, 256][seed]
    W, H = int(rng.integers(1, 150)), int(rng.integers(1, 70))
    layers = _over_layers(rng, n, W, H, np.float32 if seed % 2 else np.float16)
    order = list(rng.permutation(n))
    vp = (int(rng.integers(-2, 3)), int(rng.integers(-2, 3)), W, H)
    G = rng.standard_normal((H, W, 4))
    note(f"over backward seed={seed} n={n}")
    _bwd_check(layers, order, vp, G)


def test_over_backward_grad_target_workload():
    """32 layers at 1024x1024 with loss = sum (out - t)^2 (G = 2 (out - t)):
    every gradient element against the FP64 adjoint."""
    note("over backward 32x1024x1024")
    ow = synth.over_bricks(seed=4, n=32, W=1024, H=1024, device=DEV, with_target=True)
    layers = [l.rgba.requires_grad_(True) for l in ow.layers]
    rois = [l.roi for l in ow.layers]
    out = cmp.OverComposite.apply(ow.order, ow.viewport, rois, *layers)
    loss = ((out - ow.target) ** 2).sum()
    loss.backward()
    torch.cuda.synchronize()
    G = (2.0 * (out.detach() - ow.target)).cpu().numpy().astype(np.float64)
    Ls = [l.detach().cpu().numpy() for l in layers]
    ref, scale = oracle.composite_over_backward(Ls, rois, ow.order, ow.viewport, G, want_scale=True)
    for k in range(32):
        got = layers[k].grad.cpu().numpy().astype(np.float64)
        assert not (np.abs(got - ref[k]) > 2e-6 * scale[k] + 1e-30).any(), k
    # the forward output against the oracle, every element
    del Ls
    total, worst, p9999 = _over_frame_vs_oracle(ow.layers, ow.order, out.detach(), band_rows=256)
    print(f"[over error] 32x1024x1024 forward: {total} elements, max rel {worst:.3e}, "
          f"p99.99 rel {p9999:.3e}", flush=True)


# ------------------------------------------------------------------ batch
def _cjobs(jobs, outs):
    keep = []
    arr = (cmp.CJob * len(jobs))()
    for k, (job, out) in enumerate(zip(jobs, outs)):
        wl = job.work
        if job.kind == "depth":
            imgs = cmp._images(wl.images, "u32")
            arr[k] = cmp.CJob(0, cmp.RGBA8, len(wl.images), imgs, None, cmp._rect(wl.viewport),
                              out[0].data_ptr(), out[1].data_ptr(), out[0].stride(0))
            keep.append(imgs)
        else:
            imgs = cmp._images(wl.layers, "rgba")
            import ctypes
            order = (ctypes.c_int32 * len(wl.order))(*wl.order)
            arr[k] = cmp.CJob(1, cmp.RGBA32F, len(wl.layers), imgs, order, cmp._rect(wl.viewport),
                              out.data_ptr(), None, out.stride(0) // 4)
            keep += [imgs, order]
    return arr, keep


def _alloc_outs(jobs):
    outs = []
    for job in jobs:
        _, _, w, h = job.work.viewport
        if job.kind == "depth":
            outs.append((torch.full((h, w), 7, dtype=torch.int32, device=DEV),
                         torch.full((h, w), 7, dtype=torch.int32, device=DEV)))
        else:
            outs.append(torch.full((h, w, 4), 7.0, dtype=torch.float32, device=DEV))
    return outs


def test_batch_persistent_equals_plain_and_oracle():
    import ctypes
    jobs = synth.batch_jobs(seed=5, njobs=24, device=DEV, log2_range=(3.0, 8.0), n_range=(2, 9))
    outs_a, outs_b = _alloc_outs(jobs), _alloc_outs(jobs)
    arr_a, keep_a = _cjobs(jobs, outs_a)
    arr_b, keep_b = _cjobs(jobs, outs_b)
    L = cmp.lib()
    plan_a, plan_b = ctypes.c_void_p(), ctypes.c_void_p()
    assert L.cmp_batch_plan_create(arr_a, len(jobs), None, ctypes.byref(plan_a)) == 0
    assert L.cmp_batch_plan_create(arr_b, len(jobs), None, ctypes.byref(plan_b)) == 0
    ws = torch.zeros(L.cmp_batch_workspace_size(plan_a) + 64, dtype=torch.uint8, device=DEV)
    s = torch.cuda.current_stream().cuda_stream
    note("batch 24 jobs")
    assert L.cmp_batch_upload(plan_a, ws.data_ptr(), ws.numel(), s) == 0
    torch.cuda.synchronize()
    for rep in range(3):   # the queue resets itself between launches
        assert L.cmp_batch_run(plan_a, ws.data_ptr(), s) == 0
    assert L.cmp_batch_run_plain(plan_b, s) == 0
    torch.cuda.synchronize()
    for job, a, b in zip(jobs, outs_a, outs_b):
        if job.kind == "depth":
            assert torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
        else:
            assert torch.equal(a, b)
    for k, (job, a) in enumerate(zip(jobs, outs_a)):
        assert _job_check_oracle(job, a), k
    L.cmp_batch_plan_destroy(plan_a)
    L.cmp_batch_plan_destroy(plan_b)
    del keep_a, keep_b


def _job_check_oracle(job, out):
    """One batched job's output against the oracle: depth bit for bit, over
    within 2e-6 of the FP64 result."""
    wl = job.work
    if job.kind == "depth":
        rc, rd = _oracle_depth(wl.images, wl.viewport)
        return bool((u32(out[0]) == rc).all() and (u32(out[1]) == rd).all())
    ref = oracle.composite_over([l.rgba.cpu().numpy() for l in wl.layers],
                                [l.roi for l in wl.layers], wl.order, wl.viewport)
    return bool(_close(out.cpu().numpy(), ref).all())


def _same(a, b):
    if isinstance(a, tuple):
        return torch.equal(a[0], b[0]) and torch.equal(a[1], b[1])
    return torch.equal(a, b)


def _scribble(outs):
    for o in outs:
        for t in (o if isinstance(o, tuple) else (o,)):
            t.fill_(3)


def _plan(L, arr, njobs, cache):
    import ctypes
    plan = ctypes.c_void_p()
    st = L.cmp_batch_plan_create(arr, njobs, cache.encode() if cache else None, ctypes.byref(plan))
    assert st == 0, L.cmp_last_error()
    return plan


def test_batch_full_size_autotuned(tmp_path):
    """The 256-job batch (sides log-uniform 64..2048, 2..32 contributors,
    half depth and half over, ROI-cropped) with tiles from cmp_autotune: the
    persistent launch, its graph replays and one plain launch per job give
    the same bits for every job, and every job matches the oracle."""
    jobs = synth.batch_jobs(seed=5, njobs=256, device=DEV)
    note("batch 256 jobs, autotuned tiles")
    L = cmp.lib()
    s = torch.cuda.current_stream().cuda_stream
    cache = str(tmp_path / "tune.txt")
    outs_p, outs_g, outs_l = _alloc_outs(jobs), _alloc_outs(jobs), _alloc_outs(jobs)
    (arr_p, keep_p), (arr_g, keep_g), (arr_l, keep_l) = (_cjobs(jobs, o) for o in (outs_p, outs_g, outs_l))
    assert L.cmp_autotune(arr_l, len(jobs), cache.encode(), 2, s) == 0, L.cmp_last_error()
    lines = [ln for ln in open(cache) if not ln.startswith("#")]
    assert len(lines) > 0
    plan_p, plan_g, plan_l = (_plan(L, a, len(jobs), cache) for a in (arr_p, arr_g, arr_l))
    ws_p = torch.zeros(L.cmp_batch_workspace_size(plan_p) + 64, dtype=torch.uint8, device=DEV)
    ws_g = torch.zeros(L.cmp_batch_workspace_size(plan_g) + 64, dtype=torch.uint8, device=DEV)
    assert L.cmp_batch_upload(plan_p, ws_p.data_ptr(), ws_p.numel(), s) == 0
    assert L.cmp_batch_upload(plan_g, ws_g.data_ptr(), ws_g.numel(), s) == 0
    torch.cuda.synchronize()
    for _ in range(2):   # the queue resets itself between launches
        assert L.cmp_batch_run(plan_p, ws_p.data_ptr(), s) == 0
    _scribble(outs_l)
    assert L.cmp_batch_run_plain(plan_l, s) == 0
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.graph(g, stream=side):
        assert L.cmp_batch_run(plan_g, ws_g.data_ptr(), side.cuda_stream) == 0
    torch.cuda.synchronize()
    for rep in range(3):   # eager work between replays
        _scribble(outs_g)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        bad = [k for k in range(len(jobs)) if not _same(outs_g[k], outs_p[k])]
        assert not bad, (rep, bad[:8])
    bad = [k for k in range(len(jobs)) if not _same(outs_l[k], outs_p[k])]
    assert not bad, bad[:8]
    bad = [k for k, (job, o) in enumerate(zip(jobs, outs_p)) if not _job_check_oracle(job, o)]
    assert not bad, bad[:8]
    for p in (plan_p, plan_g, plan_l):
        L.cmp_batch_plan_destroy(p)
    del g, keep_p, keep_g, keep_l


def test_batch_tune_cache_tiles_do_not_change_results(tmp_path):
    """A plan whose tiles come from a tune cache (rewritten to tiles other
    than the defaults, plus entries the library must reject: a zero width,
    an area above 65536, a negative height) gives the same bits as the
    default-tile plan, persistent and plain."""
    jobs = synth.batch_jobs(seed=7, njobs=40, device=DEV, log2_range=(5.0, 9.5))
    note("batch tune cache vs default tiles")
    L = cmp.lib()
    s = torch.cuda.current_stream().cuda_stream
    cache = str(tmp_path / "tune.txt")
    outs_d, outs_t, outs_l = _alloc_outs(jobs), _alloc_outs(jobs), _alloc_outs(jobs)
    (arr_d, keep_d), (arr_t, keep_t), (arr_l, keep_l) = (_cjobs(jobs, o) for o in (outs_d, outs_t, outs_l))
    assert L.cmp_autotune(arr_l, len(jobs), cache.encode(), 1, s) == 0, L.cmp_last_error()
    head = [ln for ln in open(cache) if ln.startswith("#")]
    rows = [ln.split() for ln in open(cache) if not ln.startswith("#")]
    alt = {0: [(128, 8), (32, 4), (64, 64)], 1: [(16, 16), (256, 1), (32, 2)]}
    with open(cache, "w") as f:
        f.writelines(head)
        for k, r in enumerate(rows):
            if k % 4 == 3:   # invalid tiles: ignored, the default is used
                r[4], r[5] = [("0", "16"), ("512", "256"), ("64", "-4")][k % 3]
            else:
                r[4], r[5] = (str(v) for v in alt[int(r[0])][k % 3])
            f.write(" ".join(r) + "\n")
    plan_d, plan_t, plan_l = _plan(L, arr_d, len(jobs), None), _plan(L, arr_t, len(jobs), cache), \
        _plan(L, arr_l, len(jobs), cache)
    for plan, outs in ((plan_d, outs_d), (plan_t, outs_t)):
        ws = torch.zeros(L.cmp_batch_workspace_size(plan) + 64, dtype=torch.uint8, device=DEV)
        assert L.cmp_batch_upload(plan, ws.data_ptr(), ws.numel(), s) == 0
        assert L.cmp_batch_run(plan, ws.data_ptr(), s) == 0
        torch.cuda.synchronize()
    assert L.cmp_batch_run_plain(plan_l, s) == 0
    torch.cuda.synchronize()
    for k, job in enumerate(jobs):
        assert _same(outs_t[k], outs_d[k]), k
        assert _same(outs_l[k], outs_d[k]), k
    for k in (0, 1, 2, 3):
        assert _job_check_oracle(jobs[k], outs_d[k]), k
    for p in (plan_d, plan_t, plan_l):
        L.cmp_batch_plan_destroy(p)
    del keep_d, keep_t, keep_l


def test_batch_many_contributors():
    """Batched jobs past the 64 a workgroup stages at once: depth jobs of
    65..130 contributors (staged in chunks of 64, later chunks combined with
    the output of earlier ones) and over jobs of 65..130 layers (descriptors
    read from the workspace): the persistent launch equals one plain launch
    per job, and every job matches the oracle."""
    import ctypes
    jobs = synth.batch_jobs(seed=12, njobs=6, device=DEV, log2_range=(5.0, 7.5), n_range=(65, 130))
    assert min(len(j.work.images if j.kind == "depth" else j.work.layers) for j in jobs) >= 65
    outs_p, outs_l = _alloc_outs(jobs), _alloc_outs(jobs)
    arr_p, keep_p = _cjobs(jobs, outs_p)
    arr_l, keep_l = _cjobs(jobs, outs_l)
    L = cmp.lib()
    s = torch.cuda.current_stream().cuda_stream
    plan_p, plan_l = _plan(L, arr_p, len(jobs), None), _plan(L, arr_l, len(jobs), None)
    ws = torch.zeros(L.cmp_batch_workspace_size(plan_p) + 64, dtype=torch.uint8, device=DEV)
    note("batch, 65..130 contributors per job")
    assert L.cmp_batch_upload(plan_p, ws.data_ptr(), ws.numel(), s) == 0
    assert L.cmp_batch_run(plan_p, ws.data_ptr(), s) == 0
    assert L.cmp_batch_run_plain(plan_l, s) == 0
    torch.cuda.synchronize()
    for k, job in enumerate(jobs):
        assert _same(outs_p[k], outs_l[k]), k
        assert _job_check_oracle(job, outs_p[k]), k
    for p in (plan_p, plan_l):
        L.cmp_batch_plan_destroy(p)
    del keep_p, keep_l


def test_batch_plan_reads_tune_cache_from_environment(tmp_path):
    """cmp_batch_plan_create with no path uses the tune cache named by
    CMP_TUNE_CACHE: in a child process with CMP_LOG=1, the plan's log line
    names that file and the entries it read for this device."""
    import subprocess
    import sys
    jobs = synth.batch_jobs(seed=9, njobs=6, device=DEV, log2_range=(5.0, 7.0))
    L = cmp.lib()
    s = torch.cuda.current_stream().cuda_stream
    cache = str(tmp_path / "tune.txt")
    outs = _alloc_outs(jobs)
    arr, keep = _cjobs(jobs, outs)
    note("batch tune cache from CMP_TUNE_CACHE")
    assert L.cmp_autotune(arr, len(jobs), cache.encode(), 1, s) == 0, L.cmp_last_error()
    torch.cuda.synchronize()
    code = (
        "import ctypes, paper_1902_08755_amd as cmp\n"
        "L = cmp.lib()\n"
        "img = (cmp.CImage * 1)(cmp.CImage(0x10000, 0x20000, 64, cmp.Rect(0, 0, 64, 64)))\n"
        "job = cmp.CJob(0, cmp.RGBA8, 1, img, None, cmp.Rect(0, 0, 64, 64), 0x30000, 0x40000, 64)\n"
        "plan = ctypes.c_void_p()\n"
        "assert L.cmp_batch_plan_create(ctypes.byref(job), 1, None, ctypes.byref(plan)) == 0\n"
        "L.cmp_batch_plan_destroy(plan)\n")
    env = dict(os.environ, CMP_LOG="1", CMP_TUNE_CACHE=cache)
    r = subprocess.run([sys.executable, "-c", code], cwd=os.path.dirname(os.path.dirname(
        os.path.abspath(__file__))), env=env, capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stderr.splitlines() if ln.startswith("[cmp] batch plan")]
    assert len(lines) == 1 and f"tune cache {cache} (" in lines[0], r.stderr[-2000:]
    entries = int(lines[0].split(f"tune cache {cache} (")[1].split()[0])
    assert entries > 0, lines[0]
    del keep


def test_batch_graph_replay():
    """The persistent launch captured in a HIP graph and replayed several times,
    with eager work in between; every replay matches the eager result."""
    import ctypes
    jobs = synth.batch_jobs(seed=6, njobs=12, device=DEV, log2_range=(4.0, 8.0), n_range=(2, 6))
    outs = _alloc_outs(jobs)
    arr, keep = _cjobs(jobs, outs)
    L = cmp.lib()
    plan = ctypes.c_void_p()
    assert L.cmp_batch_plan_create(arr, len(jobs), None, ctypes.byref(plan)) == 0
    ws = torch.zeros(L.cmp_batch_workspace_size(plan) + 64, dtype=torch.uint8, device=DEV)
    stream = torch.cuda.Stream()
    note("batch graph replay")
    with torch.cuda.stream(stream):
        assert L.cmp_batch_upload(plan, ws.data_ptr(), ws.numel(), stream.cuda_stream) == 0
        assert L.cmp_batch_run(plan, ws.data_ptr(), stream.cuda_stream) == 0
    stream.synchronize()
    eager = [tuple(t.clone() for t in o) if isinstance(o, tuple) else o.clone() for o in outs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        assert L.cmp_batch_run(plan, ws.data_ptr(), stream.cuda_stream) == 0
    for rep in range(4):
        for o in outs:   # scribble, then replay
            (o[0] if isinstance(o, tuple) else o).fill_(3)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for o, e in zip(outs, eager):
            if isinstance(o, tuple):
                assert torch.equal(o[0], e[0]) and torch.equal(o[1], e[1])
            else:
                assert torch.equal(o, e)
    L.cmp_batch_plan_destroy(plan)
    del keep


# --------------------------------------------------------- whole pipeline
def test_ramp_pipeline_full_size():
    """16 x 1920x1080: roi_detect -> RLE compress -> decompress -> depth
    compositing (binary swap over 16 owners), against the oracle chain."""
    note("pipeline 16x1920x1080")
    wl = synth.depth_ramps_full(seed=2, n=16, W=1920, H=1080, device=DEV)
    roi = cmp.roi_detect(wl.images)
    batch = cmp.RleBatch(wl.images, roi_dev=roi)
    streams, sizes, _ = batch.run()
    blocks = [cmp.Image(torch.zeros((1080, 1920), dtype=torch.int32, device=DEV),
                        torch.zeros((1080, 1920), dtype=torch.int32, device=DEV), (0, 0, 1920, 1080))
              for _ in range(16)]
    ro, st = cmp.rle_decompress(streams, blocks)
    placed = [cmp.Image(b.color, b.depth, (0, 0, 1920, 1080)) for b in blocks]
    oc, od = cmp.composite_depth(placed, wl.viewport, roi_dev=ro, schedule=("binary_swap", 16))
    torch.cuda.synchronize()
    assert (st == 0).all() and int(batch.status.abs().sum()) == 0
    # oracle chain
    rois = [oracle.roi_detect_depth(u32(im.depth)) for im in wl.images]
    assert [tuple(r) for r in roi.cpu().tolist()] == rois
    crops_c, crops_d = [], []
    for k, im in enumerate(wl.images):
        c, d = u32(im.color), u32(im.depth)
        ref = oracle.rle_compress(c, d, rois[k])
        n = int(sizes[k])
        assert n == ref.size and (streams[k][:n].cpu().numpy() == ref).all(), k
        r2, c2, d2 = oracle.rle_decompress(ref)
        crops_c.append(c2)
        crops_d.append(d2)
    ref_c, ref_d = oracle.composite_depth(crops_c, crops_d, rois, wl.viewport)
    assert (u32(oc) == ref_c).all() and (u32(od) == ref_d).all()
    # cropping is lossless: the same as compositing the full frames
    full_c, full_d = _oracle_depth(wl.images, wl.viewport)
    assert (ref_c == full_c).all() and (ref_d == full_d).all()


@pytest.mark.parametrize("nframes,groups_per_cu,own_streams", [(2, 0, False), (4, 3, False),
                                                              (4, 2, True)])
def test_frames_in_flight_match_one_at_a_time(nframes, groups_per_cu, own_streams):
    """The benchmark's asynchronous mode: several frames' whole chains (ROI,
    RLE compress, decompress, depth compositing) on as many streams at once
    (torch's or the library's own, cmp_streams_create), with the RLE
    kernels' occupancy capped or not, give the same streams and
    composites as running them one after the other (compressions on
    different streams overlap freely: blocks come from per-image tickets)."""
    note(f"{nframes} frames in flight, RLE groups per CU {groups_per_cu}, own {own_streams}")
    frames = [synth.depth_ramps_full(seed=s, n=16, W=1920, H=1080, device=DEV)
              for s in range(2, 2 + nframes)]

    def chain(wl, stream):
        with torch.cuda.stream(stream):
            # calls that may overlap need their own ROI workspace
            need = cmp.lib().cmp_roi_workspace_size(cmp._images(wl.images, "u32"), len(wl.images))
            ws = torch.zeros(need, dtype=torch.uint8, device=DEV)
            roi = cmp.roi_detect(wl.images, ws=ws)
            batch = cmp.RleBatch(wl.images, roi_dev=roi)
            streams, sizes, _ = batch.run()
            blocks = [cmp.Image(torch.zeros((1080, 1920), dtype=torch.int32, device=DEV),
                                torch.zeros((1080, 1920), dtype=torch.int32, device=DEV),
                                (0, 0, 1920, 1080)) for _ in range(16)]
            ro, st = cmp.rle_decompress(streams, blocks)
            placed = [cmp.Image(b.color, b.depth, (0, 0, 1920, 1080)) for b in blocks]
            oc, od = cmp.composite_depth(placed, wl.viewport, roi_dev=ro,
                                         schedule=("binary_swap", 16))
        return roi, streams, sizes, st, oc, od, batch.status

    main = torch.cuda.current_stream()
    seq = [chain(wl, main) for wl in frames]
    torch.cuda.synchronize()
    cmp.rle_set_groups_per_cu(groups_per_cu, groups_per_cu)
    own = cmp.Streams(nframes) if own_streams else None
    try:
        side = own.streams if own else [torch.cuda.Stream() for _ in frames]
        for st in side:
            st.wait_stream(main)
        par = [chain(wl, st) for wl, st in zip(frames, side)]
        for st in side:
            main.wait_stream(st)
        torch.cuda.synchronize()
    finally:
        cmp.rle_set_groups_per_cu(0, 0)
        if own:
            own.close()
    for a, b in zip(seq, par):
        assert torch.equal(a[0], b[0])
        assert (a[6] == 0).all() and (b[6] == 0).all()   # compression finished in time
        assert torch.equal(a[2], b[2]) and (a[3] == 0).all() and (b[3] == 0).all()
        for k in range(16):
            n = int(a[2][k])
            assert torch.equal(a[1][k][:n], b[1][k][:n]), k
        assert torch.equal(a[4], b[4]) and torch.equal(a[5], b[5])


def test_rle_swizzled_streams():
    """Bit-swizzled colour planes: byte-identical streams and round trips."""
    wl = synth.depth_ramps_full(seed=2, n=4, W=640, H=360, device=DEV)
    rng = np.random.default_rng(8)
    noise = torch.from_numpy(rng.integers(0, 2 ** 32, (90, 200), dtype=np.uint64)
                             .astype(np.uint32).view(np.int32)).to(DEV)
    imgs = list(wl.images) + [cmp.Image(noise, noise.clone(), (0, 0, 200, 90)),
                              cmp.Image(noise.clone(), None, (0, 0, 200, 90))]
    roi = cmp.roi_detect(imgs[:4])
    rois = [tuple(r) for r in roi.cpu().tolist()] + [(3, 4, 190, 81), (0, 0, 200, 90)]
    rd = torch.tensor(rois, dtype=torch.int32, device=DEV)
    note("rle swizzled")
    streams, sizes, cst = cmp.rle_compress(imgs, roi_dev=rd, swizzle=True)
    torch.cuda.synchronize()
    assert (cst == 0).all()
    for k, im in enumerate(imgs):
        c = u32(im.color)
        d = u32(im.depth) if im.depth is not None else None
        ref = oracle.rle_compress(c, d, rois[k], swizzle=True)
        n = int(sizes[k])
        assert n == ref.size and (streams[k][:n].cpu().numpy() == ref).all(), k
    outs = [cmp.Image(torch.zeros_like(im.color), None if im.depth is None else torch.zeros_like(im.depth),
                      im.roi) for im in imgs]
    _, st = cmp.rle_decompress(streams, outs)
    torch.cuda.synchronize()
    assert (st == 0).all()
    for im, o, (x, y, w, h) in zip(imgs, outs, rois):
        assert torch.equal(o.color[:h, :w], im.color[y:y + h, x:x + w])


# ------------------------------------------------------ subpixel / pixel
@pytest.mark.parametrize("n", [1, 2, 3, 8, 16, 64])
def test_composite_average(n):
    """Subpixel compositing: 4 x 640x480 style samples, partial placements,
    every schedule and tile bit-identical to the oracle."""
    rng = np.random.default_rng(500 + n)
    W, H = 333, 201
    imgs = []
    for i in range(n):
        full = i % 3 != 2
        w, h = (W, H) if full else (int(rng.integers(1, W)), int(rng.integers(1, H)))
        x, y = (0, 0) if full else (int(rng.integers(-5, W)), int(rng.integers(-5, H)))
        P = w + int(rng.integers(0, 4))
        c = rng.integers(0, 2 ** 32, (h, P), dtype=np.uint64).astype(np.uint32)
        imgs.append(cmp.Image(torch.from_numpy(c.view(np.int32)).to(DEV), None, (x, y, w, h)))
    vp = (2, 3, W, H)
    note(f"average n={n}")
    ref = oracle.composite_average([u32(i.color) for i in imgs], [i.roi for i in imgs], vp)
    for sched, tile in [(("seq", 1), (0, 0)), (("direct_send", 5), (64, 8)),
                        (("binary_swap", 16), (128, 4)), (("seq", 1), (50, 3))]:
        out = cmp.composite_average(imgs, vp, schedule=sched, tile=tile)
        torch.cuda.synchronize()
        assert (u32(out) == ref).all(), (sched, tile)


@pytest.mark.parametrize("kx,ky", [(2, 2), (3, 2), (1, 4), (8, 8), (4, 1)])
def test_assemble_pixels(kx, ky):
    rng = np.random.default_rng(kx * 31 + ky)
    W, H = 517, 203
    img = rng.integers(0, 2 ** 32, (H, W), dtype=np.uint64).astype(np.uint32)
    imgs, offs = [], []
    classes = [(ox, oy) for oy in range(ky) for ox in range(kx)]
    rng.shuffle(classes)
    drop = classes[-1] if len(classes) > 2 else None
    for (ox, oy) in classes:
        if (ox, oy) == drop:
            continue      # one class without a source stays 0
        part = np.ascontiguousarray(img[oy::ky, ox::kx])
        P = part.shape[1] + 3
        buf = np.zeros((part.shape[0], P), np.uint32)
        buf[:, :part.shape[1]] = part
        imgs.append(cmp.Image(torch.from_numpy(buf.view(np.int32)).to(DEV), None,
                              (0, 0, part.shape[1], part.shape[0])))
        offs.append((ox, oy))
    note(f"assemble {kx}x{ky}")
    out = cmp.assemble_pixels(imgs, offs, (kx, ky), (0, 0, W, H))
    torch.cuda.synchronize()
    ref = oracle.assemble_pixels([u32(i.color) for i in imgs], offs, (kx, ky), (0, 0, W, H))
    assert (u32(out) == ref).all()
    exp = img.copy()
    if drop is not None:
        exp[drop[1]::ky, drop[0]::kx] = 0
    assert (ref == exp).all()


@pytest.mark.parametrize("fmt,cell", [("depth", (64, 64)), ("depth", (7, 5)), ("rgba8", (16, 16)),
                                      ("f32", (32, 8)), ("f16", (3, 3)), ("depth", (5000, 2))])
def test_roi_grid_holes(fmt, cell):
    rng = np.random.default_rng(len(fmt) * 100 + cell[0])
    imgs, refs = [], []
    for k, (h, w) in enumerate([(130, 257), (64, 64), (1, 1), (211, 333)]):
        P = w + (k % 2) * 4
        m = np.zeros((h, P), bool)
        for _ in range(4):   # a few blobs leave holes between them
            y, x = rng.integers(0, h), rng.integers(0, w)
            m[y:y + 9, x:x + 13] = True
        m[:, w:] = False
        if fmt in ("depth", "rgba8"):
            a = np.where(m, rng.integers(1, F - 1, (h, P), dtype=np.uint64), F if fmt == "depth" else 0).astype(np.uint32)
            t = torch.from_numpy(a.view(np.int32)).to(DEV)
            imgs.append(cmp.Image(t, t if fmt == "depth" else None, (0, 0, w, h)))
            refs.append(oracle.roi_grid(a, cell, mode=fmt, w=w, h=h))
        else:
            L = np.zeros((h, P, 4), np.float32)
            L[m, 2] = 0.75
            L[~m, 0] = -0.0
            L = L.astype(np.float16 if fmt == "f16" else np.float32)
            imgs.append(cmp.Image(torch.from_numpy(L).to(DEV), None, (0, 0, w, h)))
            refs.append(oracle.roi_grid(L, cell, mode="float", w=w, h=h))
    note(f"roi grid {fmt} {cell}")
    f = {"depth": cmp.RGBA8, "rgba8": cmp.RGBA8, "f32": cmp.RGBA32F, "f16": cmp.RGBA16F}[fmt]
    grids = cmp.roi_grid(imgs, cell, fmt=f)
    torch.cuda.synchronize()
    for g, r in zip(grids, refs):
        assert (g.cpu().numpy() == r).all()


def _rle_outputs_ok(imgs, rois, streams, sizes, status):
    """Every stream either matches the oracle (status 0) or reports
    CMP_ETIMEOUT and is rejected by decompression."""
    st = status.cpu().tolist()
    outs = [cmp.Image(torch.zeros_like(im.color), torch.zeros_like(im.depth), im.roi) for im in imgs]
    _, dst = cmp.rle_decompress(streams, outs)
    torch.cuda.synchronize()
    dst = dst.cpu().tolist()
    timed_out = 0
    for k, im in enumerate(imgs):
        if st[k] == cmp.CMP_ETIMEOUT:
            timed_out += 1
            assert dst[k] == cmp.CMP_ECORRUPT, k
            continue
        assert st[k] == 0, k
        ref = oracle.rle_compress(u32(im.color), u32(im.depth), rois[k])
        n = int(sizes[k])
        assert n == ref.size and (streams[k][:n].cpu().numpy() == ref).all(), k
        assert dst[k] == 0, k
    return timed_out


def test_rle_compress_gives_up_cleanly():
    """The compressor's failure path, forced from the host: with a wait limit
    of zero polls a block whose predecessors are not done gives up at once.
    Such a stream must report CMP_ETIMEOUT and fail to decode (its offset
    entry is invalid); every other stream is still exact. Afterwards the
    default limit gives exact streams everywhere."""
    wl = synth.depth_ramps_full(seed=2, n=16, W=1920, H=1080, device=DEV)
    roi = cmp.roi_detect(wl.images)
    torch.cuda.synchronize()
    rois = [tuple(r) for r in roi.cpu().tolist()]
    note("rle forced wait limit 0")
    cmp.rle_set_wait_limit(0)
    try:
        seen = 0
        for _ in range(3):
            streams, sizes, st = cmp.rle_compress(wl.images, roi_dev=roi)
            seen += _rle_outputs_ok(wl.images, rois, streams, sizes, st)
    finally:
        cmp.rle_set_wait_limit(-1)
    print(f"[rle] streams that gave up with a zero wait limit: {seen} of 48", flush=True)
    streams, sizes, st = cmp.rle_compress(wl.images, roi_dev=roi)
    assert _rle_outputs_ok(wl.images, rois, streams, sizes, st) == 0


def test_rle_graph_replay_alongside_eager():
    """A compression captured in a HIP graph and replayed while eager
    compressions of other frames run on another stream (each call with its
    own workspace): every replay and every eager call gives the oracle's
    streams."""
    frames = [synth.depth_ramps_full(seed=s, n=8, W=1280, H=720, device=DEV) for s in (11, 12)]
    rois = []
    for wl in frames:
        r = cmp.roi_detect(wl.images, ws=torch.zeros(1 << 16, dtype=torch.uint8, device=DEV))
        rois.append(r.clone())
    torch.cuda.synchronize()
    note("rle graph replay alongside eager")
    cap_stream, eager_stream = torch.cuda.Stream(), torch.cuda.Stream()
    b_graph = cmp.RleBatch(frames[0].images, roi_dev=rois[0])
    b_eager = cmp.RleBatch(frames[1].images, roi_dev=rois[1])
    cap_stream.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=cap_stream):
        b_graph.run(stream=cap_stream)
    torch.cuda.synchronize()
    refs = [[oracle.rle_compress(u32(im.color), u32(im.depth), tuple(r))
             for im, r in zip(wl.images, ro.cpu().tolist())] for wl, ro in zip(frames, rois)]
    for rep in range(4):
        for o in b_graph.outs + b_eager.outs:
            o.fill_(0xAB)
        b_graph.status.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(cap_stream):
            g.replay()
        for _ in range(2):
            b_eager.run(stream=eager_stream)
        torch.cuda.synchronize()
        for b, ref in ((b_graph, refs[0]), (b_eager, refs[1])):
            assert (b.status == 0).all(), rep
            for k, r in enumerate(ref):
                n = int(b.sizes[k])
                assert n == r.size and (b.outs[k][:n].cpu().numpy() == r).all(), (rep, k)
