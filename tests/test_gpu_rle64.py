"""GPU parity of the basic 64-bit RLE (RL64, thesis Section 5.5.1: two RGBA8
pixels per 64-bit token): streams byte-identical to the oracle's, round
trips, malformed streams rejected with the oracle's verdict, and the 16 x
1920x1080 workload at full size."""
import numpy as np
import pytest
import torch

import oracle
import paper_1902_08755_amd as cmp
import synth
from conftest import read_golden

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)
F = 0xFFFFFFFF


def note(msg):
    print(f"[gpu case] {msg}", flush=True)


def _golden(name):
    sec = read_golden("rl64_examples.txt")[name]
    return np.array([int(t, 16) for row in sec for t in row], np.uint8)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a).view(np.int32)).to(DEV)


def _check(imgs, rois, streams, sizes, status):
    """Every GPU stream equals the oracle's for the same ROI."""
    assert int(status.abs().sum()) == 0
    for k, im in enumerate(imgs):
        c = synth.as_u32(im.color)
        d = None if im.depth is None else synth.as_u32(im.depth)
        ref = oracle.rle64_compress(c, d, rois[k])
        n = int(sizes[k])
        assert n == ref.size, (k, n, ref.size)
        assert (streams[k][:n].cpu().numpy() == ref).all(), k


def _round_trip(imgs, rois, streams):
    outs = [cmp.Image(torch.zeros_like(im.color),
                      None if im.depth is None else torch.zeros_like(im.depth), im.roi)
            for im in imgs]
    ro, st = cmp.rle64_decompress(streams, outs)
    torch.cuda.synchronize()
    assert (st == 0).all(), st.tolist()
    assert [tuple(r) for r in ro.cpu().tolist()] == [tuple(r) for r in rois]
    for im, o, (x, y, w, h) in zip(imgs, outs, rois):
        if w * h == 0:
            continue
        assert torch.equal(o.color[:h, :w], im.color[y:y + h, x:x + w])
        if im.depth is not None:
            assert torch.equal(o.depth[:h, :w], im.depth[y:y + h, x:x + w])


def test_rle64_hand_worked_streams():
    """The three hand-derived streams of tests/golden/rl64_examples.txt."""
    run = np.full((1, 300), 0x7E7E7E7E, np.uint32)
    odd = np.array([[7] * 8 + [9]], np.uint32)
    depth = np.array([[5, 5, F, F], [5, 3, F, F], [F, F, F, F], [F, F, 7, F]], np.uint32)
    color = np.where(depth != F, 0xFF332211, 0).astype(np.uint32)
    imgs = [cmp.Image(_dev(run), None, (0, 0, 300, 1)), cmp.Image(_dev(odd), None, (0, 0, 9, 1)),
            cmp.Image(_dev(color), _dev(depth), (0, 0, 4, 4))]
    rois = [(0, 0, 300, 1), (0, 0, 9, 1), (0, 0, 3, 4)]
    note("rl64 hand-worked")
    streams, sizes, st = cmp.rle64_compress(imgs, torch.tensor(rois, dtype=torch.int32, device=DEV))
    torch.cuda.synchronize()
    assert int(st.abs().sum()) == 0
    for k, name in enumerate(["run300", "odd9", "worked_A"]):
        g = _golden(name)
        assert int(sizes[k]) == g.size and (streams[k][:g.size].cpu().numpy() == g).all(), name
    _round_trip(imgs, rois, streams)


def test_rle64_adversarial_images():
    """Pixel-pair runs of 127/128/129 symbols (crossing 128-symbol segments),
    odd ROI widths and block tails, single pixels, one-block and block+1
    ROIs, empty ROIs, noise, colour-only images, several images per launch,
    the workspace reused."""
    rng = np.random.default_rng(64)
    specs = [((1, 1), (0, 0, 1, 1)), ((130, 150), (7, 3, 129, 101)), ((64, 128), (0, 0, 128, 32)),
             ((65, 64), (0, 0, 64, 65)), ((20, 30), (5, 5, 0, 7)), ((300, 301), (0, 0, 301, 300)),
             ((40, 4100), (1, 2, 4097, 3)), ((33, 33), (32, 32, 1, 1)), ((9, 11), (0, 0, 11, 9))]
    imgs, rois = [], []
    for k, ((H, W), roi) in enumerate(specs):
        c = np.zeros((H, W), np.uint32)
        d = np.full((H, W), F, np.uint32)
        flat, dflat = c.reshape(-1), d.reshape(-1)
        pos = 0
        # runs in pixels: pairs of 127, 128 and 129 symbols, odd runs that
        # split pairs, single pixels
        for run in [254, 256, 258, 1, 3, 2, 255, 257, 4095, 4096, 4097, 8190]:
            if pos >= flat.size:
                break
            flat[pos:pos + run] = rng.integers(0, 2 ** 32, dtype=np.uint64)
            dflat[pos:pos + run] = rng.integers(0, 4, dtype=np.uint64) + 100
            pos = min(flat.size, pos + run)
        k2 = min(flat.size, pos + 3000)
        flat[pos:k2] = rng.integers(0, 2 ** 32, k2 - pos, dtype=np.uint64).astype(np.uint32)
        imgs.append(cmp.Image(_dev(c), _dev(d) if k % 3 else None, (0, 0, W, H)))
        rois.append(roi)
    rd = torch.tensor(rois, dtype=torch.int32, device=DEV)
    note("rl64 adversarial")
    clean = [r if r[2] * r[3] else (0, 0, 0, 0) for r in rois]
    for rep in range(3):
        streams, sizes, st = cmp.rle64_compress(imgs, rd)
        torch.cuda.synchronize()
        _check(imgs, clean, streams, sizes, st)
    _round_trip(imgs, clean, streams)


def test_rle64_ramps_full_size():
    """The 16 x 1920x1080 workload: ROIs found on the device, RL64 streams
    byte-identical to the oracle's, round trip; prints the space saved by
    RL64, per-component RLE and swizzled per-component RLE."""
    wl = synth.depth_ramps_full(seed=2, n=16, W=1920, H=1080, device=DEV)
    roi = cmp.roi_detect(wl.images)
    note("rl64 ramps 16 x 1920x1080")
    streams, sizes, st = cmp.rle64_compress(wl.images, roi)
    torch.cuda.synchronize()
    rois = [tuple(r) for r in roi.cpu().tolist()]
    _check(wl.images, rois, streams, sizes, st)
    _round_trip(wl.images, rois, streams)
    raw = sum(8 * w * h for _, _, w, h in rois)
    _, s1, _ = cmp.rle_compress(wl.images, roi_dev=roi)
    _, s2, _ = cmp.rle_compress(wl.images, roi_dev=roi, swizzle=True)
    torch.cuda.synchronize()
    for name, tot in (("rl64", int(sizes.sum())), ("rle1", int(s1.sum())),
                      ("rle1_swizzled", int(s2.sum()))):
        print(f"[space] {name}: {tot} of {raw} raw bytes, saves {100 * (1 - tot / raw):.1f}%")


def test_rle64_decompress_rejects_malformed_streams():
    """Each corruption of a valid stream is rejected by the oracle and by the
    GPU (CMP_ECORRUPT); the valid stream decodes; a small destination or a
    missing depth buffer gives CMP_ENOSPC."""
    run = np.full((1, 300), 0x7E7E7E7E, np.uint32)
    dep = np.full((1, 300), 0x01020304, np.uint32)
    dep[0, 299] = 5                     # odd count 300 -> last symbol (5-pair) differs
    good = oracle.rle64_compress(run, dep, (0, 0, 300, 1))
    # layout: header 32, boff 4, sizes 8 -> payload at 48; colour tokens
    # (2 runs: 8 + 16 bytes) at 48, depth tokens (3 runs) at 72
    assert good[48] == 0x7F and good[49] == 0x15 and good[72:75].tolist() == [0x7F, 0x14, 0]
    odd = oracle.rle64_compress(np.array([[7] * 8 + [9]], np.uint32), None, (0, 0, 9, 1))
    raw = oracle.rle64_compress(np.arange(5, dtype=np.uint32).reshape(1, 5) * 77 + 1, None,
                                (0, 0, 5, 1))
    assert raw[36] == 24   # 3 raw symbols
    cases = []
    def corrupt(base, edits, name):
        s = base.copy()
        for pos, val in edits.items():
            s[pos] = val
        cases.append((name, s))
    corrupt(good, {0: 0x53}, "magic")
    corrupt(good, {20: 3}, "nstreams")
    corrupt(good, {28: 2}, "nblocks")
    corrupt(good, {36: 25}, "size_not_multiple_of_8")
    corrupt(good, {36: 8}, "size_of_no_run_count")
    corrupt(good, {48: 99, 49: 49}, "run_crosses_segment")   # runs 100 + 50: the second crosses 128
    corrupt(good, {49: 0x16}, "lengths_overrun")             # 128 + 23 > 150 symbols
    corrupt(good, {48: 0x7E}, "lengths_short")               # 127 + 22 < 150 symbols
    corrupt(good, {50: 1}, "length_padding")
    corrupt(good, {33: 1}, "boff")
    corrupt(odd, {68: 1}, "odd_partner")                     # last symbol (9, 0) -> (9, 1)
    corrupt(raw, {72: 1}, "block_padding")
    for name, s in cases:
        with pytest.raises(oracle.CorruptStream):
            oracle.rle64_decompress(s)
    names = [n for n, _ in cases] + ["good", "small", "nodepth"]
    streams = [torch.from_numpy(s).to(DEV) for _, s in cases] + \
              [torch.from_numpy(good).to(DEV)] * 3
    def out(w, h, depth=True):
        return cmp.Image(torch.zeros((h, w), dtype=torch.int32, device=DEV),
                         torch.zeros((h, w), dtype=torch.int32, device=DEV) if depth else None,
                         (0, 0, w, h))
    outs = [out(300, 1) for _ in cases] + [out(300, 1), out(299, 1), out(300, 1, depth=False)]
    note("rl64 malformed")
    _, st = cmp.rle64_decompress(streams, outs)
    torch.cuda.synchronize()
    st = st.cpu().tolist()
    for name, s in zip(names, st):
        if name == "good":
            assert s == 0
        elif name in ("small", "nodepth"):
            assert s == cmp.CMP_ENOSPC, name
        else:
            assert s == cmp.CMP_ECORRUPT, name
    g = outs[names.index("good")]
    assert (synth.as_u32(g.color) == run).all() and (synth.as_u32(g.depth) == dep).all()
