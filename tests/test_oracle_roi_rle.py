"""Pins of the oracle's ROI detection and per-component RLE.

ROI: brute force with numpy's nonzero, rectangles the generator placed itself,
corner, empty and full images, and the float emptiness readings.
RLE: the hand-derived RLE1 byte streams in tests/golden, an independent parser
and decoder written here in plain Python (structure, maximal runs, the raw
rule, the layout), round trips on adversarial planes, and corrupt streams."""
import struct

import numpy as np
import pytest

import oracle
import synth
from conftest import read_hex

F = 0xFFFFFFFF


# ------------------------------------------------------------------- ROI
def _np_bbox(mask):
    ys, xs = np.nonzero(mask)
    if len(xs) == 0:
        return (0, 0, 0, 0)
    return (int(xs.min()), int(ys.min()), int(xs.max() - xs.min() + 1), int(ys.max() - ys.min() + 1))


@pytest.mark.parametrize("seed", range(8))
def test_roi_brute_force(seed):
    rng = np.random.default_rng(seed)
    H, W, P = int(rng.integers(1, 20)), int(rng.integers(1, 20)), 0
    P = W + int(rng.integers(0, 4))
    d = np.full((H, P), F, np.uint32)
    m = rng.random((H, P)) < (0.02 if seed % 2 else 0.3)
    d[m] = rng.integers(0, F, m.sum(), dtype=np.uint64).astype(np.uint32)
    assert oracle.roi_detect_depth(d, W, H) == _np_bbox(m[:, :W])
    c = np.where(m, rng.integers(1, 2 ** 32, (H, P), dtype=np.uint64), 0).astype(np.uint32)
    assert oracle.roi_detect_rgba8(c, W, H) == _np_bbox(c[:, :W] != 0)
    f = np.zeros((H, P, 4), np.float32)
    f[m, int(seed % 4)] = rng.random(m.sum()).astype(np.float32) + 0.5
    assert oracle.roi_detect_rgbaf(f, W, H) == _np_bbox(m[:, :W])


def test_roi_special_images():
    d = np.full((7, 9), F, np.uint32)
    assert oracle.roi_detect_depth(d) == (0, 0, 0, 0)
    d[6, 8] = 0
    assert oracle.roi_detect_depth(d) == (8, 6, 1, 1)
    d[0, 0] = F - 1
    assert oracle.roi_detect_depth(d) == (0, 0, 9, 7)
    assert oracle.roi_detect_depth(np.zeros((7, 9), np.uint32)) == (0, 0, 9, 7)
    # float readings: -0.0 is empty, NaN is data
    f = np.zeros((4, 5, 4), np.float32)
    f[1, 2, 0] = -0.0
    assert oracle.roi_detect_rgbaf(f) == (0, 0, 0, 0)
    f[2, 3, 3] = np.nan
    assert oracle.roi_detect_rgbaf(f) == (3, 2, 1, 1)
    h = np.zeros((4, 5, 4), np.float16)
    h[3, 1, 2] = np.float16(6e-8)  # smallest fp16 subnormal is data
    assert oracle.roi_detect_rgbaf(h) == (1, 3, 1, 1)


def test_roi_of_generated_contributors_is_exact():
    """The ramp generator knows the rectangle it drew; depth noise stays below
    the clear value, so detection must return it exactly."""
    for i in range(6):
        img = synth.ramp_image(2, i, i, 160, 90, pitch_pad=64)
        d = synth.as_u32(img.depth)
        assert oracle.roi_detect_depth(d, 160, 90) == img.true_roi


# ------------------------------------------------------------------- RLE
class Parsed:
    pass


def parse_rle1(s: bytes):
    """Independent reader of the RLE1 layout (plain Python)."""
    p = Parsed()
    magic, x, y, w, h, npl, blk, nb = struct.unpack_from("<IiiiiIII", s, 0)
    assert magic == 0x31454C52 and blk == 4096
    p.roi, p.nplanes, p.nblocks = (x, y, w, h), npl, nb
    npx = w * h
    assert nb == -(-npx // 4096)
    boff = struct.unpack_from(f"<{nb}I", s, 32)
    sizes = struct.unpack_from(f"<{nb * npl}I", s, 32 + 4 * nb)
    p0 = 32 + 4 * nb * (1 + npl)
    p0 = (p0 + 15) // 16 * 16
    assert all(b == 0 for b in s[32 + 4 * nb * (1 + npl):p0])
    planes = [bytearray() for _ in range(npl)]
    pos = 0
    p.tokens = []
    for b in range(nb):
        ln = min(4096, npx - 4096 * b)
        assert boff[b] == pos and pos % 16 == 0
        q = p0 + pos
        tot = 0
        for k in range(npl):
            sz = sizes[b * npl + k]
            enc = s[q:q + sz]
            if sz == ln:
                planes[k] += enc
                p.tokens.append(None)
            else:
                assert sz % 2 == 0 and 0 < sz < ln
                toks = [(enc[2 * t] + 1, enc[2 * t + 1]) for t in range(sz // 2)]
                assert sum(r for r, _ in toks) == ln
                # the raw rule: tokens only when strictly smaller
                assert 2 * len(toks) < ln
                # maximal runs that never cross a multiple of 256 pixels
                start = 4096 * b
                for (r, v), nxt in zip(toks, toks[1:] + [None]):
                    assert start // 256 == (start + r - 1) // 256
                    if nxt is not None and (start + r) % 256 != 0:
                        assert nxt[1] != v
                    start += r
                for r, v in toks:
                    planes[k] += bytes([v]) * r
                p.tokens.append(toks)
            q += sz
            tot += sz
        padded = (tot + 15) // 16 * 16
        assert all(c == 0 for c in s[p0 + pos + tot:p0 + pos + padded])
        pos += padded
    assert len(s) == p0 + pos
    p.planes = [bytes(pl) for pl in planes]
    return p


def _planes_of(color, depth, roi):
    x, y, w, h = roi
    words = [color[y:y + h, x:x + w].reshape(-1)]
    if depth is not None:
        words.append(depth[y:y + h, x:x + w].reshape(-1))
    out = []
    for wd in words:
        for k in range(4):
            out.append(((wd >> (8 * k)) & 0xFF).astype(np.uint8).tobytes())
    return out


def test_golden_stream_of_worked_example():
    depth = np.array([[5, 5, F, F], [5, 3, F, F], [F, F, F, F], [F, F, 7, F]], np.uint32)
    color = np.where(depth != F, 0xFF332211, 0).astype(np.uint32)
    roi = oracle.roi_detect_depth(depth)
    assert roi == (0, 0, 3, 4)
    exp = read_hex("rle_A_roi.txt")
    assert len(exp) == 176
    got = oracle.rle_compress(color, depth, roi).tobytes()
    assert got == exp
    r, c, d = oracle.rle_decompress(np.frombuffer(exp, np.uint8))
    assert r == roi and (c == color[:, :3]).all() and (d == depth[:, :3]).all()
    parse_rle1(exp)


def test_golden_stream_run_across_256():
    color = np.full((1, 300), 0x7E7E7E7E, np.uint32)
    exp = read_hex("rle_run300.txt")
    got = oracle.rle_compress(color, color.copy(), (0, 0, 300, 1)).tobytes()
    assert got == exp


def test_hand_built_two_block_stream():
    """4097 pixels of colour 0 and clear depth: block 0 holds 16 runs of 256
    per plane (32 bytes), block 1 one pixel per plane, stored raw (2 >= 1)."""
    color = np.zeros((1, 4097), np.uint32)
    depth = np.full((1, 4097), F, np.uint32)
    hdr = struct.pack("<IiiiiIII", 0x31454C52, 0, 0, 4097, 1, 8, 4096, 2)
    boff = struct.pack("<2I", 0, 256)
    sizes = struct.pack("<16I", *([32] * 8 + [1] * 8))
    tables = hdr + boff + sizes
    tables += b"\0" * (112 - len(tables))
    block0 = b"\xff\x00" * 16 * 4 + b"\xff\xff" * 16 * 4
    block1 = b"\x00" * 4 + b"\xff" * 4 + b"\0" * 8
    exp = tables + block0 + block1
    assert len(exp) == 384
    assert oracle.rle_compress(color, depth, (0, 0, 4097, 1)).tobytes() == exp


def _adversarial_images(rng, H, W):
    c = np.zeros((H, W), np.uint32)
    d = np.full((H, W), F, np.uint32)
    flat = c.reshape(-1)
    dflat = d.reshape(-1)
    n = flat.size
    # runs of 255, 256, 257 and 1, noise, and a long constant tail
    pos = 0
    for run in [255, 256, 257, 1, 1, 2, 511, 513, 4095, 4096, 4097]:
        if pos >= n:
            break
        flat[pos:pos + run] = rng.integers(0, 2 ** 32, dtype=np.uint64)
        dflat[pos:pos + run] = rng.integers(0, 2 ** 32, dtype=np.uint64)
        pos = min(n, pos + run)
    k = min(n, pos + 3000)
    flat[pos:k] = rng.integers(0, 2 ** 32, k - pos, dtype=np.uint64).astype(np.uint32)
    dflat[pos:k] = rng.integers(0, 2 ** 32, k - pos, dtype=np.uint64).astype(np.uint32)
    return c, d


@pytest.mark.parametrize("shape,roi", [
    ((1, 1), (0, 0, 1, 1)),
    ((130, 150), (0, 0, 150, 130)),
    ((130, 150), (7, 3, 129, 101)),
    ((64, 128), (0, 0, 128, 32)),    # exactly one block
    ((65, 64), (0, 0, 64, 65)),      # one block + 64 pixels
    ((20, 30), (5, 5, 0, 7)),        # empty ROI
])
def test_round_trip_and_structure(shape, roi):
    rng = np.random.default_rng(sum(shape) + sum(roi))
    c, d = _adversarial_images(rng, *shape)
    for depth in (d, None):
        s = oracle.rle_compress(c, depth, roi)
        assert s.size <= oracle.rle_max_size(roi[2], roi[3], 8 if depth is not None else 4)
        p = parse_rle1(s.tobytes())
        assert p.roi == (roi if roi[2] * roi[3] else (0, 0, 0, 0))
        assert p.planes == _planes_of(c, depth, roi)
        r, c2, d2 = oracle.rle_decompress(s)
        x, y, w, h = roi
        # an empty ROI is stored in its canonical form (0, 0, 0, 0)
        assert r == (roi if w * h else (0, 0, 0, 0))
        assert c2.size == w * h and (c2.reshape(-1) == c[y:y + h, x:x + w].reshape(-1)).all()
        if depth is not None:
            assert d2.size == w * h and (d2.reshape(-1) == d[y:y + h, x:x + w].reshape(-1)).all()
        else:
            assert d2 is None


def test_generated_ramp_contributor_round_trip():
    img = synth.ramp_image(2, 3, 3, 320, 180, pitch_pad=64)
    c, d = synth.as_u32(img.color), synth.as_u32(img.depth)
    roi = oracle.roi_detect_depth(d, 320, 180)
    s = oracle.rle_compress(c, d, roi)
    p = parse_rle1(s.tobytes())
    assert p.planes == _planes_of(c, d, roi)
    # the smooth colour gradients and clear-free interior compress; the noisy
    # low depth byte is stored raw
    assert s.size < 8 * roi[2] * roi[3]
    assert all(t is None for t in p.tokens[4::8])


def test_corrupt_streams_are_rejected():
    depth = np.array([[5, 5, F], [5, 3, F], [F, F, F], [F, F, 7]], np.uint32)
    color = np.where(depth != F, 0xFF332211, 0).astype(np.uint32)
    good = oracle.rle_compress(color, depth, (0, 0, 3, 4))
    oracle.rle_decompress(good)

    def bad(mut):
        s = good.copy()
        mut(s)
        with pytest.raises(oracle.CorruptStream):
            oracle.rle_decompress(s)

    bad(lambda s: s.__setitem__(0, 0x53))                     # magic
    bad(lambda s: s.__setitem__(20, 5))                       # nplanes
    bad(lambda s: s.__setitem__(25, 0x20))                    # block size
    bad(lambda s: s.__setitem__(28, 2))                       # nblocks
    bad(lambda s: s.__setitem__(32, 16))                      # block offset
    bad(lambda s: s.__setitem__(36, 11))                      # odd token size
    bad(lambda s: s.__setitem__(36, 13))                      # size > block length
    bad(lambda s: s.__setitem__(80, 0x05))                    # runs overflow block
    bad(lambda s: s.__setitem__(80, 0x00))                    # runs short of block
    with pytest.raises(oracle.CorruptStream):
        oracle.rle_decompress(good[:100])                     # truncated
    with pytest.raises(oracle.CorruptStream):
        oracle.rle_decompress(good[:20])


def test_run_across_segment_is_rejected():
    """Runs end at multiples of 256 pixels at the latest (the RLE1 format):
    the 300-pixel constant row is 256 + 44 per plane; moving the split to
    200 + 100 keeps the sum but makes the second run cross pixel 256."""
    color = np.full((1, 300), 0x7E7E7E7E, np.uint32)
    good = oracle.rle_compress(color, color.copy(), (0, 0, 300, 1))
    assert good[80] == 0xFF and good[82] == 43        # plane 0: (255, v), (43, v)
    oracle.rle_decompress(good)
    s = good.copy()
    s[80], s[82] = 199, 99
    with pytest.raises(oracle.CorruptStream):
        oracle.rle_decompress(s)
    s = good.copy()
    s[80], s[82] = 254, 44                            # 255 + 45: ends at 300, crosses 256
    with pytest.raises(oracle.CorruptStream):
        oracle.rle_decompress(s)


def test_max_size_formula():
    for w, h, npl in [(0, 0, 8), (1, 1, 8), (4096, 1, 4), (4097, 1, 8), (1920, 1080, 8)]:
        nb = -(-w * h // 4096)
        p0 = (32 + 4 * nb * (1 + npl) + 15) // 16 * 16
        body = sum(((min(4096, w * h - 4096 * b) * npl) + 15) // 16 * 16 for b in range(nb))
        assert oracle.rle_max_size(w, h, npl) == p0 + body


# ------------------------------------------------------------ swizzling
def test_swizzle_hand_values():
    """Byte j of the swizzled word holds bits 2j+1, 2j of R, G, B, A (from its
    low end). Values derived by hand from that description."""
    cases = {
        0x000000FF: 0x03030303,   # all of R: the low two bits of every byte
        0x0000FF00: 0x0C0C0C0C,   # G
        0x00FF0000: 0x30303030,   # B
        0xFF000000: 0xC0C0C0C0,   # A
        0x80808080: 0xAA000000,   # the top bit of every component: top byte
        0x01010101: 0x00000055,   # the bottom bit of every component: low byte
        0x000000C0: 0x03000000,   # R bits 7, 6 -> bits 25, 24
        0x00000003: 0x00000003,
        0x00000000: 0x00000000,
        0xFFFFFFFF: 0xFFFFFFFF,
    }
    for v, exp in cases.items():
        assert oracle.swizzle(v) == exp, hex(v)
        assert oracle.unswizzle(exp) == v


def test_swizzle_is_a_bijection_and_an_involution():
    rng = np.random.default_rng(1)
    for v in rng.integers(0, 2 ** 32, 20000, dtype=np.uint64).tolist():
        s = oracle.swizzle(v)
        assert oracle.unswizzle(s) == v
        assert oracle.swizzle(s) == v          # a transpose of 2-bit fields
        assert bin(s).count("1") == bin(v).count("1")
    for k in range(32):
        assert bin(oracle.swizzle(1 << k)).count("1") == 1


def test_swizzled_stream_hand_built():
    """300 px of colour 0x80808080 (swizzled: 0xAA000000) and depth 0x7E7E7E7E:
    every plane is two runs (256 + 44); header word 5 is 8 | 0x100."""
    color = np.full((1, 300), 0x80808080, np.uint32)
    depth = np.full((1, 300), 0x7E7E7E7E, np.uint32)
    hdr = struct.pack("<IiiiiIII", 0x31454C52, 0, 0, 300, 1, 0x108, 4096, 1)
    tables = hdr + struct.pack("<I", 0) + struct.pack("<8I", *([4] * 8))
    tables += b"\0" * (80 - len(tables))
    payload = (b"\xff\x00\x2b\x00" * 3 + b"\xff\xaa\x2b\xaa" + b"\xff\x7e\x2b\x7e" * 4)
    exp = tables + payload
    got = oracle.rle_compress(color, depth, (0, 0, 300, 1), swizzle=True).tobytes()
    assert got == exp
    r, c, d = oracle.rle_decompress(np.frombuffer(exp, np.uint8))
    assert (c == color).all() and (d == depth).all()


def test_swizzle_round_trip_and_gain_on_shaded_colour():
    """Swizzling is lossless, and on shaded colour (R, G and B changing
    together and slowly) the high-order bits of all components share planes
    of long runs, so the stream shrinks: the effect the thesis reports for its
    swizzling preconditioner. (It is data dependent: a gradient in one
    component alone compresses better unswizzled.)"""
    yy, xx = np.mgrid[0:360, 0:640]
    lum = ((xx + 2 * yy) // 5) % 256
    c = (lum | (lum << 8) | (lum << 16) | (255 << 24)).astype(np.uint32)
    roi = (0, 0, 640, 360)
    plain = oracle.rle_compress(c, None, roi)
    swz = oracle.rle_compress(c, None, roi, swizzle=True)
    _, c2, _ = oracle.rle_decompress(swz)
    assert (c2 == c).all()
    assert swz.size < 0.8 * plain.size
    rng = np.random.default_rng(3)
    noise = rng.integers(0, 2 ** 32, (37, 53), dtype=np.uint64).astype(np.uint32)
    s = oracle.rle_compress(noise, noise, (1, 2, 50, 30), swizzle=True)
    _, c3, d3 = oracle.rle_decompress(s)
    assert (c3 == noise[2:32, 1:51]).all() and (d3 == noise[2:32, 1:51]).all()


# ------------------------------------------------------- ROI with holes
def test_roi_grid_hand_worked():
    """A 6x5 depth image, 2x2 cells: data at (0,0), (5,1) and (2,4); the
    occupancy is worked out by hand; the hole in the middle stays 0."""
    d = np.full((5, 6), F, np.uint32)
    d[0, 0] = 1
    d[1, 5] = 7
    d[4, 2] = 3
    g = oracle.roi_grid(d, (2, 2))
    assert g.tolist() == [[1, 0, 1], [0, 0, 0], [0, 1, 0]]
    assert oracle.roi_grid(np.full((5, 6), F, np.uint32), (4, 3)).tolist() == [[0, 0], [0, 0]]


@pytest.mark.parametrize("seed", range(4))
def test_roi_grid_brute_force(seed):
    rng = np.random.default_rng(900 + seed)
    H, W = int(rng.integers(1, 70)), int(rng.integers(1, 90))
    cw, ch = int(rng.integers(1, 17)), int(rng.integers(1, 17))
    m = rng.random((H, W)) < 0.01
    d = np.where(m, 5, F).astype(np.uint32)
    g = oracle.roi_grid(d, (cw, ch))
    for cy in range(g.shape[0]):
        for cx in range(g.shape[1]):
            assert g[cy, cx] == int(m[cy * ch:(cy + 1) * ch, cx * cw:(cx + 1) * cw].any())
    # the bounding box of the occupied cells contains the ROI
    x, y, w, h = oracle.roi_detect_depth(d)
    if w:
        ys, xs = np.nonzero(g)
        assert xs.min() * cw <= x and (xs.max() + 1) * cw >= x + w
        assert ys.min() * ch <= y and (ys.max() + 1) * ch >= y + h
    # float layers: -0.0 is empty, NaN is data
    f = np.zeros((H, W, 4), np.float32)
    f[m, 1] = 0.5
    f[~m, 3] = -0.0
    assert (oracle.roi_grid(f, (cw, ch), mode="float") == g).all()
