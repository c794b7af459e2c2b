"""Pins of the oracle's basic 64-bit RLE (thesis Section 5.5.1: the basic
compressor compares two RGBA8 pixels at a time as one 64-bit token).

Independent facts used: streams derived by hand from the format definition
(tests/golden/rl64_examples.txt), a pure-Python parser written from the
format definition that checks every structural rule (maximal runs, the
128-symbol segment limit, the raw rule, zero padding, table offsets),
round-trip identity on adversarial images, and corrupt streams."""
import numpy as np
import pytest

import oracle
from conftest import read_golden

F = 0xFFFFFFFF


def _golden(name):
    sec = read_golden("rl64_examples.txt")[name]
    return np.array([int(t, 16) for row in sec for t in row], np.uint8)


def test_hand_worked_streams():
    run = np.full((1, 300), 0x7E7E7E7E, np.uint32)
    assert (oracle.rle64_compress(run, None, (0, 0, 300, 1)) == _golden("run300")).all()
    odd = np.array([[7] * 8 + [9]], np.uint32)
    assert (oracle.rle64_compress(odd, None, (0, 0, 9, 1)) == _golden("odd9")).all()
    depth = np.array([[5, 5, F, F], [5, 3, F, F], [F, F, F, F], [F, F, 7, F]], np.uint32)
    color = np.where(depth != F, 0xFF332211, 0).astype(np.uint32)
    assert (oracle.rle64_compress(color, depth, (0, 0, 3, 4)) == _golden("worked_A")).all()
    for name, c, d, roi in (("run300", run, None, (0, 0, 300, 1)), ("odd9", odd, None, (0, 0, 9, 1)),
                            ("worked_A", color, depth, (0, 0, 3, 4))):
        r, c2, d2 = oracle.rle64_decompress(_golden(name))
        x, y, w, h = roi
        assert r == roi and (c2 == c[y:y + h, x:x + w]).all()
        assert (d2 is None) == (d is None)
        if d is not None:
            assert (d2 == d[y:y + h, x:x + w]).all()


def _py_parse(stream):
    """Decodes an RL64 stream with plain Python, checking every rule of the
    format; returns (roi, colour, depth) as lists of rows."""
    b = bytes(stream)
    u32 = lambda o: int.from_bytes(b[o:o + 4], "little")
    assert u32(0) == 0x34364C52 and u32(24) == 4096
    x, y, w, h, ns = (u32(4 * k) for k in (1, 2, 3, 4, 5))
    assert ns in (1, 2)
    npx = w * h
    nb = (npx + 4095) // 4096
    assert u32(28) == nb
    p0 = (32 + 4 * nb * (1 + ns) + 15) // 16 * 16
    assert all(v == 0 for v in b[32 + 4 * nb * (1 + ns):p0])
    out = [[0] * npx for _ in range(ns)]
    pos = 0
    for blk in range(nb):
        assert u32(32 + 4 * blk) == pos
        q0 = 4096 * blk
        ln = min(4096, npx - q0)
        m = (ln + 1) // 2
        used = 0
        for k in range(ns):
            sz = u32(32 + 4 * nb + 4 * (blk * ns + k))
            src = b[p0 + pos + used:p0 + pos + used + sz]
            sym = [int.from_bytes(src[8 * j:8 * j + 8], "little") for j in range(m)] if sz == 8 * m else None
            if sym is None:
                lens, j = [], 0
                while j < m:
                    lens.append(src[len(lens)] + 1)
                    j += lens[-1]
                R = len(lens)
                vo = (R + 7) // 8 * 8
                assert sz == vo + 8 * R < 8 * m
                assert all(v == 0 for v in src[R:vo])
                vals = [int.from_bytes(src[vo + 8 * t:vo + 8 * t + 8], "little") for t in range(R)]
                sym, j = [], 0
                for t, (L, v) in enumerate(zip(lens, vals)):
                    assert (j % 128) + L <= 128                      # inside a segment
                    if t > 0 and j % 128 != 0:
                        assert v != vals[t - 1]                      # maximal runs
                    sym += [v] * L
                    j += L
            else:
                # raw only when tokens would not be smaller
                R = 1 + sum(1 for j in range(1, m) if j % 128 == 0 or sym[j] != sym[j - 1])
                assert (R + 7) // 8 * 8 + 8 * R >= 8 * m
            if ln % 2:
                assert sym[-1] >> 32 == 0
            for p in range(ln):
                out[k][q0 + p] = (sym[p // 2] >> (32 * (p % 2))) & 0xFFFFFFFF
            used += sz
        pad = (used + 15) // 16 * 16
        assert all(v == 0 for v in b[p0 + pos + used:p0 + pos + pad])
        pos += pad
    assert len(b) == p0 + pos
    rows = lambda v: [v[r * w:(r + 1) * w] for r in range(h)]
    return (x, y, w, h), rows(out[0]), rows(out[1]) if ns == 2 else None


def _adversarial(rng, H, W):
    """Runs of equal pixels of many lengths (odd and even, around the
    256-pixel segment), equal pairs and noise."""
    c = np.zeros((H, W), np.uint32)
    d = np.full((H, W), F, np.uint32)
    flat, dflat = c.reshape(-1), d.reshape(-1)
    pos = 0
    for run in [1, 2, 3, 255, 256, 257, 254, 511, 513, 4095, 4096, 4097, 7]:
        if pos >= flat.size:
            break
        flat[pos:pos + run] = rng.integers(0, 2 ** 32, dtype=np.uint64)
        dflat[pos:pos + run] = rng.integers(0, 4, dtype=np.uint64)
        pos = min(flat.size, pos + run)
    k2 = min(flat.size, pos + 2000)
    flat[pos:k2] = rng.integers(0, 2 ** 32, k2 - pos, dtype=np.uint64).astype(np.uint32)
    return c, d


@pytest.mark.parametrize("shape,roi", [((1, 1), (0, 0, 1, 1)), ((130, 150), (7, 3, 129, 101)),
                                       ((65, 64), (0, 0, 64, 65)), ((20, 30), (5, 5, 0, 7)),
                                       ((40, 4100), (1, 2, 4097, 3)), ((9, 9), (0, 0, 9, 9)),
                                       ((300, 301), (0, 0, 301, 300))])
def test_round_trip_and_structure(shape, roi):
    rng = np.random.default_rng(shape[0] * 7 + shape[1])
    c, d = _adversarial(rng, *shape)
    for depth in (None, d):
        s = oracle.rle64_compress(c, depth, roi)
        x, y, w, h = roi if roi[2] * roi[3] else (0, 0, 0, 0)
        got_roi, pc, pd = _py_parse(s)
        assert got_roi == (x, y, w, h)
        assert np.array_equal(np.array(pc, np.uint32).reshape(h, w), c[y:y + h, x:x + w])
        r, c2, d2 = oracle.rle64_decompress(s)
        assert r == (x, y, w, h) and (c2 == c[y:y + h, x:x + w]).all()
        if depth is not None:
            assert np.array_equal(np.array(pd, np.uint32).reshape(h, w), d[y:y + h, x:x + w])
            assert (d2 == d[y:y + h, x:x + w]).all()
        assert s.size <= oracle.rle64_max_size(w, h, 1 if depth is None else 2)


def test_compression_needs_equal_pairs():
    """Runs compress only as runs of equal pixel pairs: a constant image and
    an image of repeating (1, 2) pairs shrink to one token per 128-symbol
    segment, while pixels that repeat with a period of 3 give no two equal
    neighbouring pairs and stay raw (the thesis: the basic codec can only
    compress adjacent pixels of the same colour)."""
    const = np.full((64, 256), 0x11223344, np.uint32)
    s = oracle.rle64_compress(const, None, (0, 0, 256, 64))
    # 16384 px = 4 blocks of 2048 symbols = 16 segments each: 16 runs per
    # block, 16 length bytes + 16 values; header + table = align16(32 + 32)
    assert s.size == 64 + 4 * (16 + 16 * 8)
    alt = np.tile(np.array([1, 2], np.uint32), (64, 128))
    s2 = oracle.rle64_compress(alt, None, (0, 0, 256, 64))
    assert s2.size == 64 + 4 * (16 + 16 * 8)     # pairs (1, 2) are all equal
    shifted = np.tile(np.array([1, 1, 2], np.uint32), (64, 86))[:, :256].copy()
    s3 = oracle.rle64_compress(shifted, None, (0, 0, 256, 64))
    assert s3.size == oracle.rle64_max_size(256, 64, 1)   # no equal neighbouring pairs: raw


def test_corrupt_streams_rejected():
    good = _golden("run300")
    oracle.rle64_decompress(good)
    cases = {"magic": (0, 0x51), "streams": (20, 3), "block": (25, 0x20), "nblocks": (28, 2),
             "boff": (32, 16), "size_odd": (36, 0x19), "size_big": (37, 0x10),
             "run_crosses_segment": (48, 0x80), "run_too_long": (49, 0x20), "pad": (50, 1),
             "block_pad": (79, 1)}
    for name, (pos, val) in cases.items():
        s = good.copy()
        s[pos] = val
        with pytest.raises(oracle.CorruptStream):
            oracle.rle64_decompress(s)
    with pytest.raises(oracle.CorruptStream):
        oracle.rle64_decompress(good[:60])
    # the partner of an odd last pixel must be 0
    s = _golden("odd9").copy()
    s[68] = 1
    with pytest.raises(oracle.CorruptStream):
        oracle.rle64_decompress(s)
