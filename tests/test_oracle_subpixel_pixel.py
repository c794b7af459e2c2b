"""Pins of the oracle's subpixel (accumulate-and-average) compositing and
pixel-compound assembly: hand-worked values, closed-form special cases,
invariants, and a round trip through numpy strided slicing (a different
mechanism for the same interleave)."""
import numpy as np
import pytest

import oracle


def _rgba(r, g, b, a):
    return np.uint32(r | (g << 8) | (b << 16) | (a << 24))


def test_average_hand_worked():
    """Means rounded half up, per channel (Section 4.2.3: samples of a pixel
    are accumulated and averaged)."""
    # two sources: (1+2)/2 = 1.5 -> 2; (0+255)/2 = 127.5 -> 128; (4+4)/2 = 4; (9+0)/2 = 4.5 -> 5
    a = np.array([[_rgba(1, 0, 4, 9)]], np.uint32)
    b = np.array([[_rgba(2, 255, 4, 0)]], np.uint32)
    out = oracle.composite_average([a, b], [(0, 0, 1, 1)] * 2, (0, 0, 1, 1))
    assert out[0, 0] == _rgba(2, 128, 4, 5)
    # three sources: (1+1+2)/3 = 1.33 -> 1; (255*3)/3 = 255; (0+0+2)/3 = 0.67 -> 1; (5+6+7)/3 = 6
    s = [np.array([[_rgba(1, 255, 0, 5)]], np.uint32), np.array([[_rgba(1, 255, 0, 6)]], np.uint32),
         np.array([[_rgba(2, 255, 2, 7)]], np.uint32)]
    out = oracle.composite_average(s, [(0, 0, 1, 1)] * 3, (0, 0, 1, 1))
    assert out[0, 0] == _rgba(1, 255, 1, 6)
    # a source that does not cover the pixel contributes a black sample
    out = oracle.composite_average([a, b], [(0, 0, 1, 1), (5, 5, 1, 1)], (0, 0, 1, 1))
    assert out[0, 0] == _rgba(1, 0, 2, 5)   # (1+0)/2 -> 1, (0+0)/2, (4+0)/2, (9+0)/2 -> 5


def test_average_properties():
    rng = np.random.default_rng(4)
    H, W = 9, 13
    imgs = [rng.integers(0, 2 ** 32, (H, W), dtype=np.uint64).astype(np.uint32) for _ in range(5)]
    rois = [(0, 0, W, H)] * 5
    vp = (0, 0, W, H)
    # n identical sources: the identity
    same = oracle.composite_average([imgs[0]] * 7, [rois[0]] * 7, vp)
    assert (same == imgs[0]).all()
    # order does not matter (integer sums)
    out = oracle.composite_average(imgs, rois, vp)
    p = rng.permutation(5)
    assert (oracle.composite_average([imgs[i] for i in p], rois, vp) == out).all()
    # each channel lies between the smallest and the largest sample
    for k in range(4):
        ch = np.stack([(im >> (8 * k)) & 0xFF for im in imgs])
        o = (out >> (8 * k)) & 0xFF
        assert (o >= ch.min(0)).all() and (o <= ch.max(0)).all()
    # two sources: the mean of x and y is within half a step of (x+y)/2
    two = oracle.composite_average(imgs[:2], rois[:2], vp)
    for k in range(4):
        x = ((imgs[0] >> (8 * k)) & 0xFF).astype(float)
        y = ((imgs[1] >> (8 * k)) & 0xFF).astype(float)
        o = ((two >> (8 * k)) & 0xFF).astype(float)
        assert (np.abs(o - (x + y) / 2) <= 0.5).all()
    assert (oracle.composite_average([], [], vp) == 0).all()


def _split(img, kx, ky):
    """The kx x ky interleave of an image by strided slicing."""
    return {(ox, oy): np.ascontiguousarray(img[oy::ky, ox::kx])
            for oy in range(ky) for ox in range(kx)}


@pytest.mark.parametrize("kx,ky,W,H", [(2, 2, 4, 4), (3, 2, 10, 7), (1, 4, 5, 9), (4, 1, 9, 3),
                                       (3, 3, 1, 1)])
def test_assemble_round_trip(kx, ky, W, H):
    """Splitting a frame into its pixel-kernel classes and assembling them
    gives the frame back (Section 4.2.2)."""
    rng = np.random.default_rng(kx * 10 + ky)
    img = rng.integers(0, 2 ** 32, (H, W), dtype=np.uint64).astype(np.uint32)
    parts = _split(img, kx, ky)
    keys = list(parts)
    rng.shuffle(keys)
    out = oracle.assemble_pixels([parts[k] for k in keys], keys, (kx, ky), (0, 0, W, H))
    assert (out == img).all()


def test_assemble_hand_worked_and_missing_classes():
    """2x2 kernel over 4x4: the four sources' constant colours form the
    checkerboard of their offsets; a class without a source stays 0; a
    duplicate class goes to the lower index."""
    A, B, C, D = 0xA, 0xB, 0xC, 0xD
    srcs = [np.full((2, 2), v, np.uint32) for v in (A, B, C, D)]
    offs = [(0, 0), (1, 0), (0, 1), (1, 1)]
    out = oracle.assemble_pixels(srcs, offs, (2, 2), (0, 0, 4, 4))
    exp = np.array([[A, B, A, B], [C, D, C, D], [A, B, A, B], [C, D, C, D]], np.uint32)
    assert (out == exp).all()
    out = oracle.assemble_pixels(srcs[:3], offs[:3], (2, 2), (0, 0, 4, 4))
    exp2 = exp.copy()
    exp2[1::2, 1::2] = 0
    assert (out == exp2).all()
    dup = oracle.assemble_pixels([srcs[1], srcs[0]] + srcs[2:], [(0, 0)] * 2 + offs[2:], (2, 2),
                                 (0, 0, 4, 4))
    assert dup[0, 0] == B and dup[0, 1] == 0
