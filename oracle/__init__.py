"""Oracle for the sort-last compositing path: plain single-threaded CPU code.

TEST INFRASTRUCTURE ONLY. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package. The product path
(``paper_1902_08755_amd``) never imports it and shares no code with it.

The arithmetic lives in ``oracle.c`` (built with ``gcc -O2 -ffp-contract=off``
into ``liboracle.so``); this module only marshals numpy arrays. Every function
cites the thesis passage it follows (S. Eilemann, "Parallel Rendering and
Large Data Visualization", 2019, chapter 5 "Compositing").

Images are described by the same plain fields everywhere:
  color  uint32 array (H, pitch)        RGBA8, little-endian R,G,B,A bytes
  depth  uint32 array (H, pitch)        smaller is nearer, 0xFFFFFFFF = clear
  layer  float array (H, pitch, 4)      premultiplied RGBA (fp16/fp32/fp64)
  roi    (x, y, w, h)                   placement in destination pixels
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CLEAR_DEPTH = 0xFFFFFFFF


class Rect(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int32), ("y", ctypes.c_int32),
                ("w", ctypes.c_int32), ("h", ctypes.c_int32)]

    def tup(self):
        return (self.x, self.y, self.w, self.h)


def build() -> str:
    """Compile oracle.c with gcc (no contraction of float operations)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                           "-Wall", "-Wextra", "-Wno-unused-parameter",
                           "-shared", "-fPIC", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        i32, i64, u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
        L.orc_composite_depth.argtypes = [i32, P, P, P, P, Rect, P, P, i64]
        L.orc_composite_depth.restype = None
        L.orc_composite_over.argtypes = [i32, P, P, P, P, Rect, P, i64]
        L.orc_composite_over.restype = None
        L.orc_composite_over_tree.argtypes = [i32, P, P, P, P, i32, Rect, P, i64]
        L.orc_composite_over_tree.restype = None
        L.orc_composite_over_f32.argtypes = [i32, P, P, P, P, i32, Rect, P, i64]
        L.orc_composite_over_f32.restype = None
        L.orc_composite_over_backward.argtypes = [i32, P, P, P, P, Rect, P, i64, P, P]
        L.orc_composite_over_backward.restype = None
        for name in ("orc_roi_detect_depth", "orc_roi_detect_rgba8", "orc_roi_detect_rgbaf"):
            getattr(L, name).argtypes = [P, i32, i32, i64]
            getattr(L, name).restype = Rect
        L.orc_rle_max_size.argtypes = [i32, i32, i32]
        L.orc_rle_max_size.restype = u64
        L.orc_rle_compress.argtypes = [P, P, i64, Rect, i32, P, u64]
        L.orc_rle_compress.restype = u64
        L.orc_rle_header.argtypes = [P, u64, ctypes.POINTER(Rect), ctypes.POINTER(i32),
                                     ctypes.POINTER(i32), ctypes.POINTER(u64)]
        L.orc_swizzle.argtypes = [ctypes.c_uint32]
        L.orc_swizzle.restype = ctypes.c_uint32
        L.orc_unswizzle.argtypes = [ctypes.c_uint32]
        L.orc_unswizzle.restype = ctypes.c_uint32
        L.orc_rle_header.restype = ctypes.c_int
        L.orc_rle_decompress.argtypes = [P, u64, P, P, i64, ctypes.POINTER(Rect)]
        L.orc_rle_decompress.restype = ctypes.c_int
        L.orc_rle64_max_size.argtypes = [i32, i32, i32]
        L.orc_rle64_max_size.restype = u64
        L.orc_rle64_compress.argtypes = [P, P, i64, Rect, P, u64]
        L.orc_rle64_compress.restype = u64
        L.orc_rle64_decompress.argtypes = [P, u64, P, P, i64, ctypes.POINTER(Rect)]
        L.orc_rle64_decompress.restype = ctypes.c_int
        L.orc_composite_average_rgba8.argtypes = [i32, P, P, P, Rect, P, i64]
        L.orc_composite_average_rgba8.restype = None
        L.orc_assemble_pixels.argtypes = [i32, P, P, P, P, i32, i32, Rect, P, i64]
        L.orc_assemble_pixels.restype = None
        L.orc_roi_grid.argtypes = [i32, P, i32, i32, i64, i32, i32, P]
        L.orc_roi_grid.restype = None
        L.orc_roi_rects.argtypes = [P, i32, i32, i32, i32, i32, i32, i32, P]
        L.orc_roi_rects.restype = i32
        _lib = L
    return _lib


# ---------------------------------------------------------------- helpers
def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def _ptr_array(arrs):
    return (ctypes.c_void_p * max(1, len(arrs)))(*[_ptr(a) for a in arrs])


def _contig(a, dtype):
    a = np.asarray(a)
    if a.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {a.dtype}")
    # keep row pitch: only the innermost layout must be dense
    if not a.flags.c_contiguous:
        a = np.ascontiguousarray(a)
    return a


def _rects(rois):
    arr = (Rect * max(1, len(rois)))()
    for i, r in enumerate(rois):
        arr[i] = Rect(*[int(v) for v in r])
    return arr


# ------------------------------------------------------ depth compositing
def composite_depth(colors, depths, rois, viewport):
    """Depth-sorted sort-last compositing (Section 5.2.1).

    colors[i], depths[i]: uint32 arrays of shape (roi_i.h, pitch_i) whose first
    roi_i.w columns hold the image. Returns (out_color, out_depth), each
    uint32 of shape (viewport.h, viewport.w).
    """
    n = len(colors)
    colors = [_contig(c, np.uint32) for c in colors]
    depths = [_contig(d, np.uint32) for d in depths]
    pitch = np.array([c.shape[1] if c.ndim == 2 else 0 for c in colors], dtype=np.int64)
    for c, d, r in zip(colors, depths, rois):
        assert c.shape == d.shape and c.shape[0] >= r[3] and c.shape[1] >= r[2]
    vp = Rect(*viewport)
    oc = np.zeros((viewport[3], viewport[2]), np.uint32)
    od = np.zeros((viewport[3], viewport[2]), np.uint32)
    lib().orc_composite_depth(n, _ptr_array(colors), _ptr_array(depths),
                              _ptr(pitch) if n else None, _rects(rois), vp,
                              _ptr(oc), _ptr(od), viewport[2])
    return oc, od


# -------------------------------------------------------- over compositing
def _layers_f64(layers):
    out = []
    for L in layers:
        L = np.asarray(L)
        assert L.ndim == 3 and L.shape[2] == 4
        out.append(np.ascontiguousarray(L.astype(np.float64)))  # exact upcast
    return out


def composite_over(layers, rois, order_b2f, viewport, groups=None):
    """Ordered premultiplied-alpha compositing (Section 5.2.1), FP64.

    layers[i]: float array (roi_i.h, pitch_i, 4). order_b2f: layer indices back
    to front. groups=None is the sequential order; groups=P is the binary-swap
    merge tree over P contiguous groups (Section 5.2.2).
    Returns float64 (viewport.h, viewport.w, 4).
    """
    n = len(layers)
    L = _layers_f64(layers)
    pitch = np.array([a.shape[1] for a in L], dtype=np.int64)
    order = np.ascontiguousarray(np.asarray(order_b2f, dtype=np.int32))
    assert sorted(order.tolist()) == list(range(n))
    out = np.zeros((viewport[3], viewport[2], 4), np.float64)
    vp = Rect(*viewport)
    if groups is None:
        lib().orc_composite_over(n, _ptr_array(L), _ptr(pitch) if n else None, _rects(rois),
                                 _ptr(order) if n else None, vp, _ptr(out), viewport[2])
    else:
        lib().orc_composite_over_tree(n, _ptr_array(L), _ptr(pitch) if n else None, _rects(rois),
                                      _ptr(order) if n else None, int(groups), vp, _ptr(out),
                                      viewport[2])
    return out


def composite_over_f32(layers, rois, order_b2f, viewport, groups=1):
    """The same two orders evaluated in single precision (no contraction)."""
    n = len(layers)
    L = [np.ascontiguousarray(np.asarray(a, dtype=np.float32)) for a in layers]
    pitch = np.array([a.shape[1] for a in L], dtype=np.int64)
    order = np.ascontiguousarray(np.asarray(order_b2f, dtype=np.int32))
    out = np.zeros((viewport[3], viewport[2], 4), np.float32)
    lib().orc_composite_over_f32(n, _ptr_array(L), _ptr(pitch) if n else None, _rects(rois),
                                 _ptr(order) if n else None, int(groups), Rect(*viewport),
                                 _ptr(out), viewport[2])
    return out


def composite_over_backward(layers, rois, order_b2f, viewport, grad_out, want_scale=False):
    """Adjoint of ordered over compositing, FP64.

    grad_out: (viewport.h, viewport.w, 4) = d loss / d out. Returns the list of
    per-layer gradients (same shape as layers[i]) and, with want_scale, the
    componentwise condition scales used as test tolerances.
    """
    n = len(layers)
    L = _layers_f64(layers)
    pitch = np.array([a.shape[1] for a in L], dtype=np.int64)
    order = np.ascontiguousarray(np.asarray(order_b2f, dtype=np.int32))
    G = np.ascontiguousarray(np.asarray(grad_out, dtype=np.float64))
    assert G.shape == (viewport[3], viewport[2], 4)
    grads = [np.zeros_like(a) for a in L]
    scales = [np.zeros_like(a) for a in L] if want_scale else None
    lib().orc_composite_over_backward(n, _ptr_array(L), _ptr(pitch) if n else None, _rects(rois),
                                      _ptr(order) if n else None, Rect(*viewport), _ptr(G),
                                      viewport[2], _ptr_array(grads),
                                      _ptr_array(scales) if want_scale else None)
    return (grads, scales) if want_scale else grads


# ------------------------------------------------------------------- ROI
def roi_detect_depth(depth, w=None, h=None):
    """Bounding box of pixels with depth != 0xFFFFFFFF (Section 5.3)."""
    d = _contig(depth, np.uint32)
    h = d.shape[0] if h is None else h
    w = d.shape[1] if w is None else w
    return lib().orc_roi_detect_depth(_ptr(d), w, h, d.shape[1]).tup()


def roi_detect_rgba8(color, w=None, h=None):
    """Bounding box of pixels whose RGBA8 word is not 0 (Section 5.3)."""
    c = _contig(color, np.uint32)
    h = c.shape[0] if h is None else h
    w = c.shape[1] if w is None else w
    return lib().orc_roi_detect_rgba8(_ptr(c), w, h, c.shape[1]).tup()


def roi_detect_rgbaf(layer, w=None, h=None):
    """Bounding box of pixels with any channel != 0.0 (Section 5.3)."""
    a = np.ascontiguousarray(np.asarray(layer).astype(np.float64))
    h = a.shape[0] if h is None else h
    w = a.shape[1] if w is None else w
    return lib().orc_roi_detect_rgbaf(_ptr(a), w, h, a.shape[1]).tup()


# ------------------------------------------------------------------- RLE
def rle_max_size(w, h, nplanes):
    return int(lib().orc_rle_max_size(w, h, nplanes))


def swizzle(word: int) -> int:
    """The bit-swizzling preconditioner of Section 5.5.1 on one RGBA8 word."""
    return int(lib().orc_swizzle(word))


def unswizzle(word: int) -> int:
    return int(lib().orc_unswizzle(word))


def rle_compress(color, depth, roi, swizzle=False):
    """Per-component RLE of the ROI of an RGBA8 (+ depth) image (Section 5.5.1).

    color/depth: uint32 (H, pitch) full images; roi: image-local (x, y, w, h).
    swizzle: bit-swizzle the colour words first (Section 5.5.1).
    Returns the RLE1 stream as a uint8 array.
    """
    c = _contig(color, np.uint32)
    d = None if depth is None else _contig(depth, np.uint32)
    if d is not None:
        assert d.shape == c.shape
    x, y, w, h = roi
    assert 0 <= x and 0 <= y and x + w <= c.shape[1] and y + h <= c.shape[0]
    nplanes = 4 if d is None else 8
    cap = rle_max_size(w, h, nplanes)
    out = np.zeros(cap, np.uint8)
    sz = lib().orc_rle_compress(_ptr(c), None if d is None else _ptr(d), c.shape[1],
                                Rect(*roi), int(bool(swizzle)), _ptr(out), cap)
    if sz == 0:
        raise ValueError("rle_compress failed")
    return out[:sz].copy()


def rle_header(stream):
    s = np.ascontiguousarray(np.asarray(stream, dtype=np.uint8))
    r, npl, swz, tot = Rect(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_uint64()
    rc = lib().orc_rle_header(_ptr(s), s.size, ctypes.byref(r), ctypes.byref(npl),
                              ctypes.byref(swz), ctypes.byref(tot))
    if rc != 0:
        return None
    return r.tup(), npl.value, tot.value


class CorruptStream(ValueError):
    pass


def rle_decompress(stream):
    """Decode an RLE1 stream. Returns (roi, color, depth or None)."""
    s = np.ascontiguousarray(np.asarray(stream, dtype=np.uint8))
    hdr = rle_header(s)
    if hdr is None:
        raise CorruptStream("bad header")
    (x, y, w, h), npl, _ = hdr
    c = np.zeros((max(h, 0), max(w, 0)), np.uint32)
    d = np.zeros((max(h, 0), max(w, 0)), np.uint32) if npl == 8 else None
    r = Rect()
    rc = lib().orc_rle_decompress(_ptr(s), s.size, _ptr(c), None if d is None else _ptr(d),
                                  max(w, 1), ctypes.byref(r))
    if rc != 0:
        raise CorruptStream("corrupt payload")
    return r.tup(), c, d


def rle64_max_size(w, h, nstreams):
    return int(lib().orc_rle64_max_size(w, h, nstreams))


def rle64_compress(color, depth, roi):
    """Basic 64-bit RLE of the ROI of an RGBA8 (+ depth) image (Section
    5.5.1: two pixels per 64-bit token). Returns the RL64 stream (uint8)."""
    c = _contig(color, np.uint32)
    d = None if depth is None else _contig(depth, np.uint32)
    if d is not None:
        assert d.shape == c.shape
    x, y, w, h = roi
    assert 0 <= x and 0 <= y and x + w <= c.shape[1] and y + h <= c.shape[0]
    ns = 1 if d is None else 2
    cap = rle64_max_size(w, h, ns)
    out = np.zeros(cap, np.uint8)
    sz = lib().orc_rle64_compress(_ptr(c), None if d is None else _ptr(d), c.shape[1],
                                  Rect(*roi), _ptr(out), cap)
    if sz == 0:
        raise ValueError("rle64_compress failed")
    return out[:sz].copy()


def rle64_decompress(stream):
    """Decode an RL64 stream. Returns (roi, color, depth or None)."""
    s = np.ascontiguousarray(np.asarray(stream, dtype=np.uint8))
    if s.size < 32:
        raise CorruptStream("short header")
    hw = s[:32].view(np.uint32)
    w, h, ns = int(hw[3]), int(hw[4]), int(hw[5])
    if w < 0 or h < 0 or w > (1 << 20) or h > (1 << 20):
        raise CorruptStream("bad size")
    c = np.zeros((h, w), np.uint32)
    d = np.zeros((h, w), np.uint32) if ns == 2 else None
    r = Rect()
    rc = lib().orc_rle64_decompress(_ptr(s), s.size, _ptr(c), None if d is None else _ptr(d),
                                    max(w, 1), ctypes.byref(r))
    if rc != 0:
        raise CorruptStream("corrupt stream")
    return r.tup(), c, d


# ------------------------------------------------------ subpixel / pixel
def composite_average(colors, rois, viewport):
    """Subpixel compositing (Section 4.2.3): per-channel mean of the n
    sources' RGBA8 samples, rounded half up; 0 outside a source's ROI."""
    n = len(colors)
    colors = [_contig(c, np.uint32) for c in colors]
    pitch = np.array([c.shape[1] for c in colors], dtype=np.int64)
    out = np.zeros((viewport[3], viewport[2]), np.uint32)
    lib().orc_composite_average_rgba8(n, _ptr_array(colors), _ptr(pitch) if n else None,
                                      _rects(rois), Rect(*viewport), _ptr(out), viewport[2])
    return out


def assemble_pixels(colors, offsets, kernel, viewport):
    """Pixel-compound assembly (Section 4.2.2). colors[i] holds the pixels of
    offset class offsets[i] = (ox, oy) of the kernel (kx, ky)."""
    n = len(colors)
    colors = [_contig(c, np.uint32) for c in colors]
    pitch = np.array([c.shape[1] for c in colors], dtype=np.int64)
    ox = np.array([o[0] for o in offsets], dtype=np.int32)
    oy = np.array([o[1] for o in offsets], dtype=np.int32)
    out = np.zeros((viewport[3], viewport[2]), np.uint32)
    lib().orc_assemble_pixels(n, _ptr_array(colors), _ptr(pitch) if n else None,
                              _ptr(ox) if n else None, _ptr(oy) if n else None,
                              int(kernel[0]), int(kernel[1]), Rect(*viewport), _ptr(out),
                              viewport[2])
    return out


def roi_grid(image, cell, mode="depth", w=None, h=None):
    """Occupancy of cw x ch cells (Section 5.3, holes in the ROI): uint8
    array (ceil(h / ch), ceil(w / cw)). mode: "depth", "rgba8" or "float"."""
    cw, ch = cell
    if mode == "float":
        a = np.ascontiguousarray(np.asarray(image).astype(np.float64))
        m = 2
    else:
        a = _contig(image, np.uint32)
        m = 0 if mode == "depth" else 1
    h = a.shape[0] if h is None else h
    w = a.shape[1] if w is None else w
    g = np.zeros(((h + ch - 1) // ch, (w + cw - 1) // cw), np.uint8)
    lib().orc_roi_grid(m, _ptr(a), w, h, a.shape[1], cw, ch, _ptr(g))
    return g


def roi_rects(grid, cell, w, h, max_rects=64):
    """Rectangles covering the occupied cells of a roi_grid (Section 5.3, ROI
    with holes): per row of cells its maximal runs, a run equal to a run of
    the row above extends that rectangle, others start one; more than
    max_rects gives the bounding box. List of (x, y, w, h) in pixels."""
    g = np.ascontiguousarray(np.asarray(grid, dtype=np.uint8))
    gh, gw = g.shape
    out = np.zeros(4 * max(1, gw * gh), np.int32)
    n = lib().orc_roi_rects(_ptr(g), gw, gh, cell[0], cell[1], w, h, max_rects, _ptr(out))
    return [tuple(int(v) for v in out[4 * k:4 * k + 4]) for k in range(n)]
