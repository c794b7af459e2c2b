"""Sort-last image compositing on MI355X: Python binding of ``libcmp.so``.

The binding only marshals arguments: torch supplies device memory and the
current HIP stream, and every step runs in the library's HIP kernels. If the
library is missing the import of :func:`lib` raises; there is no fallback.

Thesis: S. Eilemann, "Parallel Rendering and Large Data Visualization" (2019),
chapter 5 "Compositing". The C entry points (include/cmp.h) cite the passages.

Image conventions (matching cmp.h):
  depth images   color, depth: int32 tensors (h, pitch) holding uint32 bits
  float layers   rgba: float32 / float16 tensor (h, pitch, 4)
  roi            (x, y, w, h): placement in destination pixels
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass
from typing import Optional, Sequence

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcmp.so")

CMP_OK, CMP_EINVAL, CMP_ENOSPC, CMP_EHIP, CMP_EUNSUPPORTED, CMP_ECORRUPT, CMP_ETIMEOUT = (
    0, -1, -2, -3, -4, -5, -6)
RGBA8, RGBA32F, RGBA16F = 0, 1, 2
RLE_SWIZZLE = 1
SEQ, DIRECT_SEND, BINARY_SWAP = 0, 1, 2
_SCHED = {"seq": SEQ, "direct_send": DIRECT_SEND, "binary_swap": BINARY_SWAP}


class CmpError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str = ""):
        self.status = status
        super().__init__(f"{where}: status {status}" + (f" ({detail})" if detail else ""))


class Rect(ctypes.Structure):
    _fields_ = [("x", ctypes.c_int32), ("y", ctypes.c_int32),
                ("w", ctypes.c_int32), ("h", ctypes.c_int32)]


class Schedule(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("owners", ctypes.c_int32)]


class Tile(ctypes.Structure):
    _fields_ = [("w", ctypes.c_int32), ("h", ctypes.c_int32)]


class CImage(ctypes.Structure):
    _fields_ = [("color", ctypes.c_void_p), ("depth", ctypes.c_void_p),
                ("pitch", ctypes.c_int64), ("roi", Rect)]


class CJob(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("fmt", ctypes.c_int32), ("n", ctypes.c_int32),
                ("in_", ctypes.POINTER(CImage)), ("order_b2f", ctypes.POINTER(ctypes.c_int32)),
                ("viewport", Rect), ("out_color", ctypes.c_void_p),
                ("out_depth", ctypes.c_void_p), ("out_pitch", ctypes.c_int64)]


_lib = None


def lib() -> ctypes.CDLL:
    """Loads libcmp.so (built in place by ``python -m paper_1902_08755_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run python -m paper_1902_08755_amd.build")
    L = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u64, sz = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                            ctypes.c_size_t)
    IMG = ctypes.POINTER(CImage)
    sig = {
        "cmp_version": ([], ctypes.c_char_p),
        "cmp_status_string": ([i32], ctypes.c_char_p),
        "cmp_last_error": ([], ctypes.c_char_p),
        "cmp_schedule_regions": ([Schedule, Rect, ctypes.POINTER(Rect), i32], i32),
        "cmp_composite_depth": ([IMG, i32, P, Rect, P, P, i64, Schedule, Tile, P], i32),
        "cmp_composite_depth_crop": ([IMG, i32, P, Rect, P, P, i64, Schedule, Tile, P], i32),
        "cmp_composite_average": ([IMG, i32, Rect, P, i64, Schedule, Tile, P], i32),
        "cmp_assemble_pixels": ([IMG, i32, P, i32, i32, Rect, P, i64, P], i32),
        "cmp_composite_over": ([IMG, i32, i32, P, Rect, P, i64, Schedule, Tile, P], i32),
        "cmp_composite_over_backward": ([IMG, i32, i32, P, Rect, P, i64, P, P, P, sz, P], i32),
        "cmp_over_backward_workspace_size": ([i32], sz),
        "cmp_roi_workspace_size": ([IMG, i32], sz),
        "cmp_roi_detect": ([IMG, i32, i32, P, P, sz, P], i32),
        "cmp_roi_grid": ([IMG, i32, i32, i32, i32, P, P], i32),
        "cmp_roi_rects": ([IMG, i32, i32, i32, P, i32, P, P, P], i32),
        "cmp_rle_max_size": ([i32, i32, i32], sz),
        "cmp_rle_workspace_size": ([IMG, i32], sz),
        "cmp_rle_compress": ([IMG, i32, i32, ctypes.c_uint32, P, P, P, P, P, P, sz, P], i32),
        "cmp_rle_compress_noalloc": ([IMG, i32, i32, ctypes.c_uint32, P, P, P, P, P, P], i32),
        "cmp_rle_decompress": ([P, P, i32, IMG, P, P, P], i32),
        "cmp_rle_decompress_at_roi": ([P, P, i32, IMG, P, P, P], i32),
        "cmp_rle64_max_size": ([i32, i32, i32], sz),
        "cmp_rle64_compress": ([IMG, i32, i32, P, P, P, P, P, P, sz, P], i32),
        "cmp_rle64_decompress": ([P, P, i32, IMG, P, P, P], i32),
        "cmp_rle_set_groups_per_cu": ([i32, i32], i32),
        "cmp_rle_set_wait_limit": ([i32], i32),
        "cmp_streams_create": ([i32, ctypes.POINTER(P)], i32),
        "cmp_streams_destroy": ([i32, ctypes.POINTER(P)], i32),
        "cmp_batch_plan_create": ([ctypes.POINTER(CJob), i32, ctypes.c_char_p,
                                   ctypes.POINTER(P)], i32),
        "cmp_batch_workspace_size": ([P], sz),
        "cmp_batch_upload": ([P, P, sz, P], i32),
        "cmp_batch_run": ([P, P, P], i32),
        "cmp_batch_run_plain": ([P, P], i32),
        "cmp_batch_info": ([P, ctypes.POINTER(i64), ctypes.POINTER(i32)], i32),
        "cmp_batch_plan_destroy": ([P], None),
        "cmp_bandwidth_probe": ([i32, P, P, sz, P], i32),
        "cmp_autotune": ([ctypes.POINTER(CJob), i32, ctypes.c_char_p, i32, P], i32),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def _check(st: int, where: str) -> None:
    if st != CMP_OK:
        raise CmpError(st, where, lib().cmp_last_error().decode())


def _stream(stream=None) -> int:
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def _u32_pitch(t: torch.Tensor) -> int:
    if t.dim() != 2 or t.stride(1) != 1 or t.element_size() != 4:
        raise ValueError("expected a (h, pitch) tensor of 4-byte elements, unit column stride")
    return t.stride(0)


def _rgba_pitch(t: torch.Tensor) -> int:
    if t.dim() != 3 or t.shape[2] != 4 or t.stride(2) != 1 or t.stride(1) != 4 or t.stride(0) % 4:
        raise ValueError("expected a (h, pitch, 4) RGBA tensor")
    return t.stride(0) // 4


def _cuda(t: Optional[torch.Tensor], what: str):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{what} must be a device tensor")
    return t.data_ptr()


def _rect(r) -> Rect:
    return Rect(*[int(v) for v in r])


@dataclass
class Image:
    """A contributor: RGBA8 colour (+ depth) or a float RGBA layer, and its ROI."""
    color: torch.Tensor
    depth: Optional[torch.Tensor]
    roi: tuple


def _images(imgs: Sequence, kind: str):
    arr = (CImage * max(1, len(imgs)))()
    for i, im in enumerate(imgs):
        color, depth, roi = im.color if hasattr(im, "color") else im.rgba, getattr(im, "depth", None), im.roi
        if kind == "rgba":
            pitch = _rgba_pitch(color) if color.numel() else int(roi[2])
        else:
            pitch = _u32_pitch(color) if color.numel() else int(roi[2])
            if depth is not None and depth.numel() and _u32_pitch(depth) != pitch:
                raise ValueError(f"image {i}: colour and depth pitches differ")
        arr[i] = CImage(_cuda(color, "color") if color.numel() else None,
                        _cuda(depth, "depth") if depth is not None and depth.numel() else None,
                        pitch, _rect(roi))
    return arr


def _fmt_of(t: torch.Tensor) -> int:
    if t.dtype == torch.float32:
        return RGBA32F
    if t.dtype == torch.float16:
        return RGBA16F
    raise ValueError(f"unsupported layer dtype {t.dtype}")


def _schedule(schedule) -> Schedule:
    if isinstance(schedule, Schedule):
        return schedule
    kind, owners = schedule if isinstance(schedule, tuple) else (schedule, 1)
    return Schedule(_SCHED[kind] if isinstance(kind, str) else int(kind), int(owners))


# ------------------------------------------------------------ compositing
def composite_depth(images: Sequence, viewport, out_color=None, out_depth=None, roi_dev=None,
                    schedule=("seq", 1), tile=(0, 0), want_depth=True, stream=None, crop=False):
    """Depth-sorted sort-last compositing (cmp_composite_depth; with
    crop=True cmp_composite_depth_crop: roi_dev crops the placed images)."""
    x, y, w, h = viewport
    dev = torch.device("cuda", torch.cuda.current_device())
    if out_color is None:
        out_color = torch.empty((h, w), dtype=torch.int32, device=dev)
    if out_depth is None and want_depth:
        out_depth = torch.empty((h, w), dtype=torch.int32, device=dev)
    pitch = _u32_pitch(out_color)
    if out_depth is not None and _u32_pitch(out_depth) != pitch:
        raise ValueError("out_color and out_depth pitches differ")
    arr = _images(images, "u32")
    fn = lib().cmp_composite_depth_crop if crop else lib().cmp_composite_depth
    st = fn(arr, len(images), _cuda(roi_dev, "roi_dev"), _rect(viewport), out_color.data_ptr(),
            _cuda(out_depth, "out_depth"), pitch, _schedule(schedule), Tile(*tile),
            _stream(stream))
    _check(st, "cmp_composite_depth_crop" if crop else "cmp_composite_depth")
    return out_color, out_depth


def composite_over(layers: Sequence, order, viewport, out=None, schedule=("seq", 1), tile=(0, 0),
                   stream=None):
    """Ordered premultiplied-alpha compositing (cmp_composite_over); FP32 output."""
    x, y, w, h = viewport
    n = len(layers)
    fmt = _fmt_of(layers[0].rgba if hasattr(layers[0], "rgba") else layers[0].color) if n else RGBA32F
    if out is None:
        out = torch.empty((h, w, 4), dtype=torch.float32,
                          device=torch.device("cuda", torch.cuda.current_device()))
    order_arr = (ctypes.c_int32 * max(1, n))(*[int(v) for v in order])
    st = lib().cmp_composite_over(_images(layers, "rgba"), n, fmt, order_arr, _rect(viewport),
                                  out.data_ptr(), _rgba_pitch(out), _schedule(schedule),
                                  Tile(*tile), _stream(stream))
    _check(st, "cmp_composite_over")
    return out


def composite_over_backward(layers: Sequence, order, viewport, grad_out, grads=None, stream=None):
    """Adjoint of composite_over: d loss / d layer for every layer."""
    n = len(layers)
    rgba = [l.rgba if hasattr(l, "rgba") else l.color for l in layers]
    fmt = _fmt_of(rgba[0]) if n else RGBA32F
    if grads is None:
        grads = [torch.empty((int(l.roi[3]), int(l.roi[2]), 4), dtype=torch.float32,
                             device=r.device) for l, r in zip(layers, rgba)]
    ptrs = (ctypes.c_void_p * max(1, n))(*[g.data_ptr() for g in grads])
    pitches = (ctypes.c_int64 * max(1, n))(*[_rgba_pitch(g) for g in grads])
    order_arr = (ctypes.c_int32 * max(1, n))(*[int(v) for v in order])
    grad_out = grad_out.contiguous()
    need = lib().cmp_over_backward_workspace_size(n)
    ws = workspace("over_backward", need) if need else None
    st = lib().cmp_composite_over_backward(_images(layers, "rgba"), n, fmt, order_arr,
                                           _rect(viewport), grad_out.data_ptr(),
                                           _rgba_pitch(grad_out), ptrs, pitches,
                                           ws.data_ptr() if ws is not None else None,
                                           ws.numel() if ws is not None else 0, _stream(stream))
    _check(st, "cmp_composite_over_backward")
    return grads


class OverComposite(torch.autograd.Function):
    """Differentiable ordered over compositing: forward and backward both run
    in libcmp's kernels; the transmittance is recomputed, never stored.

    ``OverComposite.apply(order, viewport, rois, *layers)`` with layers as
    (h, pitch, 4) float tensors; returns the (H, W, 4) FP32 composite.
    """

    @staticmethod
    def forward(ctx, order, viewport, rois, *layers):
        imgs = [Image(l.detach(), None, r) for l, r in zip(layers, rois)]
        out = composite_over(imgs, order, viewport)
        ctx.order, ctx.viewport, ctx.rois = list(order), tuple(viewport), list(rois)
        ctx.save_for_backward(*layers)
        return out

    @staticmethod
    def backward(ctx, grad_out):
        layers = ctx.saved_tensors
        imgs = [Image(l.detach(), None, r) for l, r in zip(layers, ctx.rois)]
        grads = composite_over_backward(imgs, ctx.order, ctx.viewport, grad_out.float())
        out = []
        for l, g in zip(layers, grads):
            if l.shape[1] != g.shape[1]:   # layer stored with a wider pitch
                full = torch.zeros(l.shape, dtype=torch.float32, device=g.device)
                full[:, :g.shape[1]] = g
                g = full
            out.append(g.to(l.dtype))
        return (None, None, None, *out)


def composite_average(images: Sequence, viewport, out=None, schedule=("seq", 1), tile=(0, 0),
                      stream=None):
    """Subpixel compositing (cmp_composite_average): per-channel RGBA8 mean."""
    x, y, w, h = viewport
    if out is None:
        out = torch.empty((h, w), dtype=torch.int32,
                          device=torch.device("cuda", torch.cuda.current_device()))
    st = lib().cmp_composite_average(_images(images, "u32"), len(images), _rect(viewport),
                                     out.data_ptr(), _u32_pitch(out), _schedule(schedule),
                                     Tile(*tile), _stream(stream))
    _check(st, "cmp_composite_average")
    return out


def assemble_pixels(images: Sequence, offsets, kernel, viewport, out=None, stream=None):
    """Pixel-compound assembly (cmp_assemble_pixels); images[i].roi gives the
    source image size, offsets[i] = (ox, oy) its class in the kernel."""
    x, y, w, h = viewport
    if out is None:
        out = torch.empty((h, w), dtype=torch.int32,
                          device=torch.device("cuda", torch.cuda.current_device()))
    n = len(images)
    offs = (ctypes.c_int32 * max(2, 2 * n))(*[int(v) for o in offsets for v in o])
    st = lib().cmp_assemble_pixels(_images(images, "u32"), n, offs, int(kernel[0]),
                                   int(kernel[1]), _rect(viewport), out.data_ptr(),
                                   _u32_pitch(out), _stream(stream))
    _check(st, "cmp_assemble_pixels")
    return out


# -------------------------------------------------------------------- ROI
_workspaces = {}


def workspace(tag: str, nbytes: int, device=None) -> torch.Tensor:
    """A zero-filled device workspace cached per (tag, device); grown on demand.
    The library leaves every workspace ready for its next call."""
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    key = (tag, str(dev))
    ws = _workspaces.get(key)
    if ws is None or ws.numel() < nbytes:
        ws = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=dev)
        _workspaces[key] = ws
    return ws


def roi_detect(images: Sequence, fmt: int = RGBA8, roi_out=None, ws=None, stream=None):
    """Automatic ROI detection (cmp_roi_detect); returns an int32 (n, 4) tensor.
    Without `ws` the call uses a workspace shared by all calls on the device:
    calls that may overlap (on other streams) must each pass their own."""
    n = len(images)
    arr = _images(images, "rgba" if fmt != RGBA8 else "u32")
    if roi_out is None:
        roi_out = torch.empty((n, 4), dtype=torch.int32,
                              device=torch.device("cuda", torch.cuda.current_device()))
    need = lib().cmp_roi_workspace_size(arr, n)
    if ws is None:
        ws = workspace("roi", need)
    st = lib().cmp_roi_detect(arr, n, fmt, roi_out.data_ptr(), ws.data_ptr(), ws.numel(),
                              _stream(stream))
    _check(st, "cmp_roi_detect")
    return roi_out


def roi_grid(images: Sequence, cell, fmt: int = RGBA8, stream=None):
    """Cell occupancy of each image (cmp_roi_grid): a list of uint8 device
    tensors (ceil(h / ch), ceil(w / cw))."""
    cw, ch = cell
    dims = [((int(im.roi[3]) + ch - 1) // ch, (int(im.roi[2]) + cw - 1) // cw) for im in images]
    total = sum(a * b for a, b in dims)
    buf = torch.zeros(max(1, total), dtype=torch.uint8,
                      device=torch.device("cuda", torch.cuda.current_device()))
    st = lib().cmp_roi_grid(_images(images, "rgba" if fmt != RGBA8 else "u32"), len(images), fmt,
                            cw, ch, buf.data_ptr(), _stream(stream))
    _check(st, "cmp_roi_grid")
    out, o = [], 0
    for gh, gw in dims:
        out.append(buf[o:o + gh * gw].view(gh, gw))
        o += gh * gw
    return out


def roi_rects(images: Sequence, cell, grids, max_rects: int = 4, stream=None):
    """ROI with holes (cmp_roi_rects): rectangles covering each image's
    occupied cells, from the grids of :func:`roi_grid` (same images and
    cells). Returns (rects int32 (n, max_rects, 4), counts int32 (n,)) on
    the device; unused rows are empty ROIs."""
    n = len(images)
    dev = torch.device("cuda", torch.cuda.current_device())
    flat = torch.cat([g.reshape(-1) for g in grids]) if n else torch.zeros(1, dtype=torch.uint8, device=dev)
    rects = torch.zeros((n, max_rects, 4), dtype=torch.int32, device=dev)
    counts = torch.zeros(n, dtype=torch.int32, device=dev)
    st = lib().cmp_roi_rects(_images(images, "u32"), n, int(cell[0]), int(cell[1]),
                             flat.data_ptr(), int(max_rects), rects.data_ptr(), counts.data_ptr(),
                             _stream(stream))
    _check(st, "cmp_roi_rects")
    return rects, counts


# -------------------------------------------------------------------- RLE
def rle_max_size(w: int, h: int, nplanes: int) -> int:
    return int(lib().cmp_rle_max_size(w, h, nplanes))


class RleBatch:
    """Pre-marshalled arguments of one cmp_rle_compress call over n images."""

    def __init__(self, images: Sequence, roi_dev=None, outs=None, swizzle=False):
        self.flags = RLE_SWIZZLE if swizzle else 0
        self.images = list(images)
        n = self.n = len(images)
        self.arr = _images(images, "u32")
        dev = torch.device("cuda", torch.cuda.current_device())
        self.caps = [rle_max_size(int(im.roi[2]), int(im.roi[3]), 8 if im.depth is not None else 4)
                     for im in images]
        self.outs = outs or [torch.empty(c, dtype=torch.uint8, device=dev) for c in self.caps]
        self.out_ptrs = (ctypes.c_void_p * max(1, n))(*[o.data_ptr() for o in self.outs])
        self.cap_arr = (ctypes.c_uint64 * max(1, n))(*[o.numel() for o in self.outs])
        self.sizes = torch.zeros(n, dtype=torch.int64, device=dev)
        self.status = torch.zeros(n, dtype=torch.int32, device=dev)
        self.roi_dev = roi_dev
        need = lib().cmp_rle_workspace_size(self.arr, n)
        self.ws = torch.zeros(max(need, 256), dtype=torch.uint8, device=dev)

    def run(self, stream=None):
        self.status.zero_()
        st = lib().cmp_rle_compress(self.arr, self.n, RGBA8, self.flags, _cuda(self.roi_dev, "roi_dev"),
                                    self.out_ptrs, self.cap_arr, self.sizes.data_ptr(),
                                    self.status.data_ptr(), self.ws.data_ptr(), self.ws.numel(),
                                    _stream(stream))
        _check(st, "cmp_rle_compress")
        return self.outs, self.sizes, self.status


def rle_compress(images: Sequence, roi_dev=None, swizzle=False, stream=None):
    """Per-component RLE of n images (cmp_rle_compress). Returns (streams,
    sizes, status): full-capacity uint8 buffers, an int64 tensor of stream
    sizes and an int32 tensor of per-image statuses (0, or CMP_ETIMEOUT for
    a stream that must not be used)."""
    return RleBatch(images, roi_dev, swizzle=swizzle).run(stream)


def rle_set_wait_limit(polls: int) -> None:
    """Test hook (cmp_rle_set_wait_limit): polls before a compressing block
    gives up waiting for its predecessors; negative restores the default."""
    _check(lib().cmp_rle_set_wait_limit(int(polls)), "cmp_rle_set_wait_limit")


def rle_set_groups_per_cu(compress: int, decompress: int) -> None:
    """Cap the RLE kernels' workgroups per compute unit (cmp_rle_set_groups_per_cu);
    0 = as many as fit."""
    _check(lib().cmp_rle_set_groups_per_cu(compress, decompress), "cmp_rle_set_groups_per_cu")


class Streams:
    """``count`` streams of the library's own (cmp_streams_create), as
    torch.cuda.ExternalStream objects in ``.streams``; destroyed by close()
    after a device synchronisation. Create them before anything else makes a
    stream for the hardware queue placement described in include/cmp.h."""

    def __init__(self, count: int):
        arr = (ctypes.c_void_p * count)()
        _check(lib().cmp_streams_create(count, arr), "cmp_streams_create")
        self._arr = arr
        self.streams = [torch.cuda.ExternalStream(h) for h in arr]

    def close(self):
        if self._arr is not None:
            torch.cuda.synchronize()
            _check(lib().cmp_streams_destroy(len(self._arr), self._arr), "cmp_streams_destroy")
            self._arr, self.streams = None, []


def rle_decompress(streams: Sequence[torch.Tensor], outs: Sequence, stream=None, roi_out=None,
                   status=None, at_roi=False):
    """Decodes n RLE1 streams into ``outs`` (Image-like; roi w/h bound the
    size): at their top left, or with at_roi=True (cmp_rle_decompress_at_roi)
    at the ROI's position in each frame. Returns (roi_out (n, 4) int32,
    status (n,) int32) device tensors."""
    n = len(streams)
    dev = torch.device("cuda", torch.cuda.current_device())
    arr = _images(outs, "u32")
    ins = (ctypes.c_void_p * max(1, n))(*[s.data_ptr() for s in streams])
    nbytes = (ctypes.c_uint64 * max(1, n))(*[s.numel() for s in streams])
    if roi_out is None:
        roi_out = torch.empty((n, 4), dtype=torch.int32, device=dev)
    if status is None:
        status = torch.zeros(n, dtype=torch.int32, device=dev)
    fn = lib().cmp_rle_decompress_at_roi if at_roi else lib().cmp_rle_decompress
    st = fn(ins, nbytes, n, arr, roi_out.data_ptr(), status.data_ptr(), _stream(stream))
    _check(st, "cmp_rle_decompress")
    return roi_out, status


def rle64_compress(images: Sequence, roi_dev=None, stream=None):
    """Basic 64-bit RLE of n images (cmp_rle64_compress, two pixels per
    token). Returns (streams, sizes, status) like :func:`rle_compress`."""
    n = len(images)
    L = lib()
    dev = torch.device("cuda", torch.cuda.current_device())
    arr = _images(images, "u32")
    caps = [int(L.cmp_rle64_max_size(int(im.roi[2]), int(im.roi[3]),
                                     2 if im.depth is not None else 1)) for im in images]
    outs = [torch.empty(c, dtype=torch.uint8, device=dev) for c in caps]
    out_ptrs = (ctypes.c_void_p * max(1, n))(*[o.data_ptr() for o in outs])
    cap_arr = (ctypes.c_uint64 * max(1, n))(*caps)
    sizes = torch.zeros(n, dtype=torch.int64, device=dev)
    status = torch.zeros(n, dtype=torch.int32, device=dev)
    ws = workspace("rle64", int(L.cmp_rle_workspace_size(arr, n)))
    st = L.cmp_rle64_compress(arr, n, RGBA8, _cuda(roi_dev, "roi_dev"), out_ptrs, cap_arr,
                              sizes.data_ptr(), status.data_ptr(), ws.data_ptr(), ws.numel(),
                              _stream(stream))
    _check(st, "cmp_rle64_compress")
    return outs, sizes, status


def rle64_decompress(streams: Sequence[torch.Tensor], outs: Sequence, stream=None, roi_out=None,
                     status=None):
    """Decodes n RL64 streams into ``outs`` (cmp_rle64_decompress). Returns
    (roi_out (n, 4) int32, status (n,) int32) device tensors."""
    n = len(streams)
    dev = torch.device("cuda", torch.cuda.current_device())
    arr = _images(outs, "u32")
    ins = (ctypes.c_void_p * max(1, n))(*[s.data_ptr() for s in streams])
    nbytes = (ctypes.c_uint64 * max(1, n))(*[s.numel() for s in streams])
    if roi_out is None:
        roi_out = torch.empty((n, 4), dtype=torch.int32, device=dev)
    if status is None:
        status = torch.zeros(n, dtype=torch.int32, device=dev)
    st = lib().cmp_rle64_decompress(ins, nbytes, n, arr, roi_out.data_ptr(), status.data_ptr(),
                                    _stream(stream))
    _check(st, "cmp_rle64_decompress")
    return roi_out, status


def schedule_regions(schedule, viewport):
    """The owner regions of a schedule over a viewport (host-only query)."""
    out = (Rect * 64)()
    n = lib().cmp_schedule_regions(_schedule(schedule), _rect(viewport), out, 64)
    if n < 0:
        _check(n, "cmp_schedule_regions")
    return [(r.x, r.y, r.w, r.h) for r in out[:n]]


def version() -> str:
    return lib().cmp_version().decode()
