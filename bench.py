"""Benchmark of the sort-last compositing path on one MI355X.

One step = the whole hot path over one frame of the 16-contributor workload
(16 x 1920x1080 RGBA8 + uint32 depth framebuffers, each holding a ~30%
region of interest with a smooth depth ramp plus noise):
    ROI detection of the 16 framebuffers
 -> per-component RLE compression of the 16 ROIs
 -> decompression of the 16 streams into 16 frames, each ROI block at its
    position in the frame
 -> depth compositing of the 16 frames cropped to the decoded ROIs into
    1920x1080 with the binary-swap schedule over 16 owners (tiles of
    480x270).
Inputs are resident in HBM before timing starts; the step rotates over
several copies of every buffer so that the 256 MB Infinity Cache cannot
serve a step from the previous one.

Prints one JSON line: Mpixel/s of composited input (the sum of the ROI areas
supplied per frame) with frames composited asynchronously, four in flight
on four streams of the library's own, compression capped at one workgroup
and decompression at three per compute unit (one frame at a time, as a HIP graph and eagerly, at full occupancy, is
reported beside it), the roofline of the dominant stage (algorithmic bytes
over its event-timed average duration, one frame at a time), and the oracle
timed on the host.
"""
from __future__ import annotations

import argparse
import math
import ctypes
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

import paper_1902_08755_amd as cmp  # noqa: E402
import synth  # noqa: E402

PEAK_HBM_GBPS = 8000.0
METRIC = "composited input Mpixel/s and achieved HBM GB/s (% peak), plain vs batched/backward"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


class Frame:
    """One copy of every buffer of the pipeline."""

    def __init__(self, wl, dev):
        self.images = wl.images
        self.roi = torch.zeros((16, 4), dtype=torch.int32, device=dev)
        self.rle = cmp.RleBatch(self.images, roi_dev=self.roi)
        W, H = wl.viewport[2], wl.viewport[3]
        # the decoded frames: each ROI block lands at its position, and only
        # the ROIs are read from them
        self.placed = [cmp.Image(torch.zeros((H, W), dtype=torch.int32, device=dev),
                                 torch.zeros((H, W), dtype=torch.int32, device=dev), (0, 0, W, H))
                       for _ in self.images]
        self.roi_dec = torch.zeros((16, 4), dtype=torch.int32, device=dev)
        self.status = torch.zeros(16, dtype=torch.int32, device=dev)
        self.out_c = torch.zeros((H, W), dtype=torch.int32, device=dev)
        self.out_d = torch.zeros((H, W), dtype=torch.int32, device=dev)
        self.viewport = wl.viewport
        # pre-marshalled C arguments: the timed loop only calls the library
        L = cmp.lib()
        self.img_arr = cmp._images(self.images, "u32")
        self.roi_ws = torch.zeros(L.cmp_roi_workspace_size(self.img_arr, 16), dtype=torch.uint8,
                                  device=dev)
        self.dec_in = (ctypes.c_void_p * 16)(*[o.data_ptr() for o in self.rle.outs])
        self.dec_bytes = (ctypes.c_uint64 * 16)(*[o.numel() for o in self.rle.outs])
        self.dec_out = cmp._images(self.placed, "u32")
        self.comp_in = cmp._images(self.placed, "u32")

    def stage(self, k, s):
        L = cmp.lib()
        if k == 0:
            st = L.cmp_roi_detect(self.img_arr, 16, cmp.RGBA8, self.roi.data_ptr(),
                                  self.roi_ws.data_ptr(), self.roi_ws.numel(), s)
        elif k == 1:
            r = self.rle
            st = L.cmp_rle_compress(r.arr, 16, cmp.RGBA8, 0, self.roi.data_ptr(), r.out_ptrs,
                                    r.cap_arr, r.sizes.data_ptr(), r.status.data_ptr(),
                                    r.ws.data_ptr(), r.ws.numel(), s)
        elif k == 2:
            # each ROI block into its frame at the ROI's position: the
            # compositor's 64-pixel row reads then start on the same column
            # alignment as the viewport (blocks at the buffer origin made
            # every wave's 256-byte read span three 128-byte lines: 1.40x
            # the algorithmic bytes, against 1.09x)
            st = L.cmp_rle_decompress_at_roi(self.dec_in, self.dec_bytes, 16, self.dec_out,
                                             self.roi_dec.data_ptr(), self.status.data_ptr(), s)
        else:
            st = L.cmp_composite_depth_crop(self.comp_in, 16, self.roi_dec.data_ptr(),
                                            cmp._rect(self.viewport), self.out_c.data_ptr(),
                                            self.out_d.data_ptr(), self.out_c.stride(0),
                                            cmp.Schedule(cmp.BINARY_SWAP, 16), cmp.Tile(0, 0), s)
        if st != 0:
            raise cmp.CmpError(st, f"stage {k}", L.cmp_last_error().decode())


STAGES = ["roi_detect", "rle_compress", "rle_decompress", "composite_depth"]
# the kernels each stage launches (one library call per stage)
STAGE_KERNELS = {"roi_detect": "roi_kernel<0>",
                 "rle_compress": "rle_compress_kernel",
                 "rle_decompress": "rle_decompress_kernel",
                 "composite_depth": "depth_kernel"}


def algorithmic_bytes(frame, rois, stream_sizes):
    """Bytes each stage must move (reads + writes), from the frame's ROIs."""
    W, H = frame.viewport[2], frame.viewport[3]
    roi_px = sum(w * h for _, _, w, h in rois)
    cover = np.zeros((H, W), np.int32)
    for x, y, w, h in rois:
        cover[y:y + h, x:x + w] += 1
    covered = int((cover > 0).sum())
    comp = int(stream_sizes.sum())
    return {
        "roi_detect": 16 * W * H * 4 + 16 * 16,
        "rle_compress": 8 * roi_px + comp,
        "rle_decompress": comp + 8 * roi_px,
        # depth of every covering contributor, the winner's colour, and the
        # output colour + depth
        "composite_depth": 4 * int(cover.sum()) + 4 * covered + 8 * W * H,
    }, roi_px


class DevEvent:
    """A HIP timing event whose record releases to device scope only
    (hipEventReleaseToDevice): torch's events release to system scope, which
    writes back and invalidates the L2 at every record and would charge that
    to the stage that follows."""
    _hip = None

    def __init__(self):
        if DevEvent._hip is None:
            DevEvent._hip = ctypes.CDLL("libamdhip64.so")
        self.h = ctypes.c_void_p()
        st = DevEvent._hip.hipEventCreateWithFlags(ctypes.byref(self.h), ctypes.c_uint(0x40000000))
        assert st == 0, f"hipEventCreateWithFlags: {st}"

    def record(self, stream_handle):
        st = DevEvent._hip.hipEventRecord(self.h, ctypes.c_void_p(stream_handle))
        assert st == 0, f"hipEventRecord: {st}"

    def elapsed_ms(self, end):
        ms = ctypes.c_float()
        st = DevEvent._hip.hipEventElapsedTime(ctypes.byref(ms), self.h, end.h)
        assert st == 0, f"hipEventElapsedTime: {st}"
        return ms.value

    def __del__(self):
        if self.h and DevEvent._hip is not None:
            DevEvent._hip.hipEventDestroy(self.h)


def time_stages(frames, steps, warmup, s_obj):
    """One frame at a time on one stream, each stage between two events."""
    s = s_obj.cuda_stream
    nf = len(frames)
    for i in range(warmup):
        f = frames[i % nf]
        for k in range(4):
            f.stage(k, s)
    torch.cuda.synchronize()
    ev = [[DevEvent() for _ in range(5)] for _ in range(steps)]
    t0, t1 = DevEvent(), DevEvent()
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(s)
    for i in range(steps):
        f = frames[i % nf]
        for k in range(4):
            ev[i][k].record(s)
            f.stage(k, s)
        ev[i][4].record(s)
    t1.record(s)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    total_ms = t0.elapsed_ms(t1)
    per = np.array([[ev[i][k].elapsed_ms(ev[i][k + 1]) for k in range(4)] for i in range(steps)])
    return total_ms, wall, per


def time_stage_alone(frames, k, steps, warmup, s_obj):
    """Stage k launched `steps` times back to back over the buffer copies
    (its inputs are valid from the set-up pass), between two events: the
    average milliseconds per launch, i.e. the stage's kernel time without
    the gaps that per-stage events in the chain add."""
    s = s_obj.cuda_stream
    nf = len(frames)
    for i in range(warmup):
        frames[i % nf].stage(k, s)
    t0, t1 = DevEvent(), DevEvent()
    torch.cuda.synchronize()
    t0.record(s)
    for i in range(steps):
        frames[i % nf].stage(k, s)
    t1.record(s)
    torch.cuda.synchronize()
    return t0.elapsed_ms(t1) / steps


# Frames in flight in the headline run and the RLE kernels' workgroups per
# compute unit there, on streams created before any other (us per step with
# 12 buffer copies: 4 frames with both RLE kernels at 2 groups 110.0-111.1,
# both at 3 111.5-112.4, 3 frames at 2 113.5-114.3; with 4 frames, compress x
# decompress caps 1x3 106.1-106.5, 1x2 106.5-106.9, 1x4 106.3-106.8, 1x1
# 106.9-108.9, 2x3 108.4-108.6, 2x2 109.0-109.7, 3x2 111.3-111.9, 4x2 113.3-113.5)
PIPE_IN_FLIGHT = 4
PIPE_COMPRESS_GROUPS = 1
PIPE_DECOMPRESS_GROUPS = 3


def time_pipelined(frames, steps, warmup, s_obj, streams):
    """Frames composited asynchronously (the thesis's pipelined compositing of
    consecutive frames, Section 5.4): step i runs the whole chain for buffer
    copy i mod (copies) on stream i mod len(streams), so that many frames overlap
    (a ROI scan or a compositing pass of one frame next to the RLE kernels
    of another). Each copy's steps stay in order on their stream. Returns
    the milliseconds and wall seconds of `steps` steps between a
    synchronize on each side."""
    nf = len(frames)
    in_flight = len(streams)
    assert nf % in_flight == 0, "each buffer copy must stay on one stream"

    def run(count):
        for i in range(count):
            st = streams[i % in_flight].cuda_stream
            f = frames[i % nf]
            for k in range(4):
                f.stage(k, st)

    # the runtime's per-stream pools grow during the first few dozen steps
    # with several streams busy: at least 64 untimed steps
    run(max(warmup, nf, 64))
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    t0.record(s_obj)
    for st in streams:
        st.wait_event(t0)
    run(steps)
    for st in streams:
        e = torch.cuda.Event()
        e.record(st)
        s_obj.wait_event(e)
    t1.record(s_obj)
    torch.cuda.synchronize()
    return t0.elapsed_time(t1), time.perf_counter() - w0


def time_graph(frames, steps, warmup, s_obj):
    """The same steps captured as HIP graphs (one per frame copy, holding the
    step's five launches) and replayed: `warmup` untimed replays, then
    `steps` timed ones between a synchronize on each side."""
    graphs = []
    for f in frames:
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g):   # captured on torch's side stream
            for k in range(4):
                f.stage(k, torch.cuda.current_stream().cuda_stream)
        graphs.append(g)
    torch.cuda.synchronize()
    for i in range(max(warmup, len(graphs))):
        graphs[i % len(graphs)].replay()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    w0 = time.perf_counter()
    t0.record()
    for i in range(steps):
        graphs[i % len(graphs)].replay()
    t1.record()
    torch.cuda.synchronize()
    return t0.elapsed_time(t1), time.perf_counter() - w0


def bandwidth_probe(dev, nbytes=2 << 30, reps=10):
    """Measured streaming bandwidth (read-only and copy) of a buffer far
    larger than the Infinity Cache: the practical ceiling next to the spec."""
    src = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
    dst = torch.empty_like(src)
    L = cmp.lib()
    s = torch.cuda.current_stream().cuda_stream
    res = {}
    for mode, name, moved in [(0, "read_GBps", nbytes), (1, "copy_GBps", 2 * nbytes)]:
        for _ in range(2):
            L.cmp_bandwidth_probe(mode, src.data_ptr(), dst.data_ptr(), nbytes, s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            st = L.cmp_bandwidth_probe(mode, src.data_ptr(), dst.data_ptr(), nbytes, s)
            if st != 0:
                raise cmp.CmpError(st, "cmp_bandwidth_probe", L.cmp_last_error().decode())
        e1.record()
        torch.cuda.synchronize()
        res[name] = moved / (e0.elapsed_time(e1) / reps) / 1e6
    del src, dst
    torch.cuda.empty_cache()
    return res


def cpu_baseline(frame_host, min_s=10.0, budget_s=25.0):
    """The oracle chain of one full frame on the host (single thread),
    repeated for at least `min_s` seconds (and 3 runs), at most `budget_s`."""
    import oracle
    colors, depths, viewport = frame_host
    times = []
    t_start = time.perf_counter()
    while True:
        elapsed = time.perf_counter() - t_start
        if elapsed >= budget_s or (len(times) >= 3 and elapsed >= min_s):
            break
        t = time.perf_counter()
        rois = [oracle.roi_detect_depth(d) for d in depths]
        crops_c, crops_d = [], []
        for c, d, r in zip(colors, depths, rois):
            s = oracle.rle_compress(c, d, r)
            _, cc, dd = oracle.rle_decompress(s)
            crops_c.append(cc)
            crops_d.append(dd)
        oracle.composite_depth(crops_c, crops_d, rois, viewport)
        times.append(time.perf_counter() - t)
    return float(np.median(times)), len(times), rois, float(sum(times))


# ------------------------------------------------------------------ extras
def bench_over(dev, dtype, reps=10):
    ow = synth.over_bricks(seed=3, n=64, W=3840, H=2160, device=dev, dtype=dtype)
    out = torch.empty((2160, 3840, 4), dtype=torch.float32, device=dev)
    for _ in range(2):
        cmp.composite_over(ow.layers, ow.order, ow.viewport, out=out)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        cmp.composite_over(ow.layers, ow.order, ow.viewport, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    esz = 16 if dtype == torch.float32 else 8
    nbytes = 64 * 3840 * 2160 * esz + 3840 * 2160 * 16
    del ow, out
    torch.cuda.empty_cache()
    return {"ms": ms, "Mpx_per_s": 64 * 3840 * 2160 / ms / 1e3, "GBps": nbytes / ms / 1e6,
            "hbm_frac": nbytes / ms / 1e6 / PEAK_HBM_GBPS, "bytes": nbytes}


EXTRAS_ONLY = ("over_fp32", "over_fp16", "over_backward", "batch")


def bench_codecs(frames, s_obj, reps=50):
    """The compressor family of Section 5.5.1 on the 16 x 1920x1080 frames
    with their device ROIs: stream bytes of per-component RLE, swizzled
    per-component RLE and the basic 64-bit two-pixel RLE (space saved
    against the raw ROI bytes), and the RL64 kernels' times (each launched
    `reps` times back to back over the buffer copies)."""
    s = s_obj.cuda_stream
    f0 = frames[0]
    rois = [tuple(r) for r in f0.roi.cpu().tolist()]
    raw = sum(8 * w * h for _, _, w, h in rois)
    rle1 = int(f0.rle.sizes.sum())
    _, sw, _ = cmp.rle_compress(f0.images, roi_dev=f0.roi, swizzle=True)
    out = {"raw_roi_bytes": raw}
    # RL64: one set of streams and decoded blocks per buffer copy
    L = cmp.lib()
    per = []
    for f in frames:
        caps = [int(L.cmp_rle64_max_size(1920, 1080, 2))] * 16
        outs = [torch.empty(c, dtype=torch.uint8, device=f.roi.device) for c in caps]
        ptrs = (ctypes.c_void_p * 16)(*[o.data_ptr() for o in outs])
        cap_arr = (ctypes.c_uint64 * 16)(*caps)
        sizes = torch.zeros(16, dtype=torch.int64, device=f.roi.device)
        status = torch.zeros(16, dtype=torch.int32, device=f.roi.device)
        ws = torch.zeros(L.cmp_rle_workspace_size(f.img_arr, 16), dtype=torch.uint8,
                         device=f.roi.device)
        dec_bytes = (ctypes.c_uint64 * 16)(*caps)
        per.append((f, outs, ptrs, cap_arr, sizes, status, ws, dec_bytes))

    def comp(p):
        f, outs, ptrs, cap_arr, sizes, status, ws, _ = p
        st = L.cmp_rle64_compress(f.img_arr, 16, cmp.RGBA8, f.roi.data_ptr(), ptrs, cap_arr,
                                  sizes.data_ptr(), status.data_ptr(), ws.data_ptr(), ws.numel(), s)
        assert st == 0, L.cmp_last_error().decode()

    def decomp(p):
        f, outs, ptrs, cap_arr, sizes, status, ws, dec_bytes = p
        st = L.cmp_rle64_decompress(ptrs, dec_bytes, 16, f.dec_out, f.roi_dec.data_ptr(),
                                    f.status.data_ptr(), s)
        assert st == 0, L.cmp_last_error().decode()

    res = {}
    for name, fn in (("rl64_compress", comp), ("rl64_decompress", decomp)):
        for i in range(len(per)):
            fn(per[i])
        t0, t1 = DevEvent(), DevEvent()
        torch.cuda.synchronize()
        t0.record(s)
        for i in range(reps):
            fn(per[i % len(per)])
        t1.record(s)
        torch.cuda.synchronize()
        res[name] = t0.elapsed_ms(t1) / reps * 1e3
    torch.cuda.synchronize()
    # the RL64 round trip must give the frames' ROIs back, with clean statuses
    for p in per:
        assert int(p[5].abs().sum()) == 0 and int(p[0].status.abs().sum()) == 0
    rl64 = int(per[0][4].sum())
    for name, b in (("rle1_per_component", rle1), ("rle1_swizzled", int(sw.sum())),
                    ("rl64_two_pixel", rl64)):
        out[name] = {"bytes": b, "saved": 1 - b / raw}
    roi_px = raw // 8
    for name in ("rl64_compress", "rl64_decompress"):
        out[name] = {"us": res[name], "GBps": (8 * roi_px + rl64) / res[name] / 1e3}
    return out


def read_error_summary(path):
    """`key: value` lines of the committed over-error summary (the parity
    test's full-frame comparison with the FP64 oracle), or None."""
    if not os.path.exists(path):
        return None
    out = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out


def bench_next_rows(frames, s_obj, reps=50):
    """The rows built beyond the hot path, on the 16 x 1920x1080 frames, each
    kernel launched `reps` times back to back over the buffer copies between
    two events: subpixel compositing (Section 4.2.3: the per-channel mean of
    the 16 colour frames), pixel-compound assembly (Section 4.2.2: 4 x 4
    sources of 480x270 interleaved into one 1920x1080 frame) and ROI with
    holes (Section 5.3: the 64x64-cell occupancy grids of the 16 depth frames,
    then their rectangles). Outputs are checked equal across the copies."""
    L = cmp.lib()
    s = s_obj.cuda_stream
    W, H, kx, ky, cell = 1920, 1080, 4, 4, 64
    vp = cmp._rect((0, 0, W, H))
    seq = cmp.Schedule(cmp.SEQ, 1)
    gh, gw = -(-H // cell), -(-W // cell)
    offs = (ctypes.c_int32 * 32)(*[v for i in range(16) for v in (i % kx, i // kx)])
    per = []
    for f in frames:
        dev = f.out_c.device
        colour = cmp._images([cmp.Image(im.color, None, (0, 0, W, H)) for im in f.images], "u32")
        srcs = cmp._images([cmp.Image(im.color[:H // ky, :W // kx], None, (0, 0, W // kx, H // ky))
                            for im in f.images], "u32")
        grid = torch.zeros(16 * gh * gw, dtype=torch.uint8, device=dev)
        rects = torch.zeros((16, 4, 4), dtype=torch.int32, device=dev)
        counts = torch.zeros(16, dtype=torch.int32, device=dev)
        per.append((f, colour, srcs, torch.empty((H, W), dtype=torch.int32, device=dev),
                    torch.empty((H, W), dtype=torch.int32, device=dev), grid, rects, counts))

    def average(p):
        st = L.cmp_composite_average(p[1], 16, vp, p[3].data_ptr(), W, seq, cmp.Tile(0, 0), s)
        assert st == 0, L.cmp_last_error().decode()

    def assemble(p):
        st = L.cmp_assemble_pixels(p[2], 16, offs, kx, ky, vp, p[4].data_ptr(), W, s)
        assert st == 0, L.cmp_last_error().decode()

    def grid(p):
        st = L.cmp_roi_grid(p[0].img_arr, 16, cmp.RGBA8, cell, cell, p[5].data_ptr(), s)
        assert st == 0, L.cmp_last_error().decode()

    def rects(p):
        st = L.cmp_roi_rects(p[0].img_arr, 16, cell, cell, p[5].data_ptr(), 4, p[6].data_ptr(),
                             p[7].data_ptr(), s)
        assert st == 0, L.cmp_last_error().decode()

    px = W * H
    nbytes = {"subpixel_average": 16 * 4 * px + 4 * px, "pixel_assembly": 4 * px + 4 * px,
              "roi_grid": 16 * 4 * px + 16 * gh * gw, "roi_rects": 16 * gh * gw}
    res = {}
    for name, fn in (("subpixel_average", average), ("pixel_assembly", assemble),
                     ("roi_grid", grid), ("roi_rects", rects)):
        for p in per:
            fn(p)
        torch.cuda.synchronize()
        t0, t1 = DevEvent(), DevEvent()
        t0.record(s)
        for i in range(reps):
            fn(per[i % len(per)])
        t1.record(s)
        torch.cuda.synchronize()
        us = t0.elapsed_ms(t1) / reps * 1e3
        res[name] = {"us": us, "bytes": nbytes[name], "GBps": nbytes[name] / us / 1e3,
                     "hbm_frac": nbytes[name] / us / 1e3 / PEAK_HBM_GBPS}
    for p in per[1:]:   # every copy holds the same frames
        assert torch.equal(p[3], per[0][3]) and torch.equal(p[4], per[0][4])
        assert torch.equal(p[5], per[0][5]) and torch.equal(p[6], per[0][6])
    res["workloads"] = ("subpixel: mean of 16 colour frames 1920x1080; assembly: 4x4 sources of "
                        "480x270 into 1920x1080; roi_grid: 64x64 cells of 16 depth frames "
                        "1920x1080; roi_rects: up to 4 rectangles per frame from those grids")
    return res


def bench_backward(dev, reps=10, which=("forward", "backward", "forward_backward")):
    ow = synth.over_bricks(seed=4, n=32, W=1024, H=1024, device=dev, with_target=True)
    imgs = ow.layers
    out = torch.empty((1024, 1024, 4), dtype=torch.float32, device=dev)
    grads = [torch.empty((1024, 1024, 4), dtype=torch.float32, device=dev) for _ in range(32)]
    G = torch.randn((1024, 1024, 4), dtype=torch.float32, device=dev)

    def fwd():
        cmp.composite_over(imgs, ow.order, ow.viewport, out=out)

    def bwd():
        cmp.composite_over_backward(imgs, ow.order, ow.viewport, G, grads=grads)

    res = {}
    px = 1024 * 1024
    for name, fn, nbytes in [("forward", fwd, px * (32 * 16 + 16)),
                             ("backward", bwd, px * (32 * 16 + 16 + 32 * 16)),
                             ("forward_backward", lambda: (fwd(), bwd()), px * (2 * 32 * 16 + 32 + 32 * 16))]:
        if name not in which:
            continue
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"ms": ms, "Mpx_per_s": 32 * px / ms / 1e3, "GBps": nbytes / ms / 1e6,
                     "hbm_frac": nbytes / ms / 1e6 / PEAK_HBM_GBPS, "bytes": nbytes}
    return res


def _union_area(rois, W, H):
    """Pixels of the W x H viewport covered by at least one placement."""
    cover = np.zeros((H, W), bool)
    for x, y, w, h in rois:
        cover[max(0, y):max(0, min(H, y + h)), max(0, x):max(0, min(W, x + w))] = True
    return int(cover.sum())


def bench_batch(dev, reps=5, tune_path=None, which=("persistent_graph", "persistent", "plain_launches")):
    jobs = synth.batch_jobs(seed=5, njobs=256, device=dev)
    outs, keep = [], []
    arr = (cmp.CJob * len(jobs))()
    in_px, nbytes = 0, 0
    for k, job in enumerate(jobs):
        wl = job.work
        _, _, w, h = wl.viewport
        if job.kind == "depth":
            oc = torch.empty((h, w), dtype=torch.int32, device=dev)
            od = torch.empty((h, w), dtype=torch.int32, device=dev)
            imgs = cmp._images(wl.images, "u32")
            arr[k] = cmp.CJob(0, cmp.RGBA8, len(wl.images), imgs, None, cmp._rect(wl.viewport),
                              oc.data_ptr(), od.data_ptr(), w)
            outs.append((oc, od))
            keep.append(imgs)
            cover = sum(r[2] * r[3] for r in (i.roi for i in wl.images))
            covered = _union_area([i.roi for i in wl.images], w, h)
            nbytes += 4 * cover + 4 * covered + 8 * w * h
            in_px += cover
        else:
            o = torch.empty((h, w, 4), dtype=torch.float32, device=dev)
            imgs = cmp._images(wl.layers, "rgba")
            order = (ctypes.c_int32 * len(wl.order))(*wl.order)
            arr[k] = cmp.CJob(1, cmp.RGBA32F, len(wl.layers), imgs, order, cmp._rect(wl.viewport),
                              o.data_ptr(), None, w)
            outs.append(o)
            keep += [imgs, order]
            cover = sum(l.roi[2] * l.roi[3] for l in wl.layers)
            nbytes += 16 * cover + 16 * w * h
            in_px += cover
    L = cmp.lib()
    s = torch.cuda.current_stream()
    if tune_path:
        st = L.cmp_autotune(arr, len(jobs), tune_path.encode(), 3, s.cuda_stream)
        if st != 0:
            raise cmp.CmpError(st, "cmp_autotune", L.cmp_last_error().decode())
    plan = ctypes.c_void_p()
    st = L.cmp_batch_plan_create(arr, len(jobs), tune_path.encode() if tune_path else None,
                                 ctypes.byref(plan))
    if st != 0:
        raise cmp.CmpError(st, "cmp_batch_plan_create", L.cmp_last_error().decode())
    ws = torch.zeros(L.cmp_batch_workspace_size(plan) + 64, dtype=torch.uint8, device=dev)
    L.cmp_batch_upload(plan, ws.data_ptr(), ws.numel(), s.cuda_stream)
    torch.cuda.synchronize()
    items, wgs = ctypes.c_int64(), ctypes.c_int32()
    L.cmp_batch_info(plan, ctypes.byref(items), ctypes.byref(wgs))
    g = torch.cuda.CUDAGraph()
    if "persistent_graph" in which:
        with torch.cuda.graph(g):
            L.cmp_batch_run(plan, ws.data_ptr(), torch.cuda.current_stream().cuda_stream)
    res = {}
    for name, fn in [("persistent_graph", lambda: g.replay()),
                     ("persistent", lambda: L.cmp_batch_run(plan, ws.data_ptr(), s.cuda_stream)),
                     ("plain_launches", lambda: L.cmp_batch_run_plain(plan, s.cuda_stream))]:
        if name not in which:
            continue
        for _ in range(2):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / reps
        res[name] = {"ms": ms, "Mpx_per_s": in_px / ms / 1e3, "GBps": nbytes / ms / 1e6,
                     "hbm_frac": nbytes / ms / 1e6 / PEAK_HBM_GBPS, "bytes": nbytes}
    res["jobs"] = len(jobs)
    res["work_items"] = int(items.value)
    res["workgroups"] = int(wgs.value)
    res["input_Mpx"] = in_px / 1e6
    res["algorithmic_GB"] = nbytes / 1e9
    L.cmp_batch_plan_destroy(plan)
    del keep, outs
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--copies", type=int, default=12,
                    help="buffer copies rotated per step (a multiple of the frames in flight)")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--only", default="", help="profile helper: run only this stage (or probe_copy, a 1 GiB copy; "
                    "or an extra: over_fp32, over_fp16, over_backward, batch, rle64, next_rows) repeatedly")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the library runs the whole path on one GPU; how it would shard is a design "
              "only)", file=sys.stderr)
        sys.exit(2)
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    # the streams of the asynchronous run, made before any other stream: each
    # then runs on a hardware queue of its own (cmp_streams_create)
    in_flight = math.gcd(PIPE_IN_FLIGHT, args.copies)
    pipe_streams = None if args.only else cmp.Streams(in_flight)
    if args.only in EXTRAS_ONLY:
        # profile helper for the extras: `steps` timed launches after two warm-up ones
        if args.only == "over_fp32":
            r = bench_over(dev, torch.float32, reps=args.steps)
        elif args.only == "over_fp16":
            r = bench_over(dev, torch.float16, reps=args.steps)
        elif args.only == "over_backward":
            r = bench_backward(dev, reps=args.steps, which=("backward",))["backward"]
        else:
            r = bench_batch(dev, reps=args.steps, which=("persistent",), tune_path=os.path.join(
                os.environ.get("TMPDIR", "/tmp"), "cmp_tune_cache.txt"))["persistent"]
        log(f"ran {args.only} {args.steps} times: {r['ms']:.3f} ms, {r['bytes']} algorithmic bytes per launch")
        print(json.dumps({"only": args.only, **r}))
        return
    if args.only == "probe_copy":
        # reference kernel for scaling HBM counters: a 1 GiB copy (1 GiB read + 1 GiB written)
        nbytes = 1 << 30
        src = torch.ones(nbytes // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        L = cmp.lib()
        for _ in range(args.steps):
            st = L.cmp_bandwidth_probe(1, src.data_ptr(), dst.data_ptr(), nbytes,
                                       torch.cuda.current_stream().cuda_stream)
            if st != 0:
                raise cmp.CmpError(st, "cmp_bandwidth_probe", L.cmp_last_error().decode())
        torch.cuda.synchronize()
        log(f"copied {nbytes} bytes {args.steps} times")
        return
    log("generating 16 x 1920x1080 contributors")
    frames = []
    for c in range(args.copies):
        wl = synth.depth_ramps_full(seed=2, n=16, W=1920, H=1080, device=dev)
        frames.append(Frame(wl, dev))
    s_obj = torch.cuda.current_stream()
    # one pass over every copy (each holds valid ROIs and streams from here
    # on), checked on the first: ROIs and stream sizes for the byte counts
    for f in frames:
        for k in range(4):
            f.stage(k, s_obj.cuda_stream)
    torch.cuda.synchronize()
    rois = [tuple(r) for r in frames[0].roi.cpu().tolist()]
    assert rois == [im.true_roi for im in frames[0].images], "ROI detection mismatch"
    assert int(frames[0].status.abs().sum()) == 0 and int(frames[0].rle.status.abs().sum()) == 0
    sizes = frames[0].rle.sizes.cpu().numpy()
    abytes, roi_px = algorithmic_bytes(frames[0], rois, sizes)
    ref_color = frames[0].out_c.clone()   # every copy holds the same workload

    if args.only == "rle64":
        # profile helper: the RL64 kernels, `steps` launches each
        r = bench_codecs(frames, s_obj, reps=args.steps)
        log(f"ran rl64 compress and decompress {args.steps} times each")
        print(json.dumps({"only": args.only, **r}))
        return
    if args.only == "next_rows":
        # profile helper: subpixel, assembly, ROI grid and rectangles, `steps` launches each
        r = bench_next_rows(frames, s_obj, reps=args.steps)
        log(f"ran the subpixel, assembly, ROI grid and rectangle kernels {args.steps} times each")
        print(json.dumps({"only": args.only, **r}))
        return
    if args.only:
        k = STAGES.index(args.only)
        for i in range(args.steps):
            frames[i % len(frames)].stage(k, s_obj.cuda_stream)
        torch.cuda.synchronize()
        log(f"ran {args.only} {args.steps} times")
        return

    log(f"timing {args.steps} steps after {args.warmup} warmup")
    total_ms, wall, per = time_stages(frames, args.steps, args.warmup, s_obj)
    ms_step = total_ms / args.steps
    stage_ms = per.mean(axis=0)
    alone_ms = [time_stage_alone(frames, k, args.steps, args.warmup, s_obj) for k in range(4)]
    stages = {}
    for k, name in enumerate(STAGES):
        stages[name] = {"us": float(alone_ms[k] * 1e3), "bytes": int(abytes[name]),
                        "GBps": float(abytes[name] / alone_ms[k] / 1e6),
                        "us_in_chain": float(stage_ms[k] * 1e3)}
    dom = max(STAGES, key=lambda n: stages[n]["us"])
    # several frames in flight: the RLE kernels leave room on every compute
    # unit to the other streams' kernels
    cmp.rle_set_groups_per_cu(PIPE_COMPRESS_GROUPS, PIPE_DECOMPRESS_GROUPS)
    try:
        pipe_total, pipe_wall = time_pipelined(frames, args.steps, args.warmup, s_obj,
                                               pipe_streams.streams)
    finally:
        cmp.rle_set_groups_per_cu(0, 0)
        pipe_streams.close()
    pipe_ms = pipe_total / args.steps
    # one frame at a time as HIP graphs, after the asynchronous run: measured
    # before it, graph capture left the first asynchronous run ~15% slower
    graph_total, graph_wall = time_graph(frames, args.steps, args.warmup, s_obj)
    graph_ms = graph_total / args.steps
    # the timed runs left every copy's statuses clear and its composite intact
    for f in frames:
        assert int(f.status.abs().sum()) == 0 and int(f.rle.status.abs().sum()) == 0, "RLE status"
        assert torch.equal(f.out_c, ref_color), "composite changed during the timed runs"
    probe = bandwidth_probe(dev)
    step_bytes = sum(abytes.values())
    achieved = stages[dom]["GBps"]
    traffic = None
    t = read_traffic(os.path.join(ROOT, "profiles", f"hbm_traffic_{dom}.txt"))
    if t and t.get("source_hash") == _source_hash(dom):
        traffic = float(t["bytes_per_launch"])
    result = {
        "metric": METRIC,
        "value": roi_px / (pipe_ms * 1e3),
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": pipe_ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {"workload": "sort-last depth pipeline: roi_detect + per-component RLE "
                               "compress/decompress + depth compositing",
                   "contributors": 16, "width": 1920, "height": 1080,
                   "roi_area_fraction": "0.25-0.35", "schedule": "binary_swap(16)",
                   "composited_input_px_per_step": roi_px, "buffer_copies": args.copies},
        "timing": f"value and ms_per_step: frames composited asynchronously, {in_flight} in "
                  f"flight (each frame's whole chain on one of {in_flight} streams, compression at "
                  f"{PIPE_COMPRESS_GROUPS} and decompression at {PIPE_DECOMPRESS_GROUPS} "
                  "workgroups per CU); graph: one frame at a time, its four "
                  "launches replayed as a HIP graph; eager: the chain one frame at a time; stages "
                  "and roofline: each stage launched back to back over the buffer copies between two "
                  "events (us_in_chain: between per-stage events inside the eager chain), RLE "
                  "kernels at full occupancy",
        "frames_in_flight": in_flight,
        "pipelined_rle_groups_per_cu": {"compress": PIPE_COMPRESS_GROUPS,
                                        "decompress": PIPE_DECOMPRESS_GROUPS},
        "graph_ms_per_step": graph_ms,
        "eager_ms_per_step": ms_step,
        "hbm_GBps_step": step_bytes / pipe_ms / 1e6,
        "hbm_frac_step": step_bytes / pipe_ms / 1e6 / PEAK_HBM_GBPS,
        "stages": stages,
        "roofline": {"bound": "hbm", "kernel": f"{dom}: {STAGE_KERNELS[dom]}", "achieved": achieved,
                     "peak": PEAK_HBM_GBPS,
                     "unit": "GB/s", "frac": achieved / PEAK_HBM_GBPS, "traffic": traffic},
        "probe": dict(probe, frac_of_read_probe=achieved / probe["read_GBps"]),
        "wall_s_timed": pipe_wall,
        "wall_s_timed_graph": graph_wall,
        "wall_s_timed_eager": wall,
    }
    if not args.no_extras:
        log("extras: over 64x3840x2160 fp32/fp16, backward 32x1024x1024, batch of 256 jobs")
        ex = {}
        ex["over_fp32_64x3840x2160"] = bench_over(dev, torch.float32)
        ex["over_fp16_64x3840x2160"] = bench_over(dev, torch.float16)
        ex["over_grad_32x1024x1024"] = bench_backward(dev)
        ex["batch_256_jobs"] = bench_batch(dev, tune_path=os.path.join(
            os.environ.get("TMPDIR", "/tmp"), "cmp_tune_cache.txt"))
        ex["codecs_16x1920x1080"] = bench_codecs(frames, s_obj)
        ex["next_rows_16x1920x1080"] = bench_next_rows(frames, s_obj)
        err = read_error_summary(os.path.join(ROOT, "profiles", "over_error_64x3840x2160.txt"))
        if err:
            ex["over_fp32_64x3840x2160"]["rel_err"] = {k[5:]: v for k, v in err.items() if k.startswith("fp32_")}
            ex["over_fp16_64x3840x2160"]["rel_err"] = {k[5:]: v for k, v in err.items() if k.startswith("fp16_")}
        result["extras"] = ex
    if not args.no_cpu:
        log("cpu baseline: the oracle chain on one full frame")
        f = frames[0]
        host = ([synth.as_u32(im.color) for im in f.images], [synth.as_u32(im.depth) for im in f.images],
                f.viewport)
        t, reps, _, total = cpu_baseline(host)
        result["cpu_baseline"] = {"value": roi_px / (t * 1e6), "unit": "Mpixel/s", "cores": 1,
                                  "kind": "oracle",
                                  "sample": f"one full frame (16 x 1920x1080) of the same pipeline, "
                                            f"median of {reps} runs ({t:.2f} s each, {total:.1f} s "
                                            f"of CPU work)"}
    print(json.dumps(result), flush=True)


def read_traffic(path):
    """`key: value` lines of a committed HBM-counter summary (None if absent).
    The counters are only valid for the kernel sources they were taken on,
    so the summary carries a hash of those sources."""
    if not os.path.exists(path):
        return None
    out = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            out[k.strip()] = v.strip()
    return out if "bytes_per_launch" in out else None


# The sources each stage's kernels are built from: a counter summary stays
# valid while these are unchanged.
STAGE_SOURCES = {"roi_detect": ("roi.hip", "cmp_internal.hpp"),
                 "rle_compress": ("rle.hip", "rle_common.hpp", "cmp_internal.hpp"),
                 "rle_decompress": ("rle.hip", "rle_common.hpp", "cmp_internal.hpp"),
                 "composite_depth": ("depth.hip", "depth_tile.hpp", "cmp_internal.hpp")}


def _source_hash(stage=None):
    """sha256[:16] of the stage's kernel sources (all of csrc/ without a stage)."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1902_08755_amd", "csrc")
    names = STAGE_SOURCES[stage] if stage else sorted(os.listdir(csrc))
    for name in names:
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


if __name__ == "__main__":
    main()
