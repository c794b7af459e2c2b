"""Seeded synthetic workloads for the sort-last compositing path.

This module only draws inputs; it holds none of the compositing, ROI or RLE
arithmetic. Both the oracle-side tests and the GPU path use it, and it runs
unchanged on the CPU or on a GPU: every value comes from integer hashing and
single exactly-rounded float operations, so the same seed gives the same bits
on any device.

Randomness: a counter-based generator. The key for (seed, stream) is derived
with the splitmix64 finaliser, and value number ``c`` of that stream is the
(c+1)-th output of the splitmix64 generator started at the key (Steele, Lea
and Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).

Workload shapes follow the thesis's sort-last setting (chapter 5): compact
per-source regions of interest on otherwise clear framebuffers (Section 5.3),
smooth rendered depth surfaces, and depth-sorted volume bricks blended in order
(Section 5.2.1). The thesis's datasets are not available; these stand in.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import torch

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
CLEAR_DEPTH = 0xFFFFFFFF


# ------------------------------------------------------------ scalar (host)
def mix64(z: int) -> int:
    """splitmix64 output finaliser on a Python int (mod 2^64)."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def stream_key(seed: int, stream: int) -> int:
    return mix64(mix64(seed * GAMMA + 1) ^ ((stream + 1) * GAMMA))


def hash64(seed: int, stream: int, ctr: int) -> int:
    """Value number ``ctr`` of stream ``stream``: splitmix64 output ctr+1."""
    return mix64(stream_key(seed, stream) + (ctr + 1) * GAMMA)


class HostRng:
    """Sequential draws from one (seed, stream) on the host."""

    def __init__(self, seed: int, stream: int):
        self.key = stream_key(seed, stream)
        self.ctr = 0

    def next64(self) -> int:
        self.ctr += 1
        return mix64(self.key + self.ctr * GAMMA)

    def uniform(self) -> float:
        """Uniform in [0, 1) with 24 bits (exact in fp32)."""
        return (self.next64() >> 40) * 2.0 ** -24

    def randint(self, lo: int, hi: int) -> int:
        """Uniform integer in [lo, hi] (inclusive)."""
        m = hi - lo + 1
        return lo + (((self.next64() >> 32) * m) >> 32)

    def permutation(self, n: int):
        """Fisher-Yates shuffle of 0..n-1."""
        p = list(range(n))
        for i in range(n - 1, 0, -1):
            j = self.randint(0, i)
            p[i], p[j] = p[j], p[i]
        return p


# ---------------------------------------------------------- vector (torch)
def _s64(v: int) -> int:
    v &= MASK64
    return v - (1 << 64) if v >= (1 << 63) else v


def _lsr(x: torch.Tensor, k: int) -> torch.Tensor:
    """Logical right shift of int64 bit patterns."""
    return (x >> k) & ((1 << (64 - k)) - 1)


def mix64_t(z: torch.Tensor) -> torch.Tensor:
    """splitmix64 finaliser on int64 tensors (two's complement wrap-around)."""
    z = (z ^ _lsr(z, 30)) * _s64(M1)
    z = (z ^ _lsr(z, 27)) * _s64(M2)
    return z ^ _lsr(z, 31)


def hash64_t(seed: int, stream: int, ctr: torch.Tensor) -> torch.Tensor:
    """Vector form of :func:`hash64`; ``ctr`` is an int64 tensor."""
    key = _s64(stream_key(seed, stream))
    return mix64_t(key + (ctr + 1) * _s64(GAMMA))


def uniform_t(h: torch.Tensor) -> torch.Tensor:
    """24-bit uniform in [0, 1) as float32 (exact)."""
    return _lsr(h, 40).to(torch.float32) * (2.0 ** -24)


def randint_t(h: torch.Tensor, lo: int, hi: int) -> torch.Tensor:
    m = hi - lo + 1
    return lo + ((_lsr(h, 32) * m) >> 32)


# ----------------------------------------------------------------- images
@dataclass
class DepthImage:
    """RGBA8 colour + uint32 depth, row-major with a pitch (pixels)."""
    color: torch.Tensor      # int32 bit patterns (H, pitch)
    depth: torch.Tensor      # int32 bit patterns (H, pitch)
    roi: tuple               # (x, y, w, h) placement in destination pixels
    true_roi: tuple = None   # generator's own knowledge of the data's bounding box


@dataclass
class OverLayer:
    rgba: torch.Tensor       # float (H, pitch, 4)
    roi: tuple


def u32_to_i32(v: int) -> int:
    return v - (1 << 32) if v >= (1 << 31) else v


def _padded(w: int, pad: int) -> int:
    return ((w + pad - 1) // pad) * pad if pad > 1 else w


def rect_image(seed, stream, W, H, nrects=20, device="cpu", pitch_pad=1):
    """A clear W x H framebuffer with ``nrects`` random rectangles drawn in
    order with a strict-less depth test; uniform random depth and colour per
    rectangle (the 640x480 correctness workload)."""
    rng = HostRng(seed, stream)
    P = _padded(W, pitch_pad)
    depth = torch.full((H, P), u32_to_i32(CLEAR_DEPTH), dtype=torch.int64, device=device)
    color = torch.zeros((H, P), dtype=torch.int64, device=device)
    for _ in range(nrects):
        x0 = rng.randint(0, W - 1)
        y0 = rng.randint(0, H - 1)
        w = rng.randint(1, W // 2)
        h = rng.randint(1, H // 2)
        d = rng.randint(0, CLEAR_DEPTH - 1)
        c = rng.randint(0, CLEAR_DEPTH)
        x1, y1 = min(W, x0 + w), min(H, y0 + h)
        dv = depth[y0:y1, x0:x1] & 0xFFFFFFFF
        closer = d < dv
        depth[y0:y1, x0:x1] = torch.where(closer, torch.full_like(dv, u32_to_i32(d)), depth[y0:y1, x0:x1])
        color[y0:y1, x0:x1] = torch.where(closer, torch.full_like(dv, u32_to_i32(c)), color[y0:y1, x0:x1])
    return DepthImage(color.to(torch.int32), depth.to(torch.int32), (0, 0, W, H))


def ramp_roi_params(seed, stream, W, H, area=(0.25, 0.35)):
    """ROI rectangle and depth-ramp parameters of one sort-last contributor."""
    rng = HostRng(seed, stream)
    a = area[0] + (area[1] - area[0]) * rng.uniform()
    s = 0.8 + 0.45 * rng.uniform()
    w = min(W, max(1, int(round(W * math.sqrt(a) * s))))
    h = min(H, max(1, int(round(H * math.sqrt(a) / s))))
    x0 = rng.randint(0, W - w)
    y0 = rng.randint(0, H - h)
    d0 = rng.randint(1 << 30, 3 << 30)
    gx = rng.randint(-4096, 4096)
    gy = rng.randint(-4096, 4096)
    return (x0, y0, w, h), d0, gx, gy


def ramp_block(seed, stream, index, roi, d0, gx, gy, device="cpu"):
    """Colour and depth of a contributor's w x h ROI block: a smooth depth
    ramp plus small noise, and a colour gradient over the block."""
    x0, y0, w, h = roi
    yy = torch.arange(h, device=device, dtype=torch.int64).view(-1, 1)
    xx = torch.arange(w, device=device, dtype=torch.int64).view(1, -1)
    ctr = yy * w + xx
    nu = randint_t(hash64_t(seed, 1000 + stream, ctr), -128, 127)
    d = d0 + gx * xx + gy * yy + nu
    d = d.clamp(0, CLEAR_DEPTH - 1)
    r = (255 * xx) // max(1, w - 1) if w > 1 else torch.zeros_like(xx)
    g = (255 * yy) // max(1, h - 1) if h > 1 else torch.zeros_like(yy)
    b = (16 * index) % 256
    c = (r + (g << 8) + (b << 16) + (255 << 24)).expand(h, w)
    return c, d


def _to_i32(t: torch.Tensor) -> torch.Tensor:
    t = t & 0xFFFFFFFF
    return torch.where(t >= (1 << 31), t - (1 << 32), t).to(torch.int32)


def ramp_image(seed, stream, index, W, H, device="cpu", pitch_pad=1, area=(0.25, 0.35)):
    """A full W x H clear framebuffer holding one contributor's ramp ROI."""
    roi, d0, gx, gy = ramp_roi_params(seed, stream, W, H, area)
    x0, y0, w, h = roi
    P = _padded(W, pitch_pad)
    depth = torch.full((H, P), u32_to_i32(CLEAR_DEPTH), dtype=torch.int32, device=device)
    color = torch.zeros((H, P), dtype=torch.int32, device=device)
    c, d = ramp_block(seed, stream, index, roi, d0, gx, gy, device)
    depth[y0:y0 + h, x0:x0 + w] = _to_i32(d)
    color[y0:y0 + h, x0:x0 + w] = _to_i32(c)
    return DepthImage(color, depth, (0, 0, W, H), true_roi=roi)


def ramp_contributor(seed, stream, index, W, H, device="cpu", pitch_pad=1, area=(0.25, 0.35)):
    """Only the ROI block of a ramp contributor, placed by its ROI."""
    roi, d0, gx, gy = ramp_roi_params(seed, stream, W, H, area)
    x0, y0, w, h = roi
    P = _padded(w, pitch_pad)
    c, d = ramp_block(seed, stream, index, roi, d0, gx, gy, device)
    color = torch.zeros((h, P), dtype=torch.int32, device=device)
    depth = torch.full((h, P), u32_to_i32(CLEAR_DEPTH), dtype=torch.int32, device=device)
    color[:, :w] = _to_i32(c)
    depth[:, :w] = _to_i32(d)
    return DepthImage(color, depth, roi, true_roi=(0, 0, w, h))


def brick_layer(seed, stream, w, h, device="cpu", pitch_pad=1, dtype=torch.float32,
                row0=0, nrows=None):
    """One volume-brick layer: alpha ~ Beta(2,5) drawn as the second smallest
    of six uniforms; colour channel k = u_k * alpha (premultiplied).
    ``row0``/``nrows`` draw a horizontal band of the layer only (same values
    as the full layer in those rows)."""
    nrows = h - row0 if nrows is None else nrows
    P = _padded(w, pitch_pad)
    yy = torch.arange(row0, row0 + nrows, device=device, dtype=torch.int64).view(-1, 1)
    xx = torch.arange(w, device=device, dtype=torch.int64).view(1, -1)
    base = (yy * w + xx) * 9
    slots = torch.arange(9, device=device, dtype=torch.int64)
    u = uniform_t(hash64_t(seed, stream, base.unsqueeze(-1) + slots))  # (rows, w, 9)
    alpha = torch.sort(u[..., :6], dim=-1).values[..., 1]
    rgb = u[..., 6:9] * alpha.unsqueeze(-1)
    out = torch.zeros((nrows, P, 4), dtype=torch.float32, device=device)
    out[:, :w, :3] = rgb
    out[:, :w, 3] = alpha
    return out.to(dtype)


def target_image(seed, stream, w, h, device="cpu"):
    """Uniform [0,1) RGBA target image (float32)."""
    yy = torch.arange(h, device=device, dtype=torch.int64).view(-1, 1, 1)
    xx = torch.arange(w, device=device, dtype=torch.int64).view(1, -1, 1)
    k = torch.arange(4, device=device, dtype=torch.int64).view(1, 1, -1)
    return uniform_t(hash64_t(seed, stream, (yy * w + xx) * 4 + k))


# -------------------------------------------------------------- workloads
@dataclass
class DepthWorkload:
    viewport: tuple
    images: list             # DepthImage list
    name: str = ""


@dataclass
class OverWorkload:
    viewport: tuple
    layers: list             # OverLayer list
    order: list              # back to front
    name: str = ""
    target: torch.Tensor = None


def depth_rects(seed=1, n=4, W=640, H=480, nrects=20, device="cpu", pitch_pad=1):
    """n full-frame contributors with random rectangles (correctness case)."""
    imgs = [rect_image(seed, i, W, H, nrects, device, pitch_pad) for i in range(n)]
    return DepthWorkload((0, 0, W, H), imgs, f"depth_rects_{n}x{W}x{H}")


def depth_ramps_full(seed=2, n=16, W=1920, H=1080, device="cpu", pitch_pad=1):
    """n full-frame clear framebuffers, each with one ~30% ramp ROI."""
    imgs = [ramp_image(seed, i, i, W, H, device, pitch_pad) for i in range(n)]
    return DepthWorkload((0, 0, W, H), imgs, f"depth_ramps_{n}x{W}x{H}")


def depth_ramps_roi(seed=2, n=16, W=1920, H=1080, device="cpu", pitch_pad=1):
    """The same contributors as :func:`depth_ramps_full`, ROI blocks only."""
    imgs = [ramp_contributor(seed, i, i, W, H, device, pitch_pad) for i in range(n)]
    return DepthWorkload((0, 0, W, H), imgs, f"depth_ramps_roi_{n}x{W}x{H}")


def over_bricks(seed=3, n=64, W=3840, H=2160, device="cpu", dtype=torch.float32, pitch_pad=1,
                with_target=False):
    """n full-frame brick layers and a random back-to-front order."""
    layers = [OverLayer(brick_layer(seed, i, W, H, device, pitch_pad, dtype), (0, 0, W, H))
              for i in range(n)]
    order = HostRng(seed, 10_000).permutation(n)
    tgt = target_image(seed, 20_000, W, H, device) if with_target else None
    return OverWorkload((0, 0, W, H), layers, order, f"over_bricks_{n}x{W}x{H}", tgt)


def over_bricks_roi(seed, n, W, H, device="cpu", dtype=torch.float32, pitch_pad=1,
                    frac=(0.25, 1.0)):
    """n brick layers, each covering a random sub-rectangle of the viewport."""
    rng = HostRng(seed, 30_000)
    layers = []
    for i in range(n):
        w = max(1, int(round(W * (frac[0] + (frac[1] - frac[0]) * rng.uniform()))))
        h = max(1, int(round(H * (frac[0] + (frac[1] - frac[0]) * rng.uniform()))))
        w, h = min(w, W), min(h, H)
        x0 = rng.randint(0, W - w)
        y0 = rng.randint(0, H - h)
        layers.append(OverLayer(brick_layer(seed, i, w, h, device, pitch_pad, dtype), (x0, y0, w, h)))
    order = HostRng(seed, 10_000).permutation(n)
    return OverWorkload((0, 0, W, H), layers, order, f"over_bricks_roi_{n}x{W}x{H}")


@dataclass
class Job:
    kind: str                # "depth" or "over"
    work: object             # DepthWorkload or OverWorkload (viewport at origin)


def batch_jobs(seed=5, njobs=256, device="cpu", log2_range=(6.0, 11.0), n_range=(2, 32),
               max_side=None):
    """Uneven compositing jobs: sides log-uniform in 2^[6, 11], 2..32
    contributors, even jobs depth, odd jobs over, ROI-cropped contributors."""
    rng = HostRng(seed, 40_000)
    jobs = []
    for j in range(njobs):
        w = int(round(2.0 ** (log2_range[0] + (log2_range[1] - log2_range[0]) * rng.uniform())))
        h = int(round(2.0 ** (log2_range[0] + (log2_range[1] - log2_range[0]) * rng.uniform())))
        if max_side:
            w, h = min(w, max_side), min(h, max_side)
        n = rng.randint(*n_range)
        jseed = seed * 1_000_003 + j
        if j % 2 == 0:
            imgs = []
            for i in range(n):
                roi, d0, gx, gy = _job_roi(HostRng(jseed, i), w, h)
                c, d = ramp_block(jseed, i, i, roi, d0, gx, gy, device)
                imgs.append(DepthImage(_line_aligned(_to_i32(c), roi[0], 32),
                                       _line_aligned(_to_i32(d), roi[0], 32), roi))
            jobs.append(Job("depth", DepthWorkload((0, 0, w, h), imgs, f"job{j}")))
        else:
            lay = []
            for i in range(n):
                roi, _, _, _ = _job_roi(HostRng(jseed, i), w, h)
                layer = brick_layer(jseed, i, roi[2], roi[3], device)[:, :roi[2]]
                lay.append(OverLayer(_line_aligned(layer, roi[0], 8), roi))
            order = HostRng(jseed, 10_000).permutation(n)
            jobs.append(Job("over", OverWorkload((0, 0, w, h), lay, order, f"job{j}")))
    return jobs


def _line_aligned(block: torch.Tensor, x0: int, px_per_line: int) -> torch.Tensor:
    """The (h, w[, 4]) block as a view into a zeroed buffer whose pitch is a
    multiple of one 128-byte line (px_per_line pixels), the block starting at
    column x0 mod px_per_line: a row segment of the block then sits on the same
    line boundaries as the destination columns it lands on, so a wave's row
    access touches whole lines (the layout the frames placed at their ROIs
    have). The pixel values are those of the block."""
    h, w = block.shape[0], block.shape[1]
    off = x0 % px_per_line
    pitch = -(-(off + w) // px_per_line) * px_per_line
    buf = torch.zeros((h, pitch) + tuple(block.shape[2:]), dtype=block.dtype, device=block.device)
    buf[:, off:off + w] = block
    return buf[:, off:off + w]


def _job_roi(rng: HostRng, W, H):
    fw = 0.25 + 0.75 * rng.uniform()
    fh = 0.25 + 0.75 * rng.uniform()
    w = min(W, max(1, int(round(W * fw))))
    h = min(H, max(1, int(round(H * fh))))
    x0 = rng.randint(0, W - w)
    y0 = rng.randint(0, H - h)
    d0 = rng.randint(1 << 30, 3 << 30)
    gx = rng.randint(-4096, 4096)
    gy = rng.randint(-4096, 4096)
    return (x0, y0, w, h), d0, gx, gy


# ------------------------------------------------------------ numpy views
def as_u32(t: torch.Tensor):
    """uint32 numpy view of an int32 bit-pattern tensor (copied to host)."""
    return t.detach().cpu().contiguous().numpy().view("uint32")
