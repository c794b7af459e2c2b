// cmp_roi_detect: automatic region-of-interest detection, the 2D bounding box
// of the pixels that hold data (Section 5.3, Region of Interest).
//
// One pass over every image, several images per launch. A workgroup scans a
// band of rows with 16-byte loads (4 depth or RGBA8 pixels, 2 RGBA16F pixels
// or 1 RGBA32F pixel per load, several in flight per lane), keeps per-lane
// min/max of the data pixels' columns and rows, reduces them across the wave
// and the workgroup, and stores the workgroup's box in a slot of its own.
// The last workgroup of an image (counted with an atomic ticket, one per
// image on its own cache line) folds the image's slots into the rectangle and
// clears the ticket, so the workspace is ready for the next call. One
// read-modify-write per workgroup: atomics on a shared line are serialised,
// and per-workgroup atomic maxima on a few shared words cost several
// microseconds at the end of the launch. No fence is needed: every access to
// the shared words is a device-scope atomic.
#include <string.h>

#include "cmp_internal.hpp"

namespace cmp {

constexpr int kRoiMax = 64;
constexpr int kRoiBatch = 8;
// workspace: one int32 ticket per image, each on its own 128-byte line
// (8 KiB), then one int32[4] partial box per workgroup
constexpr int kTicketStride = 32;
constexpr size_t kRoiTickets = (size_t)kRoiMax * kTicketStride * 4;

struct RoiImg {
  const void* color;
  const uint32_t* depth;
  int64_t pitch;
  int32_t w, h;
  int32_t wg_begin;   // first workgroup of this image
  int32_t nwg;        // workgroups of this image
  int32_t rows;       // rows per workgroup
  int32_t pad;
};

struct RoiArgs {
  RoiImg im[kRoiMax];
  int32_t* roi_out;
  int32_t* ticket;    // workspace: a ticket per image, kTicketStride words apart
  int4* part;         // workspace: a partial box per workgroup
  int32_t n;
  int32_t mode;       // 0 depth, 1 RGBA8 colour, 2 RGBA32F, 3 RGBA16F
};
static_assert(sizeof(RoiArgs) <= 4096, "kernel arguments must fit in 4 KiB");

// Bit k of the result is set when pixel k of the 16-byte unit holds data.
template <int MODE>
__device__ __forceinline__ uint32_t unit_mask(u32x4 v) {
  if constexpr (MODE == 0) {
    return (v.x != kClearDepth) | ((v.y != kClearDepth) << 1) | ((v.z != kClearDepth) << 2) |
           ((v.w != kClearDepth) << 3);
  } else if constexpr (MODE == 1) {
    return (v.x != 0u) | ((v.y != 0u) << 1) | ((v.z != 0u) << 2) | ((v.w != 0u) << 3);
  } else if constexpr (MODE == 2) {
    // any channel != 0.0: -0.0 is empty, NaN holds data
    return ((v.x | v.y | v.z | v.w) & 0x7FFFFFFFu) != 0u;
  } else {
    const uint32_t a = (v.x & 0x7FFF7FFFu) | (v.y & 0x7FFF7FFFu);
    const uint32_t b = (v.z & 0x7FFF7FFFu) | (v.w & 0x7FFF7FFFu);
    return (a != 0u) | ((b != 0u) << 1);
  }
}

template <int MODE>
__device__ __forceinline__ uint32_t px_mask(const uint8_t* row, int x) {
  if constexpr (MODE == 0 || MODE == 1) {
    const uint32_t v = reinterpret_cast<const uint32_t*>(row)[x];
    return MODE == 0 ? v != kClearDepth : v != 0u;
  } else if constexpr (MODE == 2) {
    const u32x4 v = reinterpret_cast<const u32x4*>(row)[x];
    return ((v.x | v.y | v.z | v.w) & 0x7FFFFFFFu) != 0u;
  } else {
    const uint2 v = reinterpret_cast<const uint2*>(row)[x];
    return ((v.x | v.y) & 0x7FFF7FFFu) != 0u;
  }
}

template <int MODE>
__global__ __launch_bounds__(kThreads) void roi_kernel(const RoiArgs a) {
  constexpr int bpp = MODE == 2 ? 16 : MODE == 3 ? 8 : 4;
  constexpr int ppu = 16 / bpp;  // pixels per 16-byte unit
  const int blk = blockIdx.x;
  int s = 0;
  s = segment_of([&](int i) { return a.im[i].wg_begin; }, a.n, blk);
  const RoiImg I = a.im[s];
  const int local = blk - I.wg_begin;
  const int y0 = local * I.rows;
  const int y1 = min(I.h, y0 + I.rows);
  const uint8_t* base =
      reinterpret_cast<const uint8_t*>(MODE == 0 ? (const void*)I.depth : I.color);
  const int64_t row_bytes = I.pitch * bpp;
  // 16-byte units per row, and whether the row start is 16-byte aligned
  const bool aligned = ((reinterpret_cast<uintptr_t>(base) | (uintptr_t)row_bytes) & 15) == 0;
  const int full_units = aligned ? I.w / ppu : 0;
  const int tail = I.w - full_units * ppu;   // pixels handled one by one

  int minx = 0x7FFFFFFF, miny = 0x7FFFFFFF, maxx = -1, maxy = -1;
  const int nrows = y1 - y0;
  // Full 16-byte units, flat over (row, unit): lane t takes units t, t + 256,
  // ...; kRoiBatch loads are issued unconditionally (an index past the end
  // reads unit 0 of the band instead and is ignored) so they are all in
  // flight before the first is examined.
  const int uwork = full_units * nrows;
  if (uwork > 0) {
    const int dq = kThreads / full_units, dr = kThreads - dq * full_units;
    int ry = (int)threadIdx.x / full_units;
    int u = (int)threadIdx.x - ry * full_units;
    for (int t0 = threadIdx.x; t0 < uwork; t0 += kThreads * kRoiBatch) {
      u32x4 v[kRoiBatch];
      int xs[kRoiBatch], ys[kRoiBatch];
#pragma unroll
      for (int k = 0; k < kRoiBatch; ++k) {
        const bool ok = t0 + k * kThreads < uwork;
        xs[k] = ok ? u * ppu : -1;
        ys[k] = y0 + ry;
        const u32x4* row =
            reinterpret_cast<const u32x4*>(base + (int64_t)(y0 + (ok ? ry : 0)) * row_bytes);
        v[k] = __builtin_nontemporal_load(&row[ok ? u : 0]);   // read once
        u += dr;
        ry += dq;
        if (u >= full_units) { u -= full_units; ++ry; }
      }
#pragma unroll
      for (int k = 0; k < kRoiBatch; ++k) {
        const uint32_t m = xs[k] >= 0 ? unit_mask<MODE>(v[k]) : 0u;
        if (m) {
          minx = min(minx, xs[k] + (int)__builtin_ctz(m));
          maxx = max(maxx, xs[k] + 31 - (int)__builtin_clz(m));
          miny = min(miny, ys[k]);
          maxy = max(maxy, ys[k]);
        }
      }
    }
  }
  // The remaining pixels of each row (all of them when rows are not 16-byte
  // aligned), one load per pixel, batched the same way.
  const int twork = tail * nrows;
  for (int t0 = threadIdx.x; t0 < twork; t0 += kThreads * kRoiBatch) {
    uint32_t m[kRoiBatch];
    int xs[kRoiBatch], ys[kRoiBatch];
#pragma unroll
    for (int k = 0; k < kRoiBatch; ++k) {
      const int t = t0 + k * kThreads;
      const bool ok = t < twork;
      const int tc = ok ? t : 0;
      const int r = tc / tail;
      xs[k] = full_units * ppu + (tc - r * tail);
      ys[k] = y0 + r;
      const uint32_t mm = px_mask<MODE>(base + (int64_t)(y0 + r) * row_bytes, xs[k]);
      m[k] = ok ? mm : 0u;
    }
#pragma unroll
    for (int k = 0; k < kRoiBatch; ++k) {
      if (m[k]) {
        minx = min(minx, xs[k]);
        maxx = max(maxx, xs[k]);
        miny = min(miny, ys[k]);
        maxy = max(maxy, ys[k]);
      }
    }
  }
  __shared__ int4 red[kThreads / kWave];
  __shared__ bool s_last;
  minx = wave_min(minx);
  miny = wave_min(miny);
  maxx = wave_max(maxx);
  maxy = wave_max(maxy);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == 0) red[wave] = int4{minx, miny, maxx, maxy};
  __syncthreads();
  if (threadIdx.x == 0) {
    int4 b = red[0];
#pragma unroll
    for (int w = 1; w < kThreads / kWave; ++w) {
      b.x = min(b.x, red[w].x);
      b.y = min(b.y, red[w].y);
      b.z = max(b.z, red[w].z);
      b.w = max(b.w, red[w].w);
    }
    // the workgroup's box goes to its own slot, then the image's ticket is
    // taken; the slot stores complete (s_waitcnt) before the ticket, so the
    // image's last workgroup sees every slot. Device-scope atomic stores and
    // loads, no fence; one read-modify-write per workgroup.
    int* slot = reinterpret_cast<int*>(a.part + blk);
    __hip_atomic_store(&slot[0], b.x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&slot[1], b.y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&slot[2], b.z, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(&slot[3], b.w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    const int t = __hip_atomic_fetch_add(&a.ticket[s * kTicketStride], 1, __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_AGENT);
    s_last = t == I.nwg - 1;
  }
  __syncthreads();
  if (s_last) {   // the image's last workgroup folds the image's slots
    int4 r{0x7FFFFFFF, 0x7FFFFFFF, -1, -1};
#pragma unroll 4
    for (int i = threadIdx.x; i < I.nwg; i += kThreads) {
      const int* slot = reinterpret_cast<const int*>(a.part + I.wg_begin + i);
      r.x = min(r.x, __hip_atomic_load(&slot[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      r.y = min(r.y, __hip_atomic_load(&slot[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      r.z = max(r.z, __hip_atomic_load(&slot[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
      r.w = max(r.w, __hip_atomic_load(&slot[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
    }
    r.x = wave_min(r.x);
    r.y = wave_min(r.y);
    r.z = wave_max(r.z);
    r.w = wave_max(r.w);
    __syncthreads();   // red[] is reused
    if (lane == 0) red[wave] = r;
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
      for (int w = 1; w < kThreads / kWave; ++w) {
        r.x = min(r.x, red[w].x);
        r.y = min(r.y, red[w].y);
        r.z = max(r.z, red[w].z);
        r.w = max(r.w, red[w].w);
      }
      int4 box{0, 0, 0, 0};
      if (r.z >= 0) box = int4{r.x, r.y, r.z - r.x + 1, r.w - r.y + 1};
      reinterpret_cast<int4*>(a.roi_out)[s] = box;
      __hip_atomic_store(&a.ticket[s * kTicketStride], 0, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// Rows per workgroup: about 128 KiB of reads per workgroup, and at most
// kRoiSlotsMax workgroups per image (the slots its last workgroup folds).
constexpr int kRoiSlotsMax = 1024;
static int roi_rows(const cmp_image& I, int bpp) {
  const int64_t row_bytes = (int64_t)(I.roi.w > 0 ? I.roi.w : 1) * bpp;
  int64_t r = (128 * 1024 + row_bytes - 1) / row_bytes;
  r = std::max<int64_t>(r, ((int64_t)I.roi.h + kRoiSlotsMax - 1) / kRoiSlotsMax);
  if (r < 1) r = 1;
  if (r > I.roi.h) r = I.roi.h > 0 ? I.roi.h : 1;
  return (int)r;
}

// Workgroups of a launch over images [0, n): an empty image takes one.
static int64_t roi_workgroups(const cmp_image* imgs, int n, int bpp) {
  int64_t wg = 0;
  for (int i = 0; i < n; ++i) {
    const cmp_image& I = imgs[i];
    if (!rect_valid(I.roi) || rect_empty(I.roi)) {
      wg += 1;
      continue;
    }
    const int rows = roi_rows(I, bpp);
    wg += (I.roi.h + rows - 1) / rows;
  }
  return wg;
}

static int roi_bpp(cmp_format fmt) { return fmt == CMP_RGBA32F ? 16 : fmt == CMP_RGBA16F ? 8 : 4; }

// ---------------------------------------------------------------- holes
// Occupancy of cw x ch cells (Section 5.3: analysing the framebuffer also
// finds holes in the rendered area). A workgroup scans the rows of one cell
// row and a chunk of whole cells about kGridChunkCols columns wide (so each
// cell has one writer). Lane = column: each thread walks its column down the
// cell row, kRoiBatch rows of loads in flight (every wave access one
// coalesced row segment), and ORs whether any of its pixels holds data; a
// thread that saw data sets its cell's byte flag in LDS once, and the flags
// are written out at the end.
constexpr int kGridChunkCells = 1024;   // LDS flags per workgroup
constexpr int kGridChunkCols = 256;     // columns of a chunk (one per thread)

struct GridImg {
  const void* data;
  int64_t pitch;
  int32_t w, h;
  int32_t gw, gh;
  int32_t chunks;        // cell chunks per cell row
  int32_t wg_begin;
  int64_t grid_off;      // byte offset of this image's grid
};

struct GridArgs {
  GridImg im[kRoiMax];
  uint8_t* grid;
  int32_t n;
  int32_t cw, ch;
  int32_t chunk_cells;
};
static_assert(sizeof(GridArgs) <= 4096, "kernel arguments must fit in 4 KiB");

template <int MODE>
__global__ __launch_bounds__(kThreads) void roi_grid_kernel(const GridArgs a) {
  constexpr int bpp = MODE == 2 ? 16 : MODE == 3 ? 8 : 4;
  __shared__ uint8_t flags[kGridChunkCells];
  const int blk = blockIdx.x;
  int s = 0;
  s = segment_of([&](int i) { return a.im[i].wg_begin; }, a.n, blk);
  const GridImg I = a.im[s];
  const int local = blk - I.wg_begin;
  const int band = local / I.chunks, chunk = local - band * I.chunks;
  const int c0 = chunk * a.chunk_cells;                      // first cell of the chunk
  const int ncells = min(a.chunk_cells, I.gw - c0);
  const int x0 = c0 * a.cw, x1 = min(I.w, (c0 + ncells) * a.cw);
  const int y0 = band * a.ch, y1 = min(I.h, y0 + a.ch);
  for (int k = threadIdx.x; k < ncells; k += kThreads) flags[k] = 0;
  __syncthreads();
  const int rows = y1 - y0;
  const int64_t row_bytes = I.pitch * bpp;
  const uint8_t* base = reinterpret_cast<const uint8_t*>(I.data) + (int64_t)y0 * row_bytes;
  for (int x = x0 + (int)threadIdx.x; x < x1; x += kThreads) {
    uint32_t any = 0;
    for (int r0 = 0; r0 < rows; r0 += kRoiBatch) {
      uint32_t m[kRoiBatch];
#pragma unroll
      for (int k = 0; k < kRoiBatch; ++k) {
        // unconditional loads (a row past the band's end reads its first row
        // and is ignored), so that the batch is in flight together
        const int r = r0 + k < rows ? r0 + k : 0;
        m[k] = px_mask<MODE>(base + r * row_bytes, x);
      }
#pragma unroll
      for (int k = 0; k < kRoiBatch; ++k)
        if (r0 + k < rows) any |= m[k];
    }
    if (any) flags[(x - x0) / a.cw] = 1;   // every writer stores the same value
  }
  __syncthreads();
  uint8_t* g = a.grid + I.grid_off + (int64_t)band * I.gw + c0;
  for (int k = threadIdx.x; k < ncells; k += kThreads) g[k] = flags[k];
}

}  // namespace cmp

using namespace cmp;

extern "C" size_t cmp_roi_workspace_size(const cmp_image* imgs, int32_t n) {
  if (n < 0 || (n > 0 && !imgs)) return 0;
  // 16-byte pixels give the most workgroups
  return kRoiTickets + sizeof(int4) * (size_t)roi_workgroups(imgs, n, 16);
}

extern "C" cmp_status cmp_roi_detect(const cmp_image* imgs, int32_t n, cmp_format fmt,
                                     int32_t* roi_out_dev, void* workspace, size_t ws_bytes,
                                     void* stream) {
  CMP_RANGE("cmp_roi_detect");
  CMP_REQUIRE(n >= 0 && n <= kRoiMax, "n = %d must be 0..%d", n, kRoiMax);
  if (n == 0) return CMP_OK;
  CMP_REQUIRE(imgs && roi_out_dev && workspace, "NULL argument");
  CMP_REQUIRE(((uintptr_t)roi_out_dev & 15) == 0 && ((uintptr_t)workspace & 15) == 0,
              "roi_out_dev and workspace must be 16-byte aligned");
  CMP_REQUIRE(fmt == CMP_RGBA8 || fmt == CMP_RGBA32F || fmt == CMP_RGBA16F, "bad format %d", fmt);
  const int bpp = roi_bpp(fmt);
  int mode = fmt == CMP_RGBA32F ? 2 : fmt == CMP_RGBA16F ? 3 : 1;
  if (fmt == CMP_RGBA8) {
    // all images must agree: depth test or colour test
    const bool d0 = imgs[0].depth != nullptr;
    for (int i = 1; i < n; ++i)
      CMP_REQUIRE((imgs[i].depth != nullptr) == d0,
                  "either every image has a depth buffer or none has");
    mode = d0 ? 0 : 1;
  }
  RoiArgs a;
  memset(&a, 0, sizeof a);
  int64_t wg = 0;
  for (int i = 0; i < n; ++i) {
    const cmp_image& I = imgs[i];
    CMP_REQUIRE(rect_valid(I.roi), "imgs[%d] has a negative size", i);
    const bool empty = rect_empty(I.roi);
    if (!empty) {
      CMP_REQUIRE(mode == 0 ? I.depth != nullptr : I.color != nullptr, "imgs[%d]: NULL buffer", i);
      CMP_REQUIRE(I.pitch >= I.roi.w, "imgs[%d].pitch < width", i);
      const uintptr_t p = (uintptr_t)(mode == 0 ? (const void*)I.depth : I.color);
      CMP_REQUIRE(p % (uintptr_t)(bpp < 16 ? bpp : 16) == 0, "imgs[%d]: misaligned buffer", i);
    }
    const int rows = empty ? 1 : roi_rows(I, bpp);
    const int nwg = empty ? 1 : (I.roi.h + rows - 1) / rows;
    a.im[i] = RoiImg{I.color, I.depth, I.pitch, empty ? 0 : I.roi.w, empty ? 0 : I.roi.h,
                     (int32_t)wg, nwg, rows, 0};
    wg += nwg;
  }
  CMP_REQUIRE(wg < (1 << 24), "too many workgroups");
  const size_t need = kRoiTickets + sizeof(int4) * (size_t)wg;
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than %zu", ws_bytes, need);
    return CMP_ENOSPC;
  }
  a.roi_out = roi_out_dev;
  a.ticket = (int32_t*)workspace;
  a.part = (int4*)((char*)workspace + kRoiTickets);
  a.n = n;
  a.mode = mode;
  hipStream_t s = (hipStream_t)stream;
  log_plan("roi detect: %d images, format mode %d, %lld workgroups", n, mode, (long long)wg);
  switch (mode) {
    case 0: hipLaunchKernelGGL(roi_kernel<0>, dim3((unsigned)wg), dim3(kThreads), 0, s, a); break;
    case 1: hipLaunchKernelGGL(roi_kernel<1>, dim3((unsigned)wg), dim3(kThreads), 0, s, a); break;
    case 2: hipLaunchKernelGGL(roi_kernel<2>, dim3((unsigned)wg), dim3(kThreads), 0, s, a); break;
    default: hipLaunchKernelGGL(roi_kernel<3>, dim3((unsigned)wg), dim3(kThreads), 0, s, a); break;
  }
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}

extern "C" cmp_status cmp_roi_grid(const cmp_image* imgs, int32_t n, cmp_format fmt,
                                   int32_t cell_w, int32_t cell_h, uint8_t* grid_dev,
                                   void* stream) {
  CMP_RANGE("cmp_roi_grid");
  CMP_REQUIRE(n >= 0 && n <= kRoiMax, "n = %d must be 0..%d", n, kRoiMax);
  if (n == 0) return CMP_OK;
  CMP_REQUIRE(imgs && grid_dev, "NULL argument");
  CMP_REQUIRE(cell_w >= 1 && cell_h >= 1, "cells must be at least 1x1");
  CMP_REQUIRE(fmt == CMP_RGBA8 || fmt == CMP_RGBA32F || fmt == CMP_RGBA16F, "bad format %d", fmt);
  int mode = fmt == CMP_RGBA32F ? 2 : fmt == CMP_RGBA16F ? 3 : 1;
  if (fmt == CMP_RGBA8) {
    const bool d0 = imgs[0].depth != nullptr;
    for (int i = 1; i < n; ++i)
      CMP_REQUIRE((imgs[i].depth != nullptr) == d0,
                  "either every image has a depth buffer or none has");
    mode = d0 ? 0 : 1;
  }
  const int bpp = roi_bpp(fmt);
  GridArgs a;
  memset(&a, 0, sizeof a);
  a.cw = cell_w;
  a.ch = cell_h;
  // chunks of whole cells about kGridChunkCols columns wide (one column per
  // thread, enough workgroups to fill the device), wider for short cells so
  // that a workgroup still scans about 16K pixels
  const int chunk_cols = std::max(kGridChunkCols, 16384 / cell_h);
  a.chunk_cells = std::min(kGridChunkCells, std::max(1, chunk_cols / cell_w));
  int64_t wg = 0, goff = 0;
  for (int i = 0; i < n; ++i) {
    const cmp_image& I = imgs[i];
    CMP_REQUIRE(rect_valid(I.roi), "imgs[%d] has a negative size", i);
    const bool empty = rect_empty(I.roi);
    const int W = empty ? 0 : I.roi.w, H = empty ? 0 : I.roi.h;
    const void* data = mode == 0 ? (const void*)I.depth : I.color;
    if (!empty) {
      CMP_REQUIRE(data, "imgs[%d]: NULL buffer", i);
      CMP_REQUIRE(I.pitch >= W, "imgs[%d].pitch < width", i);
      CMP_REQUIRE((uintptr_t)data % (uintptr_t)(bpp < 16 ? bpp : 16) == 0,
                  "imgs[%d]: misaligned buffer", i);
    }
    const int gw = (W + cell_w - 1) / cell_w, gh = (H + cell_h - 1) / cell_h;
    const int chunks = (gw + a.chunk_cells - 1) / a.chunk_cells;
    a.im[i] = GridImg{data, I.pitch, W, H, gw, gh, chunks, (int32_t)wg, goff};
    wg += (int64_t)gh * chunks;
    goff += (int64_t)gw * gh;
  }
  CMP_REQUIRE(wg < (1 << 24), "too many workgroups");
  if (wg == 0) return CMP_OK;
  a.grid = grid_dev;
  a.n = n;
  hipStream_t s = (hipStream_t)stream;
  const dim3 grid((unsigned)wg), block(kThreads);
  switch (mode) {
    case 0: hipLaunchKernelGGL(roi_grid_kernel<0>, grid, block, 0, s, a); break;
    case 1: hipLaunchKernelGGL(roi_grid_kernel<1>, grid, block, 0, s, a); break;
    case 2: hipLaunchKernelGGL(roi_grid_kernel<2>, grid, block, 0, s, a); break;
    default: hipLaunchKernelGGL(roi_grid_kernel<3>, grid, block, 0, s, a); break;
  }
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}

namespace cmp {

// --------------------------------------------------------- ROI rectangles
// cmp_roi_rects: the occupied cells of each image's occupancy grid covered
// by disjoint rectangles (Section 5.3: the framebuffer analysis also finds
// the holes of the rendered area), built row by row of cells: a row's
// maximal runs of occupied cells, left to right; a run with the same first
// and last cell as a run of the row above extends that run's rectangle,
// any other run starts a new one; numbered in the order they start. More
// than max_rects rectangles give one, the bounding box of the occupied
// cells.
//
// One wave per image. A grid row is read as 64-bit ballot words (lane j:
// column 64 w + j); its runs are walked with bit scans, uniformly over the
// wave; the run ends of the row above are kept in LDS per start column,
// tagged with their row so that they never need clearing.
constexpr int kRectMaxWords = 64;   // grid rows of at most 64 x 64 cells
constexpr int kRectMax = 64;        // rectangles per image

struct RectArgs {
  const uint8_t* grid;
  int32_t* rects;
  int32_t* count;
  int64_t goff[kRoiMax];   // first cell of each image's grid
  int32_t w[kRoiMax], h[kRoiMax];
  int32_t n, cw, ch, max_rects;
};
static_assert(sizeof(RectArgs) <= 4096, "kernel arguments must fit in 4 KiB");

__global__ __launch_bounds__(kWave) void roi_rects_kernel(const RectArgs a) {
  __shared__ uint64_t row[kRectMaxWords];                 // occupancy of the current row
  __shared__ int32_t end_above[kRectMaxWords * 64];      // run end by start column (row above)
  __shared__ int32_t tag_above[kRectMaxWords * 64];      // the row that entry belongs to
  __shared__ int32_t rect_above[kRectMaxWords * 64];     // its rectangle
  __shared__ int32_t rc[kRectMax][4];                    // c0, r0, c1, r1 (cells)
  const int s = blockIdx.x, lane = threadIdx.x;
  const int W = a.w[s], H = a.h[s];
  const int gw = W > 0 ? (W + a.cw - 1) / a.cw : 0, gh = H > 0 ? (H + a.ch - 1) / a.ch : 0;
  const int nw = (gw + 63) / 64;
  const uint8_t* g = a.grid + a.goff[s];
  for (int i = lane; i < nw * 64; i += kWave) tag_above[i] = -2;
  int n = 0;                                   // rectangles started (uniform)
  int bc0 = gw, br0 = gh, bc1 = 0, br1 = 0;    // bounding box of the occupied cells
  for (int r = 0; r < gh; ++r) {
    // the row's occupancy words: all loads issued, then one ballot per word
    for (int w = 0; w < nw; ++w) {
      const int c = 64 * w + lane;
      const bool occ = c < gw && g[(int64_t)r * gw + c] != 0;
      const uint64_t m = __ballot(occ);
      if (lane == 0) row[w] = m;
    }
    __builtin_amdgcn_wave_barrier();
    // walk the runs (uniform)
    uint64_t prev_top = 0;   // bit 63 of the previous word
    for (int w = 0; w < nw; ++w) {
      const uint64_t m = row[w];
      uint64_t starts = m & ~((m << 1) | prev_top);
      prev_top = m >> 63;
      while (starts) {
        const int c0 = 64 * w + (int)__builtin_ctzll(starts);
        starts &= starts - 1;
        // the run's end: the first empty column at or after c0
        int e = gw;
        for (int w2 = w; w2 < nw; ++w2) {
          uint64_t z = ~row[w2];
          if (w2 == w) z &= ~0ull << (c0 & 63);
          if (z) {
            e = min(gw, 64 * w2 + (int)__builtin_ctzll(z));
            break;
          }
        }
        int k = -1;
        if (tag_above[c0] == r - 1 && end_above[c0] == e) k = rect_above[c0];
        if (k >= 0) {
          if (k < kRectMax && lane == 0) rc[k][3] = r + 1;
        } else {
          k = n++;
          if (k < kRectMax && lane == 0) {
            rc[k][0] = c0; rc[k][1] = r; rc[k][2] = e; rc[k][3] = r + 1;
          }
        }
        bc0 = min(bc0, c0); bc1 = max(bc1, e);
        br0 = min(br0, r); br1 = r + 1;
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) {   // this row's entry, read when the next row is walked
          tag_above[c0] = r;
          end_above[c0] = e;
          rect_above[c0] = k;
        }
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
  __builtin_amdgcn_wave_barrier();
  // out: pixels, clipped; the bounding box when there are too many
  const int out = n > a.max_rects ? 1 : n;
  int32_t* dst = a.rects + (int64_t)s * a.max_rects * 4;
  for (int k = lane; k < a.max_rects; k += kWave) {
    int4 v = int4{0, 0, 0, 0};
    if (k < out) {
      const int c0 = n > a.max_rects ? bc0 : rc[k][0], r0 = n > a.max_rects ? br0 : rc[k][1];
      const int c1 = n > a.max_rects ? bc1 : rc[k][2], r1 = n > a.max_rects ? br1 : rc[k][3];
      const int x0 = c0 * a.cw, y0 = r0 * a.ch;
      v = int4{x0, y0, min(c1 * a.cw, W) - x0, min(r1 * a.ch, H) - y0};
    }
    reinterpret_cast<int4*>(dst)[k] = v;
  }
  if (lane == 0) a.count[s] = out;
}

}  // namespace cmp

extern "C" cmp_status cmp_roi_rects(const cmp_image* imgs, int32_t n, int32_t cell_w,
                                    int32_t cell_h, const uint8_t* grid_dev, int32_t max_rects,
                                    int32_t* rects_dev, int32_t* count_dev, void* stream) {
  CMP_RANGE("cmp_roi_rects");
  using namespace cmp;
  CMP_REQUIRE(n >= 0 && n <= kRoiMax, "n = %d must be 0..%d", n, kRoiMax);
  if (n == 0) return CMP_OK;
  CMP_REQUIRE(imgs && grid_dev && rects_dev && count_dev, "NULL argument");
  CMP_REQUIRE(cell_w >= 1 && cell_h >= 1, "cells must be at least 1x1");
  CMP_REQUIRE(max_rects >= 1 && max_rects <= kRectMax, "max_rects = %d must be 1..%d", max_rects,
              kRectMax);
  CMP_REQUIRE(((uintptr_t)rects_dev & 15) == 0 && ((uintptr_t)count_dev & 3) == 0,
              "rects_dev must be 16-byte and count_dev 4-byte aligned");
  RectArgs a;
  memset(&a, 0, sizeof a);
  int64_t off = 0;
  for (int i = 0; i < n; ++i) {
    CMP_REQUIRE(rect_valid(imgs[i].roi), "imgs[%d] has a negative size", i);
    const int W = rect_empty(imgs[i].roi) ? 0 : imgs[i].roi.w;
    const int H = rect_empty(imgs[i].roi) ? 0 : imgs[i].roi.h;
    const int64_t gw = W ? (W + cell_w - 1) / cell_w : 0, gh = H ? (H + cell_h - 1) / cell_h : 0;
    CMP_REQUIRE(gw <= 64 * kRectMaxWords, "imgs[%d]: %lld cells per row; at most %d", i,
                (long long)gw, 64 * kRectMaxWords);
    a.goff[i] = off;
    a.w[i] = W;
    a.h[i] = H;
    off += gw * gh;
  }
  a.grid = grid_dev;
  a.rects = rects_dev;
  a.count = count_dev;
  a.n = n;
  a.cw = cell_w;
  a.ch = cell_h;
  a.max_rects = max_rects;
  hipLaunchKernelGGL(roi_rects_kernel, dim3((unsigned)n), dim3(kWave), 0, (hipStream_t)stream, a);
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}
