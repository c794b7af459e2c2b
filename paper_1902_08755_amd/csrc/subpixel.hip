// Subpixel and pixel compounds: the two compositing steps that the
// decomposition modes of Section 4.2.2 (Pixel) and Section 4.2.3 (Subpixel)
// need on the destination.
//
// cmp_composite_average: accumulate and average the samples of every pixel
// (subpixel compounds). Integer sums, so every schedule and tile gives the
// same bits. Mapping as in depth compositing: lane = column, four rows per
// step, the loads of four sources x four rows in flight; the four 8-bit
// channels are summed in two registers as 16-bit pairs (n <= 64 keeps every
// pair below 2^16).
//
// cmp_assemble_pixels: put the interleaved pixels of pixel-compound sources
// back in place. Each destination pixel looks up the source of its offset
// class (a table in LDS) and gathers its value; stores are coalesced along
// the row.
#include <string.h>

#include "cmp_internal.hpp"

namespace cmp {

constexpr int kAvgMax = 64;

struct AvgDesc {
  const uint32_t* color;
  int64_t pitch;
  int32_t x, y, w, h;
};

struct AvgArgs {
  AvgDesc c[kAvgMax];
  Region reg[kMaxRegions];
  uint32_t* out;
  int64_t out_pitch;
  int32_t vx, vy;
  int32_t n, nreg;
  int32_t tile_w, tile_h;
  float rcp_n;
};
static_assert(sizeof(AvgArgs) <= 4096, "kernel arguments must fit in 4 KiB");

// floor(t / n) for t < 2^24: a float estimate corrected by one step.
__device__ __forceinline__ uint32_t div_small(uint32_t t, uint32_t n, float rcp) {
  uint32_t q = (uint32_t)((float)t * rcp);
  if ((q + 1) * n <= t) ++q;
  else if (q * n > t) --q;
  return q;
}

__global__ __launch_bounds__(kThreads) void average_kernel(const AvgArgs a) {
  // region and tile of this workgroup
  const int blk = blockIdx.x;
  int r = 0;
  r = segment_of([&](int i) { return a.reg[i].tile_begin; }, a.nreg, blk);
  const Region R = a.reg[r];
  const int local = blk - R.tile_begin;
  const int tiles_x = (R.w + a.tile_w - 1) / a.tile_w;
  const int ty = local / tiles_x, tx = local - ty * tiles_x;
  const int x0 = R.x + tx * a.tile_w, y0 = R.y + ty * a.tile_h;
  const int tw = min(a.tile_w, R.x + R.w - x0), th = min(a.tile_h, R.y + R.h - y0);

  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  constexpr int kRows = 4, kBatch = 4;
  constexpr int kStepRows = kRows * (kThreads / kWave);
  const uint32_t n = (uint32_t)a.n, half = n / 2;
  for (int cx = 0; cx < tw; cx += kWave) {
    const int X = x0 + cx + lane;
    const bool col_ok = cx + lane < tw;
    for (int r0 = wave * kRows; r0 < th; r0 += kStepRows) {
      const int Y0 = y0 + r0;
      const int nrows = min(kRows, th - r0);
      uint32_t s02[kRows], s13[kRows];   // channels 0,2 and 1,3 as 16-bit pairs
#pragma unroll
      for (int k = 0; k < kRows; ++k) s02[k] = s13[k] = 0;
      for (int i0 = 0; i0 < a.n; i0 += kBatch) {
        uint32_t v[kBatch][kRows];
#pragma unroll
        for (int j = 0; j < kBatch; ++j) {
#pragma unroll
          for (int k = 0; k < kRows; ++k) v[j][k] = 0;
          const int i = i0 + j;
          if (i >= a.n) continue;
          const AvgDesc& D = a.c[i];
          if (D.w <= 0 || D.h <= 0 || D.x >= x0 + tw || D.x + D.w <= x0 || D.y >= Y0 + nrows ||
              D.y + D.h <= Y0)
            continue;
          const bool in_col = col_ok && X >= D.x && X < D.x + D.w;
          const int64_t off0 = (int64_t)(Y0 - D.y) * D.pitch + (X - D.x);
#pragma unroll
          for (int k = 0; k < kRows; ++k) {
            const int yy = Y0 + k - D.y;
            if (k < nrows && yy >= 0 && yy < D.h && in_col) v[j][k] = D.color[off0 + (int64_t)k * D.pitch];
          }
        }
#pragma unroll
        for (int j = 0; j < kBatch; ++j)
#pragma unroll
          for (int k = 0; k < kRows; ++k) {
            s02[k] += v[j][k] & 0x00FF00FFu;
            s13[k] += (v[j][k] >> 8) & 0x00FF00FFu;
          }
      }
      if (!col_ok) continue;
#pragma unroll
      for (int k = 0; k < kRows; ++k) {
        if (k >= nrows) continue;
        uint32_t res = 0;
        if (n > 0) {
          res = div_small((s02[k] & 0xFFFFu) + half, n, a.rcp_n) |
                (div_small((s13[k] & 0xFFFFu) + half, n, a.rcp_n) << 8) |
                (div_small((s02[k] >> 16) + half, n, a.rcp_n) << 16) |
                (div_small((s13[k] >> 16) + half, n, a.rcp_n) << 24);
        }
        a.out[(int64_t)(Y0 + k - a.vy) * a.out_pitch + (X - a.vx)] = res;
      }
    }
  }
}

// ------------------------------------------------------------ pixel compounds
constexpr int kAsmMax = 64;

struct AsmSrc {
  const uint32_t* color;
  int64_t pitch;
};

struct AsmArgs {
  AsmSrc src[kAsmMax];
  int8_t cls[kAsmMax];   // offset class (ox + kx oy) -> source, -1 for none
  uint32_t* out;
  int64_t out_pitch;
  int32_t vx, vy, vw, vh;
  int32_t kx, ky, n;
  int32_t tiles_x;
};
static_assert(sizeof(AsmArgs) <= 4096, "kernel arguments must fit in 4 KiB");

constexpr int kAsmTileW = 64, kAsmTileH = 16;

__global__ __launch_bounds__(kThreads) void assemble_kernel(const AsmArgs a) {
  __shared__ AsmSrc s_src[kAsmMax];
  __shared__ int s_cls[kAsmMax];
  if (threadIdx.x < kAsmMax) {
    if (threadIdx.x < a.n) s_src[threadIdx.x] = a.src[threadIdx.x];
    s_cls[threadIdx.x] = a.cls[threadIdx.x];
  }
  __syncthreads();
  const int ty = blockIdx.x / a.tiles_x, tx = blockIdx.x - ty * a.tiles_x;
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  const int u = tx * kAsmTileW + lane;              // viewport-relative column
  if (u >= a.vw) return;
  const int cu = u % a.kx, su = u / a.kx;
  for (int rr = wave; rr < kAsmTileH; rr += kThreads / kWave) {
    const int v = ty * kAsmTileH + rr;
    if (v >= a.vh) break;
    const int s = s_cls[cu + a.kx * (v % a.ky)];
    uint32_t val = 0;
    if (s >= 0) val = s_src[s].color[(int64_t)(v / a.ky) * s_src[s].pitch + su];
    a.out[(int64_t)v * a.out_pitch + u] = val;
  }
}

}  // namespace cmp

using namespace cmp;

extern "C" cmp_status cmp_composite_average(const cmp_image* in, int32_t n, cmp_rect viewport,
                                            uint32_t* out, int64_t out_pitch, cmp_schedule sched,
                                            cmp_tile tile, void* stream) {
  CMP_RANGE("cmp_composite_average");
  CMP_REQUIRE(n >= 0 && n <= kAvgMax, "n = %d must be 0..%d", n, kAvgMax);
  CMP_REQUIRE(n == 0 || in, "in is NULL");
  for (int i = 0; i < n; ++i) {
    const cmp_image& I = in[i];
    CMP_REQUIRE(rect_valid(I.roi), "in[%d].roi has a negative size", i);
    if (rect_empty(I.roi)) continue;
    CMP_REQUIRE(I.color && ((uintptr_t)I.color & 3) == 0, "in[%d].color: NULL or misaligned", i);
    CMP_REQUIRE(I.pitch >= I.roi.w, "in[%d].pitch < roi.w", i);
  }
  CMP_REQUIRE(rect_valid(viewport), "viewport has a negative size");
  if (rect_empty(viewport)) return CMP_OK;
  CMP_REQUIRE(out && ((uintptr_t)out & 3) == 0, "out: NULL or misaligned");
  CMP_REQUIRE(out_pitch >= viewport.w, "out_pitch < viewport.w");
  const int tw = tile.w ? tile.w : 64, th = tile.h ? tile.h : 16;
  CMP_REQUIRE(tw > 0 && th > 0 && (int64_t)tw * th <= 65536, "bad tile %dx%d", tw, th);
  AvgArgs a;
  memset(&a, 0, sizeof a);
  int64_t tiles = 0;
  const int nreg = plan_regions(sched, viewport, tw, th, a.reg, &tiles);
  if (nreg < 0) return nreg;
  CMP_REQUIRE(tiles < (1ll << 24), "too many tiles");
  for (int i = 0; i < n; ++i) {
    const cmp_image& I = in[i];
    const bool e = rect_empty(I.roi);
    a.c[i] = AvgDesc{(const uint32_t*)I.color, I.pitch, I.roi.x, I.roi.y, e ? 0 : I.roi.w,
                     e ? 0 : I.roi.h};
  }
  a.out = out;
  a.out_pitch = out_pitch;
  a.vx = viewport.x;
  a.vy = viewport.y;
  a.n = n;
  a.nreg = nreg;
  a.tile_w = tw;
  a.tile_h = th;
  a.rcp_n = n > 0 ? 1.0f / (float)n : 0.f;
  hipLaunchKernelGGL(average_kernel, dim3((unsigned)tiles), dim3(kThreads), 0,
                     (hipStream_t)stream, a);
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}

extern "C" cmp_status cmp_assemble_pixels(const cmp_image* in, int32_t n, const int32_t* offsets,
                                          int32_t kx, int32_t ky, cmp_rect viewport,
                                          uint32_t* out, int64_t out_pitch, void* stream) {
  CMP_RANGE("cmp_assemble_pixels");
  CMP_REQUIRE(n >= 0 && n <= kAsmMax, "n = %d must be 0..%d", n, kAsmMax);
  CMP_REQUIRE(kx >= 1 && ky >= 1 && kx * ky <= kAsmMax, "pixel kernel %dx%d: 1..64 classes", kx,
              ky);
  CMP_REQUIRE(n == 0 || (in && offsets), "in or offsets is NULL");
  CMP_REQUIRE(rect_valid(viewport), "viewport has a negative size");
  if (rect_empty(viewport)) return CMP_OK;
  CMP_REQUIRE(out && ((uintptr_t)out & 3) == 0, "out: NULL or misaligned");
  CMP_REQUIRE(out_pitch >= viewport.w, "out_pitch < viewport.w");
  AsmArgs a;
  memset(&a, 0, sizeof a);
  for (int c = 0; c < kAsmMax; ++c) a.cls[c] = -1;
  for (int i = 0; i < n; ++i) {
    const int ox = offsets[2 * i], oy = offsets[2 * i + 1];
    CMP_REQUIRE(ox >= 0 && ox < kx && oy >= 0 && oy < ky, "offsets[%d] = (%d, %d) outside the kernel",
                i, ox, oy);
    const cmp_image& I = in[i];
    // the source must hold every pixel of its class
    const int need_w = viewport.w > ox ? (viewport.w - ox + kx - 1) / kx : 0;
    const int need_h = viewport.h > oy ? (viewport.h - oy + ky - 1) / ky : 0;
    CMP_REQUIRE(I.roi.w >= need_w && I.roi.h >= need_h,
                "in[%d] is %dx%d, its class needs %dx%d", i, I.roi.w, I.roi.h, need_w, need_h);
    if (need_w > 0 && need_h > 0) {
      CMP_REQUIRE(I.color && ((uintptr_t)I.color & 3) == 0, "in[%d].color: NULL or misaligned", i);
      CMP_REQUIRE(I.pitch >= need_w, "in[%d].pitch too small", i);
    }
    a.src[i] = AsmSrc{(const uint32_t*)I.color, I.pitch};
    if (a.cls[ox + kx * oy] < 0) a.cls[ox + kx * oy] = (int8_t)i;
  }
  a.out = out;
  a.out_pitch = out_pitch;
  a.vx = viewport.x;
  a.vy = viewport.y;
  a.vw = viewport.w;
  a.vh = viewport.h;
  a.kx = kx;
  a.ky = ky;
  a.n = n;
  a.tiles_x = (viewport.w + kAsmTileW - 1) / kAsmTileW;
  const int64_t tiles = (int64_t)a.tiles_x * ((viewport.h + kAsmTileH - 1) / kAsmTileH);
  CMP_REQUIRE(tiles < (1ll << 24), "too many tiles");
  hipLaunchKernelGGL(assemble_kernel, dim3((unsigned)tiles), dim3(kThreads), 0, (hipStream_t)stream,
                     a);
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}
