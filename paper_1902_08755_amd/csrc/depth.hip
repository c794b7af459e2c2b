// cmp_composite_depth: plain launch of depth-sorted compositing
// (Section 5.2.1), with the direct-send / binary-swap schedules of
// Section 5.2.2 as tile assignments inside one launch.
#include <string.h>

#include "depth_tile.hpp"

namespace cmp {

constexpr int kDepthPerPass = 48;
static_assert(kDepthPerPass <= kPlaceMax, "placements of a pass are staged in LDS");

struct DepthArgs {
  DepthDesc c[kDepthPerPass];
  Region reg[kMaxRegions];
  const int32_t* roi_dev;
  uint32_t* out_color;
  uint32_t* out_depth;
  int64_t out_pitch;
  int32_t vx, vy;
  int32_t n, nreg;
  int32_t tile_w, tile_h;
  int32_t accumulate;
  int32_t index_base;
  int32_t crop;   // roi_dev crops the placed contributors (else it places them)
};
static_assert(sizeof(DepthArgs) <= 4096, "kernel arguments must fit in 4 KiB");

__device__ __forceinline__ void tile_of_block(const Region* reg, int nreg, int tile_w, int tile_h,
                                              int& x0, int& y0, int& tw, int& th) {
  const int blk = blockIdx.x;
  int r = 0;
  r = segment_of([&](int i) { return reg[i].tile_begin; }, nreg, blk);
  const Region R = reg[r];
  const int local = blk - R.tile_begin;
  const int tiles_x = (R.w + tile_w - 1) / tile_w;
  const int ty = local / tiles_x, tx = local - ty * tiles_x;
  x0 = R.x + tx * tile_w;
  y0 = R.y + ty * tile_h;
  tw = min(tile_w, R.x + R.w - x0);
  th = min(tile_h, R.y + R.h - y0);
}

// Eight waves per SIMD: at the compiler's default the kernel used 106 SGPRs,
// which held it to seven (measured on 16 x 1920x1080 cropped frames:
// 22.85 -> 21.7 us; forcing eight on the over and batch kernels made them
// spill and run slower).
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(8, 8))) void depth_kernel(
    const DepthArgs a) {
  int x0, y0, tw, th;
  tile_of_block(a.reg, a.nreg, a.tile_w, a.tile_h, x0, y0, tw, th);
  const DepthSrc src{a.c, a.roi_dev, a.index_base, a.crop};
  __shared__ DepthRec s_rec[kPlaceMax];
  stage_contributors(src, a.n, s_rec);   // a.n <= kDepthPerPass <= kPlaceMax
  depth_tile(s_rec, a.n, x0, y0, tw, th, a.out_color, a.out_depth, a.out_pitch, a.vx, a.vy,
             a.accumulate != 0);
}

// Host-side validation of one contributor list; shared with the batch planner.
cmp_status validate_depth_inputs(const cmp_image* in, int32_t n) {
  CMP_REQUIRE(n >= 0, "n = %d is negative", n);
  CMP_REQUIRE(n == 0 || in, "in is NULL");
  for (int i = 0; i < n; ++i) {
    const cmp_image& I = in[i];
    CMP_REQUIRE(rect_valid(I.roi), "in[%d].roi has a negative size", i);
    if (rect_empty(I.roi)) continue;
    CMP_REQUIRE(I.color && I.depth, "in[%d]: color and depth are required", i);
    CMP_REQUIRE(I.pitch >= I.roi.w, "in[%d].pitch %lld < roi.w %d", i, (long long)I.pitch,
                I.roi.w);
    CMP_REQUIRE(((uintptr_t)I.color & 3) == 0 && ((uintptr_t)I.depth & 3) == 0,
                "in[%d]: buffers must be 4-byte aligned", i);
  }
  return CMP_OK;
}

}  // namespace cmp

using namespace cmp;

static cmp_status composite_depth_impl(const cmp_image* in, int32_t n, const int32_t* roi_dev,
                                       bool crop, cmp_rect viewport, uint32_t* out_color,
                                       uint32_t* out_depth, int64_t out_pitch,
                                       cmp_schedule sched, cmp_tile tile, void* stream) {
  cmp_status st = validate_depth_inputs(in, n);
  if (st != CMP_OK) return st;
  CMP_REQUIRE(rect_valid(viewport), "viewport has a negative size");
  if (rect_empty(viewport)) return CMP_OK;
  CMP_REQUIRE(out_color, "out_color is NULL");
  CMP_REQUIRE(out_pitch >= viewport.w, "out_pitch %lld < viewport.w %d", (long long)out_pitch,
              viewport.w);
  CMP_REQUIRE(((uintptr_t)out_color & 3) == 0 && ((uintptr_t)out_depth & 3) == 0,
              "outputs must be 4-byte aligned");
  CMP_REQUIRE(n <= kDepthPerPass || out_depth,
              "out_depth is required when n > %d (it carries the result between passes)",
              kDepthPerPass);
  CMP_REQUIRE(((uintptr_t)roi_dev & 15) == 0, "roi_dev must be 16-byte aligned");
  const int tw = tile.w ? tile.w : 64, th = tile.h ? tile.h : 16;
  CMP_REQUIRE(tw > 0 && th > 0 && (int64_t)tw * th <= 65536,
              "tile %dx%d: sizes must be positive, area <= 65536", tw, th);

  DepthArgs a;
  memset(&a, 0, sizeof a);
  int64_t tiles = 0;
  const int nreg = plan_regions(sched, viewport, tw, th, a.reg, &tiles);
  if (nreg < 0) return nreg;
  CMP_REQUIRE(tiles < (1ll << 24), "too many tiles (%lld)", (long long)tiles);
  a.roi_dev = roi_dev;
  a.crop = crop ? 1 : 0;
  a.out_color = out_color;
  a.out_depth = out_depth;
  a.out_pitch = out_pitch;
  a.vx = viewport.x;
  a.vy = viewport.y;
  a.nreg = nreg;
  a.tile_w = tw;
  a.tile_h = th;
  hipStream_t s = (hipStream_t)stream;
  int base = 0;
  do {
    const int cnt = n - base < kDepthPerPass ? n - base : kDepthPerPass;
    for (int i = 0; i < cnt; ++i) {
      const cmp_image& I = in[base + i];
      a.c[i] = DepthDesc{I.depth ? (const uint32_t*)I.color : nullptr, I.depth, I.pitch,
                         I.roi.x, I.roi.y, rect_empty(I.roi) ? 0 : I.roi.w,
                         rect_empty(I.roi) ? 0 : I.roi.h};
    }
    a.n = cnt;
    a.accumulate = base > 0;
    a.index_base = base;
    hipLaunchKernelGGL(depth_kernel, dim3((unsigned)tiles), dim3(kThreads), 0, s, a);
    CMP_CHECK_HIP(hipGetLastError());
    base += cnt;
  } while (base < n);
  return CMP_OK;
}

extern "C" cmp_status cmp_composite_depth(const cmp_image* in, int32_t n, const int32_t* roi_dev,
                                          cmp_rect viewport, uint32_t* out_color,
                                          uint32_t* out_depth, int64_t out_pitch,
                                          cmp_schedule sched, cmp_tile tile, void* stream) {
  CMP_RANGE("cmp_composite_depth");
  return composite_depth_impl(in, n, roi_dev, false, viewport, out_color, out_depth, out_pitch,
                              sched, tile, stream);
}

extern "C" cmp_status cmp_composite_depth_crop(const cmp_image* in, int32_t n,
                                               const int32_t* roi_dev, cmp_rect viewport,
                                               uint32_t* out_color, uint32_t* out_depth,
                                               int64_t out_pitch, cmp_schedule sched,
                                               cmp_tile tile, void* stream) {
  CMP_RANGE("cmp_composite_depth_crop");
  CMP_REQUIRE(roi_dev, "roi_dev is required");
  return composite_depth_impl(in, n, roi_dev, true, viewport, out_color, out_depth, out_pitch,
                              sched, tile, stream);
}
