// Workgroup tile body of ordered "over" compositing, shared by the plain
// launch and the persistent batched launch.
//
// Thesis Section 5.2.1: partial images of convex regions are sorted by depth
// and blended in that order. Per pixel, back to front from transparent black:
//     acc <- L + (1 - L.a) * acc        (FP32 fused multiply-add per channel)
// A layer that does not cover the pixel leaves acc unchanged.
//
// Mapping: one pixel per lane per step, consecutive lanes on consecutive
// pixels of a tile row, so each layer row segment is one coalesced stream of
// 16-byte (RGBA32F) or 8-byte (RGBA16F) loads. Loads of kBatch layers are
// issued before the first of them is blended, so every lane keeps several
// requests in flight; the blend chain itself stays strictly in order.
#pragma once

#include "cmp_internal.hpp"

namespace cmp {

struct OverDesc {
  const void* color;   // RGBA32F or RGBA16F
  int64_t pitch;
  int32_t x, y, w, h;  // placement
};

// A stored pixel before widening: FP16 pixels stay packed in two registers
// until they are blended.
template <int FMT>
struct RawPx { typedef f32x4 type; };
template <>
struct RawPx<CMP_RGBA16F> { typedef f16x4 type; };

template <int FMT>
__device__ __forceinline__ typename RawPx<FMT>::type ld_raw(const void* base, int64_t px) {
  return reinterpret_cast<const typename RawPx<FMT>::type*>(base)[px];
}
__device__ __forceinline__ f32x4 widen(f32x4 v) { return v; }
__device__ __forceinline__ f32x4 widen(f16x4 h) {
  return f32x4{(float)h.x, (float)h.y, (float)h.z, (float)h.w};
}

// Layers whose loads are in flight together: 128 bytes per lane either way.
template <int FMT>
constexpr int over_batch() { return FMT == CMP_RGBA32F ? 8 : 16; }
constexpr int kOverBatch = 8;   // the backward pass (FP32 and FP16 alike)

__device__ __forceinline__ f32x4 over_op(f32x4 front, f32x4 back) {
  const float t = 1.0f - front.w;
  return f32x4{__builtin_fmaf(t, back.x, front.x), __builtin_fmaf(t, back.y, front.y),
               __builtin_fmaf(t, back.z, front.z), __builtin_fmaf(t, back.w, front.w)};
}

__device__ __forceinline__ bool tile_misses(int rx, int ry, int rw, int rh, int x0, int y0,
                                            int tw, int th) {
  return rw <= 0 || rh <= 0 || rx >= x0 + tw || rx + rw <= x0 || ry >= y0 + th || ry + rh <= y0;
}

// Blends layers [j0, j1) of `d` (back-to-front positions) at pixel (X, Y)
// onto acc. The loads of a batch are unconditional, so that no branch
// separates them: a layer that misses the tile (a uniform test) reads from
// `safe` (any readable address, e.g. the output), and a lane outside a
// layer reads the layer's first pixel; both results are discarded.
template <int FMT>
__device__ __forceinline__ f32x4 over_range(const OverDesc* __restrict__ d, int j0, int j1,
                                            int X, int Y, int x0, int y0, int tw, int th,
                                            const void* safe, f32x4 acc) {
  constexpr int B = over_batch<FMT>();
  typedef typename RawPx<FMT>::type Raw;
  for (int jb = j0; jb < j1; jb += B) {
    Raw L[B];
    bool cov[B];
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const int j = min(jb + k, j1 - 1);
      const OverDesc& D = d[j];
      const bool hit = jb + k < j1 && !tile_misses(D.x, D.y, D.w, D.h, x0, y0, tw, th);
      cov[k] = hit && X >= D.x && X < D.x + D.w && Y >= D.y && Y < D.y + D.h;
      const void* base = hit ? D.color : safe;
      L[k] = ld_raw<FMT>(base, cov[k] ? (int64_t)(Y - D.y) * D.pitch + (X - D.x) : 0);
    }
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (cov[k]) acc = over_op(widen(L[k]), acc);
  }
  return acc;
}

// Sequential order (also direct send: same per-pixel chain).
template <int FMT>
__device__ __forceinline__ void over_tile_seq(const OverDesc* __restrict__ d, int n, int x0, int y0,
                                              int tw, int th, float* __restrict__ out,
                                              int64_t out_pitch, int vx, int vy,
                                              bool accumulate) {
  const int np = tw * th;
  for (int p = threadIdx.x; p < np; p += kThreads) {
    const int r = p / tw;
    const int c = p - r * tw;
    const int X = x0 + c, Y = y0 + r;
    f32x4* o = reinterpret_cast<f32x4*>(out) + ((int64_t)(Y - vy) * out_pitch + (X - vx));
    f32x4 acc = accumulate ? *o : f32x4{0.f, 0.f, 0.f, 0.f};
    acc = over_range<FMT>(d, 0, n, X, Y, x0, y0, tw, th, out, acc);
    *o = acc;
  }
}

// Binary-swap merge order (Section 5.2.2): `groups` (a power of two, <= 64)
// contiguous groups of the back-to-front list, group g = positions
// [gb[g], gb[g+1]), each composited alone, then merged pairwise level by
// level: merge(back, front) = front + (1 - front.a) * back. The pending
// partial of each level is kept in LDS (a binary counter over the groups).
constexpr int kTreeLevels = 7;

template <int FMT>
__device__ __forceinline__ void over_tile_tree(const OverDesc* __restrict__ d,
                                               const uint8_t* __restrict__ gb, int groups, int x0,
                                               int y0, int tw, int th, float* __restrict__ out,
                                               int64_t out_pitch, int vx, int vy) {
  __shared__ f32x4 lvl[kTreeLevels][kThreads];
  const int np = tw * th;
  int levels = 0;
  while ((1 << levels) < groups) ++levels;
  for (int p = threadIdx.x; p < np; p += kThreads) {
    const int r = p / tw;
    const int c = p - r * tw;
    const int X = x0 + c, Y = y0 + r;
    for (int g = 0; g < groups; ++g) {
      f32x4 carry = over_range<FMT>(d, gb[g], gb[g + 1], X, Y, x0, y0, tw, th, out,
                                    f32x4{0.f, 0.f, 0.f, 0.f});
      int l = 0;
      for (; (g >> l) & 1; ++l) carry = over_op(carry, lvl[l][threadIdx.x]);
      lvl[l][threadIdx.x] = carry;
    }
    f32x4* o = reinterpret_cast<f32x4*>(out) + ((int64_t)(Y - vy) * out_pitch + (X - vx));
    *o = lvl[levels][threadIdx.x];
  }
}

}  // namespace cmp
