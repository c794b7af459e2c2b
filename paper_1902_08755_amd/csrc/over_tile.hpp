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
  typedef const __attribute__((address_space(1))) typename RawPx<FMT>::type* GPtr;
  // non-temporal: each layer pixel is read once (measured faster than the
  // default policy for this kernel and the backward pass)
  return __builtin_nontemporal_load(&((GPtr)base)[px]);
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

// Copies the descriptors of layers [0, n) (n <= 64) to LDS: a tile reads a
// layer's placement and buffer from there (uniform LDS reads), not from the
// kernel arguments or the batch workspace. All threads; ends with a barrier.
constexpr int kOverStage = 64;
__device__ __forceinline__ void stage_layers(const OverDesc* __restrict__ src, int n,
                                             OverDesc* s_d) {
  for (int i = threadIdx.x; i < n; i += kThreads) s_d[i] = src[i];
  __syncthreads();
}

// Layers [c0, c1) (c1 - c0 <= 64) that reach the tile, as a bit mask
// (bit i: layer c0 + i). Uniform.
__device__ __forceinline__ uint64_t tile_hits(const OverDesc* __restrict__ d, int c0, int c1,
                                              int x0, int y0, int tw, int th) {
  uint64_t m = 0;
  for (int j = c0; j < c1; ++j) {
    const OverDesc& D = d[j];
    if (!tile_misses(uniform(D.x), uniform(D.y), uniform(D.w), uniform(D.h), x0, y0, tw, th))
      m |= 1ull << (j - c0);
  }
  return (uint64_t)uniform64((int64_t)m);
}

// tile_hits by one ballot: lane i tests layer c0 + i (c1 - c0 <= 64). Every
// lane of the wave must be active (a lane outside the wave's work casts no
// vote): callers take it before their per-pixel loops.
__device__ __forceinline__ uint64_t tile_hits_wave(const OverDesc* __restrict__ d, int c0, int c1,
                                                   int x0, int y0, int tw, int th) {
  const int j = c0 + (int)(threadIdx.x % kWave);
  bool hit = false;
  if (j < c1) {
    const OverDesc& D = d[j];
    hit = !tile_misses(D.x, D.y, D.w, D.h, x0, y0, tw, th);
  }
  return (uint64_t)__ballot(hit);
}

// Blends, in increasing order, the layers base + i for the set bits i of
// `hits` (layers that reach the tile) at pixel (X, Y) onto acc. A batch's
// loads are unconditional, so that no branch separates them: a slot past
// the last layer repeats the batch's first layer, and a lane outside a
// layer reads the layer's first pixel; both results are discarded.
template <int FMT>
__device__ __forceinline__ f32x4 over_hits(const OverDesc* __restrict__ d, int base,
                                           uint64_t hits, int X, int Y, f32x4 acc) {
  constexpr int B = over_batch<FMT>();
  typedef typename RawPx<FMT>::type Raw;
  while (hits) {   // uniform
    Raw L[B];
    bool cov[B];
    const int first = (int)__builtin_ctzll(hits);
#pragma unroll
    for (int k = 0; k < B; ++k) {
      const bool has = hits != 0;
      const OverDesc& D = d[base + (has ? (int)__builtin_ctzll(hits) : first)];
      hits &= hits - 1;
      const int dx = uniform(D.x), dy = uniform(D.y), dw = uniform(D.w), dh = uniform(D.h);
      const void* color = uniform_ptr(D.color);
      const int64_t pitch = uniform64(D.pitch);
      cov[k] = has && X >= dx && X < dx + dw && Y >= dy && Y < dy + dh;
      L[k] = ld_raw<FMT>(color, cov[k] ? (int64_t)(Y - dy) * pitch + (X - dx) : 0);
    }
#pragma unroll
    for (int k = 0; k < B; ++k)
      if (cov[k]) acc = over_op(widen(L[k]), acc);
  }
  return acc;
}

// Layers [j0, j1) at pixel (X, Y) onto acc, 64 at a time.
template <int FMT>
__device__ __forceinline__ f32x4 over_range(const OverDesc* __restrict__ d, int j0, int j1,
                                            int X, int Y, int x0, int y0, int tw, int th,
                                            f32x4 acc) {
  for (int c0 = j0; c0 < j1; c0 += 64)
    acc = over_hits<FMT>(d, c0, tile_hits(d, c0, min(j1, c0 + 64), x0, y0, tw, th), X, Y, acc);
  return acc;
}

// Sequential order (also direct send: same per-pixel chain).
template <int FMT>
__device__ __forceinline__ void over_tile_seq(const OverDesc* __restrict__ d, int n, int x0, int y0,
                                              int tw, int th, float* __restrict__ out,
                                              int64_t out_pitch, int vx, int vy,
                                              bool accumulate) {
  const int np = tw * th;
  // the layers that reach the tile, found once for all its pixels (n <= 64)
  const uint64_t hits = n <= 64 ? tile_hits_wave(d, 0, n, x0, y0, tw, th) : 0;
  for (int p = threadIdx.x; p < np; p += kThreads) {
    const int r = p / tw;
    const int c = p - r * tw;
    const int X = x0 + c, Y = y0 + r;
    f32x4* o = reinterpret_cast<f32x4*>(out) + ((int64_t)(Y - vy) * out_pitch + (X - vx));
    f32x4 acc = accumulate ? *o : f32x4{0.f, 0.f, 0.f, 0.f};
    acc = n <= 64 ? over_hits<FMT>(d, 0, hits, X, Y, acc)
                  : over_range<FMT>(d, 0, n, X, Y, x0, y0, tw, th, acc);
    __builtin_nontemporal_store(acc, o);
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
  // n <= 64 layers in all (one pass): the tile's layers found once
  const uint64_t hits = tile_hits_wave(d, 0, gb[groups], x0, y0, tw, th);
  for (int p = threadIdx.x; p < np; p += kThreads) {
    const int r = p / tw;
    const int c = p - r * tw;
    const int X = x0 + c, Y = y0 + r;
    for (int g = 0; g < groups; ++g) {
      const int j0 = gb[g], j1 = gb[g + 1];
      const uint64_t span = (j1 - j0 >= 64 ? ~0ull : ((1ull << (j1 - j0)) - 1ull)) << j0;
      f32x4 carry = over_hits<FMT>(d, 0, hits & span, X, Y, f32x4{0.f, 0.f, 0.f, 0.f});
      int l = 0;
      for (; (g >> l) & 1; ++l) carry = over_op(carry, lvl[l][threadIdx.x]);
      lvl[l][threadIdx.x] = carry;
    }
    f32x4* o = reinterpret_cast<f32x4*>(out) + ((int64_t)(Y - vy) * out_pitch + (X - vx));
    __builtin_nontemporal_store(lvl[levels][threadIdx.x], o);
  }
}

}  // namespace cmp
