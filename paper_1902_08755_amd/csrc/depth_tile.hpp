// Workgroup tile body of depth-sorted compositing, shared by the plain launch
// and the persistent batched launch.
//
// Thesis Section 5.2.1 (Spatial and Depth-Sorted Sort-Last Compositing): a
// final pixel takes the colour of the source with the front-most depth. Here:
// the smallest (depth, index) pair over the contributors covering the pixel;
// the clear depth never wins.
//
// Mapping: lane = column. A wave covers 64 consecutive pixels of a tile row
// and steps over 4 rows at a time (the four waves of a workgroup take
// interleaved row groups), so every load of a contributor row is one
// coalesced 256-byte access per wave, and a contributor's left or right edge
// is only a per-lane mask. Per contributor only the depth is read; the
// colour is gathered once, from the winner, at the end ("lean" traffic: 4
// bytes per covering contributor plus 4 for the winner). Contributors are
// visited in index order with a strict "<", so ties keep the lower index.
// The loads of four contributors x four rows are issued before any compare.
#pragma once

#include "cmp_internal.hpp"

namespace cmp {

struct DepthDesc {
  const uint32_t* color;
  const uint32_t* depth;
  int64_t pitch;
  int32_t x, y, w, h;   // placement (host rectangle; bounds the buffer)
};

// Source of contributor descriptors; `roi_dev` may override placements.
struct DepthSrc {
  const DepthDesc* d;
  const int32_t* roi_dev;   // device int32[n][4] or nullptr
  int index_base;           // row of roi_dev that corresponds to d[0]
};

// Composites the tile [x0, x0+tw) x [y0, y0+th) (destination pixels) of a
// viewport whose origin is (vx, vy) into out_color/out_depth. With
// `accumulate`, the outputs already hold the result of earlier contributors
// (a previous pass) and are combined under the same rule.
constexpr int kDepthRows = 4;    // rows per lane per step
constexpr int kDepthBatch = 4;   // contributors whose loads are in flight together

__device__ __forceinline__ void depth_tile(const DepthSrc src, int n, int x0, int y0, int tw,
                                           int th, uint32_t* __restrict__ out_color,
                                           uint32_t* __restrict__ out_depth, int64_t out_pitch,
                                           int vx, int vy, bool accumulate) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  constexpr int kStepRows = kDepthRows * (kThreads / kWave);
  for (int cx = 0; cx < tw; cx += kWave) {
    const int X = x0 + cx + lane;
    const bool col_ok = cx + lane < tw;
    for (int r0 = wave * kDepthRows; r0 < th; r0 += kStepRows) {
      const int Y0 = y0 + r0;                       // rows Y0 .. Y0 + 3 (uniform)
      const int nrows = min(kDepthRows, th - r0);
      uint32_t bd[kDepthRows], pc[kDepthRows];
      const uint32_t* bc[kDepthRows];
#pragma unroll
      for (int k = 0; k < kDepthRows; ++k) {
        bd[k] = kClearDepth;
        pc[k] = 0;
        bc[k] = nullptr;
        if (accumulate && col_ok && k < nrows) {
          const int64_t oo = (int64_t)(Y0 + k - vy) * out_pitch + (X - vx);
          bd[k] = out_depth[oo];
          pc[k] = out_color[oo];
        }
      }
      for (int i0 = 0; i0 < n; i0 += kDepthBatch) {
        uint32_t dv[kDepthBatch][kDepthRows];
        const uint32_t* crow[kDepthBatch];   // colour of this lane's pixel in row Y0 - ry
        int64_t cpitch[kDepthBatch];
#pragma unroll
        for (int j = 0; j < kDepthBatch; ++j) {
#pragma unroll
          for (int k = 0; k < kDepthRows; ++k) dv[j][k] = kClearDepth;
          crow[j] = nullptr;
          cpitch[j] = 0;
          const int i = i0 + j;
          if (i >= n) continue;
          const DepthDesc& D = src.d[i];
          int32_t rx, ry, rw, rh;
          placement(src.roi_dev, src.index_base + i, D.x, D.y, D.w, D.h, rx, ry, rw, rh);
          // whole-step rejection (uniform): columns of the tile, rows of the step
          if (rw <= 0 || rh <= 0 || rx >= x0 + tw || rx + rw <= x0 || ry >= Y0 + nrows ||
              ry + rh <= Y0)
            continue;
          const bool in_col = col_ok && X >= rx && X < rx + rw;
          const int64_t off0 = (int64_t)(Y0 - ry) * D.pitch + (X - rx);
          crow[j] = D.color + off0;
          cpitch[j] = D.pitch;
#pragma unroll
          for (int k = 0; k < kDepthRows; ++k) {
            const int yy = Y0 + k - ry;           // uniform
            if (k < nrows && yy >= 0 && yy < rh && in_col)
              dv[j][k] = D.depth[off0 + (int64_t)k * D.pitch];
          }
        }
#pragma unroll
        for (int j = 0; j < kDepthBatch; ++j) {
#pragma unroll
          for (int k = 0; k < kDepthRows; ++k) {
            if (dv[j][k] < bd[k]) {
              bd[k] = dv[j][k];
              bc[k] = crow[j] + (int64_t)k * cpitch[j];
            }
          }
        }
      }
      // gather the winners' colours and store (4-byte accesses, coalesced
      // along the row across the wave)
      if (col_ok) {
#pragma unroll
        for (int k = 0; k < kDepthRows; ++k) {
          if (k >= nrows) continue;
          const int64_t oo = (int64_t)(Y0 + k - vy) * out_pitch + (X - vx);
          out_color[oo] = bc[k] ? *bc[k] : pc[k];
          if (out_depth) out_depth[oo] = bd[k];
        }
      }
    }
  }
}

}  // namespace cmp
