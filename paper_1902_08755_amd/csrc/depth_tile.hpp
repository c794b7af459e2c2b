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

// Source of contributor descriptors; `roi_dev` may override placements
// (crop == 0) or crop the contributors to the rectangles that hold their
// data (crop == 1: the buffers stay where the descriptors place them).
struct DepthSrc {
  const DepthDesc* d;
  const int32_t* roi_dev;   // device int32[n][4] or nullptr
  int index_base;           // row of roi_dev that corresponds to d[0]
  int crop;
};

// Composites the tile [x0, x0+tw) x [y0, y0+th) (destination pixels) of a
// viewport whose origin is (vx, vy) into out_color/out_depth. With
// `accumulate`, the outputs already hold the result of earlier contributors
// (a previous pass) and are combined under the same rule.
constexpr int kDepthRows = 4;    // rows per lane per step
constexpr int kDepthBatch = 4;   // covering contributors whose loads are in flight together
constexpr int kPlaceMax = 64;    // contributors staged in LDS per call

typedef const __attribute__((address_space(1))) uint32_t* GlobalU32;

// A contributor as the tile reads it: placement and buffers.
struct DepthRec {
  int32_t x, y, w, h;
  const uint32_t* depth;
  const uint32_t* color;
  int64_t pitch;
};

// Stages contributors [0, n) (n <= kPlaceMax) in LDS: their placements (the
// host rectangle or the device ROI, clamped to the host size) and buffers.
// All threads of the workgroup; ends with a barrier.
__device__ __forceinline__ void stage_contributors(const DepthSrc& src, int n, DepthRec* rec) {
  for (int i = threadIdx.x; i < n; i += kThreads) {
    const DepthDesc& D = src.d[i];
    DepthRec r{D.x, D.y, D.w, D.h, D.depth, D.color, D.pitch};
    if (src.roi_dev && src.crop) {
      // the part of the placed buffer inside the device rectangle
      const int4 q = reinterpret_cast<const int4*>(src.roi_dev)[src.index_base + i];
      const int x0 = max(q.x, D.x), y0 = max(q.y, D.y);
      const int x1 = min(q.x + max(q.z, 0), D.x + D.w), y1 = min(q.y + max(q.w, 0), D.y + D.h);
      r.x = x0;
      r.y = y0;
      r.w = max(0, x1 - x0);
      r.h = max(0, y1 - y0);
      if (r.w > 0 && r.h > 0) {
        const int64_t o = (int64_t)(y0 - D.y) * D.pitch + (x0 - D.x);
        r.depth = D.depth + o;
        r.color = D.color + o;
      }
    } else if (src.roi_dev) {
      const int4 q = reinterpret_cast<const int4*>(src.roi_dev)[src.index_base + i];
      r.x = q.x;
      r.y = q.y;
      r.w = max(0, min(q.z, D.w));
      r.h = max(0, min(q.w, D.h));
    }
    if (!D.depth || r.w <= 0 || r.h <= 0) r.w = r.h = 0;
    rec[i] = r;
  }
  __syncthreads();
}

// `rec`: contributors staged by stage_contributors (n <= kPlaceMax).
// Per step a wave first finds which contributors cover its rows and the
// tile's columns: lane i tests contributor i and one ballot gives the 64-bit
// mask (a loop over the contributors with uniform compares took a quarter of
// the kernel's vector instructions). It then loads kDepthBatch covering
// contributors x 4 rows at a time, so the depth loads of a typical step are
// one round trip; the winner's colour is gathered at the end.
__device__ __forceinline__ void depth_tile(const DepthRec* rec, int n, int x0, int y0, int tw,
                                           int th, uint32_t* __restrict__ out_color,
                                           uint32_t* __restrict__ out_depth, int64_t out_pitch,
                                           int vx, int vy, bool accumulate) {
  const int lane = threadIdx.x % kWave, wave = threadIdx.x / kWave;
  constexpr int kStepRows = kDepthRows * (kThreads / kWave);
  for (int cx = 0; cx < tw; cx += kWave) {
    const int X = x0 + cx + lane;
    const bool col_ok = cx + lane < tw;
    const int cx0 = x0 + cx, cx1 = x0 + min(tw, cx + kWave);   // the wave's columns
    for (int r0 = wave * kDepthRows; r0 < th; r0 += kStepRows) {
      const int Y0 = y0 + r0;                       // rows Y0 .. Y0 + 3 (uniform)
      const int nrows = min(kDepthRows, th - r0);
      // covering contributors of this step: lane i tests contributor i
      // (n <= 64), one ballot gives the mask (bit i: contributor i). Every
      // lane of the wave is active here: the loops above are uniform over
      // the wave and callers run depth_tile with the whole workgroup.
      bool covers_i = false;
      if (lane < n) {
        const DepthRec& R = rec[lane];
        covers_i = R.w > 0 && R.x < cx1 && R.x + R.w > cx0 && R.y < Y0 + nrows && R.y + R.h > Y0;
      }
      uint64_t cover = (uint64_t)__ballot(covers_i);
      uint32_t bd[kDepthRows], pc[kDepthRows];
      int bi[kDepthRows];
#pragma unroll
      for (int k = 0; k < kDepthRows; ++k) {
        bd[k] = kClearDepth;
        pc[k] = 0;
        bi[k] = -1;
        if (accumulate && col_ok && k < nrows) {
          const int64_t oo = (int64_t)(Y0 + k - vy) * out_pitch + (X - vx);
          bd[k] = out_depth[oo];
          pc[k] = out_color[oo];
        }
      }
      while (cover) {   // uniform
        // the next kDepthBatch covering contributors (a slot past the last
        // one repeats the first and is ignored), then every load of the
        // batch, then the compares: no branch between the loads
        int ids[kDepthBatch];
        bool has[kDepthBatch];
        const int first = (int)__builtin_ctzll(cover);
#pragma unroll
        for (int j = 0; j < kDepthBatch; ++j) {
          has[j] = cover != 0;
          ids[j] = has[j] ? (int)__builtin_ctzll(cover) : first;
          cover &= cover - 1;
        }
        uint32_t dv[kDepthBatch][kDepthRows];
        bool ok[kDepthBatch][kDepthRows];
#pragma unroll
        for (int j = 0; j < kDepthBatch; ++j) {
          const int i = ids[j];
          // the column test is per lane anyway: x and w stay in vector registers
          const int rx = rec[i].x, ry = uniform(rec[i].y);
          const int rw = rec[i].w, rh = uniform(rec[i].h);
          // global (not flat) loads: flat ones would also hold up the LDS counter
          const GlobalU32 dep = (GlobalU32)uniform_ptr(rec[i].depth);
          const int64_t pitch = uniform64(rec[i].pitch);
          const bool in_col = has[j] && col_ok && X >= rx && X < rx + rw;
          const int lo = in_col ? X - rx : 0;   // this lane's column in the contributor
          // a uniform row offset (one multiply per contributor, then one
          // pitch per row) plus the lane's column; a pixel outside the
          // contributor reads the first pixel of a valid row instead
          const int yy0 = Y0 - ry;               // uniform
          int64_t roff = (int64_t)yy0 * pitch;
#pragma unroll
          for (int k = 0; k < kDepthRows; ++k) {
            const int yy = yy0 + k;
            const bool rok = k < nrows && yy >= 0 && yy < rh;
            dv[j][k] = dep[(rok ? roff : 0) + lo];
            ok[j][k] = rok && in_col;
            roff += pitch;
          }
        }
        // ascending indices and a strict "<": ties keep the lower index
#pragma unroll
        for (int j = 0; j < kDepthBatch; ++j) {
#pragma unroll
          for (int k = 0; k < kDepthRows; ++k) {
            if (ok[j][k] && dv[j][k] < bd[k]) {
              bd[k] = dv[j][k];
              bi[k] = ids[j];
            }
          }
        }
      }
      // gather the winners' colours and store (4-byte accesses, coalesced
      // along the row across the wave; non-temporal stores, measured faster
      // here, while non-temporal loads were slower)
      if (col_ok) {
        uint32_t cv[kDepthRows];
#pragma unroll
        for (int k = 0; k < kDepthRows; ++k) {
          cv[k] = pc[k];
          if (k < nrows && bi[k] >= 0) {
            const DepthRec& R = rec[bi[k]];
            cv[k] = ((GlobalU32)R.color)[(int64_t)(Y0 + k - R.y) * R.pitch + (X - R.x)];
          }
        }
#pragma unroll
        for (int k = 0; k < kDepthRows; ++k) {
          if (k >= nrows) continue;
          const int64_t oo = (int64_t)(Y0 + k - vy) * out_pitch + (X - vx);
          __builtin_nontemporal_store(cv[k], &out_color[oo]);
          if (out_depth) __builtin_nontemporal_store(bd[k], &out_depth[oo]);
        }
      }
    }
  }
}

}  // namespace cmp
