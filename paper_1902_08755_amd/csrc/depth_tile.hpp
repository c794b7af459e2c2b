// Workgroup tile body of depth-sorted compositing, shared by the plain launch
// and the persistent batched launch.
//
// Thesis Section 5.2.1 (Spatial and Depth-Sorted Sort-Last Compositing): a
// final pixel takes the colour of the source with the front-most depth. Here:
// the smallest (depth, index) pair over the contributors covering the pixel;
// the clear depth never wins.
//
// Mapping: each lane owns quads of 4 horizontally adjacent pixels; a wave
// covers 64 consecutive quads of a tile row, so every contributor row segment
// is read with coalesced 16-byte loads. Per contributor only the depth is
// read; the colour is gathered once, from the winner, at the end ("lean"
// traffic: 4 bytes per covering contributor plus 4 for the winner).
// Contributors are visited in index order with a strict "<", so ties keep the
// lower index. Loads are issued for four contributors before any of them is
// compared, to keep several 16-byte requests per lane in flight.
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

__device__ __forceinline__ void depth_update(uint32_t d, uint32_t& bd, const uint32_t*& bc,
                                             const uint32_t* cptr) {
  if (d < bd) { bd = d; bc = cptr; }
}

// Composites the tile [x0, x0+tw) x [y0, y0+th) (destination pixels) of a
// viewport whose origin is (vx, vy) into out_color/out_depth. With
// `accumulate`, the outputs already hold the result of earlier contributors
// (a previous pass) and are combined under the same rule.
__device__ __forceinline__ void depth_tile(const DepthSrc src, int n, int x0, int y0, int tw,
                                           int th, uint32_t* __restrict__ out_color,
                                           uint32_t* __restrict__ out_depth, int64_t out_pitch,
                                           int vx, int vy, bool accumulate) {
  const int qpr = (tw + 3) >> 2;
  const int nq = qpr * th;
  for (int q = threadIdx.x; q < nq; q += kThreads) {
    const int r = q / qpr;
    const int c = q - r * qpr;
    const int X = x0 + 4 * c;
    const int Y = y0 + r;
    const int cnt = min(4, x0 + tw - X);
    const int64_t oo = (int64_t)(Y - vy) * out_pitch + (X - vx);

    uint32_t bd0 = kClearDepth, bd1 = kClearDepth, bd2 = kClearDepth, bd3 = kClearDepth;
    const uint32_t *bc0 = nullptr, *bc1 = nullptr, *bc2 = nullptr, *bc3 = nullptr;
    uint32_t pc0 = 0, pc1 = 0, pc2 = 0, pc3 = 0;   // colour from a previous pass
    if (accumulate) {
      if (cnt == 4) {
        const u32x4 d = ld_u32x4(out_depth + oo);
        const u32x4 cc = ld_u32x4(out_color + oo);
        bd0 = d.x; bd1 = d.y; bd2 = d.z; bd3 = d.w;
        pc0 = cc.x; pc1 = cc.y; pc2 = cc.z; pc3 = cc.w;
      } else {
        bd0 = out_depth[oo]; pc0 = out_color[oo];
        if (cnt > 1) { bd1 = out_depth[oo + 1]; pc1 = out_color[oo + 1]; }
        if (cnt > 2) { bd2 = out_depth[oo + 2]; pc2 = out_color[oo + 2]; }
      }
    }

    for (int i0 = 0; i0 < n; i0 += 4) {
      u32x4 dv[4];
      const uint32_t* cp[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        dv[j] = u32x4{kClearDepth, kClearDepth, kClearDepth, kClearDepth};
        cp[j] = nullptr;
        const int i = i0 + j;
        if (i >= n) continue;
        const DepthDesc& D = src.d[i];
        int32_t rx, ry, rw, rh;
        placement(src.roi_dev, src.index_base + i, D.x, D.y, D.w, D.h, rx, ry, rw, rh);
        // whole-tile rejection (uniform)
        if (rw <= 0 || rh <= 0 || rx >= x0 + tw || rx + rw <= x0 || ry >= y0 + th ||
            ry + rh <= y0)
          continue;
        if (Y < ry || Y >= ry + rh) continue;
        const int64_t off = (int64_t)(Y - ry) * D.pitch + (X - rx);
        cp[j] = D.color + off;
        if (cnt == 4 && X >= rx && X + 4 <= rx + rw) {
          dv[j] = ld_u32x4(D.depth + off);
        } else {
          const uint32_t* dp = D.depth + off;
          if (X + 0 >= rx && X + 0 < rx + rw) dv[j].x = dp[0];
          if (cnt > 1 && X + 1 >= rx && X + 1 < rx + rw) dv[j].y = dp[1];
          if (cnt > 2 && X + 2 >= rx && X + 2 < rx + rw) dv[j].z = dp[2];
          if (cnt > 3 && X + 3 >= rx && X + 3 < rx + rw) dv[j].w = dp[3];
        }
      }
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        depth_update(dv[j].x, bd0, bc0, cp[j] + 0);
        depth_update(dv[j].y, bd1, bc1, cp[j] + 1);
        depth_update(dv[j].z, bd2, bc2, cp[j] + 2);
        depth_update(dv[j].w, bd3, bc3, cp[j] + 3);
      }
    }

    // gather the winners' colours
    const uint32_t c0 = bc0 ? *bc0 : pc0;
    const uint32_t c1 = bc1 ? *bc1 : pc1;
    const uint32_t c2 = bc2 ? *bc2 : pc2;
    const uint32_t c3 = bc3 ? *bc3 : pc3;
    if (cnt == 4) {
      st_u32x4(out_color + oo, u32x4{c0, c1, c2, c3});
      if (out_depth) st_u32x4(out_depth + oo, u32x4{bd0, bd1, bd2, bd3});
    } else {
      out_color[oo] = c0;
      if (cnt > 1) out_color[oo + 1] = c1;
      if (cnt > 2) out_color[oo + 2] = c2;
      if (out_depth) {
        out_depth[oo] = bd0;
        if (cnt > 1) out_depth[oo + 1] = bd1;
        if (cnt > 2) out_depth[oo + 2] = bd2;
      }
    }
  }
}

}  // namespace cmp
