// cmp_composite_over / cmp_composite_over_backward: ordered premultiplied
// "over" compositing (Section 5.2.1) and its adjoint.
#include <stdlib.h>
#include <string.h>

#include "over_tile.hpp"

namespace cmp {

constexpr int kOverPerPass = 64;
static_assert(kOverPerPass <= kOverStage, "a pass's layers are staged in LDS");

struct OverArgs {
  OverDesc c[kOverPerPass];      // back to front
  Region reg[kMaxRegions];
  uint8_t gb[kOverPerPass + 1];  // binary-swap group bounds (positions)
  float* out;
  int64_t out_pitch;
  int32_t vx, vy;
  int32_t n, nreg;
  int32_t tile_w, tile_h;
  int32_t accumulate;
  int32_t groups;                // 0: sequential chain
};
static_assert(sizeof(OverArgs) <= 4096, "kernel arguments must fit in 4 KiB");

__device__ __forceinline__ void region_tile(const Region* reg, int nreg, int tile_w, int tile_h,
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

template <int FMT>
__global__ __launch_bounds__(kThreads) void over_kernel(const OverArgs a) {
  int x0, y0, tw, th;
  region_tile(a.reg, a.nreg, a.tile_w, a.tile_h, x0, y0, tw, th);
  __shared__ OverDesc s_d[kOverStage];
  stage_layers(a.c, a.n, s_d);   // a.n <= kOverPerPass == kOverStage
  over_tile_seq<FMT>(s_d, a.n, x0, y0, tw, th, a.out, a.out_pitch, a.vx, a.vy,
                     a.accumulate != 0);
}

template <int FMT>
__global__ __launch_bounds__(kThreads) void over_tree_kernel(const OverArgs a) {
  int x0, y0, tw, th;
  region_tile(a.reg, a.nreg, a.tile_w, a.tile_h, x0, y0, tw, th);
  __shared__ OverDesc s_d[kOverStage];
  stage_layers(a.c, a.n, s_d);
  over_tile_tree<FMT>(s_d, a.gb, a.groups, x0, y0, tw, th, a.out, a.out_pitch, a.vx, a.vy);
}

// ------------------------------------------------------------- backward
// For the pixel's covering layers in front-to-back order i, with
// T_0 = 1, T_{i+1} = T_i (1 - a_i) and S_i = L_i + (1 - a_i) S_{i+1}:
//     grad L_i = G T_i,   grad a_i += -T_i <G, S_{i+1}>.
// The back-to-front sweep reads every layer once, builds S (FP64) and keeps
// a_i and D_i = <G, S_{i+1}> per lane in LDS; the front-to-back sweep then
// forms T (FP64) from the kept a_i and writes the gradients. Nothing per
// layer goes to memory. With more than kChunk layers, the back kChunk
// positions are handled first, with T at their front edge computed by a
// front-to-back pass over the alpha of the front chunk.
constexpr int kBwdMax = 64;
constexpr int kChunk = 32;

struct BwdDesc {
  const void* color;
  float* grad;
  int64_t pitch;
  int64_t gpitch;
  int32_t x, y, w, h;
};

struct BwdArgs {
  BwdDesc c[kBwdMax];   // back to front
  const float* gout;
  int64_t gout_pitch;
  int32_t vx, vy, vw, vh;
  int32_t n;
  int32_t tile_w, tile_h, tiles_x;
};
static_assert(sizeof(BwdArgs) <= 4096, "kernel arguments must fit in 4 KiB");

__device__ __forceinline__ bool covers(const BwdDesc& D, int X, int Y) {
  return X >= D.x && X < D.x + D.w && Y >= D.y && Y < D.y + D.h;
}

// One chunk: positions [j0, j1). S (in/out) is the composite of everything
// behind the chunk; T is the transmittance in front of it.
template <int FMT>
__device__ __forceinline__ void bwd_chunk(const BwdDesc* __restrict__ d, int j0, int j1, int X,
                                          int Y, const f32x4 G, double (&S)[4], double T,
                                          float2 (*st)[kThreads]) {
  const double g0 = G.x, g1 = G.y, g2 = G.z, g3 = G.w;
  const int tid = threadIdx.x;
  for (int jb = j0; jb < j1; jb += kOverBatch) {
    f32x4 L[kOverBatch];
    bool cov[kOverBatch];
#pragma unroll
    for (int k = 0; k < kOverBatch; ++k) {
      const int j = jb + k;
      L[k] = f32x4{0.f, 0.f, 0.f, 0.f};
      cov[k] = j < j1 && covers(d[j], X, Y);
      if (cov[k]) L[k] = ld_rgba<FMT>(d[j].color, (int64_t)(Y - d[j].y) * d[j].pitch + (X - d[j].x));
    }
#pragma unroll
    for (int k = 0; k < kOverBatch; ++k) {
      const int j = jb + k;
      if (j >= j1) break;
      float2 e = make_float2(0.f, 0.f);   // (alpha, D); alpha 0 leaves T unchanged
      if (cov[k]) {
        e.y = (float)(g0 * S[0] + g1 * S[1] + g2 * S[2] + g3 * S[3]);
        e.x = L[k].w;
        const double t = 1.0 - (double)L[k].w;
        S[0] = (double)L[k].x + t * S[0];
        S[1] = (double)L[k].y + t * S[1];
        S[2] = (double)L[k].z + t * S[2];
        S[3] = (double)L[k].w + t * S[3];
      }
      st[j - j0][tid] = e;
    }
  }
  for (int j = j1 - 1; j >= j0; --j) {
    const BwdDesc& Dd = d[j];
    if (!covers(Dd, X, Y)) continue;
    const float2 e = st[j - j0][tid];
    f32x4 g;
    g.x = (float)(g0 * T);
    g.y = (float)(g1 * T);
    g.z = (float)(g2 * T);
    g.w = (float)(g3 * T - T * (double)e.y);
    // a global-address-space store cannot alias the kernel-argument copy
    ((__attribute__((address_space(1))) f32x4*)(Dd.grad))
        [(int64_t)(Y - Dd.y) * Dd.gpitch + (X - Dd.x)] = g;
    T = T * (1.0 - (double)e.x);
  }
}

template <int FMT>
__global__ __launch_bounds__(kThreads) void over_bwd_kernel(const BwdArgs a) {
  __shared__ float2 st[kChunk][kThreads];
  const int ty = blockIdx.x / a.tiles_x, tx = blockIdx.x - ty * a.tiles_x;
  const int x0 = a.vx + tx * a.tile_w, y0 = a.vy + ty * a.tile_h;
  const int tw = min(a.tile_w, a.vx + a.vw - x0), th = min(a.tile_h, a.vy + a.vh - y0);
  const int np = tw * th;
  for (int p = threadIdx.x; p < np; p += kThreads) {
    const int r = p / tw;
    const int c = p - r * tw;
    const int X = x0 + c, Y = y0 + r;
    const f32x4 G =
        reinterpret_cast<const f32x4*>(a.gout)[(int64_t)(Y - a.vy) * a.gout_pitch + (X - a.vx)];
    double S[4] = {0.0, 0.0, 0.0, 0.0};
    if (a.n <= kChunk) {
      bwd_chunk<FMT>(a.c, 0, a.n, X, Y, G, S, 1.0, st);
    } else {
      // transmittance in front of the back chunk: front chunk, front to back
      double T1 = 1.0;
      for (int j = a.n - 1; j >= kChunk; --j) {
        const BwdDesc& D = a.c[j];
        if (covers(D, X, Y))
          T1 = T1 * (1.0 - (double)ld_rgba<FMT>(D.color, (int64_t)(Y - D.y) * D.pitch + (X - D.x)).w);
      }
      bwd_chunk<FMT>(a.c, 0, kChunk, X, Y, G, S, T1, st);
      bwd_chunk<FMT>(a.c, kChunk, a.n, X, Y, G, S, 1.0, st);
    }
  }
}

__global__ __launch_bounds__(kThreads) void zero_rgba_kernel(float* p, int64_t pitch, int w,
                                                             int h) {
  const int64_t npx = (int64_t)w * h;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < npx;
       i += (int64_t)gridDim.x * kThreads) {
    const int64_t y = i / w, x = i - y * w;
    reinterpret_cast<f32x4*>(p)[y * pitch + x] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
}

cmp_status validate_over_inputs(const cmp_image* in, int32_t n, cmp_format fmt,
                                const int32_t* order) {
  CMP_REQUIRE(n >= 0, "n = %d is negative", n);
  CMP_REQUIRE(n == 0 || (in && order), "in or order_b2f is NULL");
  CMP_REQUIRE(fmt == CMP_RGBA32F || fmt == CMP_RGBA16F, "format %d is not a float format", fmt);
  const uintptr_t align = fmt == CMP_RGBA32F ? 16 : 8;
  for (int i = 0; i < n; ++i) {
    const cmp_image& I = in[i];
    CMP_REQUIRE(rect_valid(I.roi), "in[%d].roi has a negative size", i);
    if (rect_empty(I.roi)) continue;
    CMP_REQUIRE(I.color, "in[%d].color is NULL", i);
    CMP_REQUIRE(I.pitch >= I.roi.w, "in[%d].pitch < roi.w", i);
    CMP_REQUIRE(((uintptr_t)I.color % align) == 0, "in[%d].color must be %d-byte aligned", i,
                (int)align);
  }
  // order must be a permutation
  if (n > 0) {
    uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);
    if (!seen) return CMP_EINVAL;
    bool ok = true;
    for (int j = 0; j < n && ok; ++j) {
      const int v = order[j];
      if (v < 0 || v >= n || seen[v]) ok = false;
      else seen[v] = 1;
    }
    free(seen);
    CMP_REQUIRE(ok, "order_b2f is not a permutation of 0..%d", n - 1);
  }
  return CMP_OK;
}

}  // namespace cmp

using namespace cmp;

extern "C" cmp_status cmp_composite_over(const cmp_image* in, int32_t n, cmp_format fmt,
                                         const int32_t* order_b2f, cmp_rect viewport,
                                         float* out_rgba, int64_t out_pitch, cmp_schedule sched,
                                         cmp_tile tile, void* stream) {
  cmp_status st = validate_over_inputs(in, n, fmt, order_b2f);
  if (st != CMP_OK) return st;
  CMP_REQUIRE(rect_valid(viewport), "viewport has a negative size");
  if (rect_empty(viewport)) return CMP_OK;
  CMP_REQUIRE(out_rgba && ((uintptr_t)out_rgba & 15) == 0, "out_rgba must be 16-byte aligned");
  CMP_REQUIRE(out_pitch >= viewport.w, "out_pitch < viewport.w");
  const int tw = tile.w ? tile.w : 64, th = tile.h ? tile.h : 4;
  CMP_REQUIRE(tw > 0 && th > 0 && (int64_t)tw * th <= 65536, "bad tile %dx%d", tw, th);
  const bool tree = sched.kind == CMP_SCHED_BINARY_SWAP;
  if (tree && n > kOverPerPass) {
    set_error("binary-swap order supports at most %d layers", kOverPerPass);
    return CMP_EUNSUPPORTED;
  }

  OverArgs a;
  memset(&a, 0, sizeof a);
  int64_t tiles = 0;
  const int nreg = plan_regions(sched, viewport, tw, th, a.reg, &tiles);
  if (nreg < 0) return nreg;
  CMP_REQUIRE(tiles < (1ll << 24), "too many tiles");
  a.out = out_rgba;
  a.out_pitch = out_pitch;
  a.vx = viewport.x;
  a.vy = viewport.y;
  a.nreg = nreg;
  a.tile_w = tw;
  a.tile_h = th;
  hipStream_t s = (hipStream_t)stream;
  auto launch = [&]() -> cmp_status {
    const dim3 grid((unsigned)tiles), block(kThreads);
    if (a.groups > 0) {
      if (fmt == CMP_RGBA32F)
        hipLaunchKernelGGL(over_tree_kernel<CMP_RGBA32F>, grid, block, 0, s, a);
      else
        hipLaunchKernelGGL(over_tree_kernel<CMP_RGBA16F>, grid, block, 0, s, a);
    } else {
      if (fmt == CMP_RGBA32F)
        hipLaunchKernelGGL(over_kernel<CMP_RGBA32F>, grid, block, 0, s, a);
      else
        hipLaunchKernelGGL(over_kernel<CMP_RGBA16F>, grid, block, 0, s, a);
    }
    CMP_CHECK_HIP(hipGetLastError());
    return CMP_OK;
  };
  if (tree) {
    const int P = sched.owners;
    for (int j = 0; j < n; ++j) {
      const cmp_image& I = in[order_b2f[j]];
      a.c[j] = OverDesc{I.color, I.pitch, I.roi.x, I.roi.y, rect_empty(I.roi) ? 0 : I.roi.w,
                        rect_empty(I.roi) ? 0 : I.roi.h};
    }
    for (int g = 0; g <= P; ++g) a.gb[g] = (uint8_t)(((int64_t)g * n) / P);
    a.n = n;
    a.groups = P;
    return launch();
  }
  int base = 0;
  do {
    const int cnt = n - base < kOverPerPass ? n - base : kOverPerPass;
    for (int j = 0; j < cnt; ++j) {
      const cmp_image& I = in[order_b2f[base + j]];
      a.c[j] = OverDesc{I.color, I.pitch, I.roi.x, I.roi.y, rect_empty(I.roi) ? 0 : I.roi.w,
                        rect_empty(I.roi) ? 0 : I.roi.h};
    }
    a.n = cnt;
    a.accumulate = base > 0;
    st = launch();
    if (st != CMP_OK) return st;
    base += cnt;
  } while (base < n);
  return CMP_OK;
}

extern "C" cmp_status cmp_composite_over_backward(const cmp_image* in, int32_t n, cmp_format fmt,
                                                  const int32_t* order_b2f, cmp_rect viewport,
                                                  const float* grad_out, int64_t grad_pitch,
                                                  float* const* grad_layers,
                                                  const int64_t* grad_pitch_layers,
                                                  void* stream) {
  cmp_status st = validate_over_inputs(in, n, fmt, order_b2f);
  if (st != CMP_OK) return st;
  if (n > kBwdMax) {
    set_error("the backward pass supports at most %d layers", kBwdMax);
    return CMP_EUNSUPPORTED;
  }
  CMP_REQUIRE(rect_valid(viewport), "viewport has a negative size");
  CMP_REQUIRE(n == 0 || (grad_layers && grad_pitch_layers), "grad_layers is NULL");
  for (int i = 0; i < n; ++i) {
    if (rect_empty(in[i].roi)) continue;
    CMP_REQUIRE(grad_layers[i] && ((uintptr_t)grad_layers[i] & 15) == 0,
                "grad_layers[%d] must be 16-byte aligned", i);
    CMP_REQUIRE(grad_pitch_layers[i] >= in[i].roi.w, "grad_pitch_layers[%d] < roi.w", i);
  }
  hipStream_t s = (hipStream_t)stream;
  // zero the parts of the layer gradients that the viewport does not reach
  for (int i = 0; i < n; ++i) {
    const cmp_rect r = in[i].roi;
    if (rect_empty(r)) continue;
    const bool inside = !rect_empty(viewport) && r.x >= viewport.x && r.y >= viewport.y &&
                        (int64_t)r.x + r.w <= (int64_t)viewport.x + viewport.w &&
                        (int64_t)r.y + r.h <= (int64_t)viewport.y + viewport.h;
    if (inside) continue;
    const int64_t npx = (int64_t)r.w * r.h;
    const unsigned blocks = (unsigned)((npx + kThreads - 1) / kThreads < 4096
                                           ? (npx + kThreads - 1) / kThreads
                                           : 4096);
    hipLaunchKernelGGL(zero_rgba_kernel, dim3(blocks), dim3(kThreads), 0, s, grad_layers[i],
                       grad_pitch_layers[i], r.w, r.h);
    CMP_CHECK_HIP(hipGetLastError());
  }
  if (rect_empty(viewport) || n == 0) return CMP_OK;
  CMP_REQUIRE(grad_out && ((uintptr_t)grad_out & 15) == 0, "grad_out must be 16-byte aligned");
  CMP_REQUIRE(grad_pitch >= viewport.w, "grad_pitch < viewport.w");

  BwdArgs a;
  memset(&a, 0, sizeof a);
  for (int j = 0; j < n; ++j) {
    const int li = order_b2f[j];
    const cmp_image& I = in[li];
    a.c[j] = BwdDesc{I.color, grad_layers[li], I.pitch, grad_pitch_layers[li], I.roi.x, I.roi.y,
                     rect_empty(I.roi) ? 0 : I.roi.w, rect_empty(I.roi) ? 0 : I.roi.h};
  }
  a.gout = grad_out;
  a.gout_pitch = grad_pitch;
  a.vx = viewport.x;
  a.vy = viewport.y;
  a.vw = viewport.w;
  a.vh = viewport.h;
  a.n = n;
  a.tile_w = 64;
  a.tile_h = 4;
  a.tiles_x = (viewport.w + a.tile_w - 1) / a.tile_w;
  const int64_t tiles = (int64_t)a.tiles_x * ((viewport.h + a.tile_h - 1) / a.tile_h);
  CMP_REQUIRE(tiles < (1ll << 24), "too many tiles");
  if (fmt == CMP_RGBA32F)
    hipLaunchKernelGGL(over_bwd_kernel<CMP_RGBA32F>, dim3((unsigned)tiles), dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(over_bwd_kernel<CMP_RGBA16F>, dim3((unsigned)tiles), dim3(kThreads), 0, s, a);
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}
