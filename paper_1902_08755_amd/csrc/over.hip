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
// The positions (back to front) are taken in chunks of kChunk. Per chunk, a
// back-to-front sweep reads every layer once, carries S (FP64) and keeps
// a_i and D_i = <G, S_{i+1}> per lane in LDS; a front-to-back sweep then
// forms T (FP64) from the kept a_i and writes the gradients. Nothing per
// layer goes to memory. The chunks run back to front, so S carries over;
// the transmittance in front of each chunk (a checkpoint) comes from a first
// pass over the alpha of the layers in front of the back chunk, front to
// back, kept per lane in LDS (FP64). Only layers that reach the tile are
// visited, kOverBatch of them per batch of unconditional loads (a lane the
// layer does not cover reads the layer's first pixel and discards it).
constexpr int kChunk = 32;
constexpr int kBwdInline = 64;                        // descriptors in the kernel arguments
constexpr int kBwdMaxLayers = 256;                    // with a descriptor workspace
constexpr int kBwdCkpt = kBwdMaxLayers / kChunk - 1;  // checkpoints of the general kernel
constexpr int kBwdMaxChunks = kBwdMaxLayers / kChunk;

struct BwdDesc {
  const void* color;
  float* grad;
  int64_t pitch;
  int64_t gpitch;
  int32_t x, y, w, h;
};

struct BwdArgs {
  BwdDesc c[kBwdInline];   // back to front (n <= kBwdInline)
  const BwdDesc* desc;     // device copy, back to front (n > kBwdInline)
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

template <int FMT>
__device__ __forceinline__ float ld_alpha(const void* base, int64_t px) {
  if constexpr (FMT == CMP_RGBA32F) {
    return ((const __attribute__((address_space(1))) float*)base)[4 * px + 3];
  } else {
    return (float)((const __attribute__((address_space(1))) _Float16*)base)[4 * px + 3];
  }
}

// T <- T * prod (1 - a_j) over the hit positions of [j0, j0 + 32), front to
// back (descending positions).
template <int FMT>
__device__ __forceinline__ double bwd_alpha_product(const BwdDesc* __restrict__ d, int j0,
                                                    uint32_t hits, int X, int Y, double T) {
  while (hits) {   // uniform
    float al[kOverBatch];
    bool cov[kOverBatch];
    const int first = 31 - __builtin_clz(hits);
#pragma unroll
    for (int k = 0; k < kOverBatch; ++k) {
      const bool has = hits != 0;
      const int i = has ? 31 - __builtin_clz(hits) : first;
      hits &= ~(1u << i);
      const BwdDesc& D = d[j0 + i];
      const int dx = uniform(D.x), dy = uniform(D.y), dw = uniform(D.w), dh = uniform(D.h);
      cov[k] = has && X >= dx && X < dx + dw && Y >= dy && Y < dy + dh;
      al[k] = ld_alpha<FMT>(uniform_ptr(D.color),
                            cov[k] ? (int64_t)(Y - dy) * uniform64(D.pitch) + (X - dx) : 0);
    }
#pragma unroll
    for (int k = 0; k < kOverBatch; ++k)
      if (cov[k]) T = T * (1.0 - (double)al[k]);
  }
  return T;
}

// One chunk: positions j0 + i for the set bits i of `hits`. S (in/out) is the
// composite of everything behind the chunk; T is the transmittance in front
// of it.
template <int FMT>
__device__ __forceinline__ void bwd_chunk(const BwdDesc* __restrict__ d, int j0, uint32_t hits,
                                          int X, int Y, const f32x4 G, double (&S)[4], double T,
                                          float2 (*st)[kThreads]) {
  const double g0 = G.x, g1 = G.y, g2 = G.z, g3 = G.w;
  const int tid = threadIdx.x;
  uint32_t m = hits;
  while (m) {   // uniform: back to front over the hit positions
    f32x4 L[kOverBatch];
    bool cov[kOverBatch], has[kOverBatch];
    int pos[kOverBatch];
    const int first = (int)__builtin_ctz(m);
#pragma unroll
    for (int k = 0; k < kOverBatch; ++k) {
      has[k] = m != 0;
      pos[k] = has[k] ? (int)__builtin_ctz(m) : first;
      m &= m - 1u;
      const BwdDesc& D = d[j0 + pos[k]];
      const int dx = uniform(D.x), dy = uniform(D.y), dw = uniform(D.w), dh = uniform(D.h);
      cov[k] = has[k] && X >= dx && X < dx + dw && Y >= dy && Y < dy + dh;
      L[k] = widen(ld_raw<FMT>(uniform_ptr(D.color),
                               cov[k] ? (int64_t)(Y - dy) * uniform64(D.pitch) + (X - dx) : 0));
    }
#pragma unroll
    for (int k = 0; k < kOverBatch; ++k) {
      if (!has[k]) break;   // uniform
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
      st[pos[k]][tid] = e;
    }
  }
  m = hits;
  while (m) {   // uniform: front to back
    const int i = 31 - __builtin_clz(m);
    m &= ~(1u << i);
    const BwdDesc& Dd = d[j0 + i];
    if (!covers(Dd, X, Y)) continue;
    const float2 e = st[i][tid];
    f32x4 g;
    g.x = (float)(g0 * T);
    g.y = (float)(g1 * T);
    g.z = (float)(g2 * T);
    g.w = (float)(g3 * T - T * (double)e.y);
    // a global-address-space store cannot alias the kernel-argument copy
    __builtin_nontemporal_store(g, &((__attribute__((address_space(1))) f32x4*)(Dd.grad))
        [(int64_t)(Y - Dd.y) * Dd.gpitch + (X - Dd.x)]);
    T = T * (1.0 - (double)e.x);
  }
}

// kInline: n <= kBwdInline, descriptors in the arguments, at most two chunks
// (the back chunk's checkpoint stays in a register); otherwise descriptors
// from the workspace and up to kBwdCkpt checkpoints in LDS.
template <int FMT, bool kInline>
__global__ __launch_bounds__(kThreads) void over_bwd_kernel(const BwdArgs a) {
  __shared__ float2 st[kChunk][kThreads];
  __shared__ double tck[kInline ? 1 : kBwdCkpt][kThreads];
  __shared__ uint32_t s_hits[kBwdMaxChunks];
  const BwdDesc* d = kInline ? a.c : a.desc;
  const int ty = blockIdx.x / a.tiles_x, tx = blockIdx.x - ty * a.tiles_x;
  const int x0 = a.vx + tx * a.tile_w, y0 = a.vy + ty * a.tile_h;
  const int tw = min(a.tile_w, a.vx + a.vw - x0), th = min(a.tile_h, a.vy + a.vh - y0);
  const int np = tw * th;
  const int n = a.n, nch = (n + kChunk - 1) / kChunk;
  // each chunk's layer mask for this tile, found once, before the per-pixel
  // loop (every lane active): wave w takes chunks w, w + 4, ...; lane i
  // tests position i of the chunk and one ballot gives the mask
  {
    const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    for (int ch = wave; ch < nch; ch += kThreads / kWave) {
      const int j = ch * kChunk + lane;
      bool hit = false;
      if (lane < kChunk && j < n) {
        const BwdDesc& D = d[j];
        hit = !tile_misses(D.x, D.y, D.w, D.h, x0, y0, tw, th);
      }
      const uint32_t m = (uint32_t)__ballot(hit);
      if (lane == 0) s_hits[ch] = m;
    }
  }
  __syncthreads();
  for (int p = threadIdx.x; p < np; p += kThreads) {
    const int r = p / tw;
    const int c = p - r * tw;
    const int X = x0 + c, Y = y0 + r;
    const f32x4 G =
        reinterpret_cast<const f32x4*>(a.gout)[(int64_t)(Y - a.vy) * a.gout_pitch + (X - a.vx)];
    // checkpoints: the transmittance in front of chunks nch-2 .. 0
    double T1 = 1.0;
    {
      double T = 1.0;
      for (int ch = nch - 1; ch >= 1; --ch) {
        const int j0 = ch * kChunk;
        T = bwd_alpha_product<FMT>(d, j0, s_hits[ch], X, Y, T);
        if (kInline) T1 = T;
        else tck[ch - 1][threadIdx.x] = T;
      }
    }
    double S[4] = {0.0, 0.0, 0.0, 0.0};
    for (int ch = 0; ch < nch; ++ch) {
      const int j0 = ch * kChunk;
      const double T = ch == nch - 1 ? 1.0 : kInline ? T1 : tck[ch][threadIdx.x];
      bwd_chunk<FMT>(d, j0, s_hits[ch], X, Y, G, S, T, st);
    }
  }
}

// Copies up to kBwdInline descriptors from the arguments to device memory
// (the workspace of a backward pass with more layers): a kernel rather than
// a host copy, so that a captured graph carries the descriptors with it.
struct BwdDescCopy {
  BwdDesc c[kBwdInline];
  BwdDesc* dst;
  int32_t n;
};
static_assert(sizeof(BwdDescCopy) <= 4096, "kernel arguments must fit in 4 KiB");

__global__ __launch_bounds__(kThreads) void bwd_desc_kernel(const BwdDescCopy a) {
  for (int i = threadIdx.x; i < a.n; i += kThreads) a.dst[i] = a.c[i];
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
  CMP_RANGE("cmp_composite_over");
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

extern "C" size_t cmp_over_backward_workspace_size(int32_t n) {
  return n > kBwdInline && n <= kBwdMaxLayers ? (size_t)n * sizeof(BwdDesc) : 0;
}

extern "C" cmp_status cmp_composite_over_backward(const cmp_image* in, int32_t n, cmp_format fmt,
                                                  const int32_t* order_b2f, cmp_rect viewport,
                                                  const float* grad_out, int64_t grad_pitch,
                                                  float* const* grad_layers,
                                                  const int64_t* grad_pitch_layers,
                                                  void* workspace, size_t ws_bytes,
                                                  void* stream) {
  CMP_RANGE("cmp_composite_over_backward");
  cmp_status st = validate_over_inputs(in, n, fmt, order_b2f);
  if (st != CMP_OK) return st;
  if (n > kBwdMaxLayers) {
    set_error("the backward pass supports at most %d layers", kBwdMaxLayers);
    return CMP_EUNSUPPORTED;
  }
  if (n > kBwdInline) {
    CMP_REQUIRE(workspace && ((uintptr_t)workspace & 15) == 0,
                "n = %d > %d layers needs a 16-byte aligned workspace", n, kBwdInline);
    if (ws_bytes < cmp_over_backward_workspace_size(n)) {
      set_error("workspace of %zu bytes is smaller than %zu", ws_bytes,
                cmp_over_backward_workspace_size(n));
      return CMP_ENOSPC;
    }
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
  auto desc = [&](int j) {
    const int li = order_b2f[j];
    const cmp_image& I = in[li];
    return BwdDesc{I.color, grad_layers[li], I.pitch, grad_pitch_layers[li], I.roi.x, I.roi.y,
                   rect_empty(I.roi) ? 0 : I.roi.w, rect_empty(I.roi) ? 0 : I.roi.h};
  };
  if (n <= kBwdInline) {
    for (int j = 0; j < n; ++j) a.c[j] = desc(j);
  } else {
    // the descriptors go to the workspace, kBwdInline per copy kernel
    BwdDesc* dst = (BwdDesc*)workspace;
    for (int j0 = 0; j0 < n; j0 += kBwdInline) {
      BwdDescCopy cp;
      memset(&cp, 0, sizeof cp);
      cp.n = n - j0 < kBwdInline ? n - j0 : kBwdInline;
      for (int j = 0; j < cp.n; ++j) cp.c[j] = desc(j0 + j);
      cp.dst = dst + j0;
      hipLaunchKernelGGL(bwd_desc_kernel, dim3(1), dim3(kThreads), 0, s, cp);
      CMP_CHECK_HIP(hipGetLastError());
    }
    a.desc = dst;
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
  const dim3 grid((unsigned)tiles), block(kThreads);
  if (n <= kBwdInline) {
    if (fmt == CMP_RGBA32F)
      hipLaunchKernelGGL((over_bwd_kernel<CMP_RGBA32F, true>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((over_bwd_kernel<CMP_RGBA16F, true>), grid, block, 0, s, a);
  } else {
    if (fmt == CMP_RGBA32F)
      hipLaunchKernelGGL((over_bwd_kernel<CMP_RGBA32F, false>), grid, block, 0, s, a);
    else
      hipLaunchKernelGGL((over_bwd_kernel<CMP_RGBA16F, false>), grid, block, 0, s, a);
  }
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}
