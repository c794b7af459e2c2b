// Internal definitions shared by the HIP translation units of libcmp.
// Target: gfx950 (CDNA4), wave64.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

#include "cmp.h"

namespace cmp {

constexpr uint32_t kClearDepth = 0xFFFFFFFFu;
constexpr int kThreads = 256;   // every kernel runs 256-thread workgroups (4 waves)
constexpr int kWave = 64;

// ----------------------------------------------------------------- host
void set_error(const char* fmt, ...);
cmp_status hip_fail(hipError_t e, const char* what);
// Plan logging: with CMP_LOG=1 in the environment (read once per process),
// log_plan writes one "[cmp] ..." line to stderr; otherwise it does nothing.
bool log_enabled();
void log_plan(const char* fmt, ...) __attribute__((format(printf, 1, 2)));

// roctx ranges around the entry points: with CMP_ROCTX=1 in the environment
// (read once per process) each call that enqueues work is one named range on
// the calling thread (rocprofv3 --marker-trace shows them beside the
// kernels); the roctx library is loaded on first use, so nothing depends on
// it otherwise. A range covers the host-side call (validation and enqueue).
class ApiRange {
 public:
  explicit ApiRange(const char* name);
  ~ApiRange();
  ApiRange(const ApiRange&) = delete;
  ApiRange& operator=(const ApiRange&) = delete;

 private:
  bool on_;
};
#define CMP_RANGE(name) ::cmp::ApiRange cmp_api_range_(name)

#define CMP_CHECK_HIP(expr)                                  \
  do {                                                       \
    hipError_t e_ = (expr);                                  \
    if (e_ != hipSuccess) return ::cmp::hip_fail(e_, #expr); \
  } while (0)

#define CMP_REQUIRE(cond, ...)                \
  do {                                        \
    if (!(cond)) {                            \
      ::cmp::set_error(__VA_ARGS__);          \
      return CMP_EINVAL;                      \
    }                                         \
  } while (0)

inline bool rect_valid(cmp_rect r) { return r.w >= 0 && r.h >= 0; }
inline bool rect_empty(cmp_rect r) { return r.w <= 0 || r.h <= 0; }

// Launch geometry of a schedule: a list of regions of the viewport, each cut
// into workgroup tiles (row-major inside the region).
struct Region {
  int32_t x, y, w, h;     // destination pixels
  int32_t tile_begin;     // first workgroup of this region
};
constexpr int kMaxRegions = 64;

// Builds the regions of `sched` over `vp`. Returns the number of regions (or
// a negative cmp_status) and the total number of workgroup tiles.
int plan_regions(cmp_schedule sched, cmp_rect vp, int tile_w, int tile_h, Region* out,
                 int64_t* total_tiles);

// --------------------------------------------------------------- device
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));

// 16-byte load/store from an address that is only 4-byte aligned. gfx950
// handles dword-aligned multi-dword global accesses.
__device__ __forceinline__ u32x4 ld_u32x4(const uint32_t* p) {
  u32x4 v;
  __builtin_memcpy(&v, __builtin_assume_aligned(p, 4), 16);
  return v;
}
// A 16-byte global store marked non-temporal (streaming: the line is not
// kept for reuse), at 4-byte alignment.
typedef uint32_t u32x4u __attribute__((ext_vector_type(4), aligned(4)));
__device__ __forceinline__ void st_u32x4_nt(uint32_t* p, u32x4 v) {
  __builtin_nontemporal_store(u32x4u{v.x, v.y, v.z, v.w}, (__attribute__((address_space(1))) u32x4u*)p);
}
__device__ __forceinline__ void st_u32x4(uint32_t* p, u32x4 v) {
  __builtin_memcpy(__builtin_assume_aligned(p, 4), &v, 16);
}

// One RGBA pixel of a float layer as float4 (RGBA32F: 16-byte aligned load;
// RGBA16F: 8-byte aligned load, exact widening).
template <int FMT>
__device__ __forceinline__ f32x4 ld_rgba(const void* base, int64_t px) {
  if constexpr (FMT == CMP_RGBA32F) {
    return reinterpret_cast<const f32x4*>(base)[px];
  } else {
    const f16x4 h = reinterpret_cast<const f16x4*>(base)[px];
    return f32x4{(float)h.x, (float)h.y, (float)h.z, (float)h.w};
  }
}

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = min(v, __shfl_xor(v, m));
  return v;
}
__device__ __forceinline__ int wave_max(int v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v = max(v, __shfl_xor(v, m));
  return v;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uniform64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T* uniform_ptr(T* p) {
  return reinterpret_cast<T*>(uniform64((int64_t)reinterpret_cast<uintptr_t>(p)));
}

// The segment holding workgroup blk: the last i < n whose first workgroup
// begin_of(i) is <= blk (begin_of(0) == 0, ascending). Every begin_of(i) is
// read up front (independent scalar loads from the kernel arguments) rather
// than one after another, which costs a cache miss per step on a CU's first
// workgroup.
template <int kN, typename F>
__device__ __forceinline__ int count_begins_le(F begin_of, int n, int blk) {
  int r = 0;
#pragma unroll
  for (int i = 1; i < kN; ++i) r += (i < n && begin_of(i) <= blk) ? 1 : 0;
  return r;
}
template <typename F>
__device__ __forceinline__ int segment_of(F begin_of, int n, int blk) {
  if (n <= 1) return 0;
  if (n <= 16) return count_begins_le<16>(begin_of, n, blk);
  return count_begins_le<64>(begin_of, n, blk);
}

// The placement of contributor i: the host rectangle, or the device one
// (clamped to the host rectangle's size, which bounds the buffer).
__device__ __forceinline__ void placement(const int32_t* roi_dev, int idx, int32_t hx, int32_t hy,
                                          int32_t hw, int32_t hh, int32_t& x, int32_t& y,
                                          int32_t& w, int32_t& h) {
  if (roi_dev) {
    const int4 r = reinterpret_cast<const int4*>(roi_dev)[idx];
    x = uniform(r.x);
    y = uniform(r.y);
    w = uniform(max(0, min(r.z, hw)));
    h = uniform(max(0, min(r.w, hh)));
  } else {
    x = hx; y = hy; w = hw; h = hh;
  }
}

}  // namespace cmp
