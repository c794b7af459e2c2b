// Host-side helpers of libcmp: version, status strings, the per-thread error
// text and the schedule planner shared by the compositing entry points.
#include <dlfcn.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <mutex>

#include "cmp_internal.hpp"

namespace cmp {

static thread_local char g_err[512];

void set_error(const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof g_err, fmt, ap);
  va_end(ap);
}

cmp_status hip_fail(hipError_t e, const char* what) {
  set_error("%s: %s", what, hipGetErrorString(e));
  return CMP_EHIP;
}

static std::atomic<int> g_log{-1};   // -1: CMP_LOG not read yet

bool log_enabled() {
  int v = g_log.load(std::memory_order_relaxed);
  if (v < 0) {
    const char* e = getenv("CMP_LOG");
    v = (e && *e && strcmp(e, "0") != 0) ? 1 : 0;
    g_log.store(v, std::memory_order_relaxed);
  }
  return v == 1;
}

void log_plan(const char* fmt, ...) {
  if (!log_enabled()) return;
  char line[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(line, sizeof line, fmt, ap);
  va_end(ap);
  fprintf(stderr, "[cmp] %s\n", line);
}

// roctx, resolved on first use when CMP_ROCTX is set: -1 not looked up yet,
// 0 off (unset, or the library is missing), 1 on.
typedef int (*roctx_push_fn)(const char*);
typedef int (*roctx_pop_fn)();
static std::atomic<int> g_roctx{-1};
static roctx_push_fn g_roctx_push = nullptr;
static roctx_pop_fn g_roctx_pop = nullptr;

static bool roctx_on() {
  int v = g_roctx.load(std::memory_order_acquire);
  if (v >= 0) return v == 1;
  static std::mutex mu;
  std::lock_guard<std::mutex> lock(mu);
  v = g_roctx.load(std::memory_order_relaxed);
  if (v >= 0) return v == 1;
  v = 0;
  const char* e = getenv("CMP_ROCTX");
  if (e && *e && strcmp(e, "0") != 0) {
    void* h = dlopen("librocprofiler-sdk-roctx.so.1", RTLD_NOW | RTLD_GLOBAL);
    if (!h) h = dlopen("librocprofiler-sdk-roctx.so", RTLD_NOW | RTLD_GLOBAL);
    if (h) {
      g_roctx_push = (roctx_push_fn)dlsym(h, "roctxRangePushA");
      g_roctx_pop = (roctx_pop_fn)dlsym(h, "roctxRangePop");
      v = g_roctx_push && g_roctx_pop ? 1 : 0;
    }
    log_plan("roctx ranges %s", v ? "on" : "requested, but the roctx library was not found");
  }
  g_roctx.store(v, std::memory_order_release);
  return v == 1;
}

ApiRange::ApiRange(const char* name) : on_(roctx_on()) {
  if (on_) g_roctx_push(name);
}
ApiRange::~ApiRange() {
  if (on_) g_roctx_pop();
}

static void push_region(Region* out, int& nreg, int64_t& tiles, int x, int y, int w, int h,
                        int tw, int th) {
  if (w <= 0 || h <= 0) return;
  out[nreg] = Region{x, y, w, h, (int32_t)tiles};
  tiles += (int64_t)((w + tw - 1) / tw) * ((h + th - 1) / th);
  ++nreg;
}

// Section 5.2.2 (Direct Send and Binary Swap): both spread the compositing
// work over all resources, each of which completes one tile of the final
// image. Here a resource is a set of workgroup tiles.
int plan_regions(cmp_schedule sched, cmp_rect vp, int tw, int th, Region* out,
                 int64_t* total_tiles) {
  const int P = sched.owners;
  int nreg = 0;
  int64_t tiles = 0;
  if (tw <= 0 || th <= 0) {
    set_error("tile %dx%d must be positive", tw, th);
    return CMP_EINVAL;
  }
  switch (sched.kind) {
    case CMP_SCHED_SEQ:
      push_region(out, nreg, tiles, vp.x, vp.y, vp.w, vp.h, tw, th);
      break;
    case CMP_SCHED_DIRECT_SEND:
      if (P < 1 || P > kMaxRegions) {
        set_error("direct send needs 1..%d owners, got %d", kMaxRegions, P);
        return CMP_EINVAL;
      }
      for (int k = 0; k < P; ++k) {
        const int r0 = (int)(((int64_t)k * vp.h) / P), r1 = (int)(((int64_t)(k + 1) * vp.h) / P);
        push_region(out, nreg, tiles, vp.x, vp.y + r0, vp.w, r1 - r0, tw, th);
      }
      break;
    case CMP_SCHED_BINARY_SWAP: {
      if (P < 1 || P > kMaxRegions || (P & (P - 1)) != 0) {
        set_error("binary swap needs a power-of-two owner count <= %d, got %d", kMaxRegions, P);
        return CMP_EINVAL;
      }
      int rounds = 0;
      while ((1 << rounds) < P) ++rounds;
      for (int k = 0; k < P; ++k) {
        int x = vp.x, y = vp.y, w = vp.w, h = vp.h;
        for (int r = 0; r < rounds; ++r) {
          const bool second = (k >> r) & 1;
          if (w > h) {
            const int w1 = w / 2;
            if (second) { x += w1; w -= w1; } else { w = w1; }
          } else {
            const int h1 = h / 2;
            if (second) { y += h1; h -= h1; } else { h = h1; }
          }
        }
        push_region(out, nreg, tiles, x, y, w, h, tw, th);
      }
      break;
    }
    default:
      set_error("unknown schedule kind %d", sched.kind);
      return CMP_EINVAL;
  }
  *total_tiles = tiles;
  log_plan("schedule kind %d (%d owners) over %dx%d at (%d,%d): %d regions, tiles %dx%d, %lld "
           "workgroups", (int)sched.kind, (int)sched.owners, vp.w, vp.h, vp.x, vp.y, nreg, tw, th,
           (long long)tiles);
  return nreg;
}

}  // namespace cmp

extern "C" {

const char* cmp_version(void) { return "cmp 0.1.0 (gfx950)"; }

const char* cmp_status_string(cmp_status s) {
  switch (s) {
    case CMP_OK: return "ok";
    case CMP_EINVAL: return "invalid argument";
    case CMP_ENOSPC: return "output or workspace too small";
    case CMP_EHIP: return "HIP runtime error";
    case CMP_EUNSUPPORTED: return "unsupported";
    case CMP_ECORRUPT: return "corrupt RLE stream";
    case CMP_ETIMEOUT: return "device wait timed out";
    default: return "unknown status";
  }
}

const char* cmp_last_error(void) { return cmp::g_err; }

cmp_status cmp_streams_create(int32_t count, void** streams) {
  CMP_REQUIRE(streams && count >= 1 && count <= 16, "count %d: 1..16 streams", (int)count);
  for (int i = 0; i < count; ++i) streams[i] = nullptr;
  for (int i = 0; i < count; ++i) {
    hipStream_t s = nullptr;
    const hipError_t e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
    if (e != hipSuccess) {
      for (int j = 0; j < i; ++j) {
        (void)hipStreamDestroy((hipStream_t)streams[j]);
        streams[j] = nullptr;
      }
      return cmp::hip_fail(e, "hipStreamCreateWithFlags");
    }
    streams[i] = s;
  }
  return CMP_OK;
}

cmp_status cmp_streams_destroy(int32_t count, void* const* streams) {
  CMP_REQUIRE(count >= 0 && (count == 0 || streams), "count %d, streams %p", (int)count,
              (const void*)streams);
  for (int i = 0; i < count; ++i)
    if (streams[i]) CMP_CHECK_HIP(hipStreamDestroy((hipStream_t)streams[i]));
  return CMP_OK;
}

int32_t cmp_schedule_regions(cmp_schedule sched, cmp_rect viewport, cmp_rect* out, int32_t max) {
  if (viewport.w < 0 || viewport.h < 0 || max < 0 || (max > 0 && !out)) {
    cmp::set_error("invalid arguments");
    return CMP_EINVAL;
  }
  cmp::Region reg[cmp::kMaxRegions];
  int64_t tiles = 0;
  const int n = cmp::plan_regions(sched, viewport, 1, 1, reg, &tiles);
  if (n < 0) return n;
  for (int i = 0; i < n && i < max; ++i) out[i] = cmp_rect{reg[i].x, reg[i].y, reg[i].w, reg[i].h};
  return n;
}

}  // extern "C"
