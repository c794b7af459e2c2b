// Batched compositing: many uneven jobs in one persistent launch.
//
// The plan cuts every job into workgroup tiles, groups runs of consecutive
// tiles into work items of about kItemBytes of traffic (so the shared queue
// counter is touched rarely), orders the items largest first
// (longest-processing-time order: big items start early, small ones fill the
// tail) and uploads the job records,
// contributor descriptors and items to the caller's workspace. The kernel's
// workgroups, sized to fill the GPU once, pull items from an atomic queue
// counter until it runs dry, like render clients pulling tile work packages
// from a server-side queue (Section 4.2.4, Tiles; Section 6.2.1, Dynamic Work
// Packages). A completion counter lets the last workgroup reset the queue, so
// a captured graph can replay the launch without any reset node.
//
// Each item runs the same tile body as the plain launch, so a job's pixels
// are bit-identical to cmp_composite_depth / cmp_composite_over (SEQ).
//
// The autotuner times candidate tiles per (kind, format, contributor bucket,
// size bucket) with plain launches and stores the winners in a text cache.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "depth_tile.hpp"
#include "over_tile.hpp"

namespace cmp {

cmp_status validate_depth_inputs(const cmp_image* in, int32_t n);
cmp_status validate_over_inputs(const cmp_image* in, int32_t n, cmp_format fmt,
                                const int32_t* order);

struct JobRec {
  int32_t kind, fmt, n, desc_off;
  int32_t vx, vy, vw, vh;
  void* out_color;
  uint32_t* out_depth;
  int64_t out_pitch;
  int32_t tile_w, tile_h, tiles_x, pad;
};

struct Item {
  int32_t job, tile0, ntiles, pad;   // tiles [tile0, tile0 + ntiles) of one job
};

struct BatchArgs {
  uint32_t* ctl;            // [0] next item, [1] finished workgroups
  const JobRec* jobs;
  const DepthDesc* ddesc;
  const OverDesc* odesc;
  const Item* items;
  int32_t nitems;
};

// Built for at least six waves per SIMD: at the compiler's default the
// kernel took 84 VGPRs (five waves); asked for six it fits in 72 with no
// spill and runs at seven (256 jobs: 1.947 -> 1.895 ms). Eight spills.
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(6, 8))) void batch_kernel(
    const BatchArgs a) {
  __shared__ int s_item;
  __shared__ DepthRec s_rec[kPlaceMax];   // contributors of the current depth job
  __shared__ OverDesc s_od[kOverStage];   // layers of the current over job
  const int tid = threadIdx.x;
  while (true) {
    if (tid == 0)
      s_item = (int)__hip_atomic_fetch_add(&a.ctl[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int it = uniform(s_item);
    __syncthreads();
    if (it >= a.nitems) break;
    const Item I = a.items[it];
    const JobRec& J = a.jobs[uniform(I.job)];
    const int t1 = uniform(I.tile0) + uniform(I.ntiles);
    if (J.kind == 0) {
      // contributors in chunks of kPlaceMax staged in LDS; later chunks
      // combine with the output of earlier ones (the planner requires a
      // depth buffer when there is more than one chunk)
      const int jn = uniform(J.n);
      for (int c0 = 0; c0 < jn || c0 == 0; c0 += kPlaceMax) {
        const int cn = min(kPlaceMax, jn - c0);
        if (c0 > 0) __syncthreads();   // the previous chunk's records are no longer read
        stage_contributors(DepthSrc{a.ddesc + J.desc_off + c0, nullptr, 0, 0}, cn, s_rec);
        for (int tile = uniform(I.tile0); tile < t1; ++tile) {
          const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
          const int x0 = J.vx + tx * J.tile_w, y0 = J.vy + ty * J.tile_h;
          const int tw = min(J.tile_w, J.vx + J.vw - x0), th = min(J.tile_h, J.vy + J.vh - y0);
          depth_tile(s_rec, cn, x0, y0, tw, th, (uint32_t*)J.out_color, J.out_depth, J.out_pitch,
                     J.vx, J.vy, c0 > 0);
        }
      }
      continue;
    }
    // an over job's layer descriptors go to LDS when they fit
    const int on = uniform(J.n);
    const OverDesc* od = a.odesc + J.desc_off;
    if (on <= kOverStage) {
      stage_layers(od, on, s_od);
      od = s_od;
    }
    for (int tile = uniform(I.tile0); tile < t1; ++tile) {
      const int ty = tile / J.tiles_x, tx = tile - ty * J.tiles_x;
      const int x0 = J.vx + tx * J.tile_w, y0 = J.vy + ty * J.tile_h;
      const int tw = min(J.tile_w, J.vx + J.vw - x0), th = min(J.tile_h, J.vy + J.vh - y0);
      if (J.fmt == CMP_RGBA32F) {
        over_tile_seq<CMP_RGBA32F>(od, J.n, x0, y0, tw, th, (float*)J.out_color,
                                   J.out_pitch, J.vx, J.vy, false);
      } else {
        over_tile_seq<CMP_RGBA16F>(od, J.n, x0, y0, tw, th, (float*)J.out_color,
                                   J.out_pitch, J.vx, J.vy, false);
      }
    }
  }
  if (tid == 0) {
    // no fence: nothing but the counters is shared with the last workgroup
    const uint32_t done =
        __hip_atomic_fetch_add(&a.ctl[1], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (done == gridDim.x - 1) {
      __hip_atomic_store(&a.ctl[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&a.ctl[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ------------------------------------------------------------ autotuning
struct TileShape {
  int w, h;
};
static const TileShape kDepthTiles[] = {{64, 16}, {64, 32}, {64, 64}, {128, 16}, {128, 32},
                                        {256, 16}};
static const TileShape kOverTiles[] = {{64, 4}, {128, 2}, {256, 1}, {32, 8}, {64, 8},
                                       {16, 16}, {64, 16}, {128, 8}};
static const TileShape kDepthDefault = {64, 16}, kOverDefault = {64, 8};
constexpr double kItemBytes = 512.0 * 1024.0;   // target traffic of one work item

static int ilog2(int64_t v) {
  int r = 0;
  while (v > 1) { v >>= 1; ++r; }
  return r;
}

struct TuneKey {
  int kind, fmt, nb, sb;
  bool operator==(const TuneKey& o) const {
    return kind == o.kind && fmt == o.fmt && nb == o.nb && sb == o.sb;
  }
};

static TuneKey key_of(const cmp_job& j) {
  const int64_t area = (int64_t)(j.viewport.w > 0 ? j.viewport.w : 1) * (j.viewport.h > 0 ? j.viewport.h : 1);
  return TuneKey{j.kind, j.kind == 0 ? CMP_RGBA8 : j.fmt, std::min(6, ilog2(j.n > 0 ? j.n : 1)),
                 std::min(12, ilog2(area) / 2)};
}

struct TuneEntry {
  TuneKey key;
  TileShape tile;
  double us;
};

static std::string device_arch() {
  int dev = 0;
  hipDeviceProp_t p;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&p, dev) != hipSuccess)
    return "unknown";
  std::string a = p.gcnArchName;
  const size_t c = a.find(':');
  return c == std::string::npos ? a : a.substr(0, c);
}

static std::vector<TuneEntry> read_cache(const char* path) {
  std::vector<TuneEntry> v;
  if (!path) return v;
  FILE* f = fopen(path, "r");
  if (!f) return v;
  char line[256];
  const std::string arch = device_arch();
  bool arch_ok = false;
  while (fgets(line, sizeof line, f)) {
    char a[64];
    if (sscanf(line, "# cmp tune cache v1 %63s", a) == 1) {
      arch_ok = arch == a;
      continue;
    }
    TuneEntry e;
    // a tile must be what the plain entry points accept (positive sides,
    // area <= 65536); anything else is ignored and the default tile is used
    if (arch_ok && sscanf(line, "%d %d %d %d %d %d %lf", &e.key.kind, &e.key.fmt, &e.key.nb,
                          &e.key.sb, &e.tile.w, &e.tile.h, &e.us) == 7 &&
        e.tile.w > 0 && e.tile.h > 0 && (int64_t)e.tile.w * e.tile.h <= 65536)
      v.push_back(e);
  }
  fclose(f);
  return v;
}

static TileShape pick_tile(const std::vector<TuneEntry>& cache, const cmp_job& j) {
  const TuneKey k = key_of(j);
  for (const TuneEntry& e : cache)
    if (e.key == k) return e.tile;
  return j.kind == 0 ? kDepthDefault : kOverDefault;
}

static cmp_status plain_job(const cmp_job& j, TileShape t, hipStream_t s) {
  const cmp_schedule seq{CMP_SCHED_SEQ, 1};
  const cmp_tile tile{t.w, t.h};
  if (j.kind == 0)
    return cmp_composite_depth(j.in, j.n, nullptr, j.viewport, (uint32_t*)j.out_color, j.out_depth,
                               j.out_pitch, seq, tile, s);
  return cmp_composite_over(j.in, j.n, j.fmt, j.order_b2f, j.viewport, (float*)j.out_color,
                            j.out_pitch, seq, tile, s);
}

static cmp_status validate_job(const cmp_job& j, int idx) {
  CMP_REQUIRE(j.kind == 0 || j.kind == 1, "job %d: kind %d", idx, j.kind);
  CMP_REQUIRE(rect_valid(j.viewport), "job %d: negative viewport", idx);
  CMP_REQUIRE(j.out_color || rect_empty(j.viewport), "job %d: out_color is NULL", idx);
  CMP_REQUIRE(j.out_pitch >= j.viewport.w, "job %d: out_pitch < viewport.w", idx);
  cmp_status st = j.kind == 0 ? validate_depth_inputs(j.in, j.n)
                              : validate_over_inputs(j.in, j.n, j.fmt, j.order_b2f);
  if (st == CMP_OK && j.kind == 0)
    CMP_REQUIRE(j.n <= kPlaceMax || j.out_depth,
                "job %d: out_depth is required when n > %d (it carries the result between "
                "contributor chunks)", idx, kPlaceMax);
  if (st != CMP_OK) return st;
  if (j.kind == 0)
    CMP_REQUIRE(((uintptr_t)j.out_color & 3) == 0 && ((uintptr_t)j.out_depth & 3) == 0,
                "job %d: outputs must be 4-byte aligned", idx);
  else
    CMP_REQUIRE(((uintptr_t)j.out_color & 15) == 0, "job %d: output must be 16-byte aligned", idx);
  return CMP_OK;
}

}  // namespace cmp

using namespace cmp;

struct cmp_batch_plan {
  std::vector<cmp_job> jobs;                // the caller's jobs (pointers stay the caller's)
  std::vector<std::vector<cmp_image>> ins;  // copies of the per-job image arrays
  std::vector<std::vector<int32_t>> orders;
  std::vector<TileShape> tiles;
  std::vector<unsigned char> blob;          // the device tables, host copy
  size_t off_jobs = 0, off_ddesc = 0, off_odesc = 0, off_items = 0;
  int32_t nitems = 0;
  int32_t grid = 0;
};

static size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

extern "C" cmp_status cmp_batch_plan_create(const cmp_job* jobs, int32_t njobs,
                                            const char* tune_cache_path, cmp_batch_plan** plan) {
  CMP_REQUIRE(plan, "plan is NULL");
  *plan = nullptr;
  CMP_REQUIRE(njobs >= 0 && (njobs == 0 || jobs), "bad job list");
  for (int i = 0; i < njobs; ++i) {
    cmp_status st = validate_job(jobs[i], i);
    if (st != CMP_OK) return st;
  }
  cmp_batch_plan* P = new cmp_batch_plan();
  // no path given: the cache named by CMP_TUNE_CACHE, if any
  if (!tune_cache_path) tune_cache_path = getenv("CMP_TUNE_CACHE");
  const std::vector<TuneEntry> cache = read_cache(tune_cache_path);
  std::vector<JobRec> recs;
  std::vector<DepthDesc> dd;
  std::vector<OverDesc> od;
  struct Cand {
    Item it;
    int64_t cost;
  };
  std::vector<Cand> cands;
  // estimated bytes per pixel of a job: every contributor's share of the
  // viewport it covers, plus the output
  auto px_bytes = [](const cmp_job& j) -> double {
    const double area = (double)std::max(1, j.viewport.w) * std::max(1, j.viewport.h);
    double cover = 0;
    for (int k = 0; k < j.n; ++k)
      if (!rect_empty(j.in[k].roi)) cover += (double)j.in[k].roi.w * j.in[k].roi.h;
    const double per = j.kind == 0 ? 4.0 : (j.fmt == CMP_RGBA32F ? 16.0 : 8.0);
    return per * cover / area + (j.kind == 0 ? 12.0 : 16.0);
  };
  for (int i = 0; i < njobs; ++i) {
    const cmp_job& j = jobs[i];
    P->ins.emplace_back(j.in, j.in + j.n);
    P->orders.emplace_back();
    if (j.kind == 1) P->orders.back().assign(j.order_b2f, j.order_b2f + j.n);
    cmp_job c = j;
    c.in = P->ins.back().data();
    c.order_b2f = j.kind == 1 ? P->orders.back().data() : nullptr;
    P->jobs.push_back(c);
    const TileShape t = pick_tile(cache, j);
    P->tiles.push_back(t);
    JobRec r;
    memset(&r, 0, sizeof r);
    r.kind = j.kind;
    r.fmt = j.kind == 0 ? CMP_RGBA8 : j.fmt;
    r.n = j.n;
    r.vx = j.viewport.x;
    r.vy = j.viewport.y;
    r.vw = rect_empty(j.viewport) ? 0 : j.viewport.w;
    r.vh = rect_empty(j.viewport) ? 0 : j.viewport.h;
    r.out_color = j.out_color;
    r.out_depth = j.out_depth;
    r.out_pitch = j.out_pitch;
    r.tile_w = t.w;
    r.tile_h = t.h;
    r.tiles_x = r.vw ? (r.vw + t.w - 1) / t.w : 0;
    if (j.kind == 0) {
      r.desc_off = (int32_t)dd.size();
      for (int k = 0; k < j.n; ++k) {
        const cmp_image& I = j.in[k];
        const bool e = rect_empty(I.roi);
        dd.push_back(DepthDesc{(const uint32_t*)I.color, I.depth, I.pitch, I.roi.x, I.roi.y,
                               e ? 0 : I.roi.w, e ? 0 : I.roi.h});
      }
    } else {
      r.desc_off = (int32_t)od.size();
      for (int k = 0; k < j.n; ++k) {
        const cmp_image& I = j.in[j.order_b2f[k]];
        const bool e = rect_empty(I.roi);
        od.push_back(OverDesc{I.color, I.pitch, I.roi.x, I.roi.y, e ? 0 : I.roi.w, e ? 0 : I.roi.h});
      }
    }
    recs.push_back(r);
    // work items: runs of consecutive tiles worth about kItemBytes of traffic,
    // so the shared queue counter is touched rarely
    const int tiles_y = r.vh ? (r.vh + t.h - 1) / t.h : 0;
    const int ntiles = tiles_y * r.tiles_x;
    const double tile_bytes = px_bytes(j) * t.w * t.h;
    const int per_item = std::max(1, (int)(kItemBytes / std::max(1.0, tile_bytes)));
    for (int t0 = 0; t0 < ntiles; t0 += per_item) {
      const int cnt = std::min(per_item, ntiles - t0);
      cands.push_back(Cand{Item{i, t0, cnt, 0}, (int64_t)(cnt * tile_bytes)});
    }
  }
  std::stable_sort(cands.begin(), cands.end(),
                   [](const Cand& x, const Cand& y) { return x.cost > y.cost; });
  P->nitems = (int32_t)cands.size();
  // device table layout
  P->off_jobs = 64;
  P->off_ddesc = align_up(P->off_jobs + recs.size() * sizeof(JobRec), 64);
  P->off_odesc = align_up(P->off_ddesc + dd.size() * sizeof(DepthDesc), 64);
  P->off_items = align_up(P->off_odesc + od.size() * sizeof(OverDesc), 64);
  const size_t total = align_up(P->off_items + cands.size() * sizeof(Item), 64);
  P->blob.assign(total, 0);
  if (!recs.empty()) memcpy(P->blob.data() + P->off_jobs, recs.data(), recs.size() * sizeof(JobRec));
  if (!dd.empty()) memcpy(P->blob.data() + P->off_ddesc, dd.data(), dd.size() * sizeof(DepthDesc));
  if (!od.empty()) memcpy(P->blob.data() + P->off_odesc, od.data(), od.size() * sizeof(OverDesc));
  Item* items = (Item*)(P->blob.data() + P->off_items);
  for (size_t k = 0; k < cands.size(); ++k) items[k] = cands[k].it;
  // one wave of resident workgroups
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_kernel, kThreads, 0) !=
          hipSuccess) {
    delete P;
    set_error("could not query the device for the persistent grid size");
    return CMP_EHIP;
  }
  P->grid = std::max(1, cus * std::max(1, per_cu));
  log_plan("batch plan: %d jobs, %d work items, %d resident workgroups, tune cache %s (%zu "
           "entries for this device)", njobs, P->nitems, P->grid,
           tune_cache_path ? tune_cache_path : "none", cache.size());
  *plan = P;
  return CMP_OK;
}

extern "C" size_t cmp_batch_workspace_size(const cmp_batch_plan* plan) {
  return plan ? plan->blob.size() : 0;
}

extern "C" cmp_status cmp_batch_upload(const cmp_batch_plan* plan, void* workspace,
                                       size_t ws_bytes, void* stream) {
  CMP_RANGE("cmp_batch_upload");
  CMP_REQUIRE(plan && workspace, "NULL argument");
  CMP_REQUIRE(((uintptr_t)workspace & 63) == 0, "workspace must be 64-byte aligned");
  if (ws_bytes < plan->blob.size()) {
    set_error("workspace of %zu bytes is smaller than %zu", ws_bytes, plan->blob.size());
    return CMP_ENOSPC;
  }
  CMP_CHECK_HIP(hipMemcpyAsync(workspace, plan->blob.data(), plan->blob.size(),
                               hipMemcpyHostToDevice, (hipStream_t)stream));
  return CMP_OK;
}

extern "C" cmp_status cmp_batch_run(const cmp_batch_plan* plan, void* workspace, void* stream) {
  CMP_RANGE("cmp_batch_run");
  CMP_REQUIRE(plan && workspace, "NULL argument");
  if (plan->nitems == 0) return CMP_OK;
  char* w = (char*)workspace;
  BatchArgs a;
  a.ctl = (uint32_t*)w;
  a.jobs = (const JobRec*)(w + plan->off_jobs);
  a.ddesc = (const DepthDesc*)(w + plan->off_ddesc);
  a.odesc = (const OverDesc*)(w + plan->off_odesc);
  a.items = (const Item*)(w + plan->off_items);
  a.nitems = plan->nitems;
  hipLaunchKernelGGL(batch_kernel, dim3((unsigned)plan->grid), dim3(kThreads), 0,
                     (hipStream_t)stream, a);
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}

extern "C" cmp_status cmp_batch_run_plain(const cmp_batch_plan* plan, void* stream) {
  CMP_RANGE("cmp_batch_run_plain");
  CMP_REQUIRE(plan, "NULL plan");
  for (size_t i = 0; i < plan->jobs.size(); ++i) {
    const cmp_status st = plain_job(plan->jobs[i], plan->tiles[i], (hipStream_t)stream);
    if (st != CMP_OK) return st;
  }
  return CMP_OK;
}

extern "C" cmp_status cmp_batch_info(const cmp_batch_plan* plan, int64_t* items,
                                     int32_t* workgroups) {
  CMP_REQUIRE(plan, "NULL plan");
  if (items) *items = plan->nitems;
  if (workgroups) *workgroups = plan->grid;
  return CMP_OK;
}

extern "C" void cmp_batch_plan_destroy(cmp_batch_plan* plan) { delete plan; }

extern "C" cmp_status cmp_autotune(const cmp_job* jobs, int32_t njobs, const char* cache_path,
                                   int32_t reps, void* stream) {
  CMP_RANGE("cmp_autotune");
  if (!cache_path) cache_path = getenv("CMP_TUNE_CACHE");
  CMP_REQUIRE(njobs >= 0 && (njobs == 0 || jobs) && cache_path,
              "bad arguments (no cache path given and CMP_TUNE_CACHE unset)");
  CMP_REQUIRE(reps >= 1, "reps must be >= 1");
  for (int i = 0; i < njobs; ++i) {
    cmp_status st = validate_job(jobs[i], i);
    if (st != CMP_OK) return st;
  }
  hipStream_t s = (hipStream_t)stream;
  // representative job per key: the largest viewport
  std::vector<TuneKey> keys;
  std::vector<int> rep;
  for (int i = 0; i < njobs; ++i) {
    const TuneKey k = key_of(jobs[i]);
    size_t p = 0;
    while (p < keys.size() && !(keys[p] == k)) ++p;
    const int64_t area = (int64_t)jobs[i].viewport.w * jobs[i].viewport.h;
    if (p == keys.size()) {
      keys.push_back(k);
      rep.push_back(i);
    } else if (area > (int64_t)jobs[rep[p]].viewport.w * jobs[rep[p]].viewport.h) {
      rep[p] = i;
    }
  }
  hipEvent_t e0, e1;
  CMP_CHECK_HIP(hipEventCreate(&e0));
  CMP_CHECK_HIP(hipEventCreate(&e1));
  std::vector<TuneEntry> out;
  cmp_status st = CMP_OK;
  for (size_t p = 0; p < keys.size() && st == CMP_OK; ++p) {
    const cmp_job& j = jobs[rep[p]];
    const TileShape* cand = j.kind == 0 ? kDepthTiles : kOverTiles;
    const int nc = j.kind == 0 ? (int)(sizeof kDepthTiles / sizeof *kDepthTiles)
                               : (int)(sizeof kOverTiles / sizeof *kOverTiles);
    TuneEntry best{keys[p], cand[0], 1e30};
    for (int c = 0; c < nc && st == CMP_OK; ++c) {
      st = plain_job(j, cand[c], s);   // warm-up
      if (st != CMP_OK) break;
      if (hipEventRecord(e0, s) != hipSuccess) { st = CMP_EHIP; break; }
      for (int r = 0; r < reps && st == CMP_OK; ++r) st = plain_job(j, cand[c], s);
      if (st != CMP_OK) break;
      float ms = 0.f;
      if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
        st = CMP_EHIP;
        break;
      }
      const double us = 1000.0 * ms / reps;
      if (us < best.us) best = TuneEntry{keys[p], cand[c], us};
    }
    out.push_back(best);
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != CMP_OK) return st;
  FILE* f = fopen(cache_path, "w");
  if (!f) {
    set_error("cannot write %s", cache_path);
    return CMP_EINVAL;
  }
  fprintf(f, "# cmp tune cache v1 %s\n# kind fmt nbucket sbucket tile_w tile_h us\n",
          device_arch().c_str());
  for (const TuneEntry& e : out)
    fprintf(f, "%d %d %d %d %d %d %.3f\n", e.key.kind, e.key.fmt, e.key.nb, e.key.sb, e.tile.w,
            e.tile.h, e.us);
  fclose(f);
  return CMP_OK;
}
