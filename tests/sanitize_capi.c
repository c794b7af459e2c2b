/* The host side of libcmp under AddressSanitizer and UndefinedBehaviorSanitizer
 * (built by tests/test_capi_sanitized.py with the sanitizers on the host code
 * only). Every call here either computes on the host or is rejected before
 * anything reaches the HIP runtime: version and status strings, schedule
 * regions, stream and workspace sizes, the argument checks of the compositing,
 * ROI and RLE entry points, and the batch planner over a few hundred synthetic
 * jobs, with tune caches that are valid, malformed or truncated. Device
 * pointers are fake and never dereferenced. argv[1]: a scratch directory. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "cmp.h"

static int fails = 0;
#define EXPECT(c)                                                        \
  do {                                                                   \
    if (!(c)) {                                                          \
      fprintf(stderr, "FAIL %s:%d: %s (%s)\n", __FILE__, __LINE__, #c,   \
              cmp_last_error());                                         \
      ++fails;                                                           \
    }                                                                    \
  } while (0)

/* a fake device address, 256-byte aligned */
static void* fake(uint64_t k) { return (void*)(uintptr_t)(0x7f0000000000ull + (k << 12)); }

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint32_t rnd(uint32_t n) { /* xorshift64*, uniform enough for test shapes */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return (uint32_t)((rng_state * 2685821657736338717ull) >> 33) % (n ? n : 1);
}

static void strings(void) {
  EXPECT(strstr(cmp_version(), "gfx950") != NULL);
  for (int s = -10; s <= 3; ++s) EXPECT(cmp_status_string(s) != NULL);
  EXPECT(cmp_last_error() != NULL);
}

static void schedules(void) {
  const cmp_rect vps[] = {{0, 0, 0, 0},  {0, 0, 1, 1},    {3, 4, 5, 5},   {0, 0, 1920, 1080},
                          {0, 0, 7, 3},  {-5, -5, 100, 1}, {0, 0, 1, 4096}, {10, 20, 33, 17}};
  const int owners[] = {-1, 0, 1, 2, 3, 4, 5, 16, 63, 64, 65, 128};
  cmp_rect out[128];
  for (int kind = -1; kind <= 3; ++kind)
    for (size_t v = 0; v < sizeof vps / sizeof vps[0]; ++v)
      for (size_t o = 0; o < sizeof owners / sizeof owners[0]; ++o) {
        const cmp_schedule s = {kind, owners[o]};
        const int n = cmp_schedule_regions(s, vps[v], out, 128);
        if (n < 0) continue;
        EXPECT(n <= 128);
        int64_t area = 0;
        for (int i = 0; i < n; ++i) area += (int64_t)out[i].w * out[i].h;
        EXPECT(area == (int64_t)vps[v].w * vps[v].h);
        EXPECT(cmp_schedule_regions(s, vps[v], NULL, 0) == n);
        EXPECT(cmp_schedule_regions(s, vps[v], out, 1) == n);
      }
  EXPECT(cmp_schedule_regions((cmp_schedule){CMP_SCHED_SEQ, 1}, (cmp_rect){0, 0, -1, 4}, out, 8) < 0);
  EXPECT(cmp_schedule_regions((cmp_schedule){CMP_SCHED_SEQ, 1}, (cmp_rect){0, 0, 4, 4}, NULL, 8) < 0);
}

static void sizes(void) {
  const int32_t dims[] = {-1, 0, 1, 7, 64, 4095, 4096, 4097, 65535};
  for (size_t a = 0; a < sizeof dims / sizeof dims[0]; ++a)
    for (size_t b = 0; b < sizeof dims / sizeof dims[0]; ++b) {
      for (int np = 3; np <= 9; ++np) (void)cmp_rle_max_size(dims[a], dims[b], np);
      for (int ns = 0; ns <= 3; ++ns) (void)cmp_rle64_max_size(dims[a], dims[b], ns);
    }
  cmp_image im[70];
  for (int i = 0; i < 70; ++i) {
    im[i] = (cmp_image){fake(i), (const uint32_t*)fake(100 + i), 2000,
                        {0, 0, (int32_t)rnd(2000), (int32_t)rnd(1100)}};
  }
  for (int n = 0; n <= 64; n += 7) {
    EXPECT(cmp_rle_workspace_size(im, n) >= 8192);
    (void)cmp_roi_workspace_size(im, n);
  }
  for (int n = -1; n <= 300; n += 13) (void)cmp_over_backward_workspace_size(n);
}

static void argument_errors(void) {
  /* every array holds as many entries as the count passed with it */
  enum { MANY = 300 };
  static cmp_image im[MANY];
  static int32_t perm_many[MANY];
  static const uint8_t* ins_many[MANY];
  static uint64_t inb_many[MANY];
  for (int i = 0; i < MANY; ++i) {
    im[i] = (cmp_image){fake(i), (const uint32_t*)fake(1000 + i), 640, {0, 0, 640, 480}};
    perm_many[i] = MANY - 1 - i;
    ins_many[i] = (const uint8_t*)fake(2000 + i);
    inb_many[i] = 64;
  }
  const cmp_rect vp = {0, 0, 640, 480};
  const cmp_schedule seq = {CMP_SCHED_SEQ, 1}, bad = {CMP_SCHED_BINARY_SWAP, 3};
  const cmp_tile dflt = {0, 0}, huge = {4096, 4096};
  uint32_t* oc = (uint32_t*)fake(50);
  uint32_t* od = (uint32_t*)fake(51);
  EXPECT(cmp_composite_depth(NULL, 2, NULL, vp, oc, od, 640, seq, dflt, NULL) == CMP_EINVAL);
  EXPECT(cmp_composite_depth(im, -1, NULL, vp, oc, od, 640, seq, dflt, NULL) == CMP_EINVAL);
  EXPECT(cmp_composite_depth(im, 4, NULL, vp, NULL, od, 640, seq, dflt, NULL) == CMP_EINVAL);
  EXPECT(cmp_composite_depth(im, 4, NULL, vp, oc, od, 100, seq, dflt, NULL) == CMP_EINVAL);
  EXPECT(cmp_composite_depth(im, 4, NULL, vp, oc, od, 640, bad, dflt, NULL) == CMP_EINVAL);
  EXPECT(cmp_composite_depth(im, 4, NULL, vp, oc, od, 640, seq, huge, NULL) == CMP_EINVAL);
  EXPECT(cmp_composite_depth_crop(im, 4, NULL, vp, oc, od, 640, seq, dflt, NULL) == CMP_EINVAL);
  cmp_image bad_im = im[0];
  bad_im.pitch = 10;
  EXPECT(cmp_composite_depth(&bad_im, 1, NULL, vp, oc, od, 640, seq, dflt, NULL) == CMP_EINVAL);

  float* orgba = (float*)fake(60);
  const int32_t perm[4] = {2, 0, 3, 1}, notperm[4] = {0, 0, 1, 2}, outside[4] = {0, 1, 2, 7};
  EXPECT(cmp_composite_over(im, 4, CMP_RGBA32F, notperm, vp, orgba, 640, seq, dflt, NULL) ==
         CMP_EINVAL);
  EXPECT(cmp_composite_over(im, 4, CMP_RGBA32F, outside, vp, orgba, 640, seq, dflt, NULL) ==
         CMP_EINVAL);
  EXPECT(cmp_composite_over(im, 4, CMP_RGBA32F, NULL, vp, orgba, 640, seq, dflt, NULL) ==
         CMP_EINVAL);
  EXPECT(cmp_composite_over(im, 4, 7, perm, vp, orgba, 640, seq, dflt, NULL) < 0);
  float* gl[4] = {(float*)fake(70), (float*)fake(71), (float*)fake(72), (float*)fake(73)};
  const int64_t gp[4] = {640, 640, 640, 10};
  EXPECT(cmp_composite_over_backward(im, 4, CMP_RGBA32F, perm, vp, orgba, 640, gl, gp, NULL, 0,
                                     NULL) == CMP_EINVAL);
  static float* gl_many[MANY];
  static int64_t gp_many[MANY];
  for (int i = 0; i < MANY; ++i) {
    gl_many[i] = (float*)fake(3000 + i);
    gp_many[i] = 640;
  }
  EXPECT(cmp_composite_over_backward(im, MANY, CMP_RGBA32F, perm_many, vp, orgba, 640, gl_many,
                                     gp_many, NULL, 0, NULL) == CMP_EUNSUPPORTED);
  EXPECT(cmp_composite_average(im, 65, vp, oc, 640, seq, dflt, NULL) < 0);
  const int32_t offs[8] = {0, 0, 1, 0, 0, 1, 1, 1};
  EXPECT(cmp_assemble_pixels(im, 4, offs, 0, 2, vp, oc, 640, NULL) < 0);

  int32_t* roi = (int32_t*)fake(80);
  EXPECT(cmp_roi_detect(im, 65, CMP_RGBA8, roi, fake(81), 1 << 20, NULL) < 0);
  EXPECT(cmp_roi_detect(im, 4, CMP_RGBA8, roi, fake(81), 16, NULL) == CMP_ENOSPC);
  EXPECT(cmp_roi_grid(im, 4, CMP_RGBA8, 0, 16, (uint8_t*)fake(82), NULL) < 0);
  EXPECT(cmp_roi_rects(im, 4, 16, 16, (const uint8_t*)fake(82), 0, roi, roi, NULL) < 0);

  uint8_t* outs[4] = {(uint8_t*)fake(90), (uint8_t*)fake(91), (uint8_t*)fake(92),
                      (uint8_t*)fake(93)};
  uint64_t caps[4] = {1, 1, 1, 1};
  uint64_t* osz = (uint64_t*)fake(94);
  int32_t* st = (int32_t*)fake(95);
  EXPECT(cmp_rle_compress(im, 0, CMP_RGBA8, 0, NULL, outs, caps, osz, st, fake(96), 1 << 20,
                          NULL) == CMP_OK);
  EXPECT(cmp_rle_compress(im, 65, CMP_RGBA8, 0, NULL, outs, caps, osz, st, fake(96), 1 << 20,
                          NULL) == CMP_EINVAL);
  EXPECT(cmp_rle_compress(im, 4, CMP_RGBA32F, 0, NULL, outs, caps, osz, st, fake(96), 1 << 20,
                          NULL) == CMP_EUNSUPPORTED);
  EXPECT(cmp_rle_compress(im, 4, CMP_RGBA8, 0x80, NULL, outs, caps, osz, st, fake(96), 1 << 20,
                          NULL) == CMP_EINVAL);
  EXPECT(cmp_rle_compress(im, 4, CMP_RGBA8, 0, NULL, outs, caps, osz, st, fake(96), 1 << 20,
                          NULL) == CMP_ENOSPC);
  EXPECT(cmp_rle_compress(im, 4, CMP_RGBA8, 0, NULL, outs, caps, NULL, st, fake(96), 1 << 20,
                          NULL) == CMP_EINVAL);
  EXPECT(cmp_rle64_compress(im, 4, CMP_RGBA8, NULL, outs, caps, osz, st, fake(96), 1 << 20,
                            NULL) == CMP_ENOSPC);
  cmp_image big[64];
  for (int i = 0; i < 64; ++i)
    big[i] = (cmp_image){fake(i), (const uint32_t*)fake(i + 64), 8192, {0, 0, 8192, 8192}};
  uint8_t* bouts[64];
  uint64_t bcaps[64];
  for (int i = 0; i < 64; ++i) {
    bouts[i] = (uint8_t*)fake(200 + i);
    bcaps[i] = 1ull << 40;
  }
  EXPECT(cmp_rle_compress_noalloc(big, 64, CMP_RGBA8, 0, NULL, bouts, bcaps, osz, st, NULL) ==
         CMP_ENOSPC);
  const uint8_t* ins[4] = {outs[0], outs[1], outs[2], outs[3]};
  const uint64_t inb[4] = {64, 64, 64, 64};
  EXPECT(cmp_rle_decompress(ins_many, inb_many, 65, im, roi, st, NULL) < 0);
  EXPECT(cmp_rle_decompress(NULL, inb, 4, im, roi, st, NULL) < 0);
  EXPECT(cmp_rle_decompress_at_roi(ins, inb, 4, im, roi, NULL, NULL) < 0);
  EXPECT(cmp_rle64_decompress(ins, NULL, 4, im, roi, st, NULL) < 0);

  EXPECT(cmp_rle_set_groups_per_cu(-1, 0) == CMP_EINVAL);
  EXPECT(cmp_rle_set_groups_per_cu(2, 3) == CMP_OK);
  EXPECT(cmp_rle_set_groups_per_cu(0, 0) == CMP_OK);
  EXPECT(cmp_rle_set_wait_limit(-5) == CMP_OK);
  void* streams[17];
  EXPECT(cmp_streams_create(0, streams) == CMP_EINVAL);
  EXPECT(cmp_streams_create(17, streams) == CMP_EINVAL);
  EXPECT(cmp_streams_create(2, NULL) == CMP_EINVAL);
  EXPECT(cmp_streams_destroy(0, NULL) == CMP_OK);
  EXPECT(cmp_bandwidth_probe(1, fake(1), fake(2), 17, NULL) < 0);
}

/* ---- batch planning over synthetic jobs */
typedef struct {
  cmp_job job;
  cmp_image in[70];
  int32_t order[70];
} JobBuf;

static void make_jobs(JobBuf* b, int njobs) {
  for (int j = 0; j < njobs; ++j) {
    cmp_job* J = &b[j].job;
    const int kind = j % 2;
    const int w = 1 + (int)rnd(2048), h = 1 + (int)rnd(2048);
    const int n = kind == 0 ? 1 + (int)rnd(70) : 1 + (int)rnd(40);
    for (int i = 0; i < n; ++i) {
      const int rw = (int)rnd((uint32_t)w + 1), rh = (int)rnd((uint32_t)h + 1);
      const int rx = (int)rnd((uint32_t)(w - rw + 1)), ry = (int)rnd((uint32_t)(h - rh + 1));
      b[j].in[i] = (cmp_image){fake(1000 + 100 * j + i),
                               kind == 0 ? (const uint32_t*)fake(50000 + 100 * j + i) : NULL,
                               rw + (int)rnd(3), {rx, ry, rw, rh}};
      b[j].order[i] = n - 1 - i;
    }
    *J = (cmp_job){kind,
                   kind ? (j % 4 == 1 ? CMP_RGBA32F : CMP_RGBA16F) : CMP_RGBA8,
                   n,
                   b[j].in,
                   kind ? b[j].order : NULL,
                   (cmp_rect){0, 0, w, h},
                   fake(90000 + j),
                   kind == 0 ? (uint32_t*)fake(95000 + j) : NULL,
                   w + (int)rnd(5)};
  }
}

static void write_file(const char* path, const char* text) {
  FILE* f = fopen(path, "w");
  if (!f) {
    fprintf(stderr, "cannot write %s\n", path);
    ++fails;
    return;
  }
  fputs(text, f);
  fclose(f);
}

static void batch(const char* dir) {
  enum { NJOBS = 300 };
  JobBuf* b = (JobBuf*)calloc(NJOBS, sizeof(JobBuf));
  make_jobs(b, NJOBS);
  cmp_job jobs[NJOBS];
  for (int j = 0; j < NJOBS; ++j) jobs[j] = b[j].job;

  char good[512], junk[512], cut[512], missing[512];
  snprintf(good, sizeof good, "%s/tune_good.txt", dir);
  snprintf(junk, sizeof junk, "%s/tune_junk.txt", dir);
  snprintf(cut, sizeof cut, "%s/tune_cut.txt", dir);
  snprintf(missing, sizeof missing, "%s/no_such_file.txt", dir);
  /* the header names the architecture the plan runs on: with no GPU, "unknown" */
  write_file(good,
             "# cmp tune cache v1 unknown\n"
             "0 0 0 0 64 8 1.5\n0 0 1 1 128 4 2.0\n1 1 0 0 64 16 3.0\n1 2 2 3 256 2 1.0\n");
  char longline[1200];
  memset(longline, '7', sizeof longline - 2);
  longline[sizeof longline - 2] = '\n';
  longline[sizeof longline - 1] = 0;
  FILE* f = fopen(junk, "w");
  if (f) {
    fputs("# cmp tune cache v1 unknown\n", f);
    fputs("0 0 0 0 0 8 1\n0 0 0 0 -64 8 1\n0 0 0 0 65536 65536 1\n0 0 0 0 2147483647 2 1\n", f);
    fputs("garbage\n\n# cmp tune cache v1 gfx000\n0 0 0 0 64 8 1\n", f);
    fputs(longline, f);
    fputs("# cmp tune cache v1 unknown\n1 1 99 99 32 32 nan\n1 1 -1 -1 32 32 inf\n", f);
    fclose(f);
  } else {
    ++fails;
  }
  write_file(cut, "# cmp tune cache v1 unknown\n0 0 0 0 64");

  const char* caches[] = {NULL, good, junk, cut, missing};
  for (size_t c = 0; c < sizeof caches / sizeof caches[0]; ++c) {
    for (int njobs = 0; njobs <= NJOBS; njobs += 100) {
      cmp_batch_plan* plan = NULL;
      const cmp_status s = cmp_batch_plan_create(jobs, njobs, caches[c], &plan);
      /* the plan is built on the host; only its grid size needs the device,
         so without a GPU the call ends there with CMP_EHIP and no plan */
      EXPECT(s == CMP_OK || (s == CMP_EHIP && plan == NULL));
      if (s != CMP_OK) continue;
      int64_t items = -1;
      int32_t groups = -1;
      EXPECT(cmp_batch_info(plan, &items, &groups) == CMP_OK);
      EXPECT(items >= 0 && (njobs == 0 || items > 0));
      EXPECT(cmp_batch_workspace_size(plan) > 0 || njobs == 0);
      cmp_batch_plan_destroy(plan);
    }
  }
  /* invalid jobs are rejected and leave no plan */
  cmp_job bad = jobs[1];
  int32_t dup[70];
  memcpy(dup, b[1].order, sizeof dup);
  dup[0] = dup[1];
  bad.order_b2f = dup;
  cmp_batch_plan* plan = (cmp_batch_plan*)fake(7);
  EXPECT(cmp_batch_plan_create(&bad, 1, NULL, &plan) == CMP_EINVAL && plan == NULL);
  bad = jobs[0];
  bad.kind = 3;
  EXPECT(cmp_batch_plan_create(&bad, 1, NULL, &plan) == CMP_EINVAL && plan == NULL);
  bad = jobs[0];
  bad.viewport.w = -1;
  EXPECT(cmp_batch_plan_create(&bad, 1, NULL, &plan) == CMP_EINVAL);
  bad = jobs[0];
  bad.out_pitch = 0;
  EXPECT(cmp_batch_plan_create(&bad, 1, NULL, &plan) == CMP_EINVAL);
  EXPECT(cmp_batch_plan_create(NULL, 3, NULL, &plan) == CMP_EINVAL);
  EXPECT(cmp_batch_plan_create(jobs, 3, NULL, NULL) == CMP_EINVAL);
  cmp_batch_plan_destroy(NULL);
  if (!getenv("CMP_TUNE_CACHE"))   /* no path and none in the environment */
    EXPECT(cmp_autotune(jobs, 4, NULL, 1, NULL) == CMP_EINVAL);
  free(b);
}

int main(int argc, char** argv) {
  const char* dir = argc > 1 ? argv[1] : ".";
  strings();
  schedules();
  sizes();
  argument_errors();
  batch(dir);
  if (fails) {
    fprintf(stderr, "%d checks failed\n", fails);
    return 1;
  }
  printf("sanitized capi run: ok\n");
  return 0;
}
