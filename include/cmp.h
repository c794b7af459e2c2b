/*
 * cmp.h - sort-last image compositing on one MI355X (gfx950).
 *
 * The data-parallel hot path of sort-last parallel rendering as described in
 * S. Eilemann, "Parallel Rendering and Large Data Visualization" (thesis,
 * 2019), chapter 5 "Compositing": depth-sorted and ordered (alpha) sort-last
 * compositing of many contributors' partial framebuffers, automatic region of
 * interest (ROI) detection, and per-component run-length encoding (RLE) of
 * pixel data; plus the adjoint of ordered compositing and a batched,
 * persistent launch of many uneven compositing jobs.
 *
 * Plain C ABI. Every pointer documented as "device" is HIP device memory on
 * the current device; every "host" pointer is ordinary host memory that is
 * only read during the call. `stream` is a hipStream_t (NULL = the null
 * stream). All calls are stream-ordered and asynchronous: a CMP_OK return
 * means the work is enqueued. Arguments are validated on the host before
 * anything is enqueued, so an error return means nothing was launched;
 * cmp_last_error() then describes the problem. Apart from the opaque batch
 * plan (host memory) the library never allocates: scratch memory is the
 * caller's "workspace", sized by the *_workspace_size functions.
 *
 * Conventions (the thesis fixes none of these; they are this library's):
 *  - Buffers are row-major, row 0 first in memory; pitches count pixels.
 *  - cmp_rect {x, y, w, h} is the half-open [x, x+w) x [y, y+h); an empty
 *    rectangle has w == 0 or h == 0.
 *  - RGBA8 pixels are little-endian uint32 words with bytes R, G, B, A.
 *  - Depth is uint32, smaller is nearer, 0xFFFFFFFF is the clear depth.
 *  - Float layers hold premultiplied RGBA, alpha in channel 3.
 *  - A contributor's `roi` places its w x h block of pixels at (roi.x, roi.y)
 *    in destination pixel space (Section 5.3, Region of Interest: the ROI is
 *    sent with the pixels and used to place them on the input frame).
 *
 * Environment (read by the library, never required):
 *  - CMP_LOG=1: each plan (schedule regions and tiles, ROI, RLE and batch
 *    launch geometry, the tune cache a batch plan used) is written to stderr
 *    as one "[cmp] ..." line. Read once per process.
 *  - CMP_TUNE_CACHE=<path>: the tune cache that cmp_batch_plan_create and
 *    cmp_autotune use when their path argument is NULL.
 *  - CMP_ROCTX=1: every call that enqueues work is one roctx range, named
 *    after the entry point, around its host side (validation and enqueue);
 *    the roctx library is loaded at the first such call. Read once per
 *    process.
 */
#ifndef CMP_H
#define CMP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t cmp_status;
#define CMP_OK            0
#define CMP_EINVAL       -1   /* an argument is invalid                        */
#define CMP_ENOSPC       -2   /* an output or workspace is too small           */
#define CMP_EHIP         -3   /* the HIP runtime reported an error             */
#define CMP_EUNSUPPORTED -4   /* a valid request the library does not handle   */
#define CMP_ECORRUPT     -5   /* an RLE stream is malformed (device status)    */
#define CMP_ETIMEOUT     -6   /* a bounded device-side wait gave up (status)   */

typedef int32_t cmp_format;
#define CMP_RGBA8   0   /* uint32 per pixel                                  */
#define CMP_RGBA32F 1   /* 4 x float per pixel (16 bytes)                    */
#define CMP_RGBA16F 2   /* 4 x IEEE half per pixel (8 bytes)                 */

typedef struct { int32_t x, y, w, h; } cmp_rect;

/*
 * Parallel compositing schedule (Section 5.2.2, Direct Send and Binary Swap).
 * On one GPU the P "owners" are tile assignments inside the launch:
 *   CMP_SCHED_SEQ          one region, the whole viewport.
 *   CMP_SCHED_DIRECT_SEND  P row strips; strip k covers the rows
 *                          [floor(k H / P), floor((k+1) H / P)).
 *   CMP_SCHED_BINARY_SWAP  P a power of two; log2 P rounds each halve every
 *                          region along its longer side (rows on a tie; the
 *                          first half is floor(len / 2) long). For ordered
 *                          compositing, the back-to-front list is cut into P
 *                          contiguous groups, group g = positions
 *                          [floor(g n / P), floor((g+1) n / P)), and the group
 *                          composites are merged pairwise in the binary tree
 *                          of the exchange rounds. For depth compositing the
 *                          merge order cannot change the result (see
 *                          cmp_composite_depth), so the schedule only decides
 *                          the tiles.
 * owners (P) is 1..64.
 */
#define CMP_SCHED_SEQ          0
#define CMP_SCHED_DIRECT_SEND  1
#define CMP_SCHED_BINARY_SWAP  2
typedef struct { int32_t kind; int32_t owners; } cmp_schedule;

/* The regions a schedule assigns to its owners over `viewport`, in owner
 * order, empty regions left out; writes at most `max` rectangles to `out`
 * (host) and returns how many there are, or a negative cmp_status. Host-only. */
int32_t cmp_schedule_regions(cmp_schedule sched, cmp_rect viewport, cmp_rect* out, int32_t max);

/* Workgroup tile in destination pixels; {0, 0} picks the default. Widths that
 * are multiples of 64 keep every lane busy. The tile never changes results. */
typedef struct { int32_t w, h; } cmp_tile;

/* One contributor image or layer. */
typedef struct {
  const void*     color;  /* device; RGBA8 | RGBA32F | RGBA16F per the call  */
  const uint32_t* depth;  /* device uint32 depth, or NULL                     */
  int64_t         pitch;  /* row pitch in pixels, >= roi.w                    */
  cmp_rect        roi;    /* placement in destination pixels (w x h block)   */
} cmp_image;

const char* cmp_version(void);
const char* cmp_status_string(cmp_status s);
/* Text of the last host-side error on the calling thread ("" if none). */
const char* cmp_last_error(void);

/*
 * Depth-sorted sort-last compositing.
 * Section 5.2.1 (Spatial and Depth-Sorted Sort-Last Compositing): every final
 * pixel takes the colour of the source with the front-most depth.
 *   For each destination pixel p in `viewport`, over the contributors i whose
 *   placement covers p, pick the smallest (depth, i) pair; the clear depth
 *   0xFFFFFFFF never wins. out_color = the winner's colour, or 0 if none;
 *   out_depth = the winner's depth, or 0xFFFFFFFF if none.
 * Ties go to the lower index, which makes the result independent of the
 * order in which frames are combined (Section 5.6, Out-of-Order Assembly).
 *   in[n]      host array; color = RGBA8 (uint32), depth required.
 *   roi_dev    NULL, or device int32[n][4] (x, y, w, h) placements that
 *              replace in[i].roi.x/y/w/h at run time (e.g. ROIs detected on
 *              the device). in[i].roi.w/h then bound the buffer: a device
 *              w or h beyond them is clamped, and negative sizes are empty.
 *   out_color  device uint32, viewport.w x viewport.h, pitch out_pitch.
 *   out_depth  device uint32 or NULL (same pitch). Required when n > 48.
 * n == 0 writes the background. Errors: CMP_EINVAL (n < 0, NULL buffers,
 * negative sizes, pitch < width, bad schedule or tile), CMP_EHIP.
 */
cmp_status cmp_composite_depth(const cmp_image* in, int32_t n, const int32_t* roi_dev,
                               cmp_rect viewport, uint32_t* out_color, uint32_t* out_depth,
                               int64_t out_pitch, cmp_schedule sched, cmp_tile tile,
                               void* stream);

/*
 * cmp_composite_depth with the device rectangles cropping the contributors
 * instead of placing them: in[i] stays where in[i].roi places it (e.g. a
 * whole frame at its viewport), and only its part inside roi_dev[i] (e.g.
 * its detected ROI, in destination pixels) is read. Section 5.3: the input
 * frame places the pixel data at the ROI's position; a frame whose ROI
 * blocks were decompressed into place (cmp_rle_decompress_at_roi) is read
 * at its own columns, so a contributor row starts where the destination's
 * does (whole cache lines when the frame's pitch and the tiles are aligned).
 * roi_dev is required; other arguments, results and errors as
 * cmp_composite_depth.
 */
cmp_status cmp_composite_depth_crop(const cmp_image* in, int32_t n, const int32_t* roi_dev,
                                    cmp_rect viewport, uint32_t* out_color, uint32_t* out_depth,
                                    int64_t out_pitch, cmp_schedule sched, cmp_tile tile,
                                    void* stream);

/*
 * Ordered (spatial) sort-last compositing with alpha blending.
 * Section 5.2.1: the partial images of convex regions are sorted by depth and
 * blended in order; ordering is the application's part (Section 3.6,
 * Compositing: ordered compositing reorders the input frames).
 *   out(p) = fold over j = 0..n-1 of  acc <- L + (1 - L.alpha) * acc
 * with L = layer order_b2f[j] at p (transparent outside its placement),
 * starting from acc = 0; i.e. Porter-Duff "over" of premultiplied colour,
 * back to front. Arithmetic: FP32 fused multiply-add per channel, FP32
 * accumulation for RGBA32F and RGBA16F storage.
 *   in[n]      host array; color = RGBA32F or RGBA16F (fmt), depth unused.
 *   order_b2f  host int32[n], a permutation of 0..n-1, back to front.
 *   out_rgba   device float[viewport.h][out_pitch][4].
 * CMP_SCHED_SEQ and CMP_SCHED_DIRECT_SEND give identical bits; BINARY_SWAP
 * evaluates the merge tree described above (n <= 64 for it).
 * Errors: CMP_EINVAL (also a non-permutation order), CMP_EUNSUPPORTED, CMP_EHIP.
 */
cmp_status cmp_composite_over(const cmp_image* in, int32_t n, cmp_format fmt,
                              const int32_t* order_b2f, cmp_rect viewport, float* out_rgba,
                              int64_t out_pitch, cmp_schedule sched, cmp_tile tile,
                              void* stream);

/*
 * Adjoint of cmp_composite_over (SEQ order). The thesis has no backward pass;
 * this differentiates the forward operation above.
 * With the layers that cover p in front-to-back order i = 0 (nearest) ..,
 * T_0 = 1, T_{i+1} = T_i (1 - a_i), and S_i the composite of layers i and
 * everything behind it (S_end = 0), out = (front part) + T_i S_i, so for
 * G = grad_out(p):
 *   grad L_i[k] = G_k T_i,      grad a_i += -T_i * sum_m G_m S_{i+1}[m].
 * T and S are recomputed per pixel (never stored to memory); the recurrences
 * run in FP64 and the results are rounded once to FP32.
 *   grad_out       device float[viewport.h][grad_pitch][4].
 *   grad_layers    host array of n device float RGBA pointers; layer i's
 *                  gradient has in[i].roi.w x in[i].roi.h pixels with pitch
 *                  grad_pitch_layers[i] (host int64[n]) and is fully written
 *                  (zero where the layer does not reach the viewport).
 *   workspace      device, 16-byte aligned, >= cmp_over_backward_workspace_size(n)
 *                  bytes (0, and NULL allowed, for n <= 64): the layer
 *                  descriptors of a pass with more layers. Calls sharing a
 *                  workspace must not overlap.
 * The layers are visited in chunks of 32 positions: with more than 32, the
 * alpha of the layers in front of the back chunk is read once more (a first
 * pass that keeps the transmittance at every chunk's front edge).
 * n <= 256. Errors: CMP_EINVAL, CMP_ENOSPC (workspace), CMP_EUNSUPPORTED
 * (n > 256), CMP_EHIP.
 */
size_t     cmp_over_backward_workspace_size(int32_t n);
cmp_status cmp_composite_over_backward(const cmp_image* in, int32_t n, cmp_format fmt,
                                       const int32_t* order_b2f, cmp_rect viewport,
                                       const float* grad_out, int64_t grad_pitch,
                                       float* const* grad_layers,
                                       const int64_t* grad_pitch_layers, void* workspace,
                                       size_t ws_bytes, void* stream);

/*
 * Subpixel compositing (Section 4.2.3, Subpixel: the default compositing
 * accumulates and averages all computed fragments of a pixel, reusing the
 * parallel compositing of sort-last rendering). Each of the n sources gives
 * one RGBA8 sample per pixel (0 where the pixel lies outside its placement);
 * per channel out = floor((sum + floor(n / 2)) / n), the mean rounded half
 * up. Integer arithmetic: every schedule and tile gives the same bits.
 *   in[n]   host array, color = RGBA8; n <= 64.
 *   out     device uint32, viewport.w x viewport.h, pitch out_pitch.
 * Errors: CMP_EINVAL, CMP_EHIP.
 */
cmp_status cmp_composite_average(const cmp_image* in, int32_t n, cmp_rect viewport,
                                 uint32_t* out, int64_t out_pitch, cmp_schedule sched,
                                 cmp_tile tile, void* stream);

/*
 * Pixel-compound assembly (Section 4.2.2, Pixel: sources render interleaved
 * pixels described by a pixel kernel, its 2D size kx x ky and the 2D offset
 * of the source inside it). Source i holds the destination pixels
 * (vx + ox_i + kx u, vy + oy_i + ky v) at (u, v) of its RGBA8 image
 * (in[i].color, in[i].pitch; in[i].roi.w/h give its size, roi.x/y are
 * ignored). offsets: host int32[n][2] = (ox_i, oy_i). A class that no source
 * has gives 0; if several sources share a class the lowest index wins.
 * n <= 64, kx * ky <= 64. Errors: CMP_EINVAL (also a source too small for
 * its class), CMP_EHIP.
 */
cmp_status cmp_assemble_pixels(const cmp_image* in, int32_t n, const int32_t* offsets,
                               int32_t kx, int32_t ky, cmp_rect viewport, uint32_t* out,
                               int64_t out_pitch, void* stream);

/*
 * Automatic ROI detection: the 2D bounding box of the pixels that hold data
 * (Section 5.3, Region of Interest: the ROI encloses the rendered data and can
 * be found by analysing the framebuffer).
 *   imgs[i] is an image of imgs[i].roi.w x imgs[i].roi.h pixels (roi.x/y are
 *   ignored). A pixel holds data when: fmt CMP_RGBA8 with depth != NULL:
 *   depth != 0xFFFFFFFF; CMP_RGBA8 without depth: the colour word != 0;
 *   CMP_RGBA32F / CMP_RGBA16F: any channel != 0.0 (-0.0 is empty, NaN is data).
 *   roi_out_dev  device int32[n][4]: image-local (x, y, w, h); an image
 *                without data gives (0, 0, 0, 0).
 *   workspace    device, >= cmp_roi_workspace_size(imgs, n) bytes (per-image
 *                tickets, then a partial box per workgroup), zero-filled
 *                before its first use; every call leaves the tickets zeroed
 *                again.
 * Calls that share a workspace must not overlap. n <= 64.
 * Errors: CMP_EINVAL, CMP_ENOSPC (workspace), CMP_EHIP.
 */
size_t     cmp_roi_workspace_size(const cmp_image* imgs, int32_t n);
cmp_status cmp_roi_detect(const cmp_image* imgs, int32_t n, cmp_format fmt, int32_t* roi_out_dev,
                          void* workspace, size_t ws_bytes, void* stream);

/*
 * ROI with holes: the occupancy of cell_w x cell_h cells (Section 5.3: the
 * framebuffer analysis can also detect holes in the rendered area). A cell
 * is 1 when any of its pixels holds data (the same test as cmp_roi_detect),
 * else 0; the last row and column of cells may be smaller. The grids of the
 * n images lie back to back in grid_dev (device bytes): image i's grid has
 * gh_i = ceil(h_i / cell_h) rows of gw_i = ceil(w_i / cell_w) bytes and
 * starts after the grids of images 0..i-1. n <= 64.
 * Errors: CMP_EINVAL, CMP_EHIP.
 */
cmp_status cmp_roi_grid(const cmp_image* imgs, int32_t n, cmp_format fmt, int32_t cell_w,
                        int32_t cell_h, uint8_t* grid_dev, void* stream);

/*
 * ROI with holes as rectangles (Section 5.3: the framebuffer analysis also
 * finds the holes of the rendered area): the occupied cells of each image's
 * occupancy grid (cmp_roi_grid's layout and cells) covered by disjoint
 * rectangles, built row by row of cells. A row's maximal runs of occupied
 * cells are taken left to right; a run with the same first and last cell as
 * a run of the row above extends that run's rectangle, any other run starts
 * a new one; rectangles are numbered in the order they start. With more
 * than max_rects rectangles an image gets one, the bounding box of its
 * occupied cells.
 *   imgs[i].roi.w/h   the image size the grid was made for.
 *   grid_dev          device, the grids of cmp_roi_grid (same cells).
 *   rects_dev         device int32[n][max_rects][4], 16-byte aligned:
 *                     image-local (x, y, w, h) in pixels, clipped to the
 *                     image; rows past an image's count are (0, 0, 0, 0),
 *                     i.e. empty ROIs. They are ready to be roi_dev of
 *                     cmp_rle_compress (each image listed max_rects times)
 *                     and, as placements, of cmp_composite_depth: the
 *                     rectangles of a frame leave out only cells without
 *                     data, so compositing them gives the composite of the
 *                     frames.
 *   count_dev         device int32[n]: rectangles per image.
 * max_rects 1..64; a grid row of at most 4096 cells. n <= 64.
 * Errors: CMP_EINVAL, CMP_EHIP.
 */
cmp_status cmp_roi_rects(const cmp_image* imgs, int32_t n, int32_t cell_w, int32_t cell_h,
                         const uint8_t* grid_dev, int32_t max_rects, int32_t* rects_dev,
                         int32_t* count_dev, void* stream);

/*
 * Per-component run-length encoding (Section 5.5.1, Enhanced RLE Compression:
 * one RLE stream per component of the pixel, and the image decomposed into
 * sub-images that are compressed in parallel). Stream format "RLE1"; all
 * integers little-endian uint32:
 *   header  magic 0x31454C52, roi.x, roi.y, roi.w, roi.h, nplanes (| 0x100
 *           when the colour is bit-swizzled), 4096, nblocks = ceil(w h / 4096)
 *   boff[nblocks]           payload offset of block b (multiple of 16)
 *   size[nblocks][nplanes]  encoded bytes of (block b, plane k)
 *   zero bytes to a multiple of 16; then the payload: per block, its planes'
 *   encodings back to back, zero-padded to a multiple of 16 bytes.
 * Planes: byte k of the pixel record, which is the RGBA8 word (planes 0..3,
 * R G B A) followed, when a depth buffer is given, by the depth word (planes
 * 4..7, least significant byte first). Pixels are taken row-major over the
 * ROI; block b covers pixels [4096 b, 4096 b + len_b). A plane of a block is
 * its maximal runs of equal bytes that do not cross a multiple of 256 pixels,
 * each stored as (run length - 1, value), when 2 * runs < len_b, and its
 * len_b raw bytes otherwise (size == len_b marks raw).
 */
size_t cmp_rle_max_size(int32_t w, int32_t h, int32_t nplanes);

/* Bit swizzling of the colour words before their planes are taken (Section
 * 5.5.1: a preconditioner that groups the colour bits by significance). The
 * bit pattern is this library's: byte j of the swizzled word holds bits
 * 2j+1 and 2j of R, G, B and A (component c at bits 8j + 2c .. 8j + 2c + 1).
 * The stream records it as 0x100 in header word 5 (next to nplanes);
 * decompression undoes it. */
#define CMP_RLE_SWIZZLE 1u

/*
 * Compress n images (fmt CMP_RGBA8; 8 planes when imgs[i].depth != NULL,
 * else 4) in one launch. flags: 0 or CMP_RLE_SWIZZLE.
 *   imgs[i]       image of imgs[i].roi.w x imgs[i].roi.h pixels (x/y ignored).
 *   roi_dev       NULL (whole images) or device int32[n][4] image-local ROIs,
 *                 e.g. the output of cmp_roi_detect; clamped to the image.
 *   out           host array of n device pointers, 16-byte aligned.
 *   capacity      host uint64[n]; must be >= cmp_rle_max_size(image w, h,
 *                 nplanes), which bounds every ROI's stream.
 *   out_size_dev  device uint64[n]: the stream sizes.
 *   status_dev    device int32[n] (required), zero before the call; receives
 *                 CMP_ETIMEOUT if a block's bounded wait for its predecessors
 *                 gave up (not expected: see below). Such a stream is
 *                 unusable: the block's offset entry is set to 0xFFFFFFFF
 *                 (decompression rejects it with CMP_ECORRUPT), its payload is
 *                 not written, and out_size may be 0.
 *   workspace     device, >= cmp_rle_workspace_size(imgs, n) bytes (per-image
 *                 tickets, a call counter, a look-back flag per block),
 *                 zero-filled before its first use; every call leaves it
 *                 ready for the next (the last workgroup to finish zeroes
 *                 the tickets; flags carry the 30-bit call counter, so they
 *                 are cleared only by the call that wraps it, once in 2^30
 *                 calls). Calls sharing a workspace must not overlap.
 * A block's payload offset is the sum of the sizes of the blocks before it
 * in its image, found on the device while the blocks are encoded (one
 * pass). Workgroups draw blocks from a ticket counter per image, in order,
 * so a block only waits for blocks held by running workgroups: any number of
 * compressions may run at once, on any streams, eagerly or replayed from
 * HIP graphs, each with its own workspace.
 * n <= 64. Errors: CMP_EINVAL, CMP_ENOSPC, CMP_EUNSUPPORTED, CMP_EHIP.
 */
size_t     cmp_rle_workspace_size(const cmp_image* imgs, int32_t n);
cmp_status cmp_rle_compress(const cmp_image* imgs, int32_t n, cmp_format fmt, uint32_t flags,
                            const int32_t* roi_dev, uint8_t* const* out,
                            const uint64_t* capacity, uint64_t* out_size_dev,
                            int32_t* status_dev, void* workspace, size_t ws_bytes,
                            void* stream);

/*
 * cmp_rle_compress without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). The tickets and look-back flags live in
 * a fixed array inside the library: CMP_RLE_SCRATCH_BYTES bytes on every
 * device it runs on, held until the process ends, its address looked up on
 * the first call on each device. The call allocates nothing.
 * Every call on a device shares that array: calls that overlap on one device
 * (on other streams, or graph replays running at the same time) race and
 * corrupt each other's streams; order them. The array starts zeroed and
 * every call leaves it ready for the next.
 * Limit: cmp_rle_workspace_size(imgs, n) <= CMP_RLE_SCRATCH_BYTES, i.e. at
 * most 131072 blocks of 4096 pixels over the n images (64 images of
 * 3840x2160 fit); beyond it CMP_ENOSPC and nothing is launched. Arguments,
 * results and other errors as cmp_rle_compress; CMP_EHIP if the array's
 * address cannot be found.
 */
#define CMP_RLE_SCRATCH_BYTES ((size_t)8192 + (size_t)256 + (size_t)8 * 131072)
cmp_status cmp_rle_compress_noalloc(const cmp_image* imgs, int32_t n, cmp_format fmt,
                                    uint32_t flags, const int32_t* roi_dev, uint8_t* const* out,
                                    const uint64_t* capacity, uint64_t* out_size_dev,
                                    int32_t* status_dev, void* stream);

/*
 * Decompress n RLE1 streams in one launch.
 *   in            host array of n device pointers (16-byte aligned).
 *   in_bytes      host uint64[n]: readable bytes of each stream buffer.
 *   out[i]        destination: color (uint32) and, for 8-plane streams,
 *                 depth; pitch; out[i].roi.w/h bound the decoded ROI size.
 *   roi_out_dev   NULL or device int32[n][4]: the ROI from each header.
 *   status_dev    device int32[n], zero before the call; receives
 *                 CMP_ECORRUPT (malformed stream) or CMP_ENOSPC (ROI larger
 *                 than out[i].roi.w/h, or 8 planes without a depth buffer).
 *                 Blocks of a bad stream may be left unwritten.
 * n <= 64. Errors: CMP_EINVAL, CMP_EHIP.
 */
cmp_status cmp_rle_decompress(const uint8_t* const* in, const uint64_t* in_bytes, int32_t n,
                              const cmp_image* out, int32_t* roi_out_dev, int32_t* status_dev,
                              void* stream);

/*
 * Basic 64-bit RLE (Section 5.5.1, Enhanced RLE Compression: the basic
 * compressor compares two RGBA8 pixels at a time as one 64-bit token, so it
 * only shortens runs of equal pixel pairs; the per-component codec above is
 * the thesis's improvement on it). Stream format "RL64" (the thesis gives
 * none; this library's), all integers little-endian:
 *   header  magic 0x34364C52, roi.x, roi.y, roi.w, roi.h, nstreams (1:
 *           colour; 2: colour + depth), 4096, nblocks = ceil(w h / 4096)
 *   boff[nblocks], size[nblocks][nstreams] (uint32), zero bytes to a
 *   multiple of 16, then per block its streams back to back, zero-padded to
 *   a multiple of 16 bytes (the layout of RLE1).
 * Symbols: the ROI's pixels row-major in pairs, symbol j = pixel 2j (low 32
 * bits) | pixel 2j+1 (high 32 bits), an odd last pixel of a block paired
 * with 0; colour words form stream 0, depth words stream 1. A block of len
 * pixels has m = ceil(len / 2) symbols. Its runs are the maximal runs of
 * equal symbols that do not cross a multiple of 128 symbols (256 pixels).
 * A stream with R runs is stored as tokens when align8(R) + 8 R < 8 m: the
 * R bytes (run length - 1), zero bytes to a multiple of 8, then the R run
 * values as 64-bit words; otherwise as its m symbols (size == 8 m marks raw).
 */
size_t cmp_rle64_max_size(int32_t w, int32_t h, int32_t nstreams);

/* Compress n images to RL64 streams in one launch: the arguments, workspace
 * (cmp_rle_workspace_size), statuses, ordering and errors of
 * cmp_rle_compress without its flags; capacity[i] >= cmp_rle64_max_size(w,
 * h, depth ? 2 : 1). */
cmp_status cmp_rle64_compress(const cmp_image* imgs, int32_t n, cmp_format fmt,
                              const int32_t* roi_dev, uint8_t* const* out,
                              const uint64_t* capacity, uint64_t* out_size_dev,
                              int32_t* status_dev, void* workspace, size_t ws_bytes, void* stream);

/* Decompress n RL64 streams in one launch: the arguments, statuses and
 * errors of cmp_rle_decompress (2-stream streams need a depth buffer).
 * CMP_ECORRUPT also for nonzero padding bytes and a nonzero partner of an
 * odd last pixel. Not affected by cmp_rle_set_groups_per_cu. */
cmp_status cmp_rle64_decompress(const uint8_t* const* in, const uint64_t* in_bytes, int32_t n,
                                const cmp_image* out, int32_t* roi_out_dev, int32_t* status_dev,
                                void* stream);

/*
 * cmp_rle_decompress into frames: out[i] is a whole frame (colour and depth
 * pointers at its pixel (0, 0), pitch, out[i].roi.w/h its size), and stream
 * i's ROI block is written at the ROI's position in it (Section 5.3: the
 * input frame places the pixel data where the ROI says). CMP_ENOSPC (status)
 * when the ROI does not lie inside the frame. Other arguments, results and
 * errors as cmp_rle_decompress.
 */
cmp_status cmp_rle_decompress_at_roi(const uint8_t* const* in, const uint64_t* in_bytes,
                                     int32_t n, const cmp_image* out, int32_t* roi_out_dev,
                                     int32_t* status_dev, void* stream);

/*
 * Occupancy of the RLE kernels, for frames composited asynchronously
 * (Section 5.4: the stages of consecutive frames overlap). Both kernels run
 * a resident grid that by default fills every compute unit; a cap of c
 * workgroups per compute unit (1..) leaves room for the kernels of other
 * streams, which pays when several frames are in flight and costs a
 * single frame some speed. 0 restores the default. Process-wide, for all
 * devices; affects calls issued afterwards. Results do not depend on it.
 * Errors: CMP_EINVAL (a negative cap).
 */
cmp_status cmp_rle_set_groups_per_cu(int32_t compress, int32_t decompress);

/*
 * Streams for frames composited asynchronously (Section 5.4): writes
 * `count` (1..16) new non-blocking streams of the default priority to
 * streams[0..count) on the current device. The HIP runtime ties a stream to
 * one of its hardware queues (GPU_MAX_HW_QUEUES of them, 4 by default) when
 * the stream is created, and two busy streams on one queue run one after
 * the other. Streams created before any stream but the null one ran side by
 * side in every process measured; four taken from a framework's stream pool
 * created later ran up to 14% slower in some processes and not in others.
 * The caller owns the streams and releases them with cmp_streams_destroy
 * (after their work). Errors: CMP_EINVAL (count out of range, NULL array),
 * CMP_EHIP (creation failed: the streams created so far are destroyed and
 * streams[] is left NULL).
 */
cmp_status cmp_streams_create(int32_t count, void** streams);
/* Destroys count streams made by cmp_streams_create (NULL entries are skipped). */
cmp_status cmp_streams_destroy(int32_t count, void* const* streams);

/*
 * Test hook for the failure path of compression: the number of polls a
 * block makes for its predecessors' sizes before it gives up (negative:
 * the default of about a million). With a small limit, blocks whose
 * predecessors are not yet done give up and report CMP_ETIMEOUT instead of
 * waiting. Process-wide; affects calls issued afterwards.
 */
cmp_status cmp_rle_set_wait_limit(int32_t polls);

/*
 * Batched compositing: many independent jobs in one persistent launch whose
 * workgroups pull (job, tile) work items from a device queue, largest first
 * (the pull model of tile work packages, Section 4.2.4 Tiles and Section
 * 6.2.1 Dynamic Work Packages).
 *   kind 0: a cmp_composite_depth job (SEQ), kind 1: cmp_composite_over (SEQ).
 * Each job's results are bit-identical to the plain call.
 */
typedef struct {
  int32_t          kind;       /* 0 depth, 1 over                              */
  cmp_format       fmt;        /* over: CMP_RGBA32F or CMP_RGBA16F             */
  int32_t          n;
  const cmp_image* in;         /* host array of n                              */
  const int32_t*   order_b2f;  /* over: host, back to front                    */
  cmp_rect         viewport;
  void*            out_color;  /* depth: uint32; over: float RGBA              */
  uint32_t*        out_depth;  /* depth: NULL or uint32                        */
  int64_t          out_pitch;
} cmp_job;

typedef struct cmp_batch_plan cmp_batch_plan;

/* Builds the work list on the host. tune_cache_path: a text file written by
 * cmp_autotune whose tile choices are used, or NULL: the file named by
 * CMP_TUNE_CACHE, if set, else the default tiles. */
cmp_status cmp_batch_plan_create(const cmp_job* jobs, int32_t njobs, const char* tune_cache_path,
                                 cmp_batch_plan** plan);
size_t     cmp_batch_workspace_size(const cmp_batch_plan* plan);
/* Copies the plan's tables into `workspace` (device) and prepares its queue
 * counters. The plan must stay alive until the copy has completed. */
cmp_status cmp_batch_upload(const cmp_batch_plan* plan, void* workspace, size_t ws_bytes,
                            void* stream);
/* One persistent launch over every work item; stream-capturable. */
cmp_status cmp_batch_run(const cmp_batch_plan* plan, void* workspace, void* stream);
/* The same jobs as one plain launch per job (the comparison baseline). */
cmp_status cmp_batch_run_plain(const cmp_batch_plan* plan, void* stream);
/* Work items and tiles of the plan (for reporting). */
cmp_status cmp_batch_info(const cmp_batch_plan* plan, int64_t* items, int32_t* workgroups);
void       cmp_batch_plan_destroy(cmp_batch_plan* plan);

/*
 * Autotuner: for every (kind, format, contributor-count bucket, size bucket)
 * that occurs in `jobs`, times each candidate tile with plain launches of a
 * representative job on `stream` (synchronising it) and writes the fastest
 * tile per bucket to the text file `cache_path` (NULL: the file named by
 * CMP_TUNE_CACHE; CMP_EINVAL if that is unset too). Results never depend on
 * the tile. Writes only the jobs' outputs.
 */
cmp_status cmp_autotune(const cmp_job* jobs, int32_t njobs, const char* cache_path, int32_t reps,
                        void* stream);

/*
 * Bandwidth probes (measurement helpers, not part of the method): mode 0
 * reads `bytes` from src with 16-byte loads (dst: device, at least 4 bytes,
 * written only in an (almost) impossible case that keeps the loads alive);
 * mode 1 copies `bytes` from src to dst. 16-byte aligned, bytes % 16 == 0.
 */
cmp_status cmp_bandwidth_probe(int32_t mode, const void* src, void* dst, size_t bytes,
                               void* stream);

#ifdef __cplusplus
}
#endif
#endif /* CMP_H */
