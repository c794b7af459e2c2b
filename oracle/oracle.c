/*
 * Oracle for the sort-last compositing path: a plain, slow, single-threaded CPU
 * implementation of every operation the GPU library performs.
 *
 * TEST INFRASTRUCTURE ONLY. Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library. The product path (the
 * HIP library and its Python binding) never calls, links or imports it, and
 * this file shares no code, header, table or helper with the product path.
 *
 * Source: S. Eilemann, "Parallel Rendering and Large Data Visualization"
 * (thesis, 2019), chapter 5 "Compositing". Every function below names the
 * passage it follows. Where the thesis is silent, the reading taken is stated
 * in the function's comment.
 *
 * Built with `gcc -O2 -ffp-contract=off` so that no multiply-add is fused:
 * every floating-point operation rounds exactly as written.
 *
 * Conventions shared by all functions (readings; the thesis fixes none of them):
 *  - Buffers are row-major, row 0 first in memory; pitches are in pixels.
 *  - Rectangles {x, y, w, h} are half-open: [x, x+w) x [y, y+h).
 *  - An RGBA8 pixel is a little-endian uint32 whose bytes are R, G, B, A.
 *  - Depth is a uint32; smaller is nearer; 0xFFFFFFFF is the clear depth.
 *  - A contributor's ROI places its w x h pixel block at (roi.x, roi.y) in
 *    destination pixel space (Section 5.3, Region of Interest: the ROI travels
 *    with the pixels and places them on the input frame).
 *  - Float layers are premultiplied RGBA, alpha in channel 3, passed here as
 *    double (the exact upcast of the stored fp32 or fp16 values).
 */
#include <stdint.h>
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

typedef struct { int32_t x, y, w, h; } orc_rect;

#define ORC_CLEAR_DEPTH 0xFFFFFFFFu

static int in_rect(orc_rect r, int64_t X, int64_t Y)
{
    return X >= r.x && X < (int64_t)r.x + r.w && Y >= r.y && Y < (int64_t)r.y + r.h;
}

/* ------------------------------------------------------------------------ */
/* Depth-sorted sort-last compositing.                                      */
/* Section 5.2.1 (Spatial and Depth-Sorted Sort-Last Compositing): each     */
/* final pixel takes the colour of the source whose depth value is the      */
/* front-most.                                                              */
/* Readings: ties go to the lowest contributor index (strict "<" in index   */
/* order), so the result does not depend on arrival order (Section 5.6,     */
/* Out-of-Order Assembly); the clear depth never wins, so an uncovered      */
/* pixel gets colour 0 and depth 0xFFFFFFFF.                                */
/* ------------------------------------------------------------------------ */
void orc_composite_depth(int32_t n,
                         const uint32_t* const* color, const uint32_t* const* depth,
                         const int64_t* pitch, const orc_rect* roi,
                         orc_rect viewport,
                         uint32_t* out_color, uint32_t* out_depth, int64_t out_pitch)
{
    for (int64_t v = 0; v < viewport.h; ++v) {
        for (int64_t u = 0; u < viewport.w; ++u) {
            const int64_t X = viewport.x + u, Y = viewport.y + v;
            uint32_t best_d = ORC_CLEAR_DEPTH, best_c = 0;
            for (int32_t i = 0; i < n; ++i) {
                if (!in_rect(roi[i], X, Y)) continue;
                const int64_t off = (Y - roi[i].y) * pitch[i] + (X - roi[i].x);
                const uint32_t d = depth[i][off];
                if (d < best_d) { best_d = d; best_c = color[i][off]; }
            }
            out_color[v * out_pitch + u] = best_c;
            if (out_depth) out_depth[v * out_pitch + u] = best_d;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Ordered (spatial) sort-last compositing with alpha blending.             */
/* Section 5.2.1: the partial images of convex regions are depth-sorted     */
/* and blended in that order. Reading: the blend is Porter-Duff "over" on   */
/* premultiplied RGBA, composited back to front onto transparent black:     */
/*     acc <- L + (1 - L.a) * acc     (all four channels)                   */
/* `order` lists layer indices from back to front. A layer contributes only */
/* inside its ROI.                                                          */
/* ------------------------------------------------------------------------ */
static void over_pixel_f64(const double* L, double* acc)
{
    const double t = 1.0 - L[3];
    for (int k = 0; k < 4; ++k) acc[k] = L[k] + t * acc[k];
}

static const double* layer_px(const double* const* layer, const int64_t* pitch,
                              const orc_rect* roi, int32_t i, int64_t X, int64_t Y)
{
    if (!in_rect(roi[i], X, Y)) return NULL;
    return layer[i] + 4 * ((Y - roi[i].y) * pitch[i] + (X - roi[i].x));
}

void orc_composite_over(int32_t n, const double* const* layer, const int64_t* pitch,
                        const orc_rect* roi, const int32_t* order_b2f,
                        orc_rect viewport, double* out, int64_t out_pitch)
{
    for (int64_t v = 0; v < viewport.h; ++v) {
        for (int64_t u = 0; u < viewport.w; ++u) {
            const int64_t X = viewport.x + u, Y = viewport.y + v;
            double acc[4] = {0.0, 0.0, 0.0, 0.0};
            for (int32_t j = 0; j < n; ++j) {
                const double* L = layer_px(layer, pitch, roi, order_b2f[j], X, Y);
                if (L) over_pixel_f64(L, acc);
            }
            for (int k = 0; k < 4; ++k) out[4 * (v * out_pitch + u) + k] = acc[k];
        }
    }
}

/* Binary-swap merge order (Section 5.2.2, Direct Send and Binary Swap):    */
/* the back-to-front list is cut into `groups` contiguous runs; group g     */
/* holds positions [floor(g n / P), floor((g+1) n / P)). Each group is      */
/* composited on its own, then neighbours are merged pairwise, level by     */
/* level, as the pairs of a binary compositing tree exchange and combine    */
/* their halves: merge(back, front) = front + (1 - front.a) * back.         */
/* `groups` must be a power of two.                                         */
void orc_composite_over_tree(int32_t n, const double* const* layer, const int64_t* pitch,
                             const orc_rect* roi, const int32_t* order_b2f, int32_t groups,
                             orc_rect viewport, double* out, int64_t out_pitch)
{
    double part[64][4];
    if (groups < 1 || groups > 64) return;
    for (int64_t v = 0; v < viewport.h; ++v) {
        for (int64_t u = 0; u < viewport.w; ++u) {
            const int64_t X = viewport.x + u, Y = viewport.y + v;
            for (int32_t g = 0; g < groups; ++g) {
                const int32_t j0 = (int32_t)(((int64_t)g * n) / groups);
                const int32_t j1 = (int32_t)(((int64_t)(g + 1) * n) / groups);
                for (int k = 0; k < 4; ++k) part[g][k] = 0.0;
                for (int32_t j = j0; j < j1; ++j) {
                    const double* L = layer_px(layer, pitch, roi, order_b2f[j], X, Y);
                    if (L) over_pixel_f64(L, part[g]);
                }
            }
            for (int32_t width = 1; width < groups; width *= 2) {
                for (int32_t g = 0; g + width < groups; g += 2 * width) {
                    const double* front = part[g + width];
                    double* back = part[g];
                    const double t = 1.0 - front[3];
                    for (int k = 0; k < 4; ++k) back[k] = front[k] + t * back[k];
                }
            }
            for (int k = 0; k < 4; ++k) out[4 * (v * out_pitch + u) + k] = part[0][k];
        }
    }
}

/* FP32 forms of the two orders above, for the check that the tree order   */
/* and the sequential order agree in single precision. Every operation is   */
/* a separately rounded float operation (no contraction).                   */
static const float* layer_px_f32(const float* const* layer, const int64_t* pitch,
                                 const orc_rect* roi, int32_t i, int64_t X, int64_t Y)
{
    if (!in_rect(roi[i], X, Y)) return NULL;
    return layer[i] + 4 * ((Y - roi[i].y) * pitch[i] + (X - roi[i].x));
}

void orc_composite_over_f32(int32_t n, const float* const* layer, const int64_t* pitch,
                            const orc_rect* roi, const int32_t* order_b2f, int32_t groups,
                            orc_rect viewport, float* out, int64_t out_pitch)
{
    float part[64][4];
    if (groups < 1 || groups > 64) return;
    for (int64_t v = 0; v < viewport.h; ++v) {
        for (int64_t u = 0; u < viewport.w; ++u) {
            const int64_t X = viewport.x + u, Y = viewport.y + v;
            for (int32_t g = 0; g < groups; ++g) {
                const int32_t j0 = (int32_t)(((int64_t)g * n) / groups);
                const int32_t j1 = (int32_t)(((int64_t)(g + 1) * n) / groups);
                for (int k = 0; k < 4; ++k) part[g][k] = 0.0f;
                for (int32_t j = j0; j < j1; ++j) {
                    const float* L = layer_px_f32(layer, pitch, roi, order_b2f[j], X, Y);
                    if (!L) continue;
                    const float t = 1.0f - L[3];
                    for (int k = 0; k < 4; ++k) {
                        const float p = t * part[g][k];
                        part[g][k] = L[k] + p;
                    }
                }
            }
            for (int32_t width = 1; width < groups; width *= 2) {
                for (int32_t g = 0; g + width < groups; g += 2 * width) {
                    const float* front = part[g + width];
                    float* back = part[g];
                    const float t = 1.0f - front[3];
                    for (int k = 0; k < 4; ++k) {
                        const float p = t * back[k];
                        back[k] = front[k] + p;
                    }
                }
            }
            for (int k = 0; k < 4; ++k) out[4 * (v * out_pitch + u) + k] = part[0][k];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Adjoint of ordered "over" compositing (no counterpart in the thesis; the */
/* forward operation is the one of Section 5.2.1 as read above).            */
/* With front-to-back positions i = 0 (nearest) .. m-1 over the layers that */
/* cover the pixel, T_0 = 1, T_{i+1} = T_i (1 - a_i), and S_i the composite */
/* of layers i..m-1 (S_m = 0), the output is out = P_i + T_i S_i where P_i  */
/* does not depend on layer i and S_i = L_i + (1 - a_i) S_{i+1}. Hence      */
/*     d out_k / d L_i[k]  = T_i                                            */
/*     d out_k / d a_i    -= T_i S_{i+1}[k]                                 */
/* and with G = d loss / d out:                                             */
/*     grad L_i[k] = G_k T_i,  grad a_i += -T_i sum_m G_m S_{i+1}[m].       */
/* `gscale`, when given, receives the componentwise condition scale         */
/*     T_i (|G_k| + [k = 3] sum_m |G_m| S_{i+1}[m])                         */
/* which the tests use as the tolerance scale.                              */
/* Pixels outside layer i's ROI give it no gradient; its gradient buffer    */
/* has the layer's own ROI shape and pitch and is fully written.            */
/* ------------------------------------------------------------------------ */
void orc_composite_over_backward(int32_t n, const double* const* layer, const int64_t* pitch,
                                 const orc_rect* roi, const int32_t* order_b2f,
                                 orc_rect viewport, const double* grad_out, int64_t grad_pitch,
                                 double* const* grad_layer, double* const* gscale)
{
    int32_t cover[1024];
    double S[1025][4];
    if (n > 1024) return;
    for (int32_t i = 0; i < n; ++i) {
        for (int64_t y = 0; y < roi[i].h; ++y)
            for (int64_t x = 0; x < roi[i].w; ++x)
                for (int k = 0; k < 4; ++k) {
                    grad_layer[i][4 * (y * pitch[i] + x) + k] = 0.0;
                    if (gscale) gscale[i][4 * (y * pitch[i] + x) + k] = 0.0;
                }
    }
    for (int64_t v = 0; v < viewport.h; ++v) {
        for (int64_t u = 0; u < viewport.w; ++u) {
            const int64_t X = viewport.x + u, Y = viewport.y + v;
            const double* G = grad_out + 4 * (v * grad_pitch + u);
            /* covering layers, front to back */
            int32_t m = 0;
            for (int32_t j = n - 1; j >= 0; --j)
                if (in_rect(roi[order_b2f[j]], X, Y)) cover[m++] = order_b2f[j];
            /* S_i from the back */
            for (int k = 0; k < 4; ++k) S[m][k] = 0.0;
            for (int32_t i = m - 1; i >= 0; --i) {
                const double* L = layer_px(layer, pitch, roi, cover[i], X, Y);
                for (int k = 0; k < 4; ++k) S[i][k] = L[k] + (1.0 - L[3]) * S[i + 1][k];
            }
            /* T_i from the front, and the gradients */
            double T = 1.0;
            for (int32_t i = 0; i < m; ++i) {
                const int32_t li = cover[i];
                const double* L = layer_px(layer, pitch, roi, li, X, Y);
                const int64_t off = 4 * ((Y - roi[li].y) * pitch[li] + (X - roi[li].x));
                double dot = 0.0, adot = 0.0;
                for (int k = 0; k < 4; ++k) {
                    dot += G[k] * S[i + 1][k];
                    adot += (G[k] < 0 ? -G[k] : G[k]) * S[i + 1][k];
                }
                for (int k = 0; k < 4; ++k) grad_layer[li][off + k] = G[k] * T;
                grad_layer[li][off + 3] += -T * dot;
                if (gscale) {
                    for (int k = 0; k < 4; ++k)
                        gscale[li][off + k] = T * (G[k] < 0 ? -G[k] : G[k]);
                    gscale[li][off + 3] += T * adot;
                }
                T = T * (1.0 - L[3]);
            }
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Region of interest: the screen-space 2D bounding box of the data an      */
/* image holds (Section 5.3, Region of Interest), found by analysing the    */
/* framebuffer. Coordinates are image-local; an image with no data gives    */
/* {0,0,0,0}. Readings for "holds data":                                    */
/*   depth images: depth != 0xFFFFFFFF (colour ignored);                    */
/*   RGBA8 colour-only images: the pixel word != 0;                         */
/*   float images: any channel != 0.0 (so -0.0 is empty, NaN is data).      */
/* ------------------------------------------------------------------------ */
typedef struct { int64_t x0, y0, x1, y1; } bbox;

static void bbox_add(bbox* b, int64_t x, int64_t y)
{
    if (x < b->x0) b->x0 = x;
    if (y < b->y0) b->y0 = y;
    if (x > b->x1) b->x1 = x;
    if (y > b->y1) b->y1 = y;
}

static orc_rect bbox_rect(bbox b)
{
    orc_rect r = {0, 0, 0, 0};
    if (b.x1 < 0) return r;
    r.x = (int32_t)b.x0; r.y = (int32_t)b.y0;
    r.w = (int32_t)(b.x1 - b.x0 + 1); r.h = (int32_t)(b.y1 - b.y0 + 1);
    return r;
}

orc_rect orc_roi_detect_depth(const uint32_t* depth, int32_t w, int32_t h, int64_t pitch)
{
    bbox b = {INT64_MAX, INT64_MAX, -1, -1};
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x)
            if (depth[y * pitch + x] != ORC_CLEAR_DEPTH) bbox_add(&b, x, y);
    return bbox_rect(b);
}

orc_rect orc_roi_detect_rgba8(const uint32_t* color, int32_t w, int32_t h, int64_t pitch)
{
    bbox b = {INT64_MAX, INT64_MAX, -1, -1};
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x)
            if (color[y * pitch + x] != 0u) bbox_add(&b, x, y);
    return bbox_rect(b);
}

orc_rect orc_roi_detect_rgbaf(const double* rgba, int32_t w, int32_t h, int64_t pitch)
{
    bbox b = {INT64_MAX, INT64_MAX, -1, -1};
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x) {
            const double* p = rgba + 4 * (y * pitch + x);
            if (p[0] != 0.0 || p[1] != 0.0 || p[2] != 0.0 || p[3] != 0.0) bbox_add(&b, x, y);
        }
    return bbox_rect(b);
}

/* ------------------------------------------------------------------------ */
/* Per-component run-length encoding (Section 5.5.1, Enhanced RLE           */
/* Compression): every byte of the pixel record is its own stream (plane),  */
/* and the image is cut into sub-images that are compressed independently.  */
/* The thesis gives no stream format; the "RLE1" format is defined here.    */
/*                                                                          */
/* Pixel record: RGBA8 colour bytes R, G, B, A (planes 0..3), then, when a  */
/* depth buffer is given, depth bytes from least to most significant        */
/* (planes 4..7). Pixels are taken row-major over the ROI.                  */
/* Blocks: 4096 pixels; block b covers pixels [4096 b, 4096 b + len_b).     */
/* Runs are maximal runs of equal bytes within one plane of one block that  */
/* do not cross a multiple of 256 pixels, so a run is 1..256 bytes. A token */
/* is two bytes (run length - 1, value). A plane of a block is stored as    */
/* tokens when 2 * ntokens < len_b, otherwise as its len_b raw bytes; the   */
/* decoder tells the two apart by size == len_b.                            */
/* Layout (all integers little-endian uint32):                              */
/*   [0..32)  magic 0x31454C52, roi.x, roi.y, roi.w, roi.h, nplanes,        */
/*            4096, nblocks = ceil(w h / 4096); an empty ROI is stored as   */
/*            (0, 0, 0, 0)                                                  */
/*   boff[nblocks]          payload-relative offset of block b (16-aligned) */
/*   size[nblocks][nplanes] encoded bytes of (block, plane)                 */
/*   zero bytes up to the next multiple of 16: payload start P0             */
/*   payload: per block, its planes' encodings back to back, then zero      */
/*            bytes up to a multiple of 16                                  */
/* Total = P0 + sum over blocks of align16(sum of the block's sizes).       */
/* ------------------------------------------------------------------------ */
#define RLE_MAGIC 0x31454C52u
#define RLE_BLOCK 4096
#define RLE_SEG 256

static uint64_t align16(uint64_t v) { return (v + 15u) & ~(uint64_t)15u; }

static void put32(uint8_t* p, uint32_t v)
{
    p[0] = (uint8_t)v; p[1] = (uint8_t)(v >> 8); p[2] = (uint8_t)(v >> 16); p[3] = (uint8_t)(v >> 24);
}

static uint32_t get32(const uint8_t* p)
{
    return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

static uint64_t rle_nblocks(int64_t npx) { return (uint64_t)((npx + RLE_BLOCK - 1) / RLE_BLOCK); }

static uint64_t rle_payload_start(uint64_t nblocks, int32_t nplanes)
{
    return align16(32 + 4 * nblocks * (1 + (uint64_t)nplanes));
}

uint64_t orc_rle_max_size(int32_t w, int32_t h, int32_t nplanes)
{
    const int64_t npx = (int64_t)w * h;
    const uint64_t nb = rle_nblocks(npx);
    uint64_t total = rle_payload_start(nb, nplanes);
    for (uint64_t b = 0; b < nb; ++b) {
        const int64_t len = (npx - (int64_t)b * RLE_BLOCK) < RLE_BLOCK ? (npx - (int64_t)b * RLE_BLOCK) : RLE_BLOCK;
        total += align16((uint64_t)len * nplanes);
    }
    return total;
}

/* Bit swizzling (Section 5.5.1: a preconditioner that regroups the colour */
/* bits by significance, so that per-component RLE compresses the high,     */
/* middle and low bits of all four components in separate streams). The    */
/* bit pattern is this library's own: byte j of the swizzled word holds     */
/* bits 2j+1 and 2j of R, G, B and A, in that order from its low end, i.e.  */
/* bit 2j+b of component c moves to bit 8j + 2c + b.                        */
uint32_t orc_swizzle(uint32_t rgba)
{
    uint32_t out = 0;
    for (int c = 0; c < 4; ++c)
        for (int j = 0; j < 4; ++j)
            for (int b = 0; b < 2; ++b) {
                const uint32_t bit = (rgba >> (8 * c + 2 * j + b)) & 1u;
                out |= bit << (8 * j + 2 * c + b);
            }
    return out;
}

uint32_t orc_unswizzle(uint32_t s)
{
    uint32_t out = 0;
    for (int c = 0; c < 4; ++c)
        for (int j = 0; j < 4; ++j)
            for (int b = 0; b < 2; ++b) {
                const uint32_t bit = (s >> (8 * j + 2 * c + b)) & 1u;
                out |= bit << (8 * c + 2 * j + b);
            }
    return out;
}

/* byte k of pixel q of the ROI (q row-major over the ROI) */
static uint8_t plane_byte(const uint32_t* color, const uint32_t* depth, int64_t pitch,
                          orc_rect roi, int64_t q, int k, int swizzle)
{
    const int64_t yy = q / roi.w, xx = q % roi.w;
    const int64_t off = (roi.y + yy) * pitch + (roi.x + xx);
    uint32_t word = k < 4 ? color[off] : depth[off];
    if (k < 4 && swizzle) word = orc_swizzle(word);
    return (uint8_t)(word >> (8 * (k & 3)));
}

/* Returns the stream size, or 0 if `cap` is too small or the ROI invalid. */
/* With `swizzle`, the colour words are bit-swizzled before their planes    */
/* are taken, and header word 5 carries the flag 0x100 next to nplanes.     */
uint64_t orc_rle_compress(const uint32_t* color, const uint32_t* depth, int64_t pitch,
                          orc_rect roi, int32_t swizzle, uint8_t* out, uint64_t cap)
{
    const int32_t nplanes = depth ? 8 : 4;
    if (roi.w < 0 || roi.h < 0) return 0;
    if (roi.w == 0 || roi.h == 0) { roi.x = 0; roi.y = 0; roi.w = 0; roi.h = 0; } /* canonical empty ROI */
    const int64_t npx = (int64_t)roi.w * roi.h;
    const uint64_t nb = rle_nblocks(npx);
    const uint64_t P0 = rle_payload_start(nb, nplanes);
    if (cap < orc_rle_max_size(roi.w, roi.h, nplanes)) return 0;
    memset(out, 0, P0);
    put32(out + 0, RLE_MAGIC);
    put32(out + 4, (uint32_t)roi.x); put32(out + 8, (uint32_t)roi.y);
    put32(out + 12, (uint32_t)roi.w); put32(out + 16, (uint32_t)roi.h);
    put32(out + 20, (uint32_t)nplanes | (swizzle ? 0x100u : 0u));
    put32(out + 24, RLE_BLOCK); put32(out + 28, (uint32_t)nb);
    uint8_t* boff = out + 32;
    uint8_t* sizes = out + 32 + 4 * nb;
    uint64_t pos = 0; /* payload-relative */
    uint8_t plane[RLE_BLOCK];
    for (uint64_t b = 0; b < nb; ++b) {
        const int64_t q0 = (int64_t)b * RLE_BLOCK;
        const int64_t len = (npx - q0) < RLE_BLOCK ? (npx - q0) : RLE_BLOCK;
        put32(boff + 4 * b, (uint32_t)pos);
        uint64_t block_bytes = 0;
        for (int k = 0; k < nplanes; ++k) {
            for (int64_t j = 0; j < len; ++j)
                plane[j] = plane_byte(color, depth, pitch, roi, q0 + j, k, swizzle);
            /* count maximal runs that stay inside a 256-pixel segment */
            int64_t ntok = 0;
            for (int64_t j = 0; j < len;) {
                int64_t e = j + 1;
                while (e < len && plane[e] == plane[j] && (q0 + e) % RLE_SEG != 0) ++e;
                ++ntok;
                j = e;
            }
            uint8_t* dst = out + P0 + pos + block_bytes;
            uint32_t sz;
            if (2 * ntok < len) {
                int64_t t = 0;
                for (int64_t j = 0; j < len;) {
                    int64_t e = j + 1;
                    while (e < len && plane[e] == plane[j] && (q0 + e) % RLE_SEG != 0) ++e;
                    dst[2 * t] = (uint8_t)(e - j - 1);
                    dst[2 * t + 1] = plane[j];
                    ++t;
                    j = e;
                }
                sz = (uint32_t)(2 * ntok);
            } else {
                memcpy(dst, plane, (size_t)len);
                sz = (uint32_t)len;
            }
            put32(sizes + 4 * (b * nplanes + k), sz);
            block_bytes += sz;
        }
        const uint64_t padded = align16(block_bytes);
        for (uint64_t p = block_bytes; p < padded; ++p) out[P0 + pos + p] = 0;
        pos += padded;
    }
    return P0 + pos;
}

/* Parses the header. Returns 0 and fills the outputs, or -1 if corrupt. */
int orc_rle_header(const uint8_t* in, uint64_t size, orc_rect* roi, int32_t* nplanes,
                   int32_t* swizzle, uint64_t* total)
{
    if (size < 32) return -1;
    if (get32(in) != RLE_MAGIC) return -1;
    orc_rect r;
    r.x = (int32_t)get32(in + 4); r.y = (int32_t)get32(in + 8);
    r.w = (int32_t)get32(in + 12); r.h = (int32_t)get32(in + 16);
    const uint32_t w5 = get32(in + 20);
    const uint32_t np = w5 & 0xFFu;
    if (w5 & ~0x1FFu) return -1;
    if (r.w < 0 || r.h < 0) return -1;
    if (np != 4 && np != 8) return -1;
    if (get32(in + 24) != RLE_BLOCK) return -1;
    const int64_t npx = (int64_t)r.w * r.h;
    const uint64_t nb = rle_nblocks(npx);
    if (get32(in + 28) != nb) return -1;
    const uint64_t P0 = rle_payload_start(nb, (int32_t)np);
    if (size < P0) return -1;
    uint64_t pos = 0;
    for (uint64_t b = 0; b < nb; ++b) {
        const int64_t len = (npx - (int64_t)b * RLE_BLOCK) < RLE_BLOCK ? (npx - (int64_t)b * RLE_BLOCK) : RLE_BLOCK;
        if (get32(in + 32 + 4 * b) != pos) return -1;
        uint64_t block_bytes = 0;
        for (uint32_t k = 0; k < np; ++k) {
            const uint32_t sz = get32(in + 32 + 4 * nb + 4 * (b * np + k));
            if (sz > (uint64_t)len) return -1;
            if (sz < (uint64_t)len && (sz == 0 || (sz & 1u))) return -1;
            block_bytes += sz;
        }
        pos += align16(block_bytes);
    }
    if (size < P0 + pos) return -1;
    *roi = r; *nplanes = (int32_t)np; *swizzle = (w5 >> 8) & 1; *total = P0 + pos;
    return 0;
}

/* Decodes into ROI-sized buffers (w x h, out_pitch). `out_depth` must be    */
/* given for 8-plane streams. Returns 0, or -1 if the stream is corrupt      */
/* (bad header, tables that disagree, token runs that do not add up to the  */
/* block length, a run that crosses a multiple of 256 pixels).              */
int orc_rle_decompress(const uint8_t* in, uint64_t size, uint32_t* out_color, uint32_t* out_depth,
                       int64_t out_pitch, orc_rect* roi_out)
{
    orc_rect r; int32_t np, swz; uint64_t total;
    if (orc_rle_header(in, size, &r, &np, &swz, &total) != 0) return -1;
    if (np == 8 && !out_depth) return -1;
    const int64_t npx = (int64_t)r.w * r.h;
    const uint64_t nb = rle_nblocks(npx);
    const uint64_t P0 = rle_payload_start(nb, np);
    uint8_t plane[RLE_BLOCK];
    for (uint64_t b = 0; b < nb; ++b) {
        const int64_t q0 = (int64_t)b * RLE_BLOCK;
        const int64_t len = (npx - q0) < RLE_BLOCK ? (npx - q0) : RLE_BLOCK;
        const uint8_t* src = in + P0 + get32(in + 32 + 4 * b);
        for (int32_t k = 0; k < np; ++k) {
            const uint32_t sz = get32(in + 32 + 4 * nb + 4 * (b * (uint64_t)np + k));
            if (sz == (uint64_t)len) {
                memcpy(plane, src, (size_t)len);
            } else {
                int64_t j = 0;
                for (uint32_t t = 0; t < sz / 2; ++t) {
                    const int64_t run = (int64_t)src[2 * t] + 1;
                    if (j + run > len) return -1;
                    /* runs end at multiples of 256 pixels at the latest */
                    if ((j % RLE_SEG) + run > RLE_SEG) return -1;
                    for (int64_t e = 0; e < run; ++e) plane[j + e] = src[2 * t + 1];
                    j += run;
                }
                if (j != len) return -1;
            }
            src += sz;
            for (int64_t j = 0; j < len; ++j) {
                const int64_t q = q0 + j;
                const int64_t yy = q / r.w, xx = q % r.w;
                uint32_t* word = k < 4 ? &out_color[yy * out_pitch + xx] : &out_depth[yy * out_pitch + xx];
                const int sh = 8 * (k & 3);
                *word = (*word & ~(0xFFu << sh)) | ((uint32_t)plane[j] << sh);
            }
        }
    }
    if (swz)
        for (int64_t yy = 0; yy < r.h; ++yy)
            for (int64_t xx = 0; xx < r.w; ++xx)
                out_color[yy * out_pitch + xx] = orc_unswizzle(out_color[yy * out_pitch + xx]);
    if (roi_out) *roi_out = r;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Basic 64-bit RLE (Section 5.5.1, Enhanced RLE Compression: the basic     */
/* compressor compares two RGBA8 pixels at a time, as one 64-bit token, so  */
/* it only compresses runs of equal pixel pairs). The thesis gives no       */
/* stream format; the "RL64" format is defined here, with the block and     */
/* table layout of RLE1.                                                    */
/*                                                                          */
/* Symbols: the ROI's colour words row-major, in pairs: symbol j holds      */
/* pixel 2j in its low 32 bits and pixel 2j+1 in its high 32 bits (an odd   */
/* last pixel of a block pairs with 0). With a depth buffer the depth words */
/* form a second symbol stream the same way. Blocks of 4096 pixels, i.e.    */
/* m = ceil(len / 2) symbols. Runs are maximal runs of equal symbols that   */
/* do not cross a multiple of 128 symbols (256 pixels): 1..128 symbols. A   */
/* stream of a block with R runs is stored as tokens when                   */
/* align8(R) + 8 R < 8 m: the R bytes (run length - 1), zero bytes up to a  */
/* multiple of 8, then the R run values as little-endian 64-bit words;      */
/* otherwise as its m symbols (8 m bytes). size == 8 m marks raw.           */
/* Layout: as RLE1 (header, boff[nblocks], size[nblocks][nstreams], zero    */
/* bytes to a multiple of 16, payloads padded to 16) with magic 0x34364C52  */
/* ("RL64") and header word 5 = nstreams (1: colour, 2: colour + depth).    */
/* ------------------------------------------------------------------------ */
#define RL64_MAGIC 0x34364C52u
#define RL64_SEG 128   /* symbols per 256-pixel segment */

static uint64_t align8(uint64_t v) { return (v + 7u) & ~(uint64_t)7u; }

static void put64(uint8_t* p, uint64_t v)
{
    for (int i = 0; i < 8; ++i) p[i] = (uint8_t)(v >> (8 * i));
}

static uint64_t get64(const uint8_t* p)
{
    uint64_t v = 0;
    for (int i = 0; i < 8; ++i) v |= (uint64_t)p[i] << (8 * i);
    return v;
}

static int64_t blk_len(int64_t npx, uint64_t b)
{
    const int64_t rest = npx - (int64_t)b * RLE_BLOCK;
    return rest < RLE_BLOCK ? rest : RLE_BLOCK;
}

uint64_t orc_rle64_max_size(int32_t w, int32_t h, int32_t nstreams)
{
    const int64_t npx = (int64_t)w * h;
    const uint64_t nb = rle_nblocks(npx);
    uint64_t total = rle_payload_start(nb, nstreams);
    for (uint64_t b = 0; b < nb; ++b)
        total += align16(8 * (uint64_t)nstreams * (uint64_t)((blk_len(npx, b) + 1) / 2));
    return total;
}

/* symbol j of stream k (0 colour, 1 depth) of the block starting at pixel q0 */
static uint64_t rl64_symbol(const uint32_t* color, const uint32_t* depth, int64_t pitch,
                            orc_rect roi, int64_t q0, int64_t len, int k, int64_t j)
{
    const uint32_t* src = k == 0 ? color : depth;
    uint64_t v = 0;
    for (int half = 0; half < 2; ++half) {
        const int64_t p = 2 * j + half;   /* block-relative pixel */
        if (p >= len) break;              /* the odd last pixel pairs with 0 */
        const int64_t q = q0 + p;
        const int64_t yy = q / roi.w, xx = q % roi.w;
        v |= (uint64_t)src[(roi.y + yy) * pitch + (roi.x + xx)] << (32 * half);
    }
    return v;
}

/* Returns the stream size, or 0 if `cap` is too small or the ROI invalid. */
uint64_t orc_rle64_compress(const uint32_t* color, const uint32_t* depth, int64_t pitch,
                            orc_rect roi, uint8_t* out, uint64_t cap)
{
    const int32_t ns = depth ? 2 : 1;
    if (roi.w < 0 || roi.h < 0) return 0;
    if (roi.w == 0 || roi.h == 0) { roi.x = 0; roi.y = 0; roi.w = 0; roi.h = 0; }
    const int64_t npx = (int64_t)roi.w * roi.h;
    const uint64_t nb = rle_nblocks(npx);
    const uint64_t P0 = rle_payload_start(nb, ns);
    if (cap < orc_rle64_max_size(roi.w, roi.h, ns)) return 0;
    memset(out, 0, P0);
    put32(out + 0, RL64_MAGIC);
    put32(out + 4, (uint32_t)roi.x); put32(out + 8, (uint32_t)roi.y);
    put32(out + 12, (uint32_t)roi.w); put32(out + 16, (uint32_t)roi.h);
    put32(out + 20, (uint32_t)ns);
    put32(out + 24, RLE_BLOCK); put32(out + 28, (uint32_t)nb);
    uint8_t* boff = out + 32;
    uint8_t* sizes = out + 32 + 4 * nb;
    uint64_t pos = 0;
    static uint64_t sym[RLE_BLOCK / 2];
    for (uint64_t b = 0; b < nb; ++b) {
        const int64_t q0 = (int64_t)b * RLE_BLOCK;
        const int64_t len = blk_len(npx, b);
        const int64_t m = (len + 1) / 2;
        put32(boff + 4 * b, (uint32_t)pos);
        uint64_t block_bytes = 0;
        for (int k = 0; k < ns; ++k) {
            for (int64_t j = 0; j < m; ++j) sym[j] = rl64_symbol(color, depth, pitch, roi, q0, len, k, j);
            /* runs of equal symbols inside a 128-symbol segment */
            int64_t R = 0;
            for (int64_t j = 0; j < m;) {
                int64_t e = j + 1;
                while (e < m && sym[e] == sym[j] && e % RL64_SEG != 0) ++e;
                ++R;
                j = e;
            }
            uint8_t* dst = out + P0 + pos + block_bytes;
            uint32_t sz;
            if (align8((uint64_t)R) + 8 * (uint64_t)R < 8 * (uint64_t)m) {
                const uint64_t vals = align8((uint64_t)R);
                int64_t t = 0;
                for (int64_t j = 0; j < m;) {
                    int64_t e = j + 1;
                    while (e < m && sym[e] == sym[j] && e % RL64_SEG != 0) ++e;
                    dst[t] = (uint8_t)(e - j - 1);
                    put64(dst + vals + 8 * t, sym[j]);
                    ++t;
                    j = e;
                }
                for (uint64_t p = (uint64_t)R; p < vals; ++p) dst[p] = 0;
                sz = (uint32_t)(vals + 8 * (uint64_t)R);
            } else {
                for (int64_t j = 0; j < m; ++j) put64(dst + 8 * j, sym[j]);
                sz = (uint32_t)(8 * m);
            }
            put32(sizes + 4 * (b * ns + k), sz);
            block_bytes += sz;
        }
        const uint64_t padded = align16(block_bytes);
        for (uint64_t p = block_bytes; p < padded; ++p) out[P0 + pos + p] = 0;
        pos += padded;
    }
    return P0 + pos;
}

/* Decodes an RL64 stream into ROI-sized buffers (w x h, out_pitch);        */
/* out_depth is needed for two-stream streams. Returns 0, or -1 if the      */
/* stream is corrupt: a bad header, tables that disagree, runs that do not  */
/* add up to the block's symbols or cross a multiple of 128 symbols, a      */
/* token size that does not match its run count, nonzero padding bytes, or  */
/* a nonzero partner of an odd last pixel.                                   */
int orc_rle64_decompress(const uint8_t* in, uint64_t size, uint32_t* out_color,
                         uint32_t* out_depth, int64_t out_pitch, orc_rect* roi_out)
{
    if (size < 32 || get32(in) != RL64_MAGIC) return -1;
    orc_rect r;
    r.x = (int32_t)get32(in + 4); r.y = (int32_t)get32(in + 8);
    r.w = (int32_t)get32(in + 12); r.h = (int32_t)get32(in + 16);
    const uint32_t ns = get32(in + 20);
    if (r.w < 0 || r.h < 0 || (ns != 1 && ns != 2) || get32(in + 24) != RLE_BLOCK) return -1;
    const int64_t npx = (int64_t)r.w * r.h;
    const uint64_t nb = rle_nblocks(npx);
    if (get32(in + 28) != nb) return -1;
    const uint64_t P0 = rle_payload_start(nb, (int32_t)ns);
    if (size < P0) return -1;
    if (ns == 2 && !out_depth) return -1;
    static uint64_t sym[RLE_BLOCK / 2];
    uint64_t pos = 0;
    for (uint64_t b = 0; b < nb; ++b) {
        const int64_t q0 = (int64_t)b * RLE_BLOCK;
        const int64_t len = blk_len(npx, b);
        const int64_t m = (len + 1) / 2;
        if (get32(in + 32 + 4 * b) != pos) return -1;
        uint64_t block_bytes = 0;
        for (uint32_t k = 0; k < ns; ++k) {
            const uint64_t sz = get32(in + 32 + 4 * nb + 4 * (b * ns + k));
            if (P0 + pos + block_bytes + sz > size) return -1;
            const uint8_t* src = in + P0 + pos + block_bytes;
            if (sz > 8 * (uint64_t)m) return -1;
            if (sz == 8 * (uint64_t)m) {
                for (int64_t j = 0; j < m; ++j) sym[j] = get64(src + 8 * j);
            } else {
                /* run lengths until the block's symbols are covered */
                int64_t j = 0, t = 0;
                while (j < m) {
                    if ((uint64_t)t >= sz) return -1;
                    const int64_t run = (int64_t)src[t] + 1;
                    if (j + run > m || (j % RL64_SEG) + run > RL64_SEG) return -1;
                    j += run;
                    ++t;
                }
                const uint64_t vals = align8((uint64_t)t);
                if (sz != vals + 8 * (uint64_t)t) return -1;
                for (uint64_t p = (uint64_t)t; p < vals; ++p)
                    if (src[p] != 0) return -1;
                j = 0;
                for (int64_t u = 0; u < t; ++u) {
                    const int64_t run = (int64_t)src[u] + 1;
                    const uint64_t v = get64(src + vals + 8 * u);
                    for (int64_t e = 0; e < run; ++e) sym[j + e] = v;
                    j += run;
                }
            }
            if ((len & 1) && (sym[m - 1] >> 32) != 0) return -1;
            uint32_t* dst = k == 0 ? out_color : out_depth;
            for (int64_t p = 0; p < len; ++p) {
                const int64_t q = q0 + p;
                const int64_t yy = q / r.w, xx = q % r.w;
                dst[yy * out_pitch + xx] = (uint32_t)(sym[p / 2] >> (32 * (p & 1)));
            }
            block_bytes += sz;
        }
        const uint64_t padded = align16(block_bytes);
        if (P0 + pos + padded > size) return -1;
        for (uint64_t p = block_bytes; p < padded; ++p)
            if (in[P0 + pos + p] != 0) return -1;
        pos += padded;
    }
    if (roi_out) *roi_out = r;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Subpixel compositing (Section 4.2.3, Subpixel: the default compositing   */
/* accumulates and averages all the computed fragments of a pixel; it       */
/* reuses the parallel compositing of sort-last rendering except for this   */
/* combination step). Readings: each of the n sources supplies one sample   */
/* per pixel, transparent black (0) where the pixel lies outside its ROI;   */
/* an RGBA8 channel is the integer mean rounded half up:                    */
/*     out = floor((sum + floor(n / 2)) / n).                               */
/* ------------------------------------------------------------------------ */
void orc_composite_average_rgba8(int32_t n, const uint32_t* const* color, const int64_t* pitch,
                                 const orc_rect* roi, orc_rect viewport, uint32_t* out,
                                 int64_t out_pitch)
{
    for (int64_t v = 0; v < viewport.h; ++v) {
        for (int64_t u = 0; u < viewport.w; ++u) {
            const int64_t X = viewport.x + u, Y = viewport.y + v;
            uint64_t sum[4] = {0, 0, 0, 0};
            for (int32_t i = 0; i < n; ++i) {
                if (!in_rect(roi[i], X, Y)) continue;
                const uint32_t c = color[i][(Y - roi[i].y) * pitch[i] + (X - roi[i].x)];
                for (int k = 0; k < 4; ++k) sum[k] += (c >> (8 * k)) & 0xFFu;
            }
            uint32_t res = 0;
            if (n > 0)
                for (int k = 0; k < 4; ++k) {
                    const uint64_t mean = (sum[k] + (uint64_t)(n / 2)) / (uint64_t)n;
                    res |= (uint32_t)mean << (8 * k);
                }
            out[v * out_pitch + u] = res;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Pixel-compound assembly (Section 4.2.2, Pixel: sources render            */
/* interleaved pixels given by a pixel kernel, its 2D size and the 2D       */
/* offset of the source inside it; the destination puts every pixel back). */
/* Source i holds the destination pixels (vx + ox_i + kx u, vy + oy_i +     */
/* ky v) at (u, v). Readings: a destination pixel whose offset class no     */
/* source has gets 0; if several sources share a class, the lowest index   */
/* wins.                                                                    */
/* ------------------------------------------------------------------------ */
void orc_assemble_pixels(int32_t n, const uint32_t* const* color, const int64_t* pitch,
                         const int32_t* offx, const int32_t* offy, int32_t kx, int32_t ky,
                         orc_rect viewport, uint32_t* out, int64_t out_pitch)
{
    for (int64_t v = 0; v < viewport.h; ++v) {
        for (int64_t u = 0; u < viewport.w; ++u) {
            uint32_t val = 0;
            for (int32_t i = 0; i < n; ++i) {
                if (u % kx == offx[i] && v % ky == offy[i]) {
                    val = color[i][(v / ky) * pitch[i] + (u / kx)];
                    break;
                }
            }
            out[v * out_pitch + u] = val;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* ROI with holes (Section 5.3: analysing the framebuffer also detects      */
/* holes in the rendered area). Reading: the image is cut into cells of     */
/* cw x ch pixels (the last row and column of cells may be smaller); a      */
/* cell is occupied (1) when any of its pixels holds data under the same    */
/* emptiness test as the bounding box, else 0. `mode`: 0 depth != clear,    */
/* 1 RGBA8 word != 0, 2 float RGBA (passed as double) any channel != 0.     */
/* grid: gh x gw bytes, row-major, gw = ceil(w / cw), gh = ceil(h / ch).    */
/* ------------------------------------------------------------------------ */
void orc_roi_grid(int32_t mode, const void* data, int32_t w, int32_t h, int64_t pitch,
                  int32_t cw, int32_t ch, uint8_t* grid)
{
    const int64_t gw = (w + cw - 1) / cw, gh = (h + ch - 1) / ch;
    for (int64_t i = 0; i < gw * gh; ++i) grid[i] = 0;
    for (int64_t y = 0; y < h; ++y)
        for (int64_t x = 0; x < w; ++x) {
            int full = 0;
            if (mode == 0) full = ((const uint32_t*)data)[y * pitch + x] != ORC_CLEAR_DEPTH;
            else if (mode == 1) full = ((const uint32_t*)data)[y * pitch + x] != 0u;
            else {
                const double* p = (const double*)data + 4 * (y * pitch + x);
                full = p[0] != 0.0 || p[1] != 0.0 || p[2] != 0.0 || p[3] != 0.0;
            }
            if (full) grid[(y / ch) * gw + (x / cw)] = 1;
        }
}

/* ------------------------------------------------------------------------ */
/* ROI with holes as rectangles (Section 5.3, Region of Interest: analysing */
/* the framebuffer also finds the holes in the rendered area). The thesis   */
/* says no more; the reading used here: the occupied cells of a cell grid   */
/* (orc_roi_grid) are covered by disjoint rectangles, built row by row of   */
/* cells. A row's maximal runs of occupied cells are taken left to right;   */
/* a run whose first and last cell equal those of a run of the row above    */
/* extends that run's rectangle by one row, any other run starts a new      */
/* rectangle. Rectangles are numbered in the order they start. With more    */
/* than max_rects of them the image gets one rectangle, the bounding box of */
/* its occupied cells. Rectangles are returned in pixels, clipped to the    */
/* w x h image: (x, y, w, h) at rects[4 k]. Returns the count.              */
/* ------------------------------------------------------------------------ */
int32_t orc_roi_rects(const uint8_t* grid, int32_t gw, int32_t gh, int32_t cw, int32_t ch,
                      int32_t w, int32_t h, int32_t max_rects, int32_t* rects)
{
    /* rectangles in cells: c0, r0, c1, r1 (half-open), at most gw * gh */
    int32_t n = 0, cap = gw * gh > 0 ? gw * gh : 1;
    int32_t* rc = (int32_t*)malloc(sizeof(int32_t) * 4 * (size_t)cap);
    int32_t* above = (int32_t*)malloc(sizeof(int32_t) * (size_t)(gw > 0 ? gw : 1));   /* rect of the run starting at c in the row above, or -1 */
    int32_t* here = (int32_t*)malloc(sizeof(int32_t) * (size_t)(gw > 0 ? gw : 1));
    for (int32_t c = 0; c < gw; ++c) above[c] = -1;
    for (int32_t r = 0; r < gh; ++r) {
        for (int32_t c = 0; c < gw; ++c) here[c] = -1;
        int32_t c = 0;
        while (c < gw) {
            if (!grid[(int64_t)r * gw + c]) { ++c; continue; }
            int32_t e = c;
            while (e < gw && grid[(int64_t)r * gw + e]) ++e;   /* the run is [c, e) */
            int32_t k = above[c];
            if (k >= 0 && rc[4 * k + 2] == e) {
                rc[4 * k + 3] = r + 1;
            } else {
                k = n++;
                rc[4 * k + 0] = c; rc[4 * k + 1] = r; rc[4 * k + 2] = e; rc[4 * k + 3] = r + 1;
            }
            here[c] = k;
            c = e;
        }
        int32_t* t = above; above = here; here = t;
    }
    int32_t out = n;
    if (n > max_rects) {
        /* the bounding box of the occupied cells */
        int32_t c0 = gw, r0 = gh, c1 = 0, r1 = 0;
        for (int32_t k = 0; k < n; ++k) {
            if (rc[4 * k + 0] < c0) c0 = rc[4 * k + 0];
            if (rc[4 * k + 1] < r0) r0 = rc[4 * k + 1];
            if (rc[4 * k + 2] > c1) c1 = rc[4 * k + 2];
            if (rc[4 * k + 3] > r1) r1 = rc[4 * k + 3];
        }
        rc[0] = c0; rc[1] = r0; rc[2] = c1; rc[3] = r1;
        out = 1;
    }
    for (int32_t k = 0; k < out; ++k) {
        const int32_t x0 = rc[4 * k + 0] * cw, y0 = rc[4 * k + 1] * ch;
        const int32_t x1 = rc[4 * k + 2] * cw < w ? rc[4 * k + 2] * cw : w;
        const int32_t y1 = rc[4 * k + 3] * ch < h ? rc[4 * k + 3] * ch : h;
        rects[4 * k + 0] = x0; rects[4 * k + 1] = y0;
        rects[4 * k + 2] = x1 - x0; rects[4 * k + 3] = y1 - y0;
    }
    free(rc); free(above); free(here);
    return out;
}
