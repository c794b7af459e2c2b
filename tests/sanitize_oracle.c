/*
 * Exercises every function of oracle/oracle.c on small seeded inputs, for a
 * build with AddressSanitizer and UndefinedBehaviorSanitizer (see
 * test_oracle_sanitized.py): round trips of both RLE formats, composites of
 * ragged placements (partly outside the viewport, empty ROIs), and the two
 * decoders on thousands of corrupted and truncated streams, which must be
 * rejected or decoded without any access outside the given buffers.
 * Exit status 0 when every round trip matched; the sanitizers abort on any
 * out-of-bounds access, leak or undefined behaviour.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct { int32_t x, y, w, h; } orc_rect;

void orc_composite_depth(int32_t n, const uint32_t* const* color, const uint32_t* const* depth,
                         const int64_t* pitch, const orc_rect* roi, orc_rect viewport,
                         uint32_t* out_color, uint32_t* out_depth, int64_t out_pitch);
void orc_composite_over(int32_t n, const double* const* layer, const int64_t* pitch,
                        const orc_rect* roi, const int32_t* order_b2f, orc_rect viewport,
                        double* out, int64_t out_pitch);
void orc_composite_over_tree(int32_t n, const double* const* layer, const int64_t* pitch,
                             const orc_rect* roi, const int32_t* order_b2f, int32_t groups,
                             orc_rect viewport, double* out, int64_t out_pitch);
void orc_composite_over_f32(int32_t n, const float* const* layer, const int64_t* pitch,
                            const orc_rect* roi, const int32_t* order_b2f, int32_t groups,
                            orc_rect viewport, float* out, int64_t out_pitch);
void orc_composite_over_backward(int32_t n, const double* const* layer, const int64_t* pitch,
                                 const orc_rect* roi, const int32_t* order_b2f,
                                 orc_rect viewport, const double* grad_out, int64_t grad_pitch,
                                 double* const* grad_layer, double* const* gscale);
orc_rect orc_roi_detect_depth(const uint32_t* depth, int32_t w, int32_t h, int64_t pitch);
orc_rect orc_roi_detect_rgba8(const uint32_t* color, int32_t w, int32_t h, int64_t pitch);
orc_rect orc_roi_detect_rgbaf(const double* rgba, int32_t w, int32_t h, int64_t pitch);
uint64_t orc_rle_max_size(int32_t w, int32_t h, int32_t nplanes);
uint64_t orc_rle_compress(const uint32_t* color, const uint32_t* depth, int64_t pitch,
                          orc_rect roi, int32_t swizzle, uint8_t* out, uint64_t cap);
int orc_rle_header(const uint8_t* in, uint64_t size, orc_rect* roi, int32_t* nplanes,
                   int32_t* swizzle, uint64_t* total);
int orc_rle_decompress(const uint8_t* in, uint64_t size, uint32_t* out_color, uint32_t* out_depth,
                       int64_t out_pitch, orc_rect* roi_out);
uint64_t orc_rle64_max_size(int32_t w, int32_t h, int32_t nstreams);
uint64_t orc_rle64_compress(const uint32_t* color, const uint32_t* depth, int64_t pitch,
                            orc_rect roi, uint8_t* out, uint64_t cap);
int orc_rle64_decompress(const uint8_t* in, uint64_t size, uint32_t* out_color,
                         uint32_t* out_depth, int64_t out_pitch, orc_rect* roi_out);
void orc_composite_average_rgba8(int32_t n, const uint32_t* const* color, const int64_t* pitch,
                                 const orc_rect* roi, orc_rect viewport, uint32_t* out,
                                 int64_t out_pitch);
void orc_assemble_pixels(int32_t n, const uint32_t* const* color, const int64_t* pitch,
                         const int32_t* offx, const int32_t* offy, int32_t kx, int32_t ky,
                         orc_rect viewport, uint32_t* out, int64_t out_pitch);
void orc_roi_grid(int32_t mode, const void* data, int32_t w, int32_t h, int64_t pitch, int32_t cw,
                  int32_t ch, uint8_t* grid);
int32_t orc_roi_rects(const uint8_t* grid, int32_t gw, int32_t gh, int32_t cw, int32_t ch,
                      int32_t w, int32_t h, int32_t max_rects, int32_t* rects);

/* splitmix64 (Steele, Lea and Flood 2014) */
static uint64_t g_state = 0x2545F4914F6CDD1Dull;
static uint64_t rnd(void) {
    uint64_t z = (g_state += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static int rndi(int lo, int hi) { return lo + (int)(rnd() % (uint64_t)(hi - lo + 1)); }

static uint32_t get32(const uint8_t* p) {
    return (uint32_t)p[0] | (uint32_t)p[1] << 8 | (uint32_t)p[2] << 16 | (uint32_t)p[3] << 24;
}

static void* xmalloc(size_t n) {
    void* p = malloc(n ? n : 1);
    if (!p) { fprintf(stderr, "out of memory\n"); exit(2); }
    return p;
}

/* An image of w x h (pitch w + pad): runs of random lengths, some noise, and
 * clear pixels (depth 0xFFFFFFFF, colour 0) around a rectangle of data. */
static void make_image(int w, int h, int pad, uint32_t** color, uint32_t** depth) {
    const int64_t pitch = w + pad;
    *color = (uint32_t*)xmalloc((size_t)(pitch * h) * 4);
    *depth = (uint32_t*)xmalloc((size_t)(pitch * h) * 4);
    const int x0 = rndi(0, w / 2), y0 = rndi(0, h / 2);
    const int x1 = rndi(x0, w), y1 = rndi(y0, h);
    uint32_t c = (uint32_t)rnd(), d = (uint32_t)rnd() >> 4;
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < pitch; ++x) {
            if (rndi(0, 9) == 0) c = (uint32_t)rnd();
            if (rndi(0, 3) == 0) d = (uint32_t)(rnd() >> 40);
            const int in = x < w && x >= x0 && x < x1 && y >= y0 && y < y1;
            (*color)[y * pitch + x] = in ? c : 0u;
            (*depth)[y * pitch + x] = in ? d : 0xFFFFFFFFu;
        }
}

static int check_rle(int w, int h, int pad, int swizzle, int with_depth) {
    uint32_t *color, *depth;
    make_image(w, h, pad, &color, &depth);
    const int64_t pitch = w + pad;
    orc_rect roi = orc_roi_detect_depth(depth, w, h, pitch);
    if (rndi(0, 2) == 0) roi = (orc_rect){0, 0, w, h};
    const int np = with_depth ? 8 : 4;
    const uint64_t cap = orc_rle_max_size(w, h, np);
    uint8_t* s = (uint8_t*)xmalloc(cap);
    const uint32_t* c0 = color + (int64_t)roi.y * pitch + roi.x;
    const uint32_t* d0 = with_depth ? depth + (int64_t)roi.y * pitch + roi.x : NULL;
    /* both compressors take the image and apply the ROI themselves */
    const uint64_t n = orc_rle_compress(color, with_depth ? depth : NULL, pitch, roi, swizzle, s, cap);
    int bad = n == 0 || n > cap;
    const int64_t npx = (int64_t)roi.w * roi.h;
    uint32_t* oc = (uint32_t*)xmalloc((size_t)npx * 4);
    uint32_t* od = (uint32_t*)xmalloc((size_t)npx * 4);
    orc_rect r2;
    if (!bad && orc_rle_decompress(s, n, oc, with_depth ? od : NULL, roi.w, &r2) != 0) bad = 1;
    for (int y = 0; !bad && y < roi.h; ++y)
        for (int x = 0; x < roi.w; ++x) {
            if (oc[y * roi.w + x] != c0[y * pitch + x]) bad = 1;
            if (with_depth && od[y * roi.w + x] != d0[y * pitch + x]) bad = 1;
        }
    /* corrupted and truncated copies: rejected or decoded, never out of bounds */
    for (int t = 0; !bad && t < 200; ++t) {
        const uint64_t len = rndi(0, 3) == 0 ? (uint64_t)rndi(0, (int)n) : n;
        uint8_t* m = (uint8_t*)xmalloc(len);
        memcpy(m, s, len);
        for (int k = rndi(1, 4); k > 0 && len > 0; --k) m[rnd() % len] ^= (uint8_t)(1u << rndi(0, 7));
        orc_rect hr; int32_t hnp, hsw; uint64_t tot;
        if (orc_rle_header(m, len, &hr, &hnp, &hsw, &tot) != 0) {
            /* rejected by the header check, before any output is written */
            if (orc_rle_decompress(m, len, oc, od, roi.w, &r2) == 0) bad = 1;
        } else if ((int64_t)hr.w * hr.h <= (1 << 22)) {
            const int64_t hp = (int64_t)hr.w * hr.h;
            uint32_t* a = (uint32_t*)xmalloc((size_t)hp * 4);
            uint32_t* b = (uint32_t*)xmalloc((size_t)hp * 4);
            (void)orc_rle_decompress(m, len, a, b, hr.w, &r2);
            free(a); free(b);
        }
        free(m);
    }
    /* RL64: the same image */
    const int ns = with_depth ? 2 : 1;
    const uint64_t cap64 = orc_rle64_max_size(w, h, ns);
    uint8_t* s64 = (uint8_t*)xmalloc(cap64);
    const uint64_t n64 = orc_rle64_compress(color, with_depth ? depth : NULL, pitch, roi, s64, cap64);
    if (!bad && (n64 == 0 || n64 > cap64)) bad = 1;
    if (!bad && orc_rle64_decompress(s64, n64, oc, with_depth ? od : NULL, roi.w, &r2) != 0) bad = 1;
    for (int y = 0; !bad && y < roi.h; ++y)
        for (int x = 0; x < roi.w; ++x) {
            if (oc[y * roi.w + x] != c0[y * pitch + x]) bad = 1;
            if (with_depth && od[y * roi.w + x] != d0[y * pitch + x]) bad = 1;
        }
    for (int t = 0; !bad && t < 200; ++t) {
        const uint64_t len = rndi(0, 3) == 0 ? (uint64_t)rndi(0, (int)n64) : n64;
        uint8_t* m = (uint8_t*)xmalloc(len);
        memcpy(m, s64, len);
        for (int k = rndi(1, 4); k > 0 && len > 0; --k) m[rnd() % len] ^= (uint8_t)(1u << rndi(0, 7));
        /* output buffers of the size the stream's header states (words 3
         * and 4, as in the RLE1 header), so that a corrupted size that
         * still passes the format checks is decoded in bounds */
        if (len >= 32) {
            const int64_t hw = (int64_t)get32(m + 12), hh = (int64_t)get32(m + 16);
            if (hw >= 0 && hh >= 0 && hw <= (1 << 20) && hh <= (1 << 20) && hw * hh <= (1 << 22)) {
                uint32_t* a = (uint32_t*)xmalloc((size_t)(hw * hh) * 4);
                uint32_t* b = (uint32_t*)xmalloc((size_t)(hw * hh) * 4);
                (void)orc_rle64_decompress(m, len, a, b, hw, &r2);
                free(a); free(b);
            }
        } else if (orc_rle64_decompress(m, len, oc, od, roi.w, &r2) == 0) {
            bad = 1;   /* shorter than a header */
        }
        free(m);
    }
    if (bad) fprintf(stderr, "RLE round trip failed: %dx%d pad %d swizzle %d depth %d\n", w, h, pad,
                     swizzle, with_depth);
    free(s); free(s64); free(oc); free(od); free(color); free(depth);
    return bad;
}

static void run_composites(void) {
    enum { N = 6 };
    const uint32_t* cc[N]; const uint32_t* dd[N]; const double* ll[N]; const float* ff[N];
    uint32_t* cbuf[N]; uint32_t* dbuf[N]; double* lbuf[N]; float* fbuf[N];
    double* gl[N]; double* gs[N];
    int64_t pitch[N]; orc_rect roi[N]; int32_t order[N], offx[N], offy[N];
    const orc_rect vp = {3, 2, 37, 29};
    for (int i = 0; i < N; ++i) {
        const int w = rndi(0, 45), h = rndi(0, 40);
        pitch[i] = w + rndi(0, 3);
        roi[i] = (orc_rect){rndi(-10, 40), rndi(-10, 30), w, h};
        if (i == 2) roi[i].w = 0;   /* an empty contributor */
        make_image(w > 0 ? w : 1, h > 0 ? h : 1, (int)(pitch[i] - w) + (w > 0 ? 0 : 1), &cbuf[i], &dbuf[i]);
        const int64_t np = pitch[i] * (h > 0 ? h : 1);
        lbuf[i] = (double*)xmalloc((size_t)np * 4 * sizeof(double));
        fbuf[i] = (float*)xmalloc((size_t)np * 4 * sizeof(float));
        gl[i] = (double*)xmalloc((size_t)np * 4 * sizeof(double));
        gs[i] = (double*)xmalloc((size_t)np * 4 * sizeof(double));
        for (int64_t p = 0; p < np; ++p) {
            const double a = (double)(rnd() % 1000) / 1000.0;
            for (int k = 0; k < 3; ++k) lbuf[i][4 * p + k] = a * (double)(rnd() % 1000) / 1000.0;
            lbuf[i][4 * p + 3] = a;
            for (int k = 0; k < 4; ++k) fbuf[i][4 * p + k] = (float)lbuf[i][4 * p + k];
        }
        cc[i] = cbuf[i]; dd[i] = dbuf[i]; ll[i] = lbuf[i]; ff[i] = fbuf[i];
        order[i] = (i * 5 + 3) % N;
        offx[i] = i % 2; offy[i] = i / 2 % 3;
    }
    const int64_t op = vp.w + 2;
    uint32_t* oc = (uint32_t*)xmalloc((size_t)(op * vp.h) * 4);
    uint32_t* od = (uint32_t*)xmalloc((size_t)(op * vp.h) * 4);
    double* o = (double*)xmalloc((size_t)(op * vp.h) * 4 * sizeof(double));
    float* of = (float*)xmalloc((size_t)(op * vp.h) * 4 * sizeof(float));
    double* g = (double*)xmalloc((size_t)(op * vp.h) * 4 * sizeof(double));
    for (int64_t p = 0; p < op * vp.h * 4; ++p) g[p] = (double)(rnd() % 2001) / 1000.0 - 1.0;
    orc_composite_depth(N, cc, dd, pitch, roi, vp, oc, od, op);
    orc_composite_over(N, ll, pitch, roi, order, vp, o, op);
    orc_composite_over_tree(N, ll, pitch, roi, order, 4, vp, o, op);
    orc_composite_over_f32(N, ff, pitch, roi, order, 1, vp, of, op);
    orc_composite_over_f32(N, ff, pitch, roi, order, 2, vp, of, op);
    orc_composite_over_backward(N, ll, pitch, roi, order, vp, g, op, gl, gs);
    orc_composite_average_rgba8(N, cc, pitch, roi, vp, oc, op);
    {
        /* assembly: each source covers every kx-th column and ky-th row */
        const int kx = 2, ky = 3;
        const uint32_t* src[N];
        int64_t sp[N];
        uint32_t* sb[N];
        for (int i = 0; i < N; ++i) {
            const int sw = (vp.w + kx - 1) / kx, sh = (vp.h + ky - 1) / ky;
            sp[i] = sw;
            sb[i] = (uint32_t*)xmalloc((size_t)(sw * sh) * 4);
            for (int64_t p = 0; p < (int64_t)sw * sh; ++p) sb[i][p] = (uint32_t)rnd();
            src[i] = sb[i];
        }
        orc_assemble_pixels(N, src, sp, offx, offy, kx, ky, vp, oc, op);
        for (int i = 0; i < N; ++i) free(sb[i]);
    }
    for (int i = 0; i < N; ++i) {
        free(cbuf[i]); free(dbuf[i]); free(lbuf[i]); free(fbuf[i]); free(gl[i]); free(gs[i]);
    }
    free(oc); free(od); free(o); free(of); free(g);
}

static void run_roi(void) {
    for (int t = 0; t < 20; ++t) {
        const int w = rndi(1, 70), h = rndi(1, 50);
        uint32_t *c, *d;
        make_image(w, h, t % 3, &c, &d);
        const int64_t pitch = w + t % 3;
        (void)orc_roi_detect_depth(d, w, h, pitch);
        (void)orc_roi_detect_rgba8(c, w, h, pitch);
        double* f = (double*)xmalloc((size_t)(pitch * h) * 4 * sizeof(double));
        for (int64_t p = 0; p < pitch * h; ++p)
            for (int k = 0; k < 4; ++k) f[4 * p + k] = c[p] ? 0.5 : 0.0;
        (void)orc_roi_detect_rgbaf(f, w, h, pitch);
        const int cw = rndi(1, 9), ch = rndi(1, 9);
        const int gw = (w + cw - 1) / cw, gh = (h + ch - 1) / ch;
        uint8_t* grid = (uint8_t*)xmalloc((size_t)(gw * gh));
        orc_roi_grid(0, d, w, h, pitch, cw, ch, grid);
        orc_roi_grid(1, c, w, h, pitch, cw, ch, grid);
        int32_t rects[64 * 4];
        (void)orc_roi_rects(grid, gw, gh, cw, ch, w, h, 1 + t % 8, rects);
        (void)orc_roi_rects(grid, gw, gh, cw, ch, w, h, 64, rects);
        free(grid); free(f); free(c); free(d);
    }
}

int main(void) {
    int bad = 0;
    const int sizes[][2] = {{1, 1}, {7, 3}, {64, 64}, {130, 70}, {4097, 2}, {300, 301}, {17, 1}};
    for (size_t i = 0; i < sizeof sizes / sizeof sizes[0]; ++i)
        for (int v = 0; v < 4; ++v)
            bad |= check_rle(sizes[i][0], sizes[i][1], v % 3, v & 1, v >> 1 & 1);
    for (int t = 0; t < 4; ++t) run_composites();
    run_roi();
    printf("sanitized oracle run: %s\n", bad ? "MISMATCH" : "ok");
    return bad;
}
