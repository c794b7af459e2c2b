// Parts shared by the run-length codecs (the per-component RLE1 codec and
// the basic 64-bit RL64 codec of Section 5.5.1, Enhanced RLE Compression):
// block geometry, the slot tickets and decoupled look-back of the
// single-pass compressors, the pixel loads of a block, and wave / workgroup
// scans. Streams of both codecs share one layout (header, block offsets,
// per-block sizes, 16-byte aligned payloads).
#pragma once

#include <atomic>

#include "cmp_internal.hpp"

namespace cmp {

constexpr uint32_t kRleMagic = 0x31454C52u;
constexpr int kBlock = 4096;
constexpr int kSeg = 256;
constexpr int kPxPerLane = 16;
constexpr int kRleMax = 64;
constexpr int kStage = 8 * kBlock + 16;

__host__ __device__ inline int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }
__host__ __device__ inline uint64_t align16(uint64_t v) { return (v + 15u) & ~(uint64_t)15u; }
__host__ __device__ inline uint64_t rle_nblocks(int64_t npx) {
  return (uint64_t)((npx + kBlock - 1) / kBlock);
}
__host__ __device__ inline uint64_t rle_p0(uint64_t nb, int np) {
  return align16(32 + 4 * nb * (1 + (uint64_t)np));
}

// ------------------------------------------------------------- helpers
__device__ __forceinline__ uint64_t wave_incl_scan(uint64_t v) {
  // DPP inside rows of 16 lanes (both halves of the word, then a 64-bit
  // add), then the row totals of the lower rows read lane by lane
#pragma unroll
  for (int d = 1; d < 16; d <<= 1) {
    uint32_t lo = 0, hi = 0;
    switch (d) {
      case 1: lo = __builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);
              hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0x111, 0xF, 0xF, true); break;
      case 2: lo = __builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);
              hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0x112, 0xF, 0xF, true); break;
      case 4: lo = __builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);
              hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0x114, 0xF, 0xF, true); break;
      default: lo = __builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);
               hi = __builtin_amdgcn_update_dpp(0, (int)(v >> 32), 0x118, 0xF, 0xF, true); break;
    }
    v += ((uint64_t)hi << 32) | lo;
  }
  const uint32_t vlo = (uint32_t)v, vhi = (uint32_t)(v >> 32);
  const uint64_t r0 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)vhi, 15) << 32) |
                      (uint32_t)__builtin_amdgcn_readlane((int)vlo, 15);
  const uint64_t r1 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)vhi, 31) << 32) |
                      (uint32_t)__builtin_amdgcn_readlane((int)vlo, 31);
  const uint64_t r2 = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane((int)vhi, 47) << 32) |
                      (uint32_t)__builtin_amdgcn_readlane((int)vlo, 47);
  const int row = (threadIdx.x % kWave) >> 4;
  return v + (row >= 1 ? r0 : 0ull) + (row >= 2 ? r1 : 0ull) + (row >= 3 ? r2 : 0ull);
}

// Exclusive workgroup scan of two packed words (4 x 16-bit counters each);
// also returns the workgroup totals. `sh` holds 8 words; ends with a barrier.
__device__ __forceinline__ void block_scan2(uint64_t a, uint64_t b, uint64_t& ea, uint64_t& eb,
                                            uint64_t& ta, uint64_t& tb, uint64_t* sh) {
  const uint64_t ia = wave_incl_scan(a), ib = wave_incl_scan(b);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == kWave - 1) {
    sh[wave] = ia;
    sh[4 + wave] = ib;
  }
  __syncthreads();
  uint64_t pa = 0, pb = 0;
  ta = 0;
  tb = 0;
#pragma unroll
  for (int w = 0; w < kThreads / kWave; ++w) {
    if (w < wave) {
      pa += sh[w];
      pb += sh[4 + w];
    }
    ta += sh[w];
    tb += sh[4 + w];
  }
  ea = pa + ia - a;
  eb = pb + ib - b;
  __syncthreads();
}

__device__ __forceinline__ uint32_t field16(uint64_t lo, uint64_t hi, int k) {
  const uint64_t w = k < 4 ? lo : hi;
  return (uint32_t)((w >> (16 * (k & 3))) & 0xFFFFu);
}

__device__ __forceinline__ uint32_t byte_of(uint32_t w, int k) { return (w >> (8 * (k & 3))) & 0xFFu; }

// Bit swizzling (Section 5.5.1): bit 2j+b of component c moves to bit
// 8j + 2c + b, i.e. the 4x4 matrix of 2-bit fields (component, significance
// group) is transposed. Two delta swaps do the transpose: the off-diagonal
// 2x2 blocks, then the off-diagonal fields inside each block. A transpose is
// its own inverse, so the same function undoes it.
__device__ __forceinline__ uint32_t swizzle_bits(uint32_t x) {
  uint32_t t = ((x >> 12) ^ x) & 0x0000F0F0u;
  x ^= t ^ (t << 12);
  t = ((x >> 6) ^ x) & 0x00CC00CCu;
  x ^= t ^ (t << 6);
  return x;
}

// Clamp a device ROI to a W x H image.
__device__ __forceinline__ void clamp_roi(const int32_t* roi_dev, int s, int W, int H, int& x,
                                          int& y, int& w, int& h) {
  if (!roi_dev) {
    x = 0; y = 0; w = W; h = H;
    return;
  }
  const int4 r = reinterpret_cast<const int4*>(roi_dev)[s];
  x = min(max(r.x, 0), W);
  y = min(max(r.y, 0), H);
  w = min(max(r.z, 0), W - x);
  h = min(max(r.w, 0), H - y);
  if (w == 0 || h == 0) { x = 0; y = 0; w = 0; h = 0; }
  x = uniform(x); y = uniform(y); w = uniform(w); h = uniform(h);
}

// ------------------------------------------------------------ compress
struct RleCImg {
  const uint32_t* color;
  const uint32_t* depth;   // nullptr: 4 planes
  int64_t pitch;
  int32_t W, H;            // image size
  uint8_t* out;
  int32_t flag_base;       // first look-back flag of this image
  int32_t pad;
};

struct RleCArgs {
  RleCImg im[kRleMax];
  const int32_t* roi_dev;
  uint64_t* out_size;
  int32_t* status;
  uint32_t* tickets;       // workspace: a ticket counter per image, kTicketStride words apart
  uint32_t* ctl;           // workspace: the call epoch (word 0), finished workgroups (word
                           // kCtlDone), the most flags any call has used (word kCtlHwm)
  uint64_t* flags;         // workspace: one flag per (image, block)
  int32_t nflags;          // flags of this call
  int32_t n;
  int32_t swizzle;         // CMP_RLE_SWIZZLE
  uint32_t wait_limit;     // look-back polls before a block gives up
};
static_assert(sizeof(RleCArgs) <= 4096, "kernel arguments must fit in 4 KiB");

// Workspace: the ticket counters (one per image, each on its own 128-byte
// line), control words (the call epoch on one line; the count of finished
// workgroups and the most flags any call has used on another), then the
// look-back flags. It is zero-filled once, before its first use; every call
// leaves it ready for the next: the last workgroup to finish zeroes the
// tickets and the count and advances the epoch, and a flag written by an
// earlier call (another epoch) reads as not ready, so the flags are not
// cleared, except when the 30-bit epoch wraps to 0: then the flags that
// calls have used so far are zeroed, since those of the calls 2^30 earlier
// would read as current again.
constexpr int kTicketStride = 32;
constexpr size_t kTicketBytes = (size_t)kRleMax * kTicketStride * 4;
constexpr int kCtlDone = 32;   // word index of the finished-workgroup count
constexpr int kCtlHwm = 33;    // word index of the most flags any call has used
constexpr size_t kCtlBytes = 256;
constexpr uint32_t kEpochMask = (1u << 30) - 1;

// look-back flag: epoch (30 bits) << 34 | status (2 bits) << 32 | value (32
// bits); status 0, or another call's epoch, = not ready. kPoison marks a
// block whose offset is unknown (a bounded wait gave up): neither it nor
// any later block of the image writes its payload.
constexpr uint64_t kAgg = 1, kIncl = 2, kPoison = 3;
constexpr int kLookback = 4;   // flags per lane per look-back step
__device__ __forceinline__ uint64_t mkflag(uint64_t st, uint32_t v, uint32_t ep) {
  return ((uint64_t)ep << 34) | (st << 32) | v;
}
__device__ __forceinline__ uint64_t flag_state(uint64_t f, uint32_t ep) {
  return (uint32_t)(f >> 34) == ep ? (f >> 32) & 3u : 0u;
}

// The epoch of this call (every workgroup reads it at its start; only the
// previous call's last workgroup wrote it). Loaded into a vector register
// and first used at the block's flag, so that the load's latency passes
// while the pixels arrive (made uniform there, it held up the first ticket
// draw).
__device__ __forceinline__ uint32_t call_epoch(const RleCArgs& a) {
  return __hip_atomic_load(a.ctl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) & kEpochMask;
}

// Every workgroup ends here, after its last use of the tickets and flags:
// the last one to arrive zeroes the tickets of this call's images and the
// count, raises the flag high-water mark to this call's flags, and advances
// the epoch, ready for the next call on the workspace; if the epoch wraps to
// 0 it first zeroes the flags below the high-water mark.
// Relaxed atomics suffice: every ticket access is a device-scope atomic, and
// a workgroup's last draw has returned before its count is added; the next
// call reads the epoch after this kernel has ended. (An acquire-release
// count, which writes back the L2 at each workgroup's exit, made a 16 x
// 1920x1080 compression 40% slower.)
__device__ __forceinline__ void finish_call(const RleCArgs& a, uint32_t ep) {
  __shared__ int s_last;
  __syncthreads();
  if (threadIdx.x == 0)
    s_last = __hip_atomic_fetch_add(a.ctl + kCtlDone, 1u, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  __syncthreads();
  if (s_last) {
    for (int i = threadIdx.x; i < a.n; i += kThreads)
      __hip_atomic_store(a.tickets + i * kTicketStride, 0u, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t hwm =
        max(__hip_atomic_load(a.ctl + kCtlHwm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT),
            (uint32_t)a.nflags);
    const uint32_t next = (ep + 1) & kEpochMask;
    if (next == 0) {
      for (uint32_t i = threadIdx.x; i < hwm; i += kThreads)
        __hip_atomic_store(a.flags + i, (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();   // every thread has read the high-water mark
    if (threadIdx.x == 0) {
      __hip_atomic_store(a.ctl + kCtlHwm, hwm, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(a.ctl + kCtlDone, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(a.ctl, next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}


// Byte k of each of four words, gathered into one word: one column of a
// 4x4 byte transpose (pixel-major RGBA words -> plane-major bytes).
__device__ __forceinline__ uint32_t gather_byte(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                                int k) {
  const int sh = 8 * k;
  return ((a >> sh) & 0xFFu) | (((b >> sh) & 0xFFu) << 8) | (((c >> sh) & 0xFFu) << 16) |
         (((d >> sh) & 0xFFu) << 24);
}

// Bit i (i < 4) set when byte i of x is nonzero.
__device__ __forceinline__ uint32_t nonzero_bytes(uint32_t x) {
  const uint32_t t = (((x & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | x) & 0x80808080u;
  return ((t >> 7) | (t >> 14) | (t >> 21) | (t >> 28)) & 0xFu;
}

// Bit j of the result is bit k of nibble j of the 64-bit value lo | hi << 32
// (16 nibbles): one row of a 4 x 16 bit-matrix transpose.
__device__ __forceinline__ uint32_t nibble_bits(uint32_t lo, uint32_t hi, int k) {
  uint32_t x = (lo >> k) & 0x11111111u, y = (hi >> k) & 0x11111111u;
  x = (x | (x >> 3)) & 0x03030303u;  y = (y | (y >> 3)) & 0x03030303u;
  x = (x | (x >> 6)) & 0x000F000Fu;  y = (y | (y >> 6)) & 0x000F000Fu;
  x = (x | (x >> 12)) & 0xFFu;       y = (y | (y >> 12)) & 0xFFu;
  return x | (y << 8);
}

// DPP row shift left by D lanes inside rows of 16 lanes (lane r reads lane
// r + D); lanes whose source lies outside the row keep `fill`.
template <int D>
__device__ __forceinline__ int row_shl_fill(int v, int fill) {
  return __builtin_amdgcn_update_dpp(fill, v, 0x100 + D, 0xF, 0xF, false);
}

// Inclusive scan over the 64 lanes: DPP inside rows of 16, then the row
// totals of the lower rows (read lane by lane).
__device__ __forceinline__ uint32_t wave_incl_scan32(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);
  const uint32_t r0 = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
  const uint32_t r1 = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
  const uint32_t r2 = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
  const int row = (threadIdx.x % kWave) >> 4;
  return v + (row >= 1 ? r0 : 0u) + (row >= 2 ? r1 : 0u) + (row >= 3 ? r2 : 0u);
}

// Exclusive workgroup scan of kW 32-bit words of packed counters that cannot
// overflow; also returns the totals. `sh` holds 4 * kW words; two barriers.
template <int kW>
__device__ __forceinline__ void block_scan32(const uint32_t (&v)[kW], uint32_t (&ex)[kW],
                                             uint32_t (&tot)[kW], uint32_t* sh) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  uint32_t inc[kW];
#pragma unroll
  for (int i = 0; i < kW; ++i) {
    inc[i] = wave_incl_scan32(v[i]);
    if (lane == kWave - 1) sh[4 * i + wave] = inc[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kW; ++i) {
    uint32_t p = 0, t = 0;
#pragma unroll
    for (int w = 0; w < kThreads / kWave; ++w) {
      const uint32_t x = sh[4 * i + w];
      if (w < wave) p += x;
      t += x;
    }
    ex[i] = p + inc[i] - v[i];
    tot[i] = t;
  }
  __syncthreads();
}

// One compression slot: image s, block b, and the image's clamped ROI.
struct CSlot {
  int s, b, rx, ry, rw, rh;
};

__device__ __forceinline__ CSlot compress_slot(int2 sb, const int4* t_roi) {
  CSlot c;
  c.s = uniform(sb.x);
  c.b = uniform(sb.y);
  const int4 r = t_roi[c.s];
  c.rx = uniform(r.x);
  c.ry = uniform(r.y);
  c.rw = uniform(r.z);
  c.rh = uniform(r.w);
  return c;
}

// Draws the next slot for the calling workgroup (one wave calls it; the
// result is uniform): ticket t of image s is block t of s. The blocks of an
// image are handed out in order, and only to running workgroups, so every
// block a look-back waits for belongs to a workgroup that runs; no launch
// order, grid size or other kernel on the device can stall it. A workgroup
// keeps drawing from its current image `img`; when that one is exhausted,
// the wave reads every image's counter at once and moves to the image with
// the most blocks left. Returns (-1, 0) when every image is exhausted.
// The first ticket is drawn by draw_ticket (lane 0 of the wave), so that its
// latency can pass while the wave works; draw_slot completes the draw.
__device__ __forceinline__ uint32_t draw_ticket(uint32_t* tickets, int img) {
  uint32_t t = 0;
  if (threadIdx.x % kWave == 0)
    t = __hip_atomic_fetch_add(&tickets[img * kTicketStride], 1u, __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
  return t;
}

__device__ __forceinline__ int2 draw_slot(uint32_t t0, uint32_t* tickets, const uint32_t* t_slots,
                                          int n, int& img) {
  const int lane = threadIdx.x % kWave;
  uint32_t t = t0;
  while (true) {
    t = (uint32_t)__builtin_amdgcn_readlane((int)t, 0);
    if (t < t_slots[img]) return int2{img, (int)t};
    // exhausted: the image with the most blocks left (lane i reads image i)
    uint32_t left = 0;
    if (lane < n) {
      const uint32_t c = __hip_atomic_load(&tickets[lane * kTicketStride], __ATOMIC_RELAXED,
                                           __HIP_MEMORY_SCOPE_AGENT);
      left = c < t_slots[lane] ? t_slots[lane] - c : 0u;
    }
    uint32_t best = left;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) best = max(best, (uint32_t)__shfl_xor((int)best, m));
    if (best == 0) return int2{-1, 0};
    img = uniform((int)__builtin_ctzll(__ballot(left == best)));
    t = draw_ticket(tickets, img);
  }
}

// Issues the loads of this lane's 16 pixels of slot c (zeros past the block).
__device__ __forceinline__ void compress_load(const RleCArgs& a, const CSlot& c, int tid,
                                              uint32_t (&col)[kPxPerLane],
                                              uint32_t (&dep)[kPxPerLane]) {
  const RleCImg& I = a.im[c.s];
  const int64_t npx = (int64_t)c.rw * c.rh;
  const int len = (int)imin64(kBlock, npx - (int64_t)c.b * kBlock);   // <= 0: no pixels
  const int q0 = tid * kPxPerLane;
  // the block's first pixel (uniform), then this lane's row by a 32-bit division
  const int64_t qb = (int64_t)c.b * kBlock;
  const int rw = c.rw > 0 ? c.rw : 1;
  const int yb = uniform((int)(qb / rw));
  const int xb = uniform((int)(qb - (int64_t)yb * rw));
  const uint32_t xl = (uint32_t)xb + (uint32_t)q0;
  const uint32_t dy = xl / (uint32_t)rw;
  int yy = yb + (int)dy, xx = (int)(xl - dy * (uint32_t)rw);
  const bool fast = (q0 + kPxPerLane <= len) && (xx + kPxPerLane <= rw);
  if (fast) {
    const int64_t off = (int64_t)(c.ry + yy) * I.pitch + c.rx + xx;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const u32x4 c4 = ld_u32x4(I.color + off + 4 * v);
      col[4 * v + 0] = c4.x; col[4 * v + 1] = c4.y; col[4 * v + 2] = c4.z; col[4 * v + 3] = c4.w;
      if (I.depth) {
        const u32x4 d4 = ld_u32x4(I.depth + off + 4 * v);
        dep[4 * v + 0] = d4.x; dep[4 * v + 1] = d4.y; dep[4 * v + 2] = d4.z; dep[4 * v + 3] = d4.w;
      } else {
        dep[4 * v + 0] = dep[4 * v + 1] = dep[4 * v + 2] = dep[4 * v + 3] = 0;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < kPxPerLane; ++j) {
      col[j] = 0;
      dep[j] = 0;
      if (q0 + j < len) {
        const int64_t off = (int64_t)(c.ry + yy) * I.pitch + c.rx + xx;
        col[j] = I.color[off];
        if (I.depth) dep[j] = I.depth[off];
        if (++xx == rw) { xx = 0; ++yy; }
      }
    }
  }
}


// Arguments of a decompression: the streams and their destinations.
struct RleDImg {
  const uint8_t* in;
  uint64_t in_bytes;
  uint32_t* color;
  uint32_t* depth;
  int64_t pitch;
  int32_t cap_w, cap_h;
};

struct RleDArgs {
  RleDImg im[kRleMax];
  int32_t* roi_out;
  int32_t* status;
  int32_t at_roi;   // blocks go to their ROI's position in a frame (else to its top left)
  int32_t n;
};
static_assert(sizeof(RleDArgs) <= 4096, "kernel arguments must fit in 4 KiB");

// 4 x 4 byte transpose: byte j of o_i is byte i of input j (pixel words to
// plane words and back). v_perm takes bytes 0..3 from its second operand and
// 4..7 from its first: two rounds of four.
__device__ __forceinline__ void transpose4x4(uint32_t a, uint32_t b, uint32_t c, uint32_t d,
                                             uint32_t& o0, uint32_t& o1, uint32_t& o2,
                                             uint32_t& o3) {
  const uint32_t t0 = __builtin_amdgcn_perm(b, a, 0x05010400u);   // a0 b0 a1 b1
  const uint32_t t1 = __builtin_amdgcn_perm(b, a, 0x07030602u);   // a2 b2 a3 b3
  const uint32_t t2 = __builtin_amdgcn_perm(d, c, 0x05010400u);   // c0 d0 c1 d1
  const uint32_t t3 = __builtin_amdgcn_perm(d, c, 0x07030602u);   // c2 d2 c3 d3
  o0 = __builtin_amdgcn_perm(t2, t0, 0x05040100u);                // a0 b0 c0 d0
  o1 = __builtin_amdgcn_perm(t2, t0, 0x07060302u);                // a1 b1 c1 d1
  o2 = __builtin_amdgcn_perm(t3, t1, 0x05040100u);                // a2 b2 c2 d2
  o3 = __builtin_amdgcn_perm(t3, t1, 0x07060302u);                // a3 b3 c3 d3
}

// DPP row shift right by D lanes inside rows of 16 lanes; lanes whose source
// lies outside the row read 0.
template <int D>
__device__ __forceinline__ uint32_t row_shr(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x110 + D, 0xF, 0xF, true);
}

// The slot table of a compression (all threads call it; ends before the
// caller's barrier): wave 0 clamps image i's device ROI in lane i (n <= 64,
// one load) and counts its blocks; an empty ROI still takes one slot, whose
// workgroup writes the header-only stream.
__device__ __forceinline__ void slot_table(const RleCArgs& a, int4* t_roi, uint32_t* t_slots) {
  const int tid = threadIdx.x, lane = tid % kWave;
  if (tid < kWave) {
    int lx = 0, ly = 0, lw = 0, lh = 0;
    uint32_t lslots = 0;
    if (lane < a.n) {
      const int W = a.im[lane].W, H = a.im[lane].H;
      if (a.roi_dev) {
        const int4 r = reinterpret_cast<const int4*>(a.roi_dev)[lane];
        lx = min(max(r.x, 0), W);
        ly = min(max(r.y, 0), H);
        lw = min(max(r.z, 0), W - lx);
        lh = min(max(r.w, 0), H - ly);
        if (lw == 0 || lh == 0) { lx = 0; ly = 0; lw = 0; lh = 0; }
      } else {
        lw = W; lh = H;
      }
      const uint32_t nb = (uint32_t)rle_nblocks((int64_t)lw * lh);
      lslots = nb ? nb : 1;
    }
    t_roi[lane] = int4{lx, ly, lw, lh};
    t_slots[lane] = lslots;
  }
}

// Decoupled look-back (Merrill and Garland 2016) for block b of one image,
// run by all 64 lanes of one wave: the sum of the payload sizes of blocks
// 0..b-1, read from their flags 256 at a time (4 per lane, each load
// instruction contiguous over the lanes), summing aggregates back to the
// nearest inclusive prefix. A wait that runs out of polls, or a poisoned
// prefix, sets `poisoned`. The caller publishes b's inclusive (or poisoned)
// flag with publish_incl once its own next loads are issued: a wave that
// still has that store in flight waits for its completion at its next full
// memory wait, which the loads' issue would otherwise sit behind.
__device__ __forceinline__ uint32_t lookback_excl(uint64_t* flags, int b, uint32_t padded,
                                                  uint32_t wait_limit, uint32_t ep,
                                                  bool& poisoned) {
  const int lane = threadIdx.x % kWave;
  uint32_t excl = 0;
  poisoned = false;
  if (b == 0) return 0;
  int top = b - 1;   // flag i of lane l: predecessor top - (64 i + l)
  uint32_t spins = 0;
  while (true) {
    uint64_t f[kLookback];
#pragma unroll
    for (int i = 0; i < kLookback; ++i) {
      const int p = top - (kWave * i + lane);
      f[i] = mkflag(kIncl, 0, ep);   // before block 0: an empty prefix
      if (p >= 0) f[i] = __hip_atomic_load(&flags[p], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the nearest inclusive (or poisoned) prefix, at distance 64 i + lane,
    // and whether every flag up to it is ready
    int first = kWave * kLookback;
    bool waiting = false;
#pragma unroll
    for (int i = kLookback - 1; i >= 0; --i) {
      const uint64_t st = flag_state(f[i], ep);
      const uint64_t incl = __ballot(st >= kIncl);
      if (incl) first = kWave * i + (int)__builtin_ctzll(incl);
    }
    uint64_t pz = 0;
#pragma unroll
    for (int i = 0; i < kLookback; ++i) {
      const uint64_t st = flag_state(f[i], ep);
      if (__ballot(st == 0 && kWave * i + lane <= first)) waiting = true;
      pz |= __ballot(st == kPoison && kWave * i + lane == first);
    }
    if (waiting) {
      if (++spins > wait_limit) {   // never expected: see draw_slot
        poisoned = true;
        break;
      }
      __builtin_amdgcn_s_sleep(1);
      continue;
    }
    if (pz) {   // the prefix this block needs is unknown
      poisoned = true;
      break;
    }
    uint32_t v = 0;
#pragma unroll
    for (int i = 0; i < kLookback; ++i)
      if (kWave * i + lane <= first) v += (uint32_t)f[i];
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m);
    excl += v;
    if (first < kWave * kLookback) break;
    top -= kWave * kLookback;
  }
  return excl;
}

// Block b's inclusive prefix (excl + padded), or its poisoned flag; lane 0
// of the wave that ran lookback_excl. Block 0 published its inclusive
// prefix with its size.
__device__ __forceinline__ void publish_incl(uint64_t* flags, int b, uint32_t excl,
                                             uint32_t padded, bool poisoned, uint32_t ep) {
  if (b != 0 && threadIdx.x % kWave == 0)
    __hip_atomic_store(&flags[b],
                       poisoned ? mkflag(kPoison, 0, ep) : mkflag(kIncl, excl + padded, ep),
                       __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---------------------------------------------------------------- host
// Workgroups of `kernel` that fit on the device at once, at most `cap` per
// compute unit when cap > 0 (the per-unit occupancy is cached per device).
int resident_groups(const void* kernel, std::atomic<int>* cache, int cap);
// Look-back flags a compression needs: one per block of each image's
// largest possible ROI (one for an empty image).
int64_t rle_flag_count(const cmp_image* imgs, int32_t n);
// Polls before a compressing block gives up (cmp_rle_set_wait_limit).
uint32_t rle_wait_limit();
// Caps on the compressors' workgroups per compute unit (0: as many as fit).
int rle_compress_cap();
// Validates a compression call of n images whose streams need at most
// max_size(w, h, has depth) bytes and fills `a` (all but the codec's flags)
// and `grid` (the number of slots). Enqueues nothing.
cmp_status rle_compress_prepare(const cmp_image* imgs, int32_t n, const int32_t* roi_dev,
                                uint8_t* const* out, const uint64_t* capacity,
                                uint64_t* out_size_dev, int32_t* status_dev, void* workspace,
                                size_t ws_bytes, size_t (*max_size)(int32_t, int32_t, bool),
                                RleCArgs& a, int64_t& grid);

}  // namespace cmp
