// cmp_rle_compress / cmp_rle_decompress: per-component run-length encoding of
// RGBA8 (+ depth) pixels in the RLE1 format (Section 5.5.1, Enhanced RLE
// Compression: one stream per pixel component; the image is decomposed into
// sub-images compressed in parallel). Format: see cmp.h.
//
// Compression is a single pass over the input. A workgroup owns one block of
// 4096 pixels of one image (16 consecutive pixels per lane) and encodes all
// planes of it from registers:
//   - run starts: byte != previous byte, or a multiple of 256 pixels; the
//     previous lane's last byte comes from a lane shuffle (a wave boundary is
//     always a 256-pixel boundary);
//   - token slots: a workgroup-wide exclusive scan of the per-lane run counts
//     (eight 16-bit counters packed in two 64-bit words);
//   - run ends: the next start in the lane, else a suffix minimum of the first
//     starts over the following lanes of the same 256-pixel segment;
//   - the encoded block is staged in LDS, and its payload offset comes from a
//     decoupled look-back over the blocks of the image (Merrill and Garland,
//     "Single-pass Parallel Prefix Scan with Decoupled Look-back", 2016),
//     one wave reading 64 predecessors' flags at a time.
// The grid is at most one resident wave of workgroups. Workgroups draw
// (image, block) slots from a ticket counter per image (each on its own
// cache line), so the blocks of an image go out in order and only to
// running workgroups: every block a look-back waits for is held by a
// workgroup that makes progress, whatever else runs on the device. No
// kernel clears the workspace: the last workgroup to finish zeroes the
// tickets, and the look-back flags carry a per-call epoch.
// Every workgroup derives the slot count from the device ROIs, so blocks that
// the ROIs leave out cost nothing.
//
// Decompression: a grid-stride loop over the blocks of all streams (counted
// from the stream headers); per block: table checks (uniform loads, every
// lane checks), payload to LDS, each lane's 16-byte window of every plane
// (its 16 raw bytes or its 8 tokens), one workgroup scan of the run-length
// sums of all run-coded planes, each run's value and start bit scattered
// into LDS, and per lane a fill of its 16 pixels from the last run start.
// The value entering a lane comes from a scan over its DPP row of 16 lanes:
// a row covers one 256-pixel segment, which no run crosses. Pixels are
// assembled in registers and written with 16-byte stores.
#include <string.h>

#include <atomic>
#include <mutex>

#include "rle_common.hpp"

namespace cmp {

// The tokens (run length - 1, value) of this lane's runs of one plane, from
// token index idx on; 16-bit stores when the plane starts at an even offset.
template <bool kEven>
__device__ __forceinline__ void emit_tokens(uint8_t* stage, uint32_t off, uint32_t idx, uint32_t m,
                                            const uint32_t (&pw)[4], int q0, int next_after) {
  while (m) {
    const int j = __builtin_ctz(m);
    m &= m - 1u;
    const int end = m ? q0 + __builtin_ctz(m) : next_after;
    const uint32_t w = j < 4 ? pw[0] : j < 8 ? pw[1] : j < 12 ? pw[2] : pw[3];
    const uint32_t tokv = (uint32_t)(end - q0 - j - 1) | (((w >> (8 * (j & 3))) & 0xFFu) << 8);
    if (kEven) {
      *reinterpret_cast<uint16_t*>(stage + off + 2 * idx) = (uint16_t)tokv;
    } else {
      stage[off + 2 * idx] = (uint8_t)tokv;
      stage[off + 2 * idx + 1] = (uint8_t)(tokv >> 8);
    }
    ++idx;
  }
}

// kSwizzle: the colour words are bit-swizzled before their planes are taken
// (a template parameter, so that the plain kernel carries no branch and no
// copies of the pixel registers for it).
template <bool kSwizzle>
__global__ __launch_bounds__(kThreads, 4) void rle_compress_kernel(const RleCArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t stage[kStage];
  __shared__ uint32_t sh[16];
  __shared__ uint32_t s_excl;
  __shared__ int32_t s_poison;

  // Slots: one per block of every image's ROI (an empty ROI still takes one
  // slot, whose workgroup writes the header-only stream). Wave 0 computes the
  // table (lane i: image i, n <= 64; one load) into LDS.
  __shared__ int4 t_roi[kRleMax];
  __shared__ uint32_t t_slots[kRleMax];
  __shared__ int2 s_next;   // the slot drawn for the next iteration
  slot_table(a, t_roi, t_slots);
  const uint32_t ep = call_epoch(a);
  __syncthreads();

  // Slots come from per-image tickets (draw_slot), drawn by wave 1: the
  // next slot's ticket is drawn once the current block's size is published,
  // and its pixels are loaded while the current block finishes (look-back
  // and writes). Drawing late keeps a ticket from waiting behind a whole
  // block of encoding, which its successors would wait for too (measured:
  // drawn at the start of the current block instead, 16 x 1920x1080 took
  // 63.6 us; drawn here, 59.5 us). Holding a drawn slot while finishing the
  // current one cannot deadlock: a block only waits for blocks whose tickets
  // were drawn earlier, so every chain of waits ends at a workgroup that
  // makes progress.
  int img = (int)(blockIdx.x % (uint32_t)a.n);   // wave 1's current image
  if (threadIdx.x / kWave == 1) {
    const int2 sb = draw_slot(draw_ticket(a.tickets, img), a.tickets, t_slots, a.n, img);
    if (threadIdx.x == kWave) s_next = sb;
  }
  __syncthreads();
  int2 cur = s_next;
  if (cur.x < 0) {   // uniform: nothing left for this workgroup
    finish_call(a, ep);
    return;
  }
  uint32_t col[kPxPerLane], dep[kPxPerLane];
  CSlot nx = compress_slot(cur, t_roi);
  compress_load(a, nx, threadIdx.x, col, dep);
  while (true) {
  // an opaque copy of the thread index: keeps per-lane values from being
  // hoisted out of the loop and held in registers across iterations
  int tid = threadIdx.x;
  __asm__ volatile("" : "+v"(tid));
  const int lane = tid % kWave;
  const CSlot c = nx;
  const int s = c.s, b = c.b, rx = c.rx, ry = c.ry, rw = c.rw, rh = c.rh;
  // the next slot: its ticket is drawn after the scan, the draw is
  // completed (and written to s_next) after the staging, before a barrier
  const bool drawer = tid / kWave == 1;
  uint32_t t_next = 0u;
  auto finish_draw = [&]() {
    if (drawer) {
      const int2 sb = draw_slot(t_next, a.tickets, t_slots, a.n, img);
      if (lane == 0) s_next = sb;
    }
  };
  bool more = false;
  {
    const RleCImg I = a.im[s];
    const int np = I.depth ? 8 : 4;
    const int64_t npx = (int64_t)rw * rh;
    const uint64_t nb = rle_nblocks(npx);
    const uint64_t P0 = rle_p0(nb, np);
    uint8_t* out = I.out;
    if (nb == 0) {
      if (drawer) t_next = draw_ticket(a.tickets, img);
      finish_draw();
      __syncthreads();   // s_next is written
      cur = s_next;
      more = cur.x >= 0;
      if (more) {
        nx = compress_slot(cur, t_roi);
        compress_load(a, nx, tid, col, dep);
      }
      if (tid < 8) {
        const uint32_t hdr[8] = {kRleMagic, (uint32_t)rx, (uint32_t)ry, 0u, 0u,
                                 (uint32_t)np | (kSwizzle ? 0x100u : 0u), (uint32_t)kBlock, 0u};
        reinterpret_cast<uint32_t*>(out)[tid] = hdr[tid];
      }
      if (tid == 0) a.out_size[s] = 32;
    } else {
      const int len = (int)imin64(kBlock, npx - (int64_t)b * kBlock);
      const int q0 = tid * kPxPerLane;   // block-relative first pixel
      if (kSwizzle) {
#pragma unroll
        for (int j = 0; j < kPxPerLane; ++j) col[j] = swizzle_bits(col[j]);
      }
      const uint32_t pcol = __shfl_up(col[kPxPerLane - 1], 1);
      const uint32_t pdep = __shfl_up(dep[kPxPerLane - 1], 1);
      // plane words, made when needed: byte j of pw[j / 4] is plane k of pixel j
      auto plane_words = [&](int k, uint32_t (&pw)[4]) {
        const uint32_t* w = k < 4 ? col : dep;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          pw[i] = gather_byte(w[4 * i], w[4 * i + 1], w[4 * i + 2], w[4 * i + 3], k & 3);
      };
      const bool seg_start = (tid % (kSeg / kPxPerLane)) == 0;
      const int nvalid = min(kPxPerLane, max(0, len - q0));
      const uint32_t vmask = (1u << nvalid) - 1u;

      // ---- run starts (byte != previous byte, or a segment start) and counts:
      // per pixel, which bytes differ from the previous pixel's (a nibble),
      // then the 16 nibbles transposed into one 16-bit mask per plane
      uint32_t nc_lo = 0, nc_hi = 0, nd_lo = 0, nd_hi = 0;
#pragma unroll
      for (int j = 0; j < kPxPerLane; ++j) {
        const uint32_t c = nonzero_bytes(col[j] ^ (j ? col[j - 1] : pcol));
        const uint32_t d = nonzero_bytes(dep[j] ^ (j ? dep[j - 1] : pdep));
        if (j < 8) { nc_lo |= c << (4 * j); nd_lo |= d << (4 * j); }
        else { nc_hi |= c << (4 * (j - 8)); nd_hi |= d << (4 * (j - 8)); }
      }
      uint32_t masks[8];
      uint32_t cnt[4] = {0, 0, 0, 0};
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        masks[k] = 0;
        if (k >= np) continue;
        uint32_t m = k < 4 ? nibble_bits(nc_lo, nc_hi, k) : nibble_bits(nd_lo, nd_hi, k - 4);
        if (seg_start) m |= 1u;
        m &= vmask;
        masks[k] = m;
        cnt[k >> 1] |= (uint32_t)__builtin_popcount(m) << (16 * (k & 1));
      }
      uint32_t ex[4], tot[4];
      block_scan32<4>(cnt, ex, tot, sh);
      if (drawer) t_next = draw_ticket(a.tickets, img);

      // ---- plane sizes and offsets (uniform)
      uint32_t size[8], poff[8];
      uint32_t total = 0;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        size[k] = 0;
        poff[k] = total;
        if (k >= np) continue;
        const uint32_t ntok = (tot[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
        size[k] = (2 * ntok < (uint32_t)len) ? 2 * ntok : (uint32_t)len;
        total += size[k];
      }
      const uint32_t padded = (uint32_t)align16(total);
      // the block's size is known: publish it now (block 0: as the inclusive
      // prefix), so that successors need not wait for the staging below
      uint64_t* flags = a.flags + I.flag_base;
      if (tid == 0)
        __hip_atomic_store(&flags[b], mkflag(b == 0 ? kIncl : kAgg, padded, ep), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);

      // ---- stage the encoded block in LDS
      const int seg_end = min(len, ((q0 / kSeg) + 1) * kSeg);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (k >= np) continue;
        const uint32_t m = masks[k];
        const uint32_t off = poff[k];
        uint32_t pw[4];
        plane_words(k, pw);
        if (size[k] != (uint32_t)len) {
          // a run ends at the next start: in this lane, else the first start
          // of the following lanes of the segment (a suffix minimum over the
          // lane's DPP row), else the segment end
          int fs = m ? q0 + __builtin_ctz(m) : seg_end;
          fs = min(fs, row_shl_fill<1>(fs, seg_end));
          fs = min(fs, row_shl_fill<2>(fs, seg_end));
          fs = min(fs, row_shl_fill<4>(fs, seg_end));
          fs = min(fs, row_shl_fill<8>(fs, seg_end));
          const int next_after = row_shl_fill<1>(fs, seg_end);
          const uint32_t tok0 = (ex[k >> 1] >> (16 * (k & 1))) & 0xFFFFu;
          if ((off & 1u) == 0)
            emit_tokens<true>(stage, off, tok0, m, pw, q0, next_after);
          else
            emit_tokens<false>(stage, off, tok0, m, pw, q0, next_after);
        } else if ((off & 3u) == 0 && q0 + kPxPerLane <= len) {
          // raw plane, 4-byte aligned: four 32-bit stores per lane
#pragma unroll
          for (int i = 0; i < 4; ++i)
            *reinterpret_cast<uint32_t*>(stage + off + q0 + 4 * i) = pw[i];
        } else {
#pragma unroll
          for (int j = 0; j < kPxPerLane; ++j)
            if (q0 + j < len) stage[off + q0 + j] = (uint8_t)(pw[j >> 2] >> (8 * (j & 3)));
        }
      }
      if (tid < (int)(padded - total)) stage[total + tid] = 0;
      finish_draw();
      __syncthreads();   // s_next is written
      cur = s_next;
      more = cur.x >= 0;

      // ---- decoupled look-back for the payload offset: wave 0 reads the
      // flags of 256 predecessors at once (4 per lane, each load instruction
      // contiguous over the lanes), sums the aggregates up to the nearest
      // inclusive prefix, and moves the window back if it has none
      bool lb_poison = false;
      uint32_t lb_excl = 0;
      if (tid < kWave) {
        lb_excl = lookback_excl(flags, b, padded, a.wait_limit, ep, lb_poison);
        if (lane == 0) {
          s_excl = lb_excl;
          s_poison = lb_poison ? 1 : 0;
          if (lb_poison) a.status[s] = CMP_ETIMEOUT;
        }
      }
      // the next slot's pixels go in flight: waves 1..3 during the look-back,
      // wave 0 after it (its flag loads must not wait behind these loads),
      // then wave 0 publishes the block's inclusive prefix
      if (more) {
        nx = compress_slot(cur, t_roi);
        compress_load(a, nx, tid, col, dep);
      }
      if (tid < kWave) publish_incl(flags, b, lb_excl, padded, lb_poison, ep);
      __syncthreads();
      const uint32_t excl = s_excl;
      const bool poisoned = s_poison != 0;

      // ---- tables, header, payload
      uint32_t* tbl = reinterpret_cast<uint32_t*>(out + 32);
      if (tid < np) {
        uint32_t v = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k)
          if (k == tid) v = size[k];
        tbl[nb + (uint64_t)b * np + tid] = v;
      }
      // a poisoned block's offset is unknown: its table entry is made invalid
      // (not a multiple of 16, which decompression rejects) and its payload
      // is not written
      if (tid == 0) tbl[b] = poisoned ? 0xFFFFFFFFu : excl;
      if (b == 0) {
        if (tid < 8) {
          const uint32_t hdr[8] = {kRleMagic, (uint32_t)rx, (uint32_t)ry, (uint32_t)rw,
                                   (uint32_t)rh, (uint32_t)np | (kSwizzle ? 0x100u : 0u),
                                   (uint32_t)kBlock, (uint32_t)nb};
          reinterpret_cast<uint32_t*>(out)[tid] = hdr[tid];
        }
        const uint64_t tend = 32 + 4 * nb * (1 + (uint64_t)np);
        if ((uint64_t)tid < P0 - tend) out[tend + tid] = 0;
      }
      if ((uint64_t)b == nb - 1 && tid == 0) a.out_size[s] = poisoned ? 0 : P0 + excl + padded;
      if (!poisoned) {
        u32x4* dst = reinterpret_cast<u32x4*>(out + P0 + excl);
        const u32x4* src = reinterpret_cast<const u32x4*>(stage);
        for (uint32_t i = tid; i < padded / 16; i += kThreads)
          __builtin_nontemporal_store(src[i], &dst[i]);   // streamed out, not re-read
      }
    }
  }
  __syncthreads();   // the stage, the scan words and s_next are reused by the next slot
  if (!more) break;
  }
  finish_call(a, ep);
}

// ---------------------------------------------------------- decompress
// Run-length sums of a block's planes, 21-bit fields, three per word: a
// plane of < 2048 tokens of <= 256 pixels sums to < 2^21, so no field can
// overflow into the next, whatever the stream holds.
__device__ __forceinline__ int fld_word(int k) { return k / 3; }
__device__ __forceinline__ int fld_shift(int k) { return 21 * (k % 3); }
constexpr uint64_t kFld = (1u << 21) - 1;


// Exclusive workgroup scan with a single barrier: the caller keeps a barrier
// between these reads of `sh` and its next writes.
template <int kW>
__device__ __forceinline__ void block_scan_once(const uint64_t (&v)[kW], uint64_t (&ex)[kW],
                                                uint64_t (&tot)[kW], uint64_t* sh) {
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  uint64_t inc[kW];
#pragma unroll
  for (int i = 0; i < kW; ++i) {
    inc[i] = wave_incl_scan(v[i]);
    if (lane == kWave - 1) sh[4 * i + wave] = inc[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kW; ++i) {
    uint64_t p = 0, t = 0;
#pragma unroll
    for (int w = 0; w < kThreads / kWave; ++w) {
      const uint64_t x = sh[4 * i + w];
      if (w < wave) p += x;
      t += x;
    }
    ex[i] = p + inc[i] - v[i];
    tot[i] = t;
  }
}

// 16 bytes at any byte offset `off` of a buffer whose first `end` bytes
// (end >= 16) may be read: load16_from reads them with one 16-byte load from
// src = min(off, end - 16); when the bytes run past `end`, load16_fix shifts
// the 16 bytes that end there into place (bytes past `end` read 0). Split in
// two so that a lane's loads are all issued before any of them is waited for.
// Offsets are 32-bit: a stream is smaller than 4 GiB.
__device__ __forceinline__ u32x4 load16_from(const uint8_t* base, uint32_t src) {
  u32x4 v;
  __builtin_memcpy(&v, base + src, 16);
  return v;
}
__device__ __forceinline__ u32x4 load16_fix(u32x4 v, uint32_t src, uint32_t off) {
  if (src != off) {   // rare: the last bytes of an exactly sized buffer
    uint32_t d = (uint32_t)(off - src);   // 1..15
    uint64_t lo = (uint64_t)v.x | ((uint64_t)v.y << 32), hi = (uint64_t)v.z | ((uint64_t)v.w << 32);
    if (d >= 8) { lo = hi; hi = 0; d -= 8; }
    if (d) { lo = (lo >> (8 * d)) | (hi << (64 - 8 * d)); hi >>= 8 * d; }
    v = u32x4{(uint32_t)lo, (uint32_t)(lo >> 32), (uint32_t)hi, (uint32_t)(hi >> 32)};
  }
  return v;
}

__global__ __launch_bounds__(kThreads, 4) void rle_decompress_kernel(const RleDArgs a) {
  // the bytes of each run-coded plane's runs at their start positions
  __shared__ __attribute__((aligned(16))) uint8_t vals[8 * kBlock];
  __shared__ __attribute__((aligned(16))) uint32_t starts[8][kBlock / 32];   // run-start bits
  __shared__ uint64_t sh[12];
  __shared__ int32_t s_bad[3];   // a malformed block, in rotation over consecutive slots
  // byte selectors that fill a word from its run starts: for start nibble n,
  // byte j takes the word's byte at the last start <= j, else byte 3 of the
  // previous word (v_perm numbering: 0..3 this word, 4..7 the previous one)
  __shared__ uint32_t fill_sel[16];
  const int tid = threadIdx.x;
  if (tid < 16) {
    uint32_t sel = 0;
    int last = 7;
    for (int j = 0; j < 4; ++j) {
      if ((tid >> j) & 1) last = j;
      sel |= (uint32_t)last << (8 * j);
    }
    fill_sel[tid] = sel;
  }
  reinterpret_cast<u32x4*>(&starts[0][0])[tid] = u32x4{0, 0, 0, 0};
  if (tid < 3) s_bad[tid] = 0;
  const int lane = tid % kWave;

  // Wave 0 reads and checks the header of stream i in lane i (n <= 64) into
  // LDS; a stream takes one slot per block, or one slot if it has no blocks
  // or a bad header (that slot reports the status or writes the ROI).
  __shared__ uint32_t t_hdr[kRleMax][8];
  __shared__ int32_t t_err[kRleMax];
  __shared__ uint32_t t_slots[kRleMax], t_incl[kRleMax], t_total;
  if (tid < kWave) {
    uint32_t lh[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    int lerr = 0;
    uint32_t lslots = 0;
    if (lane < a.n) {
      const RleDImg& I = a.im[lane];
      if (I.in_bytes < 32) {
        lerr = CMP_ECORRUPT;
      } else {
        const u32x4 h0 = reinterpret_cast<const u32x4*>(I.in)[0];
        const u32x4 h1 = reinterpret_cast<const u32x4*>(I.in)[1];
        lh[0] = h0.x; lh[1] = h0.y; lh[2] = h0.z; lh[3] = h0.w;
        lh[4] = h1.x; lh[5] = h1.y; lh[6] = h1.z; lh[7] = h1.w;
        const int32_t w = (int32_t)lh[3], hh = (int32_t)lh[4];
        const uint32_t np = lh[5] & 0xFFu;
        if (lh[0] != kRleMagic || w < 0 || hh < 0 || (np != 4 && np != 8) ||
            lh[6] != (uint32_t)kBlock || (lh[5] & ~0x1FFu))
          lerr = CMP_ECORRUPT;
        else if ((uint64_t)lh[7] != rle_nblocks((int64_t)w * hh))
          lerr = CMP_ECORRUPT;
        else if (I.in_bytes < rle_p0(lh[7], (int)np))
          lerr = CMP_ECORRUPT;
        else if ((np == 8 && !I.depth) ||
                 (a.at_roi ? (int32_t)lh[1] < 0 || (int32_t)lh[2] < 0 ||
                                 (int64_t)(int32_t)lh[1] + w > I.cap_w ||
                                 (int64_t)(int32_t)lh[2] + hh > I.cap_h
                           : w > I.cap_w || hh > I.cap_h))
          lerr = CMP_ENOSPC;
      }
      lslots = (lerr || lh[7] == 0) ? 1u : lh[7];
    }
    uint32_t lincl = lslots;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const uint32_t o = __shfl_up(lincl, d);
      if (lane >= d) lincl += o;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) t_hdr[lane][k] = lh[k];
    t_err[lane] = lerr;
    t_slots[lane] = lslots;
    t_incl[lane] = lincl;
    if (lane == kWave - 1) t_total = lincl;
  }
  __syncthreads();
  const uint32_t total = t_total;

  uint32_t tslot = 0;   // slots with run-coded planes so far (uniform): picks the s_bad entry
  for (uint32_t g = blockIdx.x; g < total; g += gridDim.x) {
  int tid = threadIdx.x;   // opaque per iteration (see the compressor)
  __asm__ volatile("" : "+v"(tid));
  const int lane = tid % kWave;
  const uint64_t hit = __ballot(lane < a.n && g < t_incl[lane]);
  const int s = uniform(__builtin_ctzll(hit));
  const int b = uniform((int)(g - (t_incl[s] - t_slots[s])));
  const RleDImg I = a.im[s];
  uint32_t h[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) h[k] = (uint32_t)uniform((int)t_hdr[s][k]);
  const int err = uniform(t_err[s]);
  if (err) {
    if (tid == 0) a.status[s] = err;
    continue;   // uniform; no LDS was touched in this slot
  }
  const int32_t rw = (int32_t)h[3], rh = (int32_t)h[4];
  const int np = (int)(h[5] & 0xFFu);
  const bool swizzled = (h[5] >> 8) & 1u;
  const uint64_t nb = h[7];
  if (b == 0 && a.roi_out && tid == 0)
    reinterpret_cast<int4*>(a.roi_out)[s] = int4{(int)h[1], (int)h[2], (int)h[3], (int)h[4]};
  if ((uint64_t)b >= nb) continue;   // uniform: a stream without blocks
  const int64_t npx = (int64_t)rw * rh;
  const int len = (int)imin64(kBlock, npx - (int64_t)b * kBlock);
  // block table: uniform addresses, every lane checks the same values
  // (three loads issued together; all inside the table the header check
  // found readable, since np is 4 or 8 and entry nb is the first size)
  const uint32_t* tbl = reinterpret_cast<const uint32_t*>(I.in + 32);
  const uint32_t* srow = tbl + nb + (uint64_t)b * np;
  const u32x4 s03 = ld_u32x4(srow);
  const u32x4 s47 = ld_u32x4(srow + (np == 8 ? 4 : 0));
  uint2 bo;   // boff[b], boff[b + 1]: a 4-byte aligned pair
  __builtin_memcpy(&bo, __builtin_assume_aligned(tbl + b, 4), 8);
  const uint32_t boff = bo.x;
  const uint32_t bnext = bo.y;   // the first size entry when b is the last block
  uint32_t size[8], poff[8], btotal = 0;
  int e = 0;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    size[k] = k < 4 ? s03[k] : np == 8 ? s47[k - 4] : 0u;
    if (k < np && (size[k] > (uint32_t)len ||
                   (size[k] < (uint32_t)len && (size[k] == 0 || (size[k] & 1u)))))
      e = CMP_ECORRUPT;
    poff[k] = btotal;
    btotal += size[k];
  }
  if ((boff & 15u) || (b == 0 && boff != 0)) e = CMP_ECORRUPT;
  if ((uint64_t)b + 1 < nb && (uint64_t)bnext != boff + align16(btotal)) e = CMP_ECORRUPT;
  // (a stream smaller than 4 GiB: all its offsets are 32-bit)
  if (rle_p0(nb, np) + boff + align16(btotal) > imin64((int64_t)I.in_bytes, 0xFFFFFFFFll))
    e = CMP_ECORRUPT;
  if (e) {   // uniform; no LDS was touched in this slot
    if (tid == 0) a.status[s] = e;
    continue;
  }
  uint32_t tokmask = 0;   // planes stored as runs
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k < np && size[k] != (uint32_t)len) tokmask |= 1u << k;

  // Every plane's 16-byte window of this lane, straight from the stream:
  // the raw bytes of its 16 pixels, or its tokens (run length - 1, value).
  // A run-coded plane of T tokens gives each lane tpl = ceil(T / 256) of
  // them (at most 8), so that all four waves share the scatter below. A lane
  // without bytes in a plane reads the payload's first bytes.
  const int q0 = tid * kPxPerLane;
  const uint32_t pay = (uint32_t)(rle_p0(nb, np) + boff);
  const uint32_t last16 = (uint32_t)imin64((int64_t)I.in_bytes, 0xFFFFFFFFll) - 16u;
  int tpl[8], nv[8];   // tokens per lane (uniform), this lane's tokens
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int ntok = (int)(size[k] / 2);
    tpl[k] = uniform(max(1, (ntok + kThreads - 1) / kThreads));
    nv[k] = min(tpl[k], max(0, ntok - tid * tpl[k]));
  }
  u32x4 win[8];
  uint32_t woff[8], wsrc[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const bool tok = (tokmask >> k) & 1u;
    const uint32_t lo = tok ? 2u * (uint32_t)tpl[k] * (uint32_t)tid : (uint32_t)q0;   // lane's byte
    const uint32_t base = (uint32_t)uniform((int)(pay + poff[k]));
    woff[k] = k < np && lo < size[k] ? base + lo : pay;
    wsrc[k] = min(woff[k], last16);
    win[k] = load16_from(I.in, wsrc[k]);   // every plane's load, unconditionally
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) win[k] = k < np ? load16_fix(win[k], wsrc[k], woff[k]) : u32x4{0, 0, 0, 0};
  bool bad = false;
  if (tokmask) {   // uniform
    // this slot's flag; the next one's is cleared now: its last readers (two
    // such slots ago) have all passed the previous slot's barriers
    int32_t* bad_flag = &s_bad[tslot % 3];
    if (tid == 0) s_bad[(tslot + 1) % 3] = 0;
    ++tslot;
    // start position of this lane's first token in every run-coded plane
    uint64_t v3[3] = {0, 0, 0}, ex3[3], tot3[3];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (tokmask & (1u << k)) {
        const uint32_t wv[4] = {win[k].x, win[k].y, win[k].z, win[k].w};
        uint32_t sum = (uint32_t)nv[k];   // + the (length - 1) bytes of its tokens
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const uint32_t keep = (nv[k] > 2 * i ? 0xFFu : 0u) | (nv[k] > 2 * i + 1 ? 0xFF0000u : 0u);
          sum = __builtin_amdgcn_sad_u8(wv[i] & keep, 0u, sum);
        }
        v3[fld_word(k)] |= (uint64_t)sum << fld_shift(k);
      }
    }
    block_scan_once<3>(v3, ex3, tot3, sh);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if ((tokmask & (1u << k)) && ((tot3[fld_word(k)] >> fld_shift(k)) & kFld) != (uint64_t)len)
        bad = true;   // uniform
    // each run's value at its start position, and its start bit; a run must
    // not cross a multiple of 256 pixels
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (tokmask & (1u << k)) {
        const uint32_t wv[4] = {win[k].x, win[k].y, win[k].z, win[k].w};
        uint32_t pos = (uint32_t)((ex3[fld_word(k)] >> fld_shift(k)) & kFld);
        uint8_t* vk = vals + k * kBlock;
        uint32_t* bits = starts[k];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          if (j < nv[k]) {
            const uint32_t t = wv[j >> 1] >> (16 * (j & 1));
            const uint32_t rl = (t & 0xFFu) + 1u;
            if ((pos % kSeg) + rl > (uint32_t)kSeg) bad = true;
            if (pos < (uint32_t)kBlock) {
              vk[pos] = (uint8_t)(t >> 8);
              __hip_atomic_fetch_or(&bits[pos >> 5], 1u << (pos & 31), __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_WORKGROUP);
            }
            pos += rl;
          }
        }
      }
    }
    // one vote per wave into this slot's flag, then the barrier that also
    // publishes the runs
    if (__ballot(bad) && lane == 0)
      __hip_atomic_fetch_or(bad_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    __syncthreads();
    const bool block_bad = *bad_flag != 0;
    // Expand (a malformed block skips it): a pixel takes the value of the
    // last run start at or before it. A 256-pixel segment (the 16 lanes of
    // one DPP row) starts with a run, so the value entering a lane comes from
    // a scan over its row.
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if ((tokmask & (1u << k)) && !block_bad) {
        const u32x4 d = *reinterpret_cast<const u32x4*>(vals + k * kBlock + q0);
        const uint32_t m = (starts[k][q0 >> 5] >> (q0 & 31)) & 0xFFFFu;
        const uint32_t dv[4] = {d.x, d.y, d.z, d.w};
        const int hb = 31 - __builtin_clz(m | 1u);
        const uint32_t hw = hb < 4 ? d.x : hb < 8 ? d.y : hb < 12 ? d.z : d.w;
        const uint32_t last = (hw >> (8 * (hb & 3))) & 0xFFu;
        uint32_t x = m ? (0x100u | last) : 0u;
        uint32_t y;
        y = row_shr<1>(x); if (!(x & 0x100u)) x = y;
        y = row_shr<2>(x); if (!(x & 0x100u)) x = y;
        y = row_shr<4>(x); if (!(x & 0x100u)) x = y;
        y = row_shr<8>(x); if (!(x & 0x100u)) x = y;
        // word by word: each byte from the last start in the word, else the
        // previous word's last byte (the value entering the lane for word 0)
        uint32_t o[4];
        uint32_t prev = row_shr<1>(x) << 24;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          prev = __builtin_amdgcn_perm(prev, dv[i], fill_sel[(m >> (4 * i)) & 0xFu]);
          o[i] = prev;
        }
        win[k] = u32x4{o[0], o[1], o[2], o[3]};
      }
    }
    // clear this slot's start bits: word q0 / 32 is read only by this lane
    // and its neighbour in the same wave, which have both read it
    if ((tid & 1) == 0) {
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (tokmask & (1u << k)) starts[k][q0 >> 5] = 0;
    }
    if (block_bad) {   // uniform
      if (tid == 0) a.status[s] = CMP_ECORRUPT;
      continue;
    }
  }
  // pixels from the planes: byte k of pixel 4 i + j is byte j of plane k's
  // word i (a 4 x 4 byte transpose per word of colour and of depth)
  uint32_t col[kPxPerLane], dep[kPxPerLane];
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    transpose4x4(win[0][i], win[1][i], win[2][i], win[3][i], col[4 * i], col[4 * i + 1],
                 col[4 * i + 2], col[4 * i + 3]);
    transpose4x4(win[4][i], win[5][i], win[6][i], win[7][i], dep[4 * i], dep[4 * i + 1],
                 dep[4 * i + 2], dep[4 * i + 3]);
  }
  if (swizzled) {
#pragma unroll
    for (int j = 0; j < kPxPerLane; ++j) col[j] = swizzle_bits(col[j]);
  }
  // ---- write the pixels (row-major over the ROI). A lane holds 16
  // consecutive pixels, but stores are issued so that consecutive lanes
  // write consecutive 16-byte quads: the wave's 1024 pixels are restaged
  // through LDS (the wave's eighth of every plane's run values, which only
  // this wave reads), and in store v lane i writes pixels 256 v + 4 i .. + 3
  // of the wave's range (16-byte stores at a 64-byte lane stride cost four
  // times the memory requests).
  {
    const int wave = tid / kWave;
    uint8_t* wbase = vals + (kBlock / 4) * wave;
    // quad q of the wave (pixels 4 q ..) sits in piece q / 64 at slot
    // swz(q % 64): within each group of 8 slots (128 bytes, all banks) the
    // slots rotate by the group index, so that the 8 lanes served together
    // hit 8 different 16-byte bank groups both when lane L writes its quads
    // 4 L + c and when lane i reads quad 64 v + i
    auto swz = [](int x) { return (x & ~7) | ((x + (x >> 3)) & 7); };
    uint8_t* wl = wbase + (lane / 16) * kBlock;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int slot = 16 * swz((4 * lane + c) % 64);
      *reinterpret_cast<u32x4*>(wl + slot) =
          u32x4{col[4 * c], col[4 * c + 1], col[4 * c + 2], col[4 * c + 3]};
      if (np == 8)
        *reinterpret_cast<u32x4*>(wl + 4 * kBlock + slot) =
            u32x4{dep[4 * c], dep[4 * c + 1], dep[4 * c + 2], dep[4 * c + 3]};
    }
    __builtin_amdgcn_wave_barrier();
    u32x4 cq[4], dq[4];
    const int rslot = 16 * swz(lane);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      cq[v] = *reinterpret_cast<const u32x4*>(wbase + v * kBlock + rslot);
      dq[v] = np == 8 ? *reinterpret_cast<const u32x4*>(wbase + (4 + v) * kBlock + rslot)
                      : u32x4{0, 0, 0, 0};
    }
    // the block's first pixel (uniform), then the quad's by a 32-bit division
    const int qw = (kBlock / 4) * wave + 4 * lane;   // block pixel of store 0
    // the block's origin: the frame's top left, or its ROI's position there
    const int64_t org = a.at_roi ? (int64_t)(int32_t)h[2] * I.pitch + (int32_t)h[1] : 0;
    uint32_t* const ocol = I.color + org;
    uint32_t* const odep = np == 8 ? I.depth + org : nullptr;
    const int64_t qb = (int64_t)b * kBlock;
    const int yb = uniform((int)(qb / rw)), xb = uniform((int)(qb - (int64_t)yb * rw));
    const uint32_t xl = (uint32_t)xb + (uint32_t)qw;
    const uint32_t dy = xl / (uint32_t)rw;
    int yy = yb + (int)dy, xx = (int)(xl - dy * (uint32_t)rw);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int qq = qw + (kBlock / 16) * v;
      if (qq < len) {
        if (qq + 4 <= len && xx + 4 <= rw) {
          const int64_t o = (int64_t)yy * I.pitch + xx;
          st_u32x4_nt(ocol + o, cq[v]);
          if (np == 8) st_u32x4_nt(odep + o, dq[v]);
        } else {   // a quad at the end of a row or of the block
          int y2 = yy, x2 = xx;
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (qq + j < len) {
              const int64_t o = (int64_t)y2 * I.pitch + x2;
              ocol[o] = cq[v][j];
              if (np == 8) odep[o] = dq[v][j];
              if (++x2 == rw) { x2 = 0; ++y2; }
            }
          }
        }
      }
      // advance 256 pixels
      xx += kBlock / 16;
      if (xx >= rw) {
        const int d = xx / rw;
        yy += d;
        xx -= d * rw;
      }
    }
  }
  }
}

// Workgroups of `kernel` that fit on the device at once, at most `cap` per
// compute unit when cap > 0 (the per-unit occupancy is cached per device).
int resident_groups(const void* kernel, std::atomic<int>* cache, int cap) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 1024;
  int packed = cache[dev].load(std::memory_order_relaxed);
  if (packed <= 0) {
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, kThreads, 0) != hipSuccess ||
        cus <= 0 || per_cu <= 0)
      return 1024;
    packed = cus * 256 + per_cu;   // both fit: cus < 2^23, per_cu < 256
    cache[dev].store(packed, std::memory_order_relaxed);
  }
  const int cus = packed / 256, per_cu = packed % 256;
  return cus * (cap > 0 && cap < per_cu ? cap : per_cu);
}
static std::atomic<int> g_compress_groups[64], g_decompress_groups[64];
// Caps on the workgroups per compute unit (0: as many as fit).
static std::atomic<int> g_compress_cap{0}, g_decompress_cap{0};
// Look-back polls before a compressing block gives up (negative: the default).
constexpr uint32_t kDefaultWaitLimit = 1u << 20;
static std::atomic<int32_t> g_wait_limit{-1};
uint32_t rle_wait_limit() {
  const int32_t wl = g_wait_limit.load(std::memory_order_relaxed);
  return wl < 0 ? kDefaultWaitLimit : (uint32_t)wl;
}
int rle_compress_cap() { return g_compress_cap.load(std::memory_order_relaxed); }

// Look-back flags: one per block of each image's largest possible ROI.
int64_t rle_flag_count(const cmp_image* imgs, int32_t n) {
  int64_t f = 0;
  for (int i = 0; i < n; ++i) {
    const int64_t npx = (int64_t)(imgs[i].roi.w > 0 ? imgs[i].roi.w : 0) *
                        (imgs[i].roi.h > 0 ? imgs[i].roi.h : 0);
    const int64_t nb = (int64_t)rle_nblocks(npx);
    f += nb ? nb : 1;
  }
  return f;
}

// Scratch memory of cmp_rle_compress_noalloc: the tickets and look-back
// flags that cmp_rle_compress keeps in the caller's workspace. Each device
// holds its own copy until the process ends. Host code never passes this
// name to a kernel (on the host it is only a stand-in for the symbol): it
// passes the device address that hipGetSymbolAddress returns for the
// current device, looked up once per device and kept in g_scratch_ptr.
static_assert(CMP_RLE_SCRATCH_BYTES == kTicketBytes + kCtlBytes + 8 * 131072,
              "the scratch holds the tickets, the control words and 131072 look-back flags");
static __device__ __align__(256) uint8_t scratch[CMP_RLE_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[64];

// The current device's address of `scratch` (nullptr, with the error set,
// if it cannot be found).
static void* scratch_address() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) {
    set_error("no current HIP device (or more than 64 devices)");
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      set_error("hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = p;
  }
  return g_scratch_ptr[dev];
}

}  // namespace cmp

using namespace cmp;

extern "C" size_t cmp_rle_max_size(int32_t w, int32_t h, int32_t nplanes) {
  if (w < 0 || h < 0 || nplanes <= 0) return 0;
  const int64_t npx = (int64_t)w * h;
  const uint64_t nb = rle_nblocks(npx);
  uint64_t total = rle_p0(nb, nplanes);
  if (nb) total += (nb - 1) * align16((uint64_t)kBlock * nplanes) +
                   align16((uint64_t)(npx - (int64_t)(nb - 1) * kBlock) * nplanes);
  return (size_t)total;
}

extern "C" size_t cmp_rle_workspace_size(const cmp_image* imgs, int32_t n) {
  if (n < 0 || (n > 0 && !imgs)) return 0;
  return kTicketBytes + kCtlBytes + (size_t)(8 * rle_flag_count(imgs, n));
}

namespace cmp {

cmp_status rle_compress_prepare(const cmp_image* imgs, int32_t n, const int32_t* roi_dev,
                                uint8_t* const* out, const uint64_t* capacity,
                                uint64_t* out_size_dev, int32_t* status_dev, void* workspace,
                                size_t ws_bytes, size_t (*max_size)(int32_t, int32_t, bool),
                                RleCArgs& a, int64_t& grid) {
  CMP_REQUIRE(imgs && out && capacity && out_size_dev && status_dev && workspace, "NULL argument");
  CMP_REQUIRE(((uintptr_t)roi_dev & 15) == 0 && ((uintptr_t)workspace & 15) == 0 &&
                  ((uintptr_t)out_size_dev & 7) == 0 && ((uintptr_t)status_dev & 3) == 0,
              "roi_dev/workspace must be 16-byte, out_size_dev 8-byte and status_dev "
              "4-byte aligned");
  memset(&a, 0, sizeof a);
  int64_t nflags = 0;
  grid = 0;
  for (int i = 0; i < n; ++i) {
    const cmp_image& I = imgs[i];
    CMP_REQUIRE(rect_valid(I.roi), "imgs[%d] has a negative size", i);
    const int W = rect_empty(I.roi) ? 0 : I.roi.w, H = rect_empty(I.roi) ? 0 : I.roi.h;
    if (W > 0) {
      CMP_REQUIRE(I.color, "imgs[%d].color is NULL", i);
      CMP_REQUIRE(I.pitch >= W, "imgs[%d].pitch < width", i);
      CMP_REQUIRE(((uintptr_t)I.color & 3) == 0 && ((uintptr_t)I.depth & 3) == 0,
                  "imgs[%d]: buffers must be 4-byte aligned", i);
    }
    CMP_REQUIRE(out[i] && ((uintptr_t)out[i] & 15) == 0, "out[%d] must be 16-byte aligned", i);
    const size_t need = max_size(W, H, I.depth != nullptr);
    CMP_REQUIRE(need < (1ull << 32), "image %d too large for 32-bit stream offsets", i);
    if (capacity[i] < need) {
      set_error("capacity[%d] = %llu < %zu", i, (unsigned long long)capacity[i], need);
      return CMP_ENOSPC;
    }
    const int64_t nb = (int64_t)rle_nblocks((int64_t)W * H);
    a.im[i] = RleCImg{(const uint32_t*)I.color, I.depth, I.pitch, W, H, out[i], (int32_t)nflags, 0};
    nflags += nb ? nb : 1;
    grid += nb ? nb : 1;
  }
  CMP_REQUIRE(grid < (1ll << 24), "too many blocks");
  const size_t need = kTicketBytes + kCtlBytes + (size_t)(8 * nflags);
  if (ws_bytes < need) {
    set_error("workspace of %zu bytes is smaller than %zu", ws_bytes, need);
    return CMP_ENOSPC;
  }
  a.roi_dev = roi_dev;
  a.out_size = out_size_dev;
  a.status = status_dev;
  a.tickets = (uint32_t*)workspace;
  a.ctl = (uint32_t*)((uint8_t*)workspace + kTicketBytes);
  a.flags = (uint64_t*)((uint8_t*)workspace + kTicketBytes + kCtlBytes);
  a.nflags = (int32_t)nflags;
  a.n = n;
  a.wait_limit = rle_wait_limit();
  return CMP_OK;
}

}  // namespace cmp

static size_t rle1_max_size(int32_t w, int32_t h, bool depth) {
  return cmp_rle_max_size(w, h, depth ? 8 : 4);
}

extern "C" cmp_status cmp_rle_compress(const cmp_image* imgs, int32_t n, cmp_format fmt,
                                       uint32_t flags, const int32_t* roi_dev, uint8_t* const* out,
                                       const uint64_t* capacity, uint64_t* out_size_dev,
                                       int32_t* status_dev, void* workspace, size_t ws_bytes,
                                       void* stream) {
  CMP_RANGE("cmp_rle_compress");
  CMP_REQUIRE(n >= 0 && n <= kRleMax, "n = %d must be 0..%d", n, kRleMax);
  if (n == 0) return CMP_OK;
  if (fmt != CMP_RGBA8) {
    set_error("RLE compression handles RGBA8 (+ depth) pixels");
    return CMP_EUNSUPPORTED;
  }
  CMP_REQUIRE((flags & ~CMP_RLE_SWIZZLE) == 0, "unknown flags 0x%x", flags);
  RleCArgs a;
  int64_t grid = 0;
  hipStream_t s = (hipStream_t)stream;
  const cmp_status st = rle_compress_prepare(imgs, n, roi_dev, out, capacity, out_size_dev,
                                             status_dev, workspace, ws_bytes, rle1_max_size, a,
                                             grid);
  if (st != CMP_OK) return st;
  a.swizzle = (flags & CMP_RLE_SWIZZLE) ? 1 : 0;
  // one wave of workgroups at most: more would find the tickets drawn
  // (both instances have the same resources, so one occupancy serves both)
  const int64_t cap = resident_groups((const void*)rle_compress_kernel<false>, g_compress_groups,
                                      rle_compress_cap());
  const dim3 grid_dim((unsigned)(grid < cap ? grid : cap));
  log_plan("rle compress: %d images, %lld block slots, %u resident workgroups%s", n,
           (long long)grid, grid_dim.x, a.swizzle ? ", swizzled" : "");
  if (a.swizzle)
    hipLaunchKernelGGL(rle_compress_kernel<true>, grid_dim, dim3(kThreads), 0, s, a);
  else
    hipLaunchKernelGGL(rle_compress_kernel<false>, grid_dim, dim3(kThreads), 0, s, a);
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}

extern "C" cmp_status cmp_rle_compress_noalloc(const cmp_image* imgs, int32_t n, cmp_format fmt,
                                               uint32_t flags, const int32_t* roi_dev,
                                               uint8_t* const* out, const uint64_t* capacity,
                                               uint64_t* out_size_dev, int32_t* status_dev,
                                               void* stream) {
  CMP_RANGE("cmp_rle_compress_noalloc");
  CMP_REQUIRE(n >= 0 && n <= kRleMax, "n = %d must be 0..%d", n, kRleMax);
  if (n == 0) return CMP_OK;
  CMP_REQUIRE(imgs, "imgs is NULL");
  for (int i = 0; i < n; ++i)
    CMP_REQUIRE(rect_valid(imgs[i].roi), "imgs[%d] has a negative size", i);
  const size_t need = cmp_rle_workspace_size(imgs, n);
  if (need > CMP_RLE_SCRATCH_BYTES) {
    set_error("these images need %zu bytes of scratch; the static maximum is %zu "
              "(131072 blocks of 4096 pixels): use cmp_rle_compress with a workspace",
              need, (size_t)CMP_RLE_SCRATCH_BYTES);
    return CMP_ENOSPC;
  }
  void* ws = scratch_address();
  if (!ws) return CMP_EHIP;
  return cmp_rle_compress(imgs, n, fmt, flags, roi_dev, out, capacity, out_size_dev, status_dev,
                          ws, CMP_RLE_SCRATCH_BYTES, stream);
}

extern "C" cmp_status cmp_rle_set_wait_limit(int32_t polls) {
  g_wait_limit.store(polls < 0 ? -1 : polls, std::memory_order_relaxed);
  return CMP_OK;
}

extern "C" cmp_status cmp_rle_set_groups_per_cu(int32_t compress, int32_t decompress) {
  CMP_REQUIRE(compress >= 0 && decompress >= 0, "caps must be >= 0 (0: as many as fit)");
  g_compress_cap.store(compress, std::memory_order_relaxed);
  g_decompress_cap.store(decompress, std::memory_order_relaxed);
  return CMP_OK;
}

static cmp_status rle_decompress_impl(const uint8_t* const* in, const uint64_t* in_bytes,
                                      int32_t n, const cmp_image* out, int32_t* roi_out_dev,
                                      int32_t* status_dev, bool at_roi, void* stream) {
  CMP_REQUIRE(n >= 0 && n <= kRleMax, "n = %d must be 0..%d", n, kRleMax);
  if (n == 0) return CMP_OK;
  CMP_REQUIRE(in && in_bytes && out && status_dev, "NULL argument");
  CMP_REQUIRE(((uintptr_t)roi_out_dev & 15) == 0 && ((uintptr_t)status_dev & 3) == 0,
              "roi_out_dev must be 16-byte aligned");
  RleDArgs a;
  memset(&a, 0, sizeof a);
  int64_t grid = 0;
  for (int i = 0; i < n; ++i) {
    const cmp_image& O = out[i];
    CMP_REQUIRE(in[i] && ((uintptr_t)in[i] & 15) == 0, "in[%d] must be 16-byte aligned", i);
    CMP_REQUIRE(rect_valid(O.roi), "out[%d] has a negative size", i);
    const int W = rect_empty(O.roi) ? 0 : O.roi.w, H = rect_empty(O.roi) ? 0 : O.roi.h;
    if (W > 0) {
      CMP_REQUIRE(O.color && O.pitch >= W, "out[%d]: NULL colour or pitch < width", i);
      CMP_REQUIRE(((uintptr_t)O.color & 3) == 0 && ((uintptr_t)O.depth & 3) == 0,
                  "out[%d]: buffers must be 4-byte aligned", i);
    }
    const int64_t nb = (int64_t)rle_nblocks((int64_t)W * H);
    a.im[i] = RleDImg{in[i], in_bytes[i], (uint32_t*)O.color, (uint32_t*)O.depth, O.pitch, W, H};
    grid += nb ? nb : 1;
  }
  CMP_REQUIRE(grid < (1ll << 24), "too many blocks");
  a.roi_out = roi_out_dev;
  a.status = status_dev;
  a.n = n;
  a.at_roi = at_roi ? 1 : 0;
  const int64_t cap = resident_groups((const void*)rle_decompress_kernel, g_decompress_groups,
                                      g_decompress_cap.load(std::memory_order_relaxed));
  log_plan("rle decompress: %d streams, at most %lld blocks, %lld resident workgroups%s", n,
           (long long)grid, (long long)(grid < cap ? grid : cap), at_roi ? ", at the ROIs" : "");
  hipLaunchKernelGGL(rle_decompress_kernel, dim3((unsigned)(grid < cap ? grid : cap)),
                     dim3(kThreads), 0, (hipStream_t)stream, a);
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}

extern "C" cmp_status cmp_rle_decompress(const uint8_t* const* in, const uint64_t* in_bytes,
                                         int32_t n, const cmp_image* out, int32_t* roi_out_dev,
                                         int32_t* status_dev, void* stream) {
  CMP_RANGE("cmp_rle_decompress");
  return rle_decompress_impl(in, in_bytes, n, out, roi_out_dev, status_dev, false, stream);
}

extern "C" cmp_status cmp_rle_decompress_at_roi(const uint8_t* const* in,
                                                const uint64_t* in_bytes, int32_t n,
                                                const cmp_image* out, int32_t* roi_out_dev,
                                                int32_t* status_dev, void* stream) {
  CMP_RANGE("cmp_rle_decompress_at_roi");
  return rle_decompress_impl(in, in_bytes, n, out, roi_out_dev, status_dev, true, stream);
}
