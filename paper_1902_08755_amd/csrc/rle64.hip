// cmp_rle64_compress / cmp_rle64_decompress: the basic 64-bit run-length
// encoding of Section 5.5.1 (Enhanced RLE Compression), which compares two
// RGBA8 pixels at a time as one 64-bit token and therefore only shortens
// runs of equal pixel pairs. Stream format "RL64": see cmp.h.
//
// The machinery is that of the per-component compressor (rle.hip): one
// workgroup encodes a block of 4096 pixels (16 per lane, i.e. 8 symbols per
// lane and stream) from registers, the block's size is published as soon as
// a workgroup scan has counted its runs, its payload offset comes from a
// decoupled look-back over the blocks of the image, and blocks are drawn
// from a ticket counter per image. A run starts at symbol j when j is a
// multiple of 128 or symbol j differs from symbol j - 1; runs therefore
// never cross a 256-pixel segment (16 lanes), and a run's end is the next
// start in its lane or the first start of the following lanes of its DPP
// row.
//
// Decompression: a grid-stride loop over the blocks of all streams; per
// block the payload goes to LDS, each lane sums the run lengths of 8 tokens,
// a workgroup scan places the runs, every run start is marked (a bit and the
// run's token index), and each lane fills its 8 symbols from the last start
// at or before each of them (the start entering a lane comes from a scan
// over its DPP row). Every check of the format is made: a malformed stream
// gets CMP_ECORRUPT and its blocks are not written.
#include <string.h>

#include "rle_common.hpp"

namespace cmp {

constexpr uint32_t kRl64Magic = 0x34364C52u;
constexpr int kSymLane = kPxPerLane / 2;   // symbols per lane and stream
constexpr int kSymSeg = kSeg / 2;          // symbols per 256-pixel segment
constexpr int kSymBlock = kBlock / 2;      // symbols per block

__host__ __device__ inline uint32_t align8u(uint32_t v) { return (v + 7u) & ~7u; }
// Bytes of a token-coded stream with R runs: R length bytes, zeros to a
// multiple of 8, then R 64-bit values.
__host__ __device__ inline uint32_t rl64_token_bytes(uint32_t r) { return align8u(r) + 8u * r; }

// Runs of a token-coded stream of `bytes` bytes (the inverse of
// rl64_token_bytes), or 0 if no run count gives that size.
__device__ __forceinline__ uint32_t rl64_runs_of(uint32_t bytes) {
  if (bytes == 0 || (bytes & 7u)) return 0;
  const uint32_t u = bytes / 8, q = u / 9, r = u % 9;
  // R = 8q gives u = 9q; R = 8q + r' (1 <= r' <= 8) gives u = 9q + r' + 1
  const uint32_t R = r == 0 ? 8 * q : r == 1 ? 0 : 8 * q + r - 1;
  return R && rl64_token_bytes(R) == bytes ? R : 0;
}

// ------------------------------------------------------------ compress
__global__ __launch_bounds__(kThreads, 4) void rle64_compress_kernel(const RleCArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t stage[kStage];
  __shared__ uint32_t sh[16];
  __shared__ uint32_t s_excl;
  __shared__ int32_t s_poison;
  __shared__ int4 t_roi[kRleMax];
  __shared__ uint32_t t_slots[kRleMax];
  __shared__ int2 s_next;   // the slot drawn for the next iteration
  slot_table(a, t_roi, t_slots);
  const uint32_t ep = call_epoch(a);
  __syncthreads();

  // Slots as in the per-component compressor: per-image tickets drawn by
  // wave 1, the next one after the current block's size is published.
  int img = (int)(blockIdx.x % (uint32_t)a.n);
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
  int tid = threadIdx.x;   // opaque per iteration (see the per-component compressor)
  __asm__ volatile("" : "+v"(tid));
  const int lane = tid % kWave;
  const CSlot c = nx;
  const int s = c.s, b = c.b, rx = c.rx, ry = c.ry, rw = c.rw, rh = c.rh;
  const bool drawer = tid / kWave == 1;
  uint32_t t_next = 0u;
  auto finish_draw = [&]() {
    if (drawer) {
      const int2 sb = draw_slot(t_next, a.tickets, t_slots, a.n, img);
      if (lane == 0) s_next = sb;
    }
  };
  bool more = false;
  const RleCImg I = a.im[s];
  const int ns = I.depth ? 2 : 1;
  const int64_t npx = (int64_t)rw * rh;
  const uint64_t nb = rle_nblocks(npx);
  const uint64_t P0 = rle_p0(nb, ns);
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
      const uint32_t hdr[8] = {kRl64Magic, (uint32_t)rx, (uint32_t)ry, 0u, 0u, (uint32_t)ns,
                               (uint32_t)kBlock, 0u};
      reinterpret_cast<uint32_t*>(out)[tid] = hdr[tid];
    }
    if (tid == 0) a.out_size[s] = 32;
  } else {
    const int len = (int)imin64(kBlock, npx - (int64_t)b * kBlock);
    const int m = (len + 1) / 2;   // symbols of the block (an odd last pixel pairs with 0)
    const int j0 = tid * kSymLane;
    const int nsv = min(kSymLane, max(0, m - j0));
    const uint32_t vmask = (1u << nsv) - 1u;
    const bool seg_start = (tid % (kSeg / kPxPerLane)) == 0;

    // ---- run starts of the symbols (pixel 2i low, 2i + 1 high) per stream:
    // symbol i differs from the one before it (the previous lane's last
    // symbol for i = 0), or starts a segment
    uint32_t mask[2] = {0u, 0u};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k >= ns) continue;
      const uint32_t* w = k ? dep : col;
      const uint32_t plo = __shfl_up(w[kPxPerLane - 2], 1), phi = __shfl_up(w[kPxPerLane - 1], 1);
      uint32_t mm = 0;
#pragma unroll
      for (int i = 0; i < kSymLane; ++i) {
        const uint32_t lo0 = i ? w[2 * i - 2] : plo, hi0 = i ? w[2 * i - 1] : phi;
        if ((w[2 * i] ^ lo0) | (w[2 * i + 1] ^ hi0)) mm |= 1u << i;
      }
      if (seg_start) mm |= 1u;
      mask[k] = mm & vmask;
    }
    uint32_t cnt[1] = {(uint32_t)__builtin_popcount(mask[0]) |
                       ((uint32_t)__builtin_popcount(mask[1]) << 16)};
    uint32_t ex[1], tot[1];
    block_scan32<1>(cnt, ex, tot, sh);
    if (drawer) t_next = draw_ticket(a.tickets, img);

    // ---- stream sizes and offsets (uniform; multiples of 8)
    uint32_t size[2], poff[2], runs[2];
    uint32_t total = 0;
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      size[k] = 0;
      poff[k] = total;
      runs[k] = (tot[0] >> (16 * k)) & 0xFFFFu;
      if (k >= ns) continue;
      const uint32_t tb = rl64_token_bytes(runs[k]);
      size[k] = tb < 8u * (uint32_t)m ? tb : 8u * (uint32_t)m;
      total += size[k];
    }
    const uint32_t padded = (uint32_t)align16(total);
    uint64_t* flags = a.flags + I.flag_base;
    if (tid == 0)
      __hip_atomic_store(&flags[b], mkflag(b == 0 ? kIncl : kAgg, padded, ep), __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);

    // ---- stage the encoded block in LDS
    const int seg_end = min(m, (j0 / kSymSeg + 1) * kSymSeg);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      if (k >= ns) continue;
      const uint32_t* w = k ? dep : col;
      const uint32_t off = poff[k];
      if (size[k] != 8u * (uint32_t)m) {
        // a run ends at the next start: in this lane, else the first start
        // of the following lanes of the segment, else the segment end
        uint32_t mm = mask[k];
        int fs = mm ? j0 + __builtin_ctz(mm) : seg_end;
        fs = min(fs, row_shl_fill<1>(fs, seg_end));
        fs = min(fs, row_shl_fill<2>(fs, seg_end));
        fs = min(fs, row_shl_fill<4>(fs, seg_end));
        fs = min(fs, row_shl_fill<8>(fs, seg_end));
        const int next_after = row_shl_fill<1>(fs, seg_end);
        uint32_t idx = (ex[0] >> (16 * k)) & 0xFFFFu;
        const uint32_t vals = off + align8u(runs[k]);
        // one unrolled step per symbol slot, so that the symbol registers are
        // indexed by constants: indexed by the run's position instead, they
        // went to scratch memory (144 bytes per lane, 2.3x the kernel's HBM
        // bytes)
#pragma unroll
        for (int i = 0; i < kSymLane; ++i) {
          if (mm & (1u << i)) {
            const uint32_t later = mm & ~((2u << i) - 1u);   // starts after symbol i
            const int end = later ? j0 + __builtin_ctz(later) : next_after;
            stage[off + idx] = (uint8_t)(end - j0 - i - 1);
            *reinterpret_cast<uint2*>(stage + vals + 8 * idx) = uint2{w[2 * i], w[2 * i + 1]};
            ++idx;
          }
        }
        if (tid < (int)(align8u(runs[k]) - runs[k])) stage[off + runs[k] + tid] = 0;
      } else {
#pragma unroll
        for (int i = 0; i < kSymLane; ++i)
          if (i < nsv)
            *reinterpret_cast<uint2*>(stage + off + 8 * (j0 + i)) = uint2{w[2 * i], w[2 * i + 1]};
      }
    }
    if (tid < (int)(padded - total)) stage[total + tid] = 0;
    finish_draw();
    __syncthreads();   // s_next is written
    cur = s_next;
    more = cur.x >= 0;

    // ---- payload offset (wave 0); the next slot's pixels go in flight
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
    if (tid < ns) tbl[nb + (uint64_t)b * ns + tid] = tid ? size[1] : size[0];
    if (tid == 0) tbl[b] = poisoned ? 0xFFFFFFFFu : excl;
    if (b == 0) {
      if (tid < 8) {
        const uint32_t hdr[8] = {kRl64Magic, (uint32_t)rx, (uint32_t)ry, (uint32_t)rw,
                                 (uint32_t)rh, (uint32_t)ns, (uint32_t)kBlock, (uint32_t)nb};
        reinterpret_cast<uint32_t*>(out)[tid] = hdr[tid];
      }
      const uint64_t tend = 32 + 4 * nb * (1 + (uint64_t)ns);
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
  __syncthreads();   // the stage, the scan words and s_next are reused by the next slot
  if (!more) break;
  }
  finish_call(a, ep);
}

// ---------------------------------------------------------- decompress
__global__ __launch_bounds__(kThreads) void rle64_decompress_kernel(const RleDArgs a) {
  __shared__ __attribute__((aligned(16))) uint8_t stage[kStage];
  __shared__ uint32_t starts[2][kSymBlock / 32];   // run-start bits per stream
  __shared__ uint16_t tok_at[2][kSymBlock];        // token index at each run start
  __shared__ uint32_t sh[16];
  __shared__ int32_t s_bad[kThreads / kWave];
  const int tid = threadIdx.x, lane = tid % kWave;

  // Wave 0 reads and checks the header of stream i in lane i (n <= 64); a
  // stream takes one slot per block, or one slot if it has no blocks or a
  // bad header (that slot reports the status or writes the ROI).
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
        if (lh[0] != kRl64Magic || w < 0 || hh < 0 || (lh[5] != 1 && lh[5] != 2) ||
            lh[6] != (uint32_t)kBlock)
          lerr = CMP_ECORRUPT;
        else if ((uint64_t)lh[7] != rle_nblocks((int64_t)w * hh))
          lerr = CMP_ECORRUPT;
        else if (I.in_bytes < rle_p0(lh[7], (int)lh[5]))
          lerr = CMP_ECORRUPT;
        else if (w > I.cap_w || hh > I.cap_h || (lh[5] == 2 && !I.depth))
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
  const uint32_t total_slots = t_total;

  for (uint32_t g = blockIdx.x; g < total_slots; g += gridDim.x) {
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
  const int ns = (int)h[5];
  const uint64_t nb = h[7];
  if (b == 0 && a.roi_out && tid == 0)
    reinterpret_cast<int4*>(a.roi_out)[s] = int4{(int)h[1], (int)h[2], (int)h[3], (int)h[4]};
  if ((uint64_t)b >= nb) continue;   // uniform: a stream without blocks
  const int64_t npx = (int64_t)rw * rh;
  const int len = (int)imin64(kBlock, npx - (int64_t)b * kBlock);
  const int m = (len + 1) / 2;
  // block table (uniform loads; inside the table the header check found
  // readable)
  const uint32_t* tbl = reinterpret_cast<const uint32_t*>(I.in + 32);
  const uint32_t* srow = tbl + nb + (uint64_t)b * ns;
  uint32_t size[2] = {srow[0], ns == 2 ? srow[1] : 0u};
  uint2 bo;   // boff[b], boff[b + 1]: a 4-byte aligned pair
  __builtin_memcpy(&bo, __builtin_assume_aligned(tbl + b, 4), 8);
  uint32_t poff[2], runs[2] = {0u, 0u}, btotal = 0;
  int e = 0;
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    poff[k] = btotal;
    if (k >= ns) continue;
    if (size[k] > 8u * (uint32_t)m) e = CMP_ECORRUPT;
    if (size[k] < 8u * (uint32_t)m) {
      runs[k] = rl64_runs_of(size[k]);
      if (!runs[k]) e = CMP_ECORRUPT;
    }
    btotal += size[k];
  }
  const uint32_t boff = bo.x, bnext = bo.y;   // bnext: the first size entry when b is the last block
  if ((boff & 15u) || (b == 0 && boff != 0)) e = CMP_ECORRUPT;
  if ((uint64_t)b + 1 < nb && (uint64_t)bnext != boff + align16(btotal)) e = CMP_ECORRUPT;
  if (rle_p0(nb, ns) + boff + align16(btotal) > I.in_bytes) e = CMP_ECORRUPT;
  if (e) {   // uniform; no LDS was touched in this slot
    if (tid == 0) a.status[s] = e;
    continue;
  }
  const uint32_t padded = (uint32_t)align16(btotal);
  if (tid < 2 * kSymBlock / 32) (&starts[0][0])[tid] = 0;
  {
    // the whole block payload to LDS: all loads in flight before the stores
    const u32x4* src = reinterpret_cast<const u32x4*>(I.in + rle_p0(nb, ns) + boff);
    u32x4* dst = reinterpret_cast<u32x4*>(stage);
    constexpr int kMaxPer = (8 * kBlock / 16 + kThreads - 1) / kThreads;
    u32x4 tmp[kMaxPer];
    const int nvi = (int)(padded / 16);
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k)
      tmp[k] = tid + k * kThreads < nvi ? src[tid + k * kThreads] : u32x4{0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < kMaxPer; ++k)
      if (tid + k * kThreads < nvi) dst[tid + k * kThreads] = tmp[k];
  }
  __syncthreads();

  bool bad = false;
  // zero padding: after the run lengths of a token stream, after the block
  if (tid < 16 && (uint32_t)tid < padded - btotal && stage[btotal + tid]) bad = true;
#pragma unroll
  for (int k = 0; k < 2; ++k)
    if (runs[k] && (uint32_t)tid < align8u(runs[k]) - runs[k] && stage[poff[k] + runs[k] + tid])
      bad = true;
  // run positions: lane t covers tokens 8t .. 8t + 7 of each token stream
  const int t0 = tid * kSymLane;
  // (a stream's lengths sum to < 2^20 whatever it holds: < 2048 tokens of
  // <= 256 symbols; each stream has a 32-bit word of its own in the scan)
  uint32_t lens[2][kSymLane];
  uint32_t sums[2] = {0u, 0u};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
#pragma unroll
    for (int i = 0; i < kSymLane; ++i) {
      lens[k][i] = 0;
      if ((uint32_t)(t0 + i) < runs[k]) {
        lens[k][i] = (uint32_t)stage[poff[k] + t0 + i] + 1u;
        sums[k] += lens[k][i];
      }
    }
  }
  uint32_t ex[2], tot[2];
  block_scan32<2>(sums, ex, tot, sh);
#pragma unroll
  for (int k = 0; k < 2; ++k)
    if (runs[k] && tot[k] != (uint32_t)m) bad = true;
  // mark every run start, and check that no run crosses a multiple of 128
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    if (!runs[k]) continue;
    uint32_t pos = ex[k];
#pragma unroll
    for (int i = 0; i < kSymLane; ++i) {
      if (lens[k][i]) {
        if ((pos % kSymSeg) + lens[k][i] > (uint32_t)kSymSeg || pos + lens[k][i] > (uint32_t)m) {
          bad = true;
        } else {
          tok_at[k][pos] = (uint16_t)(t0 + i);
          __hip_atomic_fetch_or(&starts[k][pos >> 5], 1u << (pos & 31), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        pos += lens[k][i];
      }
    }
  }
  // a malformed block must not be written: one vote per wave, then a
  // barrier that also publishes the marks
  {
    const uint64_t vote = __ballot(bad);
    if (lane == 0) s_bad[tid / kWave] = vote != 0;
  }
  __syncthreads();
  if (s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3]) {
    if (tid == 0) a.status[s] = CMP_ECORRUPT;
    __syncthreads();   // every lane has read s_bad before the next slot writes it
    continue;
  }

  // ---- symbols of this lane: symbol j0 + i, i < 8
  const int j0 = tid * kSymLane;
  const int nsv = min(kSymLane, max(0, m - j0));
  uint32_t col[kPxPerLane], dep[kPxPerLane];
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    uint32_t* px = k ? dep : col;
#pragma unroll
    for (int i = 0; i < kPxPerLane; ++i) px[i] = 0;
    if (k >= ns) continue;
    if (!runs[k]) {
#pragma unroll
      for (int i = 0; i < kSymLane; ++i) {
        if (i < nsv) {
          const uint2 v = *reinterpret_cast<const uint2*>(stage + poff[k] + 8 * (j0 + i));
          px[2 * i] = v.x;
          px[2 * i + 1] = v.y;
        }
      }
    } else {
      // the token of the last start at or before each symbol; the one
      // entering the lane comes from the lanes before it in its DPP row
      // (a row is one segment, which starts with a run)
      const uint32_t mm = (starts[k][j0 >> 5] >> (j0 & 31)) & 0xFFu;
      uint32_t x = mm ? (0x10000u | tok_at[k][j0 + 31 - __builtin_clz(mm)]) : 0u;
      uint32_t y;
      y = row_shr<1>(x); if (!(x & 0x10000u)) x = y;
      y = row_shr<2>(x); if (!(x & 0x10000u)) x = y;
      y = row_shr<4>(x); if (!(x & 0x10000u)) x = y;
      y = row_shr<8>(x); if (!(x & 0x10000u)) x = y;
      uint32_t t = row_shr<1>(x) & 0xFFFFu;
      const uint32_t vals = poff[k] + align8u(runs[k]);
#pragma unroll
      for (int i = 0; i < kSymLane; ++i) {
        if (i < nsv) {
          if ((mm >> i) & 1u) t = tok_at[k][j0 + i];
          const uint2 v = *reinterpret_cast<const uint2*>(stage + vals + 8 * t);
          px[2 * i] = v.x;
          px[2 * i + 1] = v.y;
        }
      }
    }
    // the partner of an odd last pixel must be 0
#pragma unroll
    for (int i = 0; i < kSymLane; ++i)
      if ((len & 1) && j0 + i == m - 1 && px[2 * i + 1]) bad = true;
  }
  {
    const uint64_t vote = __ballot(bad);
    if (lane == 0) s_bad[tid / kWave] = vote != 0;
  }
  __syncthreads();   // also ends every LDS access of this slot
  if (s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3]) {
    if (tid == 0) a.status[s] = CMP_ECORRUPT;
    __syncthreads();
    continue;
  }
  // ---- write the pixels (row-major over the ROI)
  const int q0 = tid * kPxPerLane;
  if (q0 < len) {
    const int64_t qb = (int64_t)b * kBlock;
    const int yb = uniform((int)(qb / rw)), xb = uniform((int)(qb - (int64_t)yb * rw));
    const uint32_t xl = (uint32_t)xb + (uint32_t)q0;
    const uint32_t dy = xl / (uint32_t)rw;
    int yy = yb + (int)dy, xx = (int)(xl - dy * (uint32_t)rw);
    if ((q0 + kPxPerLane <= len) && (xx + kPxPerLane <= rw)) {
      const int64_t o = (int64_t)yy * I.pitch + xx;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        st_u32x4(I.color + o + 4 * v,
                 u32x4{col[4 * v], col[4 * v + 1], col[4 * v + 2], col[4 * v + 3]});
        if (ns == 2)
          st_u32x4(I.depth + o + 4 * v,
                   u32x4{dep[4 * v], dep[4 * v + 1], dep[4 * v + 2], dep[4 * v + 3]});
      }
    } else {
#pragma unroll
      for (int j = 0; j < kPxPerLane; ++j) {
        if (q0 + j < len) {
          const int64_t o = (int64_t)yy * I.pitch + xx;
          I.color[o] = col[j];
          if (ns == 2) I.depth[o] = dep[j];
          if (++xx == rw) { xx = 0; ++yy; }
        }
      }
    }
  }
  __syncthreads();   // s_bad and the LDS tables are reused by the next slot
  }
}

static std::atomic<int> g_rl64_compress_groups[64], g_rl64_decompress_groups[64];

// The largest RL64 stream of a w x h ROI: every stream of every block raw.
static size_t rl64_max_size(int32_t w, int32_t h, int32_t nstreams) {
  if (w < 0 || h < 0 || nstreams < 1 || nstreams > 2) return 0;
  const int64_t npx = (int64_t)w * h;
  const uint64_t nb = rle_nblocks(npx);
  uint64_t total = rle_p0(nb, nstreams);
  if (nb) {
    const uint64_t last = (uint64_t)(npx - (int64_t)(nb - 1) * kBlock);
    total += (nb - 1) * align16(8ull * nstreams * kSymBlock) +
             align16(8ull * nstreams * ((last + 1) / 2));
  }
  return (size_t)total;
}

static size_t rl64_max_size_of(int32_t w, int32_t h, bool depth) {
  return rl64_max_size(w, h, depth ? 2 : 1);
}

}  // namespace cmp

using namespace cmp;

extern "C" size_t cmp_rle64_max_size(int32_t w, int32_t h, int32_t nstreams) {
  return rl64_max_size(w, h, nstreams);
}

extern "C" cmp_status cmp_rle64_compress(const cmp_image* imgs, int32_t n, cmp_format fmt,
                                         const int32_t* roi_dev, uint8_t* const* out,
                                         const uint64_t* capacity, uint64_t* out_size_dev,
                                         int32_t* status_dev, void* workspace, size_t ws_bytes,
                                         void* stream) {
  CMP_RANGE("cmp_rle64_compress");
  CMP_REQUIRE(n >= 0 && n <= kRleMax, "n = %d must be 0..%d", n, kRleMax);
  if (n == 0) return CMP_OK;
  if (fmt != CMP_RGBA8) {
    set_error("RL64 compression handles RGBA8 (+ depth) pixels");
    return CMP_EUNSUPPORTED;
  }
  RleCArgs a;
  int64_t grid = 0;
  hipStream_t s = (hipStream_t)stream;
  const cmp_status st = rle_compress_prepare(imgs, n, roi_dev, out, capacity, out_size_dev,
                                             status_dev, workspace, ws_bytes, rl64_max_size_of, a,
                                             grid);
  if (st != CMP_OK) return st;
  const int64_t cap = resident_groups((const void*)rle64_compress_kernel,
                                      g_rl64_compress_groups, rle_compress_cap());
  hipLaunchKernelGGL(rle64_compress_kernel, dim3((unsigned)(grid < cap ? grid : cap)),
                     dim3(kThreads), 0, s, a);
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}

extern "C" cmp_status cmp_rle64_decompress(const uint8_t* const* in, const uint64_t* in_bytes,
                                           int32_t n, const cmp_image* out, int32_t* roi_out_dev,
                                           int32_t* status_dev, void* stream) {
  CMP_RANGE("cmp_rle64_decompress");
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
  const int64_t cap = resident_groups((const void*)rle64_decompress_kernel,
                                      g_rl64_decompress_groups, 0);
  hipLaunchKernelGGL(rle64_decompress_kernel, dim3((unsigned)(grid < cap ? grid : cap)),
                     dim3(kThreads), 0, (hipStream_t)stream, a);
  CMP_CHECK_HIP(hipGetLastError());
  return CMP_OK;
}
