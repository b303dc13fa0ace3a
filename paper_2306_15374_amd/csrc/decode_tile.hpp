// One tile of the LeCo decoder (section 3.3, range decompression): the
// values of global positions [g0, g1) of one blob, decoded by one 256-thread
// workgroup.  The tile is cut at partition boundaries into segments and each
// segment into chunks whose packed residual words fit the LDS stage; each
// chunk's words are read from HBM once, with coalesced 16-byte loads, and
// every thread then decodes values t = c0 + tid, c0 + tid + 256, ... from
// LDS, so each wave stores a contiguous run of outputs.
#pragma once

#include "leco_dev.hpp"

namespace leco {

constexpr int kBlock = 256;
// 32-bit words of LDS per stage (16 KiB of residual words plus slack for
// the alignment of the first load and the two words read past a field).
constexpr uint32_t kStageWords = 4096 + 16;

__device__ inline uint32_t chunk_values(uint32_t bits) {
  return bits == 0 ? 0xffffffffu : ((kStageWords - 12) * 32u) / bits;
}

// Sink receives (global position g, decoded value v) for every value.
// Returns false if the blob failed validation (the caller raises the flag);
// all control flow depending on it is uniform across the workgroup.
template <class Sink>
__device__ bool decode_tile(const uint8_t* __restrict__ blob, const Header& h, uint64_t g0,
                            uint64_t g1, uint32_t* __restrict__ stage, Sink& sink) {
  const uint32_t tid = threadIdx.x;
  uint64_t j = locate(blob, h, g0);
  const uint32_t* words32 = reinterpret_cast<const uint32_t*>(blob + h.words_off);
  while (g0 < g1) {
    Part p;
    if (!load_part(blob, h, j, p)) return false;
    if (g0 < p.start || g0 - p.start >= p.len) return false;
    const uint64_t seg_end = (p.start + p.len < g1) ? p.start + p.len : g1;
    const uint32_t t_end = uint32_t(seg_end - p.start);
    const uint32_t b = p.bits;
    const bool small_pred = prediction_fits_i32(p.theta1, p.len);
    if (!sink.visit_segment(p, uint32_t(g0 - p.start), t_end)) {
      g0 = seg_end;
      ++j;
      continue;
    }
    const uint32_t step = chunk_values(b);
    for (uint32_t c0 = uint32_t(g0 - p.start); c0 < t_end;) {
      const uint32_t c1 = (t_end - c0 > step) ? c0 + step : t_end;
      int64_t qoff = 0;
      if (b != 0) {
        // 32-bit word range of bits [b*c0, b*c1), widened to 16-byte loads.
        const uint64_t w_first = 2 * p.word_off + ((uint64_t(b) * c0) >> 5);
        const uint64_t w_last = 2 * p.word_off + ((uint64_t(b) * c1 + 31) >> 5);
        const uint64_t a0 = w_first & ~uint64_t(3);
        const uint32_t nvec = uint32_t((w_last - a0 + 3) >> 2);
        const uint4* src = reinterpret_cast<const uint4*>(words32 + a0);
        uint4* dst = reinterpret_cast<uint4*>(stage);
        for (uint32_t i = tid; i < nvec; i += kBlock) dst[i] = src[i];
        qoff = int64_t(64 * p.word_off) - int64_t(32 * a0);
        __syncthreads();
      }
      // values handled by this thread: t = c0 + tid + kBlock * i, i < cnt
      const uint32_t first = c0 + tid;
      const uint32_t cnt = first < c1 ? (c1 - first + kBlock - 1) / kBlock : 0;
      const uint32_t mask32 = b >= 32 ? 0xffffffffu : ((1u << b) - 1u);
      const uint32_t mask_hi = b >= 64 ? 0xffffffffu : (b > 32 ? ((1u << (b - 32)) - 1u) : 0u);
      const uint32_t q0 = uint32_t(qoff + int64_t(b) * first);
      const uint32_t dq = b * kBlock;
      const uint64_t g_first = p.start + first;
      if (b <= 32 && small_pred) {
#pragma unroll 4
        for (uint32_t i = 0; i < cnt; ++i) {
          const uint32_t t = first + i * kBlock;
          const uint32_t u = b ? extract32(stage, q0 + i * dq, mask32) : 0u;
          const int32_t pr = predict32(p.theta1, t);
          sink.put(g_first + i * kBlock, p.base + uint64_t(int64_t(pr)) + u);
        }
      } else if (b <= 32) {
#pragma unroll 2
        for (uint32_t i = 0; i < cnt; ++i) {
          const uint32_t t = first + i * kBlock;
          const uint32_t u = b ? extract32(stage, q0 + i * dq, mask32) : 0u;
          sink.put(g_first + i * kBlock, p.base + uint64_t(predict(p.theta1, t)) + u);
        }
      } else {
#pragma unroll 2
        for (uint32_t i = 0; i < cnt; ++i) {
          const uint32_t t = first + i * kBlock;
          const uint64_t u = extract64(stage, q0 + i * dq, mask_hi);
          sink.put(g_first + i * kBlock, p.base + uint64_t(predict(p.theta1, t)) + u);
        }
      }
      if (b != 0) __syncthreads();
      c0 = c1;
    }
    g0 = seg_end;
    ++j;
  }
  return true;
}

// Writes each value to out[g - origin] with the column's width, bypassing
// the caches (outputs are written once and not read back by the kernel).
template <typename OutT>
struct StoreSink {
  OutT* out;
  uint64_t origin;
  __device__ bool visit_segment(const Part&, uint32_t, uint32_t) { return true; }
  __device__ void put(uint64_t g, uint64_t v) {
    __builtin_nontemporal_store(OutT(v), out + (g - origin));
  }
};

// Maps a workgroup to a virtual index so that each XCD (workgroups are
// dispatched round-robin over the 8 XCDs) walks a contiguous run of tiles;
// grid must be a multiple of 8 for the mapping to be a permutation.
__device__ inline uint64_t xcd_virtual_block(uint32_t b, uint32_t grid, bool remap) {
  if (!remap || (grid & 7u)) return b;
  return uint64_t(b & 7u) * (grid >> 3) + (b >> 3);
}

}  // namespace leco
