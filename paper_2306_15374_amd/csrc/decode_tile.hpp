// The LeCo decoder's inner loop (section 3.3, range decompression), built
// around wavefront tiles: each 64-lane wavefront decodes the values of
// global positions [g0, g1) (1024 of them by default) on its own, with its
// own slice of LDS and no workgroup barrier.  The tile is cut at partition
// boundaries into segments; the residual words of all its segments (which
// lie back to back in the blob) are copied once into the wavefront's LDS
// slice with coalesced 16-byte loads, then each lane decodes values
// t = c0 + lane, c0 + lane + 64, ... so that every store of the wavefront
// covers 64 consecutive outputs.  Tiles whose words do not fit the slice
// are decoded segment by segment in chunks.
#pragma once

#include "leco_dev.hpp"

namespace leco {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kWavesPerBlock = kBlock / kWave;
// 32-bit words of LDS per wavefront: 1024 words of residuals (1024 values
// at up to 32 bits) plus slack for the alignment of the first load and the
// two words read past a field.
constexpr uint32_t kWaveStageWords = 1024 + 16;

__device__ inline uint32_t lane_id() { return threadIdx.x & (kWave - 1); }
// Wavefront index, read from the first lane so the compiler treats it (and
// every tile bound, partition index and record derived from it) as uniform:
// scalar registers and scalar loads instead of per-lane ones.
__device__ inline uint32_t wave_id() {
  return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
}

// Orders this wavefront's LDS writes before its later LDS reads (and the
// reverse); the lanes of a wavefront need no other synchronisation.
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ inline uint32_t chunk_values(uint32_t bits) {
  return bits == 0 ? 0xffffffffu : ((kWaveStageWords - 12) * 32u) / bits;
}

// Decodes values t in [c0, c1) of partition p from the staged words, in
// which residual t starts at bit qoff + b t.  Lane l takes t = c0 + l,
// c0 + l + 64, ...
//
// The round count is uniform: rounds 0 .. full-1 have every lane active
// and run unrolled by kUnroll with all residual reads of a group issued
// before any is used, so the LDS latency is paid once per group; the
// partial last round (lanes below rem) runs once under the lane mask.
// Residual extraction, prediction and the sink are chosen per partition
// outside the loops: U(i) gives the residual of round i, P(t) the
// prediction at t.
constexpr uint32_t kUnroll = 4;

template <class Sink, class Residual, class Predict>
__device__ inline void decode_rounds(const Part& p, uint32_t c0, uint32_t c1, Sink& sink,
                                     Residual U, Predict P) {
  const uint32_t lane = lane_id();
  const uint32_t n = c1 - c0;
  const uint32_t full = n / kWave, rem = n % kWave;
  const uint32_t first = c0 + lane;
  const uint64_t g_first = p.start + first;
  uint32_t i = 0;
  for (; i + kUnroll <= full; i += kUnroll) {
    decltype(U(0u)) u[kUnroll];
#pragma unroll
    for (uint32_t k = 0; k < kUnroll; ++k) u[k] = U(i + k);
#pragma unroll
    for (uint32_t k = 0; k < kUnroll; ++k) {
      const uint32_t r = i + k;
      sink.put(g_first + r * kWave, p.base + uint64_t(P(first + r * kWave)) + u[k]);
    }
  }
  for (; i < full; ++i) sink.put(g_first + i * kWave, p.base + uint64_t(P(first + i * kWave)) + U(i));
  if (lane < rem)
    sink.put(g_first + full * kWave, p.base + uint64_t(P(first + full * kWave)) + U(full));
}

template <class Sink>
__device__ inline void decode_values(const Part& p, uint32_t c0, uint32_t c1, int64_t qoff,
                                     const uint32_t* stage, Sink& sink) {
  const uint32_t b = p.bits;
  const double theta1 = p.theta1;
  const uint32_t first = c0 + lane_id();
  // Residual of round i starts at bit q0 + 64 b i of the stage.  64 b is a
  // multiple of 32, so the bit offset within a word (sh) is the same in
  // every round and the word index advances by 2 b per round.
  const uint32_t q0 = uint32_t(qoff + int64_t(b) * first);
  const uint32_t* lw = stage + (q0 >> 5);
  const uint32_t sh = q0 & 31, wstep = 2 * b;
  // With a non-negative slope every product is >= 0 (or +-0), so the floor
  // is the conversion's truncation toward zero.
  const bool nonneg = !(theta1 < 0.0);
  auto pred32 = [=](uint32_t t) { return int64_t(predict32(theta1, t)); };
  auto pred32_nn = [=](uint32_t t) { return int64_t(int32_t(__dmul_rn(theta1, double(t)))); };
  auto pred64 = [=](uint32_t t) { return predict(theta1, t); };
  auto zero = [](uint32_t) { return 0u; };
  const bool fits32 = prediction_fits_i32(theta1, p.len);
  if (b == 0) {
    if (fits32 && nonneg)
      decode_rounds(p, c0, c1, sink, zero, pred32_nn);
    else if (fits32)
      decode_rounds(p, c0, c1, sink, zero, pred32);
    else
      decode_rounds(p, c0, c1, sink, zero, pred64);
  } else if (b <= 32) {
    const uint32_t mask = b == 32 ? 0xffffffffu : ((1u << b) - 1u);
    auto res = [=](uint32_t i) {
      const uint32_t* w = lw + i * wstep;
      return __builtin_amdgcn_alignbit(w[1], w[0], sh) & mask;
    };
    if (fits32 && nonneg)
      decode_rounds(p, c0, c1, sink, res, pred32_nn);
    else if (fits32)
      decode_rounds(p, c0, c1, sink, res, pred32);
    else
      decode_rounds(p, c0, c1, sink, res, pred64);
  } else {
    const uint32_t mask_hi = b >= 64 ? 0xffffffffu : ((1u << (b - 32)) - 1u);
    auto res = [=](uint32_t i) {
      const uint32_t* w = lw + i * wstep;
      const uint32_t w0 = w[0], w1 = w[1], w2 = w[2];
      const uint32_t lo = __builtin_amdgcn_alignbit(w1, w0, sh);
      const uint32_t hi = __builtin_amdgcn_alignbit(w2, w1, sh) & mask_hi;
      return (uint64_t(hi) << 32) | lo;
    };
    decode_rounds(p, c0, c1, sink, res, pred64);
  }
}

// 32-bit word range [ws, we) (relative to the words section) holding the
// residuals t in [t0, t1) of partition p.
__device__ inline void word_span(const Part& p, uint32_t t0, uint32_t t1, uint64_t& ws,
                                 uint64_t& we) {
  ws = 2 * p.word_off + ((uint64_t(p.bits) * t0) >> 5);
  we = 2 * p.word_off + ((uint64_t(p.bits) * t1 + 31) >> 5);
}

// Copies 32-bit words [a0, w_end) (a0 a multiple of 4) into the stage with
// coalesced 16-byte loads by the lanes of one wavefront.
__device__ inline void stage_words(const uint32_t* __restrict__ words32, uint64_t a0,
                                   uint64_t w_end, uint32_t* stage) {
  const uint32_t nvec = uint32_t((w_end - a0 + 3) >> 2);
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const auto src = global_ptr(reinterpret_cast<const u32x4*>(words32 + a0));
  u32x4* dst = reinterpret_cast<u32x4*>(stage);
  for (uint32_t i = lane_id(); i < nvec; i += kWave) dst[i] = src[i];
}

constexpr uint32_t kMaxTileSegments = 64;

// Decodes one wavefront tile [g0, g1) of a blob into the sink.  Returns
// false if the blob failed validation (the caller raises the flag); all
// control flow is uniform across the wavefront.
//
// When the sink visits every segment (Sink::kWholeTile) and the words of
// all segments fit the slice, they are staged in one round trip; otherwise
// each segment is staged and decoded in chunks on its own.
template <class Sink>
__device__ bool decode_tile(const uint8_t* __restrict__ blob, const Header& h, uint64_t g0,
                            uint64_t g1, uint32_t* stage, Sink& sink) {
  const uint64_t j0 = locate(blob, h, g0);
  const uint32_t* words32 = reinterpret_cast<const uint32_t*>(blob + h.words_off);
  if (Sink::kWholeTile) {
    uint64_t j = j0, g = g0, span_lo = 0, span_hi = 0;
    uint32_t nseg = 0;
    bool one_round = true;
    while (g < g1) {
      Part p;
      if (!load_part(blob, h, j, p)) return false;
      if (g < p.start || g - p.start >= p.len) return false;
      const uint64_t seg_end = (p.start + p.len < g1) ? p.start + p.len : g1;
      uint64_t ws, we;
      word_span(p, uint32_t(g - p.start), uint32_t(seg_end - p.start), ws, we);
      if (nseg == 0) span_lo = ws;
      else if (ws < span_hi) one_round = false;  // spans must follow each other
      if (we > span_hi) span_hi = we;
      g = seg_end;
      ++j;
      if (++nseg >= kMaxTileSegments && g < g1) {
        one_round = false;
        break;
      }
    }
    const uint64_t a0 = span_lo & ~uint64_t(3);
    if (one_round && span_hi - a0 + 8 <= kWaveStageWords) {
      if (span_hi > span_lo) stage_words(words32, a0, span_hi, stage);
      wave_sync();
      j = j0;
      g = g0;
      while (g < g1) {
        Part p;
        load_part(blob, h, j, p);  // validated above
        const uint64_t seg_end = (p.start + p.len < g1) ? p.start + p.len : g1;
        const int64_t qoff = int64_t(64 * p.word_off) - int64_t(32 * a0);
        decode_values(p, uint32_t(g - p.start), uint32_t(seg_end - p.start), qoff, stage, sink);
        g = seg_end;
        ++j;
      }
      wave_sync();
      return true;
    }
  }
  uint64_t j = j0;
  while (g0 < g1) {
    Part p;
    if (!load_part(blob, h, j, p)) return false;
    if (g0 < p.start || g0 - p.start >= p.len) return false;
    const uint64_t seg_end = (p.start + p.len < g1) ? p.start + p.len : g1;
    const uint32_t t_end = uint32_t(seg_end - p.start);
    const uint32_t b = p.bits;
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
        uint64_t ws, we;
        word_span(p, c0, c1, ws, we);
        const uint64_t a0 = ws & ~uint64_t(3);
        stage_words(words32, a0, we, stage);
        qoff = int64_t(64 * p.word_off) - int64_t(32 * a0);
        wave_sync();
      }
      decode_values(p, c0, c1, qoff, stage, sink);
      if (b != 0) wave_sync();
      c0 = c1;
    }
    g0 = seg_end;
    ++j;
  }
  return true;
}

// The wavefront's share [g0, g1) of the workgroup tile [t0, t1): quarter w
// of it (tile boundaries are multiples of 4 values, so quarters are exact
// for full tiles; a ragged last tile gives empty quarters at its end).
__device__ inline void wave_share(uint64_t t0, uint64_t t1, uint32_t tile_log2, uint64_t& g0,
                                  uint64_t& g1) {
  const uint64_t q = uint64_t(1) << (tile_log2 - 2);
  const uint64_t w = wave_id();
  g0 = t0 + w * q;
  g1 = g0 + q;
  if (g0 > t1) g0 = t1;
  if (g1 > t1) g1 = t1;
}

// Writes each value to out[g - origin] with the column's width, bypassing
// the caches (outputs are written once and not read back by the kernel).
template <typename OutT>
struct StoreSink {
  static constexpr bool kWholeTile = true;
  OutT* out;
  uint64_t origin;
  __device__ bool visit_segment(const Part&, uint32_t, uint32_t) { return true; }
  __device__ void put(uint64_t g, uint64_t v) {
    __builtin_nontemporal_store(OutT(v), global_ptr(out + (g - origin)));
  }
};

// Maps a workgroup to a virtual index so that each XCD (workgroups are
// dispatched round-robin over the 8 XCDs) walks a contiguous run of tiles;
// grid must be a multiple of 8 for the mapping to be a permutation.
__device__ inline uint64_t xcd_virtual_block(uint32_t b, uint32_t grid, bool remap) {
  if (!remap || (grid & 7u)) return b;
  return uint64_t(b & 7u) * (grid >> 3) + (b >> 3);
}

__device__ inline void raise(int* err, int bits) { atomicOr(err, bits); }

// Random access (section 3.3): the value at position g < h.n, from the
// partition's record and the one or two words holding the residual.  False
// if the records around g are malformed.
__device__ inline bool lookup_value(const uint8_t* __restrict__ blob, const Header& h,
                                    uint64_t g, uint64_t& v) {
  const uint64_t j = locate(blob, h, g);
  Part p;
  if (!load_part(blob, h, j, p) || g < p.start || g - p.start >= p.len) return false;
  const uint32_t t = uint32_t(g - p.start);
  uint64_t u = 0;
  if (p.bits) {
    const uint64_t* words = reinterpret_cast<const uint64_t*>(blob + h.words_off);
    const uint64_t q = 64 * p.word_off + uint64_t(p.bits) * t;
    const uint32_t s = uint32_t(q & 63);
    const uint64_t lo = words[q >> 6];
    const uint64_t hi = (s + p.bits > 64) ? words[(q >> 6) + 1] : 0;
    u = (lo >> s) | ((hi << 1) << (63 - s));
    if (p.bits < 64) u &= (uint64_t(1) << p.bits) - 1;
  }
  v = p.base + uint64_t(predict(p.theta1, t)) + u;
  return true;
}

// Accumulates sum and count of values in [lo, hi).  A segment is skipped
// without reading its residuals when the model bounds its values outside
// [lo, hi): values of a partition lie in
//   [base + min_t floor(theta1 t), base + max_t floor(theta1 t) + 2^b - 1]
// (the prediction is monotone in t), and the bound is used only when that
// interval, evaluated exactly, lies inside [0, 2^64) so that no value wraps.
struct FilterSink {
  static constexpr bool kWholeTile = false;  // may skip segments by their model bounds
  uint64_t lo, hi;
  uint64_t sum_lo, sum_hi, count;
  int prune;
  __device__ bool visit_segment(const Part& p, uint32_t t0, uint32_t t1) {
    if (!prune) return true;
    const int64_t pa = predict(p.theta1, t0), pb = predict(p.theta1, t1 - 1);
    const int64_t pmin = pa < pb ? pa : pb, pmax = pa < pb ? pb : pa;
    // exact [base + pmin, base + pmax + 2^b - 1] as 128-bit signed values
    const __int128 base = __int128(p.base);
    const __int128 vmin = base + pmin;
    const __int128 span = p.bits >= 64 ? (__int128(1) << 64) - 1 : (__int128(1) << p.bits) - 1;
    const __int128 vmax = base + pmax + span;
    const __int128 top = __int128(1) << 64;
    if (vmin < 0 || vmax >= top) return true;  // no safe bound
    return !(vmax < __int128(lo) || vmin >= __int128(hi));
  }
  __device__ void put(uint64_t, uint64_t v) {
    if (v >= lo && v < hi) {
      const uint64_t s = sum_lo + v;
      sum_hi += (s < sum_lo);
      sum_lo = s;
      ++count;
    }
  }
};

// Adds a workgroup's (sum_lo, sum_hi, count) into out3 exactly.  Called by
// every thread of the workgroup.
__device__ inline void block_add_sum(uint64_t sum_lo, uint64_t sum_hi, uint64_t count,
                                     uint64_t* out3) {
  __shared__ uint64_t red[3][kBlock];
  const uint32_t tid = threadIdx.x;
  red[0][tid] = sum_lo;
  red[1][tid] = sum_hi;
  red[2][tid] = count;
  __syncthreads();
  for (uint32_t s = kBlock / 2; s > 0; s >>= 1) {
    if (tid < s) {
      const uint64_t a = red[0][tid], b = red[0][tid + s];
      red[0][tid] = a + b;
      red[1][tid] += red[1][tid + s] + (a + b < a);
      red[2][tid] += red[2][tid + s];
    }
    __syncthreads();
  }
  if (tid == 0 && (red[0][0] | red[1][0] | red[2][0])) {
    const uint64_t x = red[0][0];
    const uint64_t old = atomicAdd(reinterpret_cast<unsigned long long*>(out3), x);
    const uint64_t carry = (old + x < old) ? 1 : 0;
    atomicAdd(reinterpret_cast<unsigned long long*>(out3 + 1), red[1][0] + carry);
    atomicAdd(reinterpret_cast<unsigned long long*>(out3 + 2), red[2][0]);
  }
  __syncthreads();
}

}  // namespace leco
