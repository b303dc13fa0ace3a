// The LeCo decoder's inner loop (section 3.3, range decompression), built
// around wavefront tiles: each 64-lane wavefront decodes the values of
// global positions [g0, g1) (up to 4096 of them, as many as the blob's bits
// per value let its words fit the slice) on its own, with its own slice of
// LDS and no workgroup barrier.  The tile is cut at partition boundaries
// into segments; the residual words of all its segments (which lie back to
// back in the blob) are copied once into the wavefront's LDS slice with
// coalesced 16-byte loads, then each lane decodes values t = c0 + lane,
// c0 + lane + 64, ... so that every store of the wavefront covers 64
// consecutive outputs; runs of short partitions are decoded in full
// 64-value rounds across their boundaries.  Tiles whose words do not fit
// the slice are decoded segment by segment in chunks.
#pragma once

#include "leco_dev.hpp"

namespace leco {

constexpr int kBlock = 256;
constexpr int kWave = 64;
constexpr int kWavesPerBlock = kBlock / kWave;
// 32-bit words of LDS per wavefront for residuals: 1024 words (1024 values
// at up to 32 bits) plus slack for the alignment of the first load and the
// two words read past a field.
constexpr uint32_t kWaveStageWords = 1024 + 16;
// A piece of a tile covers at most kPieceSegs partitions (kFlatPieceSegs
// when runs of short partitions may be decoded in full rounds); their
// records sit in LDS after the residual words while the piece is decoded.
constexpr uint32_t kPieceSegs = 16;
constexpr uint32_t kFlatPieceSegs = 64;
struct PieceRec {
  uint64_t base, theta_bits;
  int32_t start;  // partition start minus the piece's first position
  uint32_t len;
  int32_t qoff;   // stage bit of residual t = 0 (0 when b = 0)
  uint32_t bits;
};
static_assert(sizeof(PieceRec) == 32, "two 16-byte LDS reads per record");
// Pieces of at most kFlatSpan values whose partitions are shorter than
// kFlatMeanLen on average are decoded lane by lane across partition
// boundaries, with a bitmap of the piece's partition starts in LDS.
constexpr uint32_t kFlatSpan = 4096;
constexpr uint32_t kFlatMeanLen = 256;
constexpr uint32_t kBitmapWords = kFlatSpan / 32;
constexpr uint32_t kFlatUnroll = 4;
// LDS per wavefront: residual words, the piece's records and, for a sink
// that allows full-round decoding (Sink::kFlat), the start bitmap.  A sink
// that may skip segments decodes segment by segment and needs the residual
// words only.
template <class Sink>
constexpr uint32_t piece_segs() {
  return Sink::kFlat ? kFlatPieceSegs : kPieceSegs;
}
template <class Sink>
constexpr uint32_t slot_words() {
  return !Sink::kWholeTile ? kWaveStageWords
                           : kWaveStageWords + piece_segs<Sink>() * sizeof(PieceRec) / 4 +
                                 (Sink::kFlat ? kBitmapWords : 0);
}

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

// Decodes the piece [g0, g0 + span) whose records are in `table` and whose
// residual words are staged, 64 consecutive values per round whatever the
// partition boundaries: bit x of `starts` marks a partition start at g0 + x
// (the first partition, which holds g0, has none), so the partition of
// value x is the number of marked bits at or below x, counted for the
// whole round from the wavefront's ballot.
//
// kRes: 0 when every width is 0 (no residual), 1 when every width is at
// most 32, 2 otherwise; kFast: every slope is >= 0 and every prediction
// below 2^31; kConst: every width and slope is 0 (runs of one value), so
// each value is its partition's intercept.  kN rounds from r0 are decoded with their LDS reads grouped;
// kMasked: the last round of the piece, where lanes past the span decode
// its last value and store nothing.
constexpr uint32_t kResZero = 0, kResNarrow = 1, kResWide = 2;

template <uint32_t kN, bool kMasked, uint32_t kRes, bool kFast, bool kConst, class Sink>
__device__ inline void flat_rounds(uint32_t r0, uint32_t& k_before, uint64_t g0, uint32_t span,
                                   const PieceRec* table, const uint32_t* starts,
                                   const uint32_t* stage, Sink& sink) {
  const uint32_t lane = lane_id();
  uint32_t x[kN], k[kN];
#pragma unroll
  for (uint32_t i = 0; i < kN; ++i) {
    x[i] = (r0 + i) * kWave + lane;
    k[i] = __builtin_amdgcn_ubfe(starts[x[i] >> 5], x[i] & 31, 1);
  }
#pragma unroll
  for (uint32_t i = 0; i < kN; ++i) {
    const uint64_t m = __ballot(k[i]);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi(
        uint32_t(m >> 32), __builtin_amdgcn_mbcnt_lo(uint32_t(m), 0u));
    k[i] += k_before + below;
    k_before += uint32_t(__popcll(m));
  }
  if (kConst) {
    uint64_t base[kN];
#pragma unroll
    for (uint32_t i = 0; i < kN; ++i) base[i] = table[k[i]].base;
#pragma unroll
    for (uint32_t i = 0; i < kN; ++i)
      if (!kMasked || x[i] < span) sink.put(g0 + x[i], base[i]);
    return;
  }
  PieceRec rec[kN];
#pragma unroll
  for (uint32_t i = 0; i < kN; ++i) rec[i] = table[k[i]];
  uint32_t t[kN];
  uint64_t u[kN];
#pragma unroll
  for (uint32_t i = 0; i < kN; ++i) {
    const uint32_t xc = (kMasked && x[i] >= span) ? span - 1 : x[i];
    t[i] = uint32_t(int32_t(xc) - rec[i].start);
    const uint32_t b = rec[i].bits;
    const uint32_t q = uint32_t(rec[i].qoff) + b * t[i];
    const uint32_t* w = stage + (q >> 5);
    const uint32_t sh = q & 31;
    if (kRes == kResZero) {
      u[i] = 0;
    } else if (kRes == kResWide) {
      const uint32_t w0 = w[0], w1 = w[1], w2 = w[2];
      const uint64_t v = (uint64_t(__builtin_amdgcn_alignbit(w2, w1, sh)) << 32) |
                         __builtin_amdgcn_alignbit(w1, w0, sh);
      u[i] = b >= 64 ? v : v & ((uint64_t(1) << b) - 1);
    } else {
      const uint32_t v = __builtin_amdgcn_alignbit(w[1], w[0], sh);
      u[i] = b >= 32 ? v : v & ((1u << b) - 1u);
    }
  }
#pragma unroll
  for (uint32_t i = 0; i < kN; ++i) {
    const double th = __longlong_as_double(static_cast<long long>(rec[i].theta_bits));
    const int64_t p = kFast ? int64_t(int32_t(__dmul_rn(th, double(t[i])))) : predict(th, t[i]);
    if (!kMasked || x[i] < span) sink.put(g0 + x[i], rec[i].base + uint64_t(p) + u[i]);
  }
}

template <uint32_t kRes, bool kFast, bool kConst = false, class Sink>
__device__ inline void decode_piece_flat(uint64_t g0, uint32_t span, const PieceRec* table,
                                         const uint32_t* starts, const uint32_t* stage,
                                         Sink& sink) {
  const uint32_t full = span / kWave;
  uint32_t k_before = 0;  // partition of the value before the round, uniform
  uint32_t r = 0;
  for (; r + kFlatUnroll <= full; r += kFlatUnroll)
    flat_rounds<kFlatUnroll, false, kRes, kFast, kConst>(r, k_before, g0, span, table, starts,
                                                         stage, sink);
  for (; r < full; ++r)
    flat_rounds<1, false, kRes, kFast, kConst>(r, k_before, g0, span, table, starts, stage, sink);
  if (span % kWave)
    flat_rounds<1, true, kRes, kFast, kConst>(r, k_before, g0, span, table, starts, stage, sink);
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

// A value the wavefront holds in every lane, moved to scalar registers.
__device__ inline uint64_t uniform_u64(uint64_t x) {
  const uint32_t lo = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(x))));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(x >> 32))));
  return (uint64_t(hi) << 32) | lo;
}

// Lane k's value of x, k uniform across the wavefront.
__device__ inline uint64_t lane_u64(uint64_t x, uint32_t k) {
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x)), int(k)));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x >> 32)), int(k)));
  return (uint64_t(hi) << 32) | lo;
}

// Partition holding g (as locate), searched by the whole wavefront: each
// round probes 64 evenly spaced starts at once, so a variable-length blob
// of m partitions needs about log_65(m) dependent loads instead of
// log_2(m).  Fixed lengths are located arithmetically.
__device__ inline uint64_t locate_wave(const uint8_t* blob, const Header& h, uint64_t g) {
  if (!h.variable) return locate(blob, h, g);
  const MetaPtr s = meta_words(blob, h.starts_off);
  const uint32_t lane = lane_id();
  uint64_t lo = 0, hi = h.m;  // the last start <= g lies in [lo, hi)
  while (hi - lo > kWave) {
    const uint64_t q = lo + (hi - lo) * (lane + 1) / (kWave + 1);  // lo < q < hi
    const uint64_t below = __ballot(s[q] <= g);
    const uint32_t c = uint32_t(__popcll(below & (~0ull >> (64 - kWave))));
    const uint64_t q_lo = lane_u64(q, c ? c - 1 : 0), q_hi = lane_u64(q, c < kWave ? c : 0);
    if (c) lo = q_lo;
    if (c < kWave) hi = q_hi;
  }
  const uint64_t q = lo + lane;
  const uint64_t below = __ballot(q < hi && s[q] <= g);
  const uint32_t c = uint32_t(__popcll(below));
  return c ? lo + c - 1 : lo;
}

// Decodes one wavefront tile [g0, g1) of a blob into the sink.  Returns
// false if the blob failed validation (the caller raises the flag); all
// control flow is uniform across the wavefront.
//
// When the sink visits every segment (Sink::kWholeTile) the tile goes in
// pieces of up to piece_segs<Sink>() partitions: lane k loads and checks the
// record of the piece's k-th partition (one round trip for all of them)
// and parks it in the wavefront's LDS slot, the residual words of the whole
// piece are staged in one round trip, and the segments are decoded from
// the stage one after the other, or, for a piece of short partitions and a
// sink that allows it (Sink::kFlat), lane by lane across the partition
// boundaries (decode_piece_flat).  A piece whose words do not fit the slot,
// and every tile of a sink that may skip segments, is decoded segment by
// segment in chunks instead.
template <class Sink>
__device__ bool decode_tile(const uint8_t* __restrict__ blob, const Header& h, uint64_t g0,
                            uint64_t g1, uint32_t* stage, Sink& sink) {
  uint64_t j0 = locate_wave(blob, h, g0);
  const uint32_t* words32 = reinterpret_cast<const uint32_t*>(blob + h.words_off);
  if (Sink::kWholeTile) {
    const uint32_t lane = lane_id();
    PieceRec* table = reinterpret_cast<PieceRec*>(stage + kWaveStageWords);
    constexpr uint32_t kSegs = piece_segs<Sink>();
    uint32_t* bitmap = stage + kWaveStageWords + kSegs * sizeof(PieceRec) / 4;
    while (g0 < g1) {
      // lane k < kSegs: partition j0 + k, a segment of the piece if it
      // starts before g1
      const uint64_t jl = j0 + lane;
      const bool want = lane < kSegs && jl < h.m && (lane == 0 || part_start(blob, h, jl) < g1);
      Part lp{0, 0, 0, 0.0, 0, 0};
      const bool ok = want && load_part(blob, h, jl, lp);
      if (__ballot(want && !ok)) return false;
      const uint64_t segs = __ballot(want);
      const uint32_t nseg = uint32_t(__popcll(segs));
      if (nseg == 0 || segs != (~0ull >> (64 - nseg))) return false;  // starts must increase
      const uint64_t end_l = lp.start + lp.len;
      if (g0 < lane_u64(lp.start, 0) || g0 >= lane_u64(end_l, 0)) return false;
      // the piece [g0, ge): its segments' residual word spans must follow
      // each other for one staging round trip (partitions are contiguous by
      // construction, each length coming from the next start; the spans
      // are contiguous only in a valid blob)
      const uint64_t last_end = lane_u64(end_l, nseg - 1);
      const uint64_t ge = last_end < g1 ? last_end : g1;
      const uint64_t t0 = (g0 > lp.start ? g0 : lp.start) - lp.start;
      const uint64_t t1 = (ge < end_l ? ge : end_l) - lp.start;
      uint64_t ws = 0, we = 0;
      if (want) word_span(lp, uint32_t(t0), uint32_t(t1), ws, we);
      const uint64_t prev_we = uint64_t(__shfl_up(static_cast<unsigned long long>(we), 1, kWave));
      const bool gap = want && lane > 0 && ws < prev_we;
      const uint64_t span_lo = lane_u64(ws, 0), span_hi = lane_u64(we, nseg - 1);
      const uint64_t a0 = span_lo & ~uint64_t(3);
      if (__ballot(gap) || span_hi - a0 + 8 > kWaveStageWords) break;  // chunked path
      const uint32_t span = uint32_t(ge - g0);
      const bool flat =
          Sink::kFlat && nseg > 1 && span <= kFlatSpan && span < kFlatMeanLen * nseg;
      if (flat) {
        for (uint32_t i = lane; i < kBitmapWords; i += kWave) bitmap[i] = 0;
        wave_sync();
      }
      if (want) {
        // lane 0's partition holds g0; the others start inside the piece
        const int32_t qoff = lp.bits ? int32_t(int64_t(64 * lp.word_off) - int64_t(32 * a0)) : 0;
        table[lane] = PieceRec{lp.base, uint64_t(__double_as_longlong(lp.theta1)),
                               int32_t(int64_t(lp.start) - int64_t(g0)), uint32_t(lp.len), qoff,
                               lp.bits};
        if (flat && lane > 0) {
          const uint32_t x = uint32_t(lp.start - g0);
          atomicOr(&bitmap[x >> 5], 1u << (x & 31));
        }
      }
      const bool wide = flat && __ballot(want && lp.bits > 32) != 0;
      const bool zero = flat && __ballot(want && lp.bits != 0) == 0;
      const bool cnst = zero && __ballot(want && lp.theta1 != 0.0) == 0;
      const bool fast =
          flat && __ballot(want && (lp.theta1 < 0.0 || !prediction_fits_i32(lp.theta1, lp.len))) == 0;
      if (span_hi > span_lo) stage_words(words32, a0, span_hi, stage);
      wave_sync();
      if (flat) {
        if (wide)
          decode_piece_flat<kResWide, false>(g0, span, table, bitmap, stage, sink);
        else if (cnst)
          decode_piece_flat<kResZero, true, true>(g0, span, table, bitmap, stage, sink);
        else if (zero && fast)
          decode_piece_flat<kResZero, true>(g0, span, table, bitmap, stage, sink);
        else if (zero)
          decode_piece_flat<kResZero, false>(g0, span, table, bitmap, stage, sink);
        else if (fast)
          decode_piece_flat<kResNarrow, true>(g0, span, table, bitmap, stage, sink);
        else
          decode_piece_flat<kResNarrow, false>(g0, span, table, bitmap, stage, sink);
      } else {
        for (uint32_t k = 0; k < nseg; ++k) {
          const PieceRec r = table[k];
          Part p;
          p.start = uint64_t(int64_t(g0) + int32_t(__builtin_amdgcn_readfirstlane(r.start)));
          p.len = uint32_t(__builtin_amdgcn_readfirstlane(int(r.len)));
          p.base = uniform_u64(r.base);
          p.theta1 = __longlong_as_double(static_cast<long long>(uniform_u64(r.theta_bits)));
          p.word_off = 0;  // the stage offset is qoff
          p.bits = uint32_t(__builtin_amdgcn_readfirstlane(int(r.bits)));
          const int64_t qoff = int32_t(__builtin_amdgcn_readfirstlane(r.qoff));
          const uint64_t s0 = g0 > p.start ? g0 : p.start;
          const uint64_t s1 = ge < p.start + p.len ? ge : p.start + p.len;
          decode_values(p, uint32_t(s0 - p.start), uint32_t(s1 - p.start), qoff, stage, sink);
        }
      }
      wave_sync();
      g0 = ge;
      j0 += nseg;
    }
    if (g0 >= g1) return true;
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
// kFlatRuns: runs of short partitions may be decoded in full rounds (which
// costs the kernel LDS and registers).
template <typename OutT, bool kFlatRuns = true>
struct StoreSink {
  static constexpr bool kWholeTile = true;
  static constexpr bool kFlat = kFlatRuns;
  static constexpr bool kGramWalk = true;
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

// ---- blobs with a polynomial coefficient section -----------------------------------
//
// Such blobs (header flag kFlagPoly) mix linear records (kind 0) and
// polynomial ones (kind 1: c1 in the slope field, c2 and c3 in the
// coefficient section).  They are decoded value by value from global
// memory: one wavefront walks the partitions of its share, reading each
// record and its coefficients with scalar loads, and its lanes take
// consecutive values of the partition.

// Kind and coefficients of partition j (kind 1 needs the coefficient
// section and at most kPolyMaxLen values); false if malformed.
__device__ inline bool load_model_kind(const uint8_t* blob, const Header& h, uint64_t j,
                                       const Part& p, uint32_t& kind, double& c2, double& c3) {
  kind = uint32_t(meta_words(blob, kHeaderBytes + kRecordBytes * j)[3] >> 8) & 0xff;
  c2 = c3 = 0.0;
  if (kind == 0) return true;
  if (kind > 1 || !h.poly || p.len > kPolyMaxLen) return false;
  const MetaPtr cf = meta_words(blob, h.coef_off + 16 * j);
  c2 = __longlong_as_double(static_cast<long long>(cf[0]));
  c3 = __longlong_as_double(static_cast<long long>(cf[1]));
  return true;
}

// The residual of position t of partition p, read from global memory.
__device__ inline uint64_t residual_at(const uint64_t* words, const Part& p, uint64_t t) {
  if (p.bits == 0) return 0;
  const uint64_t q = 64 * p.word_off + uint64_t(p.bits) * t;
  const uint32_t s = uint32_t(q & 63);
  const uint64_t lo = words[q >> 6];
  const uint64_t hi = (s + p.bits > 64) ? words[(q >> 6) + 1] : 0;
  uint64_t u = (lo >> s) | ((hi << 1) << (63 - s));
  if (p.bits < 64) u &= (uint64_t(1) << p.bits) - 1;
  return u;
}

// Values [g0, g1) of a blob with coefficient section, by one wavefront;
// false if a record is malformed.  Each partition's residual words are
// staged in the wavefront's LDS slice (in chunks that fit it) with
// coalesced 16-byte loads, then lane l decodes t = c0 + l, c0 + l + 64, ...
// from the stage, so no lane waits on a global load of its own.
template <class Sink>
__device__ bool decode_range_poly(const uint8_t* __restrict__ blob, const Header& h, uint64_t g0,
                                  uint64_t g1, uint32_t* stage, Sink& sink) {
  const uint32_t* words32 = reinterpret_cast<const uint32_t*>(blob + h.words_off);
  const uint32_t lane = lane_id();
  uint64_t j = uniform_u64(locate(blob, h, g0));
  for (uint64_t g = g0; g < g1; ++j) {
    Part p;
    uint32_t kind;
    double c2, c3;
    if (!load_part(blob, h, j, p) || g < p.start || g - p.start >= p.len ||
        !load_model_kind(blob, h, j, p, kind, c2, c3))
      return false;
    const uint64_t end = p.start + p.len < g1 ? p.start + p.len : g1;
    const uint32_t b = p.bits, t_end = uint32_t(end - p.start);
    const uint64_t mask = b >= 64 ? ~uint64_t(0) : (uint64_t(1) << b) - 1;
    const uint32_t step = chunk_values(b);
    for (uint32_t c0 = uint32_t(g - p.start); c0 < t_end;) {
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
      // three words cover any field of up to 64 bits; the words past the
      // staged ones only meet masked bits
      const auto field = [&](uint32_t t) -> uint64_t {
        if (b == 0) return 0;
        const uint32_t q = uint32_t(qoff + int64_t(b) * t);
        const uint32_t* w = stage + (q >> 5);
        const uint32_t w0 = w[0], w1 = w[1], w2 = w[2];
        return ((uint64_t(__builtin_amdgcn_alignbit(w2, w1, q & 31)) << 32) |
                __builtin_amdgcn_alignbit(w1, w0, q & 31)) & mask;
      };
      if (kind && Sink::kGramWalk) {
        // sinks that only store: the lane's Gram polynomials by forward
        // differences (its positions are kWave apart); the filtering sinks
        // evaluate them per value, which keeps those kernels within their
        // register budgets on every blob
        GramWalk gw;
        gw.start(c0 + lane, uint32_t(p.len), kWave);
        for (uint32_t t = c0 + lane; t < c1; t += kWave) {
          const uint64_t u = field(t);
          sink.put(p.start + t, p.base + uint64_t(gw.predict(p.theta1, c2, c3)) + u);
          gw.next();
        }
      } else if (kind) {
        for (uint32_t t = c0 + lane; t < c1; t += kWave)
          sink.put(p.start + t,
                   p.base + uint64_t(poly_predict(p.theta1, c2, c3, t, uint32_t(p.len))) + field(t));
      } else {
        for (uint32_t t = c0 + lane; t < c1; t += kWave)
          sink.put(p.start + t, p.base + uint64_t(predict(p.theta1, t)) + field(t));
      }
      if (b != 0) wave_sync();
      c0 = c1;
    }
    g = end;
  }
  return true;
}

// Random access into a blob with coefficient section.
__device__ inline bool lookup_value_poly(const uint8_t* __restrict__ blob, const Header& h,
                                         uint64_t g, uint64_t& v) {
  const uint64_t j = locate(blob, h, g);
  Part p;
  uint32_t kind;
  double c2, c3;
  if (!load_part(blob, h, j, p) || g < p.start || g - p.start >= p.len ||
      !load_model_kind(blob, h, j, p, kind, c2, c3))
    return false;
  const uint32_t t = uint32_t(g - p.start);
  const int64_t pred = kind ? poly_predict(p.theta1, c2, c3, t, uint32_t(p.len))
                            : predict(p.theta1, t);
  v = p.base + uint64_t(pred) + residual_at(reinterpret_cast<const uint64_t*>(blob + h.words_off),
                                            p, t);
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
  static constexpr bool kFlat = false;
  static constexpr bool kGramWalk = false;
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
  // wavefront sums by butterfly shuffles (128-bit adds with carry), then
  // the workgroup's kWavesPerBlock partials through LDS
  __shared__ uint64_t red[kWavesPerBlock][3];
  for (int m = kWave / 2; m > 0; m >>= 1) {
    const uint64_t lo = __shfl_xor(static_cast<unsigned long long>(sum_lo), m, kWave);
    const uint64_t hi = __shfl_xor(static_cast<unsigned long long>(sum_hi), m, kWave);
    const uint64_t c = __shfl_xor(static_cast<unsigned long long>(count), m, kWave);
    const uint64_t s = sum_lo + lo;
    sum_hi += hi + (s < sum_lo ? 1 : 0);
    sum_lo = s;
    count += c;
  }
  const uint32_t w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    red[w][0] = sum_lo;
    red[w][1] = sum_hi;
    red[w][2] = count;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t lo = 0, hi = 0, c = 0;
    for (uint32_t i = 0; i < kWavesPerBlock; ++i) {
      const uint64_t s = lo + red[i][0];
      hi += red[i][1] + (s < lo ? 1 : 0);
      lo = s;
      c += red[i][2];
    }
    if (lo | hi | c) {
      const uint64_t old = atomicAdd(reinterpret_cast<unsigned long long*>(out3), lo);
      const uint64_t carry = (old + lo < old) ? 1 : 0;
      atomicAdd(reinterpret_cast<unsigned long long*>(out3 + 1), hi + carry);
      atomicAdd(reinterpret_cast<unsigned long long*>(out3 + 2), c);
    }
  }
  __syncthreads();
}

}  // namespace leco
