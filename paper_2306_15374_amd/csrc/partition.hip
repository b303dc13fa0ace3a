// Variable-length partitioner (section 3.2.2) on the GPU.
//
// Split: the greedy of the paper, which includes the next value in the
// current partition while the approximate cost of doing so,
//   C = (len + 1) * D~new - len * D~old,  D~ = bitlen(max d - min d)
// over the partition's first differences d, stays within tau * S_M, and
// the partition holds fewer than max_len values.  The column is cut into
// 2^14-value sub-chunks that are first split speculatively in parallel, as
// if a partition began at each one's start.  One wavefront per 2^20-value
// segment then walks the segment's sub-chunks in order from the true state,
// each until the true run starts a partition where the speculative run did
// (from there on the two runs are the same), rewriting the starts it
// passes; a last wavefront does the same across segments, from the end
// state of each segment to the next.  The wavefront walks 64 candidates at a
// time (see greedy_walk).  This reproduces the sequential greedy exactly.
// Optionally the split also honours starting partitions (section 3.2.2,
// selecting good starting positions): runs of smallest second-order delta,
// whose first value begins a partition and whose other values join it
// without the cost test.
//
// Merge: the paper's scan.  The current partition merges with its right
// neighbour when the union (sized with the encoder's own fit: 32-byte
// record, 8-byte start, residual words) is strictly smaller than the two
// apart and fits max_len, and then tries the next neighbour; passes repeat
// until one merges nothing.  The scan's state is the current partition
// (its first index and size), and it is reset by every refused merge, so
// the same speculation applies: chunks of the partition list are scanned
// in parallel as if a partition began at each chunk's start; then, in
// rounds of alternating parity, every chunk whose left neighbour's end
// state changed is walked again from it until it keeps a boundary its
// recorded run also kept.  A run of merges spanning c chunks takes about c
// rounds.  Within a run, 64 steps are sized at once (one per lane), and a
// long current partition is represented by the convex hulls of its points,
// which bound its residuals exactly for any slope, so a step costs the
// values it adds rather than the whole union.
#include <math.h>

#include <utility>
#include <vector>

#include "fit.hpp"
#include "internal.hpp"
#include "leco_dev.hpp"

namespace leco {

constexpr uint32_t kSegLog2 = 20;
constexpr uint32_t kSubLog2 = 14;  // speculative split sub-chunks of a segment
constexpr uint32_t kSplitWindow = 1024;  // values staged in LDS per window
constexpr uint32_t kScanBlock = 256;
constexpr uint32_t kItemsPerBlock = 1024;  // bitmap words or flags per scan block
constexpr uint64_t kNoMerge = ~uint64_t(0);

// A first difference d = v_j - v_{j-1} of (up to) 64-bit values as the
// 65-bit unsigned number d + 2^64 = (hi, lo), which orders like d.
struct DKey {
  uint32_t hi;
  uint64_t lo;
};

__device__ inline bool key_less(const DKey& a, const DKey& b) {
  return a.hi != b.hi ? a.hi < b.hi : a.lo < b.lo;
}

__device__ inline DKey key_shfl_up(const DKey& k, int delta) {
  DKey r;
  r.hi = uint32_t(__shfl_up(int(k.hi), delta, 64));
  r.lo = uint64_t(__shfl_up(static_cast<unsigned long long>(k.lo), delta, 64));
  return r;
}

__device__ inline DKey key_readlane(const DKey& k, int lane) {
  DKey r;
  r.hi = uint32_t(__shfl(int(k.hi), lane, 64));
  r.lo = uint64_t(__shfl(static_cast<unsigned long long>(k.lo), lane, 64));
  return r;
}

// bitlen(max - min) of two keys (at most 65).
__device__ inline uint32_t key_span_bits(const DKey& mn, const DKey& mx) {
  const uint64_t lo = mx.lo - mn.lo;
  const uint32_t hi = mx.hi - mn.hi - (mx.lo < mn.lo ? 1u : 0u);
  return hi ? 65u : bitlen64(lo);
}

// For 32-bit columns a first difference fits 33 bits: the key d + 2^32 is
// one 64-bit word (two 32-bit shuffles instead of three).
__device__ inline bool key_less(uint64_t a, uint64_t b) { return a < b; }
__device__ inline uint64_t key_shfl_up(uint64_t k, int delta) {
  return uint64_t(__shfl_up(static_cast<unsigned long long>(k), delta, 64));
}
__device__ inline uint64_t key_readlane(uint64_t k, int lane) {
  return uint64_t(__shfl(static_cast<unsigned long long>(k), lane, 64));
}
__device__ inline uint32_t key_span_bits(uint64_t mn, uint64_t mx) { return bitlen64(mx - mn); }

// Key of the first difference v_j - v_{j-1}, and the state's stored form.
__device__ inline DKey make_key(DKey*, uint64_t vj, uint64_t vp) {
  return DKey{vj >= vp ? 1u : 0u, vj - vp};
}
__device__ inline uint64_t make_key(uint64_t*, uint64_t vj, uint64_t vp) {
  return vj - vp + (uint64_t(1) << 32);  // v < 2^32
}
__device__ inline DKey key_from(DKey*, uint32_t hi, uint64_t lo) { return DKey{hi, lo}; }
__device__ inline uint64_t key_from(uint64_t*, uint32_t, uint64_t lo) { return lo; }
__device__ inline uint32_t key_hi(const DKey& k) { return k.hi; }
__device__ inline uint32_t key_hi(uint64_t) { return 0; }
__device__ inline uint64_t key_lo(const DKey& k) { return k.lo; }
__device__ inline uint64_t key_lo(uint64_t k) { return k; }

__device__ inline void mark(unsigned long long* bitmap, uint64_t j) {
  atomicOr(bitmap + (j >> 6), 1ull << (j & 63));
}

// The greedy's state: the current partition's first value i, and whether
// it has first differences yet with their min / max keys and D~.
struct SplitState {
  uint64_t i;
  uint64_t kmin_lo, kmax_lo;
  uint32_t kmin_hi, kmax_hi;
  uint32_t w_old, have;
};

// Clears bits [x, y) of the bitmap (y - x <= 128, so at most three words).
__device__ inline void clear_bits(unsigned long long* bitmap, uint64_t x, uint64_t y) {
  while (x < y) {
    const uint64_t w = x >> 6;
    const uint64_t hi = (y - (w << 6)) < 64 ? y - (w << 6) : 64;  // bit bound in word w
    const uint64_t lo = x & 63;
    const uint64_t mask = (hi == 64 ? ~0ull : ((1ull << hi) - 1)) & ~((1ull << lo) - 1);
    atomicAnd(bitmap + w, ~mask);
    x = (w + 1) << 6;
  }
}

__device__ inline bool bit_set(unsigned long long* bitmap, uint64_t j) {
  const unsigned long long word =
      __hip_atomic_load(bitmap + (j >> 6), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return (word >> (j & 63)) & 1ull;
}

// Runs the greedy over candidates [p, b) from state st, 64 candidates per
// step: lane l assumes the values before its own are all included, takes
// the inclusive prefix min / max of the first differences over the lanes
// below it and evaluates C; the first lane that fails starts the next
// partition and the lanes after it are retried from there.
//
// kFix = false: sets the bit of every start.  kFix = true: the bits in
// [p, b) are a speculative run's, made from a different state; the walk
// rewrites them until it starts a partition where the speculative run also
// did (from there on both runs are the same), returning true at that point.
//
// forced and inside (both null, or both bitmaps over the column): bit j of
// forced set means a partition begins at j (the first value of a starting
// partition), whatever the cost; bit j of inside set means v[j] joins the
// current partition without the cost test (a later value of a starting
// partition).  The length cap applies to both.
//
// K: the key type, DKey for 64-bit columns, one 64-bit word for 32-bit ones.
template <bool kFix, class K>
__device__ bool greedy_walk(const uint8_t* __restrict__ col, uint32_t dtype, uint64_t p,
                            uint64_t b, double thr, uint64_t max_len, SplitState& st,
                            uint64_t* win, unsigned long long* __restrict__ bitmap,
                            const uint64_t* __restrict__ forced,
                            const uint64_t* __restrict__ inside) {
  const uint32_t lane = threadIdx.x & 63;
  K kmin = key_from(static_cast<K*>(nullptr), st.kmin_hi, st.kmin_lo);
  K kmax = key_from(static_cast<K*>(nullptr), st.kmax_hi, st.kmax_lo);
  uint64_t i = st.i;
  bool have = st.have != 0;
  uint32_t w_old = st.w_old;
  uint64_t base = 0, wend = 0;  // the window holds v[base - 1, wend)
  bool synced = false;
  while (p < b) {
    const uint64_t need = p + 64 < b ? p + 64 : b;
    if (wend < need) {
      __syncthreads();  // every lane is done with the old window
      base = p;
      wend = b - p < kSplitWindow ? b : p + kSplitWindow;
      for (uint64_t k = lane; k <= wend - base; k += 64)
        win[k] = load_value(col, dtype, base - 1 + k);
      __syncthreads();
    }
    const uint64_t j = p + lane;
    const bool valid = j < b;
    K d = make_key(static_cast<K*>(nullptr), 0, 0);
    if (valid) d = make_key(static_cast<K*>(nullptr), win[j - base + 1], win[j - base]);
    // inclusive prefix min / max over the lanes up to this one; the invalid
    // lanes are the last ones and never feed a valid lane
    K mn = d, mx = d;
#pragma unroll
    for (int delta = 1; delta < 64; delta <<= 1) {
      const K lo = key_shfl_up(mn, delta), hi = key_shfl_up(mx, delta);
      if (int(lane) >= delta) {
        if (key_less(lo, mn)) mn = lo;
        if (key_less(mx, hi)) mx = hi;
      }
    }
    if (have) {
      if (key_less(kmin, mn)) mn = kmin;
      if (key_less(mx, kmax)) mx = kmax;
    }
    const uint32_t w_new = key_span_bits(mn, mx);
    uint32_t w_prev = uint32_t(__shfl_up(int(w_new), 1, 64));
    if (lane == 0) w_prev = w_old;
    const uint64_t len = j - i;
    const int64_t cost = int64_t((len + 1) * w_new) - int64_t(len * w_prev);
    const bool start_here = forced && valid && ((forced[j >> 6] >> (j & 63)) & 1ull);
    const bool in_start = forced && valid && ((inside[j >> 6] >> (j & 63)) & 1ull);
    const bool include = len < max_len && !start_here && (in_start || double(cost) <= thr);
    const uint64_t split = __ballot(valid && !include);
    if (split == 0) {
      const int last = int(b - p - 1 < 63 ? b - p - 1 : 63);
      if (kFix && lane == 0) clear_bits(bitmap, p, p + uint64_t(last) + 1);
      kmin = key_readlane(mn, last);
      kmax = key_readlane(mx, last);
      w_old = uint32_t(__shfl(int(w_new), last, 64));
      have = true;
      p += uint64_t(last) + 1;
    } else {
      const uint64_t js = p + uint64_t(__ffsll(static_cast<long long>(split)) - 1);
      if (kFix) {
        bool hit = false;
        if (lane == 0) {
          clear_bits(bitmap, p, js);
          hit = bit_set(bitmap, js);
          if (!hit) mark(bitmap, js);
        }
        synced = __ballot(hit) != 0;
      } else if (lane == 0) {
        mark(bitmap, js);
      }
      i = js;
      have = false;
      w_old = 0;
      p = js + 1;
      if (synced) break;
    }
  }
  st.i = i;
  st.have = have ? 1u : 0u;
  st.kmin_hi = key_hi(kmin);
  st.kmin_lo = key_lo(kmin);
  st.kmax_hi = key_hi(kmax);
  st.kmax_lo = key_lo(kmax);
  st.w_old = w_old;
  return synced;
}

// Speculative split: one 64-lane workgroup per 2^kSubLog2-value sub-chunk.
// Sub-chunk 0 of the column begins where a partition really begins; the
// others begin a partition at their own start, which the fix-up passes
// correct.  Each records its final state.
__global__ __launch_bounds__(64) void k_split_spec(const uint8_t* __restrict__ col,
                                                   uint32_t dtype, uint64_t n, double thr,
                                                   uint64_t max_len,
                                                   unsigned long long* __restrict__ bitmap,
                                                   SplitState* __restrict__ states,
                                                   const uint64_t* __restrict__ forced,
                                                   const uint64_t* __restrict__ inside) {
  __shared__ uint64_t win[kSplitWindow + 1];  // win[k] = v[base - 1 + k]
  const uint64_t a = uint64_t(blockIdx.x) << kSubLog2;
  if (a >= n) return;
  const uint64_t b = n - a < (uint64_t(1) << kSubLog2) ? n : a + (uint64_t(1) << kSubLog2);
  if (threadIdx.x == 0) mark(bitmap, a);
  SplitState st{a, 0, 0, 0, 0, 0, 0};
  if (dtype == 4)
    greedy_walk<false, uint64_t>(col, dtype, a + 1, b, thr, max_len, st, win, bitmap, forced,
                                 inside);
  else
    greedy_walk<false, DKey>(col, dtype, a + 1, b, thr, max_len, st, win, bitmap, forced, inside);
  if (threadIdx.x == 0) states[blockIdx.x] = st;
}

// Walks sub-chunks [q, q_end) of the column in order from state st (fix
// mode), each from the state the previous one ends in; returns at the
// first sub-chunk where the walk meets the starts already there (st is
// then that meeting's state, and the caller continues from the run already
// recorded), or after the last one with st its end state.
__device__ bool walk_subchunks(const uint8_t* col, uint32_t dtype, uint64_t n, double thr,
                               uint64_t max_len, uint64_t q, uint64_t q_end, SplitState& st,
                               uint64_t* win, unsigned long long* bitmap, const uint64_t* forced,
                               const uint64_t* inside) {
  for (; q < q_end; ++q) {
    const uint64_t aq = q << kSubLog2;
    if (aq >= n) break;
    const uint64_t bq = n - aq < (uint64_t(1) << kSubLog2) ? n : aq + (uint64_t(1) << kSubLog2);
    const bool synced =
        dtype == 4
            ? greedy_walk<true, uint64_t>(col, dtype, aq, bq, thr, max_len, st, win, bitmap, forced,
                                          inside)
            : greedy_walk<true, DKey>(col, dtype, aq, bq, thr, max_len, st, win, bitmap, forced,
                                      inside);
    if (synced) return true;
  }
  return false;
}

// Fix-up within segments: one workgroup per 2^20-value segment walks its
// sub-chunks 1.. in order, each from the state the previous one ends in,
// until its starts meet the speculative ones; the segment's end state (as
// if a partition began at the segment start) goes to seg_states.
__global__ __launch_bounds__(64) void k_split_fix(const uint8_t* __restrict__ col,
                                                  uint32_t dtype, uint64_t n, double thr,
                                                  uint64_t max_len,
                                                  unsigned long long* __restrict__ bitmap,
                                                  const SplitState* __restrict__ states,
                                                  SplitState* __restrict__ seg_states,
                                                  const uint64_t* __restrict__ forced,
                                                  const uint64_t* __restrict__ inside) {
  __shared__ uint64_t win[kSplitWindow + 1];
  constexpr uint64_t kSubs = uint64_t(1) << (kSegLog2 - kSubLog2);
  const uint64_t a = uint64_t(blockIdx.x) << kSegLog2;
  if (a >= n) return;
  const uint64_t q0 = uint64_t(blockIdx.x) * kSubs;
  const uint64_t nsub = (n + (uint64_t(1) << kSubLog2) - 1) >> kSubLog2;
  const uint64_t q_end = q0 + kSubs < nsub ? q0 + kSubs : nsub;
  SplitState st = states[q0];
  for (uint64_t q = q0 + 1; q < q_end; ++q) {
    // a meeting makes the rest of sub-chunk q the speculative run's
    if (walk_subchunks(col, dtype, n, thr, max_len, q, q + 1, st, win, bitmap, forced, inside))
      st = states[q];
  }
  if (threadIdx.x == 0) seg_states[blockIdx.x] = st;
}

// Fix-up across segments: one wavefront walks each segment from the true
// state the previous segment ends in, until it meets the starts already
// there (from then on the segment's run, and its end state, are right).
__global__ __launch_bounds__(64) void k_split_join(const uint8_t* __restrict__ col,
                                                   uint32_t dtype, uint64_t n, double thr,
                                                   uint64_t max_len,
                                                   unsigned long long* __restrict__ bitmap,
                                                   const SplitState* __restrict__ seg_states,
                                                   uint64_t nseg, const uint64_t* __restrict__ forced,
                                                   const uint64_t* __restrict__ inside) {
  __shared__ uint64_t win[kSplitWindow + 1];
  constexpr uint64_t kSubs = uint64_t(1) << (kSegLog2 - kSubLog2);
  const uint64_t nsub = (n + (uint64_t(1) << kSubLog2) - 1) >> kSubLog2;
  SplitState st = seg_states[0];
  for (uint64_t g = 1; g < nseg; ++g) {
    const uint64_t q0 = g * kSubs, q_end = q0 + kSubs < nsub ? q0 + kSubs : nsub;
    if (walk_subchunks(col, dtype, n, thr, max_len, q0, q_end, st, win, bitmap, forced, inside))
      st = seg_states[g];
  }
}

// ---- starting partitions ---------------------------------------------------------
//
// Second-order deltas dd_k = v_k - 2 v_{k-1} + v_{k-2} (k >= 2, exact in
// 128 bits, |dd| < 2^66).  Positions whose |dd| is the column's smallest
// are good; a maximal run k..k' of them is the starting partition
// v[k-2, k'+1), and of two that would share a value the later keeps it
// (section 3.2.2, selecting good starting positions, for a degree-1 model).

typedef unsigned __int128 u128_t;

__device__ inline u128_t dd_magnitude(const uint8_t* col, uint32_t dtype, uint64_t k) {
  const __int128 a = __int128(load_value(col, dtype, k));
  const __int128 b = __int128(load_value(col, dtype, k - 1));
  const __int128 c = __int128(load_value(col, dtype, k - 2));
  const __int128 dd = a - 2 * b + c;
  return dd < 0 ? u128_t(-dd) : u128_t(dd);
}

__device__ inline u128_t wave_min_u128(u128_t x) {
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t lo = uint64_t(__shfl_xor(static_cast<unsigned long long>(uint64_t(x)), off, 64));
    const uint64_t hi =
        uint64_t(__shfl_xor(static_cast<unsigned long long>(uint64_t(x >> 64)), off, 64));
    const u128_t y = (u128_t(hi) << 64) | lo;
    x = y < x ? y : x;
  }
  return x;
}

// partial[block] = the smallest |dd_k| over the block's grid-stride share of
// k = 2 .. n-1 (all ones when it has none), as (low, high) words.
__global__ __launch_bounds__(kScanBlock) void k_dd_min(const uint8_t* __restrict__ col,
                                                      uint32_t dtype, uint64_t n,
                                                      uint64_t* __restrict__ partial) {
  __shared__ uint64_t red[kScanBlock / 64][2];
  u128_t best = ~u128_t(0);
  for (uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x + 2; k < n;
       k += uint64_t(gridDim.x) * blockDim.x) {
    const u128_t x = dd_magnitude(col, dtype, k);
    best = x < best ? x : best;
  }
  best = wave_min_u128(best);
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[wave][0] = uint64_t(best);
    red[wave][1] = uint64_t(best >> 64);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (uint32_t w = 1; w < kScanBlock / 64; ++w) {
      const u128_t y = (u128_t(red[w][1]) << 64) | red[w][0];
      best = y < best ? y : best;
    }
    partial[2 * blockIdx.x] = uint64_t(best);
    partial[2 * blockIdx.x + 1] = uint64_t(best >> 64);
  }
}

// out[0..1] = the smallest of `count` partial minima (one wavefront).
__global__ __launch_bounds__(64) void k_dd_min_final(const uint64_t* __restrict__ partial,
                                                    uint64_t count, uint64_t* __restrict__ out) {
  u128_t best = ~u128_t(0);
  for (uint64_t i = threadIdx.x; i < count; i += 64) {
    const u128_t y = (u128_t(partial[2 * i + 1]) << 64) | partial[2 * i];
    best = y < best ? y : best;
  }
  best = wave_min_u128(best);
  if (threadIdx.x == 0) {
    out[0] = uint64_t(best);
    out[1] = uint64_t(best >> 64);
  }
}

// good(k): k >= 2 and |dd_k| is the smallest.
__device__ inline bool dd_good(const uint8_t* col, uint32_t dtype, uint64_t n, uint64_t k,
                               u128_t best) {
  return k >= 2 && k < n && dd_magnitude(col, dtype, k) == best;
}

// first[w] bit l: value p = 64 w + l begins a starting partition (p + 2 is
// good, p + 1 is not); inside[w] bit l: p is a later value of one (p or
// p + 1 is good, and p does not begin one).  One lane per value; the
// wavefront's ballots are the words.
__global__ __launch_bounds__(kScanBlock) void k_mark_starting(const uint8_t* __restrict__ col,
                                                             uint32_t dtype, uint64_t n,
                                                             const uint64_t* __restrict__ best_dd,
                                                             uint64_t* __restrict__ first,
                                                             uint64_t* __restrict__ inside) {
  const u128_t best = (u128_t(best_dd[1]) << 64) | best_dd[0];
  const uint64_t nwords = (n + 63) / 64;
  for (uint64_t p0 = (uint64_t(blockIdx.x) * blockDim.x + (threadIdx.x & ~63u));
       p0 < nwords * 64; p0 += uint64_t(gridDim.x) * blockDim.x) {
    const uint64_t p = p0 + (threadIdx.x & 63);
    bool begins = false, in = false;
    if (p < n) {
      const bool g0 = dd_good(col, dtype, n, p, best);
      const bool g1 = dd_good(col, dtype, n, p + 1, best);
      const bool g2 = dd_good(col, dtype, n, p + 2, best);
      begins = g2 && !g1;
      in = !begins && (g0 || g1);
    }
    const uint64_t wb = __ballot(begins), wi = __ballot(in);
    if ((threadIdx.x & 63) == 0) {
      first[p0 >> 6] = wb;
      inside[p0 >> 6] = wi;
    }
  }
}

// ---- block-wide scan of counts -------------------------------------------------

// Exclusive prefix sum of x over the workgroup's threads; *total receives
// the workgroup sum.
__device__ inline uint32_t block_exclusive_scan(uint32_t x, uint32_t* total) {
  __shared__ uint32_t wsum[kScanBlock / 64];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t inc = x;
#pragma unroll
  for (int delta = 1; delta < 64; delta <<= 1) {
    const uint32_t y = uint32_t(__shfl_up(int(inc), delta, 64));
    if (int(lane) >= delta) inc += y;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint32_t before = 0, all = 0;
#pragma unroll
  for (uint32_t w = 0; w < kScanBlock / 64; ++w) {
    if (w < wave) before += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return before + inc - x;
}

// Set bits of bitmap words [blockIdx * 1024, +1024).
__global__ __launch_bounds__(kScanBlock) void k_bitmap_count(const uint64_t* __restrict__ bitmap,
                                                             uint64_t nwords,
                                                             uint64_t* __restrict__ counts) {
  const uint64_t w0 = uint64_t(blockIdx.x) * kItemsPerBlock + threadIdx.x * 4;
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (w0 + k < nwords) c += uint32_t(__popcll(bitmap[w0 + k]));
  uint32_t total;
  block_exclusive_scan(c, &total);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// Writes the positions of the set bits, in order, from starts[offsets[block]].
__global__ __launch_bounds__(kScanBlock) void k_bitmap_emit(const uint64_t* __restrict__ bitmap,
                                                            uint64_t nwords,
                                                            const uint64_t* __restrict__ offsets,
                                                            uint64_t* __restrict__ starts) {
  const uint64_t w0 = uint64_t(blockIdx.x) * kItemsPerBlock + threadIdx.x * 4;
  uint64_t words[4];
  uint32_t c = 0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    words[k] = w0 + k < nwords ? bitmap[w0 + k] : 0;
    c += uint32_t(__popcll(words[k]));
  }
  uint32_t total;
  uint64_t out = offsets[blockIdx.x] + block_exclusive_scan(c, &total);
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    uint64_t w = words[k];
    while (w) {
      const int bit = __ffsll(static_cast<long long>(w)) - 1;
      starts[out++] = (w0 + k) * 64 + uint64_t(bit);
      w &= w - 1;
    }
  }
}

// ---- sizes -----------------------------------------------------------------------

struct FitShared {
  uint64_t red[kEncWaves][4];
  double theta1;
};

// Bytes that the partition v[s, e) costs in a variable-length blob: its
// 32-byte record, its 8-byte start and its residual words, with the model
// the encoder would choose.  Called by every thread of the workgroup.
__device__ uint64_t range_cost(FitShared& sh, const uint8_t* col, uint32_t dtype, uint64_t s,
                               uint64_t e) {
  const uint64_t len = e - s;
  const uint8_t* src = col + s * dtype;
  uint64_t vmin = ~uint64_t(0), vmax = 0;
  U128 sv{0, 0}, stv{0, 0};
  for (uint64_t t = threadIdx.x; t < len; t += kEncBlock) {
    const uint64_t x = load_value(src, dtype, t);
    vmin = x < vmin ? x : vmin;
    vmax = x > vmax ? x : vmax;
    sv = add128(sv, U128{x, 0});
    stv = add128(stv, mul64x64(t, x));
  }
  block_minmax_u64(sh, vmin, vmax);
  const uint64_t range = vmax - vmin;
  Model md{vmin, vmin, 0.0, bitlen64(range), false, 0, range};
  if (len > 1 && range < (uint64_t(1) << 61)) {
    block_sum_u128x2(sh, sv, stv);
    const double th = block_slope(sh, len, sv, stv);
    int64_t rmin = INT64_MAX, rmax = INT64_MIN;
    for (uint64_t t = threadIdx.x; t < len; t += kEncBlock) {
      const int64_t rr = int64_t(load_value(src, dtype, t) - vmin) - predict(th, uint32_t(t));
      rmin = rr < rmin ? rr : rmin;
      rmax = rr > rmax ? rr : rmax;
    }
    block_minmax_i64(sh, rmin, rmax);
    choose_model(md, th, rmin, rmax);
  }
  return kRecordBytes + 8 + 8 * ((len * md.bits + 63) >> 6);
}

// Ranges up to kLaneRangeMax values are sized by one lane, up to
// kWaveRangeMax by one wavefront, longer ones by a whole workgroup.
constexpr uint64_t kLaneRangeMax = 32;
constexpr uint64_t kWaveRangeMax = 8192;

// range_cost computed by one lane alone.
__device__ uint64_t range_cost_lane(const uint8_t* col, uint32_t dtype, uint64_t s, uint64_t e) {
  const uint64_t len = e - s;
  const uint8_t* src = col + s * dtype;
  uint64_t vmin = ~uint64_t(0), vmax = 0;
  U128 sv{0, 0}, stv{0, 0};
  for (uint64_t t = 0; t < len; ++t) {
    const uint64_t x = load_value(src, dtype, t);
    vmin = x < vmin ? x : vmin;
    vmax = x > vmax ? x : vmax;
    sv = add128(sv, U128{x, 0});
    stv = add128(stv, mul64x64(t, x));
  }
  const uint64_t range = vmax - vmin;
  Model md{vmin, vmin, 0.0, bitlen64(range), false, 0, range};
  if (len > 1 && range < (uint64_t(1) << 61)) {
    const double th = ls_slope(len, sv, stv);
    int64_t rmin = INT64_MAX, rmax = INT64_MIN;
    for (uint64_t t = 0; t < len; ++t) {
      const int64_t rr = int64_t(load_value(src, dtype, t) - vmin) - predict(th, uint32_t(t));
      rmin = rr < rmin ? rr : rmin;
      rmax = rr > rmax ? rr : rmax;
    }
    choose_model(md, th, rmin, rmax);
  }
  return kRecordBytes + 8 + 8 * ((len * md.bits + 63) >> 6);
}

// The ranges of at most kLaneRangeMax values (and the ones too long to
// merge): one lane each.
__global__ __launch_bounds__(kEncBlock) void k_costs_short(const uint8_t* __restrict__ col,
                                                           uint32_t dtype,
                                                           const uint64_t* __restrict__ starts,
                                                           uint64_t count, uint32_t span,
                                                           uint64_t max_len,
                                                           const uint8_t* __restrict__ dirty,
                                                           uint64_t* __restrict__ out) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t j = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; j < count; j += stride) {
    if (dirty && !dirty[j]) continue;
    const uint64_t s = starts[j], e = starts[j + span];
    if (e - s > max_len) out[j] = kNoMerge;
    else if (e - s <= kLaneRangeMax) out[j] = range_cost_lane(col, dtype, s, e);
  }
}

// range_cost computed by one wavefront alone (no workgroup barrier), the
// same arithmetic in the same order of operations where it matters: the
// sums are exact and the slope is one function of them.
//
// Ranges of at most 64 kCostRegs values are held in registers: every load
// is issued before any is used and the residual pass reads the registers
// (a loop of dependent loads per pass made the wavefront wait once per 64
// values, twice).  The sums are exact, so their order does not matter.
constexpr int kCostRegs = 8;

template <class T>
__device__ uint64_t range_cost_wave_regs(const T* src, uint64_t len) {
  const uint32_t lane = threadIdx.x & 63;
  const auto g = global_ptr(src);
  uint64_t x[kCostRegs];
#pragma unroll
  for (int k = 0; k < kCostRegs; ++k) {
    const uint32_t t = lane + 64u * k;
    x[k] = uint64_t(g[t < len ? t : len - 1]);
  }
  uint64_t vmin = ~uint64_t(0), vmax = 0;
  U128 sv{0, 0}, stv{0, 0};
#pragma unroll
  for (int k = 0; k < kCostRegs; ++k) {
    const uint32_t t = lane + 64u * k;
    if (t < len) {
      vmin = x[k] < vmin ? x[k] : vmin;
      vmax = x[k] > vmax ? x[k] : vmax;
      sv = add128(sv, U128{x[k], 0});
      stv = add128(stv, mul64x64(t, x[k]));
    }
  }
  wave_minmax_u64(vmin, vmax);
  const uint64_t range = vmax - vmin;
  Model md{vmin, vmin, 0.0, bitlen64(range), false, 0, range};
  if (len > 1 && range < (uint64_t(1) << 61)) {
    wave_sum_u128x2(sv, stv);
    const double th = ls_slope(len, sv, stv);
    int64_t rmin = INT64_MAX, rmax = INT64_MIN;
#pragma unroll
    for (int k = 0; k < kCostRegs; ++k) {
      const uint32_t t = lane + 64u * k;
      if (t < len) {
        const int64_t rr = int64_t(x[k] - vmin) - predict(th, t);
        rmin = rr < rmin ? rr : rmin;
        rmax = rr > rmax ? rr : rmax;
      }
    }
    wave_minmax_i64(rmin, rmax);
    choose_model(md, th, rmin, rmax);
  }
  return kRecordBytes + 8 + 8 * ((len * md.bits + 63) >> 6);
}

__device__ uint64_t range_cost_wave(const uint8_t* col, uint32_t dtype, uint64_t s, uint64_t e) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t len = e - s;
  const uint8_t* src = col + s * dtype;
  if (len <= 64u * kCostRegs)
    return dtype == 8 ? range_cost_wave_regs(reinterpret_cast<const uint64_t*>(src), len)
                      : range_cost_wave_regs(reinterpret_cast<const uint32_t*>(src), len);
  // longer ranges in blocks of 64 kCostRegs values, each block's loads
  // issued together (indices clamped, the extra lanes masked)
  uint64_t vmin = ~uint64_t(0), vmax = 0;
  U128 sv{0, 0}, stv{0, 0};
  for (uint64_t t0 = 0; t0 < len; t0 += 64u * kCostRegs) {
    uint64_t x[kCostRegs];
#pragma unroll
    for (int k = 0; k < kCostRegs; ++k) {
      const uint64_t t = t0 + lane + 64u * k;
      x[k] = load_value(src, dtype, t < len ? t : len - 1);
    }
#pragma unroll
    for (int k = 0; k < kCostRegs; ++k) {
      const uint64_t t = t0 + lane + 64u * k;
      if (t < len) {
        vmin = x[k] < vmin ? x[k] : vmin;
        vmax = x[k] > vmax ? x[k] : vmax;
        sv = add128(sv, U128{x[k], 0});
        stv = add128(stv, mul64x64(t, x[k]));
      }
    }
  }
  wave_minmax_u64(vmin, vmax);
  const uint64_t range = vmax - vmin;
  Model md{vmin, vmin, 0.0, bitlen64(range), false, 0, range};
  if (len > 1 && range < (uint64_t(1) << 61)) {
    wave_sum_u128x2(sv, stv);
    const double th = ls_slope(len, sv, stv);
    int64_t rmin = INT64_MAX, rmax = INT64_MIN;
    for (uint64_t t0 = 0; t0 < len; t0 += 64u * kCostRegs) {
      uint64_t x[kCostRegs];
#pragma unroll
      for (int k = 0; k < kCostRegs; ++k) {
        const uint64_t t = t0 + lane + 64u * k;
        x[k] = load_value(src, dtype, t < len ? t : len - 1);
      }
#pragma unroll
      for (int k = 0; k < kCostRegs; ++k) {
        const uint64_t t = t0 + lane + 64u * k;
        if (t < len) {
          const int64_t rr = int64_t(x[k] - vmin) - predict(th, uint32_t(t));
          rmin = rr < rmin ? rr : rmin;
          rmax = rr > rmax ? rr : rmax;
        }
      }
    }
    wave_minmax_i64(rmin, rmax);
    choose_model(md, th, rmin, rmax);
  }
  return kRecordBytes + 8 + 8 * ((len * md.bits + 63) >> 6);
}

// Ranges are screened `chunk` (at most kCostChunk) at a time: the chunk's
// lanes read their dirty flag and bounds together (one round trip), and the
// wavefront or workgroup then sizes the chunk's ranges of its class one
// after another.  (Walking one range per iteration made every idle launch
// cost a chain of dependent loads per range.)  The host picks the chunk so
// that there are at least as many chunks as resident wavefronts or
// workgroups: few, long ranges still get one each.
constexpr uint32_t kCostChunk = 64;

// Bounds of range j0 + lane for lanes below kCostChunk; true if it needs
// sizing by the caller's class [lo_len, hi_len] (and is within max_len).
__device__ inline bool cost_candidate(const uint64_t* starts, uint64_t count, uint32_t span,
                                      uint64_t max_len, const uint8_t* dirty, uint64_t j,
                                      uint64_t lo_len, uint64_t hi_len) {
  if (j >= count) return false;
  // the flag and both bounds in one round trip
  const bool d = !dirty || dirty[j];
  const uint64_t len = starts[j + span] - starts[j];
  return d && len <= max_len && len > lo_len && len <= hi_len;
}

// out[j] = cost of v[starts[j], starts[j + span]) for j < count (only
// where dirty[j], if dirty is given), or kNoMerge when that is longer than
// max_len: one wavefront per range of more than kLaneRangeMax and at most
// kWaveRangeMax values; the others are left to k_costs_short and
// k_costs_long.
__global__ __launch_bounds__(kEncBlock) void k_costs(const uint8_t* __restrict__ col,
                                                     uint32_t dtype,
                                                     const uint64_t* __restrict__ starts,
                                                     uint64_t count, uint32_t span,
                                                     uint64_t max_len,
                                                     const uint8_t* __restrict__ dirty,
                                                     uint64_t* __restrict__ out, uint32_t chunk) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t waves = uint64_t(gridDim.x) * kEncWaves;
  for (uint64_t j0 = (uint64_t(blockIdx.x) * kEncWaves + (threadIdx.x >> 6)) * chunk;
       j0 < count; j0 += waves * chunk) {
    const bool mine = lane < chunk &&
                      cost_candidate(starts, count, span, max_len, dirty, j0 + lane,
                                     kLaneRangeMax, kWaveRangeMax);
    uint64_t todo = __ballot(mine);
    while (todo) {
      const uint64_t j = j0 + uint64_t(__ffsll(static_cast<long long>(todo)) - 1);
      todo &= todo - 1;
      const uint64_t c = range_cost_wave(col, dtype, starts[j], starts[j + span]);
      if (lane == 0) out[j] = c;
    }
  }
}

// The ranges k_costs left: one workgroup each.
__global__ __launch_bounds__(kEncBlock) void k_costs_long(const uint8_t* __restrict__ col,
                                                          uint32_t dtype,
                                                          const uint64_t* __restrict__ starts,
                                                          uint64_t count, uint32_t span,
                                                          uint64_t max_len,
                                                          const uint8_t* __restrict__ dirty,
                                                          uint64_t* __restrict__ out,
                                                          uint32_t chunk) {
  __shared__ FitShared sh;
  __shared__ uint64_t todo_sh;
  for (uint64_t j0 = uint64_t(blockIdx.x) * chunk; j0 < count;
       j0 += uint64_t(gridDim.x) * chunk) {
    if (threadIdx.x < 64) {
      const bool mine =
          threadIdx.x < chunk && cost_candidate(starts, count, span, max_len, dirty,
                                                     j0 + threadIdx.x, kWaveRangeMax, max_len);
      const uint64_t b = __ballot(mine);
      if (threadIdx.x == 0) todo_sh = b;
    }
    __syncthreads();
    uint64_t todo = todo_sh;
    while (todo) {
      const uint64_t j = j0 + uint64_t(__ffsll(static_cast<long long>(todo)) - 1);
      todo &= todo - 1;
      const uint64_t c = range_cost(sh, col, dtype, starts[j], starts[j + span]);
      if (threadIdx.x == 0) out[j] = c;
    }
    __syncthreads();  // todo_sh is rewritten by the next chunk
  }
}

// ---- merge scan -------------------------------------------------------------------
//
// Boundary k (1 <= k < m) is the start of partition k.  Step k of a pass
// tries to merge the current partition, which begins at boundary a (a < k)
// and costs cc bytes, with partition k:
//   union = pair[k - 1] when a = k - 1 (two unmerged partitions, sized in
//           advance), else the size of v[s[a], s[k+1]) fitted now; none
//           when longer than max_len;
//   merge when union < cc + cost[k]: the current partition grows (cc =
//   union); else boundary k is kept, and partition k is the current one
//   (a = k, cc = cost[k]).
// The pass keeps a bitmap of kept boundaries (bit 0 always set); the
// partitions that absorbed others are sized once the pass is done.

constexpr uint32_t kMergeChunkLog2 = 8;  // boundaries per speculative chunk
constexpr uint64_t kMergeChunk = uint64_t(1) << kMergeChunkLog2;

__device__ inline uint64_t shfl_up64(uint64_t x, int d) {
  return uint64_t(__shfl_up(static_cast<unsigned long long>(x), d, 64));
}

// Lane k's value of x, k uniform across the wavefront.
__device__ inline uint64_t readlane64(uint64_t x, uint32_t k) {
  const uint32_t lo = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x)), int(k)));
  const uint32_t hi = uint32_t(__builtin_amdgcn_readlane(int(uint32_t(x >> 32)), int(k)));
  return (uint64_t(hi) << 32) | lo;
}

// Value summary of a range of the column: smallest and largest value, and
// the sums of v and of t * v (t counted from the range's first position)
// modulo 2^128: the least-squares slope needs no more (N is the same for
// shifted values, and exact because |N| < 2^121).
struct RangeSum {
  uint64_t vmin, vmax;
  U128 sy, sty;
};

// The summary of [x, z) from those of [x, y) and [y, z).
__device__ inline RangeSum join(const RangeSum& a, const RangeSum& b, uint64_t a_len) {
  RangeSum r;
  r.vmin = a.vmin < b.vmin ? a.vmin : b.vmin;
  r.vmax = a.vmax > b.vmax ? a.vmax : b.vmax;
  r.sy = add128(a.sy, b.sy);
  r.sty = add128(add128(a.sty, b.sty), mul128x64(b.sy, a_len));
  return r;
}

struct MergeState {
  uint64_t a;   // boundary where the current partition begins
  uint64_t cc;  // its size in bytes
  RangeSum sum; // its values' summary
};

// Convex hulls of the current partition's points (t, v_t), t counted from
// its first value: the upper hull (left to right, right turns only) and the
// lower one.  Over any set of points, v_t - theta1 * t is largest at an
// upper-hull vertex and smallest at a lower-hull vertex, whatever theta1;
// so is the exact residual v_t - floor(theta1 * t), the ceiling of that real
// number.  The encoder's residual takes the binary64 product, whose floor
// exceeds the exact one by 1 exactly when the product rounds up onto an
// integer (merge_walk checks for that).  A long run of merges then sizes
// each union from the hulls and the values it adds, not from all its values.
constexpr uint32_t kHullMax = 64;              // vertices per hull
constexpr uint64_t kHullBuildMin = 256;        // shorter partitions are scanned whole
constexpr uint64_t kHullBuildMax = 16384;      // values a hull is first built from
constexpr uint64_t kHullAppendMax = 8192;      // values one step may append
constexpr uint64_t kHullNewMax = 4096;         // new values a batch sizes by scanning
enum : uint32_t { kHullNone = 0, kHullValid = 1, kHullDead = 2 };

struct ChainHull {  // hull 0: upper, hull 1: lower
  uint32_t nu, nl, state, pad;
  uint32_t t[2][kHullMax];
  uint64_t x[2][kHullMax];
};

// A wavefront's LDS: the hulls and a window of values with a 16-value halo
// on either side.
constexpr uint32_t kHalo = 16;
struct HullLds {
  ChainHull h;
  uint64_t stage[64 + 2 * kHalo];
};

// The hulls' counts and state, identical in every lane of the wavefront.
struct HullRegs {
  uint32_t nu, nl, state;
};

__device__ inline void wave_lds_order() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Sign of (b - a) x (c - a) for points with ta < tb < tc whose values lie
// within 2^61 of each other.  kW = 64: within 2^43, so that with t < 2^20
// each product fits in 64 bits; kW = 32: within 2^31, so that each factor
// fits in 32 bits as well (one 32 x 32 -> 64 multiply).
template <int kW = 128>
__device__ inline int turn(uint32_t ta, uint64_t xa, uint32_t tb, uint64_t xb, uint32_t tc,
                           uint64_t xc) {
  if (kW == 32) {
    const int64_t l = int64_t(int32_t(tb - ta)) * int64_t(int32_t(uint32_t(xc - xa)));
    const int64_t r = int64_t(int32_t(uint32_t(xb - xa))) * int64_t(int32_t(tc - ta));
    return l > r ? 1 : (l < r ? -1 : 0);
  }
  if (kW == 64) {
    const int64_t l = int64_t(tb - ta) * int64_t(xc - xa);
    const int64_t r = int64_t(xb - xa) * int64_t(tc - ta);
    return l > r ? 1 : (l < r ? -1 : 0);
  }
  const __int128 l = __int128(int64_t(tb - ta)) * __int128(int64_t(xc - xa));
  const __int128 r = __int128(int64_t(xb - xa)) * __int128(int64_t(tc - ta));
  return l > r ? 1 : (l < r ? -1 : 0);
}

// Appends the points [u0, u1) of the partition beginning at column position
// sa to both hulls; too many vertices mark them dead.  Each lane first tests
// its point against chords through points of [0, u1) at distances 1..16 on
// either side: a point on or below such a chord is no upper-hull vertex of
// any set holding both ends, one on or above it no lower-hull vertex.  The
// survivors then go through the monotone chain in order, lane 0 keeping the
// upper hull and lane 1 the lower one side by side, each with its two last
// vertices in registers.  Called by a whole wavefront, uniform arguments.
template <int kW>
__device__ inline void hull_append_t(const uint8_t* __restrict__ col, uint32_t dtype, uint64_t sa,
                                     uint64_t u0, uint64_t u1, HullLds& w, HullRegs& hr) {
  const uint32_t lane = threadIdx.x & 63;
  const uint8_t* src = col + sa * dtype;
  ChainHull& h = w.h;
  const uint32_t side = lane & 1;  // lanes 0 and 1: the hull they keep
  uint32_t n = side ? hr.nl : hr.nu;
  uint32_t t1 = 0, t2 = 0;  // last and second-last vertex
  uint64_t x1 = 0, x2 = 0;
  if (lane < 2) {
    if (n >= 1) { t1 = h.t[side][n - 1]; x1 = h.x[side][n - 1]; }
    if (n >= 2) { t2 = h.t[side][n - 2]; x2 = h.x[side][n - 2]; }
  }
  bool over = false;
  for (uint64_t b = u0; b < u1; b += 64) {
    // positions b - kHalo .. b + 63 + kHalo that lie in [0, u1), staged once
    for (uint32_t i = lane; i < 64 + 2 * kHalo; i += 64) {
      if (b + i >= kHalo && b + i - kHalo < u1) w.stage[i] = load_value(src, dtype, b + i - kHalo);
    }
    wave_lds_order();
    const uint64_t t = b + lane;
    const bool in = t < u1;
    const uint64_t x = w.stage[kHalo + lane];  // used only where in
    bool cu = in, cl = in;
#pragma unroll
    for (uint32_t ia = 0; ia < 5; ++ia) {
      const uint32_t a = 1u << ia;
      if (!in || t < a) break;
      const uint64_t xa = w.stage[kHalo + lane - a];
#pragma unroll
      for (uint32_t ic = 0; ic < 5; ++ic) {
        const uint32_t c = 1u << ic;
        if (t + c >= u1) break;
        const int tr = turn<kW>(0, xa, a, x, a + c, w.stage[kHalo + lane + c]);
        if (tr >= 0) cu = false;
        if (tr <= 0) cl = false;
      }
    }
    wave_lds_order();  // every read of the window precedes the next block's
    const uint64_t mu = __ballot(cu), ml = __ballot(cl);
    uint64_t todo = mu | ml;
    while (todo) {
      const uint32_t q = uint32_t(__ffsll(static_cast<long long>(todo)) - 1);
      todo &= todo - 1;
      const uint64_t xq = readlane64(x, q);
      const uint32_t tq = uint32_t(b + q);
      const bool mine = lane < 2 && (((side ? ml : mu) >> q) & 1);
      if (mine && !over) {
        while (n >= 2) {
          const int tr = turn<kW>(t2, x2, t1, x1, tq, xq);
          if (side ? tr > 0 : tr < 0) break;  // a strict turn keeps the last vertex
          --n;
          t1 = t2;
          x1 = x2;
          if (n >= 2) {
            t2 = h.t[side][n - 2];
            x2 = h.x[side][n - 2];
          }
        }
        if (n == kHullMax) {
          over = true;
        } else {
          h.t[side][n] = tq;
          h.x[side][n] = xq;
          ++n;
          t2 = t1;
          x2 = x1;
          t1 = tq;
          x1 = xq;
        }
      }
    }
    if (__ballot(over)) break;
  }
  const uint32_t nu = uint32_t(__builtin_amdgcn_readlane(int(n), 0));
  const uint32_t nl = uint32_t(__builtin_amdgcn_readlane(int(n), 1));
  hr = __ballot(over) ? HullRegs{0, 0, kHullDead} : HullRegs{nu, nl, kHullValid};
  wave_lds_order();  // the vertices are read by every lane next
}

// Values spread below 2^31 take the 32-bit turn test, below 2^43 the 64-bit one.
__device__ inline void hull_append(const uint8_t* __restrict__ col, uint32_t dtype, uint64_t sa,
                                   uint64_t u0, uint64_t u1, uint64_t spread, HullLds& w,
                                   HullRegs& hr) {
  if (spread < (uint64_t(1) << 31))
    hull_append_t<32>(col, dtype, sa, u0, u1, w, hr);
  else if (spread < (uint64_t(1) << 43))
    hull_append_t<64>(col, dtype, sa, u0, u1, w, hr);
  else
    hull_append_t<128>(col, dtype, sa, u0, u1, w, hr);
}

__device__ inline void hull_store(ChainHull* __restrict__ g, const ChainHull& h, const HullRegs& hr) {
  const uint32_t lane = threadIdx.x & 63;
  if (hr.state == kHullValid) {
    if (lane < hr.nu) {
      g->t[0][lane] = h.t[0][lane];
      g->x[0][lane] = h.x[0][lane];
    }
    if (lane < hr.nl) {
      g->t[1][lane] = h.t[1][lane];
      g->x[1][lane] = h.x[1][lane];
    }
  }
  if (lane == 0) {
    g->nu = hr.nu;
    g->nl = hr.nl;
    g->state = hr.state;
  }
}

__device__ inline HullRegs hull_load(const ChainHull* __restrict__ g, ChainHull& h) {
  const uint32_t lane = threadIdx.x & 63;
  HullRegs hr{g->nu, g->nl, g->state};
  if (hr.state == kHullValid) {
    if (lane < hr.nu) {
      h.t[0][lane] = g->t[0][lane];
      h.x[0][lane] = g->x[0][lane];
    }
    if (lane < hr.nl) {
      h.t[1][lane] = g->t[1][lane];
      h.x[1][lane] = g->x[1][lane];
    }
  }
  wave_lds_order();
  return hr;
}

// The encoder's residual v - vmin - floor(fl(theta1 * t)) at a hull vertex,
// plus 1 when the binary64 product rounded up onto an integer (then the
// exact residual is one more; `up` says so).  `gap` is 1 - frac(theta1 * t)
// of the exact product, to within 2^-50, when up is false.
__device__ inline int64_t vertex_residual(double th, uint32_t t, uint64_t x, uint64_t vmin,
                                          bool& up, double& gap) {
  const double p = __dmul_rn(th, double(t));
  const double fp = floor(p);
  const double e = __fma_rn(th, double(t), -p);  // exact: theta1 * t - p
  up = fp == p && e < 0.0;
  gap = ((fp + 1.0) - p) - e;
  return int64_t(x - vmin) - int64_t(fp) + (up ? 1 : 0);
}

__device__ inline void set_bits(unsigned long long* bits, uint64_t k, uint64_t mask) {
  const uint64_t w = k >> 6, off = k & 63;
  atomicOr(bits + w, static_cast<unsigned long long>(mask << off));
  if (off && (mask >> (64 - off))) atomicOr(bits + w + 1, static_cast<unsigned long long>(mask >> (64 - off)));
}

__device__ inline void clear_bit(unsigned long long* bits, uint64_t k) {
  atomicAnd(bits + (k >> 6), ~(1ull << (k & 63)));
}

// Runs steps [kb, ke) from state st.  kFix = false: the bitmap holds zeros
// there and the walk sets the kept bits.  kFix = true: the bits are another
// run's, made from a different state; the walk rewrites them until it keeps
// a boundary that run also kept (from there on both runs are the same) and
// returns true at that point.  h / hr: the current partition's hulls, valid
// when hr.state is kHullValid and a merge is pending.  Called by a whole
// wavefront.
template <bool kFix>
__device__ bool merge_walk(const uint8_t* __restrict__ col, uint32_t dtype,
                           const uint64_t* __restrict__ s, const uint64_t* __restrict__ cost,
                           const uint64_t* __restrict__ pair, const RangeSum* __restrict__ psum,
                           uint64_t max_len, uint64_t kb, uint64_t ke, MergeState& st,
                           unsigned long long* __restrict__ keep, HullLds& w, HullRegs& hr) {
  const ChainHull& h = w.h;
  const uint32_t lane = threadIdx.x & 63;
  constexpr uint64_t kWide = uint64_t(1) << 61;  // value spread beyond which no line is fitted
  uint64_t k = kb;
  while (k < ke) {
    if (st.a + 1 == k) {
      // No merge pending: the next 64 steps are decided from the sizes
      // known in advance, each as if the steps before it kept their
      // boundary; the first merge (or meeting) ends the batch.
      const uint64_t kk = k + lane;
      const bool valid = kk < ke;
      bool merge = false, met = false;
      if (valid) {
        const uint64_t u = pair[kk - 1];
        merge = u != kNoMerge && u < cost[kk - 1] + cost[kk];
        if (kFix && !merge) met = bit_set(keep, kk);
      }
      const uint64_t vmask = __ballot(valid), mmask = __ballot(merge),
                     smask = kFix ? __ballot(met) : 0;
      const int fm = mmask ? __ffsll(static_cast<long long>(mmask)) - 1 : 64;
      const int fs = smask ? __ffsll(static_cast<long long>(smask)) - 1 : 64;
      const int stop = fm < fs ? fm : fs;
      const uint64_t kept = stop >= 64 ? vmask : vmask & ((1ull << stop) - 1);
      if (lane == 0 && kept) set_bits(keep, k, kept);
      if (fs < fm) return true;  // kFix: both runs keep boundary k + fs
      if (fm == 64) {            // every valid step kept its boundary
        const uint64_t last = uint64_t(63 - __clzll(static_cast<long long>(vmask)));
        st.a = k + last;
        st.cc = cost[st.a];
        st.sum = psum[st.a];
        k += last + 1;
        continue;
      }
      const uint64_t km = k + uint64_t(fm);
      if (kFix && lane == 0) clear_bit(keep, km);
      st.a = km - 1;
      st.cc = pair[km - 1];
      st.sum = join(psum[km - 1], psum[km], s[km] - s[km - 1]);
      hr = HullRegs{0, 0, kHullNone};
      k = km + 1;
      continue;
    }
    // The current partition absorbed others.  Lane l sizes its union with
    // partitions k .. k+l: the union's sums and extremes from the
    // partitions' summaries (a prefix across lanes), its slope from them,
    // and its residual range from the current partition's hulls and one
    // pass over the added values, every value broadcast to all lanes, each
    // lane predicting with its own slope.  Without hulls the pass covers
    // every value of the longest union, and the lanes taken are those
    // whose union is at most about twice the current length, so a run that
    // stops early wastes little of it.
    const uint64_t sa = s[st.a];
    const uint64_t lold = s[k] - sa;
    if (hr.state == kHullNone && lold >= kHullBuildMin) {
      if (lold <= kHullBuildMax && st.sum.vmax - st.sum.vmin < kWide) {
        hr = HullRegs{0, 0, kHullValid};
        hull_append(col, dtype, sa, 0, lold, st.sum.vmax - st.sum.vmin, w, hr);
      } else {
        hr.state = kHullDead;
      }
    }
    const bool via_hull = hr.state == kHullValid;
    const uint64_t j = k + lane;
    const uint64_t len0 = s[k + 1] - sa;
    const uint64_t lcap = len0 + (len0 > 512 ? len0 : 512);
    const uint64_t e_l = j < ke ? s[j + 1] : 0;
    const bool act =
        j < ke && (lane == 0 || (via_hull ? e_l - sa - lold <= kHullNewMax : e_l - sa <= lcap));
    const uint32_t nact = uint32_t(__popcll(__ballot(act)));  // a prefix of the lanes
    const uint64_t len_l = act ? e_l - sa : 0;
    RangeSum u{~uint64_t(0), 0, U128{0, 0}, U128{0, 0}};
    if (act) {
      u = psum[j];
      u.sty = add128(u.sty, mul128x64(u.sy, s[j] - sa));
    }
    // inclusive prefix over the lanes (the inactive ones add nothing)
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
      const uint64_t mn = shfl_up64(u.vmin, d), mx = shfl_up64(u.vmax, d);
      const U128 y{shfl_up64(u.sy.lo, d), shfl_up64(u.sy.hi, d)};
      const U128 ty{shfl_up64(u.sty.lo, d), shfl_up64(u.sty.hi, d)};
      if (int(lane) >= d) {
        u.vmin = mn < u.vmin ? mn : u.vmin;
        u.vmax = mx > u.vmax ? mx : u.vmax;
        u.sy = add128(u.sy, y);
        u.sty = add128(u.sty, ty);
      }
    }
    const uint64_t vmin = st.sum.vmin < u.vmin ? st.sum.vmin : u.vmin;
    const uint64_t vmax = st.sum.vmax > u.vmax ? st.sum.vmax : u.vmax;
    const uint64_t range = vmax - vmin;
    const bool fits = act && len_l <= max_len;
    const bool lin = fits && len_l > 1 && range < kWide;
    double th = 0.0;
    if (lin) th = ls_slope(len_l, add128(st.sum.sy, u.sy), add128(st.sum.sty, u.sty));
    int64_t rmin = INT64_MAX, rmax = INT64_MIN;
    const uint64_t lmax = readlane64(len_l, nact - 1);
    const uint8_t* src = col + sa * dtype;
    // 32 bits suffice when, on every lane fitting a line, the union's values
    // lie within 2^31 of its minimum and every |prediction| is below 2^31
    const bool narrow =
        __ballot(lin && !(range < (uint64_t(1) << 31) &&
                          __dmul_rn(fabs(th), double(len_l)) < 2147483648.0)) == 0;
    // the values of [tb, lmax) staged 64 at a time in LDS, each read by
    // every lane at once, every lane predicting with its own slope
    auto scan = [&](uint64_t tb) {
      for (uint64_t t0 = tb; t0 < lmax; t0 += 64) {
        const uint64_t t = t0 + lane;
        w.stage[lane] = load_value(src, dtype, t < lmax ? t : lmax - 1);
        wave_lds_order();
        const uint32_t cnt = lmax - t0 < 64 ? uint32_t(lmax - t0) : 64u;
        if (narrow) {
          const uint32_t vmin32 = uint32_t(vmin);
          int32_t mn = INT32_MAX, mx = INT32_MIN;
          for (uint32_t q = 0; q < cnt; ++q) {
            const uint32_t tq = uint32_t(t0) + q;
            const bool in = lin && tq < len_l;
            const int32_t rr = int32_t(uint32_t(w.stage[q]) - vmin32) - predict32(th, in ? tq : 0);
            mn = in ? min(mn, rr) : mn;
            mx = in ? max(mx, rr) : mx;
          }
          rmin = mn < rmin ? mn : rmin;
          rmax = mx > rmax ? mx : rmax;
        } else {
          for (uint32_t q = 0; q < cnt; ++q) {
            const uint64_t tq = t0 + q;
            if (lin && tq < len_l) {
              const int64_t rr = int64_t(w.stage[q] - vmin) - predict(th, uint32_t(tq));
              rmin = rr < rmin ? rr : rmin;
              rmax = rr > rmax ? rr : rmax;
            }
          }
        }
        wave_lds_order();  // every read of the block precedes the next one's staging
      }
    };
    bool scan_all = !via_hull;
    if (via_hull) {
      scan(lold);  // the added values
      bool unsure = false;
      if (lin) {
        const double pmax = __dmul_rn(fabs(th), double(len_l));  // bounds every |product|
        if (!(pmax < 2147483648.0)) {
          unsure = true;  // products too large for the rounding test below
        } else {
          // Old values.  Exact residuals: the largest, R, is at an upper
          // vertex and the smallest, Q, at a lower one.  The encoder's
          // largest is R unless every value reaching R rounds up; its
          // smallest is Q - 1 if some value reaching Q rounds up, which
          // needs a product within half an ulp of pmax under an integer:
          // ruled out when the lower vertices reaching Q, among them the
          // one minimising v - theta1 * t, have a larger gap (margin: two
          // ulps of pmax, at least 2^-48 against the gap's own rounding).
          const double margin = pmax >= 0x1p-3 ? fmax(ldexp(1.0, ilogb(pmax) - 51), 0x1p-48)
                                               : 0x1p-48;
          int64_t R = INT64_MIN, Q = INT64_MAX;
          bool r_exact = false, q_up = false, q_gap = true;
          for (uint32_t i = 0; i < hr.nu; ++i) {
            bool up;
            double gap;
            const int64_t rr = vertex_residual(th, h.t[0][i], h.x[0][i], vmin, up, gap);
            if (rr > R) {
              R = rr;
              r_exact = !up;
            } else if (rr == R) {
              r_exact = r_exact || !up;
            }
          }
          for (uint32_t i = 0; i < hr.nl; ++i) {
            bool up;
            double gap;
            const int64_t rr = vertex_residual(th, h.t[1][i], h.x[1][i], vmin, up, gap);
            const bool wide_gap = gap >= margin;
            if (rr < Q) {
              Q = rr;
              q_up = up;
              q_gap = wide_gap;
            } else if (rr == Q) {
              q_up = q_up || up;
              q_gap = q_gap && wide_gap;
            }
          }
          if (r_exact || rmax >= R) rmax = rmax > R ? rmax : R;
          else unsure = true;
          if (q_up) rmin = rmin < Q - 1 ? rmin : Q - 1;
          else if (q_gap) rmin = rmin < Q ? rmin : Q;
          else if (rmin > Q - 1) unsure = true;
        }
      }
      scan_all = __ballot(unsure) != 0;
      if (scan_all) {
        rmin = INT64_MAX;
        rmax = INT64_MIN;
      }
    }
    if (scan_all) scan(0);
    uint32_t bits = bitlen64(range);
    if (lin) {
      const uint32_t b_ls = bitlen64(uint64_t(rmax) - uint64_t(rmin));
      if (b_ls < bits) bits = b_ls;
    }
    const uint64_t size = fits ? kRecordBytes + 8 + 8 * ((len_l * bits + 63) >> 6) : kNoMerge;
    uint64_t prev = shfl_up64(size, 1);
    if (lane == 0) prev = st.cc;
    const bool merge = act && size != kNoMerge && size < prev + (act ? cost[j] : 0);
    const uint64_t refuse = __ballot(act && !merge);
    const uint32_t f = refuse ? uint32_t(__ffsll(static_cast<long long>(refuse)) - 1) : nact;
    if (kFix && lane == 0 && f > 0) {  // steps k .. k+f-1 merged
      for (uint32_t i = 0; i < f; ++i) clear_bit(keep, k + i);
    }
    if (f == nact) {  // the chain goes on past the batch
      st.cc = readlane64(size, f - 1);
      st.sum.vmin = readlane64(vmin, f - 1);
      st.sum.vmax = readlane64(vmax, f - 1);
      st.sum.sy = add128(st.sum.sy, U128{readlane64(u.sy.lo, f - 1), readlane64(u.sy.hi, f - 1)});
      st.sum.sty = add128(st.sum.sty, U128{readlane64(u.sty.lo, f - 1), readlane64(u.sty.hi, f - 1)});
      if (hr.state == kHullValid) {
        const uint64_t lnew = s[k + f] - sa;
        if (lnew - lold > kHullAppendMax || st.sum.vmax - st.sum.vmin >= kWide)
          hr.state = kHullDead;
        else
          hull_append(col, dtype, sa, lold, lnew, st.sum.vmax - st.sum.vmin, w, hr);
      }
      k += f;
      continue;
    }
    // step k+f refuses: boundary k+f is kept and partition k+f is current
    const uint64_t kk = k + f;
    bool met = false;
    if (lane == 0) {
      if (kFix) met = bit_set(keep, kk);
      if (!met) set_bits(keep, kk, 1);
    }
    met = __ballot(met) != 0;
    st.a = kk;
    st.cc = cost[kk];
    st.sum = psum[kk];
    hr = HullRegs{0, 0, kHullNone};
    k = kk + 1;
    if (met) return true;
  }
  return false;
}


// psum[j] = the summary of partition j, j < m: one lane per partition of at
// most 64 values, the wavefront together for the longer ones of its 64.
__global__ __launch_bounds__(kEncBlock) void k_part_sums(const uint8_t* __restrict__ col,
                                                        uint32_t dtype,
                                                        const uint64_t* __restrict__ s,
                                                        uint64_t m, RangeSum* __restrict__ psum) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t waves = uint64_t(gridDim.x) * kEncWaves;
  for (uint64_t j0 = (uint64_t(blockIdx.x) * kEncWaves + (threadIdx.x >> 6)) * 64; j0 < m;
       j0 += waves * 64) {
    const uint64_t j = j0 + lane;
    uint64_t a = 0, e = 0;
    if (j < m) {
      a = s[j];
      e = s[j + 1];
    }
    const bool shortp = j < m && e - a <= 64;
    if (shortp) {
      RangeSum r{~uint64_t(0), 0, U128{0, 0}, U128{0, 0}};
      for (uint64_t t = 0; t < e - a; ++t) {
        const uint64_t x = load_value(col, dtype, a + t);
        r.vmin = x < r.vmin ? x : r.vmin;
        r.vmax = x > r.vmax ? x : r.vmax;
        r.sy = add128(r.sy, U128{x, 0});
        r.sty = add128(r.sty, mul64x64(t, x));
      }
      psum[j] = r;
    }
    uint64_t todo = __ballot(j < m && !shortp);
    while (todo) {
      const uint32_t l = uint32_t(__ffsll(static_cast<long long>(todo)) - 1);
      todo &= todo - 1;
      const uint64_t la = readlane64(a, l), le = readlane64(e, l);
      RangeSum r{~uint64_t(0), 0, U128{0, 0}, U128{0, 0}};
      for (uint64_t t = lane; t < le - la; t += 64) {
        const uint64_t x = load_value(col, dtype, la + t);
        r.vmin = x < r.vmin ? x : r.vmin;
        r.vmax = x > r.vmax ? x : r.vmax;
        r.sy = add128(r.sy, U128{x, 0});
        r.sty = add128(r.sty, mul64x64(t, x));
      }
      wave_minmax_u64(r.vmin, r.vmax);
      wave_sum_u128x2(r.sy, r.sty);
      if (lane == 0) psum[j0 + l] = r;
    }
  }
}


// Speculative pass: one wavefront per chunk of kMergeChunk boundaries,
// scanned as if its first boundary were kept (chunk 0 from the true start);
// each chunk's end state and hulls go to out and hulls, and seen[q] records
// the entry state the chunk was walked from.
__global__ __launch_bounds__(kEncBlock) void k_merge_spec(
    const uint8_t* __restrict__ col, uint32_t dtype, const uint64_t* __restrict__ s,
    const uint64_t* __restrict__ cost, const uint64_t* __restrict__ pair,
    const RangeSum* __restrict__ psum, uint64_t m, uint64_t max_len,
    unsigned long long* __restrict__ keep, MergeState* __restrict__ out,
    ChainHull* __restrict__ hulls, uint64_t* __restrict__ seen) {
  __shared__ HullLds lds[kEncWaves];
  const uint32_t wv = threadIdx.x >> 6;
  const uint64_t q = uint64_t(blockIdx.x) * kEncWaves + wv;
  const uint64_t k0 = q << kMergeChunkLog2;
  if (k0 >= m) return;
  const uint64_t ke = m - k0 < kMergeChunk ? m : k0 + kMergeChunk;
  MergeState st;
  uint64_t kb = k0;
  if (q == 0) {
    if ((threadIdx.x & 63) == 0) set_bits(keep, 0, 1);
    st = MergeState{0, cost[0], psum[0]};
    kb = 1;
  } else {
    st = MergeState{k0 - 1, cost[k0 - 1], psum[k0 - 1]};
    if ((threadIdx.x & 63) == 0) seen[q] = k0 - 1;
  }
  HullRegs hr{0, 0, kHullNone};
  merge_walk<false>(col, dtype, s, cost, pair, psum, max_len, kb, ke, st, keep, lds[wv], hr);
  if ((threadIdx.x & 63) == 0) out[q] = st;
  hull_store(hulls + q, lds[wv].h, hr);
}

// Fix-up rounds.  out[q] is the end state (hulls[q] its hulls) of the run
// recorded in chunk q's bits, and seen[q] the state that run began in.  A
// round walks the chunks of one parity whose left neighbour's end state
// differs from seen: from that state, rewriting the chunk's bits until it
// keeps a boundary the recorded run also kept (from there on that run is
// right, and so is its end state) or reaches the chunk's end (its end state
// is the new out[q]).  The neighbours, of the other parity, do not run in
// the same round.  Chunk 0 begins where the column does, so after round r
// (parities 1, 0, 1, ...) at least chunks 0..r are right; rounds repeat
// until two in a row walk nothing.
__global__ __launch_bounds__(kEncBlock) void k_merge_round(
    const uint8_t* __restrict__ col, uint32_t dtype, const uint64_t* __restrict__ s,
    const uint64_t* __restrict__ cost, const uint64_t* __restrict__ pair,
    const RangeSum* __restrict__ psum, uint64_t m, uint64_t max_len,
    unsigned long long* __restrict__ keep, MergeState* __restrict__ out,
    ChainHull* __restrict__ hulls, uint64_t* __restrict__ seen, uint64_t nchunks,
    uint32_t parity, unsigned long long* __restrict__ walks) {
  __shared__ HullLds lds[kEncWaves];
  const uint32_t wv = threadIdx.x >> 6;
  const uint64_t q = 2 * (uint64_t(blockIdx.x) * kEncWaves + wv) + parity;
  if (q == 0 || q >= nchunks) return;
  MergeState st = out[q - 1];
  if (st.a == seen[q]) return;
  const uint64_t kb = q << kMergeChunkLog2;
  const uint64_t ke = m - kb < kMergeChunk ? m : kb + kMergeChunk;
  HullRegs hr{0, 0, kHullNone};
  if (st.a + 1 < kb) hr = hull_load(hulls + (q - 1), lds[wv].h);
  const bool met =
      merge_walk<true>(col, dtype, s, cost, pair, psum, max_len, kb, ke, st, keep, lds[wv], hr);
  if ((threadIdx.x & 63) == 0) {
    seen[q] = out[q - 1].a;
    if (!met) out[q] = st;
    atomicAdd(walks, 1ull);
  }
  if (!met) hull_store(hulls + q, lds[wv].h, hr);
}

// ---- compaction after a pass --------------------------------------------------------

__device__ inline uint32_t kept_bit(const unsigned long long* keep, uint64_t k, uint64_t m) {
  return k < m && ((keep[k >> 6] >> (k & 63)) & 1ull) ? 1u : 0u;
}

// Kept boundaries in words [blockIdx * 1024, +1024) of the bitmap.
__global__ __launch_bounds__(kScanBlock) void k_keep_count(const unsigned long long* __restrict__ keep,
                                                           uint64_t m, uint64_t* __restrict__ counts) {
  const uint64_t nwords = (m + 63) / 64;
  const uint64_t w0 = uint64_t(blockIdx.x) * kItemsPerBlock + threadIdx.x * 4;
  uint32_t c = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint64_t w = w0 + q;
    if (w < nwords) {
      uint64_t x = keep[w];
      if ((w + 1) * 64 > m) x &= (m & 63) ? ((1ull << (m & 63)) - 1) : ~0ull;
      c += uint32_t(__popcll(x));
    }
  }
  uint32_t total;
  block_exclusive_scan(c, &total);
  if (threadIdx.x == 0) counts[blockIdx.x] = total;
}

// Copies the kept starts to their new places with their sizes (a
// partition that absorbed others is sized afterwards), whether it absorbed
// others, and its old index.
__global__ __launch_bounds__(kScanBlock) void k_keep_emit(
    const unsigned long long* __restrict__ keep, uint64_t m, const uint64_t* __restrict__ offsets,
    const uint64_t* __restrict__ starts, const uint64_t* __restrict__ cost,
    uint64_t* __restrict__ starts_out, uint64_t* __restrict__ cost_out,
    uint8_t* __restrict__ changed_out, uint64_t* __restrict__ old_out) {
  const uint64_t w0 = uint64_t(blockIdx.x) * kItemsPerBlock + threadIdx.x * 4;
  uint32_t c = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    for (uint64_t k = (w0 + q) * 64; k < (w0 + q + 1) * 64 && k < m; ++k) c += kept_bit(keep, k, m);
  uint32_t total;
  uint64_t out = offsets[blockIdx.x] + block_exclusive_scan(c, &total);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    for (uint64_t k = (w0 + q) * 64; k < (w0 + q + 1) * 64 && k < m; ++k) {
      if (!kept_bit(keep, k, m)) continue;
      const bool absorbed = k + 1 < m && !kept_bit(keep, k + 1, m);
      starts_out[out] = starts[k];
      cost_out[out] = cost[k];
      changed_out[out] = absorbed ? 1 : 0;
      old_out[out] = k;
      ++out;
    }
  }
}

// After a pass: the pair (k, k+1) of the new partitions keeps its union
// size when neither absorbed a neighbour (they were adjacent before, as old
// partitions old[k] and old[k] + 1); the others are marked for sizing.
__global__ void k_pair_reuse(uint64_t m, const uint8_t* __restrict__ changed,
                             const uint64_t* __restrict__ old, const uint64_t* __restrict__ pair,
                             uint64_t* __restrict__ pair_out, uint8_t* __restrict__ dirty) {
  const uint64_t k = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k + 1 >= m) return;
  const bool fresh = changed[k] || changed[k + 1];
  if (!fresh) pair_out[k] = pair[old[k]];
  dirty[k] = fresh ? 1 : 0;
}

}  // namespace leco

// ---- host side ------------------------------------------------------------------

namespace {

// Device buffers of one call, freed on every exit path.
struct Buffers {
  std::vector<void*> ptrs;
  ~Buffers() {
    for (void* p : ptrs) (void)hipFree(p);
  }
  template <class T>
  bool alloc(T** p, uint64_t count) {
    void* q = nullptr;
    if (hipMalloc(&q, count ? count * sizeof(T) : sizeof(T)) != hipSuccess) return false;
    ptrs.push_back(q);
    *p = static_cast<T*>(q);
    return true;
  }
};

leco_status pfail(leco_ctx* ctx, leco_status st, const char* msg) {
  ctx->last_error = msg;
  return st;
}

// Exclusive scan of per-block counts on the host (a few thousand entries).
hipError_t scan_counts(uint64_t* counts_dev, uint64_t nblocks, uint64_t* total,
                       hipStream_t stream) {
  std::vector<uint64_t> c(nblocks);
  hipError_t e = hipMemcpyAsync(c.data(), counts_dev, 8 * nblocks, hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return e;
  uint64_t run = 0;
  for (uint64_t i = 0; i < nblocks; ++i) {
    const uint64_t x = c[i];
    c[i] = run;
    run += x;
  }
  *total = run;
  e = hipMemcpyAsync(counts_dev, c.data(), 8 * nblocks, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);  // c is freed on return
  return e;
}

}  // namespace

#define P_TRY(call)                                                  \
  do {                                                               \
    const hipError_t e_ = (call);                                    \
    if (e_ != hipSuccess) return pfail(ctx, LECO_EDEVICE, hipGetErrorString(e_)); \
  } while (0)

extern "C" {

leco_status leco_partition(leco_ctx* ctx, const void* col_dev, uint64_t n, leco_dtype dtype,
                           const leco_partition_params* prm, uint64_t* starts_host,
                           uint64_t starts_cap, uint64_t* m_out, hipStream_t stream) {
  if (!ctx) return LECO_EINVAL;
  if (!prm || !m_out || (dtype != LECO_U32 && dtype != LECO_U64))
    return pfail(ctx, LECO_EINVAL, "partition: null argument or bad dtype");
  if (prm->max_len == 0 || prm->max_len > leco::kMaxPartLen || !(prm->tau == prm->tau))
    return pfail(ctx, LECO_EINVAL, "partition: max_len outside 1..2^20 or tau NaN");
  if ((prm->start_positions != 0 && prm->start_positions != 1) || prm->reserved != 0)
    return pfail(ctx, LECO_EINVAL, "partition: start_positions not 0 or 1, or reserved not 0");
  if (n && (!col_dev || (reinterpret_cast<uintptr_t>(col_dev) & (uint64_t(dtype) - 1))))
    return pfail(ctx, LECO_EINVAL, "partition: null or misaligned column");
  if (starts_cap && !starts_host) return pfail(ctx, LECO_EINVAL, "partition: null starts buffer");
  *m_out = 0;
  if (n == 0) {
    if (starts_cap < 1) return pfail(ctx, LECO_ENOSPC, "partition: starts buffer too small");
    starts_host[0] = 0;
    return LECO_OK;
  }
  P_TRY(hipSetDevice(ctx->device));
  const uint8_t* col = static_cast<const uint8_t*>(col_dev);
  const uint32_t w = uint32_t(dtype);
  const double thr = prm->tau * double(prm->sm_bits);
  Buffers buf;

  // split: bitmap of partition starts
  const uint64_t nwords = (n + 63) / 64;
  const uint64_t nseg = (n + (uint64_t(1) << leco::kSegLog2) - 1) >> leco::kSegLog2;
  unsigned long long* bitmap = nullptr;
  if (!buf.alloc(&bitmap, nwords)) return pfail(ctx, LECO_ENOMEM, "partition: bitmap");
  P_TRY(hipMemsetAsync(bitmap, 0, 8 * nwords, stream));
  const uint64_t nsub = (n + (uint64_t(1) << leco::kSubLog2) - 1) >> leco::kSubLog2;
  leco::SplitState *states = nullptr, *seg_states = nullptr;
  if (!buf.alloc(&states, nsub) || !buf.alloc(&seg_states, nseg))
    return pfail(ctx, LECO_ENOMEM, "partition: split states");
  // starting partitions: bitmaps of their first and later values
  uint64_t *first = nullptr, *inside = nullptr;
  if (prm->start_positions) {
    const uint64_t cap = uint64_t(ctx->num_cus) * 8;
    const uint64_t gd0 = (n + leco::kScanBlock - 1) / leco::kScanBlock;
    const uint64_t gd = gd0 < cap ? gd0 : cap;
    uint64_t *partial = nullptr, *best = nullptr;
    if (!buf.alloc(&first, nwords) || !buf.alloc(&inside, nwords) ||
        !buf.alloc(&partial, 2 * gd) || !buf.alloc(&best, 2))
      return pfail(ctx, LECO_ENOMEM, "partition: starting partitions");
    hipLaunchKernelGGL(leco::k_dd_min, dim3(uint32_t(gd)), dim3(leco::kScanBlock), 0, stream, col,
                       w, n, partial);
    P_TRY(hipGetLastError());
    hipLaunchKernelGGL(leco::k_dd_min_final, dim3(1), dim3(64), 0, stream, partial, gd, best);
    P_TRY(hipGetLastError());
    hipLaunchKernelGGL(leco::k_mark_starting, dim3(uint32_t(gd)), dim3(leco::kScanBlock), 0, stream,
                       col, w, n, best, first, inside);
    P_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(leco::k_split_spec, dim3(uint32_t(nsub)), dim3(64), 0, stream, col, w, n,
                     thr, prm->max_len, bitmap, states, first, inside);
  P_TRY(hipGetLastError());
  hipLaunchKernelGGL(leco::k_split_fix, dim3(uint32_t(nseg)), dim3(64), 0, stream, col, w, n, thr,
                     prm->max_len, bitmap, states, seg_states, first, inside);
  P_TRY(hipGetLastError());
  if (nseg > 1) {
    hipLaunchKernelGGL(leco::k_split_join, dim3(1), dim3(64), 0, stream, col, w, n, thr,
                       prm->max_len, bitmap, seg_states, nseg, first, inside);
    P_TRY(hipGetLastError());
  }

  // starts from the bitmap
  const uint64_t nb = (nwords + leco::kItemsPerBlock - 1) / leco::kItemsPerBlock;
  uint64_t* counts = nullptr;
  if (!buf.alloc(&counts, nb)) return pfail(ctx, LECO_ENOMEM, "partition: counts");
  hipLaunchKernelGGL(leco::k_bitmap_count, dim3(uint32_t(nb)), dim3(leco::kScanBlock), 0, stream,
                     reinterpret_cast<const uint64_t*>(bitmap), nwords, counts);
  P_TRY(hipGetLastError());
  uint64_t m = 0;
  P_TRY(scan_counts(counts, nb, &m, stream));
  uint64_t *starts = nullptr, *starts2 = nullptr, *cost = nullptr, *cost2 = nullptr,
           *pair = nullptr, *pair2 = nullptr, *old = nullptr, *keep_counts = nullptr;
  uint8_t *changed = nullptr, *dirty = nullptr;
  unsigned long long *keep = nullptr, *walks = nullptr;
  leco::MergeState* mout = nullptr;
  leco::ChainHull* hulls = nullptr;
  leco::RangeSum* psum = nullptr;
  uint64_t* seen = nullptr;
  constexpr int kRoundGroup = 8;  // fix-up rounds launched between checks
  const uint64_t kwords = (m + 63) / 64;
  const uint64_t nbk = (kwords + leco::kItemsPerBlock - 1) / leco::kItemsPerBlock;
  const uint64_t nchunks0 = (m + leco::kMergeChunk - 1) / leco::kMergeChunk;
  if (!buf.alloc(&starts, m + 1) || !buf.alloc(&starts2, m + 1) || !buf.alloc(&cost, m) ||
      !buf.alloc(&cost2, m) || !buf.alloc(&pair, m) || !buf.alloc(&pair2, m) ||
      !buf.alloc(&old, m) || !buf.alloc(&changed, m) || !buf.alloc(&dirty, m) ||
      !buf.alloc(&keep, kwords) || !buf.alloc(&keep_counts, nbk) ||
      !buf.alloc(&mout, nchunks0) || !buf.alloc(&hulls, nchunks0) || !buf.alloc(&psum, m) ||
      !buf.alloc(&seen, nchunks0) || !buf.alloc(&walks, kRoundGroup))
    return pfail(ctx, LECO_ENOMEM, "partition: partition arrays");
  hipLaunchKernelGGL(leco::k_bitmap_emit, dim3(uint32_t(nb)), dim3(leco::kScanBlock), 0, stream,
                     reinterpret_cast<const uint64_t*>(bitmap), nwords, counts, starts);
  P_TRY(hipGetLastError());
  P_TRY(hipMemcpyAsync(starts + m, &n, 8, hipMemcpyHostToDevice, stream));

  // merge passes
  const uint64_t grid_cap = uint64_t(ctx->num_cus) * 16;
  auto costs = [&](const uint64_t* s, uint64_t count, uint32_t span, const uint8_t* dirty,
                   uint64_t* out) {
    if (count == 0) return hipSuccess;
    const uint64_t gs = (count + leco::kEncBlock - 1) / leco::kEncBlock;
    hipLaunchKernelGGL(leco::k_costs_short, dim3(uint32_t(gs < grid_cap ? gs : grid_cap)),
                       dim3(leco::kEncBlock), 0, stream, col, w, s, count, span, prm->max_len,
                       dirty, out);
    hipError_t e0 = hipGetLastError();
    if (e0 != hipSuccess) return e0;
    // chunks of ranges: at least one per resident wavefront (k_costs) or
    // workgroup (k_costs_long), at most kCostChunk ranges each
    auto chunk_for = [&](uint64_t units) {
      const uint64_t c = count / units;
      return uint32_t(c < 1 ? 1 : (c > leco::kCostChunk ? leco::kCostChunk : c));
    };
    const uint32_t cw = chunk_for(grid_cap * leco::kEncWaves);
    const uint64_t chunks_w = (count + cw - 1) / cw;
    const uint64_t gw = (chunks_w + leco::kEncWaves - 1) / leco::kEncWaves;
    hipLaunchKernelGGL(leco::k_costs, dim3(uint32_t(gw < grid_cap ? gw : grid_cap)),
                       dim3(leco::kEncBlock), 0, stream, col, w, s, count, span, prm->max_len,
                       dirty, out, cw);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const uint32_t cl = chunk_for(grid_cap);
    const uint64_t chunks_l = (count + cl - 1) / cl;
    const uint64_t gl = chunks_l < grid_cap ? chunks_l : grid_cap;
    hipLaunchKernelGGL(leco::k_costs_long, dim3(uint32_t(gl)), dim3(leco::kEncBlock), 0, stream,
                       col, w, s, count, span, prm->max_len, dirty, out, cl);
    return hipGetLastError();
  };
  P_TRY(costs(starts, m, 1, nullptr, cost));
  if (m >= 2) P_TRY(costs(starts, m - 1, 2, nullptr, pair));
  for (uint64_t pass = 0; prm->max_passes == 0 || pass < prm->max_passes; ++pass) {
    if (m < 2) break;
    const uint64_t words = (m + 63) / 64;
    const uint64_t nchunks = (m + leco::kMergeChunk - 1) / leco::kMergeChunk;
    P_TRY(hipMemsetAsync(keep, 0, 8 * words, stream));
    const uint64_t gsum = (m + 64 * leco::kEncWaves - 1) / (64 * leco::kEncWaves);
    hipLaunchKernelGGL(leco::k_part_sums, dim3(uint32_t(gsum < grid_cap ? gsum : grid_cap)),
                       dim3(leco::kEncBlock), 0, stream, col, w, starts, m, psum);
    P_TRY(hipGetLastError());
    const uint32_t gch = uint32_t((nchunks + leco::kEncWaves - 1) / leco::kEncWaves);
    hipLaunchKernelGGL(leco::k_merge_spec, dim3(gch), dim3(leco::kEncBlock), 0, stream, col, w,
                       starts, cost, pair, psum, m, prm->max_len, keep, mout, hulls, seen);
    P_TRY(hipGetLastError());
    // fix-up rounds, parities 1, 0, 1, ..., until two in a row walk nothing;
    // chunk r is right after round r, so nchunks rounds always suffice
    const uint64_t half = (nchunks + 1) / 2;
    const uint32_t ghalf = uint32_t((half + leco::kEncWaves - 1) / leco::kEncWaves);
    for (uint64_t r0 = 0; nchunks > 1 && r0 < nchunks + 2 * kRoundGroup; r0 += kRoundGroup) {
      P_TRY(hipMemsetAsync(walks, 0, 8 * kRoundGroup, stream));
      for (int i = 0; i < kRoundGroup; ++i) {
        hipLaunchKernelGGL(leco::k_merge_round, dim3(ghalf), dim3(leco::kEncBlock), 0, stream, col,
                           w, starts, cost, pair, psum, m, prm->max_len, keep, mout, hulls, seen,
                           nchunks, uint32_t((r0 + i + 1) & 1), walks + i);
        P_TRY(hipGetLastError());
      }
      unsigned long long nwalk[kRoundGroup];
      P_TRY(hipMemcpyAsync(nwalk, walks, 8 * kRoundGroup, hipMemcpyDeviceToHost, stream));
      P_TRY(hipStreamSynchronize(stream));
      if (nwalk[kRoundGroup - 2] == 0 && nwalk[kRoundGroup - 1] == 0) break;
    }
    const uint64_t blocks = (words + leco::kItemsPerBlock - 1) / leco::kItemsPerBlock;
    hipLaunchKernelGGL(leco::k_keep_count, dim3(uint32_t(blocks)), dim3(leco::kScanBlock), 0,
                       stream, keep, m, keep_counts);
    P_TRY(hipGetLastError());
    uint64_t m2 = 0;
    P_TRY(scan_counts(keep_counts, blocks, &m2, stream));
    if (m2 == m) break;  // the pass merged nothing
    hipLaunchKernelGGL(leco::k_keep_emit, dim3(uint32_t(blocks)), dim3(leco::kScanBlock), 0,
                       stream, keep, m, keep_counts, starts, cost, starts2, cost2, changed, old);
    P_TRY(hipGetLastError());
    P_TRY(hipMemcpyAsync(starts2 + m2, &n, 8, hipMemcpyHostToDevice, stream));
    // sizes of the partitions that absorbed others
    P_TRY(costs(starts2, m2, 1, changed, cost2));
    if (m2 >= 2) {
      // pair sizes for the next pass: reused, or sized where a merge happened
      hipLaunchKernelGGL(leco::k_pair_reuse, dim3(uint32_t((m2 - 1 + 255) / 256)), dim3(256), 0,
                         stream, m2, changed, old, pair, pair2, dirty);
      P_TRY(hipGetLastError());
      P_TRY(costs(starts2, m2 - 1, 2, dirty, pair2));
    }
    P_TRY(hipStreamSynchronize(stream));  // &n stays valid until the copy is done
    std::swap(starts, starts2);
    std::swap(cost, cost2);
    std::swap(pair, pair2);
    m = m2;
  }
  *m_out = m;
  if (starts_cap < m + 1) return pfail(ctx, LECO_ENOSPC, "partition: starts buffer too small");
  P_TRY(hipMemcpyAsync(starts_host, starts, 8 * (m + 1), hipMemcpyDeviceToHost, stream));
  P_TRY(hipStreamSynchronize(stream));
  return LECO_OK;
}

}  // extern "C"
