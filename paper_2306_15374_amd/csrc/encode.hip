// LeCo encoder for gfx950 (section 3.1 regressor, section 3.3 encoder), in
// two passes over the input that need no ordering between partitions:
//
//   fit    every partition's model: range, exact least-squares sums, slope,
//          residual range, the choice between the line and the constant
//          model (section 3.1), hence its width b and its word count; with
//          the minimax regressor also the minimax line (k_fit_minimax*,
//          hulls in minimax.hpp), with the polynomial regressor the
//          degree-2 and degree-3 polynomials (k_fit_poly*);
//   scan   the exclusive prefix of the word counts gives every partition's
//          word offset; the records, starts, header and padding are written;
//   pack   every partition's residuals, recomputed from its stored model,
//          are bit-packed into its word span (section 3.3 storage format).
//
// The fits take one wavefront per partition when every partition holds at
// most kWaveEncodeMax values (16 per lane) or twice that (32 per lane; not
// the minimax fit): values in registers, shuffle reductions, no workgroup
// barrier.  Longer partitions get a whole workgroup.  Works on a table of columns, so one sequence of
// launches encodes one column or thousands.  The column is read twice; in
// exchange no partition waits on another.
//
// Register-resident partitions whose range is below 2^30 (the usual case)
// fit on a narrow path: y = v - vmin fits 32 bits, the exact sums fit 64-bit
// lanes, and predictions and residuals fit int32.  The arithmetic and its
// results are the same as on the general path, only carried in fewer bits.
#include "fit.hpp"
#include "internal.hpp"
#include "leco_dev.hpp"
#include "minimax.hpp"

namespace leco {

constexpr int kEncRegs = 16;                           // values per thread in registers
constexpr uint32_t kEncRegLen = kEncBlock * kEncRegs;  // 4096
constexpr uint32_t kWaveEncMax = uint32_t(kWaveEncodeMax);
constexpr int kWaveRegs = int(kWaveEncMax / 64);      // values per lane, one wavefront
constexpr uint64_t kNarrowRange = 1ull << 30;
constexpr uint32_t kScanItems = 1024;                  // word counts per scan workgroup

__device__ inline void raise(int* err, int bits) { atomicOr(err, bits); }

__device__ inline void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct FitShared {
  uint64_t red[kEncWaves][4];
  double theta1;
};

// ORs a residual u (< 2^b) into a stream of 32-bit words at bit q.
__device__ inline void or_bits(uint32_t* w, uint32_t q, uint32_t b, uint64_t u) {
  if (u == 0) return;
  const uint32_t i = q >> 5, s = q & 31;
  atomicOr(&w[i], uint32_t(u << s));
  if (s + b > 32) atomicOr(&w[i + 1], uint32_t(u >> (32 - s)));
  if (s + b > 64) atomicOr(&w[i + 2], uint32_t(u >> (64 - s)));
}

// p[i] read through the constant address space: a scalar load when i is
// uniform across the wavefront.  Only for data written before the launch.
template <class T>
__device__ inline T meta_load(const T* p, uint64_t i) {
  return ((const __attribute__((address_space(4))) T*)p)[i];
}

constexpr uint32_t kColWords = sizeof(EncColumn) / 8;
static_assert(sizeof(EncColumn) == 104 && offsetof(EncColumn, part_base) == 72 &&
                  offsetof(EncColumn, dtype) == 80 && offsetof(EncColumn, regressor) == 88 &&
                  offsetof(EncColumn, val_base) == 96,
              "column entry layout");
static_assert(kHullTile == kHullTileValues, "hull tile");

// The column holding partition P: the kernel argument of a one-column
// launch, else the last table entry with part_base <= P, read word by word
// with scalar loads when P is uniform.
__device__ inline EncColumn column_of(const EncColumn* cols, uint64_t ncols,
                                      const EncColumn& single, uint64_t P) {
  if (cols == nullptr) return single;
  const uint64_t* t = reinterpret_cast<const uint64_t*>(cols);
  uint64_t lo = 0, hi = ncols;
  while (hi - lo > 1) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (meta_load(t, mid * kColWords + 9) <= P) lo = mid; else hi = mid;
  }
  const uint64_t e = lo * kColWords;
  EncColumn c;
  c.col = reinterpret_cast<const uint8_t*>(meta_load(t, e + 0));
  c.blob = reinterpret_cast<uint8_t*>(meta_load(t, e + 1));
  c.starts = reinterpret_cast<const uint64_t*>(meta_load(t, e + 2));
  c.size_out = reinterpret_cast<uint64_t*>(meta_load(t, e + 3));
  c.n = meta_load(t, e + 4);
  c.m = meta_load(t, e + 5);
  c.fixed_len = meta_load(t, e + 6);
  c.cap = meta_load(t, e + 7);
  c.words_off = meta_load(t, e + 8);
  c.part_base = meta_load(t, e + 9);
  const uint64_t w = meta_load(t, e + 10);
  c.dtype = uint32_t(w);
  c.force_constant = uint32_t(w >> 32);
  c.regressor = uint32_t(meta_load(t, e + 11));
  c.pad = 0;
  c.val_base = meta_load(t, e + 12);
  return c;
}

// First value and length of partition j of column c.
__device__ inline void part_bounds(const EncColumn& c, uint64_t j, uint64_t& start,
                                   uint64_t& len) {
  if (c.fixed_len) {
    start = j * c.fixed_len;
    len = (start + c.fixed_len < c.n ? start + c.fixed_len : c.n) - start;
  } else {
    start = meta_load(c.starts, j);
    len = meta_load(c.starts, j + 1) - start;
  }
}

__device__ inline void write_header(const EncColumn& c, uint64_t total_words) {
  uint64_t* hd = reinterpret_cast<uint64_t*>(c.blob);
  const bool variable = c.fixed_len == 0;
  const uint64_t flags = (variable ? kFlagVariable : 0) | (c.regressor == 2 ? kFlagPoly : 0);
  hd[0] = uint64_t(kMagic) | (uint64_t(kVersion) << 32) | (uint64_t(c.dtype) << 48) |
          (flags << 56);
  hd[1] = c.n;
  hd[2] = c.m;
  hd[3] = c.fixed_len;
  hd[4] = kHeaderBytes;
  hd[5] = variable ? kHeaderBytes + kRecordBytes * c.m : 0;
  hd[6] = c.words_off;
  hd[7] = total_words;
}

// Header, the last start and the zero padding of a column whose total word
// count is known; size checked against the capacity.
__device__ inline void finish_column(const EncColumn& c, uint64_t total_words, int* err) {
  const uint64_t size = align16(c.words_off + 8 * total_words);
  if (c.size_out) *c.size_out = size;
  if (size > c.cap) {
    raise(err, kErrNoSpace);
    return;
  }
  write_header(c, total_words);
  const bool variable = c.fixed_len == 0;
  const uint64_t meta_end = kHeaderBytes + kRecordBytes * c.m + (variable ? 8 * (c.m + 1) : 0);
  if (variable) reinterpret_cast<uint64_t*>(c.blob + kHeaderBytes + kRecordBytes * c.m)[c.m] = c.n;
  // padding around the coefficient section, which k_records fills
  const uint64_t coef = c.regressor == 2 ? align16(meta_end) : c.words_off;
  const uint64_t coef_end = c.regressor == 2 ? coef + 16 * c.m : c.words_off;
  for (uint64_t i = meta_end; i < coef; ++i) c.blob[i] = 0;
  for (uint64_t i = coef_end; i < c.words_off; ++i) c.blob[i] = 0;
  for (uint64_t i = c.words_off + 8 * total_words; i < size; ++i) c.blob[i] = 0;
}

// Writes the fitted model of partition P.
__device__ inline void store_model(const EncScratch& s, uint64_t P, const Model& md,
                                   uint64_t len) {
  s.base[P] = md.base;
  s.theta[P] = uint64_t(__double_as_longlong(md.theta1));
  s.bits[P] = md.bits;
  s.nwords[P] = (len * md.bits + 63) >> 6;
}

// ---- fit: one thread per partition ------------------------------------------------

// Partitions of at most this many values are fitted by one thread each when
// a launch holds no longer ones (a wavefront per partition left 63 of its
// 64 lanes idle at one value per partition: 1.4 ms for the 2e6 sampled
// partitions of a size search's first length).
constexpr uint64_t kLaneFitMax = 32;

// The model fit_wave_regs computes, by one thread: the same exact sums (the
// slope is one function of them, whatever their order), the same residual
// range and the same choice.
__device__ inline Model fit_lane(const uint8_t* src, uint32_t dtype, uint64_t len,
                                 bool force_constant) {
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
  if (len > 1 && !force_constant && range < (uint64_t(1) << 61)) {
    const double th = ls_slope(len, sv, stv);
    int64_t rmin = INT64_MAX, rmax = INT64_MIN;
    for (uint64_t t = 0; t < len; ++t) {
      const int64_t rr = int64_t(load_value(src, dtype, t) - vmin) - predict(th, uint32_t(t));
      rmin = rr < rmin ? rr : rmin;
      rmax = rr > rmax ? rr : rmax;
    }
    choose_model(md, th, rmin, rmax);
  }
  return md;
}

// Least-squares partitions of at most kLaneFitMax values, one thread each
// (grid-stride over the launch's partitions).
__global__ __launch_bounds__(256) void k_fit_lane(const EncColumn* __restrict__ cols,
                                                  uint64_t ncols, EncColumn single,
                                                  uint64_t nparts, EncScratch scr) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t P = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; P < nparts; P += stride) {
    const EncColumn c = column_of(cols, ncols, single, P);
    uint64_t start, len;
    part_bounds(c, P - c.part_base, start, len);
    const Model md = fit_lane(c.col + start * c.dtype, c.dtype, len, c.force_constant != 0);
    store_model(scr, P, md, len);
  }
}

// ---- fit: one wavefront per partition ---------------------------------------------

// Exact sums of y = v - vmin (below 2^61) and of t y over kN register-held
// values (value k at position t0 + k * kStride, positions from len on
// ignored), each y split at bit 32: s = {sum y_lo, sum y_hi} and
// st = {sum t y_lo, sum t y_hi}.  With at most 4096 values (t < 2^12) every
// component stays below 2^56, so the wavefront and workgroup sums of U128
// pairs add them component-wise (no carry leaves a low half), and
// join_split makes the 128-bit sums.  The slope of the offsets is the
// slope of the values.
template <int kN, uint32_t kStride, class W>
__device__ __attribute__((always_inline)) inline void split_sums_regs(
    const W (&v)[kN], uint32_t t0, uint64_t len, uint64_t vmin, U128& s, U128& st) {
  uint64_t slo = 0, shi = 0, stlo = 0, sthi = 0;
#pragma unroll
  for (int k = 0; k < kN; ++k) {
    const uint32_t t = t0 + k * kStride;
    const uint64_t y = t < len ? uint64_t(v[k]) - vmin : 0;
    const uint64_t yl = y & 0xffffffffu, yh = y >> 32;
    slo += yl;
    shi += yh;
    stlo += uint64_t(t) * yl;
    sthi += uint64_t(t) * yh;
  }
  s = U128{slo, shi};
  st = U128{stlo, sthi};
}

__device__ inline U128 join_split(U128 p) {
  return add128(U128{p.lo, 0}, U128{p.hi << 32, p.hi >> 32});
}

// Range of the least-squares residuals of kN register-held values, value k
// at position t0 + k * kStride (positions from len on ignored).  When small
// (values below vmin + 2^30, every |floor(theta1 t)| below 2^30, the same
// in every lane) each residual fits int32 and the range is taken in 32-bit
// operations; otherwise in 64-bit ones with the full prediction.
template <int kN, uint32_t kStride, class W>
__device__ __attribute__((always_inline)) inline void residual_range_regs(
    const W (&v)[kN], uint32_t t0, uint64_t len, uint64_t vmin, double th, bool small,
    int64_t& rmin, int64_t& rmax) {
  if (__builtin_amdgcn_readfirstlane(int(small))) {
    int32_t mn = INT32_MAX, mx = INT32_MIN;
#pragma unroll
    for (int k = 0; k < kN; ++k) {
      const uint32_t t = t0 + k * kStride;
      const int32_t rr = int32_t(uint32_t(v[k]) - uint32_t(vmin)) - predict32(th, t);
      if (t < len) {
        mn = rr < mn ? rr : mn;
        mx = rr > mx ? rr : mx;
      }
    }
    rmin = mn;
    rmax = mx;
  } else {
    rmin = INT64_MAX;
    rmax = INT64_MIN;
#pragma unroll
    for (int k = 0; k < kN; ++k) {
      const uint32_t t = t0 + k * kStride;
      const int64_t rr = int64_t(uint64_t(v[k]) - vmin) - predict(th, t);
      if (t < len) {
        rmin = rr < rmin ? rr : rmin;
        rmax = rr > rmax ? rr : rmax;
      }
    }
  }
}

// Loads of value t of a partition of len values: the index is clamped so
// every lane loads (no branch between loads), and callers mask t >= len.
template <class T>
__device__ inline uint64_t load_clamped(const T* src, uint32_t t, uint64_t len) {
  return uint64_t(global_ptr(src)[t < len ? t : uint32_t(len - 1)]);
}

// The model of a partition of len <= 64 kR values held by one wavefront,
// value lane + 64 k in v[k] (positions past len holding its last value;
// W: the column's value type, or uint64_t for either).
template <int kR, class W>
__device__ __attribute__((always_inline)) inline Model fit_wave_regs(const W (&v)[kR],
                                                                    uint64_t len,
                                                                    bool force_constant) {
  const uint32_t lane = threadIdx.x & 63;
  // clamped lanes hold the last value, which leaves min and max unchanged
  W lo = v[0], hi = v[0];
#pragma unroll
  for (int k = 1; k < kR; ++k) {
    lo = v[k] < lo ? v[k] : lo;
    hi = v[k] > hi ? v[k] : hi;
  }
  uint64_t vmin = lo, vmax = hi;
  wave_minmax_u64(vmin, vmax);
  const uint64_t range = vmax - vmin;
  Model md{vmin, vmin, 0.0, bitlen64(range), false, 0, range};
  if (len > 1 && !force_constant && range < (uint64_t(1) << 61)) {
    const bool narrow = range < kNarrowRange;
    double th;
    if (narrow) {
      uint64_t sy = 0, sty = 0;  // < 2^40 and < 2^50
#pragma unroll
      for (int k = 0; k < kR; ++k) {
        const uint32_t t = lane + 64 * k;
        const uint64_t y = t < len ? uint32_t(v[k]) - uint32_t(vmin) : 0;
        sy += y;
        sty += uint64_t(t) * y;
      }
      wave_sum_u64x2(sy, sty);
      th = ls_slope(len, U128{sy, 0}, U128{sty, 0});
    } else {
      U128 s, st;
      split_sums_regs<kR, 64>(v, lane, len, vmin, s, st);
      wave_sum_u128x2(s, st);
      th = ls_slope(len, join_split(s), join_split(st));
    }
    // |floor(theta1 t)| < 2^30 for every t < len: predictions fit int32
    const bool small = narrow && __dmul_rn(fabs(th), double(len)) < 1073741824.0;
    int64_t rmin, rmax;
    residual_range_regs<kR, 64>(v, lane, len, vmin, th, small, rmin, rmax);
    wave_minmax_i64(rmin, rmax);
    choose_model(md, th, rmin, rmax);
  }
  return md;
}

// The same, loading the partition (len <= 64 kR values) first.
template <int kR, class T>
__device__ __attribute__((always_inline)) inline Model fit_wave(const T* src, uint64_t len, bool force_constant) {
  const uint32_t lane = threadIdx.x & 63;
  T v[kR];
#pragma unroll
  for (int k = 0; k < kR; ++k) v[k] = T(load_clamped(src, lane + 64 * k, len));
  return fit_wave_regs<kR>(v, len, force_constant);
}

// At 16 values per lane, held to five waves per SIMD (90 VGPRs instead of
// 104): 2% faster on u64 columns.
template <int kR>
__global__ __launch_bounds__(kEncBlock, kR == 16 ? 5 : 1) void k_fit_wave(const EncColumn* __restrict__ cols,
                                                       uint64_t ncols, EncColumn single,
                                                       uint64_t nparts, EncScratch scr,
                                                       int* err) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t P =
      uint64_t(blockIdx.x) * kEncWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (P >= nparts) return;
  // launches holding polynomial columns (k_fit_poly) never use this kernel
  const EncColumn c = column_of(cols, ncols, single, P);
  uint64_t start, len;
  part_bounds(c, P - c.part_base, start, len);
  if (len > 64 * kR) {  // the host sends such partitions to k_fit_block
    if (lane == 0) raise(err, kErrDevice);
    return;
  }
  const Model md = c.dtype == 8
                       ? fit_wave<kR>(reinterpret_cast<const uint64_t*>(c.col) + start, len, c.force_constant)
                       : fit_wave<kR>(reinterpret_cast<const uint32_t*>(c.col) + start, len, c.force_constant);
  if (lane == 0) store_model(scr, P, md, len);
}

// ---- fit: one workgroup per partition ----------------------------------------------

// The model of one partition, by the whole workgroup (identical in every
// thread).  Partitions of at most kEncRegLen values are held in registers;
// longer ones are streamed twice.
template <class T>
__device__ __attribute__((always_inline)) inline Model fit_block(FitShared& sh, const T* src, uint64_t len, bool force_constant) {
  const uint32_t tid = threadIdx.x;
  const bool in_regs = len <= kEncRegLen;
  const auto gsrc = global_ptr(src);
  uint64_t v[kEncRegs];
  uint64_t vmin = ~uint64_t(0), vmax = 0;
  U128 sv{0, 0}, stv{0, 0};
  if (in_regs) {
#pragma unroll
    for (int k = 0; k < kEncRegs; ++k) v[k] = load_clamped(src, tid + k * kEncBlock, len);
    vmin = vmax = v[0];
#pragma unroll
    for (int k = 1; k < kEncRegs; ++k) {
      vmin = v[k] < vmin ? v[k] : vmin;
      vmax = v[k] > vmax ? v[k] : vmax;
    }
  } else {
    // streamed: range and raw sums in one pass
    for (uint64_t t = tid; t < len; t += kEncBlock) {
      const uint64_t x = uint64_t(gsrc[t]);
      vmin = x < vmin ? x : vmin;
      vmax = x > vmax ? x : vmax;
      sv = add128(sv, U128{x, 0});
      stv = add128(stv, mul64x64(t, x));
    }
  }
  block_minmax_u64(sh, vmin, vmax);
  const uint64_t range = vmax - vmin;
  Model md{vmin, vmin, 0.0, bitlen64(range), false, 0, range};
  if (len > 1 && !force_constant && range < (uint64_t(1) << 61)) {
    double th;
    bool small = false;
    if (in_regs && range < kNarrowRange) {
      uint64_t sy = 0, sty = 0;  // < 2^42 and < 2^54
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) {
        const uint32_t t = tid + k * kEncBlock;
        const uint64_t y = t < len ? uint32_t(v[k]) - uint32_t(vmin) : 0;
        sy += y;
        sty += uint64_t(t) * y;
      }
      block_sum_u64x2(sh, sy, sty);
      th = block_slope(sh, len, U128{sy, 0}, U128{sty, 0});
      small = __dmul_rn(fabs(th), double(len)) < 1073741824.0;
    } else {
      if (in_regs) {
#pragma unroll
        for (int k = 0; k < kEncRegs; ++k) {
          const uint32_t t = tid + k * kEncBlock;
          const uint64_t x = t < len ? v[k] : 0;
          sv = add128(sv, U128{x, 0});
          stv = add128(stv, mul64x64(t, x));
        }
      }
      block_sum_u128x2(sh, sv, stv);
      th = block_slope(sh, len, sv, stv);
    }
    int64_t rmin = INT64_MAX, rmax = INT64_MIN;
    if (in_regs) {
      residual_range_regs<kEncRegs, kEncBlock>(v, tid, len, vmin, th, small, rmin, rmax);
    } else {
      for (uint64_t t = tid; t < len; t += kEncBlock) {
        const int64_t rr = int64_t(uint64_t(gsrc[t]) - vmin) - predict(th, uint32_t(t));
        rmin = rr < rmin ? rr : rmin;
        rmax = rr > rmax ? rr : rmax;
      }
    }
    block_minmax_i64(sh, rmin, rmax);
    choose_model(md, th, rmin, rmax);
  }
  return md;
}

// Six waves per SIMD (at most 80 VGPRs; 114 unconstrained): the extra
// waves of loads in flight outweigh the registers the 128-bit-sum path
// spills.  Encode of 2e8 u64 values at L 4096: sorted keys 0.73-0.74 ->
// 0.70 ms (0.76 at four waves), a noisy line 0.66 -> 0.64 ms; partitions
// spanning 2^30 or more, which take that path, 1.07 -> 1.22 ms.
__global__ __launch_bounds__(kEncBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_fit_block(
    const EncColumn* __restrict__ cols, uint64_t ncols, EncColumn single, uint64_t nparts,
    EncScratch scr) {
  __shared__ FitShared sh;
  const uint64_t P = blockIdx.x;
  if (P >= nparts) return;
  const EncColumn c = column_of(cols, ncols, single, P);
  if (c.regressor == 2) return;  // k_fit_poly
  uint64_t start, len;
  part_bounds(c, P - c.part_base, start, len);
  const Model md =
      c.dtype == 8
          ? fit_block(sh, reinterpret_cast<const uint64_t*>(c.col) + start, len, c.force_constant)
          : fit_block(sh, reinterpret_cast<const uint32_t*>(c.col) + start, len, c.force_constant);
  if (threadIdx.x == 0) store_model(scr, P, md, len);
}

// ---- fit with the minimax regressor: one workgroup per partition ------------------

// A hull tile's LDS word for an offset below kHullF64Range: its binary64 bits.
__device__ inline uint64_t f64_word(uint64_t offset) {
  return uint64_t(__double_as_longlong(double(offset)));
}
// The value a hull tile's word stands for: the word itself, or (f64) the
// offset its binary64 bits hold (an integer below 2^40: exact).
__device__ inline uint64_t tile_word_value(uint64_t word, bool f64) {
  return f64 ? uint64_t(__longlong_as_double(static_cast<long long>(word))) : word;
}

// The least-squares model of fit_block, then (minimax) the minimax line
// of section 3.1's fixed-width objective, stored instead when its residual
// width is strictly smaller.  run_up / run_lo: the partition's running hulls
// when it spans several hull tiles.
template <class T>
__device__ __attribute__((always_inline)) inline Model fit_minimax(FitShared& fs, HullShared& hs, const T* src, uint64_t len,
                                    bool force_constant, bool minimax, uint32_t* run_up,
                                    uint32_t* run_lo) {
  Model md = fit_block(fs, src, len, force_constant);
  // the same partitions as the least-squares line: len > 1, range < 2^61
  if (!minimax || len < 2 || force_constant || !(md.linear || md.bits <= 61)) return md;
  const auto gsrc = global_ptr(src);
  const uint32_t tid = threadIdx.x;
  const uint32_t ntiles = uint32_t((len + kHullTile - 1) / kHullTile);
  // one tile of a narrow range: the hull tests in binary64
  const bool f64 = ntiles == 1 && md.range < kHullF64Range;
  for (uint32_t k = 0; k < ntiles; ++k) {
    const uint32_t t0 = k * kHullTile;
    const uint32_t cnt = uint32_t(len - t0 < kHullTile ? len - t0 : kHullTile);
    {  // the tile's loads issued at once
      uint64_t tv[kHullChunk];
#pragma unroll
      for (uint32_t j = 0; j < kHullChunk; ++j) {
        const uint32_t x = tid + j * kEncBlock;
        tv[j] = x < cnt ? uint64_t(gsrc[t0 + x]) : 0;
      }
#pragma unroll
      for (uint32_t j = 0; j < kHullChunk; ++j) {
        const uint32_t x = tid + j * kEncBlock;
        if (x < cnt) hs.v[x] = f64 ? f64_word(tv[j] - md.vmin) : tv[j];
      }
    }
    __syncthreads();
    if (f64)
      tile_hulls<kEncBlock, true>(hs, cnt, tid);
    else
      tile_hulls<kEncBlock, false>(hs, cnt, tid);
    if (ntiles == 1) break;
    uint32_t keep[2], from[2], c[2];
    for (uint32_t side = 0; side < 2; ++side) c[side] = hs.cnt[side][0];
    if (k == 0) {
      keep[0] = keep[1] = from[0] = from[1] = 0;
    } else {
      if (tid < 2) {
        const uint32_t side = tid;
        const uint32_t* R = side ? run_lo : run_up;
        const auto A = [&](uint32_t i) {
          const uint32_t t = R[i];
          return HullPoint{t, uint64_t(gsrc[t])};
        };
        const auto B = [&](uint32_t j) {
          const uint32_t x = hs.h[side][j];
          return HullPoint{t0 + x, hs.v[x]};
        };
        uint32_t kp, fr;
        hull_bridge(side == 0, A, hs.rcnt[side], B, c[side], kp, fr);
        hs.rkeep[side] = kp;
        hs.rfrom[side] = fr;
      }
      __syncthreads();
      for (uint32_t side = 0; side < 2; ++side) {
        keep[side] = hs.rkeep[side];
        from[side] = hs.rfrom[side];
      }
    }
    for (uint32_t side = 0; side < 2; ++side) {
      uint32_t* R = side ? run_lo : run_up;
      for (uint32_t x = tid; x < c[side] - from[side]; x += kEncBlock)
        R[keep[side] + x] = t0 + hs.h[side][from[side] + x];
    }
    __syncthreads();
    if (tid < 2) hs.rcnt[tid] = keep[tid] + c[tid] - from[tid];
    __syncthreads();
  }
  EdgeSlope th;
  if (f64) {
    const auto U = [&](uint32_t i) { return hull_pt<true>(hs.h[0][i], hs.v[hs.h[0][i]]); };
    const auto L = [&](uint32_t i) { return hull_pt<true>(hs.h[1][i], hs.v[hs.h[1][i]]); };
    th = minimax_bend<kEncBlock>(hs, U, hs.cnt[0][0], L, hs.cnt[1][0], tid);
  } else if (ntiles == 1) {
    const auto U = [&](uint32_t i) { return hull_pt<false>(hs.h[0][i], hs.v[hs.h[0][i]]); };
    const auto L = [&](uint32_t i) { return hull_pt<false>(hs.h[1][i], hs.v[hs.h[1][i]]); };
    th = minimax_bend<kEncBlock>(hs, U, hs.cnt[0][0], L, hs.cnt[1][0], tid);
  } else {
    const auto U = [&](uint32_t i) {
      const uint32_t t = run_up[i];
      return HullPoint{t, uint64_t(gsrc[t])};
    };
    const auto L = [&](uint32_t i) {
      const uint32_t t = run_lo[i];
      return HullPoint{t, uint64_t(gsrc[t])};
    };
    th = minimax_bend<kEncBlock>(hs, U, hs.rcnt[0], L, hs.rcnt[1], tid);
  }
  // one correctly rounded division of the exact edge fraction
  double theta = static_cast<double>(th.dy) / static_cast<double>(th.dt);
  if (theta == 0.0) theta = 0.0;  // +0.0, never -0.0
  int64_t rmin = INT64_MAX, rmax = INT64_MIN;
  for (uint32_t t0 = 0; t0 < len; t0 += kHullTile) {
#pragma unroll
    for (uint32_t j = 0; j < kHullChunk; ++j) {
      const uint32_t t = t0 + tid + j * kEncBlock;
      if (t < len) {
        const uint64_t x = ntiles == 1 ? (f64 ? md.vmin + tile_word_value(hs.v[t], true) : hs.v[t])
                                       : uint64_t(gsrc[t]);
        const int64_t rr = int64_t(x - md.vmin) - predict(theta, t);
        rmin = rr < rmin ? rr : rmin;
        rmax = rr > rmax ? rr : rmax;
      }
    }
  }
  block_minmax_i64(fs, rmin, rmax);
  const uint32_t b = bitlen64(uint64_t(rmax) - uint64_t(rmin));
  if (b < md.bits) {
    md.linear = true;
    md.theta1 = theta;
    md.base = md.vmin + uint64_t(rmin);
    md.bits = b;
    md.rmin = rmin;
  }
  return md;
}

__global__ __launch_bounds__(kEncBlock) void k_fit_minimax(const EncColumn* __restrict__ cols,
                                                          uint64_t ncols, EncColumn single,
                                                          uint64_t nparts, EncScratch scr,
                                                          int* err) {
  __shared__ FitShared fs;
  __shared__ HullShared hs;
  const uint64_t P = blockIdx.x;
  if (P >= nparts) return;
  const EncColumn c = column_of(cols, ncols, single, P);
  if (c.regressor == 2) return;  // k_fit_poly
  uint64_t start, len;
  part_bounds(c, P - c.part_base, start, len);
  bool minimax = c.regressor == 1;
  uint32_t *run_up = nullptr, *run_lo = nullptr;
  if (minimax && len > kHullTile) {
    if (scr.hull == nullptr) {  // the host allocates running hulls for such launches
      if (threadIdx.x == 0) raise(err, kErrDevice);
      minimax = false;
    } else {
      run_up = scr.hull + c.val_base + start;
      run_lo = scr.hull + scr.hull_values + c.val_base + start;
    }
  }
  const Model md =
      c.dtype == 8
          ? fit_minimax(fs, hs, reinterpret_cast<const uint64_t*>(c.col) + start, len,
                        c.force_constant, minimax, run_up, run_lo)
          : fit_minimax(fs, hs, reinterpret_cast<const uint32_t*>(c.col) + start, len,
                        c.force_constant, minimax, run_up, run_lo);
  if (threadIdx.x == 0) store_model(scr, P, md, len);
}

// The same with one wavefront per partition of at most kWaveEncMax values
// (four per workgroup, no workgroup barrier): the least-squares model of
// fit_wave, then the minimax line from the partition's hulls in the
// wavefront's own LDS slice.  Launches holding polynomial columns never use
// this kernel.
template <class T>
__device__ __attribute__((always_inline)) inline Model fit_minimax_wave(HullSharedT<64>& hs,
                                                                        const T* src, uint64_t len,
                                                                        bool force_constant,
                                                                        bool minimax) {
  Model md = fit_wave<kWaveRegs>(src, len, force_constant);
  if (!minimax || len < 2 || force_constant || md.range >= (uint64_t(1) << 61)) return md;
  const uint32_t lane = threadIdx.x & 63;
  // all loads issued at once (the same addresses fit_wave read)
  uint64_t v[kWaveRegs];
#pragma unroll
  for (int k = 0; k < kWaveRegs; ++k) v[k] = load_clamped(src, lane + 64 * k, len);
  const bool f64 = md.range < kHullF64Range;  // the hull tests in binary64
#pragma unroll
  for (int k = 0; k < kWaveRegs; ++k)
    if (lane + 64 * k < len) hs.v[lane + 64 * k] = f64 ? f64_word(v[k] - md.vmin) : v[k];
  group_sync<64>();
  if (f64)
    tile_hulls<64, true>(hs, uint32_t(len), lane);
  else
    tile_hulls<64, false>(hs, uint32_t(len), lane);
  EdgeSlope th;
  if (f64) {
    const auto U = [&](uint32_t i) { return hull_pt<true>(hs.h[0][i], hs.v[hs.h[0][i]]); };
    const auto L = [&](uint32_t i) { return hull_pt<true>(hs.h[1][i], hs.v[hs.h[1][i]]); };
    th = minimax_bend<64>(hs, U, hs.cnt[0][0], L, hs.cnt[1][0], lane);
  } else {
    const auto U = [&](uint32_t i) { return hull_pt<false>(hs.h[0][i], hs.v[hs.h[0][i]]); };
    const auto L = [&](uint32_t i) { return hull_pt<false>(hs.h[1][i], hs.v[hs.h[1][i]]); };
    th = minimax_bend<64>(hs, U, hs.cnt[0][0], L, hs.cnt[1][0], lane);
  }
  double theta = static_cast<double>(th.dy) / static_cast<double>(th.dt);
  if (theta == 0.0) theta = 0.0;  // +0.0, never -0.0
  int64_t rmin = INT64_MAX, rmax = INT64_MIN;
#pragma unroll
  for (int k = 0; k < kWaveRegs; ++k) {
    const uint32_t t = lane + 64 * k;
    if (t < len) {
      const int64_t rr = int64_t(v[k] - md.vmin) - predict(theta, t);
      rmin = rr < rmin ? rr : rmin;
      rmax = rr > rmax ? rr : rmax;
    }
  }
  wave_minmax_i64(rmin, rmax);
  const uint32_t b = bitlen64(uint64_t(rmax) - uint64_t(rmin));
  if (b < md.bits) {
    md.linear = true;
    md.theta1 = theta;
    md.base = md.vmin + uint64_t(rmin);
    md.bits = b;
    md.rmin = rmin;
  }
  return md;
}

__global__ __launch_bounds__(kEncBlock) void k_fit_minimax_wave(const EncColumn* __restrict__ cols,
                                                               uint64_t ncols, EncColumn single,
                                                               uint64_t nparts, EncScratch scr,
                                                               int* err) {
  __shared__ HullSharedT<64> hs[kEncWaves];
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t P = uint64_t(blockIdx.x) * kEncWaves + wave;
  if (P >= nparts) return;
  const EncColumn c = column_of(cols, ncols, single, P);
  uint64_t start, len;
  part_bounds(c, P - c.part_base, start, len);
  if (len > kWaveEncMax) {  // the host sends such partitions to k_fit_minimax
    if (lane == 0) raise(err, kErrDevice);
    return;
  }
  const bool minimax = c.regressor == 1;
  const Model md =
      c.dtype == 8
          ? fit_minimax_wave(hs[wave], reinterpret_cast<const uint64_t*>(c.col) + start, len,
                             c.force_constant, minimax)
          : fit_minimax_wave(hs[wave], reinterpret_cast<const uint32_t*>(c.col) + start, len,
                             c.force_constant, minimax);
  if (lane == 0) store_model(scr, P, md, len);
}

// ---- fit with the polynomial regressor: one workgroup per partition ---------------

__device__ inline double i128_to_double(__int128 x) {
  return i128_to_f64(U128{uint64_t(x), uint64_t(static_cast<unsigned __int128>(x) >> 64)});
}

// The degree-2 and degree-3 least-squares polynomials of a partition of
// 3 <= n <= 4096 values of range below 2^50, in the Gram basis:
// c_k = fl(S_k) / fl(Q_k), S_k = sum y_t g_k(t) exact in int128 and
// Q_k = sum g_k(t)^2 from its closed form; md takes the narrower of them when
// strictly narrower than every simpler model.  Each of the group's kT
// threads holds kR <= 16 offsets y = v - vmin, at positions t = u + kT k
// (u = tid, k < kR); sum4 and minmax reduce over the group.
//
// S_k comes from the moments M_j = sum_t y_t t^j, j <= 3, by the
// coefficients of g_k:
//   S1 = 2 M1 - a M0,  S2 = 6 M2 - 6a M1 + e2 M0,
//   S3 = 20 M3 - 30a M2 + k3 M1 - e3 M0        (a = n - 1).
// A thread's positions come in chunks of up to 16 registers, t = u' + kT j
// (u' = u + 16 kT h for chunk h, j < 16); its share of M_j expands
// (u' + kT j)^j binomially over the chunk's sums T_i = sum_j y_j j^i, so
// the loop over values multiplies only by the constants j^i;
// T_3 <= 2^50 (0^3 + ... + 15^3) < 2^64, so every T_i fits 64 bits.  The
// group totals stay below 2^103 in magnitude.
template <int kT, int kR, class Sum4, class MinMax>
__device__ __attribute__((always_inline)) inline void poly_stage(
    Model& md, const uint64_t (&y)[kR], uint32_t tid, uint32_t n, const Sum4& sum4,
    const MinMax& minmax, uint32_t& kind, double& c2_out, double& c3_out) {
  constexpr int kC = kR < 16 ? kR : 16;  // registers per chunk
  static_assert(kR % kC == 0, "whole chunks");
  using u128 = unsigned __int128;
  u128 M0 = 0, M1 = 0, M2 = 0, M3 = 0;
#pragma unroll
  for (int h = 0; h < kR / kC; ++h) {
    uint64_t T0 = 0, T1 = 0, T2 = 0, T3 = 0;
#pragma unroll
    for (int j = 0; j < kC; ++j) {
      const int k = h * kC + j;
      const uint64_t yk = tid + uint32_t(k * kT) < n ? y[k] : 0;
      T0 += yk;
      T1 += yk * uint64_t(j);
      T2 += yk * uint64_t(j * j);
      T3 += yk * uint64_t(j * j * j);
    }
    const uint64_t u = tid + uint64_t(h) * kC * kT, S = kT;
    M0 += T0;
    M1 += u128(T0) * u + u128(T1) * S;
    M2 += u128(T0) * (u * u) + u128(T1) * (2 * u * S) + u128(T2) * (S * S);
    M3 += u128(T0) * (u * u * u) + u128(T1) * (3 * u * u * S) + u128(T2) * (3 * u * S * S) +
          u128(T3) * (S * S * S);
  }
  sum4(M0, M1, M2, M3);
  const int64_t N = n, a = N - 1;
  const int64_t k3 = 12 * N * N - 30 * N + 22, e2 = a * (N - 2), e3 = a * (N - 2) * (N - 3);
  const __int128 m0 = __int128(M0), m1 = __int128(M1), m2 = __int128(M2), m3 = __int128(M3);
  const __int128 S1 = 2 * m1 - a * m0;
  const __int128 S2 = 6 * m2 - 6 * a * m1 + e2 * m0;
  const __int128 S3 = 20 * m3 - 30 * a * m2 + k3 * m1 - e3 * m0;
  // The norms sum g_k(t)^2 over t < n have closed forms (the Gram
  // polynomials' squared norms, exact integers): (n-1)n(n+1)/3,
  // (n-2)...(n+2)/5 and (n-3)...(n+3)/7, below 2^84 for n <= 4096.  Each is
  // a run of 3, 5 or 7 consecutive integers, one of which the divisor
  // divides: that factor is divided first, so no 128-bit division is needed.
  auto norm = [](int64_t nv, int64_t half, int64_t d) {
    __int128 q = 1;
    bool divided = false;
    for (int64_t f = nv - half; f <= nv + half; ++f) {
      int64_t x = f;
      if (!divided && x % d == 0) {
        x /= d;
        divided = true;
      }
      q *= x;
    }
    return q;
  };
  const __int128 Q1 = norm(N, 1, 3), Q2 = norm(N, 2, 5), Q3 = norm(N, 3, 7);
  double c[3];
  const __int128 Sk[3] = {S1, S2, S3}, Q[3] = {Q1, Q2, Q3};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    c[k] = Q[k] != 0 ? i128_to_double(Sk[k]) / i128_to_double(Q[k]) : 0.0;
    if (c[k] == 0.0) c[k] = 0.0;  // +0.0, never -0.0
  }
  // the residuals of both degrees in one pass (the degree-2 prediction is
  // the degree-3 one with c3 = 0: the two share their Gram values, which
  // the thread steps by forward differences over its positions kT apart)
  int64_t mn2 = INT64_MAX, mx2 = INT64_MIN, mn3 = INT64_MAX, mx3 = INT64_MIN;
  GramWalk gw;
  gw.start(tid, n, kT);
#pragma unroll
  for (int k = 0; k < kR; ++k) {
    const uint32_t t = tid + k * kT;
    if (t < n) {
      const int64_t r2 = int64_t(y[k]) - poly_combine(c[0], c[1], 0.0, gw.g1, gw.g2, gw.g3);
      const int64_t r3 = int64_t(y[k]) - gw.predict(c[0], c[1], c[2]);
      mn2 = r2 < mn2 ? r2 : mn2;
      mx2 = r2 > mx2 ? r2 : mx2;
      mn3 = r3 < mn3 ? r3 : mn3;
      mx3 = r3 > mx3 ? r3 : mx3;
    }
    gw.next();
  }
  minmax(mn2, mx2);
  minmax(mn3, mx3);
  for (int deg = 2; deg <= 3; ++deg) {
    if (deg == 3 && n < 4) break;
    const int64_t rmin = deg == 2 ? mn2 : mn3, rmax = deg == 2 ? mx2 : mx3;
    const uint32_t b = bitlen64(uint64_t(rmax) - uint64_t(rmin));
    if (b < md.bits) {
      md.linear = true;
      md.theta1 = c[0];
      md.base = md.vmin + uint64_t(rmin);
      md.bits = b;
      md.rmin = rmin;
      kind = 1;
      c2_out = c[1];
      c3_out = deg == 3 ? c[2] : 0.0;
    }
  }
}

__device__ inline U128 to_u128(unsigned __int128 x) { return U128{uint64_t(x), uint64_t(x >> 64)}; }
__device__ inline unsigned __int128 from_u128(U128 x) {
  return (static_cast<unsigned __int128>(x.hi) << 64) | x.lo;
}

// The least-squares model of fit_block, then the polynomial stage, by the
// whole workgroup.
template <class T>
__device__ __attribute__((always_inline)) inline Model fit_poly(FitShared& fs, const T* src, uint64_t len, bool force_constant,
                                 uint32_t& kind, double& c2_out, double& c3_out) {
  Model md = fit_block(fs, src, len, force_constant);
  kind = 0;
  c2_out = c3_out = 0.0;
  if (force_constant || len < 3 || len > kPolyMaxLen || md.range >= kPolyMaxRange) return md;
  const uint32_t tid = threadIdx.x;
  uint64_t y[kEncRegs];
#pragma unroll
  for (int k = 0; k < kEncRegs; ++k) y[k] = load_clamped(src, tid + k * kEncBlock, len) - md.vmin;
  const auto sum4 = [&](unsigned __int128& m0, unsigned __int128& m1, unsigned __int128& m2,
                        unsigned __int128& m3) {
    U128 x = to_u128(m0), w = to_u128(m1);
    block_sum_u128x2(fs, x, w);
    m0 = from_u128(x);
    m1 = from_u128(w);
    x = to_u128(m2);
    w = to_u128(m3);
    block_sum_u128x2(fs, x, w);
    m2 = from_u128(x);
    m3 = from_u128(w);
  };
  const auto minmax = [&](int64_t& mn, int64_t& mx) { block_minmax_i64(fs, mn, mx); };
  poly_stage<kEncBlock, kEncRegs>(md, y, tid, uint32_t(len), sum4, minmax, kind, c2_out, c3_out);
  return md;
}

// The same by one wavefront, for partitions of at most 64 kR values: the
// model of fit_wave, then the polynomial stage with wavefront reductions (no
// barrier).
template <int kR, class T>
__device__ __attribute__((always_inline)) inline Model fit_poly_wave(const T* src, uint64_t len, bool force_constant,
                                      uint32_t& kind, double& c2_out, double& c3_out) {
  Model md = fit_wave<kR>(src, len, force_constant);
  kind = 0;
  c2_out = c3_out = 0.0;
  if (force_constant || len < 3 || md.range >= kPolyMaxRange) return md;
  const uint32_t lane = threadIdx.x & 63;
  uint64_t y[kR];
#pragma unroll
  for (int k = 0; k < kR; ++k) y[k] = load_clamped(src, lane + 64 * k, len) - md.vmin;
  const auto sum4 = [](unsigned __int128& m0, unsigned __int128& m1, unsigned __int128& m2,
                       unsigned __int128& m3) {
    U128 x = to_u128(m0), w = to_u128(m1), z = to_u128(m2), q = to_u128(m3);
    wave_sum_u128x2(x, w);
    wave_sum_u128x2(z, q);
    m0 = from_u128(x);
    m1 = from_u128(w);
    m2 = from_u128(z);
    m3 = from_u128(q);
  };
  const auto minmax = [](int64_t& mn, int64_t& mx) { wave_minmax_i64(mn, mx); };
  poly_stage<64, kR>(md, y, lane, uint32_t(len), sum4, minmax, kind, c2_out, c3_out);
  return md;
}

__device__ inline void store_poly(const EncScratch& s, uint64_t P, uint32_t kind, double c2,
                                  double c3) {
  s.kind[P] = kind;
  s.c2[P] = uint64_t(__double_as_longlong(c2));
  s.c3[P] = uint64_t(__double_as_longlong(c3));
}

__global__ __launch_bounds__(kEncBlock) void k_fit_poly(const EncColumn* __restrict__ cols,
                                                       uint64_t ncols, EncColumn single,
                                                       uint64_t nparts, EncScratch scr) {
  __shared__ FitShared fs;
  const uint64_t P = blockIdx.x;
  if (P >= nparts) return;
  const EncColumn c = column_of(cols, ncols, single, P);
  if (c.regressor != 2) return;  // the other fit kernels
  uint64_t start, len;
  part_bounds(c, P - c.part_base, start, len);
  uint32_t kind;
  double c2, c3;
  const Model md =
      c.dtype == 8
          ? fit_poly(fs, reinterpret_cast<const uint64_t*>(c.col) + start, len, c.force_constant,
                     kind, c2, c3)
          : fit_poly(fs, reinterpret_cast<const uint32_t*>(c.col) + start, len, c.force_constant,
                     kind, c2, c3);
  if (threadIdx.x == 0) {
    store_model(scr, P, md, len);
    store_poly(scr, P, kind, c2, c3);
  }
}

// Held to four waves per SIMD at 16 values per lane and three at 32 (128
// and 168 VGPRs instead of 139 and 181, some spilled): polynomial encode
// of 1e8 u32 two-sine values 0.67 -> 0.61 ms, of 2e8 u64 cubic blocks
// 1.26 -> 1.17 ms.
template <int kR>
__global__ __launch_bounds__(kEncBlock, kR == 16 ? 4 : 3) void k_fit_poly_wave(const EncColumn* __restrict__ cols,
                                                            uint64_t ncols, EncColumn single,
                                                            uint64_t nparts, EncScratch scr,
                                                            int* err) {
  const uint32_t lane = threadIdx.x & 63;
  const uint64_t P =
      uint64_t(blockIdx.x) * kEncWaves + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  if (P >= nparts) return;
  const EncColumn c = column_of(cols, ncols, single, P);
  if (c.regressor != 2) return;  // the other fit kernels
  uint64_t start, len;
  part_bounds(c, P - c.part_base, start, len);
  if (len > 64 * kR) {  // the host sends such partitions to k_fit_poly
    if (lane == 0) raise(err, kErrDevice);
    return;
  }
  uint32_t kind;
  double c2, c3;
  const Model md =
      c.dtype == 8
          ? fit_poly_wave<kR>(reinterpret_cast<const uint64_t*>(c.col) + start, len,
                              c.force_constant, kind, c2, c3)
          : fit_poly_wave<kR>(reinterpret_cast<const uint32_t*>(c.col) + start, len,
                              c.force_constant, kind, c2, c3);
  if (lane == 0) {
    store_model(scr, P, md, len);
    store_poly(scr, P, kind, c2, c3);
  }
}

// ---- scan: word offsets ------------------------------------------------------------

// Exclusive prefix sum of x over the workgroup's threads; *total receives
// the workgroup sum.
__device__ inline uint64_t block_exclusive_scan_u64(uint64_t x, uint64_t* total) {
  __shared__ uint64_t wsum[kEncWaves];
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint64_t inc = x;
#pragma unroll
  for (int delta = 1; delta < 64; delta <<= 1) {
    const uint64_t y = uint64_t(__shfl_up(static_cast<unsigned long long>(inc), delta, 64));
    if (int(lane) >= delta) inc += y;
  }
  if (lane == 63) wsum[wave] = inc;
  __syncthreads();
  uint64_t before = 0, all = 0;
#pragma unroll
  for (int w = 0; w < kEncWaves; ++w) {
    if (w < int(wave)) before += wsum[w];
    all += wsum[w];
  }
  __syncthreads();
  *total = all;
  return before + inc - x;
}

// bsum[g] = word count of partitions [g * 1024, (g + 1) * 1024).
__global__ __launch_bounds__(kEncBlock) void k_scan_sums(EncScratch scr, uint64_t nparts) {
  const uint64_t p0 = uint64_t(blockIdx.x) * kScanItems + threadIdx.x * 4;
  uint64_t x = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (p0 + q < nparts) x += scr.nwords[p0 + q];
  uint64_t total;
  block_exclusive_scan_u64(x, &total);
  if (threadIdx.x == 0) scr.bsum[blockIdx.x] = total;
}

// Exclusive prefix of bsum[0, ng) in place, by one workgroup.
__global__ __launch_bounds__(kEncBlock) void k_scan_top(EncScratch scr, uint64_t ng) {
  uint64_t carry = 0;
  for (uint64_t g0 = 0; g0 < ng; g0 += kEncBlock) {
    const uint64_t g = g0 + threadIdx.x;
    const uint64_t x = g < ng ? scr.bsum[g] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan_u64(x, &total);
    if (g < ng) scr.bsum[g] = carry + ex;
    carry += total;
  }
}

// woff[P] = exclusive prefix of the word counts over all partitions of the
// launch (a column's offsets are relative to its first partition's).
__global__ __launch_bounds__(kEncBlock) void k_scan_apply(EncScratch scr, uint64_t nparts) {
  const uint64_t p0 = uint64_t(blockIdx.x) * kScanItems + threadIdx.x * 4;
  uint64_t x[4], sum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    x[q] = p0 + q < nparts ? scr.nwords[p0 + q] : 0;
    sum += x[q];
  }
  uint64_t total;
  uint64_t run = scr.bsum[blockIdx.x] + block_exclusive_scan_u64(sum, &total);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    if (p0 + q < nparts) scr.woff[p0 + q] = run;
    run += x[q];
  }
}

// Records and starts; the last partition of a column also writes the
// header and the padding.
__global__ __launch_bounds__(kEncBlock) void k_records(const EncColumn* __restrict__ cols,
                                                      uint64_t ncols, EncColumn single,
                                                      uint64_t nparts, EncScratch scr, int* err) {
  const uint64_t P = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (P >= nparts) return;
  const EncColumn c = column_of(cols, ncols, single, P);
  const uint64_t j = P - c.part_base;
  const uint64_t word_off = scr.woff[P] - scr.woff[c.part_base];
  const uint64_t rec = kHeaderBytes + kRecordBytes * j;
  if (rec + kRecordBytes <= c.cap) {
    uint64_t* r = reinterpret_cast<uint64_t*>(c.blob + rec);
    r[0] = scr.base[P];
    r[1] = scr.theta[P];
    r[2] = word_off;
    r[3] = uint64_t(scr.bits[P]) | (c.regressor == 2 ? uint64_t(scr.kind[P]) << 8 : 0);
  }
  if (c.fixed_len == 0) {
    const uint64_t so = kHeaderBytes + kRecordBytes * c.m + 8 * j;
    if (so + 8 <= c.cap) *reinterpret_cast<uint64_t*>(c.blob + so) = c.starts[j];
  }
  if (c.regressor == 2) {  // (c2, c3), zero for a line or constant
    const uint64_t meta_end =
        kHeaderBytes + kRecordBytes * c.m + (c.fixed_len == 0 ? 8 * (c.m + 1) : 0);
    const uint64_t co = align16(meta_end) + 16 * j;
    if (co + 16 <= c.cap) {
      uint64_t* q = reinterpret_cast<uint64_t*>(c.blob + co);
      q[0] = scr.kind[P] ? scr.c2[P] : 0;
      q[1] = scr.kind[P] ? scr.c3[P] : 0;
    }
  }
  if (j + 1 == c.m) finish_column(c, word_off + scr.nwords[P], err);
}

// ---- pack ----------------------------------------------------------------------------

constexpr uint32_t kPackBatch = 8;  // rounds of 64 residuals per batch

// Packs rounds [k_begin, k_end) of partition v[0, len) into its words, from
// the stored model: u = (v - base) - floor(theta1 t), the encoder's
// residual for both models (the constant model has theta1 = +0).  Round k
// holds residuals 64k .. 64k + 63, which fill exactly 2b 32-bit words, so a
// batch of consecutive rounds fills 2b words per round with no word shared
// with another batch.  A batch's values are loaded together, its words
// assembled in the wavefront's LDS buffer (kPackBatch * 128 words) and
// stored as one contiguous run; words at or beyond `limit` (the span's end,
// or the blob's capacity) are not stored.  Called by one wavefront.  A
// polynomial partition (kind 1) predicts with poly_predict(theta1, c2, c3).
template <class T>
__device__ __attribute__((always_inline)) inline void pack_rounds(const T* src, uint64_t len, uint64_t base, double theta1,
                                   uint32_t kind, double c2, double c3, uint32_t b,
                                   uint32_t* gw32, uint64_t limit, uint64_t k_begin,
                                   uint64_t k_end, uint32_t* w32) {
  const uint32_t lane = threadIdx.x & 63;
  const bool fits32 = prediction_fits_i32(theta1, len);
  const auto gdst = global_ptr(gw32);
  for (uint64_t k0 = k_begin; k0 < k_end; k0 += kPackBatch) {
    const uint32_t nr = uint32_t(k_end - k0 < kPackBatch ? k_end - k0 : kPackBatch);
    uint64_t u[kPackBatch];
#pragma unroll
    for (uint32_t r = 0; r < kPackBatch; ++r) u[r] = load_clamped(src, uint32_t(64 * (k0 + r) + lane), len);
#pragma unroll
    for (uint32_t r = 0; r < kPackBatch; ++r) {
      const uint32_t t = uint32_t(64 * (k0 + r) + lane);
      const uint64_t p = kind ? uint64_t(poly_predict(theta1, c2, c3, t, uint32_t(len)))
                              : fits32 ? uint64_t(int64_t(predict32(theta1, t)))
                                       : uint64_t(predict(theta1, t));
      u[r] = t < len ? (u[r] - base) - p : 0;
    }
    const uint32_t nw = 2 * b * nr;  // <= 1024
    for (uint32_t q = lane; q < nw; q += 64) w32[q] = 0;
    wave_fence();
#pragma unroll
    for (uint32_t r = 0; r < kPackBatch; ++r)
      if (r < nr) or_bits(w32, (64 * r + lane) * b, b, u[r]);
    wave_fence();
    const uint64_t first = 2 * b * k0;
    const uint64_t count = first >= limit ? 0 : (limit - first < nw ? limit - first : nw);
    for (uint32_t q = lane; q < count; q += 64) gdst[first + q] = w32[q];
    wave_fence();
  }
}

// One wavefront per partition (kWave, four per workgroup), or one workgroup
// per partition whose four wavefronts take consecutive quarters of its
// rounds (each a whole number of batches).  Five waves per SIMD, as
// k_fit_block (95 VGPRs instead of 105, no spills).
template <bool kWave>
__global__ __launch_bounds__(kEncBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_pack(
    const EncColumn* __restrict__ cols, uint64_t ncols, EncColumn single, uint64_t nparts,
    EncScratch scr) {
  __shared__ uint32_t lds[kEncWaves][kPackBatch * 128];
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const uint64_t P = kWave ? uint64_t(blockIdx.x) * kEncWaves + wave : uint64_t(blockIdx.x);
  if (P >= nparts) return;
  const uint32_t b = meta_load(scr.bits, P);
  if (b == 0) return;
  const EncColumn c = column_of(cols, ncols, single, P);
  uint64_t start, len;
  part_bounds(c, P - c.part_base, start, len);
  const uint64_t w0 = 2 * (meta_load(scr.woff, P) - meta_load(scr.woff, c.part_base));
  uint32_t* gw32 = reinterpret_cast<uint32_t*>(c.blob + c.words_off) + w0;
  const uint64_t cap_w32 = c.cap > c.words_off ? (c.cap - c.words_off) / 4 : 0;
  const uint64_t nwords32 = 2 * ((len * b + 63) >> 6);
  const uint64_t avail = cap_w32 > w0 ? cap_w32 - w0 : 0;
  const uint64_t limit = nwords32 < avail ? nwords32 : avail;
  const uint64_t rounds = (len + 63) / 64;
  uint64_t k_begin = 0, k_end = rounds;
  if (!kWave) {
    const uint64_t quarter = ((rounds + kEncWaves - 1) / kEncWaves + kPackBatch - 1) / kPackBatch * kPackBatch;
    k_begin = wave * quarter < rounds ? wave * quarter : rounds;
    k_end = k_begin + quarter < rounds ? k_begin + quarter : rounds;
  }
  const double theta1 = __longlong_as_double(static_cast<long long>(meta_load(scr.theta, P)));
  const uint64_t base = meta_load(scr.base, P);
  uint32_t kind = 0;
  double c2 = 0.0, c3 = 0.0;
  if (c.regressor == 2) {
    kind = meta_load(scr.kind, P);
    c2 = __longlong_as_double(static_cast<long long>(meta_load(scr.c2, P)));
    c3 = __longlong_as_double(static_cast<long long>(meta_load(scr.c3, P)));
  }
  if (c.dtype == 8)
    pack_rounds(reinterpret_cast<const uint64_t*>(c.col) + start, len, base, theta1, kind, c2, c3,
                b, gw32, limit, k_begin, k_end, lds[wave]);
  else
    pack_rounds(reinterpret_cast<const uint32_t*>(c.col) + start, len, base, theta1, kind, c2, c3,
                b, gw32, limit, k_begin, k_end, lds[wave]);
}

// ---- one pass: fit, word offset by look-back, record and pack ----------------------
//
// For least-squares columns whose partitions hold at most kEncRegLen
// values: one workgroup per partition reads the values once into registers
// (wavefront w holds values 1024 w .. 1024 w + 1023, 16 per lane, so its
// rounds of 64 residuals are consecutive), fits the model as fit_block
// does, and takes the partition's word offset from the word counts of the
// partitions before it in its column (decoupled look-back: each partition
// publishes its count as soon as it is fitted, and its inclusive prefix as
// soon as it knows it).  Partitions take their index from a ticket in the
// order their workgroups start, so every partition a workgroup waits on is
// already running and publishes without waiting on later ones: the waits
// end.  It then writes its record (and start) and packs its residuals from
// the registers; the last partition of a column writes the header.

// A look-back state: flag in the top two bits, a word count below them.
// Each state is one 64-bit word read and written with relaxed atomics at
// device scope: the word is the whole message, so nothing needs ordering
// around it (acquire / release at device scope would write back or
// invalidate the L2 of an XCD at every access).
constexpr uint64_t kLbCount = uint64_t(1) << 62;      // the partition's own count
constexpr uint64_t kLbInclusive = uint64_t(2) << 62;  // counts of its column up to it
constexpr uint64_t kLbValue = kLbCount - 1;

__device__ inline void lb_publish(uint64_t* st, uint64_t P, uint64_t v) {
  __hip_atomic_store(st + P, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Words of partitions [first, P) of a column, by one wavefront: lane l reads
// the state of partition hi - 1 - l, 64 predecessors per round, down to the
// nearest one with an inclusive prefix; rounds wait (sleeping between
// reads) while a partition closer than that has published nothing yet.
__device__ inline uint64_t lb_exclusive(const uint64_t* st, uint64_t first, uint64_t P) {
  const uint32_t lane = threadIdx.x & 63;
  uint64_t acc = 0, hi = P;
  while (hi > first) {
    const uint64_t span = hi - first < 64 ? hi - first : 64;
    const bool in = lane < span;
    const uint64_t j = hi - 1 - lane;
    uint64_t s = 0;
    int stop;
    while (true) {
      s = in ? __hip_atomic_load(st + j, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
      const uint64_t inc = __ballot(in && (s >> 62) == 2);
      stop = inc ? __ffsll(static_cast<long long>(inc)) - 1 : int(span) - 1;
      const uint64_t need = stop >= 63 ? ~0ull : (2ull << stop) - 1;  // lanes 0..stop
      if (__ballot(in && (s >> 62) == 0) & need) {
        __builtin_amdgcn_s_sleep(8);
        continue;
      }
      break;
    }
    uint64_t x = in && int(lane) <= stop ? (s & kLbValue) : 0;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) x += shfl_xor64(x, m);
    acc += x;
    const bool found = __ballot(in && int(lane) == stop && (s >> 62) == 2) != 0;
    if (found) break;
    hi -= span;
  }
  return acc;
}

// Every thread receives the workgroup's min and max of int32 values.
__device__ inline void block_minmax_i32(FitShared& sh, int32_t& mn, int32_t& mx) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    mn = min(mn, __shfl_xor(mn, m, 64));
    mx = max(mx, __shfl_xor(mx, m, 64));
  }
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh.red[wave][0] = uint64_t(uint32_t(mn));
    sh.red[wave][1] = uint64_t(uint32_t(mx));
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kEncWaves; ++w) {
    mn = min(mn, int32_t(uint32_t(sh.red[w][0])));
    mx = max(mx, int32_t(uint32_t(sh.red[w][1])));
  }
  __syncthreads();
}

// The model of a partition held in registers as described above.  When
// the residuals v - vmin - floor(theta1 t) fit int32 (`small`), r32 keeps
// them for the packing.
__device__ __attribute__((always_inline)) inline Model fit_regs(FitShared& sh, const uint64_t (&v)[kEncRegs],
                                                               uint32_t t0, uint64_t len,
                                                               bool force_constant,
                                                               int32_t (&r32)[kEncRegs],
                                                               bool& small_out) {
  small_out = false;
  const bool full = len == kEncRegLen;  // no position needs masking
  // clamped loads hold the partition's last value: min and max unchanged
  uint64_t vmin = v[0], vmax = v[0];
#pragma unroll
  for (int k = 1; k < kEncRegs; ++k) {
    vmin = v[k] < vmin ? v[k] : vmin;
    vmax = v[k] > vmax ? v[k] : vmax;
  }
  block_minmax_u64(sh, vmin, vmax);
  const uint64_t range = vmax - vmin;
  Model md{vmin, vmin, 0.0, bitlen64(range), false, 0, range};
  if (len > 1 && !force_constant && range < (uint64_t(1) << 61)) {
    double th;
    bool small = false;
    if (range < kNarrowRange) {
      uint64_t sy = 0, sty = 0;  // < 2^42 and < 2^54
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) {
        const uint32_t t = t0 + 64 * k;
        const uint64_t y = full || t < len ? uint32_t(v[k]) - uint32_t(vmin) : 0;
        sy += y;
        sty += uint64_t(t) * y;
      }
      block_sum_u64x2(sh, sy, sty);
      th = block_slope(sh, len, U128{sy, 0}, U128{sty, 0});
      small = __dmul_rn(fabs(th), double(len)) < 1073741824.0;
    } else {
      U128 sv{0, 0}, stv{0, 0};
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) {
        const uint32_t t = t0 + 64 * k;
        const uint64_t x = full || t < len ? v[k] : 0;
        sv = add128(sv, U128{x, 0});
        stv = add128(stv, mul64x64(t, x));
      }
      block_sum_u128x2(sh, sv, stv);
      th = block_slope(sh, len, sv, stv);
    }
    int64_t rmin = INT64_MAX, rmax = INT64_MIN;
    if (small) {
      int32_t mn = INT32_MAX, mx = INT32_MIN;
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) {
        const uint32_t t = t0 + 64 * k;
        r32[k] = int32_t(uint32_t(v[k]) - uint32_t(vmin)) - predict32(th, t);
        if (full || t < len) {
          mn = min(mn, r32[k]);
          mx = max(mx, r32[k]);
        }
      }
      block_minmax_i32(sh, mn, mx);
      small_out = true;
      choose_model(md, th, mn, mx);
      return md;
    } else {
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) {
        const uint32_t t = t0 + 64 * k;
        const int64_t rr = int64_t(v[k] - vmin) - predict(th, t);
        if (t < len) {
          rmin = rr < rmin ? rr : rmin;
          rmax = rr > rmax ? rr : rmax;
        }
      }
    }
    block_minmax_i64(sh, rmin, rmax);
    choose_model(md, th, rmin, rmax);
    small_out = small;
  }
  return md;
}

struct FusedShared {
  FitShared fit;
  uint64_t P, woff;
  // each wavefront's 16 rounds of residuals, packed: 2 b words per round
  uint32_t words[kEncWaves][2 * 64 * kEncRegs];
};

// One workgroup per partition (its index from a ticket): values loaded
// once, model fitted, word count published; the residuals packed into LDS
// (which needs no offset) while the partitions before it publish theirs;
// then the look-back, the record, and the packed words copied out.
__device__ __attribute__((always_inline)) inline void encode_fused_part(
    FusedShared& sh, const EncColumn& c, uint64_t P, const EncScratch& scr, int* err) {
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  uint64_t start, len;
  const uint64_t j = P - c.part_base;
  part_bounds(c, j, start, len);
  const uint32_t t0 = wave * 64 * kEncRegs + lane;  // value t0 + 64 k is v[k]
  uint64_t v[kEncRegs];
  const bool full = len == kEncRegLen;  // no load clamped, no position masked
  if (c.dtype == 8) {
    const auto src = global_ptr(reinterpret_cast<const uint64_t*>(c.col) + start);
    if (full) {
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) v[k] = src[t0 + 64 * k];
    } else {
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) v[k] = load_clamped(src, t0 + 64 * k, len);
    }
  } else {
    const auto src = global_ptr(reinterpret_cast<const uint32_t*>(c.col) + start);
    if (full) {
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) v[k] = src[t0 + 64 * k];
    } else {
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) v[k] = load_clamped(src, t0 + 64 * k, len);
    }
  }
  int32_t r32[kEncRegs];
  bool small;
  const Model md = fit_regs(sh.fit, v, t0, len, c.force_constant != 0, r32, small);
  const uint64_t nw = (len * md.bits + 63) >> 6;
  uint64_t* st = scr.woff;
  if (threadIdx.x == 0) lb_publish(st, P, (j == 0 ? kLbInclusive : kLbCount) | nw);
  // pack this wavefront's rounds 16 w .. 16 w + 15 into its LDS words
  const uint32_t b = md.bits;
  const uint64_t rounds = (len + 63) / 64;
  const uint64_t r0 = uint64_t(wave) * kEncRegs;
  const uint32_t nr = r0 >= rounds ? 0 : uint32_t(rounds - r0 < kEncRegs ? rounds - r0 : kEncRegs);
  const uint32_t nwb = 2 * b * nr;
  uint32_t* w32 = sh.words[wave];
  if (nwb) {
    for (uint32_t q = lane; q < nwb; q += 64) w32[q] = 0;
    wave_fence();
    // the encoder's residual: (v - vmin) - floor(theta1 t) - rmin for the
    // line (from the fit's registers when they hold it), v - vmin for the
    // constant model
    const bool fits32 = prediction_fits_i32(md.theta1, len);
    const bool reuse = md.linear && small;
    if (reuse && full) {
      // every round whole, widths below 32: each residual ORs into two words
      // (the second gets zero bits when it fits in one)
      const int32_t rmin = int32_t(md.rmin);
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) {
        const uint32_t q = (64 * k + lane) * b;
        const uint64_t x = uint64_t(uint32_t(r32[k] - rmin)) << (q & 31);
        atomicOr(&w32[q >> 5], uint32_t(x));
        atomicOr(&w32[(q >> 5) + 1], uint32_t(x >> 32));
      }
    } else {
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) {
        const uint32_t t = t0 + 64 * k;
        uint64_t u;
        if (reuse) {
          u = uint64_t(uint32_t(r32[k] - int32_t(md.rmin)));
        } else {
          const uint64_t p = !md.linear ? 0
                             : fits32   ? uint64_t(int64_t(predict32(md.theta1, t)))
                                        : uint64_t(predict(md.theta1, t));
          u = (v[k] - md.base) - p;
        }
        if (t >= len) u = 0;
        if (uint32_t(k) < nr) or_bits(w32, (64 * k + lane) * b, b, u);
      }
    }
    wave_fence();
  }
  if (j != 0 && wave == 0) {
    const uint64_t before = lb_exclusive(st, c.part_base, P);
    if (lane == 0) {
      lb_publish(st, P, kLbInclusive | (before + nw));
      sh.woff = before;
    }
  }
  __syncthreads();
  const uint64_t woff = j == 0 ? 0 : sh.woff;
  if (threadIdx.x == 0) {
    const uint64_t rec = kHeaderBytes + kRecordBytes * j;
    if (rec + kRecordBytes <= c.cap) {
      uint64_t* r = reinterpret_cast<uint64_t*>(c.blob + rec);
      r[0] = md.base;
      r[1] = uint64_t(__double_as_longlong(md.theta1));
      r[2] = woff;
      r[3] = uint64_t(md.bits);
    }
    if (c.fixed_len == 0) {
      const uint64_t so = kHeaderBytes + kRecordBytes * c.m + 8 * j;
      if (so + 8 <= c.cap) *reinterpret_cast<uint64_t*>(c.blob + so) = start;
    }
    if (j + 1 == c.m) finish_column(c, woff + nw, err);
  }
  if (nwb) {
    const auto gdst = global_ptr(reinterpret_cast<uint32_t*>(c.blob + c.words_off) + 2 * woff);
    const uint64_t cap_w32 = c.cap > c.words_off ? (c.cap - c.words_off) / 4 : 0;
    const uint64_t avail = cap_w32 > 2 * woff ? cap_w32 - 2 * woff : 0;
    const uint64_t limit = 2 * nw < avail ? 2 * nw : avail;
    const uint64_t first = 2 * b * r0;
    const uint64_t count = first >= limit ? 0 : (limit - first < nwb ? limit - first : nwb);
    for (uint32_t q = lane; q < count; q += 64) gdst[first + q] = w32[q];
  }
}

// Before a one-pass encode: the look-back states (scr.woff) and the ticket
// (scr.bsum[0]) start at 0, and every empty column's blob is written whole
// (as k_encode_prepare does; one launch instead of two).
__global__ void k_fused_prepare(const EncColumn* __restrict__ cols, uint64_t ncols,
                                EncColumn single, EncScratch scr, uint64_t nparts, int* err) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  const uint64_t first = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (uint64_t i = first; i < nparts; i += stride) scr.woff[i] = 0;
  if (first == 0) scr.bsum[0] = 0;
  for (uint64_t i = first; i < ncols; i += stride) {
    const EncColumn& c = cols ? cols[i] : single;
    if (c.m == 0) finish_column(c, 0, err);
  }
}

__global__ __launch_bounds__(kEncBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_encode_fused(
    const EncColumn* __restrict__ cols, uint64_t ncols, EncColumn single, uint64_t nparts,
    EncScratch scr, int* err) {
  __shared__ FusedShared sh;
  if (threadIdx.x == 0)
    sh.P = atomicAdd(reinterpret_cast<unsigned long long*>(scr.bsum), 1ull);
  __syncthreads();
  const uint64_t Pw = sh.P;  // the same in every lane: made scalar
  const uint64_t P = (uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(Pw >> 32))))) << 32) |
                     uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(Pw))));
  if (P >= nparts) return;
  const EncColumn c = column_of(cols, ncols, single, P);
  encode_fused_part(sh, c, P, scr, err);
}

// The one-pass encoder for partitions of at most 64 kR values: one
// wavefront per partition, no workgroup barrier after the ticket.  Values in
// registers, model by wavefront shuffles, word count published, residuals
// packed in the wavefront's LDS slice, look-back, record and words written.
template <int kR>
__global__ __launch_bounds__(kEncBlock) void k_encode_fused_wave(
    const EncColumn* __restrict__ cols, uint64_t ncols, EncColumn single, uint64_t nparts,
    EncScratch scr, int* err) {
  __shared__ uint32_t words[kEncWaves][2 * 64 * kR];
  __shared__ uint64_t ticket;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // one ticket per workgroup, whose waves take partitions 4 ticket ..
  // 4 ticket + 3 (a ticket per wavefront, 2e6 device-scope atomics on one
  // word for 2e9 values, doubled the time of such a launch)
  if (threadIdx.x == 0)
    ticket = atomicAdd(reinterpret_cast<unsigned long long*>(scr.bsum), 1ull);
  __syncthreads();
  const uint64_t tk = ticket;
  const uint64_t P = kEncWaves * ((uint64_t(uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(tk >> 32))))) << 32) |
                                  uint32_t(__builtin_amdgcn_readfirstlane(int(uint32_t(tk))))) +
                     wave;
  if (P >= nparts) return;
  const EncColumn c = column_of(cols, ncols, single, P);
  uint64_t start, len;
  const uint64_t j = P - c.part_base;
  part_bounds(c, j, start, len);
  if (len > 64 * kR) {  // the host sends such launches to the two passes
    if (lane == 0) raise(err, kErrDevice);
    return;
  }
  uint64_t v[kR];
  if (c.dtype == 8) {
    const uint64_t* src = reinterpret_cast<const uint64_t*>(c.col) + start;
#pragma unroll
    for (int k = 0; k < kR; ++k) v[k] = load_clamped(src, lane + 64 * k, len);
  } else {
    const uint32_t* src = reinterpret_cast<const uint32_t*>(c.col) + start;
#pragma unroll
    for (int k = 0; k < kR; ++k) v[k] = load_clamped(src, lane + 64 * k, len);
  }
  const Model md = fit_wave_regs<kR>(v, len, c.force_constant != 0);
  const uint64_t nw = (len * md.bits + 63) >> 6;
  uint64_t* st = scr.woff;
  if (lane == 0) lb_publish(st, P, (j == 0 ? kLbInclusive : kLbCount) | nw);
  const uint32_t b = md.bits;
  const uint32_t nr = uint32_t((len + 63) / 64);
  const uint32_t nwb = 2 * b * nr;
  uint32_t* w32 = words[wave];
  if (nwb) {
    for (uint32_t q = lane; q < nwb; q += 64) w32[q] = 0;
    wave_fence();
    const bool fits32 = prediction_fits_i32(md.theta1, len);
#pragma unroll
    for (int k = 0; k < kR; ++k) {
      const uint32_t t = lane + 64 * k;
      const uint64_t p = !md.linear ? 0
                         : fits32   ? uint64_t(int64_t(predict32(md.theta1, t)))
                                    : uint64_t(predict(md.theta1, t));
      const uint64_t u = t < len ? (v[k] - md.base) - p : 0;
      if (uint32_t(k) < nr) or_bits(w32, t * b, b, u);
    }
    wave_fence();
  }
  uint64_t woff = 0;
  if (j != 0) {
    woff = lb_exclusive(st, c.part_base, P);
    if (lane == 0) lb_publish(st, P, kLbInclusive | (woff + nw));
  }
  if (lane == 0) {
    const uint64_t rec = kHeaderBytes + kRecordBytes * j;
    if (rec + kRecordBytes <= c.cap) {
      uint64_t* r = reinterpret_cast<uint64_t*>(c.blob + rec);
      r[0] = md.base;
      r[1] = uint64_t(__double_as_longlong(md.theta1));
      r[2] = woff;
      r[3] = uint64_t(md.bits);
    }
    if (c.fixed_len == 0) {
      const uint64_t so = kHeaderBytes + kRecordBytes * c.m + 8 * j;
      if (so + 8 <= c.cap) *reinterpret_cast<uint64_t*>(c.blob + so) = start;
    }
    if (j + 1 == c.m) finish_column(c, woff + nw, err);
  }
  if (nwb) {
    const auto gdst = global_ptr(reinterpret_cast<uint32_t*>(c.blob + c.words_off) + 2 * woff);
    const uint64_t cap_w32 = c.cap > c.words_off ? (c.cap - c.words_off) / 4 : 0;
    const uint64_t avail = cap_w32 > 2 * woff ? cap_w32 - 2 * woff : 0;
    const uint64_t limit = 2 * nw < avail ? 2 * nw : avail;
    const uint64_t count = limit < nwb ? limit : nwb;
    for (uint32_t q = lane; q < count; q += 64) gdst[q] = w32[q];
  }
}

// Writes the complete blob of every empty column (no partitions, so no
// other kernel sees it).
__global__ void k_encode_prepare(const EncColumn* __restrict__ cols, uint64_t ncols,
                                 EncColumn single, int* err) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < ncols; i += stride) {
    const EncColumn& c = cols ? cols[i] : single;
    if (c.m != 0) continue;
    finish_column(c, 0, err);  // also writes starts[0] = 0 of a variable column
  }
}

uint64_t encode_scratch_bytes(uint64_t nparts) {
  const uint64_t k = nparts ? nparts : 1;
  const uint64_t ng = (k + kScanItems - 1) / kScanItems;
  return 8 * (6 * k + ng + 1) + 8 * k + 64;
}

EncScratch carve_encode_scratch(void* p, uint64_t nparts) {
  const uint64_t k = nparts ? nparts : 1;
  const uint64_t ng = (k + kScanItems - 1) / kScanItems;
  uint64_t* q = static_cast<uint64_t*>(p);
  EncScratch s;
  s.nwords = q;
  s.woff = q + k;
  s.base = q + 2 * k;
  s.theta = q + 3 * k;
  s.bsum = q + 4 * k;
  s.c2 = q + 4 * k + ng + 1;
  s.c3 = q + 5 * k + ng + 1;
  s.bits = reinterpret_cast<uint32_t*>(q + 6 * k + ng + 1);
  s.kind = s.bits + k;
  s.hull = nullptr;
  s.hull_values = 0;
  return s;
}

hipError_t launch_fit_columns(leco_ctx* ctx, const EncColumn* cols_dev, uint64_t ncols,
                              const EncColumn& single, uint64_t nparts, uint64_t max_len,
                              uint32_t regs, const EncScratch& scr, hipStream_t stream) {
  if (nparts == 0) return hipSuccess;
  // each fit kernel fits the columns of its regressors and skips the others
  const uint64_t pw = (nparts + kEncWaves - 1) / kEncWaves;
  // one wavefront per partition: 16 values per lane up to 1024 values, 32
  // up to 2048 (not the minimax fit, whose hull slice holds 1024)
  const bool wave16 = max_len <= kWaveEncMax && ctx->tune.encode_wave;
  const bool wave32 =
      max_len <= 2 * kWaveEncMax && ctx->tune.encode_wave && ctx->tune.encode_wave32;
  if ((regs & kRegPoly) && wave16)
    hipLaunchKernelGGL(k_fit_poly_wave<kWaveRegs>, dim3(uint32_t(pw)), dim3(kEncBlock), 0, stream,
                       cols_dev, ncols, single, nparts, scr, ctx->err_dev);
  else if ((regs & kRegPoly) && wave32)
    hipLaunchKernelGGL(k_fit_poly_wave<2 * kWaveRegs>, dim3(uint32_t(pw)), dim3(kEncBlock), 0,
                       stream, cols_dev, ncols, single, nparts, scr, ctx->err_dev);
  else if (regs & kRegPoly)
    hipLaunchKernelGGL(k_fit_poly, dim3(uint32_t(nparts)), dim3(kEncBlock), 0, stream, cols_dev,
                       ncols, single, nparts, scr);
  if (!(regs & (kRegLS | kRegMinimax))) return hipGetLastError();
  if (regs == kRegLS && max_len <= kLaneFitMax && ctx->tune.encode_wave) {
    const uint64_t g = (nparts + 255) / 256, cap = uint64_t(ctx->num_cus) * 16;
    hipLaunchKernelGGL(k_fit_lane, dim3(uint32_t(g < cap ? g : cap)), dim3(256), 0, stream,
                       cols_dev, ncols, single, nparts, scr);
    return hipGetLastError();
  }
  // k_fit_wave fits every column it is given: not with polynomial columns
  const bool poly = regs & kRegPoly;
  if ((regs & kRegMinimax) && wave16 && !poly)
    hipLaunchKernelGGL(k_fit_minimax_wave, dim3(uint32_t(pw)), dim3(kEncBlock), 0, stream, cols_dev,
                       ncols, single, nparts, scr, ctx->err_dev);
  else if (regs & kRegMinimax)
    hipLaunchKernelGGL(k_fit_minimax, dim3(uint32_t(nparts)), dim3(kEncBlock), 0, stream, cols_dev,
                       ncols, single, nparts, scr, ctx->err_dev);
  else if (wave16 && !poly)
    hipLaunchKernelGGL(k_fit_wave<kWaveRegs>, dim3(uint32_t(pw)), dim3(kEncBlock), 0, stream,
                       cols_dev, ncols, single, nparts, scr, ctx->err_dev);
  else if (wave32 && !poly)
    hipLaunchKernelGGL(k_fit_wave<2 * kWaveRegs>, dim3(uint32_t(pw)), dim3(kEncBlock), 0, stream,
                       cols_dev, ncols, single, nparts, scr, ctx->err_dev);
  else
    hipLaunchKernelGGL(k_fit_block, dim3(uint32_t(nparts)), dim3(kEncBlock), 0, stream, cols_dev,
                       ncols, single, nparts, scr);
  return hipGetLastError();
}

hipError_t launch_encode_columns(leco_ctx* ctx, const EncColumn* cols_dev, uint64_t ncols,
                                 const EncColumn& single, uint64_t nparts, uint64_t max_len,
                                 uint32_t regs, const EncScratch& scr, hipStream_t stream) {
  const bool wave_fit = max_len <= kWaveEncMax ||
                        (max_len <= 2 * kWaveEncMax && ctx->tune.encode_wave32);
  const uint64_t pw = (nparts + kEncWaves - 1) / kEncWaves;
  const auto fused = [&](uint32_t mode, uint64_t workgroups) {
    return mode == 1 || (mode == 2 && workgroups <= uint64_t(kFusedAutoPerCu) * ctx->num_cus);
  };
  const bool one_pass_wave = nparts != 0 && regs == kRegLS && ctx->tune.encode_wave &&
                             max_len <= kWaveEncMax && fused(ctx->tune.encode_fused_wave, pw);
  const bool one_pass = nparts != 0 && regs == kRegLS && !one_pass_wave &&
                        max_len <= kEncRegLen && !(wave_fit && ctx->tune.encode_wave) &&
                        fused(ctx->tune.encode_fused, nparts);
  if (one_pass_wave || one_pass) {
    const uint64_t items = nparts > ncols ? nparts : ncols;
    const uint64_t g = (items + 255) / 256;
    hipLaunchKernelGGL(k_fused_prepare, dim3(uint32_t(g < 4096 ? g : 4096)), dim3(256), 0, stream,
                       cols_dev, ncols, single, scr, nparts, ctx->err_dev);
    if (one_pass_wave)
      hipLaunchKernelGGL(k_encode_fused_wave<kWaveRegs>, dim3(uint32_t(pw)), dim3(kEncBlock), 0,
                         stream, cols_dev, ncols, single, nparts, scr, ctx->err_dev);
    else
      hipLaunchKernelGGL(k_encode_fused, dim3(uint32_t(nparts)), dim3(kEncBlock), 0, stream,
                         cols_dev, ncols, single, nparts, scr, ctx->err_dev);
    return hipGetLastError();
  }
  const uint64_t cg = (ncols + 255) / 256;
  hipLaunchKernelGGL(k_encode_prepare, dim3(uint32_t(cg < 4096 ? cg : 4096)), dim3(256), 0,
                     stream, cols_dev, ncols, single, ctx->err_dev);
  if (nparts == 0) return hipGetLastError();
  const hipError_t e = launch_fit_columns(ctx, cols_dev, ncols, single, nparts, max_len, regs,
                                          scr, stream);
  if (e != hipSuccess) return e;
  const bool wave = max_len <= kWaveEncMax && ctx->tune.encode_wave;  // pack only
  const uint64_t ng = (nparts + kScanItems - 1) / kScanItems;
  hipLaunchKernelGGL(k_scan_sums, dim3(uint32_t(ng)), dim3(kEncBlock), 0, stream, scr, nparts);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kEncBlock), 0, stream, scr, ng);
  hipLaunchKernelGGL(k_scan_apply, dim3(uint32_t(ng)), dim3(kEncBlock), 0, stream, scr, nparts);
  hipLaunchKernelGGL(k_records, dim3(uint32_t((nparts + 255) / 256)), dim3(256), 0, stream,
                     cols_dev, ncols, single, nparts, scr, ctx->err_dev);
  if (wave)
    hipLaunchKernelGGL(k_pack<true>, dim3(uint32_t(pw)), dim3(kEncBlock), 0, stream, cols_dev,
                       ncols, single, nparts, scr);
  else
    hipLaunchKernelGGL(k_pack<false>, dim3(uint32_t(nparts)), dim3(kEncBlock), 0, stream, cols_dev,
                       ncols, single, nparts, scr);
  return hipGetLastError();
}

// ---- sampled cost of a partitioning -------------------------------------------------

// *out += sum over P < nparts of 32 + 8 * nwords[P]: the record and word
// bytes the fitted partitions add to a blob.
__global__ __launch_bounds__(kEncBlock) void k_cost_sum(EncScratch scr, uint64_t nparts,
                                                       uint64_t extra, unsigned long long* out) {
  __shared__ uint64_t part[kEncWaves];
  uint64_t x = 0;
  const uint64_t stride = uint64_t(gridDim.x) * kEncBlock;
  for (uint64_t P = uint64_t(blockIdx.x) * kEncBlock + threadIdx.x; P < nparts; P += stride)
    x += kRecordBytes + extra + 8 * scr.nwords[P];
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) x += shfl_xor64(x, m);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int w = 0; w < kEncWaves; ++w) t += part[w];
    atomicAdd(out, static_cast<unsigned long long>(t));
  }
}

hipError_t launch_cost_sum(const EncScratch& scr, uint64_t nparts, uint64_t extra_per_part,
                           uint64_t* out, hipStream_t stream) {
  uint64_t blocks = (nparts + kEncBlock - 1) / kEncBlock;
  blocks = blocks < 1 ? 1 : (blocks > 2048 ? 2048 : blocks);
  hipLaunchKernelGGL(k_cost_sum, dim3(uint32_t(blocks)), dim3(kEncBlock), 0, stream, scr, nparts,
                     extra_per_part, reinterpret_cast<unsigned long long*>(out));
  return hipGetLastError();
}

// ---- diagnostics --------------------------------------------------------------

__global__ void k_diag_slope(const uint64_t* __restrict__ in, uint64_t k, double* __restrict__ out) {
  const uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const U128 N{in[4 * i], in[4 * i + 1]};
  const U128 D{in[4 * i + 2], in[4 * i + 3]};
  double s = i128_to_f64(N) / u128_to_f64(D);
  if (s == 0.0) s = 0.0;
  out[i] = s;
}

hipError_t launch_diag_slope(const uint64_t* in, uint64_t k, double* out, hipStream_t stream) {
  if (k == 0) return hipSuccess;
  hipLaunchKernelGGL(k_diag_slope, dim3(uint32_t((k + 255) / 256)), dim3(256), 0, stream, in, k, out);
  return hipGetLastError();
}

}  // namespace leco
