// LeCo encoder for gfx950 (section 3.1 regressor, section 3.3 encoder), one
// pass over the input: each workgroup takes the next partition in ticket
// order, keeps its values in registers (4096 per partition; longer
// partitions are streamed in chunks), reduces the range and the exact
// least-squares sums with wavefront shuffles, derives the slope and the
// residual width, obtains its word offset from a decoupled look-back over
// the partitions before it in the same column, and bit-packs its residuals
// through LDS into the blob.  Works on a table of columns, so one launch
// encodes one column or thousands.
//
// Register-resident partitions whose range is below 2^30 (the usual case)
// take a narrow path: y = v - vmin fits 32 bits, the exact sums fit 64-bit
// lanes, and predictions and residuals fit int32.  The arithmetic and its
// results are the same as on the general path, only carried in fewer bits.
#include "fit.hpp"
#include "internal.hpp"
#include "leco_dev.hpp"

namespace leco {

constexpr int kEncRegs = 16;                           // values per thread in registers
constexpr uint32_t kEncRegLen = kEncBlock * kEncRegs;  // 4096
constexpr uint32_t kPackWords = 2048;                  // 64-bit words in the LDS pack buffer
constexpr uint64_t kFlagAgg = 1ull << 62;              // look-back status: aggregate
constexpr uint64_t kFlagPrefix = 2ull << 62;           //                   inclusive prefix
constexpr uint64_t kValueMask = (1ull << 62) - 1;
constexpr uint32_t kSpinLimit = 1u << 24;              // bounded wait on a predecessor
constexpr uint64_t kNarrowRange = 1ull << 30;

__device__ inline void raise(int* err, int bits) { atomicOr(err, bits); }

struct EncShared {
  uint64_t words[kPackWords];
  uint64_t red[kEncWaves][4];
  double theta1;
  uint64_t word_off;
  uint64_t ticket;
};

// ORs a residual u (< 2^b) into the LDS stream at bit q.
__device__ inline void or_bits(uint32_t* w, uint32_t q, uint32_t b, uint64_t u) {
  if (u == 0) return;
  const uint32_t i = q >> 5, s = q & 31;
  atomicOr(&w[i], uint32_t(u << s));
  if (s + b > 32) atomicOr(&w[i + 1], uint32_t(u >> (32 - s)));
  if (s + b > 64) atomicOr(&w[i + 2], uint32_t(u >> (64 - s)));
}
// Same for b <= 32.
__device__ inline void or_bits32(uint32_t* w, uint32_t q, uint32_t b, uint32_t u) {
  if (u == 0) return;
  const uint32_t i = q >> 5, s = q & 31;
  atomicOr(&w[i], u << s);
  if (s + b > 32) atomicOr(&w[i + 1], u >> (32 - s));
}

__device__ inline const EncColumn& column_of(const EncColumn* cols, uint64_t ncols,
                                             const EncColumn& single, uint64_t P) {
  if (cols == nullptr) return single;
  uint64_t lo = 0, hi = ncols;  // last column with part_base <= P
  while (hi - lo > 1) {
    const uint64_t mid = lo + ((hi - lo) >> 1);
    if (cols[mid].part_base <= P) lo = mid; else hi = mid;
  }
  return cols[lo];
}

__device__ inline void write_header(const EncColumn& c, uint64_t total_words) {
  uint64_t* hd = reinterpret_cast<uint64_t*>(c.blob);
  const bool variable = c.fixed_len == 0;
  hd[0] = uint64_t(kMagic) | (uint64_t(kVersion) << 32) | (uint64_t(c.dtype) << 48) |
          (uint64_t(variable ? 1 : 0) << 56);
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
  for (uint64_t i = meta_end; i < c.words_off; ++i) c.blob[i] = 0;
  for (uint64_t i = c.words_off + 8 * total_words; i < size; ++i) c.blob[i] = 0;
}

// Word offset of partition P inside its column by decoupled look-back, then
// its record (and start); the last partition also finishes the column.
// Wave 0 reads kRows rows of 64 predecessors per round trip (row r, lane l
// holds partition top - 64 r - l; partitions before the column's first
// count as an inclusive prefix of 0), so the inclusive-prefix frontier
// advances kRows * 64 partitions per global-memory round trip.  The status
// words carry their own value, so relaxed device-scope atomics suffice.
// Run by one whole wavefront; every lane receives the word offset.
__device__ uint64_t look_back_wave(const EncColumn& c, uint64_t P, uint64_t j, uint64_t start,
                                  uint64_t nwords, const Model& md, uint64_t* status, int* err) {
  const uint32_t lane = threadIdx.x & 63;
  {
    if (lane == 0)
      __hip_atomic_store(&status[P], (j == 0 ? kFlagPrefix : kFlagAgg) | nwords, __ATOMIC_RELAXED,
                         __HIP_MEMORY_SCOPE_AGENT);
    uint64_t excl = 0;
    if (j != 0) {
      // The first round reads one row (the frontier is usually near); a
      // round that consumes its whole window without a prefix widens it.
      constexpr int kRows = 4;
      int rows = 1;
      int64_t top = int64_t(P) - 1;
      uint32_t spins = 0;
      bool done = false;
      while (!done) {
        uint64_t s[kRows];
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          const int64_t q = top - 64 * r - int64_t(lane);
          s[r] = (r < rows && q >= int64_t(c.part_base))
                     ? __hip_atomic_load(&status[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                     : kFlagPrefix;
        }
        uint64_t add = 0;
        int rows_used = 0;
        bool wait = false;
#pragma unroll
        for (int r = 0; r < kRows; ++r) {
          if (done || wait || r >= rows) continue;
          const uint64_t not_ready = __ballot((s[r] >> 62) == 0);
          const uint64_t prefix = __ballot((s[r] >> 62) == 2);
          const uint32_t first =
              prefix ? uint32_t(__ffsll(static_cast<long long>(prefix)) - 1) : 64u;
          const uint64_t needed = first >= 63 ? ~uint64_t(0) : ((uint64_t(2) << first) - 1);
          if (not_ready & needed) {
            wait = true;
            continue;
          }
          uint64_t x = lane <= first ? (s[r] & kValueMask) : 0;
#pragma unroll
          for (int m = 32; m > 0; m >>= 1) x += shfl_xor64(x, m);
          add += x;
          ++rows_used;
          if (first < 64) done = true;
        }
        // rows before the first unready one are final: keep them, move on
        excl += add;
        top -= 64 * rows_used;
        if (wait && !done) {
          if (++spins > kSpinLimit) {
            if (lane == 0) raise(err, kErrDevice);
            break;
          }
          __builtin_amdgcn_s_sleep(1);
        } else {
          rows = kRows;
        }
      }
      if (lane == 0)
        __hip_atomic_store(&status[P], kFlagPrefix | ((excl + nwords) & kValueMask),
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (lane == 0) {
      const uint64_t rec = kHeaderBytes + kRecordBytes * j;
      if (rec + kRecordBytes <= c.cap) {
        uint64_t* r = reinterpret_cast<uint64_t*>(c.blob + rec);
        r[0] = md.base;
        r[1] = uint64_t(__double_as_longlong(md.theta1));
        r[2] = excl;
        r[3] = uint64_t(md.bits);
      }
      if (c.fixed_len == 0) {
        const uint64_t so = kHeaderBytes + kRecordBytes * c.m + 8 * j;
        if (so + 8 <= c.cap) *reinterpret_cast<uint64_t*>(c.blob + so) = start;
      }
      if (j + 1 == c.m) finish_column(c, excl + nwords, err);
    }
    return excl;
  }
}

// The workgroup version: wave 0 looks back, every thread gets the offset.
__device__ uint64_t publish_and_look_back(EncShared& sh, const EncColumn& c, uint64_t P,
                                          uint64_t j, uint64_t start, uint64_t nwords,
                                          const Model& md, uint64_t* status, int* err) {
  if ((threadIdx.x >> 6) == 0) {
    const uint64_t excl = look_back_wave(c, P, j, start, nwords, md, status, err);
    if ((threadIdx.x & 63) == 0) sh.word_off = excl;
  }
  __syncthreads();
  return sh.word_off;
}

// Copies packed words [0, cw) of the LDS buffer to global words [w0, w0+cw).
__device__ inline void store_words(const EncShared& sh, uint64_t* gwords, uint64_t w0,
                                   uint32_t cw, uint64_t cap_words) {
  for (uint32_t i = threadIdx.x; i < cw; i += kEncBlock)
    if (w0 + i < cap_words) gwords[w0 + i] = sh.words[i];
}

__device__ inline void zero_words(EncShared& sh, uint32_t cw) {
  for (uint32_t i = threadIdx.x; i < cw; i += kEncBlock) sh.words[i] = 0;
}

__global__ __launch_bounds__(kEncBlock) void k_encode(const EncColumn* __restrict__ cols,
                                                     uint64_t ncols, EncColumn single,
                                                     uint64_t* __restrict__ status,
                                                     unsigned long long* __restrict__ ticket,
                                                     int* err) {
  __shared__ EncShared sh;
  const uint32_t tid = threadIdx.x;
  // Partition order: a ticket from one counter (no assumption on dispatch
  // order), or the workgroup index (workgroups are dispatched in index
  // order, so every predecessor of a running workgroup has started).
  uint64_t P = blockIdx.x;
  if (ticket) {
    if (tid == 0) sh.ticket = atomicAdd(ticket, 1ull);
    __syncthreads();
    P = sh.ticket;
  }
  const EncColumn& c = column_of(cols, ncols, single, P);
  const uint64_t j = P - c.part_base;
  uint64_t start, len;
  if (c.fixed_len) {
    start = j * c.fixed_len;
    len = (start + c.fixed_len < c.n ? start + c.fixed_len : c.n) - start;
  } else {
    start = c.starts[j];
    len = c.starts[j + 1] - start;
  }
  const uint8_t* src = c.col + start * c.dtype;
  const bool in_regs = len <= kEncRegLen;
  const bool fit_allowed = !(len == 1 || c.force_constant);
  uint64_t* gwords = reinterpret_cast<uint64_t*>(c.blob + c.words_off);
  const uint64_t cap_words = c.cap > c.words_off ? (c.cap - c.words_off) / 8 : 0;
  uint32_t* w32 = reinterpret_cast<uint32_t*>(sh.words);

  uint64_t v[kEncRegs];
  uint64_t vmin = ~uint64_t(0), vmax = 0;
  U128 sv{0, 0}, stv{0, 0};
  if (in_regs) {
#pragma unroll
    for (int k = 0; k < kEncRegs; ++k) {
      const uint32_t t = tid + k * kEncBlock;
      v[k] = t < len ? load_value(src, c.dtype, t) : 0;
      if (t < len) {
        vmin = v[k] < vmin ? v[k] : vmin;
        vmax = v[k] > vmax ? v[k] : vmax;
      }
    }
  } else {
    // streamed: range and raw sums in one pass
    for (uint64_t t = tid; t < len; t += kEncBlock) {
      const uint64_t x = load_value(src, c.dtype, t);
      vmin = x < vmin ? x : vmin;
      vmax = x > vmax ? x : vmax;
      sv = add128(sv, U128{x, 0});
      stv = add128(stv, mul64x64(t, x));
    }
  }
  block_minmax_u64(sh, vmin, vmax);
  const uint64_t range = vmax - vmin;
  Model md{vmin, vmin, 0.0, bitlen64(range), false, 0};
  const bool fit = fit_allowed && range < (uint64_t(1) << 61);

  if (in_regs && range < kNarrowRange) {
    // ---- narrow path ----
    uint32_t y[kEncRegs];
#pragma unroll
    for (int k = 0; k < kEncRegs; ++k) y[k] = uint32_t(v[k]) - uint32_t(vmin);  // y < 2^30
    int32_t r[kEncRegs];
    bool small = false;
    if (fit) {
      uint64_t sy = 0, sty = 0;  // < 2^42 and < 2^54
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) {
        const uint32_t t = tid + k * kEncBlock;
        if (t < len) {
          sy += y[k];
          sty += uint64_t(t) * y[k];
        }
      }
      block_sum_u64x2(sh, sy, sty);
      const double th = block_slope(sh, len, U128{sy, 0}, U128{sty, 0});
      // |floor(theta1 t)| < 2^30 for every t < len, so residuals fit int32
      small = __dmul_rn(fabs(th), double(len)) < 1073741824.0;
      int64_t rmin = INT64_MAX, rmax = INT64_MIN;
      if (small) {
        int32_t mn = INT32_MAX, mx = INT32_MIN;
#pragma unroll
        for (int k = 0; k < kEncRegs; ++k) {
          const uint32_t t = tid + k * kEncBlock;
          r[k] = 0;
          if (t < len) {
            r[k] = int32_t(y[k]) - predict32(th, t);
            mn = r[k] < mn ? r[k] : mn;
            mx = r[k] > mx ? r[k] : mx;
          }
        }
        rmin = mn;
        rmax = mx;
      } else {
#pragma unroll
        for (int k = 0; k < kEncRegs; ++k) {
          const uint32_t t = tid + k * kEncBlock;
          if (t < len) {
            const int64_t rr = int64_t(y[k]) - predict(th, t);
            rmin = rr < rmin ? rr : rmin;
            rmax = rr > rmax ? rr : rmax;
          }
        }
      }
      block_minmax_i64(sh, rmin, rmax);
      choose_model(md, th, rmin, rmax);
    }
    const uint32_t b = md.bits;  // <= 30
    const uint64_t nwords = (len * b + 63) >> 6;
    const uint64_t word_off =
        publish_and_look_back(sh, c, P, j, start, nwords, md, status, err);
    if (b == 0) return;
    const uint32_t cw = uint32_t(nwords);  // <= 4096 * 30 / 64 < kPackWords
    zero_words(sh, cw);
    __syncthreads();
    const int32_t rmin32 = int32_t(md.rmin);
#pragma unroll
    for (int k = 0; k < kEncRegs; ++k) {
      const uint32_t t = tid + k * kEncBlock;
      if (t < len) {
        uint32_t u;
        if (!md.linear) u = y[k];
        else if (small) u = uint32_t(r[k] - rmin32);
        else u = uint32_t(uint64_t(int64_t(y[k]) - predict(md.theta1, t)) - uint64_t(md.rmin));
        or_bits32(w32, t * b, b, u);
      }
    }
    __syncthreads();
    store_words(sh, gwords, word_off, cw, cap_words);
    return;
  }

  // ---- general path: 128-bit sums, 64-bit residuals ----
  if (fit) {
    if (in_regs) {
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) {
        const uint32_t t = tid + k * kEncBlock;
        if (t < len) {
          sv = add128(sv, U128{v[k], 0});
          stv = add128(stv, mul64x64(t, v[k]));
        }
      }
    }
    block_sum_u128x2(sh, sv, stv);
    const double th = block_slope(sh, len, sv, stv);
    int64_t rmin = INT64_MAX, rmax = INT64_MIN;
    if (in_regs) {
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) {
        const uint32_t t = tid + k * kEncBlock;
        if (t < len) {
          const int64_t rr = int64_t(v[k] - vmin) - predict(th, t);
          rmin = rr < rmin ? rr : rmin;
          rmax = rr > rmax ? rr : rmax;
        }
      }
    } else {
      for (uint64_t t = tid; t < len; t += kEncBlock) {
        const int64_t rr = int64_t(load_value(src, c.dtype, t) - vmin) - predict(th, uint32_t(t));
        rmin = rr < rmin ? rr : rmin;
        rmax = rr > rmax ? rr : rmax;
      }
    }
    block_minmax_i64(sh, rmin, rmax);
    choose_model(md, th, rmin, rmax);
  }
  const uint32_t b = md.bits;
  const uint64_t nwords = (len * b + 63) >> 6;
  const uint64_t word_off = publish_and_look_back(sh, c, P, j, start, nwords, md, status, err);
  if (b == 0) return;

  // residual t at bits [b t, b t + b) of the partition's span, in chunks
  // whose words fit the LDS buffer (chunk * b / 64 <= kPackWords)
  const uint32_t chunk = b <= 32 ? 4096u : 2048u;
  for (uint64_t c0 = 0; c0 < len; c0 += chunk) {
    const uint64_t c1 = c0 + chunk < len ? c0 + chunk : len;
    const uint32_t cw = uint32_t(((c1 - c0) * b + 63) >> 6);
    zero_words(sh, cw);
    __syncthreads();
    if (in_regs) {
#pragma unroll
      for (int k = 0; k < kEncRegs; ++k) {
        const uint32_t t = tid + k * kEncBlock;
        if (t >= c0 && t < c1) {
          const uint64_t yy = v[k] - md.base;
          const uint64_t u = md.linear ? yy - uint64_t(predict(md.theta1, t)) : yy;
          or_bits(w32, uint32_t(t - c0) * b, b, u);
        }
      }
    } else {
      for (uint64_t t = c0 + tid; t < c1; t += kEncBlock) {
        const uint64_t yy = load_value(src, c.dtype, t) - md.base;
        const uint64_t u = md.linear ? yy - uint64_t(predict(md.theta1, uint32_t(t))) : yy;
        or_bits(w32, uint32_t(t - c0) * b, b, u);
      }
    }
    __syncthreads();
    store_words(sh, gwords, word_off + ((c0 * b) >> 6), cw, cap_words);
    __syncthreads();
  }
}

// ---- one wavefront per partition ------------------------------------------------

// Partitions of at most kWaveEncMax values are encoded by one wavefront
// each (16 values per lane in registers, shuffle reductions, no workgroup
// barrier), four per workgroup.
constexpr uint32_t kWaveEncMax = uint32_t(kWaveEncodeMax);
constexpr int kWaveRegs = int(kWaveEncMax / 64);

__device__ inline void wave_fence() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Same model, bytes and look-back as k_encode for every partition of the
// launch, which the host only sends here when none is longer than
// kWaveEncMax.  Packing goes one round of 64 residuals at a time: round k
// holds residuals 64k .. 64k + 63, which fill exactly 2b 32-bit words, so
// the rounds never share a word; the round is assembled in the
// wavefront's LDS buffer and stored.
__global__ __launch_bounds__(kEncBlock) void k_encode_wave(const EncColumn* __restrict__ cols,
                                                          uint64_t ncols, EncColumn single,
                                                          uint64_t* __restrict__ status,
                                                          unsigned long long* __restrict__ ticket,
                                                          uint64_t nparts, int* err) {
  __shared__ uint32_t pack_lds[kEncWaves][128];
  __shared__ unsigned long long block_ticket;
  const uint32_t lane = threadIdx.x & 63;
  const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  // one ticket per workgroup for its four partitions: same-address atomics
  // serialize, so fewer of them shorten the launch
  uint64_t P;
  if (ticket) {
    if (threadIdx.x == 0) block_ticket = atomicAdd(ticket, 1ull);
    __syncthreads();
    P = uint64_t(block_ticket) * kEncWaves + wave;
  } else {
    P = uint64_t(blockIdx.x) * kEncWaves + wave;
  }
  if (P >= nparts) return;
  const EncColumn& c = column_of(cols, ncols, single, P);
  const uint64_t j = P - c.part_base;
  uint64_t start, len;
  if (c.fixed_len) {
    start = j * c.fixed_len;
    len = (start + c.fixed_len < c.n ? start + c.fixed_len : c.n) - start;
  } else {
    start = c.starts[j];
    len = c.starts[j + 1] - start;
  }
  if (len > kWaveEncMax) {  // the host routes such partitions to k_encode
    if (lane == 0) raise(err, kErrDevice);
    return;
  }
  const uint8_t* src = c.col + start * c.dtype;
  const bool fit_allowed = !(len == 1 || c.force_constant);
  uint32_t* gw32 = reinterpret_cast<uint32_t*>(c.blob + c.words_off);
  const uint64_t cap_w32 = c.cap > c.words_off ? (c.cap - c.words_off) / 4 : 0;
  uint32_t* w32 = pack_lds[wave];

  uint64_t v[kWaveRegs];
  uint64_t vmin = ~uint64_t(0), vmax = 0;
#pragma unroll
  for (int k = 0; k < kWaveRegs; ++k) {
    const uint32_t t = lane + 64 * k;
    v[k] = t < len ? load_value(src, c.dtype, t) : 0;
    if (t < len) {
      vmin = v[k] < vmin ? v[k] : vmin;
      vmax = v[k] > vmax ? v[k] : vmax;
    }
  }
  wave_minmax_u64(vmin, vmax);
  const uint64_t range = vmax - vmin;
  Model md{vmin, vmin, 0.0, bitlen64(range), false, 0};
  const bool fit = fit_allowed && range < (uint64_t(1) << 61);
  const bool narrow = range < kNarrowRange;
  bool small = false;
  if (fit) {
    double th;
    if (narrow) {
      uint64_t sy = 0, sty = 0;  // < 2^40 and < 2^50
#pragma unroll
      for (int k = 0; k < kWaveRegs; ++k) {
        const uint32_t t = lane + 64 * k;
        if (t < len) {
          const uint64_t y = uint32_t(v[k]) - uint32_t(vmin);
          sy += y;
          sty += uint64_t(t) * y;
        }
      }
      wave_sum_u64x2(sy, sty);
      th = ls_slope(len, U128{sy, 0}, U128{sty, 0});
    } else {
      U128 sv{0, 0}, stv{0, 0};
#pragma unroll
      for (int k = 0; k < kWaveRegs; ++k) {
        const uint32_t t = lane + 64 * k;
        if (t < len) {
          sv = add128(sv, U128{v[k], 0});
          stv = add128(stv, mul64x64(t, v[k]));
        }
      }
      wave_sum_u128x2(sv, stv);
      th = ls_slope(len, sv, stv);
    }
    // |floor(theta1 t)| < 2^30 for every t < len: predictions fit int32
    small = narrow && __dmul_rn(fabs(th), double(len)) < 1073741824.0;
    int64_t rmin = INT64_MAX, rmax = INT64_MIN;
#pragma unroll
    for (int k = 0; k < kWaveRegs; ++k) {
      const uint32_t t = lane + 64 * k;
      if (t < len) {
        const int64_t rr = small ? int64_t(int32_t(uint32_t(v[k]) - uint32_t(vmin)) - predict32(th, t))
                                 : int64_t(v[k] - vmin) - predict(th, t);
        rmin = rr < rmin ? rr : rmin;
        rmax = rr > rmax ? rr : rmax;
      }
    }
    wave_minmax_i64(rmin, rmax);
    choose_model(md, th, rmin, rmax);
  }
  const uint32_t b = md.bits;
  const uint64_t nwords = (len * b + 63) >> 6;
  const uint64_t word_off = look_back_wave(c, P, j, start, nwords, md, status, err);
  if (b == 0) return;
  const uint64_t w0 = 2 * word_off;  // first 32-bit word of the span
  const uint32_t rounds = uint32_t((len + 63) / 64);
#pragma unroll
  for (int k = 0; k < kWaveRegs; ++k) {
    if (uint32_t(k) >= rounds) break;
    w32[lane] = 0;
    w32[lane + 64] = 0;
    wave_fence();
    const uint32_t t = lane + 64 * k;
    if (t < len) {
      uint64_t u;
      if (!md.linear) u = v[k] - md.vmin;
      else if (small)
        u = uint64_t(uint32_t(int32_t(uint32_t(v[k]) - uint32_t(vmin)) - predict32(md.theta1, t) -
                              int32_t(md.rmin)));
      else u = (v[k] - md.base) - uint64_t(predict(md.theta1, t));
      or_bits(w32, lane * b, b, u);
    }
    wave_fence();
    // 32-bit words of this round: 2b, the last round up to the span's end
    const uint64_t first = uint64_t(2 * b) * k;
    const uint64_t count = (first + 2 * b <= 2 * nwords) ? 2 * b : 2 * nwords - first;
    for (uint32_t q = lane; q < count; q += 64) {
      const uint64_t dst = w0 + first + q;
      if (dst < cap_w32) gw32[dst] = w32[q];
    }
    wave_fence();
  }
}

// Clears the look-back state and ticket, and writes the complete blob of
// every empty column (no partitions, so no workgroup of k_encode sees it).
__global__ void k_encode_prepare(const EncColumn* __restrict__ cols, uint64_t ncols,
                                 EncColumn single, uint64_t* __restrict__ status,
                                 uint64_t nparts, unsigned long long* ticket, int* err) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  const uint64_t gid = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  for (uint64_t i = gid; i < nparts; i += stride) status[i] = 0;
  if (gid == 0) *ticket = 0;
  for (uint64_t i = gid; i < ncols; i += stride) {
    const EncColumn& c = cols ? cols[i] : single;
    if (c.m != 0) continue;
    finish_column(c, 0, err);  // also writes starts[0] = 0 of a variable column
  }
}

hipError_t launch_encode_columns(leco_ctx* ctx, const EncColumn* cols_dev, uint64_t ncols,
                                 const EncColumn& single, uint64_t nparts, uint64_t max_len,
                                 uint64_t* status, unsigned long long* ticket,
                                 hipStream_t stream) {
  const uint64_t pg = (nparts + 255) / 256;
  const uint64_t cg = (ncols + 255) / 256;
  uint64_t g = pg > cg ? pg : cg;
  if (g == 0) g = 1;
  if (g > 4096) g = 4096;
  hipLaunchKernelGGL(k_encode_prepare, dim3(uint32_t(g)), dim3(256), 0, stream, cols_dev, ncols,
                     single, status, nparts, ticket, ctx->err_dev);
  if (nparts == 0) return hipGetLastError();
  unsigned long long* tk = ctx->tune.encode_ticket ? ticket : nullptr;
  if (max_len <= kWaveEncMax && ctx->tune.encode_wave)
    hipLaunchKernelGGL(k_encode_wave, dim3(uint32_t((nparts + kEncWaves - 1) / kEncWaves)),
                       dim3(kEncBlock), 0, stream, cols_dev, ncols, single, status, tk, nparts,
                       ctx->err_dev);
  else
    hipLaunchKernelGGL(k_encode, dim3(uint32_t(nparts)), dim3(kEncBlock), 0, stream, cols_dev,
                       ncols, single, status, tk, ctx->err_dev);
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
