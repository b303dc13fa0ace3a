// Device-side building blocks of the LeCo codec for gfx950: blob header and
// record access with in-kernel validation, exact 128-bit integer helpers,
// correctly rounded int128 -> binary64 conversion, and residual extraction.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace leco {

constexpr uint32_t kMagic = 0x4F43454Cu;  // bytes 'L','E','C','O'
constexpr uint32_t kVersion = 1;
constexpr uint64_t kHeaderBytes = 64;
constexpr uint64_t kRecordBytes = 32;
constexpr uint64_t kMaxPartLen = 1ull << 20;
// Header flag bits (byte 7).
constexpr uint32_t kFlagVariable = 1;  // starts section present
constexpr uint32_t kFlagPoly = 2;      // (c2, c3) coefficient section present
// Polynomial partitions: at most this many values, range below 2^50.
constexpr uint64_t kPolyMaxLen = 4096;
constexpr uint64_t kPolyMaxRange = 1ull << 50;

// Device error bits, reported by leco_sync.
constexpr int kErrRange = 1;
constexpr int kErrFormat = 2;
constexpr int kErrNoSpace = 4;
constexpr int kErrDevice = 8;  // a bounded wait gave up (never expected)

__host__ __device__ inline uint64_t align16(uint64_t x) { return (x + 15) & ~uint64_t(15); }

// Blob metadata (header, records, starts) is read through the constant
// address space: no kernel writes a blob while it decodes it, so loads whose
// address is uniform across the wavefront can use scalar loads, also when
// the blob pointer was itself read from a table in memory (batched and
// served decoding), and their results stay in scalar registers.
typedef const __attribute__((address_space(4))) uint64_t* MetaPtr;
__device__ inline MetaPtr meta_words(const uint8_t* blob, uint64_t byte_off) {
  return (MetaPtr)(blob + byte_off);
}

// Residual words and outputs live in global memory; saying so lets the
// compiler use global instead of flat loads and stores where the pointer
// came from a table in memory.
template <class T>
__device__ inline __attribute__((address_space(1))) T* global_ptr(T* p) {
  return (__attribute__((address_space(1))) T*)p;
}

struct Header {
  uint64_t n, m, fixed_len, starts_off, words_off, total_words;
  uint32_t dtype;     // 4 or 8
  uint32_t variable;  // 1 = variable-length partitions
  uint32_t poly;      // 1 = polynomial coefficient section present
  uint64_t coef_off;  // its offset (poly only)
};

// Reads and checks the 64-byte header against the caller-supplied blob size.
// Every later access of a kernel stays inside [0, blob_bytes) when this
// returns true and the per-record checks below pass.
__device__ inline bool load_header(const uint8_t* blob, uint64_t blob_bytes, Header& h) {
  if (blob_bytes < kHeaderBytes) return false;
  const MetaPtr q = meta_words(blob, 0);
  uint64_t w0 = q[0];
  h.n = q[1];
  h.m = q[2];
  h.fixed_len = q[3];
  uint64_t records_off = q[4];
  h.starts_off = q[5];
  h.words_off = q[6];
  h.total_words = q[7];
  uint32_t magic = uint32_t(w0);
  uint32_t version = uint32_t(w0 >> 32) & 0xffff;
  h.dtype = uint32_t(w0 >> 48) & 0xff;
  const uint32_t flags = uint32_t(w0 >> 56);
  h.variable = flags & kFlagVariable;
  h.poly = (flags & kFlagPoly) ? 1u : 0u;
  if (magic != kMagic || version != kVersion) return false;
  if (h.dtype != 4 && h.dtype != 8) return false;
  if (flags > (kFlagVariable | kFlagPoly) || records_off != kHeaderBytes) return false;
  if (h.m > blob_bytes / kRecordBytes) return false;
  uint64_t meta_end = kHeaderBytes + kRecordBytes * h.m;
  if (h.variable) {
    if (h.fixed_len != 0 || h.starts_off != meta_end) return false;
    if (h.m + 1 > blob_bytes / 8) return false;
    meta_end += 8 * (h.m + 1);
  } else {
    if (h.fixed_len == 0 || h.fixed_len > kMaxPartLen || h.starts_off != 0) return false;
    if (h.n / h.fixed_len + (h.n % h.fixed_len != 0) != h.m) return false;
  }
  h.coef_off = 0;
  if (h.poly) {
    h.coef_off = align16(meta_end);
    meta_end = h.coef_off + 16 * h.m;
  }
  if (h.words_off != align16(meta_end)) return false;
  if (h.total_words > blob_bytes / 8) return false;
  if (align16(h.words_off + 8 * h.total_words) > blob_bytes) return false;
  return true;
}

struct Part {
  uint64_t start, len;   // global index of t = 0 and partition length
  uint64_t base;         // integer intercept
  double theta1;         // slope
  uint64_t word_off;     // first word of the residual span
  uint32_t bits;         // residual width b
};

__device__ inline uint64_t part_start(const uint8_t* blob, const Header& h, uint64_t j) {
  if (h.variable) return meta_words(blob, h.starts_off)[j];
  uint64_t s = j * h.fixed_len;
  return s < h.n ? s : h.n;
}

// Loads partition j and checks it; false means the blob is corrupt.
__device__ inline bool load_part(const uint8_t* blob, const Header& h, uint64_t j, Part& p) {
  if (j >= h.m) return false;
  const MetaPtr r = meta_words(blob, kHeaderBytes + kRecordBytes * j);
  p.base = r[0];
  p.theta1 = __longlong_as_double(static_cast<long long>(r[1]));
  p.word_off = r[2];
  p.bits = uint32_t(r[3] & 0xff);
  p.start = part_start(blob, h, j);
  uint64_t end = part_start(blob, h, j + 1);
  if (end <= p.start || end > h.n || end - p.start > kMaxPartLen) return false;
  p.len = end - p.start;
  if (p.bits > 8 * h.dtype) return false;
  uint64_t words = (p.len * p.bits + 63) >> 6;
  if (p.word_off > h.total_words || words > h.total_words - p.word_off) return false;
  return true;
}

// Partition holding global index g: floor(g / L) for fixed partitions, the
// last start <= g for variable ones (binary search; the result is checked by
// the caller against the partition bounds).
__device__ inline uint64_t locate(const uint8_t* blob, const Header& h, uint64_t g) {
  if (!h.variable) {
    // floor(g / L) through a binary64 reciprocal, then exact correction.
    uint64_t L = h.fixed_len;
    uint64_t j = uint64_t(double(g) * (1.0 / double(L)));
    while (j > 0 && j * L > g) --j;
    while ((j + 1) * L <= g) ++j;
    return j;
  }
  const MetaPtr s = meta_words(blob, h.starts_off);
  uint64_t lo = 0, hi = h.m;  // answer in [lo, hi)
  while (hi - lo > 1) {
    uint64_t mid = lo + ((hi - lo) >> 1);
    if (s[mid] <= g) lo = mid; else hi = mid;
  }
  return lo;
}

// ---- exact integer helpers --------------------------------------------------

struct U128 {
  uint64_t lo, hi;
};

__device__ __host__ inline U128 add128(U128 a, U128 b) {
  U128 r;
  r.lo = a.lo + b.lo;
  r.hi = a.hi + b.hi + (r.lo < a.lo);
  return r;
}
__device__ __host__ inline U128 sub128(U128 a, U128 b) {
  U128 r;
  r.lo = a.lo - b.lo;
  r.hi = a.hi - b.hi - (a.lo < b.lo);
  return r;
}
__device__ inline U128 mul64x64(uint64_t a, uint64_t b) {
  U128 r;
  r.lo = a * b;
  r.hi = __umul64hi(a, b);
  return r;
}
// Low 128 bits of a 128 x 64 product.
__device__ inline U128 mul128x64(U128 a, uint64_t b) {
  U128 r = mul64x64(a.lo, b);
  r.hi += a.hi * b;
  return r;
}

__device__ inline uint32_t bitlen64(uint64_t x) { return x ? 64u - uint32_t(__clzll(x)) : 0u; }

// Correctly rounded (nearest-even) conversion of an unsigned 64-bit integer:
// the high and low halves convert exactly and their sum rounds once.
__device__ inline double u64_to_f64(uint64_t x) {
  double hi = double(uint32_t(x >> 32)) * 4294967296.0;
  double lo = double(uint32_t(x));
  return __dadd_rn(hi, lo);
}

// Correctly rounded conversion of an unsigned 128-bit integer.  Values of 65
// or more bits are shifted down to exactly 64 bits with every dropped bit
// ORed into bit 0 (a sticky bit below the rounding position, which lies 11
// bits down), converted, and scaled back by an exact power of two.
__device__ inline double u128_to_f64(U128 x) {
  if (x.hi == 0) return u64_to_f64(x.lo);
  uint32_t s = bitlen64(x.hi);  // 1..64 bits above the low word
  uint64_t kept = (s == 64) ? x.hi : ((x.hi << (64 - s)) | (x.lo >> s));
  uint64_t dropped = (s == 64) ? x.lo : (x.lo << (64 - s));
  kept |= (dropped != 0);
  return ldexp(u64_to_f64(kept), int(s));
}

// Correctly rounded conversion of a two's-complement 128-bit integer.
__device__ inline double i128_to_f64(U128 x) {
  bool neg = int64_t(x.hi) < 0;
  if (neg) x = sub128(U128{0, 0}, x);
  double m = u128_to_f64(x);
  return neg ? -m : m;
}

// floor(theta1 * t) as an integer: one binary64 multiply (no contraction
// is possible: nothing is added), an exact floor and an exact conversion.
__device__ inline int64_t predict(double theta1, uint32_t t) {
  double prod = __dmul_rn(theta1, double(t));
  return static_cast<int64_t>(floor(prod));
}
// Same when every |floor(theta1 * t)| of the partition is below 2^31.
__device__ inline int32_t predict32(double theta1, uint32_t t) {
  double prod = __dmul_rn(theta1, double(t));
  return static_cast<int32_t>(floor(prod));
}

// True when floor(theta1 * t) fits in int32 for every t < len.  Rounding is
// monotone, so |fl(theta1 * t)| <= fl(|theta1| * len) for t < len.
__device__ inline bool prediction_fits_i32(double theta1, uint64_t len) {
  return __dmul_rn(fabs(theta1), double(len)) < 2147483648.0;
}

// Polynomial prediction of a partition of n <= 4096 values: the Gram
// polynomials of the positions, g1 = 2t - (n-1), g2 = 6t^2 - 6(n-1)t +
// (n-1)(n-2), g3 = 20t^3 - 30(n-1)t^2 + (12n^2 - 30n + 22)t - (n-1)(n-2)(n-3),
// are integers below 2^37 in magnitude, and
//   p_t = floor(fl(fl(fl(c1 g1) + fl(c2 g2)) + fl(c3 g3))).
// The g_k are evaluated in binary64 in Horner form: for t, n <= 4096 every
// intermediate is an integer below 2^42, so each operation is exact and the
// values equal the integer polynomials.
__device__ inline int64_t poly_combine(double c1, double c2, double c3, double g1, double g2,
                                       double g3) {
  double s = __dadd_rn(__dmul_rn(c1, g1), __dmul_rn(c2, g2));
  s = __dadd_rn(s, __dmul_rn(c3, g3));
  return static_cast<int64_t>(floor(s));
}

__device__ inline int64_t poly_predict(double c1, double c2, double c3, uint32_t t, uint32_t n) {
  const double x = double(t), N = double(n), a = N - 1.0;
  const double g1 = __dadd_rn(__dmul_rn(2.0, x), -a);
  const double e2 = __dmul_rn(a, N - 2.0);
  const double g2 = __dadd_rn(__dmul_rn(__dadd_rn(__dmul_rn(6.0, x), __dmul_rn(-6.0, a)), x), e2);
  const double k3 = __dadd_rn(__dmul_rn(__dadd_rn(__dmul_rn(12.0, N), -30.0), N), 22.0);
  const double e3 = __dmul_rn(e2, N - 3.0);
  const double h3 = __dadd_rn(__dmul_rn(20.0, x), __dmul_rn(-30.0, a));
  const double g3 = __dadd_rn(__dmul_rn(__dadd_rn(__dmul_rn(h3, x), k3), x), -e3);
  return poly_combine(c1, c2, c3, g1, g2, g3);
}

// The same predictions at positions t, t + h, t + 2h, ... (a lane's
// positions, h its stride): the Gram polynomials advanced by forward
// differences.  With a = n - 1, their first differences are 2h,
// 12ht + 6h^2 - 6ah and 60ht^2 + (60h^2 - 60ah)t + 20h^3 - 30ah^2 + k3 h,
// the second 12h^2 and 120h^2 t + 120h^3 - 60ah^2, the third 120h^3.  For
// n <= 4096, h <= 256 and positions below n + 3h every value, difference
// and product here is an integer below 2^53, so each step is exact and
// gives the g1, g2, g3 that poly_predict evaluates.
struct GramWalk {
  double g1, g2, g3, d1, d2, dd2, d3, dd3, ddd3;

  __device__ void start(uint32_t t, uint32_t n, uint32_t h) {
    const double x = double(t), N = double(n), a = N - 1.0, H = double(h);
    const double e2 = a * (N - 2.0);
    const double k3 = (12.0 * N - 30.0) * N + 22.0;
    const double e3 = e2 * (N - 3.0);
    g1 = 2.0 * x - a;
    g2 = (6.0 * x - 6.0 * a) * x + e2;
    g3 = ((20.0 * x - 30.0 * a) * x + k3) * x - e3;
    const double H2 = H * H, H3 = H2 * H;
    d1 = 2.0 * H;
    d2 = 12.0 * H * x + (6.0 * H2 - 6.0 * a * H);
    dd2 = 12.0 * H2;
    d3 = (60.0 * H * x + (60.0 * H2 - 60.0 * a * H)) * x + (20.0 * H3 - 30.0 * a * H2 + k3 * H);
    dd3 = 120.0 * H2 * x + (120.0 * H3 - 60.0 * a * H2);
    ddd3 = 120.0 * H3;
  }
  __device__ int64_t predict(double c1, double c2, double c3) const {
    return poly_combine(c1, c2, c3, g1, g2, g3);
  }
  __device__ void next() {
    g1 += d1;
    g2 += d2;
    d2 += dd2;
    g3 += d3;
    d3 += dd3;
    dd3 += ddd3;
  }
};

// ---- residual extraction from 32-bit words ---------------------------------

// Width-b field at bit q of a little-endian stream held as 32-bit words,
// b <= 32: funnel shift of two consecutive words.
__device__ inline uint32_t extract32(const uint32_t* w, uint32_t q, uint32_t mask) {
  uint32_t i = q >> 5;
  return __builtin_amdgcn_alignbit(w[i + 1], w[i], q & 31) & mask;
}
// Width-b field, 32 < b <= 64: three consecutive words.
__device__ inline uint64_t extract64(const uint32_t* w, uint32_t q, uint32_t mask_hi) {
  uint32_t i = q >> 5, s = q & 31;
  uint32_t w0 = w[i], w1 = w[i + 1], w2 = w[i + 2];
  uint32_t lo = __builtin_amdgcn_alignbit(w1, w0, s);
  uint32_t hi = __builtin_amdgcn_alignbit(w2, w1, s) & mask_hi;
  return (uint64_t(hi) << 32) | lo;
}

}  // namespace leco
