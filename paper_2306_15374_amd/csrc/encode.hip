// LeCo encoder kernels for gfx950 (section 3.1 regressor, section 3.3
// encoder): per-partition exact least-squares fit and residual width, an
// exclusive scan of the word counts, and word-centric bit-packing (one
// writer per 64-bit word, so the bytes are deterministic).
#include "internal.hpp"
#include "leco_dev.hpp"

namespace leco {

constexpr int kFitBlock = 256;
constexpr int kFitRegs = 16;  // values kept in registers per thread (4096 per partition)

__device__ inline uint64_t load_value(const uint8_t* col, uint32_t dtype, uint64_t i) {
  return dtype == 8 ? reinterpret_cast<const uint64_t*>(col)[i]
                    : uint64_t(reinterpret_cast<const uint32_t*>(col)[i]);
}

struct PartBounds {
  uint64_t start, len;
};

__device__ inline PartBounds enc_bounds(uint64_t j, uint64_t n, uint64_t fixed_len,
                                        const uint64_t* starts) {
  if (fixed_len) {
    const uint64_t s = j * fixed_len;
    const uint64_t e = s + fixed_len < n ? s + fixed_len : n;
    return {s, e - s};
  }
  return {starts[j], starts[j + 1] - starts[j]};
}

// ---- workgroup reductions (256 threads, LDS trees) -------------------------

struct FitScratch {
  uint64_t a[kFitBlock], b[kFitBlock], c[kFitBlock], d[kFitBlock], e[kFitBlock], f[kFitBlock];
  // results broadcast by thread 0
  uint64_t vmin, vmax;
  double theta1;
  int do_fit;
};

// min/max of u64 and two exact u128 sums.
__device__ void reduce_pass1(FitScratch& s, uint64_t& vmin, uint64_t& vmax, U128& sv, U128& stv) {
  const uint32_t tid = threadIdx.x;
  s.a[tid] = vmin;
  s.b[tid] = vmax;
  s.c[tid] = sv.lo;
  s.d[tid] = sv.hi;
  s.e[tid] = stv.lo;
  s.f[tid] = stv.hi;
  __syncthreads();
  for (uint32_t w = kFitBlock / 2; w > 0; w >>= 1) {
    if (tid < w) {
      s.a[tid] = s.a[tid] < s.a[tid + w] ? s.a[tid] : s.a[tid + w];
      s.b[tid] = s.b[tid] > s.b[tid + w] ? s.b[tid] : s.b[tid + w];
      U128 x = add128(U128{s.c[tid], s.d[tid]}, U128{s.c[tid + w], s.d[tid + w]});
      s.c[tid] = x.lo;
      s.d[tid] = x.hi;
      U128 y = add128(U128{s.e[tid], s.f[tid]}, U128{s.e[tid + w], s.f[tid + w]});
      s.e[tid] = y.lo;
      s.f[tid] = y.hi;
    }
    __syncthreads();
  }
  vmin = s.a[0];
  vmax = s.b[0];
  sv = U128{s.c[0], s.d[0]};
  stv = U128{s.e[0], s.f[0]};
}

__device__ void reduce_minmax_i64(FitScratch& s, int64_t& rmin, int64_t& rmax) {
  const uint32_t tid = threadIdx.x;
  __syncthreads();
  s.a[tid] = uint64_t(rmin);
  s.b[tid] = uint64_t(rmax);
  __syncthreads();
  for (uint32_t w = kFitBlock / 2; w > 0; w >>= 1) {
    if (tid < w) {
      const int64_t x = int64_t(s.a[tid]), y = int64_t(s.a[tid + w]);
      s.a[tid] = uint64_t(x < y ? x : y);
      const int64_t u = int64_t(s.b[tid]), v = int64_t(s.b[tid + w]);
      s.b[tid] = uint64_t(u > v ? u : v);
    }
    __syncthreads();
  }
  rmin = int64_t(s.a[0]);
  rmax = int64_t(s.b[0]);
}

// Least-squares slope from exact sums over raw values v_t.  With
// y_t = v_t - c for any constant c, n*S_ty - S_t*S_y equals
// n*S_tv - S_t*S_v, so N is formed from the raw sums modulo 2^128; its true
// magnitude is below 2^121, so the wrapped result is exact.
__device__ double ls_slope(uint64_t len, U128 sv, U128 stv) {
  const uint64_t st = len * (len - 1) / 2;                     // < 2^39
  const uint64_t stt = ((len - 1) * len / 2) * (2 * len - 1) / 3;  // < 2^61, exact
  const U128 N = sub128(mul128x64(stv, len), mul128x64(sv, st));
  const U128 D = sub128(mul64x64(len, stt), mul64x64(st, st));
  double slope = i128_to_f64(N) / u128_to_f64(D);
  if (slope == 0.0) slope = 0.0;  // +0.0, never -0.0
  return slope;
}

__global__ __launch_bounds__(kFitBlock) void k_fit(const uint8_t* __restrict__ col, uint64_t n,
                                                   uint32_t dtype, uint64_t fixed_len,
                                                   const uint64_t* __restrict__ starts, uint64_t m,
                                                   int force_constant,
                                                   PartModel* __restrict__ models) {
  __shared__ FitScratch s;
  const uint32_t tid = threadIdx.x;
  for (uint64_t j = blockIdx.x; j < m; j += gridDim.x) {
    const PartBounds pb = enc_bounds(j, n, fixed_len, starts);
    const uint64_t len = pb.len;
    const uint8_t* base_ptr = col + pb.start * dtype;
    const bool in_regs = len <= uint64_t(kFitBlock) * kFitRegs;
    uint64_t regs[kFitRegs];

    // Pass 1: range and exact sums.
    uint64_t vmin = ~uint64_t(0), vmax = 0;
    U128 sv{0, 0}, stv{0, 0};
    if (in_regs) {
#pragma unroll
      for (int k = 0; k < kFitRegs; ++k) {
        const uint32_t t = tid + k * kFitBlock;
        if (t < len) {
          const uint64_t v = load_value(base_ptr, dtype, t);
          regs[k] = v;
          vmin = v < vmin ? v : vmin;
          vmax = v > vmax ? v : vmax;
          sv = add128(sv, U128{v, 0});
          stv = add128(stv, mul64x64(t, v));
        }
      }
    } else {
      for (uint64_t t = tid; t < len; t += kFitBlock) {
        const uint64_t v = load_value(base_ptr, dtype, t);
        vmin = v < vmin ? v : vmin;
        vmax = v > vmax ? v : vmax;
        sv = add128(sv, U128{v, 0});
        stv = add128(stv, mul64x64(t, v));
      }
    }
    reduce_pass1(s, vmin, vmax, sv, stv);
    const uint64_t range = vmax - vmin;
    const uint32_t b_for = bitlen64(range);
    const bool fit = !(len == 1 || force_constant || range >= (uint64_t(1) << 61));

    PartModel pm;
    pm.base = vmin;
    pm.theta1 = 0.0;
    pm.bits = b_for;
    pm.pad = 0;
    if (fit) {
      if (tid == 0) s.theta1 = ls_slope(len, sv, stv);
      __syncthreads();
      const double th = s.theta1;
      // Pass 2: residual range of the linear model.
      int64_t rmin = INT64_MAX, rmax = INT64_MIN;
      if (in_regs) {
#pragma unroll
        for (int k = 0; k < kFitRegs; ++k) {
          const uint32_t t = tid + k * kFitBlock;
          if (t < len) {
            const int64_t r = int64_t(regs[k] - vmin) - predict(th, t);
            rmin = r < rmin ? r : rmin;
            rmax = r > rmax ? r : rmax;
          }
        }
      } else {
        for (uint64_t t = tid; t < len; t += kFitBlock) {
          const int64_t r = int64_t(load_value(base_ptr, dtype, t) - vmin) - predict(th, uint32_t(t));
          rmin = r < rmin ? r : rmin;
          rmax = r > rmax ? r : rmax;
        }
      }
      reduce_minmax_i64(s, rmin, rmax);
      const uint32_t b_ls = bitlen64(uint64_t(rmax) - uint64_t(rmin));
      if (b_ls < b_for) {  // ties keep the constant model
        pm.base = vmin + uint64_t(rmin);
        pm.theta1 = th;
        pm.bits = b_ls;
      }
    }
    pm.nwords = (len * pm.bits + 63) >> 6;
    if (tid == 0) models[j] = pm;
    __syncthreads();
  }
}

// ---- word-offset scan ---------------------------------------------------------

constexpr int kScanBlock = 256;
constexpr int kScanItems = 16;
constexpr uint64_t kScanTile = uint64_t(kScanBlock) * kScanItems;

__device__ uint64_t block_exclusive_scan(uint64_t x, uint64_t* sh, uint64_t& total) {
  const uint32_t tid = threadIdx.x;
  sh[tid] = x;
  __syncthreads();
  for (uint32_t off = 1; off < kScanBlock; off <<= 1) {
    const uint64_t y = tid >= off ? sh[tid - off] : 0;
    __syncthreads();
    sh[tid] += y;
    __syncthreads();
  }
  total = sh[kScanBlock - 1];
  const uint64_t incl = sh[tid];
  __syncthreads();
  return incl - x;
}

__global__ __launch_bounds__(kScanBlock) void k_scan_partial(const PartModel* __restrict__ models,
                                                             uint64_t m, uint64_t* partial) {
  __shared__ uint64_t sh[kScanBlock];
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile + uint64_t(threadIdx.x) * kScanItems;
  uint64_t x = 0;
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < m) x += models[base + k].nwords;
  uint64_t total;
  block_exclusive_scan(x, sh, total);
  if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Exclusive scan of the per-tile sums in place (one workgroup, looping with
// a running carry), then the blob size and the capacity check.
__global__ __launch_bounds__(kScanBlock) void k_scan_top(uint64_t* partial, uint64_t nb,
                                                         uint64_t words_off, uint64_t cap,
                                                         uint64_t* total_words, uint64_t* size_out,
                                                         int* err) {
  __shared__ uint64_t sh[kScanBlock];
  uint64_t carry = 0;
  for (uint64_t c = 0; c < nb; c += kScanBlock) {
    const uint64_t i = c + threadIdx.x;
    const uint64_t x = i < nb ? partial[i] : 0;
    uint64_t total;
    const uint64_t ex = block_exclusive_scan(x, sh, total);
    if (i < nb) partial[i] = carry + ex;
    carry += total;
  }
  if (threadIdx.x == 0) {
    const uint64_t size = align16(words_off + 8 * carry);
    *total_words = carry;
    *size_out = size;
    if (size > cap) atomicOr(err, kErrNoSpace);
  }
}

// Word offsets of every partition, then (when the blob fits) its records,
// header, starts and padding.
__global__ __launch_bounds__(kScanBlock) void k_scan_final(
    const PartModel* __restrict__ models, uint64_t m, const uint64_t* __restrict__ partial,
    uint64_t* __restrict__ word_off, uint8_t* __restrict__ blob, uint64_t cap,
    const uint64_t* __restrict__ total_words, const uint64_t* __restrict__ size_in, uint64_t n,
    uint32_t dtype, uint64_t fixed_len, const uint64_t* __restrict__ starts, uint64_t words_off) {
  __shared__ uint64_t sh[kScanBlock];
  const uint64_t size = *size_in;
  const bool fits = size <= cap;
  const uint64_t base = uint64_t(blockIdx.x) * kScanTile + uint64_t(threadIdx.x) * kScanItems;
  uint64_t x = 0;
  for (int k = 0; k < kScanItems; ++k)
    if (base + k < m) x += models[base + k].nwords;
  uint64_t total;
  uint64_t off = block_exclusive_scan(x, sh, total) + (blockIdx.x < gridDim.x && m ? partial[blockIdx.x] : 0);
  for (int k = 0; k < kScanItems; ++k) {
    const uint64_t j = base + k;
    if (j >= m) break;
    const PartModel pm = models[j];
    word_off[j] = off;
    if (fits) {
      uint64_t* r = reinterpret_cast<uint64_t*>(blob + kHeaderBytes + kRecordBytes * j);
      r[0] = pm.base;
      r[1] = uint64_t(__double_as_longlong(pm.theta1));
      r[2] = off;
      r[3] = uint64_t(pm.bits & 0xff);
    }
    off += pm.nwords;
  }
  if (!fits) return;
  const bool variable = fixed_len == 0;
  const uint64_t meta_end = kHeaderBytes + kRecordBytes * m + (variable ? 8 * (m + 1) : 0);
  const uint64_t tw = *total_words;
  if (variable) {
    uint64_t* sdst = reinterpret_cast<uint64_t*>(blob + kHeaderBytes + kRecordBytes * m);
    for (uint64_t i = uint64_t(blockIdx.x) * kScanBlock + threadIdx.x; i <= m;
         i += uint64_t(gridDim.x) * kScanBlock)
      sdst[i] = starts[i];
  }
  if (blockIdx.x == 0) {
    // zero padding before the words and after the last word
    for (uint64_t i = meta_end + threadIdx.x; i < words_off; i += kScanBlock) blob[i] = 0;
    for (uint64_t i = words_off + 8 * tw + threadIdx.x; i < size; i += kScanBlock) blob[i] = 0;
    if (threadIdx.x == 0) {
      uint64_t* hd = reinterpret_cast<uint64_t*>(blob);
      hd[0] = uint64_t(kMagic) | (uint64_t(kVersion) << 32) | (uint64_t(dtype) << 48) |
              (uint64_t(variable ? 1 : 0) << 56);
      hd[1] = n;
      hd[2] = m;
      hd[3] = fixed_len;
      hd[4] = kHeaderBytes;
      hd[5] = variable ? kHeaderBytes + kRecordBytes * m : 0;
      hd[6] = words_off;
      hd[7] = tw;
    }
  }
}

// ---- bit-packing -----------------------------------------------------------------

// Word w of partition j holds bits [64 w, 64 w + 64) of the partition's
// residual stream; residual t occupies bits [b t, b t + b).  Each thread
// assembles whole words from the residuals that overlap them.
__global__ __launch_bounds__(256) void k_pack(const uint8_t* __restrict__ col, uint64_t n,
                                              uint32_t dtype, uint64_t fixed_len,
                                              const uint64_t* __restrict__ starts, uint64_t m,
                                              const PartModel* __restrict__ models,
                                              const uint64_t* __restrict__ word_off,
                                              uint8_t* __restrict__ blob, uint64_t cap,
                                              const uint64_t* __restrict__ size_in,
                                              uint64_t words_off) {
  if (*size_in > cap) return;
  uint64_t* words = reinterpret_cast<uint64_t*>(blob + words_off);
  for (uint64_t j = blockIdx.x; j < m; j += gridDim.x) {
    const PartModel pm = models[j];
    const uint32_t b = pm.bits;
    if (b == 0) continue;
    const PartBounds pb = enc_bounds(j, n, fixed_len, starts);
    const uint8_t* src = col + pb.start * dtype;
    const uint64_t wbase = word_off[j];
    for (uint64_t w = threadIdx.x; w < pm.nwords; w += blockDim.x) {
      const uint32_t bit0 = uint32_t(64 * w);  // < 2^26: partitions hold <= 2^20 values
      uint64_t t = bit0 / b;
      uint64_t t_last = (bit0 + 63) / b;
      if (t_last >= pb.len) t_last = pb.len - 1;
      uint64_t word = 0;
      for (; t <= t_last; ++t) {
        const uint64_t u = load_value(src, dtype, t) - pm.base -
                           uint64_t(predict(pm.theta1, uint32_t(t)));
        const int64_t off = int64_t(b * t) - int64_t(bit0);
        word |= off >= 0 ? (u << off) : (u >> -off);
      }
      words[wbase + w] = word;
    }
  }
}

// ---- launcher ---------------------------------------------------------------------

hipError_t launch_encode(leco_ctx* ctx, const EncodePlan& pl, hipStream_t stream) {
  const uint64_t m = pl.m;
  const uint64_t fit_cap = uint64_t(ctx->num_cus) * 8;
  if (m > 0) {
    const uint64_t g = m < fit_cap ? m : fit_cap;
    hipLaunchKernelGGL(k_fit, dim3(uint32_t(g)), dim3(kFitBlock), 0, stream,
                       static_cast<const uint8_t*>(pl.col), pl.n, pl.dtype, pl.fixed_len,
                       pl.starts_dev, m, pl.force_constant, pl.models);
  }
  const uint64_t nb = (m + kScanTile - 1) / kScanTile;
  if (nb > 0)
    hipLaunchKernelGGL(k_scan_partial, dim3(uint32_t(nb)), dim3(kScanBlock), 0, stream,
                       pl.models, m, pl.partial);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(kScanBlock), 0, stream, pl.partial, nb,
                     pl.words_off, pl.cap, pl.total_words, pl.size_dev, ctx->err_dev);
  const uint64_t nf = nb > 0 ? nb : 1;
  hipLaunchKernelGGL(k_scan_final, dim3(uint32_t(nf)), dim3(kScanBlock), 0, stream, pl.models, m,
                     pl.partial, pl.word_off, static_cast<uint8_t*>(pl.blob), pl.cap,
                     pl.total_words, pl.size_dev, pl.n, pl.dtype, pl.fixed_len, pl.starts_dev,
                     pl.words_off);
  if (m > 0) {
    const uint64_t g = m < fit_cap ? m : fit_cap;
    hipLaunchKernelGGL(k_pack, dim3(uint32_t(g)), dim3(256), 0, stream,
                       static_cast<const uint8_t*>(pl.col), pl.n, pl.dtype, pl.fixed_len,
                       pl.starts_dev, m, pl.models, pl.word_off, static_cast<uint8_t*>(pl.blob),
                       pl.cap, pl.size_dev, pl.words_off);
  }
  return hipGetLastError();
}

}  // namespace leco

// ---- diagnostics --------------------------------------------------------------

namespace leco {

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
