// Model fitting shared by the encoder and the partitioner (section 3.1):
// the least-squares slope from exact integer sums, the residual width, and
// the choice between the fitted line and the constant model, with
// workgroup-wide reductions over 256 threads.  The reductions take any
// shared-memory struct with a `red[kEncWaves][4]` array and a `theta1` slot.
#pragma once

#include "leco_dev.hpp"

namespace leco {

constexpr int kEncBlock = 256;
constexpr int kEncWaves = kEncBlock / 64;

__device__ inline uint64_t load_value(const uint8_t* col, uint32_t dtype, uint64_t i) {
  return dtype == 8 ? reinterpret_cast<const uint64_t*>(col)[i]
                    : uint64_t(reinterpret_cast<const uint32_t*>(col)[i]);
}

// ---- workgroup reductions: wavefront shuffles, then one LDS slot per wave ----

__device__ inline uint64_t shfl_xor64(uint64_t x, int m) {
  return static_cast<uint64_t>(__shfl_xor(static_cast<unsigned long long>(x), m, 64));
}

// Wavefront-wide reductions (every lane receives the result, no barrier).
__device__ inline void wave_minmax_u64(uint64_t& mn, uint64_t& mx) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const uint64_t a = shfl_xor64(mn, m), b = shfl_xor64(mx, m);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
}

__device__ inline void wave_minmax_i64(int64_t& mn, int64_t& mx) {
  // order-preserving map of int64 onto uint64
  uint64_t a = uint64_t(mn) ^ (1ull << 63), b = uint64_t(mx) ^ (1ull << 63);
  wave_minmax_u64(a, b);
  mn = int64_t(a ^ (1ull << 63));
  mx = int64_t(b ^ (1ull << 63));
}

__device__ inline void wave_sum_u128x2(U128& x, U128& y) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    x = add128(x, U128{shfl_xor64(x.lo, m), shfl_xor64(x.hi, m)});
    y = add128(y, U128{shfl_xor64(y.lo, m), shfl_xor64(y.hi, m)});
  }
}

__device__ inline void wave_sum_u64x2(uint64_t& x, uint64_t& y) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    x += shfl_xor64(x, m);
    y += shfl_xor64(y, m);
  }
}

// Every thread receives the workgroup's min and max (two barriers).
template <class Sh>
__device__ inline void block_minmax_u64(Sh& sh, uint64_t& mn, uint64_t& mx) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    const uint64_t a = shfl_xor64(mn, m), b = shfl_xor64(mx, m);
    mn = a < mn ? a : mn;
    mx = b > mx ? b : mx;
  }
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh.red[wave][0] = mn;
    sh.red[wave][1] = mx;
  }
  __syncthreads();
#pragma unroll
  for (int w = 0; w < kEncWaves; ++w) {
    mn = sh.red[w][0] < mn ? sh.red[w][0] : mn;
    mx = sh.red[w][1] > mx ? sh.red[w][1] : mx;
  }
  __syncthreads();
}

template <class Sh>
__device__ inline void block_minmax_i64(Sh& sh, int64_t& mn, int64_t& mx) {
  // order-preserving map of int64 onto uint64
  uint64_t a = uint64_t(mn) ^ (1ull << 63), b = uint64_t(mx) ^ (1ull << 63);
  block_minmax_u64(sh, a, b);
  mn = int64_t(a ^ (1ull << 63));
  mx = int64_t(b ^ (1ull << 63));
}

// Exact workgroup sums of two unsigned 128-bit values.
template <class Sh>
__device__ inline void block_sum_u128x2(Sh& sh, U128& x, U128& y) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    x = add128(x, U128{shfl_xor64(x.lo, m), shfl_xor64(x.hi, m)});
    y = add128(y, U128{shfl_xor64(y.lo, m), shfl_xor64(y.hi, m)});
  }
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh.red[wave][0] = x.lo;
    sh.red[wave][1] = x.hi;
    sh.red[wave][2] = y.lo;
    sh.red[wave][3] = y.hi;
  }
  __syncthreads();
  x = U128{0, 0};
  y = U128{0, 0};
#pragma unroll
  for (int w = 0; w < kEncWaves; ++w) {
    x = add128(x, U128{sh.red[w][0], sh.red[w][1]});
    y = add128(y, U128{sh.red[w][2], sh.red[w][3]});
  }
  __syncthreads();
}

// Exact workgroup sums of two 64-bit values that cannot overflow.
template <class Sh>
__device__ inline void block_sum_u64x2(Sh& sh, uint64_t& x, uint64_t& y) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) {
    x += shfl_xor64(x, m);
    y += shfl_xor64(y, m);
  }
  const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    sh.red[wave][0] = x;
    sh.red[wave][1] = y;
  }
  __syncthreads();
  x = y = 0;
#pragma unroll
  for (int w = 0; w < kEncWaves; ++w) {
    x += sh.red[w][0];
    y += sh.red[w][1];
  }
  __syncthreads();
}

// Least-squares slope from exact sums S_y = sum y_t and S_ty = sum t y_t.
// Shifting every value by a constant c changes neither n S_ty - S_t S_y nor
// the slope, so the sums may be taken over v_t or over v_t - vmin; N is
// formed modulo 2^128 and its true magnitude is below 2^121, so it is exact.
__device__ inline double ls_slope(uint64_t len, U128 sv, U128 stv) {
  const uint64_t st = len * (len - 1) / 2;                         // < 2^39
  const uint64_t stt = ((len - 1) * len / 2) * (2 * len - 1) / 3;  // < 2^61, exact
  const U128 N = sub128(mul128x64(stv, len), mul128x64(sv, st));
  const U128 D = sub128(mul64x64(len, stt), mul64x64(st, st));
  double slope = i128_to_f64(N) / u128_to_f64(D);
  if (slope == 0.0) slope = 0.0;  // +0.0, never -0.0
  return slope;
}

// The slope computed once (by wave 0) and broadcast through LDS.
template <class Sh>
__device__ inline double block_slope(Sh& sh, uint64_t len, U128 sv, U128 stv) {
  if ((threadIdx.x >> 6) == 0) {
    const double th = ls_slope(len, sv, stv);
    if (threadIdx.x == 0) sh.theta1 = th;
  }
  __syncthreads();
  return sh.theta1;
}

// The model of one partition, identical in every thread of the workgroup.
struct Model {
  uint64_t vmin, base;
  double theta1;
  uint32_t bits;
  bool linear;
  int64_t rmin;
  uint64_t range;  // vmax - vmin
};

// Chooses between the constant model and the fitted line (ties keep the
// constant model, whose width never exceeds bitlen(vmax - vmin)).
__device__ inline void choose_model(Model& md, double th, int64_t rmin, int64_t rmax) {
  const uint32_t b_ls = bitlen64(uint64_t(rmax) - uint64_t(rmin));
  if (b_ls < md.bits) {
    md.linear = true;
    md.theta1 = th;
    md.base = md.vmin + uint64_t(rmin);
    md.bits = b_ls;
    md.rmin = rmin;
  }
}

}  // namespace leco
