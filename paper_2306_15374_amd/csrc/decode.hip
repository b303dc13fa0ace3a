// LeCo decoder kernels for gfx950 (section 3.3): full and range decode,
// random access, and the range-filter sum with model-bound pruning
// (section 5.1).  Launch helpers at the bottom are called by the C ABI.
#include "decode_tile.hpp"
#include "internal.hpp"

namespace leco {


// Decode positions [begin, end) into out[g - begin].  Tile k of the launch
// covers [(first_tile + k) * 2^tile_log2, ...) clipped to [begin, end); a
// workgroup walks tiles vb, vb + grid, ... (vb: its XCD-aware index).  With
// `all` set, end is taken from the header and checked against out_cap.
template <typename OutT>
__device__ void decode_tiles(const uint8_t* __restrict__ blob, const Header& h,
                             OutT* __restrict__ out, uint64_t begin, uint64_t e,
                             uint32_t tile_log2, uint64_t num_tiles, bool remap, uint32_t* stage,
                             int* err) {
  StoreSink<OutT> sink{out, begin};
  const uint64_t first = begin >> tile_log2;
  for (uint64_t k = xcd_virtual_block(blockIdx.x, gridDim.x, remap); k < num_tiles;
       k += gridDim.x) {
    uint64_t t0 = (first + k) << tile_log2;
    uint64_t t1 = t0 + (uint64_t(1) << tile_log2);
    if (t0 < begin) t0 = begin;
    if (t1 > e) t1 = e;
    if (t0 >= t1) break;
    uint64_t g0, g1;
    wave_share(t0, t1, tile_log2, g0, g1);
    if (g0 < g1 && !decode_tile(blob, h, g0, g1, stage, sink)) {
      if (lane_id() == 0) raise(err, kErrFormat);
      return;  // no workgroup barrier follows
    }
  }
}

// The tiles of decode_tiles for a blob with coefficient section, each
// wavefront's share decoded value by value.
template <typename OutT>
__device__ void decode_tiles_poly(const uint8_t* __restrict__ blob, const Header& h,
                                  OutT* __restrict__ out, uint64_t begin, uint64_t e,
                                  uint32_t tile_log2, uint64_t num_tiles, uint32_t* stage,
                                  int* err) {
  StoreSink<OutT> sink{out, begin};
  const uint64_t first = begin >> tile_log2;
  for (uint64_t k = blockIdx.x; k < num_tiles; k += gridDim.x) {
    uint64_t t0 = (first + k) << tile_log2;
    uint64_t t1 = t0 + (uint64_t(1) << tile_log2);
    if (t0 < begin) t0 = begin;
    if (t1 > e) t1 = e;
    if (t0 >= t1) break;
    uint64_t g0, g1;
    wave_share(t0, t1, tile_log2, g0, g1);
    if (g0 < g1 && !decode_range_poly(blob, h, g0, g1, stage, sink)) {
      if (lane_id() == 0) raise(err, kErrFormat);
      return;
    }
  }
}

// Six waves per SIMD: the register allocator is held to 80 VGPRs, which
// the decode paths fit without spilling.
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_decode(
    const uint8_t* __restrict__ blob, uint64_t blob_bytes, uint8_t* __restrict__ out,
    uint64_t begin, uint64_t end, uint64_t out_cap, uint32_t tile_log2, uint64_t num_tiles,
    int all, int remap, int* err) {
  constexpr uint32_t kSlot = slot_words<StoreSink<uint64_t>>();
  __shared__ uint4 stage_v[kWavesPerBlock * kSlot / 4];
  uint32_t* stage = reinterpret_cast<uint32_t*>(stage_v) + wave_id() * kSlot;
  Header h;
  if (!load_header(blob, blob_bytes, h)) {
    if (threadIdx.x == 0 && blockIdx.x == 0) raise(err, kErrFormat);
    return;
  }
  uint64_t e = end;
  if (all) {
    if (h.n > out_cap) {
      if (threadIdx.x == 0 && blockIdx.x == 0) raise(err, kErrNoSpace);
      return;
    }
    e = h.n;
  } else if (end > h.n) {
    if (threadIdx.x == 0 && blockIdx.x == 0) raise(err, kErrRange);
    return;
  }
  if (h.poly) {
    if (h.dtype == 8)
      decode_tiles_poly(blob, h, reinterpret_cast<uint64_t*>(out), begin, e, tile_log2, num_tiles,
                        stage, err);
    else
      decode_tiles_poly(blob, h, reinterpret_cast<uint32_t*>(out), begin, e, tile_log2, num_tiles,
                        stage, err);
    return;
  }
  if (h.dtype == 8)
    decode_tiles(blob, h, reinterpret_cast<uint64_t*>(out), begin, e, tile_log2, num_tiles,
                 remap != 0, stage, err);
  else
    decode_tiles(blob, h, reinterpret_cast<uint32_t*>(out), begin, e, tile_log2, num_tiles,
                 remap != 0, stage, err);
}

// ---- random access -------------------------------------------------------------

// kLpt positions per lane, strided by the workgroup size so that position
// loads and output stores stay coalesced; the lane issues all record loads,
// then all word loads, so up to 2 kLpt independent loads are in flight.
template <int kLpt>
__global__ __launch_bounds__(kBlock) void k_random_access(const uint8_t* __restrict__ blob,
                                                          uint64_t blob_bytes,
                                                          const uint64_t* __restrict__ pos,
                                                          uint64_t k, uint8_t* __restrict__ out,
                                                          int* err) {
  Header h;
  if (!load_header(blob, blob_bytes, h)) {
    if (threadIdx.x == 0 && blockIdx.x == 0) raise(err, kErrFormat);
    return;
  }
  const uint64_t i0 = uint64_t(blockIdx.x) * (kBlock * kLpt) + threadIdx.x;
  if (h.poly) {
    for (int r = 0; r < kLpt; ++r) {
      const uint64_t i = i0 + uint64_t(r) * kBlock;
      if (i >= k) break;
      const uint64_t g = pos[i];
      uint64_t v = 0;
      if (g >= h.n) raise(err, kErrRange);
      else if (!lookup_value_poly(blob, h, g, v)) raise(err, kErrFormat);
      if (h.dtype == 8)
        reinterpret_cast<uint64_t*>(out)[i] = v;
      else
        reinterpret_cast<uint32_t*>(out)[i] = uint32_t(v);
    }
    return;
  }
  const uint64_t* words = reinterpret_cast<const uint64_t*>(blob + h.words_off);
  uint64_t g[kLpt];
  bool ok[kLpt];
#pragma unroll
  for (int r = 0; r < kLpt; ++r) {
    const uint64_t i = i0 + uint64_t(r) * kBlock;
    g[r] = i < k ? pos[i] : 0;
    ok[r] = i < k;
  }
  uint4 r0[kLpt], r1[kLpt];
  uint64_t start[kLpt], len[kLpt];
  bool bad = false;
#pragma unroll
  for (int r = 0; r < kLpt; ++r) {
    if (ok[r] && g[r] >= h.n) {
      raise(err, kErrRange);
      ok[r] = false;
    }
    const uint64_t j = ok[r] ? locate(blob, h, g[r]) : 0;
    start[r] = 0;
    len[r] = 0;
    if (ok[r]) {
      const uint4* rec = reinterpret_cast<const uint4*>(blob + kHeaderBytes + kRecordBytes * j);
      r0[r] = rec[0];
      r1[r] = rec[1];
      start[r] = part_start(blob, h, j);
      len[r] = part_start(blob, h, j + 1) - start[r];
    }
  }
  uint64_t lo[kLpt], hi[kLpt];
  uint32_t sh[kLpt], bits[kLpt];
#pragma unroll
  for (int r = 0; r < kLpt; ++r) {
    lo[r] = hi[r] = 0;
    sh[r] = 0;
    bits[r] = 0;
    if (!ok[r]) continue;
    const uint64_t word_off = uint64_t(r1[r].x) | (uint64_t(r1[r].y) << 32);
    const uint32_t b = r1[r].z & 0xff;
    const uint64_t nwords = (len[r] * b + 63) >> 6;
    if (g[r] < start[r] || g[r] - start[r] >= len[r] || len[r] > kMaxPartLen || b > 8 * h.dtype ||
        word_off > h.total_words || nwords > h.total_words - word_off) {
      bad = true;
      ok[r] = false;
      continue;
    }
    bits[r] = b;
    if (b) {
      const uint64_t q = 64 * word_off + uint64_t(b) * (g[r] - start[r]);
      sh[r] = uint32_t(q & 63);
      lo[r] = words[q >> 6];
      if (sh[r] + b > 64) hi[r] = words[(q >> 6) + 1];
    }
  }
  if (bad) raise(err, kErrFormat);
#pragma unroll
  for (int r = 0; r < kLpt; ++r) {
    const uint64_t i = i0 + uint64_t(r) * kBlock;
    if (i >= k) continue;
    uint64_t v = 0;
    if (ok[r]) {
      const uint32_t b = bits[r];
      uint64_t u = (lo[r] >> sh[r]) | ((hi[r] << 1) << (63 - sh[r]));
      if (b < 64) u &= (uint64_t(1) << b) - 1;
      const uint64_t base = uint64_t(r0[r].x) | (uint64_t(r0[r].y) << 32);
      const double th = __longlong_as_double(
          static_cast<long long>(uint64_t(r0[r].z) | (uint64_t(r0[r].w) << 32)));
      v = base + uint64_t(predict(th, uint32_t(g[r] - start[r]))) + u;
    }
    if (h.dtype == 8)
      reinterpret_cast<uint64_t*>(out)[i] = v;
    else
      reinterpret_cast<uint32_t*>(out)[i] = uint32_t(v);
  }
}

// ---- range-filter sum ------------------------------------------------------

__global__ void k_zero_u64(uint64_t* p, uint64_t n) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += uint64_t(gridDim.x) * blockDim.x)
    p[i] = 0;
}

__global__ __launch_bounds__(kBlock) void k_filter_sum(const uint8_t* __restrict__ blob,
                                                       uint64_t blob_bytes, uint64_t lo,
                                                       uint64_t hi, uint64_t* out3,
                                                       uint32_t tile_log2, int prune, int* err) {
  constexpr uint32_t kSlot = slot_words<FilterSink>();
  __shared__ uint4 stage_v[kWavesPerBlock * kSlot / 4];
  uint32_t* stage = reinterpret_cast<uint32_t*>(stage_v) + wave_id() * kSlot;
  Header h;
  if (!load_header(blob, blob_bytes, h)) {
    if (threadIdx.x == 0 && blockIdx.x == 0) raise(err, kErrFormat);
    return;
  }
  FilterSink sink{lo, hi, 0, 0, 0, prune};
  bool bad = false;
  // Persistent grid: the tile count comes from the header.
  const uint64_t num_tiles = h.n == 0 ? 0 : ((h.n - 1) >> tile_log2) + 1;
  for (uint64_t k = blockIdx.x; k < num_tiles; k += gridDim.x) {
    const uint64_t t0 = k << tile_log2;
    uint64_t t1 = t0 + (uint64_t(1) << tile_log2);
    if (t1 > h.n) t1 = h.n;
    uint64_t g0, g1;
    wave_share(t0, t1, tile_log2, g0, g1);
    // blobs with polynomial partitions: every value decoded, no pruning
    if (!bad && g0 < g1 &&
        !(h.poly ? decode_range_poly(blob, h, g0, g1, stage, sink)
                 : decode_tile(blob, h, g0, g1, stage, sink)))
      bad = true;
  }
  if (bad && lane_id() == 0) raise(err, kErrFormat);
  block_add_sum(sink.sum_lo, sink.sum_hi, sink.count, out3);
}

// ---- diagnostics: streaming copy / fill for HBM calibration -----------------------

// 16 bytes per lane and iteration, four workgroups per CU (the fastest
// shape of a sweep over 1-16 bytes per lane, 256-1024 threads per
// workgroup and 2-32 workgroups per CU on MI355X: about 5.5 TB/s of
// read + write for a 2 GiB copy).
__global__ __launch_bounds__(256) void k_diag_copy(const uint4* __restrict__ src,
                                                   uint4* __restrict__ dst, uint64_t n16) {
  const uint64_t stride = uint64_t(gridDim.x) * blockDim.x;
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src ? src[i] : make_uint4(0, 0, 0, 0);
}

// ---- launchers ---------------------------------------------------------------

uint32_t pick_tile_log2(const Tune& t, uint64_t blob_bytes, uint64_t n) {
  if (t.tile_log2) return t.tile_log2;
  if (n == 0) return 12;
  // bits per value over the whole blob (records and padding included, so an
  // overestimate of the residual bits), with 1/16 slack for the per-partition
  // word alignment and 16 words for the first load's alignment
  const double bpv = 8.0 * double(blob_bytes) / double(n);
  uint32_t share_log2 = 12;
  while (share_log2 > 6 &&
         double(uint64_t(1) << share_log2) * bpv / 32.0 * 1.0625 + 16.0 > double(kWaveStageWords))
    --share_log2;
  return share_log2 + 2;
}

hipError_t launch_decode(leco_ctx* ctx, const void* blob, uint64_t blob_bytes, void* out,
                         uint64_t begin, uint64_t end, uint64_t out_cap, bool all,
                         hipStream_t stream) {
  const uint64_t e = all ? out_cap : end;
  // the total count is not known on the host: out_cap (decode_all) or end
  // (range) stands in for it
  const uint32_t tl = pick_tile_log2(ctx->tune, blob_bytes, e);
  if (!all && e <= begin) return hipSuccess;
  // decode_all always launches, so an empty output still checks n <= 0
  const uint64_t tiles = e <= begin ? 1 : ((e - 1) >> tl) - (begin >> tl) + 1;
  const uint64_t cap = uint64_t(ctx->num_cus) * ctx->tune.decode_blocks_per_cu;
  uint64_t grid = (cap == 0 || tiles < cap) ? tiles : cap;
  if (ctx->tune.xcd_remap) grid = (grid + 7) & ~uint64_t(7);
  hipLaunchKernelGGL(k_decode, dim3(uint32_t(grid)), dim3(kBlock), 0, stream,
                     static_cast<const uint8_t*>(blob), blob_bytes, static_cast<uint8_t*>(out),
                     begin, end, out_cap, tl, tiles, all ? 1 : 0, ctx->tune.xcd_remap ? 1 : 0,
                     ctx->err_dev);
  return hipGetLastError();
}

template <int kLpt>
static void launch_ra(const void* blob, uint64_t blob_bytes, const uint64_t* pos, uint64_t k,
                      void* out, int* err, hipStream_t stream) {
  const uint64_t per = uint64_t(kBlock) * kLpt;
  const uint64_t grid = (k + per - 1) / per;
  hipLaunchKernelGGL(k_random_access<kLpt>, dim3(uint32_t(grid)), dim3(kBlock), 0, stream,
                     static_cast<const uint8_t*>(blob), blob_bytes, pos, k,
                     static_cast<uint8_t*>(out), err);
}

hipError_t launch_random_access(leco_ctx* ctx, const void* blob, uint64_t blob_bytes,
                                const uint64_t* pos, uint64_t k, void* out, hipStream_t stream) {
  if (k == 0) return hipSuccess;
  switch (ctx->tune.ra_lookups_per_lane) {
    case 1: launch_ra<1>(blob, blob_bytes, pos, k, out, ctx->err_dev, stream); break;
    case 2: launch_ra<2>(blob, blob_bytes, pos, k, out, ctx->err_dev, stream); break;
    case 8: launch_ra<8>(blob, blob_bytes, pos, k, out, ctx->err_dev, stream); break;
    default: launch_ra<4>(blob, blob_bytes, pos, k, out, ctx->err_dev, stream); break;
  }
  return hipGetLastError();
}

hipError_t launch_zero_u64(uint64_t* p, uint64_t n, hipStream_t stream) {
  if (n == 0) return hipSuccess;
  const uint64_t grid = (n + 255) / 256 < 1024 ? (n + 255) / 256 : 1024;
  hipLaunchKernelGGL(k_zero_u64, dim3(uint32_t(grid)), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t launch_filter_sum(leco_ctx* ctx, const void* blob, uint64_t blob_bytes, uint64_t lo,
                             uint64_t hi, uint64_t* out3, bool prune, hipStream_t stream) {
  hipError_t e = launch_zero_u64(out3, 3, stream);
  if (e != hipSuccess) return e;
  // n is read on the device; the filter's segments are staged one by one,
  // so the tile only sets how the work is cut
  const uint32_t tl = ctx->tune.tile_log2 ? ctx->tune.tile_log2 : 12;
  const uint64_t grid = uint64_t(ctx->num_cus) * 4;
  hipLaunchKernelGGL(k_filter_sum, dim3(uint32_t(grid)), dim3(kBlock), 0, stream,
                     static_cast<const uint8_t*>(blob), blob_bytes, lo, hi, out3, tl,
                     prune ? 1 : 0, ctx->err_dev);
  return hipGetLastError();
}

hipError_t launch_diag_copy(leco_ctx* ctx, const void* src, void* dst, uint64_t bytes,
                            hipStream_t stream) {
  const uint64_t n16 = bytes / 16;
  if (n16 == 0) return hipSuccess;
  const uint64_t grid = uint64_t(ctx->num_cus) * 4;
  hipLaunchKernelGGL(k_diag_copy, dim3(uint32_t(grid)), dim3(256), 0, stream,
                     static_cast<const uint4*>(src), static_cast<uint4*>(dst), n16);
  return hipGetLastError();
}

}  // namespace leco
