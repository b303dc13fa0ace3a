// Batched LeCo decoding and encoding: one persistent decode launch over the
// tiles of thousands of columns (flattened into one table, mixed uint32 and
// uint64, optional fused range-filter sum), HIP-graph replay, a launch-shape
// tuner, and a one-launch encoder over a table of columns.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <string>
#include <vector>

#include "decode_tile.hpp"
#include "internal.hpp"

namespace leco {

// One column of a decode batch in device memory.  tile_base is the index of
// the column's first tile in the flattened table; its tiles hold
// 2^tile_log2 values each.
struct DecCol {
  const uint8_t* blob;
  uint64_t blob_bytes;
  uint64_t n;
  uint8_t* out;
  uint64_t lo, hi;
  uint64_t* sum3;
  uint64_t tile_base;
  uint32_t tile_log2, pad;
};

// Stores each value (when kStore) and accumulates the filter sum (when
// kFilter).  Pruning by model bounds is only possible when nothing is stored.
template <typename OutT, bool kStore, bool kFilter>
struct BatchSink {
  static constexpr bool kWholeTile = kStore;
  // runs of short partitions in full rounds when only storing: the fused
  // filter's accumulators would push the kernel past its register budget
  static constexpr bool kFlat = kStore && !kFilter;
  // polynomial predictions by forward differences (decode_range_poly) only
  // when storing alone, for the same reason
  static constexpr bool kGramWalk = kStore && !kFilter;
  OutT* out;
  FilterSink f;
  __device__ bool visit_segment(const Part& p, uint32_t t0, uint32_t t1) {
    return kStore ? true : f.visit_segment(p, t0, t1);
  }
  __device__ void put(uint64_t g, uint64_t v) {
    if (kStore) __builtin_nontemporal_store(OutT(v), global_ptr(out + g));
    if (kFilter) f.put(g, v);
  }
};

// Decodes this wavefront's share [g0, g1) of a column tile; with kFilter,
// every thread of the workgroup then joins the exact sum (a workgroup
// barrier, reached by all waves whatever their share held).
template <typename OutT, bool kStore, bool kFilter>
__device__ __attribute__((always_inline)) bool run_tile(const DecCol& c, const Header& h,
                                                        uint64_t g0, uint64_t g1,
                                                        uint32_t* stage) {
  BatchSink<OutT, kStore, kFilter> sink{reinterpret_cast<OutT*>(c.out),
                                        FilterSink{c.lo, c.hi, 0, 0, 0, kStore ? 0 : 1}};
  // blobs with polynomial partitions: value by value, every value decoded
  const bool ok = g0 >= g1 || (h.poly ? decode_range_poly(c.blob, h, g0, g1, stage, sink)
                                      : decode_tile(c.blob, h, g0, g1, stage, sink));
  if (kFilter) block_add_sum(sink.f.sum_lo, sink.f.sum_hi, sink.f.count, c.sum3);
  return ok;
}

// Six waves per SIMD: the register allocator is held to 80 VGPRs.
template <bool kStore, bool kFilter>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(6))) void k_batch_decode(
    const DecCol* __restrict__ cols, const uint32_t* __restrict__ tile_col, uint64_t total_tiles,
    int* err) {
  // (the sink's type does not depend on the column's width)
  constexpr uint32_t kSlot = slot_words<BatchSink<uint32_t, kStore, kFilter>>();
  __shared__ uint4 stage_v[kWavesPerBlock * kSlot / 4];
  uint32_t* stage = reinterpret_cast<uint32_t*>(stage_v) + wave_id() * kSlot;
  for (uint64_t k = blockIdx.x; k < total_tiles; k += gridDim.x) {
    const DecCol& c = cols[tile_col[k]];
    Header h;
    if (!load_header(c.blob, c.blob_bytes, h) || h.n != c.n) {
      if (threadIdx.x == 0) raise(err, kErrFormat);
      continue;
    }
    const uint32_t tile_log2 = c.tile_log2;
    const uint64_t t0 = (k - c.tile_base) << tile_log2;
    uint64_t t1 = t0 + (uint64_t(1) << tile_log2);
    if (t1 > c.n) t1 = c.n;
    uint64_t g0, g1;
    wave_share(t0, t1, tile_log2, g0, g1);
    const bool filter = kFilter && c.sum3 != nullptr;
    const bool store = kStore && c.out != nullptr;
    bool ok;
    if (h.dtype == 8) {
      if (store && filter) ok = run_tile<uint64_t, true, true>(c, h, g0, g1, stage);
      else if (store) ok = run_tile<uint64_t, true, false>(c, h, g0, g1, stage);
      else if (filter) ok = run_tile<uint64_t, false, true>(c, h, g0, g1, stage);
      else ok = true;
    } else {
      if (store && filter) ok = run_tile<uint32_t, true, true>(c, h, g0, g1, stage);
      else if (store) ok = run_tile<uint32_t, true, false>(c, h, g0, g1, stage);
      else if (filter) ok = run_tile<uint32_t, false, true>(c, h, g0, g1, stage);
      else ok = true;
    }
    if (!ok && lane_id() == 0) raise(err, kErrFormat);
  }
}

__global__ void k_batch_zero_sums(const DecCol* __restrict__ cols, uint64_t ncols) {
  for (uint64_t i = uint64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < ncols;
       i += uint64_t(gridDim.x) * blockDim.x) {
    uint64_t* s = cols[i].sum3;
    if (s) s[0] = s[1] = s[2] = 0;
  }
}

}  // namespace leco

// ---- host side ------------------------------------------------------------------

struct leco_batch {
  leco_ctx* ctx = nullptr;
  std::vector<leco_decode_job> jobs;
  leco::DecCol* cols_dev = nullptr;
  uint32_t* tile_col_dev = nullptr;  // column of every tile
  uint64_t tile_col_cap = 0;
  uint64_t total_tiles = 0;
  uint32_t tile_log2 = 0;  // 0 = each column's own, from its bits per value
  uint32_t blocks_per_cu = 0;
  hipStream_t capture_stream = nullptr;
  hipGraphExec_t graphs[4] = {nullptr, nullptr, nullptr, nullptr};
};

namespace {

leco_status bfail(leco_batch* b, leco_status st, const char* msg) {
  if (b && b->ctx) b->ctx->last_error = msg;
  return st;
}

void drop_graphs(leco_batch* b) {
  for (auto& g : b->graphs)
    if (g) {
      (void)hipGraphExecDestroy(g);
      g = nullptr;
    }
}

// Rebuilds and uploads the flattened tile table for the batch's tile size
// (or each column's own).
leco_status upload_table(leco_batch* b) {
  const uint64_t ncols = b->jobs.size();
  std::vector<leco::DecCol> cols(ncols);
  uint64_t tiles = 0;
  for (uint64_t i = 0; i < ncols; ++i) {
    const leco_decode_job& j = b->jobs[i];
    leco::DecCol& c = cols[i];
    c.blob = static_cast<const uint8_t*>(j.blob_dev);
    c.blob_bytes = j.blob_bytes;
    c.n = j.n;
    c.out = static_cast<uint8_t*>(j.out_dev);
    c.lo = j.lo;
    c.hi = j.hi;
    c.sum3 = j.sum3_dev;
    c.tile_base = tiles;
    c.tile_log2 = b->tile_log2 ? b->tile_log2 : leco::pick_tile_log2(leco::Tune{}, j.blob_bytes, j.n);
    c.pad = 0;
    tiles += (j.n + (uint64_t(1) << c.tile_log2) - 1) >> c.tile_log2;
  }
  b->total_tiles = tiles;
  if (ncols == 0) return LECO_OK;
  if (ncols > 0xffffffffull) return bfail(b, LECO_EINVAL, "too many columns in one batch");
  std::vector<uint32_t> tile_col(tiles ? tiles : 1);
  for (uint64_t i = 0; i < ncols; ++i) {
    const uint64_t end = i + 1 < ncols ? cols[i + 1].tile_base : tiles;
    for (uint64_t k = cols[i].tile_base; k < end; ++k) tile_col[k] = uint32_t(i);
  }
  if (!b->cols_dev && hipMalloc(&b->cols_dev, sizeof(leco::DecCol) * ncols) != hipSuccess)
    return bfail(b, LECO_ENOMEM, "batch table allocation failed");
  if (tile_col.size() > b->tile_col_cap) {
    if (b->tile_col_dev) (void)hipFree(b->tile_col_dev);
    b->tile_col_dev = nullptr;
    b->tile_col_cap = 0;
    if (hipMalloc(&b->tile_col_dev, 4 * tile_col.size()) != hipSuccess)
      return bfail(b, LECO_ENOMEM, "batch tile map allocation failed");
    b->tile_col_cap = tile_col.size();
  }
  if (hipMemcpy(b->cols_dev, cols.data(), sizeof(leco::DecCol) * ncols, hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(b->tile_col_dev, tile_col.data(), 4 * tile_col.size(), hipMemcpyHostToDevice) !=
          hipSuccess)
    return bfail(b, LECO_EDEVICE, "batch table upload failed");
  drop_graphs(b);
  return LECO_OK;
}

using BatchKernel = void (*)(const leco::DecCol*, const uint32_t*, uint64_t, int*);

BatchKernel batch_kernel(int op) {
  const bool filter = (op & LECO_BATCH_FILTER) != 0, store = (op & LECO_BATCH_DECODE) != 0;
  return store && filter ? leco::k_batch_decode<true, true>
         : store         ? leco::k_batch_decode<true, false>
                         : leco::k_batch_decode<false, true>;
}

hipError_t launch_batch(leco_batch* b, int op, hipStream_t stream) {
  const uint64_t ncols = b->jobs.size();
  if (ncols == 0) return hipSuccess;
  const bool filter = (op & LECO_BATCH_FILTER) != 0;
  if (filter) {
    const uint64_t g = (ncols + 255) / 256;
    hipLaunchKernelGGL(leco::k_batch_zero_sums, dim3(uint32_t(g < 1024 ? g : 1024)), dim3(256), 0,
                       stream, b->cols_dev, ncols);
  }
  if (b->total_tiles == 0) return hipGetLastError();
  const uint64_t cap = uint64_t(b->ctx->num_cus) * b->blocks_per_cu;
  const uint64_t grid = (cap == 0 || b->total_tiles < cap) ? b->total_tiles : cap;
  hipLaunchKernelGGL(batch_kernel(op), dim3(uint32_t(grid)), dim3(leco::kBlock), 0, stream,
                     b->cols_dev,
                     b->tile_col_dev, b->total_tiles, b->ctx->err_dev);
  return hipGetLastError();
}

bool valid_op(int op) { return op >= 1 && op <= 3; }

}  // namespace

extern "C" {

leco_status leco_batch_create(leco_ctx* ctx, const leco_decode_job* jobs, uint64_t ncols,
                              leco_batch** out) {
  if (!ctx || !out || (ncols && !jobs)) return LECO_EINVAL;
  *out = nullptr;
  for (uint64_t i = 0; i < ncols; ++i) {
    const leco_decode_job& j = jobs[i];
    if (!j.blob_dev || (reinterpret_cast<uintptr_t>(j.blob_dev) & 15) || j.blob_bytes < 64) {
      ctx->last_error = "batch job with a null, unaligned or short blob";
      return LECO_EINVAL;
    }
    if (j.out_dev && (reinterpret_cast<uintptr_t>(j.out_dev) & 3)) {
      ctx->last_error = "batch job with a misaligned output";
      return LECO_EINVAL;
    }
  }
  leco_batch* b = new leco_batch();
  b->ctx = ctx;
  b->jobs.assign(jobs, jobs + ncols);
  b->tile_log2 = ctx->tune.tile_log2;
  b->blocks_per_cu = ctx->tune.decode_blocks_per_cu;
  if (hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking) != hipSuccess) {
    delete b;
    return LECO_EDEVICE;
  }
  const leco_status st = upload_table(b);
  if (st != LECO_OK) {
    leco_batch_destroy(b);
    return st;
  }
  *out = b;
  return LECO_OK;
}

leco_status leco_batch_destroy(leco_batch* b) {
  if (!b) return LECO_OK;
  (void)hipDeviceSynchronize();
  drop_graphs(b);
  if (b->cols_dev) (void)hipFree(b->cols_dev);
  if (b->tile_col_dev) (void)hipFree(b->tile_col_dev);
  if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
  delete b;
  return LECO_OK;
}

leco_status leco_batch_set_shape(leco_batch* b, uint32_t tile_log2, uint32_t blocks_per_cu) {
  if (!b || (tile_log2 != 0 && (tile_log2 < 8 || tile_log2 > 16)) || blocks_per_cu > 64)
    return LECO_EINVAL;
  if (tile_log2 == b->tile_log2 && blocks_per_cu == b->blocks_per_cu) return LECO_OK;
  (void)hipDeviceSynchronize();
  b->blocks_per_cu = blocks_per_cu;
  if (tile_log2 != b->tile_log2) {
    b->tile_log2 = tile_log2;
    return upload_table(b);
  }
  drop_graphs(b);
  return LECO_OK;
}

leco_status leco_batch_run(leco_batch* b, int op, hipStream_t stream) {
  if (!b || !valid_op(op)) return LECO_EINVAL;
  const hipError_t e = launch_batch(b, op, stream);
  if (e != hipSuccess) return bfail(b, LECO_EDEVICE, hipGetErrorString(e));
  return LECO_OK;
}

leco_status leco_batch_run_graph(leco_batch* b, int op, hipStream_t stream) {
  if (!b || !valid_op(op)) return LECO_EINVAL;
  hipGraphExec_t& exec = b->graphs[op];
  if (!exec) {
    // Captured on the batch's own stream (the legacy default stream cannot
    // be captured); the instantiated graph is then launched on `stream`.
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal) != hipSuccess)
      return bfail(b, LECO_EDEVICE, "stream capture failed to start");
    const hipError_t le = launch_batch(b, op, b->capture_stream);
    const hipError_t ce = hipStreamEndCapture(b->capture_stream, &g);
    if (le != hipSuccess || ce != hipSuccess || !g)
      return bfail(b, LECO_EDEVICE, "batch capture failed");
    const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ie != hipSuccess) {
      exec = nullptr;
      return bfail(b, LECO_EDEVICE, "graph instantiation failed");
    }
  }
  if (hipGraphLaunch(exec, stream) != hipSuccess) return bfail(b, LECO_EDEVICE, "graph launch failed");
  return LECO_OK;
}

leco_status leco_batch_tune(leco_batch* b, int op, hipStream_t stream, uint32_t* tile_log2,
                            uint32_t* blocks_per_cu) {
  if (!b || !valid_op(op)) return LECO_EINVAL;
  // persistent grids are tried at the number of workgroups a CU holds at
  // once, so that no workgroup waits for another one to finish
  int resident = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&resident, batch_kernel(op), leco::kBlock, 0) !=
          hipSuccess ||
      resident < 1)
    resident = 4;
  static const uint32_t kTiles[] = {0, 12, 13, 14};
  const uint32_t bpcs[] = {0, uint32_t(resident)};
  hipEvent_t e0 = nullptr, e1 = nullptr;
  leco_status st = LECO_OK;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) st = LECO_EDEVICE;
  float best = 1e30f;
  uint32_t bt = b->tile_log2, bb = b->blocks_per_cu;
  for (uint32_t tl : kTiles) {
    for (uint32_t bpc : bpcs) {
      if (st != LECO_OK) break;
      st = leco_batch_set_shape(b, tl, bpc);
      if (st != LECO_OK) break;
      float total = 0.0f;
      hipError_t e = launch_batch(b, op, stream);  // warm-up
      for (int r = 0; r < 3 && e == hipSuccess; ++r) {
        float ms = 0.0f;
        if ((e = hipEventRecord(e0, stream)) != hipSuccess ||
            (e = launch_batch(b, op, stream)) != hipSuccess ||
            (e = hipEventRecord(e1, stream)) != hipSuccess ||
            (e = hipEventSynchronize(e1)) != hipSuccess ||
            (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
          break;
        total += ms;
      }
      if (e != hipSuccess) {
        st = bfail(b, LECO_EDEVICE, hipGetErrorString(e));
        break;
      }
      if (total < best) {
        best = total;
        bt = tl;
        bb = bpc;
      }
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  const leco_status st2 = leco_batch_set_shape(b, bt, bb);
  if (tile_log2) *tile_log2 = bt;
  if (blocks_per_cu) *blocks_per_cu = bb;
  return st != LECO_OK ? st : st2;
}

}  // extern "C"

namespace {

// The tuner's cache file: a JSON object with one member per line,
//   "<key>": {"tile_log2": T, "blocks_per_cu": B},
// keyed by device, operation and batch shape.
std::string tune_key(const leco_batch* b, int op) {
  hipDeviceProp_t prop;
  std::string arch = "unknown";
  if (hipGetDeviceProperties(&prop, b->ctx->device) == hipSuccess) arch = prop.gcnArchName;
  for (char& ch : arch)
    if (ch == '"' || ch == '\\') ch = '_';
  uint64_t values = 0, bytes = 0;
  for (const leco_decode_job& j : b->jobs) {
    values += j.n;
    bytes += j.blob_bytes;
  }
  char buf[512];
  snprintf(buf, sizeof(buf), "%s cu%d op%d cols%llu values%llu bytes%llu", arch.c_str(),
           b->ctx->num_cus, op, (unsigned long long)b->jobs.size(), (unsigned long long)values,
           (unsigned long long)bytes);
  return buf;
}

struct TuneEntry {
  std::string key;
  uint32_t tile_log2, blocks_per_cu;
};

std::vector<TuneEntry> read_tune_cache(const char* path) {
  std::vector<TuneEntry> out;
  FILE* f = fopen(path, "r");
  if (!f) return out;
  char line[1024];
  while (fgets(line, sizeof(line), f)) {
    const char* q0 = strchr(line, '"');
    const char* q1 = q0 ? strchr(q0 + 1, '"') : nullptr;
    if (!q1) continue;
    unsigned t = 0, bpc = 0;
    const char* rest = strstr(q1, "\"tile_log2\":");
    const char* rest2 = strstr(q1, "\"blocks_per_cu\":");
    if (!rest || !rest2 || sscanf(rest, "\"tile_log2\": %u", &t) != 1 ||
        sscanf(rest2, "\"blocks_per_cu\": %u", &bpc) != 1)
      continue;
    out.push_back(TuneEntry{std::string(q0 + 1, q1), t, bpc});
  }
  fclose(f);
  return out;
}

bool write_tune_cache(const char* path, const std::vector<TuneEntry>& entries) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = fopen(tmp.c_str(), "w");
  if (!f) return false;
  fprintf(f, "{\n");
  for (size_t i = 0; i < entries.size(); ++i)
    fprintf(f, "\"%s\": {\"tile_log2\": %u, \"blocks_per_cu\": %u}%s\n", entries[i].key.c_str(),
            entries[i].tile_log2, entries[i].blocks_per_cu, i + 1 < entries.size() ? "," : "");
  fprintf(f, "}\n");
  const bool ok = fclose(f) == 0;
  return ok && rename(tmp.c_str(), path) == 0;
}

}  // namespace

extern "C" {

leco_status leco_batch_tune_cached(leco_batch* b, int op, const char* cache_path,
                                   hipStream_t stream, uint32_t* tile_log2,
                                   uint32_t* blocks_per_cu, int32_t* from_cache) {
  if (!b || !valid_op(op)) return LECO_EINVAL;
  if (from_cache) *from_cache = 0;
  const char* path = cache_path ? cache_path : getenv("LECO_AUTOTUNE_CACHE");
  if (!path || !*path) return leco_batch_tune(b, op, stream, tile_log2, blocks_per_cu);
  const std::string key = tune_key(b, op);
  std::vector<TuneEntry> entries = read_tune_cache(path);
  for (const TuneEntry& e : entries) {
    if (e.key != key) continue;
    const leco_status st = leco_batch_set_shape(b, e.tile_log2, e.blocks_per_cu);
    if (st != LECO_OK) break;  // an unusable entry is tuned again below
    if (tile_log2) *tile_log2 = e.tile_log2;
    if (blocks_per_cu) *blocks_per_cu = e.blocks_per_cu;
    if (from_cache) *from_cache = 1;
    return LECO_OK;
  }
  uint32_t t = 0, bpc = 0;
  leco_status st = leco_batch_tune(b, op, stream, &t, &bpc);
  if (st != LECO_OK) return st;
  if (tile_log2) *tile_log2 = t;
  if (blocks_per_cu) *blocks_per_cu = bpc;
  std::vector<TuneEntry> kept;
  for (const TuneEntry& e : entries)
    if (e.key != key) kept.push_back(e);
  kept.push_back(TuneEntry{key, t, bpc});
  if (!write_tune_cache(path, kept)) return bfail(b, LECO_EINVAL, "cannot write the tuner cache file");
  return LECO_OK;
}

}  // extern "C"
