// Host-side internals shared by the LeCo HIP library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/leco.h"

namespace leco {

// Launch parameters chosen per context (see tune.hip).
struct Tune {
  uint32_t tile_log2 = 0;            // values per decode tile = 2^tile_log2; 0 = per blob
  uint32_t decode_blocks_per_cu = 0; // 0 = one workgroup per tile
  uint32_t xcd_remap = 0;            // 1 = contiguous tile runs per XCD
  uint32_t ra_lookups_per_lane = 1;  // 1, 2, 4 or 8 positions per lane
  uint32_t encode_wave = 1;          // 1 = one wavefront per partition when all are short
  uint32_t encode_wave32 = 1;        // 1 = the same up to 2048 values (32 per lane)
  // One pass over the column with a decoupled look-back: a workgroup per
  // partition (partitions of 2049..4096) or a wavefront per partition (at
  // most 1024).  0 = never, 1 = always where it applies, 2 = for launches of
  // at most kFusedAutoPerCu workgroups per CU.
  uint32_t encode_fused = 2;
  uint32_t encode_fused_wave = 2;
};

// Past about two workgroups per CU (2e6 8-byte values at partitions of 1024
// or 4096) the two-pass encoder is faster; below, its seven launches cost more
// than the one-pass kernel's look-back.
constexpr uint32_t kFusedAutoPerCu = 2;

// Reads LECO_TILE_LOG2, LECO_DECODE_BLOCKS_PER_CU, LECO_XCD_REMAP,
// LECO_RA_LPT, LECO_ENCODE_WAVE, LECO_ENCODE_WAVE32, LECO_ENCODE_FUSED and
// LECO_ENCODE_FUSED_WAVE overrides from the environment.
void tune_from_env(Tune& t);

// One column for the encoder: input, partitioning, output blob.  A table of
// these (device memory) drives one encode launch over many columns.
struct EncColumn {
  const uint8_t* col;      // n values of dtype
  uint8_t* blob;           // cap bytes
  const uint64_t* starts;  // m + 1 starts in device memory (variable), else null
  uint64_t* size_out;      // device word receiving the blob size, or null
  uint64_t n, m, fixed_len, cap;
  uint64_t words_off;      // offset of the words section
  uint64_t part_base;      // index of the column's first partition in the launch
  uint32_t dtype, force_constant;
  uint32_t regressor;      // 0 least squares, 1 minimax as well, 2 polynomials as well
  uint32_t pad;
  uint64_t val_base;       // index of the column's first value in the launch
};

// Decode tile size (log2 of values per workgroup tile) for a blob of
// blob_bytes holding about n values, unless the environment fixed it: the
// largest tile (up to 4096 values per wavefront) whose residual words,
// estimated from the blob's bits per value, fit one wavefront's LDS slice,
// so that every wavefront stages its words in one round trip.
uint32_t pick_tile_log2(const Tune& t, uint64_t blob_bytes, uint64_t n);

hipError_t launch_decode(leco_ctx* ctx, const void* blob, uint64_t blob_bytes, void* out,
                         uint64_t begin, uint64_t end, uint64_t out_cap, bool all,
                         hipStream_t stream);
hipError_t launch_random_access(leco_ctx* ctx, const void* blob, uint64_t blob_bytes,
                                const uint64_t* pos, uint64_t k, void* out, hipStream_t stream);
hipError_t launch_filter_sum(leco_ctx* ctx, const void* blob, uint64_t blob_bytes, uint64_t lo,
                             uint64_t hi, uint64_t* out3, bool prune, hipStream_t stream);
hipError_t launch_zero_u64(uint64_t* p, uint64_t n, hipStream_t stream);
// Partitions of at most this many values are encoded one per wavefront.
constexpr uint64_t kWaveEncodeMax = 1024;
// Minimax partitions longer than this many values keep running hulls in
// EncScratch::hull.
constexpr uint64_t kHullTileValues = 4096;

// Device scratch of one encode launch (nparts partitions): the fitted
// models, their word counts and offsets, and the scan's per-workgroup sums.
struct EncScratch {
  uint64_t* nwords;
  uint64_t* woff;
  uint64_t* base;
  uint64_t* theta;  // bits of the binary64 slope
  uint64_t* bsum;
  uint32_t* bits;
  // running hulls of minimax partitions longer than one hull tile: upper
  // vertex k of the partition at launch value s is hull[s + k], lower is
  // hull[hull_values + s + k]; null when no such partition is encoded
  uint32_t* hull;
  uint64_t hull_values;
  // polynomial models (columns with the polynomial regressor): kind 0/1 and
  // the bits of c2, c3 per partition
  uint32_t* kind;
  uint64_t* c2;
  uint64_t* c3;
};
uint64_t encode_scratch_bytes(uint64_t nparts);
EncScratch carve_encode_scratch(void* p, uint64_t nparts);

// Regressors present in a launch, as bits of a mask.
constexpr uint32_t kRegLS = 1, kRegMinimax = 2, kRegPoly = 4;
inline uint32_t regressor_bit(uint32_t regressor) { return 1u << regressor; }

// Encodes ncols columns (table cols_dev, or `single` when cols_dev is null)
// with nparts partitions in total.  max_len: the longest partition of the
// launch; regs: the regressors its columns ask for (selects the kernels).
hipError_t launch_encode_columns(leco_ctx* ctx, const EncColumn* cols_dev, uint64_t ncols,
                                 const EncColumn& single, uint64_t nparts, uint64_t max_len,
                                 uint32_t regs, const EncScratch& scr, hipStream_t stream);
// *out += the record and word bytes (plus extra_per_part) of the nparts
// partitions fitted in scr.
hipError_t launch_cost_sum(const EncScratch& scr, uint64_t nparts, uint64_t extra_per_part,
                           uint64_t* out, hipStream_t stream);
// The fit step alone: every partition's model, width and word count in scr.
hipError_t launch_fit_columns(leco_ctx* ctx, const EncColumn* cols_dev, uint64_t ncols,
                              const EncColumn& single, uint64_t nparts, uint64_t max_len,
                              uint32_t regs, const EncScratch& scr, hipStream_t stream);
hipError_t launch_diag_slope(const uint64_t* in, uint64_t k, double* out, hipStream_t stream);
hipError_t launch_diag_copy(leco_ctx* ctx, const void* src, void* dst, uint64_t bytes,
                            hipStream_t stream);

}  // namespace leco

struct leco_ctx {
  int device = 0;
  int num_cus = 0;
  int* err_dev = nullptr;          // device error bits (leco::kErr*)
  int* err_host = nullptr;         // pinned host mirror used by leco_sync
  uint64_t* pinned_u64 = nullptr;  // pinned host words for small readbacks
  void* scratch = nullptr;
  size_t scratch_bytes = 0;
  void* noalloc_scratch = nullptr;  // this device's fixed encode scratch
  leco::Tune tune;
  std::string last_error;
};
