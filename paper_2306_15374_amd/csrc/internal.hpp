// Host-side internals shared by the LeCo HIP library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "../../include/leco.h"

namespace leco {

// Per-partition model produced by the fit kernel (32 bytes).
struct PartModel {
  uint64_t base;
  double theta1;
  uint64_t nwords;
  uint32_t bits;
  uint32_t pad;
};

// Launch parameters chosen per context (see the tuner in tune.hip).
struct Tune {
  uint32_t tile_log2 = 12;           // values per decode tile = 2^tile_log2
  uint32_t decode_blocks_per_cu = 0; // 0 = one workgroup per tile
  uint32_t xcd_remap = 0;            // 1 = contiguous tile runs per XCD
  uint32_t ra_lookups_per_lane = 1;  // 1, 2, 4 or 8 positions per lane
};

// Reads LECO_TILE_LOG2, LECO_DECODE_BLOCKS_PER_CU, LECO_XCD_REMAP and
// LECO_RA_LPT overrides from the environment.
void tune_from_env(Tune& t);

// Everything the encode kernels need, with scratch already carved out.
struct EncodePlan {
  const void* col;
  uint64_t n, m, fixed_len;
  uint32_t dtype;
  int force_constant;
  const uint64_t* starts_dev;  // m + 1 starts (variable) or null
  void* blob;
  uint64_t cap;
  uint64_t words_off;
  PartModel* models;     // m
  uint64_t* word_off;    // m
  uint64_t* partial;     // ceil(m / 4096)
  uint64_t* total_words; // 1
  uint64_t* size_dev;    // 1
};

hipError_t launch_decode(leco_ctx* ctx, const void* blob, uint64_t blob_bytes, void* out,
                         uint64_t begin, uint64_t end, uint64_t out_cap, bool all,
                         hipStream_t stream);
hipError_t launch_random_access(leco_ctx* ctx, const void* blob, uint64_t blob_bytes,
                                const uint64_t* pos, uint64_t k, void* out, hipStream_t stream);
hipError_t launch_filter_sum(leco_ctx* ctx, const void* blob, uint64_t blob_bytes, uint64_t lo,
                             uint64_t hi, uint64_t* out3, bool prune, hipStream_t stream);
hipError_t launch_zero_u64(uint64_t* p, uint64_t n, hipStream_t stream);
hipError_t launch_encode(leco_ctx* ctx, const EncodePlan& plan, hipStream_t stream);
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
  leco::Tune tune;
  std::string last_error;
};
