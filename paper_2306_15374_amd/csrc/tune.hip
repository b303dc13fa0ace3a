// Launch-shape settings of the decoder and their environment overrides.
#include <stdlib.h>

#include "internal.hpp"

namespace leco {

static bool env_u32(const char* name, uint32_t lo, uint32_t hi, uint32_t* out) {
  const char* s = getenv(name);
  if (!s || !*s) return false;
  char* end = nullptr;
  const unsigned long v = strtoul(s, &end, 10);
  if (*end != '\0' || v < lo || v > hi) return false;
  *out = uint32_t(v);
  return true;
}

void tune_from_env(Tune& t) {
  env_u32("LECO_TILE_LOG2", 8, 20, &t.tile_log2);
  env_u32("LECO_DECODE_BLOCKS_PER_CU", 0, 64, &t.decode_blocks_per_cu);
  env_u32("LECO_XCD_REMAP", 0, 1, &t.xcd_remap);
  env_u32("LECO_ENCODE_WAVE", 0, 1, &t.encode_wave);
  env_u32("LECO_ENCODE_WAVE32", 0, 1, &t.encode_wave32);
  env_u32("LECO_ENCODE_FUSED", 0, 2, &t.encode_fused);
  env_u32("LECO_ENCODE_FUSED_WAVE", 0, 2, &t.encode_fused_wave);
  uint32_t lpt = t.ra_lookups_per_lane;
  if (env_u32("LECO_RA_LPT", 1, 8, &lpt) && (lpt == 1 || lpt == 2 || lpt == 4 || lpt == 8))
    t.ra_lookups_per_lane = lpt;
}

}  // namespace leco
