/*
 * Drives every entry point of the CPU oracle (test infrastructure) on
 * deterministic inputs, for a build with AddressSanitizer and
 * UndefinedBehaviorSanitizer: shifts by 64, int128 overflow, reads outside
 * a blob or a column abort the run.  Exit status 0 means every call
 * returned and every round trip reproduced its column.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/leco_oracle.h"

static uint64_t rng_state = 0x9E3779B97F4A7C15ull;
static uint64_t next(void) { /* xorshift64* */
  rng_state ^= rng_state >> 12;
  rng_state ^= rng_state << 25;
  rng_state ^= rng_state >> 27;
  return rng_state * 2685821657736338717ull;
}

#define CHECK(cond)                                                    \
  do {                                                                 \
    if (!(cond)) {                                                     \
      fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
      exit(1);                                                         \
    }                                                                  \
  } while (0)

/* Column kinds: 0 noise on a line, 1 full-range random, 2 constant runs,
 * 3 extremes (0 and 2^64-1), 4 a cubic, 5 sorted keys. */
static void make_column(int kind, int dtype, uint64_t n, uint64_t *v) {
  uint64_t acc = 1000, run = 0, val = 0;
  for (uint64_t i = 0; i < n; i++) {
    uint64_t x;
    switch (kind) {
      case 0: x = 1000 + 7 * i + (next() & 63); break;
      case 1: x = next(); break;
      case 2:
        if (run == 0) {
          run = 1 + (next() & 127);
          val = next();
        }
        run--;
        x = val;
        break;
      case 3: x = (next() & 1) ? ~0ull : 0; break;
      case 4: x = (i * i * i) / 40 + 3 * i + (next() & 15); break;
      default: acc += 1 + (next() & 255); x = acc; break;
    }
    v[i] = dtype == 4 ? (x & 0xffffffffull) : x;
  }
}

static void *pack(const uint64_t *v, uint64_t n, int dtype) {
  void *col = malloc(n ? n * (uint64_t)dtype : 1);
  for (uint64_t i = 0; i < n; i++) {
    if (dtype == 4) ((uint32_t *)col)[i] = (uint32_t)v[i];
    else ((uint64_t *)col)[i] = v[i];
  }
  return col;
}

static uint64_t value_at(const void *col, int dtype, uint64_t i) {
  return dtype == 4 ? ((const uint32_t *)col)[i] : ((const uint64_t *)col)[i];
}

static void round_trip(const void *col, uint64_t n, int dtype, uint64_t L, const uint64_t *starts,
                       uint64_t m, int regressor) {
  uint64_t size = 0;
  int st = leco_ref_encode(col, n, dtype, L, starts, m, 0, regressor, NULL, 0, &size);
  CHECK(st == LREF_ENOSPC);
  uint8_t *blob = (uint8_t *)malloc(size);
  CHECK(leco_ref_encode(col, n, dtype, L, starts, m, 0, regressor, blob, size, &size) == LREF_OK);
  uint64_t bytes = 0;
  CHECK(leco_ref_blob_bytes(col, n, dtype, L, starts, m, 0, regressor, &bytes) == LREF_OK);
  CHECK(bytes == size);
  uint64_t n2, m2;
  int dt2;
  CHECK(leco_ref_blob_info(blob, size, &n2, &dt2, &m2) == LREF_OK && n2 == n && dt2 == dtype);
  void *out = malloc(n ? n * (uint64_t)dtype : 1);
  CHECK(leco_ref_decode_all(blob, size, out, n) == LREF_OK);
  CHECK(n == 0 || memcmp(out, col, n * (uint64_t)dtype) == 0);
  if (n) {
    uint64_t pos[64];
    for (int q = 0; q < 64; q++) pos[q] = next() % n;
    pos[0] = 0;
    pos[1] = n - 1;
    uint64_t got[64];
    CHECK(leco_ref_random_access(blob, size, pos, 64, got) == LREF_OK);
    for (int q = 0; q < 64; q++) {
      uint64_t g = dtype == 4 ? ((uint32_t *)got)[q] : got[q];
      CHECK(g == value_at(col, dtype, pos[q]));
    }
    uint64_t b = next() % n, e = b + next() % (n - b + 1);
    CHECK(leco_ref_decode_range(blob, size, b, e, out) == LREF_OK);
    uint64_t fs[3];
    CHECK(leco_ref_filter_sum(blob, size, 0, ~0ull, fs) == LREF_OK);
    for (uint64_t j = 0; j < m2; j++) {
      uint64_t base, woff, bits, s0, len;
      double th;
      CHECK(leco_ref_blob_record(blob, size, j, &base, &th, &woff, &bits, &s0, &len) == LREF_OK);
    }
    uint64_t bad = n;
    CHECK(leco_ref_random_access(blob, size, &bad, 1, got) == LREF_ERANGE);
  }
  /* corrupted and truncated copies must be rejected or decoded, never read
   * outside the buffer */
  for (int trial = 0; trial < 24; trial++) {
    uint64_t cut = trial < 8 ? next() % (size + 1) : size;
    uint8_t *c = (uint8_t *)malloc(cut ? cut : 1);
    memcpy(c, blob, cut);
    if (trial >= 8 && cut) c[next() % cut] ^= (uint8_t)(1u << (next() & 7));
    uint64_t sink[3];
    (void)leco_ref_decode_all(c, cut, out, n);
    (void)leco_ref_filter_sum(c, cut, 0, ~0ull, sink);
    free(c);
  }
  free(out);
  free(blob);
}

int main(void) {
  uint64_t lens[] = {0, 1, 2, 3, 5, 64, 700, 4097, 20000};
  for (int dt = 4; dt <= 8; dt += 4)
    for (int kind = 0; kind < 6; kind++)
      for (size_t li = 0; li < sizeof(lens) / sizeof(lens[0]); li++) {
        uint64_t n = lens[li];
        uint64_t *v = (uint64_t *)malloc((n ? n : 1) * 8);
        make_column(kind, dt, n, v);
        void *col = pack(v, n, dt);
        for (int reg = 0; reg <= 2; reg++) {
          round_trip(col, n, dt, 1 + next() % 1500, NULL, 0, reg);
          round_trip(col, n, dt, 4096, NULL, 0, reg);
          if (n) { /* variable partitions */
            uint64_t *s = (uint64_t *)malloc((n + 1) * 8), m = 0;
            s[0] = 0;
            while (s[m] < n) {
              uint64_t step = 1 + next() % 3000;
              s[m + 1] = s[m] + step < n ? s[m] + step : n;
              m++;
            }
            round_trip(col, n, dt, 0, s, m, reg);
            free(s);
          }
        }
        if (n >= 2) {
          const uint64_t k = n < 5000 ? n : 5000;
          uint64_t lo = v[0], hi = v[0];
          for (uint64_t i = 1; i < k; i++) {
            lo = v[i] < lo ? v[i] : lo;
            hi = v[i] > hi ? v[i] : hi;
          }
          int64_t dy;
          uint64_t dtt;
          leco_ref_model md;
          /* the slope needs a range below 2^61 and refuses others */
          const int want = hi - lo < (1ull << 61) ? LREF_OK : LREF_EINVAL;
          CHECK(leco_ref_minimax_slope(v, k, &dy, &dtt) == want);
          CHECK(leco_ref_fit(v, n < 4096 ? n : 4096, 0, LREF_REG_POLY, &md) == LREF_OK);
        }
        if (n >= 2) {
          uint64_t *st = (uint64_t *)malloc((n + 1) * 8), m = 0, bytes = 0;
          CHECK(leco_ref_partition_greedy(col, n, dt, 0.05, 320, 1u << 20, 0, 0, st, &m) == LREF_OK);
          CHECK(leco_ref_partition_greedy(col, n, dt, 0.05, 320, 1u << 20, 0, 1, st, &m) == LREF_OK);
          CHECK(leco_ref_partition_split(col, n, dt, 0.05, 320, 1u << 20, 1, st, &m) == LREF_OK);
          CHECK(leco_ref_partition_split(col, n, dt, 0.0, 320, 5, 1, st, &m) == LREF_OK);
          CHECK(leco_ref_partitioning_cost(col, n, dt, st, m, &bytes) == LREF_OK);
          {
            uint64_t *en = (uint64_t *)malloc(n * 8), c = 0;
            CHECK(leco_ref_start_positions(col, n, dt, st, en, &c) == LREF_OK);
            CHECK(leco_ref_start_positions(col, n, dt, st, NULL, &c) == LREF_OK);
            CHECK(leco_ref_start_positions_delta(col, n, dt, en, &c) == LREF_OK);
            free(en);
          }
          for (uint64_t L = 1; L <= 4096; L *= 8) {
            uint64_t need = 0;
            CHECK(leco_ref_delta_fix_bytes(col, n, dt, L, &need) == LREF_OK);
            uint8_t *df = (uint8_t *)malloc(need);
            void *back = malloc(n * (uint64_t)dt);
            CHECK(leco_ref_delta_fix_encode(col, n, dt, L, df, need, &need) == LREF_OK);
            CHECK(leco_ref_delta_fix_decode(df, need, back, n) == LREF_OK);
            CHECK(memcmp(back, col, n * (uint64_t)dt) == 0);
            for (int f = 0; f < 8; f++) { /* damaged copies must not read out of bounds */
              uint64_t cut = need - (next() % (need < 64 ? need : 64));
              uint8_t *bad = (uint8_t *)malloc(cut ? cut : 1);
              memcpy(bad, df, cut);
              if (cut > 32) bad[next() % cut] ^= (uint8_t)(1u << (next() & 7));
              (void)leco_ref_delta_fix_decode(bad, cut, back, n);
              free(bad);
            }
            free(back);
            free(df);
          }
          CHECK(leco_ref_partition_merge(col, n, dt, st, &m, 1u << 20, 2) == LREF_OK);
          (void)leco_ref_split_cost(v, 0, n - 1, 0);
          (void)leco_ref_split_cost(v, 0, n - 1, 1);
          (void)leco_ref_delta_partition_bits(v, 0, n, 320);
          (void)leco_ref_partition_cost_bytes(v, 0, n);
          if (n <= 64) {
            CHECK(leco_ref_partition_dp(col, n, dt, 1u << 20, st, &m, &bytes) == LREF_OK);
            if (n <= 14)
              CHECK(leco_ref_partition_bruteforce(col, n, dt, 1u << 20, st, &m, &bytes) == LREF_OK);
          }
          free(st);
        }
        if (n >= 700) {
          uint64_t starts[3] = {0, (n - 700) / 3, n - 700}, L, cost, tr[64], tl;
          for (int reg = 0; reg <= 2; reg++)
            CHECK(leco_ref_size_search(col, n, dt, starts, 3, 700, reg, &L, &cost, tr, 64, &tl) ==
                  LREF_OK);
        }
        free(col);
        free(v);
      }
  for (int i = 0; i < 200; i++) (void)leco_ref_bitlen(next() >> (next() & 63));
  printf("oracle sanitizer run ok\n");
  return 0;
}
