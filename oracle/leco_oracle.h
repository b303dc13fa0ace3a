/*
 * LeCo CPU oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, scalar C implementation of what the learned-compression hot
 * path computes, written from the LeCo paper (Liu, Zeng, Zhang, "LeCo:
 * Lightweight Compression via Learning Serial Correlations", SIGMOD 2024).
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  The product path (the HIP library) shares no code,
 * header, table or constant with it.
 *
 * Every function names the passage of the paper it follows.  Where the paper
 * is silent or ambiguous the reading taken is stated next to the code.
 *
 * Conventions: all arrays are host memory owned by the caller.  Columns are
 * little-endian uint32 (dtype 4) or uint64 (dtype 8).  Functions return one
 * of the LREF_* status codes below and never abort.
 */
#ifndef LECO_ORACLE_H
#define LECO_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LREF_OK = 0,
  LREF_EINVAL = 1,  /* bad argument (dtype, partitioning, sizes)      */
  LREF_ENOMEM = 2,  /* host allocation failed                          */
  LREF_ENOSPC = 3,  /* output buffer too small; required size returned */
  LREF_EFORMAT = 4, /* blob fails validation                           */
  LREF_ERANGE = 5   /* a position or range lies outside [0, n)         */
};

/* Result of fitting one partition (section 3.1 least squares, section 3.3
 * storage).  mode 0 = constant model (FOR, section 2), 1 = linear. */
typedef struct {
  uint64_t vmin, vmax;
  uint64_t b_for;      /* bitlen(vmax - vmin)                               */
  int32_t fitted;      /* 1 when the least-squares fit was evaluated        */
  int32_t mode;        /* 0 = FOR (slope +0.0), 1 = least-squares line,
                          2 = minimax line                                 */
  uint64_t N_lo;       /* N = n*S_ty - S_t*S_y as two's-complement int128   */
  int64_t N_hi;
  uint64_t D_lo;       /* D = n*S_tt - S_t^2 as uint128                     */
  uint64_t D_hi;
  double theta1_ls;    /* fl(N)/fl(D), the fitted slope (0 if not fitted)   */
  int64_t r_min, r_max;/* residual extremes of the linear model             */
  uint64_t b_ls;       /* bitlen(r_max - r_min)                             */
  double theta1;       /* stored slope: theta1_ls or theta1_mm, else +0.0   */
  uint64_t base;       /* stored integer intercept                          */
  uint64_t bits;       /* stored residual width b                           */
  /* Minimax line (evaluated only with LREF_REG_MINIMAX). */
  int32_t mm_fitted;   /* 1 when the minimax slope was evaluated            */
  int32_t mm_pad;
  int64_t mm_dy;       /* exact minimax slope mm_dy / mm_dt, mm_dt > 0      */
  uint64_t mm_dt;
  double theta1_mm;    /* fl(mm_dy) / fl(mm_dt)                             */
  int64_t r_min_mm, r_max_mm;
  uint64_t b_mm;       /* bitlen(r_max_mm - r_min_mm)                       */
  /* Polynomials (evaluated only with LREF_REG_POLY). */
  int32_t poly_fitted; /* 1 when the degree-2 (and -3) fits were evaluated  */
  int32_t poly_degree; /* degree of the stored polynomial (mode 3), else 0  */
  double pc[3];        /* fitted Gram coefficients c1, c2, c3               */
  uint64_t b_p2, b_p3; /* widths of the degree-2 and degree-3 fits (99 = none) */
  double stored_c[3];  /* stored coefficients (c3 = 0 for degree 2)         */
} leco_ref_model;

/* bitlen(x) = floor(log2 x) + 1, bitlen(0) = 0 (the paper's ceil(log2 .)
 * read as "bits needed to store x"). */
uint64_t leco_ref_bitlen(uint64_t x);

/* Regressors (section 3.1).  LREF_REG_LS fits the least-squares line.
 * LREF_REG_MINIMAX also fits the line of smallest maximum deviation (the
 * fixed-width objective of section 3.1) and stores whichever of the
 * constant model, the least-squares line and the minimax line is narrowest,
 * ties going in that order. */
enum { LREF_REG_LS = 0, LREF_REG_MINIMAX = 1, LREF_REG_POLY = 2 };

/* Polynomial regressor (section 3.1 model terms; the higher-order models of
 * the evaluation).  For a partition of 3..4096 values whose range is below
 * 2^50, the least-squares polynomials of degree 2 and 3 (degree 3 from 4
 * values) are fitted in the basis of the discrete orthogonal (Gram)
 * polynomials of the positions t = 0..n-1:
 *   g1(t) = 2t - (n-1)
 *   g2(t) = 6t^2 - 6(n-1)t + (n-1)(n-2)
 *   g3(t) = 20t^3 - 30(n-1)t^2 + (12n^2 - 30n + 22)t - (n-1)(n-2)(n-3),
 * exactly orthogonal over those positions, so each coefficient is
 *   c_k = fl(S_k) / fl(Q_k),  S_k = sum y_t g_k(t),  Q_k = sum g_k(t)^2,
 * with exact integer sums (y_t = v_t - min v) each rounded to nearest-even
 * binary64 and one division; degree 2 stores c3 = 0.  Prediction:
 *   p_t = floor(fl(fl(fl(c1 * g1(t)) + fl(c2 * g2(t))) + fl(c3 * g3(t)))).
 * The stored model is the narrowest of the constant model, the
 * least-squares line, degree 2 and degree 3 (ties in that order).  A blob
 * encoded with this regressor sets header flag bit 1 and carries, after the
 * records (and starts), a 16-byte-aligned section of m (c2, c3) binary64
 * pairs; a polynomial partition's record has kind byte 25 = 1 and c1 in
 * the slope field. */

/* Fit one partition of n values (section 3.1, section 3.3). */
int leco_ref_fit(const uint64_t *v, uint64_t n, int force_constant,
                 int regressor, leco_ref_model *out);

/* Minimax slope of y_t = v_t, t = 0..n-1 (section 3.1 objective): the
 * smallest theta minimising max_t (v_t - theta t) - min_t (v_t - theta t),
 * as the exact fraction *dy / *dt (dt > 0).  Needs 2 <= n <= 2^20 and
 * max(v) - min(v) < 2^61. */
int leco_ref_minimax_slope(const uint64_t *v, uint64_t n, int64_t *dy,
                           uint64_t *dt);

/* Exact compressed size in bytes for a column under the given partitioning.
 * fixed_len > 0 selects fixed partitions; otherwise starts[0..m] is used. */
int leco_ref_blob_bytes(const void *col, uint64_t n, int dtype,
                        uint64_t fixed_len, const uint64_t *starts, uint64_t m,
                        int force_constant, int regressor, uint64_t *bytes);

/* Encode a column into a self-describing blob (section 3, section 3.3).
 * On LREF_ENOSPC *blob_bytes holds the required size. */
int leco_ref_encode(const void *col, uint64_t n, int dtype, uint64_t fixed_len,
                    const uint64_t *starts, uint64_t m, int force_constant,
                    int regressor, uint8_t *blob, uint64_t cap, uint64_t *blob_bytes);

/* Blob header fields. */
int leco_ref_blob_info(const uint8_t *blob, uint64_t blob_bytes, uint64_t *n,
                       int *dtype, uint64_t *m);

/* Per-partition model as stored in a blob (for diagnostics). */
int leco_ref_blob_record(const uint8_t *blob, uint64_t blob_bytes, uint64_t j,
                         uint64_t *base, double *theta1, uint64_t *word_off,
                         uint64_t *bits, uint64_t *start, uint64_t *len);

/* Decoder (section 3.3): every position is decoded on its own. */
int leco_ref_decode_all(const uint8_t *blob, uint64_t blob_bytes, void *out,
                        uint64_t out_cap_elems);
int leco_ref_decode_range(const uint8_t *blob, uint64_t blob_bytes,
                          uint64_t begin, uint64_t end, void *out);
int leco_ref_random_access(const uint8_t *blob, uint64_t blob_bytes,
                           const uint64_t *pos, uint64_t k, void *out);

/* Sum and count of decoded values v with lo <= v < hi (section 5.1 filter).
 * out[0] = low 64 bits of the sum, out[1] = high 64 bits, out[2] = count. */
int leco_ref_filter_sum(const uint8_t *blob, uint64_t blob_bytes, uint64_t lo,
                        uint64_t hi, uint64_t out[3]);

/* ---- Variable-length partitioner (section 3.2.2) ------------------------ */

/* Split-phase inclusion cost C of appending v[j] to v[i, j):
 *   model 0 = linear regressor with the approximation Delta~ (bitlen of the
 *             range of first differences),
 *   model 1 = Delta encoding with signed first-difference widths.
 * Result in bits. */
int64_t leco_ref_split_cost(const uint64_t *v, uint64_t i, uint64_t j,
                            int model);

/* Delta-encoding partition size S_M + len * Delta(v[i, j)) in bits, with
 * Delta = the widest signed first difference inside [i, j). */
uint64_t leco_ref_delta_partition_bits(const uint64_t *v, uint64_t i,
                                       uint64_t j, uint64_t sm_bits);

/* Size in bytes that a partition v[i, j) costs in a variable-length blob:
 * 32-byte record + 8-byte start + its residual words. */
uint64_t leco_ref_partition_cost_bytes(const uint64_t *v, uint64_t i,
                                       uint64_t j);

/* Greedy split + merge (section 3.2.2).  starts_out needs room for n + 1
 * entries.  max_len caps partition length (<= 2^20): a partition holding
 * max_len values takes no further value.  With start_positions the split
 * also begins a partition at the first value of every starting partition
 * (leco_ref_start_positions) and includes that starting partition's other
 * values without the cost test.  The merge then scans the partition list
 * (see leco_ref_partition_merge), at most max_passes passes (0: until a
 * pass merges nothing). */
int leco_ref_partition_greedy(const void *col, uint64_t n, int dtype,
                              double tau, uint64_t sm_bits, uint64_t max_len,
                              uint64_t max_passes, int start_positions,
                              uint64_t *starts_out, uint64_t *m_out);

/* The split phase of leco_ref_partition_greedy alone. */
int leco_ref_partition_split(const void *col, uint64_t n, int dtype, double tau,
                             uint64_t sm_bits, uint64_t max_len, int start_positions,
                             uint64_t *starts_out, uint64_t *m_out);

/* Starting partitions for the linear regressor (section 3.2.2, selecting
 * good starting positions: the segments where the second-order deltas,
 * dd_k = v_k - 2 v_{k-1} + v_{k-2}, are smallest).  Each maximal run k..k'
 * of positions whose |dd_k| equals the column's smallest |dd| is one
 * starting partition v[k-2, k'+1) (when two runs are one position apart
 * the later one takes the shared value).  first_out[i] and end_out[i] (end
 * may be null) receive the first value and one past the last value of the
 * i-th starting partition; both need room for n entries; *count_out
 * receives their number.  n < 3 has none. */
int leco_ref_start_positions(const void *col, uint64_t n, int dtype, uint64_t *first_out,
                             uint64_t *end_out, uint64_t *count_out);

/* Starting positions for Delta encoding (section 3.2.2 and the Delta
 * partitioning figure): with rb_k the signed width of d_k = v_k - v_{k-1}
 * ("required bits") and db_k = |rb_k - rb_{k-1}| ("delta bits"), each
 * maximal run k..k' of positions whose db equals the column's smallest db
 * starts a partition at k - 2.  pos_out needs room for n entries. */
int leco_ref_start_positions_delta(const void *col, uint64_t n, int dtype, uint64_t *pos_out,
                                   uint64_t *count_out);

/* Merge phase alone, applied to a given partitioning (in place): the
 * partition list is scanned from the left; the current partition merges
 * with its right neighbour when the merged partition costs strictly fewer
 * bytes than the two apart (leco_ref_partition_cost_bytes) and holds at
 * most max_len values, and the merged partition then tries its new right
 * neighbour; after a refusal the neighbour becomes the current partition.
 * Passes repeat until one merges nothing or max_passes have run (0: no
 * limit). */
int leco_ref_partition_merge(const void *col, uint64_t n, int dtype,
                             uint64_t *starts, uint64_t *m, uint64_t max_len,
                             uint64_t max_passes);

/* ---- Delta-fix codec (section 2, Delta encoding over fixed partitions) -----
 * Partitions of L values; each stores its first value and the offsets
 * e_k = d_k - d_min of its first differences d_k = v_k - v_{k-1} at width
 * w = bitlen(d_max - d_min) (w <= 65), least-significant bit first.
 * Size: 32 + 32 m + 8 * sum_j ceil((n_j - 1) w_j / 64) bytes. */
int leco_ref_delta_fix_bytes(const void *col, uint64_t n, int dtype, uint64_t L,
                             uint64_t *bytes);
int leco_ref_delta_fix_encode(const void *col, uint64_t n, int dtype, uint64_t L,
                              uint8_t *blob, uint64_t cap, uint64_t *blob_bytes);
int leco_ref_delta_fix_decode(const uint8_t *blob, uint64_t blob_bytes, void *out,
                              uint64_t out_cap_elems);

/* Optimal partitioning by dynamic programming (section 3.2), O(n^3). */
int leco_ref_partition_dp(const void *col, uint64_t n, int dtype,
                          uint64_t max_len, uint64_t *starts_out,
                          uint64_t *m_out, uint64_t *bytes_out);

/* Exhaustive search over all 2^(n-1) partitionings (n <= 24). */
int leco_ref_partition_bruteforce(const void *col, uint64_t n, int dtype,
                                  uint64_t max_len, uint64_t *starts_out,
                                  uint64_t *m_out, uint64_t *bytes_out);

/* Sum of leco_ref_partition_cost_bytes over a partitioning. */
int leco_ref_partitioning_cost(const void *col, uint64_t n, int dtype,
                               const uint64_t *starts, uint64_t m,
                               uint64_t *bytes_out);

/* ---- Fixed partition size search (section 3.2.1) ---------------------------
 *
 * Sampled cost of fixed partitions of length L: the windows
 * [starts[i], starts[i] + window), i < k, each cut into partitions of L
 * values (the last one shorter), and
 *   cost(L) = sum over all those partitions of 32 + 8 * ceil(len * b / 64),
 * the record and residual words each partition adds to a blob (b from
 * leco_ref_fit with `regressor`; the polynomial regressor adds its 16
 * coefficient bytes per partition).  The random window starts are inputs. */
int leco_ref_fixed_cost(const void *col, uint64_t n, int dtype,
                        const uint64_t *starts, uint64_t k, uint64_t window,
                        uint64_t L, int regressor, uint64_t *cost);

/* Search of L in [1, window] for the smallest cost (section 3.2.1, steps
 * 2-3).  Reading of the steps:
 *   exponential phase: L = 1, 2, 4, ... up to window, then window itself if
 *     it is not a power of two, stopping after the first L whose cost is
 *     strictly above the previous one; best = the cheapest L seen (the
 *     smallest on ties);
 *   back search: for s = best / 2, best / 4, ..., 1 evaluate best - s and
 *     then best + s (those in [1, window] not evaluated before) and move to
 *     the cheapest when strictly cheaper than best; stop after s = 1, or
 *     after a move that lowers the cost by less than 0.01% of it.
 * Every evaluation is appended to trace[] as (L, cost) pairs while
 * 2 * *trace_len < trace_cap.  cost_fn(ctx, L) supplies the costs. */
typedef uint64_t (*leco_ref_cost_fn)(void *ctx, uint64_t L);
int leco_ref_size_search_fn(uint64_t window, leco_ref_cost_fn cost_fn, void *ctx,
                            uint64_t *L_out, uint64_t *cost_out, uint64_t *trace,
                            uint64_t trace_cap, uint64_t *trace_len);

/* The search over leco_ref_fixed_cost of a column's sampled windows. */
int leco_ref_size_search(const void *col, uint64_t n, int dtype,
                         const uint64_t *starts, uint64_t k, uint64_t window,
                         int regressor, uint64_t *L_out, uint64_t *cost_out,
                         uint64_t *trace, uint64_t trace_cap, uint64_t *trace_len);

#ifdef __cplusplus
}
#endif
#endif
