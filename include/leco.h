/*
 * leco.h -- C ABI of the MI355X (gfx950) LeCo codec.
 *
 * LeCo (Liu, Zeng, Zhang, "LeCo: Lightweight Compression via Learning Serial
 * Correlations", SIGMOD 2024) stores an integer column as partitions, each
 * with a regression model and a fixed-width bit-packed array of residuals;
 * value[i] = model_j(i - start_j) + residual[i] (section 3, problem
 * statement; section 3.3, encoder and decoder).  This library runs every
 * step of encoding and decoding in HIP kernels on one GPU.
 *
 * Memory and ownership
 *   - Arguments ending in `_dev` are device pointers owned by the caller
 *     (allocated with hipMalloc or as torch tensors).  Arguments ending in
 *     `_host` are host pointers owned by the caller.  The library never frees
 *     or retains caller memory beyond the call, except resident blobs handed
 *     to a server (see leco_server_*), which must stay valid until
 *     leco_server_stop returns.
 *   - Calls taking a `stream` only enqueue work on that stream and return;
 *     results are valid once the stream has reached that point.  Calls marked
 *     [sync] wait for the stream before returning.
 *   - A context is not thread-safe: use one per host thread.  Contexts on the
 *     same device may be used concurrently.
 *
 * Errors
 *   - Every call returns a leco_status.  Argument errors are detected on the
 *     host before any work is enqueued (LECO_EINVAL, LECO_ENOSPC).
 *   - Conditions only the GPU can see (a position >= n, a blob whose header,
 *     records or starts fail validation, an encode output larger than its
 *     capacity) raise a per-context device flag.  The kernels never read or
 *     write outside the buffers described by the call's sizes, whatever the
 *     blob holds; the output for the offending elements is unspecified.  The
 *     flag is reported, and cleared, by the next leco_sync on the context.
 *   - leco_last_error returns a description of the last failure.
 *
 * Blob format (section 3.3, storage format; little-endian, zero padding)
 *   header, 64 B: magic "LECO" u32, version u16 = 1, dtype u8 (4 or 8),
 *     flags u8 (bit 0 = variable-length partitions), n u64, m u64,
 *     fixed_len u64 (0 if variable), records_off u64 (= 64), starts_off u64
 *     (0 if fixed), words_off u64, total_words u64;
 *   records, m x 32 B: intercept `base` u64, slope theta1 as binary64 bits,
 *     word_off u64 (in 64-bit words, relative to words_off), bit width b u8,
 *     7 zero bytes;
 *   starts (variable only): m + 1 u64, starts[0] = 0, starts[m] = n;
 *   words: begins at the 16-byte-aligned end of the previous section;
 *     residual t of partition j occupies bits [b*t, b*t + b) of the span that
 *     begins at word word_off_j, least-significant bit first; each partition
 *     starts on a fresh word; the blob ends on a 16-byte boundary.
 *   Total size: align16(align16(64 + 32 m [+ 8 (m + 1)]) + 8 * total_words).
 *
 * Model arithmetic (section 3.1 regressor; section 3.3 decoder)
 *   For partition values v_t (t = 0..n_j-1), vmin/vmax and R = vmax - vmin:
 *   if n_j = 1, R >= 2^61, or the constant model is forced, the partition
 *   uses the constant model (frame of reference): theta1 = +0.0,
 *   base = vmin, b = bitlen(R).  Otherwise the least-squares slope is
 *   theta1 = fl(N) / fl(D) with N = n*S_ty - S_t*S_y and D = n*S_tt - S_t^2
 *   from exact integer sums over y_t = v_t - vmin, each converted to binary64
 *   with round-to-nearest-even and divided once (IEEE); -0.0 becomes +0.0.
 *   Residuals r_t = y_t - floor(theta1 * t) (one binary64 multiply, no fused
 *   multiply-add).  If bitlen(R) <= bitlen(max r - min r) the constant model
 *   is kept; else base = vmin + min r (mod 2^64), b = bitlen(max r - min r).
 *   Decoding: v = base + floor(theta1 * t) + u (mod 2^64), truncated to the
 *   column's dtype.
 */
#ifndef LECO_H
#define LECO_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct leco_ctx leco_ctx;

typedef enum {
  LECO_OK = 0,
  LECO_EINVAL = 1,  /* bad argument or partitioning                         */
  LECO_ENOMEM = 2,  /* device or host allocation failed                     */
  LECO_ENOSPC = 3,  /* output buffer too small (required size is returned)  */
  LECO_EFORMAT = 4, /* blob failed validation                               */
  LECO_ERANGE = 5,  /* position or range outside [0, n)                     */
  LECO_EDEVICE = 6  /* HIP runtime error                                    */
} leco_status;

typedef enum { LECO_U32 = 4, LECO_U64 = 8 } leco_dtype;

/* Partition assignment (section 3, problem statement; section 3.2).
 *   fixed_len > 0: fixed partitions of fixed_len values (section 3.2.1), the
 *                  last one possibly shorter; starts_host is ignored.
 *   fixed_len = 0: variable partitions (section 3.2.2) given by
 *                  starts_host[0..num_partitions], strictly increasing,
 *                  starts_host[0] = 0 and starts_host[num_partitions] = n.
 *   Every partition holds 1..2^20 values.
 *   force_constant_model = 1 stores every partition with slope +0.0, which is
 *   exactly frame-of-reference encoding (section 2).
 *   regressor (section 3.1): LECO_REGRESSOR_LS fits the least-squares line;
 *   LECO_REGRESSOR_MINIMAX also fits the line of smallest maximum deviation
 *   (the fixed-width objective of section 3.1: the smallest slope that
 *   minimises the vertical width of the strip holding the partition's
 *   points, taken exactly from their convex hulls, stored as fl(dy)/fl(dt)
 *   of the hull edge it lies on) and stores it when its residual width is
 *   strictly below both the constant model's and the least-squares line's.
 *   Minimax partitions longer than 4096 values need 8 bytes of device
 *   scratch per value of the column.
 *   LECO_REGRESSOR_POLY (section 3.1's model terms; the higher-order models
 *   of the evaluation) also fits, for partitions of 3..4096 values whose
 *   range is below 2^50, the least-squares polynomials of degree 2 and 3
 *   (degree 3 from 4 values) in the discrete orthogonal (Gram) basis of the
 *   positions t = 0..n-1:
 *     g1 = 2t - (n-1), g2 = 6t^2 - 6(n-1)t + (n-1)(n-2),
 *     g3 = 20t^3 - 30(n-1)t^2 + (12n^2 - 30n + 22)t - (n-1)(n-2)(n-3);
 *   c_k = fl(S_k) / fl(Q_k) with S_k = sum (v_t - min v) g_k(t) and
 *   Q_k = sum g_k(t)^2 exact integers, degree 2 storing c3 = 0; prediction
 *   floor(fl(fl(fl(c1 g1) + fl(c2 g2)) + fl(c3 g3))).  The narrowest of the
 *   constant model, the line, degree 2 and degree 3 is stored (ties: the
 *   simpler).  Its blobs set header flag bit 1 and hold, 16-byte aligned
 *   after the records (and starts), one (c2, c3) binary64 pair per
 *   partition (zero for a line); a polynomial record has kind byte 25 = 1
 *   and c1 in the slope field.  Every decoder (single-column, batched and
 *   served) decodes such blobs, value by value and without model-bound
 *   pruning.  Least-squares and minimax blobs keep flag bit 1 clear and
 *   every kind byte 0. */
typedef enum {
  LECO_REGRESSOR_LS = 0,
  LECO_REGRESSOR_MINIMAX = 1,
  LECO_REGRESSOR_POLY = 2
} leco_regressor;

typedef struct {
  uint64_t fixed_len;
  const uint64_t *starts_host;
  uint64_t num_partitions;
  int32_t force_constant_model;
  int32_t regressor; /* leco_regressor; any other value is LECO_EINVAL */
} leco_partitioning;

/* Context on HIP device `hip_device`.  Owns the device error flag, scratch
 * buffers and the tuning table. */
leco_status leco_create(int hip_device, leco_ctx **out);
leco_status leco_destroy(leco_ctx *ctx); /* [sync] on the whole device */
const char *leco_last_error(const leco_ctx *ctx);

/* Waits for `stream`, then reports and clears the context's device flag:
 * LECO_ERANGE, LECO_EFORMAT or LECO_ENOSPC if a kernel raised one. [sync] */
leco_status leco_sync(leco_ctx *ctx, hipStream_t stream);

/* Upper bound of the blob size for any column of n values of this dtype
 * under this partitioning (every residual at full dtype width). */
leco_status leco_max_blob_bytes(uint64_t n, leco_dtype dtype,
                                const leco_partitioning *part, uint64_t *bytes);

/* Parses a host copy of the 64-byte blob header. */
leco_status leco_blob_info(const void *header_host, uint64_t *n,
                           leco_dtype *dtype, uint64_t *num_partitions);

/* Full host-side validation of a blob in device memory: copies its header,
 * records and starts to the host and checks every field. [sync] */
leco_status leco_validate_blob(leco_ctx *ctx, const void *blob_dev,
                               uint64_t blob_bytes, hipStream_t stream);

/* Encoder (section 3.3): fits every partition (section 3.1), computes the
 * residuals and their width, and bit-packs them into blob_dev.
 *   col_dev: n values of `dtype`.  blob_dev: blob_cap bytes.
 *   On success *blob_bytes_host is the blob size.  If blob_cap is smaller
 *   than the size, returns LECO_ENOSPC with the required size in
 *   *blob_bytes_host and the contents of blob_dev unspecified.  [sync] */
leco_status leco_encode(leco_ctx *ctx, const void *col_dev, uint64_t n,
                        leco_dtype dtype, const leco_partitioning *part,
                        void *blob_dev, uint64_t blob_cap,
                        uint64_t *blob_bytes_host, hipStream_t stream);

/* Same as leco_encode without waiting: requires blob_cap >=
 * leco_max_blob_bytes(...) and writes the blob size to *blob_bytes_dev. */
leco_status leco_encode_async(leco_ctx *ctx, const void *col_dev, uint64_t n,
                              leco_dtype dtype, const leco_partitioning *part,
                              void *blob_dev, uint64_t blob_cap,
                              uint64_t *blob_bytes_dev, hipStream_t stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the
 * encode of leco_encode_async, producing the same bytes, that allocates
 * nothing.  Its scratch (per-partition models, word counts and offsets,
 * variable starts, running hulls) lives in a fixed array of
 * LECO_NOALLOC_SCRATCH_BYTES in each GPU's memory, held by the library
 * until the process ends; every call on a GPU shares that GPU's array, so
 * calls that overlap on one GPU (other streams, other threads, other
 * contexts) race and must be ordered by the caller.  About 56 bytes per
 * partition are needed (plus 8 (m + 1) for variable starts and 8 n for
 * minimax partitions longer than 4096 values); a call needing more than the
 * array returns LECO_ENOSPC before anything is enqueued.  Requires
 * blob_cap >= leco_max_blob_bytes(...); the blob size goes to
 * *blob_bytes_dev. */
#define LECO_NOALLOC_SCRATCH_BYTES (32u << 20)
leco_status leco_encode_noalloc(leco_ctx *ctx, const void *col_dev, uint64_t n,
                                leco_dtype dtype, const leco_partitioning *part,
                                void *blob_dev, uint64_t blob_cap,
                                uint64_t *blob_bytes_dev, hipStream_t stream);

/* Decoder, full column (section 3.3, range decompression over [0, n)).
 *   out_dev: room for out_cap_elems values of the blob's dtype.  A blob with
 *   n > out_cap_elems raises LECO_ENOSPC on the device flag. */
leco_status leco_decode_all(leco_ctx *ctx, const void *blob_dev,
                            uint64_t blob_bytes, void *out_dev,
                            uint64_t out_cap_elems, hipStream_t stream);

/* Decoder, positions [begin, end) into out_dev[0 .. end - begin)
 * (section 3.3, range decompression).  end > n raises LECO_ERANGE. */
leco_status leco_decode_range(leco_ctx *ctx, const void *blob_dev,
                              uint64_t blob_bytes, uint64_t begin, uint64_t end,
                              void *out_dev, hipStream_t stream);

/* Random access (section 3.3): out_dev[q] = value at pos_dev[q], q < k, in
 * request order.  pos_dev: k uint64 positions in device memory.  A position
 * >= n raises LECO_ERANGE and leaves out_dev[q] unspecified. */
leco_status leco_random_access(leco_ctx *ctx, const void *blob_dev,
                               uint64_t blob_bytes, const uint64_t *pos_dev,
                               uint64_t k, void *out_dev, hipStream_t stream);

/* Range-filter sum over the decoded column (the filter of section 5.1,
 * with the model-bound pruning described there): writes
 * out3_dev[0] = low 64 bits and out3_dev[1] = high 64 bits of the exact sum
 * of values v with lo <= v < hi, out3_dev[2] = their count. */
leco_status leco_filter_sum(leco_ctx *ctx, const void *blob_dev,
                            uint64_t blob_bytes, uint64_t lo, uint64_t hi,
                            uint64_t *out3_dev, hipStream_t stream);

/* ---- Batched mode -------------------------------------------------------------
 * Many columns in one launch per direction.  The paper encodes and decodes
 * one sequence at a time (section 3.3); batching only changes how the work
 * is scheduled on the GPU, never a value or a byte. */

/* One column to encode with fixed partitions (section 3.2.1).  blob_cap
 * must be at least leco_max_blob_bytes(n, dtype, {fixed_len}); the blob size
 * is written to *blob_bytes_dev. */
typedef struct {
  const void *col_dev;
  uint64_t n;
  leco_dtype dtype;
  int32_t force_constant_model;
  uint64_t fixed_len;
  void *blob_dev;
  uint64_t blob_cap;
  uint64_t *blob_bytes_dev;
  int32_t regressor; /* leco_regressor, as in leco_partitioning */
  int32_t reserved;  /* must be 0 */
} leco_encode_job;

/* Encodes every job with one sequence of launches per group of columns
 * (columns whose partitions fit one wavefront, the other least-squares and
 * minimax columns, and the polynomial-regressor columns): a fit
 * launch writes every partition's model and word count, a scan gives the
 * word offsets within each column, and a pack launch writes the residual
 * words; no partition waits for another.  Produces exactly the blobs of
 * leco_encode.  Enqueues only; jobs_host is copied before the call
 * returns. */
leco_status leco_encode_batch(leco_ctx *ctx, const leco_encode_job *jobs_host,
                              uint64_t ncols, hipStream_t stream);

/* One column to decode.  n must equal the blob's value count (checked on
 * the device).  out_dev receives the n decoded values (or is null); when
 * sum3_dev is not null it receives the exact sum (low, high 64 bits) and the
 * count of decoded values v with lo <= v < hi (the filter of section 5.1). */
typedef struct {
  const void *blob_dev;
  uint64_t blob_bytes;
  uint64_t n;
  void *out_dev;
  uint64_t lo, hi;
  uint64_t *sum3_dev;
} leco_decode_job;

typedef struct leco_batch leco_batch;

enum { LECO_BATCH_DECODE = 1, LECO_BATCH_FILTER = 2 };

/* Builds the flattened tile table of a set of columns and keeps it in
 * device memory; the jobs' buffers must stay valid while the batch is used.
 * [sync] */
leco_status leco_batch_create(leco_ctx *ctx, const leco_decode_job *jobs_host,
                              uint64_t ncols, leco_batch **out);
leco_status leco_batch_destroy(leco_batch *batch);

/* One persistent launch over all tiles of all columns: op is
 * LECO_BATCH_DECODE, LECO_BATCH_FILTER or both (fused: values are written and
 * summed in the same pass).  Capturable in a HIP graph. */
leco_status leco_batch_run(leco_batch *batch, int op, hipStream_t stream);

/* Same work replayed from a HIP graph captured on first use per op. */
leco_status leco_batch_run_graph(leco_batch *batch, int op, hipStream_t stream);

/* Times the candidate launch shapes (tile size, workgroups per CU) of this
 * batch for `op` and keeps the fastest; every candidate produces identical
 * results.  Writes the chosen shape to *tile_log2 (0: each column's own) and
 * *blocks_per_cu if not null.  [sync] */
leco_status leco_batch_tune(leco_batch *batch, int op, hipStream_t stream,
                            uint32_t *tile_log2, uint32_t *blocks_per_cu);

/* leco_batch_tune with its choice kept in a file (the tuner cache): the
 * shape chosen for a key of the device (architecture name and CU count),
 * op and batch shape (column count, total values, total blob bytes) is
 * stored as a member "<key>": {"tile_log2": T, "blocks_per_cu": B} of a
 * JSON object in cache_path (or, when cache_path is null, the file named by
 * the environment variable LECO_AUTOTUNE_CACHE; with neither this is
 * leco_batch_tune).  A key found in the file is applied without timing and
 * *from_cache (if not null) is set to 1; otherwise the batch is tuned and
 * the file rewritten with the new member (LECO_EINVAL if it cannot be
 * written).  [sync] */
leco_status leco_batch_tune_cached(leco_batch *batch, int op, const char *cache_path,
                                   hipStream_t stream, uint32_t *tile_log2,
                                   uint32_t *blocks_per_cu, int32_t *from_cache);

/* Sets the launch shape explicitly: tiles of 2^tile_log2 values (8..16) for
 * every column, or 0 for each column's own size, the largest whose residual
 * words (estimated from the column's blob bytes per value) fit one
 * wavefront's LDS slice (the default); blocks_per_cu = 0 for one workgroup
 * per tile.  EINVAL outside these ranges. */
leco_status leco_batch_set_shape(leco_batch *batch, uint32_t tile_log2,
                                 uint32_t blocks_per_cu);

/* ---- Variable-length partitioning (section 3.2.2) --------------------------------
 * Chooses partition starts for a column on the GPU, for use as
 * leco_partitioning.starts_host:
 *   split  left to right, a value joins the current partition while the
 *          approximate cost C = (len + 1) * D~new - len * D~old of including
 *          it stays within tau * sm_bits (compared in binary64), where
 *          D~ = bitlen(max d - min d) over the partition's first differences
 *          d, and while the partition holds fewer than max_len values;
 *   merge  the paper's scan over the partition list: the current partition
 *          merges with its right neighbour when the union costs strictly
 *          fewer bytes than the two apart and holds at most max_len values,
 *          sizes being the exact bytes a partition costs in a
 *          variable-length blob (32-byte record, 8-byte start, residual
 *          words, with the model the encoder chooses); after a merge the
 *          merged partition tries its next neighbour, after a refusal the
 *          neighbour becomes the current partition; passes repeat until one
 *          merges nothing or max_passes have run.
 * col_dev: n values of dtype in device memory, aligned to the dtype.  On
 * success starts_host[0..m] holds the starts (starts_host[0] = 0,
 * starts_host[m] = n) and *m_out = m; LECO_ENOSPC if starts_cap < m + 1
 * (*m_out still set).  Scratch device memory is allocated and freed by the
 * call.  [sync] */
typedef struct {
  double tau;          /* split threshold factor (the paper's range: 0..0.15) */
  uint64_t sm_bits;    /* model size S_M in bits (320: record + start)        */
  uint64_t max_len;    /* longest partition, 1..2^20                          */
  uint64_t max_passes; /* merge passes at most (0: until one merges nothing)  */
  /* 1: the split honours starting partitions (section 3.2.2, selecting good
   * starting positions, for the linear regressor): with the second-order
   * deltas dd_k = v_k - 2 v_{k-1} + v_{k-2}, each maximal run k..k' of
   * positions whose |dd_k| is the column's smallest is a starting partition
   * v[k-2, k'+1) (the later of two that would share a value keeps it); its
   * first value begins a partition and its other values join it without
   * the cost test (max_len still applies).  0: plain split. */
  int32_t start_positions;
  int32_t reserved;    /* must be 0 */
} leco_partition_params;

leco_status leco_partition(leco_ctx *ctx, const void *col_dev, uint64_t n, leco_dtype dtype,
                           const leco_partition_params *params, uint64_t *starts_host,
                           uint64_t starts_cap, uint64_t *m_out, hipStream_t stream);

/* ---- Fixed partition size search (section 3.2.1) ------------------------------
 * Picks the fixed partition length from a sample of the column: k windows
 * of `window` values at starts_host[0..k) (the caller draws the random
 * starts; the paper samples under 1% of the data), and for a length L
 *   cost(L) = sum, over every length-L partition of every window (the last
 *             one of a window shorter), of 32 + 8 * ceil(len * b / 64):
 * the record and residual words the partition adds to a blob, b being the
 * encoder's width with `regressor` (exactly what leco_encode stores), plus
 * 16 coefficient bytes per partition with LECO_REGRESSOR_POLY.
 * Requires 1 <= window <= min(n, 2^20) and starts_host[i] + window <= n;
 * col_dev is aligned to the dtype.  Scratch device memory comes from the
 * context.  [sync] */
leco_status leco_fixed_cost(leco_ctx *ctx, const void *col_dev, uint64_t n, leco_dtype dtype,
                            const uint64_t *starts_host, uint64_t k, uint64_t window,
                            uint64_t L, int32_t regressor, uint64_t *cost_host,
                            hipStream_t stream);

/* The search of section 3.2.1 over cost(L), L in [1, window]:
 *   exponential phase: L = 1, 2, 4, ... up to window, then window itself if
 *     it is not a power of two, stopping after the first L whose cost is
 *     strictly above the previous one; best = the cheapest L seen (the
 *     smallest on ties);
 *   back search: for s = best/2, best/4, ..., 1 evaluate best - s, then
 *     best + s (those in [1, window] not evaluated yet), move to the
 *     cheapest when strictly cheaper than best, and stop after s = 1 or
 *     after a move that lowers the cost by less than 0.01% of it.
 * *L_out and *cost_out receive the result; the evaluations, in order, go to
 * trace_host as (L, cost) pairs while 2 * *trace_len < trace_cap (trace_host
 * may be null).  One device evaluation per length.  [sync] */
leco_status leco_size_search(leco_ctx *ctx, const void *col_dev, uint64_t n, leco_dtype dtype,
                             const uint64_t *starts_host, uint64_t k, uint64_t window,
                             int32_t regressor, uint64_t *L_out, uint64_t *cost_out,
                             uint64_t *trace_host, uint64_t trace_cap, uint64_t *trace_len,
                             hipStream_t stream);

/* ---- Served mode --------------------------------------------------------------
 * Compressed columns stay resident in device memory while a request loop
 * answers point lookups and range scans (the decoder of section 3.3 for "one
 * or a range of positions").  Requests are admitted in arrival order when
 * output memory and an in-flight slot are free; the admitted requests are
 * packed into steps, one kernel launch each, and consecutive steps run on
 * different streams so they overlap.  A request's result stays in a
 * server-owned device buffer until the caller releases it.  Every result
 * equals what the same request returns alone. */

typedef struct leco_server leco_server;

typedef struct {
  const void *blob_dev; /* resident blob, valid until leco_server_stop */
  uint64_t blob_bytes;
  uint64_t n;           /* value count of the blob (checked at start) */
} leco_resident_col;

typedef struct {
  uint64_t out_budget_bytes;   /* device memory for results                */
  uint32_t max_inflight;       /* admitted, not yet released requests      */
  uint32_t num_streams;        /* steps that may run concurrently (>= 1)   */
  uint32_t max_step_items;     /* workgroups per step launch               */
  uint32_t max_step_positions; /* host-memory positions staged per step    */
  /* Batching: while a step is running, the next one is launched only once
   * its admitted requests produce min_step_bytes of results, fill half the
   * step, or the oldest of them has waited max_wait_us.  An idle GPU always
   * gets the next step at once.  0 disables either rule. */
  uint64_t min_step_bytes;
  uint32_t max_wait_us;
  uint32_t reserved;           /* must be 0 */
  /* Pinned host memory holding the positions of queued random-access
   * requests until their step has run (0 selects 64 MiB).  The step kernel
   * reads positions from it directly. */
  uint64_t position_ring_bytes;
} leco_server_config;

/* Request kinds.  LECO_REQ_RANDOM_ACCESS: k positions in host memory,
 * checked against n and copied into the position ring at submission (the
 * caller's buffer is free again when submit returns).
 * LECO_REQ_RANDOM_ACCESS_DEV: k positions in device memory (8-byte aligned),
 * read in place by the step kernel; the buffer must stay valid and unchanged
 * until the request completes.  They are checked on the device: a position
 * >= n yields 0 and raises the context's range flag (leco_sync reports
 * LECO_ERANGE).  LECO_REQ_RANGE: values [begin, end). */
enum { LECO_REQ_RANDOM_ACCESS = 1, LECO_REQ_RANGE = 2, LECO_REQ_RANDOM_ACCESS_DEV = 3 };

typedef struct {
  uint32_t kind;                 /* one of the request kinds above             */
  uint32_t col;                  /* resident column index                      */
  const uint64_t *positions;     /* random access: k positions (host or device) */
  uint64_t k;
  uint64_t begin, end;           /* range: positions [begin, end)              */
} leco_request;

typedef struct {
  uint64_t ticket;
  int32_t status;          /* LECO_OK, or the error that ended the request     */
  int32_t dtype;           /* 4 or 8                                           */
  /* count values, valid until leco_server_release; aligned to the value
   * width (a range's values are placed with value g at g * width modulo
   * 256 bytes, so that the decoder's stores line up with cache lines) */
  const void *out_dev;
  uint64_t count;
  double latency_us;       /* submit to observed completion of its step        */
} leco_completion;

typedef struct {
  uint64_t submitted, completed, steps, values_out, positions;
  uint64_t out_bytes_in_use, out_bytes_peak, queued;
  uint64_t items; /* work items launched (workgroups of the step kernels) */
  /* Host time of the request loop in nanoseconds: submission (checks,
   * position copies, queueing), admission of queued requests into a step
   * (under the server's lock), building the step's work items, launching it
   * (work-item copy, kernel launch, events), retiring finished steps
   * (event queries, completions), and the loop's waits for work or for a
   * step to finish. */
  uint64_t host_submit_ns, host_admit_ns, host_build_ns, host_launch_ns, host_retire_ns,
      host_wait_ns;
  /* Device time from timing events recorded around each step on its
   * stream: the sum of the steps' durations, the time covered by at least
   * one step (the union of their intervals) and the span from the earliest
   * start to the latest end, in nanoseconds, over the steps retired. */
  uint64_t gpu_step_ns, gpu_busy_ns, gpu_span_ns;
} leco_server_stats;

/* Starts the request loop (one host thread) over resident columns. [sync] */
leco_status leco_server_start(leco_ctx *ctx, const leco_resident_col *cols_host,
                              uint64_t ncols, const leco_server_config *cfg,
                              leco_server **out);
/* Queues a request; never blocks on the GPU.  Host positions are checked
 * against n and copied into the position ring here (LECO_ERANGE; LECO_ENOMEM
 * when the ring is momentarily full: retry once earlier requests complete);
 * a request larger than the whole budget is refused (LECO_ENOSPC), one
 * larger than a step (max_step_items workgroups: 256 lookups each, or for a
 * range one each per tile of the column's decode grid that it touches,
 * tiles of 2^8 to 2^14 values from position 0, the most whose residual
 * words fit a workgroup's staging memory at the column's bits per value) is
 * LECO_EINVAL.  A request's latency runs from the start of this call. */
leco_status leco_server_submit(leco_server *s, const leco_request *req,
                               uint64_t *ticket);
/* Queues reqs[0..n) in order with one acquisition of the server's lock,
 * stopping at the first request that fails (its status is returned;
 * *accepted, if not null, receives how many were queued and tickets[0..
 * *accepted) their tickets).  The checks and errors are leco_server_submit's. */
leco_status leco_server_submit_batch(leco_server *s, const leco_request *reqs, uint64_t n,
                                     uint64_t *tickets, uint64_t *accepted);
/* Returns up to max completions (non-blocking). */
leco_status leco_server_poll(leco_server *s, leco_completion *out, uint64_t max,
                             uint64_t *got);
/* Frees a completed request's result memory. */
leco_status leco_server_release(leco_server *s, uint64_t ticket);
leco_status leco_server_stats_get(leco_server *s, leco_server_stats *out);
/* Zeroes the counters and timers above (not out_bytes_in_use or queued) and
 * forgets the step intervals retired so far. */
leco_status leco_server_stats_reset(leco_server *s);
/* Waits for every admitted step, stops the loop and frees the server. */
leco_status leco_server_stop(leco_server *s);

/* Open-loop load generator: submits reqs[i] at arrival_s[i] seconds after
 * the call (busy-waiting), releases each result as it completes, and waits
 * for all of them.  latency_us_out (n entries, may be null) receives each
 * request's latency from its scheduled arrival (so a generator that falls
 * behind is charged for it) to the observed completion of its step;
 * *elapsed_s the time from the first arrival to the last completion. */
leco_status leco_server_replay(leco_server *s, const leco_request *reqs,
                               const double *arrival_s, uint64_t n,
                               double *latency_us_out, double *elapsed_s);

/* The plain path, the baseline the served loop is measured against: the
 * same request stream replayed at arrival_s[i] seconds after the call
 * (busy-waiting), each request as its own leco_random_access or
 * leco_decode_range launch on `stream` (no batching, no overlap), in
 * arrival order, with an event after each.  Requests are ranges or
 * random-access batches with device positions (LECO_REQ_RANDOM_ACCESS_DEV)
 * on cols_host[req.col]; every result goes to out_dev, which must hold the
 * largest request's values (out_bytes; LECO_ENOSPC otherwise).
 * latency_us_out[i] (may be null) receives the time from request i's
 * scheduled arrival to the observed completion of its event; *elapsed_s
 * the time from the first arrival to the last completion.  [sync] */
leco_status leco_plain_replay(leco_ctx *ctx, const leco_resident_col *cols_host, uint64_t ncols,
                              const leco_request *reqs, const double *arrival_s, uint64_t n,
                              void *out_dev, uint64_t out_bytes, hipStream_t stream,
                              double *latency_us_out, double *elapsed_s);

/* ---- Diagnostics ------------------------------------------------------------
 * Evaluates the slope arithmetic of the encoder (section 3.1, least-squares
 * closed form) on the GPU for k given pairs: in_dev holds 4 uint64 per pair,
 * (N low, N high) as a two's-complement int128 and (D low, D high) as an
 * unsigned int128 (D > 0); out_dev[i] = fl(N) / fl(D), with each integer
 * rounded to nearest-even binary64 and one IEEE division, -0.0 mapped to
 * +0.0 -- exactly the encoder's theta1. */
leco_status leco_diag_slope(leco_ctx *ctx, const uint64_t *in_dev, uint64_t k,
                            double *out_dev, hipStream_t stream);

/* Streaming copy of `bytes` (a multiple of 16, both buffers 16-byte
 * aligned) from src_dev to dst_dev, or a zero fill of dst_dev when src_dev
 * is null: a plain HBM-bound reference kernel of known traffic, used to
 * calibrate bandwidth measurements and hardware traffic counters. */
leco_status leco_diag_copy(leco_ctx *ctx, const void *src_dev, void *dst_dev,
                           uint64_t bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* LECO_H */
