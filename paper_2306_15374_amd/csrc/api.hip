// C ABI of the LeCo HIP library: argument checks on the host, scratch
// management, the device error flag, and dispatch to the kernels.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <map>
#include <mutex>
#include <vector>

#include "internal.hpp"
#include "leco_dev.hpp"

using leco::kMaxPartLen;

// Device scratch of the encoder variant that allocates nothing
// (leco_encode_noalloc): a fixed array in every GPU's memory for the whole
// process.  Its name is only a host-side stand-in; host code uses the
// per-device address that noalloc_scratch_address looks up.
constexpr size_t kNoAllocScratchBytes = size_t(LECO_NOALLOC_SCRATCH_BYTES);
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {

// Address of `scratch` on the current device, looked up once per device.
hipError_t noalloc_scratch_address(int device, void** out) {
  static std::mutex mu;
  static std::map<int, void*> addr;
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(device);
  if (it != addr.end()) {
    *out = it->second;
    return hipSuccess;
  }
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  addr[device] = ptr;
  *out = ptr;
  return hipSuccess;
}

leco_status fail(leco_ctx* ctx, leco_status st, const char* fmt, ...) {
  if (ctx) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    ctx->last_error = buf;
  }
  return st;
}

leco_status hip_fail(leco_ctx* ctx, hipError_t e, const char* what) {
  return fail(ctx, LECO_EDEVICE, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                               \
  do {                                                   \
    hipError_t e_ = (expr);                              \
    if (e_ != hipSuccess) return hip_fail(ctx, e_, #expr); \
  } while (0)

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; }

// Returns a device scratch area of at least `bytes`.  Growing it waits for
// the whole device first, so no queued kernel still uses the old area.
leco_status get_scratch(leco_ctx* ctx, size_t bytes, void** out) {
  if (bytes <= ctx->scratch_bytes) {
    *out = ctx->scratch;
    return LECO_OK;
  }
  HIP_TRY(ctx, hipDeviceSynchronize());
  if (ctx->scratch) HIP_TRY(ctx, hipFree(ctx->scratch));
  ctx->scratch = nullptr;
  ctx->scratch_bytes = 0;
  size_t sz = bytes + bytes / 4 + 4096;
  hipError_t e = hipMalloc(&ctx->scratch, sz);
  if (e != hipSuccess) return fail(ctx, LECO_ENOMEM, "scratch allocation of %zu bytes failed", sz);
  ctx->scratch_bytes = sz;
  *out = ctx->scratch;
  return LECO_OK;
}

bool valid_regressor(int32_t r) {
  return r == LECO_REGRESSOR_LS || r == LECO_REGRESSOR_MINIMAX || r == LECO_REGRESSOR_POLY;
}

// Partition count and validation of a partitioning for n values.
leco_status check_partitioning(leco_ctx* ctx, uint64_t n, const leco_partitioning* part,
                               uint64_t* m_out, uint64_t* max_len_out = nullptr) {
  if (!part) return fail(ctx, LECO_EINVAL, "partitioning is null");
  if (!valid_regressor(part->regressor))
    return fail(ctx, LECO_EINVAL, "unknown regressor %d", int(part->regressor));
  if (part->fixed_len > 0) {
    if (part->fixed_len > kMaxPartLen)
      return fail(ctx, LECO_EINVAL, "fixed_len %llu exceeds 2^20",
                  (unsigned long long)part->fixed_len);
    *m_out = n / part->fixed_len + (n % part->fixed_len != 0);
    if (max_len_out) *max_len_out = n < part->fixed_len ? n : part->fixed_len;
    return LECO_OK;
  }
  const uint64_t m = part->num_partitions;
  const uint64_t* s = part->starts_host;
  if (!s) return fail(ctx, LECO_EINVAL, "starts_host is null for variable partitioning");
  if (s[0] != 0 || s[m] != n)
    return fail(ctx, LECO_EINVAL, "starts must begin at 0 and end at n");
  uint64_t longest = 0;
  for (uint64_t j = 0; j < m; ++j) {
    if (s[j + 1] <= s[j])
      return fail(ctx, LECO_EINVAL, "starts not strictly increasing at %llu",
                  (unsigned long long)j);
    if (s[j + 1] - s[j] > kMaxPartLen)
      return fail(ctx, LECO_EINVAL, "partition %llu longer than 2^20", (unsigned long long)j);
    if (s[j + 1] - s[j] > longest) longest = s[j + 1] - s[j];
  }
  *m_out = m;
  if (max_len_out) *max_len_out = longest;
  return LECO_OK;
}

// Offset of the words section: header, records, starts (variable), and the
// (c2, c3) coefficient section of the polynomial regressor.
uint64_t meta_words_off(uint64_t m, bool variable, bool poly) {
  uint64_t end = leco::kHeaderBytes + leco::kRecordBytes * m + (variable ? 8 * (m + 1) : 0);
  if (poly) end = leco::align16(end) + 16 * m;
  return leco::align16(end);
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// One single-column encode: the column descriptor plus its scratch.
struct EncodeCall {
  leco::EncColumn col;
  uint64_t max_len;             // longest partition
  leco::EncScratch scr;         // models, word counts and offsets
  uint64_t* size_dev;           // blob size (scratch; used when the caller gives none)
};

// Checks the arguments, carves the encode scratch and copies variable starts.
// The scratch is the context's (grown as needed), or when fixed is given the
// fixed_bytes at fixed (LECO_ENOSPC if the call needs more).
leco_status prepare_encode(leco_ctx* ctx, const void* col, uint64_t n, leco_dtype dtype,
                           const leco_partitioning* part, void* blob, uint64_t cap,
                           hipStream_t stream, EncodeCall* call, void* fixed = nullptr,
                           size_t fixed_bytes = 0) {
  if (dtype != LECO_U32 && dtype != LECO_U64) return fail(ctx, LECO_EINVAL, "bad dtype");
  if (n > 0 && !col) return fail(ctx, LECO_EINVAL, "column is null");
  if (!blob) return fail(ctx, LECO_EINVAL, "blob is null");
  if (!aligned16(blob) || (n > 0 && (reinterpret_cast<uintptr_t>(col) % dtype) != 0))
    return fail(ctx, LECO_EINVAL, "blob must be 16-byte aligned and column dtype-aligned");
  if (cap < leco::kHeaderBytes) return fail(ctx, LECO_ENOSPC, "blob capacity below 64 bytes");
  uint64_t m = 0;
  leco_status st = check_partitioning(ctx, n, part, &m, &call->max_len);
  if (st != LECO_OK) return st;
  if (m >= (uint64_t(1) << 31)) return fail(ctx, LECO_EINVAL, "too many partitions");
  const bool variable = part->fixed_len == 0;
  size_t off = 0;
  const size_t o_enc = off;    off = align256(off + leco::encode_scratch_bytes(m));
  const size_t o_misc = off;   off = align256(off + 16);
  const size_t o_starts = off; off = align256(off + (variable ? 8 * (m + 1) : 8));
  const bool hulls = part->regressor == LECO_REGRESSOR_MINIMAX && call->max_len > leco::kHullTileValues;
  const size_t o_hull = off;   off = align256(off + (hulls ? 8 * n : 0));
  void* scr = nullptr;
  if (fixed) {
    if (off > fixed_bytes)
      return fail(ctx, LECO_ENOSPC, "encode needs %zu bytes of scratch, the fixed scratch holds %zu",
                  off, fixed_bytes);
    scr = fixed;
  } else {
    st = get_scratch(ctx, off, &scr);
    if (st != LECO_OK) return st;
  }
  char* b = static_cast<char*>(scr);
  leco::EncColumn& c = call->col;
  c.col = static_cast<const uint8_t*>(col);
  c.blob = static_cast<uint8_t*>(blob);
  c.starts = nullptr;
  c.n = n;
  c.m = m;
  c.fixed_len = part->fixed_len;
  c.cap = cap;
  c.words_off = meta_words_off(m, variable, part->regressor == LECO_REGRESSOR_POLY);
  c.part_base = 0;
  c.dtype = uint32_t(dtype);
  c.force_constant = part->force_constant_model ? 1 : 0;
  c.regressor = uint32_t(part->regressor);
  c.pad = 0;
  c.val_base = 0;
  call->scr = leco::carve_encode_scratch(b + o_enc, m);
  if (hulls) {
    call->scr.hull = reinterpret_cast<uint32_t*>(b + o_hull);
    call->scr.hull_values = n;
  }
  call->size_dev = reinterpret_cast<uint64_t*>(b + o_misc);
  c.size_out = call->size_dev;
  if (variable) {
    uint64_t* sd = reinterpret_cast<uint64_t*>(b + o_starts);
    HIP_TRY(ctx, hipMemcpyAsync(sd, part->starts_host, 8 * (m + 1), hipMemcpyHostToDevice, stream));
    c.starts = sd;
  }
  return LECO_OK;
}

leco_status check_blob_args(leco_ctx* ctx, const void* blob, uint64_t blob_bytes) {
  if (!ctx) return LECO_EINVAL;
  if (!blob) return fail(ctx, LECO_EINVAL, "blob is null");
  if (!aligned16(blob)) return fail(ctx, LECO_EINVAL, "blob must be 16-byte aligned");
  if (blob_bytes < leco::kHeaderBytes) return fail(ctx, LECO_EFORMAT, "blob shorter than its header");
  return LECO_OK;
}

uint64_t rd64(const uint8_t* p) {
  uint64_t x;
  memcpy(&x, p, 8);
  return x;
}

}  // namespace

extern "C" {

leco_status leco_create(int hip_device, leco_ctx** out) {
  if (!out) return LECO_EINVAL;
  *out = nullptr;
  int count = 0;
  if (hipGetDeviceCount(&count) != hipSuccess || hip_device < 0 || hip_device >= count)
    return LECO_EDEVICE;
  if (hipSetDevice(hip_device) != hipSuccess) return LECO_EDEVICE;
  leco_ctx* ctx = new leco_ctx();
  ctx->device = hip_device;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess) {
    delete ctx;
    return LECO_EDEVICE;
  }
  ctx->num_cus = prop.multiProcessorCount;
  leco::tune_from_env(ctx->tune);
  if (hipMalloc(&ctx->err_dev, 256) != hipSuccess ||
      hipHostMalloc(&ctx->err_host, 256, hipHostMallocDefault) != hipSuccess) {
    leco_destroy(ctx);
    return LECO_ENOMEM;
  }
  ctx->pinned_u64 = reinterpret_cast<uint64_t*>(reinterpret_cast<char*>(ctx->err_host) + 64);
  if (hipMemset(ctx->err_dev, 0, 256) != hipSuccess ||
      noalloc_scratch_address(hip_device, &ctx->noalloc_scratch) != hipSuccess) {
    leco_destroy(ctx);
    return LECO_EDEVICE;
  }
  *out = ctx;
  return LECO_OK;
}

leco_status leco_destroy(leco_ctx* ctx) {
  if (!ctx) return LECO_OK;
  (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (ctx->scratch) (void)hipFree(ctx->scratch);
  if (ctx->err_dev) (void)hipFree(ctx->err_dev);
  if (ctx->err_host) (void)hipHostFree(ctx->err_host);
  delete ctx;
  return LECO_OK;
}

const char* leco_last_error(const leco_ctx* ctx) {
  return ctx ? ctx->last_error.c_str() : "no context";
}

leco_status leco_sync(leco_ctx* ctx, hipStream_t stream) {
  if (!ctx) return LECO_EINVAL;
  HIP_TRY(ctx, hipMemcpyAsync(ctx->err_host, ctx->err_dev, sizeof(int), hipMemcpyDeviceToHost, stream));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  const int bits = *ctx->err_host;
  if (bits == 0) return LECO_OK;
  *ctx->err_host = 0;
  HIP_TRY(ctx, hipMemcpyAsync(ctx->err_dev, ctx->err_host, sizeof(int), hipMemcpyHostToDevice, stream));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  if (bits & leco::kErrDevice) return fail(ctx, LECO_EDEVICE, "a kernel's bounded wait expired");
  if (bits & leco::kErrFormat) return fail(ctx, LECO_EFORMAT, "a kernel found the blob malformed");
  if (bits & leco::kErrRange) return fail(ctx, LECO_ERANGE, "a position or range lies outside [0, n)");
  return fail(ctx, LECO_ENOSPC, "an output buffer was too small");
}

leco_status leco_max_blob_bytes(uint64_t n, leco_dtype dtype, const leco_partitioning* part,
                                uint64_t* bytes) {
  if (!bytes || (dtype != LECO_U32 && dtype != LECO_U64)) return LECO_EINVAL;
  uint64_t m = 0;
  leco_status st = check_partitioning(nullptr, n, part, &m);
  if (st != LECO_OK) return st;
  // every partition at full width: ceil(n_j * 8w / 64) <= n_j * w / 8 + 1
  const uint64_t words = (n * uint64_t(dtype) + 7) / 8 + m;
  *bytes = leco::align16(meta_words_off(m, part->fixed_len == 0,
                                        part->regressor == LECO_REGRESSOR_POLY) + 8 * words);
  return LECO_OK;
}

leco_status leco_blob_info(const void* header_host, uint64_t* n, leco_dtype* dtype, uint64_t* m) {
  if (!header_host) return LECO_EINVAL;
  const uint8_t* h = static_cast<const uint8_t*>(header_host);
  uint32_t magic;
  memcpy(&magic, h, 4);
  const uint16_t version = uint16_t(h[4] | (h[5] << 8));
  if (magic != leco::kMagic || version != leco::kVersion || (h[6] != 4 && h[6] != 8))
    return LECO_EFORMAT;
  if (n) *n = rd64(h + 8);
  if (dtype) *dtype = leco_dtype(h[6]);
  if (m) *m = rd64(h + 16);
  return LECO_OK;
}

leco_status leco_validate_blob(leco_ctx* ctx, const void* blob_dev, uint64_t blob_bytes,
                               hipStream_t stream) {
  leco_status st = check_blob_args(ctx, blob_dev, blob_bytes);
  if (st != LECO_OK) return st;
  uint8_t hdr[64];
  HIP_TRY(ctx, hipMemcpyAsync(hdr, blob_dev, 64, hipMemcpyDeviceToHost, stream));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  uint32_t magic;
  memcpy(&magic, hdr, 4);
  const uint16_t version = uint16_t(hdr[4] | (hdr[5] << 8));
  const uint32_t dtype = hdr[6], flags = hdr[7];
  const uint32_t variable = flags & leco::kFlagVariable;
  const bool poly = (flags & leco::kFlagPoly) != 0;
  const uint64_t n = rd64(hdr + 8), m = rd64(hdr + 16), L = rd64(hdr + 24);
  const uint64_t rec_off = rd64(hdr + 32), st_off = rd64(hdr + 40), w_off = rd64(hdr + 48),
                 tw = rd64(hdr + 56);
  if (magic != leco::kMagic || version != leco::kVersion)
    return fail(ctx, LECO_EFORMAT, "bad magic or version");
  if ((dtype != 4 && dtype != 8) || flags > (leco::kFlagVariable | leco::kFlagPoly) || rec_off != 64)
    return fail(ctx, LECO_EFORMAT, "bad dtype, flags or records offset");
  if (m > blob_bytes / 32) return fail(ctx, LECO_EFORMAT, "partition count exceeds blob");
  if (variable) {
    if (L != 0 || st_off != 64 + 32 * m) return fail(ctx, LECO_EFORMAT, "bad starts section");
  } else {
    if (L == 0 || L > kMaxPartLen || st_off != 0 || m != n / L + (n % L != 0))
      return fail(ctx, LECO_EFORMAT, "bad fixed partitioning");
  }
  if (w_off != meta_words_off(m, variable, poly)) return fail(ctx, LECO_EFORMAT, "bad words offset");
  if (tw > blob_bytes / 8 || leco::align16(w_off + 8 * tw) > blob_bytes)
    return fail(ctx, LECO_EFORMAT, "words section exceeds blob");
  std::vector<uint8_t> meta(w_off);
  HIP_TRY(ctx, hipMemcpyAsync(meta.data(), blob_dev, w_off, hipMemcpyDeviceToHost, stream));
  HIP_TRY(ctx, hipStreamSynchronize(stream));
  uint64_t expect_off = 0;
  for (uint64_t j = 0; j < m; ++j) {
    const uint8_t* r = meta.data() + 64 + 32 * j;
    uint64_t s0, s1;
    if (variable) {
      s0 = rd64(meta.data() + st_off + 8 * j);
      s1 = rd64(meta.data() + st_off + 8 * (j + 1));
      if (j == 0 && s0 != 0) return fail(ctx, LECO_EFORMAT, "starts[0] != 0");
      if (s1 <= s0 || s1 - s0 > kMaxPartLen) return fail(ctx, LECO_EFORMAT, "bad start %llu", (unsigned long long)j);
    } else {
      s0 = j * L;
      s1 = s0 + L < n ? s0 + L : n;
    }
    const uint64_t bits = r[24];
    if (bits > 8 * dtype) return fail(ctx, LECO_EFORMAT, "width too large in partition %llu", (unsigned long long)j);
    if (r[25] > (poly ? 1 : 0)) return fail(ctx, LECO_EFORMAT, "bad model kind in partition %llu", (unsigned long long)j);
    if (r[25] && s1 - s0 > leco::kPolyMaxLen)
      return fail(ctx, LECO_EFORMAT, "polynomial partition %llu longer than 4096", (unsigned long long)j);
    for (int k = 26; k < 32; ++k)
      if (r[k]) return fail(ctx, LECO_EFORMAT, "nonzero record padding");
    if (rd64(r + 16) != expect_off) return fail(ctx, LECO_EFORMAT, "word offsets not contiguous");
    expect_off += ((s1 - s0) * bits + 63) / 64;
  }
  if (variable && m > 0 && rd64(meta.data() + st_off + 8 * m) != n)
    return fail(ctx, LECO_EFORMAT, "starts[m] != n");
  if (expect_off != tw) return fail(ctx, LECO_EFORMAT, "word count mismatch");
  return LECO_OK;
}

static leco_status encode_common(leco_ctx* ctx, const void* col, uint64_t n, leco_dtype dtype,
                                 const leco_partitioning* part, void* blob, uint64_t cap,
                                 uint64_t* size_dev, hipStream_t stream, EncodeCall* call,
                                 void* fixed = nullptr, size_t fixed_bytes = 0) {
  if (!ctx) return LECO_EINVAL;
  leco_status st = prepare_encode(ctx, col, n, dtype, part, blob, cap, stream, call, fixed,
                                  fixed_bytes);
  if (st != LECO_OK) return st;
  if (size_dev) call->col.size_out = size_dev;
  HIP_TRY(ctx, leco::launch_encode_columns(ctx, nullptr, 1, call->col, call->col.m, call->max_len,
                                           leco::regressor_bit(call->col.regressor), call->scr,
                                           stream));
  return LECO_OK;
}

leco_status leco_encode(leco_ctx* ctx, const void* col_dev, uint64_t n, leco_dtype dtype,
                        const leco_partitioning* part, void* blob_dev, uint64_t blob_cap,
                        uint64_t* blob_bytes_host, hipStream_t stream) {
  EncodeCall call;
  leco_status st = encode_common(ctx, col_dev, n, dtype, part, blob_dev, blob_cap, nullptr,
                                 stream, &call);
  if (st != LECO_OK) return st;
  HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned_u64, call.size_dev, 8, hipMemcpyDeviceToHost, stream));
  st = leco_sync(ctx, stream);
  const uint64_t size = *ctx->pinned_u64;
  if (blob_bytes_host) *blob_bytes_host = size;
  if (st == LECO_ENOSPC || size > blob_cap)
    return fail(ctx, LECO_ENOSPC, "blob needs %llu bytes, capacity is %llu",
                (unsigned long long)size, (unsigned long long)blob_cap);
  return st;
}

leco_status leco_encode_async(leco_ctx* ctx, const void* col_dev, uint64_t n, leco_dtype dtype,
                              const leco_partitioning* part, void* blob_dev, uint64_t blob_cap,
                              uint64_t* blob_bytes_dev, hipStream_t stream) {
  if (!ctx) return LECO_EINVAL;
  if (!blob_bytes_dev) return fail(ctx, LECO_EINVAL, "blob_bytes_dev is null");
  uint64_t bound = 0;
  leco_status st = leco_max_blob_bytes(n, dtype, part, &bound);
  if (st != LECO_OK) return fail(ctx, st, "bad encode arguments");
  if (blob_cap < bound)
    return fail(ctx, LECO_ENOSPC, "async encode needs capacity %llu", (unsigned long long)bound);
  EncodeCall call;
  return encode_common(ctx, col_dev, n, dtype, part, blob_dev, blob_cap, blob_bytes_dev, stream,
                       &call);
}

leco_status leco_encode_noalloc(leco_ctx* ctx, const void* col_dev, uint64_t n, leco_dtype dtype,
                                const leco_partitioning* part, void* blob_dev, uint64_t blob_cap,
                                uint64_t* blob_bytes_dev, hipStream_t stream) {
  if (!ctx) return LECO_EINVAL;
  if (!blob_bytes_dev) return fail(ctx, LECO_EINVAL, "blob_bytes_dev is null");
  if (!ctx->noalloc_scratch) return fail(ctx, LECO_EDEVICE, "no fixed scratch on this device");
  uint64_t bound = 0;
  leco_status st = leco_max_blob_bytes(n, dtype, part, &bound);
  if (st != LECO_OK) return fail(ctx, st, "bad encode arguments");
  if (blob_cap < bound)
    return fail(ctx, LECO_ENOSPC, "encode needs capacity %llu", (unsigned long long)bound);
  HIP_TRY(ctx, hipSetDevice(ctx->device));
  EncodeCall call;
  return encode_common(ctx, col_dev, n, dtype, part, blob_dev, blob_cap, blob_bytes_dev, stream,
                       &call, ctx->noalloc_scratch, kNoAllocScratchBytes);
}

leco_status leco_encode_batch(leco_ctx* ctx, const leco_encode_job* jobs, uint64_t ncols,
                              hipStream_t stream) {
  if (!ctx) return LECO_EINVAL;
  if (ncols && !jobs) return fail(ctx, LECO_EINVAL, "jobs is null");
  // Columns whose partitions fit one wavefront go to one sequence of
  // launches, the others to a second, columns with the polynomial regressor
  // to a third.
  constexpr int kGroups = 3;
  std::vector<leco::EncColumn> cols[kGroups];
  uint64_t parts[kGroups] = {0, 0, 0}, longest[kGroups] = {0, 0, 0}, values[kGroups] = {0, 0, 0};
  bool minimax[kGroups] = {false, false, false};
  uint32_t regs[kGroups] = {0, 0, 0};
  for (uint64_t i = 0; i < ncols; ++i) {
    const leco_encode_job& j = jobs[i];
    if (j.dtype != LECO_U32 && j.dtype != LECO_U64) return fail(ctx, LECO_EINVAL, "job %llu: bad dtype", (unsigned long long)i);
    if (j.fixed_len == 0 || j.fixed_len > kMaxPartLen)
      return fail(ctx, LECO_EINVAL, "job %llu: fixed_len must be in [1, 2^20]", (unsigned long long)i);
    if ((j.n && !j.col_dev) || !j.blob_dev || !j.blob_bytes_dev || !aligned16(j.blob_dev) ||
        (reinterpret_cast<uintptr_t>(j.col_dev) % j.dtype))
      return fail(ctx, LECO_EINVAL, "job %llu: null or misaligned buffer", (unsigned long long)i);
    if (!valid_regressor(j.regressor) || j.reserved != 0)
      return fail(ctx, LECO_EINVAL, "job %llu: bad regressor or reserved field", (unsigned long long)i);
    leco_partitioning part{j.fixed_len, nullptr, 0, j.force_constant_model, j.regressor};
    uint64_t bound = 0;
    leco_max_blob_bytes(j.n, j.dtype, &part, &bound);
    if (j.blob_cap < bound)
      return fail(ctx, LECO_ENOSPC, "job %llu: capacity below %llu", (unsigned long long)i,
                  (unsigned long long)bound);
    const uint64_t len = j.n < j.fixed_len ? j.n : j.fixed_len;
    const int g = j.regressor == LECO_REGRESSOR_POLY ? 2 : len <= leco::kWaveEncodeMax ? 0 : 1;
    leco::EncColumn c;
    c.col = static_cast<const uint8_t*>(j.col_dev);
    c.blob = static_cast<uint8_t*>(j.blob_dev);
    c.starts = nullptr;
    c.size_out = j.blob_bytes_dev;
    c.n = j.n;
    c.m = j.n / j.fixed_len + (j.n % j.fixed_len != 0);
    c.fixed_len = j.fixed_len;
    c.cap = j.blob_cap;
    c.words_off = meta_words_off(c.m, false, j.regressor == LECO_REGRESSOR_POLY);
    c.part_base = parts[g];
    c.dtype = uint32_t(j.dtype);
    c.force_constant = j.force_constant_model ? 1 : 0;
    c.regressor = uint32_t(j.regressor);
    c.pad = 0;
    c.val_base = values[g];
    parts[g] += c.m;
    values[g] += c.n;
    if (len > longest[g]) longest[g] = len;
    if (j.regressor == LECO_REGRESSOR_MINIMAX) minimax[g] = true;
    regs[g] |= leco::regressor_bit(uint32_t(j.regressor));
    cols[g].push_back(c);
  }
  if (ncols == 0) return LECO_OK;
  for (int g = 0; g < kGroups; ++g)
    if (parts[g] >= (uint64_t(1) << 31))
      return fail(ctx, LECO_EINVAL, "too many partitions in one batch");
  size_t off = 0, o_enc[kGroups], o_cols[kGroups], o_hull[kGroups];
  bool hulls[kGroups];
  for (int g = 0; g < kGroups; ++g) {
    hulls[g] = minimax[g] && longest[g] > leco::kHullTileValues;
    o_enc[g] = off;  off = align256(off + leco::encode_scratch_bytes(parts[g]));
    o_cols[g] = off; off = align256(off + sizeof(leco::EncColumn) * (cols[g].size() + 1));
    o_hull[g] = off; off = align256(off + (hulls[g] ? 8 * values[g] : 0));
  }
  void* scr = nullptr;
  leco_status st = get_scratch(ctx, off, &scr);
  if (st != LECO_OK) return st;
  char* b = static_cast<char*>(scr);
  for (int g = 0; g < kGroups; ++g) {
    if (cols[g].empty()) continue;
    leco::EncColumn* cols_dev = reinterpret_cast<leco::EncColumn*>(b + o_cols[g]);
    HIP_TRY(ctx, hipMemcpyAsync(cols_dev, cols[g].data(), sizeof(leco::EncColumn) * cols[g].size(),
                                hipMemcpyHostToDevice, stream));
    leco::EncScratch es = leco::carve_encode_scratch(b + o_enc[g], parts[g]);
    if (hulls[g]) {
      es.hull = reinterpret_cast<uint32_t*>(b + o_hull[g]);
      es.hull_values = values[g];
    }
    HIP_TRY(ctx, leco::launch_encode_columns(ctx, cols_dev, cols[g].size(), cols[g][0], parts[g],
                                             longest[g], regs[g], es, stream));
  }
  return LECO_OK;
}

leco_status leco_decode_all(leco_ctx* ctx, const void* blob_dev, uint64_t blob_bytes,
                            void* out_dev, uint64_t out_cap_elems, hipStream_t stream) {
  leco_status st = check_blob_args(ctx, blob_dev, blob_bytes);
  if (st != LECO_OK) return st;
  if (!out_dev && out_cap_elems) return fail(ctx, LECO_EINVAL, "output is null");
  if (!aligned16(out_dev)) return fail(ctx, LECO_EINVAL, "output must be 16-byte aligned");
  HIP_TRY(ctx, leco::launch_decode(ctx, blob_dev, blob_bytes, out_dev, 0, 0, out_cap_elems, true, stream));
  return LECO_OK;
}

leco_status leco_decode_range(leco_ctx* ctx, const void* blob_dev, uint64_t blob_bytes,
                              uint64_t begin, uint64_t end, void* out_dev, hipStream_t stream) {
  leco_status st = check_blob_args(ctx, blob_dev, blob_bytes);
  if (st != LECO_OK) return st;
  if (begin > end) return fail(ctx, LECO_ERANGE, "begin > end");
  if (end > begin && !out_dev) return fail(ctx, LECO_EINVAL, "output is null");
  HIP_TRY(ctx, leco::launch_decode(ctx, blob_dev, blob_bytes, out_dev, begin, end, 0, false, stream));
  return LECO_OK;
}

leco_status leco_random_access(leco_ctx* ctx, const void* blob_dev, uint64_t blob_bytes,
                               const uint64_t* pos_dev, uint64_t k, void* out_dev,
                               hipStream_t stream) {
  leco_status st = check_blob_args(ctx, blob_dev, blob_bytes);
  if (st != LECO_OK) return st;
  if (k && (!pos_dev || !out_dev)) return fail(ctx, LECO_EINVAL, "positions or output is null");
  if (k > (uint64_t(1) << 40)) return fail(ctx, LECO_EINVAL, "too many positions");
  HIP_TRY(ctx, leco::launch_random_access(ctx, blob_dev, blob_bytes, pos_dev, k, out_dev, stream));
  return LECO_OK;
}

leco_status leco_filter_sum(leco_ctx* ctx, const void* blob_dev, uint64_t blob_bytes, uint64_t lo,
                            uint64_t hi, uint64_t* out3_dev, hipStream_t stream) {
  leco_status st = check_blob_args(ctx, blob_dev, blob_bytes);
  if (st != LECO_OK) return st;
  if (!out3_dev) return fail(ctx, LECO_EINVAL, "output is null");
  HIP_TRY(ctx, leco::launch_filter_sum(ctx, blob_dev, blob_bytes, lo, hi, out3_dev, true, stream));
  return LECO_OK;
}

// ---- fixed partition size search (section 3.2.1) ----------------------------------

static leco_status check_windows(leco_ctx* ctx, const void* col, uint64_t n, leco_dtype dtype,
                                 const uint64_t* starts, uint64_t k, uint64_t window,
                                 int32_t regressor) {
  if (!ctx) return LECO_EINVAL;
  if (dtype != LECO_U32 && dtype != LECO_U64) return fail(ctx, LECO_EINVAL, "bad dtype");
  if (!col || (reinterpret_cast<uintptr_t>(col) % dtype) != 0)
    return fail(ctx, LECO_EINVAL, "column is null or misaligned");
  if (!valid_regressor(regressor))
    return fail(ctx, LECO_EINVAL, "unknown regressor %d", int(regressor));
  if (k == 0 || !starts) return fail(ctx, LECO_EINVAL, "no sample windows");
  if (window == 0 || window > n || window > kMaxPartLen)
    return fail(ctx, LECO_EINVAL, "window must be in [1, min(n, 2^20)]");
  if (k > (uint64_t(1) << 31) / window) return fail(ctx, LECO_EINVAL, "too many sampled values");
  for (uint64_t i = 0; i < k; ++i)
    if (starts[i] > n - window)
      return fail(ctx, LECO_EINVAL, "window %llu runs past the column", (unsigned long long)i);
  return LECO_OK;
}

// cost(L) over the windows: every window is a column of the fit launch.
static leco_status sampled_cost(leco_ctx* ctx, const void* col, leco_dtype dtype,
                                const uint64_t* starts, uint64_t k, uint64_t window, uint64_t L,
                                int32_t regressor, hipStream_t stream, uint64_t* cost) {
  const uint64_t m = window / L + (window % L != 0);
  const uint64_t nparts = k * m;
  if (nparts >= (uint64_t(1) << 31)) return fail(ctx, LECO_EINVAL, "too many sampled partitions");
  const bool minimax = regressor == LECO_REGRESSOR_MINIMAX;
  const bool hulls = minimax && L > leco::kHullTileValues;
  size_t off = 0;
  const size_t o_enc = off;  off = align256(off + leco::encode_scratch_bytes(nparts));
  const size_t o_cols = off; off = align256(off + sizeof(leco::EncColumn) * k);
  const size_t o_sum = off;  off = align256(off + 8);
  const size_t o_hull = off; off = align256(off + (hulls ? 8 * k * window : 0));
  void* scr = nullptr;
  leco_status st = get_scratch(ctx, off, &scr);
  if (st != LECO_OK) return st;
  char* b = static_cast<char*>(scr);
  std::vector<leco::EncColumn> cols(k);
  for (uint64_t i = 0; i < k; ++i) {
    leco::EncColumn& c = cols[i];
    c.col = static_cast<const uint8_t*>(col) + starts[i] * uint64_t(dtype);
    c.blob = nullptr;
    c.starts = nullptr;
    c.size_out = nullptr;
    c.n = window;
    c.m = m;
    c.fixed_len = L;
    c.cap = 0;
    c.words_off = 0;
    c.part_base = i * m;
    c.dtype = uint32_t(dtype);
    c.force_constant = 0;
    c.regressor = uint32_t(regressor);
    c.pad = 0;
    c.val_base = i * window;
  }
  leco::EncScratch es = leco::carve_encode_scratch(b + o_enc, nparts);
  if (hulls) {
    es.hull = reinterpret_cast<uint32_t*>(b + o_hull);
    es.hull_values = k * window;
  }
  auto* cols_dev = reinterpret_cast<leco::EncColumn*>(b + o_cols);
  auto* sum_dev = reinterpret_cast<uint64_t*>(b + o_sum);
  HIP_TRY(ctx, hipMemcpyAsync(cols_dev, cols.data(), sizeof(leco::EncColumn) * k,
                              hipMemcpyHostToDevice, stream));
  HIP_TRY(ctx, hipMemsetAsync(sum_dev, 0, 8, stream));
  HIP_TRY(ctx, leco::launch_fit_columns(ctx, cols_dev, k, cols[0], nparts, L,
                                        leco::regressor_bit(uint32_t(regressor)), es, stream));
  // a polynomial blob also stores 16 coefficient bytes per partition
  HIP_TRY(ctx, leco::launch_cost_sum(es, nparts, regressor == LECO_REGRESSOR_POLY ? 16 : 0, sum_dev,
                                     stream));
  HIP_TRY(ctx, hipMemcpyAsync(ctx->pinned_u64, sum_dev, 8, hipMemcpyDeviceToHost, stream));
  st = leco_sync(ctx, stream);  // also waits for the table's copy before `cols` goes
  if (st != LECO_OK) return st;
  *cost = *ctx->pinned_u64;
  return LECO_OK;
}

leco_status leco_fixed_cost(leco_ctx* ctx, const void* col_dev, uint64_t n, leco_dtype dtype,
                            const uint64_t* starts_host, uint64_t k, uint64_t window, uint64_t L,
                            int32_t regressor, uint64_t* cost_host, hipStream_t stream) {
  leco_status st = check_windows(ctx, col_dev, n, dtype, starts_host, k, window, regressor);
  if (st != LECO_OK) return st;
  if (L == 0 || L > window) return fail(ctx, LECO_EINVAL, "L must be in [1, window]");
  if (!cost_host) return fail(ctx, LECO_EINVAL, "cost_host is null");
  return sampled_cost(ctx, col_dev, dtype, starts_host, k, window, L, regressor, stream, cost_host);
}

leco_status leco_size_search(leco_ctx* ctx, const void* col_dev, uint64_t n, leco_dtype dtype,
                             const uint64_t* starts_host, uint64_t k, uint64_t window,
                             int32_t regressor, uint64_t* L_out, uint64_t* cost_out,
                             uint64_t* trace_host, uint64_t trace_cap, uint64_t* trace_len,
                             hipStream_t stream) {
  leco_status st = check_windows(ctx, col_dev, n, dtype, starts_host, k, window, regressor);
  if (st != LECO_OK) return st;
  if (!L_out || !cost_out) return fail(ctx, LECO_EINVAL, "outputs are null");
  // known[L] = cost(L) once evaluated (UINT64_MAX before)
  std::vector<uint64_t> known(window + 1, UINT64_MAX);
  uint64_t evaluated = 0;
  leco_status err = LECO_OK;
  auto cost = [&](uint64_t L) -> uint64_t {
    if (known[L] != UINT64_MAX || err != LECO_OK) return known[L];
    uint64_t c = UINT64_MAX;
    err = sampled_cost(ctx, col_dev, dtype, starts_host, k, window, L, regressor, stream, &c);
    known[L] = c;
    if (trace_host && 2 * evaluated + 2 <= trace_cap) {
      trace_host[2 * evaluated] = L;
      trace_host[2 * evaluated + 1] = c;
    }
    ++evaluated;
    return c;
  };
  // exponential phase: past the bottom of the U
  uint64_t best = 1, best_cost = cost(1);
  for (uint64_t L = 1, prev = best_cost; L < window && err == LECO_OK;) {
    L = L <= window / 2 ? 2 * L : window;
    const uint64_t c = cost(L);
    if (c < best_cost) {
      best_cost = c;
      best = L;
    }
    if (c > prev) break;
    prev = c;
  }
  // back search with halving steps until the gain converges
  for (uint64_t s = best / 2; s > 0 && err == LECO_OK; s /= 2) {
    uint64_t to = best, to_cost = best_cost;
    if (best > s) {
      const uint64_t c = cost(best - s);
      if (c < to_cost) {
        to = best - s;
        to_cost = c;
      }
    }
    if (best + s <= window) {
      const uint64_t c = cost(best + s);
      if (c < to_cost) {
        to = best + s;
        to_cost = c;
      }
    }
    if (to == best) continue;
    const bool converged = (best_cost - to_cost) * 10000 < best_cost;
    best = to;
    best_cost = to_cost;
    if (converged) break;
  }
  if (err != LECO_OK) return err;
  *L_out = best;
  *cost_out = best_cost;
  if (trace_len) *trace_len = evaluated;
  return LECO_OK;
}

leco_status leco_diag_slope(leco_ctx* ctx, const uint64_t* in_dev, uint64_t k, double* out_dev,
                            hipStream_t stream) {
  if (!ctx) return LECO_EINVAL;
  if (k && (!in_dev || !out_dev)) return fail(ctx, LECO_EINVAL, "input or output is null");
  if (k > (uint64_t(1) << 32)) return fail(ctx, LECO_EINVAL, "too many pairs");
  HIP_TRY(ctx, leco::launch_diag_slope(in_dev, k, out_dev, stream));
  return LECO_OK;
}

leco_status leco_diag_copy(leco_ctx* ctx, const void* src_dev, void* dst_dev, uint64_t bytes,
                           hipStream_t stream) {
  if (!ctx) return LECO_EINVAL;
  if (!dst_dev || !aligned16(dst_dev) || (src_dev && !aligned16(src_dev)) || bytes % 16)
    return fail(ctx, LECO_EINVAL, "copy needs 16-byte aligned buffers and a multiple of 16 bytes");
  HIP_TRY(ctx, leco::launch_diag_copy(ctx, src_dev, dst_dev, bytes, stream));
  return LECO_OK;
}

}  // extern "C"
