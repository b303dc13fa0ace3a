// Served mode: compressed columns resident in HBM, a host request loop with
// admission by output memory, and steps of mixed random-access and range
// work executed by one kernel launch each on rotating streams.
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "decode_tile.hpp"
#include "internal.hpp"

namespace leco {

struct ServeCol {
  const uint8_t* blob;
  uint64_t blob_bytes;
  uint64_t n;
  uint32_t dtype;
  uint32_t tile_log2;  // values per range work item, as decode_all's tiles
};

// One workgroup of a step.  Random access: b positions, at index a of the
// position ring (LECO_REQ_RANDOM_ACCESS) or at device address a
// (LECO_REQ_RANDOM_ACCESS_DEV), results to out_off.  Range: values [a, b)
// of the column within one tile of its grid (tiles of 2^tile_log2 values
// from position 0, as decode_all's), results to out_off.
struct WorkItem {
  uint32_t kind;
  uint32_t col;
  uint64_t a, b;
  uint64_t out_off;  // bytes into the result arena
};

// The position ring lives in pinned host memory; the lanes of a workgroup
// read 256 consecutive positions (from the ring or from device memory), so
// each wave reads 512 contiguous bytes.  Ring positions were checked against
// n at submission, device positions are checked here: one >= n raises the
// range flag and gives 0.
__global__ __launch_bounds__(kBlock) void k_serve_step(const ServeCol* __restrict__ cols,
                                                       const WorkItem* __restrict__ items,
                                                       const uint64_t* __restrict__ positions,
                                                       uint8_t* __restrict__ arena, int* err) {
  // range work items decode partition by partition: the full-round decoder
  // of short partitions would cost the step kernel a wave per SIMD
  constexpr uint32_t kSlot = slot_words<StoreSink<uint64_t, false>>();
  __shared__ uint4 stage_v[kWavesPerBlock * kSlot / 4];
  uint32_t* stage = reinterpret_cast<uint32_t*>(stage_v) + wave_id() * kSlot;
  const WorkItem it = items[blockIdx.x];
  const ServeCol c = cols[it.col];
  Header h;
  if (!load_header(c.blob, c.blob_bytes, h) || h.n != c.n) {
    if (threadIdx.x == 0) raise(err, kErrFormat);
    return;
  }
  uint8_t* out = arena + it.out_off;
  if (it.kind != LECO_REQ_RANGE) {
    const uint64_t i = threadIdx.x;
    if (i >= it.b) return;
    const uint64_t g = it.kind == LECO_REQ_RANDOM_ACCESS
                           ? positions[it.a + i]
                           : global_ptr(reinterpret_cast<const uint64_t*>(it.a))[i];
    uint64_t v = 0;
    if (g >= h.n || !(h.poly ? lookup_value_poly(c.blob, h, g, v) : lookup_value(c.blob, h, g, v)))
      raise(err, g >= h.n ? kErrRange : kErrFormat);
    if (h.dtype == 8)
      reinterpret_cast<uint64_t*>(out)[i] = v;
    else
      reinterpret_cast<uint32_t*>(out)[i] = uint32_t(v);
    return;
  }
  // the item lies in one tile of the column's grid; wavefront w takes
  // quarter w of that tile, clipped to the item, so a share starts on the
  // grid (as in decode_all) except where the request itself begins
  const uint64_t q = uint64_t(1) << (c.tile_log2 - 2);
  const uint64_t base = (it.a >> c.tile_log2) << c.tile_log2;
  uint64_t g0 = base + wave_id() * q, g1 = g0 + q;
  g0 = g0 > it.a ? g0 : it.a;
  g1 = g1 < it.b ? g1 : it.b;
  if (g0 >= g1) return;
  bool ok;
  if (h.dtype == 8) {
    StoreSink<uint64_t, false> sink{reinterpret_cast<uint64_t*>(out), it.a};
    ok = h.poly ? decode_range_poly(c.blob, h, g0, g1, stage, sink) : decode_tile(c.blob, h, g0, g1, stage, sink);
  } else {
    StoreSink<uint32_t, false> sink{reinterpret_cast<uint32_t*>(out), it.a};
    ok = h.poly ? decode_range_poly(c.blob, h, g0, g1, stage, sink) : decode_tile(c.blob, h, g0, g1, stage, sink);
  }
  if (!ok && lane_id() == 0) raise(err, kErrFormat);
}

}  // namespace leco

// ---- host side ------------------------------------------------------------------

namespace {

using Clock = std::chrono::steady_clock;

// First-fit allocator over [0, size) bytes, 256-byte granules: the result
// arena in device memory and the position ring in pinned host memory.
class Arena {
 public:
  explicit Arena(uint64_t size) { free_[0] = size; }
  bool alloc(uint64_t bytes, uint64_t* off) {
    bytes = round(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const uint64_t rest = it->second - bytes;
        const uint64_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        used_ += bytes;
        peak_ = used_ > peak_ ? used_ : peak_;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
    bytes = round(bytes);
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto next = std::next(it);
    if (next != free_.end() && it->first + it->second == next->first) {
      it->second += next->second;
      free_.erase(next);
    }
    if (it != free_.begin()) {
      auto prev = std::prev(it);
      if (prev->first + prev->second == it->first) {
        prev->second += it->second;
        free_.erase(it);
      }
    }
  }
  uint64_t used() const { return used_; }
  uint64_t peak() const { return peak_; }
  void reset_peak() { peak_ = used_; }
  static uint64_t round(uint64_t b) { return (b + 255) & ~uint64_t(255); }

 private:
  uint64_t used_ = 0, peak_ = 0;
  std::map<uint64_t, uint64_t> free_;
};

struct Pending {
  uint64_t ticket;
  leco_request req;
  uint64_t pos_off;  // byte offset of the positions in the ring (host positions)
  uint64_t count, out_bytes;
  uint64_t items;    // work items (workgroups) of the request
  // bytes between the result's allocation and its first value: a range's
  // values are placed so that value g sits at g * dtype modulo 256, which
  // lines up the stores of work items on the column's tile grid with
  // cache lines
  uint64_t pad;
  Clock::time_point t_submit;
};

struct Result {
  uint64_t off, bytes;
  bool done;
};

// A step slot: its stream, completion event and work-item staging.
struct Slot {
  hipStream_t stream = nullptr;
  hipEvent_t start = nullptr;  // timing events around the step
  hipEvent_t done = nullptr;
  leco::WorkItem* items_host = nullptr;  // pinned
  leco::WorkItem* items_dev = nullptr;
  bool busy = false;              // admitted requests, step being built or running
  bool launched = false;          // the step's completion event is recorded
  leco_status status = LECO_OK;  // EDEVICE if the step's launch failed
  std::vector<Pending> reqs;     // requests the running step completes
  std::vector<uint64_t> offs;
};

}  // namespace

struct leco_server {
  leco_ctx* ctx = nullptr;
  leco_server_config cfg{};
  std::vector<leco::ServeCol> cols;
  leco::ServeCol* cols_dev = nullptr;
  uint8_t* arena_dev = nullptr;
  Arena* arena = nullptr;
  uint64_t* ring_host = nullptr;  // pinned, device-accessible
  uint64_t* ring_dev = nullptr;
  Arena* ring = nullptr;
  std::vector<Slot> slots;
  size_t next_slot = 0;

  std::mutex mu;  // guards everything below and the two allocators
  std::condition_variable cv;
  std::deque<Pending> queue;
  std::unordered_map<uint64_t, Result> results;
  std::deque<leco_completion> completions;
  uint64_t next_ticket = 1;
  uint64_t inflight = 0;  // admitted and not yet released
  leco_server_stats stats{};
  std::atomic<bool> stop{false};
  std::thread worker;

  // Host time of the loop's phases (ns), written by the worker thread
  // outside the lock and by submitting threads.
  std::atomic<uint64_t> t_submit{0}, t_admit{0}, t_build{0}, t_launch{0}, t_retire{0}, t_wait{0};
  // Device intervals of retired steps, in ms after the reference event
  // (guarded by mu).
  hipEvent_t ref = nullptr;
  std::vector<std::pair<double, double>> intervals;
};

namespace {

uint64_t ns_since(Clock::time_point t0) {
  return uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count());
}

leco_status sfail(leco_server* s, leco_status st, const char* msg) {
  if (s && s->ctx) s->ctx->last_error = msg;
  return st;
}

uint64_t step_items(const Pending& p) { return p.items; }

// While a step is running, the next one waits until the queued work that
// fits it is worth a launch: enough result bytes, half the step's items,
// the step's position capacity, or an old enough request.  Work that does
// not fit the free memory or slots cannot grow by waiting, so it goes.
bool batch_ready(const leco_server* s) {
  const leco_server_config& cfg = s->cfg;
  if (cfg.max_wait_us &&
      Clock::now() - s->queue.front().t_submit >= std::chrono::microseconds(cfg.max_wait_us))
    return true;
  uint64_t bytes = 0, items = 0, pos = 0, admitted = 0;
  for (const Pending& p : s->queue) {
    const uint64_t it = step_items(p);
    const bool ra = p.req.kind == LECO_REQ_RANDOM_ACCESS;  // positions in the ring
    if (items + it > cfg.max_step_items || (ra && pos + p.count > cfg.max_step_positions) ||
        s->inflight + admitted >= cfg.max_inflight)
      return true;  // the step is full
    bytes += p.out_bytes;
    items += it;
    pos += ra ? p.count : 0;
    ++admitted;
    if (cfg.min_step_bytes && bytes >= cfg.min_step_bytes) return true;
    if (2 * items >= cfg.max_step_items) return true;
  }
  return false;  // the whole queue is a small step: wait for more
}

// Admits queued requests into a free slot and launches the step.  Called
// by the worker with s->mu held; admission (memory, slots) happens under the
// lock, the work items are built and the step launched without it (the slot
// belongs to the worker until it is marked busy).  Returns true if a step
// was launched.
bool launch_step(leco_server* s, std::unique_lock<std::mutex>& lk) {
  const Clock::time_point t_enter = Clock::now();
  Slot* slot = nullptr;
  for (size_t i = 0; i < s->slots.size(); ++i) {
    Slot& c = s->slots[(s->next_slot + i) % s->slots.size()];
    if (!c.busy) {
      slot = &c;
      s->next_slot = (s->next_slot + i + 1) % s->slots.size();
      break;
    }
  }
  if (!slot || s->queue.empty()) return false;
  bool any_busy = false;
  for (const Slot& c : s->slots) any_busy = any_busy || c.busy;
  if (any_busy && !batch_ready(s)) return false;
  uint64_t nitems = 0, npos = 0;
  slot->reqs.clear();
  slot->offs.clear();
  while (!s->queue.empty()) {
    Pending& p = s->queue.front();
    const bool ra = p.req.kind == LECO_REQ_RANDOM_ACCESS;  // positions in the ring
    const uint64_t items = step_items(p);
    if (nitems + items > s->cfg.max_step_items) break;
    if (ra && npos + p.count > s->cfg.max_step_positions) break;
    if (s->inflight >= s->cfg.max_inflight) break;
    uint64_t off = 0;
    const uint64_t bytes = p.out_bytes + p.pad ? p.out_bytes + p.pad : 1;
    if (!s->arena->alloc(bytes, &off)) break;  // wait for memory
    nitems += items;
    if (ra) npos += p.count;
    s->results[p.ticket] = Result{off, bytes, false};
    ++s->inflight;
    slot->offs.push_back(off + p.pad);
    slot->reqs.push_back(p);
    s->queue.pop_front();
  }
  if (slot->reqs.empty()) return false;
  s->stats.steps += 1;
  slot->busy = true;  // keeps other launches off this slot while unlocked
  lk.unlock();
  const Clock::time_point t_built0 = Clock::now();
  s->t_admit += uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(t_built0 - t_enter).count());
  uint32_t k = 0;
  for (size_t r = 0; r < slot->reqs.size(); ++r) {
    const Pending& p = slot->reqs[r];
    const uint64_t off = slot->offs[r];
    const leco::ServeCol& col = s->cols[p.req.col];
    if (p.req.kind != LECO_REQ_RANGE) {
      const bool ra = p.req.kind == LECO_REQ_RANDOM_ACCESS;
      // ring index, or device address, of the request's first position
      const uint64_t base = ra ? p.pos_off / 8 : reinterpret_cast<uint64_t>(p.req.positions);
      const uint64_t stride = ra ? 1 : 8;
      for (uint64_t first = 0; first < p.count; first += leco::kBlock) {
        const uint64_t cnt = p.count - first < uint64_t(leco::kBlock) ? p.count - first : leco::kBlock;
        slot->items_host[k++] = leco::WorkItem{p.req.kind, p.req.col, base + first * stride, cnt,
                                               off + first * col.dtype};
      }
    } else {
      // one item per tile of the column's grid that the range touches
      const uint64_t tile = uint64_t(1) << col.tile_log2;
      for (uint64_t g = p.req.begin; g < p.req.end;) {
        const uint64_t next = (g | (tile - 1)) + 1;
        const uint64_t e = next < p.req.end ? next : p.req.end;
        slot->items_host[k++] = leco::WorkItem{LECO_REQ_RANGE, p.req.col, g, e,
                                               off + (g - p.req.begin) * col.dtype};
        g = e;
      }
    }
  }
  const Clock::time_point t_launch0 = Clock::now();
  s->t_build += uint64_t(std::chrono::duration_cast<std::chrono::nanoseconds>(t_launch0 - t_built0).count());
  hipError_t e = hipEventRecord(slot->start, slot->stream);
  if (k && e == hipSuccess) {
    e = hipMemcpyAsync(slot->items_dev, slot->items_host, sizeof(leco::WorkItem) * k,
                       hipMemcpyHostToDevice, slot->stream);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(leco::k_serve_step, dim3(k), dim3(leco::kBlock), 0, slot->stream,
                         s->cols_dev, slot->items_dev, s->ring_dev, s->arena_dev,
                         s->ctx->err_dev);
      e = hipGetLastError();
    }
  }
  if (e == hipSuccess) e = hipEventRecord(slot->done, slot->stream);
  // a failed step completes its requests with EDEVICE once its stream drains
  if (e != hipSuccess) (void)hipStreamSynchronize(slot->stream);
  s->t_launch += ns_since(t_launch0);
  lk.lock();
  s->stats.items += k;
  slot->status = e == hipSuccess ? LECO_OK : LECO_EDEVICE;
  slot->launched = true;
  return true;
}

// Retires finished steps: completions, and the ring space of their
// positions.  Called with s->mu held.
bool retire_steps(leco_server* s) {
  bool any = false;
  for (Slot& slot : s->slots) {
    if (!slot.busy || !slot.launched ||
        (slot.status == LECO_OK && hipEventQuery(slot.done) != hipSuccess))
      continue;
    const Clock::time_point now = Clock::now();
    float t0_ms = 0.f, t1_ms = 0.f;
    if (slot.status == LECO_OK && hipEventElapsedTime(&t0_ms, s->ref, slot.start) == hipSuccess &&
        hipEventElapsedTime(&t1_ms, s->ref, slot.done) == hipSuccess)
      s->intervals.emplace_back(double(t0_ms), double(t1_ms));
    for (size_t i = 0; i < slot.reqs.size(); ++i) {
      const Pending& p = slot.reqs[i];
      if (p.req.kind == LECO_REQ_RANDOM_ACCESS && p.count) s->ring->release(p.pos_off, 8 * p.count);
      auto it = s->results.find(p.ticket);
      if (it != s->results.end()) it->second.done = true;
      leco_completion c{};
      c.ticket = p.ticket;
      c.status = slot.status;
      c.dtype = int32_t(s->cols[p.req.col].dtype);
      c.out_dev = s->arena_dev + slot.offs[i];
      c.count = p.count;
      c.latency_us = std::chrono::duration<double, std::micro>(now - p.t_submit).count();
      s->completions.push_back(c);
      s->stats.completed += 1;
      s->stats.values_out += p.count;
    }
    slot.reqs.clear();
    slot.busy = false;
    slot.launched = false;
    any = true;
  }
  if (any) s->cv.notify_all();
  return any;
}

void worker_main(leco_server* s) {
  (void)hipSetDevice(s->ctx->device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (true) {
    const Clock::time_point t0 = Clock::now();
    retire_steps(s);
    s->t_retire += ns_since(t0);
    const bool launched = launch_step(s, lk);
    bool busy = false;
    for (const Slot& slot : s->slots) busy = busy || slot.busy;
    if (s->stop && s->queue.empty() && !busy) break;
    if (!launched) {
      const Clock::time_point tw = Clock::now();
      if (busy) {
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else {
        s->cv.wait_for(lk, std::chrono::microseconds(200));
      }
      s->t_wait += ns_since(tw);
    }
  }
}

void free_server(leco_server* s) {
  for (Slot& slot : s->slots) {
    if (slot.stream) (void)hipStreamSynchronize(slot.stream);
    if (slot.done) (void)hipEventDestroy(slot.done);
    if (slot.start) (void)hipEventDestroy(slot.start);
    // teardown: an error here leaves nothing to undo, so it is not reported
    if (slot.stream) (void)hipStreamDestroy(slot.stream);
    if (slot.items_host) (void)hipHostFree(slot.items_host);
    if (slot.items_dev) (void)hipFree(slot.items_dev);
  }
  if (s->ref) (void)hipEventDestroy(s->ref);
  if (s->cols_dev) (void)hipFree(s->cols_dev);
  if (s->arena_dev) (void)hipFree(s->arena_dev);
  if (s->ring_host) (void)hipHostFree(s->ring_host);
  delete s->arena;
  delete s->ring;
  delete s;
}

}  // namespace

extern "C" {

leco_status leco_server_start(leco_ctx* ctx, const leco_resident_col* cols, uint64_t ncols,
                              const leco_server_config* cfg, leco_server** out) {
  if (!ctx || !out || !cfg || (ncols && !cols)) return LECO_EINVAL;
  *out = nullptr;
  if (ncols == 0 || ncols > 0xffffffffull || cfg->out_budget_bytes == 0 || cfg->num_streams == 0 ||
      cfg->reserved != 0 || cfg->max_step_items == 0 || cfg->max_inflight == 0) {
    ctx->last_error = "server needs columns, a budget, a stream, step items and in-flight slots";
    return LECO_EINVAL;
  }
  leco_server* s = new leco_server();
  s->ctx = ctx;
  s->cfg = *cfg;
  if (s->cfg.max_step_positions == 0) s->cfg.max_step_positions = 1u << 20;
  if (s->cfg.position_ring_bytes == 0) s->cfg.position_ring_bytes = uint64_t(64) << 20;
  if (hipSetDevice(ctx->device) != hipSuccess) {
    delete s;
    return LECO_EDEVICE;
  }
  for (uint64_t i = 0; i < ncols; ++i) {
    uint8_t hdr[64];
    if (!cols[i].blob_dev || (reinterpret_cast<uintptr_t>(cols[i].blob_dev) & 15) ||
        cols[i].blob_bytes < 64 ||
        hipMemcpy(hdr, cols[i].blob_dev, 64, hipMemcpyDeviceToHost) != hipSuccess) {
      free_server(s);
      ctx->last_error = "resident column with a bad blob";
      return LECO_EINVAL;
    }
    uint64_t n = 0;
    leco_dtype dt;
    if (leco_blob_info(hdr, &n, &dt, nullptr) != LECO_OK || n != cols[i].n) {
      free_server(s);
      ctx->last_error = "resident blob header does not match its column";
      return LECO_EFORMAT;
    }
    s->cols.push_back(leco::ServeCol{static_cast<const uint8_t*>(cols[i].blob_dev),
                                     cols[i].blob_bytes, n, uint32_t(dt),
                                     leco::pick_tile_log2(leco::Tune{}, cols[i].blob_bytes, n)});
  }
  bool ok = hipMalloc(&s->cols_dev, sizeof(leco::ServeCol) * ncols) == hipSuccess &&
            hipMemcpy(s->cols_dev, s->cols.data(), sizeof(leco::ServeCol) * ncols,
                      hipMemcpyHostToDevice) == hipSuccess &&
            hipMalloc(&s->arena_dev, cfg->out_budget_bytes) == hipSuccess &&
            hipHostMalloc(&s->ring_host, s->cfg.position_ring_bytes, hipHostMallocDefault) ==
                hipSuccess &&
            hipHostGetDevicePointer(reinterpret_cast<void**>(&s->ring_dev), s->ring_host, 0) ==
                hipSuccess;
  s->slots.resize(cfg->num_streams);
  for (Slot& slot : s->slots) {
    ok = ok && hipStreamCreateWithFlags(&slot.stream, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreate(&slot.start) == hipSuccess && hipEventCreate(&slot.done) == hipSuccess &&
         hipHostMalloc(&slot.items_host, sizeof(leco::WorkItem) * s->cfg.max_step_items,
                       hipHostMallocDefault) == hipSuccess &&
         hipMalloc(&slot.items_dev, sizeof(leco::WorkItem) * s->cfg.max_step_items) == hipSuccess;
  }
  // the reference the step events are timed against
  ok = ok && hipEventCreate(&s->ref) == hipSuccess &&
       hipEventRecord(s->ref, s->slots[0].stream) == hipSuccess &&
       hipEventSynchronize(s->ref) == hipSuccess;
  if (!ok) {
    free_server(s);
    ctx->last_error = "server allocation failed";
    return LECO_ENOMEM;
  }
  s->arena = new Arena(cfg->out_budget_bytes);
  s->ring = new Arena(s->cfg.position_ring_bytes);
  s->worker = std::thread(worker_main, s);
  *out = s;
  return LECO_OK;
}

}  // extern "C"

namespace {

// Validates one request and, for host positions, reserves ring space and
// copies the positions into it (checking them on the way).  The request is
// not queued yet.
leco_status prepare_request(leco_server* s, const leco_request* r, Pending& p) {
  if (r->col >= s->cols.size()) return sfail(s, LECO_EINVAL, "no such resident column");
  const leco::ServeCol& col = s->cols[r->col];
  p.req = *r;
  p.pos_off = 0;
  const bool ring = r->kind == LECO_REQ_RANDOM_ACCESS;
  if (ring || r->kind == LECO_REQ_RANDOM_ACCESS_DEV) {
    if (r->k && !r->positions) return sfail(s, LECO_EINVAL, "positions are null");
    if (ring && (r->k > s->cfg.max_step_positions ||
                 Arena::round(8 * r->k) > s->cfg.position_ring_bytes))
      return sfail(s, LECO_EINVAL, "more positions than a step or the position ring holds");
    if (!ring && (reinterpret_cast<uintptr_t>(r->positions) & 7))
      return sfail(s, LECO_EINVAL, "device positions must be 8-byte aligned");
    if ((r->k + leco::kBlock - 1) / leco::kBlock > s->cfg.max_step_items)
      return sfail(s, LECO_EINVAL, "more positions than a step holds");
    p.count = r->k;
    p.items = (p.count + leco::kBlock - 1) / leco::kBlock;
  } else if (r->kind == LECO_REQ_RANGE) {
    if (r->begin > r->end || r->end > col.n) return sfail(s, LECO_ERANGE, "range outside [0, n)");
    p.count = r->end - r->begin;
    // tiles of the column's grid that [begin, end) touches
    p.items = p.count ? ((r->end - 1) >> col.tile_log2) - (r->begin >> col.tile_log2) + 1 : 0;
    if (p.items > s->cfg.max_step_items) return sfail(s, LECO_EINVAL, "range larger than a step");
  } else {
    return sfail(s, LECO_EINVAL, "unknown request kind");
  }
  p.out_bytes = p.count * col.dtype;
  p.pad = r->kind == LECO_REQ_RANGE ? (r->begin * col.dtype) & 255 : 0;
  if (Arena::round(p.out_bytes + p.pad) > s->cfg.out_budget_bytes)
    return sfail(s, LECO_ENOSPC, "request larger than the output budget");
  if (ring && p.count) {
    // Reserve ring space under the lock, then check and copy the positions
    // without it: the request is invisible to the loop until it is queued.
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (!s->ring->alloc(8 * p.count, &p.pos_off))
        return sfail(s, LECO_ENOMEM, "position ring full: retry after earlier requests complete");
    }
    uint64_t* dst = reinterpret_cast<uint64_t*>(reinterpret_cast<uint8_t*>(s->ring_host) + p.pos_off);
    uint64_t bad = 0;
    for (uint64_t i = 0; i < p.count; ++i) {
      const uint64_t g = r->positions[i];
      bad |= uint64_t(g >= col.n);
      dst[i] = g;
    }
    if (bad) {
      std::lock_guard<std::mutex> lk(s->mu);
      s->ring->release(p.pos_off, 8 * p.count);
      return sfail(s, LECO_ERANGE, "position >= n");
    }
  }
  return LECO_OK;
}

// Frees a completed request's result memory; s->mu held.
leco_status release_locked(leco_server* s, uint64_t ticket) {
  auto it = s->results.find(ticket);
  if (it == s->results.end() || !it->second.done)
    return sfail(s, LECO_EINVAL, "ticket is not a completed, unreleased request");
  s->arena->release(it->second.off, it->second.bytes);
  s->results.erase(it);
  --s->inflight;
  return LECO_OK;
}

}  // namespace

extern "C" {

leco_status leco_server_submit_batch(leco_server* s, const leco_request* reqs, uint64_t n,
                                     uint64_t* tickets, uint64_t* accepted) {
  if (accepted) *accepted = 0;
  if (!s || (n && !reqs)) return LECO_EINVAL;
  const Clock::time_point t_enter = Clock::now();  // latency counts the copies below
  std::vector<Pending> ready;
  ready.reserve(n);
  leco_status st = LECO_OK;
  for (uint64_t i = 0; i < n; ++i) {
    Pending p;
    if ((st = prepare_request(s, &reqs[i], p)) != LECO_OK) break;
    ready.push_back(p);
  }
  if (!ready.empty()) {
    std::lock_guard<std::mutex> lk(s->mu);
    for (uint64_t i = 0; i < ready.size(); ++i) {
      Pending& p = ready[i];
      p.t_submit = t_enter;
      p.ticket = s->next_ticket++;
      if (tickets) tickets[i] = p.ticket;
      s->stats.submitted += 1;
      if (p.req.kind != LECO_REQ_RANGE) s->stats.positions += p.count;
      s->queue.push_back(p);
    }
    s->cv.notify_all();
  }
  s->t_submit += ns_since(t_enter);
  if (accepted) *accepted = ready.size();
  return st;
}

leco_status leco_server_submit(leco_server* s, const leco_request* r, uint64_t* ticket) {
  if (!s || !r) return LECO_EINVAL;
  return leco_server_submit_batch(s, r, 1, ticket, nullptr);
}

leco_status leco_server_poll(leco_server* s, leco_completion* out, uint64_t max, uint64_t* got) {
  if (!s || (max && !out) || !got) return LECO_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  uint64_t k = 0;
  while (k < max && !s->completions.empty()) {
    out[k++] = s->completions.front();
    s->completions.pop_front();
  }
  *got = k;
  return LECO_OK;
}

leco_status leco_server_release(leco_server* s, uint64_t ticket) {
  if (!s) return LECO_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  const leco_status st = release_locked(s, ticket);
  if (st == LECO_OK) s->cv.notify_all();
  return st;
}

leco_status leco_server_stats_get(leco_server* s, leco_server_stats* out) {
  if (!s || !out) return LECO_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  out->out_bytes_in_use = s->arena->used();
  out->out_bytes_peak = s->arena->peak();
  out->queued = s->queue.size();
  out->host_submit_ns = s->t_submit;
  out->host_admit_ns = s->t_admit;
  out->host_build_ns = s->t_build;
  out->host_launch_ns = s->t_launch;
  out->host_retire_ns = s->t_retire;
  out->host_wait_ns = s->t_wait;
  // step durations, their union and their span
  std::vector<std::pair<double, double>> iv = s->intervals;
  std::sort(iv.begin(), iv.end());
  double sum = 0, busy = 0, cur_a = 0, cur_b = 0, lo = 0, hi = 0;
  bool open = false;
  for (const auto& x : iv) {
    sum += x.second - x.first;
    if (!open) {
      cur_a = x.first;
      cur_b = x.second;
      lo = x.first;
      hi = x.second;
      open = true;
      continue;
    }
    hi = x.second > hi ? x.second : hi;
    if (x.first > cur_b) {
      busy += cur_b - cur_a;
      cur_a = x.first;
      cur_b = x.second;
    } else if (x.second > cur_b) {
      cur_b = x.second;
    }
  }
  if (open) busy += cur_b - cur_a;
  out->gpu_step_ns = uint64_t(sum * 1e6);
  out->gpu_busy_ns = uint64_t(busy * 1e6);
  out->gpu_span_ns = uint64_t((hi - lo) * 1e6);
  return LECO_OK;
}

leco_status leco_server_stats_reset(leco_server* s) {
  if (!s) return LECO_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  const uint64_t in_use = s->stats.out_bytes_in_use;
  s->stats = leco_server_stats{};
  s->stats.out_bytes_in_use = in_use;
  s->arena->reset_peak();
  s->t_submit = s->t_admit = s->t_build = s->t_launch = s->t_retire = s->t_wait = 0;
  s->intervals.clear();
  return LECO_OK;
}

leco_status leco_server_stop(leco_server* s) {
  if (!s) return LECO_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv.notify_all();
  }
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->ctx->device);  // teardown continues either way
  free_server(s);
  return LECO_OK;
}

leco_status leco_server_replay(leco_server* s, const leco_request* reqs, const double* arrival_s,
                               uint64_t n, double* latency_us_out, double* elapsed_s) {
  if (!s || (n && (!reqs || !arrival_s))) return LECO_EINVAL;
  std::unordered_map<uint64_t, uint64_t> index;  // ticket -> request number
  std::vector<double> lag_us(n, 0.0);            // submission start - scheduled arrival
  std::vector<leco_completion> buf(1024);
  std::vector<uint64_t> tickets(1024);
  uint64_t done = 0;
  const Clock::time_point t0 = Clock::now();
  Clock::time_point last = t0;
  auto due_at = [&](uint64_t i) {
    return t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[i]));
  };
  // Polls completions and releases their results under one lock.
  auto drain = [&]() {
    uint64_t got = 0;
    leco_server_poll(s, buf.data(), buf.size(), &got);
    if (!got) return;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      for (uint64_t i = 0; i < got; ++i) release_locked(s, buf[i].ticket);
      s->cv.notify_all();
    }
    for (uint64_t i = 0; i < got; ++i) {
      auto it = index.find(buf[i].ticket);
      if (it != index.end() && latency_us_out)
        latency_us_out[it->second] = lag_us[it->second] + buf[i].latency_us;
    }
    done += got;
    last = Clock::now();
  };
  uint64_t i = 0;
  while (i < n) {
    while (Clock::now() < due_at(i)) drain();
    // every request already due goes in one batch
    const Clock::time_point now = Clock::now();
    uint64_t j = i + 1;
    while (j < n && j - i < tickets.size() && due_at(j) <= now) ++j;
    for (uint64_t q = i; q < j; ++q)
      // latency runs from the scheduled arrival: the lag until the accepted
      // submission, plus the server's submit-to-completion time
      lag_us[q] = std::chrono::duration<double, std::micro>(now - due_at(q)).count();
    uint64_t accepted = 0;
    const leco_status st = leco_server_submit_batch(s, reqs + i, j - i, tickets.data(), &accepted);
    for (uint64_t q = 0; q < accepted; ++q) index[tickets[q]] = i + q;
    i += accepted;
    if (st == LECO_ENOMEM) {
      drain();  // the position ring frees as earlier steps finish
      std::this_thread::yield();
    } else if (st != LECO_OK) {
      return st;
    }
    drain();  // keep releasing results while submitting
  }
  while (done < n) {
    drain();
    std::this_thread::yield();
  }
  if (elapsed_s) {
    const double first = n ? arrival_s[0] : 0.0;
    *elapsed_s = std::chrono::duration<double>(last - t0).count() - first;
  }
  return LECO_OK;
}

}  // extern "C"

extern "C" {

leco_status leco_plain_replay(leco_ctx* ctx, const leco_resident_col* cols, uint64_t ncols,
                              const leco_request* reqs, const double* arrival_s, uint64_t n,
                              void* out_dev, uint64_t out_bytes, hipStream_t stream,
                              double* latency_us_out, double* elapsed_s) {
  if (!ctx) return LECO_EINVAL;
  if ((ncols && !cols) || (n && (!reqs || !arrival_s)) || !out_dev) {
    ctx->last_error = "plain replay: null argument";
    return LECO_EINVAL;
  }
  if (hipSetDevice(ctx->device) != hipSuccess) return LECO_EDEVICE;
  // dtypes of the columns, and the checks the served loop makes at submission
  std::vector<uint32_t> dt(ncols);
  for (uint64_t c = 0; c < ncols; ++c) {
    uint8_t hdr[64];
    leco_dtype d;
    uint64_t nn = 0;
    if (!cols[c].blob_dev || hipMemcpy(hdr, cols[c].blob_dev, 64, hipMemcpyDeviceToHost) != hipSuccess ||
        leco_blob_info(hdr, &nn, &d, nullptr) != LECO_OK || nn != cols[c].n) {
      ctx->last_error = "plain replay: column with a bad blob";
      return LECO_EINVAL;
    }
    dt[c] = uint32_t(d);
  }
  for (uint64_t i = 0; i < n; ++i) {
    const leco_request& r = reqs[i];
    if (r.col >= ncols) {
      ctx->last_error = "plain replay: no such column";
      return LECO_EINVAL;
    }
    uint64_t count = 0;
    if (r.kind == LECO_REQ_RANDOM_ACCESS_DEV) {
      if (r.k && !r.positions) {
        ctx->last_error = "plain replay: positions are null";
        return LECO_EINVAL;
      }
      count = r.k;
    } else if (r.kind == LECO_REQ_RANGE) {
      if (r.begin > r.end || r.end > cols[r.col].n) {
        ctx->last_error = "plain replay: range outside [0, n)";
        return LECO_ERANGE;
      }
      count = r.end - r.begin;
    } else {
      ctx->last_error = "plain replay: requests must be ranges or device-position lookups";
      return LECO_EINVAL;
    }
    if (count * dt[r.col] > out_bytes) {
      ctx->last_error = "plain replay: output buffer smaller than a request";
      return LECO_ENOSPC;
    }
  }
  // a ring of completion events, retired in launch order
  constexpr uint64_t kEvents = 1024;
  std::vector<hipEvent_t> ev(kEvents, nullptr);
  for (auto& e : ev)
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
      for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
      return LECO_EDEVICE;
    }
  const Clock::time_point t0 = Clock::now();
  auto due_at = [&](uint64_t i) {
    return t0 + std::chrono::duration_cast<Clock::duration>(std::chrono::duration<double>(arrival_s[i]));
  };
  Clock::time_point last = t0;
  uint64_t head = 0, tail = 0;  // requests [head, tail) are launched and not yet seen complete
  leco_status st = LECO_OK;
  auto retire = [&](bool wait) {
    while (head < tail) {
      hipEvent_t e = ev[head % kEvents];
      const hipError_t q = wait ? hipEventSynchronize(e) : hipEventQuery(e);
      if (q == hipErrorNotReady) return;
      if (q != hipSuccess) st = LECO_EDEVICE;
      last = Clock::now();
      if (latency_us_out)
        latency_us_out[head] = std::chrono::duration<double, std::micro>(last - due_at(head)).count();
      ++head;
      wait = false;
    }
  };
  for (uint64_t i = 0; i < n && st == LECO_OK; ++i) {
    while (Clock::now() < due_at(i)) retire(false);
    while (tail - head >= kEvents) retire(true);  // the ring is full
    const leco_request& r = reqs[i];
    const leco_resident_col& c = cols[r.col];
    const leco_status ls =
        r.kind == LECO_REQ_RANGE
            ? leco_decode_range(ctx, c.blob_dev, c.blob_bytes, r.begin, r.end, out_dev, stream)
            : leco_random_access(ctx, c.blob_dev, c.blob_bytes, r.positions, r.k, out_dev, stream);
    if (ls != LECO_OK) {
      st = ls;
      break;
    }
    if (hipEventRecord(ev[tail % kEvents], stream) != hipSuccess) {
      st = LECO_EDEVICE;
      break;
    }
    ++tail;
    retire(false);
  }
  while (head < tail) {
    const leco_status before = st;
    retire(true);
    if (st != before) break;
  }
  (void)hipStreamSynchronize(stream);
  for (auto& e : ev) (void)hipEventDestroy(e);
  if (elapsed_s) *elapsed_s = std::chrono::duration<double>(last - t0).count() - (n ? arrival_s[0] : 0.0);
  return st;
}

}  // extern "C"
