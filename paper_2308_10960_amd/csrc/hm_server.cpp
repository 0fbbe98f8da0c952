// Request loop of libhm: continuous batching of H-matrix-vector products
// against device-resident matrices.
//
// Clients call hm_submit(matrix, X) from any thread; a dispatcher thread
//  * admits requests by device-memory budget: a batch's vectors and
//    workspace are carved out of the caller's arena with a first-fit
//    allocator, and a batch that does not fit waits for running ones to
//    release memory;
//  * batches queued requests of the same matrix (FIFO, up to the matrix's
//    max_nrhs right-hand sides) into one hm_mvm_batch call;
//  * keeps up to n_streams batches in flight, one per stream slot, so
//    requests arriving while others run start as soon as a slot and memory
//    free up (no waiting for the whole previous batch set).
// Each slot has a worker thread that brings its batch's right-hand sides to
// the device (directly from page-locked client buffers, else gathered
// through its pinned staging buffer), enqueues product and copy-back on its
// stream, waits for them, hands the results over and completes the tickets
// (latency recorded at completion); the host work of different slots runs
// in parallel, outside the server lock.
// A request's result does not depend on the batch it lands in: every column
// of a batch is computed by the same kernels in the same order.
//
// Test hook: HM_SERVER_FAULT_EVERY=N (environment, read at creation) fails
// every N-th batch with HM_EDEVICE before anything is enqueued for it, so the
// failure path can be exercised without a device fault.

#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#include <hip/hip_runtime_api.h>

#include "../../include/hm.h"
#include "hm_internal.hpp"

using Clock = std::chrono::steady_clock;

namespace {

struct Request {
  uint64_t ticket;
  int32_t mat, nrhs;
  const void* hx;
  int64_t ldx;
  void* hy;
  int64_t ldy;
  bool x_pinned = false, y_pinned = false;   // page-locked client buffers: copied without staging
  Clock::time_point t_submit;
  bool done = false;
  hm_status result = HM_OK;
};

// Whether [p, p + bytes) lies in page-locked host memory the device can
// reach directly (hipHostMalloc); a failed query (ordinary pageable memory)
// is cleared so that it does not surface in a later call.
bool host_pinned(const void* p, size_t bytes) {
  hipPointerAttribute_t at{};
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (at.type != hipMemoryTypeHost) return false;
  hipPointerAttribute_t end{};
  if (hipPointerGetAttributes(&end, static_cast<const uint8_t*>(p) + bytes - 1) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return end.type == hipMemoryTypeHost;
}

// First-fit allocator over [0, size) in 256-byte units.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + 255) / 256 * 256;
    for (auto it = free_.begin(); it != free_.end(); ++it)
      if (it->second >= bytes) {
        *off = it->first;
        size_t rest = it->second - bytes, start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + 255) / 256 * 256;
    used_ -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
  size_t size() const { return size_; }

 private:
  size_t size_, used_ = 0;
  std::map<size_t, size_t> free_;
};

enum class SlotState { kIdle, kAssigned, kRunning };

struct Slot {
  hipStream_t stream = nullptr;
  SlotState state = SlotState::kIdle;   // guarded by the server lock
  bool fault = false;                   // injected failure for this batch
  std::vector<std::shared_ptr<Request>> reqs;
  size_t off = 0, bytes = 0;
  int32_t mat = 0, nrhs = 0;
  void* pinned = nullptr;               // owned by the slot's worker
  size_t pinned_bytes = 0;
  std::thread worker;
};

}  // namespace

struct hm_server {
  std::vector<hm_matrix*> mats;
  uint8_t* arena_base = nullptr;
  std::unique_ptr<Arena> arena;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done, cv_assign;
  int device = 0;
  bool stop_workers = false;
  std::deque<std::shared_ptr<Request>> queue;
  std::map<uint64_t, std::shared_ptr<Request>> tickets;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread thread;
  // stats: latencies of the most recent kLatWindow completed requests (a ring)
  static constexpr size_t kLatWindow = size_t(1) << 20;
  std::vector<double> lat_us;
  size_t lat_next = 0;
  int64_t rhs_done = 0;
  Clock::time_point t_first{}, t_last{};
  bool have_first = false;
  int64_t batches = 0;
  int64_t fault_every = 0;
  size_t max_queue = 1 << 20;
};

namespace {

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

size_t footprint(const hm_matrix* A, int32_t r) {
  const size_t vs = A->acc_dtype == HM_F64 ? 8 : 4;
  return align256((size_t)A->hdr.n_cols * r * vs) + align256((size_t)A->hdr.n_rows * r * vs) +
         (size_t)hm::batch_slots(A->acc_dtype, r) * A->work_bytes_per_rhs + 256;
}

void finish(hm_server* S, const std::shared_ptr<Request>& q, hm_status st, Clock::time_point now) {
  q->result = st;
  q->done = true;
  const double us = std::chrono::duration<double, std::micro>(now - q->t_submit).count();
  if (S->lat_us.size() < hm_server::kLatWindow) S->lat_us.push_back(us);
  else S->lat_us[S->lat_next] = us;
  S->lat_next = (S->lat_next + 1) % hm_server::kLatWindow;
  if (st == HM_OK) S->rhs_done += q->nrhs;
  if (!S->have_first || q->t_submit < S->t_first) S->t_first = q->t_submit;
  S->have_first = true;
  S->t_last = now;
}

// Run one batch on its slot (worker thread, server lock not held): bring
// the right-hand sides to the device, enqueue the product and the
// copy-back, wait, and hand the results over.  A request in page-locked
// client memory is copied by the device straight between its buffers and
// its columns of the batch (2-D copies with the caller's leading
// dimensions); the others go through the slot's pinned staging buffer
// (gathered before, scattered after).
hm_status run_batch(hm_server* S, Slot& sl) {
  const hm_matrix* A = S->mats[sl.mat];
  const size_t vs = A->acc_dtype == HM_F64 ? 8 : 4;
  const int64_t nr = A->hdr.n_rows, nc = A->hdr.n_cols;
  const size_t xbytes = (size_t)nc * sl.nrhs * vs, ybytes = (size_t)nr * sl.nrhs * vs;
  bool staged = false;
  for (auto& q : sl.reqs) staged |= !q->x_pinned || !q->y_pinned;
  if (staged && sl.pinned_bytes < xbytes + ybytes) {
    if (sl.pinned) (void)hipHostFree(sl.pinned);
    sl.pinned = nullptr;
    sl.pinned_bytes = 0;
    if (hipHostMalloc(&sl.pinned, xbytes + ybytes, hipHostMallocDefault) != hipSuccess)
      return HM_ENOMEM;
    sl.pinned_bytes = xbytes + ybytes;
  }
  uint8_t* px = (uint8_t*)sl.pinned;
  uint8_t* py = px ? px + xbytes : nullptr;
  uint8_t* base = S->arena_base + sl.off;
  uint8_t* dX = base;
  uint8_t* dY = base + align256(xbytes);
  uint8_t* dW = dY + align256(ybytes);
  const size_t wbytes = (size_t)hm::batch_slots(A->acc_dtype, sl.nrhs) * A->work_bytes_per_rhs;
  hm_status st = HM_OK;
  auto ok = [&](hipError_t e) { if (e != hipSuccess && st == HM_OK) st = HM_EDEVICE; };
  int32_t col = 0;
  for (auto& q : sl.reqs) {
    const size_t o = (size_t)col * nc * vs;
    if (q->x_pinned) {
      if (q->ldx == nc)
        ok(hipMemcpyAsync(dX + o, q->hx, (size_t)nc * q->nrhs * vs, hipMemcpyHostToDevice, sl.stream));
      else
        for (int32_t c = 0; c < q->nrhs; ++c)
          ok(hipMemcpyAsync(dX + o + (size_t)c * nc * vs, (const uint8_t*)q->hx + (size_t)c * q->ldx * vs,
                            (size_t)nc * vs, hipMemcpyHostToDevice, sl.stream));
    } else {
      for (int32_t c = 0; c < q->nrhs; ++c)
        std::memcpy(px + o + (size_t)c * nc * vs, (const uint8_t*)q->hx + (size_t)c * q->ldx * vs,
                    (size_t)nc * vs);
      ok(hipMemcpyAsync(dX + o, px + o, (size_t)nc * q->nrhs * vs, hipMemcpyHostToDevice, sl.stream));
    }
    col += q->nrhs;
  }
  ok(hipMemsetAsync(dY, 0, ybytes, sl.stream));
  if (st == HM_OK) st = hm_mvm_batch(A, sl.nrhs, 1.0, dX, nc, dY, nr, dW, wbytes, sl.stream);
  col = 0;
  for (auto& q : sl.reqs) {
    const size_t o = (size_t)col * nr * vs;
    if (q->y_pinned) {
      if (q->ldy == nr)
        ok(hipMemcpyAsync(q->hy, dY + o, (size_t)nr * q->nrhs * vs, hipMemcpyDeviceToHost, sl.stream));
      else
        for (int32_t c = 0; c < q->nrhs; ++c)
          ok(hipMemcpyAsync((uint8_t*)q->hy + (size_t)c * q->ldy * vs, dY + o + (size_t)c * nr * vs,
                            (size_t)nr * vs, hipMemcpyDeviceToHost, sl.stream));
    } else {
      ok(hipMemcpyAsync(py + o, dY + o, (size_t)nr * q->nrhs * vs, hipMemcpyDeviceToHost, sl.stream));
    }
    col += q->nrhs;
  }
  if (hipStreamSynchronize(sl.stream) != hipSuccess && st == HM_OK) st = HM_EDEVICE;
  if (st != HM_OK) return st;
  col = 0;
  for (auto& q : sl.reqs) {
    if (!q->y_pinned)
      for (int32_t c = 0; c < q->nrhs; ++c)
        std::memcpy((uint8_t*)q->hy + (size_t)c * q->ldy * vs, py + (size_t)(col + c) * nr * vs,
                    (size_t)nr * vs);
    col += q->nrhs;
  }
  return HM_OK;
}

void worker(hm_server* S, Slot* sl) {
  (void)hipSetDevice(S->device);
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    S->cv_assign.wait(lk, [&] { return sl->state == SlotState::kAssigned || S->stop_workers; });
    if (sl->state != SlotState::kAssigned) break;
    sl->state = SlotState::kRunning;
    lk.unlock();
    const hm_status st = sl->fault ? HM_EDEVICE : run_batch(S, *sl);
    lk.lock();
    const auto now = Clock::now();
    for (auto& q : sl->reqs) finish(S, q, st, now);
    S->arena->release(sl->off, sl->bytes);
    sl->reqs.clear();
    sl->state = SlotState::kIdle;
    S->cv_done.notify_all();
    S->cv_work.notify_all();
  }
}

// Dispatcher: forms batches and hands them to idle slots.
void loop(hm_server* S) {
  std::unique_lock<std::mutex> lk(S->mu);
  for (;;) {
    bool assigned = false;
    for (auto& sl : S->slots) {
      if (sl.state != SlotState::kIdle || S->queue.empty()) continue;
      auto head = S->queue.front();
      const hm_matrix* A = S->mats[head->mat];
      if (footprint(A, head->nrhs) > S->arena->size()) {   // can never fit
        S->queue.pop_front();
        finish(S, head, HM_ENOMEM, Clock::now());
        S->cv_done.notify_all();
        continue;
      }
      // gather same-matrix requests in FIFO order up to max_nrhs
      std::vector<std::shared_ptr<Request>> take;
      int32_t r = 0;
      for (auto it = S->queue.begin(); it != S->queue.end();) {
        if ((*it)->mat == head->mat && r + (*it)->nrhs <= A->max_nrhs) {
          r += (*it)->nrhs;
          take.push_back(*it);
          it = S->queue.erase(it);
        } else {
          ++it;
        }
      }
      // admission by memory budget; shrink the batch until it fits
      size_t off = 0;
      while (!take.empty() && !S->arena->alloc(footprint(A, r), &off)) {
        r -= take.back()->nrhs;
        S->queue.push_front(take.back());
        take.pop_back();
      }
      // keep FIFO order of what went back to the queue
      std::stable_sort(S->queue.begin(), S->queue.end(),
                       [](const std::shared_ptr<Request>& a, const std::shared_ptr<Request>& b) {
                         return a->ticket < b->ticket;
                       });
      if (take.empty()) break;   // no memory now: wait for completions
      sl.reqs = std::move(take);
      sl.off = off;
      sl.bytes = footprint(A, r);
      sl.mat = head->mat;
      sl.nrhs = r;
      ++S->batches;
      sl.fault = S->fault_every > 0 && S->batches % S->fault_every == 0;
      sl.state = SlotState::kAssigned;
      assigned = true;
    }
    if (assigned) S->cv_assign.notify_all();
    bool any_busy = false;
    for (auto& sl : S->slots) any_busy |= sl.state != SlotState::kIdle;
    if (S->stop && S->queue.empty() && !any_busy) break;
    // woken by a submission, a completed batch or a stop (bounded wait as a backstop)
    S->cv_work.wait_for(lk, std::chrono::milliseconds(5));
  }
}

}  // namespace

extern "C" {

hm_status hm_server_create(hm_matrix* const* mats, int32_t n_mats, void* d_arena,
                           size_t arena_bytes, void* const* streams, int32_t n_streams,
                           hm_server** out) {
  using hm::fail;
  if (!out || !mats || n_mats <= 0 || !d_arena || !streams || n_streams <= 0)
    return fail(HM_EINVAL, "bad server arguments");
  *out = nullptr;
  if (((uintptr_t)d_arena) % 256) return fail(HM_EINVAL, "arena must be 256-byte aligned");
  for (int32_t i = 0; i < n_mats; ++i)
    if (!mats[i]) return fail(HM_EINVAL, "matrix %d is NULL", i);
  auto S = std::make_unique<hm_server>();
  S->mats.assign(mats, mats + n_mats);
  S->arena_base = (uint8_t*)d_arena;
  S->arena = std::make_unique<Arena>(arena_bytes / 256 * 256);
  S->slots.resize(n_streams);
  for (int32_t i = 0; i < n_streams; ++i) S->slots[i].stream = (hipStream_t)streams[i];
  S->device = mats[0]->device;
  if (const char* f = std::getenv("HM_SERVER_FAULT_EVERY")) S->fault_every = std::atoll(f);
  hm_server* raw = S.release();
  for (auto& sl : raw->slots) sl.worker = std::thread(worker, raw, &sl);
  raw->thread = std::thread(loop, raw);
  *out = raw;
  return hm::ok();
}

hm_status hm_submit(hm_server* s, int32_t mat, int32_t nrhs, const void* h_X, int64_t ldx,
                    void* h_Y, int64_t ldy, uint64_t* ticket) {
  using hm::fail;
  if (!s || !h_X || !h_Y || !ticket) return fail(HM_EINVAL, "NULL argument");
  if (mat < 0 || mat >= (int32_t)s->mats.size()) return fail(HM_EINVAL, "matrix index %d", mat);
  const hm_matrix* A = s->mats[mat];
  if (nrhs < 1 || nrhs > A->max_nrhs) return fail(HM_EINVAL, "nrhs %d outside [1, %d]", nrhs, A->max_nrhs);
  if (ldx < A->hdr.n_cols || ldy < A->hdr.n_rows) return fail(HM_EINVAL, "leading dimension too small");
  auto q = std::make_shared<Request>();
  q->mat = mat; q->nrhs = nrhs; q->hx = h_X; q->ldx = ldx; q->hy = h_Y; q->ldy = ldy;
  q->t_submit = Clock::now();
  const size_t vs = A->acc_dtype == HM_F64 ? 8 : 4;
  q->x_pinned = host_pinned(h_X, ((size_t)(nrhs - 1) * ldx + A->hdr.n_cols) * vs);
  q->y_pinned = host_pinned(h_Y, ((size_t)(nrhs - 1) * ldy + A->hdr.n_rows) * vs);
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) return fail(HM_ESTATE, "server is stopping");
    if (s->queue.size() >= s->max_queue) return fail(HM_EBUSY, "queue full");
    q->ticket = s->next_ticket++;
    s->tickets[q->ticket] = q;
    s->queue.push_back(q);
  }
  s->cv_work.notify_one();
  *ticket = q->ticket;
  return hm::ok();
}

hm_status hm_poll(hm_server* s, uint64_t ticket, int32_t* done, hm_status* result) {
  if (!s || !done) return hm::fail(HM_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> g(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return hm::fail(HM_ESTATE, "unknown ticket %llu", (unsigned long long)ticket);
  *done = it->second->done ? 1 : 0;
  if (result) *result = it->second->done ? it->second->result : HM_OK;
  if (it->second->done) s->tickets.erase(it);       // reported: the ticket is released
  return hm::ok();
}

hm_status hm_wait(hm_server* s, uint64_t ticket, int64_t timeout_us, hm_status* result) {
  if (!s) return hm::fail(HM_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return hm::fail(HM_ESTATE, "unknown ticket %llu", (unsigned long long)ticket);
  auto q = it->second;
  auto pred = [&] { return q->done; };
  if (timeout_us < 0) s->cv_done.wait(lk, pred);
  else if (!s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), pred))
    return hm::fail(HM_ETIMEOUT, "ticket %llu not done after %lld us", (unsigned long long)ticket,
                    (long long)timeout_us);
  if (result) *result = q->result;
  s->tickets.erase(ticket);                         // reported: the ticket is released
  return hm::ok();
}

hm_status hm_server_stats(hm_server* s, double* p50_us, double* p99_us, double* matvecs_per_s) {
  if (!s) return hm::fail(HM_EINVAL, "NULL argument");
  std::vector<double> v;
  int64_t rhs_done = 0;
  double secs = 0;
  {
    std::lock_guard<std::mutex> g(s->mu);     // copy under the lock, sort outside it
    v = s->lat_us;
    rhs_done = s->rhs_done;
    secs = s->have_first ? std::chrono::duration<double>(s->t_last - s->t_first).count() : 0;
  }
  auto pct = [&](double p) {
    if (v.empty()) return 0.0;
    size_t k = (size_t)std::min<double>((double)v.size() - 1, std::ceil(p * v.size()) - 1);
    std::nth_element(v.begin(), v.begin() + k, v.end());
    return v[k];
  };
  if (p50_us) *p50_us = pct(0.50);
  if (p99_us) *p99_us = pct(0.99);
  if (matvecs_per_s) *matvecs_per_s = secs > 0 ? rhs_done / secs : 0.0;
  return hm::ok();
}

void hm_server_destroy(hm_server* s) {
  if (!s) return;
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->thread.joinable()) s->thread.join();       // queue drained, every slot idle
  {
    std::lock_guard<std::mutex> g(s->mu);
    s->stop_workers = true;
  }
  s->cv_assign.notify_all();
  for (auto& sl : s->slots) {
    if (sl.worker.joinable()) sl.worker.join();
    if (sl.pinned) (void)hipHostFree(sl.pinned);
  }
  delete s;
}

}  // extern "C"
