// hp_serve.hip -- the served form: independent requests (one cloud each)
// joined into batches by a scheduler thread (continuous batching).
//
// Admission: every request needs one block of the server's device arena
// (its points when they come from the host, its workspace slots, its device
// outputs and info words).  The arena is allocated once, at creation, with
// the caller's budget; a request waits in FIFO order until its block fits.
//
// Scheduling: up to kSlots batches are in flight, each on a stream of its
// own.  Whenever a slot is free and requests are waiting, the thread admits
// as many as fit (at most max_batch) and enqueues on the slot's stream, in
// order: their points and the batch's work tables (host to device), one
// batched launch sequence for the small requests or the single-cloud
// sequence for each request of at least kServeSingleN points (which fills
// the device by itself), and every request's outputs (device to host) right
// behind its kernels.  A request completes when its last copy has landed; it
// is then marked done with the completion time and its block returns to the
// arena.  Batches in different slots run concurrently: the copies and
// kernels of a request that arrives while another is being served start at
// once on the next free slot's stream instead of queueing behind it.  A
// request that finds nothing waiting and a slot free is issued by the
// submitting thread itself.  When idle, the scheduler keeps polling for
// kIdleSpinNs before it sleeps, so completions are seen without a wake-up.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "hp_arena.h"
#include "hp_batch.h"

namespace hp {

namespace {

constexpr int kSlots = 4;                   // batches in flight, one stream each
constexpr int64_t kIdleSpinNs = 2000000;    // polling before the thread sleeps
constexpr size_t kTableBytes = 8u << 20;    // work-table image capacity of one batch
// Requests with at least this many points run the single-cloud launch
// sequence, which spreads one cloud over the whole device; smaller ones
// share one batched launch sequence.
constexpr int64_t kServeSingleN = 1 << 18;
// Smaller requests share a batched launch sequence only when at least this
// many are issued together; fewer run the single-cloud sequence each, which
// has the lower latency for one cloud.
constexpr size_t kServeMinBatch = 8;

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

struct Request {
  int64_t id = 0;
  int64_t n = 0;
  int32_t p = 1;
  const int32_t *pts = nullptr;
  bool on_device = false;
  int32_t *cx = nullptr, *clo = nullptr, *chi = nullptr, *hx = nullptr, *hy = nullptr, *info = nullptr;
  int32_t cap = 0;               // chain capacity min(n, p); the hull has 2 cap
  bool single = false;           // always runs the single-cloud launch sequence
  TreeShape tree;
  CloudSlots slots;              // batched workspace (single: one workspace of ws_bytes)
  size_t ws_bytes = 0;
  size_t o_pts = 0, o_slots = 0, o_chain = 0, o_hull = 0, o_info = 0, bytes = 0;
  size_t table_bound = 0;
  size_t block = Arena::kFail;
  hipEvent_t ev = nullptr;       // recorded after the request's last output copy; none for the
                                 // slot's last request, which completes when the stream is idle
  bool done = false;
  int64_t done_ns = 0;
};

using RequestPtr = std::shared_ptr<Request>;

struct Slot {
  hipStream_t stream = nullptr;  // copies in, kernels and copies out of this slot's batches
  std::atomic<bool> busy{false}; // claimed (changed under the lock)
  std::atomic<bool> live{false}; // reqs published: the scheduler may poll the slot
  std::vector<RequestPtr> reqs;  // in the order their events are recorded
  size_t head = 0;               // reqs[0, head) have completed and are not touched again
  std::vector<hipEvent_t> events;  // taken from the pool for this batch
  char *himg = nullptr;          // pinned host image of the work tables
  void *dimg = nullptr;          // its device copy
};

}  // namespace

}  // namespace hp

struct hp_server {
  int device = 0;
  size_t budget = 0;
  int32_t max_batch = 1;
  int64_t lds_p_max = 1;
  hp::Arena arena;
  char *dmem = nullptr;
  hp::Slot slot[hp::kSlots];
  std::mutex ev_mu;                  // guards ev_pool (issuing threads and the scheduler)
  std::vector<hipEvent_t> ev_pool;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<hp::RequestPtr> pending;
  std::atomic<int64_t> npending{0};   // pending.size(), readable without the lock
  std::unordered_map<int64_t, hp::RequestPtr> live;   // submitted and not yet waited for
  int64_t next_id = 0;
  bool stop = false;
  std::thread thread;
  // statistics
  int64_t batches = 0, served = 0, peak_in_use = 0, batched_requests = 0;
};

namespace hp {

namespace {

void layout_request(Request &r) {
  tree_shape(r.p, &r.tree);
  r.single = r.n >= kServeSingleN;
  r.slots = cloud_slots(r.p, r.tree);
  // every request can run the single-cloud sequence; small ones can also
  // join a batched sequence (their slots fit the same space)
  r.ws_bytes = std::max(align256(single_ws_bytes(r.n, r.p)), r.slots.total);
  r.cap = (int32_t)chain_cap_for(r.n, r.p);
  size_t o = 0;
  r.o_pts = o;
  if (!r.on_device) o = align256(o + 8 * (size_t)r.n);
  r.o_slots = o;
  o += r.ws_bytes;
  // chain, hull and info back to back, as one host buffer may hold them
  r.o_chain = o;
  r.o_hull = o + 3 * sizeof(int32_t) * (size_t)r.cap;
  r.o_info = r.o_hull + 4 * sizeof(int32_t) * (size_t)r.cap;
  o = align256(r.o_info + sizeof(int32_t) * HP_INFO_WORDS);
  r.bytes = o;
  r.table_bound = r.single ? 0 : BatchTables::cloud_image_bound(r.n, r.p, r.tree);
}

// Mark one request done and return its block.  Called with the lock held.
void finish(hp_server *S, Request *r, int status, int64_t t) {
  if (status != HP_OK) r->info[HP_INFO_STATUS] = status;
  r->done = true;
  r->done_ns = t;
  S->arena.release(r->block);
  r->block = Arena::kFail;
  ++S->served;
}

// Free a slot whose requests are all done: its events go back to the pool.
void release_slot(hp_server *S, Slot &sl) {
  {
    std::lock_guard<std::mutex> g(S->ev_mu);
    for (hipEvent_t e : sl.events) S->ev_pool.push_back(e);
  }
  sl.events.clear();
  sl.reqs.clear();
  sl.head = 0;
  sl.live.store(false, std::memory_order_release);
  sl.busy = false;
}

// Whether a request's copies have landed: its event, or for the slot's last
// request (no event recorded behind it) the slot's stream being idle, which
// the runtime reports sooner than an event placed after the same copy.
hipError_t request_state(const Slot &sl, const Request *r) {
  return r->ev ? hipEventQuery(r->ev) : hipStreamQuery(sl.stream);
}

// Complete the requests of a slot whose events have fired (in recording
// order).  Called with the lock held; returns true if any completed.
bool poll_slot(hp_server *S, Slot &sl, bool &busy) {
  bool any = false;
  const int64_t t = now_ns();
  while (sl.head < sl.reqs.size()) {
    Request *r = sl.reqs[sl.head].get();
    const hipError_t q = request_state(sl, r);
    if (q == hipErrorNotReady) break;
    finish(S, r, q == hipSuccess ? HP_OK : HP_EDEVICE, t);
    ++sl.head;
    any = true;
  }
  if (any) S->cv_done.notify_all();
  if (sl.head == sl.reqs.size()) release_slot(S, sl);
  else busy = true;
  return any;
}

hipEvent_t pool_event(hp_server *S, Slot &sl) {
  hipEvent_t e = nullptr;
  {
    std::lock_guard<std::mutex> g(S->ev_mu);
    if (!S->ev_pool.empty()) {
      e = S->ev_pool.back();
      S->ev_pool.pop_back();
    }
  }
  if (!e && hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  sl.events.push_back(e);
  return e;
}

// Copies and launches for the requests in `take` (blocks already
// allocated), all on the slot's stream.  Runs without the lock, on the
// thread that launches the slot (the scheduler, or a submitting thread that
// found the server idle).  The small requests' points and the work tables
// are copied first and computed in one batched launch sequence; the other
// requests follow one by one with the single-cloud sequence.  Every
// request's outputs are copied back right behind its own kernels and an
// event is recorded after them (none after the slot's last request, which
// completes when the stream is idle), so it completes independently of the
// rest of the batch.  Reorders `take` into completion order.
hipError_t issue(hp_server *S, Slot &sl, std::vector<RequestPtr> &take) {
  std::stable_partition(take.begin(), take.end(), [](const RequestPtr &r) { return !r->single; });
  size_t small = 0;
  while (small < take.size() && !take[small]->single) ++small;
  const size_t nbatched = small >= kServeMinBatch ? small : 0;   // the rest run one by one
  BatchTables t;
  std::vector<BCloud> clouds;
  std::vector<const int32_t *> cpts;
  std::vector<const int32_t *> dpts(take.size());
  hipError_t e = hipSuccess;
  const hipStream_t st = sl.stream;
  auto outputs = [&](Request &r) {
    char *base = S->dmem + r.block;
    CloudOut o;
    int32_t *chain = reinterpret_cast<int32_t *>(base + r.o_chain);
    int32_t *hull = reinterpret_cast<int32_t *>(base + r.o_hull);
    o.cx = chain;
    o.clo = chain + r.cap;
    o.chi = chain + 2 * (size_t)r.cap;
    o.chain_cap = r.cap;
    o.hx = hull;
    o.hy = hull + 2 * (size_t)r.cap;
    o.hull_cap = 2 * r.cap;
    o.info = reinterpret_cast<int32_t *>(base + r.o_info);
    o.mask = nullptr;
    return o;
  };
  auto copy_in = [&](size_t b) -> hipError_t {
    Request &r = *take[b];
    if (r.on_device) {
      dpts[b] = r.pts;
      return hipSuccess;
    }
    int32_t *dst = reinterpret_cast<int32_t *>(S->dmem + r.block + r.o_pts);
    dpts[b] = dst;
    if (r.n == 0) return hipSuccess;
    return hipMemcpyAsync(dst, r.pts, 8 * (size_t)r.n, hipMemcpyHostToDevice, st);
  };
  auto copy_out = [&](Request &r) -> hipError_t {
    const char *base = S->dmem + r.block;
    const int32_t *h = r.cx;
    const size_t c4 = (size_t)r.cap;
    if (h && r.clo == h + c4 && r.chi == h + 2 * c4 && r.hx == h + 3 * c4 && r.hy == h + 5 * c4 &&
        r.info == h + 7 * c4)   // one host buffer laid out as the device block
      return hipMemcpyAsync(r.cx, base + r.o_chain, sizeof(int32_t) * (7 * c4 + HP_INFO_WORDS),
                            hipMemcpyDeviceToHost, st);
    const int32_t *chain = reinterpret_cast<const int32_t *>(base + r.o_chain);
    const int32_t *hull = reinterpret_cast<const int32_t *>(base + r.o_hull);
    const size_t c = sizeof(int32_t) * (size_t)r.cap;
    hipError_t x = hipSuccess;
    if (r.cap > 0) {
      if ((x = hipMemcpyAsync(r.cx, chain, c, hipMemcpyDeviceToHost, st)) != hipSuccess) return x;
      if ((x = hipMemcpyAsync(r.clo, chain + r.cap, c, hipMemcpyDeviceToHost, st)) != hipSuccess) return x;
      if ((x = hipMemcpyAsync(r.chi, chain + 2 * (size_t)r.cap, c, hipMemcpyDeviceToHost, st)) != hipSuccess) return x;
      if ((x = hipMemcpyAsync(r.hx, hull, 2 * c, hipMemcpyDeviceToHost, st)) != hipSuccess) return x;
      if ((x = hipMemcpyAsync(r.hy, hull + 2 * (size_t)r.cap, 2 * c, hipMemcpyDeviceToHost, st)) != hipSuccess) return x;
    }
    return hipMemcpyAsync(r.info, base + r.o_info, sizeof(int32_t) * HP_INFO_WORDS, hipMemcpyDeviceToHost, st);
  };
  // small requests: points, tables, one batched launch, outputs, one event
  size_t nsmall = 0;
  while (nsmall < nbatched) {
    Request &r = *take[nsmall];
    if ((e = copy_in(nsmall)) != hipSuccess) return e;
    t.add_cloud(r.n, r.p, r.tree, S->lds_p_max);
    clouds.push_back(make_bcloud(r.p, r.tree, S->dmem + r.block + r.o_slots, r.slots, outputs(r)));
    cpts.push_back(dpts[nsmall]);
    ++nsmall;
  }
  if (nsmall > 0) {
    t.sort_items();
    const size_t img = batch_image_bytes(t);
    if (img > kTableBytes) return hipErrorInvalidValue;   // excluded by admission
    DeviceBatch D;
    batch_image(t, clouds, cpts, sl.himg, static_cast<char *>(sl.dimg), D);
    if ((e = hipMemcpyAsync(sl.dimg, sl.himg, img, hipMemcpyHostToDevice, st)) != hipSuccess) return e;
    if ((e = enqueue_batch(D, st)) != hipSuccess) return e;
    for (size_t b = 0; b < nsmall; ++b)
      if ((e = copy_out(*take[b])) != hipSuccess) return e;
    hipEvent_t done = nullptr;   // the slot's last work: completes with its stream
    if (nsmall < take.size()) {
      if (!(done = pool_event(S, sl))) return hipErrorOutOfMemory;
      if ((e = hipEventRecord(done, st)) != hipSuccess) return e;
    }
    for (size_t b = 0; b < nsmall; ++b) take[b]->ev = done;
  }
  // the other requests one by one, each with its own copies
  for (size_t b = nsmall; b < take.size(); ++b) {
    Request &r = *take[b];
    if ((e = copy_in(b)) != hipSuccess) return e;
    const CloudOut o = outputs(r);
    if (run_single(dpts[b], r.n, r.p, nullptr, nullptr, nullptr, o.cx, o.clo, o.chi, o.chain_cap, o.hx, o.hy,
                   o.hull_cap, o.info, S->dmem + r.block + r.o_slots, r.ws_bytes, st, true) != HP_OK)
      return hipErrorLaunchFailure;
    if ((e = copy_out(r)) != hipSuccess) return e;
    hipEvent_t done = nullptr;
    if (b + 1 < take.size()) {
      if (!(done = pool_event(S, sl))) return hipErrorOutOfMemory;
      if ((e = hipEventRecord(done, st)) != hipSuccess) return e;
    }
    r.ev = done;
  }
  return hipSuccess;
}

// Admit the waiting requests that fit (FIFO, stop at the first that does
// not) into a free slot and issue them.  Called with the lock held, by the
// scheduler thread or by a submitting thread that found the server idle;
// drops the lock around the device calls.  Returns true if a batch was
// issued.
bool launch(hp_server *S, Slot &sl, std::unique_lock<std::mutex> &lk) {
  std::vector<RequestPtr> take;
  size_t table = BatchTables::kImageSlack;
  while (!S->pending.empty() && (int32_t)take.size() < S->max_batch) {
    const RequestPtr &r = S->pending.front();
    if (table + r->table_bound > kTableBytes) break;
    const size_t at = S->arena.alloc(r->bytes);
    if (at == Arena::kFail) break;
    r->block = at;
    table += r->table_bound;
    take.push_back(r);
    S->pending.pop_front();
  }
  S->npending.store((int64_t)S->pending.size(), std::memory_order_release);
  if (take.empty()) return false;
  S->peak_in_use = std::max<int64_t>(S->peak_in_use, (int64_t)S->arena.in_use());
  sl.busy = true;
  ++S->batches;
  S->batched_requests += (int64_t)take.size();
  lk.unlock();
  const hipError_t e = issue(S, sl, take);
  if (e != hipSuccess) {
    // nothing of this batch may still touch its blocks when they are freed
    (void)hipStreamSynchronize(sl.stream);
  }
  lk.lock();
  sl.reqs = take;
  sl.head = 0;
  if (e != hipSuccess) {
    const int64_t t = now_ns();
    for (const RequestPtr &r : take) finish(S, r.get(), HP_EDEVICE, t);
    S->cv_done.notify_all();
    release_slot(S, sl);
  } else {
    sl.live.store(true, std::memory_order_release);
  }
  return true;
}

void serve_loop(hp_server *S) {
  (void)hipSetDevice(S->device);
  int64_t active = now_ns();   // the last time there was work
  for (;;) {
    // Only this thread completes requests, and a slot's requests and head
    // change after it is published (live) only here, so the published
    // slots are polled without the lock; the lock is taken only when a
    // request has completed, when requests wait, and to sleep.  A
    // submitting thread therefore rarely finds the lock held.
    bool busy = false, ready = false;
    for (Slot &sl : S->slot) {
      if (!sl.live.load(std::memory_order_acquire)) continue;
      busy = true;
      if (request_state(sl, sl.reqs[sl.head].get()) != hipErrorNotReady) ready = true;
    }
    if (ready || S->npending.load(std::memory_order_acquire) > 0) {
      std::unique_lock<std::mutex> lk(S->mu);
      bool progressed = false, still = false;
      for (Slot &sl : S->slot)
        if (sl.live.load(std::memory_order_relaxed) && poll_slot(S, sl, still)) progressed = true;
      for (Slot &sl : S->slot) {
        if (sl.busy || S->pending.empty()) continue;
        if (launch(S, sl, lk)) progressed = true;
      }
      lk.unlock();
      active = now_ns();
      if (!progressed) std::this_thread::yield();   // waiting for room
      continue;
    }
    bool claimed = false;   // a slot a submitting thread is still issuing into
    for (Slot &sl : S->slot) claimed |= sl.busy && !sl.live.load(std::memory_order_acquire);
    if (busy || claimed) {
      active = now_ns();
      std::this_thread::yield();
      continue;
    }
    if (now_ns() - active < kIdleSpinNs) {
      std::this_thread::yield();
      continue;
    }
    std::unique_lock<std::mutex> lk(S->mu);
    auto any_busy = [&] {
      for (Slot &sl : S->slot)
        if (sl.busy) return true;
      return false;
    };
    if (any_busy()) continue;   // claimed by a submitting thread meanwhile
    if (S->stop && S->pending.empty()) break;
    // woken by a request queued for this thread or issued by its submitter
    S->cv_work.wait(lk, [&] { return S->stop || !S->pending.empty() || any_busy(); });
    active = now_ns();
  }
}

}  // namespace

}  // namespace hp

using namespace hp;

extern "C" int hp_server_destroy(hp_server *S) {
  if (!S) return HP_OK;
  if (S->thread.joinable()) {
    {
      std::lock_guard<std::mutex> g(S->mu);
      S->stop = true;
    }
    S->cv_work.notify_all();
    S->thread.join();
  }
  S->live.clear();
  for (Slot &sl : S->slot) {
    for (hipEvent_t e : sl.events) (void)hipEventDestroy(e);
    if (sl.himg) (void)hipHostFree(sl.himg);
    if (sl.dimg) (void)hipFree(sl.dimg);
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
  }
  for (hipEvent_t e : S->ev_pool) (void)hipEventDestroy(e);
  if (S->dmem) (void)hipFree(S->dmem);
  delete S;
  return HP_OK;
}

extern "C" int hp_server_create(size_t device_budget_bytes, int32_t max_batch, hp_server **out) {
  if (!out) return set_error(HP_EINVAL, "server pointer is NULL");
  *out = nullptr;
  if (max_batch < 1) return set_error(HP_EINVAL, "max_batch = %d < 1", max_batch);
  if (device_budget_bytes < Arena::kAlign) return set_error(HP_EINVAL, "device budget of %zu bytes is too small", device_budget_bytes);
  hp_server *S = new (std::nothrow) hp_server;
  if (!S) return set_error(HP_ENOMEM, "host allocation failed");
  if (hipGetDevice(&S->device) != hipSuccess) {
    hp_server_destroy(S);
    return set_error(HP_EDEVICE, "no current device");
  }
  const DeviceInfo &D = device_info();
  S->lds_p_max = D.lds_max_p - 8;
  S->budget = device_budget_bytes / Arena::kAlign * Arena::kAlign;
  S->max_batch = max_batch;
  int rc = HP_OK;
  if (hipMalloc(reinterpret_cast<void **>(&S->dmem), S->budget) != hipSuccess)
    rc = set_error(HP_ENOMEM, "device arena of %zu bytes could not be allocated", S->budget);
  for (Slot &sl : S->slot) {
    if (rc != HP_OK) break;
    if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess) {
      rc = set_error(HP_EDEVICE, "stream creation failed");
      break;
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&sl.himg), kTableBytes, hipHostMallocDefault) != hipSuccess ||
        hipMalloc(&sl.dimg, kTableBytes) != hipSuccess)
      rc = set_error(HP_ENOMEM, "server slot resources could not be allocated");
  }
  if (rc == HP_OK && prepare_b_reduce() != hipSuccess) rc = set_error(HP_EDEVICE, "reduce kernel setup failed");
  if (rc != HP_OK) {
    hp_server_destroy(S);
    return rc;
  }
  S->arena.reset(S->budget);
  try {
    S->thread = std::thread(serve_loop, S);
  } catch (...) {
    hp_server_destroy(S);
    return set_error(HP_EDEVICE, "scheduler thread could not start");
  }
  *out = S;
  return HP_OK;
}

extern "C" int hp_server_request_bytes(int64_t n, int32_t p, int32_t on_device, size_t *bytes) {
  if (!bytes) return set_error(HP_EINVAL, "bytes is NULL");
  if (n < 0) return set_error(HP_EINVAL, "n = %lld < 0", (long long)n);
  if (p < 1 || p > kBatchPMax) return set_error(HP_EINVAL, "p = %d outside [1, %d]", p, kBatchPMax);
  Request r;
  r.n = n;
  r.p = p;
  r.on_device = on_device != 0;
  layout_request(r);
  *bytes = r.bytes;
  return HP_OK;
}

extern "C" int hp_server_submit(hp_server *S, const int32_t *pts, int64_t n, int32_t p, int32_t on_device,
                                int32_t *cx, int32_t *clo, int32_t *chi, int32_t chain_cap, int32_t *hx,
                                int32_t *hy, int32_t *info, int64_t *ticket) {
  if (!S) return set_error(HP_EINVAL, "server is NULL");
  if (!ticket) return set_error(HP_EINVAL, "ticket is NULL");
  if (n < 0) return set_error(HP_EINVAL, "n = %lld < 0", (long long)n);
  if (p < 1 || p > kBatchPMax) return set_error(HP_EINVAL, "p = %d outside [1, %d]", p, kBatchPMax);
  if (n > 0 && !pts) return set_error(HP_EINVAL, "pts is NULL");
  if (pts && ((uintptr_t)pts & 7)) return set_error(HP_EINVAL, "pts is not 8-byte aligned");
  if (!info) return set_error(HP_EINVAL, "info is NULL");
  const int64_t cap = chain_cap_for(n, p);
  if (chain_cap < cap) return set_error(HP_ECAPACITY, "chain_cap %d < min(n, p) = %lld", chain_cap, (long long)cap);
  if (cap > 0 && (!cx || !clo || !chi || !hx || !hy)) return set_error(HP_EINVAL, "NULL output buffer");
  RequestPtr r;
  try {
    r = std::make_shared<Request>();
  } catch (...) {
    return set_error(HP_ENOMEM, "host allocation failed");
  }
  r->n = n;
  r->p = p;
  r->pts = pts;
  r->on_device = on_device != 0;
  r->cx = cx;
  r->clo = clo;
  r->chi = chi;
  r->hx = hx;
  r->hy = hy;
  r->info = info;
  layout_request(*r);
  if (r->bytes > S->arena.size() || r->table_bound + BatchTables::kImageSlack > kTableBytes) {
    const size_t need = r->bytes;
    return set_error(HP_ECAPACITY, "request needs %zu device bytes, the server budget is %zu", need, S->budget);
  }
  // A request that finds nothing waiting and a slot free is issued here, on
  // the submitting thread (when its current device is the server's), which
  // saves the hand-over to the scheduler thread; the scheduler still
  // completes it.
  int cur = -1;
  const bool direct = hipGetDevice(&cur) == hipSuccess && cur == S->device;
  {
    std::unique_lock<std::mutex> lk(S->mu);
    r->id = S->next_id++;
    S->live[r->id] = r;
    const bool idle = S->pending.empty();
    S->pending.push_back(r);
    S->npending.store((int64_t)S->pending.size(), std::memory_order_release);
    *ticket = r->id;
    if (direct && idle && !S->stop)
      for (Slot &sl : S->slot)
        if (!sl.busy) {
          launch(S, sl, lk);
          break;
        }
  }
  S->cv_work.notify_one();   // a sleeping scheduler polls the issued request too
  return HP_OK;
}

extern "C" int hp_server_wait(hp_server *S, int64_t ticket, int64_t timeout_us, int64_t *done_ns) {
  if (!S) return set_error(HP_EINVAL, "server is NULL");
  std::unique_lock<std::mutex> lk(S->mu);
  auto it = S->live.find(ticket);
  if (it == S->live.end()) return set_error(HP_EINVAL, "unknown ticket %lld", (long long)ticket);
  const RequestPtr r = it->second;
  auto ready = [&] { return r->done; };
  if (timeout_us < 0) {
    S->cv_done.wait(lk, ready);
  } else if (!S->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return HP_ETIMEOUT;
  }
  if (done_ns) *done_ns = r->done_ns;
  S->live.erase(ticket);
  return HP_OK;
}

extern "C" int hp_server_stats(hp_server *S, int64_t *stats) {
  if (!S || !stats) return set_error(HP_EINVAL, "server or stats is NULL");
  std::lock_guard<std::mutex> g(S->mu);
  stats[0] = S->batches;
  stats[1] = S->served;
  stats[2] = S->batched_requests;
  stats[3] = S->peak_in_use;
  stats[4] = (int64_t)S->pending.size();
  stats[5] = (int64_t)S->arena.size();
  return HP_OK;
}

extern "C" int64_t hp_clock_ns(void) { return now_ns(); }
