// Serving form: a continuous-batching engine around the persistent batched
// kernel.
//
// One scheduler thread owns every HIP call after creation.  Its loop:
//   1. admission -- queued requests are admitted in arrival order while their
//      input and output bytes fit the device arena (first-fit free list over a
//      single allocation, 256-byte granules, neighbours merged on free); the
//      input copy is issued on the copy stream and an event recorded;
//   2. requests whose input copy has completed become ready (the scheduler
//      polls the copy events: with few hardware queues per process, device-side
//      waits across streams were measured to stall unrelated copies);
//      when a compute slot is free, every ready request (up to max_batch) is
//      put into one batch: the descriptors and tile list are staged in pinned
//      memory and copied to the slot's device buffer in one copy, and the
//      batched kernel is launched; batches in
//      different slots overlap on the device, and requests that arrive while
//      batches run join the next one;
//   3. when the scheduler sees a batch's kernel complete (its event polled
//      again), the slot is free and the batch's outputs go back on one
//      device-to-host stream, smallest output first, so the PCIe link serves
//      copies one at a time instead of splitting its bandwidth over concurrent
//      ones; each request completes, and returns its arena space, when its
//      own output copy has landed (an event per request), not when its whole
//      batch has.  No stream ever waits on another on the device.
// The coefficient table of the four transforms stays resident.
//
// Errors: every HIP call the scheduler makes is checked.  A request whose
// descriptors are rejected, whose copy or launch cannot be enqueued, or whose
// events report a device error completes at once with that status (and its
// arena space returned); poll and wait return the status, so a failure never
// shows up as a request that is done with its output unwritten, nor as a wait
// that times out.  Only hipSuccess and hipErrorNotReady of an event query
// count as "complete" and "pending".
//
// Locking: the scheduler owns the request pipeline and makes its HIP calls
// without holding any lock that callers take.  Callers meet it at three small
// locks: `mu_in` (incoming requests and the id map), `mu_done` (completion
// wake-ups; a request's done flag is atomic) and `mu_stats` (counters).  A
// submit, poll or wait therefore never waits behind a run of HIP calls.
// Events come from a pool owned by the scheduler, and creation warms every
// stream and the batched kernel with one tiny request, so that the first real
// requests pay no one-time costs.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdarg>
#include <sys/prctl.h>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "launch.h"

using namespace mact;

namespace {

using Clock = std::chrono::steady_clock;

constexpr size_t kGranule = 256;

// First-fit allocator over [0, size) with coalescing.
class Arena {
 public:
  explicit Arena(size_t size) : size_(size) { free_[0] = size; }
  bool alloc(size_t bytes, size_t* off) {
    bytes = (bytes + kGranule - 1) / kGranule * kGranule;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const size_t rest = it->second - bytes;
        const size_t start = it->first + bytes;
        free_.erase(it);
        if (rest) free_[start] = rest;
        used_ += bytes;
        return true;
      }
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    bytes = (bytes + kGranule - 1) / kGranule * kGranule;
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

struct Req {
  int64_t id = 0;
  mact_request r{};
  size_t in_bytes = 0, out_bytes = 0, in_off = 0, out_off = 0;
  bool placed = false;  // holds arena space
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  Clock::time_point t_submit, t_done;  // t_done, status and err are written before done is set
  mact_status status = MACT_OK;
  char err[256] = "";
  std::atomic<bool> done{false};
  // 0 waiting for admission, 1 admitted, 2 cancelled: the scheduler (admission) and
  // mact_server_cancel each move it out of 0 once, so exactly one of them owns the request
  std::atomic<int> phase{0};
};

struct Slot {
  hipStream_t stream = nullptr;
  char* d_buf = nullptr;  // descriptors, then the tile list
  char* h_buf = nullptr;  // pinned staging of the same
  size_t buf_bytes = 0;
  std::vector<Req*> reqs;
  bool busy = false;
  Clock::time_point t_launch;
  hipEvent_t ev_k0 = nullptr, ev_k1 = nullptr;
};

size_t esize(int dtype) { return dtype == MACT_U8 ? 1 : (dtype == MACT_F16 || dtype == MACT_U16) ? 2 : 4; }

}  // namespace

struct mact_server {
  int device = 0;
  mact_server_config cfg{};
  int deg = 5;
  mact_tune tune{512, 8192, 4, 32, 0};  // small tiles: a single request still spreads over the CUs
  std::unique_ptr<Arena> arena;
  char* d_arena = nullptr;
  KCoef* d_coefs = nullptr;
  hipStream_t copy_stream = nullptr;  // host -> device, in admission order
  hipStream_t d2h_stream = nullptr;   // device -> host, in launch order
  std::vector<Slot> slots;

  // shared with callers
  std::mutex mu_in;  // incoming, all, next_id, submitted, rejected, stop
  std::condition_variable cv_work;
  std::deque<Req*> incoming;
  std::unordered_map<int64_t, std::unique_ptr<Req>> all;
  int64_t next_id = 1, submitted = 0, rejected = 0;
  bool stop = false;
  std::atomic<int64_t> waiting{0};  // submitted, not yet admitted to the arena
  std::mutex mu_done;
  std::condition_variable cv_done;
  std::mutex mu_stats;  // lat_ms, completed, batches, batched_reqs, busy_ms
  std::vector<double> lat_ms;
  int64_t completed = 0, failed = 0, cancelled = 0, batches = 0, batched_reqs = 0;
  double busy_ms = 0.0;

  // the scheduler's own
  std::deque<Req*> queued;   // submitted, not admitted
  std::vector<Req*> copying;  // input copy in flight
  std::vector<Req*> ready;    // input on the device, not yet in a batch
  std::vector<Req*> draining;  // output copy in flight
  std::vector<hipEvent_t> ev_pool;
  std::thread th;

  void loop();
  void release(Req* q);
  void fail_req(Req* q, mact_status st, const char* fmt, ...);
  hipEvent_t get_event();
  bool take_incoming();
  bool admit();
  void poll_copies();
  bool launch(Slot& s);
  bool finish_slots();
  bool finish_requests();
};

// nullptr if the pool is empty and a new event cannot be created
hipEvent_t mact_server::get_event() {
  if (!ev_pool.empty()) {
    hipEvent_t e = ev_pool.back();
    ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
  return e;
}

// Returns the request's arena space and events.
void mact_server::release(Req* q) {
  if (q->placed) {
    arena->release(q->in_off, q->in_bytes);
    arena->release(q->out_off, q->out_bytes);
    q->placed = false;
  }
  if (q->ev_in) ev_pool.push_back(q->ev_in);
  if (q->ev_out) ev_pool.push_back(q->ev_out);
  q->ev_in = q->ev_out = nullptr;
}

// Completes request q with an error: its status and detail are what poll and
// wait report.  The caller has removed q from the scheduler's lists.
void mact_server::fail_req(Req* q, mact_status st, const char* fmt, ...) {
  release(q);
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(q->err, sizeof q->err, fmt, ap);
  va_end(ap);
  q->status = st;
  q->t_done = Clock::now();
  {
    std::lock_guard<std::mutex> g(mu_done);
    q->done.store(true);
  }
  {
    std::lock_guard<std::mutex> g(mu_stats);
    ++failed;
  }
  cv_done.notify_all();
}

bool mact_server::take_incoming() {
  std::lock_guard<std::mutex> g(mu_in);
  if (incoming.empty()) return false;
  queued.insert(queued.end(), incoming.begin(), incoming.end());
  incoming.clear();
  return true;
}

bool mact_server::admit() {
  bool any = false;
  while (!queued.empty()) {
    Req* q = queued.front();
    if (q->phase.load() == 2) {  // cancelled while waiting: mact_server_cancel has completed it
      queued.pop_front();
      waiting.fetch_sub(1);
      any = true;
      continue;
    }
    size_t in_off, out_off;
    if (!arena->alloc(q->in_bytes, &in_off)) break;
    if (!arena->alloc(q->out_bytes, &out_off)) {
      arena->release(in_off, q->in_bytes);
      break;
    }
    queued.pop_front();
    waiting.fetch_sub(1);
    int expect = 0;
    if (!q->phase.compare_exchange_strong(expect, 1)) {  // cancelled just now
      arena->release(in_off, q->in_bytes);
      arena->release(out_off, q->out_bytes);
      any = true;
      continue;
    }
    q->in_off = in_off;
    q->out_off = out_off;
    q->placed = true;
    any = true;
    q->ev_in = get_event();
    q->ev_out = get_event();
    if (!q->ev_in || !q->ev_out) {
      fail_req(q, MACT_E_DEVICE, "request %lld: no event for its copies", (long long)q->id);
      continue;
    }
    hipError_t e = hipMemcpyAsync(d_arena + in_off, q->r.host_in, q->in_bytes, hipMemcpyHostToDevice, copy_stream);
    if (e == hipSuccess) e = hipEventRecord(q->ev_in, copy_stream);
    if (e != hipSuccess) {
      fail_req(q, MACT_E_DEVICE, "request %lld: input copy: %s", (long long)q->id, hipGetErrorString(e));
      continue;
    }
    copying.push_back(q);
  }
  return any;
}

void mact_server::poll_copies() {
  // copies complete in admission order (one copy stream): stop at the first pending one; a
  // device error fails the request instead of leaving it pending for ever
  size_t i = 0;
  while (i < copying.size()) {
    Req* q = copying[i];
    const hipError_t e = hipEventQuery(q->ev_in);
    if (e == hipErrorNotReady) break;
    if (e == hipSuccess) {
      ready.push_back(q);
    } else {
      fail_req(q, MACT_E_DEVICE, "request %lld: input copy: %s", (long long)q->id, hipGetErrorString(e));
    }
    ++i;
  }
  copying.erase(copying.begin(), copying.begin() + i);
}

bool mact_server::launch(Slot& s) {
  if (ready.empty()) return false;
  const size_t n = std::min<size_t>(ready.size(), (size_t)cfg.max_batch);
  std::vector<Req*> take(ready.begin(), ready.begin() + n);  // admission order is arrival order
  ready.erase(ready.begin(), ready.begin() + n);
  s.reqs.clear();
  std::vector<BDesc> descs;
  descs.reserve(n);
  for (Req* q : take) {
    mact_image in{}, out{};
    in.data = d_arena + q->in_off;
    in.dtype = q->r.in_dtype;
    in.layout = MACT_HWC;
    in.width = q->r.width;
    in.height = q->r.height;
    in.gamma = q->r.gamma;
    out.data = d_arena + q->out_off;
    out.dtype = q->r.out_dtype;
    out.layout = MACT_HWC;
    out.width = q->r.width;
    out.height = q->r.height;
    int d = 5;
    const size_t before = descs.size();
    mact_status st = cfg.fail_request != 0 && q->id == cfg.fail_request
                         ? fail(MACT_E_INVALID, "descriptors rejected (the configuration's fail_request)")
                         : make_batch_descs(cfg.params[q->r.xform], &in, &out, q->r.xform, &descs, &d, "mact_server");
    if (st != MACT_OK) {
      descs.resize(before);
      fail_req(q, st, "request %lld: %s", (long long)q->id, mact_last_error());
      clear_error();
      continue;
    }
    s.reqs.push_back(q);
  }
  if (s.reqs.empty()) return true;  // every request of the batch failed: progress, the slot stays free
  std::vector<uint32_t> ts;
  const uint32_t total = build_tiles(descs, (uint32_t)tune.tile, &ts);
  const size_t db = descs.size() * sizeof(BDesc), tb = ts.size() * sizeof(uint32_t);
  std::memcpy(s.h_buf, descs.data(), db);
  std::memcpy(s.h_buf + db, ts.data(), tb);
  hipError_t e = hipMemcpyAsync(s.d_buf, s.h_buf, db + tb, hipMemcpyHostToDevice, s.stream);
  if (e == hipSuccess) e = hipEventRecord(s.ev_k0, s.stream);
  if (e == hipSuccess)
    e = launch_batch_kernel(reinterpret_cast<const BDesc*>(s.d_buf), d_coefs,
                            reinterpret_cast<const uint32_t*>(s.d_buf + db), (int32_t)descs.size(), total, tune, deg,
                            s.stream);
  if (e == hipSuccess) e = hipEventRecord(s.ev_k1, s.stream);
  if (e != hipSuccess) {
    // the batch may or may not have been enqueued: wait for the slot's stream before its
    // requests' arena space can be handed out again
    (void)hipStreamSynchronize(s.stream);
    for (Req* q : s.reqs) fail_req(q, MACT_E_DEVICE, "request %lld: batch launch: %s", (long long)q->id, hipGetErrorString(e));
    s.reqs.clear();
    return true;
  }
  s.busy = true;
  s.t_launch = Clock::now();
  std::lock_guard<std::mutex> g(mu_stats);
  ++batches;
  batched_reqs += (int64_t)s.reqs.size();
  return true;
}

// A slot whose kernel has finished: its requests' outputs go back on the
// device-to-host stream, smallest first, and the slot is free again.  The
// copies are enqueued only once the kernel is seen complete, so the
// device-to-host stream never holds a wait on another stream: with few
// hardware queues per process, streams share queues, and such a wait
// measured to stall the copies queued behind it (the served form then ran
// 30-40% below the plain per-request path under load).
bool mact_server::finish_slots() {
  bool any = false;
  for (Slot& s : slots) {
    if (!s.busy) continue;
    const hipError_t e = hipEventQuery(s.ev_k1);
    if (e == hipErrorNotReady) continue;
    any = true;
    s.busy = false;
    if (e != hipSuccess) {
      for (Req* q : s.reqs) fail_req(q, MACT_E_DEVICE, "request %lld: batch kernel: %s", (long long)q->id, hipGetErrorString(e));
      s.reqs.clear();
      continue;
    }
    float kms = 0.0f;
    if (hipEventElapsedTime(&kms, s.ev_k0, s.ev_k1) == hipSuccess) {
      std::lock_guard<std::mutex> g(mu_stats);
      busy_ms += kms;
    }
    std::vector<Req*> by_size(s.reqs);
    s.reqs.clear();
    std::stable_sort(by_size.begin(), by_size.end(), [](const Req* a, const Req* b) { return a->out_bytes < b->out_bytes; });
    for (Req* q : by_size) {
      hipError_t ce = hipMemcpyAsync(q->r.host_out, d_arena + q->out_off, q->out_bytes, hipMemcpyDeviceToHost, d2h_stream);
      if (ce == hipSuccess) ce = hipEventRecord(q->ev_out, d2h_stream);
      if (ce != hipSuccess) {
        (void)hipStreamSynchronize(d2h_stream);
        fail_req(q, MACT_E_DEVICE, "request %lld: output copy: %s", (long long)q->id, hipGetErrorString(ce));
        continue;
      }
      draining.push_back(q);
    }
  }
  return any;
}

bool mact_server::finish_requests() {
  std::vector<double> lat;
  bool any = false;
  const auto now = Clock::now();
  for (size_t i = 0; i < draining.size();) {
    Req* q = draining[i];
    const hipError_t e = hipEventQuery(q->ev_out);
    if (e == hipErrorNotReady) {
      ++i;
      continue;
    }
    draining[i] = draining.back();
    draining.pop_back();
    any = true;
    if (e != hipSuccess) {
      fail_req(q, MACT_E_DEVICE, "request %lld: output copy: %s", (long long)q->id, hipGetErrorString(e));
      continue;
    }
    release(q);
    q->t_done = now;
    lat.push_back(std::chrono::duration<double, std::milli>(q->t_done - q->t_submit).count());
    {
      std::lock_guard<std::mutex> g(mu_done);  // a waiter checks done under this lock
      q->done.store(true);
    }
  }
  if (lat.empty()) return any;
  {
    std::lock_guard<std::mutex> g(mu_stats);
    lat_ms.insert(lat_ms.end(), lat.begin(), lat.end());
    completed += (int64_t)lat.size();
  }
  cv_done.notify_all();
  return true;
}

void mact_server::loop() {
  (void)hipSetDevice(device);
  // the loop polls device events with 5 us sleeps; Linux's default timer slack (50 us) would
  // stretch each of them tenfold and add it to every stage of a request's latency
  (void)prctl(PR_SET_TIMERSLACK, 1000UL, 0UL, 0UL, 0UL);
  for (;;) {
    bool progress = false;
    progress |= finish_requests();
    progress |= finish_slots();
    progress |= take_incoming();
    progress |= admit();
    poll_copies();
    for (Slot& s : slots)
      if (!s.busy) progress |= launch(s);
    const bool in_flight = !copying.empty() || !draining.empty() ||
                           std::any_of(slots.begin(), slots.end(), [](const Slot& s) { return s.busy; });
    if (progress) continue;
    if (in_flight || !ready.empty()) {
      // device work outstanding: poll its events again shortly
      std::this_thread::sleep_for(std::chrono::microseconds(5));
      continue;
    }
    std::unique_lock<std::mutex> lk(mu_in);
    if (stop && incoming.empty() && queued.empty()) break;
    if (incoming.empty() && queued.empty()) cv_work.wait_for(lk, std::chrono::milliseconds(50));
  }
  for (hipEvent_t e : ev_pool) (void)hipEventDestroy(e);
  ev_pool.clear();
  cv_done.notify_all();
}

static void server_free(mact_server* s) {
  if (!s) return;
  for (hipEvent_t e : s->ev_pool) (void)hipEventDestroy(e);
  s->ev_pool.clear();
  for (Slot& sl : s->slots) {
    if (sl.stream) (void)hipStreamDestroy(sl.stream);
    if (sl.ev_k0) (void)hipEventDestroy(sl.ev_k0);
    if (sl.ev_k1) (void)hipEventDestroy(sl.ev_k1);
    if (sl.d_buf) (void)hipFree(sl.d_buf);
    if (sl.h_buf) (void)hipHostFree(sl.h_buf);
  }
  if (s->copy_stream) (void)hipStreamDestroy(s->copy_stream);
  if (s->d2h_stream) (void)hipStreamDestroy(s->d2h_stream);
  if (s->d_arena) (void)hipFree(s->d_arena);
  if (s->d_coefs) (void)hipFree(s->d_coefs);
  delete s;
}

// The arena cleared once, one 16 x 16 8-bit CIELAB request through the copy
// stream, every slot and the output stream, synchronously, and a stock of
// events: first-use costs (page set-up, queue set-up, kernel loading, event
// creation) are paid here rather than by the first requests.
static mact_status warm_up(mact_server* s) {
  const int64_t w = 16, h = 16;
  const size_t in_b = (size_t)(w * h * 3), out_off = 4096, out_b = (size_t)(w * h * 12);
  char* hs = nullptr;
  if (hipHostMalloc((void**)&hs, out_b) != hipSuccess) return fail(MACT_E_NOMEM, "mact_server_create: warm-up buffer");
  std::memset(hs, 0, out_b);
  // touch the whole arena once, so that no request is the first to reach its pages
  mact_status st = hip_check(hipMemsetAsync(s->d_arena, 0, s->cfg.arena_bytes, s->copy_stream),
                             "mact_server_create: arena clear");
  if (st == MACT_OK)
    st = hip_check(hipMemcpyAsync(s->d_arena, hs, in_b, hipMemcpyHostToDevice, s->copy_stream),
                   "mact_server_create: warm-up copy");
  if (st == MACT_OK) st = hip_check(hipStreamSynchronize(s->copy_stream), "mact_server_create: warm-up copy");
  for (Slot& sl : s->slots) {
    if (st != MACT_OK) break;
    mact_image in{}, out{};
    in.data = s->d_arena;
    in.dtype = MACT_U8;
    in.layout = MACT_HWC;
    in.width = w;
    in.height = h;
    in.gamma = MACT_GAMMA_BT709;
    out.data = s->d_arena + out_off;
    out.dtype = MACT_F32;
    out.layout = MACT_HWC;
    out.width = w;
    out.height = h;
    std::vector<BDesc> descs;
    int d = 5;
    st = make_batch_descs(s->cfg.params[MACT_LAB], &in, &out, MACT_LAB, &descs, &d, "mact_server_create");
    if (st != MACT_OK) break;
    std::vector<uint32_t> ts;
    const uint32_t total = build_tiles(descs, (uint32_t)s->tune.tile, &ts);
    const size_t db = descs.size() * sizeof(BDesc), tb = ts.size() * sizeof(uint32_t);
    std::memcpy(sl.h_buf, descs.data(), db);
    std::memcpy(sl.h_buf + db, ts.data(), tb);
    st = hip_check(hipMemcpyAsync(sl.d_buf, sl.h_buf, db + tb, hipMemcpyHostToDevice, sl.stream), "mact_server_create: warm-up");
    if (st == MACT_OK)
      st = hip_check(launch_batch_kernel(reinterpret_cast<const BDesc*>(sl.d_buf), s->d_coefs,
                                         reinterpret_cast<const uint32_t*>(sl.d_buf + db), (int32_t)descs.size(), total,
                                         s->tune, s->deg, sl.stream),
                     "mact_server_create: warm-up launch");
    if (st == MACT_OK) st = hip_check(hipStreamSynchronize(sl.stream), "mact_server_create: warm-up");
  }
  if (st == MACT_OK)
    st = hip_check(hipMemcpyAsync(hs, s->d_arena + out_off, out_b, hipMemcpyDeviceToHost, s->d2h_stream),
                   "mact_server_create: warm-up copy");
  if (st == MACT_OK) st = hip_check(hipStreamSynchronize(s->d2h_stream), "mact_server_create: warm-up copy");
  (void)hipHostFree(hs);
  const int n_ev = 2 * std::min(s->cfg.max_batch, 256) * (int)s->slots.size();
  for (int i = 0; i < n_ev && st == MACT_OK; ++i) {
    hipEvent_t e = nullptr;
    st = hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "mact_server_create: event");
    if (st == MACT_OK) s->ev_pool.push_back(e);
  }
  return st;
}

extern "C" mact_status mact_server_create(const mact_server_config* cfg, mact_server** srv) {
  clear_error();
  if (!cfg || !srv) return fail(MACT_E_INVALID, "mact_server_create: NULL argument");
  *srv = nullptr;
  if (cfg->arena_bytes < (1u << 20)) return fail(MACT_E_INVALID, "mact_server_create: arena_bytes < 1 MiB");
  if (cfg->max_batch < 1 || cfg->max_batch > 4096) return fail(MACT_E_INVALID, "mact_server_create: max_batch %d", cfg->max_batch);
  if (cfg->compute_streams < 1 || cfg->compute_streams > 8)
    return fail(MACT_E_INVALID, "mact_server_create: compute_streams %d outside 1..8", cfg->compute_streams);
  if (cfg->max_queue < 1) return fail(MACT_E_INVALID, "mact_server_create: max_queue %d", cfg->max_queue);
  if (cfg->fail_request < 0) return fail(MACT_E_INVALID, "mact_server_create: fail_request %d < 0", cfg->fail_request);
  for (int x = 0; x < 4; ++x) {
    if (cfg->params[x].xform != x)
      return fail(MACT_E_INVALID, "mact_server_create: params[%d].xform must be %d", x, x);
    mact_status st = check_params(&cfg->params[x]);
    if (st != MACT_OK) return st;
  }
  mact_server* s = new (std::nothrow) mact_server();
  if (!s) return fail(MACT_E_NOMEM, "mact_server_create: host allocation");
  s->cfg = *cfg;
  s->device = current_device();
  KCoef k[4];
  for (int x = 0; x < 4; ++x) s->deg = std::max(s->deg, pack_coef(cfg->params[x], &k[x]));
  s->arena.reset(new Arena(cfg->arena_bytes));
  mact_status st = MACT_OK;
  if (hipMalloc(&s->d_arena, cfg->arena_bytes) != hipSuccess || hipMalloc(&s->d_coefs, sizeof k) != hipSuccess) {
    server_free(s);
    return fail(MACT_E_NOMEM, "mact_server_create: device allocation of %zu bytes", cfg->arena_bytes);
  }
  st = hip_check(hipMemcpy(s->d_coefs, k, sizeof k, hipMemcpyHostToDevice), "mact_server_create: coefficients");
  if (st == MACT_OK) st = hip_check(hipStreamCreateWithFlags(&s->copy_stream, hipStreamNonBlocking), "mact_server_create: stream");
  if (st == MACT_OK) st = hip_check(hipStreamCreateWithFlags(&s->d2h_stream, hipStreamNonBlocking), "mact_server_create: stream");
  s->slots.resize(cfg->compute_streams);
  // descriptors per slot: an image of 2^31 pixels or more splits, but requests are single images
  const size_t nd = (size_t)cfg->max_batch;
  for (Slot& sl : s->slots) {
    if (st != MACT_OK) break;
    st = hip_check(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking), "mact_server_create: stream");
    if (st == MACT_OK) st = hip_check(hipEventCreate(&sl.ev_k0), "mact_server_create: event");
    if (st == MACT_OK) st = hip_check(hipEventCreate(&sl.ev_k1), "mact_server_create: event");
    sl.buf_bytes = nd * sizeof(BDesc) + (nd + 1) * sizeof(uint32_t);
    if (st == MACT_OK && (hipMalloc((void**)&sl.d_buf, sl.buf_bytes) != hipSuccess ||
                          hipHostMalloc((void**)&sl.h_buf, sl.buf_bytes) != hipSuccess))
      st = fail(MACT_E_NOMEM, "mact_server_create: slot buffers");
  }
  if (st == MACT_OK) st = warm_up(s);
  if (st != MACT_OK) {
    server_free(s);
    return st;
  }
  s->th = std::thread([s] { s->loop(); });
  *srv = s;
  return MACT_OK;
}

extern "C" mact_status mact_server_submit(mact_server* s, const mact_request* r, int64_t* id) {
  clear_error();
  if (!s || !r || !id) return fail(MACT_E_INVALID, "mact_server_submit: NULL argument");
  if (!r->host_in || !r->host_out) return fail(MACT_E_INVALID, "mact_server_submit: NULL host buffer");
  if (r->in_dtype != MACT_U8 && r->in_dtype != MACT_U16 && r->in_dtype != MACT_F16 && r->in_dtype != MACT_F32)
    return fail(MACT_E_INVALID, "mact_server_submit: in_dtype %d", r->in_dtype);
  if (r->out_dtype != MACT_F32 && r->out_dtype != MACT_F16) return fail(MACT_E_INVALID, "mact_server_submit: out_dtype %d", r->out_dtype);
  if (r->xform < MACT_LAB || r->xform > MACT_LUV) return fail(MACT_E_INVALID, "mact_server_submit: xform %d", r->xform);
  if (r->gamma < MACT_GAMMA_BT709 || r->gamma > MACT_GAMMA_NONE) return fail(MACT_E_INVALID, "mact_server_submit: gamma %d", r->gamma);
  if (r->width <= 0 || r->height <= 0 || (uint64_t)r->width * (uint64_t)r->height >= (1ull << 31))
    return fail(MACT_E_INVALID, "mact_server_submit: size %lld x %lld", (long long)r->width, (long long)r->height);
  const size_t px = (size_t)r->width * (size_t)r->height;
  const size_t in_b = px * 3 * esize(r->in_dtype), out_b = px * 3 * esize(r->out_dtype);
  const size_t need = (in_b + kGranule - 1) / kGranule * kGranule + (out_b + kGranule - 1) / kGranule * kGranule;
  if (need > s->cfg.arena_bytes) return fail(MACT_E_INVALID, "mact_server_submit: request needs %zu bytes, arena has %zu", need, s->cfg.arena_bytes);
  std::unique_ptr<Req> q(new (std::nothrow) Req());
  if (!q) return fail(MACT_E_NOMEM, "mact_server_submit: host allocation");
  q->r = *r;
  q->in_bytes = in_b;
  q->out_bytes = out_b;
  {
    std::lock_guard<std::mutex> g(s->mu_in);
    if (s->stop) return fail(MACT_E_INVALID, "mact_server_submit: server is stopping");
    if (s->waiting.load() >= s->cfg.max_queue) {
      ++s->rejected;
      return fail(MACT_E_BUSY, "mact_server_submit: %d requests already waiting", s->cfg.max_queue);
    }
    q->id = s->next_id++;
    q->t_submit = Clock::now();
    *id = q->id;
    s->incoming.push_back(q.get());
    s->all[q->id] = std::move(q);
    ++s->submitted;
    s->waiting.fetch_add(1);
  }
  s->cv_work.notify_one();
  return MACT_OK;
}

// The request with handle `id`, or null.  Requests live until the server is destroyed.
static Req* find_req(mact_server* s, int64_t id) {
  std::lock_guard<std::mutex> g(s->mu_in);
  auto it = s->all.find(id);
  return it == s->all.end() ? nullptr : it->second.get();
}

extern "C" mact_status mact_server_poll(mact_server* s, int64_t id, int32_t* done) {
  clear_error();
  if (!s || !done) return fail(MACT_E_INVALID, "mact_server_poll: NULL argument");
  Req* q = find_req(s, id);
  if (!q) return fail(MACT_E_INVALID, "mact_server_poll: unknown request %lld", (long long)id);
  *done = q->done.load() ? 1 : 0;
  if (*done && q->status != MACT_OK) return fail(q->status, "mact_server_poll: %s", q->err);
  return MACT_OK;
}

extern "C" mact_status mact_server_wait(mact_server* s, int64_t id, int32_t timeout_ms) {
  clear_error();
  if (!s) return fail(MACT_E_INVALID, "mact_server_wait: NULL server");
  Req* q = find_req(s, id);
  if (!q) return fail(MACT_E_INVALID, "mact_server_wait: unknown request %lld", (long long)id);
  std::unique_lock<std::mutex> lk(s->mu_done);
  if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [q] { return q->done.load(); }))
    return fail(MACT_E_BUSY, "mact_server_wait: request %lld not done after %d ms", (long long)id, timeout_ms);
  if (q->status != MACT_OK) return fail(q->status, "mact_server_wait: %s", q->err);
  return MACT_OK;
}

extern "C" mact_status mact_server_cancel(mact_server* s, int64_t id) {
  clear_error();
  if (!s) return fail(MACT_E_INVALID, "mact_server_cancel: NULL server");
  Req* q = find_req(s, id);
  if (!q) return fail(MACT_E_INVALID, "mact_server_cancel: unknown request %lld", (long long)id);
  int expect = 0;
  if (!q->phase.compare_exchange_strong(expect, 2))
    return fail(MACT_E_BUSY, "mact_server_cancel: request %lld already admitted", (long long)id);
  // the request is ours: complete it; the scheduler drops it from its queue without touching it
  std::snprintf(q->err, sizeof q->err, "request %lld cancelled before admission", (long long)id);
  q->status = MACT_E_CANCELLED;
  q->t_done = Clock::now();
  {
    std::lock_guard<std::mutex> g(s->mu_done);
    q->done.store(true);
  }
  {
    std::lock_guard<std::mutex> g(s->mu_stats);
    ++s->cancelled;
  }
  s->cv_done.notify_all();
  return MACT_OK;
}

extern "C" mact_status mact_server_latency(mact_server* s, int64_t id, double* ms) {
  clear_error();
  if (!s || !ms) return fail(MACT_E_INVALID, "mact_server_latency: NULL argument");
  Req* q = find_req(s, id);
  if (!q) return fail(MACT_E_INVALID, "mact_server_latency: unknown request %lld", (long long)id);
  if (!q->done.load()) return fail(MACT_E_BUSY, "mact_server_latency: request %lld not done", (long long)id);
  if (q->status != MACT_OK) return fail(q->status, "mact_server_latency: %s", q->err);
  *ms = std::chrono::duration<double, std::milli>(q->t_done - q->t_submit).count();
  return MACT_OK;
}

extern "C" mact_status mact_server_stats_get(mact_server* s, mact_server_stats* st) {
  clear_error();
  if (!s || !st) return fail(MACT_E_INVALID, "mact_server_stats_get: NULL argument");
  std::memset(st, 0, sizeof *st);
  {
    std::lock_guard<std::mutex> g(s->mu_in);
    st->submitted = s->submitted;
    st->rejected = s->rejected;
  }
  std::lock_guard<std::mutex> g(s->mu_stats);
  st->completed = s->completed;
  st->failed = s->failed;
  st->cancelled = s->cancelled;
  st->batches = s->batches;
  st->mean_batch = s->batches ? (double)s->batched_reqs / s->batches : 0.0;
  st->device_busy_ms = s->busy_ms;
  if (!s->lat_ms.empty()) {
    std::vector<double> v = s->lat_ms;
    std::sort(v.begin(), v.end());
    auto q = [&v](double f) { return v[std::min(v.size() - 1, (size_t)(f * (v.size() - 1) + 0.5))]; };
    st->p50_ms = q(0.50);
    st->p99_ms = q(0.99);
    double sum = 0.0;
    for (double x : v) sum += x;
    st->mean_ms = sum / v.size();
  }
  return MACT_OK;
}

extern "C" mact_status mact_server_destroy(mact_server* s) {
  clear_error();
  if (!s) return MACT_OK;
  {
    std::lock_guard<std::mutex> g(s->mu_in);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  for (Slot& sl : s->slots)
    if (sl.stream) (void)hipStreamSynchronize(sl.stream);
  if (s->copy_stream) (void)hipStreamSynchronize(s->copy_stream);
  if (s->d2h_stream) (void)hipStreamSynchronize(s->d2h_stream);
  server_free(s);
  return MACT_OK;
}
