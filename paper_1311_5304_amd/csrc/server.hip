// Serving loop with continuous batching (host code).
//
// A server thread owns three streams and one device arena.  Requests are
// admitted in submission order once they have arrived and their coefficient,
// quant-table and RGB buffers fit in the arena; their host->device copies
// start at once.  Whenever a batch-table slot is free, everything admitted
// since the last launch becomes one persistent batch launch (the segment
// queue of batch.hip); its RGB8 results go device->host on a third stream
// and the arena space returns when that copy completes (requests whose RGB
// goes to the caller's device memory are written there by the kernel and
// copy nothing back).  In sync mode the same thread decodes one request at
// a time and waits for each.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "mjd_internal.h"

namespace mjd {
namespace serve {

using Clock = std::chrono::steady_clock;
constexpr uint64_t kAlign = 256;
constexpr uint64_t kQtBytes = 512;  // uint16[4][64], a multiple of kAlign

static uint64_t round_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

// First-fit allocator over [0, size) with coalescing free ranges.
class Arena {
 public:
  void reset(uint64_t size) {
    free_.clear();
    free_[0] = size;
  }
  bool alloc(uint64_t bytes, uint64_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second >= bytes) {
        *off = it->first;
        const uint64_t rest = it->second - bytes;
        const uint64_t at = it->first + bytes;
        free_.erase(it);
        if (rest) free_[at] = rest;
        return true;
      }
    }
    return false;
  }
  void release(uint64_t off, uint64_t bytes) {
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

 private:
  std::map<uint64_t, uint64_t> free_;
};

struct Request {
  mjd_request r;
  mjd_geometry g;
  uint64_t coef_bytes = 0, rgb_pitch = 0, rgb_bytes = 0, total = 0;
  uint64_t off = 0;  // arena offset: coefficients, then quant tables, then RGB
  mjd_request_times t{};
  double pred_s = 0.0;  // predicted GPU seconds (with a model)
  bool done = false;
};

// Device tables of one batch launch and the requests riding in it.
struct TableSlot {
  ImageView* d_views = nullptr;
  BatchItem* d_items = nullptr;
  unsigned* d_counters = nullptr;
  uint8_t* h_stage = nullptr;  // pinned: views, then items
  size_t view_cap = 0, item_cap = 0;
  hipEvent_t copied = nullptr;  // host->device copies of its requests done
  hipEvent_t done = nullptr;    // its last device->host copy done
  bool busy = false;
  uint64_t seq = 0;  // launch order
  std::vector<uint64_t> reqs;
};

}  // namespace serve
}  // namespace mjd

struct mjd_server {
  mjd_ctx* ctx = nullptr;
  int device = 0;
  mjd_server_config cfg{};
  mjd_model model{};
  bool has_model = false;
  mjd::serve::Clock::time_point t0;
  uint8_t* d_arena = nullptr;
  mjd::serve::Arena arena;
  hipStream_t s_h2d = nullptr, s_kernel = nullptr, s_d2h = nullptr;
  std::vector<mjd::serve::TableSlot> slots;
  uint64_t launches = 0;

  std::mutex mu;
  std::condition_variable cv_work;  // the server thread waits for submissions
  std::condition_variable cv_done;  // callers wait for completions
  std::deque<mjd::serve::Request> reqs;  // by id; deque keeps references stable
  uint64_t next_admit = 0;               // first id not yet admitted
  uint64_t n_done = 0;
  uint64_t last_arrival = 0;
  bool stop = false;
  std::thread th;

  uint64_t now_ns() const {
    return static_cast<uint64_t>(
        std::chrono::duration_cast<std::chrono::nanoseconds>(mjd::serve::Clock::now() - t0).count());
  }
};

namespace mjd {
namespace serve {

static void finish(mjd_server* s, uint64_t id, int status, uint64_t now) {
  Request& q = s->reqs[id];
  q.t.done_ns = now;
  q.t.status = status;
  q.done = true;
  s->n_done += 1;
}

// Grow a table slot to hold a plan (only while the slot is idle).
static hipError_t fit_slot(TableSlot& t, size_t views, size_t items) {
  if (views <= t.view_cap && items <= t.item_cap) return hipSuccess;
  const size_t vc = std::max(views, t.view_cap), ic = std::max(items, 2 * t.item_cap);
  if (t.h_stage) (void)hipHostFree(t.h_stage);
  if (t.d_views) (void)hipFree(t.d_views);
  if (t.d_items) (void)hipFree(t.d_items);
  t.h_stage = nullptr;
  t.d_views = nullptr;
  t.d_items = nullptr;
  t.view_cap = t.item_cap = 0;
  hipError_t e;
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&t.h_stage), vc * sizeof(ImageView) + ic * sizeof(BatchItem),
                         hipHostMallocDefault)) != hipSuccess)
    return e;
  if ((e = hipMalloc(&t.d_views, vc * sizeof(ImageView))) != hipSuccess) return e;
  if ((e = hipMalloc(&t.d_items, ic * sizeof(BatchItem))) != hipSuccess) return e;
  t.view_cap = vc;
  t.item_cap = ic;
  return hipSuccess;
}

// Enqueue host->device copies of an admitted request.
static hipError_t copy_in(mjd_server* s, Request& q) {
  uint8_t* base = s->d_arena + q.off;
  hipError_t e = hipMemcpyAsync(base, q.r.h_coef, q.coef_bytes, hipMemcpyHostToDevice, s->s_h2d);
  if (e != hipSuccess) return e;
  return hipMemcpyAsync(base + q.coef_bytes, q.r.h_qt, kQtBytes, hipMemcpyHostToDevice, s->s_h2d);
}

static hipError_t copy_out(mjd_server* s, Request& q) {
  if (q.r.d_rgb) return hipSuccess;  // the kernel wrote the caller's device rows
  const uint8_t* rgb = s->d_arena + q.off + q.coef_bytes + kQtBytes;
  // rows without padding on both sides: one linear copy (with padding, the
  // host bytes beyond 3 * width must stay untouched)
  if (q.r.pitch == 3ull * q.r.frame.width && q.rgb_pitch == q.r.pitch)
    return hipMemcpyAsync(q.r.h_rgb, rgb, q.rgb_pitch * q.r.frame.height, hipMemcpyDeviceToHost, s->s_d2h);
  return hipMemcpy2DAsync(q.r.h_rgb, q.r.pitch, rgb, q.rgb_pitch, 3ull * q.r.frame.width, q.r.frame.height,
                          hipMemcpyDeviceToHost, s->s_d2h);
}

static mjd_job job_of(mjd_server* s, const Request& q) {
  mjd_job j{};
  j.frame = q.r.frame;
  uint8_t* base = s->d_arena + q.off;
  j.d_coef = reinterpret_cast<const int16_t*>(base);
  j.d_qt = reinterpret_cast<const uint16_t*>(base + q.coef_bytes);
  j.d_rgb = q.r.d_rgb ? q.r.d_rgb : base + q.coef_bytes + kQtBytes;
  j.pitch = q.r.d_rgb ? q.r.pitch : q.rgb_pitch;
  return j;
}

// Launch everything in `forming` as one batch in table slot `t`.
static int launch(mjd_server* s, TableSlot& t, std::vector<uint64_t>& forming, uint64_t now) {
  std::vector<mjd_job> jobs;
  jobs.reserve(forming.size());
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (uint64_t id : forming) jobs.push_back(job_of(s, s->reqs[id]));
  }
  BatchPlan plan;
  int rc = batch_plan(s->ctx, jobs.data(), jobs.size(), static_cast<int>(s->cfg.upsample), &plan);
  if (rc != MJD_OK) return rc;
  hipError_t e = fit_slot(t, plan.views.size(), plan.items.size());
  if (e != hipSuccess) return fail(MJD_ENOMEM, "batch tables: %s", hipGetErrorString(e));
  const size_t vb = plan.views.size() * sizeof(ImageView), ib = plan.items.size() * sizeof(BatchItem);
  memcpy(t.h_stage, plan.views.data(), vb);
  memcpy(t.h_stage + t.view_cap * sizeof(ImageView), plan.items.data(), ib);
  if ((e = hipEventRecord(t.copied, s->s_h2d)) != hipSuccess ||
      (e = hipStreamWaitEvent(s->s_kernel, t.copied, 0)) != hipSuccess ||
      (e = hipMemcpyAsync(t.d_views, t.h_stage, vb, hipMemcpyHostToDevice, s->s_kernel)) != hipSuccess ||
      (e = hipMemcpyAsync(t.d_items, t.h_stage + t.view_cap * sizeof(ImageView), ib, hipMemcpyHostToDevice,
                          s->s_kernel)) != hipSuccess ||
      (e = batch_enqueue(t.d_views, t.d_items, static_cast<int>(plan.items.size()), t.d_counters, plan.grid,
                         s->s_kernel)) != hipSuccess ||
      (e = hipEventRecord(t.done, s->s_kernel)) != hipSuccess ||
      (e = hipStreamWaitEvent(s->s_d2h, t.done, 0)) != hipSuccess)
    return fail(MJD_EDEVICE, "batch launch: %s", hipGetErrorString(e));
  {
    std::lock_guard<std::mutex> g(s->mu);
    for (uint64_t id : forming) {
      Request& q = s->reqs[id];
      if ((e = copy_out(s, q)) != hipSuccess) return fail(MJD_EDEVICE, "result copy: %s", hipGetErrorString(e));
      q.t.launch_ns = now;
      q.t.batch = static_cast<uint32_t>(forming.size());
    }
  }
  if ((e = hipEventRecord(t.done, s->s_d2h)) != hipSuccess)
    return fail(MJD_EDEVICE, "hipEventRecord: %s", hipGetErrorString(e));
  t.reqs.swap(forming);
  forming.clear();
  t.busy = true;
  t.seq = s->launches++;
  return MJD_OK;
}

static void run_continuous(mjd_server* s) {
  std::vector<uint64_t> forming;
  double forming_s = 0.0;  // predicted GPU seconds of the forming batch
  const bool capped = s->has_model && s->cfg.max_batch_s > 0.0;
  for (;;) {
    bool progressed = false;
    if (forming.empty()) forming_s = 0.0;
    const uint64_t now = s->now_ns();
    // retire finished batches, oldest first
    for (;;) {
      TableSlot* oldest = nullptr;
      for (auto& t : s->slots)
        if (t.busy && (!oldest || t.seq < oldest->seq)) oldest = &t;
      if (!oldest) break;
      const hipError_t q = hipEventQuery(oldest->done);
      if (q == hipErrorNotReady) break;
      const int st = q == hipSuccess ? MJD_OK : MJD_EDEVICE;
      std::lock_guard<std::mutex> g(s->mu);
      for (uint64_t id : oldest->reqs) {
        Request& r = s->reqs[id];
        s->arena.release(r.off, r.total);
        finish(s, id, st, now);
      }
      oldest->reqs.clear();
      oldest->busy = false;
      s->cv_done.notify_all();
      progressed = true;
    }
    // admit arrived requests in order while their buffers fit
    uint64_t next_arrival = UINT64_MAX;
    bool pending = false;
    {
      std::lock_guard<std::mutex> g(s->mu);
      while (s->next_admit < s->reqs.size() && forming.size() < s->cfg.max_batch) {
        Request& q = s->reqs[s->next_admit];
        if (q.r.arrival_ns > now) {
          next_arrival = q.r.arrival_ns;
          break;
        }
        // batch sizing by the performance model: the batch closes once its
        // predicted GPU time would pass the cap
        if (capped && !forming.empty() && forming_s + q.pred_s > s->cfg.max_batch_s) break;
        if (!s->arena.alloc(q.total, &q.off)) break;
        const hipError_t e = copy_in(s, q);
        q.t.admit_ns = now;
        if (e != hipSuccess) {
          s->arena.release(q.off, q.total);
          finish(s, s->next_admit, MJD_EDEVICE, now);
          s->cv_done.notify_all();
        } else {
          forming.push_back(s->next_admit);
          forming_s += q.pred_s;
        }
        ++s->next_admit;
        progressed = true;
      }
      pending = s->next_admit < s->reqs.size();
    }
    // launch what is admitted as soon as a table slot is free
    if (!forming.empty()) {
      for (auto& t : s->slots) {
        if (t.busy) continue;
        const int rc = launch(s, t, forming, now);
        if (rc != MJD_OK) {
          // nothing of this batch may still touch the arena when it is reused
          (void)hipStreamSynchronize(s->s_kernel);
          (void)hipStreamSynchronize(s->s_d2h);
          std::lock_guard<std::mutex> g(s->mu);
          for (uint64_t id : forming) {
            Request& r = s->reqs[id];
            s->arena.release(r.off, r.total);
            finish(s, id, rc, s->now_ns());
          }
          forming.clear();
          s->cv_done.notify_all();
        }
        progressed = true;
        break;
      }
    }
    if (progressed) continue;
    bool busy = false;
    for (auto& t : s->slots) busy |= t.busy;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->stop && !busy && forming.empty() && s->next_admit >= s->reqs.size()) return;
    if (busy) {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));  // poll the device
    } else if (pending && next_arrival != UINT64_MAX) {
      s->cv_work.wait_until(lk, s->t0 + std::chrono::nanoseconds(next_arrival));
    } else if (!pending) {
      s->cv_work.wait(lk, [&] { return s->stop || s->next_admit < s->reqs.size(); });
    } else {
      lk.unlock();
      std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
  }
}

static void run_sync(mjd_server* s) {
  for (;;) {
    uint64_t id;
    Request* qp;
    {
      std::unique_lock<std::mutex> lk(s->mu);
      s->cv_work.wait(lk, [&] { return s->stop || s->next_admit < s->reqs.size(); });
      if (s->next_admit >= s->reqs.size()) return;  // stopped, nothing left
      id = s->next_admit;
      // The element is looked up under the lock: a concurrent submit may
      // grow the deque's map.  References to its elements stay valid across
      // push_back, so q may be used after the lock is released.
      qp = &s->reqs[id];
      const uint64_t arr = qp->r.arrival_ns;
      while (s->now_ns() < arr) s->cv_work.wait_until(lk, s->t0 + std::chrono::nanoseconds(arr));
      ++s->next_admit;
    }
    Request& q = *qp;
    q.off = 0;                 // alone in the arena
    q.t.admit_ns = s->now_ns();
    hipError_t e = copy_in(s, q);
    const mjd_job j = job_of(s, q);
    int rc = MJD_OK;
    if (e == hipSuccess) e = hipStreamSynchronize(s->s_h2d);
    q.t.launch_ns = s->now_ns();
    q.t.batch = 1;
    if (e == hipSuccess) {
      rc = mjd_decode(s->ctx, &j.frame, j.d_coef, j.d_qt, static_cast<int>(s->cfg.upsample), j.d_rgb, j.pitch, 0,
                      q.g.mcus_y, s->s_kernel);
      if (rc == MJD_OK) e = hipStreamSynchronize(s->s_kernel);
      if (rc == MJD_OK && e == hipSuccess) e = copy_out(s, q);
      if (rc == MJD_OK && e == hipSuccess) e = hipStreamSynchronize(s->s_d2h);
    }
    std::lock_guard<std::mutex> g(s->mu);
    finish(s, id, rc != MJD_OK ? rc : (e == hipSuccess ? MJD_OK : MJD_EDEVICE), s->now_ns());
    s->cv_done.notify_all();
  }
}

static void release_all(mjd_server* s) {
  for (auto& t : s->slots) {
    if (t.h_stage) (void)hipHostFree(t.h_stage);
    if (t.d_views) (void)hipFree(t.d_views);
    if (t.d_items) (void)hipFree(t.d_items);
    if (t.d_counters) (void)hipFree(t.d_counters);
    if (t.copied) (void)hipEventDestroy(t.copied);
    if (t.done) (void)hipEventDestroy(t.done);
  }
  s->slots.clear();
  if (s->d_arena) (void)hipFree(s->d_arena);
  s->d_arena = nullptr;
  if (s->s_h2d) (void)hipStreamDestroy(s->s_h2d);
  if (s->s_kernel) (void)hipStreamDestroy(s->s_kernel);
  if (s->s_d2h) (void)hipStreamDestroy(s->s_d2h);
}

static int create(mjd_server* s) {
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&s->s_h2d, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&s->s_kernel, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&s->s_d2h, hipStreamNonBlocking)) != hipSuccess)
    return fail(MJD_EDEVICE, "hipStreamCreateWithFlags: %s", hipGetErrorString(e));
  if ((e = hipMalloc(&s->d_arena, s->cfg.budget_bytes)) != hipSuccess)
    return fail(MJD_ENOMEM, "device arena of %llu bytes: %s", static_cast<unsigned long long>(s->cfg.budget_bytes),
                hipGetErrorString(e));
  s->arena.reset(s->cfg.budget_bytes);
  s->slots.resize(s->cfg.mode == MJD_SERVE_SYNC ? 0 : s->cfg.max_inflight);
  for (auto& t : s->slots) {
    if ((e = hipMalloc(&t.d_counters, 2 * sizeof(unsigned))) != hipSuccess ||
        (e = hipMemset(t.d_counters, 0, 2 * sizeof(unsigned))) != hipSuccess ||
        (e = hipEventCreateWithFlags(&t.copied, hipEventDisableTiming)) != hipSuccess ||
        (e = hipEventCreateWithFlags(&t.done, hipEventDisableTiming)) != hipSuccess ||
        (e = fit_slot(t, 64, 4096)) != hipSuccess)
      return fail(MJD_ENOMEM, "batch table slot: %s", hipGetErrorString(e));
  }
  return MJD_OK;
}

}  // namespace serve
}  // namespace mjd

extern "C" {

int mjd_server_create(mjd_ctx* ctx, const mjd_server_config* cfg, mjd_server** out) {
  if (!ctx || !cfg || !out) return mjd::fail(MJD_EINVAL, "null context, config or out-pointer");
  *out = nullptr;
  if (cfg->upsample != MJD_UPSAMPLE_SIMPLE && cfg->upsample != MJD_UPSAMPLE_FANCY)
    return mjd::fail(MJD_EINVAL, "upsample mode %u unknown", cfg->upsample);
  if (cfg->mode != MJD_SERVE_CONTINUOUS && cfg->mode != MJD_SERVE_SYNC)
    return mjd::fail(MJD_EINVAL, "serving mode %u unknown", cfg->mode);
  if (cfg->max_batch < 1 || cfg->max_batch > 4096) return mjd::fail(MJD_EINVAL, "max_batch outside 1..4096");
  if (cfg->max_inflight < 1 || cfg->max_inflight > 8) return mjd::fail(MJD_EINVAL, "max_inflight outside 1..8");
  if (cfg->budget_bytes < (1u << 20)) return mjd::fail(MJD_EINVAL, "budget below 1 MiB");
  if (!(cfg->max_batch_s >= 0.0) || cfg->max_batch_s > 1e6)
    return mjd::fail(MJD_EINVAL, "max_batch_s must be a non-negative number of seconds");
  mjd_server* s = new (std::nothrow) mjd_server;
  if (!s) return mjd::fail(MJD_ENOMEM, "server allocation failed");
  s->ctx = ctx;
  s->device = ctx->device;
  s->cfg = *cfg;
  s->cfg.budget_bytes = cfg->budget_bytes / mjd::serve::kAlign * mjd::serve::kAlign;
  if (cfg->model) {
    s->model = *cfg->model;
    s->has_model = true;
  }
  s->cfg.model = nullptr;  // the server keeps its own copy
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != s->device && hipSetDevice(s->device) != hipSuccess) {
    delete s;
    return mjd::fail(MJD_EDEVICE, "hipSetDevice(%d) failed", s->device);
  }
  int rc = mjd::serve::create(s);
  if (rc != MJD_OK) {
    mjd::serve::release_all(s);
    if (cur != s->device) (void)hipSetDevice(cur);
    delete s;
    return rc;
  }
  if (cur != s->device) (void)hipSetDevice(cur);
  s->t0 = mjd::serve::Clock::now();
  s->th = std::thread([s] {
    (void)hipSetDevice(s->device);
    if (s->cfg.mode == MJD_SERVE_SYNC) mjd::serve::run_sync(s);
    else mjd::serve::run_continuous(s);
  });
  *out = s;
  return MJD_OK;
}

uint64_t mjd_server_now_ns(const mjd_server* srv) { return srv ? srv->now_ns() : 0; }

int mjd_server_submit(mjd_server* srv, const mjd_request* req, uint64_t* id) {
  if (!srv || !req || !id) return mjd::fail(MJD_EINVAL, "null server, request or id pointer");
  mjd::serve::Request q;
  q.r = *req;
  int rc = mjd::frame_geometry(&req->frame, &q.g);
  if (rc != MJD_OK) return rc;
  if (!req->h_coef || !req->h_qt) return mjd::fail(MJD_EINVAL, "null request buffer");
  if ((req->h_rgb == nullptr) == (req->d_rgb == nullptr))
    return mjd::fail(MJD_EINVAL, "exactly one of h_rgb and d_rgb must be set");
  if (req->pitch < 3ull * req->frame.width) return mjd::fail(MJD_EINVAL, "pitch below 3*width");
  using mjd::serve::kAlign;
  using mjd::serve::round_up;
  q.coef_bytes = round_up(q.g.n_blocks * 128, kAlign);
  if (req->d_rgb) {
    // the kernel writes the caller's rows: no RGB buffer in the arena
    if (req->pitch >= (1ull << 24)) return mjd::fail(MJD_EINVAL, "row too wide");
    q.rgb_pitch = req->pitch;
    q.rgb_bytes = 0;
  } else {
    // device rows match dense host rows, so results come back in one linear
    // copy; otherwise they are padded to 16 bytes for the kernel's wide stores
    q.rgb_pitch = req->pitch == 3ull * req->frame.width ? req->pitch : round_up(3ull * req->frame.width, 16);
    if (q.rgb_pitch >= (1ull << 24)) return mjd::fail(MJD_EINVAL, "row too wide");
    q.rgb_bytes = round_up(q.rgb_pitch * req->frame.height, kAlign);
  }
  q.total = q.coef_bytes + mjd::serve::kQtBytes + q.rgb_bytes;
  if (srv->has_model) {
    mjd_prediction p;
    if (mjd_model_predict(&srv->model, req->frame.width, req->frame.height, 0, &p) == MJD_OK &&
        p.p_gpu > 0.0)
      q.pred_s = p.p_gpu;
  }
  if (q.total > srv->cfg.budget_bytes)
    return mjd::fail(MJD_EBUDGET, "request needs %llu device bytes, budget is %llu",
                     static_cast<unsigned long long>(q.total), static_cast<unsigned long long>(srv->cfg.budget_bytes));
  {
    std::lock_guard<std::mutex> g(srv->mu);
    if (srv->stop) return mjd::fail(MJD_EINVAL, "server is stopping");
    if (req->arrival_ns < srv->last_arrival) return mjd::fail(MJD_EINVAL, "arrival times must not decrease");
    srv->last_arrival = req->arrival_ns;
    q.t.arrival_ns = req->arrival_ns;
    *id = srv->reqs.size();
    srv->reqs.push_back(q);
  }
  srv->cv_work.notify_all();
  return MJD_OK;
}

int mjd_server_wait(mjd_server* srv, uint64_t id, mjd_request_times* times) {
  if (!srv) return mjd::fail(MJD_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(srv->mu);
  if (id >= srv->reqs.size()) return mjd::fail(MJD_EINVAL, "no request %llu", static_cast<unsigned long long>(id));
  srv->cv_done.wait(lk, [&] { return srv->reqs[id].done; });
  const mjd::serve::Request& q = srv->reqs[id];
  if (times) *times = q.t;
  if (q.t.status != MJD_OK) return mjd::fail(q.t.status, "request %llu failed", static_cast<unsigned long long>(id));
  return MJD_OK;
}

int mjd_server_drain(mjd_server* srv) {
  if (!srv) return mjd::fail(MJD_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(srv->mu);
  srv->cv_done.wait(lk, [&] { return srv->n_done == srv->reqs.size(); });
  return MJD_OK;
}

void mjd_server_destroy(mjd_server* srv) {
  if (!srv) return;
  {
    std::lock_guard<std::mutex> g(srv->mu);
    srv->stop = true;
  }
  srv->cv_work.notify_all();
  if (srv->th.joinable()) srv->th.join();
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != srv->device) (void)hipSetDevice(srv->device);
  (void)hipDeviceSynchronize();
  mjd::serve::release_all(srv);
  if (cur != srv->device) (void)hipSetDevice(cur);
  delete srv;
}

}  // extern "C"
