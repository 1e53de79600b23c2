// Pipelined end-to-end decode (paper Sec. 4.5, Fig. 6): host workers
// Huffman-decode the restart intervals of MCU-row bands into pinned buffers;
// each finished band is copied host->device, decoded by the fused kernel and
// copied back, on three HIP streams, while the workers continue with the
// next bands and images.
//
// Threads: the caller's thread orchestrates (parses headers, hands finished
// bands to the GPU in order, recycles slots) and runs decode tasks itself
// when it has nothing else to do; n_threads workers only run decode tasks.
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "host_jpeg.h"
#include "mjd_common.h"

namespace mjd {
namespace pipe {

using Clock = std::chrono::steady_clock;
constexpr int kMaxBands = 64;       // bands per image (timing events are preallocated for these)
constexpr int kEventsPerBand = 6;   // h2d start/end, kernel start/end, d2h start/end

struct Band {
  uint32_t r0 = 0, r1 = 0;  // MCU rows
  uint32_t s0 = 0, s1 = 0;  // restart intervals that cover them
  std::atomic<uint32_t> remaining{0};
};

struct Image {
  size_t index = 0;
  const uint8_t* jpg = nullptr;
  size_t len = 0;
  mjd_scan scan;
  uint16_t qt[4][64];
  std::vector<uint64_t> offsets;
  host::ScanLayout L;
  mjd_geometry g;
  Band bands[kMaxBands];
  int n_bands = 0;
  int slot = 0;
  uint8_t* h_rgb = nullptr;
  size_t pitch = 0;
  std::atomic<int> status{MJD_OK};
  std::mutex err_mu;
  std::string err;
};

struct Slot {
  int16_t* h_coef = nullptr;  // pinned
  uint16_t* h_qt = nullptr;   // pinned, 4 x 64
  int16_t* d_coef = nullptr;
  uint16_t* d_qt = nullptr;
  uint8_t* d_rgb = nullptr;
  hipEvent_t free_ev = nullptr;  // recorded after the image's last device->host copy
  bool busy = false;             // free_ev recorded, completion not yet observed
  Image* img = nullptr;
  int timed_bands = 0;           // bands whose timing events were recorded
  hipEvent_t tev[kMaxBands * kEventsPerBand] = {};
  std::unique_ptr<host::ScanTables> tables{new host::ScanTables};
};

struct Task {
  Image* img;
  const Slot* slot;
  uint32_t band;
  uint32_t interval;
};

}  // namespace pipe
}  // namespace mjd

struct mjd_pipeline {
  mjd_ctx* ctx = nullptr;
  int device = 0;
  mjd_pipeline_config cfg{};
  std::vector<mjd::pipe::Slot> slots;
  hipStream_t s_h2d = nullptr, s_kernel = nullptr, s_d2h = nullptr;
  // task queue
  std::mutex mu;
  std::condition_variable cv_task;  // workers wait for tasks
  std::condition_variable cv_done;  // the orchestrator waits for band completions
  std::deque<mjd::pipe::Task> queue;
  bool stop = false;
  std::vector<std::thread> workers;
  std::atomic<int64_t> busy_ns{0};

  bool try_pop(mjd::pipe::Task* t) {
    std::lock_guard<std::mutex> g(mu);
    if (queue.empty()) return false;
    *t = queue.front();
    queue.pop_front();
    return true;
  }

  void run_task(const mjd::pipe::Task& t) {
    using namespace mjd::pipe;
    Image* im = t.img;
    Band& b = im->bands[t.band];
    if (im->status.load(std::memory_order_relaxed) == MJD_OK) {
      const auto t0 = Clock::now();
      std::string err;
      const uint64_t mx = im->L.mcus_x;
      const int rc = mjd::host::decode_interval(im->jpg, &im->scan, im->L, *t.slot->tables, im->offsets.data(),
                                                t.interval, b.r0 * mx, b.r1 * mx, t.slot->h_coef, &err);
      busy_ns.fetch_add(std::chrono::duration_cast<std::chrono::nanoseconds>(Clock::now() - t0).count(),
                        std::memory_order_relaxed);
      if (rc != MJD_OK) {
        std::lock_guard<std::mutex> g(im->err_mu);
        if (im->status.load() == MJD_OK) {
          im->err = err;
          im->status.store(rc);
        }
      }
    }
    if (b.remaining.fetch_sub(1, std::memory_order_acq_rel) == 1) {
      std::lock_guard<std::mutex> g(mu);  // pairs with the orchestrator's predicate check
      cv_done.notify_all();
    }
  }

  void worker_loop() {
    for (;;) {
      mjd::pipe::Task t;
      {
        std::unique_lock<std::mutex> lk(mu);
        cv_task.wait(lk, [&] { return stop || !queue.empty(); });
        if (queue.empty()) return;  // stop requested and nothing left
        t = queue.front();
        queue.pop_front();
      }
      run_task(t);
    }
  }
};

namespace mjd {
namespace pipe {

static int hip_fail(hipError_t e, const char* what) {
  return fail(MJD_EDEVICE, "%s failed: %s", what, hipGetErrorString(e));
}

static void release(mjd_pipeline* p) {
  {
    std::lock_guard<std::mutex> g(p->mu);
    p->stop = true;
  }
  p->cv_task.notify_all();
  for (auto& t : p->workers) t.join();
  p->workers.clear();
  if (p->s_d2h) (void)hipStreamSynchronize(p->s_d2h);
  if (p->s_kernel) (void)hipStreamSynchronize(p->s_kernel);
  if (p->s_h2d) (void)hipStreamSynchronize(p->s_h2d);
  for (auto& s : p->slots) {
    if (s.h_coef) (void)hipHostFree(s.h_coef);
    if (s.h_qt) (void)hipHostFree(s.h_qt);
    if (s.d_coef) (void)hipFree(s.d_coef);
    if (s.d_qt) (void)hipFree(s.d_qt);
    if (s.d_rgb) (void)hipFree(s.d_rgb);
    if (s.free_ev) (void)hipEventDestroy(s.free_ev);
    for (auto& e : s.tev)
      if (e) (void)hipEventDestroy(e);
  }
  p->slots.clear();
  if (p->s_h2d) (void)hipStreamDestroy(p->s_h2d);
  if (p->s_kernel) (void)hipStreamDestroy(p->s_kernel);
  if (p->s_d2h) (void)hipStreamDestroy(p->s_d2h);
}

static int create(mjd_pipeline* p) {
  const mjd_pipeline_config& c = p->cfg;
  hipError_t e;
  if ((e = hipStreamCreateWithFlags(&p->s_h2d, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&p->s_kernel, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&p->s_d2h, hipStreamNonBlocking)) != hipSuccess)
    return hip_fail(e, "hipStreamCreateWithFlags");
  p->slots.resize(c.n_slots);
  for (auto& s : p->slots) {
    if ((e = hipHostMalloc(reinterpret_cast<void**>(&s.h_coef), c.max_blocks * 128, hipHostMallocDefault)) !=
            hipSuccess ||
        (e = hipHostMalloc(reinterpret_cast<void**>(&s.h_qt), 4 * 64 * sizeof(uint16_t), hipHostMallocDefault)) !=
            hipSuccess)
      return fail(MJD_ENOMEM, "pinned host allocation failed: %s", hipGetErrorString(e));
    if ((e = hipMalloc(reinterpret_cast<void**>(&s.d_coef), c.max_blocks * 128)) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&s.d_qt), 4 * 64 * sizeof(uint16_t))) != hipSuccess ||
        (e = hipMalloc(reinterpret_cast<void**>(&s.d_rgb), c.max_pixels * 3)) != hipSuccess)
      return fail(MJD_ENOMEM, "device allocation failed: %s", hipGetErrorString(e));
    if ((e = hipEventCreateWithFlags(&s.free_ev, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "hipEventCreateWithFlags");
    for (auto& ev : s.tev)
      if ((e = hipEventCreate(&ev)) != hipSuccess) return hip_fail(e, "hipEventCreate");
  }
  for (uint32_t i = 0; i < c.n_threads; ++i) p->workers.emplace_back([p] { p->worker_loop(); });
  return MJD_OK;
}

// Adds the slot's recorded stage intervals to the stats.
static void collect(Slot& s, mjd_pipeline_stats* st) {
  for (int b = 0; b < s.timed_bands; ++b) {
    float ms = 0;
    hipEvent_t* e = s.tev + b * kEventsPerBand;
    if (hipEventElapsedTime(&ms, e[0], e[1]) == hipSuccess) st->h2d_ms += ms;
    if (hipEventElapsedTime(&ms, e[2], e[3]) == hipSuccess) st->kernel_ms += ms;
    if (hipEventElapsedTime(&ms, e[4], e[5]) == hipSuccess) st->d2h_ms += ms;
  }
  s.timed_bands = 0;
}

struct Run {
  mjd_pipeline* p;
  bool entropy_only;
  mjd_pipeline_stats st{};
  std::vector<std::unique_ptr<Image>> images;
  int status = MJD_OK;
  std::string err;

  void set_error(int code, const std::string& msg) {
    if (status == MJD_OK) {
      status = code;
      err = msg;
    }
  }

  // Parse image i into its slot and queue its decode tasks.  Returns false
  // (with the error recorded) if the image cannot be decoded.
  bool publish(size_t i, const uint8_t* jpg, size_t len, uint8_t* rgb, size_t pitch) {
    const auto t0 = Clock::now();
    Slot& sl = p->slots[i % p->slots.size()];
    std::unique_ptr<Image>& ip = images[i];
    ip.reset(new Image);
    Image& im = *ip;
    im.index = i;
    im.jpg = jpg;
    im.len = len;
    im.slot = static_cast<int>(i % p->slots.size());
    im.h_rgb = rgb;
    im.pitch = pitch;
    auto bad = [&](int rc) {
      set_error(rc, "image " + std::to_string(i) + ": " + mjd_last_error());
      return false;
    };
    if (!jpg || !rgb) return bad(fail(MJD_EINVAL, "null bitstream or output pointer"));
    int rc = host::parse(jpg, len, &im.scan, im.qt);
    if (rc != MJD_OK) return bad(rc);
    if (im.scan.ncomp != 3) return bad(fail(MJD_EUNSUPPORTED, "grayscale stream (mjd_decode_variant decodes it)"));
    if ((rc = frame_geometry(&im.scan.frame, &im.g)) != MJD_OK) return bad(rc);
    const uint32_t W = im.scan.frame.width, H = im.scan.frame.height;
    if (im.g.n_blocks > p->cfg.max_blocks || static_cast<uint64_t>(W) * H > p->cfg.max_pixels)
      return bad(fail(MJD_EBUDGET, "%ux%u image (%llu blocks) exceeds the slot size", W, H,
                      static_cast<unsigned long long>(im.g.n_blocks)));
    if (pitch < 3ull * W) return bad(fail(MJD_EINVAL, "pitch %zu < 3*width", pitch));
    im.offsets.resize(static_cast<size_t>(im.scan.n_intervals) + 1);
    if ((rc = host::restart_index(jpg, len, &im.scan, im.offsets.data())) != MJD_OK) return bad(rc);
    if ((rc = host::scan_layout(&im.scan, &im.L)) != MJD_OK) return bad(rc);
    if ((rc = host::build_tables(&im.scan, sl.tables.get())) != MJD_OK) return bad(rc);
    memcpy(sl.h_qt, im.qt, sizeof(im.qt));
    // bands of MCU rows
    const uint32_t rows = im.g.mcus_y;
    uint32_t br = p->cfg.band_mcu_rows ? p->cfg.band_mcu_rows : std::max<uint32_t>(1, (rows + 7) / 8);
    br = std::max<uint32_t>(br, (rows + kMaxBands - 1) / kMaxBands);
    const uint64_t ri = im.scan.restart_interval ? im.scan.restart_interval : im.L.n_mcus;
    std::vector<Task> tasks;
    for (uint32_t r0 = 0; r0 < rows; r0 += br) {
      Band& b = im.bands[im.n_bands];
      b.r0 = r0;
      b.r1 = std::min(rows, r0 + br);
      const uint64_t m_lo = static_cast<uint64_t>(b.r0) * im.L.mcus_x;
      const uint64_t m_hi = static_cast<uint64_t>(b.r1) * im.L.mcus_x;
      b.s0 = static_cast<uint32_t>(m_lo / ri);
      b.s1 = static_cast<uint32_t>((m_hi - 1) / ri) + 1;
      b.remaining.store(b.s1 - b.s0, std::memory_order_relaxed);
      for (uint32_t s = b.s0; s < b.s1; ++s)
        tasks.push_back(Task{&im, &sl, static_cast<uint32_t>(im.n_bands), s});
      ++im.n_bands;
    }
    sl.img = &im;
    st.parse_ms += std::chrono::duration<double, std::milli>(Clock::now() - t0).count();
    if (!entropy_only) {
      hipError_t e = hipMemcpyAsync(sl.d_qt, sl.h_qt, sizeof(im.qt), hipMemcpyHostToDevice, p->s_h2d);
      if (e != hipSuccess) {
        hip_fail(e, "hipMemcpyAsync");
        return bad(MJD_EDEVICE);
      }
    }
    {
      std::lock_guard<std::mutex> g(p->mu);
      p->queue.insert(p->queue.end(), tasks.begin(), tasks.end());
    }
    p->cv_task.notify_all();
    st.images += 1;
    st.pixels += static_cast<uint64_t>(W) * H;
    st.bitstream_bytes += len;
    st.bands += im.n_bands;
    return true;
  }

  // Kernel and device->host copy of band k (its coefficients, and those of
  // every band it reads, are already on the device or queued before it).
  hipError_t launch_band(Image& im, Slot& sl, int k, hipEvent_t after) {
    const Band& b = im.bands[k];
    const uint32_t W = im.scan.frame.width, H = im.scan.frame.height;
    hipEvent_t* e = sl.tev + k * kEventsPerBand;
    hipError_t r;
    if ((r = hipStreamWaitEvent(p->s_kernel, after, 0)) != hipSuccess) return r;
    if ((r = hipEventRecord(e[2], p->s_kernel)) != hipSuccess) return r;
    const int rc = mjd_decode(p->ctx, &im.scan.frame, sl.d_coef, sl.d_qt, static_cast<int>(p->cfg.upsample),
                              sl.d_rgb, 3ull * W, b.r0, b.r1, p->s_kernel);
    if (rc != MJD_OK) return hipErrorLaunchFailure;
    if ((r = hipEventRecord(e[3], p->s_kernel)) != hipSuccess) return r;
    const size_t y0 = static_cast<size_t>(b.r0) * im.g.mcu_h;
    const size_t y1 = std::min<size_t>(H, static_cast<size_t>(b.r1) * im.g.mcu_h);
    if ((r = hipStreamWaitEvent(p->s_d2h, e[3], 0)) != hipSuccess) return r;
    if ((r = hipEventRecord(e[4], p->s_d2h)) != hipSuccess) return r;
    // dense host rows take one linear copy; strided ones a 2-D copy
    if (im.pitch == 3ull * W)
      r = hipMemcpyAsync(im.h_rgb + y0 * im.pitch, sl.d_rgb + y0 * 3ull * W, (y1 - y0) * 3ull * W,
                         hipMemcpyDeviceToHost, p->s_d2h);
    else
      r = hipMemcpy2DAsync(im.h_rgb + y0 * im.pitch, im.pitch, sl.d_rgb + y0 * 3ull * W, 3ull * W, 3ull * W,
                           y1 - y0, hipMemcpyDeviceToHost, p->s_d2h);
    if (r != hipSuccess) return r;
    return hipEventRecord(e[5], p->s_d2h);
  }

  // Band k of image im has been entropy-decoded: send it on.
  hipError_t hand_off(Image& im, int k) {
    Slot& sl = p->slots[im.slot];
    const Band& b = im.bands[k];
    const uint64_t row_blocks = static_cast<uint64_t>(im.L.mcus_x) * im.L.bpm;
    const uint64_t off = static_cast<uint64_t>(b.r0) * row_blocks * 64;
    const uint64_t bytes = static_cast<uint64_t>(b.r1 - b.r0) * row_blocks * 128;
    hipEvent_t* e = sl.tev + k * kEventsPerBand;
    hipError_t r;
    if ((r = hipEventRecord(e[0], p->s_h2d)) != hipSuccess) return r;
    if ((r = hipMemcpyAsync(sl.d_coef + off, sl.h_coef + off, bytes, hipMemcpyHostToDevice, p->s_h2d)) !=
        hipSuccess)
      return r;
    if ((r = hipEventRecord(e[1], p->s_h2d)) != hipSuccess) return r;
    sl.timed_bands = k + 1;
    // fancy 4:2:0 reads the first chroma row of the next band: its kernel
    // waits until that band is on the device too
    const bool needs_next = p->cfg.upsample == MJD_UPSAMPLE_FANCY && im.scan.frame.v[0] == 2;
    if (needs_next) {
      if (k > 0 && (r = launch_band(im, sl, k - 1, e[1])) != hipSuccess) return r;
      if (k == im.n_bands - 1 && (r = launch_band(im, sl, k, e[1])) != hipSuccess) return r;
    } else if ((r = launch_band(im, sl, k, e[1])) != hipSuccess) {
      return r;
    }
    return hipSuccess;
  }

  void execute(size_t n, const uint8_t* const* jpgs, const size_t* lens, uint8_t* const* rgb,
               const size_t* pitches) {
    const size_t S = p->slots.size();
    images.resize(n);
    size_t next_pub = 0;  // images published
    size_t gi = 0;        // image whose bands are being handed to the GPU
    int gb = 0;           // its next band
    bool failed = false;
    while (gi < next_pub || (!failed && next_pub < n)) {
      bool progressed = false;
      if (!failed && next_pub < n && next_pub < gi + S) {
        Slot& sl = p->slots[next_pub % S];
        if (sl.busy) {
          const hipError_t q = hipEventQuery(sl.free_ev);
          if (q == hipSuccess) {
            collect(sl, &st);
            sl.busy = false;
          } else if (q != hipErrorNotReady) {
            set_error(MJD_EDEVICE, std::string("device work of an earlier image failed: ") + hipGetErrorString(q));
            failed = true;
            continue;
          }
        }
        if (!sl.busy) {
          if (publish(next_pub, jpgs[next_pub], lens[next_pub], rgb[next_pub], pitches[next_pub])) {
            ++next_pub;
          } else {
            failed = true;
          }
          progressed = true;
        }
      }
      if (gi < next_pub) {
        Image& im = *images[gi];
        Band& b = im.bands[gb];
        if (b.remaining.load(std::memory_order_acquire) == 0) {
          if (im.status.load() != MJD_OK) {
            std::lock_guard<std::mutex> g(im.err_mu);
            set_error(im.status.load(), "image " + std::to_string(gi) + ": " + im.err);
            failed = true;
          } else if (!failed && !entropy_only) {
            hipError_t r = hand_off(im, gb);
            if (r != hipSuccess) {
              set_error(MJD_EDEVICE, "image " + std::to_string(gi) + ": " + hipGetErrorString(r));
              failed = true;
            }
          }
          if (++gb == im.n_bands) {
            Slot& sl = p->slots[im.slot];
            if (!entropy_only) {
              (void)hipEventRecord(sl.free_ev, p->s_d2h);
              sl.busy = true;
            }
            ++gi;
            gb = 0;
          }
          progressed = true;
        }
      }
      if (!progressed) {
        Task t;
        if (p->try_pop(&t)) {
          p->run_task(t);
        } else if (gi < next_pub) {
          Band& b = images[gi]->bands[gb];
          std::unique_lock<std::mutex> lk(p->mu);
          p->cv_done.wait_for(lk, std::chrono::microseconds(200),
                              [&] { return b.remaining.load(std::memory_order_acquire) == 0; });
        } else {
          std::this_thread::sleep_for(std::chrono::microseconds(50));  // a slot's device work is finishing
        }
      }
    }
    if (!entropy_only) {
      hipError_t r = hipStreamSynchronize(p->s_d2h);
      if (r != hipSuccess) set_error(MJD_EDEVICE, std::string("hipStreamSynchronize: ") + hipGetErrorString(r));
      for (auto& sl : p->slots) {
        if (sl.busy) {
          collect(sl, &st);
          sl.busy = false;
        }
      }
    }
  }
};

}  // namespace pipe
}  // namespace mjd

extern "C" {

int mjd_pipeline_create(mjd_ctx* ctx, const mjd_pipeline_config* cfg, mjd_pipeline** out) {
  if (!ctx || !cfg || !out) return mjd::fail(MJD_EINVAL, "null context, config or out-pointer");
  *out = nullptr;
  if (cfg->n_threads < 1 || cfg->n_threads > 256) return mjd::fail(MJD_EINVAL, "n_threads %u outside 1..256", cfg->n_threads);
  if (cfg->n_slots < 2 || cfg->n_slots > 64) return mjd::fail(MJD_EINVAL, "n_slots %u outside 2..64", cfg->n_slots);
  if (cfg->upsample != MJD_UPSAMPLE_SIMPLE && cfg->upsample != MJD_UPSAMPLE_FANCY)
    return mjd::fail(MJD_EINVAL, "upsample mode %u unknown", cfg->upsample);
  if (cfg->max_blocks == 0 || cfg->max_pixels == 0) return mjd::fail(MJD_EINVAL, "slot sizes must be nonzero");
  if (cfg->max_blocks > (1ull << 32) || cfg->max_pixels > (1ull << 33))
    return mjd::fail(MJD_EINVAL, "slot sizes beyond the largest frame");
  mjd_pipeline* p = new (std::nothrow) mjd_pipeline;
  if (!p) return mjd::fail(MJD_ENOMEM, "pipeline allocation failed");
  p->ctx = ctx;
  p->device = mjd::ctx_device(ctx);
  p->cfg = *cfg;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != p->device && hipSetDevice(p->device) != hipSuccess) {
    delete p;
    return mjd::fail(MJD_EDEVICE, "hipSetDevice(%d) failed", p->device);
  }
  int rc = mjd::pipe::create(p);
  if (rc != MJD_OK) {
    mjd::pipe::release(p);
    delete p;
  } else {
    *out = p;
  }
  if (cur != p->device) (void)hipSetDevice(cur);
  return rc;
}

int mjd_pipeline_run(mjd_pipeline* pipe, size_t n, const uint8_t* const* h_jpgs, const size_t* lens,
                     uint8_t* const* h_rgb, const size_t* pitches, uint32_t flags, mjd_pipeline_stats* stats) {
  if (!pipe) return mjd::fail(MJD_EINVAL, "null pipeline");
  if (n && (!h_jpgs || !lens || !h_rgb || !pitches)) return mjd::fail(MJD_EINVAL, "null array argument");
  if (flags & ~static_cast<uint32_t>(MJD_PIPELINE_ENTROPY_ONLY)) return mjd::fail(MJD_EINVAL, "unknown flags 0x%x", flags);
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != pipe->device && hipSetDevice(pipe->device) != hipSuccess)
    return mjd::fail(MJD_EDEVICE, "hipSetDevice(%d) failed", pipe->device);
  mjd::pipe::Run run;
  run.p = pipe;
  run.entropy_only = (flags & MJD_PIPELINE_ENTROPY_ONLY) != 0;
  pipe->busy_ns.store(0);
  const auto t0 = mjd::pipe::Clock::now();
  run.execute(n, h_jpgs, lens, h_rgb, pitches);
  run.st.wall_ms = std::chrono::duration<double, std::milli>(mjd::pipe::Clock::now() - t0).count();
  run.st.entropy_ms = pipe->busy_ns.load() * 1e-6;
  if (cur != pipe->device) (void)hipSetDevice(cur);
  if (stats) *stats = run.st;
  if (run.status != MJD_OK) return mjd::fail(run.status, "%s", run.err.c_str());
  return MJD_OK;
}

void mjd_pipeline_destroy(mjd_pipeline* pipe) {
  if (!pipe) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != pipe->device) (void)hipSetDevice(pipe->device);
  mjd::pipe::release(pipe);
  if (cur != pipe->device) (void)hipSetDevice(cur);
  delete pipe;
}

}  // extern "C"
