// Heterogeneous decode of one image (paper Sec. 5.2): the GPU decodes the
// image's first MCU rows while host threads decode the rest.
//   SPS: host Huffman decoding of the whole image, then the GPU rows are
//        copied in, decoded and copied back asynchronously while the host
//        decodes its own rows (mjd_decode_host).
//   OVERLAP: host Huffman decoding of the GPU's rows (and the MCU row below
//        them, which fancy 4:2:0 reads), the asynchronous GPU part, then the
//        host decodes its own rows' Huffman data and pixels meanwhile.
//   PPS: the GPU's rows go in chunks: each chunk's Huffman data is decoded
//        and the chunk enqueued (copy in, kernel, copy out) while the GPU
//        still works on the previous ones; then the host's rows as in
//        OVERLAP.  With a model, the split is solved again before the last
//        chunk, from the Huffman time measured so far (Eqs. 16-17).
// The split comes from the caller (mjd_partition_rows balances it).
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "cpu_decode.h"
#include "host_jpeg.h"
#include "host_pool.h"
#include "mjd_common.h"

struct mjd_hetero {
  mjd_ctx* ctx = nullptr;
  int device = 0;
  int n_threads = 1;
  uint64_t max_blocks = 0, max_pixels = 0;
  int16_t* h_coef = nullptr;  // pinned
  int16_t* d_coef = nullptr;
  uint16_t* d_qt = nullptr;
  uint8_t* d_rgb = nullptr;
  hipStream_t stream = nullptr;
  mjd::WorkerPool* pool = nullptr;  // n_threads - 1 workers, kept between images
};

namespace {

using Clock = std::chrono::steady_clock;

double secs(Clock::time_point a, Clock::time_point b) { return std::chrono::duration<double>(b - a).count(); }

void release(mjd_hetero* h) {
  if (h->h_coef) (void)hipHostFree(h->h_coef);
  if (h->d_coef) (void)hipFree(h->d_coef);
  if (h->d_qt) (void)hipFree(h->d_qt);
  if (h->d_rgb) (void)hipFree(h->d_rgb);
  if (h->stream) (void)hipStreamDestroy(h->stream);
  delete h->pool;
}

// Sets the context's device for the scope.
struct DeviceScope {
  int prev = 0;
  bool changed = false;
  explicit DeviceScope(int dev) {
    (void)hipGetDevice(&prev);
    if (prev != dev) changed = hipSetDevice(dev) == hipSuccess;
  }
  ~DeviceScope() {
    if (changed) (void)hipSetDevice(prev);
  }
};

}  // namespace

extern "C" {

int mjd_hetero_create(mjd_ctx* ctx, uint64_t max_blocks, uint64_t max_pixels, int n_threads, mjd_hetero** out) {
  if (!ctx || !out) return mjd::fail(MJD_EINVAL, "null context or out-pointer");
  *out = nullptr;
  if (!max_blocks || !max_pixels) return mjd::fail(MJD_EINVAL, "zero capacity");
  if (n_threads < 1 || n_threads > 256) return mjd::fail(MJD_EINVAL, "thread count outside 1..256");
  mjd_hetero* h = new (std::nothrow) mjd_hetero;
  if (!h) return mjd::fail(MJD_ENOMEM, "allocation failed");
  h->ctx = ctx;
  h->device = mjd::ctx_device(ctx);
  h->n_threads = n_threads;
  h->max_blocks = max_blocks;
  h->max_pixels = max_pixels;
  DeviceScope ds(h->device);
  hipError_t e;
  if ((e = hipHostMalloc(reinterpret_cast<void**>(&h->h_coef), max_blocks * 128, hipHostMallocDefault)) !=
          hipSuccess ||
      (e = hipMalloc(&h->d_coef, max_blocks * 128)) != hipSuccess ||
      (e = hipMalloc(&h->d_qt, 4 * 64 * sizeof(uint16_t))) != hipSuccess ||
      (e = hipMalloc(&h->d_rgb, max_pixels * 3)) != hipSuccess ||
      (e = hipStreamCreateWithFlags(&h->stream, hipStreamNonBlocking)) != hipSuccess) {
    release(h);
    delete h;
    return mjd::fail(MJD_ENOMEM, "heterogeneous decoder buffers: %s", hipGetErrorString(e));
  }
  // pinned, so that the host's rows of a split run on as many distinct
  // cores as the model was fitted with
  h->pool = new (std::nothrow) mjd::WorkerPool(n_threads, true);
  if (!h->pool) {
    release(h);
    delete h;
    return mjd::fail(MJD_ENOMEM, "allocation failed");
  }
  *out = h;
  return MJD_OK;
}

int mjd_hetero_decode(mjd_hetero* h, const uint8_t* h_jpg, size_t len, int upsample, const mjd_hetero_plan* plan,
                      uint8_t* h_rgb, size_t pitch, mjd_hetero_times* times) {
  const Clock::time_point t0 = Clock::now();
  if (!h || !h_jpg || !h_rgb || !plan) return mjd::fail(MJD_EINVAL, "null decoder, stream, output or plan pointer");
  const int scheme = plan->scheme;
  if (scheme != MJD_PART_SPS && scheme != MJD_PART_OVERLAP && scheme != MJD_PART_PPS)
    return mjd::fail(MJD_EINVAL, "unknown scheme %d", scheme);
  if (scheme == MJD_PART_PPS && plan->model && !(plan->huff_threads >= 1.0))
    return mjd::fail(MJD_EINVAL, "huff_threads below 1");
  mjd_scan scan;
  uint16_t qt[4][64];
  int rc = mjd::host::parse(h_jpg, len, &scan, qt);
  if (rc != MJD_OK) return rc;
  if (scan.ncomp != 3) return mjd::fail(MJD_EUNSUPPORTED, "grayscale stream (mjd_decode_variant decodes it)");
  mjd_geometry g;
  rc = mjd::frame_geometry(&scan.frame, &g);
  if (rc != MJD_OK) return rc;
  const uint32_t W = scan.frame.width, H = scan.frame.height;
  if (g.n_blocks > h->max_blocks || static_cast<uint64_t>(W) * H > h->max_pixels)
    return mjd::fail(MJD_EINVAL, "image larger than the decoder's buffers");
  if (pitch < 3ull * W) return mjd::fail(MJD_EINVAL, "pitch below 3*width");
  const uint32_t cpu_rows = plan->cpu_rows;
  if (cpu_rows > H) return mjd::fail(MJD_EINVAL, "cpu_rows beyond the image");
  // the GPU's MCU rows: the split must fall on an MCU-row boundary
  uint32_t R = cpu_rows == 0 ? g.mcus_y : (H - cpu_rows) / g.mcu_h;
  if (std::min<uint64_t>(H, static_cast<uint64_t>(R) * g.mcu_h) != H - cpu_rows)
    return mjd::fail(MJD_EINVAL, "cpu_rows %u leaves the GPU a partial MCU row", cpu_rows);
  std::vector<uint64_t> off(scan.n_intervals + 1);
  rc = mjd::host::restart_index(h_jpg, len, &scan, off.data());
  if (rc != MJD_OK) return rc;
  mjd::host::RowDecoder rows_dec;
  rc = mjd::host::prepare_rows(h_jpg, len, &scan, off.data(), &rows_dec);
  if (rc != MJD_OK) return rc;
  const mjd::ParallelFor pf = [h](int n, const mjd::TaskFn& fn) { h->pool->run(n, fn); };
  mjd_hetero_times tm{};
  const uint64_t row_blocks = static_cast<uint64_t>(g.mcus_x) * g.blocks_per_mcu;
  auto pixel_rows = [&](uint32_t mcu_rows) { return std::min<uint64_t>(H, static_cast<uint64_t>(mcu_rows) * g.mcu_h); };
  uint32_t decoded = 0;  // MCU rows whose Huffman data is in h_coef
  auto huffman_to = [&](uint32_t rows, double* acc) -> int {
    if (rows <= decoded) return MJD_OK;
    const Clock::time_point a = Clock::now();
    const int r = mjd::host::decode_rows_with(rows_dec, h->h_coef, decoded, rows, pf);
    *acc += secs(a, Clock::now());
    if (r == MJD_OK) decoded = rows;
    return r;
  };
  if (scheme == MJD_PART_SPS) {
    rc = huffman_to(g.mcus_y, &tm.huff_gpu_s);
    if (rc != MJD_OK) return rc;
  }
  DeviceScope ds(h->device);
  hipEvent_t start = nullptr, done = nullptr;
  auto drop_events = [&]() {
    if (start) (void)hipEventDestroy(start);
    if (done) (void)hipEventDestroy(done);
  };
  if (R) {
    hipError_t e;
    if ((e = hipEventCreate(&start)) != hipSuccess || (e = hipEventCreate(&done)) != hipSuccess) {
      drop_events();
      return mjd::fail(MJD_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
  }
  // GPU chunks [a, b) of MCU rows; one chunk unless PPS asks for more
  const uint32_t chunk = scheme == MJD_PART_PPS && plan->chunk_mcu_rows ? plan->chunk_mcu_rows : std::max(R, 1u);
  uint32_t a = 0, copied = 0;
  double busy_pred = 0.0;  // predicted device seconds of the chunks enqueued (re-partitioning)
  Clock::time_point first_enqueue = t0;
  while (a < R) {
    uint32_t b = std::min(R, a + chunk);
    if (scheme == MJD_PART_PPS && plan->model && a > 0 && b == R) {
      // the last chunk: solve the split of the remaining rows again
      double busy = 0.0;
      if (hipEventQuery(done) != hipSuccess)
        busy = std::max(0.0, busy_pred - secs(first_enqueue, Clock::now()));
      mjd_partition p;
      rc = mjd_repartition_rows(plan->model, W, H, H - a * g.mcu_h, g.mcu_h, len, plan->huff_threads,
                                H - static_cast<uint32_t>(pixel_rows(decoded)), tm.huff_gpu_s, busy, &p);
      if (rc != MJD_OK) break;
      R = (H - p.cpu_rows) == H ? g.mcus_y : (H - p.cpu_rows) / g.mcu_h;
      if (R <= a) {  // the CPU takes every remaining row
        R = a;
        break;
      }
      b = R;
    }
    const uint32_t need = std::min(g.mcus_y, b + 1);  // the MCU row below, which fancy 4:2:0 reads
    rc = huffman_to(need, &tm.huff_gpu_s);
    if (rc != MJD_OK) break;
    const Clock::time_point te = Clock::now();
    hipError_t e = hipSuccess;
    if (a == 0) {
      first_enqueue = te;
      if ((e = hipEventRecord(start, h->stream)) == hipSuccess)
        e = hipMemcpyAsync(h->d_qt, qt, sizeof(qt), hipMemcpyHostToDevice, h->stream);
    }
    if (e == hipSuccess)
      e = hipMemcpyAsync(h->d_coef + copied * row_blocks * 64, h->h_coef + copied * row_blocks * 64,
                         (need - copied) * row_blocks * 128, hipMemcpyHostToDevice, h->stream);
    if (e != hipSuccess) {
      rc = mjd::fail(MJD_EDEVICE, "copy in: %s", hipGetErrorString(e));
      break;
    }
    copied = need;
    rc = mjd_decode(h->ctx, &scan.frame, h->d_coef, h->d_qt, upsample, h->d_rgb, 3ull * W, a, b, h->stream);
    if (rc != MJD_OK) break;
    const uint64_t y0 = pixel_rows(a), y1 = pixel_rows(b);
    if ((e = hipMemcpy2DAsync(h_rgb + y0 * pitch, pitch, h->d_rgb + y0 * 3ull * W, 3ull * W, 3ull * W, y1 - y0,
                              hipMemcpyDeviceToHost, h->stream)) != hipSuccess ||
        (e = hipEventRecord(done, h->stream)) != hipSuccess) {
      rc = mjd::fail(MJD_EDEVICE, "copy out: %s", hipGetErrorString(e));
      break;
    }
    tm.dispatch_s += secs(te, Clock::now());
    if (plan->model) {
      mjd_prediction pr;
      if (mjd_model_predict(plan->model, W, static_cast<uint32_t>(y1 - y0), 0, &pr) == MJD_OK) busy_pred += pr.p_gpu;
    }
    ++tm.chunks;
    a = b;
  }
  if (rc != MJD_OK) {
    if (R) (void)hipStreamSynchronize(h->stream);
    drop_events();
    return rc;
  }
  tm.cpu_rows = H - static_cast<uint32_t>(pixel_rows(R));
  if (R < g.mcus_y) {
    rc = huffman_to(g.mcus_y, &tm.huff_cpu_s);
    const Clock::time_point t = Clock::now();
    if (rc == MJD_OK)
      rc = mjd::cpu::decode_host_with(&scan.frame, h->h_coef, &qt[0][0], upsample, h_rgb, pitch, R, g.mcus_y,
                                      h->n_threads, pf);
    tm.cpu_s = secs(t, Clock::now());
  }
  if (tm.chunks) {
    hipError_t e = hipEventSynchronize(done);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, start, done);
    tm.gpu_s = ms * 1e-3;  // device time from the first copy in to the last copy out
    if (e != hipSuccess && rc == MJD_OK) rc = mjd::fail(MJD_EDEVICE, "GPU part: %s", hipGetErrorString(e));
  } else if (R) {
    (void)hipStreamSynchronize(h->stream);
  }
  drop_events();
  tm.total_s = secs(t0, Clock::now());
  if (times) *times = tm;
  return rc;
}

void mjd_hetero_destroy(mjd_hetero* h) {
  if (!h) return;
  DeviceScope ds(h->device);
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  release(h);
  delete h;
}

}  // extern "C"
