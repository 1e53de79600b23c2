// Heterogeneous decode of one image (paper Sec. 5.2): the GPU decodes the
// image's first MCU rows while host threads decode the rest.
//   SPS: host Huffman decoding of the whole image, then the GPU rows are
//        copied in, decoded and copied back asynchronously while the host
//        decodes its own rows (mjd_decode_host).
//   PPS: host Huffman decoding of the GPU's rows (and the MCU row below
//        them, which fancy 4:2:0 reads), the asynchronous GPU part, then the
//        host decodes its own rows' Huffman data and pixels meanwhile.
// The split comes from the caller (mjd_partition_rows balances it).
#include <hip/hip_runtime_api.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>
#include <vector>

#include "host_jpeg.h"
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
  *out = h;
  return MJD_OK;
}

int mjd_hetero_decode(mjd_hetero* h, const uint8_t* h_jpg, size_t len, int upsample, int scheme, uint32_t cpu_rows,
                      uint8_t* h_rgb, size_t pitch, mjd_hetero_times* times) {
  const Clock::time_point t0 = Clock::now();
  if (!h || !h_jpg || !h_rgb) return mjd::fail(MJD_EINVAL, "null decoder, stream or output pointer");
  if (scheme != MJD_PART_SPS && scheme != MJD_PART_PPS) return mjd::fail(MJD_EINVAL, "unknown scheme %d", scheme);
  mjd_scan scan;
  uint16_t qt[4][64];
  int rc = mjd::host::parse(h_jpg, len, &scan, qt);
  if (rc != MJD_OK) return rc;
  mjd_geometry g;
  rc = mjd::frame_geometry(&scan.frame, &g);
  if (rc != MJD_OK) return rc;
  const uint32_t W = scan.frame.width, H = scan.frame.height;
  if (g.n_blocks > h->max_blocks || static_cast<uint64_t>(W) * H > h->max_pixels)
    return mjd::fail(MJD_EINVAL, "image larger than the decoder's buffers");
  if (pitch < 3ull * W) return mjd::fail(MJD_EINVAL, "pitch below 3*width");
  if (cpu_rows > H) return mjd::fail(MJD_EINVAL, "cpu_rows beyond the image");
  // the GPU's MCU rows: the split must fall on an MCU-row boundary
  uint32_t R = (H - cpu_rows) / g.mcu_h;
  if (H - cpu_rows == H) R = g.mcus_y;
  if (std::min<uint64_t>(H, static_cast<uint64_t>(R) * g.mcu_h) != H - cpu_rows)
    return mjd::fail(MJD_EINVAL, "cpu_rows %u leaves the GPU a partial MCU row", cpu_rows);
  std::vector<uint64_t> off(scan.n_intervals + 1);
  rc = mjd::host::restart_index(h_jpg, len, &scan, off.data());
  if (rc != MJD_OK) return rc;
  mjd_hetero_times tm{};
  // the GPU's rows and the MCU row below them, which fancy 4:2:0 reads
  const uint32_t gpu_need = R ? std::min(g.mcus_y, R + 1) : 0;
  const uint64_t row_blocks = static_cast<uint64_t>(g.mcus_x) * g.blocks_per_mcu;
  Clock::time_point t = Clock::now();
  rc = mjd::host::decode_rows(h_jpg, len, &scan, off.data(), h->h_coef, 0, scheme == MJD_PART_SPS ? g.mcus_y : gpu_need,
                              h->n_threads);
  if (rc != MJD_OK) return rc;
  Clock::time_point t1 = Clock::now();
  tm.huff_gpu_s = secs(t, t1);
  DeviceScope ds(h->device);
  hipEvent_t start = nullptr, done = nullptr;
  Clock::time_point tg = t1;
  if (R) {
    hipError_t e;
    if ((e = hipEventCreate(&start)) != hipSuccess || (e = hipEventCreate(&done)) != hipSuccess ||
        (e = hipEventRecord(start, h->stream)) != hipSuccess) {
      if (start) (void)hipEventDestroy(start);
      if (done) (void)hipEventDestroy(done);
      return mjd::fail(MJD_EDEVICE, "hipEventCreate: %s", hipGetErrorString(e));
    }
    if ((e = hipMemcpyAsync(h->d_coef, h->h_coef, gpu_need * row_blocks * 128, hipMemcpyHostToDevice, h->stream)) !=
            hipSuccess ||
        (e = hipMemcpyAsync(h->d_qt, qt, sizeof(qt), hipMemcpyHostToDevice, h->stream)) != hipSuccess) {
      (void)hipStreamSynchronize(h->stream);
      (void)hipEventDestroy(start);
      (void)hipEventDestroy(done);
      return mjd::fail(MJD_EDEVICE, "copy in: %s", hipGetErrorString(e));
    }
    rc = mjd_decode(h->ctx, &scan.frame, h->d_coef, h->d_qt, upsample, h->d_rgb, 3ull * W, 0, R, h->stream);
    const uint32_t rows = std::min<uint64_t>(H, static_cast<uint64_t>(R) * g.mcu_h);
    if (rc == MJD_OK &&
        ((e = hipMemcpy2DAsync(h_rgb, pitch, h->d_rgb, 3ull * W, 3ull * W, rows, hipMemcpyDeviceToHost,
                               h->stream)) != hipSuccess ||
         (e = hipEventRecord(done, h->stream)) != hipSuccess))
      rc = mjd::fail(MJD_EDEVICE, "copy out: %s", hipGetErrorString(e));
    if (rc != MJD_OK) {
      (void)hipStreamSynchronize(h->stream);
      (void)hipEventDestroy(start);
      (void)hipEventDestroy(done);
      return rc;
    }
    tg = Clock::now();
    tm.dispatch_s = secs(t1, tg);
  }
  if (R < g.mcus_y) {
    t = Clock::now();
    if (scheme == MJD_PART_PPS && gpu_need < g.mcus_y) {
      rc = mjd::host::decode_rows(h_jpg, len, &scan, off.data(), h->h_coef, gpu_need, g.mcus_y, h->n_threads);
      tm.huff_cpu_s = secs(t, Clock::now());
      t = Clock::now();
    }
    if (rc == MJD_OK)
      rc = mjd_decode_host(&scan.frame, h->h_coef, &qt[0][0], upsample, h_rgb, pitch, R, g.mcus_y, h->n_threads);
    tm.cpu_s = secs(t, Clock::now());
  }
  if (done) {
    hipError_t e = hipEventSynchronize(done);
    float ms = 0.0f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, start, done);
    tm.gpu_s = ms * 1e-3;  // device time from the first copy in to the last copy out
    (void)hipEventDestroy(start);
    (void)hipEventDestroy(done);
    if (e != hipSuccess && rc == MJD_OK) rc = mjd::fail(MJD_EDEVICE, "GPU part: %s", hipGetErrorString(e));
  }
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
