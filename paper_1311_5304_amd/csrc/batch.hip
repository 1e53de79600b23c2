// Batched decode: many images of mixed size and sampling in one persistent
// launch fed by a work queue of segments.
//
// The host plan cuts every image into segments (a column of sub-tiles of one
// strip, as in the single-image kernel) and lists them largest first.  The
// launch holds as many workgroups as stay resident; each pops the next
// segment index from a device counter, loads the image's view and runs the
// segment decoder of the image's sampling class.  When the last workgroup
// leaves it resets the counters, so the same launch (or a hipGraph holding
// it) can simply be replayed.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "mjd_internal.h"

namespace mjd {

// All classes run with 256 lanes so that one kernel serves the whole batch.
using B420F = SegCfg<2, 2, true, 16, 2, 256>;
using B420S = SegCfg<2, 2, false, 16, 2, 256>;
using B422F = SegCfg<2, 1, true, 8, 4, 256>;
using B422S = SegCfg<2, 1, false, 16, 4, 256>;
using B444 = SegCfg<1, 1, false, 16, 4, 256>;

constexpr int kBatchThreads = 256;
constexpr int cmax(int a, int b) { return a > b ? a : b; }
constexpr int kBatchLds =
    cmax(cmax(cmax(B420F::LDS_BYTES, B420S::LDS_BYTES), cmax(B422F::LDS_BYTES, B422S::LDS_BYTES)), B444::LDS_BYTES);

enum BatchClass : int { kC420F = 0, kC420S = 1, kC422F = 2, kC422S = 3, kC444 = 4 };

__global__ __launch_bounds__(kBatchThreads, 2) void decode_batch(const ImageView* __restrict__ views,
                                                              const BatchItem* __restrict__ items, int n_items,
                                                              unsigned* counters) {
  __shared__ __align__(16) uint8_t lds[kBatchLds];
  __shared__ int s_next;
  const int tid = static_cast<int>(threadIdx.x);
  for (;;) {
    if (tid == 0) s_next = static_cast<int>(atomicAdd(&counters[0], 1u));
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(s_next);
    __syncthreads();  // every lane has read s_next before it is overwritten
    if (it >= n_items) break;
    const BatchItem bi = items[it];
    // a reference into the device table (scalar loads), not a local copy,
    // which would have to live in scratch memory behind the decoder's
    // reference
    const ImageView& im = views[bi.img];
    SegmentRange r;
    r.mx0 = bi.mx0;
    r.r0 = bi.r0;
    r.r1 = bi.r1;
    switch (bi.cls) {
      case kC420F: {
        SegmentDecoder<B420F, true> d(lds, im, tid);
        d.run(r);
        break;
      }
      case kC420S: {
        SegmentDecoder<B420S> d(lds, im, tid);
        d.run(r);
        break;
      }
      case kC422F: {
        SegmentDecoder<B422F> d(lds, im, tid);
        d.run(r);
        break;
      }
      case kC422S: {
        SegmentDecoder<B422S> d(lds, im, tid);
        d.run(r);
        break;
      }
      default: {
        SegmentDecoder<B444> d(lds, im, tid);
        d.run(r);
        break;
      }
    }
  }
  // the last workgroup out rearms the queue for the next launch
  if (tid == 0) {
    __threadfence();
    const unsigned done = atomicAdd(&counters[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&counters[0], 0u);
      atomicExch(&counters[1], 0u);
    }
  }
}

static void class_shape(int cls, int* sx, int* sy) {
  switch (cls) {
    case kC420F: *sx = B420F::SX; *sy = B420F::SY; return;
    case kC420S: *sx = B420S::SX; *sy = B420S::SY; return;
    case kC422F: *sx = B422F::SX; *sy = B422F::SY; return;
    case kC422S: *sx = B422S::SX; *sy = B422S::SY; return;
    default: *sx = B444::SX; *sy = B444::SY; return;
  }
}

}  // namespace mjd

struct mjd_batch {
  mjd_ctx* ctx = nullptr;
  int n_items = 0;
  int grid = 0;
  mjd::ImageView* d_views = nullptr;
  mjd::BatchItem* d_items = nullptr;
  unsigned* d_counters = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  uint64_t pixels = 0;
};

namespace mjd {

static int batch_slots(mjd_ctx* ctx) {
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, decode_batch, kBatchThreads, 0) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu * (ctx->cu_count > 0 ? ctx->cu_count : 256);
}

int batch_plan(mjd_ctx* ctx, const mjd_job* jobs, size_t n, int upsample, BatchPlan* plan) {
  if (n == 0) return fail(MJD_EINVAL, "empty batch");
  if (n > (1u << 24)) return fail(MJD_EINVAL, "batch of %zu images too large", n);
  if (upsample != MJD_UPSAMPLE_SIMPLE && upsample != MJD_UPSAMPLE_FANCY)
    return fail(MJD_EINVAL, "upsample mode %d unknown", upsample);
  plan->views.resize(n);
  plan->items.clear();
  plan->pixels = 0;
  std::vector<int> cls(n);
  std::vector<mjd_geometry> geo(n);
  uint64_t subtiles = 0;
  for (size_t i = 0; i < n; ++i) {
    int rc = job_view(&jobs[i], upsample, &plan->views[i], &geo[i]);
    if (rc != MJD_OK) {
      const std::string why = mjd_last_error();
      return fail(rc, "job %zu: %s", i, why.c_str());
    }
    const int hf = jobs[i].frame.h[0], vf = jobs[i].frame.v[0];
    const bool fancy = upsample == MJD_UPSAMPLE_FANCY;
    cls[i] = (hf == 1) ? kC444 : (vf == 1 ? (fancy ? kC422F : kC422S) : (fancy ? kC420F : kC420S));
    int sx, sy;
    class_shape(cls[i], &sx, &sy);
    subtiles += static_cast<uint64_t>((geo[i].mcus_x + sx - 1) / sx) * ((geo[i].mcus_y + sy - 1) / sy);
    plan->pixels += static_cast<uint64_t>(jobs[i].frame.width) * jobs[i].frame.height;
  }
  const int slots = batch_slots(ctx);
  // Segment length: about 4 segments per resident workgroup over the whole
  // batch, so the queue balances the tail; the tuning knob overrides it.
  int seg_sub = static_cast<int>(ctx->tuning.seg_subtiles);
  if (seg_sub <= 0) {
    const uint64_t want = static_cast<uint64_t>(slots) * 4;
    seg_sub = static_cast<int>(std::max<uint64_t>(1, (subtiles + want - 1) / want));
  }
  for (size_t i = 0; i < n; ++i) {
    int sx, sy;
    class_shape(cls[i], &sx, &sy);
    const int strips = (geo[i].mcus_x + sx - 1) / sx;
    const int rows = static_cast<int>(geo[i].mcus_y);
    const int seg_rows = seg_sub * sy;
    for (int r0 = 0; r0 < rows; r0 += seg_rows)
      for (int s = 0; s < strips; ++s) {
        BatchItem it{};
        it.img = static_cast<int>(i);
        it.cls = cls[i];
        it.mx0 = s * sx;
        it.r0 = r0;
        it.r1 = std::min(rows, r0 + seg_rows);
        plan->items.push_back(it);
      }
  }
  // longest segments first: the queue then fills the tail with short ones
  std::stable_sort(plan->items.begin(), plan->items.end(), [](const BatchItem& a, const BatchItem& c) {
    return (a.r1 - a.r0) > (c.r1 - c.r0);
  });
  if (plan->items.size() > 0x7FFFFFF0u) return fail(MJD_EINVAL, "batch needs too many segments");
  // every resident slot by default; a tuned count may be smaller or larger
  // (workgroups beyond the resident ones start as others leave and find
  // what is left of the queue)
  int grid = ctx->tuning.workgroups > 0 ? static_cast<int>(ctx->tuning.workgroups) : slots;
  grid = std::min(grid, static_cast<int>(plan->items.size()));
  plan->grid = grid;
  return MJD_OK;
}

// ---- the no-allocation entry point ----
// The batch tables of mjd_decode_batch_noalloc live in this fixed device
// array (one copy per GPU, held until the process ends): the queue counters
// first, then the image views, then the segment queue.  In host code the
// array's name is not a device address; every use goes through the address
// looked up with hipGetSymbolAddress once per device.
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
constexpr size_t kNoAllocHeader = 256;  // the two queue counters, padded
static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

hipError_t noalloc_scratch_address(int device, void** out) {
  static std::mutex mu;
  static void* addr[64] = {};
  if (device < 0 || device >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = 0;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *out = addr[device];
  return hipSuccess;
}

hipError_t batch_enqueue(const ImageView* d_views, const BatchItem* d_items, int n_items, unsigned* d_counters,
                         int grid, hipStream_t stream) {
  hipLaunchKernelGGL(decode_batch, dim3(grid), dim3(kBatchThreads), 0, stream, d_views, d_items, n_items,
                     d_counters);
  return hipGetLastError();
}

int batch_build(mjd_ctx* ctx, const mjd_job* jobs, size_t n, int upsample, mjd_batch* b) {
  BatchPlan plan;
  int rc = batch_plan(ctx, jobs, n, upsample, &plan);
  if (rc != MJD_OK) return rc;
  b->pixels = plan.pixels;
  b->n_items = static_cast<int>(plan.items.size());
  b->grid = plan.grid;
  if (hipMalloc(&b->d_views, plan.views.size() * sizeof(ImageView)) != hipSuccess ||
      hipMalloc(&b->d_items, plan.items.size() * sizeof(BatchItem)) != hipSuccess ||
      hipMalloc(&b->d_counters, 2 * sizeof(unsigned)) != hipSuccess)
    return fail(MJD_ENOMEM, "device allocation for the batch tables failed");
  if (hipMemcpy(b->d_views, plan.views.data(), plan.views.size() * sizeof(ImageView), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemcpy(b->d_items, plan.items.data(), plan.items.size() * sizeof(BatchItem), hipMemcpyHostToDevice) !=
          hipSuccess ||
      hipMemset(b->d_counters, 0, 2 * sizeof(unsigned)) != hipSuccess)
    return fail(MJD_EDEVICE, "uploading the batch tables failed");
  return MJD_OK;
}

void batch_free(mjd_batch* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->d_views) (void)hipFree(b->d_views);
  if (b->d_items) (void)hipFree(b->d_items);
  if (b->d_counters) (void)hipFree(b->d_counters);
  b->exec = nullptr;
  b->graph = nullptr;
  b->d_views = nullptr;
  b->d_items = nullptr;
  b->d_counters = nullptr;
}

hipError_t batch_launch(mjd_batch* b, bool use_graph, hipStream_t stream) {
  if (!use_graph) return batch_enqueue(b->d_views, b->d_items, b->n_items, b->d_counters, b->grid, stream);
  if (!b->exec) {
    hipError_t e = hipGraphCreate(&b->graph, 0);
    if (e != hipSuccess) return e;
    void* args[] = {&b->d_views, &b->d_items, &b->n_items, &b->d_counters};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void*>(decode_batch);
    kp.gridDim = dim3(b->grid);
    kp.blockDim = dim3(kBatchThreads);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    hipGraphNode_t node;
    e = hipGraphAddKernelNode(&node, b->graph, nullptr, 0, &kp);
    if (e != hipSuccess) return e;
    e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0);
    if (e != hipSuccess) return e;
  }
  return hipGraphLaunch(b->exec, stream);
}

}  // namespace mjd

extern "C" {

int mjd_batch_create(mjd_ctx* ctx, const mjd_job* jobs, size_t n, int upsample, mjd_batch** out) {
  if (!ctx || !out) return mjd::fail(MJD_EINVAL, "null context or out-pointer");
  *out = nullptr;
  if (!jobs && n) return mjd::fail(MJD_EINVAL, "null jobs");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
    return mjd::fail(MJD_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
  mjd_batch* b = new (std::nothrow) mjd_batch;
  if (!b) return mjd::fail(MJD_ENOMEM, "batch allocation failed");
  b->ctx = ctx;
  int rc = mjd::batch_build(ctx, jobs, n, upsample, b);
  if (cur != ctx->device) (void)hipSetDevice(cur);
  if (rc != MJD_OK) {
    mjd::batch_free(b);
    delete b;
    return rc;
  }
  *out = b;
  return MJD_OK;
}

int mjd_batch_launch(mjd_batch* batch, int use_graph, void* stream) {
  if (!batch) return mjd::fail(MJD_EINVAL, "null batch");
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != batch->ctx->device && hipSetDevice(batch->ctx->device) != hipSuccess)
    return mjd::fail(MJD_EDEVICE, "hipSetDevice(%d) failed", batch->ctx->device);
  hipError_t e = mjd::batch_launch(batch, use_graph != 0, static_cast<hipStream_t>(stream));
  if (cur != batch->ctx->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return mjd::fail(MJD_EDEVICE, "batch launch failed: %s", hipGetErrorString(e));
  return MJD_OK;
}

int mjd_batch_info(const mjd_batch* batch, uint32_t* segments, uint32_t* workgroups, uint64_t* pixels) {
  if (!batch) return mjd::fail(MJD_EINVAL, "null batch");
  if (segments) *segments = static_cast<uint32_t>(batch->n_items);
  if (workgroups) *workgroups = static_cast<uint32_t>(batch->grid);
  if (pixels) *pixels = batch->pixels;
  return MJD_OK;
}

int mjd_decode_batch_noalloc(mjd_ctx* ctx, const mjd_job* jobs, size_t n, int upsample, void* stream) {
  if (!ctx) return mjd::fail(MJD_EINVAL, "null context");
  if (!jobs && n) return mjd::fail(MJD_EINVAL, "null jobs");
  if (!ctx->noalloc_scratch) return mjd::fail(MJD_EDEVICE, "no scratch address for device %d", ctx->device);
  mjd::BatchPlan plan;
  int rc = mjd::batch_plan(ctx, jobs, n, upsample, &plan);
  if (rc != MJD_OK) return rc;
  const size_t views_bytes = plan.views.size() * sizeof(mjd::ImageView);
  const size_t items_bytes = plan.items.size() * sizeof(mjd::BatchItem);
  const size_t items_off = mjd::kNoAllocHeader + ((views_bytes + 255) & ~size_t(255));
  const size_t need = items_off + items_bytes;
  if (need > mjd::kNoAllocScratchBytes)
    return mjd::fail(MJD_EBUDGET, "batch tables need %zu bytes; the no-allocation entry point holds at most %zu",
                     need, mjd::kNoAllocScratchBytes);
  // the tables as they go to the device, in this thread's reusable buffer
  // (host memory; its capacity only grows)
  thread_local std::vector<uint8_t> host;
  if (host.size() < need) host.resize(need);
  std::memset(host.data(), 0, mjd::kNoAllocHeader);  // both queue counters start at zero
  std::memcpy(host.data() + mjd::kNoAllocHeader, plan.views.data(), views_bytes);
  std::memcpy(host.data() + items_off, plan.items.data(), items_bytes);
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != ctx->device && hipSetDevice(ctx->device) != hipSuccess)
    return mjd::fail(MJD_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
  uint8_t* base = static_cast<uint8_t*>(ctx->noalloc_scratch);
  const hipStream_t st = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(base, host.data(), need, hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = mjd::batch_enqueue(reinterpret_cast<const mjd::ImageView*>(base + mjd::kNoAllocHeader),
                           reinterpret_cast<const mjd::BatchItem*>(base + items_off),
                           static_cast<int>(plan.items.size()), reinterpret_cast<unsigned*>(base), plan.grid, st);
  if (cur != ctx->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return mjd::fail(MJD_EDEVICE, "no-allocation batch launch failed: %s", hipGetErrorString(e));
  return MJD_OK;
}

void mjd_batch_destroy(mjd_batch* batch) {
  if (!batch) return;
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != batch->ctx->device) (void)hipSetDevice(batch->ctx->device);
  (void)hipDeviceSynchronize();
  mjd::batch_free(batch);
  if (cur != batch->ctx->device) (void)hipSetDevice(cur);
  delete batch;
}

}  // extern "C"
