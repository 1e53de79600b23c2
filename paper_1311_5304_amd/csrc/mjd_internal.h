// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "mjd.h"
#include "mjd_common.h"
#include "segment.h"

struct mjd_ctx {
  int device = 0;
  int cu_count = 0;
  int xcd_count = 8;
  std::string device_name;
  mjd_tuning tuning{0, 0, 0};
  void* noalloc_scratch = nullptr;  // device address of the no-allocation batch scratch on `device`
};

namespace mjd {

// Enqueues the segment kernel for MCU rows [row0, row1) of one image.
hipError_t launch_image(const ImageView& im, int row0, int row1, int hf, int vf, bool fancy, int cu_count,
                        const mjd_tuning& tuning, hipStream_t stream);
// Sub-tile shapes of the single-image kernel per sampling class: how many,
// and one's tile (SX x SY MCUs), lanes, LDS bytes and resident workgroups
// per CU (index < shape_count).
int shape_count(int hf, int vf, bool fancy);
// The decoder variants on the fused path: luma sampling hf x vf ((1,1),
// (2,1), (1,2), (2,2), (4,1)), IDCT method MJD_IDCT_*, the whole image, with
// the tuning's segment length and workgroup count (and shape, for the classes
// whose islow kernel is the single-image kernel's shape list).
hipError_t launch_variant(const ImageView& im, int hf, int vf, bool fancy, int idct, int cu_count,
                          const mjd_tuning& tu, hipStream_t stream);
hipError_t shape_info(int hf, int vf, bool fancy, int index, int* sx, int* sy, int* nt, int* lds_bytes, int* per_cu);

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);

// Validates one job and fills its view (shared by the single-image and batch entries).
int job_view(const mjd_job* j, int upsample, ImageView* im, mjd_geometry* g);

// One queue entry of the batched kernel: a segment of one image.
struct BatchItem {
  int img;
  int cls;
  int mx0, r0, r1;
  int pad[3];
};

// Host plan of a batch: per-image views and the segment queue (longest
// first), with the workgroup count of its launch.
struct BatchPlan {
  std::vector<ImageView> views;
  std::vector<BatchItem> items;
  uint64_t pixels = 0;
  int grid = 0;
};

int batch_plan(mjd_ctx* ctx, const mjd_job* jobs, size_t n, int upsample, BatchPlan* plan);

// Enqueues the persistent batch kernel over tables already on the device.
// d_counters (2 words) must be zero; the kernel leaves them zero.
hipError_t batch_enqueue(const ImageView* d_views, const BatchItem* d_items, int n_items, unsigned* d_counters,
                         int grid, hipStream_t stream);

// Device address of the no-allocation batch scratch on the current device
// (looked up once per device, then cached).
hipError_t noalloc_scratch_address(int device, void** out);

}  // namespace mjd
