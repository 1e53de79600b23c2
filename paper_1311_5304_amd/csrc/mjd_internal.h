// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "mjd.h"
#include "mjd_common.h"
#include "segment.h"

struct mjd_ctx {
  int device = 0;
  int cu_count = 0;
  int xcd_count = 8;
  std::string device_name;
  mjd_tuning tuning{0, 0};
};

namespace mjd {

// Enqueues the segment kernel for MCU rows [row0, row1) of one image.
hipError_t launch_image(const ImageView& im, int row0, int row1, int hf, int vf, bool fancy, int cu_count,
                        const mjd_tuning& tuning, hipStream_t stream);

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);

}  // namespace mjd
