// Internal declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <string>

#include "../../include/mjd.h"
#include "decode_kernel.h"

struct mjd_ctx {
  int device = 0;
  int cu_count = 0;
  int xcd_count = 8;
  std::string device_name;
};

namespace mjd {

// Records a thread-local message and returns `code`.
int fail(int code, const char* fmt, ...);

// Host-only frame validation + geometry (no HIP calls).
int frame_geometry(const mjd_frame* f, mjd_geometry* g);

// Enqueues the tile kernel for one image band.
hipError_t launch_image(const ImageParams& p, int hf, int vf, bool fancy, hipStream_t stream);

hipError_t launch_copy(void* dst, const void* src, size_t bytes, hipStream_t stream);

}  // namespace mjd
