// Declarations shared by the device-side and host-side translation units
// (no HIP headers: the host-only sources include this alone).
#pragma once

#include "mjd.h"

namespace mjd {

// Records a thread-local message and returns `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// Host-only frame validation + geometry (no HIP calls).
int frame_geometry(const mjd_frame* f, mjd_geometry* g);

// HIP device of a context.
int ctx_device(const mjd_ctx* ctx);

}  // namespace mjd
