// Declarations shared by the device-side and host-side translation units
// (no HIP headers: the host-only sources include this alone).
#pragma once

#include "mjd.h"

namespace mjd {

// Records a thread-local message and returns `code`.
int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));

// Clears the calling thread's message (at the start of each entry point).
void clear_error();

// Host-only frame validation + geometry (no HIP calls).
int frame_geometry(const mjd_frame* f, mjd_geometry* g);

// Geometry of a decoder-variant frame, the workspace its planes need, and
// the planes' pitches and offsets in that workspace (no HIP calls).
int variant_geometry(const mjd_variant* vr, mjd_geometry* g, uint64_t* work, uint32_t plane_pitch[3],
                     uint64_t plane_off[3]);

// HIP device of a context.
int ctx_device(const mjd_ctx* ctx);

}  // namespace mjd
