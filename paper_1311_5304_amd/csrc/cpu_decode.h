// Internal interface of the host back half (mjd_decode_host), for callers
// that run its bands on threads of their own.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "host_pool.h"
#include "mjd.h"

namespace mjd {
namespace cpu {

// mjd_decode_host with its n_threads bands run as tasks of pf.
int decode_host_with(const mjd_frame* frame, const int16_t* h_coef, const uint16_t* h_qt, int upsample,
                     uint8_t* h_rgb, size_t pitch, uint32_t mcu_row0, uint32_t mcu_row1, int n_threads,
                     const ParallelFor& pf);

}  // namespace cpu
}  // namespace mjd
