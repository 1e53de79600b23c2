// C ABI entry points: validation, geometry, context, dispatch.
#include <stdarg.h>
#include <stdio.h>

#include <new>

#include "mjd_internal.h"

namespace mjd {

int ctx_device(const mjd_ctx* ctx) { return ctx->device; }

int job_view(const mjd_job* j, int upsample, ImageView* im, mjd_geometry* g) {
  if (!j) return fail(MJD_EINVAL, "null job");
  int rc = frame_geometry(&j->frame, g);
  if (rc != MJD_OK) return rc;
  if (!j->d_coef || !j->d_qt || !j->d_rgb) return fail(MJD_EINVAL, "null device buffer");
  if (reinterpret_cast<uintptr_t>(j->d_coef) % 16) return fail(MJD_EINVAL, "coefficient buffer not 16-byte aligned");
  if (reinterpret_cast<uintptr_t>(j->d_qt) % 2) return fail(MJD_EINVAL, "quant table buffer not 2-byte aligned");
  if (upsample != MJD_UPSAMPLE_SIMPLE && upsample != MJD_UPSAMPLE_FANCY)
    return fail(MJD_EINVAL, "upsample mode %d unknown", upsample);
  if (j->pitch < 3ull * j->frame.width) return fail(MJD_EINVAL, "pitch %zu < 3*width", j->pitch);
  if (j->pitch >= (1ull << 24)) return fail(MJD_EINVAL, "pitch %zu not below 2^24 bytes", j->pitch);
  im->coef = j->d_coef;
  im->qt = j->d_qt;
  im->rgb = j->d_rgb;
  im->pitch = static_cast<uint32_t>(j->pitch);
  im->width = static_cast<int>(j->frame.width);
  im->height = static_cast<int>(j->frame.height);
  im->mcus_x = static_cast<int>(g->mcus_x);
  im->mcus_y = static_cast<int>(g->mcus_y);
  im->chroma_w = static_cast<int>(g->comp_w[1]);
  im->chroma_h = static_cast<int>(g->comp_h[1]);
  im->qsel0 = j->frame.qsel[0];
  im->qsel1 = j->frame.qsel[1];
  im->qsel2 = j->frame.qsel[2];
  return MJD_OK;
}

}  // namespace mjd

extern "C" {

int mjd_ctx_create(mjd_ctx** out, int device) {
  mjd::clear_error();
  if (!out) return mjd::fail(MJD_EINVAL, "null context out-pointer");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n == 0) return mjd::fail(MJD_EDEVICE, "no HIP device: %s", hipGetErrorString(e));
  if (device < 0 || device >= n) return mjd::fail(MJD_EINVAL, "device %d outside 0..%d", device, n - 1);
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return mjd::fail(MJD_EDEVICE, "hipGetDeviceProperties: %s", hipGetErrorString(e));
  mjd_ctx* ctx = new (std::nothrow) mjd_ctx;
  if (!ctx) return mjd::fail(MJD_ENOMEM, "context allocation failed");
  ctx->device = device;
  ctx->cu_count = prop.multiProcessorCount;
  ctx->device_name = prop.gcnArchName;
  e = mjd::noalloc_scratch_address(device, &ctx->noalloc_scratch);
  if (e != hipSuccess) {
    delete ctx;
    return mjd::fail(MJD_EDEVICE, "scratch address on device %d: %s", device, hipGetErrorString(e));
  }
  *out = ctx;
  return MJD_OK;
}

void mjd_ctx_destroy(mjd_ctx* ctx) {
  if (!ctx) return;
  int cur = 0;
  if (hipGetDevice(&cur) == hipSuccess && cur != ctx->device) (void)hipSetDevice(ctx->device);
  (void)hipDeviceSynchronize();
  if (cur != ctx->device) (void)hipSetDevice(cur);
  delete ctx;
}

int mjd_decode(mjd_ctx* ctx, const mjd_frame* frame, const int16_t* d_coef, const uint16_t* d_qt,
               int upsample, uint8_t* d_rgb, size_t pitch, uint32_t mcu_row0, uint32_t mcu_row1,
               void* stream) {
  mjd::clear_error();
  if (!ctx) return mjd::fail(MJD_EINVAL, "null context");
  if (!frame) return mjd::fail(MJD_EINVAL, "null frame");
  mjd_job job{*frame, d_coef, d_qt, d_rgb, pitch};
  mjd::ImageView im{};
  mjd_geometry g;
  int rc = mjd::job_view(&job, upsample, &im, &g);
  if (rc != MJD_OK) return rc;
  if (mcu_row0 >= mcu_row1 || mcu_row1 > g.mcus_y)
    return mjd::fail(MJD_EINVAL, "MCU rows [%u,%u) not inside [0,%u)", mcu_row0, mcu_row1, g.mcus_y);
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) {
    if (hipSetDevice(ctx->device) != hipSuccess) return mjd::fail(MJD_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
  }
  hipError_t e = mjd::launch_image(im, static_cast<int>(mcu_row0), static_cast<int>(mcu_row1), frame->h[0],
                                   frame->v[0], upsample == MJD_UPSAMPLE_FANCY, ctx->cu_count, ctx->tuning,
                                   static_cast<hipStream_t>(stream));
  if (cur != ctx->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return mjd::fail(MJD_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return MJD_OK;
}

int mjd_ctx_set_tuning(mjd_ctx* ctx, const mjd_tuning* tuning) {
  mjd::clear_error();
  if (!ctx || !tuning) return mjd::fail(MJD_EINVAL, "null context or tuning");
  if (tuning->seg_subtiles > 65536 || tuning->workgroups > (1u << 20) || tuning->shape > 255)
    return mjd::fail(MJD_EINVAL, "tuning values out of range");
  ctx->tuning = *tuning;
  return MJD_OK;
}

int mjd_ctx_get_tuning(const mjd_ctx* ctx, mjd_tuning* tuning) {
  mjd::clear_error();
  if (!ctx || !tuning) return mjd::fail(MJD_EINVAL, "null context or tuning");
  *tuning = ctx->tuning;
  return MJD_OK;
}

static int shape_class(uint32_t h, uint32_t v, int upsample) {
  if (upsample != MJD_UPSAMPLE_SIMPLE && upsample != MJD_UPSAMPLE_FANCY)
    return mjd::fail(MJD_EINVAL, "upsample mode %d unknown", upsample);
  if (!((h == 1 && v == 1) || (h == 2 && v == 1) || (h == 2 && v == 2)))
    return mjd::fail(MJD_EUNSUPPORTED, "no fused kernel for luma sampling %ux%u", h, v);
  return MJD_OK;
}

int mjd_shape_count(uint32_t h, uint32_t v, int upsample, uint32_t* count) {
  mjd::clear_error();
  if (!count) return mjd::fail(MJD_EINVAL, "null count");
  const int rc = shape_class(h, v, upsample);
  if (rc != MJD_OK) return rc;
  *count = static_cast<uint32_t>(mjd::shape_count(static_cast<int>(h), static_cast<int>(v), upsample == MJD_UPSAMPLE_FANCY));
  return MJD_OK;
}

int mjd_shape_info(mjd_ctx* ctx, uint32_t h, uint32_t v, int upsample, uint32_t index, mjd_shape* out) {
  mjd::clear_error();
  if (!ctx || !out) return mjd::fail(MJD_EINVAL, "null context or shape");
  const int rc = shape_class(h, v, upsample);
  if (rc != MJD_OK) return rc;
  const bool fancy = upsample == MJD_UPSAMPLE_FANCY;
  const int n = mjd::shape_count(static_cast<int>(h), static_cast<int>(v), fancy);
  if (index >= static_cast<uint32_t>(n)) return mjd::fail(MJD_EINVAL, "shape %u outside 0..%d", index, n - 1);
  int cur = 0;
  (void)hipGetDevice(&cur);
  if (cur != ctx->device) (void)hipSetDevice(ctx->device);
  int sx, sy, nt, lds, per_cu;
  const hipError_t e = mjd::shape_info(static_cast<int>(h), static_cast<int>(v), fancy, static_cast<int>(index), &sx,
                                       &sy, &nt, &lds, &per_cu);
  if (cur != ctx->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return mjd::fail(MJD_EDEVICE, "occupancy query failed: %s", hipGetErrorString(e));
  out->mcus_x = static_cast<uint32_t>(sx);
  out->mcus_y = static_cast<uint32_t>(sy);
  out->threads = static_cast<uint32_t>(nt);
  out->lds_bytes = static_cast<uint32_t>(lds);
  out->resident_per_cu = static_cast<uint32_t>(per_cu);
  out->cu_count = static_cast<uint32_t>(ctx->cu_count);
  return MJD_OK;
}

int mjd_copy(mjd_ctx* ctx, void* d_dst, const void* d_src, size_t bytes, void* stream) {
  mjd::clear_error();
  if (!ctx) return mjd::fail(MJD_EINVAL, "null context");
  if (!d_dst || !d_src) return mjd::fail(MJD_EINVAL, "null device buffer");
  if (reinterpret_cast<uintptr_t>(d_dst) % 16 || reinterpret_cast<uintptr_t>(d_src) % 16 || bytes % 16)
    return mjd::fail(MJD_EINVAL, "copy buffers and size must be multiples of 16 bytes");
  if (bytes == 0) return MJD_OK;
  hipError_t e = mjd::launch_copy(d_dst, d_src, bytes, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return mjd::fail(MJD_EDEVICE, "copy launch failed: %s", hipGetErrorString(e));
  return MJD_OK;
}

}  // extern "C"
