// Host-only parts of the C ABI shared by every translation unit: the
// thread-local error message, frame validation and geometry (no HIP).
#include <stdarg.h>
#include <stdio.h>

#include "mjd_common.h"

namespace {
thread_local char g_err[512] = "";
}

namespace mjd {

void clear_error() { g_err[0] = 0; }

int fail(int code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

int frame_geometry(const mjd_frame* f, mjd_geometry* g) {
  if (!f || !g) return fail(MJD_EINVAL, "null frame or geometry pointer");
  if (f->width < 1 || f->width > 65535 || f->height < 1 || f->height > 65535)
    return fail(MJD_EINVAL, "image size %ux%u outside 1..65535", f->width, f->height);
  for (int c = 0; c < 3; ++c) {
    if (f->h[c] < 1 || f->h[c] > 4 || f->v[c] < 1 || f->v[c] > 4)
      return fail(MJD_EINVAL, "component %d sampling factors (%u,%u) outside 1..4", c, f->h[c], f->v[c]);
    if (f->qsel[c] > 3) return fail(MJD_EINVAL, "component %d quant table selector %u > 3", c, f->qsel[c]);
  }
  if (f->reserved != 0) return fail(MJD_EINVAL, "reserved frame field must be 0");
  const bool luma_ok = (f->h[0] == 1 && f->v[0] == 1) || (f->h[0] == 2 && f->v[0] == 1) ||
                       (f->h[0] == 2 && f->v[0] == 2);
  if (!luma_ok || f->h[1] != 1 || f->v[1] != 1 || f->h[2] != 1 || f->v[2] != 1)
    return fail(MJD_EUNSUPPORTED, "sampling Y(%u,%u) Cb(%u,%u) Cr(%u,%u) not supported (4:4:4, 4:2:2, 4:2:0 only)",
                f->h[0], f->v[0], f->h[1], f->v[1], f->h[2], f->v[2]);
  const uint32_t hmax = f->h[0], vmax = f->v[0];
  g->mcu_w = 8 * hmax;
  g->mcu_h = 8 * vmax;
  g->mcus_x = (f->width + g->mcu_w - 1) / g->mcu_w;
  g->mcus_y = (f->height + g->mcu_h - 1) / g->mcu_h;
  g->blocks_per_mcu = hmax * vmax + 2;
  for (int c = 0; c < 3; ++c) {
    g->comp_w[c] = (f->width * f->h[c] + hmax - 1) / hmax;
    g->comp_h[c] = (f->height * f->v[c] + vmax - 1) / vmax;
  }
  g->n_blocks = static_cast<uint64_t>(g->mcus_x) * g->mcus_y * g->blocks_per_mcu;
  return MJD_OK;
}

// Geometry of a variant frame and the workspace its planes need.
int variant_geometry(const mjd_variant* vr, mjd_geometry* g, uint64_t* work, uint32_t plane_pitch[3],
                            uint64_t plane_off[3]) {
  if (!vr || !g) return fail(MJD_EINVAL, "null variant or geometry pointer");
  const mjd_frame& f = vr->frame;
  if (f.reserved != 0) return fail(MJD_EINVAL, "reserved frame field must be 0");
  const uint32_t scale = vr->scale ? vr->scale : 1;
  if (scale != 1 && scale != 2 && scale != 4 && scale != 8)
    return fail(MJD_EINVAL, "scale 1/%u is not 1, 1/2, 1/4 or 1/8", vr->scale);
  if (f.width < 1 || f.width > 65535 || f.height < 1 || f.height > 65535)
    return fail(MJD_EINVAL, "image size %ux%u outside 1..65535", f.width, f.height);
  if (vr->ncomp != 1 && vr->ncomp != 3) return fail(MJD_EINVAL, "ncomp %u is neither 1 nor 3", vr->ncomp);
  if (vr->idct != MJD_IDCT_ISLOW && vr->idct != MJD_IDCT_IFAST && vr->idct != MJD_IDCT_FLOAT)
    return fail(MJD_EINVAL, "IDCT method %d unknown", vr->idct);
  if (vr->upsample != MJD_UPSAMPLE_SIMPLE && vr->upsample != MJD_UPSAMPLE_FANCY)
    return fail(MJD_EINVAL, "upsample mode %d unknown", vr->upsample);
  if (scale > 1 && vr->idct != MJD_IDCT_ISLOW)
    return fail(MJD_EUNSUPPORTED, "scaled decoding has the islow-style reduced transform only");
  const int nc = static_cast<int>(vr->ncomp);
  for (int c = 0; c < nc; ++c)
    if (f.qsel[c] > 3) return fail(MJD_EINVAL, "component %d quant table selector %u > 3", c, f.qsel[c]);
  uint32_t hy = 1, vy = 1;
  if (nc == 3) {
    hy = f.h[0];
    vy = f.v[0];
    const bool luma_ok = (hy == 1 && vy == 1) || (hy == 2 && vy == 1) || (hy == 1 && vy == 2) ||
                         (hy == 2 && vy == 2) || (hy == 4 && vy == 1);
    if (!luma_ok || f.h[1] != 1 || f.v[1] != 1 || f.h[2] != 1 || f.v[2] != 1)
      return fail(MJD_EUNSUPPORTED, "sampling Y(%u,%u) Cb(%u,%u) Cr(%u,%u) not supported", f.h[0], f.v[0], f.h[1],
                  f.v[1], f.h[2], f.v[2]);
  }
  g->mcu_w = 8 * hy;
  g->mcu_h = 8 * vy;
  g->mcus_x = (f.width + g->mcu_w - 1) / g->mcu_w;
  g->mcus_y = (f.height + g->mcu_h - 1) / g->mcu_h;
  g->blocks_per_mcu = nc == 1 ? 1 : hy * vy + 2;
  g->n_blocks = static_cast<uint64_t>(g->mcus_x) * g->mcus_y * g->blocks_per_mcu;
  // component sizes at the output scale; planes of whole blocks of n
  // samples, rows padded to 16 bytes
  const uint32_t n = 8 / scale;
  uint64_t total = 0;
  for (int c = 0; c < 3; ++c) {
    const uint32_t hc = c == 0 ? hy : 1, vc = c == 0 ? vy : 1;
    const uint32_t cw = (f.width * hc + hy - 1) / hy, ch = (f.height * vc + vy - 1) / vy;
    g->comp_w[c] = c < nc ? (cw + scale - 1) / scale : 0;
    g->comp_h[c] = c < nc ? (ch + scale - 1) / scale : 0;
    plane_pitch[c] = (g->mcus_x * hc * n + 15) & ~15u;
    plane_off[c] = total;
    // full-size colour images decode in one fused pass: no planes
    if (nc == 3 && scale > 1) total += (static_cast<uint64_t>(plane_pitch[c]) * g->mcus_y * vc * n + 255) & ~255ull;
  }
  *work = total;
  return MJD_OK;
}

}  // namespace mjd

extern "C" {

const char* mjd_last_error(void) { return g_err; }

int mjd_geometry_of(const mjd_frame* frame, mjd_geometry* out) {
  g_err[0] = 0;
  return mjd::frame_geometry(frame, out);
}


int mjd_variant_geometry(const mjd_variant* variant, mjd_geometry* out, uint64_t* work_bytes) {
  uint32_t pp[3];
  uint64_t po[3], wb = 0;
  mjd_geometry g;
  const int rc = mjd::variant_geometry(variant, &g, &wb, pp, po);
  if (rc != MJD_OK) return rc;
  if (out) *out = g;
  if (work_bytes) *work_bytes = wb;
  return MJD_OK;
}

}  // extern "C"
