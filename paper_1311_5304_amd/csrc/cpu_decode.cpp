// The back half of the decoder on host cores: dequantisation, the islow
// (LL&M) 8x8 inverse DCT, chroma upsampling and YCbCr->RGB, for MCU-row
// bands.  It is the CPU side of the paper's CPU-GPU partitioning (Sec. 5.2:
// the CPU decodes the image rows the partition leaves it, while the GPU
// decodes the others), with the same arithmetic as the GPU kernel, so that
// both sides of a partition produce the bytes the whole-image decode would:
// - IDCT (Sec. 4.1, Eqs. 1-2): columns then rows, constants
//   round(k * 2^13), pass 1 keeping 2 fraction bits (descale by 11), pass 2
//   descaling by 18, +128, clamp;
// - fancy upsampling (Sec. 4.2, Algorithm 1): 3:1 triangle weights with
//   clamping at the true component edges; for h2v2 an unrounded vertical
//   sum, then the horizontal filter with rounding constants 8 and 7 on the
//   16x scale;
// - colour (Sec. 4.3, Algorithm 2): constants round(k * 2^16), one rounding
//   per chroma term, clamp.
// Host threads first transform every block row the output needs into shared
// planes, then form the output rows from them, both from queues of small
// tasks.
#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "cpu_decode.h"
#include "host_pool.h"
#include "mjd.h"
#include "mjd_common.h"

namespace mjd {
namespace cpu {

// round(k * 2^13) of the LL&M flowgraph's multipliers, k built from
// a_j = sqrt(2) cos(j pi / 16)
struct IdctConsts {
  int r, r2, r6, z5, p7, p5, p3, p1, z1, z2, z3, z4;
  IdctConsts() {
    double a[8];
    for (int j = 0; j < 8; ++j) a[j] = sqrt(2.0) * cos(j * M_PI / 16.0);
    auto fix = [](double x) { return static_cast<int>(lround(x * 8192.0)); };
    r = fix(a[6]);
    r2 = fix(a[2] - a[6]);
    r6 = fix(a[2] + a[6]);
    z5 = fix(a[3]);
    p7 = fix(-a[1] + a[3] + a[5] - a[7]);
    p5 = fix(a[1] + a[3] - a[5] + a[7]);
    p3 = fix(a[1] + a[3] + a[5] - a[7]);
    p1 = fix(a[1] + a[3] - a[5] - a[7]);
    z1 = fix(a[3] - a[7]);
    z2 = fix(a[1] + a[3]);
    z3 = fix(a[3] + a[5]);
    z4 = fix(a[3] - a[5]);
  }
};

static const IdctConsts& K() {
  static const IdctConsts k;
  return k;
}

// One 8-point LL&M IDCT on x[0], x[s], ..., x[7s]: results scaled by 2^13
// (before descale), written to y[0..7].
static inline void llm8(const int* x, int s, int* y) {
  const IdctConsts& k = K();
  const int x0 = x[0], x1 = x[s], x2 = x[2 * s], x3 = x[3 * s], x4 = x[4 * s], x5 = x[5 * s], x6 = x[6 * s],
            x7 = x[7 * s];
  const int z1 = (x2 + x6) * k.r;
  const int t2 = z1 + x2 * k.r2, t3 = z1 - x6 * k.r6;
  const int t0 = (x0 + x4) * 8192, t1 = (x0 - x4) * 8192;
  const int e0 = t0 + t2, e3 = t0 - t2, e1 = t1 + t3, e2 = t1 - t3;
  const int s17 = x7 + x1, s35 = x5 + x3, s37 = x7 + x3, s15 = x5 + x1;
  const int z5 = (s37 + s15) * k.z5;
  const int q17 = -s17 * k.z1, q35 = -s35 * k.z2, q37 = z5 - s37 * k.z3, q15 = z5 - s15 * k.z4;
  const int o0 = x1 * k.p1 + q17 + q15, o1 = x3 * k.p3 + q35 + q37, o2 = x5 * k.p5 + q35 + q15,
            o3 = x7 * k.p7 + q17 + q37;
  y[0] = e0 + o0;
  y[7] = e0 - o0;
  y[1] = e1 + o1;
  y[6] = e1 - o1;
  y[2] = e2 + o2;
  y[5] = e2 - o2;
  y[3] = e3 + o3;
  y[4] = e3 - o3;
}

// Dequantise + IDCT of one block (natural order) into an 8x8 sample tile at
// dst (row stride `stride`).
static void idct_block(const int16_t* c, const uint16_t* q, uint8_t* dst, size_t stride) {
  int d[64], ws[64], col[8], row[8];
  for (int i = 0; i < 64; ++i) d[i] = static_cast<int>(c[i]) * static_cast<int>(q[i]);
  for (int u = 0; u < 8; ++u) {  // column u: frequencies v = 0..7 at d[8v + u]
    llm8(d + u, 8, col);
    for (int y = 0; y < 8; ++y) ws[8 * y + u] = (col[y] + (1 << 10)) >> 11;
  }
  for (int y = 0; y < 8; ++y) {
    llm8(ws + 8 * y, 1, row);
    for (int x = 0; x < 8; ++x) {
      const int v = ((row[x] + (1 << 17)) >> 18) + 128;
      dst[y * stride + x] = static_cast<uint8_t>(v < 0 ? 0 : (v > 255 ? 255 : v));
    }
  }
}

struct Plan {
  mjd_frame f;
  mjd_geometry g;
  int hmax, vmax;
  int bw[3], first[3];  // blocks per component row; first block of the component in an MCU
  int bpm;
};

// Block rows [br0, br1) of component c, transformed into `plane` (stride
// bw*8 samples, plane row 0 = sample row 8*br0).
struct CompPlane {
  std::vector<uint8_t> plane;
  int br0 = 0, br1 = 0;
  size_t stride = 0;
};

static void decode_block_row(const Plan& p, const int16_t* coef, const uint16_t* qt, int c, int br,
                             CompPlane* out) {
  const int hc = p.f.h[c], vc = p.f.v[c];
  const uint16_t* q = qt + 64 * p.f.qsel[c];
  const int my = br / vc, by = br % vc;
  uint8_t* dst = &out->plane[static_cast<size_t>(br - out->br0) * 8 * out->stride];
  for (int bx = 0; bx < p.bw[c]; ++bx) {
    const int mx = bx / hc, bxi = bx % hc;
    const size_t mcu = static_cast<size_t>(my) * p.g.mcus_x + mx;
    const int16_t* blk = coef + (mcu * p.bpm + p.first[c] + by * hc + bxi) * 64;
    idct_block(blk, q, dst + 8 * bx, out->stride);
  }
}

// Output pixel rows [y0, y1) of the image from the transformed planes, row
// y at rgb + y * pitch.
static void output_rows(const Plan& p, const CompPlane* planes, bool fancy, int y0, int y1, uint8_t* rgb,
                        size_t pitch) {
  const int W = static_cast<int>(p.f.width);
  int fhs[3], fvs[3];
  for (int c = 0; c < 3; ++c) {
    fhs[c] = p.hmax / p.f.h[c];
    fvs[c] = p.vmax / p.f.v[c];
  }
  std::vector<int> up[3];
  for (int c = 0; c < 3; ++c) up[c].resize(W);
  std::vector<int> srow;
  // the planes' rows as plain pointers (the output stores are byte stores,
  // which may alias anything the loops would otherwise reload)
  const uint8_t* base[3];
  size_t stride[3];
  int row0[3];
  for (int c = 0; c < 3; ++c) {
    base[c] = planes[c].plane.data();
    stride[c] = planes[c].stride;
    row0[c] = 8 * planes[c].br0;
  }
  for (int y = y0; y < y1; ++y) {
    for (int c = 0; c < 3; ++c) {
      const uint8_t* const pl = base[c];
      const size_t st = stride[c];
      const int rz = row0[c];
      const int fh = fhs[c], fv = fvs[c], cw = static_cast<int>(p.g.comp_w[c]), ch = static_cast<int>(p.g.comp_h[c]);
      auto at = [=](int r, int x) { return static_cast<int>(pl[(r - rz) * st + x]); };
      int* o = up[c].data();
      if (fh == 1 && fv == 1) {
        for (int x = 0; x < W; ++x) o[x] = at(y, x);
      } else if (!fancy) {
        for (int x = 0; x < W; ++x) o[x] = at(y / fv, x / fh);
      } else if (fv == 1) {  // h2v1: Algorithm 1 along the row
        for (int x = 0; x < W; ++x) {
          const int k = x >> 1;
          const int m = at(y, k);
          o[x] = (x & 1) ? (3 * m + at(y, std::min(k + 1, cw - 1)) + 2) >> 2 : (3 * m + at(y, std::max(k - 1, 0)) + 1) >> 2;
        }
      } else {  // h2v2: vertical sum, then the horizontal filter
        const int r = y >> 1;
        const int rn = (y & 1) ? std::min(r + 1, ch - 1) : std::max(r - 1, 0);
        srow.resize(cw);
        for (int k = 0; k < cw; ++k) srow[k] = 3 * at(r, k) + at(rn, k);
        for (int x = 0; x < W; ++x) {
          const int k = x >> 1;
          o[x] = (x & 1) ? (3 * srow[k] + srow[std::min(k + 1, cw - 1)] + 7) >> 4
                         : (3 * srow[k] + srow[std::max(k - 1, 0)] + 8) >> 4;
        }
      }
    }
    uint8_t* out = rgb + static_cast<size_t>(y) * pitch;
    for (int x = 0; x < W; ++x) {
      const int yy = up[0][x], xb = up[1][x] - 128, xr = up[2][x] - 128;
      const int r = yy + ((91881 * xr + 32768) >> 16);
      const int g = yy + ((-22554 * xb - 46802 * xr + 32768) >> 16);
      const int b = yy + ((116130 * xb + 32768) >> 16);
      out[3 * x] = static_cast<uint8_t>(r < 0 ? 0 : (r > 255 ? 255 : r));
      out[3 * x + 1] = static_cast<uint8_t>(g < 0 ? 0 : (g > 255 ? 255 : g));
      out[3 * x + 2] = static_cast<uint8_t>(b < 0 ? 0 : (b > 255 ? 255 : b));
    }
  }
}

}  // namespace cpu
}  // namespace mjd

int mjd::cpu::decode_host_with(const mjd_frame* frame, const int16_t* h_coef, const uint16_t* h_qt, int upsample,
                               uint8_t* h_rgb, size_t pitch, uint32_t mcu_row0, uint32_t mcu_row1, int n_threads,
                               const ParallelFor& pf) {
  using namespace mjd::cpu;
  if (!frame || !h_coef || !h_qt || !h_rgb) return mjd::fail(MJD_EINVAL, "null frame or buffer pointer");
  if (upsample != MJD_UPSAMPLE_SIMPLE && upsample != MJD_UPSAMPLE_FANCY)
    return mjd::fail(MJD_EINVAL, "upsample mode %d unknown", upsample);
  Plan p;
  p.f = *frame;
  int rc = mjd::frame_geometry(frame, &p.g);
  if (rc != MJD_OK) return rc;
  if (pitch < 3ull * frame->width) return mjd::fail(MJD_EINVAL, "pitch below 3*width");
  if (mcu_row0 > mcu_row1 || mcu_row1 > p.g.mcus_y) return mjd::fail(MJD_EINVAL, "MCU rows out of range");
  if (n_threads < 1 || n_threads > 256) return mjd::fail(MJD_EINVAL, "thread count outside 1..256");
  if (mcu_row0 == mcu_row1) return MJD_OK;
  p.hmax = std::max({frame->h[0], frame->h[1], frame->h[2]});
  p.vmax = std::max({frame->v[0], frame->v[1], frame->v[2]});
  p.bpm = 0;
  for (int c = 0; c < 3; ++c) {
    p.first[c] = p.bpm;
    p.bpm += frame->h[c] * frame->v[c];
    p.bw[c] = static_cast<int>(p.g.mcus_x) * frame->h[c];
  }
  const int mh = static_cast<int>(p.g.mcu_h);
  const int H = static_cast<int>(frame->height);
  const bool fancy = upsample == MJD_UPSAMPLE_FANCY;
  // The rows go in chunks of about 4 MCU rows per thread, so the planes of
  // a chunk stay in the caches between its two phases.  Phase 1: every
  // block row the chunk's output rows read (for fancy vertical filtering
  // one chroma row above and below), transformed once into planes the
  // threads share; a block row the previous chunk already holds is copied
  // from it.  Phase 2: the output rows in bands of 8.  Both phases hand out
  // small tasks, so a thread that is held up delays the chunk by one task at
  // most.
  const int nrows = static_cast<int>(mcu_row1 - mcu_row0);
  const int max_chunk = std::max(8, 4 * n_threads);
  const int n_chunks = (nrows + max_chunk - 1) / max_chunk;
  CompPlane bufs[2][3];
  struct Task {
    int c, br;
    bool copy;
  };
  std::vector<Task> tasks;
  for (int k = 0; k < n_chunks; ++k) {
    CompPlane* cur = bufs[k & 1];
    const CompPlane* prev = k ? bufs[(k - 1) & 1] : nullptr;
    const int ra = static_cast<int>(mcu_row0) + nrows * k / n_chunks;
    const int rb = static_cast<int>(mcu_row0) + nrows * (k + 1) / n_chunks;
    const int y0 = ra * mh, y1 = std::min(H, rb * mh);
    tasks.clear();
    for (int c = 0; c < 3; ++c) {
      const int fv = p.vmax / frame->v[c];
      const int ch = static_cast<int>(p.g.comp_h[c]);
      int r0 = y0 / fv, r1 = (y1 - 1) / fv + 1;
      if (fancy && fv == 2) {
        r0 = std::max(0, r0 - 1);
        r1 = std::min(ch, r1 + 1);
      }
      CompPlane& cp = cur[c];
      cp.br0 = r0 / 8;
      cp.br1 = (r1 + 7) / 8;
      cp.stride = static_cast<size_t>(p.bw[c]) * 8;
      cp.plane.resize(static_cast<size_t>(cp.br1 - cp.br0) * 8 * cp.stride);
      for (int br = cp.br0; br < cp.br1; ++br)
        tasks.push_back(Task{c, br, prev && br >= prev[c].br0 && br < prev[c].br1});
    }
    pf(static_cast<int>(tasks.size()), [&](int t) {
      const Task& tk = tasks[t];
      CompPlane& cp = cur[tk.c];
      if (tk.copy) {
        const size_t n = 8 * cp.stride;
        memcpy(&cp.plane[(tk.br - cp.br0) * n], &prev[tk.c].plane[(tk.br - prev[tk.c].br0) * n], n);
      } else {
        decode_block_row(p, h_coef, h_qt, tk.c, tk.br, &cp);
      }
    });
    constexpr int kBand = 8;
    pf((y1 - y0 + kBand - 1) / kBand, [&](int t) {
      const int ya = y0 + kBand * t;
      output_rows(p, cur, fancy, ya, std::min(y1, ya + kBand), h_rgb, pitch);
    });
  }
  return MJD_OK;
}

extern "C" int mjd_decode_host(const mjd_frame* frame, const int16_t* h_coef, const uint16_t* h_qt, int upsample,
                               uint8_t* h_rgb, size_t pitch, uint32_t mcu_row0, uint32_t mcu_row1, int n_threads) {
  if (n_threads < 1 || n_threads > 256) return mjd::fail(MJD_EINVAL, "thread count outside 1..256");
  // threads for the whole call (each decode runs several parallel loops)
  mjd::WorkerPool pool(n_threads);
  return mjd::cpu::decode_host_with(frame, h_coef, h_qt, upsample, h_rgb, pitch, mcu_row0, mcu_row1, n_threads,
                                    [&pool](int n, const mjd::TaskFn& fn) { pool.run(n, fn); });
}
