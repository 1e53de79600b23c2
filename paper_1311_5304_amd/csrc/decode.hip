// Tile kernel of the fused JPEG back half (see decode_kernel.h) and its
// host-side launcher.
#include "decode_kernel.h"

#include "mjd_internal.h"

namespace mjd {

template <int HF, int VF, bool FANCY, int TMX, int TMY>
__global__ __launch_bounds__(256) void decode_tiles(const ImageParams p) {
  constexpr int NT = 256;
  constexpr int NY = HF * VF;       // luma blocks per MCU
  constexpr int BPM = NY + 2;       // + one Cb, one Cr block
  constexpr bool HALO_X = FANCY && HF == 2;
  constexpr bool HALO_Y = FANCY && VF == 2;
  constexpr int YW = TMX * 8 * HF;  // luma tile, bytes per row
  constexpr int YH = TMY * 8 * VF;
  constexpr int CW = (TMX + 2) * 8; // chroma tile: 8-sample margins left and right
  constexpr int CH = TMY * 8 + 2;   // one-row margins top and bottom
  __shared__ uint32_t sY[YH * YW / 4];
  __shared__ uint32_t sC[2][CH * CW / 4];
  __shared__ int sQ[3][64];

  const int tid = threadIdx.x;
  const int tx = blockIdx.x % p.tiles_x;
  const int ty = blockIdx.x / p.tiles_x;
  const int mcus_x = p.mcus_x, mcus_y = p.mcus_y;
  const int mx0 = tx * TMX;
  const int my0 = p.row0 + ty * TMY;
  const int mx1 = min(mx0 + TMX, mcus_x);
  const int my1 = min(my0 + TMY, static_cast<int>(p.row1));
  const int nmx = mx1 - mx0, nmy = my1 - my0;

  if (tid < 192) sQ[tid >> 6][tid & 63] = p.qt[p.qsel[tid >> 6] * 64 + (tid & 63)];
  __syncthreads();

  // ---- phase 1: dequantise + IDCT, one block per lane per round ----
  const int n_main = nmx * nmy * BPM;
  const int n_ring_y = HALO_Y ? 2 * (nmx + 2) : 0;  // ring rows above and below (incl. corners)
  const int n_ring_x = HALO_X ? 2 * nmy : 0;        // ring columns left and right
  const int n_jobs = n_main + 2 * (n_ring_y + n_ring_x);
  for (int j = tid; j < n_jobs; j += NT) {
    int mx, my, b, kind = 0;  // kind: 0 tile block, 1 ring above, 2 below, 3 left/right
    if (j < n_main) {
      const int m = j / BPM;
      b = j - m * BPM;
      const int lmy = m / nmx;
      mx = mx0 + (m - lmy * nmx);
      my = my0 + lmy;
    } else {
      int r = j - n_main;
      b = NY + (r & 1);
      r >>= 1;
      if (r < n_ring_y) {
        const bool below = r >= nmx + 2;
        mx = mx0 - 1 + (below ? r - (nmx + 2) : r);
        my = below ? my1 : my0 - 1;
        kind = below ? 2 : 1;
      } else {
        r -= n_ring_y;
        const bool right = r >= nmy;
        mx = right ? mx1 : mx0 - 1;
        my = my0 + (right ? r - nmy : r);
        kind = 3;
      }
      if (mx < 0 || mx >= mcus_x || my < 0 || my >= mcus_y) continue;
    }
    const int comp = b < NY ? 0 : b - NY + 1;
    const int16_t* src = p.coef + (static_cast<size_t>(my) * mcus_x + mx) * (BPM * 64) + b * 64;
    uint32_t s[16];
    decode_block(src, sQ[comp], s);
    if (comp == 0) {
      const int by = b / HF, bx = b - (b / HF) * HF;
      uint32_t* dst = sY + ((my - my0) * 8 * VF + by * 8) * (YW / 4) + ((mx - mx0) * 8 * HF + bx * 8) / 4;
#pragma unroll
      for (int r = 0; r < 8; ++r) {
        dst[r * (YW / 4)] = s[2 * r];
        dst[r * (YW / 4) + 1] = s[2 * r + 1];
      }
    } else {
      // chroma row my*8 sits at LDS row (my - my0)*8 + 1; column mx*8 at (mx - mx0)*8 + 8
      uint32_t* dst = sC[comp - 1] + ((my - my0) * 8 + 1) * (CW / 4) + ((mx - mx0) * 8 + 8) / 4;
      if (kind == 1) {         // only the bottom sample row is needed
        dst[7 * (CW / 4)] = s[14];
        dst[7 * (CW / 4) + 1] = s[15];
      } else if (kind == 2) {  // only the top sample row is needed
        dst[0] = s[0];
        dst[1] = s[1];
      } else {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          dst[r * (CW / 4)] = s[2 * r];
          dst[r * (CW / 4) + 1] = s[2 * r + 1];
        }
      }
    }
  }
  __syncthreads();

  // ---- phase 2: upsample + colour + store, 4 chroma samples per lane per round ----
  const uint8_t* y8 = reinterpret_cast<const uint8_t*>(sY);
  const uint8_t* cb8 = reinterpret_cast<const uint8_t*>(sC[0]);
  const uint8_t* cr8 = reinterpret_cast<const uint8_t*>(sC[1]);
  const int cx_org = mx0 * 8 - 8;  // global chroma column of LDS column 0
  const int cy_org = my0 * 8 - 1;  // global chroma row of LDS row 0
  const int cw_max = static_cast<int>(p.chroma_w) - 1;
  const int ch_max = static_cast<int>(p.chroma_h) - 1;
  const int units_x = nmx * 2;
  const int n_units = units_x * nmy * 8;
  const int W = p.width, H = p.height;
  for (int u = tid; u < n_units; u += NT) {
    const int cr_l = u / units_x;            // chroma row within the tile
    const int g = u - cr_l * units_x;        // group of 4 chroma columns
    const int gcy = my0 * 8 + cr_l;
    const int gcx = mx0 * 8 + 4 * g;
    const int px0 = gcx * HF;
    const int py0 = gcy * VF;
    if (px0 >= W || py0 >= H) continue;

    // chroma values for the unit's VF output rows and 4*HF output columns
    int cbv[VF][4 * HF], crv[VF][4 * HF];
    if constexpr (!FANCY || (HF == 1 && VF == 1)) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int off = (gcy - cy_org) * CW + (gcx + i - cx_org);
        const int b_ = cb8[off], r_ = cr8[off];
#pragma unroll
        for (int dy = 0; dy < VF; ++dy)
#pragma unroll
          for (int dx = 0; dx < HF; ++dx) {
            cbv[dy][i * HF + dx] = b_;
            crv[dy][i * HF + dx] = r_;
          }
      }
    } else {
      // neighbour columns gcx-1 .. gcx+4 and rows gcy-1 .. gcy+1, clamped at
      // the true chroma edge
      int col[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) col[i] = min(max(gcx - 1 + i, 0), cw_max) - cx_org;
      const int rm = (min(max(gcy - 1, 0), ch_max) - cy_org) * CW;
      const int r0 = (gcy - cy_org) * CW;
      const int rp = (min(gcy + 1, ch_max) - cy_org) * CW;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const uint8_t* C = c ? cr8 : cb8;
        int out[VF][8];
        if constexpr (VF == 1) {
          int v[6];
#pragma unroll
          for (int i = 0; i < 6; ++i) v[i] = C[r0 + col[i]];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            out[0][2 * i] = (3 * v[i + 1] + v[i] + 1) >> 2;
            out[0][2 * i + 1] = (3 * v[i + 1] + v[i + 2] + 2) >> 2;
          }
        } else {
          int su[6], sd[6];
#pragma unroll
          for (int i = 0; i < 6; ++i) {
            const int m3 = 3 * C[r0 + col[i]];
            su[i] = m3 + C[rm + col[i]];
            sd[i] = m3 + C[rp + col[i]];
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            out[0][2 * i] = (3 * su[i + 1] + su[i] + 8) >> 4;
            out[0][2 * i + 1] = (3 * su[i + 1] + su[i + 2] + 7) >> 4;
            out[VF - 1][2 * i] = (3 * sd[i + 1] + sd[i] + 8) >> 4;
            out[VF - 1][2 * i + 1] = (3 * sd[i + 1] + sd[i + 2] + 7) >> 4;
          }
        }
#pragma unroll
        for (int dy = 0; dy < VF; ++dy)
#pragma unroll
          for (int i = 0; i < 4 * HF; ++i) {
            if (c) crv[dy][i] = out[dy][i];
            else cbv[dy][i] = out[dy][i];
          }
      }
    }

    const int ly0 = cr_l * VF;                       // luma row within the tile
    const int lx0 = 4 * g * HF;
    const int nv = min(4 * HF, W - px0);             // valid pixels in this run
#pragma unroll
    for (int dy = 0; dy < VF; ++dy) {
      const int py = py0 + dy;
      if (py >= H) break;
      uint32_t pix[4 * HF];
#pragma unroll
      for (int i = 0; i < 4 * HF; ++i)
        pix[i] = ycc_rgb(y8[(ly0 + dy) * YW + lx0 + i], cbv[dy][i], crv[dy][i]);
      uint8_t* row = p.rgb + static_cast<size_t>(py) * p.pitch + static_cast<size_t>(px0) * 3;
      if (nv == 4 * HF && p.aligned_out) {
        uint32_t* w = reinterpret_cast<uint32_t*>(row);
#pragma unroll
        for (int k = 0; k < HF; ++k) {
          const uint32_t a = pix[4 * k], b_ = pix[4 * k + 1], c_ = pix[4 * k + 2], d_ = pix[4 * k + 3];
          w[3 * k] = a | (b_ << 24);
          w[3 * k + 1] = (b_ >> 8) | (c_ << 16);
          w[3 * k + 2] = (c_ >> 16) | (d_ << 8);
        }
      } else {
        for (int i = 0; i < nv; ++i) {
          row[3 * i] = static_cast<uint8_t>(pix[i]);
          row[3 * i + 1] = static_cast<uint8_t>(pix[i] >> 8);
          row[3 * i + 2] = static_cast<uint8_t>(pix[i] >> 16);
        }
      }
    }
  }
}

// ---- host launcher ----------------------------------------------------------

template <int HF, int VF, bool FANCY, int TMX, int TMY>
static hipError_t launch_tiles(ImageParams p, hipStream_t stream) {
  const uint32_t rows = p.row1 - p.row0;
  p.tiles_x = (p.mcus_x + TMX - 1) / TMX;
  const uint32_t tiles_y = (rows + TMY - 1) / TMY;
  const uint64_t n = static_cast<uint64_t>(p.tiles_x) * tiles_y;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((decode_tiles<HF, VF, FANCY, TMX, TMY>), dim3(static_cast<uint32_t>(n)), dim3(256), 0,
                     stream, p);
  return hipGetLastError();
}

hipError_t launch_image(const ImageParams& p, int hf, int vf, bool fancy, hipStream_t stream) {
  if (hf == 1 && vf == 1) return launch_tiles<1, 1, false, 8, 8>(p, stream);
  if (hf == 2 && vf == 1)
    return fancy ? launch_tiles<2, 1, true, 8, 6>(p, stream) : launch_tiles<2, 1, false, 8, 6>(p, stream);
  return fancy ? launch_tiles<2, 2, true, 8, 4>(p, stream) : launch_tiles<2, 2, false, 8, 4>(p, stream);
}

}  // namespace mjd
