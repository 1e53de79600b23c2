// Tile kernel of the fused JPEG back half and its host-side launcher.
//
// One workgroup decodes one tile of TMX x TMY MCUs of one image band:
//  phase 1  dequantise + IDCT (paper Sec. 4.1).  Each lane takes a whole 8x8
//           block of the tile and keeps both passes in registers.  For the
//           fancy filter (Sec. 4.2) the tile also needs one chroma sample of
//           ring around it: those blocks are split 8 lanes per block (one
//           column each in pass 1, as in the paper's kernel) and only the
//           outputs the filter reads are formed -- a full column pass and one
//           output per row for the left/right neighbours, one output per column
//           and one row pass for the neighbours above and below.
//  edges    where the tile holds the true edge of the chroma plane, the
//           samples beyond it are replicated into LDS, so the filter needs no
//           clamping;
//  phase 2  each lane takes 4 chroma samples of one chroma row, upsamples
//           them, converts every covered pixel (Sec. 4.3) and stores the RGB
//           bytes as dwords (Fig. 5).
// Samples live only in LDS; nothing but RGB is written to device memory.
#include "decode_kernel.h"

#include "mjd_internal.h"

namespace mjd {

namespace {

constexpr int round64(int n) { return (n + 63) & ~63; }

__device__ __forceinline__ int clamp255(int v) { return min(max(v, 0), 255); }

__device__ __forceinline__ uint32_t byte_of(uint32_t w, int i) { return (w >> (8 * i)) & 0xFFu; }

}  // namespace

template <int HF, int VF, bool FANCY, int TMX, int TMY, int NT>
__global__ __launch_bounds__(NT) void decode_tiles(const ImageParams p) {
  constexpr int NY = HF * VF;        // luma blocks per MCU
  constexpr int BPM = NY + 2;        // + one Cb, one Cr block
  constexpr bool HALO_X = FANCY && HF == 2;
  constexpr bool HALO_Y = FANCY && VF == 2;
  constexpr int YWD = TMX * 2 * HF;  // luma tile row, dwords
  constexpr int YH = TMY * 8 * VF;
  constexpr int CWD = (TMX + 2) * 2; // chroma tile row, dwords (8-sample margins left and right)
  constexpr int CH = TMY * 8 + 2;    // one-row margins top and bottom
  constexpr int MAX_SIDE = HALO_X ? 4 * TMY : 0;       // left/right neighbour tasks (x2 chroma)
  constexpr int MAX_TB = HALO_Y ? 4 * (TMX + 2) : 0;   // above/below neighbour tasks (x2 chroma)
  __shared__ uint32_t sY[YH * YWD];
  __shared__ uint32_t sC[2][CH * CWD];
  __shared__ __align__(16) uint32_t sQ[3][32];  // uint16 factors, two per dword
  __shared__ int sWS[MAX_SIDE > 0 ? MAX_SIDE * 64 : 1];  // side tasks: pass-1 block [task][row][col]
  __shared__ int sWT[MAX_TB > 0 ? MAX_TB * 8 : 1];       // top/bottom tasks: one pass-1 row [task][col]

  // Workgroups are dealt to the 8 XCDs round-robin; give each XCD a
  // contiguous run of tiles so horizontal neighbours share its L2.
  const uint32_t per_xcd = gridDim.x >> 3;
  const uint32_t t = (blockIdx.x & 7u) * per_xcd + (blockIdx.x >> 3);
  if (t >= p.tiles) return;

  const int tid = threadIdx.x;
  const int mcus_x = p.mcus_x, mcus_y = p.mcus_y;
  const int ty = t / p.tiles_x;
  const int mx0 = (t - ty * p.tiles_x) * TMX;
  const int my0 = p.row0 + ty * TMY;
  const int mx1 = min(mx0 + TMX, mcus_x);
  const int my1 = min(my0 + TMY, static_cast<int>(p.row1));
  const int nmx = mx1 - mx0, nmy = my1 - my0;

  if (tid < 96) {
    const uint16_t* q = p.qt + p.qsel[tid >> 5] * 64 + 2 * (tid & 31);
    sQ[tid >> 5][tid & 31] = static_cast<uint32_t>(q[0]) | (static_cast<uint32_t>(q[1]) << 16);
  }
  __syncthreads();

  uint8_t* const cb8 = reinterpret_cast<uint8_t*>(sC[0]);
  uint8_t* const cr8 = reinterpret_cast<uint8_t*>(sC[1]);

  // coefficient blocks of MCU (mx0 + i, my0 + j) start at tile_coef + (j*mcus_x + i)*BPM*64
  const int16_t* const tile_coef = p.coef + (static_cast<size_t>(my0) * mcus_x + mx0) * (BPM * 64);

  // ---- phase 1 ----
  // Slots: [0, BPM*TM) tile blocks, block kind major (so a wave works on one
  // component), MCU minor; then 8 lanes per left/right neighbour block; then
  // 8 lanes per above/below neighbour block.  Neighbour tasks are numbered
  // (position << 2) | (which side << 1) | chroma component.
  constexpr int TM = TMX * TMY;
  constexpr int N_MAIN = BPM * TM;
  constexpr int A_SIDE = round64(N_MAIN);
  constexpr int A_TB = A_SIDE + round64(8 * MAX_SIDE);
  constexpr int A_END = A_TB + 8 * MAX_TB;
  for (int s = tid; s < A_END; s += NT) {
    if (s < N_MAIN) {
      const int b = s / TM;               // block within the MCU (compile-time power-of-two divisor)
      const int m = s - b * TM;
      const int lmy = m / TMX, lmx = m - (m / TMX) * TMX;
      if (lmx >= nmx || lmy >= nmy) continue;
      const int comp = b < NY ? 0 : b - NY + 1;
      const int16_t* src = tile_coef + (mul24(lmy, mcus_x) + lmx) * (BPM * 64) + b * 64;
      uint32_t o[16];
      decode_block(src, sQ[comp], o);
      if (comp == 0) {
        const int by = b / HF, bx = b - (b / HF) * HF;
        uint32_t* dst = sY + (lmy * 8 * VF + by * 8) * YWD + lmx * 2 * HF + bx * 2;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          dst[r * YWD] = o[2 * r];
          dst[r * YWD + 1] = o[2 * r + 1];
        }
      } else {
        uint32_t* dst = sC[comp - 1] + (lmy * 8 + 1) * CWD + lmx * 2 + 2;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          dst[r * CWD] = o[2 * r];
          dst[r * CWD + 1] = o[2 * r + 1];
        }
      }
    } else if constexpr (HALO_X || HALO_Y) {
      const bool side = s >= A_SIDE && s < A_SIDE + 8 * MAX_SIDE;
      const bool tb = s >= A_TB;
      if (!side && !tb) continue;
      const int task = side ? (s - A_SIDE) >> 3 : (s - A_TB) >> 3;
      const int u = s & 7;  // column of the neighbour block this lane transforms
      const int comp = task & 1;
      const bool far = (task >> 1) & 1;  // right / below
      const int pos = task >> 2;         // tile row (side) or tile column + 1 (top/bottom)
      int mx, my;
      if (side) {
        if (pos >= nmy) continue;
        mx = far ? mx1 : mx0 - 1;
        my = my0 + pos;
      } else {
        if (pos >= nmx + 2) continue;
        mx = mx0 - 1 + pos;
        my = far ? my1 : my0 - 1;
      }
      if (mx < 0 || mx >= mcus_x || my < 0 || my >= mcus_y) continue;
      const int16_t* col = tile_coef + (mul24(my - my0, mcus_x) + (mx - mx0)) * (BPM * 64) + (NY + comp) * 64 + u;
      const uint16_t* q = reinterpret_cast<const uint16_t*>(sQ[1 + comp]) + u;
      int x[8];
#pragma unroll
      for (int v = 0; v < 8; ++v) x[v] = col[8 * v] * static_cast<int>(q[8 * v]);
      if (side) {
        int y[8];
        idct8_raw(x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7], kPass1Bias, y);
#pragma unroll
        for (int i = 0; i < 8; ++i) sWS[task * 64 + i * 8 + u] = y[i] >> kPass1Shift;
      } else {
        // the block above needs its bottom sample row (7), the block below its top row (0)
        const int v = far ? idct8_edge_raw<false>(x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7], kPass1Bias)
                          : idct8_edge_raw<true>(x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7], kPass1Bias);
        sWT[task * 8 + u] = v >> kPass1Shift;
      }
    }
  }

  if constexpr (HALO_X || HALO_Y) {
    __syncthreads();
    // finish the neighbour blocks: left/right tasks one lane per sample row
    // (the column the filter reads: 7 on the left, 0 on the right); above /
    // below tasks one lane per block (a full row pass)
    constexpr int B_TB = round64(8 * MAX_SIDE);
    for (int s = tid; s < B_TB + MAX_TB; s += NT) {
      if (s < 8 * MAX_SIDE) {
        const int task = s >> 3, i = s & 7;
        const bool right = (task >> 1) & 1;
        const int pos = task >> 2;
        const int mx = right ? mx1 : mx0 - 1;
        if (pos >= nmy || mx < 0 || mx >= mcus_x) continue;
        const int* w = sWS + task * 64 + i * 8;
        const int v = right ? idct8_edge_raw<false>(w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7], kPass2Bias)
                            : idct8_edge_raw<true>(w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7], kPass2Bias);
        uint8_t* c8 = (task & 1) ? cr8 : cb8;
        c8[(pos * 8 + 1 + i) * (CWD * 4) + (right ? nmx * 8 + 8 : 7)] =
            static_cast<uint8_t>(clamp255(v >> kPass2Shift));
      } else if (s >= B_TB) {
        const int task = s - B_TB;
        const bool below = (task >> 1) & 1;
        const int pos = task >> 2;
        const int mx = mx0 - 1 + pos;
        const int my = below ? my1 : my0 - 1;
        if (pos >= nmx + 2 || mx < 0 || mx >= mcus_x || my < 0 || my >= mcus_y) continue;
        const int* w = sWT + task * 8;
        int y[8];
        idct8_raw(w[0], w[1], w[2], w[3], w[4], w[5], w[6], w[7], kPass2Bias, y);
#pragma unroll
        for (int i = 0; i < 8; ++i) y[i] >>= kPass2Shift;
        uint32_t* dst = sC[task & 1] + (below ? nmy * 8 + 1 : 0) * CWD + pos * 2;
        dst[0] = pack4(y[0], y[1], y[2], y[3]);
        dst[1] = pack4(y[4], y[5], y[6], y[7]);
      }
    }
  }
  __syncthreads();

  // ---- true chroma edges inside the tile: replicate the edge samples ----
  const int gcx0 = mx0 * 8, gcy0 = my0 * 8;
  const int cw = p.chroma_w, ch = p.chroma_h;
  if constexpr (HALO_X) {
    const bool left = gcx0 == 0;
    const bool right = cw - 1 < gcx0 + 8 * nmx;
    if (left || right) {
      const int rows = nmy * 8 + 2;
      for (int s = tid; s < 2 * 2 * rows; s += NT) {
        const int c = s & 1;
        const int k = s >> 1;
        const bool is_right = k >= rows;
        const int row = is_right ? k - rows : k;
        if (is_right ? !right : !left) continue;
        uint8_t* c8 = (c ? cr8 : cb8) + row * (CWD * 4);
        if (is_right) c8[cw - gcx0 + 8] = c8[cw - 1 - gcx0 + 8];
        else c8[7] = c8[8];
      }
      if constexpr (HALO_Y) __syncthreads();
    }
  }
  if constexpr (HALO_Y) {
    const bool top = gcy0 == 0;
    const bool bottom = ch - 1 < gcy0 + 8 * nmy;
    if (top || bottom) {
      for (int s = tid; s < 2 * 2 * CWD; s += NT) {
        const int c = s & 1;
        const int k = s >> 1;
        const bool is_bottom = k >= CWD;
        const int d = is_bottom ? k - CWD : k;
        if (is_bottom ? !bottom : !top) continue;
        uint32_t* plane = sC[c];
        if (is_bottom) plane[(ch - gcy0 + 1) * CWD + d] = plane[(ch - gcy0) * CWD + d];
        else plane[d] = plane[CWD + d];
      }
    }
  }
  if constexpr (HALO_X || HALO_Y) __syncthreads();

  // ---- phase 2: upsample + colour + store ----
  const int W = p.width, H = p.height;
  // RGB of the tile's first pixel; rows inside a tile are < 2^8 apart and the
  // pitch is < 2^24 bytes, so row offsets are 24-bit products
  uint8_t* const tile_rgb = p.rgb + static_cast<size_t>(gcy0 * VF) * p.pitch + static_cast<size_t>(gcx0 * HF) * 3;
  const int pitch24 = static_cast<int>(p.pitch);
  constexpr int UX = TMX * 2;  // groups of 4 chroma samples per tile row
  for (int uidx = tid; uidx < UX * TMY * 8; uidx += NT) {
    const int cr_l = uidx / UX;  // chroma row within the tile
    const int g = uidx - cr_l * UX;
    if (g >= 2 * nmx || cr_l >= 8 * nmy) continue;
    const int px0 = (gcx0 + 4 * g) * HF;
    const int py0 = (gcy0 + cr_l) * VF;
    if (px0 >= W || py0 >= H) continue;

    int xb[VF][4 * HF], xr[VF][4 * HF];  // chroma - 128 per output pixel
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const uint32_t* plane = sC[c] + (cr_l + 1) * CWD + g + 2;
      int out[VF][4 * HF];
      if constexpr (!FANCY || HF == 1) {
        const uint32_t w = plane[0];
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int dy = 0; dy < VF; ++dy)
#pragma unroll
            for (int dx = 0; dx < HF; ++dx) out[dy][i * HF + dx] = static_cast<int>(byte_of(w, i)) - 128;
      } else {
        // C[-1..4] of each needed chroma row
        int cc[6];
        {
          const uint32_t l = plane[-1], m = plane[0], r = plane[1];
          cc[0] = byte_of(l, 3);
#pragma unroll
          for (int i = 0; i < 4; ++i) cc[1 + i] = byte_of(m, i);
          cc[5] = byte_of(r, 0);
        }
        if constexpr (VF == 1) {
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const int m3 = 3 * cc[1 + i];
            out[0][2 * i] = (m3 + cc[i] - 511) >> 2;          // (3C + Cprev + 1) / 4 - 128
            out[0][2 * i + 1] = (m3 + cc[i + 2] - 510) >> 2;  // (3C + Cnext + 2) / 4 - 128
          }
        } else {
          int su[6], sd[6];
          {
            const uint32_t* up = plane - CWD;
            const uint32_t* dn = plane + CWD;
            const uint32_t ul = up[-1], um = up[0], ur = up[1];
            const uint32_t dl = dn[-1], dm = dn[0], dr = dn[1];
            const int cu[6] = {static_cast<int>(byte_of(ul, 3)), static_cast<int>(byte_of(um, 0)),
                               static_cast<int>(byte_of(um, 1)), static_cast<int>(byte_of(um, 2)),
                               static_cast<int>(byte_of(um, 3)), static_cast<int>(byte_of(ur, 0))};
            const int cd[6] = {static_cast<int>(byte_of(dl, 3)), static_cast<int>(byte_of(dm, 0)),
                               static_cast<int>(byte_of(dm, 1)), static_cast<int>(byte_of(dm, 2)),
                               static_cast<int>(byte_of(dm, 3)), static_cast<int>(byte_of(dr, 0))};
#pragma unroll
            for (int j = 0; j < 6; ++j) {
              const int m3 = 3 * cc[j];
              su[j] = m3 + cu[j];  // unrounded vertical triangle sums
              sd[j] = m3 + cd[j];
            }
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            out[0][2 * i] = (3 * su[1 + i] + su[i] - 2040) >> 4;          // (.. + 8) / 16 - 128
            out[0][2 * i + 1] = (3 * su[1 + i] + su[i + 2] - 2041) >> 4;  // (.. + 7) / 16 - 128
            out[VF - 1][2 * i] = (3 * sd[1 + i] + sd[i] - 2040) >> 4;
            out[VF - 1][2 * i + 1] = (3 * sd[1 + i] + sd[i + 2] - 2041) >> 4;
          }
        }
      }
#pragma unroll
      for (int dy = 0; dy < VF; ++dy)
#pragma unroll
        for (int i = 0; i < 4 * HF; ++i) {
          if (c) xr[dy][i] = out[dy][i];
          else xb[dy][i] = out[dy][i];
        }
    }

    const int nv = min(4 * HF, W - px0);  // valid pixels of this run
#pragma unroll
    for (int dy = 0; dy < VF; ++dy) {
      const int py = py0 + dy;
      if (py >= H) break;
      const uint32_t* yrow = sY + (cr_l * VF + dy) * YWD + g * HF;
      uint32_t w[3 * HF];
#pragma unroll
      for (int k = 0; k < HF; ++k) {
        const uint32_t ydw = yrow[k];
        RGBWide px[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) px[i] = ycc_wide(y16_of(ydw, i), xb[dy][4 * k + i], xr[dy][4 * k + i]);
        pack_rgb4(px, w + 3 * k);
      }
      uint8_t* row = tile_rgb + (mul24(cr_l * VF + dy, pitch24) + 12 * HF * g);
      if (nv == 4 * HF && p.aligned_out) {
        uint32_t* wd = reinterpret_cast<uint32_t*>(row);
#pragma unroll
        for (int k = 0; k < 3 * HF; ++k) wd[k] = w[k];
      } else {
#pragma unroll
        for (int i = 0; i < 12 * HF; ++i)
          if (i < 3 * nv) row[i] = static_cast<uint8_t>(w[i >> 2] >> (8 * (i & 3)));
      }
    }
  }
}

// ---- host launcher ----------------------------------------------------------

template <int HF, int VF, bool FANCY, int TMX, int TMY, int NT>
static hipError_t launch_tiles(ImageParams p, hipStream_t stream) {
  const uint32_t rows = p.row1 - p.row0;
  p.tiles_x = (p.mcus_x + TMX - 1) / TMX;
  const uint64_t tiles = static_cast<uint64_t>(p.tiles_x) * ((rows + TMY - 1) / TMY);
  if (tiles == 0) return hipSuccess;
  if (tiles > 0x7FFFFFF0ull) return hipErrorInvalidValue;
  p.tiles = static_cast<uint32_t>(tiles);
  const uint32_t grid = (p.tiles + 7u) & ~7u;  // whole rounds over the 8 XCDs
  hipLaunchKernelGGL((decode_tiles<HF, VF, FANCY, TMX, TMY, NT>), dim3(grid), dim3(NT), 0, stream, p);
  return hipGetLastError();
}

hipError_t launch_image(const ImageParams& p, int hf, int vf, bool fancy, hipStream_t stream) {
  // Tile shapes: the tile's blocks fill whole waves of the workgroup, and a
  // workgroup's waves divide a CU's wave slots evenly at the kernels' register use.
  if (hf == 1 && vf == 1) return launch_tiles<1, 1, false, 8, 8, 192>(p, stream);
  if (hf == 2 && vf == 1)
    return fancy ? launch_tiles<2, 1, true, 8, 8, 256>(p, stream) : launch_tiles<2, 1, false, 8, 8, 256>(p, stream);
  return fancy ? launch_tiles<2, 2, true, 8, 8, 256>(p, stream) : launch_tiles<2, 2, false, 8, 4, 192>(p, stream);
}

}  // namespace mjd
