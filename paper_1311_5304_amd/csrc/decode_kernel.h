// Fused JPEG back-half kernel for gfx950: dequantise -> 8x8 islow IDCT ->
// chroma upsampling -> YCbCr->RGB -> interleaved RGB8 store.
//
// One workgroup decodes one tile of TMX x TMY MCUs.
//  Phase 1: every lane takes whole 8x8 blocks (the tile's blocks, plus for
//           the fancy filter the chroma blocks of the ring of MCUs around the
//           tile) and runs dequantisation and both IDCT passes in registers
//           (paper Sec. 4.1: columns first, Eq. 1, then rows, Eq. 2).  The
//           uint8 samples land in LDS planes; nothing goes back to HBM.
//  Phase 2: every lane takes a run of 4 chroma samples of one chroma row,
//           upsamples them (Sec. 4.2) and converts each pixel (Sec. 4.3), and
//           stores the RGB bytes (Fig. 5: dword stores of packed RGB).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mjd {

typedef int v4i __attribute__((ext_vector_type(4)));

// --- LL&M 8-point IDCT in 13-bit fixed point --------------------------------
// Each constant is round(2^13 * k).  With a_j = sqrt(2) cos(j*pi/16):
constexpr int kConstBits = 13;
constexpr int kR = 4433;    // a6
constexpr int kR2 = 6270;   // a2 - a6
constexpr int kR6 = 15137;  // a2 + a6
constexpr int kZ5 = 9633;   // a3
constexpr int kP7 = 2446;   // -a1 + a3 + a5 - a7
constexpr int kP5 = 16819;  // a1 + a3 - a5 + a7
constexpr int kP3 = 25172;  // a1 + a3 + a5 - a7
constexpr int kP1 = 12299;  // a1 + a3 - a5 - a7
constexpr int kZ1 = 7373;   // a3 - a7
constexpr int kZ2 = 20995;  // a1 + a3
constexpr int kZ3 = 16069;  // a3 + a5
constexpr int kZ4 = 3196;   // a3 - a5

// 24-bit signed multiply: every multiplicand in the transform is a
// dequantised coefficient, a pass-1 result or a sum of at most four of
// either, all far inside +-2^23 on the documented input domain.
__device__ __forceinline__ int m24(int a, int b) { return __mul24(a, b); }

// One sqrt(8)-scaled 1-D IDCT followed by (v + bias) >> SHIFT on each output.
template <int SHIFT>
__device__ __forceinline__ void idct8(const int x0, const int x1, const int x2, const int x3,
                                      const int x4, const int x5, const int x6, const int x7,
                                      const int bias, int* __restrict__ y, const int stride) {
  // even part: x0, x4 through shifts, (x2, x6) through a 3-multiply rotation
  const int z1 = m24(x2 + x6, kR);
  const int t2 = z1 + m24(x2, kR2);
  const int t3 = z1 - m24(x6, kR6);
  const int t0 = ((x0 + x4) << kConstBits) + bias;
  const int t1 = ((x0 - x4) << kConstBits) + bias;
  const int e0 = t0 + t2, e3 = t0 - t2;
  const int e1 = t1 + t3, e2 = t1 - t3;
  // odd part: LL&M network over pair sums
  const int s17 = x7 + x1, s35 = x5 + x3, s37 = x7 + x3, s15 = x5 + x1;
  const int z5 = m24(s37 + s15, kZ5);
  const int q17 = -m24(s17, kZ1);
  const int q35 = -m24(s35, kZ2);
  const int q37 = z5 - m24(s37, kZ3);
  const int q15 = z5 - m24(s15, kZ4);
  const int o0 = m24(x1, kP1) + q17 + q15;
  const int o1 = m24(x3, kP3) + q35 + q37;
  const int o2 = m24(x5, kP5) + q35 + q15;
  const int o3 = m24(x7, kP7) + q17 + q37;
  y[0 * stride] = (e0 + o0) >> SHIFT;
  y[7 * stride] = (e0 - o0) >> SHIFT;
  y[1 * stride] = (e1 + o1) >> SHIFT;
  y[6 * stride] = (e1 - o1) >> SHIFT;
  y[2 * stride] = (e2 + o2) >> SHIFT;
  y[5 * stride] = (e2 - o2) >> SHIFT;
  y[3 * stride] = (e3 + o3) >> SHIFT;
  y[4 * stride] = (e3 - o3) >> SHIFT;
}

__device__ __forceinline__ int clamp255(int v) { return min(max(v, 0), 255); }

// Dequantise + 2-D IDCT of one block.  coef: 64 int16 natural order (16-byte
// aligned, global); q: 64 int32 dequantisation factors (LDS).  Output: 16
// dwords, two per sample row, bytes in x order (little endian).
__device__ __forceinline__ void decode_block(const int16_t* __restrict__ coef,
                                             const int* __restrict__ q, uint32_t out[16]) {
  int ws[64];
  {
    int d[64];
    const v4i* src = reinterpret_cast<const v4i*>(coef);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const v4i v = __builtin_nontemporal_load(src + r);
      const int w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        d[8 * r + 2 * i] = static_cast<int>(static_cast<int16_t>(w[i] & 0xFFFF)) * q[8 * r + 2 * i];
        d[8 * r + 2 * i + 1] = (w[i] >> 16) * q[8 * r + 2 * i + 1];
      }
    }
    // pass 1: each column (fixed horizontal frequency u) over v = 0..7; keep
    // 2 fraction bits: descale by 13 - 2 with half-LSB rounding
#pragma unroll
    for (int u = 0; u < 8; ++u)
      idct8<kConstBits - 2>(d[u], d[8 + u], d[16 + u], d[24 + u], d[32 + u], d[40 + u], d[48 + u],
                            d[56 + u], 1 << (kConstBits - 2 - 1), ws + u, 8);
  }
  // pass 2: each row of the column results; descale by 13 + 2 + 3, +128, clamp
#pragma unroll
  for (int y = 0; y < 8; ++y) {
    int s[8];
    idct8<kConstBits + 5>(ws[8 * y], ws[8 * y + 1], ws[8 * y + 2], ws[8 * y + 3], ws[8 * y + 4],
                          ws[8 * y + 5], ws[8 * y + 6], ws[8 * y + 7], 1 << (kConstBits + 5 - 1), s, 1);
    uint32_t lo = 0, hi = 0;
#pragma unroll
    for (int x = 0; x < 4; ++x) {
      lo |= static_cast<uint32_t>(clamp255(s[x] + 128)) << (8 * x);
      hi |= static_cast<uint32_t>(clamp255(s[x + 4] + 128)) << (8 * x);
    }
    out[2 * y] = lo;
    out[2 * y + 1] = hi;
  }
}

// --- YCbCr -> RGB, 16 fraction bits ----------------------------------------
// Constants round(2^16 * k) of 1.402, 0.34414, 0.71414, 1.772 (Algorithm 2).
constexpr int kCrR = 91881;
constexpr int kCbG = 22554;
constexpr int kCrG = 46802;
constexpr int kCbB = 116130;

// Returns R | G << 8 | B << 16.
__device__ __forceinline__ uint32_t ycc_rgb(int y, int cb, int cr) {
  const int xb = cb - 128, xr = cr - 128;
  const int r = y + ((m24(xr, kCrR) + 32768) >> 16);
  const int g = y + ((m24(xb, -kCbG) + m24(xr, -kCrG) + 32768) >> 16);
  const int b = y + ((m24(xb, kCbB) + 32768) >> 16);
  return static_cast<uint32_t>(clamp255(r)) | (static_cast<uint32_t>(clamp255(g)) << 8) |
         (static_cast<uint32_t>(clamp255(b)) << 16);
}

// --- launch parameters --------------------------------------------------------
struct ImageParams {
  const int16_t* coef;
  const uint16_t* qt;
  uint8_t* rgb;
  uint64_t pitch;
  uint32_t width, height;
  uint32_t mcus_x, mcus_y;
  uint32_t chroma_w, chroma_h;  // true chroma component size
  uint32_t row0, row1;          // MCU-row band
  uint32_t qsel[3];
  uint32_t tiles_x;             // tiles per tile row
  uint32_t aligned_out;         // rgb base and pitch are multiples of 4
};

}  // namespace mjd
