// Device building blocks of the fused JPEG back-half kernel for gfx950:
// dequantise -> 8x8 islow IDCT -> chroma upsampling -> YCbCr->RGB -> RGB8.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mjd {

typedef int v4i __attribute__((ext_vector_type(4)));

// --- LL&M 8-point IDCT in 13-bit fixed point --------------------------------
// Each constant is round(2^13 * k).  With a_j = sqrt(2) cos(j*pi/16), the
// sqrt(8)-scaled 1-D IDCT is y[n] = x0 + sum_{k>=1} sqrt(2) cos((2n+1)k pi/16) x_k.
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

// Pass 1 keeps two extra fraction bits; pass 2 removes them, the 2-D gain of
// 8 and the constants' 2^13, and adds the +128 level shift through its
// rounding bias ((v + 2^17 + 128*2^18) >> 18 == ((v + 2^17) >> 18) + 128).
constexpr int kPass1Shift = kConstBits - 2;
constexpr int kPass2Shift = kConstBits + 2 + 3;
constexpr int kPass1Bias = 1 << (kPass1Shift - 1);
constexpr int kPass2Bias = (1 << (kPass2Shift - 1)) + (128 << kPass2Shift);

// 24-bit signed multiply(-add).  Every multiplicand of the transform is a
// dequantised coefficient, a pass-1 result, or a sum of at most four of them;
// on the documented input domain all stay inside +-2^23, so the 24-bit forms
// (full-rate v_mul_i32_i24 / v_mad_i32_i24) are exact.
// mad24 pins v_mad_i32_i24: left to itself the compiler may pick the
// quarter-rate v_mad_u64_u32 for a 32-bit multiply-add.  `b` is always a
// compile-time constant here and travels in an SGPR.
__device__ __forceinline__ int mul24(int a, int b) { return __mul24(a, b); }
__device__ __forceinline__ int mad24(int a, int b, int c) {
  int r;
  asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(b), "v"(c));
  return r;
}

// One sqrt(8)-scaled 1-D IDCT; returns the 8 outputs before the descale
// shift, with `bias` already added.
__device__ __forceinline__ void idct8_raw(const int x0, const int x1, const int x2, const int x3,
                                          const int x4, const int x5, const int x6, const int x7,
                                          const int bias, int y[8]) {
  // even part: x0, x4 through shifts; (x2, x6) through a 3-multiply rotation
  const int z1 = mul24(x2 + x6, kR);
  const int t2 = mad24(x2, kR2, z1);            // a2*x2 + a6*x6
  const int t3 = mad24(x6, -kR6, z1);           // a6*x2 - a2*x6
  const int t0 = ((x0 + x4) << kConstBits) + bias;
  const int t1 = mad24(x4, -(2 << kConstBits), t0);  // ((x0 - x4) << 13) + bias
  const int e0 = t0 + t2, e3 = t0 - t2;
  const int e1 = t1 + t3, e2 = t1 - t3;
  // odd part: the LL&M network over pair sums
  const int s17 = x7 + x1, s35 = x5 + x3, s37 = x7 + x3, s15 = x5 + x1;
  const int z5 = mul24(s37 + s15, kZ5);
  const int q17 = mul24(s17, -kZ1);
  const int q35 = mul24(s35, -kZ2);
  const int q37 = mad24(s37, -kZ3, z5);
  const int q15 = mad24(s15, -kZ4, z5);
  const int o0 = mad24(x1, kP1, q17 + q15);
  const int o1 = mad24(x3, kP3, q35 + q37);
  const int o2 = mad24(x5, kP5, q35 + q15);
  const int o3 = mad24(x7, kP7, q17 + q37);
  y[0] = e0 + o0;
  y[7] = e0 - o0;
  y[1] = e1 + o1;
  y[6] = e1 - o1;
  y[2] = e2 + o2;
  y[5] = e2 - o2;
  y[3] = e3 + o3;
  y[4] = e3 - o3;
}

// Output 0 (LAST = false) or output 7 (LAST = true) of idct8_raw alone.
template <bool LAST>
__device__ __forceinline__ int idct8_edge_raw(const int x0, const int x1, const int x2, const int x3,
                                              const int x4, const int x5, const int x6, const int x7,
                                              const int bias) {
  const int z1 = mul24(x2 + x6, kR);
  const int e0 = ((x0 + x4) << kConstBits) + bias + mad24(x2, kR2, z1);
  const int s15 = x5 + x1;
  const int z5 = mul24(x7 + x3 + s15, kZ5);
  const int o0 = mad24(x1, kP1, mad24(x7 + x1, -kZ1, mad24(s15, -kZ4, z5)));
  return LAST ? e0 - o0 : e0 + o0;
}

// Saturating pack of two int16-range ints to bytes: returns sat(a) | sat(b) << 8.
__device__ __forceinline__ uint32_t sat_u8x2(int a, int b) {
  const uint32_t pair = __builtin_amdgcn_perm(static_cast<uint32_t>(b), static_cast<uint32_t>(a), 0x05040100u);
  uint32_t r;
  asm("v_sat_pk_u8_i16 %0, %1" : "=v"(r) : "v"(pair));
  return r;
}

// The two saturated bytes of the int16 pair `pair` written into bytes 2..3
// of `lo`, whose bytes 0..1 are kept (an SDWA word write in place of a
// shift-or).
__device__ __forceinline__ uint32_t sat_u8x2_into_hi(uint32_t lo, uint32_t pair) {
  asm("v_sat_pk_u8_i16_sdwa %0, %1 dst_sel:WORD_1 dst_unused:UNUSED_PRESERVE src0_sel:DWORD"
      : "+v"(lo) : "v"(pair));
  return lo;
}

// (a >> 16, b >> 16) as an int16 pair (arithmetic shifts, one byte permute).
__device__ __forceinline__ uint32_t hi_halves(int a, int b) {
  return __builtin_amdgcn_perm(static_cast<uint32_t>(b), static_cast<uint32_t>(a), 0x07060302u);
}

// Same, from the high halves: sat(a >> 16) | sat(b >> 16) << 8 (a and b must
// lie in +-2^31 with (x >> 16) inside int16).
__device__ __forceinline__ uint32_t sat_u8x2_hi(int a, int b) {
  uint32_t r;
  asm("v_sat_pk_u8_i16 %0, %1" : "=v"(r) : "v"(hi_halves(a, b)));
  return r;
}

__device__ __forceinline__ uint32_t pack4(int s0, int s1, int s2, int s3) {
  return sat_u8x2(s0, s1) | (sat_u8x2(s2, s3) << 16);
}

// Four raw pass-2 sums -> four clamped samples (sum >> kPass2Shift) as bytes.
// (v >> 16) >> 2 == v >> 18 for arithmetic shifts, so the high halves are
// gathered first and shifted as int16 pairs.
__device__ __forceinline__ uint32_t descale_pack4(int s0, int s1, int s2, int s3) {
  typedef short i16x2 __attribute__((ext_vector_type(2)));
  const i16x2 sh = {kPass2Shift - 16, kPass2Shift - 16};
  const uint32_t p01 = __builtin_bit_cast(uint32_t, __builtin_bit_cast(i16x2, hi_halves(s0, s1)) >> sh);
  const uint32_t p23 = __builtin_bit_cast(uint32_t, __builtin_bit_cast(i16x2, hi_halves(s2, s3)) >> sh);
  uint32_t r;
  asm("v_sat_pk_u8_i16 %0, %1" : "=v"(r) : "v"(p01));
  return sat_u8x2_into_hi(r, p23);
}

// --- pass 1 as int16 dot products -------------------------------------------
// Before its descale shift the flowgraph is exact integer arithmetic (sums
// and multiplications by constants), so each of its outputs is an integer
// linear form in the 8 inputs.  Expanding the network gives the weights
// below; all of them, and on the documented domain every dequantised
// coefficient, fit int16, so v_dot2_i32_i16 forms two terms per instruction
// with an exact 32-bit sum.  The rows of the weight matrix are
// y_k = e_k + o_k and y_{7-k} = e_k - o_k.
constexpr int kE2a = kR + kR2;   // x2 in e0 (and -x2 in e3)
constexpr int kE6a = kR;         // x6 in e0
constexpr int kE2b = kR;         // x2 in e1 (and -x2 in e2)
constexpr int kE6b = kR - kR6;   // x6 in e1
// odd weights: o_k = sum_j kO[k][j] * x_{2j+1}
constexpr int kO[4][4] = {
    {kP1 - kZ1 - kZ4 + kZ5, kZ5, kZ5 - kZ4, kZ5 - kZ1},
    {kZ5, kP3 - kZ2 - kZ3 + kZ5, kZ5 - kZ2, kZ5 - kZ3},
    {kZ5 - kZ4, kZ5 - kZ2, kP5 - kZ2 - kZ4 + kZ5, kZ5},
    {kZ5 - kZ1, kZ5 - kZ3, kZ5, kP7 - kZ1 - kZ3 + kZ5},
};

constexpr uint32_t wpair(int lo, int hi) {
  return static_cast<uint32_t>(static_cast<uint16_t>(lo)) | (static_cast<uint32_t>(static_cast<uint16_t>(hi)) << 16);
}

// lo(a) * lo(w) + hi(a) * hi(w) + c over int16 halves (v_dot2_i32_i16, no
// clamp); the weight pair travels in an SGPR.
__device__ __forceinline__ int dot2(uint32_t a, uint32_t w, int c) {
  int r;
  asm("v_dot2_i32_i16 %0, %1, %2, %3" : "=v"(r) : "v"(a), "s"(w), "v"(c));
  return r;
}
__device__ __forceinline__ int dot2z(uint32_t a, uint32_t w) {
  int r;
  asm("v_dot2_i32_i16 %0, %1, %2, 0" : "=v"(r) : "v"(a), "s"(w));
  return r;
}

// One column of pass 1 from the input pairs (x0, x4), (x2, x6), (x1, x3),
// (x5, x7); y[] as idct8_raw returns it (bias included, before the shift).
__device__ __forceinline__ void idct8_dot(uint32_t p04, uint32_t p26, uint32_t p13, uint32_t p57,
                                          int bias, int y[8]) {
  const int t0 = dot2(p04, wpair(1 << kConstBits, 1 << kConstBits), bias);
  const int t1 = dot2(p04, wpair(1 << kConstBits, -(1 << kConstBits)), bias);
  const int e0 = dot2(p26, wpair(kE2a, kE6a), t0);
  const int e3 = dot2(p26, wpair(-kE2a, -kE6a), t0);
  const int e1 = dot2(p26, wpair(kE2b, kE6b), t1);
  const int e2 = dot2(p26, wpair(-kE2b, -kE6b), t1);
  const int o0 = dot2(p13, wpair(kO[0][0], kO[0][1]), dot2z(p57, wpair(kO[0][2], kO[0][3])));
  const int o1 = dot2(p13, wpair(kO[1][0], kO[1][1]), dot2z(p57, wpair(kO[1][2], kO[1][3])));
  const int o2 = dot2(p13, wpair(kO[2][0], kO[2][1]), dot2z(p57, wpair(kO[2][2], kO[2][3])));
  const int o3 = dot2(p13, wpair(kO[3][0], kO[3][1]), dot2z(p57, wpair(kO[3][2], kO[3][3])));
  y[0] = e0 + o0;
  y[7] = e0 - o0;
  y[1] = e1 + o1;
  y[6] = e1 - o1;
  y[2] = e2 + o2;
  y[5] = e2 - o2;
  y[3] = e3 + o3;
  y[4] = e3 - o3;
}

// Dequantise + 2-D IDCT of one block (paper Sec. 4.1: columns first, Eq. 1,
// then rows, Eq. 2).  rows: the block's 8 coefficient rows (8 int16 each, in
// registers); q: the 64 uint16 factors as 32 dwords (in LDS, 16-byte aligned).
// out: 16 dwords, two per sample row (x order, little endian), samples
// level-shifted and clamped to 0..255.
__device__ __forceinline__ void idct_block_regs(const v4i rows[8], const __attribute__((address_space(3))) uint32_t* q,
                                                uint32_t out[16]) {
  typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
  int ws[64];
  {
    // dequantised pairs (coefficient row r, columns 2i and 2i + 1): the low
    // 16 bits of each product, exact as int16 on the documented domain
    uint32_t d[8][4];
    const __attribute__((address_space(3))) v4i* qv = reinterpret_cast<const __attribute__((address_space(3))) v4i*>(q);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const v4i v = rows[r];
      const v4i qq = qv[r];
      const int w[4] = {v.x, v.y, v.z, v.w};
      const int qw[4] = {qq.x, qq.y, qq.z, qq.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
        d[r][i] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, w[i]) * __builtin_bit_cast(u16x2, qw[i]));
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      // the column's pairs (row a, row b) from the halves of two row dwords
      const int i = u >> 1;
      const uint32_t sel = (u & 1) ? 0x07060302u : 0x05040100u;
      int y[8];
      idct8_dot(__builtin_amdgcn_perm(d[4][i], d[0][i], sel), __builtin_amdgcn_perm(d[6][i], d[2][i], sel),
                __builtin_amdgcn_perm(d[3][i], d[1][i], sel), __builtin_amdgcn_perm(d[7][i], d[5][i], sel),
                kPass1Bias, y);
#pragma unroll
      for (int k = 0; k < 8; ++k) ws[8 * k + u] = y[k] >> kPass1Shift;
    }
  }
#pragma unroll
  for (int r = 0; r < 8; ++r) {
    int s[8];
    idct8_raw(ws[8 * r], ws[8 * r + 1], ws[8 * r + 2], ws[8 * r + 3], ws[8 * r + 4], ws[8 * r + 5],
              ws[8 * r + 6], ws[8 * r + 7], kPass2Bias, s);
    out[2 * r] = descale_pack4(s[0], s[1], s[2], s[3]);
    out[2 * r + 1] = descale_pack4(s[4], s[5], s[6], s[7]);
  }
}

// --- both passes as int16 dot products ---------------------------------------
// The row pass can also run on v_dot2_i32_i16 when every pass-1 result fits
// int16.  That holds whenever every dequantised coefficient lies in
// [-1024, 1023]: each pass-1 output is a linear form whose weights sum in
// magnitude to at most 61214, so |sum| < 61214 * 1024 + 1024 < 2^26 and the
// descaled value (sum >> 11) stays inside +-30607.  A conforming 8-bit
// stream stays far inside (pass 1 of an exact DCT is bounded by 4096, and
// quantisation adds at most Q/2 per coefficient).  A wave that holds a block
// outside that range takes the int32 row pass instead, so the result is the
// same on the whole documented domain.
//
// Scaled pass 1: inputs d' = 16 d (a 16-bit product with 16 Q) and doubled
// weights give 32 times the pass-1 sum, so its high half is already the
// descaled value (floor(32 s / 2^16) == floor(s / 2^11)) and one byte
// permute packs two results as the int16 pair the row pass needs.  Each
// input carries a bias of 2^14 (d' + 2^14 lies in [0, 2^15) exactly when d
// lies in [-1024, 1023], so an OR over all pairs tests the range through
// bits 15 and 31); the bias's contribution to every output is a constant,
// folded into the first accumulator of each chain.
constexpr int kInBias = 1 << 14;
constexpr int kP1ScaledBias = 1 << 15;  // 32 * 2^10
constexpr uint32_t kInBiasPair = (static_cast<uint32_t>(kInBias) << 16) | static_cast<uint32_t>(kInBias);

// Even part of output k (x0, x4, x2, x6 weights; k = 0..3) and odd part
// (x1, x3, x5, x7 weights) of the flowgraph's linear form, before doubling.
constexpr int kEw[4][4] = {
    {1 << kConstBits, 1 << kConstBits, kE2a, kE6a},
    {1 << kConstBits, -(1 << kConstBits), kE2b, kE6b},
    {1 << kConstBits, -(1 << kConstBits), -kE2b, -kE6b},
    {1 << kConstBits, 1 << kConstBits, -kE2a, -kE6a},
};
constexpr int even_corr(int k) {
  return kP1ScaledBias - kInBias * 2 * (kEw[k][0] + kEw[k][1] + kEw[k][2] + kEw[k][3]);
}
constexpr int odd_corr(int k) { return -kInBias * 2 * (kO[k][0] + kO[k][1] + kO[k][2] + kO[k][3]); }

// One column of the scaled pass 1 from biased pairs (x0, x4), (x2, x6),
// (x1, x3), (x5, x7): y[n] = 32 * (pass-1 sum of output n, rounding bias
// included), exact in 32 bits (every partial sum stays inside +-2^31).
template <int K>
__device__ __forceinline__ void p1_outputs(uint32_t p04, uint32_t p26, uint32_t p13, uint32_t p57, int y[8]) {
  const int e = dot2(p26, wpair(2 * kEw[K][2], 2 * kEw[K][3]),
                     dot2(p04, wpair(2 * kEw[K][0], 2 * kEw[K][1]), even_corr(K)));
  const int o = dot2(p13, wpair(2 * kO[K][0], 2 * kO[K][1]),
                     dot2(p57, wpair(2 * kO[K][2], 2 * kO[K][3]), odd_corr(K)));
  y[K] = e + o;
  y[7 - K] = e - o;
}
__device__ __forceinline__ void idct8_p1_scaled(uint32_t p04, uint32_t p26, uint32_t p13, uint32_t p57, int y[8]) {
  p1_outputs<0>(p04, p26, p13, p57, y);
  p1_outputs<1>(p04, p26, p13, p57, y);
  p1_outputs<2>(p04, p26, p13, p57, y);
  p1_outputs<3>(p04, p26, p13, p57, y);
}

// Dequantise + 2-D IDCT of one block (Sec. 4.1: columns first, Eq. 1, then
// rows, Eq. 2) as idct_block_regs computes it, with both passes as dot
// products when the whole wave's blocks allow it.  q16: the block's 64
// factors times 16 as 32 dwords of uint16 pairs (LDS, 16-byte aligned).
__device__ __forceinline__ void idct_block_fast(const v4i rows[8], const __attribute__((address_space(3))) uint32_t* q,
                                                const __attribute__((address_space(3))) uint32_t* q16,
                                                uint32_t out[16]) {
  typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
  uint32_t e[8][4];
  uint32_t any = 0;
  {
    const __attribute__((address_space(3))) v4i* qv = reinterpret_cast<const __attribute__((address_space(3))) v4i*>(q16);
    const u16x2 bias = __builtin_bit_cast(u16x2, kInBiasPair);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const v4i v = rows[r];
      const v4i qq = qv[r];
      const int w[4] = {v.x, v.y, v.z, v.w};
      const int qw[4] = {qq.x, qq.y, qq.z, qq.w};
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        e[r][i] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, w[i]) * __builtin_bit_cast(u16x2, qw[i]) + bias);
        any |= e[r][i];
      }
    }
  }
  if (__builtin_amdgcn_ballot_w64((any & 0x80008000u) != 0) != 0) {
    idct_block_regs(rows, q, out);
    return;
  }
  // pass 1 by column pairs (0,4), (2,6), (1,3), (5,7): the two columns'
  // results for sample row n form the pair the row pass reads for row n
  // (pr[0] (x0, x4), pr[1] (x2, x6), pr[2] (x1, x3), pr[3] (x5, x7)).  The
  // pairs are formed in the order (0,4), (1,3), (5,7), (2,6), which retires
  // the input dwords of e[][0], then e[][2], then the rest.
  uint32_t pr[4][8];
#pragma unroll
  for (int step = 0; step < 4; ++step) {
    const int cp = step == 0 ? 0 : (step == 1 ? 2 : (step == 2 ? 3 : 1));
    const int ua = cp == 0 ? 0 : (cp == 1 ? 2 : (cp == 2 ? 1 : 5));
    const int ub = cp == 0 ? 4 : (cp == 1 ? 6 : (cp == 2 ? 3 : 7));
    int ya[8], yb[8];
    {
      const int i = ua >> 1;
      const uint32_t sel = (ua & 1) ? 0x07060302u : 0x05040100u;
      idct8_p1_scaled(__builtin_amdgcn_perm(e[4][i], e[0][i], sel), __builtin_amdgcn_perm(e[6][i], e[2][i], sel),
                      __builtin_amdgcn_perm(e[3][i], e[1][i], sel), __builtin_amdgcn_perm(e[7][i], e[5][i], sel), ya);
    }
    {
      const int i = ub >> 1;
      const uint32_t sel = (ub & 1) ? 0x07060302u : 0x05040100u;
      idct8_p1_scaled(__builtin_amdgcn_perm(e[4][i], e[0][i], sel), __builtin_amdgcn_perm(e[6][i], e[2][i], sel),
                      __builtin_amdgcn_perm(e[3][i], e[1][i], sel), __builtin_amdgcn_perm(e[7][i], e[5][i], sel), yb);
    }
#pragma unroll
    for (int n = 0; n < 8; ++n) pr[cp][n] = hi_halves(ya[n], yb[n]);
  }
  // pass 2: the same linear forms on the int16 pairs
#pragma unroll
  for (int n = 0; n < 8; ++n) {
    int s[8];
    idct8_dot(pr[0][n], pr[1][n], pr[2][n], pr[3][n], kPass2Bias, s);
    out[2 * n] = descale_pack4(s[0], s[1], s[2], s[3]);
    out[2 * n + 1] = descale_pack4(s[4], s[5], s[6], s[7]);
  }
}

// --- YCbCr -> RGB, 16 fraction bits ----------------------------------------
// Constants round(2^16 * k) of 1.402, 0.34414, 0.71414, 1.772 (Algorithm 2).
constexpr int kCrR = 91881;
constexpr int kCbG = 22554;
constexpr int kCrG = 46802;
constexpr int kCbB = 116130;

// y16 = (Y << 16) + 2^15; xb = Cb - 128, xr = Cr - 128.  The channel value
// before clamping is the high half of each returned word:
// Y + ((K*x + 2^15) >> 16) == ((Y << 16) + 2^15 + K*x) >> 16.
struct RGBWide {
  int r, g, b;
};
__device__ __forceinline__ RGBWide ycc_wide(int y16, int xb, int xr) {
  return {mad24(xr, kCrR, y16), mad24(xb, -kCbG, mad24(xr, -kCrG, y16)), mad24(xb, kCbB, y16)};
}

// Y byte i (0..3) of `ydw` as (Y << 16) + 2^15, in one byte permute.
__device__ __forceinline__ int y16_of(uint32_t ydw, int i) {
  return static_cast<int>(__builtin_amdgcn_perm(0x80808080u, ydw, 0x0C00040Cu | (static_cast<uint32_t>(i) << 16)));
}

// Four pixels -> 12 RGB bytes as 3 dwords (paper Fig. 5: pixel bytes grouped
// into 4-byte vectors).
__device__ __forceinline__ void pack_rgb4(const RGBWide p[4], uint32_t w[3]) {
  w[0] = sat_u8x2_into_hi(sat_u8x2_hi(p[0].r, p[0].g), hi_halves(p[0].b, p[1].r));
  w[1] = sat_u8x2_into_hi(sat_u8x2_hi(p[1].g, p[1].b), hi_halves(p[2].r, p[2].g));
  w[2] = sat_u8x2_into_hi(sat_u8x2_hi(p[2].b, p[3].r), hi_halves(p[3].g, p[3].b));
}

}  // namespace mjd
