// The AAN-based 8-point IDCTs of the decoder variants (the paper notes that
// libjpeg builds its IDCT from AAN 1-D transforms, in integer or floating
// point, Sec. 2 and Sec. 3): the transposed AAN flowgraph, outputs in
// sample order from inputs in frequency order, sums taken left to right.
//   ifast: fixed point, multipliers q * 2^6 / (s(u) s(v)) (s(0) = 1,
//          s(k) = sqrt(2) cos(k pi / 16)), 9-bit constants with truncating
//          products, output ((v + 2^8) >> 9) + 128;
//   float: IEEE single precision, multipliers fp32(q / (8 s(u) s(v))), one
//          rounding per operation in the order written (no fused
//          multiply-adds), output floor(v + 128.5).
// Both the two-launch variant kernels and the fused segment decoder use
// these.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace mjd {

constexpr int kIfastFrac = 6;
constexpr int kIfastConstBits = 9;
constexpr int kIfastShift = kIfastFrac + 3;

// Scale factors and constants of the AAN methods, computed once on the host
// with the C library's cos and passed to the kernels by value.
struct AanConsts {
  double ss8[64];   // 8 * (s(u) * s(v)), index 8u + v
  int32_t a14[64];  // round(2^14 / (s(u) * s(v)))
  int32_t ki[4];    // round(c * 2^9) of cos(pi/4), cos(3pi/8), cos(pi/8) -+ cos(3pi/8)
  float kf[4];      // the same constants in fp32
};
const AanConsts& aan_consts();

// Dequantisation multiplier of coefficient e (0..63) for quantiser q:
// ifast in fixed point, float as the bits of an fp32.
__device__ __forceinline__ int32_t aan_ifast_mult(uint32_t q, int e, const AanConsts& k) {
  return static_cast<int32_t>((static_cast<int64_t>(q) * k.a14[e] + (1 << (13 - kIfastFrac))) >> (14 - kIfastFrac));
}
__device__ __forceinline__ int32_t aan_float_mult(uint32_t q, int e, const AanConsts& k) {
  return __float_as_int(static_cast<float>(static_cast<double>(q) / k.ss8[e]));
}

// The ifast products in 24-bit multiplies, exact on the input domain
// (|coefficient * q| <= 1155):
// - in the graph every intermediate, products included, is below 2^30 in
//   magnitude, so each operand is below 2^30 / 196 < 2^23 (196 =
//   round(cos(3 pi/8) 2^9) is the smallest constant);
// - in the dequantisation a nonzero coefficient has q <= 1155, so its
//   multiplier is below 1155 * 2^14 / (s(7) s(7)) / 2^8 < 2^20, and a zero
//   coefficient gives 0 whatever the multiplier.
struct IfastOps {
  int r, c5, c2, c4;
  __device__ int mul_r(int v) const { return __mul24(v, r) >> kIfastConstBits; }
  __device__ int mul_c5(int v) const { return __mul24(v, c5) >> kIfastConstBits; }
  __device__ int mul_c2(int v) const { return __mul24(v, c2) >> kIfastConstBits; }
  __device__ int mul_c4(int v) const { return __mul24(v, c4) >> kIfastConstBits; }
};
struct FloatOps {
  float r, c5, c2, c4;
  __device__ float mul_r(float v) const { return v * r; }
  __device__ float mul_c5(float v) const { return v * c5; }
  __device__ float mul_c2(float v) const { return v * c2; }
  __device__ float mul_c4(float v) const { return v * c4; }
};

__device__ __forceinline__ int aan_add(int a, int b) { return a + b; }
__device__ __forceinline__ int aan_sub(int a, int b) { return a - b; }
__device__ __forceinline__ float aan_add(float a, float b) {
#pragma clang fp contract(off)
  return a + b;
}
__device__ __forceinline__ float aan_sub(float a, float b) {
#pragma clang fp contract(off)
  return a - b;
}

template <class T, class Ops>
__device__ __forceinline__ void aan8(const T y[8], T x[8], const Ops& k) {
#pragma clang fp contract(off)
  // even part
  const T t10 = aan_add(y[0], y[4]);
  const T t11 = aan_sub(y[0], y[4]);
  const T u = k.mul_r(aan_sub(y[2], y[6]));
  const T t13 = aan_add(aan_add(y[2], y[6]), u);
  const T e0 = aan_add(t10, t13), e3 = aan_sub(t10, t13);
  const T e1 = aan_add(t11, u), e2 = aan_sub(t11, u);
  // odd part
  const T z13 = aan_add(y[5], y[3]);
  const T z2 = aan_sub(y[5], y[3]);
  const T z11 = aan_add(y[1], y[7]);
  const T z4 = aan_sub(y[1], y[7]);
  const T a11 = k.mul_r(aan_sub(z11, z13));
  const T t = k.mul_c5(aan_add(z2, z4));
  const T a10 = aan_add(k.mul_c2(z2), t);
  const T a12 = aan_sub(k.mul_c4(z4), t);
  const T o5 = aan_add(a10, a11);
  const T o6 = aan_add(a11, a12);
  const T o7 = aan_add(aan_add(z11, z13), a12);
  x[0] = aan_add(e0, o7);
  x[1] = aan_add(e1, o6);
  x[2] = aan_add(e2, o5);
  x[3] = aan_add(e3, a10);
  x[4] = aan_sub(e3, a10);
  x[5] = aan_sub(e2, o5);
  x[6] = aan_sub(e1, o6);
  x[7] = aan_sub(e0, o7);
}

// Output 0 (last = false) or 7 (last = true) of aan8 alone, by the same
// operations in the same order.
template <class T, class Ops>
__device__ __forceinline__ T aan8_end(const T y[8], bool last, const Ops& k) {
#pragma clang fp contract(off)
  const T t10 = aan_add(y[0], y[4]);
  const T u = k.mul_r(aan_sub(y[2], y[6]));
  const T t13 = aan_add(aan_add(y[2], y[6]), u);
  const T e0 = aan_add(t10, t13);
  const T z13 = aan_add(y[5], y[3]);
  const T z2 = aan_sub(y[5], y[3]);
  const T z11 = aan_add(y[1], y[7]);
  const T z4 = aan_sub(y[1], y[7]);
  const T t = k.mul_c5(aan_add(z2, z4));
  const T a12 = aan_sub(k.mul_c4(z4), t);
  const T o7 = aan_add(aan_add(z11, z13), a12);
  return last ? aan_sub(e0, o7) : aan_add(e0, o7);
}

// Final descale of one row-pass output to a sample.
__device__ __forceinline__ uint32_t aan_sample(int s) {
  return static_cast<uint32_t>(min(max(((s + (1 << (kIfastShift - 1))) >> kIfastShift) + 128, 0), 255));
}
__device__ __forceinline__ uint32_t aan_sample(float s) {
#pragma clang fp contract(off)
  return static_cast<uint32_t>(min(max(static_cast<int>(floorf(s + 128.5f)), 0), 255));
}

// One whole block on one lane: coefficient row r (natural order) in the
// four dwords of rows[r] (int16 pairs, low half first), multipliers m[64]
// (MJD_IDCT_IFAST: int32; MJD_IDCT_FLOAT: fp32 bits), the column pass then
// the row pass in registers; out[2r], out[2r + 1]: samples 0..3 and 4..7 of
// row r, packed little-endian.
template <int M, class V4, class MPtr>
__device__ __forceinline__ void aan_block(const V4 rows[8], MPtr m, const AanConsts& k, uint32_t out[16]) {
#pragma clang fp contract(off)
  using T = typename std::conditional<M == 1, int, float>::type;
  T ws[8][8];  // ws[y][u]: column pass output, sample row y, column u
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    T in[8], y[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int w = (u & 1) ? (rows[v][u >> 1] >> 16) : static_cast<int>(static_cast<int16_t>(rows[v][u >> 1]));
      if constexpr (M == 1) in[v] = __mul24(w, m[8 * v + u]);
      else in[v] = static_cast<float>(w) * __int_as_float(m[8 * v + u]);
    }
    if constexpr (M == 1) aan8(in, y, IfastOps{k.ki[0], k.ki[1], k.ki[2], k.ki[3]});
    else aan8(in, y, FloatOps{k.kf[0], k.kf[1], k.kf[2], k.kf[3]});
#pragma unroll
    for (int i = 0; i < 8; ++i) ws[i][u] = y[i];
  }
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    T s[8];
    if constexpr (M == 1) aan8(ws[i], s, IfastOps{k.ki[0], k.ki[1], k.ki[2], k.ki[3]});
    else aan8(ws[i], s, FloatOps{k.kf[0], k.kf[1], k.kf[2], k.kf[3]});
    out[2 * i] = aan_sample(s[0]) | (aan_sample(s[1]) << 8) | (aan_sample(s[2]) << 16) | (aan_sample(s[3]) << 24);
    out[2 * i + 1] = aan_sample(s[4]) | (aan_sample(s[5]) << 8) | (aan_sample(s[6]) << 16) | (aan_sample(s[7]) << 24);
  }
}

// Row 0 (last = false) or 7 (last = true) of a block alone, as aan_block
// forms it: each column's one output of the column pass, then the row pass
// on that row.  *lo, *hi: its packed samples 0..3 and 4..7.
template <int M, class V4, class MPtr>
__device__ __forceinline__ void aan_block_row(const V4 rows[8], MPtr m, const AanConsts& k, bool last, uint32_t* lo,
                                              uint32_t* hi) {
#pragma clang fp contract(off)
  using T = typename std::conditional<M == 1, int, float>::type;
  T w[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    T in[8];
#pragma unroll
    for (int v = 0; v < 8; ++v) {
      const int x = (u & 1) ? (rows[v][u >> 1] >> 16) : static_cast<int>(static_cast<int16_t>(rows[v][u >> 1]));
      if constexpr (M == 1) in[v] = __mul24(x, m[8 * v + u]);
      else in[v] = static_cast<float>(x) * __int_as_float(m[8 * v + u]);
    }
    if constexpr (M == 1) w[u] = aan8_end(in, last, IfastOps{k.ki[0], k.ki[1], k.ki[2], k.ki[3]});
    else w[u] = aan8_end(in, last, FloatOps{k.kf[0], k.kf[1], k.kf[2], k.kf[3]});
  }
  T s[8];
  if constexpr (M == 1) aan8(w, s, IfastOps{k.ki[0], k.ki[1], k.ki[2], k.ki[3]});
  else aan8(w, s, FloatOps{k.kf[0], k.kf[1], k.kf[2], k.kf[3]});
  *lo = aan_sample(s[0]) | (aan_sample(s[1]) << 8) | (aan_sample(s[2]) << 16) | (aan_sample(s[3]) << 24);
  *hi = aan_sample(s[4]) | (aan_sample(s[5]) << 8) | (aan_sample(s[6]) << 16) | (aan_sample(s[7]) << 24);
}

}  // namespace mjd
