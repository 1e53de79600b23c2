// Decoder variants: the IDCT methods libjpeg offers beside islow (the paper
// notes AAN-based and integer-or-float IDCTs, Sec. 2 and Sec. 3), the
// samplings beyond 4:4:4 / 4:2:2 / 4:2:0 (the paper decodes the others the
// same way, Sec. 4.2) and grayscale.  Full-size colour images run the fused
// segment kernel; the kernels here serve the rest:
//   var_gray    grayscale: one block per lane, the fused kernels'
//               dequantise + IDCT of each method, straight into the output
//               rows;
//   var_colour  chroma upsampling (simple; triangle filter for factors of 2,
//               Algorithm 1, vertical for h1v2) + YCbCr->RGB (Algorithm 2),
//               eight pixels per lane.
// IDCT methods:
//   islow  LL&M in 13-bit fixed point (the fused kernel's arithmetic);
//   ifast  the transposed AAN flowgraph in fixed point: multipliers
//          q * 2^6 / (s(u) s(v)) (s(0) = 1, s(k) = sqrt(2) cos(k pi/16)),
//          9-bit constants with truncating products, ((v + 2^8) >> 9) + 128;
//   float  the same flowgraph in IEEE single precision, multipliers
//          fp32(q / (8 s(u) s(v))), one rounding per operation in a fixed
//          order (no contraction), floor(v + 128.5).
// Scaled decoding (1/2, 1/4, 1/8 output): var_idct_red<N>, one block per
// lane, takes the block's top-left N x N coefficients through the N-point
// IDCT with the 8-point normalisation, in islow-style fixed point
// (x0 * 2^13 + sum round(2^13 sqrt(2) cos((2m+1) u pi / 2N)) x_u, pass 1
// descaled by 11, pass 2 by 18, +128); the colour kernel then runs at the
// reduced size.
#include <math.h>

#include <atomic>
#include <mutex>

#include "aan.h"
#include "mjd_internal.h"

// The float method rounds once per operation, in the order written: no
// contraction into fused multiply-adds (the file is also built with
// -ffp-contract=off).
#pragma clang fp contract(off)

namespace mjd {
// Scale factors and constants of the AAN methods (aan.h), from the C
// library's cos, once.
const AanConsts& aan_consts() {
  static AanConsts k;
  static std::once_flag once;
  std::call_once(once, [] {
    double s[8];
    s[0] = 1.0;
    for (int i = 1; i < 8; ++i) s[i] = sqrt(2.0) * cos(i * M_PI / 16.0);
    for (int u = 0; u < 8; ++u)
      for (int v = 0; v < 8; ++v) {
        const double p = s[u] * s[v];
        k.ss8[8 * u + v] = 8.0 * p;
        k.a14[8 * u + v] = static_cast<int32_t>(llround(16384.0 / p));
      }
    const double c[4] = {cos(M_PI / 4.0), cos(3.0 * M_PI / 8.0), cos(M_PI / 8.0) - cos(3.0 * M_PI / 8.0),
                         cos(M_PI / 8.0) + cos(3.0 * M_PI / 8.0)};
    for (int i = 0; i < 4; ++i) {
      k.ki[i] = static_cast<int32_t>(llround(c[i] * (1 << kIfastConstBits)));
      k.kf[i] = static_cast<float>(c[i]);
    }
  });
  return k;
}

namespace var {


// Constants of the reduced transforms: K[m][u] = round(2^13 sqrt(2)
// cos((2m+1) u pi / 2N)), index N*m + u.
struct RedConsts {
  int32_t k4[16];
  int32_t k2[4];
};

const RedConsts& red_consts() {
  static RedConsts k;
  static std::once_flag once;
  std::call_once(once, [] {
    for (int m = 0; m < 4; ++m)
      for (int u = 0; u < 4; ++u)
        k.k4[4 * m + u] = static_cast<int32_t>(llround(8192.0 * sqrt(2.0) * cos((2 * m + 1) * u * M_PI / 8.0)));
    for (int m = 0; m < 2; ++m)
      for (int u = 0; u < 2; ++u)
        k.k2[2 * m + u] = static_cast<int32_t>(llround(8192.0 * sqrt(2.0) * cos((2 * m + 1) * u * M_PI / 4.0)));
  });
  return k;
}

struct View {
  const int16_t* coef;
  const uint16_t* qt;
  uint8_t* out;
  uint8_t* work;
  uint64_t n_blocks;
  uint64_t plane_off[3];
  uint32_t plane_pitch[3];
  uint32_t pitch;
  int width, height, ncomp, hy, vy, mcus_x, bpm, fancy;
  int qsel[3];
  int comp_w, comp_h;  // the chroma components' true size
};

__device__ __forceinline__ uint32_t clamp_u8(int v) { return static_cast<uint32_t>(min(max(v, 0), 255)); }

// A dword at any byte address: output rows need not be 4-byte aligned, and
// the ROCm kernel driver runs compute queues in the GPU's unaligned access
// mode (the compiler assumes it for this target too), so whole runs take
// dword stores.
typedef uint32_t __attribute__((aligned(1))) u32u;

// --- kernel 1: grayscale, one block per lane ----------------------------------
// A grayscale MCU is one block, so the blocks lie in raster order.  Each wave
// takes runs of 64 consecutive blocks, one per lane: the block's 8
// coefficient rows go straight into registers (the wave's next run loads
// while this one is transformed), through the fused kernels' dequantise +
// IDCT of the method (islow: the dot-product passes; ifast, float: the AAN
// flowgraph on one lane), and out as 8-byte sample rows at any byte address
// (unaligned access mode, as above), cropped at the image's right and
// bottom edges.
constexpr int kGrayThreads = 256;
constexpr int kGrayWaves = kGrayThreads / 64;

template <int M>
__global__ __launch_bounds__(kGrayThreads) void var_gray(const View v, const AanConsts k) {
  // islow: the table as uint16 pairs, and times 16 (the scaled pass 1
  // reads it); ifast, float: the 64 AAN multipliers
  __shared__ __align__(16) uint32_t qs[64];
  __shared__ __align__(16) uint32_t qs16[32];
  const int t = static_cast<int>(threadIdx.x);
  const uint16_t* qt = v.qt + 64 * v.qsel[0];
  if constexpr (M == MJD_IDCT_ISLOW) {
    if (t < 32) {
      const uint32_t lo = qt[2 * t], hi = qt[2 * t + 1];
      qs[t] = lo | (hi << 16);
      qs16[t] = ((lo << 4) & 0xFFFFu) | (((hi << 4) & 0xFFFFu) << 16);
    }
  } else {
    if (t < 64)
      qs[t] = static_cast<uint32_t>(M == MJD_IDCT_IFAST ? aan_ifast_mult(qt[t], t, k) : aan_float_mult(qt[t], t, k));
  }
  __syncthreads();
  const lds32* q = (const lds32*)qs;
  const lds32* q16 = (const lds32*)qs16;
  const uint32_t n_blocks = static_cast<uint32_t>(v.n_blocks);
  const uint32_t n_runs = (n_blocks + 63) / 64;
  const uint32_t lane = static_cast<uint32_t>(t & 63);
  const uint32_t stride = gridDim.x * kGrayWaves;
  const uint32_t mcx = static_cast<uint32_t>(v.mcus_x);
  auto load = [&](uint32_t run, v4i rows[8]) {
    const uint32_t b = run * 64 + lane;
    if (run < n_runs && b < n_blocks) {
      const v4i* src = reinterpret_cast<const v4i*>(v.coef) + static_cast<size_t>(b) * 8;
#pragma unroll
      for (int r = 0; r < 8; ++r) rows[r] = src[r];
    } else {
#pragma unroll
      for (int r = 0; r < 8; ++r) rows[r] = v4i{0, 0, 0, 0};
    }
  };
  uint32_t run = blockIdx.x * kGrayWaves + static_cast<uint32_t>(t >> 6);
  v4i next[8];
  load(run, next);
  for (; run < n_runs; run += stride) {
    v4i rows[8];
#pragma unroll
    for (int r = 0; r < 8; ++r) rows[r] = next[r];
    load(run + stride, next);
    uint32_t out[16];
    if constexpr (M == MJD_IDCT_ISLOW) idct_block_fast(rows, q, q16, out);  // every lane (a wave-wide range test)
    else aan_block<M>(rows, reinterpret_cast<const ldsi*>(q), k, out);
    const uint32_t b = run * 64 + lane;
    if (b >= n_blocks) continue;
    const uint32_t by = b / mcx, bx = b - by * mcx;
    const int px0 = static_cast<int>(bx) * 8;
    const int n = min(8, v.width - px0);
    // the output as a global (not flat) pointer: the store instructions
    gbl8* dst = (gbl8*)(v.out + static_cast<size_t>(by) * 8 * v.pitch + px0);
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (static_cast<int>(by) * 8 + r >= v.height) break;
      if (n == 8) {
        gbl32u* d = reinterpret_cast<gbl32u*>(dst);
        __builtin_nontemporal_store(out[2 * r], &d[0]);
        __builtin_nontemporal_store(out[2 * r + 1], &d[1]);
      } else {
        // n = 1..7: a whole dword if n >= 4, then a 16-bit and a byte store
        if (n >= 4) *reinterpret_cast<gbl32u*>(dst) = out[2 * r];
        const uint32_t last = n >= 4 ? out[2 * r + 1] : out[2 * r];
        gbl8* tail = dst + (n & 4);
        if (n & 2) *reinterpret_cast<gbl16u*>(tail) = static_cast<uint16_t>(last);
        if (n & 1) tail[n & 2] = static_cast<uint8_t>(last >> (8 * (n & 2)));
      }
      dst += v.pitch;
    }
  }
}

// --- kernel 1b: reduced IDCT for scaled decoding -----------------------------
template <int N>
__device__ __forceinline__ void red_1d(const int x[N], int y[N], const int32_t* K, int bias) {
#pragma unroll
  for (int m = 0; m < N; ++m) {
    int acc = (x[0] << 13) + bias;
#pragma unroll
    for (int u = 1; u < N; ++u) acc += K[N * m + u] * x[u];
    y[m] = acc;
  }
}

template <int N>
__global__ __launch_bounds__(256) void var_idct_red(const View v, const RedConsts k) {
  // the four quant tables, once per workgroup
  __shared__ uint16_t qs[4 * 64];
  qs[threadIdx.x] = v.qt[threadIdx.x];
  __syncthreads();
  const uint32_t b = blockIdx.x * 256u + threadIdx.x;
  if (b >= static_cast<uint32_t>(v.n_blocks)) return;
  const int32_t* K = N == 4 ? k.k4 : k.k2;
  int comp = 0, bx, by;
  {
    const uint32_t bpm = static_cast<uint32_t>(v.bpm), mcx = static_cast<uint32_t>(v.mcus_x);
    const uint32_t m = b / bpm;
    const int j = static_cast<int>(b - m * bpm);
    const uint32_t myu = m / mcx;
    const int mx = static_cast<int>(m - myu * mcx), my = static_cast<int>(myu);
    const int ny = v.hy * v.vy;
    if (v.ncomp == 1 || j < ny) {
      const int jy = j / v.hy, jx = j - jy * v.hy;
      bx = mx * v.hy + jx;
      by = my * v.vy + jy;
    } else {
      comp = j - ny + 1;
      bx = mx;
      by = my;
    }
  }
  const int16_t* c = v.coef + static_cast<size_t>(b) * 64;
  const uint16_t* q = qs + 64 * v.qsel[comp];
  uint32_t px[N][N];
  if constexpr (N == 1) {
    px[0][0] = clamp_u8(((c[0] * static_cast<int>(q[0])) * 32768 + (1 << 17) + (128 << 18)) >> 18);
  } else {
    int ws[N][N];
#pragma unroll
    for (int vv = 0; vv < N; ++vv) {  // pass 1: column vv
      int x[N], y[N];
#pragma unroll
      for (int u = 0; u < N; ++u) x[u] = c[8 * u + vv] * static_cast<int>(q[8 * u + vv]);
      red_1d<N>(x, y, K, 1 << 10);
#pragma unroll
      for (int m = 0; m < N; ++m) ws[m][vv] = y[m] >> 11;
    }
#pragma unroll
    for (int m = 0; m < N; ++m) {  // pass 2: row m
      int z[N];
      red_1d<N>(ws[m], z, K, (1 << 17) + (128 << 18));
#pragma unroll
      for (int n = 0; n < N; ++n) px[m][n] = clamp_u8(z[n] >> 18);
    }
  }
#pragma unroll
  for (int m = 0; m < N; ++m) {
    const int y = by * N + m;
    if (v.ncomp == 1) {  // grayscale: into the output rows, cropped
      if (y >= v.height) break;
      uint8_t* dst = v.out + static_cast<size_t>(y) * v.pitch + bx * N;
#pragma unroll
      for (int n = 0; n < N; ++n)
        if (bx * N + n < v.width) dst[n] = static_cast<uint8_t>(px[m][n]);
      continue;
    }
    uint8_t* dst = v.work + v.plane_off[comp] + static_cast<size_t>(y) * v.plane_pitch[comp] + bx * N;
    if constexpr (N == 4) {
      *reinterpret_cast<uint32_t*>(dst) = px[m][0] | (px[m][1] << 8) | (px[m][2] << 16) | (px[m][3] << 24);
    } else if constexpr (N == 2) {
      *reinterpret_cast<uint16_t*>(dst) = static_cast<uint16_t>(px[m][0] | (px[m][1] << 8));
    } else {
      dst[0] = static_cast<uint8_t>(px[m][0]);
    }
  }
}

// --- kernel 2: upsample + colour -------------------------------------------
// Eight output pixels per lane: luma as one 8-byte load; chroma as the
// samples the eight pixels read, from aligned loads plus the two clamped
// neighbours of a triangle filter's window.
__device__ __forceinline__ int byte_of(uint32_t w, int i) { return static_cast<int>((w >> (8 * i)) & 0xFFu); }

// Chroma row window for a factor-2 filter: s[0..3] the samples k0..k0+3,
// l / r the clamped neighbours k0-1 and k0+4.
struct Win {
  int s[4], l, r;
};
__device__ __forceinline__ Win load_win(const uint8_t* row, int k0, int cw) {
  Win w;
  const uint32_t d = *reinterpret_cast<const uint32_t*>(row + k0);
#pragma unroll
  for (int i = 0; i < 4; ++i) w.s[i] = byte_of(d, i);
  w.l = row[max(k0 - 1, 0)];
  w.r = row[min(k0 + 4, cw - 1)];
  return w;
}

// The eight chroma values of pixels x0..x0+7 of row y.
__device__ __forceinline__ void chroma8(const View& v, const uint8_t* p, uint32_t pp, int x0, int y, int c[8]) {
  const int fh = v.hy, fv = v.vy;
  if (!v.fancy || fh == 4 || (fh == 1 && fv == 1)) {
    const uint8_t* row = p + static_cast<size_t>(y / fv) * pp;
    if (fh == 1) {
      const uint2 d = *reinterpret_cast<const uint2*>(row + x0);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        c[i] = byte_of(d.x, i);
        c[4 + i] = byte_of(d.y, i);
      }
    } else if (fh == 2) {
      const uint32_t d = *reinterpret_cast<const uint32_t*>(row + (x0 >> 1));
#pragma unroll
      for (int i = 0; i < 8; ++i) c[i] = byte_of(d, i >> 1);
    } else {
      const int a = row[x0 >> 2], b = row[(x0 >> 2) + 1];
#pragma unroll
      for (int i = 0; i < 8; ++i) c[i] = i < 4 ? a : b;
    }
    return;
  }
  if (fh == 1) {  // h1v2: Algorithm 1 turned vertical
    const int r = y >> 1, odd = y & 1;
    const int nr = odd ? min(r + 1, v.comp_h - 1) : max(r - 1, 0);
    const uint2 a = *reinterpret_cast<const uint2*>(p + static_cast<size_t>(r) * pp + x0);
    const uint2 b = *reinterpret_cast<const uint2*>(p + static_cast<size_t>(nr) * pp + x0);
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      c[i] = (3 * byte_of(a.x, i) + byte_of(b.x, i) + 1 + odd) >> 2;
      c[4 + i] = (3 * byte_of(a.y, i) + byte_of(b.y, i) + 1 + odd) >> 2;
    }
    return;
  }
  const int k0 = x0 >> 1, cw = v.comp_w;
  int s[4], l, rr;
  int sh = 2, bias_even = 1, bias_odd = 2;
  if (fv == 1) {  // h2v1: Algorithm 1
    const Win w = load_win(p + static_cast<size_t>(y) * pp, k0, cw);
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] = w.s[i];
    l = w.l;
    rr = w.r;
  } else {  // h2v2: unrounded vertical sums, then the horizontal filter on the 16x scale
    const int r = y >> 1, odd = y & 1;
    const int nr = odd ? min(r + 1, v.comp_h - 1) : max(r - 1, 0);
    const Win a = load_win(p + static_cast<size_t>(r) * pp, k0, cw);
    const Win b = load_win(p + static_cast<size_t>(nr) * pp, k0, cw);
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] = 3 * a.s[i] + b.s[i];
    l = 3 * a.l + b.l;
    rr = 3 * a.r + b.r;
    sh = 4;
    bias_even = 8;
    bias_odd = 7;
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = k0 + j;
    const int left = k - 1 < 0 ? s[j] : (j == 0 ? l : s[j - 1]);
    const int right = k + 1 > cw - 1 ? s[j] : (j == 3 ? rr : s[j + 1]);
    c[2 * j] = (3 * s[j] + left + bias_even) >> sh;
    c[2 * j + 1] = (3 * s[j] + right + bias_odd) >> sh;
  }
}

__global__ __launch_bounds__(256) void var_colour(const View v) {
  const int gpr = (v.width + 7) >> 3;
  // the grid is a multiple of 8 dealt to the XCDs round-robin: each XCD
  // takes a contiguous band of rows, so the chroma rows that neighbouring
  // output rows share are fetched once into its L2
  const uint32_t wg = (blockIdx.x & 7u) * (gridDim.x >> 3) + (blockIdx.x >> 3);
  const uint64_t g = static_cast<uint64_t>(wg) * 256 + threadIdx.x;
  if (g >= static_cast<uint64_t>(gpr) * static_cast<uint64_t>(v.height)) return;
  const int y = static_cast<int>(g / static_cast<uint64_t>(gpr));
  const int x0 = static_cast<int>(g - static_cast<uint64_t>(y) * gpr) * 8;
  const uint2 yd = *reinterpret_cast<const uint2*>(v.work + v.plane_off[0] + static_cast<size_t>(y) * v.plane_pitch[0] + x0);
  int cb[8], cr[8];
  chroma8(v, v.work + v.plane_off[1], v.plane_pitch[1], x0, y, cb);
  chroma8(v, v.work + v.plane_off[2], v.plane_pitch[2], x0, y, cr);
  uint32_t b[24];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int y16 = (byte_of(i < 4 ? yd.x : yd.y, i & 3) << 16) + 32768;
    const int xb = cb[i] - 128, xr = cr[i] - 128;
    b[3 * i] = clamp_u8((y16 + kCrR * xr) >> 16);
    b[3 * i + 1] = clamp_u8((y16 - kCbG * xb - kCrG * xr) >> 16);
    b[3 * i + 2] = clamp_u8((y16 + kCbB * xb) >> 16);
  }
  uint8_t* dst = v.out + static_cast<size_t>(y) * v.pitch + 3 * x0;
  const int n = min(8, v.width - x0);
  if (n == 8) {
    u32u* d = reinterpret_cast<u32u*>(dst);
#pragma unroll
    for (int i = 0; i < 6; ++i) d[i] = b[4 * i] | (b[4 * i + 1] << 8) | (b[4 * i + 2] << 16) | (b[4 * i + 3] << 24);
  } else {
    for (int i = 0; i < 3 * n; ++i) dst[i] = static_cast<uint8_t>(b[i]);
  }
}

// The IDCT kernel runs as many workgroups as stay resident (each loops over
// tiles), or about one per tile when there are fewer.
// Grayscale: as many workgroups as stay resident, at most one wave per run
// of 64 blocks.
template <int M>
hipError_t launch_gray(const View& v, const AanConsts& k, int cu_count, hipStream_t s) {
  static std::atomic<int> cached{0};  // resident workgroups per CU (the same on every gfx950 device)
  int per_cu = cached.load(std::memory_order_relaxed);
  if (per_cu == 0) {
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, var_gray<M>, kGrayThreads, 0);
    if (e != hipSuccess) return e;
    per_cu = n > 0 ? n : 1;
    cached.store(per_cu, std::memory_order_relaxed);
  }
  const uint64_t slots = static_cast<uint64_t>(per_cu) * (cu_count > 0 ? cu_count : 256);
  const uint64_t runs = (v.n_blocks + 63) / 64;
  const uint64_t want = (runs + kGrayWaves - 1) / kGrayWaves;
  const unsigned grid = static_cast<unsigned>(want < slots ? want : slots);
  hipLaunchKernelGGL(var_gray<M>, dim3(grid), dim3(kGrayThreads), 0, s, v, k);
  return hipGetLastError();
}

}  // namespace var

}  // namespace mjd

extern "C" {

int mjd_decode_variant(mjd_ctx* ctx, const mjd_variant* variant, const int16_t* d_coef, const uint16_t* d_qt,
                       uint8_t* d_out, size_t pitch, void* d_work, uint64_t work_bytes, void* stream) {
  using namespace mjd;
  if (!ctx) return fail(MJD_EINVAL, "null context");
  mjd_geometry g;
  var::View v{};
  uint64_t need = 0;
  int rc = variant_geometry(variant, &g, &need, v.plane_pitch, v.plane_off);
  if (rc != MJD_OK) return rc;
  if (!d_coef || !d_qt || !d_out) return fail(MJD_EINVAL, "null device buffer");
  if (reinterpret_cast<uintptr_t>(d_coef) % 16) return fail(MJD_EINVAL, "coefficient buffer not 16-byte aligned");
  if (reinterpret_cast<uintptr_t>(d_qt) % 2) return fail(MJD_EINVAL, "quant table buffer not 2-byte aligned");
  const int nc = static_cast<int>(variant->ncomp);
  const uint32_t scale = variant->scale ? variant->scale : 1;
  const uint32_t out_w = (variant->frame.width + scale - 1) / scale, out_h = (variant->frame.height + scale - 1) / scale;
  const uint64_t row_bytes = static_cast<uint64_t>(nc) * out_w;
  if (pitch < row_bytes) return fail(MJD_EINVAL, "pitch %zu < %u*width", pitch, nc);
  if (pitch >= (1ull << 31)) return fail(MJD_EINVAL, "pitch %zu not below 2^31 bytes", pitch);
  const bool fused = nc == 3 && scale == 1;
  if (fused) {
    // full-size colour images: the fused segment kernel of the sampling and
    // IDCT method, one launch, no sample planes in memory
    if (pitch >= (1ull << 24)) return fail(MJD_EINVAL, "pitch %zu not below 2^24 bytes", pitch);
    ImageView im{};
    im.coef = d_coef;
    im.qt = d_qt;
    im.rgb = d_out;
    im.pitch = static_cast<uint32_t>(pitch);
    im.width = static_cast<int>(variant->frame.width);
    im.height = static_cast<int>(variant->frame.height);
    im.mcus_x = static_cast<int>(g.mcus_x);
    im.mcus_y = static_cast<int>(g.mcus_y);
    im.chroma_w = static_cast<int>(g.comp_w[1]);
    im.chroma_h = static_cast<int>(g.comp_h[1]);
    im.qsel0 = static_cast<int>(variant->frame.qsel[0]);
    im.qsel1 = static_cast<int>(variant->frame.qsel[1]);
    im.qsel2 = static_cast<int>(variant->frame.qsel[2]);
    int cur = 0;
    if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) {
      if (hipSetDevice(ctx->device) != hipSuccess) return fail(MJD_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
    }
    const hipError_t e = launch_variant(im, static_cast<int>(variant->frame.h[0]), static_cast<int>(variant->frame.v[0]),
                                        variant->upsample == MJD_UPSAMPLE_FANCY, variant->idct, ctx->cu_count, ctx->tuning,
                                        static_cast<hipStream_t>(stream));
    if (cur != ctx->device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return fail(MJD_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
    return MJD_OK;
  }
  if (nc == 3) {
    if (!d_work) return fail(MJD_EINVAL, "null workspace");
    if (reinterpret_cast<uintptr_t>(d_work) % 16) return fail(MJD_EINVAL, "workspace not 16-byte aligned");
    if (work_bytes < need) return fail(MJD_EINVAL, "workspace of %llu bytes below the %llu needed",
                                       static_cast<unsigned long long>(work_bytes), static_cast<unsigned long long>(need));
  }
  v.coef = d_coef;
  v.qt = d_qt;
  v.out = d_out;
  v.work = static_cast<uint8_t*>(d_work);
  v.n_blocks = g.n_blocks;
  v.pitch = static_cast<uint32_t>(pitch);
  v.width = static_cast<int>(out_w);
  v.height = static_cast<int>(out_h);
  v.ncomp = nc;
  v.hy = nc == 3 ? variant->frame.h[0] : 1;
  v.vy = nc == 3 ? variant->frame.v[0] : 1;
  v.mcus_x = static_cast<int>(g.mcus_x);
  v.bpm = static_cast<int>(g.blocks_per_mcu);
  v.fancy = variant->upsample == MJD_UPSAMPLE_FANCY ? 1 : 0;
  for (int c = 0; c < 3; ++c) v.qsel[c] = c < nc ? variant->frame.qsel[c] : 0;
  v.comp_w = static_cast<int>(g.comp_w[1]);
  v.comp_h = static_cast<int>(g.comp_h[1]);
  int cur = 0;
  if (hipGetDevice(&cur) != hipSuccess || cur != ctx->device) {
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(MJD_EDEVICE, "hipSetDevice(%d) failed", ctx->device);
  }
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const AanConsts& k = aan_consts();
  hipError_t e;
  const unsigned grid_red = static_cast<unsigned>((g.n_blocks + 255) / 256);
  if (scale > 1) {
    const var::RedConsts& rk = var::red_consts();
    if (scale == 2) hipLaunchKernelGGL(var::var_idct_red<4>, dim3(grid_red), dim3(256), 0, s, v, rk);
    else if (scale == 4) hipLaunchKernelGGL(var::var_idct_red<2>, dim3(grid_red), dim3(256), 0, s, v, rk);
    else hipLaunchKernelGGL(var::var_idct_red<1>, dim3(grid_red), dim3(256), 0, s, v, rk);
    e = hipGetLastError();
  } else switch (variant->idct) {  // full-size grayscale (colour returned above)
    case MJD_IDCT_ISLOW: e = var::launch_gray<MJD_IDCT_ISLOW>(v, k, ctx->cu_count, s); break;
    case MJD_IDCT_IFAST: e = var::launch_gray<MJD_IDCT_IFAST>(v, k, ctx->cu_count, s); break;
    default: e = var::launch_gray<MJD_IDCT_FLOAT>(v, k, ctx->cu_count, s); break;
  }
  if (e == hipSuccess && nc == 3) {
    const uint64_t groups = static_cast<uint64_t>((v.width + 7) / 8) * v.height;
    const unsigned grid2 = static_cast<unsigned>(((groups + 255) / 256 + 7) & ~7ull);
    hipLaunchKernelGGL(var::var_colour, dim3(grid2), dim3(256), 0, s, v);
    e = hipGetLastError();
  }
  if (cur != ctx->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return fail(MJD_EDEVICE, "kernel launch failed: %s", hipGetErrorString(e));
  return MJD_OK;
}

}  // extern "C"
