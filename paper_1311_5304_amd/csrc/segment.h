// Pipelined segment decoder: the body shared by the single-image and the
// batched kernels.
//
// A workgroup decodes a *segment*: a column of sub-tiles (SX x SY MCUs each)
// of one image, walked top to bottom.  Per sub-tile k the stages are
//   DMA      the coefficient blocks of sub-tile k+1 (and the chroma blocks of
//            its left/right neighbour MCUs) are copied global -> LDS with
//            global_load_lds_dwordx4, fully coalesced, into a swizzled staging
//            buffer, while the lanes compute on sub-tile k.  Each wave copies
//            the blocks its own lanes read, so staging needs no barrier;
//   phase 1  dequantise + 8x8 islow IDCT (paper Sec. 4.1), one block per
//            lane, both passes in registers; samples go to an LDS luma
//            slot and an LDS chroma ring.  The neighbour chroma blocks the
//            fancy filter needs (Sec. 4.2) are split 8 lanes per block, and
//            only the one column the filter reads is formed, summed across
//            the block's lanes in the wave;
//   phase 2  upsampling + YCbCr->RGB (Sec. 4.3) + RGB8 stores (Fig. 5).
// Step k runs phase 2 of sub-tile k-1 and then phase 1 of sub-tile k, in
// different luma and chroma slots, so each step has one barrier, and a wave
// goes from its stores to its transform without waiting for the others.
// For the 4:2:0 fancy filter a sub-tile's last chroma row needs the first
// chroma row of the next sub-tile: that row pair is upsampled one step
// later still (three slots), so the rows between sub-tiles come from the
// ring instead of being decoded twice; only the rows just above and below
// the whole segment are decoded as neighbour blocks, at its start.
#pragma once

#include "aan.h"
#include "decode_kernel.h"

namespace mjd {

typedef __attribute__((address_space(3))) void lds_void_t;
// LDS pointers proper (32-bit addresses, so index arithmetic stays 32-bit)
typedef __attribute__((address_space(3))) uint8_t lds8;
typedef __attribute__((address_space(3))) uint32_t lds32;
typedef __attribute__((address_space(3))) int ldsi;
typedef __attribute__((address_space(3))) int16_t lds16;
typedef __attribute__((address_space(3))) uint16_t ldsu16;
// global-memory pointers for the RGB stores (global, not flat, instructions)
typedef __attribute__((address_space(1))) uint8_t gbl8;
typedef __attribute__((address_space(1), aligned(1))) uint16_t gbl16u;  // any byte address
typedef __attribute__((address_space(1), aligned(1))) uint32_t gbl32u;  // any byte address

constexpr int round64c(int n) { return (n + 63) & ~63; }

__device__ __forceinline__ int clamp255i(int v) { return min(max(v, 0), 255); }
__device__ __forceinline__ uint32_t byte_at(uint32_t w, int i) { return (w >> (8 * i)) & 0xFFu; }

// One image as the segment decoder sees it.
struct ImageView {
  const int16_t* coef;
  const uint16_t* qt;
  uint8_t* rgb;
  uint32_t pitch;  // < 2^24
  int width, height;
  int mcus_x, mcus_y;
  int chroma_w, chroma_h;
  int qsel0, qsel1, qsel2;
};

// Segment = MCU columns [mx0, mx0 + SX) (clipped) x MCU rows [r0, r1).
struct SegmentRange {
  int mx0, r0, r1;
};

// HF x VF: the luma blocks of an MCU, (1,1), (2,1), (1,2), (2,2) or (4,1),
// chroma one block each.  IDCT: MJD_IDCT_ISLOW (0, the paper's LL&M with
// the dot-product row pass), MJD_IDCT_IFAST (1) or MJD_IDCT_FLOAT (2), the
// AAN methods of aan.h, one whole block per lane.
template <int HF_, int VF_, bool FANCY_, int SX_, int SY_, int NT_, int IDCT_ = 0>
struct SegCfg {
  static constexpr int HF = HF_, VF = VF_, SX = SX_, SY = SY_, NT = NT_, IDCT = IDCT_;
  static constexpr bool ISLOW = IDCT == 0;
  static constexpr bool FANCY = FANCY_;
  static constexpr int NY = HF * VF;
  static constexpr int BPM = NY + 2;
  // fancy filtering applies to factors of 2 (a factor of 4 is replicated)
  static constexpr bool HALO_X = FANCY && HF == 2;
  static constexpr bool HALO_Y = FANCY && VF == 2;
  static constexpr int SM = SX * SY;                       // MCUs per sub-tile
  static constexpr int N_MAIN = BPM * SM;                  // blocks per sub-tile
  static constexpr int N_SIDE = HALO_X ? 4 * SY : 0;       // left/right neighbour chroma blocks
  static constexpr int N_SLOT = N_MAIN + N_SIDE;           // staged blocks
  static constexpr int SIDE_LANE0 = round64c(N_MAIN);      // first lane of the side tasks
  // islow forms a side block's one column on 8 lanes; the AAN methods
  // transform the whole block on one lane
  static constexpr int P1_LANES = SIDE_LANE0 + (ISLOW ? 8 : 1) * N_SIDE;
  static constexpr int N_TB = HALO_Y ? 2 * (SX + 2) : 0;   // above or below neighbour blocks
  static constexpr int YWD = SX * 2 * HF;                  // luma sub-tile row, dwords
  static constexpr int YROWS = SY * 8 * VF;
  static constexpr int CR = 8 * SY;                        // chroma rows per sub-tile
  // Luma and chroma: one slot per sub-tile in flight, two (phase 2 of k - 1
  // beside phase 1 of k), or three with the vertical fancy filter (the last
  // row pair of k - 2 is also upsampled at step k).
  static constexpr int NYB = HALO_Y ? 3 : 2;
  // Workgroups of two waves, whose residency LDS sets, keep luma in a ring
  // of two sub-tiles plus one block row instead (which still holds the last
  // two chroma rows' luma of sub-tile k-2 while k is transformed): 4 rather
  // than 3 of them fit a CU.
  static constexpr bool YCOMPACT = HALO_Y && NT <= 128;
  static constexpr int YRING = YCOMPACT ? 2 * YROWS + 8 : NYB * YROWS;
  static constexpr int Y_BYTES = YRING * YWD * 4;
  static constexpr int CWD = (SX + 2) * 2;                 // chroma ring row, dwords (8-sample margins)
  static constexpr int CROWS = NYB * CR;                   // chroma ring rows
  // with the vertical filter, one more chroma row after the ring: the row
  // below the segment
  static constexpr int CROWS_ALLOC = CROWS + (HALO_Y ? 1 : 0);
  static constexpr int UX = 2 * SX;                        // phase-2 units per chroma row
  static constexpr int UNITS = UX * 8 * SY;
  // LDS carve-up (bytes, 16-byte aligned pieces)
  static constexpr int OFF_STAGE = 0;
  static constexpr int OFF_Y = OFF_STAGE + N_SLOT * 128;
  static constexpr int OFF_C = OFF_Y + Y_BYTES;
  static constexpr int OFF_Q = OFF_C + 2 * CROWS_ALLOC * CWD * 4;     // islow: quant tables, uint16 pairs; AAN: 32-bit multipliers
  static constexpr int OFF_Q16 = OFF_Q + (ISLOW ? 3 * 128 : 3 * 256);  // islow: the same times 16
  static constexpr int LDS_BYTES = OFF_Q16 + (ISLOW ? 3 * 128 : 0);
  // Waves per SIMD that the LDS footprint allows (160 KB per CU), at most 3
  // asked of the register allocator; the 4:2:0 fancy class, which holds the
  // most state (neighbour rows and row pairs of chroma), asks for 2, which
  // leaves it 256 registers.
  static constexpr int WAVES_PER_SIMD_LDS = (160 * 1024 / LDS_BYTES) * (NT / 64) / 4;
  static constexpr int WAVES_CAP = HALO_Y && ISLOW ? 2 : 3;
  static constexpr int WAVES_PER_SIMD =
      WAVES_PER_SIMD_LDS < 1 ? 1 : (WAVES_PER_SIMD_LDS > WAVES_CAP ? WAVES_CAP : WAVES_PER_SIMD_LDS);
  static_assert(P1_LANES <= NT, "one phase-1 round per sub-tile");
  static_assert(NT % 64 == 0 && NT >= 96, "whole waves; quant table load needs 96 lanes");
  static_assert(!HALO_Y || HF <= 2, "vertical fancy filtering with HF 1 or 2");
  static_assert(N_MAIN % 64 == 0, "tile blocks fill whole waves");
  static_assert(YROWS % 8 == 0 && YRING % 8 == 0, "whole block rows; blocks never straddle the luma ring's wrap");
};

// WALK_LAST: the last row pair of a segment is upsampled in the same item
// walk as the others (one unit per lane) even where its rows could be spread
// over the waves; the batched kernel, which holds every sampling class in
// one function, takes it so (a separate pass there put the kernel over its
// register budget).
template <class C, bool WALK_LAST = false>
struct SegmentDecoder {
  static constexpr int HF = C::HF, VF = C::VF, SX = C::SX, SY = C::SY, NT = C::NT;
  static constexpr int NY = C::NY, BPM = C::BPM, SM = C::SM, N_MAIN = C::N_MAIN;
  static constexpr int N_SIDE = C::N_SIDE, N_SLOT = C::N_SLOT, N_TB = C::N_TB;
  static constexpr int YWD = C::YWD, YROWS = C::YROWS, NYB = C::NYB, YRING = C::YRING;
  static constexpr int CR = C::CR, CWD = C::CWD, CROWS = C::CROWS;
  static constexpr bool FANCY = C::FANCY, HALO_X = C::HALO_X, HALO_Y = C::HALO_Y;

  lds8* lds;
  const ImageView& im;
  const AanConsts* ak;  // the AAN methods' constants (unused by islow)
  int tid;
  // segment geometry
  int mx0, nmx, r0, r1, K;
  int gcx0;  // global chroma column of the strip's first sample

  __device__ SegmentDecoder(uint8_t* lds_, const ImageView& im_, int tid_, const AanConsts* ak_ = nullptr)
      : lds((lds8*)lds_), im(im_), ak(ak_), tid(tid_) {}

  __device__ lds8* stage() const { return lds + C::OFF_STAGE; }
  __device__ lds32* luma() const { return reinterpret_cast<lds32*>(lds + C::OFF_Y); }
  __device__ lds32* cring(int c) const { return reinterpret_cast<lds32*>(lds + C::OFF_C) + c * (C::CROWS_ALLOC * CWD); }
  __device__ lds32* qtab(int c) const { return reinterpret_cast<lds32*>(lds + C::OFF_Q) + c * (C::ISLOW ? 32 : 64); }
  __device__ lds32* qtab16(int c) const { return reinterpret_cast<lds32*>(lds + C::OFF_Q16) + c * 32; }

  // Luma row r (0 <= r < YROWS) of sub-tile k lives in row ybase(k) + r of
  // the luma area (slot k mod NYB), taken modulo YRING for the compact
  // ring (a multiple of 8 rows, so a block never straddles its wrap).
  // ybase is uniform.
  __device__ static int ybase(int k) { return C::YCOMPACT ? (YROWS * k) % YRING : (k % NYB) * YROWS; }
  __device__ static int ywrap(int i) {
    if constexpr (C::YCOMPACT) i = i >= YRING ? i - YRING : i;
    return i;
  }
  __device__ lds32* yrow(int base, int r) const { return luma() + ywrap(base + r) * YWD; }
  // Chroma row r (0 <= r < CR) of sub-tile k is ring row cbase(k) + r (a
  // sub-tile never wraps).  The row above the segment is ring row
  // CROWS - 1 (read at step 1, before sub-tile 2 takes that slot), the row
  // below it row CROWS, after the ring.
  __device__ static int cbase(int k) { return (CR * k) % CROWS; }
  static constexpr int BELOW_ROW = CROWS;
  __device__ static int ring_prev(int rc) { return rc == 0 ? CROWS - 1 : rc - 1; }
  __device__ static int ring_next(int rc) { return rc == CROWS - 1 ? 0 : rc + 1; }
  // The chroma row after the pair at ring rows rc, rc + 1 (global rows gy,
  // gy + 1): row rc + 1 itself at the image's last chroma row, the row
  // below the segment after the segment's last row, else the next ring row.
  __device__ int row_after_pair(int gy, int rc) const {
    return gy + 1 >= im.chroma_h - 1 ? rc + 1 : (gy + 2 == 8 * r1 ? BELOW_ROW : ring_next(rc + 1));
  }

  __device__ int sub_r0(int k) const { return r0 + k * SY; }
  __device__ int sub_rows(int k) const { return min(SY, r1 - (r0 + k * SY)); }

  __device__ const int16_t* block_ptr(int my, int mx, int b) const {
    return im.coef + (static_cast<size_t>(my) * im.mcus_x + mx) * (BPM * 64) + b * 64;
  }

  // ---- coefficient DMA ----
  // 16-byte chunk i of the staging buffer holds row ((i & 7) - j) & 7 of
  // staged block j = i / 8.  Blocks j < N_MAIN are the sub-tile's MCUs in
  // memory order (block j % BPM of MCU j / BPM, MCUs row by row), so each
  // MCU row of the sub-tile is one contiguous run of RUNB blocks; the rest
  // are the chroma blocks of the MCUs left and right of the strip.  Row c
  // of block j lands at ((c + j) & 7) * 16, so lanes that read whole blocks
  // later hit distinct banks, while the 8 lanes of a block still read one
  // 128-byte line.
  //
  // A DMA instruction moves 64 chunks = 8 whole blocks J..J+7 with J a
  // multiple of 8, so (RUNB being a multiple of 8) the run, and with it the
  // source base, is uniform per instruction, and a lane's offset inside the
  // 8 blocks depends on its lane number only: block J + (lane >> 3), row
  // (lane - (lane >> 3)) & 7.
  static constexpr int RUNB = SX * BPM;
  static_assert(RUNB % 8 == 0 && N_MAIN % 64 == 0, "DMA instructions never straddle a run or the side blocks");

  __device__ static int lane_chunk_offset(int lane) { return ((lane >> 3) << 7) | (((lane - (lane >> 3)) & 7) << 4); }

  // Side chunk i (i >= 8 N_MAIN): byte offset from the sub-tile's first MCU
  // (negative for the MCU left of the strip), or -1 when the MCU lies outside
  // the image or below the sub-tile's nmy rows.
  __device__ bool side_chunk(int i, int nmy, int row_bytes, int* off) const {
    const int j = i >> 3;
    const int c = ((i & 7) - j) & 7;
    const int t = j - N_MAIN;  // (row << 2) | (right << 1) | chroma component
    const int pos = t >> 2;
    const int dx = ((t >> 1) & 1) ? nmx : -1;
    const int mx = mx0 + dx;
    *off = pos * row_bytes + dx * (BPM * 128) + (NY + (t & 1)) * 128 + c * 16;
    return pos < nmy && mx >= 0 && mx < im.mcus_x;
  }

  // Copy sub-tile k's blocks into the staging buffer.  Each wave copies
  // exactly the blocks its own lanes read in read_stage (main block J is
  // read by lane J; side chunk s by the side lanes from SIDE_LANE0 + s,
  // islow, or by the first side wave, AAN), so a wave needs no other
  // wave's copies before it reads.  Lanes whose block lies outside the
  // image or below the sub-tile read the sub-tile's first block instead,
  // into a slot nothing reads, so the copy loop has no branches.
  static constexpr int SIDE_CHUNKS = 8 * N_SIDE;
  static constexpr int SIDE_W0 = C::SIDE_LANE0 / 64;
  static constexpr int SIDE_INSTR = (SIDE_CHUNKS + 63) / 64;
  __device__ void dma(int k) const {
    const uint8_t* src0 = reinterpret_cast<const uint8_t*>(block_ptr(sub_r0(k), mx0, 0));
    const int nmy = sub_rows(k);
    const int row_bytes = im.mcus_x * (BPM * 128);
    const int lane = tid & 63;
    const uint32_t lane_off = static_cast<uint32_t>(lane_chunk_offset(lane));
    const int main_blocks = nmx * BPM;  // staged blocks of each run that exist
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (wv < N_MAIN / 64) {
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int J = 64 * wv + 8 * i;  // first of the instruction's 8 blocks
        const int run = J / RUNB;
        const int jr = J - run * RUNB;
        const bool ok = run < nmy && (lane >> 3) < main_blocks - jr;
        const uint8_t* src = ok ? src0 + (run * row_bytes + jr * 128) + lane_off : src0;
        __builtin_amdgcn_global_load_lds(static_cast<const void*>(src), (lds_void_t*)(stage() + J * 128), 16, 0, 0);
      }
    } else if constexpr (N_SIDE > 0) {
      // islow: wave SIDE_W0 + m copies side chunks [64 m, 64 m + 64); AAN:
      // wave SIDE_W0 copies them all
      constexpr int PER_WAVE = C::ISLOW ? 1 : SIDE_INSTR;
      const int m0 = C::ISLOW ? wv - SIDE_W0 : 0;
      if (C::ISLOW ? (wv >= SIDE_W0 && wv < SIDE_W0 + SIDE_INSTR) : wv == SIDE_W0) {
#pragma unroll
        for (int i = 0; i < PER_WAVE; ++i) {
          const int s = 64 * (m0 + i) + lane;
          int off;
          const bool ok = side_chunk(8 * N_MAIN + s, nmy, row_bytes, &off);
          if (s < SIDE_CHUNKS)
            __builtin_amdgcn_global_load_lds(static_cast<const void*>(ok ? src0 + off : src0),
                                             (lds_void_t*)(stage() + (8 * N_MAIN + 64 * (m0 + i)) * 16), 16, 0, 0);
        }
      }
    }
  }

  // The quant tables into LDS, on the 64 lanes of one wave in rounds: the
  // global loads of every round first, then the LDS writes.  islow: 96
  // uint16 pairs (and the same times 16); AAN: the 192 multipliers.
  static constexpr int QN = C::ISLOW ? 96 : 192;
  static constexpr int QR = (QN + 63) / 64;
  struct QLoads {
    uint32_t v[QR];
  };
  __device__ QLoads qtab_loads() const {
    const int l = tid & 63;
    // the three table selectors as scalars (a per-lane choice among them
    // would otherwise become a load of its own)
    const int s0 = opaque(im.qsel0), s1 = opaque(im.qsel1), s2 = opaque(im.qsel2);
    QLoads f;
    uint32_t* v = f.v;
#pragma unroll
    for (int r = 0; r < QR; ++r) {
      const int i = l + 64 * r;
      v[r] = 0;
      if (i < QN) {
        if constexpr (C::ISLOW) {
          const int c = i >> 5;
          const int sel = c == 0 ? s0 : (c == 1 ? s1 : s2);
          const __attribute__((address_space(1))) uint16_t* q =
              (const __attribute__((address_space(1))) uint16_t*)im.qt + (sel * 64 + 2 * (i & 31));
          v[r] = static_cast<uint32_t>(q[0]) | (static_cast<uint32_t>(q[1]) << 16);
        } else {
          const int c = i >> 6;
          const int sel = c == 0 ? s0 : (c == 1 ? s1 : s2);
          v[r] = im.qt[sel * 64 + (i & 63)];
        }
      }
    }
    return f;
  }
  __device__ void qtab_stores(const QLoads& f) const {
    const int l = tid & 63;
    const uint32_t* v = f.v;
#pragma unroll
    for (int r = 0; r < QR; ++r) {
      const int i = l + 64 * r;
      if (i < QN) {
        if constexpr (C::ISLOW) {
          const int c = i >> 5;
          qtab(c)[i & 31] = v[r];
          // 16 Q per half, modulo 2^16 (the products are only used modulo 2^16)
          qtab16(c)[i & 31] = ((v[r] << 4) & 0xFFFFu) | ((v[r] >> 16) << 20);
        } else {
          const int c = i >> 6, e = i & 63;
          reinterpret_cast<ldsi*>(qtab(c))[e] =
              C::IDCT == 1 ? aan_ifast_mult(v[r], e, *ak) : aan_float_mult(v[r], e, *ak);
        }
      }
    }
  }

  // ---- neighbour blocks above/below the segment (vertical fancy filter) ----
  // The chroma blocks of the MCU rows just above and below the segment are
  // loaded straight into the registers of the lanes that form their one
  // row, by the last wave at the segment's start (run()'s prologue).

  // One lane per neighbour block forms the one sample row the filter needs
  // (row 7 of the block above, row 0 of the block below): dequantisation,
  // that row's output of the column pass for each of the 8 columns (its
  // integer linear form, four dot products per column), then the row pass
  // over the 8 results; the samples go into the ring row above/below the
  // segment.  At the true left edge and at the true right chroma edge the
  // lane also writes the replicated sample the filter reads beyond the edge.
  // The neighbour block of lane t (< N_TB) above or below the segment, or
  // false where that MCU lies outside the image.
  __device__ bool tb_block(bool below, int t, int* pos, int* mx) const {
    const int my = below ? r1 : r0 - 1;
    *pos = t >> 1;
    *mx = mx0 - 1 + *pos;
    return my >= 0 && my < im.mcus_y && t < N_TB && *pos < nmx + 2 && *mx >= 0 && *mx < im.mcus_x;
  }

  // Neighbour block t straight from global memory.
  __device__ void tb_rows_global(bool below, int t, int mx, v4i rows[8]) const {
    const __attribute__((address_space(1))) v4i* src =
        (const __attribute__((address_space(1))) v4i*)(block_ptr(below ? r1 : r0 - 1, mx, NY + (t & 1)));
#pragma unroll
    for (int c = 0; c < 8; ++c) rows[c] = src[c];
  }

  // The row of neighbour block t (component 1 + (t & 1) at MCU column mx).
  __device__ void tb_row(bool below, int t, int pos, int mx, const v4i rows[8]) const {
    if constexpr (!C::ISLOW) {
      // the AAN methods: the one row on this lane
      uint32_t lo, hi;
      aan_block_row<C::IDCT>(rows, reinterpret_cast<const ldsi*>(qtab(1 + (t & 1))), *ak, !below, &lo, &hi);
      lds32* row = cring(t & 1) + (below ? BELOW_ROW : CROWS - 1) * CWD;
      row[2 * pos] = lo;
      row[2 * pos + 1] = hi;
      lds8* row8 = reinterpret_cast<lds8*>(row);
      if (mx0 == 0 && mx == 0) row8[7] = static_cast<uint8_t>(lo);
      const int cw = im.chroma_w;
      if (cw - 1 < gcx0 + 8 * nmx && mx == ((cw - 1) >> 3)) {
        const int e = (cw - 1) & 7;
        row8[cw - gcx0 + 8] = static_cast<uint8_t>((e < 4 ? lo : hi) >> (8 * (e & 3)));
      }
      return;
    }
    typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
    const __attribute__((address_space(3))) v4i* qv =
        reinterpret_cast<const __attribute__((address_space(3))) v4i*>(qtab(1 + (t & 1)));
    uint32_t d[8][4];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const v4i v = rows[c];
      const v4i qq = qv[c];
      const int w[4] = {v.x, v.y, v.z, v.w};
      const int qw[4] = {qq.x, qq.y, qq.z, qq.w};
#pragma unroll
      for (int i = 0; i < 4; ++i)
        d[c][i] = __builtin_bit_cast(uint32_t, __builtin_bit_cast(u16x2, w[i]) * __builtin_bit_cast(u16x2, qw[i]));
    }
    int x[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = u >> 1;
      const uint32_t sel = (u & 1) ? 0x07060302u : 0x05040100u;
      const uint32_t p04 = __builtin_amdgcn_perm(d[4][i], d[0][i], sel);
      const uint32_t p26 = __builtin_amdgcn_perm(d[6][i], d[2][i], sel);
      const uint32_t p13 = __builtin_amdgcn_perm(d[3][i], d[1][i], sel);
      const uint32_t p57 = __builtin_amdgcn_perm(d[7][i], d[5][i], sel);
      const int e0 = dot2(p26, wpair(kE2a, kE6a), dot2(p04, wpair(1 << kConstBits, 1 << kConstBits), kPass1Bias));
      const int o0 = dot2(p13, wpair(kO[0][0], kO[0][1]), dot2z(p57, wpair(kO[0][2], kO[0][3])));
      x[u] = (below ? e0 + o0 : e0 - o0) >> kPass1Shift;
    }
    int y[8];
    idct8_raw(x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7], kPass2Bias, y);
#pragma unroll
    for (int i = 0; i < 8; ++i) y[i] >>= kPass2Shift;
    lds32* row = cring(t & 1) + (below ? BELOW_ROW : CROWS - 1) * CWD;
    row[2 * pos] = pack4(y[0], y[1], y[2], y[3]);
    row[2 * pos + 1] = pack4(y[4], y[5], y[6], y[7]);
    lds8* row8 = reinterpret_cast<lds8*>(row);
    // the strip starts at the image's left edge: x = -1 repeats x = 0
    if (mx0 == 0 && mx == 0) row8[7] = static_cast<uint8_t>(clamp255i(y[0]));
    // the true right chroma edge lies in this strip: x = cw repeats x = cw - 1
    const int cw = im.chroma_w;
    if (cw - 1 < gcx0 + 8 * nmx && mx == ((cw - 1) >> 3)) {
      int e = y[0];
#pragma unroll
      for (int i = 1; i < 8; ++i)
        if (((cw - 1) & 7) == i) e = y[i];  // constant indices: y stays in registers
      row8[cw - gcx0 + 8] = static_cast<uint8_t>(clamp255i(e));
    }
  }

  // ---- phase 1 of sub-tile k ----
  // Registers carried from the staging read (before the next DMA overwrites
  // the buffer) to the transform.
  struct Held {
    v4i r0, r1, r2, r3, r4, r5, r6, r7;  // named members: always promoted to registers
    __device__ __forceinline__ void set(int c, v4i v) {
      switch (c) {  // c is a compile-time constant after unrolling
        case 0: r0 = v; break;
        case 1: r1 = v; break;
        case 2: r2 = v; break;
        case 3: r3 = v; break;
        case 4: r4 = v; break;
        case 5: r5 = v; break;
        case 6: r6 = v; break;
        default: r7 = v; break;
      }
    }
  };

  __device__ void read_stage(int k, Held& h) const {
    // lanes that transform a whole block: the sub-tile's, and for the AAN
    // methods also one per side block
    const bool whole = tid < N_MAIN || (!C::ISLOW && HALO_X && tid >= C::SIDE_LANE0 && tid < C::P1_LANES);
    if (whole) {
      const int j = tid < N_MAIN ? tid : N_MAIN + (tid - C::SIDE_LANE0);
      const lds8* blk = stage() + j * 128;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        h.set(c, *reinterpret_cast<const __attribute__((address_space(3))) v4i*>(blk + (((c + j) & 7) << 4)));
    } else if constexpr (HALO_X) {
      if (tid >= C::SIDE_LANE0 && tid < C::P1_LANES) {
        const int t = (tid - C::SIDE_LANE0) >> 3, u = tid & 7;
        const int j = N_MAIN + t;
        const lds8* blk = stage() + j * 128 + 2 * u;
        int x[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) x[v] = *reinterpret_cast<const lds16*>(blk + (((v + j) & 7) << 4));
        h.r0 = v4i{x[0], x[1], x[2], x[3]};
        h.r1 = v4i{x[4], x[5], x[6], x[7]};
      }
    }
    (void)k;
  }

  // Dequantise + IDCT of one block held in registers (rows in natural
  // order), by the configured method: out[2r], out[2r + 1] the packed
  // samples 0..3 and 4..7 of row r.
  __device__ void block(const v4i rows[8], int comp, uint32_t out[16]) const {
    if constexpr (C::ISLOW) idct_block_fast(rows, qtab(comp), qtab16(comp), out);
    else aan_block<C::IDCT>(rows, reinterpret_cast<const ldsi*>(qtab(comp)), *ak, out);
  }

  __device__ void phase1(int k, const Held& h) const {
    const int nmy = sub_rows(k);
    if (tid < N_MAIN) {
      const int j = tid;
      const int m = j / BPM;
      const int b = j - m * BPM;
      const int lmy = m / SX, lmx = m - (m / SX) * SX;
      if (lmx >= nmx || lmy >= nmy) return;
      const int comp = b < NY ? 0 : b - NY + 1;
      uint32_t o[16];
      const v4i rows[8] = {h.r0, h.r1, h.r2, h.r3, h.r4, h.r5, h.r6, h.r7};
      block(rows, comp, o);
      if (comp == 0) {
        const int by = b / HF, bx = b - (b / HF) * HF;
        lds32* dst = yrow(ybase(k), lmy * 8 * VF + by * 8) + lmx * 2 * HF + bx * 2;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          dst[r * YWD] = o[2 * r];
          dst[r * YWD + 1] = o[2 * r + 1];
        }
      } else {
        lds32* dst = cring(comp - 1) + (cbase(k) + 8 * lmy) * CWD + lmx * 2 + 2;
#pragma unroll
        for (int r = 0; r < 8; ++r) {
          dst[r * CWD] = o[2 * r];
          dst[r * CWD + 1] = o[2 * r + 1];
        }
        if constexpr (HALO_X) {
          // Samples beyond the true left/right chroma edge repeat the edge
          // sample.  The lane that owns the edge sample writes the copy (no
          // other lane writes that byte: at a true edge there is no
          // neighbour MCU beyond it).
          lds8* row8 = reinterpret_cast<lds8*>(dst - lmx * 2 - 2);
          if (gcx0 == 0 && lmx == 0) {
#pragma unroll
            for (int r = 0; r < 8; ++r) row8[r * CWD * 4 + 7] = static_cast<uint8_t>(o[2 * r]);
          }
          const int e = im.chroma_w - 1 - gcx0;  // the last sample, relative to the strip
          if (e < 8 * nmx && (e >> 3) == lmx) {
            // the dword holding sample e & 7, chosen by a mask (not an
            // index, which would put o[] in scratch memory)
            const uint32_t hi = 0u - static_cast<uint32_t>((e >> 2) & 1);
            const int sh = 8 * (e & 3);
#pragma unroll
            for (int r = 0; r < 8; ++r)
              row8[r * CWD * 4 + e + 9] = static_cast<uint8_t>((o[2 * r] ^ ((o[2 * r] ^ o[2 * r + 1]) & hi)) >> sh);
          }
        }
      }
    } else if constexpr (HALO_X && !C::ISLOW) {
      // a side block on one lane: the whole block, then the one column the
      // filter reads (0 of the block right of the strip, 7 of the one left)
      if (tid >= C::SIDE_LANE0 && tid < C::P1_LANES) {
        const int t = tid - C::SIDE_LANE0;
        const int pos = t >> 2;
        const bool right = (t >> 1) & 1;
        const int mx = right ? mx0 + nmx : mx0 - 1;
        if (pos >= nmy || mx < 0 || mx >= im.mcus_x) return;
        uint32_t o[16];
        const v4i rows[8] = {h.r0, h.r1, h.r2, h.r3, h.r4, h.r5, h.r6, h.r7};
        block(rows, 1 + (t & 1), o);
        lds8* row8 = reinterpret_cast<lds8*>(cring(t & 1) + (cbase(k) + 8 * pos) * CWD);
        const int x = right ? nmx * 8 + 8 : 7;
#pragma unroll
        for (int r = 0; r < 8; ++r)
          row8[r * CWD * 4 + x] = static_cast<uint8_t>(right ? o[2 * r] : o[2 * r + 1] >> 24);
      }
    } else if constexpr (HALO_X) {
      if (tid >= C::SIDE_LANE0 && tid < C::P1_LANES) {
        const int t = (tid - C::SIDE_LANE0) >> 3, u = tid & 7;
        const int pos = t >> 2;
        const int mx = ((t >> 1) & 1) ? mx0 + nmx : mx0 - 1;
        if (pos >= nmy || mx < 0 || mx >= im.mcus_x) return;
        const ldsu16* q = reinterpret_cast<const ldsu16*>(qtab(1 + (t & 1))) + u;
        int x[8] = {h.r0.x, h.r0.y, h.r0.z, h.r0.w, h.r1.x, h.r1.y, h.r1.z, h.r1.w};
#pragma unroll
        for (int v = 0; v < 8; ++v) x[v] *= static_cast<int>(q[8 * v]);
        int y[8];
        idct8_raw(x[0], x[1], x[2], x[3], x[4], x[5], x[6], x[7], kPass1Bias, y);
        // The row pass at one output column (0 of the block right of the
        // strip, 7 of the one left of it) is the integer linear form
        // sum_u M[c][u] w[i][u] that the flowgraph computes before its
        // descale, with M[7][u] = (-1)^u M[0][u].  Each lane forms its
        // column's terms; a butterfly over the block's 8 lanes sums them,
        // and lane u keeps sample row u.
        const bool right = (t >> 1) & 1;
        const int wgt = (right || !(u & 1)) ? row0_weight(u) : -row0_weight(u);
        int sum[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) sum[i] = sum8_lanes(mul24(y[i] >> kPass1Shift, wgt));
        int v = sum[0];
#pragma unroll
        for (int i = 1; i < 8; ++i) v = u == i ? sum[i] : v;
        lds8* row8 = reinterpret_cast<lds8*>(cring(t & 1) + (cbase(k) + 8 * pos + u) * CWD);
        row8[right ? nmx * 8 + 8 : 7] = static_cast<uint8_t>(clamp255i((v + kPass2Bias) >> kPass2Shift));
      }
    }
  }

  // Weight of input u in output 0 of the flowgraph (its first row):
  // 8192, 11363, 10703, 9633, 8192, 6437, 4433, 2260.
  __device__ static int row0_weight(int u) {
    const int w01 = u & 1 ? kO[0][0] : 1 << kConstBits;
    const int w23 = u & 1 ? kO[0][1] : kE2a;
    const int w45 = u & 1 ? kO[0][2] : 1 << kConstBits;
    const int w67 = u & 1 ? kO[0][3] : kE6a;
    return u < 4 ? (u < 2 ? w01 : w23) : (u < 6 ? w45 : w67);
  }

  // Sum over the 8 lanes of an aligned 8-lane group, in every lane of it
  // (DPP: swap neighbours, swap pairs, mirror the halves of the group).
  // Integer adds wrap, so the sum is exact whenever the true sum fits 32 bits.
  __device__ static int sum8_lanes(int x) {
    x += __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
    x += __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
    x += __builtin_amdgcn_update_dpp(0, x, 0x141, 0xF, 0xF, false);  // row_half_mirror
    return x;
  }

  // ---- phase 2 helpers: fancy h2v2 on packed 16-bit pairs ----
  typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
  typedef short i16x2 __attribute__((ext_vector_type(2)));

  // Chroma samples c0..c5 around the 4 samples at p[0] (c0 = the one
  // before, c5 = the one after) as (c0, c1), (c2, c3), (c4, c5).
  __device__ static void chroma_pairs(const lds32* p, u16x2 v[3]) {
    const uint32_t l = p[-1], m = p[0], r = p[1];
    v[0] = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(m, l, 0x0C040C03u));
    v[1] = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(m, m, 0x0C020C01u));
    v[2] = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(r, m, 0x0C040C03u));
  }

  // One output row from the vertical sums s0..s5 (as pairs): for sample j
  // (1..4) the even pixel is (3 s_j + s_{j-1} + 8) >> 4 and the odd one
  // (3 s_j + s_{j+1} + 7) >> 4, each minus 128; o[] gets the 8 pixels.
  __device__ static void h2v2_row(const u16x2 s[3], int o[8]) {
    const u16x2 s12 = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, s[1]),
                                                                       __builtin_bit_cast(uint32_t, s[0]), 0x05040302u));
    const u16x2 s34 = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, s[2]),
                                                                       __builtin_bit_cast(uint32_t, s[1]), 0x05040302u));
    const u16x2 three = {3, 3}, even_bias = {2040, 2040}, odd_bias = {2041, 2041};
    const i16x2 four = {4, 4};
    const i16x2 e01 = __builtin_bit_cast(i16x2, static_cast<u16x2>(s12 * three + s[0] - even_bias)) >> four;
    const i16x2 e23 = __builtin_bit_cast(i16x2, static_cast<u16x2>(s34 * three + s[1] - even_bias)) >> four;
    const i16x2 o01 = __builtin_bit_cast(i16x2, static_cast<u16x2>(s12 * three + s[1] - odd_bias)) >> four;
    const i16x2 o23 = __builtin_bit_cast(i16x2, static_cast<u16x2>(s34 * three + s[2] - odd_bias)) >> four;
    o[0] = e01.x; o[1] = o01.x; o[2] = e01.y; o[3] = o01.y;
    o[4] = e23.x; o[5] = o23.x; o[6] = e23.y; o[7] = o23.y;
  }

  // ---- phase 2: upsample + colour + store ----
  // Uniform facts about one sub-tile that phase 2 needs.
  struct SubInfo {
    gbl8* rgb;     // output pixel of its first chroma row and the strip's first column
    int gcy0;      // global chroma row of its first row
    int yb, cb;    // luma and chroma ring bases
    int rows;      // chroma rows present
  };
  __device__ SubInfo sub_info(int k) const {
    const int gcy0 = 8 * sub_r0(k);
    return {(gbl8*)(im.rgb + static_cast<size_t>(gcy0 * VF) * im.pitch + static_cast<size_t>(gcx0 * HF) * 3), gcy0,
            ybase(k), cbase(k), 8 * sub_rows(k)};
  }

  // The same values as opaque scalars, so that a per-lane choice between
  // two sub-tiles selects finished values (the compiler would otherwise fold
  // the choice into the arithmetic and redo it per lane).
  __device__ static int opaque(int v) {
    v = __builtin_amdgcn_readfirstlane(v);
    asm volatile("" : "+s"(v));
    return v;
  }
  __device__ static SubInfo uniform(const SubInfo& si) {
    const uint64_t p = reinterpret_cast<uint64_t>(si.rgb);
    const uint32_t lo = static_cast<uint32_t>(opaque(static_cast<int>(p)));
    const uint32_t hi = static_cast<uint32_t>(opaque(static_cast<int>(p >> 32)));
    return {reinterpret_cast<gbl8*>(static_cast<uint64_t>(lo) | (static_cast<uint64_t>(hi) << 32)), opaque(si.gcy0),
            opaque(si.yb), opaque(si.cb), opaque(si.rows)};
  }

  // All chroma rows of sub-tile k.
  __device__ void phase2(int k) const {
    const SubInfo si = sub_info(k);
    // For fancy 4:2:2 the lanes that transform a block in phase 1 take one
    // unit each and the neighbour-column lanes, which have little phase-1
    // work, share the rest; otherwise all lanes share evenly.
    constexpr int L1 = (HALO_X && !HALO_Y && NT > N_MAIN) ? N_MAIN : 0;
    static_assert(C::UNITS >= L1, "one unit for every block lane");
    const int ustep = tid < L1 ? C::UNITS : NT - L1;
    for (int uidx = tid; uidx < C::UNITS; uidx += ustep) {
      const int cr_l = uidx / C::UX;
      const int g = uidx - cr_l * C::UX;
      if (g >= 2 * nmx || cr_l >= si.rows) continue;
      unit(si, cr_l, g);
    }
  }

  // Vertical fancy filter, step k (1..K): every chroma row of sub-tile k-1
  // but its last two, and the last two rows of sub-tile k-2 (the last of
  // which needs the first row of k-1), as pairs of rows: one pair of rows
  // and 4 samples per lane.  At step K also the last pair of sub-tile K-1,
  // whose last row reads the row below the segment: after phase 1, its
  // rows spread over the waves (last_pair_rows, the h2v2 filter), or in the
  // same item walk (h1v2).
  static constexpr bool LAST_IN_WALK = HF != 2 || WALK_LAST;
  static_assert(!HALO_Y || LAST_IN_WALK || C::UX % 64 == 0 || NT >= 256, "a wave for each output row");
  __device__ void phase2_pairs(int k) const {
    // work items: (pair v, unit g); v 0 the last pair of k - 2, v = CR/2
    // (step K only) the last pair of k - 1; a workgroup of fewer lanes than
    // items takes them in turns
    constexpr int ITEMS = (C::CR / 2) * C::UX;
    static_assert(ITEMS % NT == 0, "the row pairs of a sub-tile fill the workgroup a whole number of times");
    const bool has_b = k >= 2;
    const int n_items = ITEMS + (LAST_IN_WALK && k == K ? C::UX : 0);
    const SubInfo sa = uniform(sub_info(k - 1)), sb = uniform(sub_info(has_b ? k - 2 : 0));
    // every unit of the strip is whole: the plain store path alone
    const bool plain = (gcx0 + 8 * nmx) * HF <= im.width;
    for (int it0 = 0; it0 < n_items; it0 += NT) {
      const int it = it0 + tid;
      int g, v;
      if constexpr (C::UX % 64 == 0) {
        // a row pair per wave: the pair and everything derived from it
        // are scalars
        const int wb = __builtin_amdgcn_readfirstlane(it & ~63);
        v = wb / C::UX;
        g = wb - v * C::UX + (it & 63);
      } else {
        g = it % C::UX;
        v = it / C::UX;
      }
      const bool tail = v == 0;
      if (it >= n_items || g >= 2 * nmx || (tail && !has_b)) continue;
      SubInfo si;
      si.rgb = tail ? sb.rgb : sa.rgb;
      si.gcy0 = tail ? sb.gcy0 : sa.gcy0;
      si.yb = tail ? sb.yb : sa.yb;
      si.cb = tail ? sb.cb : sa.cb;
      // v = CR/2 gives sa.rows - 2 (sa.rows is CR there: only the last
      // sub-tile can be short, and its last pair is v = CR/2)
      const int cr = tail ? sb.rows - 2 : (v == C::CR / 2 ? sa.rows - 2 : 2 * (v - 1));
      if (!tail && v < C::CR / 2 && cr >= sa.rows - 2) continue;
      if constexpr (HF == 2) {
        if (plain) unit_pair<true>(si, cr, g);
        else unit_pair<false>(si, cr, g);
      } else {
        if (plain) unit_pair_v<true>(si, cr, g);
        else unit_pair_v<false>(si, cr, g);
      }
    }
  }

  // Vertical fancy filter (h2v2), step K: the last pair of sub-tile K-1
  // (its last row reads the row below the segment), its four output rows
  // spread over the waves, one row of a unit per lane, after phase 1: a
  // strip of a wave or more takes its units in turns, a narrower strip
  // gives wave j output row j.
  __device__ void last_pair_rows() const {
    const SubInfo sa = uniform(sub_info(K - 1));
    const bool plain = (gcx0 + 8 * nmx) * HF <= im.width;
    if constexpr (C::UX % 64 == 0) {
#pragma unroll
      for (int it0 = 0; it0 < 4 * C::UX; it0 += NT) {
        const int it = it0 + tid;
        if (it >= 4 * C::UX) break;
        const int wb = __builtin_amdgcn_readfirstlane(it & ~63);  // a row per wave: a scalar
        const int j = wb / C::UX, g = wb - j * C::UX + (it & 63);
        if (g >= 2 * nmx) continue;
        if (plain) unit_row<true>(sa, sa.rows - 2, g, j);
        else unit_row<false>(sa, sa.rows - 2, g, j);
      }
    } else {
      const int j = __builtin_amdgcn_readfirstlane(tid >> 6);  // a scalar
      const int g = tid & 63;
      if (j < 4 && g < C::UX && g < 2 * nmx) {
        if (plain) unit_row<true>(sa, sa.rows - 2, g, j);
        else unit_row<false>(sa, sa.rows - 2, g, j);
      }
    }
  }

  // 3 a + b on 16-bit halves (every value here is below 2^12)
  __device__ static u16x2 mad3(u16x2 a, u16x2 b) {
    uint32_t r;
    asm("v_pk_mad_u16 %0, %1, 3, %2 op_sel_hi:[1,0,1]"
        : "=v"(r) : "v"(__builtin_bit_cast(uint32_t, a)), "v"(__builtin_bit_cast(uint32_t, b)));
    return __builtin_bit_cast(u16x2, r);
  }

  // One horizontal output row of the fancy h2v2 filter from the vertical
  // sums s0..s5 (as pairs): sample j (1..4) gives the even pixel
  // (3 s_j + s_{j-1} + 8) >> 4 and the odd one (3 s_j + s_{j+1} + 7) >> 4,
  // each minus 128.  The bias (8 - 2048 or 7 - 2048) is added to the
  // neighbour term, so each 16-bit half holds the biased sum as an int16 in
  // [-2040, 2040], and one signed bit-field extract (bits 4..15) both
  // shifts and unpacks it.
  __device__ static void h2v2_row_x(const u16x2 s[3], int o[8]) {
    const u16x2 s12 = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, s[1]),
                                                                       __builtin_bit_cast(uint32_t, s[0]), 0x05040302u));
    const u16x2 s34 = __builtin_bit_cast(u16x2, __builtin_amdgcn_perm(__builtin_bit_cast(uint32_t, s[2]),
                                                                       __builtin_bit_cast(uint32_t, s[1]), 0x05040302u));
    const u16x2 three = {3, 3};
    const u16x2 eb = {static_cast<unsigned short>(8 - 2048), static_cast<unsigned short>(8 - 2048)};
    const u16x2 ob = {static_cast<unsigned short>(7 - 2048), static_cast<unsigned short>(7 - 2048)};
    const uint32_t e01 = __builtin_bit_cast(uint32_t, static_cast<u16x2>(s12 * three + (s[0] + eb)));
    const uint32_t o01 = __builtin_bit_cast(uint32_t, static_cast<u16x2>(s12 * three + (s[1] + ob)));
    const uint32_t e23 = __builtin_bit_cast(uint32_t, static_cast<u16x2>(s34 * three + (s[1] + eb)));
    const uint32_t o23 = __builtin_bit_cast(uint32_t, static_cast<u16x2>(s34 * three + (s[2] + ob)));
    o[0] = __builtin_amdgcn_sbfe(static_cast<int>(e01), 4, 12);
    o[1] = __builtin_amdgcn_sbfe(static_cast<int>(o01), 4, 12);
    o[2] = __builtin_amdgcn_sbfe(static_cast<int>(e01), 20, 12);
    o[3] = __builtin_amdgcn_sbfe(static_cast<int>(o01), 20, 12);
    o[4] = __builtin_amdgcn_sbfe(static_cast<int>(e23), 4, 12);
    o[5] = __builtin_amdgcn_sbfe(static_cast<int>(o23), 4, 12);
    o[6] = __builtin_amdgcn_sbfe(static_cast<int>(e23), 20, 12);
    o[7] = __builtin_amdgcn_sbfe(static_cast<int>(o23), 20, 12);
  }

  // Chroma rows cr and cr + 1 of a sub-tile's strip, samples 4g..4g+3
  // (4:2:0 fancy): four output rows of 8 pixels.  Each chroma row is read
  // once, with its neighbours above and below, for all four rows.
  template <bool PLAIN>
  __device__ void unit_pair(const SubInfo& si, const int cr, const int g) const {
    const int W = im.width, H = im.height;
    const int px0 = (gcx0 + 4 * g) * 2;
    const int gy = si.gcy0 + cr;
    const int py0 = 2 * gy;
    if (px0 >= W || py0 >= H) return;
    const int ch = im.chroma_h;
    const int rc = si.cb + cr;  // ring row of row cr; rc + 1 is row cr + 1 (a sub-tile never wraps the ring)
    // neighbours, repeated at the true top and bottom chroma edges
    const int ru = gy == 0 ? rc : ring_prev(rc);
    const bool last0 = gy == ch - 1;  // row cr is the last chroma row (row cr + 1 lies below the image)
    const int rd = row_after_pair(gy, rc);
    u16x2 pu[2][3], p0[2][3], p1[2][3], pd[2][3];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const lds32* ring = cring(c) + (g + 2);
      chroma_pairs(ring + mul24(ru, CWD), pu[c]);
      chroma_pairs(ring + mul24(rc, CWD), p0[c]);
      chroma_pairs(ring + mul24(rc + 1, CWD), p1[c]);
      chroma_pairs(ring + mul24(rd, CWD), pd[c]);
    }
    // the luma of the four rows, fetched together
    uint32_t yl[4][2];
    {
      const int ly = si.yb + 2 * cr;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const lds32* ysrc = luma() + (mul24(ywrap(ly + j), YWD) + 2 * g);
        yl[j][0] = ysrc[0];
        yl[j][1] = ysrc[1];
      }
    }
    // the lower neighbour of row cr: row cr + 1, or row cr itself at the
    // true bottom edge
#pragma unroll
    for (int c = 0; c < 2; ++c)
#pragma unroll
      for (int i = 0; i < 3; ++i)
        if (last0) p1[c][i] = p0[c][i];
    const int nv = min(8, W - px0);
    const int pitch24 = static_cast<int>(im.pitch);
    gbl8* row = si.rgb + (mul24(2 * cr, pitch24) + 24 * g);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (py0 + j >= H) break;
      int xs[2][8];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        u16x2 sv[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          // vertical 3:1 sums (rows cr-1|cr+1 around cr, then cr|cr+2 around cr+1)
          if (j == 0) sv[i] = mad3(p0[c][i], pu[c][i]);
          else if (j == 1) sv[i] = mad3(p0[c][i], p1[c][i]);
          else if (j == 2) sv[i] = mad3(p1[c][i], p0[c][i]);
          else sv[i] = mad3(p1[c][i], pd[c][i]);
        }
        h2v2_row_x(sv, xs[c]);
      }
      uint32_t w[6];
#pragma unroll
      for (int kk = 0; kk < 2; ++kk) {
        RGBWide px[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) px[i] = ycc_wide(y16_of(yl[j][kk], i), xs[0][4 * kk + i], xs[1][4 * kk + i]);
        pack_rgb4(px, w + 3 * kk);
      }
      if (PLAIN || nv == 8) store_unit(row, w);
      else store_ragged(row, w, 3 * nv);
      row += pitch24;
    }
  }

  // Output row j (0..3) of unit_pair's four, alone: the chroma row nearest
  // it and the other row the vertical 3:1 filter reads (j uniform across
  // the wave, so the ring rows are scalars).
  template <bool PLAIN>
  __device__ void unit_row(const SubInfo& si, const int cr, const int g, const int j) const {
    const int W = im.width, H = im.height;
    const int px0 = (gcx0 + 4 * g) * 2;
    const int gy = si.gcy0 + cr;
    const int py = 2 * gy + j;
    if (px0 >= W || py >= H) return;
    const int ch = im.chroma_h;
    const int rc = si.cb + cr;
    const int r1 = gy == ch - 1 ? rc : rc + 1;  // row cr + 1, or row cr at the true bottom edge
    int rn, rf;
    if (j == 0) {
      rn = rc;
      rf = gy == 0 ? rc : ring_prev(rc);
    } else if (j == 1) {
      rn = rc;
      rf = r1;
    } else if (j == 2) {
      rn = r1;
      rf = rc;
    } else {
      rn = r1;
      rf = row_after_pair(gy, rc);
    }
    int xs[2][8];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const lds32* ring = cring(c) + (g + 2);
      u16x2 pn[3], pf[3], sv[3];
      chroma_pairs(ring + mul24(rn, CWD), pn);
      chroma_pairs(ring + mul24(rf, CWD), pf);
#pragma unroll
      for (int i = 0; i < 3; ++i) sv[i] = mad3(pn[i], pf[i]);
      h2v2_row_x(sv, xs[c]);
    }
    const lds32* ysrc = luma() + (mul24(ywrap(si.yb + 2 * cr + j), YWD) + 2 * g);
    const uint32_t yl[2] = {ysrc[0], ysrc[1]};
    uint32_t w[6];
#pragma unroll
    for (int kk = 0; kk < 2; ++kk) {
      RGBWide px[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) px[i] = ycc_wide(y16_of(yl[kk], i), xs[0][4 * kk + i], xs[1][4 * kk + i]);
      pack_rgb4(px, w + 3 * kk);
    }
    const int nv = min(8, W - px0);
    gbl8* row = si.rgb + (mul24(2 * cr + j, static_cast<int>(im.pitch)) + 24 * g);
    if (PLAIN || nv == 8) store_unit(row, w);
    else store_ragged(row, w, 3 * nv);
  }

  // Chroma rows cr and cr + 1 of a sub-tile's strip, samples 4g..4g+3
  // (h1v2 fancy: the 3:1 filter turned vertical, no horizontal filter):
  // four output rows of 4 pixels.
  template <bool PLAIN>
  __device__ void unit_pair_v(const SubInfo& si, const int cr, const int g) const {
    const int W = im.width, H = im.height;
    const int px0 = gcx0 + 4 * g;
    const int gy = si.gcy0 + cr;
    const int py0 = 2 * gy;
    if (px0 >= W || py0 >= H) return;
    const int ch = im.chroma_h;
    const int rc = si.cb + cr;  // ring row of row cr; rc + 1 is row cr + 1
    const int ru = gy == 0 ? rc : ring_prev(rc);
    const bool last0 = gy == ch - 1;
    const int rd = row_after_pair(gy, rc);
    uint32_t cu[2], c0[2], c1[2], cd[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const lds32* ring = cring(c) + (g + 2);
      cu[c] = ring[mul24(ru, CWD)];
      c0[c] = ring[mul24(rc, CWD)];
      c1[c] = ring[mul24(rc + 1, CWD)];
      cd[c] = ring[mul24(rd, CWD)];
      if (last0) c1[c] = c0[c];
    }
    const int ly = si.yb + 2 * cr;
    const int nv = min(4, W - px0);
    const int pitch24 = static_cast<int>(im.pitch);
    gbl8* row = si.rgb + (mul24(2 * cr, pitch24) + 12 * g);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if (py0 + j >= H) break;
      const uint32_t yd = luma()[mul24(ywrap(ly + j), YWD) + g];
      int x[2][4];
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        // (3 near + far + 1) >> 2 on even output rows, + 2 on odd ones
        const uint32_t nr = j < 2 ? c0[c] : c1[c];
        const uint32_t fr = j == 0 ? cu[c] : (j == 3 ? cd[c] : (j == 1 ? c1[c] : c0[c]));
#pragma unroll
        for (int i = 0; i < 4; ++i)
          x[c][i] = ((3 * static_cast<int>(byte_at(nr, i)) + static_cast<int>(byte_at(fr, i)) + 1 + (j & 1)) >> 2) - 128;
      }
      RGBWide px[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) px[i] = ycc_wide(y16_of(yd, i), x[0][i], x[1][i]);
      uint32_t w[3];
      pack_rgb4(px, w);
      if (PLAIN || nv == 4) store_unit(row, w);
      else store_ragged(row, w, 3 * nv);
      row += pitch24;
    }
  }

  // One unit: chroma samples 4g..4g+3 of row cr_l of a sub-tile's strip,
  // i.e. 4*HF x VF pixels.
  __device__ void unit(const SubInfo& si, const int cr_l, const int g) const {
    const int W = im.width, H = im.height;
    const int pitch24 = static_cast<int>(im.pitch);
    {
      const int px0 = (gcx0 + 4 * g) * HF;
      const int py0 = (si.gcy0 + cr_l) * VF;
      if (px0 >= W || py0 >= H) return;

      int xb[VF][4 * HF], xr[VF][4 * HF];  // chroma - 128 per output pixel
      const int rc = si.cb + cr_l;
      // the rows above and below, repeated at the true top and bottom
      // chroma edges
      const int gy = si.gcy0 + cr_l;
      const int ru = gy == 0 ? rc : ring_prev(rc);
      const int rd = gy == im.chroma_h - 1 ? rc : ring_next(rc);
      (void)ru;
      (void)rd;
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        const lds32* ring = cring(c);
        const lds32* plane = ring + (mul24(rc, CWD) + g + 2);
        int out[VF][4 * HF];
        if constexpr (!FANCY || HF != 2) {
          const uint32_t w = plane[0];
#pragma unroll
          for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int dy = 0; dy < VF; ++dy)
#pragma unroll
              for (int dx = 0; dx < HF; ++dx) out[dy][i * HF + dx] = static_cast<int>(byte_at(w, i)) - 128;
        } else {
          if constexpr (VF == 1) {
            int cc[6];
            {
              const uint32_t l = plane[-1], m = plane[0], r = plane[1];
              cc[0] = byte_at(l, 3);
#pragma unroll
              for (int i = 0; i < 4; ++i) cc[1 + i] = byte_at(m, i);
              cc[5] = byte_at(r, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int m3 = 3 * cc[1 + i];
              out[0][2 * i] = (m3 + cc[i] - 511) >> 2;          // (3C + Cprev + 1) / 4 - 128
              out[0][2 * i + 1] = (m3 + cc[i + 2] - 510) >> 2;  // (3C + Cnext + 2) / 4 - 128
            }
          } else {
            // h2v2 on packed 16-bit halves: pairs of neighbouring chroma
            // samples, the unrounded 3:1 vertical sums, then the 3:1
            // horizontal filter on pairs of outputs (every intermediate is
            // below 2^12, so the halves never carry into each other)
            u16x2 pm[3], pu[3], pd[3];
            chroma_pairs(plane, pm);
            chroma_pairs(ring + (mul24(ru, CWD) + g + 2), pu);
            chroma_pairs(ring + (mul24(rd, CWD) + g + 2), pd);
            const u16x2 three = {3, 3};
            u16x2 su[3], sd[3];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
              su[j] = pm[j] * three + pu[j];
              sd[j] = pm[j] * three + pd[j];
            }
            h2v2_row(su, out[0]);
            h2v2_row(sd, out[VF - 1]);
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

      const int nv = min(4 * HF, W - px0);
#pragma unroll
      for (int dy = 0; dy < VF; ++dy) {
        const int py = py0 + dy;
        if (py >= H) break;
        const lds32* ysrc = yrow(si.yb, cr_l * VF + dy) + g * HF;
        uint32_t w[3 * HF];
#pragma unroll
        for (int kk = 0; kk < HF; ++kk) {
          const uint32_t ydw = ysrc[kk];
          RGBWide px[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) px[i] = ycc_wide(y16_of(ydw, i), xb[dy][4 * kk + i], xr[dy][4 * kk + i]);
          pack_rgb4(px, w + 3 * kk);
        }
        gbl8* row = si.rgb + (mul24(cr_l * VF + dy, pitch24) + 12 * HF * g);
        if (nv == 4 * HF) store_unit(row, w);
        else store_ragged(row, w, 3 * nv);
      }
    }
  }

  // A whole unit's 12*HF bytes, in dword stores at the row address whether
  // or not it is 4-byte aligned (a pitch or base that is not a multiple of
  // 4): the ROCm kernel driver runs compute queues in the GPU's unaligned
  // access mode, which the compiler assumes for this target as well (it
  // turns a byte-aligned 4-byte copy into one dword store).  Streaming stores, as RGB is written once
  // and never read back here; except for islow 4:1:1, whose 48-byte rows
  // left the L2 as partial lines with them (1.63x the RGB bytes written;
  // ordinary stores write 1.00x at the same speed, while the AAN 4:1:1
  // kernels run 10% slower with ordinary stores and keep streaming ones).
  __device__ static void store_unit(gbl8* row, const uint32_t* w) {
    gbl32u* wd = reinterpret_cast<gbl32u*>(row);
    if constexpr (HF == 4 && C::ISLOW) {
#pragma unroll
      for (int kk = 0; kk < 3 * HF; ++kk) wd[kk] = w[kk];
    } else {
#pragma unroll
      for (int kk = 0; kk < 3 * HF; ++kk) __builtin_nontemporal_store(w[kk], &wd[kk]);
    }
  }

  // Ragged right edge: the first nbytes bytes of w (nbytes < 12*HF, a
  // partial unit), as its whole dwords and then a 16-bit and a byte store
  // for the last 1..3 bytes, all at any byte address (unaligned access
  // mode, as above; constant register indices).
  __device__ static void store_ragged(gbl8* row, const uint32_t* w, int nbytes) {
    gbl32u* wd = reinterpret_cast<gbl32u*>(row);
    const int nd = nbytes >> 2;  // whole dwords, at most 3*HF - 1
    uint32_t last = w[0];        // the dword holding the last 1..3 bytes
#pragma unroll
    for (int kk = 0; kk < 3 * HF - 1; ++kk) {
      if (kk < nd) wd[kk] = w[kk];
      if (kk + 1 == nd) last = w[kk + 1];
    }
    gbl8* tail = row + 4 * nd;
    if (nbytes & 2) *reinterpret_cast<gbl16u*>(tail) = static_cast<uint16_t>(last);
    if (nbytes & 1) tail[nbytes & 2] = static_cast<uint8_t>(last >> (8 * (nbytes & 2)));
  }

  // ---- the pipelined walk over one segment ----
  __device__ void run(const SegmentRange& seg) {
    mx0 = seg.mx0;
    nmx = min(SX, im.mcus_x - mx0);
    r0 = seg.r0;
    r1 = seg.r1;
    K = (r1 - r0 + SY - 1) / SY;
    gcx0 = 8 * mx0;

    __syncthreads();  // the previous segment's readers are done with every buffer
    __builtin_amdgcn_s_setprio(3);
    // Every wave but the last starts its own copies of sub-tile 0 at once.
    // The last wave loads the quant tables first (so its LDS writes wait
    // for those loads alone), then makes its own copies, and after the
    // barrier loads and forms the rows just above and below the segment
    // (vertical fancy filter) while the other waves wait for their blocks.
    // The first step has no barrier: each wave starts its transform once
    // its own blocks are in.
    constexpr int AUXW = NT / 64 - 1;
    constexpr int TBP = (N_TB + 63) / 64;  // passes over the neighbour blocks of one side
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (wv != AUXW) {
      dma(0);
      asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");  // quant tables visible
    } else {
      qtab_stores(qtab_loads());
      dma(0);
      asm volatile("s_waitcnt lgkmcnt(0)\n\ts_barrier" ::: "memory");  // quant tables visible
      if constexpr (HALO_Y) {
        // the rows just above and below the segment (phase 2 first reads
        // them a step later): their blocks straight into registers, loaded
        // after the other waves' first copies
        int pos[2][TBP], mx[2][TBP];
        bool tb[2][TBP];
        v4i rows[2][TBP][8];
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int p = 0; p < TBP; ++p) {
            const int t = 64 * p + (tid & 63);
            tb[b][p] = tb_block(b == 1, t, &pos[b][p], &mx[b][p]);
            if (tb[b][p]) tb_rows_global(b == 1, t, mx[b][p], rows[b][p]);
          }
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
          for (int p = 0; p < TBP; ++p)
            if (tb[b][p]) tb_row(b == 1, 64 * p + (tid & 63), pos[b][p], mx[b][p], rows[b][p]);
      }
    }

    for (int k = 0; k <= K; ++k) {
      // The staged registers get a fresh, opaque definition every step (no
      // instruction): lanes that stage nothing never read them, and the
      // compiler need not keep the last step's values alive across the
      // loop (which costs about 32 registers, and spills with 3 waves per
      // SIMD).
      Held h;
      asm("" : "=v"(h.r0), "=v"(h.r1), "=v"(h.r2), "=v"(h.r3), "=v"(h.r4), "=v"(h.r5), "=v"(h.r6), "=v"(h.r7));
      // Wait for this wave's copies of the sub-tile (the counter also
      // covers the RGB stores, so the last step skips it).
      if (k < K) asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
      // Phase 1 of the last step (and the rows above and below) visible.
      // Each wave copies and reads its own staging blocks, and phase 2 of
      // k and phase 1 of k use different luma and chroma slots, so a step
      // needs no other barrier.
      if (k > 0) __syncthreads();
      // Wave priority: the steps left, plus one in the last step for the
      // workgroups of the grid's second half (the later of two on a CU,
      // whose waves lose every tie on age), so the two end together.
      {
        const bool later = 2 * static_cast<int>(blockIdx.x) >= static_cast<int>(gridDim.x);
        const int pr = min(3, K - k + (later && k == K ? 1 : 0));
        if (pr >= 3) __builtin_amdgcn_s_setprio(3);
        else if (pr == 2) __builtin_amdgcn_s_setprio(2);
        else if (pr == 1) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
      }
      if (k < K) {
        read_stage(k, h);
        if (k + 1 < K) {
          asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");  // this wave's staging reads done
          dma(k + 1);
        }
      }
      // Phase 2 first, so its stores drain while the transform runs.
      if (k > 0) {
        if constexpr (HALO_Y) phase2_pairs(k);
        else phase2(k - 1);
      }
      // Phase 1 also finishes the neighbour-column blocks and the edge
      // copies in place, so its LDS writes only need to be visible at the
      // next step's barrier.
      if (k < K) phase1(k, h);
      if constexpr (HALO_Y && !LAST_IN_WALK)
        if (k == K) last_pair_rows();
    }
  }
};

}  // namespace mjd
