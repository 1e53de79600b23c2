// Huffman decoding of one restart interval of a baseline scan, written once
// for one GPU lane and, through the memory environment `Env`, for any other
// caller.  The paper leaves entropy decoding on the CPU because code words
// have variable length (Sec. 1); restart intervals restart the bit stream
// and the DC predictions, so each of them decodes on its own (ITU-T T.81
// restart markers).
//
// Env supplies:
//   uint32_t lut(int t, int i)     (length << 8) | symbol for codes of at most
//                                  kGLook bits (index: the next kGLook bits),
//                                  0 for longer codes
//   uint32_t fast(int t, int i)    AC: (value << 16) | (run << 8) | bits used
//                                  when code and magnitude fit kGLook bits
//   int maxcode(int t, int l), valoff(int t, int l), val(int t, int i)
//                                  the canonical code walk for longer codes
//   int nat(int k)                 natural index of zig-zag position k
//   uint32_t byte(uint64_t p)      stream byte p
//   uint32_t dword(uint64_t p)     stream bytes p..p+3 as a little-endian
//                                  word (p is a multiple of 4)
//   void blk_clear(), blk_put(int natural_index, int value),
//   blk_store(uint64_t block)      the block being decoded and its output
// Tables t = component (DC) and 3 + component (AC).
#pragma once

#include <stdint.h>
#include <string.h>

#include "mjd.h"

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define MJD_HD __host__ __device__
#else
#define MJD_HD
#endif

namespace mjd {
namespace gent {

constexpr int kGLook = 9;  // look-ahead window of the GPU tables

enum : uint32_t { kOk = 0, kBadCode = 1, kBadRun = 2, kOverrun = 3 };

// One restart interval: its entropy-coded bytes [start, end) (end is the
// first byte of the marker that closes it) and its MCUs.
struct Interval {
  uint64_t start, end;
  uint64_t mcu0;
  uint32_t n_mcus;
  uint32_t job;
};

// Bit reader over [p, end): MSB-first window w0:w1 with `pos` bits of w0
// used; stuffed 0x00 after 0xFF dropped; at a marker or at `end` it feeds
// zero bits.  `fed` counts real bits, `used` consumed bits, so used > fed
// means the interval ran out of data.
template <class Env>
struct LaneBits {
  Env& env;
  uint64_t p, end;
  uint32_t w0 = 0, w1 = 0;
  uint32_t pos = 0;
  uint32_t fed = 0, used = 0;
  bool stop = false;

  MJD_HD LaneBits(Env& e, uint64_t start, uint64_t end_) : env(e), p(start), end(end_) {
    w0 = next32();
    w1 = next32();
  }

  MJD_HD uint32_t next_byte() {
    if (stop || p >= end) {
      stop = true;
      return 0;
    }
    const uint32_t b = env.byte(p++);
    if (b == 0xFF) {
      if (p < end && env.byte(p) == 0x00) {
        ++p;
        fed += 8;
        return 0xFF;
      }
      stop = true;
      return 0;
    }
    fed += 8;
    return b;
  }

  // The next 32 stream bits, MSB first.
  MJD_HD uint32_t next32() {
    if (!stop && (p & 3u) == 0 && p + 4 <= end) {
      const uint32_t d = env.dword(p);
      const uint32_t x = ~d;  // 0xFF bytes become zero bytes
      if (((x - 0x01010101u) & ~x & 0x80808080u) == 0) {
        p += 4;
        fed += 32;
        return (d >> 24) | ((d >> 8) & 0xFF00u) | ((d << 8) & 0xFF0000u) | (d << 24);
      }
    }
    uint32_t r = 0;
    for (int i = 0; i < 4; ++i) r = (r << 8) | next_byte();
    return r;
  }

  // The next n bits (1 <= n <= 16) as an unsigned value, not consumed.
  MJD_HD uint32_t peek(uint32_t n) const {
    const uint32_t top = pos ? (w0 << pos) | (w1 >> (32u - pos)) : w0;
    return top >> (32u - n);
  }

  MJD_HD void consume(uint32_t n) {
    used += n;
    pos += n;
    if (pos >= 32u) {
      pos -= 32u;
      w0 = w1;
      w1 = next32();
    }
  }
};

MJD_HD inline int extend_value(int raw, int s) { return raw < (1 << (s - 1)) ? raw - (1 << s) + 1 : raw; }

// One Huffman table in the form the lanes read.
struct GHuff {
  uint16_t lut[1 << kGLook];
  uint32_t fast[1 << kGLook];
  int32_t maxcode[18];
  int32_t valoff[18];
  uint8_t vals[256];
};

// A scan's tables, per component: DC of components 0..2, then AC, and the
// zig-zag map.
struct GTables {
  GHuff t[6];
  uint8_t nat[64];  // natural index of zig-zag position k
};
static_assert(sizeof(GTables) % 16 == 0, "tables copy as 16-byte chunks");

enum : int { kTableOk = 0, kTableUndefined = 1, kTableTooMany = 2, kTableOverfull = 3 };

// Builds a table from its DHT code counts and symbols (canonical codes,
// ITU-T T.81 Annex C): the look-ahead table, the AC fast table (a code and
// its magnitude bits together within kGLook bits) and the per-length code
// limits for longer codes.
inline int build_gtable(const mjd_huffman& h, bool ac, GHuff* t) {
  memset(t, 0, sizeof(*t));
  if (!h.defined) return kTableUndefined;
  int n = 0;
  for (int l = 0; l < 16; ++l) n += h.bits[l];
  if (n > 256) return kTableTooMany;
  memcpy(t->vals, h.vals, sizeof(t->vals));
  int32_t code = 0;
  int k = 0;
  for (int l = 1; l <= 16; ++l) {
    t->valoff[l] = k - code;
    for (int i = 0; i < h.bits[l - 1]; ++i) {
      if (code >= (1 << l)) return kTableOverfull;
      if (l <= kGLook) {
        const int lo = code << (kGLook - l), hi = (code + 1) << (kGLook - l);
        for (int p = lo; p < hi; ++p) t->lut[p] = static_cast<uint16_t>((l << 8) | h.vals[k]);
      }
      ++code;
      ++k;
    }
    t->maxcode[l] = h.bits[l - 1] ? code - 1 : -1;
    code <<= 1;
  }
  t->maxcode[17] = -1;
  if (ac) {
    for (int p = 0; p < (1 << kGLook); ++p) {
      const int e = t->lut[p];
      if (!e) continue;
      const int l = e >> 8, sym = e & 0xFF, run = sym >> 4, s = sym & 15;
      if (s == 0 || l + s > kGLook) continue;
      const int raw = (p >> (kGLook - l - s)) & ((1 << s) - 1);
      const int v = extend_value(raw, s);
      t->fast[p] = (static_cast<uint32_t>(static_cast<uint16_t>(static_cast<int16_t>(v))) << 16) |
                   static_cast<uint32_t>(run << 8) | static_cast<uint32_t>(l + s);
    }
  }
  return kTableOk;
}

// The next Huffman symbol of table t, or -1 for a code the table lacks.
template <class Env>
MJD_HD inline int lane_symbol(Env& env, LaneBits<Env>& br, int t) {
  const uint32_t e = env.lut(t, static_cast<int>(br.peek(kGLook)));
  if (e) {
    br.consume(e >> 8);
    return static_cast<int>(e & 0xFFu);
  }
  const int w = static_cast<int>(br.peek(16));
  for (int l = kGLook + 1; l <= 16; ++l) {
    const int c = w >> (16 - l);
    if (c <= env.maxcode(t, l)) {
      br.consume(static_cast<uint32_t>(l));
      const int idx = c + env.valoff(t, l);
      return (idx >= 0 && idx < 256) ? env.val(t, idx) : -1;
    }
  }
  return -1;
}

// Decodes interval `iv`: every block of its MCUs goes to Env::blk_store in
// MCU order (block index mcu * bpm + b).  comp_of[b]: component of block b
// of an MCU.  Returns kOk or the first error; the loops are bounded by the
// interval's MCU count and 64 coefficients per block.
template <class Env>
MJD_HD inline uint32_t decode_interval_lane(Env& env, const Interval& iv, int bpm, const uint8_t* comp_of) {
  LaneBits<Env> br(env, iv.start, iv.end);
  int pred[3] = {0, 0, 0};
  for (uint32_t m = 0; m < iv.n_mcus; ++m) {
    for (int b = 0; b < bpm; ++b) {
      const int comp = comp_of[b];
      env.blk_clear();
      const int s = lane_symbol(env, br, comp);
      if (s < 0 || s > 11) return kBadCode;
      if (s) {
        const int raw = static_cast<int>(br.peek(static_cast<uint32_t>(s)));
        br.consume(static_cast<uint32_t>(s));
        pred[comp] += extend_value(raw, s);
      }
      env.blk_put(0, pred[comp]);
      const int act = 3 + comp;
      for (int k = 1; k < 64;) {
        const uint32_t f = env.fast(act, static_cast<int>(br.peek(kGLook)));
        if (f) {
          br.consume(f & 0xFFu);
          k += static_cast<int>((f >> 8) & 0xFFu);
          if (k > 63) return kBadRun;
          env.blk_put(env.nat(k), static_cast<int>(static_cast<int16_t>(f >> 16)));
          ++k;
          continue;
        }
        const int rs = lane_symbol(env, br, act);
        if (rs < 0) return kBadCode;
        const int r = rs >> 4, sz = rs & 15;
        if (sz == 0) {
          if (r == 15) {  // ZRL: sixteen zeros
            k += 16;
            continue;
          }
          break;  // EOB
        }
        k += r;
        if (k > 63) return kBadRun;
        const int raw = static_cast<int>(br.peek(static_cast<uint32_t>(sz)));
        br.consume(static_cast<uint32_t>(sz));
        env.blk_put(env.nat(k), extend_value(raw, sz));
        ++k;
      }
      env.blk_store((iv.mcu0 + m) * static_cast<uint64_t>(bpm) + static_cast<uint64_t>(b));
    }
    if (br.used > br.fed) return kOverrun;
  }
  return kOk;
}

}  // namespace gent
}  // namespace mjd
