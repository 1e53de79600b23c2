// Baseline Huffman entropy coder for the synthetic bitstream corpus
// (T.81 F.1.2): per-block DC difference categories and AC (run, size)
// symbols in zig-zag order, 0xFF stuffing, 1-bit padding and RSTn markers
// at every restart interval.  The Python writer in synth/bitstream.py does
// the same; this one is here because the corpus holds billions of pixels.
// It is test-input generation, not part of the decoder.
#include <stdint.h>
#include <string.h>

#include <algorithm>

namespace {

struct ZigZag {
  uint8_t nat[64];
  ZigZag() {
    int k = 0;
    for (int d = 0; d < 15; ++d) {
      const int lo = std::max(0, d - 7), hi = std::min(d, 7);
      for (int i = 0; i <= hi - lo; ++i) {
        // odd anti-diagonals go down-left (row increasing), even ones up-right
        const int row = (d & 1) ? lo + i : hi - i;
        nat[k++] = static_cast<uint8_t>(8 * row + (d - row));
      }
    }
  }
};
const ZigZag kZZ;

inline int category(int v) {
  unsigned a = static_cast<unsigned>(v < 0 ? -v : v);
  int s = 0;
  while (a) {
    ++s;
    a >>= 1;
  }
  return s;
}

struct Writer {
  uint8_t* out;
  uint64_t cap, n = 0;
  uint64_t acc = 0;
  int nbits = 0;
  bool overflow = false;
  void byte(uint8_t b) {
    if (n < cap) out[n] = b;
    else overflow = true;
    ++n;
  }
  void put(uint32_t value, int bits) {
    if (!bits) return;
    acc = (acc << bits) | (value & ((1u << bits) - 1));
    nbits += bits;
    while (nbits >= 8) {
      nbits -= 8;
      const uint8_t b = static_cast<uint8_t>(acc >> nbits);
      byte(b);
      if (b == 0xFF) byte(0x00);
    }
    acc &= (nbits ? ((1ull << nbits) - 1) : 0);
  }
  void pad_ones() {
    if (nbits) put((1u << (8 - nbits)) - 1, 8 - nbits);
  }
};

template <class Sink>
void walk(const int16_t* coef, uint64_t n_mcu, int bpm, const uint8_t* tbl, const uint8_t* comp,
          uint32_t restart_interval, Sink& sink) {
  int pred[4] = {0, 0, 0, 0};
  for (uint64_t m = 0; m < n_mcu; ++m) {
    if (restart_interval && m % restart_interval == 0) {
      if (m) sink.restart(static_cast<int>(((m / restart_interval) - 1) & 7));
      pred[0] = pred[1] = pred[2] = pred[3] = 0;
    }
    for (int b = 0; b < bpm; ++b) {
      const int16_t* blk = coef + (m * bpm + b) * 64;
      const int t = tbl[b], c = comp[b];
      const int diff = blk[0] - pred[c];
      pred[c] = blk[0];
      const int s = category(diff);
      sink.symbol(2 * t, s);
      sink.bits(diff < 0 ? diff + (1 << s) - 1 : diff, s);
      int run = 0;
      int last = 0;
      for (int k = 63; k > 0; --k)
        if (blk[kZZ.nat[k]]) {
          last = k;
          break;
        }
      for (int k = 1; k <= last; ++k) {
        const int v = blk[kZZ.nat[k]];
        if (!v) {
          ++run;
          continue;
        }
        while (run > 15) {
          sink.symbol(2 * t + 1, 0xF0);
          run -= 16;
        }
        const int sz = category(v);
        sink.symbol(2 * t + 1, (run << 4) | sz);
        sink.bits(v < 0 ? v + (1 << sz) - 1 : v, sz);
        run = 0;
      }
      if (last != 63) sink.symbol(2 * t + 1, 0x00);
    }
  }
}

struct Counter {
  uint32_t* counts;
  void restart(int) {}
  void symbol(int table, int sym) { ++counts[table * 256 + sym]; }
  void bits(int, int) {}
};

struct Encoder {
  Writer w;
  const uint16_t* codes;
  const uint8_t* lens;
  bool missing = false;
  void restart(int k) {
    w.pad_ones();
    w.byte(0xFF);
    w.byte(static_cast<uint8_t>(0xD0 + k));
  }
  void symbol(int table, int sym) {
    const int l = lens[table * 256 + sym];
    if (!l) missing = true;
    w.put(codes[table * 256 + sym], l);
  }
  void bits(int v, int n) { w.put(static_cast<uint32_t>(v), n); }
};

}  // namespace

extern "C" {

// counts: uint32[4][256] = DC table 0, AC table 0, DC table 1, AC table 1.
// tbl[b]: Huffman table (0/1) of block b of an MCU; comp[b]: its component.
int se_symbol_counts(const int16_t* coef, uint64_t n_mcu, int bpm, const uint8_t* tbl, const uint8_t* comp,
                     uint32_t restart_interval, uint32_t* counts) {
  if (!coef || !tbl || !comp || !counts || bpm < 1 || bpm > 6) return -1;
  memset(counts, 0, 4 * 256 * sizeof(uint32_t));
  Counter c{counts};
  walk(coef, n_mcu, bpm, tbl, comp, restart_interval, c);
  return 0;
}

// Writes the entropy-coded data (with RSTn markers, without EOI) to out.
// Returns its length, -1 if it does not fit in cap bytes, -2 if a symbol
// has no code, -3 for bad arguments.
int64_t se_encode(const int16_t* coef, uint64_t n_mcu, int bpm, const uint8_t* tbl, const uint8_t* comp,
                  uint32_t restart_interval, const uint16_t* codes, const uint8_t* lens, uint8_t* out,
                  uint64_t cap) {
  if (!coef || !tbl || !comp || !codes || !lens || !out || bpm < 1 || bpm > 6) return -3;
  Encoder e{Writer{out, cap}, codes, lens};
  walk(coef, n_mcu, bpm, tbl, comp, restart_interval, e);
  e.w.pad_ones();
  if (e.missing) return -2;
  if (e.w.overflow) return -1;
  return static_cast<int64_t>(e.w.n);
}

}  // extern "C"
