// Huffman decoding of one restart interval of a baseline scan, written once
// for one GPU lane and, through small memory interfaces, for a CPU caller
// too.  The paper leaves entropy decoding on the CPU because code words have
// variable length (Sec. 1); restart intervals restart the bit stream and the
// DC predictions, so each of them decodes on its own (ITU-T T.81 restart
// markers).
//
// A lane advances one Huffman symbol per call of lane_step, so that the 64
// lanes of a wave, each in its own interval, run the same short path:
// - one 16-bit table entry gives the length, zero run and magnitude size of
//   any code of at most kGLook bits, and the magnitude bits are read from
//   the same 32-bit window (T.81 F.1.2.2, F.2.2.1);
// - longer codes take their length from the left-aligned code-space limits
//   of the canonical code (T.81 Annex C), without a loop over lengths;
// - a finished block leaves through the block interface.
// The stream comes through StreamRing, which serves bytes from a per-lane
// ring filled ahead of use at points the whole wave reaches together, so
// that loads are issued well before any lane waits for them.
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

constexpr int kGLook = 10;  // look-ahead bits of the first-level table

// Interval status; kRunning is internal to lane_step.
enum : uint32_t { kOk = 0, kBadCode = 1, kBadRun = 2, kOverrun = 3, kRunning = 4 };

// One restart interval: its entropy-coded bytes [start, end) (end is the
// first byte of the marker that closes it) and its MCUs.
struct Interval {
  uint32_t start, end;
  uint32_t n_mcus;
  uint32_t index;  // interval number within its scan
  uint64_t mcu0;
};

// Entry of the first-level table (index: the next kGLook bits):
//   0                no code of at most kGLook bits starts there
//   bits 0-4         code length
//   bits 5-8         magnitude size (AC: low nibble of the symbol; DC: the
//                    symbol); size 0 in an AC table is EOB, or ZRL with run 15
//   bits 9-12        zero run (AC: high nibble of the symbol)
//   kBadSym          a DC symbol above 11
constexpr uint32_t kBadSym = 1u << 13;

struct GHuff {
  uint16_t fast[1 << kGLook];
  int32_t lim[17];     // lim[l]: codes of length <= l fill [0, lim[l]) of the 16-bit left-aligned code space
  int32_t valoff[17];  // symbol index = code + valoff[length]
  uint8_t vals[256];
  uint8_t pad[8];
};

// A scan's distinct tables in up to four slots (a baseline scan uses at
// most two DC and two AC tables, T.81 B.2.4.2) and the zig-zag map.  The
// slot of each component's tables is packed in a word, four bits per
// component: DC slot in bits 4c..4c+1, AC slot in bits 4c+2..4c+3.
constexpr int kTableSlots = 4;
struct GTables {
  GHuff t[kTableSlots];
  uint8_t nat[64];  // natural index of zig-zag position k
};
static_assert(sizeof(GHuff) % 16 == 0 && sizeof(GTables) % 16 == 0, "tables copy as 16-byte chunks");

MJD_HD inline int extend_value(int raw, int s) { return raw < (1 << (s - 1)) ? raw - (1 << s) + 1 : raw; }

enum : int { kTableOk = 0, kTableUndefined = 1, kTableTooMany = 2, kTableOverfull = 3 };

// Builds a table from its DHT code counts and symbols (canonical codes,
// T.81 Annex C).
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
        const uint32_t sym = h.vals[k];
        const uint32_t e = ac ? static_cast<uint32_t>(l) | (sym & 15u) << 5 | (sym >> 4) << 9
                              : static_cast<uint32_t>(l) | (sym & 15u) << 5 | (sym > 11 ? kBadSym : 0u);
        const int lo = code << (kGLook - l), hi = (code + 1) << (kGLook - l);
        for (int p = lo; p < hi; ++p) t->fast[p] = static_cast<uint16_t>(e);
      }
      ++code;
      ++k;
    }
    t->lim[l] = code << (16 - l);
    code <<= 1;
  }
  return kTableOk;
}

enum : int { kPlanTooManyTables = 4 };

// Builds the distinct tables a scan selects into slots and returns their
// component map in *tsel; kTableOk or the first table error, or
// kPlanTooManyTables when the scan needs more than kTableSlots tables.
inline int plan_gtables(const mjd_scan& scan, GTables* g, uint32_t* tsel) {
  memset(g, 0, sizeof(*g));
  int key[kTableSlots];
  int n = 0;
  uint32_t sel = 0;
  for (int c = 0; c < 3; ++c) {
    for (int ac = 0; ac < 2; ++ac) {
      const int id = ac ? scan.ac_sel[c] : scan.dc_sel[c];
      const int k = ac * 4 + id;
      int slot = -1;
      for (int i = 0; i < n; ++i)
        if (key[i] == k) slot = i;
      if (slot < 0) {
        if (n == kTableSlots) return kPlanTooManyTables;
        const int rc = build_gtable(ac ? scan.ac[id] : scan.dc[id], ac != 0, &g->t[n]);
        if (rc != kTableOk) return rc;
        key[n] = k;
        slot = n++;
      }
      sel |= static_cast<uint32_t>(slot) << (4 * c + 2 * ac);
    }
  }
  *tsel = sel;
  return kTableOk;
}

// Stream bytes of one lane, all read from a ring of kRing bytes that holds
// stream bytes [lo, have) at offsets p % kRing.  Mem supplies
//   void g_chunk(uint32_t p, int slot)   start loading stream bytes
//                                        [p, p + 16) (p a multiple of 16)
//                                        into slot 0/1
//   void commit(int slot, uint32_t off)  put that chunk in the ring at off
//   uint32_t r_dword(uint32_t off)       ring read (off a multiple of 4)
// refill(p) commits the chunks the previous refill loaded and starts up to
// two more, each only where the ring bytes it will overwrite lie below p,
// the next byte the reader needs.  Chunks are loaded while they start
// below `lim`, the stream length rounded up to 16.  The reader never reads
// the stream directly: a lane whose ring lacks the next bytes waits for the
// next refill (ready()).
constexpr uint32_t kRing = 32;

template <class Mem>
struct StreamRing {
  Mem& mem;
  uint32_t lim;
  uint32_t lo, have;
  uint32_t npend = 0;

  MJD_HD StreamRing(Mem& m, uint32_t lim_, uint32_t start) : mem(m), lim(lim_) { lo = have = start & ~15u; }

  // Stream bytes [a, a + 12) as three little-endian words (a a multiple of
  // 4); bytes the ring does not hold yet come back stale and are not used.
  MJD_HD void triple(uint32_t a, uint32_t& d0, uint32_t& d1, uint32_t& d2) {
    d0 = mem.r_dword(a % kRing);
    d1 = mem.r_dword((a + 4) % kRing);
    d2 = mem.r_dword((a + 8) % kRing);
  }

  // The ring holds every byte one refill of the bit window can read: eight
  // bytes from p (four data bytes, each possibly stuffed), or up to `end`.
  MJD_HD bool ready(uint32_t p, uint32_t end) const { return have >= (p + 8 < end ? p + 8 : end); }

  MJD_HD void refill(uint32_t p) {
    if (npend > 0) {
      mem.commit(0, have % kRing);
      have += 16;
    }
    if (npend > 1) {
      mem.commit(1, have % kRing);
      have += 16;
    }
    if (have - lo > kRing) lo = have - kRing;
    npend = 0;
    if (have + 16 <= p + kRing && have < lim) {
      mem.g_chunk(have, 0);
      npend = 1;
      if (have + 32 <= p + kRing && have + 16 < lim) {
        mem.g_chunk(have + 16, 1);
        npend = 2;
      }
    }
  }
};

// Bytes sh..sh+3 of the little-endian pair (d0, d1), first byte most
// significant.
MJD_HD inline uint32_t be32_at(uint32_t d0, uint32_t d1, uint32_t sh) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_perm(d1, d0, 0x00010203u + sh * 0x01010101u);
#else
  const uint64_t v = ((static_cast<uint64_t>(d1) << 32) | d0) >> (8 * sh);
  const uint32_t x = static_cast<uint32_t>(v);
  return (x >> 24) | ((x >> 8) & 0xFF00u) | ((x << 8) & 0xFF0000u) | (x << 24);
#endif
}

// Byte x (0..11) of the little-endian words d0, d1, d2.
MJD_HD inline uint32_t byte_of3(uint32_t d0, uint32_t d1, uint32_t d2, uint32_t x) {
  const uint32_t w = x < 4 ? d0 : (x < 8 ? d1 : d2);
  return (w >> (8 * (x & 3u))) & 0xFFu;
}

// Bit reader over [p, end): MSB-first window w0:w1 with `pos` bits of w0
// used; stuffed 0x00 after 0xFF dropped; at a marker or at `end` it feeds
// zero bits.  `fed` counts real bits and `used` consumed bits, so used > fed
// means the interval ran out of data.  The next stream words (at p) are read
// from the ring at the start of every step, beside the table lookup, and
// used when the step's bits cross into w1.
template <class Ring>
struct LaneBits {
  Ring& ring;
  uint32_t p, end;
  uint32_t w0 = 0, w1 = 0;
  uint32_t pos = 0;
  uint32_t fed = 0, used = 0;
  bool stop = false;

  MJD_HD LaneBits(Ring& r, uint32_t start, uint32_t end_) : ring(r), p(start), end(end_) {}

  MJD_HD void fetch(uint32_t& d0, uint32_t& d1, uint32_t& d2) { ring.triple(p & ~3u, d0, d1, d2); }

  MJD_HD void prime() {
    uint32_t d0, d1, d2;
    fetch(d0, d1, d2);
    w0 = next32(d0, d1, d2);
    fetch(d0, d1, d2);
    w1 = next32(d0, d1, d2);
  }

  // The next 32 stream bits, MSB first, from the words read at p & ~3:
  // four bytes at once wherever none of them is 0xFF, else byte by byte
  // without branches (stuffed zeros dropped; a marker or `end` stops the
  // stream).
  MJD_HD uint32_t next32(uint32_t d0, uint32_t d1, uint32_t d2) {
    const uint32_t sh = p & 3u;
    if (!stop && p + 4 <= end) {
      const uint32_t d = be32_at(d0, d1, sh);
      const uint32_t x = ~d;  // 0xFF bytes become zero bytes
      if (((x - 0x01010101u) & ~x & 0x80808080u) == 0) {
        p += 4;
        fed += 32;
        return d;
      }
    }
    uint32_t r = 0, q = p;
    bool st = stop;
    for (int i = 0; i < 4; ++i) {
      const uint32_t o = q - (p & ~3u);  // at most 3 + 6
      const uint32_t b = byte_of3(d0, d1, d2, o), nb = byte_of3(d0, d1, d2, o + 1);
      const bool ff = b == 0xFFu;
      const bool stuffed = ff && q + 1 < end && nb == 0;
      st = st || q >= end || (ff && !stuffed);
      r = (r << 8) | (st ? 0u : b);
      q += st ? 0u : (stuffed ? 2u : 1u);
      fed += st ? 0u : 8u;
    }
    p = q;
    stop = st;
    return r;
  }

  // The next 32 bits of the window (at least 33 are held), not consumed.
  MJD_HD uint32_t peek32() const { return pos ? (w0 << pos) | (w1 >> (32u - pos)) : w0; }

  // Consumes n <= 31 bits; d0..d2 are the words fetch() read this step.
  MJD_HD void consume(uint32_t n, uint32_t d0, uint32_t d1, uint32_t d2) {
    used += n;
    pos += n;
    if (pos >= 32u) {
      pos -= 32u;
      w0 = w1;
      w1 = next32(d0, d1, d2);
    }
  }
};

// Decoding position of one lane inside its interval.
struct LaneState {
  uint32_t m = 0, n_mcus = 0;
  int b = 0, k = 0;
  int pred0 = 0, pred1 = 0, pred2 = 0;
};

// One symbol of the lane's interval.  Tab supplies
//   uint32_t fast(int t, int i), int lim(int t, int l), int valoff(int t, int l),
//   int val(int t, int i), int nat(int k)
// (t: a table slot), and Blk
//   void put(int natural_index, int value), void finish()  (store the block,
//   clear the buffer for the next one).
// comp_bits holds the component of block b of an MCU in bits 2b..2b+1 and
// tsel the table slots of each component (plan_gtables).
// Returns kRunning, kOk after the interval's last MCU, or the first error.
// The step has one exit and computes every case with the same operations
// where it can, so that lanes in different cases stay together.
template <class Tab, class Blk, class Ring>
MJD_HD inline uint32_t lane_step(const Tab& tab, Blk& blk, LaneBits<Ring>& br, LaneState& st, int bpm,
                                 uint32_t comp_bits, uint32_t tsel) {
  if (!br.ring.ready(br.p, br.end)) return kRunning;  // wait for the next refill
  const int comp = static_cast<int>((comp_bits >> (2 * st.b)) & 3u);
  const bool dc = st.k == 0;
  const int t = static_cast<int>((tsel >> (4 * comp + (dc ? 0 : 2))) & 3u);
  uint32_t d0, d1, d2;
  br.fetch(d0, d1, d2);
  const uint32_t top = br.peek32();
  const uint32_t e = tab.fast(t, static_cast<int>(top >> (32 - kGLook)));
  uint32_t len = e & 31u, sz = (e >> 5) & 15u, run = (e >> 9) & 15u;
  bool bad = (e & kBadSym) != 0;
  if (e == 0) {
    // a code longer than kGLook bits: its length is one more than the
    // number of left-aligned limits the next 16 bits reach
    const int w = static_cast<int>(top >> 16);
    int l = kGLook + 1;
    for (int j = kGLook + 1; j <= 16; ++j) l += w >= tab.lim(t, j) ? 1 : 0;
    const int lc = l > 16 ? 16 : l;
    const int idx = (w >> (16 - lc)) + tab.valoff(t, lc);
    const bool ok = l <= 16 && idx >= 0 && idx <= 255;
    const uint32_t sym = ok ? static_cast<uint32_t>(tab.val(t, idx)) : 0u;
    bad = !ok || (dc && sym > 11);
    len = static_cast<uint32_t>(lc);
    sz = sym & 15u;
    run = dc ? 0u : sym >> 4;
    if (dc && sym > 15) sz = 0;
  }
  // the magnitude bits follow the code inside the 32-bit window
  const int raw = sz ? static_cast<int>((top << len) >> (32 - sz)) : 0;
  const int half = static_cast<int>((1u << sz) >> 1);
  int val = raw < half ? raw - 2 * half + 1 : raw;  // EXTEND (T.81 F.2.2.1)
  br.consume(len + sz, d0, d1, d2);
  if (dc) {
    // DC prediction per component (T.81 F.2.1.3), kept in three registers
    // and chosen by masks (a select would become an indexed stack load)
    const int m0 = -static_cast<int>(comp == 0), m1 = -static_cast<int>(comp == 1), m2 = -static_cast<int>(comp == 2);
    const int p = ((st.pred0 & m0) | (st.pred1 & m1) | (st.pred2 & m2)) + val;
    st.pred0 = (p & m0) | (st.pred0 & ~m0);
    st.pred1 = (p & m1) | (st.pred1 & ~m1);
    st.pred2 = (p & m2) | (st.pred2 & ~m2);
    val = p;
  }
  // A coefficient lands at k + run.  EOB (size 0, run below 15) and ZRL
  // (size 0, run 15) write a zero at a position not yet reached, which is
  // still zero, so the store stays unconditional.
  const bool skip = !dc && sz == 0;
  const int kk = st.k + static_cast<int>(run);
  blk.put(tab.nat(kk < 63 ? kk : 63), skip ? 0 : val);
  const bool eob = skip && run != 15;
  uint32_t status = bad ? kBadCode : (!skip && kk > 63) ? kBadRun : kRunning;
  st.k = eob ? 64 : kk + 1;
  if (status == kRunning && st.k >= 64) {
    blk.finish();
    st.k = 0;
    if (++st.b == bpm) {
      st.b = 0;
      if (br.used > br.fed) status = kOverrun;
      else if (++st.m == st.n_mcus) status = kOk;
    }
  }
  return status;
}

// Every kRefillEvery steps the ring commits and restarts its loads.
constexpr uint32_t kRefillEvery = 4;

// Decodes interval iv of a stream whose bytes may be loaded up to `lim`
// (its length rounded up to 16): the ring is filled (two chunks, waited
// for) and the bit window primed, then one symbol per step until the last
// MCU or an error.  A step either waits for data, which the next refill
// brings, or advances the block position by at least one coefficient, so
// the loop ends within about 64 + 8 steps per block.
template <class Tab, class Blk, class Mem>
MJD_HD inline uint32_t decode_interval(const Tab& tab, Blk& blk, Mem& mem, uint32_t lim, const Interval& iv, int bpm,
                                       uint32_t comp_bits, uint32_t tsel) {
  StreamRing<Mem> ring(mem, lim, iv.start);
  LaneBits<StreamRing<Mem>> br(ring, iv.start, iv.end);
  ring.refill(iv.start);
  ring.refill(iv.start);
  br.prime();
  LaneState st;
  st.n_mcus = iv.n_mcus;
  uint32_t s = iv.n_mcus ? kRunning : kOk;
  for (uint32_t it = 1; s == kRunning; ++it) {
    if (it % kRefillEvery == 0) ring.refill(br.p);
    s = lane_step(tab, blk, br, st, bpm, comp_bits, tsel);
  }
  return s;
}

}  // namespace gent
}  // namespace mjd
