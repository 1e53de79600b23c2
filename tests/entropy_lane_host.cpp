// Runs the per-lane restart-interval decoder of the GPU entropy kernel on the
// CPU, through a memory environment that checks every access, so its logic
// can be compared with the oracle's reader and the host decoder without a
// GPU.  Usage: entropy_lane_host <in.jpg> <out.bin>
//   prints "<intervals> <intervals with a nonzero status>" and writes the
//   n_blocks * 64 int16 coefficients (MCU order) to out.bin.
// Exit status 3 on any out-of-range access, 2 on a parse error.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "entropy_lane.h"
#include "mjd.h"

using namespace mjd::gent;

namespace {

[[noreturn]] void out_of_range(const char* what) {
  fprintf(stderr, "out-of-range %s\n", what);
  exit(3);
}

struct CheckedTab {
  const GTables* tabs;
  uint32_t fast(int t, int i) const {
    if (t < 0 || t >= kTableSlots || i < 0 || i >= (1 << kGLook)) out_of_range("fast");
    return tabs->t[t].fast[i];
  }
  int lim(int t, int l) const {
    if (t < 0 || t >= kTableSlots || l <= kGLook || l > 16) out_of_range("lim");
    return tabs->t[t].lim[l];
  }
  int valoff(int t, int l) const {
    if (t < 0 || t >= kTableSlots || l <= kGLook || l > 16) out_of_range("valoff");
    return tabs->t[t].valoff[l];
  }
  int val(int t, int i) const {
    if (t < 0 || t >= kTableSlots || i < 0 || i > 255) out_of_range("val");
    return tabs->t[t].vals[i];
  }
  int nat(int k) const {
    if (k < 0 || k > 63) out_of_range("nat");
    return tabs->nat[k];
  }
};

struct CheckedBlk {
  int16_t buf[64];
  int16_t* coef;
  uint64_t block, n_blocks;
  void put(int i, int v) {
    if (i < 0 || i > 63) out_of_range("block index");
    buf[i] = static_cast<int16_t>(v);
  }
  void finish() {
    if (block >= n_blocks) out_of_range("block store");
    memcpy(coef + block * 64, buf, sizeof(buf));
    memset(buf, 0, sizeof(buf));
    ++block;
  }
};

// Chunk loads must stay inside the stream rounded up to 16 bytes (the
// buffer is padded with zeros to that length); ring accesses inside the
// ring.
struct CheckedMem {
  const uint8_t* jpg;
  uint32_t lim;
  uint8_t ring[kRing];
  uint8_t pend[2][16];
  void g_chunk(uint32_t p, int slot) {
    if ((p & 15) || p + 16 > lim || slot < 0 || slot > 1) out_of_range("chunk");
    memcpy(pend[slot], jpg + p, 16);
  }
  void commit(int slot, uint32_t off) {
    if ((off & 15) || off + 16 > kRing || slot < 0 || slot > 1) out_of_range("commit");
    memcpy(ring + off, pend[slot], 16);
  }
  uint32_t r_dword(uint32_t off) const {
    if ((off & 3) || off + 4 > kRing) out_of_range("ring dword");
    uint32_t d;
    memcpy(&d, ring + off, 4);
    return d;
  }
};

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  std::vector<uint8_t> jpg;
  for (int c; (c = fgetc(f)) != EOF;) jpg.push_back(static_cast<uint8_t>(c));
  fclose(f);
  mjd_scan scan;
  uint16_t qt[4][64];
  if (mjd_parse(jpg.data(), jpg.size(), &scan, qt) != MJD_OK) {
    fprintf(stderr, "parse: %s\n", mjd_last_error());
    return 2;
  }
  mjd_geometry g;
  if (mjd_geometry_of(&scan.frame, &g) != MJD_OK) return 2;
  std::vector<uint64_t> off(scan.n_intervals + 1);
  if (mjd_restart_index(jpg.data(), jpg.size(), &scan, off.data()) != MJD_OK) {
    fprintf(stderr, "restart index: %s\n", mjd_last_error());
    return 2;
  }
  std::vector<GTables> tabs(1);
  uint32_t tsel = 0;
  if (plan_gtables(scan, tabs.data(), &tsel) != kTableOk) {
    fprintf(stderr, "bad Huffman tables\n");
    return 2;
  }
  // zig-zag position -> natural index, walking the anti-diagonals
  {
    int k = 0;
    for (int s = 0; s < 15; ++s)
      for (int i = 0; i <= s; ++i) {
        const int r = (s & 1) ? i : s - i, c = s - r;
        if (r < 8 && c < 8) tabs[0].nat[k++] = static_cast<uint8_t>(8 * r + c);
      }
  }
  uint32_t comp_bits = 0;
  int bpm = 0;
  for (int c = 0; c < 3; ++c)
    for (int i = 0; i < scan.frame.h[c] * scan.frame.v[c]; ++i) comp_bits |= static_cast<uint32_t>(c) << (2 * bpm++);
  const uint64_t n_mcus = static_cast<uint64_t>(g.mcus_x) * g.mcus_y;
  std::vector<int16_t> coef(g.n_blocks * 64, 0);
  CheckedTab tab{tabs.data()};
  const uint64_t ri = scan.restart_interval ? scan.restart_interval : n_mcus;
  std::vector<uint8_t> padded(jpg);
  padded.resize((jpg.size() + 15) & ~size_t{15}, 0);
  uint32_t bad = 0;
  for (uint32_t s = 0; s < scan.n_intervals; ++s) {
    Interval iv;
    iv.start = static_cast<uint32_t>(off[s]);
    iv.end = static_cast<uint32_t>(off[s + 1] - 2);
    iv.mcu0 = s * ri;
    iv.n_mcus = static_cast<uint32_t>(n_mcus - iv.mcu0 < ri ? n_mcus - iv.mcu0 : ri);
    iv.index = s;
    CheckedBlk blk;
    memset(blk.buf, 0, sizeof(blk.buf));
    blk.coef = coef.data();
    blk.block = iv.mcu0 * static_cast<uint64_t>(bpm);
    blk.n_blocks = g.n_blocks;
    CheckedMem mem;
    mem.jpg = padded.data();
    mem.lim = static_cast<uint32_t>(padded.size());
    memset(mem.ring, 0xA5, sizeof(mem.ring));
    if (decode_interval(tab, blk, mem, mem.lim, iv, bpm, comp_bits, tsel) != kOk) ++bad;
  }
  f = fopen(argv[2], "wb");
  if (!f || fwrite(coef.data(), 2, coef.size(), f) != coef.size()) return 2;
  fclose(f);
  printf("%u %u\n", scan.n_intervals, bad);
  return 0;
}
