// Internal interface of the host entropy decoder, shared by the C entry
// points and the stream pipeline.
#pragma once

#include <stdint.h>

#include <string>

#include "host_pool.h"
#include "mjd.h"

namespace mjd {
namespace host {

constexpr int kLookBits = 10;  // look-ahead window of the table decoder

struct HuffTable {
  uint16_t lut[1 << kLookBits];   // (length << 8) | symbol for codes of <= kLookBits bits, else 0
  uint32_t fast[1 << kLookBits];  // AC: (value << 16) | (run << 8) | bits used, when code + magnitude fit
  int32_t maxcode[18];            // largest code of each length, -1 if none
  int32_t valoff[18];             // symbol index = code + valoff[length]
  uint8_t vals[256];
};

struct ScanTables {
  HuffTable dc[4], ac[4];
  bool dc_ok[4], ac_ok[4];
};

struct ScanLayout {
  uint32_t mcus_x, mcus_y;
  uint64_t n_mcus;
  int bpm;
  int comp_of[6];  // component of each block of an MCU
};

const uint8_t* zigzag_to_natural();
int build_table(const mjd_huffman& h, bool ac, HuffTable* t);
int scan_layout(const mjd_scan* scan, ScanLayout* L);
int build_tables(const mjd_scan* scan, ScanTables* T);
int parse(const uint8_t* d, size_t len, mjd_scan* scan, uint16_t qt[4][64]);
int restart_index(const uint8_t* jpg, size_t len, const mjd_scan* scan, uint64_t* off);

// Decodes restart interval s, storing the MCUs in [m_lo, m_hi) (others of
// the interval are decoded and dropped).  No thread-local state: on failure
// the message goes to *err and the status is returned.
int decode_interval(const uint8_t* jpg, const mjd_scan* scan, const ScanLayout& L, const ScanTables& T,
                    const uint64_t* offsets, uint32_t s, uint64_t m_lo, uint64_t m_hi, int16_t* coef,
                    std::string* err);

int decode_rows(const uint8_t* jpg, size_t len, const mjd_scan* scan, const uint64_t* offsets, int16_t* coef,
                uint32_t row0, uint32_t row1, int n_threads);

// One scan made ready for decoding MCU-row ranges: layout, tables, and the
// restart index checked against the stream once, for callers that decode an
// image in many ranges.  Holds pointers to jpg, scan and offsets.
struct RowDecoder {
  const uint8_t* jpg = nullptr;
  const mjd_scan* scan = nullptr;
  const uint64_t* offsets = nullptr;
  ScanLayout L;
  ScanTables T;
};
int prepare_rows(const uint8_t* jpg, size_t len, const mjd_scan* scan, const uint64_t* offsets, RowDecoder* out);

// Decodes MCU rows [row0, row1) into coef, one task per restart interval.
int decode_rows_with(const RowDecoder& D, int16_t* coef, uint32_t row0, uint32_t row1, const ParallelFor& pf);

}  // namespace host
}  // namespace mjd
