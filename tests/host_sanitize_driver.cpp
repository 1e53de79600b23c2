// Drives the library's host-only C++ (the JPEG parser, the restart index,
// the threaded Huffman decoder, the host back half, the worker pool and the
// performance-model fits) for a sanitizer build: AddressSanitizer with
// UndefinedBehaviorSanitizer, or ThreadSanitizer.  Built by
// tests/test_host_sanitizers.py together with the library's host sources.
//
//   host_sanitize_driver DIR N
// reads DIR/s0.jpg .. DIR/s{N-1}.jpg; for each it checks that 1 and 8
// threads decode the same coefficients and RGB, that a band decode writes
// the same blocks, that a stream with a damaged restart interval reports
// MJD_ECORRUPT while every other interval decodes as before, and writes the
// 8-thread RGB to DIR/s{i}.rgb.  Exit status 0 when every check holds.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <atomic>
#include <string>
#include <thread>
#include <vector>

#include "host_pool.h"
#include "mjd.h"

static std::atomic<int> g_fail{0};
#define CHECK(cond, ...)                       \
  do {                                         \
    if (!(cond)) {                             \
      fprintf(stderr, "check failed: " __VA_ARGS__); \
      fprintf(stderr, "\n");                   \
      ++g_fail;                                \
    }                                          \
  } while (0)

static std::vector<uint8_t> read_file(const std::string& path) {
  std::vector<uint8_t> d;
  FILE* f = fopen(path.c_str(), "rb");
  if (!f) return d;
  fseek(f, 0, SEEK_END);
  const long n = ftell(f);
  fseek(f, 0, SEEK_SET);
  d.resize(static_cast<size_t>(n));
  if (n > 0 && fread(d.data(), 1, d.size(), f) != d.size()) d.clear();
  fclose(f);
  return d;
}

static void one_stream(const std::string& dir, int i) {
  const std::string name = dir + "/s" + std::to_string(i);
  std::vector<uint8_t> jpg = read_file(name + ".jpg");
  CHECK(!jpg.empty(), "%s.jpg unreadable", name.c_str());
  if (jpg.empty()) return;
  mjd_scan scan;
  uint16_t qt[4][64];
  int rc = mjd_parse(jpg.data(), jpg.size(), &scan, qt);
  CHECK(rc == MJD_OK, "parse %s: %s", name.c_str(), mjd_last_error());
  if (rc != MJD_OK) return;
  std::vector<uint64_t> off(scan.n_intervals + 1);
  rc = mjd_restart_index(jpg.data(), jpg.size(), &scan, off.data());
  CHECK(rc == MJD_OK, "restart index %s: %s", name.c_str(), mjd_last_error());
  mjd_geometry g;
  CHECK(mjd_geometry_of(&scan.frame, &g) == MJD_OK, "geometry");
  const size_t nc = static_cast<size_t>(g.n_blocks) * 64;
  std::vector<int16_t> c1(nc, 0), c8(nc, 0), band(nc, 0x5555);
  CHECK(mjd_entropy_decode(jpg.data(), jpg.size(), &scan, off.data(), c1.data(), 0, g.mcus_y, 1) == MJD_OK,
        "entropy 1 thread: %s", mjd_last_error());
  CHECK(mjd_entropy_decode(jpg.data(), jpg.size(), &scan, nullptr, c8.data(), 0, g.mcus_y, 8) == MJD_OK,
        "entropy 8 threads: %s", mjd_last_error());
  CHECK(c1 == c8, "%s: 1 and 8 threads differ", name.c_str());
  // a band in the middle: only its blocks are written, and they match
  const uint32_t r0 = g.mcus_y / 3, r1 = g.mcus_y - g.mcus_y / 4;
  if (r0 < r1) {
    CHECK(mjd_entropy_decode(jpg.data(), jpg.size(), &scan, off.data(), band.data(), r0, r1, 8) == MJD_OK,
          "band decode: %s", mjd_last_error());
    const size_t row_coefs = static_cast<size_t>(g.mcus_x) * g.blocks_per_mcu * 64;
    for (size_t k = 0; k < nc; ++k) {
      const bool inside = k >= r0 * row_coefs && k < r1 * row_coefs;
      if (inside ? band[k] != c1[k] : band[k] != 0x5555) {
        CHECK(false, "%s: band [%u,%u) wrong at coefficient %zu", name.c_str(), r0, r1, k);
        break;
      }
    }
  }
  // the host back half, 1 and 8 threads
  const size_t pitch = 3 * static_cast<size_t>(scan.frame.width);
  std::vector<uint8_t> rgb1(pitch * scan.frame.height), rgb8(pitch * scan.frame.height);
  CHECK(mjd_decode_host(&scan.frame, c1.data(), &qt[0][0], MJD_UPSAMPLE_FANCY, rgb1.data(), pitch, 0, g.mcus_y, 1) ==
            MJD_OK,
        "host decode 1 thread: %s", mjd_last_error());
  CHECK(mjd_decode_host(&scan.frame, c8.data(), &qt[0][0], MJD_UPSAMPLE_FANCY, rgb8.data(), pitch, 0, g.mcus_y, 8) ==
            MJD_OK,
        "host decode 8 threads: %s", mjd_last_error());
  CHECK(rgb1 == rgb8, "%s: host decode 1 and 8 threads differ", name.c_str());
  FILE* f = fopen((name + ".rgb").c_str(), "wb");
  if (f) {
    fwrite(rgb8.data(), 1, rgb8.size(), f);
    fclose(f);
  }
  // a damaged restart interval: MJD_ECORRUPT, the other intervals unchanged
  if (scan.n_intervals >= 3) {
    std::vector<uint8_t> bad = jpg;
    const uint64_t a = off[1], b = off[2] - 2;  // interval 1's entropy-coded bytes
    // all-ones bits (0xFF with its stuffed 0x00): no Huffman code is all ones
    for (uint64_t p = a; p < b; ++p) bad[p] = ((p - a) & 1) == 0 && p + 1 < b ? 0xFF : 0x00;
    std::vector<int16_t> cb(nc, 0x2222);
    rc = mjd_entropy_decode(bad.data(), bad.size(), &scan, off.data(), cb.data(), 0, g.mcus_y, 8);
    CHECK(rc == MJD_ECORRUPT || rc == MJD_OK, "damaged stream: unexpected status %d", rc);
    const size_t per_mcu = static_cast<size_t>(g.blocks_per_mcu) * 64;
    const size_t iv = scan.restart_interval;
    for (size_t m = 0; m < static_cast<size_t>(g.mcus_x) * g.mcus_y; ++m) {
      const size_t interval = m / iv;
      if (interval == 1) continue;
      if (memcmp(&cb[m * per_mcu], &c1[m * per_mcu], per_mcu * sizeof(int16_t)) != 0) {
        CHECK(false, "%s: damaged stream changed MCU %zu of interval %zu", name.c_str(), m, interval);
        break;
      }
    }
  }
}

static void pool_checks() {
  mjd::WorkerPool pool(8);
  std::vector<long> part(64);
  for (int round = 0; round < 200; ++round) {
    pool.run(64, [&](int t) { part[t] = static_cast<long>(t) * round; });
    long s = 0;
    for (long v : part) s += v;
    CHECK(s == 2016L * round, "worker pool round %d summed %ld", round, s);
  }
  std::atomic<long> total{0};
  mjd::spawn_for(8, 1000, [&](int t) { total.fetch_add(t, std::memory_order_relaxed); });
  CHECK(total.load() == 499500, "spawn_for summed %ld", total.load());
}

static void model_checks() {
  // fits from several threads at once (each on its own data)
  std::vector<std::thread> th;
  std::atomic<int> bad{0};
  for (int t = 0; t < 6; ++t)
    th.emplace_back([t, &bad] {
      std::vector<double> a, b, y1, y2;
      for (int i = 0; i < 60; ++i) {
        const double x = 0.1 * (i + 1) + 0.01 * t, z = 0.05 * ((i * 7) % 13 + 1);
        a.push_back(x);
        b.push_back(z);
        y1.push_back(2.0 + 0.5 * x - 0.25 * x * x);
        y2.push_back(1.0 + x + 2.0 * z + 0.5 * x * z);
      }
      mjd_poly1 p1;
      mjd_poly2 p2;
      double aic1 = 0, aic2 = 0;
      if (mjd_poly1_fit(a.data(), y1.data(), a.size(), 4, &p1, &aic1) != MJD_OK) ++bad;
      if (mjd_poly2_fit(a.data(), b.data(), y2.data(), a.size(), 3, &p2, &aic2) != MJD_OK) ++bad;
      for (size_t i = 0; i < a.size(); ++i) {
        if (fabs(mjd_poly1_eval(&p1, a[i]) - y1[i]) > 1e-6) ++bad;
        if (fabs(mjd_poly2_eval(&p2, a[i], b[i]) - y2[i]) > 1e-6) ++bad;
      }
    });
  for (auto& x : th) x.join();
  CHECK(bad.load() == 0, "%d model fit checks failed", bad.load());
}

int main(int argc, char** argv) {
  if (argc < 3) {
    fprintf(stderr, "usage: %s DIR N\n", argv[0]);
    return 2;
  }
  const int n = atoi(argv[2]);
  std::vector<std::thread> th;  // the streams are decoded concurrently too
  for (int i = 0; i < n; ++i) th.emplace_back(one_stream, std::string(argv[1]), i);
  for (auto& t : th) t.join();
  pool_checks();
  model_checks();
  if (g_fail.load()) fprintf(stderr, "%d checks failed\n", g_fail.load());
  return g_fail.load() ? 1 : 0;
}
