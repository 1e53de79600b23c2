// The performance model of the paper's Sec. 5.1: least-squares polynomial
// fits whose degree is chosen by the Akaike information criterion, Horner
// evaluation, and the prediction that composes them (Eqs. 3-4 and the
// split of the GPU time into host->device copy, kernel and device->host
// copy).  Host code only.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <vector>

#include "mjd.h"
#include "mjd_common.h"

namespace mjd {
namespace model {

constexpr double kExactFloor = 1e-24;  // relative residual counted as an exact fit

// Solves min |A c - y| for an n x k column-major A (n > k) by Householder
// QR.  Returns false when a column is (numerically) dependent on the others.
static bool lstsq(std::vector<double> A, std::vector<double> y, size_t n, size_t k, double* coef, double* rss) {
  for (size_t j = 0; j < k; ++j) {
    double* col = &A[j * n];
    double norm = 0.0, scale = 0.0;
    for (size_t i = j; i < n; ++i) scale = fmax(scale, fabs(col[i]));
    if (scale == 0.0) return false;
    for (size_t i = j; i < n; ++i) norm += (col[i] / scale) * (col[i] / scale);
    norm = scale * sqrt(norm);
    const double alpha = col[j] > 0 ? -norm : norm;
    // v = x - alpha e1, stored in col[j..n); R_jj = alpha
    col[j] -= alpha;
    double vv = 0.0;
    for (size_t i = j; i < n; ++i) vv += col[i] * col[i];
    if (vv == 0.0) return false;
    for (size_t c = j + 1; c < k; ++c) {
      double* other = &A[c * n];
      double dot = 0.0;
      for (size_t i = j; i < n; ++i) dot += col[i] * other[i];
      const double f = 2.0 * dot / vv;
      for (size_t i = j; i < n; ++i) other[i] -= f * col[i];
    }
    double dot = 0.0;
    for (size_t i = j; i < n; ++i) dot += col[i] * y[i];
    const double f = 2.0 * dot / vv;
    for (size_t i = j; i < n; ++i) y[i] -= f * col[i];
    col[j] = alpha;  // the diagonal of R
  }
  // conditioning: a diagonal entry far below the largest means dependence
  double dmax = 0.0;
  for (size_t j = 0; j < k; ++j) dmax = fmax(dmax, fabs(A[j * n + j]));
  for (size_t j = 0; j < k; ++j)
    if (fabs(A[j * n + j]) <= dmax * 1e-13) return false;
  for (size_t jj = k; jj-- > 0;) {
    double s = y[jj];
    for (size_t c = jj + 1; c < k; ++c) s -= A[c * n + jj] * coef[c];
    coef[jj] = s / A[jj * n + jj];
  }
  double r = 0.0;
  for (size_t i = k; i < n; ++i) r += y[i] * y[i];
  *rss = r;
  return true;
}

static double aic_of(double rss, double sumsq, size_t n, size_t k) {
  const double floor = kExactFloor * (sumsq > 0 ? sumsq : 1.0);
  const double r = rss > floor ? rss : floor;
  return static_cast<double>(n) * log(r / static_cast<double>(n)) + 2.0 * static_cast<double>(k);
}

static size_t terms2(int degree) { return static_cast<size_t>((degree + 1) * (degree + 2) / 2); }

static size_t t2(int degree, int i, int j) { return static_cast<size_t>(i * (2 * degree + 3 - i) / 2 + j); }

// d/db of a two-variable polynomial, in Horner form.
static double poly2_db(const mjd_poly2& p, double a, double b) {
  const int deg = p.degree;
  double r = 0.0;
  for (int i = deg; i >= 0; --i) {
    double q = 0.0;
    for (int j = deg - i; j >= 1; --j) q = q * b + j * p.c[t2(deg, i, j)];
    r = r * a + q;
  }
  return r;
}

// Both sides of a partition with x image rows on the CPU (after the part of
// Huffman decoding that precedes the split), and f = cpu - gpu with its
// derivative in x.
struct Sides {
  double cpu, gpu, f, df;
};

// One split problem: the rows h being shared (the GPU takes the first h - x),
// the Huffman terms of the CPU's side and a constant added to the GPU's.
struct Split {
  int scheme;
  double w, h;
  double hpp;          // the model's Huffman seconds per pixel at the image's density
  double n;            // huff_threads
  double chunk;        // PPS: rows of the GPU's first chunk
  double huff_fixed;   // re-partitioning: seconds of Huffman decoding of all remaining rows
  double gpu_fixed;    // re-partitioning: the earlier chunks' remaining device time
};

static Sides sides(const mjd_model& m, const Split& q, double x) {
  const double w = q.w, h = q.h;
  const double a = w / 1024.0, bc = x / 1024.0, bg = (h - x) / 1024.0;
  Sides s;
  const double pgpu = mjd_poly2_eval(&m.o_w, a, bg) + mjd_poly2_eval(&m.t_kernel, a, bg) + mjd_poly2_eval(&m.o_r, a, bg);
  const double dpgpu = poly2_db(m.o_w, a, bg) + poly2_db(m.t_kernel, a, bg) + poly2_db(m.o_r, a, bg);
  s.cpu = mjd_poly2_eval(&m.t_dispatch, a, bg) + mjd_poly2_eval(&m.p_cpu, a, bc) + q.huff_fixed;
  double dcpu = (-poly2_db(m.t_dispatch, a, bg) + poly2_db(m.p_cpu, a, bc)) / 1024.0;
  if (q.scheme == MJD_PART_OVERLAP) {  // the CPU's own rows
    s.cpu += q.hpp * w * x / q.n;
    dcpu += q.hpp * w / q.n;
  } else if (q.scheme == MJD_PART_PPS) {  // every row after the GPU's first chunk
    const double c = std::min(q.chunk, h - x);
    s.cpu += q.hpp * w * (h - c) / q.n;
    if (q.chunk > h - x) dcpu += q.hpp * w / q.n;
  }
  s.gpu = pgpu + q.gpu_fixed;
  s.f = s.cpu - s.gpu;
  s.df = dcpu + dpgpu / 1024.0;  // d/dx P_gpu(w, h - x) = -dP/db / 1024
  return s;
}

// Newton's method for f(x) = 0 on [0, h]: the ends when f keeps one sign,
// else from the middle, kept inside [0, h]; it stops when a step no longer
// reduces |f| or moves less than a quarter row.  Then the GPU keeps whole
// MCU rows: the nearest split on an MCU-row boundary of the h rows.
static void solve(const mjd_model& m, const Split& q, uint32_t rows, uint32_t mcu_h, mjd_partition* out) {
  const double h = q.h;
  uint32_t it = 0;
  double x;
  if (sides(m, q, 0.0).f >= 0.0) {
    x = 0.0;  // even no rows on the CPU finish no earlier than the GPU's share
  } else if (sides(m, q, h).f <= 0.0) {
    x = h;  // the CPU alone finishes first
  } else {
    x = h / 2;
    Sides cur = sides(m, q, x);
    for (it = 0; it < 100; ++it) {
      if (!(cur.df > 0.0)) break;
      double nx = x - cur.f / cur.df;
      nx = nx < 0.0 ? 0.0 : (nx > h ? h : nx);
      const Sides nxt = sides(m, q, nx);
      if (fabs(nxt.f) >= fabs(cur.f)) break;
      const double step = fabs(nx - x);
      x = nx;
      cur = nxt;
      if (step < 0.25) {
        ++it;
        break;
      }
    }
  }
  // the splits are k * mcu_h for k < the MCU rows, and all the rows (the
  // last MCU row may be partial): take the nearest to h - x
  const double target = h - x;
  const uint32_t mcus = (rows + mcu_h - 1) / mcu_h;
  const uint32_t k = std::min(mcus, static_cast<uint32_t>(target / mcu_h));
  const uint32_t lo = std::min(rows, k * mcu_h), hi = std::min(rows, (k + 1) * mcu_h);
  const uint32_t gpu_rows = target - lo <= hi - target ? lo : hi;
  out->cpu_rows = rows - gpu_rows;
  out->iterations = it;
  out->x = x;
  const Sides fin = sides(m, q, static_cast<double>(out->cpu_rows));
  out->t_cpu = out->cpu_rows ? fin.cpu : 0.0;
  out->t_gpu = gpu_rows ? fin.gpu : 0.0;
}

}  // namespace model
}  // namespace mjd

using namespace mjd::model;

extern "C" {

int mjd_poly1_fit(const double* x, const double* y, size_t n, int max_degree, mjd_poly1* out, double* aic) {
  if (!x || !y || !out) return mjd::fail(MJD_EINVAL, "null sample or output pointer");
  if (max_degree < 0 || max_degree > MJD_POLY_MAX_DEGREE)
    return mjd::fail(MJD_EINVAL, "polynomial degree %d outside 0..%d", max_degree, MJD_POLY_MAX_DEGREE);
  if (n < 2) return mjd::fail(MJD_EINVAL, "%zu samples: at least 2 are needed", n);
  double sumsq = 0.0;
  for (size_t i = 0; i < n; ++i) sumsq += y[i] * y[i];
  bool found = false;
  double best = 0.0;
  for (int deg = 0; deg <= max_degree; ++deg) {
    const size_t k = static_cast<size_t>(deg) + 1;
    if (k >= n) break;
    std::vector<double> A(n * k);
    for (size_t i = 0; i < n; ++i) {
      double p = 1.0;
      for (size_t j = 0; j < k; ++j) {
        A[j * n + i] = p;
        p *= x[i];
      }
    }
    double c[MJD_POLY_MAX_DEGREE + 1] = {0};
    double rss = 0.0;
    if (!lstsq(A, std::vector<double>(y, y + n), n, k, c, &rss)) continue;
    const double a = aic_of(rss, sumsq, n, k);
    if (!found || a < best) {
      found = true;
      best = a;
      memset(out, 0, sizeof(*out));
      out->degree = deg;
      for (size_t j = 0; j < k; ++j) out->c[j] = c[j];
    }
  }
  if (!found) return mjd::fail(MJD_EUNSUPPORTED, "no polynomial degree could be fitted");
  if (aic) *aic = best;
  return MJD_OK;
}

int mjd_poly2_fit(const double* a, const double* b, const double* y, size_t n, int max_degree, mjd_poly2* out,
                  double* aic) {
  if (!a || !b || !y || !out) return mjd::fail(MJD_EINVAL, "null sample or output pointer");
  if (max_degree < 0 || max_degree > MJD_POLY_MAX_DEGREE)
    return mjd::fail(MJD_EINVAL, "polynomial degree %d outside 0..%d", max_degree, MJD_POLY_MAX_DEGREE);
  if (n < 2) return mjd::fail(MJD_EINVAL, "%zu samples: at least 2 are needed", n);
  double sumsq = 0.0;
  for (size_t i = 0; i < n; ++i) sumsq += y[i] * y[i];
  bool found = false;
  double best = 0.0;
  for (int deg = 0; deg <= max_degree; ++deg) {
    const size_t k = terms2(deg);
    if (k >= n) break;
    std::vector<double> A(n * k);
    for (size_t r = 0; r < n; ++r) {
      double pa = 1.0;
      for (int i = 0; i <= deg; ++i) {
        double pb = 1.0;
        for (int j = 0; j <= deg - i; ++j) {
          A[t2(deg, i, j) * n + r] = pa * pb;
          pb *= b[r];
        }
        pa *= a[r];
      }
    }
    double c[MJD_POLY2_TERMS] = {0};
    double rss = 0.0;
    if (!lstsq(A, std::vector<double>(y, y + n), n, k, c, &rss)) continue;
    const double v = aic_of(rss, sumsq, n, k);
    if (!found || v < best) {
      found = true;
      best = v;
      memset(out, 0, sizeof(*out));
      out->degree = deg;
      for (size_t j = 0; j < k; ++j) out->c[j] = c[j];
    }
  }
  if (!found) return mjd::fail(MJD_EUNSUPPORTED, "no polynomial degree could be fitted");
  if (aic) *aic = best;
  return MJD_OK;
}

double mjd_poly1_eval(const mjd_poly1* p, double x) {
  if (!p || p->degree < 0 || p->degree > MJD_POLY_MAX_DEGREE) return NAN;
  double r = 0.0;
  for (int i = p->degree; i >= 0; --i) r = r * x + p->c[i];
  return r;
}

double mjd_poly2_eval(const mjd_poly2* p, double a, double b) {
  if (!p || p->degree < 0 || p->degree > MJD_POLY_MAX_DEGREE) return NAN;
  const int deg = p->degree;
  double r = 0.0;
  for (int i = deg; i >= 0; --i) {
    double q = 0.0;  // the coefficient of a^i, a polynomial in b
    for (int j = deg - i; j >= 0; --j) q = q * b + p->c[t2(deg, i, j)];
    r = r * a + q;
  }
  return r;
}

int mjd_model_predict(const mjd_model* m, uint32_t width, uint32_t height, uint64_t file_bytes,
                      mjd_prediction* out) {
  if (!m || !out) return mjd::fail(MJD_EINVAL, "null model or output pointer");
  if (!width || !height) return mjd::fail(MJD_EINVAL, "zero image dimension");
  const double px = static_cast<double>(width) * static_cast<double>(height);
  const double a = width / 1024.0, b = height / 1024.0;
  out->d = static_cast<double>(file_bytes) / px;
  out->t_huff = mjd_poly1_eval(&m->huff_per_pixel, out->d) * px;
  out->o_w = mjd_poly2_eval(&m->o_w, a, b);
  out->t_kernel = mjd_poly2_eval(&m->t_kernel, a, b);
  out->o_r = mjd_poly2_eval(&m->o_r, a, b);
  out->p_gpu = out->o_w + out->t_kernel + out->o_r;
  out->total = out->t_huff + out->p_gpu;
  out->p_cpu = mjd_poly2_eval(&m->p_cpu, a, b);
  out->t_dispatch = mjd_poly2_eval(&m->t_dispatch, a, b);
  return MJD_OK;
}

int mjd_partition_rows(const mjd_model* m, int scheme, uint32_t width, uint32_t height, uint32_t mcu_h,
                       uint64_t file_bytes, double huff_threads, uint32_t chunk_rows, mjd_partition* out) {
  if (!m || !out) return mjd::fail(MJD_EINVAL, "null model or output pointer");
  if (!width || !height || (mcu_h != 8 && mcu_h != 16)) return mjd::fail(MJD_EINVAL, "bad image or MCU height");
  if (scheme != MJD_PART_SPS && scheme != MJD_PART_OVERLAP && scheme != MJD_PART_PPS)
    return mjd::fail(MJD_EINVAL, "unknown scheme %d", scheme);
  if (!(huff_threads >= 1.0)) return mjd::fail(MJD_EINVAL, "huff_threads below 1");
  if (scheme == MJD_PART_PPS && !chunk_rows) return mjd::fail(MJD_EINVAL, "PPS needs a chunk height");
  const double w = width, h = height;
  Split q{scheme, w, h, mjd_poly1_eval(&m->huff_per_pixel, static_cast<double>(file_bytes) / (w * h)), huff_threads,
          static_cast<double>(chunk_rows), 0.0, 0.0};
  solve(*m, q, height, mcu_h, out);
  return MJD_OK;
}

int mjd_repartition_rows(const mjd_model* m, uint32_t width, uint32_t height, uint32_t rows_left, uint32_t mcu_h,
                         uint64_t file_bytes, double huff_threads, uint32_t huff_rows_left, double huff_done_s,
                         double gpu_busy_s, mjd_partition* out) {
  if (!m || !out) return mjd::fail(MJD_EINVAL, "null model or output pointer");
  if (!width || !height || (mcu_h != 8 && mcu_h != 16)) return mjd::fail(MJD_EINVAL, "bad image or MCU height");
  if (!rows_left || rows_left > height || huff_rows_left > height)
    return mjd::fail(MJD_EINVAL, "remaining rows outside 1..height");
  if (!(huff_threads >= 1.0) || !(huff_done_s >= 0.0) || !(gpu_busy_s >= 0.0))
    return mjd::fail(MJD_EINVAL, "negative time or huff_threads below 1");
  const double w = width, h = height;
  const double d = static_cast<double>(file_bytes) / (w * h);
  const double est = mjd_poly1_eval(&m->huff_per_pixel, d) * w * h / huff_threads;
  // Eq. 17: the density of the rows still to decode, from the share of the
  // estimated Huffman time left against the share of the height left
  double d_new = 0.0;
  if (huff_rows_left && est > 0.0)
    d_new = std::max(0.0, est - huff_done_s) / est / (huff_rows_left / h) * d;
  Split q{MJD_PART_SPS, w, static_cast<double>(rows_left), 0.0, huff_threads, 0.0,
          mjd_poly1_eval(&m->huff_per_pixel, d_new) * w * huff_rows_left / huff_threads, gpu_busy_s};
  solve(*m, q, rows_left, mcu_h, out);
  return MJD_OK;
}

}  // extern "C"
