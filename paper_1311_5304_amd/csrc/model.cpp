// The performance model of the paper's Sec. 5.1: least-squares polynomial
// fits whose degree is chosen by the Akaike information criterion, Horner
// evaluation, and the prediction that composes them (Eqs. 3-4 and the
// split of the GPU time into host->device copy, kernel and device->host
// copy).  Host code only.
#include <math.h>
#include <string.h>

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
  return MJD_OK;
}

}  // extern "C"
