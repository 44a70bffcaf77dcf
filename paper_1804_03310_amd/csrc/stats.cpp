// Host-side statistics of energy series (no device work): the blocking
// analysis that gives error bars to correlated series (Sec. II remark on
// long population-controlled runs; Flyvbjerg-Petersen blocking) and the
// correlated-sampling energy difference with its error bar over independent
// repeats (Sec. I and Sec. V).  Fixed summation order.
#include <cmath>
#include <limits>
#include <vector>

#include "afqmc.h"

namespace afq {
afqmc_status set_error(afqmc_status s, const char* msg);
}

extern "C" {

afqmc_status afqmc_reblock(const double* x, int n, int max_levels, double* mean, double* sem,
                           int* n_levels, int* plateau) {
  if (!x || !mean || !sem || !n_levels || !plateau || n < 2 || max_levels < 1)
    return afq::set_error(AFQMC_ERR_ARG, "reblock: NULL pointer, n < 2 or max_levels < 1");
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return afq::set_error(AFQMC_ERR_NONFINITE, "reblock: non-finite value");
  double s = 0.0;
  for (int i = 0; i < n; ++i) s += x[i];
  *mean = s / n;
  std::vector<double> lv(x, x + n), err;
  int nl = 0;
  while ((int)lv.size() >= 2 && nl < max_levels) {
    const int m = (int)lv.size();
    double a = 0.0;
    for (int i = 0; i < m; ++i) a += lv[i];
    a /= m;
    double v = 0.0;
    for (int i = 0; i < m; ++i) v += (lv[i] - a) * (lv[i] - a);
    v /= (m - 1);
    sem[nl] = std::sqrt(v / m);
    err.push_back(sem[nl] / std::sqrt(2.0 * (m - 1)));
    ++nl;
    const int h = m / 2;
    for (int i = 0; i < h; ++i) lv[i] = 0.5 * (lv[2 * i] + lv[2 * i + 1]);
    lv.resize(h);
  }
  *n_levels = nl;
  *plateau = -1;
  for (int k = 0; k + 1 < nl; ++k)
    if (sem[k + 1] - sem[k] <= err[k]) {
      *plateau = k;
      break;
    }
  return AFQMC_OK;
}

afqmc_status afqmc_cs_difference(const double* a, const double* b, int repeats, int steps,
                                 int first, double* mean, double* sem) {
  if (!a || !b || !mean || !sem || repeats < 1 || steps < 1 || first < 0)
    return afq::set_error(AFQMC_ERR_ARG, "cs_difference: NULL pointer or bad sizes");
  const double nan = std::numeric_limits<double>::quiet_NaN();
  std::vector<double> cum((size_t)repeats * steps, nan);
  for (int r = 0; r < repeats; ++r) {
    double s = 0.0;
    long cnt = 0;
    for (int t = 0; t < steps; ++t) {
      const double av = a[(size_t)r * steps + t], bv = b[(size_t)r * steps + t];
      if (t >= first && std::isfinite(av) && std::isfinite(bv)) {
        s += bv - av;
        ++cnt;
      }
      if (t >= first && cnt > 0) cum[(size_t)r * steps + t] = s / cnt;
    }
  }
  for (int t = 0; t < steps; ++t) {
    mean[t] = nan;
    sem[t] = nan;
    bool ok = true;
    double m = 0.0;
    for (int r = 0; r < repeats; ++r) {
      const double c = cum[(size_t)r * steps + t];
      if (!std::isfinite(c)) { ok = false; break; }
      m += c;
    }
    if (!ok) continue;
    m /= repeats;
    mean[t] = m;
    if (repeats >= 2) {
      double v = 0.0;
      for (int r = 0; r < repeats; ++r) {
        const double d = cum[(size_t)r * steps + t] - m;
        v += d * d;
      }
      sem[t] = std::sqrt(v / ((double)repeats * (repeats - 1)));
    }
  }
  return AFQMC_OK;
}

}  // extern "C"
