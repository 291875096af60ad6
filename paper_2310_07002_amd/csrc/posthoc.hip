// Post-hoc diagnostics of stored log predictive draws (host code).
//
// Algorithm 1 keeps every post-warm-up draw s[k, l, i]; from one fold's L x N
// draws this computes the two-pass estimates (elpd, pooled and batch-means
// variances of f = e^s, eqs est-e, bmvar, clt) and three R-hats: the paper's
// (eq rhat), split R-hat (each chain's halves as separate chains) and the
// rank-normalised split R-hat of Vehtari, Gelman, Simpson, Carpenter and
// Buerkner (2021), the larger of its bulk and folded versions.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

#include "pcv_internal.h"

namespace pcv {
namespace {

// R-hat of chains x[m][n] (row-major), eq rhat.
double rhat_rows(const std::vector<double>& x, int m, int64_t n) {
  std::vector<double> mean(m, 0.0);
  double W = 0.0;
  for (int j = 0; j < m; ++j) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += x[j * n + i];
    mean[j] = s / n;
    double v = 0.0;
    for (int64_t i = 0; i < n; ++i) v += (x[j * n + i] - mean[j]) * (x[j * n + i] - mean[j]);
    W += v / (n - 1);
  }
  W /= m;
  double g = 0.0;
  for (int j = 0; j < m; ++j) g += mean[j];
  g /= m;
  double B = 0.0;
  for (int j = 0; j < m; ++j) B += (mean[j] - g) * (mean[j] - g);
  B *= static_cast<double>(n) / (m - 1);
  return std::sqrt((n - 1.0) / n + B / (n * W));
}

// Chains x[L][N] -> 2L half chains of h = N/2 (middle draw dropped if N is odd).
double split_rhat(const std::vector<double>& x, int L, int64_t N) {
  const int64_t h = N / 2;
  std::vector<double> y(static_cast<size_t>(2 * L) * h);
  for (int l = 0; l < L; ++l)
    for (int64_t i = 0; i < h; ++i) {
      y[(2 * l) * h + i] = x[l * N + i];
      y[(2 * l + 1) * h + i] = x[l * N + (N - h) + i];
    }
  return rhat_rows(y, 2 * L, h);
}

// Standard normal quantile: Acklam's rational approximation, refined by one
// Halley step on the exact cdf 0.5 erfc(-x/sqrt 2).
double norm_ppf(double p) {
  static const double a[] = {-3.969683028665376e+01, 2.209460984245205e+02, -2.759285104469687e+02,
                             1.383577518672690e+02, -3.066479806614716e+01, 2.506628277459239e+00};
  static const double b[] = {-5.447609879822406e+01, 1.615858368580409e+02, -1.556989798598866e+02,
                             6.680131188771972e+01, -1.328068155288572e+01};
  static const double c[] = {-7.784894002430293e-03, -3.223964580411365e-01, -2.400758277161838e+00,
                             -2.549732539343734e+00, 4.374664141464968e+00, 2.938163982698783e+00};
  static const double d[] = {7.784695709041462e-03, 3.224671290700398e-01, 2.445134137142996e+00,
                             3.754408661907416e+00};
  const double plow = 0.02425, phigh = 1 - plow;
  double x;
  if (p < plow) {
    const double q = std::sqrt(-2 * std::log(p));
    x = (((((c[0] * q + c[1]) * q + c[2]) * q + c[3]) * q + c[4]) * q + c[5]) /
        ((((d[0] * q + d[1]) * q + d[2]) * q + d[3]) * q + 1);
  } else if (p <= phigh) {
    const double q = p - 0.5, r = q * q;
    x = (((((a[0] * r + a[1]) * r + a[2]) * r + a[3]) * r + a[4]) * r + a[5]) * q /
        (((((b[0] * r + b[1]) * r + b[2]) * r + b[3]) * r + b[4]) * r + 1);
  } else {
    const double q = std::sqrt(-2 * std::log(1 - p));
    x = -(((((c[0] * q + c[1]) * q + c[2]) * q + c[3]) * q + c[4]) * q + c[5]) /
        ((((d[0] * q + d[1]) * q + d[2]) * q + d[3]) * q + 1);
  }
  const double e = 0.5 * std::erfc(-x / std::sqrt(2.0)) - p;
  const double u = e * std::sqrt(2 * M_PI) * std::exp(x * x / 2);
  return x - u / (1 + x * u / 2);
}

// Normal scores of ranks (ties averaged): Phi^-1((r - 3/8) / (S + 1/4)).
std::vector<double> normal_scores(const std::vector<double>& x) {
  const size_t S = x.size();
  std::vector<size_t> idx(S);
  std::iota(idx.begin(), idx.end(), 0);
  std::stable_sort(idx.begin(), idx.end(), [&](size_t i, size_t j) { return x[i] < x[j]; });
  std::vector<double> z(S);
  for (size_t i = 0; i < S;) {
    size_t j = i;
    while (j + 1 < S && x[idx[j + 1]] == x[idx[i]]) ++j;
    const double r = 0.5 * static_cast<double>(i + 1 + j + 1);   // average rank of the tie run
    const double v = norm_ppf((r - 0.375) / (static_cast<double>(S) + 0.25));
    for (size_t k = i; k <= j; ++k) z[idx[k]] = v;
    i = j + 1;
  }
  return z;
}

double median(std::vector<double> x) {
  const size_t n = x.size(), h = n / 2;
  std::nth_element(x.begin(), x.begin() + h, x.end());
  const double hi = x[h];
  if (n % 2) return hi;
  return 0.5 * (hi + *std::max_element(x.begin(), x.begin() + h));
}

}  // namespace

void posthoc_fold(const double* s, int L, int64_t N, int b, PosthocFold& out) {
  const size_t S = static_cast<size_t>(L) * N;
  std::vector<double> x(s, s + S);
  out.rhat = rhat_rows(x, L, N);
  out.split_rhat = split_rhat(x, L, N);
  std::vector<double> folded(S);
  const double med = median(x);
  for (size_t i = 0; i < S; ++i) folded[i] = std::fabs(x[i] - med);
  out.rank_rhat = std::max(split_rhat(normal_scores(x), L, N), split_rhat(normal_scores(folded), L, N));
  // f = e^s relative to the fold's largest draw
  const double mx = *std::max_element(x.begin(), x.end());
  double f1 = 0.0, f2 = 0.0;
  for (size_t i = 0; i < S; ++i) {
    const double f = std::exp(x[i] - mx);
    f1 += f;
    f2 += f * f;
  }
  const double fhat = f1 / S;
  out.log_fhat = mx + std::log(fhat);
  out.s2rel = (f2 - f1 * f1 / S) / (S - 1.0) / (fhat * fhat);
  const int64_t a = N / b;
  out.sig2rel = NAN;
  if (a >= 1 && L * a > 1) {
    std::vector<double> bm(static_cast<size_t>(L) * a);
    double g = 0.0;
    for (int l = 0; l < L; ++l)
      for (int64_t h = 0; h < a; ++h) {
        double t = 0.0;
        for (int i = 0; i < b; ++i) t += std::exp(x[l * N + h * b + i] - mx);
        bm[l * a + h] = t / b;
        g += t / b;
      }
    g /= static_cast<double>(L * a);
    double ss = 0.0;
    for (double v : bm) ss += (v - g) * (v - g);
    out.sig2rel = static_cast<double>(b) / (L * a - 1.0) * ss / (fhat * fhat);
  }
}

}  // namespace pcv
