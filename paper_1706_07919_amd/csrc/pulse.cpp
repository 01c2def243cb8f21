// Fourier coefficients of periodic incident pulse trains (Sec. IV: the
// fundamental pulse of Eq. pulse is replicated into an infinite train, sampled
// at N_f points per period and transformed by a DFT; the time origin enters as
// the phase factor e^{i beta}).  Host code; n_k * T complex exponentials.
#include <algorithm>
#include <cmath>
#include <complex>
#include <vector>

#include "../../include/bem.h"

namespace {

double pulse_value(int kind, const double* p, double s) {
  switch (kind) {
    case 0: {  // sin(tau) e^{-alpha |tau|} on |tau| < 2 pi N_c, tau = (8 pi N_c / w) s
      double Nc = p[0], alpha = p[1], w = p[2];
      double tau = (8.0 * M_PI * Nc / w) * s;
      return std::fabs(tau) < 2.0 * M_PI * Nc ? std::sin(tau) * std::exp(-alpha * std::fabs(tau)) : 0.0;
    }
    case 1: {
      double sg = p[0];
      return std::exp(-(s * s) / (2.0 * sg * sg));
    }
    case 2: {
      double sg = p[0];
      double q = (s * s) / (sg * sg);
      return (1.0 - q) * std::exp(-0.5 * q);
    }
    case 3: {
      double sg = p[0];
      return std::fabs(s) <= sg ? s / sg : 0.0;
    }
    case 4: {
      double ka = p[0], kb = p[1], D = p[2];
      return std::sin(ka * s + (kb - ka) * (s * s) / (2.0 * D)) * std::exp(-(s * s) / (2.0 * D * D));
    }
    case 5: {
      double k0 = p[0], sg = p[1];
      return std::sin(k0 * s) * std::exp(-(s * s) / (2.0 * sg * sg));
    }
  }
  return 0.0;
}

const int kParams[7] = {3, 1, 1, 1, 3, 2, 2};

}  // namespace

extern "C" bem_status bem_pulse_coeffs(int32_t kind, const double* params, int32_t n_params,
                                       double dk, int32_t n_k, int32_t T, double z_shift,
                                       double* c_out) {
  if (kind < 0 || kind > 6 || !params || n_params < kParams[kind] || !(dk > 0.0) ||
      !std::isfinite(dk) || n_k <= 0 || T <= 0 || !c_out || !std::isfinite(z_shift))
    return BEM_EINVAL;
  if (kind == 6) {
    double k0 = params[0], wd = params[1];
    if (!(wd > 0.0)) return BEM_EINVAL;
    for (int m = 1; m <= n_k; ++m) {
      double k = dk * m;
      double a = std::exp(-((k - k0) * (k - k0)) / (2.0 * wd * wd));
      std::complex<double> c = a * std::polar(1.0, -k * z_shift);
      c_out[2 * (m - 1)] = c.real();
      c_out[2 * (m - 1) + 1] = c.imag();
    }
    return BEM_OK;
  }
  const double L = 2.0 * M_PI / dk;
  std::vector<double> s(T), F(T);
  for (int n = 0; n < T; ++n) {
    s[n] = -0.5 * L + n * (L / T);
    F[n] = pulse_value(kind, params, s[n]);
  }
  for (int m = 1; m <= n_k; ++m) {
    const double k = dk * m;
    double re = 0.0, im = 0.0;
    for (int n = 0; n < T; ++n) {
      if (F[n] == 0.0) continue;
      re += F[n] * std::cos(k * s[n]);
      im -= F[n] * std::sin(k * s[n]);
    }
    std::complex<double> c = std::complex<double>(re / T, im / T) * std::polar(1.0, -k * z_shift);
    c_out[2 * (m - 1)] = c.real();
    c_out[2 * (m - 1) + 1] = c.imag();
  }
  return BEM_OK;
}

extern "C" bem_status bem_pulse_dominant(const double* c, int32_t n_k, int32_t n_keep,
                                         int32_t* m_index) {
  if (!c || !m_index || n_k <= 0 || n_keep <= 0 || n_keep > n_k) return BEM_EINVAL;
  std::vector<double> mag(n_k);
  for (int m = 0; m < n_k; ++m) {
    if (!std::isfinite(c[2 * m]) || !std::isfinite(c[2 * m + 1])) return BEM_EINVAL;
    mag[m] = std::hypot(c[2 * m], c[2 * m + 1]);
  }
  std::vector<int32_t> order(n_k);
  for (int m = 0; m < n_k; ++m) order[m] = m;
  // descending magnitude; the stable sort keeps equal magnitudes in index order
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t a, int32_t b) { return mag[a] > mag[b]; });
  std::sort(order.begin(), order.begin() + n_keep);
  for (int j = 0; j < n_keep; ++j) m_index[j] = order[j] + 1;
  return BEM_OK;
}
