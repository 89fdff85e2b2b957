// Daubechies low-pass filters by spectral factorisation (host, FP64; plain
// C++, also built alone with sanitizers by the CPU tests).
//
// |H(w)|^2 = 2 cos^{2N}(w/2) P(sin^2(w/2)) with P(y) = sum_{k<N} C(N-1+k, k) y^k.
// Each root y_i of P gives the pair of zeros z, 1/z of z^2 - (2 - 4 y_i) z + 1;
// keeping the one inside the unit circle makes the filter minimum phase:
//   H(z) ~ (1 + z^-1)^N prod_i (1 - z_i z^-1),   sum_k h_k = sqrt(2).
// The roots of P come from a Durand-Kerner iteration in long double.
#pragma once

#include <algorithm>
#include <cmath>
#include <complex>

namespace pr {
namespace host {

using cld = std::complex<long double>;

// All roots of the monic polynomial with coefficients c[0..deg-1] (ascending,
// leading coefficient 1 implied).
inline bool durand_kerner(const long double* c, int deg, cld* roots) {
  if (deg == 0) return true;
  long double bound = 1;
  for (int i = 0; i < deg; ++i) bound = std::max(bound, 1 + std::fabs(c[i]));
  const cld seed(0.4L, 0.9L);
  cld z = 1;
  for (int i = 0; i < deg; ++i) {
    roots[i] = z * bound * 0.5L;
    z *= seed;
  }
  for (int it = 0; it < 5000; ++it) {
    long double change = 0;
    for (int i = 0; i < deg; ++i) {
      cld pv = 1;
      for (int k = deg - 1; k >= 0; --k) pv = pv * roots[i] + c[k];
      cld den = 1;
      for (int j = 0; j < deg; ++j)
        if (j != i) den *= roots[i] - roots[j];
      const cld step = pv / den;
      roots[i] -= step;
      change = std::max(change, std::abs(step) / std::max(1.0L, std::abs(roots[i])));
    }
    if (change < 1e-17L) return true;
  }
  return false;
}

inline bool daubechies_filter(int N, double* h) {
  if (N < 1 || N > 8) return false;
  // P(y), made monic
  long double p[8];
  long double binom = 1;  // C(N-1+k, k)
  for (int k = 0; k < N; ++k) {
    p[k] = binom;
    binom = binom * (N + k) / (k + 1);
  }
  const long double lead = p[N - 1];
  long double mono[8];
  for (int k = 0; k < N - 1; ++k) mono[k] = p[k] / lead;
  cld yroots[8];
  if (!durand_kerner(mono, N - 1, yroots)) return false;
  // polynomial in z^-1, ascending powers
  cld poly[16];
  int len = 1;
  poly[0] = 1;
  auto mul_linear = [&](cld root) {  // times (1 - root z^-1)
    poly[len] = 0;
    for (int k = len; k >= 1; --k) poly[k] -= root * poly[k - 1];
    ++len;
  };
  for (int k = 0; k < N; ++k) mul_linear(cld(-1));
  for (int i = 0; i < N - 1; ++i) {
    const cld b = 2.0L - 4.0L * yroots[i];
    const cld disc = std::sqrt(b * b - 4.0L);
    const cld z1 = (b + disc) / 2.0L, z2 = (b - disc) / 2.0L;
    mul_linear(std::abs(z1) < 1 ? z1 : z2);
  }
  long double sum = 0;
  for (int k = 0; k < 2 * N; ++k) sum += poly[k].real();
  const long double norm = std::sqrt(2.0L) / sum;
  for (int k = 0; k < 2 * N; ++k) h[k] = static_cast<double>(poly[k].real() * norm);
  return true;
}

}  // namespace host
}  // namespace pr
