// Interpolation taps of the pre-sampled Kaiser-Bessel kernel (Section "Kernel
// Pre-Sampling": the kernel is sampled on 0 <= |t| <= J/2 and read either by
// zeroth-order interpolation, the nearest sample, or by first-order
// interpolation between the two samples around the tap distance).
//
// For a baseline coordinate u (radians per pixel) the continuous grid
// coordinate is s = u * K / (2 pi), formed in FP64. Tap a (a = 0..J-1) sits
// on cell floor(s) - J/2 + 1 + a at distance t_a = |s - cell|; it uses table
// sample round(t_a * D) with ties to the larger distance. With
// f = (s - floor(s)) * D and m = J/2 - 1 - a this is m*D + round_half_up(f)
// for m >= 0 and |m|*D - round_half_down(f) for m < 0. First order: the
// distance in samples is m*D + f (m >= 0) or |m|*D - f (m < 0); with
// i = floor of it and phi the rest, the weight is (1 - phi) T[i] + phi T[i+1],
// i.e. i = m*D + floor(f), phi = f - floor(f) for m >= 0, and for m < 0
// i = |m|*D - floor(f) - 1, phi = 1 - (f - floor(f)) unless f is whole
// (then i = |m|*D - f, phi = 0). All of it is FP64 with FMA contraction
// disabled, so every caller picks exactly the same samples.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

namespace pr {

struct AxisTaps {
  int j0;     // first tap cell, not reduced mod K
  int up;     // round_half_up(f)
  int dn;     // round_half_down(f)
  int ff;     // floor(f)
  double r;   // f - floor(f)
};

__device__ __forceinline__ AxisTaps axis_taps(double u, double kappa, int J, int D) {
#pragma clang fp contract(off)
  const double s = u * kappa;
  const double fl = floor(s);
  const double fr = s - fl;
  const double f = fr * static_cast<double>(D);
  const double ff = floor(f);
  const double r = f - ff;
  AxisTaps t;
  t.j0 = static_cast<int>(fl) - J / 2 + 1;
  t.up = static_cast<int>(ff) + (r >= 0.5 ? 1 : 0);
  t.dn = static_cast<int>(ff) + (r > 0.5 ? 1 : 0);
  t.ff = static_cast<int>(ff);
  t.r = r;
  return t;
}

// Compact pre-sampled taps of one visibility (nearest-sample lookup): the
// plan evaluates axis_taps once and stores, in 32 bits, the base cell within
// its tile (4 bits per axis, tiles of at most 16 cells) and, per axis,
// 2 * up + (up != dn) in 12 bits (D <= 2047). The launches then read the
// sample indices instead of recomputing them from (u, v): the same integers,
// so the same weights.
constexpr int kTapWordMaxTile = 16;
constexpr int kTapWordMaxD = 2047;

__device__ __forceinline__ uint32_t tap_word(const AxisTaps& tu, const AxisTaps& tv, int lu, int lv) {
  const uint32_t au = 2u * static_cast<uint32_t>(tu.up) + (tu.up != tu.dn ? 1u : 0u);
  const uint32_t av = 2u * static_cast<uint32_t>(tv.up) + (tv.up != tv.dn ? 1u : 0u);
  return static_cast<uint32_t>(lu) | (static_cast<uint32_t>(lv) << 4) | (au << 8) | (av << 20);
}

// The sample indices of one axis from its 12 bits (j0, ff and r are not used
// by the nearest-sample lookup and stay zero).
__device__ __forceinline__ AxisTaps word_axis(uint32_t a12) {
  AxisTaps t;
  t.j0 = 0;
  t.up = static_cast<int>(a12 >> 1);
  t.dn = t.up - static_cast<int>(a12 & 1u);
  t.ff = 0;
  t.r = 0.0;
  return t;
}

// Table index of tap a.
__device__ __forceinline__ int tap_index(const AxisTaps& t, int a, int J, int D) {
  const int m = J / 2 - 1 - a;
  return m >= 0 ? m * D + t.up : (-m) * D - t.dn;
}

// Weight of tap a from the table (tlen samples): nearest sample, or the
// first-order interpolation between samples i and i + 1 (i + 1 clamped to the
// table; it is used only with phi = 0 there).
template <bool LIN, typename R>
__device__ __forceinline__ R tap_weight(const R* tab, const AxisTaps& t, int a, int J, int D, int tlen) {
  if constexpr (!LIN) {
    (void)tlen;
    return tab[tap_index(t, a, J, D)];
  } else {
    const int m = J / 2 - 1 - a;
    int i;
    double ph;
    if (m >= 0) {
      i = m * D + t.ff;
      ph = t.r;
    } else {
      const bool frac = t.r > 0.0;
      i = (-m) * D - t.ff - (frac ? 1 : 0);
      ph = frac ? 1.0 - t.r : 0.0;
    }
    const int i1 = i + 1 < tlen ? i + 1 : tlen - 1;
    const R p = static_cast<R>(ph);
    return (R(1) - p) * tab[i] + p * tab[i1];
  }
}

// All J weights of an axis. J = 4 with the nearest sample reads the paired
// table (T[i], T[D + i]) (see the plan): two loads instead of four.
template <bool LIN, int J, typename R>
__device__ __forceinline__ void axis_weights(const R* tab, const AxisTaps& t, int D, int tlen, R* w) {
  if constexpr (J == 4 && !LIN) {
    (void)tlen;
    using R2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
    const R2* t2 = reinterpret_cast<const R2*>(tab);
    const R2 p0 = t2[t.up];        // (T[up], T[D + up]): taps m = 0, 1
    const R2 p1 = t2[D - t.dn];    // (T[D - dn], T[2D - dn]): taps m = -1, -2
    w[0] = p0.y;
    w[1] = p0.x;
    w[2] = p1.x;
    w[3] = p1.y;
  } else {
#pragma unroll
    for (int a = 0; a < J; ++a) w[a] = tap_weight<LIN>(tab, t, a, J, D, tlen);
  }
}

__device__ __forceinline__ int mod_pos(int a, int K) {
  int r = a % K;
  return r < 0 ? r + K : r;
}

// a mod K for K a power of two (two's complement keeps this right for a < 0).
__device__ __forceinline__ int mod_pow2(int a, int K) { return a & (K - 1); }

// i / d and i mod d for small non-negative i and d (i < 2^20, d < 2^12): the
// float quotient of i + 1/2 is at least 1/(2d) away from an integer, far more
// than its rounding error, so the truncation is exact.
__device__ __forceinline__ int small_div(int i, int d, float inv_d) {
  return static_cast<int>((static_cast<float>(i) + 0.5f) * inv_d);
}

}  // namespace pr
