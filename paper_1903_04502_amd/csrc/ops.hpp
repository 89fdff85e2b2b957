// Element-wise operators and reductions shared by the operator and solver code.
#pragma once

#include <cmath>

#include "phi.hpp"

namespace pr {

// *out = sum |a - b|^2 over len real values (b may be null), FP64, fixed order.
int reduce_sumsq(const void* a, const void* b, int64_t len, int prec, double* partials, double* out,
                 hipStream_t s, double* nonfinite_flag);
// *out = sum |a| over len real values, FP64, fixed order.
int reduce_abssum(const void* a, int64_t len, int prec, double* partials, double* out, hipStream_t s);
// *out = factor * max |a| * (*mul) over len real values (mul may be null), FP64.
int reduce_absmax_scaled(const void* a, int64_t len, int prec, double factor, const double* mul, double* partials,
                         double* out, hipStream_t s);
int soft_threshold(const void* in, void* out, int64_t len, int is_complex, int prec, double lam, hipStream_t s);
size_t ball_scratch_bytes();
int proj_l2ball(const void* in, const void* center, void* out, int64_t len, int prec, double eps, void* scratch,
                double* dist, hipStream_t s);
int fill_real(void* a, int64_t len, int prec, double v, hipStream_t s);
// a = b / sqrt(*s2) (device scalar)
int normalise(void* a, const void* b, int64_t len, int prec, const double* s2, hipStream_t s);
// Power method of the plan (iters applications of Phi^dagger Phi from the
// constant image) leaving 1 / ||Phi|| in device memory; no host read-back.
int phi_norm_device(pr_phi_plan_t* p, int iters, void* vis, double* inv_norm, hipStream_t s);
// dst = src over len real values.
int copy_real(void* dst, const void* src, int64_t len, int prec, hipStream_t s);
// Extrapolation of an accelerated iteration: xh = xb + c (xb - x), then x = xb
// (each element of x read before it is written).
int extrapolate(void* x, const void* xb, void* xh, int64_t len, int prec, double c, hipStream_t s);
// Reweighting of the analysis l1 norm: w_i = delta / (delta + |alpha_i|).
int l1_weights(const void* alpha, int64_t len, int prec, double delta, void* w, hipStream_t s);
// *dst = *src * f (device scalars).
int scale_scalar(const double* src, double f, double* dst, hipStream_t s);

}  // namespace pr
