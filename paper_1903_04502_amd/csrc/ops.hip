// Element-wise proximal operators (Section "Proximal Operators"), FP64
// deterministic reductions and the power method for ||Phi|| (Section
// "Distributed Images").
#include "ops.hpp"

namespace pr {

namespace {

constexpr int kThreads = 256;
constexpr int kRedBlocks = 1024;   // fixed grid of the reduction first stage

template <typename R>
__global__ void soft_threshold_kernel(const R* in, R* out, int64_t len, R lam) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const R v = in[i];
    const R m = fabs(v);
    out[i] = m > lam ? v * ((m - lam) / m) : R(0);
  }
}

template <typename R>
__global__ void soft_threshold_cx_kernel(const cx_t<R>* in, cx_t<R>* out, int64_t len, R lam) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const cx_t<R> v = in[i];
    const R m = hypot(v.x, v.y);
    const R f = m > lam ? (m - lam) / m : R(0);
    out[i] = cmk<cx_t<R>>(v.x * f, v.y * f);
  }
}

// Stage 1: per-block FP64 sums of |a - b|^2 (b may be null) over a fixed
// grid-stride partition; stage 2 sums the block results in index order.
template <typename R>
__global__ void sumsq_stage1(const R* a, const R* b, int64_t len, double* partials) {
  __shared__ double sh[kThreads];
  double acc = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double d = b ? static_cast<double>(a[i]) - static_cast<double>(b[i]) : static_cast<double>(a[i]);
    acc += d * d;
  }
  acc = block_sum_f64(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

template <typename R>
__global__ void abssum_stage1(const R* a, int64_t len, double* partials) {
  __shared__ double sh[kThreads];
  double acc = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    acc += fabs(static_cast<double>(a[i]));
  acc = block_sum_f64(acc, sh);
  if (threadIdx.x == 0) partials[blockIdx.x] = acc;
}

template <typename R>
__global__ void absmax_stage1(const R* a, int64_t len, double* partials) {
  __shared__ double sh[kThreads];
  double m = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    m = fmax(m, fabs(static_cast<double>(a[i])));
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partials[blockIdx.x] = sh[0];
}

// *out = scale_factor * max(partials) * (*mul) (mul may be null)
__global__ void max_stage2(const double* partials, int n, double factor, const double* mul, double* out) {
  __shared__ double sh[kThreads];
  double m = 0;
  for (int i = threadIdx.x; i < n; i += kThreads) m = fmax(m, partials[i]);
  sh[threadIdx.x] = m;
  __syncthreads();
  for (int w = kThreads / 2; w > 0; w >>= 1) {
    if (static_cast<int>(threadIdx.x) < w) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = factor * sh[0] * (mul ? *mul : 1.0);
}

// *inv = 1 / ||Phi|| from the power method's ||A x||^2 (A = Phi^dagger Phi)
__global__ void inv_norm_kernel(const double* s2, double* inv) { *inv = 1.0 / sqrt(sqrt(*s2)); }

__global__ void sum_stage2(const double* partials, int n, double* out, double* nonfinite_flag) {
  __shared__ double sh[kThreads];
  double acc = 0;
  for (int i = threadIdx.x; i < n; i += kThreads) acc += partials[i];
  acc = block_sum_f64(acc, sh);
  if (threadIdx.x == 0) {
    *out = acc;
    if (nonfinite_flag && !isfinite(acc)) *nonfinite_flag = 1.0;
  }
}

// out = center + (in - center) * min(1, eps / sqrt(*d2)); closed ball.
template <typename R>
__global__ void ball_apply_kernel(const cx_t<R>* in, const cx_t<R>* center, cx_t<R>* out, int64_t len,
                                  const double* d2, double eps) {
  const double d = sqrt(*d2);
  const R k = static_cast<R>(d <= eps ? 1.0 : eps / d);
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const cx_t<R> v = in[i], c = center[i];
    out[i] = cmk<cx_t<R>>(c.x + k * (v.x - c.x), c.y + k * (v.y - c.y));
  }
}

template <typename R>
__global__ void fill_kernel(R* a, int64_t len, R v) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    a[i] = v;
}

template <typename R>
__global__ void copy_kernel(R* dst, const R* __restrict__ src, int64_t len) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    dst[i] = src[i];
}

// xh = xb + c (xb - x); x = xb
template <typename R>
__global__ void extrapolate_kernel(R* x, const R* __restrict__ xb, R* __restrict__ xh, int64_t len, R c) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const R xn = xb[i], xo = x[i];
    xh[i] = xn + c * (xn - xo);
    x[i] = xn;
  }
}

template <typename R>
__global__ void l1_weights_kernel(const R* __restrict__ alpha, int64_t len, R delta, R* __restrict__ w) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    w[i] = delta / (delta + fabs(alpha[i]));
}

__global__ void scale_scalar_kernel(const double* src, double f, double* dst) { *dst = *src * f; }

// a = b / sqrt(*s2)
template <typename R>
__global__ void normalise_kernel(R* a, const R* b, int64_t len, const double* s2) {
  const R inv = static_cast<R>(1.0 / sqrt(*s2));
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    a[i] = b[i] * inv;
}

}  // namespace

int reduce_sumsq(const void* a, const void* b, int64_t len, int prec, double* partials, double* out,
                 hipStream_t s, double* nonfinite_flag) {
  const int G = grid_for(len, kThreads, kRedBlocks);
  if (prec == PR_F32)
    sumsq_stage1<float><<<G, kThreads, 0, s>>>(static_cast<const float*>(a), static_cast<const float*>(b), len, partials);
  else
    sumsq_stage1<double><<<G, kThreads, 0, s>>>(static_cast<const double*>(a), static_cast<const double*>(b), len,
                                                partials);
  PR_TRY_LAUNCH();
  sum_stage2<<<1, kThreads, 0, s>>>(partials, G, out, nonfinite_flag);
  PR_TRY_LAUNCH();
  return PR_OK;
}

int reduce_absmax_scaled(const void* a, int64_t len, int prec, double factor, const double* mul, double* partials,
                         double* out, hipStream_t s) {
  const int G = grid_for(len, kThreads, kRedBlocks);
  if (prec == PR_F32)
    absmax_stage1<float><<<G, kThreads, 0, s>>>(static_cast<const float*>(a), len, partials);
  else
    absmax_stage1<double><<<G, kThreads, 0, s>>>(static_cast<const double*>(a), len, partials);
  PR_TRY_LAUNCH();
  max_stage2<<<1, kThreads, 0, s>>>(partials, G, factor, mul, out);
  PR_TRY_LAUNCH();
  return PR_OK;
}

int reduce_abssum(const void* a, int64_t len, int prec, double* partials, double* out, hipStream_t s) {
  const int G = grid_for(len, kThreads, kRedBlocks);
  if (prec == PR_F32)
    abssum_stage1<float><<<G, kThreads, 0, s>>>(static_cast<const float*>(a), len, partials);
  else
    abssum_stage1<double><<<G, kThreads, 0, s>>>(static_cast<const double*>(a), len, partials);
  PR_TRY_LAUNCH();
  sum_stage2<<<1, kThreads, 0, s>>>(partials, G, out, nullptr);
  PR_TRY_LAUNCH();
  return PR_OK;
}

int soft_threshold(const void* in, void* out, int64_t len, int is_complex, int prec, double lam, hipStream_t s) {
  if (len == 0) return PR_OK;
  const int G = grid_for(len, kThreads, 8192);
  if (prec == PR_F32) {
    if (is_complex)
      soft_threshold_cx_kernel<float><<<G, kThreads, 0, s>>>(static_cast<const float2*>(in), static_cast<float2*>(out),
                                                             len, static_cast<float>(lam));
    else
      soft_threshold_kernel<float><<<G, kThreads, 0, s>>>(static_cast<const float*>(in), static_cast<float*>(out), len,
                                                          static_cast<float>(lam));
  } else {
    if (is_complex)
      soft_threshold_cx_kernel<double><<<G, kThreads, 0, s>>>(static_cast<const double2*>(in),
                                                              static_cast<double2*>(out), len, lam);
    else
      soft_threshold_kernel<double><<<G, kThreads, 0, s>>>(static_cast<const double*>(in), static_cast<double*>(out),
                                                           len, lam);
  }
  PR_TRY_LAUNCH();
  return PR_OK;
}

size_t ball_scratch_bytes() { return (kRedBlocks + 8) * sizeof(double); }

int proj_l2ball(const void* in, const void* center, void* out, int64_t len, int prec, double eps, void* scratch,
                double* dist, hipStream_t s) {
  if (dist) PR_TRY(no_capture(s, "the ball projection with a host distance"));
  double* partials = static_cast<double*>(scratch);
  double* d2 = partials + kRedBlocks;
  // ||in - center||^2 over the real and imaginary parts: 2 len real values
  PR_TRY(reduce_sumsq(in, center, 2 * len, prec, partials, d2, s, nullptr));
  if (len > 0) {
    const int G = grid_for(len, kThreads, 8192);
    if (prec == PR_F32)
      ball_apply_kernel<float><<<G, kThreads, 0, s>>>(static_cast<const float2*>(in), static_cast<const float2*>(center),
                                                      static_cast<float2*>(out), len, d2, eps);
    else
      ball_apply_kernel<double><<<G, kThreads, 0, s>>>(static_cast<const double2*>(in),
                                                       static_cast<const double2*>(center), static_cast<double2*>(out),
                                                       len, d2, eps);
    PR_TRY_LAUNCH();
  }
  if (dist) {
    double h = 0;
    PR_TRY_HIP(hipMemcpyAsync(&h, d2, sizeof(double), hipMemcpyDeviceToHost, s));
    PR_TRY_HIP(hipStreamSynchronize(s));
    *dist = std::sqrt(h);
  }
  return PR_OK;
}

int fill_real(void* a, int64_t len, int prec, double v, hipStream_t s) {
  const int G = grid_for(len, kThreads, 8192);
  if (prec == PR_F32)
    fill_kernel<float><<<G, kThreads, 0, s>>>(static_cast<float*>(a), len, static_cast<float>(v));
  else
    fill_kernel<double><<<G, kThreads, 0, s>>>(static_cast<double*>(a), len, v);
  PR_TRY_LAUNCH();
  return PR_OK;
}

int normalise(void* a, const void* b, int64_t len, int prec, const double* s2, hipStream_t s) {
  const int G = grid_for(len, kThreads, 8192);
  if (prec == PR_F32)
    normalise_kernel<float><<<G, kThreads, 0, s>>>(static_cast<float*>(a), static_cast<const float*>(b), len, s2);
  else
    normalise_kernel<double><<<G, kThreads, 0, s>>>(static_cast<double*>(a), static_cast<const double*>(b), len, s2);
  PR_TRY_LAUNCH();
  return PR_OK;
}

int copy_real(void* dst, const void* src, int64_t len, int prec, hipStream_t s) {
  const int G = grid_for(len, kThreads, 8192);
  if (prec == PR_F32)
    copy_kernel<float><<<G, kThreads, 0, s>>>(static_cast<float*>(dst), static_cast<const float*>(src), len);
  else
    copy_kernel<double><<<G, kThreads, 0, s>>>(static_cast<double*>(dst), static_cast<const double*>(src), len);
  PR_TRY_LAUNCH();
  return PR_OK;
}

int extrapolate(void* x, const void* xb, void* xh, int64_t len, int prec, double c, hipStream_t s) {
  const int G = grid_for(len, kThreads, 8192);
  if (prec == PR_F32)
    extrapolate_kernel<float><<<G, kThreads, 0, s>>>(static_cast<float*>(x), static_cast<const float*>(xb),
                                                     static_cast<float*>(xh), len, static_cast<float>(c));
  else
    extrapolate_kernel<double><<<G, kThreads, 0, s>>>(static_cast<double*>(x), static_cast<const double*>(xb),
                                                      static_cast<double*>(xh), len, c);
  PR_TRY_LAUNCH();
  return PR_OK;
}

int l1_weights(const void* alpha, int64_t len, int prec, double delta, void* w, hipStream_t s) {
  const int G = grid_for(len, kThreads, 8192);
  if (prec == PR_F32)
    l1_weights_kernel<float><<<G, kThreads, 0, s>>>(static_cast<const float*>(alpha), len, static_cast<float>(delta),
                                                    static_cast<float*>(w));
  else
    l1_weights_kernel<double><<<G, kThreads, 0, s>>>(static_cast<const double*>(alpha), len, delta,
                                                     static_cast<double*>(w));
  PR_TRY_LAUNCH();
  return PR_OK;
}

int scale_scalar(const double* src, double f, double* dst, hipStream_t s) {
  scale_scalar_kernel<<<1, 1, 0, s>>>(src, f, dst);
  PR_TRY_LAUNCH();
  return PR_OK;
}

int phi_norm_device(pr_phi_plan_t* p, int iters, void* vis, double* inv_norm, hipStream_t s) {
  const int64_t N = static_cast<int64_t>(p->n) * p->n;
  double* s2 = p->scalars + 8;
  PR_TRY(fill_real(p->img_a, N, p->prec, 1.0 / p->n, s));
  for (int it = 0; it < iters; ++it) {
    PR_TRY(phi_fzs(p, p->img_a, s));
    PR_TRY(phi_gw(p, vis, 1.0, s));
    PR_TRY(phi_gw_adjoint(p, vis, 1.0, s));
    PR_TRY(phi_fzs_adjoint(p, p->img_b, s));
    PR_TRY(reduce_sumsq(p->img_b, nullptr, N, p->prec, p->partials, s2, s, nullptr));
    PR_TRY(normalise(p->img_a, p->img_b, N, p->prec, s2, s));
  }
  inv_norm_kernel<<<1, 1, 0, s>>>(s2, inv_norm);
  PR_TRY_LAUNCH();
  return PR_OK;
}

int phi_norm(pr_phi_plan_t* p, int iters, double rtol, void* vis, double* norm, hipStream_t s) {
  PR_TRY(no_capture(s, "pr_phi_norm"));
  const int64_t N = static_cast<int64_t>(p->n) * p->n;
  double* s2 = p->scalars + 8;
  PR_TRY(fill_real(p->img_a, N, p->prec, 1.0 / p->n, s));
  double h = 0, lam_prev = -1.0;
  for (int it = 0; it < iters; ++it) {
    PR_TRY(phi_fzs(p, p->img_a, s));
    PR_TRY(phi_gw(p, vis, 1.0, s));
    PR_TRY(phi_gw_adjoint(p, vis, 1.0, s));
    PR_TRY(phi_fzs_adjoint(p, p->img_b, s));
    PR_TRY(reduce_sumsq(p->img_b, nullptr, N, p->prec, p->partials, s2, s, nullptr));
    PR_TRY(normalise(p->img_a, p->img_b, N, p->prec, s2, s));
    if (rtol > 0) {
      // l_k = ||A x_k||: stop once it has settled to rtol
      PR_TRY_HIP(hipMemcpyAsync(&h, s2, sizeof(double), hipMemcpyDeviceToHost, s));
      PR_TRY_HIP(hipStreamSynchronize(s));
      const double lam = std::sqrt(h);
      if (lam_prev >= 0 && std::fabs(lam - lam_prev) <= rtol * lam) break;
      lam_prev = lam;
    }
  }
  PR_TRY_HIP(hipMemcpyAsync(&h, s2, sizeof(double), hipMemcpyDeviceToHost, s));
  PR_TRY_HIP(hipStreamSynchronize(s));
  *norm = iters > 0 ? std::sqrt(std::sqrt(h)) : 0.0;
  return PR_OK;
}

}  // namespace pr
