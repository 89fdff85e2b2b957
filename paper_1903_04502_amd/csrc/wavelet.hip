// SARA dictionary on the GPU (Sections "Analysis and Synthesis", "MPI Wavelet
// Operator Benchmarks"): a Dirac basis plus periodic orthonormal 2-D
// Daubechies transforms (db1..db8) to a fixed number of levels, all wavelet
// bases of a level in one launch (blockIdx.y = basis), scaled by 1/sqrt(nb).
//
// One analysis level on the L x L low-low block: filter the rows (low half,
// then high half), then the columns; lo[m] = sum_q h[q] a[(2m + q) mod L],
// hi[m] likewise with g. Synthesis is the transpose: for output i only taps
// q = i (mod 2) contribute, from coefficient m = ((i - q) mod L) / 2.
// Coefficients are stored in the Mallat layout of each basis' n x n array.
// Levels small enough for LDS run in one launch per transform (tail kernels).
#include <cmath>

#include "ops.hpp"
#include "psi.hpp"

namespace pr {

namespace {

constexpr int kThreads = 256;
constexpr int kTapsMax = 16;

template <typename R>
struct Filt {
  R h[kTapsMax];
  R g[kTapsMax];
  int taps;
  int pad[3];
};

// d <- (1/eta) clip_gamma(eta d + a), clip_gamma(v) = v - S_gamma(v) = sign(v) min(|v|, gamma)
template <typename R>
__device__ inline R dual_clip(R d, R a, R gamma, R eta) {
  const R v = eta * d + a;
  const R c = v > gamma ? gamma : (v < -gamma ? -gamma : v);
  return c / eta;
}

template <typename R>
__global__ void dwt_rows_kernel(const R* __restrict__ src, int64_t src_basis_stride, int ld_src, int L,
                                R* __restrict__ rows, int64_t n2, const Filt<R>* __restrict__ filt) {
  const int bi = blockIdx.y;
  const Filt<R>& f = filt[bi];
  const R* in = src + bi * src_basis_stride;
  R* out = rows + bi * n2;
  // L is a power of two and L^2 < 2^31: 32-bit positions, shifts and masks
  // Two outputs per thread, m and m + 1: their windows share all but two
  // inputs, loaded once (each output is the same sum in the same order).
  const int half = L >> 1, lgq = __builtin_ctz(half >> 1);
  const int total = L * (half >> 1);
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < total; i += gridDim.x * kThreads) {
    const int r = i >> lgq, m0 = (i & ((half >> 1) - 1)) * 2;
    const R* row = in + static_cast<int64_t>(r) * ld_src;
    R v[kTapsMax + 2];
#pragma unroll
    for (int q = 0; q < kTapsMax + 2; ++q) v[q] = q < f.taps + 2 ? row[(2 * m0 + q) & (L - 1)] : R(0);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      R lo = 0, hi = 0;
#pragma unroll
      for (int q = 0; q < kTapsMax; ++q) {
        if (q < f.taps) {
          lo += f.h[q] * v[q + 2 * k];
          hi += f.g[q] * v[q + 2 * k];
        }
      }
      out[static_cast<int64_t>(r) * L + m0 + k] = lo;
      out[static_cast<int64_t>(r) * L + half + m0 + k] = hi;
    }
  }
}

// MODE 0: write scaled coefficients to alpha. MODE 1: dual update of d in place.
template <typename R, int MODE, int NO>
__global__ void dwt_cols_kernel(const R* __restrict__ rows, int64_t n2, int L, int n, R* __restrict__ ll_out,
                                int last, R* __restrict__ coef, const Filt<R>* __restrict__ filt, R scale,
                                R gamma_h, const double* __restrict__ gamma_dev, R eta, const R* __restrict__ wts) {
  const R gamma = (MODE == 1 && gamma_dev) ? static_cast<R>(*gamma_dev) : gamma_h;
  const int bi = blockIdx.y;
  const Filt<R>& f = filt[bi];
  const R* in = rows + bi * n2;
  R* cb = coef + bi * n2;
  const R* wb = wts ? wts + bi * n2 : nullptr;   // per-coefficient l1 weights (MODE 1)
  R* llb = ll_out ? ll_out + bi * (n2 / 4) : nullptr;
  // NO output rows per thread, m0 .. m0 + NO - 1: consecutive input windows
  // share all but two rows, so the thread loads taps + 2 (NO - 1) rows once
  // (each output is the same sum in the same order)
  const int half = L >> 1, lgL = __builtin_ctz(L);
  const int total = (half / NO) * L;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < total; i += gridDim.x * kThreads) {
    const int m0 = (i >> lgL) * NO, c = i & (L - 1);
    R v[kTapsMax + 2 * (NO - 1)];
#pragma unroll
    for (int q = 0; q < kTapsMax + 2 * (NO - 1); ++q)
      v[q] = q < f.taps + 2 * (NO - 1) ? in[static_cast<int64_t>((2 * m0 + q) & (L - 1)) * L + c] : R(0);
#pragma unroll
    for (int k = 0; k < NO; ++k) {
      const int m = m0 + k;
      R lo = 0, hi = 0;
#pragma unroll
      for (int q = 0; q < kTapsMax; ++q) {
        if (q < f.taps) {
          lo += f.h[q] * v[q + 2 * k];
          hi += f.g[q] * v[q + 2 * k];
        }
      }
      // low-low band goes down the chain unless this is the last level
      if (c < half && !last) {
        llb[static_cast<int64_t>(m) * half + c] = lo;
      } else {
        const int64_t o = static_cast<int64_t>(m) * n + c;
        if (MODE == 0) cb[o] = lo * scale;
        else cb[o] = dual_clip(cb[o], lo * scale, wb ? gamma * wb[o] : gamma, eta);
      }
      const int64_t o = static_cast<int64_t>(half + m) * n + c;
      if (MODE == 0) cb[o] = hi * scale;
      else cb[o] = dual_clip(cb[o], hi * scale, wb ? gamma * wb[o] : gamma, eta);
    }
  }
}

template <typename R, int MODE>
__global__ void dirac_analysis_kernel(const R* __restrict__ x, R* __restrict__ coef, int64_t n2, R scale, R gamma_h,
                                      const double* __restrict__ gamma_dev, R eta, const R* __restrict__ wts) {
  const R gamma = (MODE == 1 && gamma_dev) ? static_cast<R>(*gamma_dev) : gamma_h;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n2;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    if (MODE == 0) coef[i] = x[i] * scale;
    else coef[i] = dual_clip(coef[i], x[i] * scale, wts ? gamma * wts[i] : gamma, eta);
  }
}

// Transposed column pass of level size L: low band rows from ll_src (or from
// the coefficient array at the deepest level), high band from the coefficients.
template <typename R>
__global__ void idwt_cols_kernel(const R* __restrict__ coef, int64_t n2, int n, const R* __restrict__ ll_src,
                                 int ld_ll, int64_t ll_basis_stride, int L, R* __restrict__ rows,
                                 const Filt<R>* __restrict__ filt) {
  const int bi = blockIdx.y;
  const Filt<R>& f = filt[bi];
  const R* cb = coef + bi * n2;
  const R* ll = ll_src + bi * ll_basis_stride;
  R* out = rows + bi * n2;
  // output rows 2p (even taps) and 2p + 1 (odd taps) read the same band
  // rows m = p - j: one thread forms both from one load of each (each
  // output is the same sum in the same order)
  const int half = L >> 1, lgL = __builtin_ctz(L);
  const int total = half * L;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < total; i += gridDim.x * kThreads) {
    const int p = i >> lgL, c = i & (L - 1);
    R acc0 = 0, acc1 = 0;
#pragma unroll
    for (int j = 0; j < kTapsMax / 2; ++j) {
      const int q = 2 * j;
      if (q < f.taps) {
        const int m = (p - j) & (half - 1);
        const R lo = c < half ? ll[static_cast<int64_t>(m) * ld_ll + c] : cb[static_cast<int64_t>(m) * n + c];
        const R hi = cb[static_cast<int64_t>(half + m) * n + c];
        acc0 += f.h[q] * lo + f.g[q] * hi;
        if (q + 1 < f.taps) acc1 += f.h[q + 1] * lo + f.g[q + 1] * hi;
      }
    }
    out[static_cast<int64_t>(2 * p) * L + c] = acc0;
    out[static_cast<int64_t>(2 * p + 1) * L + c] = acc1;
  }
}

template <typename R>
__global__ void idwt_rows_kernel(const R* __restrict__ rows, int64_t n2, int L, R* __restrict__ dst,
                                 int64_t dst_basis_stride, const Filt<R>* __restrict__ filt) {
  const int bi = blockIdx.y;
  const Filt<R>& f = filt[bi];
  const R* in = rows + bi * n2;
  R* out = dst + bi * dst_basis_stride;
  // outputs 2p and 2p + 1 of a row from one load of their shared band
  // entries m = p - j (as in the column pass)
  const int half = L >> 1, lgh = __builtin_ctz(half);
  const int total = L * half;
  for (int i = blockIdx.x * kThreads + threadIdx.x; i < total; i += gridDim.x * kThreads) {
    const int r = i >> lgh, p = i & (half - 1);
    const R* row = in + static_cast<int64_t>(r) * L;
    R acc0 = 0, acc1 = 0;
#pragma unroll
    for (int j = 0; j < kTapsMax / 2; ++j) {
      const int q = 2 * j;
      if (q < f.taps) {
        const int m = (p - j) & (half - 1);
        const R lo = row[m], hi = row[half + m];
        acc0 += f.h[q] * lo + f.g[q] * hi;
        if (q + 1 < f.taps) acc1 += f.h[q + 1] * lo + f.g[q + 1] * hi;
      }
    }
    out[static_cast<int64_t>(r) * L + 2 * p] = acc0;
    out[static_cast<int64_t>(r) * L + 2 * p + 1] = acc1;
  }
}

// MODE 0: x = scale (alpha_0 + sum_b recon_b).
// MODE 1: zbar = max(z - scale (d_0 + sum_b recon_b), 0), with FP64 partials
// of ||zbar - xprev||^2 and ||zbar||^2 when xprev is given.
template <typename R, int MODE>
__global__ void combine_kernel(const R* __restrict__ dirac, const R* __restrict__ recon, int ndb, int64_t n2, R scale,
                               const R* __restrict__ z, R* out, const R* xprev, double* __restrict__ partials) {
  __shared__ double sh[kThreads];
  double dd = 0, xx = 0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(kThreads) + threadIdx.x; i < n2;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    R acc = dirac ? dirac[i] : R(0);
    for (int b = 0; b < ndb; ++b) acc += recon[b * n2 + i];
    acc *= scale;
    if (MODE == 0) {
      out[i] = acc;
    } else {
      // out may be xprev (in-place iterate): read before the store
      const R xp = xprev ? xprev[i] : R(0);
      const R v = z[i] - acc;
      const R zb = v > R(0) ? v : R(0);
      out[i] = zb;
      if (xprev) {
        const double df = static_cast<double>(zb) - static_cast<double>(xp);
        dd += df * df;
        xx += static_cast<double>(zb) * zb;
      }
    }
  }
  if (MODE == 1 && xprev) {
    dd = block_sum_f64(dd, sh);
    xx = block_sum_f64(xx, sh);
    if (threadIdx.x == 0) {
      partials[blockIdx.x] = dd;
      partials[kPartialsMax + blockIdx.x] = xx;
    }
  }
}

// Tail levels in one launch: from the first level of size L <= kTailMaxL on,
// one block per basis runs all the remaining levels with the approximation,
// the row pass and the low-low band in LDS (2 L^2 values). Each output is the
// same sum, in the same order, as in the per-level kernels. One block per
// basis is slower than the per-level launches from L = 128 up (FP32 256^2:
// ADMM iteration 0.18 -> 0.22 ms with levels 2..4 fused).
constexpr int kTailThreads = 1024;
constexpr int kTailMaxL = 64;
constexpr int kCols4MinL = 512;   // analysis column pass: four output rows per thread from this level size
constexpr size_t kTailLds = 2 * kTailMaxL * kTailMaxL * sizeof(double);

template <typename R>
bool tail_fits(int L) {
  return L <= kTailMaxL;
}

// first level (1-based) handled by the tail kernels, levels + 1 if none
template <typename R>
int tail_level(int n, int levels) {
  for (int lev = 1; lev <= levels; ++lev)
    if (tail_fits<R>(n >> (lev - 1))) return lev;
  return levels + 1;
}

int log2i(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Analysis levels lev0 .. levels (nlev of them; level lev0 has size L0 = 2^lg0)
// of basis blockIdx.x; src is that level's input as in dwt_rows_kernel.
template <typename R, int MODE>
__global__ __launch_bounds__(kTailThreads) void dwt_tail_kernel(const R* __restrict__ src, int64_t src_basis_stride,
                                                                int ld_src, int lg0, int nlev, int n, int64_t n2,
                                                                R* __restrict__ coef, const Filt<R>* __restrict__ filt,
                                                                R scale, R gamma_h, const double* __restrict__ gamma_dev,
                                                                R eta, const R* __restrict__ wts) {
  extern __shared__ char smem_raw[];
  const int L0 = 1 << lg0;
  R* A = reinterpret_cast<R*>(smem_raw);    // level input, L x L
  R* B = A + static_cast<size_t>(L0) * L0;  // row pass, L x L
  const R gamma = (MODE == 1 && gamma_dev) ? static_cast<R>(*gamma_dev) : gamma_h;
  const int bi = blockIdx.x, tid = threadIdx.x;
  const Filt<R>& f = filt[bi];
  const R* in = src + bi * src_basis_stride;
  R* cb = coef + bi * n2;
  const R* wb = wts ? wts + bi * n2 : nullptr;
  for (int i = tid; i < L0 * L0; i += kTailThreads) A[i] = in[static_cast<int64_t>(i >> lg0) * ld_src + (i & (L0 - 1))];
  int lg = lg0;
  for (int lv = 0; lv < nlev; ++lv, --lg) {
    const int L = 1 << lg, half = L >> 1;
    __syncthreads();   // A holds this level's input
    for (int i = tid; i < L * half; i += kTailThreads) {
      const int r = i >> (lg - 1), m = i & (half - 1);
      const R* row = A + r * L;
      R lo = 0, hi = 0;
#pragma unroll
      for (int q = 0; q < kTapsMax; ++q) {
        if (q < f.taps) {
          const R v = row[(2 * m + q) & (L - 1)];
          lo += f.h[q] * v;
          hi += f.g[q] * v;
        }
      }
      B[r * L + m] = lo;
      B[r * L + half + m] = hi;
    }
    __syncthreads();   // rows done; A is free for the next level's input
    const bool last = lv == nlev - 1;
    for (int i = tid; i < half * L; i += kTailThreads) {
      const int m = i >> lg, c = i & (L - 1);
      R lo = 0, hi = 0;
#pragma unroll
      for (int q = 0; q < kTapsMax; ++q) {
        if (q < f.taps) {
          const R v = B[((2 * m + q) & (L - 1)) * L + c];
          lo += f.h[q] * v;
          hi += f.g[q] * v;
        }
      }
      if (c < half && !last) {
        A[m * half + c] = lo;
      } else {
        const int64_t o = static_cast<int64_t>(m) * n + c;
        if (MODE == 0) cb[o] = lo * scale;
        else cb[o] = dual_clip(cb[o], lo * scale, wb ? gamma * wb[o] : gamma, eta);
      }
      const int64_t o = static_cast<int64_t>(half + m) * n + c;
      if (MODE == 0) cb[o] = hi * scale;
      else cb[o] = dual_clip(cb[o], hi * scale, wb ? gamma * wb[o] : gamma, eta);
    }
  }
}

// Synthesis levels levels .. lev0 (nlev of them, from the deepest, of size
// 2^lgd) of basis blockIdx.x; level lev0's output goes to dst as in
// idwt_rows_kernel, the others stay in LDS as the next level's low-low band.
template <typename R>
__global__ __launch_bounds__(kTailThreads) void idwt_tail_kernel(const R* __restrict__ coef, int64_t n2, int n, int lgd,
                                                                 int nlev, R* __restrict__ dst, int64_t dst_basis_stride,
                                                                 const Filt<R>* __restrict__ filt) {
  extern __shared__ char smem_raw[];
  const int L0 = 1 << (lgd + nlev - 1);
  R* rw = reinterpret_cast<R*>(smem_raw);      // column pass, L x L
  R* ll = rw + static_cast<size_t>(L0) * L0;   // low-low band of the next level, L x L (at most (L0/2)^2)
  const int bi = blockIdx.x, tid = threadIdx.x;
  const Filt<R>& f = filt[bi];
  const R* cb = coef + bi * n2;
  R* out = dst + bi * dst_basis_stride;
  const __attribute__((address_space(3))) R* ll_s = (const __attribute__((address_space(3))) R*)ll;
  const __attribute__((address_space(1))) R* cb_g = (const __attribute__((address_space(1))) R*)cb;
  int lg = lgd;
  for (int lv = 0; lv < nlev; ++lv, ++lg) {
    const int L = 1 << lg, half = L >> 1;
    const bool deepest = lv == 0, last = lv == nlev - 1;
    __syncthreads();   // ll holds this level's low-low band; rw is free
    for (int i = tid; i < L * L; i += kTailThreads) {
      const int r = i >> lg, c = i & (L - 1);
      R acc = 0;
#pragma unroll
      for (int q = 0; q < kTapsMax; ++q) {
        if (q < f.taps && ((q ^ r) & 1) == 0) {
          const int m = ((r - q) & (L - 1)) >> 1;
          // the two sources as LDS and global pointers: a choice between
          // two generic pointers would become a flat load
          const R lo = (c < half && !deepest) ? ll_s[m * half + c] : cb_g[static_cast<int64_t>(m) * n + c];
          const R hi = cb[static_cast<int64_t>(half + m) * n + c];
          acc += f.h[q] * lo + f.g[q] * hi;
        }
      }
      rw[i] = acc;
    }
    __syncthreads();   // columns done; ll is free
    for (int i = tid; i < L * L; i += kTailThreads) {
      const int r = i >> lg, c = i & (L - 1);
      const R* row = rw + r * L;
      R acc = 0;
#pragma unroll
      for (int q = 0; q < kTapsMax; ++q) {
        if (q < f.taps && ((q ^ c) & 1) == 0) {
          const int m = ((c - q) & (L - 1)) >> 1;
          acc += f.h[q] * row[m] + f.g[q] * row[half + m];
        }
      }
      if (last) out[i] = acc;
      else ll[i] = acc;
    }
  }
}

__global__ void combine_finish_kernel(const double* partials, int nblocks, double* sums) {
  __shared__ double sh[kThreads];
  double dd = 0, xx = 0;
  for (int i = threadIdx.x; i < nblocks; i += kThreads) {
    dd += partials[i];
    xx += partials[kPartialsMax + i];
  }
  dd = block_sum_f64(dd, sh);
  xx = block_sum_f64(xx, sh);
  if (threadIdx.x == 0) {
    sums[0] = dd;
    sums[1] = xx;
  }
}

template <typename R>
int analysis_impl(pr_psi_plan_t* p, const R* x, R* coef, int mode, double gamma, const double* gamma_dev, double eta,
                  hipStream_t s, const R* wts = nullptr) {
  const int n = p->n;
  const int64_t n2 = static_cast<int64_t>(n) * n;
  const R scale = static_cast<R>(p->scale);
  R* wave = coef + (p->has_dirac ? n2 : 0);
  const R* wwave = wts ? wts + (p->has_dirac ? n2 : 0) : nullptr;
  if (p->has_dirac) {
    const int G = grid_for(n2, kThreads, 4096);
    if (mode == 0)
      dirac_analysis_kernel<R, 0><<<G, kThreads, 0, s>>>(x, coef, n2, scale, R(gamma), gamma_dev, R(eta), nullptr);
    else
      dirac_analysis_kernel<R, 1><<<G, kThreads, 0, s>>>(x, coef, n2, scale, R(gamma), gamma_dev, R(eta), wts);
    PR_TRY_LAUNCH();
  }
  if (p->ndb == 0) return PR_OK;
  const Filt<R>* f = static_cast<const Filt<R>*>(p->filters);
  R* rows = static_cast<R*>(p->rows);
  R* lla = static_cast<R*>(p->ll_a);
  R* llb = static_cast<R*>(p->ll_b);
  const int lev0 = tail_level<R>(n, p->levels);
  int L = n;
  for (int lev = 1; lev <= p->levels; ++lev, L >>= 1) {
    const R* src = lev == 1 ? x : ((lev - 1) & 1 ? lla : llb);
    const int64_t sstride = lev == 1 ? 0 : n2 / 4;
    const int ld = lev == 1 ? n : L;
    if (lev == lev0) {
      // this level and all deeper ones in one launch
      const size_t lds = 2 * static_cast<size_t>(L) * L * sizeof(R);
      const int nlev = p->levels - lev + 1;
      if (mode == 0)
        dwt_tail_kernel<R, 0><<<p->ndb, kTailThreads, lds, s>>>(src, sstride, ld, log2i(L), nlev, n, n2, wave, f, scale,
                                                                R(gamma), gamma_dev, R(eta), nullptr);
      else
        dwt_tail_kernel<R, 1><<<p->ndb, kTailThreads, lds, s>>>(src, sstride, ld, log2i(L), nlev, n, n2, wave, f, scale,
                                                                R(gamma), gamma_dev, R(eta), wwave);
      PR_TRY_LAUNCH();
      break;
    }
    // both passes form two outputs per thread: L^2 / 4 threads
    const dim3 grid(grid_for(static_cast<int64_t>(L) * (L / 4), kThreads, 2048), p->ndb);
    dwt_rows_kernel<R><<<grid, kThreads, 0, s>>>(src, sstride, ld, L, rows, n2, f);
    PR_TRY_LAUNCH();
    const int last = lev == p->levels;
    R* llout = last ? nullptr : (lev & 1 ? lla : llb);
    // the column pass forms four output rows per thread on large levels
    const dim3 grid4(grid_for(static_cast<int64_t>(L) * (L / 8), kThreads, 2048), p->ndb);
    if (mode == 0 && L >= kCols4MinL)
      dwt_cols_kernel<R, 0, 4><<<grid4, kThreads, 0, s>>>(rows, n2, L, n, llout, last, wave, f, scale, R(gamma),
                                                          gamma_dev, R(eta), nullptr);
    else if (mode == 0)
      dwt_cols_kernel<R, 0, 2><<<grid, kThreads, 0, s>>>(rows, n2, L, n, llout, last, wave, f, scale, R(gamma),
                                                         gamma_dev, R(eta), nullptr);
    else if (L >= kCols4MinL)
      dwt_cols_kernel<R, 1, 4><<<grid4, kThreads, 0, s>>>(rows, n2, L, n, llout, last, wave, f, scale, R(gamma),
                                                          gamma_dev, R(eta), wwave);
    else
      dwt_cols_kernel<R, 1, 2><<<grid, kThreads, 0, s>>>(rows, n2, L, n, llout, last, wave, f, scale, R(gamma),
                                                         gamma_dev, R(eta), wwave);
    PR_TRY_LAUNCH();
  }
  return PR_OK;
}

// Per-basis inverse transforms into p->recon.
template <typename R>
int synthesis_bases(pr_psi_plan_t* p, const R* coef, hipStream_t s) {
  const int n = p->n;
  const int64_t n2 = static_cast<int64_t>(n) * n;
  const R* wave = coef + (p->has_dirac ? n2 : 0);
  const Filt<R>* f = static_cast<const Filt<R>*>(p->filters);
  R* rows = static_cast<R*>(p->rows);
  R* lla = static_cast<R*>(p->ll_a);
  R* llb = static_cast<R*>(p->ll_b);
  R* recon = static_cast<R*>(p->recon);
  const int lev0 = tail_level<R>(n, p->levels);
  if (lev0 <= p->levels) {
    // the deepest levels down to lev0 in one launch
    const int L0 = n >> (lev0 - 1);
    const size_t lds = (static_cast<size_t>(L0) * L0 + static_cast<size_t>(L0 / 2) * (L0 / 2)) * sizeof(R);
    R* dst = lev0 == 1 ? recon : (lev0 & 1 ? lla : llb);
    const int64_t dstride = lev0 == 1 ? n2 : n2 / 4;
    idwt_tail_kernel<R><<<p->ndb, kTailThreads, lds, s>>>(wave, n2, n, log2i(n >> (p->levels - 1)),
                                                          p->levels - lev0 + 1, dst, dstride, f);
    PR_TRY_LAUNCH();
  }
  for (int lev = lev0 - 1; lev >= 1; --lev) {
    const int L = n >> (lev - 1);
    const R* llsrc = lev == p->levels ? wave : ((lev + 1) & 1 ? lla : llb);
    const int ldll = lev == p->levels ? n : L / 2;
    const int64_t llstride = lev == p->levels ? n2 : n2 / 4;
    // both passes form two outputs per thread: L^2 / 2 threads
    const dim3 grid(grid_for(static_cast<int64_t>(L) * L / 2, kThreads, 2048), p->ndb);
    idwt_cols_kernel<R><<<grid, kThreads, 0, s>>>(wave, n2, n, llsrc, ldll, llstride, L, rows, f);
    PR_TRY_LAUNCH();
    R* dst = lev == 1 ? recon : (lev & 1 ? lla : llb);
    const int64_t dstride = lev == 1 ? n2 : n2 / 4;
    idwt_rows_kernel<R><<<grid, kThreads, 0, s>>>(rows, n2, L, dst, dstride, f);
    PR_TRY_LAUNCH();
  }
  return PR_OK;
}

template <typename R>
int synthesis_impl(pr_psi_plan_t* p, const R* coef, R* x, hipStream_t s) {
  const int64_t n2 = static_cast<int64_t>(p->n) * p->n;
  if (p->ndb) PR_TRY(synthesis_bases<R>(p, coef, s));
  const int G = grid_for(n2, kThreads, 4096);
  combine_kernel<R, 0><<<G, kThreads, 0, s>>>(p->has_dirac ? coef : nullptr, static_cast<const R*>(p->recon), p->ndb,
                                              n2, static_cast<R>(p->scale), nullptr, x, nullptr, nullptr);
  PR_TRY_LAUNCH();
  return PR_OK;
}

template <typename R>
int synthesis_step_impl(pr_psi_plan_t* p, const R* d, const R* z, R* zbar, const R* xprev, double* partials,
                        double* sums, hipStream_t s) {
  const int64_t n2 = static_cast<int64_t>(p->n) * p->n;
  if (p->ndb) PR_TRY(synthesis_bases<R>(p, d, s));
  const int G = grid_for(n2, kThreads, 1024);
  combine_kernel<R, 1><<<G, kThreads, 0, s>>>(p->has_dirac ? d : nullptr, static_cast<const R*>(p->recon), p->ndb, n2,
                                              static_cast<R>(p->scale), z, zbar, xprev, partials);
  PR_TRY_LAUNCH();
  if (xprev) {
    combine_finish_kernel<<<1, kThreads, 0, s>>>(partials, G, sums);
    PR_TRY_LAUNCH();
  }
  return PR_OK;
}

}  // namespace

int psi_validate(int n, int levels, uint32_t mask, int prec) {
  if (n < 2 || n > 8192 || (n & (n - 1))) { set_error("n = %d: must be a power of two in [2, 8192]", n); return PR_EINVAL; }
  if (levels < 1 || (n >> levels) < 1) { set_error("levels = %d: need 1 <= levels and n / 2^levels >= 1", levels); return PR_EINVAL; }
  if (mask == 0 || mask > 0x1FFu) { set_error("basis_mask = 0x%x: bits 0..8 only, at least one", mask); return PR_EINVAL; }
  if (prec != PR_F32 && prec != PR_F64) { set_error("prec = %d", prec); return PR_EINVAL; }
  return PR_OK;
}

void psi_prepare(pr_psi_plan_t* p, int n, int levels, uint32_t mask, int prec) {
  p->n = n;
  p->levels = levels;
  p->mask = mask;
  p->prec = prec;
  p->has_dirac = mask & 1u;
  p->ndb = 0;
  for (int k = 1; k <= 8; ++k)
    if (mask >> k & 1u) p->db_k[p->ndb++] = k;
  p->nb = p->ndb + p->has_dirac;
  p->scale = 1.0 / std::sqrt(static_cast<double>(p->nb));
}

int psi_layout(pr_psi_plan_t* p, void* persistent, void* scratch, size_t* persistent_bytes, size_t* scratch_bytes) {
  const size_t rs = p->prec == PR_F32 ? 4 : 8;
  const int64_t n2 = static_cast<int64_t>(p->n) * p->n;
  const int nd = p->ndb > 0 ? p->ndb : 1;
  Carver a(persistent);
  p->filters = a.take<char>(8 * (p->prec == PR_F32 ? sizeof(Filt<float>) : sizeof(Filt<double>)));
  if (persistent_bytes) *persistent_bytes = a.bytes();
  Carver b(scratch);
  p->rows = b.take<char>(nd * n2 * rs);
  p->ll_a = b.take<char>(nd * (n2 / 4 > 0 ? n2 / 4 : 1) * rs);
  p->ll_b = b.take<char>(nd * (n2 / 4 > 0 ? n2 / 4 : 1) * rs);
  p->recon = b.take<char>(nd * n2 * rs);
  if (scratch_bytes) *scratch_bytes = b.bytes();
  return PR_OK;
}

template <typename R>
static int upload_filters(pr_psi_plan_t* p, hipStream_t s) {
  Filt<R> host[8] = {};
  for (int i = 0; i < p->ndb; ++i) {
    const int k = p->db_k[i];
    const double* h = p->host_filters[k];
    host[i].taps = 2 * k;
    for (int q = 0; q < 2 * k; ++q) {
      host[i].h[q] = static_cast<R>(h[q]);
      host[i].g[q] = static_cast<R>((q & 1 ? -1.0 : 1.0) * h[2 * k - 1 - q]);
    }
  }
  PR_TRY_HIP(hipMemcpyAsync(p->filters, host, sizeof(host), hipMemcpyHostToDevice, s));
  // the host array must outlive the copy
  PR_TRY_HIP(hipStreamSynchronize(s));
  return PR_OK;
}

// the tail kernels take up to kTailLds of dynamic LDS (on the current device)
template <typename R>
static int allow_tail_lds() {
  const hipFuncAttribute attr = hipFuncAttributeMaxDynamicSharedMemorySize;
  PR_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(dwt_tail_kernel<R, 0>), attr, kTailLds));
  PR_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(dwt_tail_kernel<R, 1>), attr, kTailLds));
  PR_TRY_HIP(hipFuncSetAttribute(reinterpret_cast<const void*>(idwt_tail_kernel<R>), attr, kTailLds));
  return PR_OK;
}

int psi_create(pr_psi_plan_t* p, hipStream_t s) {
  for (int k = 1; k <= 8; ++k) {
    if (!daubechies_filter(k, p->host_filters[k])) {
      set_error("Daubechies filter %d: root finding did not converge", k);
      return PR_EINVAL;
    }
  }
  PR_TRY(p->prec == PR_F32 ? allow_tail_lds<float>() : allow_tail_lds<double>());
  return p->prec == PR_F32 ? upload_filters<float>(p, s) : upload_filters<double>(p, s);
}

int psi_analysis(pr_psi_plan_t* p, const void* x, void* alpha, hipStream_t s) {
  if (p->prec == PR_F32)
    return analysis_impl<float>(p, static_cast<const float*>(x), static_cast<float*>(alpha), 0, 0, nullptr, 1, s);
  return analysis_impl<double>(p, static_cast<const double*>(x), static_cast<double*>(alpha), 0, 0, nullptr, 1, s);
}

int psi_synthesis(pr_psi_plan_t* p, const void* alpha, void* x, hipStream_t s) {
  if (p->prec == PR_F32) return synthesis_impl<float>(p, static_cast<const float*>(alpha), static_cast<float*>(x), s);
  return synthesis_impl<double>(p, static_cast<const double*>(alpha), static_cast<double*>(x), s);
}

int psi_dual_update(pr_psi_plan_t* p, const void* zbar, int positive_in, void* d, double gamma, double eta,
                    hipStream_t s, const double* gamma_dev, const void* weights) {
  (void)positive_in;
  if (p->prec == PR_F32)
    return analysis_impl<float>(p, static_cast<const float*>(zbar), static_cast<float*>(d), 1, gamma, gamma_dev, eta, s,
                                static_cast<const float*>(weights));
  return analysis_impl<double>(p, static_cast<const double*>(zbar), static_cast<double*>(d), 1, gamma, gamma_dev, eta,
                               s, static_cast<const double*>(weights));
}

int psi_synthesis_step(pr_psi_plan_t* p, const void* d, const void* z, void* zbar, const void* xprev,
                       double* partials, double* sums, hipStream_t s) {
  if (p->prec == PR_F32)
    return synthesis_step_impl<float>(p, static_cast<const float*>(d), static_cast<const float*>(z),
                                      static_cast<float*>(zbar), static_cast<const float*>(xprev), partials, sums, s);
  return synthesis_step_impl<double>(p, static_cast<const double*>(d), static_cast<const double*>(z),
                                     static_cast<double*>(zbar), static_cast<const double*>(xprev), partials, sums, s);
}

}  // namespace pr
