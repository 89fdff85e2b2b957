// F Z S and its adjoint (eq. matrix_equation): gridding correction, zero
// padding to the oversampled K x K grid and the unnormalised 2-D FFT, as two
// passes of Stockham FFTs over lines held in LDS (radix 16, then radix 4 and
// 2 for what remains of log2 K). The zero padding is pruned: the forward row
// pass transforms only the n image rows, and the adjoint column pass keeps
// only the n rows the crop Z^T needs; within a line, the first stage reads
// its inputs straight from memory (the padding's zeros are never loaded) and
// the last stage writes straight to memory (cropped outputs are never
// stored).
//
// Layouts: image x[iy*n + ix]; intermediate A[iy*K + kx] (n rows of K);
// grid[ky*K + kx], ky = v cell, kx = u cell. Pixel offset p = i - n/2 sits at
// grid index p mod K.
#include <cstring>
#include <vector>

#include "fused.hpp"
#include "phi.hpp"

namespace pr {

namespace {

constexpr int kFftThreads = 512;

// Lines of length K held in LDS at stride LS (complex elements); element i
// of a line sits at lds_at(i) = i + i / 16, one pad slot per 16 elements, so
// that the strided stores of the early stages spread over the banks. All
// threads of the block cooperate on the W lines. Stockham stages: radix 16
// (a 4 x 4 split in registers) while four factors of two remain, then radix
// 4 and radix 2; K = 4096 takes three stages. The first stage reads through
// the caller's load function, the last writes through its store function,
// the stages between go through LDS (each reads its inputs into registers,
// synchronises, then writes in place).
__device__ __forceinline__ int lds_at(int i) { return i + (i >> 4); }

template <typename C, bool INV>
__device__ __forceinline__ void dft4(C& a0, C& a1, C& a2, C& a3) {
  const C s0 = cadd(a0, a2), d0 = csub(a0, a2);
  const C s1 = cadd(a1, a3), d1 = csub(a1, a3);
  // the rotation by -i (forward) or +i (inverse)
  const C rd1 = INV ? cmk<C>(-d1.y, d1.x) : cmk<C>(d1.y, -d1.x);
  a0 = cadd(s0, s1);
  a2 = csub(s0, s1);
  a1 = cadd(d0, rd1);
  a3 = csub(d0, rd1);
}

// 16-point DFT of v[0..15] in place, output in natural order: X[k1 + 4 k2] =
// sum_n2 W16^(n2 k1) W4^(n2 k2) sum_n1 W4^(n1 k1) v[4 n1 + n2].
template <typename C, bool INV>
__device__ __forceinline__ void dft16(C* v) {
  using R = typename CxOf<C>::R;
  constexpr R c1 = R(0.92387953251128675613), s1 = R(0.38268343236508977173), h = R(0.70710678118654752440);
#pragma unroll
  for (int n2 = 0; n2 < 4; ++n2) dft4<C, INV>(v[n2], v[n2 + 4], v[n2 + 8], v[n2 + 12]);
  // v[n2 + 4 k1] *= W16^(n2 k1), W16^m = exp(-+ 2 pi i m / 16)
  const R sg = INV ? R(1) : R(-1);
  v[5] = cmul(v[5], cmk<C>(c1, sg * s1));     // m = 1
  v[9] = cmul(v[9], cmk<C>(h, sg * h));       // m = 2
  v[13] = cmul(v[13], cmk<C>(s1, sg * c1));   // m = 3
  v[6] = cmul(v[6], cmk<C>(h, sg * h));       // m = 2
  v[10] = INV ? cmk<C>(-v[10].y, v[10].x) : cmk<C>(v[10].y, -v[10].x);   // m = 4
  v[14] = cmul(v[14], cmk<C>(-h, sg * h));    // m = 6
  v[7] = cmul(v[7], cmk<C>(s1, sg * c1));     // m = 3
  v[11] = cmul(v[11], cmk<C>(-h, sg * h));    // m = 6
  v[15] = cmul(v[15], cmk<C>(-c1, -sg * s1)); // m = 9
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1) dft4<C, INV>(v[4 * k1], v[4 * k1 + 1], v[4 * k1 + 2], v[4 * k1 + 3]);
  // v[4 k1 + k2] holds X[k1 + 4 k2]: transpose the 4 x 4 index
  C t[16];
#pragma unroll
  for (int k1 = 0; k1 < 4; ++k1)
#pragma unroll
    for (int k2 = 0; k2 < 4; ++k2) t[k1 + 4 * k2] = v[4 * k1 + k2];
#pragma unroll
  for (int i = 0; i < 16; ++i) v[i] = t[i];
}


// One Stockham stage of radix RX over W lines: butterfly j of a line reads
// elements j + r K / RX, multiplies by w^(k r) (k = j mod Ns, w the
// (Ns RX)-th root of unity), transforms, and writes element
// (j - k) RX + k + r Ns. FROM: read through ld(line, i, v) (false: zero);
// TO: write through st(line, i, v); else LDS. LF: consecutive threads take
// consecutive lines of one butterfly index (column passes: neighbouring
// columns share each row's memory), else consecutive butterflies of a line.
template <int RX, bool INV, bool FROM, bool TO, bool LF, int PER, typename C, typename Ld, typename St>
__device__ __forceinline__ void fft_stage(C* buf, int K, int W, int LS, int Ns, const C* __restrict__ tw, Ld& ld,
                                          St& st) {
  const int tid = threadIdx.x, nth = blockDim.x;
  const int q = K / RX, nbf = W * q, stride = K / (RX * Ns);
  const int logq = __builtin_ctz(q), logW = __builtin_ctz(W);   // powers of two
  C v[PER][RX];
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int bf = tid + i * nth;
    if (bf < nbf) {
      const int line = LF ? bf & (W - 1) : bf >> logq, j = LF ? bf >> logW : bf & (q - 1);
      const C* L = buf + line * LS;
#pragma unroll
      for (int r = 0; r < RX; ++r) {
        if constexpr (FROM) {
          if (!ld(line, j + r * q, v[i][r])) v[i][r] = cmk<C>(0, 0);
        } else {
          v[i][r] = L[lds_at(j + r * q)];
        }
      }
      const int k = j & (Ns - 1);
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < RX; ++r) {
          C w = tw[k * r * stride];
          if (INV) w = cconj(w);
          v[i][r] = cmul(v[i][r], w);
        }
      }
      if constexpr (RX == 16) {
        dft16<C, INV>(v[i]);
      } else if constexpr (RX == 4) {
        dft4<C, INV>(v[i][0], v[i][1], v[i][2], v[i][3]);
      } else {
        const C a0 = v[i][0];
        v[i][0] = cadd(a0, v[i][1]);
        v[i][1] = csub(a0, v[i][1]);
      }
    }
  }
  if constexpr (!FROM && !TO) __syncthreads();   // in place: every read done before the writes
#pragma unroll
  for (int i = 0; i < PER; ++i) {
    const int bf = tid + i * nth;
    if (bf < nbf) {
      const int line = LF ? bf & (W - 1) : bf >> logq, j = LF ? bf >> logW : bf & (q - 1);
      const int k = j & (Ns - 1);
      const int idxD = (j - k) * RX + k;
      C* L = buf + line * LS;
#pragma unroll
      for (int r = 0; r < RX; ++r) {
        if constexpr (TO) st(line, idxD + r * Ns, v[i][r]);
        else L[lds_at(idxD + r * Ns)] = v[i][r];
      }
    }
  }
}

// Butterflies per thread per stage (checked by fft_shape_ok): radix 16 one,
// radix 4 four, radix 2 eight.
constexpr int kPer16 = 1, kPer4 = 4, kPer2 = 8;

// The W lines' FFTs (K >= 16): ld gives the inputs, st takes the outputs.
template <bool INV, bool LF, typename C, typename Ld, typename St>
__device__ __forceinline__ void fft_lines(C* buf, int K, int logK, int W, int LS, const C* __restrict__ tw, Ld ld,
                                          St st) {
  const int n16 = logK >> 2;
  const bool r4 = (logK & 2) != 0, r2 = (logK & 1) != 0;
  const int nst = n16 + (r4 ? 1 : 0) + (r2 ? 1 : 0);
  int Ns = 1;
  for (int s = 0; s < n16; ++s, Ns *= 16) {
    const bool first = s == 0, last = s == nst - 1;
    if (first && last) {
      fft_stage<16, INV, true, true, LF, kPer16>(buf, K, W, LS, Ns, tw, ld, st);
    } else if (first) {
      fft_stage<16, INV, true, false, LF, kPer16>(buf, K, W, LS, Ns, tw, ld, st);
    } else if (last) {
      fft_stage<16, INV, false, true, LF, kPer16>(buf, K, W, LS, Ns, tw, ld, st);
    } else {
      fft_stage<16, INV, false, false, LF, kPer16>(buf, K, W, LS, Ns, tw, ld, st);
    }
    if (!last) __syncthreads();
  }
  if (r4) {
    if (!r2) {
      fft_stage<4, INV, false, true, LF, kPer4>(buf, K, W, LS, Ns, tw, ld, st);
    } else {
      fft_stage<4, INV, false, false, LF, kPer4>(buf, K, W, LS, Ns, tw, ld, st);
      __syncthreads();
    }
    Ns *= 4;
  }
  if (r2) fft_stage<2, INV, false, true, LF, kPer2>(buf, K, W, LS, Ns, tw, ld, st);
}

inline int ilog2(int v) { int l = 0; while ((1 << l) < v) ++l; return l; }

// Lines per block: a power of two that fits 128 KB of LDS at stride
// K + K/16 + 1 (the padded line plus one slot, so that neighbouring lines
// start on different banks), small enough to give at least 256 blocks when
// there are enough lines (one line may take up to 139 KB: FP64, K = 8192).
// The block has W * K / 16 threads (one radix-16 butterfly each), clamped
// to [64, 512]; W K <= 8192 for every K up to 8192, so the radix-4 and
// radix-2 stages fit in four and eight butterflies per thread.
template <typename R>
inline void lines_per_block(int K, int nlines, int* W, int* LS, int* threads) {
  const int ls = K + K / 16 + 1;
  const size_t per = static_cast<size_t>(ls) * sizeof(cx_t<R>);
  int w = 1;
  while (static_cast<size_t>(2 * w) * per <= 131072 && 2 * w <= nlines && nlines / (2 * w) >= 256) w *= 2;
  *W = w;
  *LS = ls;
  int t = w * K / 16;
  t = t < 64 ? 64 : (t > kFftThreads ? kFftThreads : t);
  *threads = t;
}

template <typename R>
int fft_shape_ok(int K, int W, int threads) {
  const int64_t wk = static_cast<int64_t>(W) * K;
  if (K < 16 || wk / 16 > static_cast<int64_t>(threads) * kPer16 || wk / 4 > static_cast<int64_t>(threads) * kPer4 ||
      wk / 2 > static_cast<int64_t>(threads) * kPer2) {
    set_error("internal: FFT of %d lines of %d points needs more than %d threads", W, K, threads);
    return PR_EUNSUPPORTED;
  }
  return PR_OK;
}

}  // namespace

// One plan's arrays in a fused FFT launch (several plans of one image size,
// blockIdx.y = member): the kernels below take their pointers from here when
// given a table.
template <typename R>
struct FftPtrs {
  const R* x;          // forward: the image
  const R* corr;
  const cx_t<R>* tw;
  cx_t<R>* A;          // n x K intermediate
  cx_t<R>* grid;       // K x K
  R* x_out;            // adjoint: the real image
};

namespace {

// Forward row pass: image rows -> S Z -> FFT along u -> A. Element g of a
// line is pixel (g + n/2) mod K of the image row, zero unless that is < n.
template <typename R, bool FUSED = false>
__global__ __launch_bounds__(kFftThreads) void fzs_rows_kernel(const R* __restrict__ x, const R* __restrict__ corr,
                                                             const cx_t<R>* __restrict__ tw, cx_t<R>* __restrict__ A,
                                                             int n, int K, int logK, int W, int LS,
                                                             const FftPtrs<R>* __restrict__ mp) {
  using C = cx_t<R>;
  if constexpr (FUSED) {
    const FftPtrs<R>* m = mp + blockIdx.y;
    x = global_ptr_at(&m->x); corr = global_ptr_at(&m->corr); tw = global_ptr_at(&m->tw); A = global_ptr_at(&m->A);
  }
  extern __shared__ char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const int h = n >> 1;
  const int row0 = blockIdx.x * W;
  const int lines = min(W, n - row0);
  auto ld = [&](int l, int g, C& v) {
    const int ix = (g + h) & (K - 1);
    if (ix >= n) return false;
    const int iy = row0 + l;
    v = cmk<C>(x[static_cast<int64_t>(iy) * n + ix] * corr[ix] * corr[iy], R(0));
    return true;
  };
  auto st = [&](int l, int g, C v) { A[static_cast<int64_t>(row0 + l) * K + g] = v; };
  fft_lines<false, false>(buf, K, logK, lines, LS, tw, ld, st);
}

// Column groups are laid out so that blocks on one XCD (blockIdx mod 8) take
// neighbouring columns and share L2 lines.
__device__ inline int xcd_group(int b, int nb) {
  if (nb % kXcds) return b;
  return (b % kXcds) * (nb / kXcds) + b / kXcds;
}

// Forward column pass: A (n nonzero rows at p mod K) -> FFT along v -> grid.
// W neighbouring columns per block; element g of a line is row
// (g + n/2) mod K of A, zero unless that is < n.
template <typename R, bool FUSED = false>
__global__ __launch_bounds__(kFftThreads) void fzs_cols_kernel(const cx_t<R>* __restrict__ A,
                                                             const cx_t<R>* __restrict__ tw, cx_t<R>* __restrict__ grid,
                                                             int n, int K, int logK, int W, int LS,
                                                             const FftPtrs<R>* __restrict__ mp) {
  using C = cx_t<R>;
  if constexpr (FUSED) {
    const FftPtrs<R>* m = mp + blockIdx.y;
    A = global_ptr_at(&m->A); tw = global_ptr_at(&m->tw); grid = global_ptr_at(&m->grid);
  }
  extern __shared__ char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const int h = n >> 1;
  const int kx0 = xcd_group(blockIdx.x, gridDim.x) * W;
  const C* Ac = A + kx0;
  C* gc = grid + kx0;
  auto ld = [&](int l, int g, C& v) {
    const int iy = (g + h) & (K - 1);
    if (iy >= n) return false;
    v = Ac[static_cast<int64_t>(iy) * K + l];
    return true;
  };
  auto st = [&](int l, int g, C v) { gc[static_cast<int64_t>(g) * K + l] = v; };
  fft_lines<false, true>(buf, K, logK, W, LS, tw, ld, st);
}

// Adjoint column pass: grid -> inverse FFT along v -> keep the n rows at p mod K -> A.
template <typename R, bool FUSED = false>
__global__ __launch_bounds__(kFftThreads) void fzs_adj_cols_kernel(const cx_t<R>* __restrict__ grid,
                                                                 const cx_t<R>* __restrict__ tw,
                                                                 cx_t<R>* __restrict__ A, int n, int K, int logK,
                                                                 int W, int LS, const FftPtrs<R>* __restrict__ mp) {
  using C = cx_t<R>;
  if constexpr (FUSED) {
    const FftPtrs<R>* m = mp + blockIdx.y;
    grid = global_ptr_at(&m->grid); tw = global_ptr_at(&m->tw); A = global_ptr_at(&m->A);
  }
  extern __shared__ char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const int h = n >> 1;
  const int kx0 = xcd_group(blockIdx.x, gridDim.x) * W;
  const C* gc = grid + kx0;
  C* Ac = A + kx0;
  auto ld = [&](int l, int g, C& v) {
    v = gc[static_cast<int64_t>(g) * K + l];
    return true;
  };
  auto st = [&](int l, int g, C v) {
    const int iy = (g + h) & (K - 1);
    if (iy < n) Ac[static_cast<int64_t>(iy) * K + l] = v;
  };
  fft_lines<true, true>(buf, K, logK, W, LS, tw, ld, st);
}

// Adjoint row pass: A rows -> inverse FFT along u -> crop, correct, real part.
// MODE 0: x = Re(.). MODE 1 (gradient step of Algorithm 1):
// x_out = x_in - rho Re(.), zbar = max(x_out, 0).
template <typename R, int MODE, bool FUSED = false>
__global__ __launch_bounds__(kFftThreads) void fzs_adj_rows_kernel(const cx_t<R>* __restrict__ A,
                                                                 const R* __restrict__ corr,
                                                                 const cx_t<R>* __restrict__ tw, R* __restrict__ x_out,
                                                                 const R* __restrict__ x_in, R* __restrict__ zbar,
                                                                 R rho, int n, int K, int logK, int W, int LS,
                                                                 const FftPtrs<R>* __restrict__ mp) {
  using C = cx_t<R>;
  if constexpr (FUSED) {   // plain adjoint only (MODE 0)
    const FftPtrs<R>* m = mp + blockIdx.y;
    A = global_ptr_at(&m->A); corr = global_ptr_at(&m->corr); tw = global_ptr_at(&m->tw);
    x_out = global_ptr_at(&m->x_out);
  }
  extern __shared__ char smem_raw[];
  C* buf = reinterpret_cast<C*>(smem_raw);
  const int h = n >> 1;
  const int row0 = blockIdx.x * W;
  const int lines = min(W, n - row0);
  auto ld = [&](int l, int g, C& v) {
    v = A[static_cast<int64_t>(row0 + l) * K + g];
    return true;
  };
  auto st = [&](int l, int g, C v) {
    const int ix = (g + h) & (K - 1);
    if (ix >= n) return;
    const int iy = row0 + l;
    const R val = v.x * corr[ix] * corr[iy];
    const int64_t o = static_cast<int64_t>(iy) * n + ix;
    if (MODE == 0) {
      x_out[o] = val;
    } else {
      const R xo = x_in[o] - rho * val;
      x_out[o] = xo;
      zbar[o] = xo > R(0) ? xo : R(0);
    }
  };
  fft_lines<true, false>(buf, K, logK, lines, LS, tw, ld, st);
}

template <typename R>
int fzs_impl(pr_phi_plan_t* p, const R* x, hipStream_t s) {
  using C = cx_t<R>;
  const int n = p->n, K = p->K, logK = ilog2(K);
  int Wr, LSr, Wc, LSc, Tr, Tc;
  lines_per_block<R>(K, n, &Wr, &LSr, &Tr);
  lines_per_block<R>(K, K, &Wc, &LSc, &Tc);
  PR_TRY(fft_shape_ok<R>(K, Wr, Tr));
  PR_TRY(fft_shape_ok<R>(K, Wc, Tc));
  const size_t lds_r = static_cast<size_t>(Wr) * LSr * sizeof(C);
  const size_t lds_c = static_cast<size_t>(Wc) * LSc * sizeof(C);
  fzs_rows_kernel<R><<<(n + Wr - 1) / Wr, Tr, lds_r, s>>>(
      x, static_cast<const R*>(p->corr), static_cast<const C*>(p->tw), static_cast<C*>(p->fft_tmp), n, K, logK, Wr, LSr,
      nullptr);
  PR_TRY_LAUNCH();
  fzs_cols_kernel<R><<<K / Wc, Tc, lds_c, s>>>(static_cast<const C*>(p->fft_tmp),
                                                       static_cast<const C*>(p->tw), static_cast<C*>(p->grid), n, K,
                                                       logK, Wc, LSc, nullptr);
  PR_TRY_LAUNCH();
  return PR_OK;
}

template <typename R, int MODE>
int fzs_adjoint_impl(pr_phi_plan_t* p, R* x_out, const R* x_in, R* zbar, double rho, hipStream_t s) {
  using C = cx_t<R>;
  const int n = p->n, K = p->K, logK = ilog2(K);
  int Wr, LSr, Wc, LSc, Tr, Tc;
  lines_per_block<R>(K, n, &Wr, &LSr, &Tr);
  lines_per_block<R>(K, K, &Wc, &LSc, &Tc);
  PR_TRY(fft_shape_ok<R>(K, Wr, Tr));
  PR_TRY(fft_shape_ok<R>(K, Wc, Tc));
  const size_t lds_r = static_cast<size_t>(Wr) * LSr * sizeof(C);
  const size_t lds_c = static_cast<size_t>(Wc) * LSc * sizeof(C);
  fzs_adj_cols_kernel<R><<<K / Wc, Tc, lds_c, s>>>(static_cast<const C*>(p->grid),
                                                           static_cast<const C*>(p->tw), static_cast<C*>(p->fft_tmp),
                                                           n, K, logK, Wc, LSc, nullptr);
  PR_TRY_LAUNCH();
  fzs_adj_rows_kernel<R, MODE><<<(n + Wr - 1) / Wr, Tr, lds_r, s>>>(
      static_cast<const C*>(p->fft_tmp), static_cast<const R*>(p->corr), static_cast<const C*>(p->tw), x_out, x_in,
      zbar, static_cast<R>(rho), n, K, logK, Wr, LSr, nullptr);
  PR_TRY_LAUNCH();
  return PR_OK;
}

// ---------------------------------------------------------------------------
// fused passes: one launch per pass for all members of one image size
// ---------------------------------------------------------------------------
template <typename R>
size_t fused_fft_bytes_t(const std::vector<int>& counts) {
  Carver c(nullptr);
  for (int k : counts) {
    c.take<FftPtrs<R>>(k);
    c.take<FftPtrs<R>>(k);
  }
  return c.bytes();
}

template <typename R>
int fused_fft_build_t(FusedStages* f, Carver& c) {
  using C = cx_t<R>;
  for (FusedStages::Cls& k : f->cls) {
    const int cnt = static_cast<int>(k.idx.size());
    k.d_fwd = c.take<FftPtrs<R>>(cnt);
    k.d_adj = c.take<FftPtrs<R>>(cnt);
    k.h_fwd.assign(cnt * sizeof(FftPtrs<R>), 0);
    k.h_adj.assign(cnt * sizeof(FftPtrs<R>), 0);
    for (int i = 0; i < cnt; ++i) {
      const pr_phi_plan_t* p = f->plans[k.idx[i]];
      FftPtrs<R> q{};
      q.corr = static_cast<const R*>(p->corr);
      q.tw = static_cast<const C*>(p->tw);
      q.A = static_cast<C*>(p->fft_tmp);
      q.grid = static_cast<C*>(p->grid);
      std::memcpy(k.h_fwd.data() + i * sizeof q, &q, sizeof q);
      std::memcpy(k.h_adj.data() + i * sizeof q, &q, sizeof q);
    }
    k.up_fwd.assign(cnt, nullptr);
    k.up_adj.assign(cnt, nullptr);
  }
  return PR_OK;
}

// Patch the members' image pointers into a class table; upload when changed
// (then wait, so the host table may change on the next call).
template <typename R, typename V>
int upload_ptrs(std::vector<char>& h, std::vector<const void*>& up, void* dev, const std::vector<int>& idx,
                V* const* vec, V* FftPtrs<R>::*field, hipStream_t s) {
  bool changed = false;
  for (size_t i = 0; i < idx.size(); ++i) {
    FftPtrs<R>* q = reinterpret_cast<FftPtrs<R>*>(h.data() + i * sizeof(FftPtrs<R>));
    q->*field = vec[idx[i]];
    if (up[i] != static_cast<const void*>(vec[idx[i]])) changed = true;
  }
  if (!changed) return PR_OK;
  PR_TRY_HIP(hipMemcpyAsync(dev, h.data(), h.size(), hipMemcpyHostToDevice, s));
  PR_TRY_HIP(hipStreamSynchronize(s));
  for (size_t i = 0; i < idx.size(); ++i) up[i] = vec[idx[i]];
  return PR_OK;
}

template <typename R>
int fused_fzs_t(FusedStages* f, const void* const* x, hipStream_t s) {
  using C = cx_t<R>;
  for (FusedStages::Cls& k : f->cls) {
    PR_TRY((upload_ptrs<R, const R>(k.h_fwd, k.up_fwd, k.d_fwd, k.idx, reinterpret_cast<const R* const*>(x),
                                    &FftPtrs<R>::x, s)));
    const int n = k.n, K = 2 * n, logK = ilog2(K);
    const unsigned cnt = static_cast<unsigned>(k.idx.size());
    int Wr, LSr, Wc, LSc, Tr, Tc;
    lines_per_block<R>(K, n, &Wr, &LSr, &Tr);
    lines_per_block<R>(K, K, &Wc, &LSc, &Tc);
    PR_TRY(fft_shape_ok<R>(K, Wr, Tr));
    PR_TRY(fft_shape_ok<R>(K, Wc, Tc));
    const FftPtrs<R>* mp = static_cast<const FftPtrs<R>*>(k.d_fwd);
    fzs_rows_kernel<R, true><<<dim3((n + Wr - 1) / Wr, cnt), Tr, static_cast<size_t>(Wr) * LSr * sizeof(C), s>>>(
        nullptr, nullptr, nullptr, nullptr, n, K, logK, Wr, LSr, mp);
    PR_TRY_LAUNCH();
    fzs_cols_kernel<R, true><<<dim3(K / Wc, cnt), Tc, static_cast<size_t>(Wc) * LSc * sizeof(C), s>>>(
        nullptr, nullptr, nullptr, n, K, logK, Wc, LSc, mp);
    PR_TRY_LAUNCH();
  }
  return PR_OK;
}

template <typename R>
int fused_fzs_adjoint_t(FusedStages* f, void* const* x, hipStream_t s) {
  using C = cx_t<R>;
  for (FusedStages::Cls& k : f->cls) {
    PR_TRY((upload_ptrs<R, R>(k.h_adj, k.up_adj, k.d_adj, k.idx, reinterpret_cast<R* const*>(x), &FftPtrs<R>::x_out,
                              s)));
    const int n = k.n, K = 2 * n, logK = ilog2(K);
    const unsigned cnt = static_cast<unsigned>(k.idx.size());
    int Wr, LSr, Wc, LSc, Tr, Tc;
    lines_per_block<R>(K, n, &Wr, &LSr, &Tr);
    lines_per_block<R>(K, K, &Wc, &LSc, &Tc);
    PR_TRY(fft_shape_ok<R>(K, Wr, Tr));
    PR_TRY(fft_shape_ok<R>(K, Wc, Tc));
    const FftPtrs<R>* mp = static_cast<const FftPtrs<R>*>(k.d_adj);
    fzs_adj_cols_kernel<R, true><<<dim3(K / Wc, cnt), Tc, static_cast<size_t>(Wc) * LSc * sizeof(C), s>>>(
        nullptr, nullptr, nullptr, n, K, logK, Wc, LSc, mp);
    PR_TRY_LAUNCH();
    fzs_adj_rows_kernel<R, 0, true><<<dim3((n + Wr - 1) / Wr, cnt), Tr, static_cast<size_t>(Wr) * LSr * sizeof(C), s>>>(
        nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, R(0), n, K, logK, Wr, LSr, mp);
    PR_TRY_LAUNCH();
  }
  return PR_OK;
}

}  // namespace

size_t fused_fft_bytes(const std::vector<int>& counts, int prec) {
  return prec == PR_F32 ? fused_fft_bytes_t<float>(counts) : fused_fft_bytes_t<double>(counts);
}

int fused_fft_build(FusedStages* f, Carver& c) {
  return f->prec == PR_F32 ? fused_fft_build_t<float>(f, c) : fused_fft_build_t<double>(f, c);
}

int fused_fzs(FusedStages* f, const void* const* x, hipStream_t s) {
  return f->prec == PR_F32 ? fused_fzs_t<float>(f, x, s) : fused_fzs_t<double>(f, x, s);
}

int fused_fzs_adjoint(FusedStages* f, void* const* x, hipStream_t s) {
  return f->prec == PR_F32 ? fused_fzs_adjoint_t<float>(f, x, s) : fused_fzs_adjoint_t<double>(f, x, s);
}

int phi_fzs(pr_phi_plan_t* p, const void* x, hipStream_t s) {
  if (p->prec == PR_F32) return fzs_impl<float>(p, static_cast<const float*>(x), s);
  return fzs_impl<double>(p, static_cast<const double*>(x), s);
}

int phi_fzs_adjoint(pr_phi_plan_t* p, void* x, hipStream_t s) {
  if (p->prec == PR_F32) return fzs_adjoint_impl<float, 0>(p, static_cast<float*>(x), nullptr, nullptr, 0.0, s);
  return fzs_adjoint_impl<double, 0>(p, static_cast<double*>(x), nullptr, nullptr, 0.0, s);
}

int phi_fzs_adjoint_step(pr_phi_plan_t* p, const void* x_in, double rho, void* x_out, void* zbar, hipStream_t s) {
  if (p->prec == PR_F32)
    return fzs_adjoint_impl<float, 1>(p, static_cast<float*>(x_out), static_cast<const float*>(x_in),
                                      static_cast<float*>(zbar), rho, s);
  return fzs_adjoint_impl<double, 1>(p, static_cast<double*>(x_out), static_cast<const double*>(x_in),
                                     static_cast<double*>(zbar), rho, s);
}

}  // namespace pr
