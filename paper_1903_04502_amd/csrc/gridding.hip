// G W (degridding) and its adjoint W G^T (gridding) with the pre-sampled
// Kaiser-Bessel kernel (eq. matrix_equation, Section "Kernel Pre-Sampling"),
// on visibilities sorted by grid tile.
//
// Degridding: one work item = a run of one tile's visibilities. The block
// stages the tile's (T+J-1)^2 grid patch in LDS and each thread interpolates
// one visibility at a time from it.
//
// Gridding is deterministic (no float atomics anywhere): within an item the
// visibilities are also sorted by their first tap cell ("base cell"). For each
// base cell c and tap (a, b) the item accumulates the moment
//   m[c][a][b] = sum_{k in c} g_a(u_k) g_b(v_k) w_k y_k
// in a fixed order: streams of J lanes walk contiguous runs of staged
// visibilities, lane a holding the J sums of column a in registers; a run that
// starts inside a stream is stored directly, a run continued from the previous
// stream is parked in a side slot and added after a barrier in stream order.
// The item's patch value at cell q is sum_{a,b} m[q - (a,b)][a][b]. Patches are
// written per item and a merge kernel adds the up to four overlapping tile
// patches of each grid cell, items in order.
#include <cstring>
#include <mutex>
#include <set>
#include <type_traits>
#include <utility>

#include "fused.hpp"
#include "phi.hpp"
#include "taps.hpp"

namespace pr {

constexpr int kSlotT2 = 0;      // ||t||^2 of the ADMM degridding epilogue
constexpr int kSlotR2 = 1;      // ||v - y||^2
constexpr int kSlotKappa = 2;   // ball scale min(1, eps / ||t||)
constexpr int kSlotNonfinite = 3;

namespace {

constexpr int kThreads = 256;
constexpr size_t kLdsSoft = 81920;    // two blocks per CU
constexpr size_t kLdsHard = 163840;   // per-workgroup limit on gfx950

__host__ __device__ constexpr size_t align16(size_t v) { return (v + 15) & ~size_t(15); }

// Visibility storage and kernel lookup of a launch (template argument LK):
// 0 nearest sample and 1 first-order lookup, both from stored (u, v, w)
// triples (taps formed in FP64 per visibility and launch); 2 nearest sample
// from stored (tap word, w) pairs (FP32 plans; the taps were formed by the
// plan with the same arithmetic).
constexpr int kLkNearest = 0, kLkLinear = 1, kLkWords = 2;

// Work-item tile field of a fused launch: tile | member << kMemberShift
// (tiles < 2^20 for K <= 8192 and tiles >= 8; members < 4096).
constexpr int kMemberShift = 20;
__host__ __device__ inline int item_tile(const int4& it) { return it.x & ((1 << kMemberShift) - 1); }
__host__ __device__ inline int item_member(const int4& it) { return static_cast<int>(static_cast<uint32_t>(it.x) >> kMemberShift); }

// Complex zero written as one 64-bit pattern for FP32 (a single 64-bit move
// per accumulator instead of two 32-bit ones).
template <typename C>
__device__ __forceinline__ C zero_cx() {
  if constexpr (sizeof(C) == 8) return __builtin_bit_cast(C, 0.0);
  else return cmk<C>(0.0, 0.0);
}

// Element at a 32-bit byte offset from a (typically block-uniform) base: the
// address is formed as base + zero-extended offset, one VALU add at most.
template <typename T>
__device__ __forceinline__ T* byte_at(T* base, uint32_t boff) {
  using B = typename std::conditional<std::is_const<T>::value, const char, char>::type;
  return reinterpret_cast<T*>(reinterpret_cast<B*>(base) + boff);
}

// Taps of one visibility and its base cell (lu, lv) relative to tile
// (tu, tv). TW: x holds the tap word's bits, y is unused; else x, y = u, v.
template <bool TW, typename R>
__device__ __forceinline__ void vis_taps(R x, R y, double kappa, int J, int D, int K, int T, int tu, int tv,
                                         AxisTaps& xu, AxisTaps& xv, int& lu, int& lv) {
  if constexpr (TW) {
    const uint32_t w = __float_as_uint(static_cast<float>(x));
    xu = word_axis((w >> 8) & 0xFFFu);
    xv = word_axis(w >> 20);
    lu = static_cast<int>(w & 15u);
    lv = static_cast<int>((w >> 4) & 15u);
  } else {
    xu = axis_taps(static_cast<double>(x), kappa, J, D);
    xv = axis_taps(static_cast<double>(y), kappa, J, D);
    lu = mod_pow2(xu.j0, K) - tu * T;
    lv = mod_pow2(xv.j0, K) - tv * T;
  }
}

// Stored inputs of plan position k: (x, y, w) as vis_taps takes them.
template <bool TW, typename R>
__device__ __forceinline__ void vis_load(const R* uv, int64_t k, R& x, R& y, R& w) {
  if constexpr (TW) {
    const uint2 q = reinterpret_cast<const uint2*>(uv)[k];
    x = __uint_as_float(q.x);
    y = R(0);
    w = __uint_as_float(q.y);
  } else {
    x = uv[3 * k];
    y = uv[3 * k + 1];
    w = uv[3 * k + 2];
  }
}

// ---------------------------------------------------------------------------
// degridding
// ---------------------------------------------------------------------------
template <typename R>
struct GwArgs {
  const cx_t<R>* grid;
  const R* table;
  const R* uv;               // (u, v, w) triples, plan order
  const int4* items;         // this launch's schedule: (tile, begin, end, item index); block b takes
  const int32_t* sched_off;  // entries [sched_off[b], sched_off[b + 1])
  int64_t nItems;
  int K, T, P, nT, lognT, D, tlen;
  double kappa;
  R scale;
  const double* scale_dev; // when set, the scale is read from device memory
  cx_t<R>* y_out;          // MODE 0
  const cx_t<R>* y_obs;    // MODE 1
  const cx_t<R>* s_in;
  const int32_t* sec;         // MODE 2: section of each visibility (plan order)
  cx_t<R>* t_out;
  double* partials;
  // Fused launch over several plans (batched channels, plain operator only):
  // member m's own arguments are mtab[m], and the tile field of each work item
  // carries the member (tile | m << kMemberShift); the table, D and kappa of
  // the launch are shared (every member has the same kernel).
  const GwArgs* mtab;
  const int4* small;         // the small items (not in the schedule), one wave each after the block's items
  int nsmall;
};

constexpr int kDegridPer = 4;   // visibilities per thread per chunk

template <typename R, int J, int MODE, bool TAB_LDS, int LK, bool FUSED = false>
__global__ __launch_bounds__(kThreads) void degrid_kernel(GwArgs<R> a) {
  using C = cx_t<R>;
  constexpr bool LIN = LK == kLkLinear, TW = LK == kLkWords;
  const R scale = a.scale_dev ? static_cast<R>(*a.scale_dev) : a.scale;
  constexpr int CH = kThreads * kDegridPer;
  extern __shared__ char smem_raw[];
  const int tid = threadIdx.x;
  C* patch = reinterpret_cast<C*>(smem_raw);
  const int P = a.P, T = a.T;          // the same for every member of a fused launch
  // the arguments of the plan an item belongs to (FUSED: from the member
  // table). The solo kernels are separate instances that read the kernel
  // arguments only: a run-time choice between the two would leave every
  // pointer generic, and flat accesses also count against the LDS wait
  // counter, so each wait on an LDS read would wait for memory as well.
  auto mem = [&](const int4& it) -> GwArgs<R> {
    if constexpr (FUSED) {
      const GwArgs<R>* t = a.mtab + item_member(it);
      GwArgs<R> m = *t;
      m.grid = global_ptr_at(&t->grid);
      m.uv = global_ptr_at(&t->uv);
      m.y_out = global_ptr_at(&t->y_out);
      return m;
    } else {
      (void)it;
      return a;
    }
  };
  double sum_t = 0.0, sum_r = 0.0;
  double sacc[MODE == 2 ? kSecAcc : 1] = {};   // MODE 2: ||t||^2 per section
  // ADMM epilogue of one visibility: t = v + s - y and the FP64 partials
  auto admm_out = [&](int64_t k, C yk, C yo, C sk, int sj) {
    const C t = cmk<C>(yk.x + sk.x - yo.x, yk.y + sk.y - yo.y);
    a.t_out[k] = t;
    const double tr = t.x, ti = t.y, dr = static_cast<double>(yk.x) - yo.x, di = static_cast<double>(yk.y) - yo.y;
    const double t2 = tr * tr + ti * ti;
    sum_t += t2;
    sum_r += dr * dr + di * di;
    if (MODE == 2) {
#pragma unroll
      for (int jj = 0; jj < (MODE == 2 ? kSecAcc : 1); ++jj) sacc[jj] += sj == jj ? t2 : 0.0;
    }
    (void)sj;
  };
  // inputs of this thread's visibilities for the current and the next chunk
  R cu_[kDegridPer], cv_[kDegridPer], cw_[kDegridPer], nu_[kDegridPer], nv_[kDegridPer], nw_[kDegridPer];
  auto load = [&](const R* uvp, int64_t c0, int64_t cend, R* u, R* v, R* w) {
#pragma unroll
    for (int j = 0; j < kDegridPer; ++j) {
      const int64_t k = c0 + tid + j * kThreads;
      if (k < cend) vis_load<TW>(uvp, k, u[j], v[j], w[j]);
    }
  };
  const int kbeg = a.sched_off[blockIdx.x], kend = a.sched_off[blockIdx.x + 1];
  // the first item's visibilities are in flight while the table is copied
  if (kbeg < kend) {
    const int4 it0 = a.items[kbeg];
    load(mem(it0).uv, it0.y, it0.z, cu_, cv_, cw_);
  }
  const R* tab = a.table;
  if (TAB_LDS) {
    R* t = reinterpret_cast<R*>(smem_raw + align16(static_cast<size_t>(a.P) * a.P * sizeof(C)));
    for (int i = tid; i < a.tlen; i += kThreads) t[i] = a.table[i];
    tab = t;
  }
  for (int ks = kbeg; ks < kend; ++ks) {
    const int4 it = a.items[ks];
    const GwArgs<R> m = mem(it);
    const int K = m.K;
    const int tile = item_tile(it);
    const int tv = tile >> m.lognT, tu = tile & (m.nT - 1);
    const R iscale = FUSED ? m.scale : scale;
    if (ks > kbeg) load(m.uv, it.y, it.z, cu_, cv_, cw_);
    __syncthreads();
    const float invP = 1.0f / P;
    for (int i = tid; i < P * P; i += kThreads) {
      const int pv = small_div(i, P, invP), pu = i - pv * P;
      const int gv = (tv * T + pv) & (K - 1), gu = (tu * T + pu) & (K - 1);
      patch[i] = m.grid[static_cast<int64_t>(gv) * K + gu];
    }
    __syncthreads();
    for (int64_t c0 = it.y; c0 < it.z; c0 += CH) {
      if (c0 + CH < it.z) load(m.uv, c0 + CH, it.z, nu_, nv_, nw_);
      // MODE 2: the chunk's y, s and section ids, issued before any of its stores
      // (for MODE 1 the same early issue measured slower: it loads them in place)
      constexpr int NA = MODE == 2 ? kDegridPer : 1;
      C yo_[NA], sk_[NA];
      int sj_[NA];
      if (MODE == 2) {
#pragma unroll
        for (int j = 0; j < NA; ++j) {
          const int64_t k = c0 + tid + j * kThreads;
          if (k < it.z) {
            yo_[j] = a.y_obs[k];
            sk_[j] = a.s_in ? a.s_in[k] : cmk<C>(R(0), R(0));
            sj_[j] = a.sec[k];
          }
        }
      }
#pragma unroll
      for (int j = 0; j < kDegridPer; ++j) {
        const int64_t k = c0 + tid + j * kThreads;
        if (k >= it.z) continue;
        AxisTaps xu, xv;
        int lu, lv;
        vis_taps<TW>(cu_[j], cv_[j], m.kappa, J, a.D, K, T, tu, tv, xu, xv, lu, lv);
        if (static_cast<unsigned>(lu) >= static_cast<unsigned>(T) || static_cast<unsigned>(lv) >= static_cast<unsigned>(T)) {
          // cannot happen for a plan's own sorted baselines; flag instead of reading out of the patch
          const R nan = R(NAN);
          if (MODE == 0) m.y_out[k] = cmk<C>(nan, nan);
          else a.t_out[k] = cmk<C>(nan, nan);
          continue;
        }
        R wu[J], wv[J];
        axis_weights<LIN, J>(tab, xu, a.D, a.tlen, wu);
        axis_weights<LIN, J>(tab, xv, a.D, a.tlen, wv);
        R accr = 0, acci = 0;
#pragma unroll
        for (int b = 0; b < J; ++b) {
          const C* row = patch + (lv + b) * P + lu;
          R rr = 0, ri = 0;
#pragma unroll
          for (int q = 0; q < J; ++q) {
            const C g = row[q];
            rr += wu[q] * g.x;
            ri += wu[q] * g.y;
          }
          accr += wv[b] * rr;
          acci += wv[b] * ri;
        }
        const R ws = cw_[j] * iscale;
        const C yk = cmk<C>(accr * ws, acci * ws);
        if (MODE == 0) {
          m.y_out[k] = yk;
        } else {
          const C yo = MODE == 2 ? yo_[MODE == 2 ? j : 0] : a.y_obs[k];
          const C sk = MODE == 2 ? sk_[MODE == 2 ? j : 0] : (a.s_in ? a.s_in[k] : cmk<C>(R(0), R(0)));
          admm_out(k, yk, yo, sk, MODE == 2 ? sj_[MODE == 2 ? j : 0] : 0);
        }
      }
#pragma unroll
      for (int j = 0; j < kDegridPer; ++j) {
        cu_[j] = nu_[j];
        cv_[j] = nv_[j];
        cw_[j] = nw_[j];
      }
    }
  }
  // The small items (plans whose gridding splits them off): one wave per
  // item, lane l computes visibility l from the grid directly (the J^2 cells
  // it reads are the patch values the item's block would have loaded; the
  // same sums in the same order), with no block barrier: the waves run their
  // items independently.
  if (a.nsmall > 0) {
    // a block without scheduled items has passed no barrier since the table
    // copy: every wave's part of the table must be in LDS before any is read
    if (TAB_LDS) __syncthreads();
    constexpr int kWaves = kThreads / 64;
    const int lane = tid & 63;
    for (int idx = static_cast<int>(blockIdx.x) * kWaves + (tid >> 6); idx < a.nsmall;
         idx += kWaves * static_cast<int>(gridDim.x)) {
      const int4 it = a.small[idx];
      if (lane >= it.z - it.y) continue;
      const GwArgs<R> m = mem(it);
      const int K = m.K;
      const int tile = item_tile(it);
      const int tv = tile >> m.lognT, tu = tile & (m.nT - 1);
      const int64_t k = static_cast<int64_t>(it.y) + lane;
      R u, v, w;
      vis_load<TW>(m.uv, k, u, v, w);
      AxisTaps xu, xv;
      int lu, lv;
      vis_taps<TW>(u, v, m.kappa, J, a.D, K, T, tu, tv, xu, xv, lu, lv);
      if (static_cast<unsigned>(lu) >= static_cast<unsigned>(T) || static_cast<unsigned>(lv) >= static_cast<unsigned>(T)) {
        const R nan = R(NAN);
        if (MODE == 0) m.y_out[k] = cmk<C>(nan, nan);
        else a.t_out[k] = cmk<C>(nan, nan);
        continue;
      }
      R wu[J], wv[J];
      axis_weights<LIN, J>(tab, xu, a.D, a.tlen, wu);
      axis_weights<LIN, J>(tab, xv, a.D, a.tlen, wv);
      R accr = 0, acci = 0;
#pragma unroll
      for (int b = 0; b < J; ++b) {
        const C* row = m.grid + static_cast<int64_t>((tv * T + lv + b) & (K - 1)) * K;
        R rr = 0, ri = 0;
#pragma unroll
        for (int q = 0; q < J; ++q) {
          const C g = row[(tu * T + lu + q) & (K - 1)];
          rr += wu[q] * g.x;
          ri += wu[q] * g.y;
        }
        accr += wv[b] * rr;
        acci += wv[b] * ri;
      }
      const R ws = w * (FUSED ? m.scale : scale);
      const C yk = cmk<C>(accr * ws, acci * ws);
      if (MODE == 0) {
        m.y_out[k] = yk;
      } else {
        admm_out(k, yk, a.y_obs[k], a.s_in ? a.s_in[k] : cmk<C>(R(0), R(0)), MODE == 2 ? a.sec[k] : 0);
      }
    }
  }
  if (MODE >= 1) {
    __syncthreads();
    double* sh = reinterpret_cast<double*>(smem_raw);
    const double bt = block_sum_f64(sum_t, sh);
    const double br = block_sum_f64(sum_r, sh);
    if (tid == 0) {
      a.partials[kSlotT2 * kPartialsMax + blockIdx.x] = bt;
      a.partials[kSlotR2 * kPartialsMax + blockIdx.x] = br;
    }
    if (MODE == 2) {
      // all section sums in one pass: a fixed xor butterfly per wave, then the
      // waves in order (sh is free again after the trees above)
      constexpr int NS = MODE == 2 ? kSecAcc : 1;
      const int lane = tid & 63, wave = tid >> 6;
#pragma unroll
      for (int jj = 0; jj < NS; ++jj) {
        double v = sacc[jj];
#pragma unroll
        for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m, 64);
        if (lane == 0) sh[wave * NS + jj] = v;
      }
      __syncthreads();
      if (tid < NS) {
        double bj = 0.0;
        for (int q = 0; q < kThreads / 64; ++q) bj += sh[q * NS + tid];
        a.partials[(kSlotSec0 + tid) * kPartialsMax + blockIdx.x] = bj;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// gridding
// ---------------------------------------------------------------------------
template <typename R>
struct GwAdjArgs {
  const R* table;
  const R* uv;               // (u, v, w) triples, plan order
  const int4* items;         // this launch's schedule: (tile, begin, end, item index); block b takes
  const int32_t* sched_off;  // entries [sched_off[b], sched_off[b + 1])
  int64_t nItems;
  int K, T, P, nT, lognT, D, tlen, B;
  double kappa;
  R scale;
  const double* scale_dev;   // when set, the scale is read from device memory
  const cx_t<R>* y_in;       // MODE 0
  const cx_t<R>* t_in;       // MODE 1: t = v + s - y
  cx_t<R>* s_io;             // MODE 1: multiplier, updated
  const double* scalars;     // MODE 1: ball scale at kSlotKappa
  R varrho;
  R vr_coef;                 // MODE 1: gridded q = vr_coef (v - r) + s' (1 Algorithm 1, 0 primal-dual)
  const int32_t* sec;        // MODE 1, local balls: section of each visibility (plan order), or null
  const double* kappa_sec;   // MODE 1, local balls: kappa of each section
  cx_t<R>* patches;
  const GwAdjArgs* mtab;     // fused launch over several plans (as GwArgs::mtab)
};

// LDS layout of the gridding kernel. Staged visibilities are stored
// segment-transposed (position p of a batch with L positions per segment lives
// at (p mod L) * NS + p / L), per-tap weights as planes of B values, moments
// and side slots entry-major: consecutive lanes touch consecutive words. The
// side slots reuse the staged area when it is large enough: they are written
// only after every thread has finished reading the staged batch.
template <typename R, int J, int NS>
struct GridLds {
  size_t tab, cell, wu, wv, yw, side, side_cell, mom, bits, total;
  __host__ __device__ GridLds(int T, int B, int tlen, bool tab_lds) {
    using C = cx_t<R>;
    size_t o = 0;
    tab = o;   o += tab_lds ? align16(static_cast<size_t>(tlen) * sizeof(R)) : 0;
    bits = o;  o += align16(static_cast<size_t>((T * T + 31) / 32) * sizeof(uint32_t));
    cell = o;  o += align16(static_cast<size_t>(B) * sizeof(int));
    const size_t st0 = o;
    wu = o;    o += align16(static_cast<size_t>(B) * J * sizeof(R));
    wv = o;    o += align16(static_cast<size_t>(B) * J * sizeof(R));
    yw = o;    o += align16(static_cast<size_t>(B) * sizeof(C));
    const size_t staged = o - st0;
    const size_t sb = align16(static_cast<size_t>(NS) * J * J * sizeof(C));
    const size_t cb = align16(static_cast<size_t>(NS) * sizeof(int));
    if (sb + cb <= staged) {
      side = st0;
      side_cell = st0 + sb;
    } else {
      side = o;      o += sb;
      side_cell = o; o += cb;
    }
    mom = o;   o += align16(static_cast<size_t>(T) * T * J * J * sizeof(C));
    total = o;
  }
};

constexpr int kGridPer = 4;   // staged visibilities per thread: B <= kThreads * kGridPer

// Gridding of one work item (a run of one tile's visibilities, sorted by base
// cell). Per batch of nb <= B staged visibilities the block is split into NS
// segments of L = ceil(nb / NS) contiguous positions; the threads of a segment
// each hold JA columns (tap a) of the J^2 moments of the current base cell in
// registers. A run that begins inside a segment is owned by it; the owner of a
// run that continues into the following segments adds their parked partial
// sums in segment order before adding the total to the cell's moments. Every
// moment is therefore a sum in a fixed order: deterministic, no atomics. The
// next batch's inputs are loaded into registers while the current one is
// accumulated.
template <typename R, int J, int JA, int MODE, bool TAB_LDS, int LK>
__global__ __launch_bounds__(kThreads) void grid_kernel(GwAdjArgs<R> a) {
  using C = cx_t<R>;
  constexpr bool LIN = LK == kLkLinear, TW = LK == kLkWords;
  const R scale = a.scale_dev ? static_cast<R>(*a.scale_dev) : a.scale;
  constexpr int JJ = J * J;
  constexpr int TPC = (J + JA - 1) / JA;
  constexpr int NS = kThreads / (TPC == 3 ? 4 : TPC);
  constexpr int TPS = kThreads / NS;            // threads per segment (TPC rounded to a divisor)
  constexpr int E = JA * J;                     // moments held per thread
  extern __shared__ char smem_raw[];
  const GridLds<R, J, NS> lay(a.T, a.B, a.tlen, TAB_LDS);
  int* st_cell = reinterpret_cast<int*>(smem_raw + lay.cell);
  R* st_wu = reinterpret_cast<R*>(smem_raw + lay.wu);
  R* st_wv = reinterpret_cast<R*>(smem_raw + lay.wv);
  C* st_yw = reinterpret_cast<C*>(smem_raw + lay.yw);
  C* side = reinterpret_cast<C*>(smem_raw + lay.side);
  int* side_cell = reinterpret_cast<int*>(smem_raw + lay.side_cell);
  C* mom = reinterpret_cast<C*>(smem_raw + lay.mom);
  uint32_t* bits = reinterpret_cast<uint32_t*>(smem_raw + lay.bits);
  const int tid = threadIdx.x;
  const int sg = tid / TPS, pa = tid - sg * TPS;
  const int q0 = pa * JA;                       // first column of this thread
  const bool cols_on = q0 < J;
  const R* tab = a.table;
  if (TAB_LDS) {
    R* t = reinterpret_cast<R*>(smem_raw + lay.tab);
    for (int i = tid; i < a.tlen; i += kThreads) t[i] = a.table[i];
    tab = t;
  }
  const int T = a.T, P = a.P, K = a.K, B = a.B;
  const int TT = T * T;
  R kappa_ball = 1;
  if (MODE == 1) kappa_ball = static_cast<R>(a.scalars[kSlotKappa]);

  const int nbits = (TT + 31) / 32;
  // Moment update of a run's total. An item of one batch has exactly one owner
  // per base cell, so the owner stores and marks the cell; items of several
  // batches accumulate into zeroed moments.
  bool single = true;
  auto flush = [&](int cell, const R* xr, const R* xi) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      if (q0 * J + e < JJ) {
        C& m = mom[(q0 * J + e) * TT + cell];
        m = single ? cmk<C>(xr[e], xi[e]) : cmk<C>(m.x + xr[e], m.y + xi[e]);
      }
    }
    if (single && pa == 0) atomicOr(&bits[cell >> 5], 1u << (cell & 31));
  };

  // raw inputs of the visibilities this thread stages (prefetched a batch ahead)
  R ru[kGridPer], rv[kGridPer], rw[kGridPer];
  C ry[kGridPer], rs[kGridPer];
  auto load_raw = [&](int b0, int n0) {
#pragma unroll
    for (int j = 0; j < kGridPer; ++j) {
      const int i = tid + j * kThreads;
      if (i < n0) {
        const int64_t k = b0 + i;
        vis_load<TW>(a.uv, k, ru[j], rv[j], rw[j]);
        if (MODE == 0) {
          ry[j] = a.y_in[k];
        } else {
          ry[j] = a.t_in[k];
          rs[j] = a.s_io[k];
        }
      }
    }
  };

  const int kend = a.sched_off[blockIdx.x + 1];
  for (int ks = a.sched_off[blockIdx.x]; ks < kend; ++ks) {
    const int4 it = a.items[ks];
    const int64_t item = it.w;
    const int tv = it.x >> a.lognT, tu = it.x & (a.nT - 1);
    const int begin = it.y, end = it.z;
    load_raw(begin, min(B, end - begin));
    single = end - begin <= B;
    __syncthreads();
    if (single) {
      for (int i = tid; i < nbits; i += kThreads) bits[i] = 0u;
    } else {
      for (int i = tid; i < TT * JJ; i += kThreads) mom[i] = cmk<C>(R(0), R(0));
      for (int i = tid; i < nbits; i += kThreads) bits[i] = ~0u;
    }
    for (int bs = begin; bs < end; bs += B) {
      const int nb = min(B, end - bs);
      // positions per segment: the smallest power of two with NS * L >= nb
      int lgL = 0;
      while ((NS << lgL) < nb) ++lgL;
      const int L = 1 << lgL;
      __syncthreads();
      // stage: first tap cell, tap weights and the weighted value of each visibility
#pragma unroll
      for (int j = 0; j < kGridPer; ++j) {
        const int i = tid + j * kThreads;
        if (i >= nb) continue;
        const int64_t k = bs + i;
        AxisTaps xu, xv;
        int lu, lv;
        vis_taps<TW>(ru[j], rv[j], a.kappa, J, a.D, K, T, tu, tv, xu, xv, lu, lv);
        const bool inside = static_cast<unsigned>(lu) < static_cast<unsigned>(T) &&
                            static_cast<unsigned>(lv) < static_cast<unsigned>(T);
        C val;
        if (MODE == 0) {
          val = ry[j];
        } else {
          // ball projection and multiplier update of Algorithm 1 from t = v + s - y:
          // r = y + kappa t, s' = s + varrho (v - r), q = vr_coef (v - r) + s'
          const C t = ry[j], sk = rs[j];
          const R omk = R(1) - (a.kappa_sec ? static_cast<R>(a.kappa_sec[a.sec[k]]) : kappa_ball);
          const C vr = cmk<C>(omk * t.x - sk.x, omk * t.y - sk.y);   // v - r
          const C sn = cmk<C>(sk.x + a.varrho * vr.x, sk.y + a.varrho * vr.y);
          a.s_io[k] = sn;
          val = cmk<C>(a.vr_coef * vr.x + sn.x, a.vr_coef * vr.y + sn.y);
        }
        const R ws = rw[j] * scale;
        val = cmk<C>(val.x * ws, val.y * ws);
        if (!inside) {
          // cannot happen for a plan's own sorted baselines; keep LDS indices in range, poison the value
          lu = lv = 0;
          val = cmk<C>(R(NAN), R(NAN));
        }
        const int si = (i & (L - 1)) * NS + (i >> lgL);
        st_cell[si] = lv * T + lu;
        st_yw[si] = val;
        R wu_[J], wv_[J];
        axis_weights<LIN, J>(tab, xu, a.D, a.tlen, wu_);
        axis_weights<LIN, J>(tab, xv, a.D, a.tlen, wv_);
#pragma unroll
        for (int q = 0; q < J; ++q) {
          st_wu[q * B + si] = wu_[q];
          st_wv[q * B + si] = wv_[q];
        }
      }
      __syncthreads();
      if (bs + B < end) load_raw(bs + B, min(B, end - bs - B));
      // accumulate the segment: positions [p0, p1), position p at (p - p0) * NS + sg
      const int p0 = sg * L;
      const int p1 = min(p0 + L, nb);
      R ar[E], ai[E], sr[E], si[E];
      bool has_side = false, defer = false;
      int cur = -1, side_c = -1;
      if (p0 < p1) {
        cur = st_cell[sg];
        bool owner = p0 == 0 || st_cell[((p0 - 1) & (L - 1)) * NS + ((p0 - 1) >> lgL)] != cur;
#pragma unroll
        for (int e = 0; e < E; ++e) ar[e] = ai[e] = R(0);
        for (int p = p0; p < p1; ++p) {
          const int ix = (p - p0) * NS + sg;
          const int c = st_cell[ix];
          if (c != cur) {
            if (owner) {
              if (cols_on) flush(cur, ar, ai);
            } else {
#pragma unroll
              for (int e = 0; e < E; ++e) { sr[e] = ar[e]; si[e] = ai[e]; }
              has_side = true;
              side_c = cur;
            }
            owner = true;
            cur = c;
#pragma unroll
            for (int e = 0; e < E; ++e) ar[e] = ai[e] = R(0);
          }
          if (cols_on) {
            const C y = st_yw[ix];
            R wv[J];
#pragma unroll
            for (int b = 0; b < J; ++b) wv[b] = st_wv[b * B + ix];
#pragma unroll
            for (int qq = 0; qq < JA; ++qq) {
              if (q0 + qq < J) {
                const R g = st_wu[(q0 + qq) * B + ix];
                const R yr = y.x * g, yi = y.y * g;
#pragma unroll
                for (int b = 0; b < J; ++b) {
                  ar[qq * J + b] += wv[b] * yr;
                  ai[qq * J + b] += wv[b] * yi;
                }
              }
            }
          }
        }
        const bool cont = p1 < nb && st_cell[(p1 & (L - 1)) * NS + (p1 >> lgL)] == cur;
        if (!owner) {
#pragma unroll
          for (int e = 0; e < E; ++e) { sr[e] = ar[e]; si[e] = ai[e]; }
          has_side = true;
          side_c = cur;
        } else if (cont) {
          defer = true;
        } else if (cols_on) {
          flush(cur, ar, ai);
        }
      }
      __syncthreads();   // the staged batch is no longer read: park the side sums
      if (pa == 0) side_cell[sg] = p0 < p1 ? (has_side ? side_c : -1) : -2;
      if (has_side && cols_on) {
#pragma unroll
        for (int e = 0; e < E; ++e)
          if (q0 * J + e < JJ) side[(q0 * J + e) * NS + sg] = cmk<C>(sr[e], si[e]);
      }
      __syncthreads();
      if (defer && cols_on) {
        // owner of a run that continues: add the following segments' parts in order
        for (int s2 = sg + 1; s2 < NS; ++s2) {
          const int c = side_cell[s2];
          if (c == -2) continue;        // empty segment
          if (c != cur) break;
#pragma unroll
          for (int e = 0; e < E; ++e) {
            if (q0 * J + e < JJ) {
              const C d = side[(q0 * J + e) * NS + s2];
              ar[e] += d.x;
              ai[e] += d.y;
            }
          }
        }
        flush(cur, ar, ai);
      }
    }
    __syncthreads();
    // patch: cell q = c + (b, a) collects moment [a][b] of base cell c
    C* out = a.patches + item * static_cast<int64_t>(P) * P;
    const float invP = 1.0f / P;
    for (int pc = tid; pc < P * P; pc += kThreads) {
      const int pv = small_div(pc, P, invP), pu = pc - pv * P;
      R sr2 = 0, si2 = 0;
#pragma unroll
      for (int b = 0; b < J; ++b) {
        const int cv = pv - b;
        if (cv < 0 || cv >= T) continue;
#pragma unroll
        for (int q = 0; q < J; ++q) {
          const int cu = pu - q;
          if (cu < 0 || cu >= T) continue;
          const int c = cv * T + cu;
          if ((bits[c >> 5] >> (c & 31)) & 1u) {
            const C m = mom[(q * J + b) * TT + c];
            sr2 += m.x;
            si2 += m.y;
          }
        }
      }
      out[pc] = cmk<C>(sr2, si2);
    }
  }
}

// ---------------------------------------------------------------------------
// gridding, segment walk with chunked staging (J <= 4)
// ---------------------------------------------------------------------------
// LDS: kernel table (optional), moments [J*J][T*T] (entry-major), one region
// holding either a staged chunk (u, v and the weighted value of WC positions
// per thread, lane-transposed) or the side slots [J*J][kThreads], and the
// first/last base cell per thread. With the table in LDS the cell lists
// borrow the table's first 2 KB after the walk (the epilogue reads no taps)
// and that part of the table is reloaded before the next item's walk: this
// keeps a 16 x 16 tile with its table within half of the 160 KB.
// Positions per thread and staged chunk: FP32 8, FP64 4 (the prefetch
// registers hold one chunk).
template <typename R> struct WalkChunk { static constexpr int value = sizeof(R) == 4 ? 8 : 4; };
// Positions per segment fetched by one prefetch: two staged chunks, so that
// the 16-lane groups that load one segment read whole 128-byte lines of each
// visibility array (8-byte values in FP32: 16 positions; FP64: 8 positions of
// 16-byte values). Loading one chunk (half a line) at a time let the L2 evict
// a line between its two halves: the walk fetched 2.3 times its bytes.
// Only where the registers allow it (two waves per SIMD): FP32 stored-tap
// walks without section ids; the others prefetch one chunk at a time.
template <typename R, int MODE, int LK> struct WalkPrefetchLen {
  static constexpr int value = (sizeof(R) == 4 && LK == kLkWords && MODE != 3 ? 2 : 1) * WalkChunk<R>::value;
};
// Row pitch of the staged chunk, in entries: one more than the thread count,
// so the WC lanes that store the WC positions of one segment hit different
// banks (a pitch of exactly kThreads puts them on one bank).
constexpr int kStagePitch = kThreads + 1;

template <typename R, int J>
struct WalkLds {
  size_t tab, mom, stage, fcell, lcell, masks, total;
  int borrow;   // table entries under the cell lists (0: lists have their own space)
  __host__ __device__ WalkLds(int T, int tlen, bool tab_lds) {
    using C = cx_t<R>;
    constexpr int WC = WalkChunk<R>::value;
    const size_t lists = 2 * align16(static_cast<size_t>(kThreads) * sizeof(int));
    const size_t tab_bytes = tab_lds ? align16(static_cast<size_t>(tlen) * sizeof(R)) : 0;
    size_t o = 0;
    tab = o;   o += tab_bytes;
    mom = o;   o += align16(static_cast<size_t>(T) * T * J * J * sizeof(C));
    const size_t staged = align16(static_cast<size_t>(kStagePitch) * WC * 2 * sizeof(C));
    const size_t sides = align16(static_cast<size_t>(kThreads) * J * J * sizeof(C));
    stage = o; o += staged > sides ? staged : sides;
    if (tab_bytes >= lists) {
      fcell = tab;
      borrow = static_cast<int>(lists / sizeof(R));
    } else {
      fcell = o;
      o += lists;
      borrow = 0;
    }
    lcell = fcell + lists / 2;
    masks = o;  o += align16(static_cast<size_t>(2 * (kThreads / 64)) * sizeof(unsigned long long));
    total = o;
  }
};

// Registers holding two chunks' inputs between the loads and the LDS stores,
// so that the loads of the next pair of chunks (or of the next item's first
// pair) are in flight while a chunk is walked. Slot r of thread tid is
// position (tid mod PF) of segment tid / PF + r * kThreads / PF; the lanes
// with (tid mod PF) < WC stage the pair's first chunk, the others its second.
template <typename R, int MODE, int LK>
struct WalkPrefetch {
  using C = cx_t<R>;
  static constexpr int WC = WalkPrefetchLen<R, MODE, LK>::value;
  // one (u, v, w) triple per slot, loaded as one piece and consumed in place
  // (a separate w register makes the compiler copy it out of the load's
  // destination, which waits for the load while the next ones are issued)
  struct Uvw { R u, v, w; };
  Uvw uvw[WC];
  C val[WC];                      // MODE 0: y; MODE 1, 3: t = v + s - y
  C s[MODE != 0 ? WC : 1];        // MODE 1, 3: multiplier before the update
  int sec[MODE == 3 ? WC : 1];    // MODE 3 (local balls): section of the position
  unsigned ok;                    // bit r: slot r holds a position of the item
};

// Thread t owns the contiguous segment [t L, (t+1) L) of the item's
// cell-sorted visibilities, L = ceil(n / 256). The block stages the segments
// chunk by chunk (WC positions per thread, loaded with consecutive threads on
// consecutive visibilities, stored lane-transposed) and each thread walks its
// positions in order, computing taps in FP64 and holding the J^2 moments of
// its current run in registers across chunks. Moments start at zero; each
// base cell's moments are stored once per item, plus at most one earlier
// store of a continuation part (below). No value atomics.
//
// Runs and segments: because the item is cell-sorted, a run that crosses
// segment boundaries covers the end of its owner segment (where it begins),
// zero or more whole middle segments and possibly the start of a final
// segment where it ends. A run that ends inside the segment where it begins is
// stored as soon as it ends. The final segment stores its part (its first run)
// in the cell's moments as soon as that run ends; a middle segment parks its
// whole sum in its side slot after the walk; the owner then adds, in segment
// order, the side slots of the middle segments and the final part already in
// the moments, and stores the total.
// TS: the tile side when fixed at compile time (16 for the stored-tap plans:
// moment and patch offsets become immediates), else 0 (read from the args).
template <typename R, int J, int MODE, bool TAB_LDS, int LK, int TS, bool FUSED = false>
__global__ __launch_bounds__(kThreads) void grid_walk_kernel(GwAdjArgs<R> a) {
  using C = cx_t<R>;
  constexpr bool LIN = LK == kLkLinear, TW = LK == kLkWords;
  // MODE 0: plain gridding; 1: fused ADMM prologue (global ball); 3: the same
  // with each visibility's section ball (local balls; section ids prefetched)
  constexpr bool ADMM = MODE != 0, SEC = MODE == 3;
  const R scale = a.scale_dev ? static_cast<R>(*a.scale_dev) : a.scale;
  constexpr int JJ = J * J;
  constexpr int WC = WalkChunk<R>::value;
  constexpr int PF = WalkPrefetchLen<R, MODE, LK>::value;
  constexpr int kSegStride = kThreads / PF;
  extern __shared__ char smem_raw[];
  const WalkLds<R, J> lay(TS ? TS : a.T, a.tlen, TAB_LDS);
  C* mom = reinterpret_cast<C*>(smem_raw + lay.mom);
  // staged position: (u, v) and the weighted value side by side (one 16-byte
  // LDS access in FP32)
  struct Staged { C uv, val; };
  Staged* st = reinterpret_cast<Staged*>(smem_raw + lay.stage);
  C* side = reinterpret_cast<C*>(smem_raw + lay.stage);          // after the walk
  int* fcell = reinterpret_cast<int*>(smem_raw + lay.fcell);
  int* lcell = reinterpret_cast<int*>(smem_raw + lay.lcell);
  unsigned long long* nonmid = reinterpret_cast<unsigned long long*>(smem_raw + lay.masks);   // per wave
  unsigned long long* helpmask = nonmid + kThreads / 64;                                       // per wave
  const int tid = threadIdx.x;
  const R* tab = a.table;
  const int T = TS ? TS : a.T, P = TS ? TS + J - 1 : a.P;   // the same for every member of a fused launch
  // the arguments of the plan an item belongs to (as in the degridding)
  auto mem = [&](const int4& it) -> GwAdjArgs<R> {
    if constexpr (FUSED) {
      const GwAdjArgs<R>* t = a.mtab + item_member(it);
      GwAdjArgs<R> m = *t;
      m.uv = global_ptr_at(&t->uv);
      m.y_in = global_ptr_at(&t->y_in);
      m.patches = global_ptr_at(&t->patches);
      return m;
    } else {
      (void)it;
      return a;
    }
  };
  const int TT = T * T;
  R kappa_ball = 1;
  if (ADMM) kappa_ball = static_cast<R>(a.scalars[kSlotKappa]);
  const int lane_q = tid & (PF - 1);      // position within the pair this thread loads
  const int lane_t = tid / PF;            // first segment this thread loads for
  const int lane_h = lane_q / WC;         // the chunk of the pair this thread stages

  WalkPrefetch<R, MODE, LK> pf;
  // issue the loads of positions q0 .. q0 + PF - 1 of every segment of item it
  // Every slot loads (a slot past its segment reads the item's first
  // position, unused): no branches around the loads, so the loaded registers
  // are not moved and nothing waits for them before the commit.
  // Positions are addressed from the item's first visibility (a block-uniform
  // base) with 32-bit item-relative offsets (items hold fewer than 2^20).
  auto issue = [&](const int4& it, int L, int d, int q0) {
    pf.ok = 0u;
    const GwAdjArgs<R> m = mem(it);
    const int n = it.z - it.y;
    const int64_t b0 = it.y;
    const C* vi = (MODE == 0 ? m.y_in : m.t_in) + b0;
#pragma unroll
    for (int r = 0; r < PF; ++r) {
      const int q = q0 + lane_q;
      const int o = (lane_t + r * kSegStride) * L + q - d;
      const bool ok = q < L && o >= 0 && o < n;
      pf.ok |= static_cast<unsigned>(ok) << r;
      const uint32_t oc = ok ? static_cast<uint32_t>(o) : 0u;
      if constexpr (TW) {
        const uint2 w2 = *byte_at(reinterpret_cast<const uint2*>(m.uv) + b0, oc * 8u);
        pf.uvw[r].u = __uint_as_float(w2.x);
        pf.uvw[r].v = R(0);
        pf.uvw[r].w = __uint_as_float(w2.y);
      } else {
        vis_load<TW>(m.uv, b0 + oc, pf.uvw[r].u, pf.uvw[r].v, pf.uvw[r].w);
      }
      pf.val[r] = *byte_at(vi, oc * static_cast<uint32_t>(sizeof(C)));
      if (ADMM) pf.s[ADMM ? r : 0] = *byte_at(m.s_io + b0, oc * static_cast<uint32_t>(sizeof(C)));
      if (SEC) pf.sec[SEC ? r : 0] = m.sec[b0 + oc];
    }
  };
  // store chunk h of the prefetched pair (positions q0 + h WC ..) lane-
  // transposed (ADMM prologue applied here). The values are formed for every
  // slot and only the stores are predicated, so every prefetched register is
  // consumed on every path (no conservative waits on them later).
  auto commit = [&](const int4& it, int L, int d, int q0, int h) {
    const GwAdjArgs<R> m = mem(it);
    const R iscale = FUSED ? m.scale : scale;
#pragma unroll
    for (int r = 0; r < PF; ++r) {
      const bool ok = ((pf.ok >> r) & 1u) && lane_h == h;
      C val;
      C sn = cmk<C>(R(0), R(0));
      if (MODE == 0) {
        val = pf.val[r];
      } else {
        // ball projection and multiplier update of Algorithm 1 from t = v + s - y:
        // r = y + kappa t, s' = s + varrho (v - r), q = vr_coef (v - r) + s'
        const C tt = pf.val[r], sk = pf.s[ADMM ? r : 0];
        const R omk = R(1) - (SEC ? static_cast<R>(a.kappa_sec[pf.sec[SEC ? r : 0]]) : kappa_ball);
        const C vr = cmk<C>(omk * tt.x - sk.x, omk * tt.y - sk.y);   // v - r
        sn = cmk<C>(sk.x + a.varrho * vr.x, sk.y + a.varrho * vr.y);
        val = cmk<C>(a.vr_coef * vr.x + sn.x, a.vr_coef * vr.y + sn.y);
      }
      const R ws = pf.uvw[r].w * iscale;
      const C uvr = cmk<C>(pf.uvw[r].u, pf.uvw[r].v);
      const C wv = cmk<C>(val.x * ws, val.y * ws);
      if (ok) {
        if (ADMM) {
          const uint32_t o = static_cast<uint32_t>((lane_t + r * kSegStride) * L + q0 + lane_q - d);
          *byte_at(m.s_io + static_cast<int64_t>(it.y), o * static_cast<uint32_t>(sizeof(C))) = sn;
        }
        const int slot = (lane_q - h * WC) * kStagePitch + lane_t + r * kSegStride;
        st[slot] = Staged{uvr, wv};
      }
    }
    // every prefetched load has landed (the values above needed them): say so
    // explicitly (vmcnt(0), other counters untouched), so the compiler does
    // not keep them pending across the predicated stores and stall the next
    // prefetch on its own registers
    __builtin_amdgcn_s_waitcnt(0x0F70);
  };
  // Segments of an item: thread t owns frame positions [t L, (t + 1) L), frame
  // position f being item position f - d. With d = 0 and L = ceil(n / 256)
  // a prefetch of PF positions per segment starts anywhere in a 128-byte line;
  // when an item needs two prefetches per segment, the two halves of a line
  // would be read by different prefetches and the line fetched twice. So, for
  // the 8-byte-per-array walks (PF values of 8 bytes fill one line), long
  // items use a frame aligned to the line (d = first position mod PF) and a
  // multiple of PF for L: every prefetch then reads whole lines.
  constexpr bool LINE_FRAME = TW && PF * sizeof(C) == 128;
  auto seg_len = [](const int4& it) {
    const int n = it.z - it.y;
    if (LINE_FRAME && n > PF * (kThreads - 1)) {
      const int d = it.y & (PF - 1);
      return PF * ((n + d + PF * kThreads - 1) / (PF * kThreads));
    }
    return (n + kThreads - 1) / kThreads;
  };
  auto seg_shift = [](const int4& it) {
    const int n = it.z - it.y;
    return LINE_FRAME && n > PF * (kThreads - 1) ? it.y & (PF - 1) : 0;
  };

  const int kbeg = a.sched_off[blockIdx.x], kend = a.sched_off[blockIdx.x + 1];
  int4 it = make_int4(0, 0, 0, 0);
  int L = 0, d = 0;
  if (kbeg < kend) {
    it = a.items[kbeg];
    L = seg_len(it);
    d = seg_shift(it);
    issue(it, L, d, 0);
  }
  // the table copy overlaps the first chunk's loads
  if (TAB_LDS) {
    R* t = reinterpret_cast<R*>(smem_raw + lay.tab);
    for (int i = tid; i < a.tlen; i += kThreads) t[i] = a.table[i];
    tab = t;
  }
  for (int ks = kbeg; ks < kend; ++ks) {
    const int64_t item = it.w;
    const bool has_next = ks + 1 < kend;
    const int4 itn = has_next ? a.items[ks + 1] : make_int4(0, 0, 0, 0);
    const int Ln = seg_len(itn), dn = seg_shift(itn);
    const GwAdjArgs<R> mi = mem(it);
    const int K = mi.K;
    const int tile = item_tile(it);
    const int tv = tile >> mi.lognT, tu = tile & (mi.nT - 1);
    // this thread's frame positions [sb, segn) (only thread 0 skips the shift)
    const int segn = max(0, min(L, d + (it.z - it.y) - tid * L));
    const int sb = tid == 0 ? d : 0;
    __syncthreads();   // the previous item is done with the moments, side slots and cell lists
    for (int i = tid; i < TT * JJ; i += kThreads) mom[i] = cmk<C>(R(0), R(0));
    if (TAB_LDS && lay.borrow) {
      // restore the table head the cell lists borrowed (its loads complete
      // with the first chunk's, which the commit below waits for anyway)
      R* t = reinterpret_cast<R*>(smem_raw + lay.tab);
      for (int i = tid; i < lay.borrow; i += kThreads) t[i] = a.table[i];
    }

    // the item's first pair was prefetched during the previous item's last
    // pair (or before the loop)
    commit(it, L, d, 0, 0);

    C acc[JJ];
    int first = -1, cur = -1, nruns = 0;
#pragma unroll
    for (int e = 0; e < JJ; ++e) acc[e] = zero_cx<C>();
    // walk the staged chunk at positions q0 .. q0 + WC - 1 of this thread's segment
    auto walk = [&](int q0) {
      const int qn = min(WC, segn - q0);
      for (int i = max(0, sb - q0); i < qn; ++i) {
        const Staged sp = st[i * kStagePitch + tid];
        C val = sp.val;
        AxisTaps xu, xv;
        int lu, lv;
        vis_taps<TW>(sp.uv.x, sp.uv.y, mi.kappa, J, a.D, K, T, tu, tv, xu, xv, lu, lv);
        if (static_cast<unsigned>(lu) >= static_cast<unsigned>(T) || static_cast<unsigned>(lv) >= static_cast<unsigned>(T)) {
          // cannot happen for a plan's own sorted baselines: keep LDS indices in range, poison the value
          lu = lv = 0;
          val = cmk<C>(R(NAN), R(NAN));
        }
        const int c = lv * T + lu;
        if (c != cur) {
          if (nruns > 0) {
            // the run on cur ended inside this segment: its sum is final
            // unless it is the segment's first run and continues the previous
            // segment, in which case the owner adds it later
#pragma unroll
            for (int e = 0; e < JJ; ++e) mom[e * TT + cur] = acc[e];
          } else {
            first = c;
          }
          cur = c;
          ++nruns;
#pragma unroll
          for (int e = 0; e < JJ; ++e) acc[e] = zero_cx<C>();
        }
        R wv[J], wu[J];
        axis_weights<LIN, J>(tab, xv, a.D, a.tlen, wv);
        axis_weights<LIN, J>(tab, xu, a.D, a.tlen, wu);
#pragma unroll
        for (int qq = 0; qq < J; ++qq) {
          const R g = wu[qq];
          const R yr = val.x * g, yi = val.y * g;
#pragma unroll
          for (int b = 0; b < J; ++b) {
            acc[qq * J + b].x += wv[b] * yr;
            acc[qq * J + b].y += wv[b] * yi;
          }
        }
      }
    };
    // Pairs of chunks: the pair's first chunk is staged; walk it, stage its
    // second chunk from the registers, then prefetch the next pair (of this
    // item, else the next item's first pair; with nothing left the slots
    // reload this item's first positions, unused) while the second chunk is
    // walked, and stage the next pair's first chunk. One prefetch call site,
    // reached once per pair.
    for (int p0 = 0; p0 < L; p0 += PF) {
      const bool second = PF > WC && p0 + WC < L;   // the pair has a second chunk
      const bool next = p0 + PF < L;           // this item has another pair
      __syncthreads();   // the first chunk is staged
      walk(p0);
      if (second) {
        __syncthreads();   // the first chunk has been walked
        commit(it, L, d, p0, 1);
      }
      issue(next || !has_next ? it : itn, next || !has_next ? L : Ln, next || !has_next ? d : dn, next ? p0 + PF : 0);
      if (second) {
        __syncthreads();   // the second chunk is staged
        walk(p0 + WC);
      }
      if (next) {
        __syncthreads();   // the second chunk has been walked
        commit(it, L, d, p0 + PF, 0);
      }
    }
    if (TAB_LDS && lay.borrow) __syncthreads();   // every walk done with the table head
    fcell[tid] = first;
    lcell[tid] = cur;
    __syncthreads();   // staging consumed; first and last cells published
    // the last run (in registers) continues the previous segment only if the
    // whole segment is one run: a middle segment, parked for its owner
    const bool middle = nruns == 1 && tid > 0 && lcell[tid - 1] == first;
    if (middle) {
#pragma unroll
      for (int e = 0; e < JJ; ++e) side[e * kThreads + tid] = acc[e];
    }
    {
      const unsigned long long bal = __ballot(!middle);
      if ((tid & 63) == 0) nonmid[tid >> 6] = bal;
    }
    __syncthreads();   // side slots and the non-middle masks written
    // A run over several segments: its owner (a non-middle segment whose last
    // run it is) and the middle segments [owner + 1, jend), jend the next
    // segment that is not a middle one; a final segment, if any, has already
    // stored its part in the moments of cur. Owner and middles find both ends
    // from the per-wave masks in constant time.
    const bool owner = nruns > 0 && !middle;
    const int wv_ = tid >> 6, lane = tid & 63;
    int base = tid, jend = tid + 1;
    if (owner || middle) {
      unsigned long long m = lane == 63 ? 0ull : (nonmid[wv_] & (~0ull << (lane + 1)));
      int ww = wv_;
      while (m == 0ull && ww + 1 < kThreads / 64) m = nonmid[++ww];
      jend = m ? ww * 64 + __builtin_ctzll(m) : kThreads;
    }
    if (middle) {
      // thread 0 is never a middle, so a non-middle segment below exists
      unsigned long long m = nonmid[wv_] & ((1ull << lane) - 1ull);
      int ww = wv_;
      while (m == 0ull && ww > 0) m = nonmid[--ww];
      base = ww * 64 + 63 - __builtin_clzll(m);
    }
    // Long runs (at least JJ middles): the middles themselves sum the parked
    // moments in two fixed-order levels. The nm middles split into
    // G = nm / JJ contiguous groups; middle k takes moment k mod JJ of group
    // k / JJ and leaves the group's sum in the group's first slot; then middle
    // e (< JJ) adds the G group sums of moment e in order into the first
    // middle's slot, which the owner reads.
    const int nm = jend - base - 1;
    const bool helped = owner && nm >= JJ;
    const bool helping = middle && nm >= JJ;
    {
      const unsigned long long bal = __ballot(helped);
      if ((tid & 63) == 0) helpmask[tid >> 6] = bal;
    }
    __syncthreads();   // the per-wave flags written
    unsigned long long anyhelp = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) anyhelp |= helpmask[w];
    if (anyhelp) {
      const int k = tid - base - 1, G = nm / JJ;
      if (helping && k / JJ < G) {
        const int e = k % JJ, g = k / JJ;
        const int lo = base + 1 + (g * nm) / G, hi = base + 1 + ((g + 1) * nm) / G;
        R sr = 0, si = 0;
        for (int j = lo; j < hi; ++j) {
          const C d = side[e * kThreads + j];
          sr += d.x;
          si += d.y;
        }
        side[e * kThreads + lo] = cmk<C>(sr, si);
      }
      __syncthreads();   // every group sum written
      if (helping && k < JJ) {
        R sr = 0, si = 0;
        for (int g = 0; g < G; ++g) {
          const C d = side[k * kThreads + base + 1 + (g * nm) / G];
          sr += d.x;
          si += d.y;
        }
        side[k * kThreads + base + 1] = cmk<C>(sr, si);
      }
      __syncthreads();   // the run totals are in the first middle slot of each run
    }
    if (owner) {
      if (helped) {
#pragma unroll
        for (int e = 0; e < JJ; ++e) {
          const C d = side[e * kThreads + tid + 1];
          acc[e].x += d.x;
          acc[e].y += d.y;
        }
      } else {
        for (int j = tid + 1; j < jend; ++j) {
#pragma unroll
          for (int e = 0; e < JJ; ++e) {
            const C d = side[e * kThreads + j];
            acc[e].x += d.x;
            acc[e].y += d.y;
          }
        }
      }
#pragma unroll
      for (int e = 0; e < JJ; ++e) {
        C* m = &mom[e * TT + cur];
        const C fin = *m;                // final segment's part, or zero
        *m = cmk<C>(acc[e].x + fin.x, acc[e].y + fin.y);
      }
    }
    __syncthreads();
    // patch: cell q = c + (b, a) collects moment [a][b] of base cell c
    C* out = mi.patches + item * static_cast<int64_t>(P) * P;
    const float invP = 1.0f / P;
    for (int pc = tid; pc < P * P; pc += kThreads) {
      const int pv = small_div(pc, P, invP), pu = pc - pv * P;
      // every load in range (clamped), out-of-tile base cells masked: the
      // J^2 loads issue together
      C m[JJ];
#pragma unroll
      for (int b = 0; b < J; ++b) {
        const int cv = min(max(pv - b, 0), T - 1);
#pragma unroll
        for (int qq = 0; qq < J; ++qq) {
          const int cu = min(max(pu - qq, 0), T - 1);
          m[b * J + qq] = mom[(qq * J + b) * TT + cv * T + cu];
        }
      }
      R sr2 = 0, si2 = 0;
#pragma unroll
      for (int b = 0; b < J; ++b) {
        const bool okv = static_cast<unsigned>(pv - b) < static_cast<unsigned>(T);
#pragma unroll
        for (int qq = 0; qq < J; ++qq) {
          const bool ok = okv && static_cast<unsigned>(pu - qq) < static_cast<unsigned>(T);
          sr2 += ok ? m[b * J + qq].x : R(0);
          si2 += ok ? m[b * J + qq].y : R(0);
        }
      }
      out[pc] = cmk<C>(sr2, si2);
    }
    it = itn;
    L = Ln;
    d = dn;
  }
}

// Gridding of the small items (at most kSmallItem visibilities), one wave
// per item: lane l takes visibility l of the item (with the ADMM prologue of
// the walk in MODE 1 / 3), evaluates its base cell and J + J weights once
// into LDS, then each lane forms patch cells l, l + 64, ... directly as the
// sum, in visibility order, of w_v (q w_u) over the visibilities whose
// footprint covers the cell. No runs and no moments: for a handful of
// visibilities the walk's per-item steps (clearing, segment carries, block
// barriers, the wait for the next item's loads) cost far more than the
// arithmetic. The weights read the table through the caches (a block would
// otherwise copy the whole table to LDS for a few hundred lookups); the four
// waves of a block take their next items together, so the block barriers
// stay uniform.
template <typename R, int J, int MODE, int LK, bool FUSED = false>
__global__ __launch_bounds__(kThreads) void grid_small_kernel(GwAdjArgs<R> a, const int4* __restrict__ small,
                                                              int nsmall) {
  using C = cx_t<R>;
  constexpr bool LIN = LK == kLkLinear, TW = LK == kLkWords;
  constexpr bool ADMM = MODE != 0, SEC = MODE == 3;
  constexpr int kWaves = kThreads / 64;
  struct Entry {
    int lu, lv;
    R wu[J], wv[J];
    C val;
  };
  extern __shared__ char smem_raw[];
  const R* tab = a.table;   // read through the caches: each visibility's weights once
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  Entry* ent = reinterpret_cast<Entry*>(smem_raw) + wave * 64;
  const R scale = a.scale_dev ? static_cast<R>(*a.scale_dev) : a.scale;
  R kappa_ball = 1;
  if (ADMM) kappa_ball = static_cast<R>(a.scalars[kSlotKappa]);
  const int T = a.T, P = a.P;   // the same for every member of a fused launch
  auto mem = [&](const int4& it) -> GwAdjArgs<R> {
    if constexpr (FUSED) {
      const GwAdjArgs<R>* t = a.mtab + item_member(it);
      GwAdjArgs<R> m = *t;
      m.uv = global_ptr_at(&t->uv);
      m.y_in = global_ptr_at(&t->y_in);
      m.patches = global_ptr_at(&t->patches);
      return m;
    } else {
      (void)it;
      return a;
    }
  };
  const int step = kWaves * static_cast<int>(gridDim.x);
  const int rounds = (nsmall + step - 1) / step;
  for (int rd = 0; rd < rounds; ++rd) {
    const int idx = rd * step + static_cast<int>(blockIdx.x) * kWaves + wave;
    const bool have = idx < nsmall;
    const int4 it = have ? small[idx] : make_int4(0, 0, 0, 0);
    const int n = it.z - it.y;
    const GwAdjArgs<R> m = mem(it);
    __syncthreads();   // the table is in LDS; the previous round is done with the entries
    if (have && lane < n) {
      const int64_t k = static_cast<int64_t>(it.y) + lane;
      R u, v, w;
      if constexpr (TW) {
        const uint2 w2 = reinterpret_cast<const uint2*>(m.uv)[k];
        u = __uint_as_float(w2.x);
        v = R(0);
        w = __uint_as_float(w2.y);
      } else {
        vis_load<TW>(m.uv, k, u, v, w);
      }
      C val;
      if constexpr (MODE == 0) {
        val = m.y_in[k];
      } else {
        // ball projection and multiplier update of Algorithm 1, as in the walk
        const C tt = m.t_in[k], sk = m.s_io[k];
        const R omk = R(1) - (SEC ? static_cast<R>(a.kappa_sec[m.sec[k]]) : kappa_ball);
        const C vr = cmk<C>(omk * tt.x - sk.x, omk * tt.y - sk.y);
        const C sn = cmk<C>(sk.x + a.varrho * vr.x, sk.y + a.varrho * vr.y);
        m.s_io[k] = sn;
        val = cmk<C>(a.vr_coef * vr.x + sn.x, a.vr_coef * vr.y + sn.y);
      }
      const R ws = w * (FUSED ? m.scale : scale);
      Entry e;
      e.val = cmk<C>(val.x * ws, val.y * ws);
      const int tile = item_tile(it);
      const int tv = tile >> m.lognT, tu = tile & (m.nT - 1);
      AxisTaps xu, xv;
      int lu, lv;
      vis_taps<TW>(u, v, m.kappa, J, a.D, m.K, T, tu, tv, xu, xv, lu, lv);
      if (static_cast<unsigned>(lu) >= static_cast<unsigned>(T) || static_cast<unsigned>(lv) >= static_cast<unsigned>(T)) {
        // cannot happen for a plan's own sorted baselines: poison the value
        lu = lv = 0;
        e.val = cmk<C>(R(NAN), R(NAN));
      }
      e.lu = lu;
      e.lv = lv;
      axis_weights<LIN, J>(tab, xu, a.D, a.tlen, e.wu);
      axis_weights<LIN, J>(tab, xv, a.D, a.tlen, e.wv);
      ent[lane] = e;
    }
    __syncthreads();   // the entries are written
    if (have) {
      C* out = m.patches + static_cast<int64_t>(it.w) * P * P;
      const float invP = 1.0f / P;
      for (int pc = lane; pc < P * P; pc += 64) {
        const int pv = small_div(pc, P, invP), pu = pc - pv * P;
        R sr = 0, si = 0;
        for (int q = 0; q < n; ++q) {
          const int du = pu - ent[q].lu, dv = pv - ent[q].lv;
          if (static_cast<unsigned>(du) < static_cast<unsigned>(J) && static_cast<unsigned>(dv) < static_cast<unsigned>(J)) {
            const R g = ent[q].wu[du], gv = ent[q].wv[dv];
            const C y = ent[q].val;
            sr += gv * (y.x * g);
            si += gv * (y.y * g);
          }
        }
        out[pc] = cmk<C>(sr, si);
      }
    }
  }
}

template <typename R, int J>
size_t small_lds_bytes() {
  struct EntrySize { int lu, lv; R wu[J], wv[J]; cx_t<R> val; };
  return static_cast<size_t>(kThreads) * sizeof(EntrySize);
}

// Columns of the moments held per gridding thread (JA): all of them for
// J <= 2, else two (2 J complex accumulators plus their parked copies). Three
// columns at J = 6 took about 300 registers in FP32, one wave per SIMD, and
// gridded at half the rate of two columns with a quarter of the threads idle
// in the walk (J / 2 = 3 threads per segment, rounded up to 4).
template <typename R, int J> struct GridSplit { static constexpr int JA = J <= 2 ? J : 2; };

// Grid cell = sum of the patches of the (up to four) tiles whose patch covers
// it, neighbour tiles first, items of a tile in order. One block per output
// tile, so the item ranges it walks are the same for all its threads.
// One plan of a fused merge: block b of the launch is tile b - tile0 of the
// member whose range [tile0, next member's tile0) holds b.
template <typename R>
struct MergeArgs {
  const cx_t<R>* patches;
  const int32_t* item_off;
  cx_t<R>* grid;
  int K, nT, tile0, pad;
};

template <typename R, bool FUSED = false>
__global__ void merge_patches_kernel(const cx_t<R>* __restrict__ patches, const int32_t* __restrict__ item_off,
                                     cx_t<R>* __restrict__ grid, int K, int T, int P, int nT, int J,
                                     const MergeArgs<R>* __restrict__ mtab, int nmembers) {
  using C = cx_t<R>;
  int t = blockIdx.x;
  if constexpr (FUSED) {
    // the member holding this block (binary search over the tile offsets)
    int lo = 0, hi = nmembers - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (mtab[mid].tile0 <= t) lo = mid; else hi = mid - 1;
    }
    const MergeArgs<R> m = mtab[lo];
    patches = global_ptr_at(&mtab[lo].patches);
    item_off = global_ptr_at(&mtab[lo].item_off);
    grid = global_ptr_at(&mtab[lo].grid);
    K = m.K;
    nT = m.nT;
    t -= m.tile0;
  }
  const int tv = t / nT, tu = t - tv * nT;
  const int64_t P2 = static_cast<int64_t>(P) * P;
  for (int c = threadIdx.x; c < T * T; c += blockDim.x) {
    const int lv = c / T, lu = c & (T - 1);
    R sr = 0, si = 0;
    for (int dv = 1; dv >= 0; --dv) {
      if (dv == 1 && lv >= J - 1) continue;
      const int tvv = tv - dv < 0 ? tv - dv + nT : tv - dv;
      const int pv = lv + dv * T;
      for (int du = 1; du >= 0; --du) {
        if (du == 1 && lu >= J - 1) continue;
        const int tuu = tu - du < 0 ? tu - du + nT : tu - du;
        const int pu = lu + du * T;
        const int src = tvv * nT + tuu;
        const int i0 = item_off[src], i1 = item_off[src + 1];
        const C* col = patches + pv * P + pu;
        int itm = i0;
        // eight loads in flight, summed in item order
        for (; itm + 8 <= i1; itm += 8) {
          C v[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) v[k] = col[(itm + k) * P2];
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            sr += v[k].x;
            si += v[k].y;
          }
        }
        for (; itm < i1; ++itm) {
          const C v = col[itm * P2];
          sr += v.x;
          si += v.y;
        }
      }
    }
    grid[static_cast<int64_t>(tv * T + lv) * K + tu * T + lu] = cmk<C>(sr, si);
  }
}

// Sum the ADMM degridding partials in a fixed order and form the ball scale.
__global__ void ball_scale_kernel(const double* partials, int nblocks, double eps, double kappa_fixed,
                                  double* scalars) {
  __shared__ double sh[kThreads];
  double t2 = 0, r2 = 0;
  for (int i = threadIdx.x; i < nblocks; i += kThreads) {
    t2 += partials[kSlotT2 * kPartialsMax + i];
    r2 += partials[kSlotR2 * kPartialsMax + i];
  }
  t2 = block_sum_f64(t2, sh);
  r2 = block_sum_f64(r2, sh);
  if (threadIdx.x == 0) {
    const double nt = sqrt(t2);
    scalars[kSlotT2] = t2;
    scalars[kSlotR2] = r2;
    scalars[kSlotKappa] = kappa_fixed >= 0.0 ? kappa_fixed : (nt <= eps ? 1.0 : eps / nt);
    if (!isfinite(t2) || !isfinite(r2)) scalars[kSlotNonfinite] = 1.0;
  }
}

// Local balls: block j sums section j's degridding partials in a fixed order
// (strided per thread, then a tree) and forms ||t_j||^2 and kappa_j.
__global__ void section_kappa_partials_kernel(const double* partials, int nblocks, const double* eps,
                                              double* kappa, double* norm2) {
  __shared__ double sh[kThreads];
  const int j = blockIdx.x;
  double s2 = 0;
  for (int i = threadIdx.x; i < nblocks; i += kThreads) s2 += partials[(kSlotSec0 + j) * kPartialsMax + i];
  s2 = block_sum_f64(s2, sh);
  if (threadIdx.x == 0) {
    norm2[j] = s2;
    const double nt = sqrt(s2);
    kappa[j] = nt <= eps[j] ? 1.0 : eps[j] / nt;
  }
}

// Degridding blocks: with small items every block also takes some after its
// scheduled items (their offsets run to kDegridBlocks).
int degrid_blocks(const pr_phi_plan_t* p) {
  if (p->nSmall > 0) return kDegridBlocks;
  return static_cast<int>(p->nItems < kDegridBlocks ? p->nItems : kDegridBlocks);
}

int grid_blocks(const pr_phi_plan_t* p) {
  return static_cast<int>(p->nGrid < kGridBlocks ? p->nGrid : kGridBlocks);
}

// Raise a kernel's dynamic LDS limit to the full 160 KB, once per kernel and
// device, so that launches (also under stream capture) set no attributes.
template <typename K>
int allow_lds(K kernel, size_t bytes) {
  if (bytes <= 65536) return PR_OK;
  static std::mutex mu;
  static std::set<std::pair<int, const void*>> done;
  int dev = 0;
  PR_TRY_HIP(hipGetDevice(&dev));
  const void* f = reinterpret_cast<const void*>(kernel);
  std::lock_guard<std::mutex> lock(mu);
  if (done.count({dev, f})) return PR_OK;
  PR_TRY_HIP(hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(kLdsHard)));
  done.insert({dev, f});
  return PR_OK;
}

template <typename R, int J, int MODE, int LK, bool FUSED = false>
int launch_degrid(pr_phi_plan_t* p, GwArgs<R> a, hipStream_t s, int G = 0) {
  using C = cx_t<R>;
  const size_t patch = align16(static_cast<size_t>(p->P) * p->P * sizeof(C));
  const size_t tabb = static_cast<size_t>(a.tlen) * sizeof(R);
  size_t lds = patch;
  if (MODE >= 1 && lds < kThreads * sizeof(double)) lds = kThreads * sizeof(double);
  if (G <= 0) G = degrid_blocks(p);
  if (lds + tabb <= kLdsSoft) {
    degrid_kernel<R, J, MODE, true, LK, FUSED><<<G, kThreads, lds + tabb, s>>>(a);
  } else if (lds <= kLdsHard) {
    PR_TRY(allow_lds(degrid_kernel<R, J, MODE, false, LK, FUSED>, lds));
    degrid_kernel<R, J, MODE, false, LK, FUSED><<<G, kThreads, lds, s>>>(a);
  } else {
    set_error("degridding patch of tile %d does not fit in LDS", p->T);
    return PR_EUNSUPPORTED;
  }
  PR_TRY_LAUNCH();
  return PR_OK;
}

// Staging depth B and table placement: fit two blocks per CU if possible,
// else use up to the whole 160 KB.
template <typename R, int J>
bool pick_grid_lds(int T, int tlen, int* B, bool* tab_lds, size_t* bytes) {
  constexpr int JA = GridSplit<R, J>::JA;
  constexpr int TPC = (J + JA - 1) / JA;
  constexpr int NS = kThreads / (TPC == 3 ? 4 : TPC);
  const size_t limits[2] = {kLdsSoft, kLdsHard};
  for (size_t lim : limits) {
    for (int tl = 1; tl >= 0; --tl) {
      for (int b = kThreads * kGridPer; b >= 64; b /= 2) {
        GridLds<R, J, NS> g(T, b, tlen, tl != 0);
        if (g.total <= lim) {
          *B = b;
          *tab_lds = tl != 0;
          *bytes = g.total;
          return true;
        }
      }
    }
  }
  return false;
}

// Segment walk (J <= 4): table in LDS if that keeps two blocks per CU, or if
// one block per CU is all that fits either way. Returns false if it does not
// fit in LDS at all (the caller then uses the J-lane kernel).
template <typename R, int J, int WMODE, int LK, bool FUSED = false>
int launch_walk(pr_phi_plan_t* p, GwAdjArgs<R>& a, hipStream_t s, int G, bool* walked) {
  const WalkLds<R, J> with(a.T, a.tlen, true), without(a.T, a.tlen, false);
  const bool tl = with.total <= kLdsSoft || (without.total > kLdsSoft && with.total <= kLdsHard);
  const size_t bytes = tl ? with.total : without.total;
  *walked = false;
  if (bytes > kLdsHard) return PR_OK;
  if (G == 0) {   // every item is a small one
    *walked = true;
    return PR_OK;
  }
  if (LK == kLkWords && a.T == 16) {
    if (tl) {
      PR_TRY(allow_lds(grid_walk_kernel<R, J, WMODE, true, LK, 16, FUSED>, bytes));
      grid_walk_kernel<R, J, WMODE, true, LK, 16, FUSED><<<G, kThreads, bytes, s>>>(a);
    } else {
      PR_TRY(allow_lds(grid_walk_kernel<R, J, WMODE, false, LK, 16, FUSED>, bytes));
      grid_walk_kernel<R, J, WMODE, false, LK, 16, FUSED><<<G, kThreads, bytes, s>>>(a);
    }
  } else if (tl) {
    PR_TRY(allow_lds(grid_walk_kernel<R, J, WMODE, true, LK, 0, FUSED>, bytes));
    grid_walk_kernel<R, J, WMODE, true, LK, 0, FUSED><<<G, kThreads, bytes, s>>>(a);
  } else {
    PR_TRY(allow_lds(grid_walk_kernel<R, J, WMODE, false, LK, 0, FUSED>, bytes));
    grid_walk_kernel<R, J, WMODE, false, LK, 0, FUSED><<<G, kThreads, bytes, s>>>(a);
  }
  *walked = true;
  return PR_OK;
}

// The small items of a walk plan (none: no launch).
template <typename R, int J, int WMODE, int LK, bool FUSED = false>
int launch_small(const GwAdjArgs<R>& a, const int4* small, int64_t nsmall, hipStream_t s) {
  if (nsmall <= 0) return PR_OK;
  const size_t bytes = small_lds_bytes<R, J>();
  const int64_t blocks = (nsmall + kThreads / 64 - 1) / (kThreads / 64);
  const int G = static_cast<int>(blocks < kDegridBlocks ? blocks : kDegridBlocks);
  PR_TRY(allow_lds(grid_small_kernel<R, J, WMODE, LK, FUSED>, bytes));
  grid_small_kernel<R, J, WMODE, LK, FUSED><<<G, kThreads, bytes, s>>>(a, small, static_cast<int>(nsmall));
  PR_TRY_LAUNCH();
  return PR_OK;
}

template <typename R, int J, int MODE, int LK>
int launch_grid(pr_phi_plan_t* p, GwAdjArgs<R> a, hipStream_t s, int parts = 3) {
  using C = cx_t<R>;
  constexpr int JA = GridSplit<R, J>::JA;
  const int G = grid_blocks(p);
  bool walked = false;
  if (!(parts & 1)) walked = true;   // patches not asked for
  if constexpr (J <= 4) {
    if (parts & 1) {
      // the ADMM prologue with section balls is its own walk instance (MODE 3)
      if (MODE == 1 && a.sec) {
        PR_TRY((launch_walk<R, J, MODE == 1 ? 3 : MODE, LK>(p, a, s, G, &walked)));
        if (walked) PR_TRY((launch_small<R, J, MODE == 1 ? 3 : MODE, LK>(a, p->small, p->nSmall, s)));
      } else {
        PR_TRY((launch_walk<R, J, MODE, LK>(p, a, s, G, &walked)));
        if (walked) PR_TRY((launch_small<R, J, MODE, LK>(a, p->small, p->nSmall, s)));
      }
    }
  }
  if (!walked) {
    int B;
    bool tab_lds;
    size_t bytes;
    if (!pick_grid_lds<R, J>(a.T, a.tlen, &B, &tab_lds, &bytes)) {
      set_error("gridding tile %d with J=%d does not fit in LDS", a.T, J);
      return PR_EUNSUPPORTED;
    }
    a.B = B;
    if (G > 0) {
      if (tab_lds) {
        PR_TRY(allow_lds(grid_kernel<R, J, JA, MODE, true, LK>, bytes));
        grid_kernel<R, J, JA, MODE, true, LK><<<G, kThreads, bytes, s>>>(a);
      } else {
        PR_TRY(allow_lds(grid_kernel<R, J, JA, MODE, false, LK>, bytes));
        grid_kernel<R, J, JA, MODE, false, LK><<<G, kThreads, bytes, s>>>(a);
      }
    }
    if (MODE == 1 && a.sec) PR_TRY((launch_small<R, J, MODE == 1 ? 3 : MODE, LK>(a, p->small, p->nSmall, s)));
    else PR_TRY((launch_small<R, J, MODE, LK>(a, p->small, p->nSmall, s)));
  }
  PR_TRY_LAUNCH();
  if (parts & 2) {
    merge_patches_kernel<R><<<p->nTiles, p->T * p->T < kThreads ? p->T * p->T : kThreads, 0, s>>>(
        static_cast<const C*>(p->patches), p->item_off, static_cast<C*>(p->grid), p->K, p->T, p->P, p->nT, p->J,
        nullptr, 0);
    PR_TRY_LAUNCH();
  }
  return PR_OK;
}

template <typename R, int J, int MODE, int LK>
int setup_mode() {
  constexpr int JA = GridSplit<R, J>::JA;
  PR_TRY((allow_lds(degrid_kernel<R, J, MODE, true, LK>, kLdsHard)));
  PR_TRY((allow_lds(degrid_kernel<R, J, MODE, false, LK>, kLdsHard)));
  if constexpr (J <= 4) {
    constexpr int WM[2] = {MODE, MODE == 1 ? 3 : MODE};
    PR_TRY((allow_lds(grid_walk_kernel<R, J, WM[0], true, LK, 0>, kLdsHard)));
    PR_TRY((allow_lds(grid_walk_kernel<R, J, WM[0], false, LK, 0>, kLdsHard)));
    PR_TRY((allow_lds(grid_walk_kernel<R, J, WM[1], true, LK, 0>, kLdsHard)));
    PR_TRY((allow_lds(grid_walk_kernel<R, J, WM[1], false, LK, 0>, kLdsHard)));
    if constexpr (LK == kLkWords) {
      PR_TRY((allow_lds(grid_walk_kernel<R, J, WM[0], true, LK, 16>, kLdsHard)));
      PR_TRY((allow_lds(grid_walk_kernel<R, J, WM[0], false, LK, 16>, kLdsHard)));
      PR_TRY((allow_lds(grid_walk_kernel<R, J, WM[1], true, LK, 16>, kLdsHard)));
      PR_TRY((allow_lds(grid_walk_kernel<R, J, WM[1], false, LK, 16>, kLdsHard)));
    }
  }
  PR_TRY((allow_lds(grid_small_kernel<R, J, MODE, LK>, kLdsHard)));
  PR_TRY((allow_lds(grid_small_kernel<R, J, MODE == 1 ? 3 : MODE, LK>, kLdsHard)));
  PR_TRY((allow_lds(grid_kernel<R, J, JA, MODE, true, LK>, kLdsHard)));
  PR_TRY((allow_lds(grid_kernel<R, J, JA, MODE, false, LK>, kLdsHard)));
  return PR_OK;
}

template <typename R, int J, int LK>
int setup_kernels() {
  PR_TRY((allow_lds(degrid_kernel<R, J, 2, true, LK>, kLdsHard)));
  PR_TRY((allow_lds(degrid_kernel<R, J, 2, false, LK>, kLdsHard)));
  PR_TRY((setup_mode<R, J, 0, LK>()));
  return setup_mode<R, J, 1, LK>();
}

// Compile-time dispatch on the kernel width and on the plan's lookup kind
// (tap words exist for FP32 plans only).
template <typename F>
int with_j(int J, F&& f) {
  switch (J) {
    case 2: return f(std::integral_constant<int, 2>{});
    case 4: return f(std::integral_constant<int, 4>{});
    case 6: return f(std::integral_constant<int, 6>{});
    case 8: return f(std::integral_constant<int, 8>{});
    default: set_error("J = %d unsupported", J); return PR_EUNSUPPORTED;
  }
}

template <typename R, typename F>
int with_lk(const pr_phi_plan_t* p, F&& f) {
  if constexpr (std::is_same<R, float>::value) {
    if (p->tapwords) return f(std::integral_constant<int, kLkWords>{});
  }
  if (p->interp) return f(std::integral_constant<int, kLkLinear>{});
  return f(std::integral_constant<int, kLkNearest>{});
}

template <typename R>
int setup_prec(const pr_phi_plan_t* p) {
  return with_j(p->J, [&](auto jj) {
    return with_lk<R>(p, [&](auto lk) { return setup_kernels<R, decltype(jj)::value, decltype(lk)::value>(); });
  });
}

template <typename R>
GwArgs<R> gw_args(pr_phi_plan_t* p, double scale) {
  GwArgs<R> a{};
  a.grid = static_cast<const cx_t<R>*>(p->grid);
  a.table = static_cast<const R*>(p->table);
  a.uv = static_cast<const R*>(p->uv);
  a.items = p->sched_d;
  a.sched_off = p->sched_d_off;
  a.nItems = p->nItems;
  a.K = p->K; a.T = p->T; a.P = p->P; a.nT = p->nT; a.D = p->D;
  a.lognT = 0;
  while ((1 << a.lognT) < p->nT) ++a.lognT;
  a.tlen = p->J * p->D / 2 + 1;
  if (p->J == 4 && !p->interp) {   // nearest sample, J = 4: the paired table
    a.table = static_cast<const R*>(p->table2);
    a.tlen = 2 * p->D + 2;
  }
  a.kappa = p->kappa;
  a.scale = static_cast<R>(scale);
  a.small = p->small;
  a.nsmall = static_cast<int>(p->nSmall);
  return a;
}

template <typename R>
GwAdjArgs<R> gwadj_args(pr_phi_plan_t* p, double scale) {
  GwAdjArgs<R> a{};
  a.table = static_cast<const R*>(p->table);
  a.uv = static_cast<const R*>(p->uv);
  a.items = p->sched_g;
  a.sched_off = p->sched_g_off;
  a.nItems = p->nItems;
  a.K = p->K; a.T = p->T; a.P = p->P; a.nT = p->nT; a.D = p->D;
  a.lognT = 0;
  while ((1 << a.lognT) < p->nT) ++a.lognT;
  a.tlen = p->J * p->D / 2 + 1;
  if (p->J == 4 && !p->interp) {   // nearest sample, J = 4: the paired table
    a.table = static_cast<const R*>(p->table2);
    a.tlen = 2 * p->D + 2;
  }
  a.kappa = p->kappa;
  a.scale = static_cast<R>(scale);
  a.patches = static_cast<cx_t<R>*>(p->patches);
  return a;
}

template <typename R>
int gw_plain(pr_phi_plan_t* p, void* y, double scale, hipStream_t s) {
  GwArgs<R> a = gw_args<R>(p, scale);
  a.y_out = static_cast<cx_t<R>*>(y);
  return with_j(p->J, [&](auto jj) {
    return with_lk<R>(p, [&](auto lk) { return launch_degrid<R, decltype(jj)::value, 0, decltype(lk)::value>(p, a, s); });
  });
}

template <typename R>
int gw_admm(pr_phi_plan_t* p, const AdmmVis& v, double scale, hipStream_t s) {
  GwArgs<R> a = gw_args<R>(p, scale);
  a.y_obs = static_cast<const cx_t<R>*>(v.y);
  a.scale_dev = v.scale_dev;
  a.s_in = static_cast<const cx_t<R>*>(v.s);
  a.t_out = static_cast<cx_t<R>*>(v.t);
  a.partials = p->partials;
  a.sec = v.sec;
  const int rc = with_j(p->J, [&](auto jj) {
    return with_lk<R>(p, [&](auto lk) {
      constexpr int JJ = decltype(jj)::value, LK = decltype(lk)::value;
      return v.sec_partials ? launch_degrid<R, JJ, 2, LK>(p, a, s) : launch_degrid<R, JJ, 1, LK>(p, a, s);
    });
  });
  if (rc != PR_OK) return rc;
  ball_scale_kernel<<<1, kThreads, 0, s>>>(p->partials, degrid_blocks(p), v.eps, v.kappa_fixed, v.sums);
  PR_TRY_LAUNCH();
  return PR_OK;
}

template <typename R>
int gwadj_plain(pr_phi_plan_t* p, const void* y, double scale, hipStream_t s, int parts,
                const double* scale_dev = nullptr) {
  GwAdjArgs<R> a = gwadj_args<R>(p, scale);
  a.y_in = static_cast<const cx_t<R>*>(y);
  a.scale_dev = scale_dev;
  return with_j(p->J, [&](auto jj) {
    return with_lk<R>(p, [&](auto lk) {
      return launch_grid<R, decltype(jj)::value, 0, decltype(lk)::value>(p, a, s, parts);
    });
  });
}

template <typename R>
int gwadj_admm(pr_phi_plan_t* p, const AdmmVis& v, double scale, hipStream_t s) {
  GwAdjArgs<R> a = gwadj_args<R>(p, scale);
  a.t_in = static_cast<const cx_t<R>*>(v.t);
  a.scale_dev = v.scale_dev;
  a.s_io = static_cast<cx_t<R>*>(v.s);
  a.scalars = v.sums;
  a.varrho = static_cast<R>(v.varrho);
  a.vr_coef = static_cast<R>(v.vr_coef);
  a.sec = v.sec;
  a.kappa_sec = v.kappa_sec;
  return with_j(p->J, [&](auto jj) {
    return with_lk<R>(p, [&](auto lk) { return launch_grid<R, decltype(jj)::value, 1, decltype(lk)::value>(p, a, s); });
  });
}

// ---------------------------------------------------------------------------
// fused launches over several plans (see fused.hpp)
// ---------------------------------------------------------------------------
template <typename R>
size_t fused_vis_bytes_t(int n, int64_t items) {
  Carver c(nullptr);
  c.take<GwArgs<R>>(n);
  c.take<GwAdjArgs<R>>(n);
  c.take<MergeArgs<R>>(n);
  c.take<int4>(items);
  c.take<int32_t>(kDegridBlocks + 1);
  c.take<int4>(items);
  c.take<int32_t>(kGridBlocks + 1);
  c.take<int4>(items);
  return c.bytes();
}

template <typename R>
int fused_vis_build_t(FusedStages* f, Carver& c, hipStream_t s) {
  const int n = static_cast<int>(f->plans.size());
  int64_t total = 0;
  for (const pr_phi_plan_t* p : f->plans) total += p->nItems;
  f->d_dg = c.take<GwArgs<R>>(n);
  f->d_ga = c.take<GwAdjArgs<R>>(n);
  MergeArgs<R>* mg = c.take<MergeArgs<R>>(n);
  f->d_mg = mg;
  f->sched_d = c.take<int4>(total);
  f->sched_d_off = c.take<int32_t>(kDegridBlocks + 1);
  f->sched_g = c.take<int4>(total);
  f->sched_g_off = c.take<int32_t>(kGridBlocks + 1);
  f->small = c.take<int4>(total);
  // every member's items, the tile field tagged with the member
  std::vector<int4> all, it;
  std::vector<int32_t> local;
  std::vector<MergeArgs<R>> hm(static_cast<size_t>(n));
  all.reserve(static_cast<size_t>(total));
  local.reserve(static_cast<size_t>(total));
  int tiles = 0;
  for (int m = 0; m < n; ++m) {
    pr_phi_plan_t* p = f->plans[m];
    it.resize(static_cast<size_t>(p->nItems));
    if (p->nItems > 0) {
      PR_TRY_HIP(hipMemcpyAsync(it.data(), p->items, p->nItems * sizeof(int4), hipMemcpyDeviceToHost, s));
      PR_TRY_HIP(hipStreamSynchronize(s));
    }
    for (int64_t i = 0; i < p->nItems; ++i) {
      int4 e = it[i];
      e.x |= m << kMemberShift;
      all.push_back(e);
      local.push_back(static_cast<int32_t>(i));
    }
    hm[m] = MergeArgs<R>{static_cast<const cx_t<R>*>(p->patches), p->item_off, static_cast<cx_t<R>*>(p->grid), p->K,
                         p->nT, tiles, 0};
    tiles += p->nTiles;
  }
  f->tiles = tiles;
  const pr_phi_plan_t* p0 = f->plans[0];
  const int64_t P2 = static_cast<int64_t>(p0->P) * p0->P;
  // the gridding items split as in a member's own plan: small ones to the
  // small-item kernel (own index in .w), the others to the walk's schedule
  std::vector<int4> big, smallv;
  std::vector<int32_t> bigl;
  // (an item goes to the small-item kernel exactly when its member's own
  // plan sends it there, so that the results stay those of the members)
  for (size_t i = 0; i < all.size(); ++i) {
    int4 e = all[i];
    const bool split = f->plans[item_member(e)]->nSmall > 0;
    if (split && e.z - e.y <= kSmallItem) {
      e.w = local[i];
      smallv.push_back(e);
    } else {
      big.push_back(e);
      bigl.push_back(local[i]);
    }
  }
  const int64_t nbig = static_cast<int64_t>(big.size());
  f->nSmall = static_cast<int64_t>(smallv.size());
  // the degridding schedules the same items as the walk; every block then
  // takes small items after its own (offsets for all kDegridBlocks)
  f->Gd = f->nSmall > 0 ? kDegridBlocks : static_cast<int>(nbig < kDegridBlocks ? nbig : kDegridBlocks);
  f->Gg = static_cast<int>(nbig < kGridBlocks ? nbig : kGridBlocks);
  std::vector<int4> sd, sg;
  std::vector<int32_t> sdo, sgo;
  if (total > 0) {
    lpt_schedule(big, static_cast<int>(nbig < kDegridBlocks ? nbig : kDegridBlocks), P2 / 2, sd, sdo);
    if (f->nSmall > 0) sdo.resize(kDegridBlocks + 1, sdo.back());
    if (!sd.empty())
      PR_TRY_HIP(hipMemcpyAsync(f->sched_d, sd.data(), sd.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    PR_TRY_HIP(hipMemcpyAsync(f->sched_d_off, sdo.data(), sdo.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  }
  if (nbig > 0) {
    lpt_schedule(big, f->Gg, P2, sg, sgo);
    for (int4& e : sg) e.w = bigl[e.w];
    PR_TRY_HIP(hipMemcpyAsync(f->sched_g, sg.data(), sg.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    PR_TRY_HIP(hipMemcpyAsync(f->sched_g_off, sgo.data(), sgo.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  }
  if (!smallv.empty())
    PR_TRY_HIP(hipMemcpyAsync(f->small, smallv.data(), smallv.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  PR_TRY_HIP(hipMemcpyAsync(mg, hm.data(), hm.size() * sizeof(MergeArgs<R>), hipMemcpyHostToDevice, s));
  PR_TRY_HIP(hipStreamSynchronize(s));   // the host vectors go out of scope
  // host argument tables: every member's own launch arguments
  f->h_dg.assign(static_cast<size_t>(n) * sizeof(GwArgs<R>), 0);
  f->h_ga.assign(static_cast<size_t>(n) * sizeof(GwAdjArgs<R>), 0);
  for (int m = 0; m < n; ++m) {
    const GwArgs<R> g = gw_args<R>(f->plans[m], 1.0);
    const GwAdjArgs<R> ga = gwadj_args<R>(f->plans[m], 1.0);
    std::memcpy(f->h_dg.data() + m * sizeof(GwArgs<R>), &g, sizeof g);
    std::memcpy(f->h_ga.data() + m * sizeof(GwAdjArgs<R>), &ga, sizeof ga);
  }
  f->up_dg.assign(static_cast<size_t>(n), nullptr);
  f->up_ga.assign(static_cast<size_t>(n), nullptr);
  return PR_OK;
}

// Patch each call's vector pointers into the host table; upload it when they
// changed (then wait for the copy, so the host table may change next call).
template <typename A, typename V>
int upload_args(std::vector<char>& h, std::vector<const void*>& up, void* dev, V* const* vec, V* A::*field,
                hipStream_t s) {
  const size_t n = up.size();
  bool changed = false;
  for (size_t m = 0; m < n; ++m) {
    A* a = reinterpret_cast<A*>(h.data() + m * sizeof(A));
    a->*field = vec[m];
    if (up[m] != static_cast<const void*>(vec[m])) changed = true;
  }
  if (!changed) return PR_OK;
  PR_TRY_HIP(hipMemcpyAsync(dev, h.data(), h.size(), hipMemcpyHostToDevice, s));
  PR_TRY_HIP(hipStreamSynchronize(s));
  for (size_t m = 0; m < n; ++m) up[m] = vec[m];
  return PR_OK;
}

template <typename R>
int fused_gw_t(FusedStages* f, void* const* y, hipStream_t s) {
  if (f->Gd == 0) return PR_OK;   // no items at all
  using C = cx_t<R>;
  PR_TRY((upload_args<GwArgs<R>, C>(f->h_dg, f->up_dg, f->d_dg, reinterpret_cast<C* const*>(y), &GwArgs<R>::y_out, s)));
  pr_phi_plan_t* p0 = f->plans[0];
  GwArgs<R> a = gw_args<R>(p0, 1.0);
  a.items = f->sched_d;
  a.sched_off = f->sched_d_off;
  a.mtab = static_cast<const GwArgs<R>*>(f->d_dg);
  a.small = f->small;
  a.nsmall = static_cast<int>(f->nSmall);
  return with_j(p0->J, [&](auto jj) {
    return with_lk<R>(p0, [&](auto lk) {
      return launch_degrid<R, decltype(jj)::value, 0, decltype(lk)::value, true>(p0, a, s, f->Gd);
    });
  });
}

template <typename R>
int fused_gw_adjoint_t(FusedStages* f, const void* const* y, hipStream_t s) {
  using C = cx_t<R>;
  pr_phi_plan_t* p0 = f->plans[0];
  if (f->Gg > 0 || f->nSmall > 0) {
    PR_TRY((upload_args<GwAdjArgs<R>, const C>(f->h_ga, f->up_ga, f->d_ga, reinterpret_cast<const C* const*>(y),
                                               &GwAdjArgs<R>::y_in, s)));
    GwAdjArgs<R> a = gwadj_args<R>(p0, 1.0);
    a.items = f->sched_g;
    a.sched_off = f->sched_g_off;
    a.mtab = static_cast<const GwAdjArgs<R>*>(f->d_ga);
    bool walked = false;
    const int rc = with_j(p0->J, [&](auto jj) -> int {
      constexpr int JJ = decltype(jj)::value;
      if constexpr (JJ <= 4) {
        return with_lk<R>(p0, [&](auto lk) -> int {
          constexpr int LK = decltype(lk)::value;
          PR_TRY((launch_walk<R, JJ, 0, LK, true>(p0, a, s, f->Gg, &walked)));
          if (walked) PR_TRY((launch_small<R, JJ, 0, LK, true>(a, f->small, f->nSmall, s)));
          return PR_OK;
        });
      } else {
        return static_cast<int>(PR_OK);
      }
    });
    if (rc != PR_OK) return rc;
    if (!walked) {
      set_error("fused gridding needs the segment walk (J <= 4, tile fitting LDS)");
      return PR_EUNSUPPORTED;
    }
    PR_TRY_LAUNCH();
  }
  merge_patches_kernel<R, true><<<f->tiles, p0->T * p0->T < kThreads ? p0->T * p0->T : kThreads, 0, s>>>(
      nullptr, nullptr, nullptr, 0, p0->T, p0->P, 0, p0->J, static_cast<const MergeArgs<R>*>(f->d_mg),
      static_cast<int>(f->plans.size()));
  PR_TRY_LAUNCH();
  return PR_OK;
}

template <typename R>
__global__ void zero_cx_kernel(cx_t<R>* a, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    a[i] = cmk<cx_t<R>>(R(0), R(0));
}

}  // namespace

bool phi_walk_fits(const pr_phi_plan_t* p) {
  if (p->J > 4) return false;
  const int tlen = p->J == 4 && !p->interp ? 2 * p->D + 2 : p->J * p->D / 2 + 1;
  auto fits = [&](auto r, auto jj) {
    using R = decltype(r);
    constexpr int J = decltype(jj)::value;
    const WalkLds<R, J> with(p->T, tlen, true), without(p->T, tlen, false);
    return (with.total < without.total ? with.total : without.total) <= kLdsHard;
  };
  auto by_j = [&](auto r) {
    switch (p->J) {
      case 2: return fits(r, std::integral_constant<int, 2>{});
      case 4: return fits(r, std::integral_constant<int, 4>{});
      default: return false;
    }
  };
  return p->prec == PR_F32 ? by_j(0.0f) : by_j(0.0);
}

int phi_gridding_setup(pr_phi_plan_t* p) {
  return p->prec == PR_F32 ? setup_prec<float>(p) : setup_prec<double>(p);
}

int phi_gw(pr_phi_plan_t* p, void* y, double scale, hipStream_t s) {
  if (p->M == 0) return PR_OK;
  return p->prec == PR_F32 ? gw_plain<float>(p, y, scale, s) : gw_plain<double>(p, y, scale, s);
}

int phi_gw_adjoint(pr_phi_plan_t* p, const void* y, double scale, hipStream_t s) {
  return phi_gw_adjoint_parts(p, y, scale, 3, s);
}

int phi_gw_adjoint_dev(pr_phi_plan_t* p, const void* y, const double* scale_dev, hipStream_t s) {
  if (p->nItems == 0) return phi_gw_adjoint_parts(p, y, 1.0, 3, s);
  return p->prec == PR_F32 ? gwadj_plain<float>(p, y, 1.0, s, 3, scale_dev)
                           : gwadj_plain<double>(p, y, 1.0, s, 3, scale_dev);
}

int phi_gw_adjoint_parts(pr_phi_plan_t* p, const void* y, double scale, int parts, hipStream_t s) {
  if (p->nItems == 0) {
    if (!(parts & 2)) return PR_OK;
    const int64_t K2 = static_cast<int64_t>(p->K) * p->K;
    if (p->prec == PR_F32)
      zero_cx_kernel<float><<<grid_for(K2, 256, 4096), 256, 0, s>>>(static_cast<float2*>(p->grid), K2);
    else
      zero_cx_kernel<double><<<grid_for(K2, 256, 4096), 256, 0, s>>>(static_cast<double2*>(p->grid), K2);
    PR_TRY_LAUNCH();
    return PR_OK;
  }
  return p->prec == PR_F32 ? gwadj_plain<float>(p, y, scale, s, parts) : gwadj_plain<double>(p, y, scale, s, parts);
}

int phi_gw_admm(pr_phi_plan_t* p, const AdmmVis& v, double scale, hipStream_t s) {
  if (p->nItems == 0) {
    set_error("ADMM needs at least one visibility");
    return PR_EINVAL;
  }
  return p->prec == PR_F32 ? gw_admm<float>(p, v, scale, s) : gw_admm<double>(p, v, scale, s);
}

int phi_section_kappa(pr_phi_plan_t* p, int nsec, const double* eps, double* kappa, double* norm2, hipStream_t s) {
  if (nsec < 1 || nsec > kSecAcc) {
    set_error("internal: %d sections in the degridding partials", nsec);
    return PR_EINVAL;
  }
  section_kappa_partials_kernel<<<nsec, kThreads, 0, s>>>(p->partials, degrid_blocks(p), eps, kappa, norm2);
  PR_TRY_LAUNCH();
  return PR_OK;
}

size_t fused_vis_bytes(int n, int64_t items, int prec) {
  return prec == PR_F32 ? fused_vis_bytes_t<float>(n, items) : fused_vis_bytes_t<double>(n, items);
}

int fused_vis_build(FusedStages* f, Carver& c, hipStream_t s) {
  return f->prec == PR_F32 ? fused_vis_build_t<float>(f, c, s) : fused_vis_build_t<double>(f, c, s);
}

int fused_gw(FusedStages* f, void* const* y, hipStream_t s) {
  return f->prec == PR_F32 ? fused_gw_t<float>(f, y, s) : fused_gw_t<double>(f, y, s);
}

int fused_gw_adjoint(FusedStages* f, const void* const* y, hipStream_t s) {
  return f->prec == PR_F32 ? fused_gw_adjoint_t<float>(f, y, s) : fused_gw_adjoint_t<double>(f, y, s);
}

int phi_gw_adjoint_admm(pr_phi_plan_t* p, const AdmmVis& v, double scale, hipStream_t s) {
  return p->prec == PR_F32 ? gwadj_admm<float>(p, v, scale, s) : gwadj_admm<double>(p, v, scale, s);
}

}  // namespace pr
