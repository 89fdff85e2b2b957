// Plan construction for the measurement operator: Kaiser-Bessel table,
// gridding correction and FFT twiddles (FP64 on the GPU), the tile sort of the
// visibilities (stable LSD radix sort on the cell key) and the gridding work
// list. The paper groups visibilities before distributing them (Section
// "Distributed Visibilities"); here the grouping key is the grid tile a
// visibility's footprint starts in, so each tile's visibilities are contiguous.
#include <cmath>
#include <cstdio>
#include <algorithm>
#include <functional>
#include <queue>
#include <utility>
#include <vector>

#include "phi.hpp"
#include "taps.hpp"

namespace pr {

// ---------------------------------------------------------------------------
// tables
// ---------------------------------------------------------------------------

// I0 by the trapezoidal rule on I0(x) = (1/2pi) int_0^{2pi} e^{x cos th} dth.
// The integrand is periodic and analytic, so the rule converges
// geometrically; 96 nodes reach rounding for x up to about 40.
__device__ double i0_trapezoid(double x) {
  const int N = 96;
  double acc = 0.0;
  for (int k = 0; k < N; ++k) acc += exp(x * cospi(2.0 * k / N));
  return acc / N;
}

template <typename R>
__global__ void build_tables_kernel(R* table, int table_len, R* corr, cx_t<R>* tw, int n, int K,
                                    int J, int D, double beta) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const double i0b = i0_trapezoid(beta);
  if (i < table_len) {
    // g(t) at t = i / D
    const double q = (2.0 * i) / (static_cast<double>(J) * D);
    const double arg = 1.0 - q * q;
    table[i] = static_cast<R>(arg >= 0.0 ? i0_trapezoid(beta * sqrt(arg)) / i0b : 0.0);
  } else if (i < table_len + n) {
    // c[p] = 1 / ghat(p / K), ghat(f) = J sinh(z) / (z I0(beta)), z^2 = beta^2 - (pi J f)^2
    const int ix = i - table_len;
    const double f = static_cast<double>(ix - n / 2) / K;
    const double a = M_PI * J * f;
    const double z2 = beta * beta - a * a;
    double shape;
    if (z2 > 0) {
      const double z = sqrt(z2);
      shape = sinh(z) / z;
    } else if (z2 < 0) {
      const double z = sqrt(-z2);
      shape = sin(z) / z;
    } else {
      shape = 1.0;
    }
    corr[ix] = static_cast<R>(i0b / (J * shape));
  } else if (i < table_len + n + K) {
    const int m = i - table_len - n;
    double sv, cv;
    sincospi(2.0 * m / K, &sv, &cv);
    tw[m] = cmk<cx_t<R>>(static_cast<R>(cv), static_cast<R>(-sv));
  }
}

// J = 4: the four nearest-sample taps of an axis read T[up], T[D + up],
// T[D - dn] and T[2D - dn]; stored as pairs (T[i], T[D + i]) they take two
// loads, T2[up] and T2[D - dn].
template <typename R>
__global__ void pair_table_kernel(const R* table, int D, R* table2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i > D) return;
  table2[2 * i] = table[i];
  table2[2 * i + 1] = table[D + i];
}

// ---------------------------------------------------------------------------
// keys, radix sort, scan
// ---------------------------------------------------------------------------
template <typename R>
__global__ void cell_keys_kernel(const R* uv, int64_t M, double kappa, int K, int J, int T, int nT,
                                 uint32_t* keys, uint32_t* vals) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= M) return;
  const AxisTaps tu = axis_taps(static_cast<double>(uv[2 * k]), kappa, J, 1);
  const AxisTaps tv = axis_taps(static_cast<double>(uv[2 * k + 1]), kappa, J, 1);
  const int bu = mod_pow2(tu.j0, K), bv = mod_pow2(tv.j0, K);
  const uint32_t tile = static_cast<uint32_t>((bv / T) * nT + bu / T);
  keys[k] = tile * static_cast<uint32_t>(T * T) + static_cast<uint32_t>((bv % T) * T + bu % T);
  vals[k] = static_cast<uint32_t>(k);
}

constexpr int kSortThreads = 256;
constexpr int kSortChunk = 4096;

__global__ void radix_upsweep(const uint32_t* keys, int64_t M, int shift, int nblocks,
                              uint32_t* hist) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t start = static_cast<int64_t>(blockIdx.x) * kSortChunk;
  const int64_t end = start + kSortChunk < M ? start + kSortChunk : M;
  for (int64_t i = start + threadIdx.x; i < end; i += kSortThreads)
    atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
  __syncthreads();
  hist[static_cast<int64_t>(threadIdx.x) * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: elements keep their input order within a digit. Ranks come
// from wave-level digit matching (8 ballots) and per-wave prefix counts.
__global__ void radix_downsweep(const uint32_t* keys_in, const uint32_t* vals_in, uint32_t* keys_out,
                                uint32_t* vals_out, const uint32_t* offsets, int64_t M, int shift,
                                int nblocks) {
  constexpr int NW = kSortThreads / 64;
  __shared__ uint32_t base[256];
  __shared__ uint32_t running[256];
  __shared__ uint32_t total[256];
  __shared__ uint32_t wcount[NW][256];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  base[tid] = offsets[static_cast<int64_t>(tid) * nblocks + blockIdx.x];
  running[tid] = 0;
  const int64_t start = static_cast<int64_t>(blockIdx.x) * kSortChunk;
  const int64_t end = start + kSortChunk < M ? start + kSortChunk : M;
  const unsigned long long lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  for (int64_t sub = start; sub < end; sub += kSortThreads) {
    for (int w = 0; w < NW; ++w) wcount[w][tid] = 0;
    __syncthreads();
    const int64_t idx = sub + tid;
    const bool valid = idx < end;
    const uint32_t key = valid ? keys_in[idx] : 0u;
    const uint32_t val = valid ? vals_in[idx] : 0u;
    const uint32_t d = (key >> shift) & 255u;
    unsigned long long peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const bool bit = (d >> b) & 1u;
      const unsigned long long bal = __ballot(bit);
      peers &= bit ? bal : ~bal;
    }
    const uint32_t rank = static_cast<uint32_t>(__popcll(peers & lt));
    if (valid && rank == 0) wcount[wave][d] = static_cast<uint32_t>(__popcll(peers));
    __syncthreads();
    {
      uint32_t s = 0;
      for (int w = 0; w < NW; ++w) {
        const uint32_t c = wcount[w][tid];
        wcount[w][tid] = s;
        s += c;
      }
      total[tid] = s;
    }
    __syncthreads();
    if (valid) {
      const uint32_t dst = base[d] + running[d] + wcount[wave][d] + rank;
      if (dst < static_cast<uint64_t>(M)) {
        keys_out[dst] = key;
        vals_out[dst] = val;
      }
    }
    __syncthreads();
    running[tid] += total[tid];
  }
}

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanChunk = kScanThreads * kScanItems;

__global__ void scan_reduce(const uint32_t* in, int64_t n, uint32_t* sums) {
  __shared__ uint32_t sh[kScanThreads];
  const int64_t start = static_cast<int64_t>(blockIdx.x) * kScanChunk;
  uint32_t acc = 0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t j = start + static_cast<int64_t>(i) * kScanThreads + threadIdx.x;
    if (j < n) acc += in[j];
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = kScanThreads / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) sums[blockIdx.x] = sh[0];
}

__global__ void scan_apply(const uint32_t* in, uint32_t* out, int64_t n, const uint32_t* carry) {
  __shared__ uint32_t sh[kScanThreads];
  const int64_t start = static_cast<int64_t>(blockIdx.x) * kScanChunk + static_cast<int64_t>(threadIdx.x) * kScanItems;
  uint32_t v[kScanItems];
  uint32_t acc = 0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t j = start + i;
    v[i] = j < n ? in[j] : 0u;
    acc += v[i];
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const uint32_t add = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  uint32_t run = sh[threadIdx.x] - acc + (carry ? carry[blockIdx.x] : 0u);
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t j = start + i;
    if (j < n) out[j] = run;
    run += v[i];
  }
}

// Scratch words scan_exclusive needs for n elements.
static int64_t scan_tmp_words(int64_t n) {
  int64_t words = 0;
  while (n > kScanChunk) {
    n = (n + kScanChunk - 1) / kScanChunk;
    words += ((n + 63) / 64) * 64;
  }
  return words;
}

static int scan_exclusive(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, hipStream_t s) {
  if (n <= 0) return PR_OK;
  const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  if (nb == 1) {
    scan_apply<<<1, kScanThreads, 0, s>>>(in, out, n, nullptr);
    PR_TRY_LAUNCH();
    return PR_OK;
  }
  uint32_t* sums = tmp;
  scan_reduce<<<static_cast<unsigned>(nb), kScanThreads, 0, s>>>(in, n, sums);
  PR_TRY_LAUNCH();
  PR_TRY(scan_exclusive(sums, sums, nb, tmp + ((nb + 63) / 64) * 64, s));
  scan_apply<<<static_cast<unsigned>(nb), kScanThreads, 0, s>>>(in, out, n, sums);
  PR_TRY_LAUNCH();
  return PR_OK;
}

size_t sort_tmp_words(int64_t M) {
  const int64_t m = M > 0 ? M : 1;
  const int64_t hn = 256 * ((m + kSortChunk - 1) / kSortChunk);
  // histogram (rounded up to 64 words), then the scan's scratch and its slack
  return static_cast<size_t>(hn + 64 + scan_tmp_words(hn) + 64);
}

int sort_pairs_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t* tmp, int64_t M, int bits,
                   hipStream_t s, uint32_t** kout, uint32_t** vout) {
  const int nblocks = static_cast<int>((M + kSortChunk - 1) / kSortChunk);
  uint32_t* hist = tmp;
  uint32_t* scan_tmp = tmp + ((int64_t(256) * nblocks + 63) / 64) * 64;
  uint32_t *kin = k0, *ko = k1, *vin = v0, *vo = v1;
  if (M > 0) {
    for (int shift = 0; shift < bits; shift += 8) {
      radix_upsweep<<<nblocks, kSortThreads, 0, s>>>(kin, M, shift, nblocks, hist);
      PR_TRY_LAUNCH();
      PR_TRY(scan_exclusive(hist, hist, int64_t(256) * nblocks, scan_tmp, s));
      radix_downsweep<<<nblocks, kSortThreads, 0, s>>>(kin, vin, ko, vo, hist, M, shift, nblocks);
      PR_TRY_LAUNCH();
      std::swap(kin, ko);
      std::swap(vin, vo);
    }
  }
  *kout = kin;
  *vout = vin;
  return PR_OK;
}

// ---------------------------------------------------------------------------
// work list
// ---------------------------------------------------------------------------
__global__ void tile_bounds_kernel(const uint32_t* keys, int64_t M, int nTiles, int T2,
                                   int32_t* tile_start) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > nTiles) return;
  const uint64_t target = static_cast<uint64_t>(t) * T2;
  int64_t lo = 0, hi = M;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (static_cast<uint64_t>(keys[mid]) < target) lo = mid + 1;
    else hi = mid;
  }
  tile_start[t] = static_cast<int32_t>(lo);
}

// Work items of a tile [b, b + c): cut at the positions (b rounded down to a
// multiple of kItemAlign) + i chunk, so that every item but a tile's first
// starts on a multiple of kItemAlign positions and every item spans at most
// chunk positions counted from the multiple of kItemAlign at or below its
// start (the gridding walk lays its segments out from there).
constexpr int kItemAlign = 16;

__global__ void item_count_kernel(const int32_t* tile_start, int nTiles, int chunk, uint32_t* counts) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > nTiles) return;
  if (t == nTiles) { counts[t] = 0; return; }
  const int b = tile_start[t], c = tile_start[t + 1] - b;
  const int d = b & (kItemAlign - 1);
  counts[t] = c == 0 ? 0u : static_cast<uint32_t>((c + d + chunk - 1) / chunk);
}

__global__ void item_fill_kernel(const int32_t* tile_start, const uint32_t* item_off_u, int nTiles, int chunk,
                                 int4* items, int32_t* item_off) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > nTiles) return;
  item_off[t] = static_cast<int32_t>(item_off_u[t]);
  if (t == nTiles) return;
  const int b = tile_start[t], c = tile_start[t + 1] - b;
  const int q = static_cast<int>(item_off_u[t + 1] - item_off_u[t]);
  const int b0 = b & ~(kItemAlign - 1);
  for (int i = 0; i < q; ++i) {
    const int lo = i == 0 ? b : b0 + i * chunk;
    const int hi = i == q - 1 ? b + c : b0 + (i + 1) * chunk;
    items[item_off_u[t] + i] = make_int4(t, lo, hi, 0);
  }
}

template <typename R>
__global__ void gather_sorted_kernel(const R* uv, const R* w, const uint32_t* perm, int64_t M,
                                     R* uvw_out, int32_t* perm_out) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= M) return;
  const uint32_t j = perm[k];
  uvw_out[3 * k] = uv[2 * static_cast<int64_t>(j)];
  uvw_out[3 * k + 1] = uv[2 * static_cast<int64_t>(j) + 1];
  uvw_out[3 * k + 2] = w ? w[j] : R(1);
  perm_out[k] = static_cast<int32_t>(j);
}

// FP32 nearest-sample plans: the taps of each visibility evaluated once, with
// the same axis_taps as the cell keys, stored as (tap word, w) in plan order.
__global__ void gather_tapwords_kernel(const float* uv, const float* w, const uint32_t* perm, int64_t M,
                                       double kappa, int K, int J, int D, int T, uint2* out, int32_t* perm_out) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= M) return;
  const uint32_t j = perm[k];
  const AxisTaps tu = axis_taps(static_cast<double>(uv[2 * static_cast<int64_t>(j)]), kappa, J, D);
  const AxisTaps tv = axis_taps(static_cast<double>(uv[2 * static_cast<int64_t>(j) + 1]), kappa, J, D);
  const int lu = mod_pow2(tu.j0, K) & (T - 1), lv = mod_pow2(tv.j0, K) & (T - 1);
  out[k] = make_uint2(tap_word(tu, tv, lu, lv), __float_as_uint(w ? w[j] : 1.0f));
  perm_out[k] = static_cast<int32_t>(j);
}

// ---------------------------------------------------------------------------
// layout, validation, creation
// ---------------------------------------------------------------------------
static bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }

// Default tile side: FP32 with J <= 4 uses 16 (moments 32 KB of LDS, table
// still in LDS, two blocks per CU; fewer, fuller work items than 8 at every
// density measured); wider kernels and FP64 use 8. pr_phi_tune measures.
static int default_tile(int J, int prec, int64_t M, int K) {
  (void)M;
  (void)K;
  return (prec == PR_F32 && J <= 4) ? 16 : 8;
}

// Smallest LDS footprint of the gridding kernel for a tile: moments, one side
// slot per segment and a 64-visibility staging batch, table in global memory
// (segments: 256 / threads per segment, threads per segment = ceil(J / JA)
// rounded up to a power of two, JA = moment columns per thread).
static size_t grid_lds_min(int T, int J, int prec) {
  const size_t sr = prec == PR_F32 ? 4 : 8, sc = 2 * sr;
  const int ja = J <= 2 ? J : 2;
  int tpc = (J + ja - 1) / ja;
  if (tpc == 3) tpc = 4;
  const size_t ns = 256 / tpc;
  return static_cast<size_t>(T) * T * J * J * sc + ns * J * J * sc + ns * 4 + 64 * (4 + 2 * J * sr + sc) + 256;
}

int phi_validate(const pr_phi_desc* d) {
  if (!d) { set_error("desc is NULL"); return PR_EINVAL; }
  if (!is_pow2(d->n) || d->n < 8 || d->n > 4096) {
    set_error("n = %d: must be a power of two in [8, 4096]", d->n);
    return PR_EINVAL;
  }
  if (d->oversample != 2) { set_error("oversample = %d: only 2 is supported", d->oversample); return PR_EUNSUPPORTED; }
  if (d->J != 2 && d->J != 4 && d->J != 6 && d->J != 8) { set_error("J = %d: must be 2, 4, 6 or 8", d->J); return PR_EINVAL; }
  if (d->D < 1 || d->D > 1000000) { set_error("D = %d: must be in [1, 1e6]", d->D); return PR_EINVAL; }
  if (d->M < 0 || d->M > kMaxVisibilities) {
    set_error("M = %lld out of range [0, %lld]", static_cast<long long>(d->M), static_cast<long long>(kMaxVisibilities));
    return PR_EINVAL;
  }
  if (d->prec != PR_F32 && d->prec != PR_F64) { set_error("prec = %d", d->prec); return PR_EINVAL; }
  if (d->interp < 0 || d->interp > 2) {
    set_error("interp = %d: must be 0 (nearest), 1 (linear) or 2 (nearest, taps recomputed per launch)", d->interp);
    return PR_EINVAL;
  }
  if (d->tile != 0 && d->tile != 8 && d->tile != 16 && d->tile != 32) {
    set_error("tile = %d: must be 0, 8, 16 or 32", d->tile);
    return PR_EINVAL;
  }
  const int K = d->oversample * d->n;
  const int T = d->tile ? d->tile : default_tile(d->J, d->prec, d->M, K);
  if (T > K || T < d->J) { set_error("tile %d must satisfy J <= tile <= K (J=%d, K=%d)", T, d->J, K); return PR_EINVAL; }
  if (grid_lds_min(T, d->J, d->prec) > 163840) {
    set_error("tile %d with J=%d in %s needs more than 160 KB of LDS", T, d->J, d->prec == PR_F32 ? "FP32" : "FP64");
    return PR_EUNSUPPORTED;
  }
  return PR_OK;
}

int phi_prepare(pr_phi_plan_t* p, const pr_phi_desc* d) {
  p->desc = *d;
  p->n = d->n;
  p->K = d->oversample * d->n;
  p->J = d->J;
  p->D = d->D;
  p->M = d->M;
  p->prec = d->prec;
  p->interp = d->interp == 1 ? 1 : 0;
  p->T = d->tile ? d->tile : default_tile(d->J, d->prec, d->M, p->K);
  p->P = p->T + p->J - 1;
  p->tapwords = d->interp == 0 && d->prec == PR_F32 && p->T <= kTapWordMaxTile && d->D <= kTapWordMaxD;
  p->nT = p->K / p->T;
  p->nTiles = p->nT * p->nT;
  // Work-item size: about M / 2048 visibilities (a power of two in [2048, 8192])
  // so that dense tiles split over many blocks while the fixed cost of an item
  // (patch load or assembly, carries between segments) stays small. A tile is
  // cut into full items and a remainder (see item_count_kernel).
  {
    int64_t c = 2048;
    while (c < 8192 && c * 2048 < p->M) c *= 2;
    p->chunk = static_cast<int>(c);
  }
  // items per tile: ceil((count + shift) / chunk), shift < kItemAlign
  p->nItemsMax = p->nTiles + (p->M + static_cast<int64_t>(kItemAlign - 1) * p->nTiles + p->chunk - 1) / p->chunk;
  p->kappa = static_cast<double>(p->K) / (2.0 * M_PI);
  const double alpha = static_cast<double>(d->oversample);
  p->beta = M_PI * std::sqrt((p->J / alpha) * (p->J / alpha) * (alpha - 0.5) * (alpha - 0.5) - 0.8);
  return PR_OK;
}

struct CreateScratch {
  uint32_t *keys0, *keys1, *vals0, *vals1, *hist, *scan_tmp, *counts, *counts_scan;
  int32_t* tile_start;
  int nblocks;
};

static CreateScratch carve_create(pr_phi_plan_t* p, Carver& c) {
  CreateScratch cs{};
  const int64_t M = p->M > 0 ? p->M : 1;
  cs.nblocks = static_cast<int>((M + kSortChunk - 1) / kSortChunk);
  cs.keys0 = c.take<uint32_t>(M);
  cs.keys1 = c.take<uint32_t>(M);
  cs.vals0 = c.take<uint32_t>(M);
  cs.vals1 = c.take<uint32_t>(M);
  const int64_t hn = int64_t(256) * cs.nblocks;
  cs.hist = c.take<uint32_t>(hn);
  const int64_t tn = p->nTiles + 1;
  cs.scan_tmp = c.take<uint32_t>(scan_tmp_words(hn > tn ? hn : tn) + 64);
  cs.counts = c.take<uint32_t>(tn);
  cs.counts_scan = c.take<uint32_t>(tn);
  cs.tile_start = c.take<int32_t>(tn);
  return cs;
}

int phi_layout(pr_phi_plan_t* p, void* persistent, void* scratch, size_t* persistent_bytes,
               size_t* scratch_bytes) {
  const size_t rs = p->prec == PR_F32 ? 4 : 8;
  const int64_t M = p->M;
  Carver a(persistent);
  // (u, v, w) or (tap word, w) per visibility, plan order
  p->uv = a.take<char>(p->tapwords ? 8 * M : 3 * M * rs);
  p->perm = a.take<int32_t>(M);
  p->item_off = a.take<int32_t>(p->nTiles + 1);
  p->items = a.take<int4>(p->nItemsMax);
  p->sched_d = a.take<int4>(p->nItemsMax);
  p->sched_d_off = a.take<int32_t>(kDegridBlocks + 1);
  p->sched_g = a.take<int4>(p->nItemsMax);
  p->sched_g_off = a.take<int32_t>(kGridBlocks + 1);
  p->small = a.take<int4>(p->nItemsMax);
  p->table = a.take<char>((p->J * static_cast<int64_t>(p->D) / 2 + 1) * rs);
  p->table2 = a.take<char>(p->J == 4 ? (2 * static_cast<int64_t>(p->D) + 2) * rs : 0);
  p->corr = a.take<char>(p->n * rs);
  p->tw = a.take<char>(p->K * 2 * rs);
  if (persistent_bytes) *persistent_bytes = a.bytes();

  Carver b(scratch);
  const int64_t K2 = static_cast<int64_t>(p->K) * p->K;
  p->grid = b.take<char>(K2 * 2 * rs);
  p->fft_tmp = b.take<char>(static_cast<int64_t>(p->n) * p->K * 2 * rs);
  p->patches = b.take<char>(p->nItemsMax * p->P * p->P * 2 * rs);
  p->partials = b.take<double>(kPartialsMax * kPartialSlots);
  p->scalars = b.take<double>(kScalars);
  p->img_a = b.take<char>(static_cast<int64_t>(p->n) * p->n * rs);
  p->img_b = b.take<char>(static_cast<int64_t>(p->n) * p->n * rs);
  size_t op = b.bytes();
  Carver c(nullptr);
  carve_create(p, c);
  size_t cr = c.bytes();
  if (scratch_bytes) *scratch_bytes = op > cr ? op : cr;
  return PR_OK;
}


static int build_schedules(pr_phi_plan_t* p, hipStream_t s) {
  const int64_t n = p->nItems;
  if (n == 0) return PR_OK;
  std::vector<int4> items(static_cast<size_t>(n));
  PR_TRY_HIP(hipMemcpyAsync(items.data(), p->items, n * sizeof(int4), hipMemcpyDeviceToHost, s));
  PR_TRY_HIP(hipStreamSynchronize(s));
  const int64_t P2 = static_cast<int64_t>(p->P) * p->P;
  std::vector<int4> sd, sg, big, small;
  std::vector<int32_t> sdo, sgo, bigi;
  // Items of at most kSmallItem visibilities go to the small-item gridding
  // kernel (item order, own index in .w) when there are enough of them to pay
  // for its launch (with the walk a few hundred ride along in its schedule,
  // hidden among its blocks; the J-lane kernel pays more per item); the
  // degridding then also takes them one wave per item after each block's
  // scheduled items.
  int64_t nsmall_items = 0;
  for (const int4& e : items) nsmall_items += e.z - e.y <= kSmallItem ? 1 : 0;
  const bool split = nsmall_items >= (phi_walk_fits(p) ? kSmallSplitMin : kSmallSplitMinLanes);
  for (int64_t i = 0; i < n; ++i) {
    int4 e = items[static_cast<size_t>(i)];
    if (split && e.z - e.y <= kSmallItem) {
      e.w = static_cast<int>(i);
      small.push_back(e);
    } else {
      big.push_back(e);
      bigi.push_back(static_cast<int32_t>(i));
    }
  }
  const int64_t nb = static_cast<int64_t>(big.size());
  const int Gd = static_cast<int>(nb < kDegridBlocks ? nb : kDegridBlocks);
  lpt_schedule(big, Gd, P2 / 2, sd, sdo);       // per item: the patch load
  if (!small.empty()) sdo.resize(kDegridBlocks + 1, sdo.back());
  const int Gg = static_cast<int>(nb < kGridBlocks ? nb : kGridBlocks);
  lpt_schedule(big, Gg, P2, sg, sgo);           // per item: clearing, assembly, patch store
  for (int4& e : sg) e.w = bigi[static_cast<size_t>(e.w)];
  p->nGrid = nb;
  p->nSmall = static_cast<int64_t>(small.size());
  if (!sd.empty()) PR_TRY_HIP(hipMemcpyAsync(p->sched_d, sd.data(), sd.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  PR_TRY_HIP(hipMemcpyAsync(p->sched_d_off, sdo.data(), sdo.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  if (nb > 0) {
    PR_TRY_HIP(hipMemcpyAsync(p->sched_g, sg.data(), sg.size() * sizeof(int4), hipMemcpyHostToDevice, s));
    PR_TRY_HIP(hipMemcpyAsync(p->sched_g_off, sgo.data(), sgo.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  }
  if (!small.empty())
    PR_TRY_HIP(hipMemcpyAsync(p->small, small.data(), small.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  PR_TRY_HIP(hipStreamSynchronize(s));   // the host vectors go out of scope
  return PR_OK;
}

template <typename R>
static int create_impl(pr_phi_plan_t* p, const R* uv, const R* w, hipStream_t s) {
  // tables
  const int tlen = p->J * p->D / 2 + 1;
  const int total = tlen + p->n + p->K;
  build_tables_kernel<R><<<(total + 255) / 256, 256, 0, s>>>(
      static_cast<R*>(p->table), tlen, static_cast<R*>(p->corr), static_cast<cx_t<R>*>(p->tw), p->n, p->K,
      p->J, p->D, p->beta);
  PR_TRY_LAUNCH();
  if (p->J == 4) {
    pair_table_kernel<R><<<(p->D + 1 + 255) / 256, 256, 0, s>>>(static_cast<const R*>(p->table), p->D,
                                                                 static_cast<R*>(p->table2));
    PR_TRY_LAUNCH();
  }

  Carver c(p->grid);  // plan-time scratch aliases the operator scratch
  CreateScratch cs = carve_create(p, c);
  const int64_t M = p->M;
  if (M > 0) {
    const unsigned gb = static_cast<unsigned>((M + 255) / 256);
    cell_keys_kernel<R><<<gb, 256, 0, s>>>(uv, M, p->kappa, p->K, p->J, p->T, p->nT, cs.keys0, cs.vals0);
    PR_TRY_LAUNCH();
    int bits = 0;
    while ((int64_t(1) << bits) < static_cast<int64_t>(p->K) * p->K) ++bits;
    uint32_t *kin = cs.keys0, *kout = cs.keys1, *vin = cs.vals0, *vout = cs.vals1;
    for (int shift = 0; shift < bits; shift += 8) {
      radix_upsweep<<<cs.nblocks, kSortThreads, 0, s>>>(kin, M, shift, cs.nblocks, cs.hist);
      PR_TRY_LAUNCH();
      PR_TRY(scan_exclusive(cs.hist, cs.hist, int64_t(256) * cs.nblocks, cs.scan_tmp, s));
      radix_downsweep<<<cs.nblocks, kSortThreads, 0, s>>>(kin, vin, kout, vout, cs.hist, M, shift, cs.nblocks);
      PR_TRY_LAUNCH();
      std::swap(kin, kout);
      std::swap(vin, vout);
    }
    if constexpr (std::is_same<R, float>::value) {
      if (p->tapwords) {
        gather_tapwords_kernel<<<gb, 256, 0, s>>>(uv, w, vin, M, p->kappa, p->K, p->J, p->D, p->T,
                                                  static_cast<uint2*>(p->uv), p->perm);
      } else {
        gather_sorted_kernel<R><<<gb, 256, 0, s>>>(uv, w, vin, M, static_cast<R*>(p->uv), p->perm);
      }
    } else {
      gather_sorted_kernel<R><<<gb, 256, 0, s>>>(uv, w, vin, M, static_cast<R*>(p->uv), p->perm);
    }
    PR_TRY_LAUNCH();
    const int nt1 = p->nTiles + 1;
    tile_bounds_kernel<<<(nt1 + 255) / 256, 256, 0, s>>>(kin, M, p->nTiles, p->T * p->T, cs.tile_start);
    PR_TRY_LAUNCH();
  } else {
    PR_TRY_HIP(hipMemsetAsync(cs.tile_start, 0, (p->nTiles + 1) * sizeof(int32_t), s));
  }
  const int nt1 = p->nTiles + 1;
  item_count_kernel<<<(nt1 + 255) / 256, 256, 0, s>>>(cs.tile_start, p->nTiles, p->chunk, cs.counts);
  PR_TRY_LAUNCH();
  PR_TRY(scan_exclusive(cs.counts, cs.counts_scan, nt1, cs.scan_tmp, s));
  item_fill_kernel<<<(nt1 + 255) / 256, 256, 0, s>>>(cs.tile_start, cs.counts_scan, p->nTiles, p->chunk,
                                                      p->items, p->item_off);
  PR_TRY_LAUNCH();
  int32_t nitems = 0;
  PR_TRY_HIP(hipMemcpyAsync(&nitems, p->item_off + p->nTiles, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PR_TRY_HIP(hipStreamSynchronize(s));
  p->nItems = nitems;
  if (p->nItems > p->nItemsMax) {
    set_error("internal: %lld work items exceed the bound %lld", static_cast<long long>(p->nItems),
              static_cast<long long>(p->nItemsMax));
    return PR_EINVAL;
  }
  return build_schedules(p, s);
}

int phi_create(pr_phi_plan_t* p, const void* uv, const void* w, hipStream_t s) {
  PR_TRY(no_capture(s, "plan creation"));
  PR_TRY(phi_gridding_setup(p));
  if (p->prec == PR_F32)
    return create_impl<float>(p, static_cast<const float*>(uv), static_cast<const float*>(w), s);
  return create_impl<double>(p, static_cast<const double*>(uv), static_cast<const double*>(w), s);
}

}  // namespace pr
