// Internal state of a measurement-operator plan and the launchers that act on
// it. The operator is Phi = W G F Z S of eq. (matrix_equation).
#pragma once

#include <vector>

#include "common.hpp"
#include "host/schedule.hpp"

struct pr_phi_plan_t {
  pr_phi_desc desc;
  int n = 0, K = 0, J = 0, D = 0, T = 0;
  int P = 0;        // patch side of one tile: T + J - 1
  int nT = 0;       // tiles per grid side
  int nTiles = 0;
  int prec = PR_F32;
  int interp = 0;   // 0 nearest sample, 1 first-order (linear) lookup
  // Storage of the sorted visibilities: false, (u, v, w) triples (Real[3M]);
  // true, for FP32 nearest-sample plans with tiles <= 16 and D <= 2047, one
  // (tap word, w) pair per visibility (uint32 + float, 8 bytes; taps.hpp)
  bool tapwords = false;
  int64_t M = 0;
  int64_t nItems = 0, nItemsMax = 0;
  int chunk = 0;    // max visibilities per gridding work item
  double kappa = 0; // K / (2 pi)
  double beta = 0;  // Kaiser-Bessel shape

  // persistent workspace
  void* uv = nullptr;          // sorted visibilities: (u, v, w) triples or (tap word, w) pairs
  int32_t* perm = nullptr;     // plan position -> user index
  int32_t* item_off = nullptr; // per tile first work item, [nTiles + 1]
  int4* items = nullptr;       // (tile, begin, end, 0)
  // Static block schedules of the work items: the items in schedule order,
  // each with its own index in .w; block b of a launch takes entries
  // [off[b], off[b+1]).
  int4* sched_d = nullptr;         // degridding, [nItemsMax]
  int32_t* sched_d_off = nullptr;  // [kDegridBlocks + 1]
  int4* sched_g = nullptr;         // gridding, [nItemsMax]
  int32_t* sched_g_off = nullptr;  // [kGridBlocks + 1]
  // Plans whose gridding uses the segment walk split the items: sched_g
  // then holds the items of more than kSmallItem visibilities, and the
  // smaller ones, in item order, go to their own kernel.
  int4* small = nullptr;           // [nItemsMax]
  int64_t nGrid = 0;               // entries of sched_g
  int64_t nSmall = 0;              // entries of small
  void* table = nullptr;       // Real[J*D/2 + 1]
  void* table2 = nullptr;      // J = 4: pairs (T[i], T[D + i]), i = 0..D (Real[2D + 2]); else unused
  void* corr = nullptr;        // Real[n]
  void* tw = nullptr;          // complex[K], e^{-2 pi i m / K}

  // scratch workspace
  void* grid = nullptr;        // complex[K*K], row = v cell, column = u cell
  void* fft_tmp = nullptr;     // complex[n*K]
  void* patches = nullptr;     // complex[nItemsMax * P * P]
  double* partials = nullptr;  // FP64 per-block partial sums
  double* scalars = nullptr;   // FP64 device scalars
  void* img_a = nullptr;       // Real[n*n]
  void* img_b = nullptr;       // Real[n*n]
};

namespace pr {

// Largest visibility count a plan accepts: positions, item bounds and the
// permutation are 32-bit, and every kernel forms (position + a per-item
// offset below 2^20) without overflow; products with positions are 64-bit.
constexpr int64_t kMaxVisibilities = (int64_t(1) << 31) - (int64_t(1) << 20);
constexpr int kPartialsMax = 4096;     // per-block partials, per quantity slot
constexpr int kDegridBlocks = 2048;    // persistent degridding blocks (8 per CU); <= kPartialsMax
constexpr int kGridBlocks = 512;       // persistent gridding blocks (2 per CU, bound by LDS)
constexpr int kSmallItem = 64;         // items of at most this many visibilities: the small-item gridding
constexpr int kSmallSplitMin = 2048;   // ... when a plan has at least this many of them (segment walk)
constexpr int kSmallSplitMinLanes = 512;   // the same with the J-lane gridding (J > 4)
constexpr int kSecAcc = 8;           // local balls: sections summed in the degridding epilogue
constexpr int kSlotSec0 = 4;         // their per-block partials: slots kSlotSec0 .. kSlotSec0 + kSecAcc - 1
constexpr int kPartialSlots = kSlotSec0 + kSecAcc;
constexpr int kScalars = 64;

// Sizes of the two workspaces for a descriptor (validated beforehand).
int phi_layout(pr_phi_plan_t* p, void* persistent, void* scratch,
               size_t* persistent_bytes, size_t* scratch_bytes);
int phi_validate(const pr_phi_desc* d);
// Geometry (sizes, tile, kernel shape) from a validated descriptor.
int phi_prepare(pr_phi_plan_t* p, const pr_phi_desc* d);
int phi_create(pr_phi_plan_t* p, const void* uv, const void* w, hipStream_t s);
// Set the LDS limits of the plan's gridding kernels (once per process and
// device), so that later launches, also under stream capture, set nothing.
int phi_gridding_setup(pr_phi_plan_t* p);
// Whether the plan's gridding uses the segment walk (J <= 4 and its LDS
// fits); those plans split their items between the walk and the
// small-item kernel.
bool phi_walk_fits(const pr_phi_plan_t* p);

// Stable LSD radix sort of M (key, value) pairs on the low `bits` bits of the
// keys, ping-ponging between (k0, v0) and (k1, v1); *kout / *vout name the
// pair holding the result. tmp: sort_tmp_words(M) words.
size_t sort_tmp_words(int64_t M);
int sort_pairs_u32(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t* tmp, int64_t M, int bits,
                   hipStream_t s, uint32_t** kout, uint32_t** vout);

// Operator stages.
int phi_fzs(pr_phi_plan_t* p, const void* x, hipStream_t s);
int phi_fzs_adjoint(pr_phi_plan_t* p, void* x, hipStream_t s);
int phi_gw(pr_phi_plan_t* p, void* y, double scale, hipStream_t s);
int phi_gw_adjoint(pr_phi_plan_t* p, const void* y, double scale, hipStream_t s);
// The two launches of phi_gw_adjoint: parts bit 0 = per-item patches from the
// visibilities, bit 1 = merge of the patches into the grid.
int phi_gw_adjoint_parts(pr_phi_plan_t* p, const void* y, double scale, int parts, hipStream_t s);
// Gridding with the scale read from device memory (1 / ||Phi|| of a solve).
int phi_gw_adjoint_dev(pr_phi_plan_t* p, const void* y, const double* scale_dev, hipStream_t s);
// Power method (host result): at most iters steps; rtol > 0 stops once
// ||A x|| changes by at most rtol of itself between steps.
int phi_norm(pr_phi_plan_t* p, int iters, double rtol, void* vis, double* norm, hipStream_t s);

// Fused ADMM stages (defined with the operator kernels).
struct AdmmVis {
  const void* y;   // observed visibilities
  void* s;         // Lagrange multiplier, updated in place by the gridding stage
  void* t;         // v + s - y, written by the degridding stage
  double* sums;    // device: [0] ||t||^2, [1] ||v - y||^2 (FP64)
  double eps, varrho;
  const double* scale_dev = nullptr;   // device 1 / ||Phi||; overrides the host scale when set
  double vr_coef = 1.0;       // gridded value q = vr_coef (v - r) + s' (1: Algorithm 1; 0: primal-dual, q = s')
  double kappa_fixed = -1.0;  // >= 0: r = y + kappa_fixed t instead of the ball projection
  const int32_t* sec = nullptr;        // local balls: section of each visibility (plan order)
  const double* kappa_sec = nullptr;   // local balls: kappa of each section (overrides the ball's)
  bool sec_partials = false;           // degridding: also FP64 ||t_j||^2 partials per section (< kSecAcc)
};
int phi_gw_admm(pr_phi_plan_t* p, const AdmmVis& a, double scale, hipStream_t s);
int phi_gw_adjoint_admm(pr_phi_plan_t* p, const AdmmVis& a, double scale, hipStream_t s);
// After phi_gw_admm with sec_partials: norm2[j] = ||t_j||^2 and
// kappa[j] = min(1, eps[j] / ||t_j||) for j < nsec <= kSecAcc (device arrays),
// the partials summed in block order.
int phi_section_kappa(pr_phi_plan_t* p, int nsec, const double* eps, double* kappa, double* norm2, hipStream_t s);
// x_out = x_in - rho * Re(S Z^T F^H grid), and zbar = max(x_out, 0).
int phi_fzs_adjoint_step(pr_phi_plan_t* p, const void* x_in, double rho, void* x_out,
                         void* zbar, hipStream_t s);

// FP64 deterministic reductions over device arrays.
int reduce_sq_f64(const void* a, const void* b, int64_t len, int prec, int is_complex,
                  double* partials, double* out, hipStream_t s);

}  // namespace pr
