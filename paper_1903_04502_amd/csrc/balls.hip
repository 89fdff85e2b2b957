// Local l2-ball constraints (Section "Local Fidelity Constraint ADMM",
// eq. proj-L2-local): the visibilities are split into sections j, each with
// its own ball ||Phi_j x - y_j|| <= eps_j, and the r step of Algorithm 1
// projects every section independently.
//
// With at most kSecAcc sections the degridding epilogue of Algorithm 1 also
// keeps one FP64 ||t_j||^2 partial per section and block, and one small kernel
// sums them in block order into kappa_j. With more sections, set-up
// (pr_balls_create) sorts the plan positions by section (stable radix sort)
// and cuts every section's range into pieces of kPiece positions; per
// iteration, after the degridding has written t = v + s - y:
//   piece sums   sum |t|^2 over a piece (FP64, fixed tree)     section_sq_kernel
//   section sums pieces of a section in order; kappa_j         section_kappa_kernel
// In both cases the fused gridding of Algorithm 1 applies, per visibility, the
// projection and multiplier update with its section's kappa_j (read through
// the section id) before gridding. Every reduction has a fixed order, so the
// result is bitwise repeatable.
#include <algorithm>
#include <cmath>
#include <vector>

#include "admm.hpp"
#include "ops.hpp"

struct pr_balls_t {
  int64_t M = 0;
  int32_t nsec = 0;
  int32_t* section = nullptr;         // copy of the section ids, plan order
  uint32_t* order = nullptr;          // plan positions sorted by section
  int4* pieces = nullptr;             // {section, first, end, 0} in sorted positions
  int64_t npieces = 0;
  int32_t* pfirst = nullptr;          // first piece of each section, [nsec + 1]
  double* piece_sum = nullptr;
  double* eps = nullptr;
  double* kappa = nullptr;
  double* norm2 = nullptr;            // ||t_j||^2 of the last iteration
  int device = 0;
};

namespace pr {
namespace {

constexpr int kPiece = 4096;
constexpr int kBallThreads = 256;

struct BallsLayout {
  int32_t* section;
  uint32_t* order;
  int4* pieces;
  int32_t* pfirst;
  double *piece_sum, *eps, *kappa, *norm2;
};

int64_t pieces_max(int64_t M, int32_t nsec) { return (M + kPiece - 1) / kPiece + nsec; }

size_t balls_layout(int64_t M, int32_t nsec, void* base, BallsLayout* L) {
  Carver c(base);
  const int64_t np = pieces_max(M, nsec);
  BallsLayout l{};
  l.section = c.take<int32_t>(M > 0 ? M : 1);
  l.order = c.take<uint32_t>(M > 0 ? M : 1);
  l.pieces = c.take<int4>(np);
  l.pfirst = c.take<int32_t>(nsec + 1);
  l.piece_sum = c.take<double>(np);
  l.eps = c.take<double>(nsec);
  l.kappa = c.take<double>(nsec);
  l.norm2 = c.take<double>(nsec);
  if (L) *L = l;
  return c.bytes();
}

struct BallsScratch {
  uint32_t *k0, *v0, *k1, *v1, *tmp;
  int32_t* off;
  int32_t* bad;
};

size_t balls_scratch_layout(int64_t M, int32_t nsec, void* base, BallsScratch* S) {
  Carver c(base);
  const int64_t m = M > 0 ? M : 1;
  BallsScratch b{};
  b.k0 = c.take<uint32_t>(m);
  b.v0 = c.take<uint32_t>(m);
  b.k1 = c.take<uint32_t>(m);
  b.v1 = c.take<uint32_t>(m);
  b.tmp = c.take<uint32_t>(sort_tmp_words(M));
  b.off = c.take<int32_t>(nsec + 1);
  b.bad = c.take<int32_t>(1);
  if (S) *S = b;
  return c.bytes();
}

__global__ void section_keys_kernel(const int32_t* section, int64_t M, int32_t nsec, uint32_t* keys,
                                    uint32_t* vals, int32_t* sec_copy, int32_t* bad) {
  const int64_t k = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x;
  if (k >= M) return;
  const int32_t j = section[k];
  const bool ok = j >= 0 && j < nsec;
  if (!ok) atomicOr(bad, 1);
  keys[k] = ok ? static_cast<uint32_t>(j) : 0u;
  sec_copy[k] = ok ? j : 0;
  vals[k] = static_cast<uint32_t>(k);
}

__global__ void zero_flag_kernel(int32_t* f) { *f = 0; }

// off[j] = first sorted position with key >= j, j in [0, nsec]
__global__ void section_bounds_kernel(const uint32_t* keys, int64_t M, int32_t nsec, int32_t* off) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j > nsec) return;
  int64_t lo = 0, hi = M;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (keys[mid] < static_cast<uint32_t>(j)) lo = mid + 1;
    else hi = mid;
  }
  off[j] = static_cast<int32_t>(lo);
}

template <typename R>
__global__ __launch_bounds__(kBallThreads) void section_sq_kernel(const cx_t<R>* t, const uint32_t* order,
                                                                  const int4* pieces, int64_t npieces,
                                                                  double* piece_sum) {
  __shared__ double sh[kBallThreads];
  for (int64_t p = blockIdx.x; p < npieces; p += gridDim.x) {
    const int4 pc = pieces[p];
    double acc = 0;
    for (int i = pc.y + static_cast<int>(threadIdx.x); i < pc.z; i += kBallThreads) {
      const cx_t<R> v = t[order[i]];
      const double a = v.x, b = v.y;
      acc += a * a + b * b;
    }
    const double tot = block_sum_f64(acc, sh);
    if (threadIdx.x == 0) piece_sum[p] = tot;
  }
}

// One wave per section: lane l sums pieces l, l + 64, ... of its section, then
// a fixed xor-butterfly over the wave.
__global__ __launch_bounds__(kBallThreads) void section_kappa_kernel(const int32_t* pfirst, const double* piece_sum,
                                                                     const double* eps, int32_t nsec, double* kappa,
                                                                     double* norm2) {
  const int j = blockIdx.x * (kBallThreads / 64) + static_cast<int>(threadIdx.x >> 6);
  const int lane = static_cast<int>(threadIdx.x & 63);
  if (j >= nsec) return;   // whole waves leave together
  double s2 = 0;
  for (int p = pfirst[j] + lane; p < pfirst[j + 1]; p += 64) s2 += piece_sum[p];
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) s2 += __shfl_xor(s2, m, 64);
  if (lane != 0) return;
  norm2[j] = s2;
  const double nt = sqrt(s2);
  kappa[j] = nt <= eps[j] ? 1.0 : eps[j] / nt;
}

// ||t_j||^2 and kappa_j = min(1, eps_j / ||t_j||) of every section.
int balls_kappa(pr_balls_t* b, const void* t, int prec, hipStream_t st) {
  if (b->npieces > 0) {
    const int G = static_cast<int>(std::min<int64_t>(b->npieces, 8192));
    if (prec == PR_F32)
      section_sq_kernel<float><<<G, kBallThreads, 0, st>>>(static_cast<const float2*>(t), b->order, b->pieces,
                                                           b->npieces, b->piece_sum);
    else
      section_sq_kernel<double><<<G, kBallThreads, 0, st>>>(static_cast<const double2*>(t), b->order, b->pieces,
                                                            b->npieces, b->piece_sum);
    PR_TRY_LAUNCH();
  }
  constexpr int kWaves = kBallThreads / 64;
  section_kappa_kernel<<<(b->nsec + kWaves - 1) / kWaves, kBallThreads, 0, st>>>(b->pfirst, b->piece_sum, b->eps,
                                                                                b->nsec, b->kappa, b->norm2);
  PR_TRY_LAUNCH();
  return PR_OK;
}

// One outer iteration of Algorithm 1 with the local balls.
int local_step(AdmmJob* j, pr_balls_t* b, hipStream_t s) {
  pr_phi_plan_t* phi = j->phi;
  pr_psi_plan_t* psi = j->psi;
  const pr_admm_params& prm = j->prm;
  AdmmWs& w = j->w;
  AdmmVis av{};
  av.y = j->y;
  av.s = w.s;
  av.t = w.t;
  av.sums = w.sums + kSumBall;
  av.eps = INFINITY;             // the global ball is not used; the sums still give ||v - y||
  av.varrho = prm.varrho;
  av.scale_dev = w.sums + kSumScale;
  const double* gamma_dev = j->device_gamma ? w.sums + kSumGamma : nullptr;
  PR_TRY(phi_fzs(phi, j->x, s));
  av.sec = b->section;
  av.sec_partials = b->nsec <= kSecAcc;
  PR_TRY(phi_gw_admm(phi, av, 1.0, s));
  if (av.sec_partials)
    PR_TRY(phi_section_kappa(phi, b->nsec, b->eps, b->kappa, b->norm2, s));
  else
    PR_TRY(balls_kappa(b, w.t, phi->prec, s));
  av.kappa_sec = b->kappa;
  PR_TRY(phi_gw_adjoint_admm(phi, av, 1.0, s));
  PR_TRY(phi_fzs_adjoint_step(phi, j->x, prm.rho, w.xt, w.zbar, s));
  for (int k = 0; k < prm.inner_iters; ++k) {
    PR_TRY(psi_dual_update(psi, w.zbar, 0, w.d, prm.gamma, prm.eta, s, gamma_dev));
    const bool last = k == prm.inner_iters - 1;
    PR_TRY(psi_synthesis_step(psi, w.d, w.xt, last ? j->x : w.zbar, last ? j->x : nullptr, w.partials,
                              w.sums + kSumVar, s));
  }
  ++j->iters_done;
  return PR_OK;
}

}  // namespace
}  // namespace pr

using namespace pr;

extern "C" {

int pr_balls_sizes(int64_t M, int32_t nsec, size_t* persistent_bytes, size_t* scratch_bytes) {
  clear_error();
  PR_NONNULL(persistent_bytes);
  PR_NONNULL(scratch_bytes);
  if (M < 0 || M > kMaxVisibilities) { set_error("M must be in [0, 2^31 - 2^20]"); return PR_EINVAL; }
  if (nsec < 1 || nsec > (1 << 24)) { set_error("nsec must be in [1, 2^24]"); return PR_EINVAL; }
  *persistent_bytes = balls_layout(M, nsec, nullptr, nullptr);
  *scratch_bytes = balls_scratch_layout(M, nsec, nullptr, nullptr);
  return PR_OK;
}

int pr_balls_create(int64_t M, int32_t nsec, const int32_t* section, void* persistent, size_t persistent_bytes,
                    void* scratch, size_t scratch_bytes, void* stream, pr_balls* out) {
  clear_error();
  PR_NONNULL(out);
  *out = nullptr;
  size_t pb = 0, sb = 0;
  PR_TRY(pr_balls_sizes(M, nsec, &pb, &sb));
  if (M > 0 && !section) { set_error("section must not be NULL"); return PR_EINVAL; }
  if (!persistent || !aligned256(persistent) || persistent_bytes < pb || !scratch || !aligned256(scratch) ||
      scratch_bytes < sb) {
    set_error("balls workspaces must be 256-byte aligned and at least %zu / %zu bytes", pb, sb);
    return PR_EWORKSPACE;
  }
  PR_TRY(check_sticky());
  hipStream_t s = as_stream(stream);
  PR_TRY(no_capture(s, "pr_balls_create"));
  BallsLayout L;
  BallsScratch S;
  balls_layout(M, nsec, persistent, &L);
  balls_scratch_layout(M, nsec, scratch, &S);
  zero_flag_kernel<<<1, 1, 0, s>>>(S.bad);
  PR_TRY_LAUNCH();
  uint32_t *kout = S.k0, *vout = S.v0;
  if (M > 0) {
    section_keys_kernel<<<static_cast<unsigned>((M + 255) / 256), 256, 0, s>>>(section, M, nsec, S.k0, S.v0, L.section,
                                                                               S.bad);
    PR_TRY_LAUNCH();
    int bits = 1;
    while ((int64_t(1) << bits) < nsec) ++bits;
    PR_TRY(sort_pairs_u32(S.k0, S.v0, S.k1, S.v1, S.tmp, M, bits, s, &kout, &vout));
    PR_TRY_HIP(hipMemcpyAsync(L.order, vout, M * sizeof(uint32_t), hipMemcpyDeviceToDevice, s));
  }
  section_bounds_kernel<<<(nsec + 1 + 255) / 256, 256, 0, s>>>(kout, M, nsec, S.off);
  PR_TRY_LAUNCH();
  std::vector<int32_t> off(static_cast<size_t>(nsec) + 1);
  int32_t bad = 0;
  PR_TRY_HIP(hipMemcpyAsync(off.data(), S.off, off.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PR_TRY_HIP(hipMemcpyAsync(&bad, S.bad, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  PR_TRY_HIP(hipStreamSynchronize(s));
  if (bad) { set_error("section ids must lie in [0, nsec)"); return PR_EINVAL; }
  std::vector<int4> pieces;
  std::vector<int32_t> pfirst(static_cast<size_t>(nsec) + 1);
  for (int32_t j = 0; j < nsec; ++j) {
    pfirst[j] = static_cast<int32_t>(pieces.size());
    for (int32_t p = off[j]; p < off[j + 1]; p += kPiece)
      pieces.push_back(make_int4(j, p, std::min(p + kPiece, off[j + 1]), 0));
  }
  pfirst[nsec] = static_cast<int32_t>(pieces.size());
  if (static_cast<int64_t>(pieces.size()) > pieces_max(M, nsec)) {
    set_error("internal: piece count exceeds its bound");
    return PR_EINVAL;
  }
  if (!pieces.empty())
    PR_TRY_HIP(hipMemcpyAsync(L.pieces, pieces.data(), pieces.size() * sizeof(int4), hipMemcpyHostToDevice, s));
  PR_TRY_HIP(hipMemcpyAsync(L.pfirst, pfirst.data(), pfirst.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
  PR_TRY_HIP(hipStreamSynchronize(s));
  pr_balls_t* b = new pr_balls_t();
  b->M = M;
  b->nsec = nsec;
  b->section = L.section;
  b->order = L.order;
  b->pieces = L.pieces;
  b->npieces = static_cast<int64_t>(pieces.size());
  b->pfirst = L.pfirst;
  b->piece_sum = L.piece_sum;
  b->eps = L.eps;
  b->kappa = L.kappa;
  b->norm2 = L.norm2;
  PR_TRY_HIP(hipGetDevice(&b->device));
  *out = b;
  return PR_OK;
}

int pr_balls_destroy(pr_balls b) {
  clear_error();
  delete b;
  return PR_OK;
}

int pr_balls_norms(pr_balls b, double* norms, void* stream) {
  clear_error();
  PR_NONNULL(b);
  PR_NONNULL(norms);
  hipStream_t s = as_stream(stream);
  PR_TRY(no_capture(s, "pr_balls_norms"));
  std::vector<double> n2(static_cast<size_t>(b->nsec));
  PR_TRY_HIP(hipMemcpyAsync(n2.data(), b->norm2, n2.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  PR_TRY_HIP(hipStreamSynchronize(s));
  for (int32_t j = 0; j < b->nsec; ++j) norms[j] = std::sqrt(n2[j]);
  return PR_OK;
}

int pr_admm_local_solve(pr_phi_plan phi, pr_psi_plan psi, pr_balls balls, const void* y,
                        const pr_admm_params* params, const double* eps, void* x, void* workspace,
                        pr_admm_report* rep, void* stream) {
  clear_error();
  PR_NONNULL(phi);
  PR_NONNULL(psi);
  PR_NONNULL(balls);
  PR_NONNULL(y);
  PR_NONNULL(params);
  PR_NONNULL(eps);
  PR_NONNULL(x);
  if (!workspace || !aligned256(workspace)) { set_error("workspace must be non-NULL and 256-byte aligned"); return PR_EWORKSPACE; }
  PR_TRY(admm_check_plans(phi, psi));
  if (balls->M != phi->M) { set_error("balls were built for %lld visibilities, the plan has %lld",
                                      static_cast<long long>(balls->M), static_cast<long long>(phi->M)); return PR_EINVAL; }
  for (int32_t j = 0; j < balls->nsec; ++j)
    if (!(eps[j] >= 0)) { set_error("eps[%d] must be >= 0", j); return PR_EINVAL; }
  pr_admm_params prm = *params;
  prm.eps = 1.0;                 // unused (the sections carry the radii); keeps the common check satisfied
  PR_TRY(admm_check_params(&prm));
  PR_TRY(check_sticky());
  hipStream_t s = as_stream(stream);
  PR_TRY(no_capture(s, "pr_admm_local_solve"));
  // the radii go to the device before the call returns (the caller's array may be freed)
  PR_TRY_HIP(hipMemcpyAsync(balls->eps, eps, balls->nsec * sizeof(double), hipMemcpyHostToDevice, s));
  PR_TRY_HIP(hipStreamSynchronize(s));
  AdmmJob j;
  PR_TRY(admm_job_init(&j, phi, psi, y, x, workspace, prm, s));
  PR_TRY(admm_device_setup(&j, s));
  double host_sums[16] = {0};
  for (int it = 0; it < prm.iters; ++it) {
    PR_TRY(local_step(&j, balls, s));
    if (prm.rel_tol > 0) {
      PR_TRY_HIP(hipMemcpyAsync(host_sums, j.w.sums, 16 * sizeof(double), hipMemcpyDeviceToHost, s));
      PR_TRY_HIP(hipStreamSynchronize(s));
      const double rv = host_sums[kSumVar + 1] > 0 ? std::sqrt(host_sums[kSumVar] / host_sums[kSumVar + 1]) : INFINITY;
      if (rv < prm.rel_tol) break;
    }
  }
  if (rep) PR_TRY(admm_report(&j, rep, s));
  return PR_OK;
}

}  // extern "C"
