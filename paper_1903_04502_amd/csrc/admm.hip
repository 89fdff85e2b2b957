// Algorithm 1 (Dual Forward-Backward ADMM) on one GPU. Each outer iteration
// is a fixed sequence of launches on the caller's stream:
//   F Z S x                                   (2 FFT passes)
//   degrid + epilogue t = v + s - y, FP64 ||t||^2, ||v - y||^2
//   ball scale kappa = min(1, eps / ||t||)    (one-block FP64 reduction)
//   gridding with the prologue r = y + kappa t, s <- s + varrho (v - r),
//     q = v - r + s, then the patch merge
//   S Z^T F^H with the epilogue xt = x - rho Re(.), zbar = max(xt, 0)
//   DualFB: d <- (1/eta) clip_gamma(eta d + Psi^dagger zbar) fused into the
//     analysis stores; zbar = max(xt - Psi d, 0) fused into the synthesis sum
// Phi enters divided by ||Phi|| (folded into the per-visibility weight scale).
// The iterate is updated in place. Nothing is read back to the host unless a
// report or a tolerance asks for it.
#include <cmath>
#include <cstring>

#include "admm.hpp"
#include "ops.hpp"

namespace pr {

namespace {

template <typename R>
__global__ void zero_kernel(R* a, int64_t len) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < len;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    a[i] = R(0);
}

__global__ void set_scalar_kernel(double* a, double v) { *a = v; }

__global__ void add_scalar_kernel(double* a, double v) { *a += v; }

__global__ void zero_f64_kernel(double* a, int len) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < len) a[i] = 0.0;
}

int zero_real(void* a, int64_t len, int prec, hipStream_t s) {
  const int G = grid_for(len, 256, 8192);
  if (prec == PR_F32) zero_kernel<float><<<G, 256, 0, s>>>(static_cast<float*>(a), len);
  else zero_kernel<double><<<G, 256, 0, s>>>(static_cast<double*>(a), len);
  PR_TRY_LAUNCH();
  return PR_OK;
}

}  // namespace

int admm_check_plans(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi) {
  if (phi->n != psi->n) { set_error("Phi plan n = %d but Psi plan n = %d", phi->n, psi->n); return PR_EINVAL; }
  if (phi->prec != psi->prec) { set_error("Phi and Psi plans differ in precision"); return PR_EINVAL; }
  if (phi->M < 1) { set_error("ADMM needs M >= 1"); return PR_EINVAL; }
  return PR_OK;
}

int admm_check_params(const pr_admm_params* p) {
  if (p->iters < 0) { set_error("iters < 0"); return PR_EINVAL; }
  if (p->inner_iters < 1) { set_error("inner_iters < 1"); return PR_EINVAL; }
  if (!(p->eps >= 0)) { set_error("eps must be >= 0"); return PR_EINVAL; }
  if (!(p->gamma > 0) && !(p->gamma_factor > 0)) {
    set_error("gamma must be > 0, or gamma <= 0 with gamma_factor > 0");
    return PR_EINVAL;
  }
  if (!(p->rho > 0) || !(p->varrho > 0) || !(p->eta > 0)) { set_error("rho, varrho, eta must be > 0"); return PR_EINVAL; }
  if (!(p->rel_tol >= 0)) { set_error("rel_tol must be >= 0"); return PR_EINVAL; }
  return PR_OK;
}

size_t admm_layout(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi, void* ws, AdmmWs* out) {
  const size_t rs = phi->prec == PR_F32 ? 4 : 8;
  const int64_t n2 = static_cast<int64_t>(phi->n) * phi->n;
  Carver c(ws);
  AdmmWs w{};
  w.s = c.take<char>(phi->M * 2 * rs);
  w.t = c.take<char>(phi->M * 2 * rs);
  w.d = c.take<char>(psi->nb * n2 * rs);
  w.alpha = c.take<char>(psi->nb * n2 * rs);
  w.xt = c.take<char>(n2 * rs);
  w.zbar = c.take<char>(n2 * rs);
  w.xb = c.take<char>(n2 * rs);
  w.partials = c.take<double>(2 * kPartialsMax);
  w.sums = c.take<double>(32);
  if (out) *out = w;
  return c.bytes();
}

size_t accel_layout(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi, void* ws, AdmmWs* out, void** xh) {
  const size_t base = admm_layout(phi, psi, ws, out);
  const size_t rs = phi->prec == PR_F32 ? 4 : 8;
  const size_t extra = (static_cast<size_t>(phi->n) * phi->n * rs + 255) & ~size_t(255);
  if (xh) *xh = ws ? static_cast<char*>(ws) + base : nullptr;
  return base + extra;
}

int admm_job_init(AdmmJob* j, pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* y, void* x, void* ws,
                  const pr_admm_params& prm, hipStream_t s) {
  j->phi = phi;
  j->psi = psi;
  j->y = y;
  j->x = x;
  j->prm = prm;
  j->iters_done = 0;
  j->device_scale = j->device_gamma = false;
  j->scale = prm.op_norm > 0 ? 1.0 / prm.op_norm : 1.0;
  admm_layout(phi, psi, ws, &j->w);
  const int64_t n2 = static_cast<int64_t>(phi->n) * phi->n;
  PR_TRY(zero_real(j->w.s, 2 * phi->M, phi->prec, s));
  PR_TRY(zero_real(j->w.d, psi->nb * n2, phi->prec, s));
  zero_f64_kernel<<<1, kSumSlots, 0, s>>>(j->w.sums, kSumSlots);
  PR_TRY_LAUNCH();
  return PR_OK;
}

int admm_job_restart(AdmmJob* j, hipStream_t s) {
  const int64_t n2 = static_cast<int64_t>(j->phi->n) * j->phi->n;
  PR_TRY(zero_real(j->w.s, 2 * j->phi->M, j->phi->prec, s));
  PR_TRY(zero_real(j->w.d, j->psi->nb * n2, j->phi->prec, s));
  return PR_OK;
}

int admm_step(AdmmJob* j, hipStream_t s) {
  pr_phi_plan_t* phi = j->phi;
  pr_psi_plan_t* psi = j->psi;
  const pr_admm_params& prm = j->prm;
  AdmmWs& w = j->w;
  AdmmVis av{};
  av.y = j->y;
  av.s = w.s;
  av.t = w.t;
  av.sums = w.sums + kSumBall;
  av.eps = prm.eps;
  av.varrho = prm.varrho;
  av.scale_dev = j->device_scale ? w.sums + kSumScale : nullptr;
  const double* gamma_dev = j->device_gamma ? w.sums + kSumGamma : nullptr;
  PR_TRY(phi_fzs(phi, j->x, s));
  PR_TRY(phi_gw_admm(phi, av, j->scale, s));
  PR_TRY(phi_gw_adjoint_admm(phi, av, j->scale, s));
  PR_TRY(phi_fzs_adjoint_step(phi, j->x, prm.rho, w.xt, w.zbar, s));
  for (int k = 0; k < prm.inner_iters; ++k) {
    PR_TRY(psi_dual_update(psi, w.zbar, 0, w.d, prm.gamma, prm.eta, s, gamma_dev, j->l1_weights));
    const bool last = k == prm.inner_iters - 1;
    // the last synthesis writes the new iterate over x (read before written)
    void* out = last ? j->x : w.zbar;
    PR_TRY(psi_synthesis_step(psi, w.d, w.xt, out, last ? j->x : nullptr, w.partials, w.sums + kSumVar, s));
  }
  ++j->iters_done;
  return PR_OK;
}

int admm_report(AdmmJob* j, pr_admm_report* rep, hipStream_t s) {
  PR_TRY(no_capture(s, "the report"));
  pr_phi_plan_t* phi = j->phi;
  pr_psi_plan_t* psi = j->psi;
  const int64_t n2 = static_cast<int64_t>(phi->n) * phi->n;
  double host_sums[kSumSlots] = {0};
  PR_TRY(psi_analysis(psi, j->x, j->w.alpha, s));
  PR_TRY(reduce_abssum(j->w.alpha, psi->nb * n2, phi->prec, j->w.partials, j->w.sums + kSumL1, s));
  PR_TRY_HIP(hipMemcpyAsync(host_sums, j->w.sums, kSumSlots * sizeof(double), hipMemcpyDeviceToHost, s));
  PR_TRY_HIP(hipStreamSynchronize(s));
  rep->iters_done = j->iters_done;
  rep->rel_var = host_sums[kSumVar + 1] > 0 ? std::sqrt(host_sums[kSumVar] / host_sums[kSumVar + 1]) : INFINITY;
  rep->resid_norm = std::sqrt(host_sums[kSumBall + 1]);
  rep->l1_norm = host_sums[kSumL1];
  rep->op_norm = j->device_scale ? 1.0 / host_sums[kSumScale] : 1.0 / j->scale;
  rep->nonfinite = (host_sums[kSumBall + 3] != 0 || !std::isfinite(rep->rel_var) || !std::isfinite(rep->l1_norm) ||
                    !std::isfinite(rep->resid_norm))
                       ? 1
                       : 0;
  return PR_OK;
}

int admm_device_setup(AdmmJob* j, hipStream_t s) {
  pr_phi_plan_t* phi = j->phi;
  const pr_admm_params& prm = j->prm;
  const int64_t n2 = static_cast<int64_t>(phi->n) * phi->n;
  double* inv = j->w.sums + kSumScale;
  if (prm.op_norm > 0) {
    set_scalar_kernel<<<1, 1, 0, s>>>(inv, 1.0 / prm.op_norm);
    PR_TRY_LAUNCH();
  } else {
    PR_TRY(phi_norm_device(phi, prm.norm_iters > 0 ? prm.norm_iters : 100, j->w.t, inv, s));
  }
  j->device_scale = true;
  if (!(prm.gamma > 0)) {
    // gamma = factor * ||Psi^dagger Re Phi^dagger y||_inf / ||Phi|| (dirty image of the normalised operator)
    PR_TRY(phi_gw_adjoint(phi, j->y, 1.0, s));
    PR_TRY(phi_fzs_adjoint(phi, j->w.xt, s));
    PR_TRY(psi_analysis(j->psi, j->w.xt, j->w.alpha, s));
    PR_TRY(reduce_absmax_scaled(j->w.alpha, j->psi->nb * n2, phi->prec, prm.gamma_factor, inv, j->w.partials,
                                j->w.sums + kSumGamma, s));
    j->device_gamma = true;
  }
  return PR_OK;
}

namespace {

// The outer loop shared by a fresh solve and a resumed one: prm.iters steps
// (or fewer once the relative change drops below rel_tol), then the device
// iteration count advances by the steps taken.
int admm_run(AdmmJob& j, const pr_admm_params& prm, pr_admm_report* rep, hipStream_t s) {
  if (prm.rel_tol > 0 || rep) PR_TRY(no_capture(s, "an ADMM solve with rel_tol or a report"));
  double host_sums[kSumSlots] = {0};
  const int start = j.iters_done;
  for (int it = 0; it < prm.iters; ++it) {
    PR_TRY(admm_step(&j, s));
    if (prm.rel_tol > 0) {
      PR_TRY_HIP(hipMemcpyAsync(host_sums, j.w.sums, kSumSlots * sizeof(double), hipMemcpyDeviceToHost, s));
      PR_TRY_HIP(hipStreamSynchronize(s));
      const double rv = host_sums[kSumVar + 1] > 0 ? std::sqrt(host_sums[kSumVar] / host_sums[kSumVar + 1]) : INFINITY;
      if (rv < prm.rel_tol) break;
    }
  }
  add_scalar_kernel<<<1, 1, 0, s>>>(j.w.sums + kSumIters, static_cast<double>(j.iters_done - start));
  PR_TRY_LAUNCH();
  if (rep) {
    PR_TRY(admm_report(&j, rep, s));
    double cnt = 0;
    PR_TRY_HIP(hipMemcpyAsync(&cnt, j.w.sums + kSumIters, sizeof(double), hipMemcpyDeviceToHost, s));
    PR_TRY_HIP(hipStreamSynchronize(s));
    rep->iters_done = static_cast<int32_t>(cnt);
  }
  return PR_OK;
}

// Checkpoint header (the first 256 bytes of a state buffer).
struct StateHeader {
  uint32_t magic;      // 'P' 'R' 'S' 'T'
  uint32_t version;
  int32_t prec, n, nb, levels;
  int64_t M;
  uint32_t basis_mask;
  int32_t slots;
};
constexpr uint32_t kStateMagic = 0x54535250u;
constexpr size_t kStateHead = 256;

struct StateParts {
  size_t x, s, d, sums, total;
};

StateParts state_parts(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi) {
  const size_t rs = phi->prec == PR_F32 ? 4 : 8;
  const size_t n2 = static_cast<size_t>(phi->n) * phi->n;
  auto up = [](size_t v) { return (v + 255) & ~size_t(255); };
  StateParts p{};
  p.x = kStateHead;
  p.s = p.x + up(n2 * rs);
  p.d = p.s + up(static_cast<size_t>(phi->M) * 2 * rs);
  p.sums = p.d + up(static_cast<size_t>(psi->nb) * n2 * rs);
  p.total = p.sums + up(kSumSlots * sizeof(double));
  return p;
}

StateHeader state_header(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi) {
  StateHeader h{};
  h.magic = kStateMagic;
  h.version = 1;
  h.prec = phi->prec;
  h.n = phi->n;
  h.nb = psi->nb;
  h.levels = psi->levels;
  h.M = phi->M;
  h.basis_mask = psi->mask;
  h.slots = kSumSlots;
  return h;
}

}  // namespace

int admm_solve(pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* y, const pr_admm_params& prm, void* x, void* ws,
               pr_admm_report* rep, hipStream_t s) {
  AdmmJob j;
  PR_TRY(admm_job_init(&j, phi, psi, y, x, ws, prm, s));
  PR_TRY(admm_device_setup(&j, s));
  return admm_run(j, prm, rep, s);
}

int admm_resume(pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* y, const pr_admm_params& prm, void* x, void* ws,
                pr_admm_report* rep, hipStream_t s) {
  AdmmJob j;
  j.phi = phi;
  j.psi = psi;
  j.y = y;
  j.x = x;
  j.prm = prm;
  j.iters_done = 0;
  admm_layout(phi, psi, ws, &j.w);
  // 1 / ||Phi|| always, and gamma unless the caller fixes it, come from the
  // device slots the first solve filled
  j.device_scale = true;
  j.device_gamma = !(prm.gamma > 0);
  return admm_run(j, prm, rep, s);
}

size_t admm_state_bytes(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi) { return state_parts(phi, psi).total; }

int admm_state_export(pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* ws, const void* x, void* state,
                      hipStream_t s) {
  PR_TRY(no_capture(s, "pr_admm_state_export"));
  AdmmWs w{};
  admm_layout(phi, psi, const_cast<void*>(ws), &w);
  const StateParts p = state_parts(phi, psi);
  const size_t rs = phi->prec == PR_F32 ? 4 : 8;
  const size_t n2 = static_cast<size_t>(phi->n) * phi->n;
  char* dst = static_cast<char*>(state);
  const StateHeader h = state_header(phi, psi);
  PR_TRY_HIP(hipMemcpyAsync(dst, &h, sizeof h, hipMemcpyDefault, s));
  PR_TRY_HIP(hipMemcpyAsync(dst + p.x, x, n2 * rs, hipMemcpyDefault, s));
  PR_TRY_HIP(hipMemcpyAsync(dst + p.s, w.s, static_cast<size_t>(phi->M) * 2 * rs, hipMemcpyDefault, s));
  PR_TRY_HIP(hipMemcpyAsync(dst + p.d, w.d, static_cast<size_t>(psi->nb) * n2 * rs, hipMemcpyDefault, s));
  PR_TRY_HIP(hipMemcpyAsync(dst + p.sums, w.sums, kSumSlots * sizeof(double), hipMemcpyDefault, s));
  PR_TRY_HIP(hipStreamSynchronize(s));   // the header lives on this call's stack
  return PR_OK;
}

int admm_state_import(pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* state, void* ws, void* x,
                      hipStream_t s) {
  PR_TRY(no_capture(s, "pr_admm_state_import"));
  const char* src = static_cast<const char*>(state);
  StateHeader h{};
  PR_TRY_HIP(hipMemcpyAsync(&h, src, sizeof h, hipMemcpyDefault, s));
  PR_TRY_HIP(hipStreamSynchronize(s));
  const StateHeader want = state_header(phi, psi);
  if (h.magic != kStateMagic || h.version != want.version) {
    set_error("state buffer does not hold an ADMM checkpoint");
    return PR_EINVAL;
  }
  if (h.prec != want.prec || h.n != want.n || h.nb != want.nb || h.levels != want.levels || h.M != want.M ||
      h.basis_mask != want.basis_mask || h.slots != want.slots) {
    set_error("checkpoint was made for other plans (n %d, M %lld, bases %d, levels %d, prec %d)", h.n,
              static_cast<long long>(h.M), h.nb, h.levels, h.prec);
    return PR_EINVAL;
  }
  AdmmWs w{};
  admm_layout(phi, psi, ws, &w);
  const StateParts p = state_parts(phi, psi);
  const size_t rs = phi->prec == PR_F32 ? 4 : 8;
  const size_t n2 = static_cast<size_t>(phi->n) * phi->n;
  PR_TRY_HIP(hipMemcpyAsync(x, src + p.x, n2 * rs, hipMemcpyDefault, s));
  PR_TRY_HIP(hipMemcpyAsync(w.s, src + p.s, static_cast<size_t>(phi->M) * 2 * rs, hipMemcpyDefault, s));
  PR_TRY_HIP(hipMemcpyAsync(w.d, src + p.d, static_cast<size_t>(psi->nb) * n2 * rs, hipMemcpyDefault, s));
  PR_TRY_HIP(hipMemcpyAsync(w.sums, src + p.sums, kSumSlots * sizeof(double), hipMemcpyDefault, s));
  PR_TRY_HIP(hipStreamSynchronize(s));
  return PR_OK;
}

}  // namespace pr
