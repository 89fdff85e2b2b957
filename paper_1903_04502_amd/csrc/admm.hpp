// Dual Forward-Backward ADMM (Algorithm 1) driver.
#pragma once

#include "phi.hpp"
#include "psi.hpp"

namespace pr {

// Device slots of the FP64 scalar block (AdmmWs::sums).
constexpr int kSumBall = 0;      // 0: ||t||^2, 1: ||v-y||^2, 2: kappa, 3: nonfinite
constexpr int kSumVar = 8;       // 8: ||x_t - x_{t-1}||^2, 9: ||x_t||^2
constexpr int kSumL1 = 12;       // ||Psi^dagger x||_1
constexpr int kSumScale = 16;    // 1 / ||Phi|| when kept on the device
constexpr int kSumGamma = 17;    // gamma when kept on the device
constexpr int kSumGammaStep = 18; // gamma * step, the FISTA prox threshold, on the device
constexpr int kSumIters = 19;    // outer iterations since the first pr_admm_solve (pr_admm_resume continues it)
constexpr int kSumSlots = 32;

struct AdmmWs {
  void *s, *t, *d, *alpha, *xt, *zbar, *xb;
  double* partials;
  double* sums;
};

// One solve's state: plans, data, workspace and parameters. The iterate x is
// updated in place by each step. The scale 1 / ||Phi|| and gamma come from
// the host values unless the device slots are selected (then they are read
// by the kernels from sums[kSumScale] and sums[kSumGamma]).
struct AdmmJob {
  pr_phi_plan_t* phi = nullptr;
  pr_psi_plan_t* psi = nullptr;
  const void* y = nullptr;
  void* x = nullptr;
  AdmmWs w{};
  pr_admm_params prm{};
  double scale = 1.0;
  bool device_scale = false;
  bool device_gamma = false;
  int iters_done = 0;
  const void* l1_weights = nullptr;   // per-coefficient weights of the l1 term (null: all 1)
};

int admm_check_plans(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi);
int admm_check_params(const pr_admm_params* prm);
size_t admm_layout(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi, void* ws, AdmmWs* out);
// Workspace of the accelerated solvers (FISTA, primal-dual): the solver's
// layout followed by the extrapolated image xh (real n*n).
size_t accel_layout(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi, void* ws, AdmmWs* out, void** xh);
// Bind the job and clear its state (s = 0, d = 0, scalars = 0) on the stream.
int admm_job_init(AdmmJob* j, pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* y, void* x, void* ws,
                  const pr_admm_params& prm, hipStream_t s);
// Restart the iteration from the current x: s = 0, d = 0 (1 / ||Phi|| and
// gamma stay in the device slots).
int admm_job_restart(AdmmJob* j, hipStream_t s);
// One outer iteration (with prm.inner_iters DualFB iterations), x in place.
int admm_step(AdmmJob* j, hipStream_t s);
// FP64 diagnostics of the current iterate (synchronises the stream).
int admm_report(AdmmJob* j, pr_admm_report* rep, hipStream_t s);
int admm_solve(pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* y, const pr_admm_params& prm, void* x,
               void* ws, pr_admm_report* rep, hipStream_t s);
// Continue from the state in ws and x (s, d, 1 / ||Phi||, gamma, the count).
int admm_resume(pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* y, const pr_admm_params& prm, void* x,
                void* ws, pr_admm_report* rep, hipStream_t s);
// Checkpoint layout: a header, then x, s, d and the FP64 scalar block.
size_t admm_state_bytes(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi);
int admm_state_export(pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* ws, const void* x, void* state,
                      hipStream_t s);
int admm_state_import(pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* state, void* ws, void* x,
                      hipStream_t s);

// Device-resident set-up after admm_job_init: 1 / ||Phi|| into sums[kSumScale]
// (from prm.op_norm, or the power method with prm.norm_iters steps), and,
// when prm.gamma <= 0, gamma = prm.gamma_factor * ||Psi^dagger Re Phi^dagger y||_inf / ||Phi||
// into sums[kSumGamma]. Asynchronous: nothing is read back to the host.
int admm_device_setup(AdmmJob* j, hipStream_t s);

}  // namespace pr
