// Dual Forward-Backward ADMM (Algorithm 1) driver.
#pragma once

#include "phi.hpp"
#include "psi.hpp"

namespace pr {

int admm_check_plans(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi);
int admm_check_params(const pr_admm_params* prm);
size_t admm_layout(const pr_phi_plan_t* phi, const pr_psi_plan_t* psi, void* ws, struct AdmmWs* out);
int admm_solve(pr_phi_plan_t* phi, pr_psi_plan_t* psi, const void* y, const pr_admm_params& prm, void* x,
               void* ws, pr_admm_report* rep, hipStream_t s);

}  // namespace pr
