// Internal state of a SARA dictionary plan (Dirac + Daubechies 1..8, periodic
// orthonormal 2-D wavelets, Mallat layout, scaled by 1/sqrt(nb)).
#pragma once

#include "common.hpp"

struct pr_psi_plan_t {
  int n = 0, levels = 0, prec = PR_F32, nb = 0, ndb = 0;
  uint32_t mask = 0;
  int has_dirac = 0;
  int db_k[8] = {0};               // Daubechies order of the i-th wavelet basis
  double host_filters[9][16] = {{0}};  // low-pass of db k at [k]
  double scale = 1.0;              // 1 / sqrt(nb)

  // persistent: Real[8][2][16] (h, g per wavelet basis, zero padded)
  void* filters = nullptr;
  // scratch, per wavelet basis
  void* rows = nullptr;   // Real[ndb][n*n]   row-pass output
  void* ll_a = nullptr;   // Real[ndb][(n/2)^2]
  void* ll_b = nullptr;   // Real[ndb][(n/2)^2]
  void* recon = nullptr;  // Real[ndb][n*n]   per-basis synthesis
};

namespace pr {

int psi_validate(int n, int levels, uint32_t mask, int prec);
void psi_prepare(pr_psi_plan_t* p, int n, int levels, uint32_t mask, int prec);
int psi_layout(pr_psi_plan_t* p, void* persistent, void* scratch, size_t* persistent_bytes,
               size_t* scratch_bytes);
int psi_create(pr_psi_plan_t* p, hipStream_t s);

// Minimum-phase Daubechies low-pass filter with N vanishing moments (2N taps),
// from spectral factorisation; returns false if the root finder fails.
bool daubechies_filter(int N, double* h);

// alpha = Psi^dagger x; x = Psi alpha.
int psi_analysis(pr_psi_plan_t* p, const void* x, void* alpha, hipStream_t s);
int psi_synthesis(pr_psi_plan_t* p, const void* alpha, void* x, hipStream_t s);

// DualFB steps of Algorithm 1 (fused forms used by the solver):
// d <- (1/eta) clip_gamma(eta d + Psi^dagger zbar), with zbar = max(z, 0) on
// load when `positive_in` is set.
// gamma_dev, when set, holds gamma in device memory and overrides `gamma`.
// weights, when set, hold one real weight per coefficient (the coefficient
// layout): the threshold of coefficient i is gamma * weights[i] (weighted l1).
int psi_dual_update(pr_psi_plan_t* p, const void* zbar, int positive_in, void* d, double gamma, double eta,
                    hipStream_t s, const double* gamma_dev = nullptr, const void* weights = nullptr);
// zbar = max(z - Psi d, 0); optional FP64 partials of ||zbar - xprev||^2 and
// ||zbar||^2 into sums[0], sums[1] (device) when xprev is not null. zbar may
// be xprev (the iterate updated in place).
int psi_synthesis_step(pr_psi_plan_t* p, const void* d, const void* z, void* zbar, const void* xprev,
                       double* partials, double* sums, hipStream_t s);

}  // namespace pr
