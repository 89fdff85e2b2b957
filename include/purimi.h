/*
 * purimi.h -- C ABI of the MI355X (gfx950) library for the sparse radio
 * interferometric imaging path of Pratley et al., "Distributed and parallel
 * sparse convex optimization for radio interferometry with PURIFY".
 *
 * The library computes, on one GPU:
 *   Phi = W G F Z S           measurement operator, eq. (matrix_equation)
 *   Phi^dagger                its adjoint (dirty map), same section
 *   Psi, Psi^dagger           SARA dictionary: Dirac + Daubechies 1..8
 *                             (Sections "Analysis and Synthesis" and
 *                             "MPI Wavelet Operator Benchmarks")
 *   S_lambda                  soft thresholding (Section "Promoting Sparsity")
 *   P_B                       l2-ball projection (eq. l2ball_prox)
 *   Algorithm 1               Dual Forward-Backward ADMM
 *
 * Conventions shared by every call
 *   - Array arguments are DEVICE pointers owned by the caller, unless stated
 *     as host. Element type follows the precision: PR_F32 -> float and
 *     complex float (two floats, re then im); PR_F64 -> double and complex
 *     double. Arrays are contiguous.
 *   - Image x: real, n*n values, row-major x[iy*n + ix]; the centred pixel
 *     offsets are p_x = ix - n/2 (pairs with u) and p_y = iy - n/2 (pairs
 *     with v).
 *   - Visibilities: complex, M values. Baselines uv: M pairs (u, v) of the
 *     precision's real type, in radians per pixel, each in [-pi, pi).
 *   - stream: a hipStream_t passed as void* (NULL = the null stream). Every
 *     call only enqueues work on it and returns, unless its comment says it
 *     synchronises. Kernel faults surface at the caller's next
 *     synchronisation and as PR_EHIP from the next call.
 *   - Workspaces: the library allocates no device memory. Each plan reports
 *     the bytes it needs (persistent: kept for the plan's life; scratch:
 *     reused by every call on the plan) and the caller passes them in,
 *     256-byte aligned. Calls on one plan must be ordered on one stream.
 *   - Return value: PR_OK or an error code; pr_last_error() gives a message
 *     (thread-local). On error nothing has been enqueued.
 */
#ifndef PURIMI_H
#define PURIMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PR_OK 0
#define PR_EINVAL 1        /* invalid argument (shape, null pointer, range)  */
#define PR_EWORKSPACE 2    /* workspace pointer missing or misaligned         */
#define PR_EHIP 3          /* a HIP runtime call failed                        */
#define PR_EUNSUPPORTED 4  /* valid request outside what this library supports */

#define PR_F32 0
#define PR_F64 1

/* Text of the last error on this thread ("" if none). */
const char* pr_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int pr_version(void);

/* ------------------------------------------------------------------------
 * Measurement operator Phi = W G F Z S (eq. matrix_equation).
 *   S: gridding correction, divides pixel p by the Kaiser-Bessel kernel's
 *      Fourier transform at p/K;
 *   Z: zero padding of the n x n image to the K x K grid, K = oversample*n,
 *      pixel p placed at grid index p mod K;
 *   F: unnormalised 2-D FFT, sign e^{-2 pi i (.)} as in eq. (meas_eq);
 *   G: interpolation off the grid with the Kaiser-Bessel kernel of support
 *      J, pre-sampled at D samples per grid cell on 0 <= |t| <= J/2 and read
 *      by nearest sample (Section "Kernel Pre-Sampling"). A visibility at
 *      grid coordinate s = u K / (2 pi) (FP64) uses cells
 *      floor(s) - J/2 + 1 + a, a = 0..J-1 (mod K), and for tap a the sample
 *      nearest to |s - cell| * D, ties to the larger distance;
 *   W: real per-visibility weights.
 * Visibility arrays passed to phi_* calls are in PLAN ORDER: the plan sorts
 * the visibilities by grid tile; pr_phi_plan_perm gives the permutation.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t n;          /* image side; power of two, 8 <= n <= 4096           */
  int32_t oversample; /* K = oversample * n; must be 2                      */
  int32_t J;          /* kernel support: 2, 4, 6 or 8                       */
  int32_t D;          /* table samples per grid cell, 1 <= D <= 1000000     */
  int64_t M;          /* visibilities, 0 <= M <= 2^31 - 2^20 (positions and
                         the permutation are int32; every product with a
                         position is formed in 64 bits). Largest count run
                         on the GPU: see the tests of the 2048^2 share.     */
  int32_t prec;       /* PR_F32 or PR_F64                                    */
  int32_t tile;       /* tile side in grid cells: 0 = default, else 8/16/32  */
  int32_t interp;     /* kernel lookup (Section "Kernel Pre-Sampling"):
                         0 = nearest sample (zeroth order), 1 = linear
                         between the two samples around the tap distance
                         (first order), 2 = nearest sample with the taps
                         recomputed from (u, v) in every launch. With 0, an
                         FP32 plan whose tile is at most 16 cells and whose
                         D is at most 2047 stores, per visibility, the
                         sample indices of its taps (32 bits) beside w
                         instead of (u, v, w): the same samples, so results
                         equal to those of 2 bitwise; other plans keep the
                         triples. Any other value: PR_EINVAL.              */
} pr_phi_desc;

typedef struct pr_phi_plan_t* pr_phi_plan;

/* Workspace bytes a plan for *desc needs. Host only, no GPU call. */
int pr_phi_plan_sizes(const pr_phi_desc* desc, size_t* persistent_bytes,
                      size_t* scratch_bytes);

/* Build a plan: the kernel table, correction and FFT twiddles (computed on
 * the GPU in FP64), the tile sort of the visibilities and the gridding work
 * list. uv: M (u,v) pairs in user order; w: M real weights or NULL for 1.
 * Synchronises the stream once (to read the work-list length). The plan
 * keeps its own sorted copy of uv and w in the persistent workspace. */
int pr_phi_plan_create(const pr_phi_desc* desc, const void* uv, const void* w,
                       void* persistent_ws, void* scratch_ws, void* stream,
                       pr_phi_plan* out);

/* Release the host-side plan object (the caller frees the workspaces). */
int pr_phi_plan_destroy(pr_phi_plan plan);

/* Device pointer to int32 perm[M]: plan position k holds user visibility
 * perm[k] (y_plan[k] = y_user[perm[k]]). Valid for the plan's lifetime. */
int pr_phi_plan_perm(pr_phi_plan plan, const int32_t** perm);

/* Copy the permutation into the caller's device buffer dst (int32[M]),
 * enqueued on stream. */
int pr_phi_plan_perm_copy(pr_phi_plan plan, int32_t* dst, void* stream);

/* Number of gridding work items (tile chunks) the plan built. Host only. */
int pr_phi_plan_items(pr_phi_plan plan, int64_t* items);

/* y = Phi x. x: real[n*n]; y: complex[M] in plan order. */
int pr_phi_apply(pr_phi_plan plan, const void* x, void* y, void* stream);

/* x = Re(Phi^dagger y), the adjoint of Phi on real images (dirty map for
 * weighted data y). y: complex[M] in plan order; x: real[n*n]. */
int pr_phi_adjoint(pr_phi_plan plan, const void* y, void* x, void* stream);

/* The two factors of Phi, for timing and for callers that keep the grid:
 * pr_phi_fzs:         plan grid = F Z S x
 * pr_phi_gw:          y = W G (plan grid)
 * pr_phi_gw_adjoint:  plan grid = G^T W y   (deterministic binned gridding)
 * pr_phi_fzs_adjoint: x = Re(S Z^T F^H plan grid)
 * pr_phi_apply == fzs then gw; pr_phi_adjoint == gw_adjoint then fzs_adjoint. */
int pr_phi_fzs(pr_phi_plan plan, const void* x, void* stream);
int pr_phi_gw(pr_phi_plan plan, void* y, void* stream);
int pr_phi_gw_adjoint(pr_phi_plan plan, const void* y, void* stream);
int pr_phi_fzs_adjoint(pr_phi_plan plan, void* x, void* stream);
/* pr_phi_gw_adjoint in its two launches: per-work-item grid patches from the
 * visibilities (each patch written once, no atomics), then the fixed-order
 * merge of the up to four overlapping patches of every grid cell. */
int pr_phi_grid_patches(pr_phi_plan plan, const void* y, void* stream);
int pr_phi_grid_merge(pr_phi_plan plan, void* stream);

/* Operator norm ||Phi|| by the power method on Re Phi^dagger Phi (Section
 * "Distributed Images"): x0 = constant image of unit norm, x <- A x / ||A x||
 * (norms in FP64), at most iters steps, result sqrt(||A x||) written to *norm
 * (host). rtol > 0: stop after step k once |l_k - l_{k-1}| <= rtol l_k, with
 * l_k = ||A x|| of step k (reads l_k back after every step); rtol = 0: exactly
 * iters steps, fully on the device until the final read. vis_ws: device
 * scratch of M complex values. Synchronises the stream. PR_EINVAL for
 * iters < 1 or rtol < 0. */
int pr_phi_norm(pr_phi_plan plan, int32_t iters, double rtol, void* vis_ws,
                double* norm, void* stream);

/* Tile-side autotuner: for each admissible tile side (8, 16, 32; desc->tile
 * is ignored) build the plan into the given workspaces and time `reps`
 * (Phi, Phi^dagger) pairs with HIP events on `stream` after one untimed pair.
 * *best_tile receives the fastest side, *best_ms (nullable) its time per pair.
 * Workspaces must hold the largest candidate (pr_phi_plan_sizes per side);
 * vis_ws: device complex[M]. Synchronises the stream; the workspaces hold no
 * usable plan afterwards. */
int pr_phi_tune(const pr_phi_desc* desc, const void* uv, const void* w,
                void* persistent_ws, void* scratch_ws, void* vis_ws,
                int32_t reps, void* stream, int32_t* best_tile,
                double* best_ms);

/* ------------------------------------------------------------------------
 * SARA dictionary (Sections "Analysis and Synthesis", "Distributed Wavelet
 * Operator"): bases selected by basis_mask (bit 0 Dirac, bit k = Daubechies
 * k, k = 1..8); each Daubechies basis is the periodic, orthonormal 2-D
 * separable transform to `levels` levels (Mallat layout: rows then columns
 * of the current low-low block, low half first), with the minimum-phase dbk
 * filter. The dictionary is scaled by 1/sqrt(nb) (nb = bases selected) so
 * Psi Psi^dagger = I.
 *   alpha: real[nb][n*n], bases in increasing bit order.
 * ---------------------------------------------------------------------- */
typedef struct pr_psi_plan_t* pr_psi_plan;

int pr_psi_plan_sizes(int32_t n, int32_t levels, uint32_t basis_mask, int32_t prec,
                      size_t* persistent_bytes, size_t* scratch_bytes);
/* Derives the Daubechies filters (host, FP64 spectral factorisation) and
 * uploads them. Does not synchronise. */
int pr_psi_plan_create(int32_t n, int32_t levels, uint32_t basis_mask, int32_t prec,
                       void* persistent_ws, void* scratch_ws, void* stream,
                       pr_psi_plan* out);
int pr_psi_plan_destroy(pr_psi_plan plan);
/* Number of bases nb selected by the plan's mask. Host only. */
int pr_psi_plan_bases(pr_psi_plan plan, int32_t* nb);
/* Filter taps of Daubechies basis k (1..8), 2k values, host FP64 copy. */
int pr_psi_filter(pr_psi_plan plan, int32_t k, double* taps);

/* x = Psi alpha (synthesis). */
int pr_psi_apply(pr_psi_plan plan, const void* alpha, void* x, void* stream);
/* alpha = Psi^dagger x (analysis). */
int pr_psi_adjoint(pr_psi_plan plan, const void* x, void* alpha, void* stream);

/* ------------------------------------------------------------------------
 * Proximal operators (Section "Proximal Operators").
 * ---------------------------------------------------------------------- */
/* out = S_lambda(in): 0 where |in_i| <= lambda, else in_i (|in_i| - lambda)
 * / |in_i|. len elements, real or complex (is_complex != 0). in == out is
 * allowed. */
int pr_prox_l1(const void* in, void* out, int64_t len, int32_t is_complex,
               int32_t prec, double lambda, void* stream);

/* Device scratch bytes pr_proj_l2ball needs for len complex elements. */
size_t pr_proj_l2ball_scratch_bytes(int64_t len);

/* out = P_B(in) for the closed ball of radius eps centred at center
 * (eq. l2ball_prox): in if ||in - center|| <= eps, else
 * center + eps (in - center) / ||in - center||. len complex elements; the
 * norm is reduced in FP64 in a fixed order (bitwise reproducible). dist: if
 * not NULL, ||in - center|| is written to this HOST pointer and the call
 * synchronises the stream. in == out is allowed. */
int pr_proj_l2ball(const void* in, const void* center, void* out, int64_t len,
                   int32_t prec, double eps, void* scratch, double* dist,
                   void* stream);

/* pr_proj_l2ball without the scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation). The FP64 partial sums live in a static
 * device array of the library (16 KB per GPU, held until the process ends;
 * its address is looked up once per device on the first call there). It
 * allocates nothing; every length the library accepts fits (the scratch does
 * not grow with len). Calls that overlap on one GPU (other streams or host
 * threads) share the array and race: serialise them. Same arguments, result
 * bits and errors as pr_proj_l2ball; PR_EUNSUPPORTED for device ids >= 64. */
int pr_proj_l2ball_noalloc(const void* in, const void* center, void* out,
                           int64_t len, int32_t prec, double eps, double* dist,
                           void* stream);

/* ------------------------------------------------------------------------
 * Dual Forward-Backward ADMM (Algorithm 1) for
 *   min ||Psi^dagger x||_1 + iota_{R+}(x) + iota_{||Phi x - y|| <= eps}
 * with Phi normalised by op_norm: each outer iteration
 *   v = Phi x / ||Phi||; r = P_B(v + s); s <- s + varrho (v - r);
 *   xt = x - rho Phi^dagger (v - r + s) / ||Phi||; x = DualFB(xt, gamma),
 * DualFB: zbar = max(xt, 0); repeat inner_iters times
 *   d <- (1/eta) (I - S_gamma)(eta d + Psi^dagger zbar); zbar = max(xt - Psi d, 0).
 * s and d start at 0 (d carried across outer iterations). The l2 norm of the
 * ball test and the diagnostics are reduced in FP64.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t iters;       /* outer iterations (>= 0)                            */
  int32_t inner_iters; /* DualFB iterations per outer iteration (>= 1)       */
  double eps;          /* l2-ball radius                                     */
  double gamma;        /* soft-threshold level (> 0)                         */
  double rho;          /* gradient step                                      */
  double varrho;       /* dual (Lagrange multiplier) step                    */
  double eta;          /* DualFB step                                        */
  double rel_tol;      /* > 0: stop when ||x_t - x_{t-1}|| / ||x_t|| < rel_tol
                          (synchronises every iteration); 0: fixed count    */
  double op_norm;      /* ||Phi||; <= 0: power method on the device (below)  */
  double gamma_factor; /* used when gamma <= 0: gamma = gamma_factor *
                          ||Psi^dagger Re Phi^dagger y||_inf / ||Phi||, formed
                          on the device (must then be > 0)                   */
  int32_t norm_iters;  /* power-method steps when op_norm <= 0 (<= 0: 100)   */
} pr_admm_params;

typedef struct {
  int32_t iters_done;
  double rel_var;      /* ||x_t - x_{t-1}|| / ||x_t|| of the last iteration  */
  double resid_norm;   /* ||Phi x_{t-1} / ||Phi|| - y|| of the last iteration */
  double l1_norm;      /* ||Psi^dagger x|| _1 of the returned x               */
  double op_norm;      /* the ||Phi|| used                                    */
  int32_t nonfinite;   /* 1 if a NaN or Inf reached a reduction               */
} pr_admm_report;

/* Device workspace bytes for pr_admm_solve on these plans. */
int pr_admm_workspace_size(pr_phi_plan phi, pr_psi_plan psi, size_t* bytes);

/* Run Algorithm 1. y: complex[M], plan order. x: real[n*n], in: x0, out:
 * the last iterate (in units of the normalised operator: the physical image
 * is x / ||Phi||), updated in place. 1 / ||Phi||, gamma and the iteration
 * count are kept in the workspace on the device (see pr_admm_resume). rep: if
 * not NULL, filled on return and the call synchronises; if NULL and
 * rel_tol == 0 the call is fully asynchronous. The two plans must have the
 * same n and precision. */
int pr_admm_solve(pr_phi_plan phi, pr_psi_plan psi, const void* y,
                  const pr_admm_params* params, void* x, void* workspace,
                  pr_admm_report* rep, void* stream);

/* Checkpoint and resume of Algorithm 1 (the state of its iteration: the
 * iterate x, the Lagrange multiplier s, the DualFB dual variable d, the
 * scalars 1 / ||Phi|| and gamma, and the outer iteration count).
 *
 * pr_admm_state_bytes: size of a checkpoint for these plans (a 256-byte
 * header, then x, s, d and the FP64 scalar block, each 256-byte aligned).
 *
 * pr_admm_state_export: copy x and the state held in `workspace` (as left by
 * pr_admm_solve or pr_admm_resume on the same plans) into `state`, host or
 * device memory of pr_admm_state_bytes bytes owned by the caller.
 * Synchronises the stream.
 *
 * pr_admm_state_import: restore a checkpoint into `workspace` (of
 * pr_admm_workspace_size bytes for these plans) and x. PR_EINVAL if `state`
 * holds no checkpoint or one made for plans of another n, M, precision or
 * dictionary. Synchronises the stream.
 *
 * pr_admm_resume: params->iters more outer iterations of Algorithm 1 from the
 * state in `workspace` and x, without clearing s and d; 1 / ||Phi|| comes from
 * the workspace (params->op_norm, norm_iters and gamma_factor are ignored),
 * and gamma too when params->gamma <= 0. The kernels and their order are
 * those of pr_admm_solve, so solve(k) then resume(m) -- also through an
 * export and an import into another workspace -- gives bitwise the x of
 * solve(k + m). rep->iters_done counts every iteration since the solve. */
int pr_admm_state_bytes(pr_phi_plan phi, pr_psi_plan psi, size_t* bytes);
int pr_admm_state_export(pr_phi_plan phi, pr_psi_plan psi, const void* workspace,
                         const void* x, void* state, void* stream);
int pr_admm_state_import(pr_phi_plan phi, pr_psi_plan psi, const void* state,
                         void* workspace, void* x, void* stream);
int pr_admm_resume(pr_phi_plan phi, pr_psi_plan psi, const void* y,
                   const pr_admm_params* params, void* x, void* workspace,
                   pr_admm_report* rep, void* stream);

/* ------------------------------------------------------------------------
 * Reweighted analysis l1 (SARA reweighting; Section "Sparse Regularization"
 * names the reweighted re-solves, without a weight rule). Round 0 is
 * pr_admm_solve; each further round r sets
 *   w_i = delta / (delta + |[Psi^dagger x]_i|),  delta = delta0 beta^(r-1),
 * from the current x and runs params->iters iterations of Algorithm 1 with
 * the weighted norm sum_i w_i |[Psi^dagger x]_i| (DualFB thresholds gamma w_i),
 * restarting from the current x with s = 0 and d = 0. 1 / ||Phi|| and gamma
 * are formed once (as for pr_admm_solve) and kept across rounds.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t rounds;      /* reweighted rounds after the first solve (>= 0)    */
  double delta0;       /* delta of the first reweighting (> 0)              */
  double beta;         /* decay of delta per round, in (0, 1]               */
} pr_reweight_params;

/* Device workspace bytes: the pr_admm_solve workspace plus one weight per
 * coefficient (nb * n * n reals). */
int pr_reweight_workspace_size(pr_phi_plan phi, pr_psi_plan psi, size_t* bytes);

/* y, x, workspace and stream as for pr_admm_solve; params->rel_tol must be 0.
 * rep (if not NULL; the call then synchronises) describes the last round:
 * iters_done counts the iterations of all rounds, l1_norm is the unweighted
 * ||Psi^dagger x||_1. PR_EINVAL for parameters out of range. */
int pr_admm_reweighted_solve(pr_phi_plan phi, pr_psi_plan psi, const void* y,
                             const pr_admm_params* params, const pr_reweight_params* rw,
                             void* x, void* workspace, pr_admm_report* rep, void* stream);

/* ------------------------------------------------------------------------
 * Local l2-ball constraints (Section "Local Fidelity Constraint ADMM",
 * eq. proj-L2-local): the visibilities are split into nsec sections, each
 * with its own ball ||Phi_j x / ||Phi|| - y_j|| <= eps_j, and the r step of
 * Algorithm 1 projects every section on its own ball (the paper's sections
 * are equal-count bins of baseline length; any assignment is accepted).
 * A pr_balls object holds the sections' order and the per-section state.
 * section: int32[M] on the device, plan order (see pr_phi_plan_perm), values
 * in [0, nsec); it is copied into the persistent workspace.
 * Workspaces: persistent (kept) and scratch (used during create only), both
 * caller-owned and 256-byte aligned, sizes from pr_balls_sizes. One solve at
 * a time per object (the radii and the section norms live in it).
 * ---------------------------------------------------------------------- */
typedef struct pr_balls_t* pr_balls;

/* M in [0, 2^31 - 2^20], nsec in [1, 2^24]. */
int pr_balls_sizes(int64_t M, int32_t nsec, size_t* persistent_bytes, size_t* scratch_bytes);
/* Sorts the plan positions by section (stable) and synchronises `stream`.
 * PR_EINVAL if a section id is out of range, PR_EWORKSPACE for a bad
 * workspace. */
int pr_balls_create(int64_t M, int32_t nsec, const int32_t* section, void* persistent,
                    size_t persistent_bytes, void* scratch, size_t scratch_bytes,
                    void* stream, pr_balls* out);
int pr_balls_destroy(pr_balls b);
/* ||t_j|| = ||v_j + s_j - y_j|| of the last iteration of the last solve, per
 * section, into the HOST array norms[nsec] (synchronises `stream`). */
int pr_balls_norms(pr_balls b, double* norms, void* stream);

/* Algorithm 1 with the local balls: as pr_admm_solve (same workspace size,
 * pr_admm_workspace_size) with params->eps ignored and eps: HOST double[nsec],
 * the radii (copied to the device; the call synchronises once at the start).
 * Per iteration the degridding forms t = v + s - y; with at most 8 sections
 * its epilogue also keeps one FP64 ||t_j||^2 partial per section and block
 * (summed in block order by one small kernel), with more sections a gather
 * over the section-sorted positions forms them. The gridding's prologue then
 * projects each visibility with its own section's kappa_j and updates the
 * multiplier before gridding, as for the global ball. */
int pr_admm_local_solve(pr_phi_plan phi, pr_psi_plan psi, pr_balls balls, const void* y,
                        const pr_admm_params* params, const double* eps, void* x,
                        void* workspace, pr_admm_report* rep, void* stream);

/* ------------------------------------------------------------------------
 * FISTA (Section "Forward-Backward Splitting", Algorithm "FISTA") for the
 * unconstrained MAP problem
 *   min gamma (||Psi^dagger x||_1 + iota_{R+}(x)) + 1/2 ||y - Phi x / ||Phi||||^2:
 * x_0 = xh_0 = x (input), theta_0 = 1; each iteration
 *   z = xh - lambda Re Phi^dagger (Phi xh / ||Phi|| - y) / ||Phi||;
 *   x_new = DualFB(z, gamma lambda) (the prox, as in Algorithm 1, d carried);
 *   theta' = (1 + sqrt(1 + 4 theta^2)) / 2;
 *   xh = x_new + (theta - 1) / theta' (x_new - x); x = x_new; theta = theta'.
 * lambda <= 1 keeps the step below 1 / L for the normalised operator (L = 1).
 * The kernels are those of pr_admm_solve (degridding with the residual
 * epilogue, gridding, adjoint FFT with the gradient step, DualFB) plus one
 * momentum pass per iteration.
 * ---------------------------------------------------------------------- */
typedef struct {
  int32_t iters;       /* iterations (>= 0)                                  */
  int32_t inner_iters; /* DualFB iterations per prox (>= 1)                  */
  double gamma;        /* regularisation weight (> 0), or <= 0 with
                          gamma_factor > 0 (formed on the device as for
                          pr_admm_params)                                    */
  double lambda;       /* gradient step (> 0)                                */
  double eta;          /* DualFB step (> 0)                                  */
  double op_norm;      /* ||Phi||; <= 0: power method on the device          */
  double gamma_factor;
  int32_t norm_iters;  /* power-method steps when op_norm <= 0 (<= 0: 100)   */
} pr_fista_params;

/* Device workspace bytes for pr_fista_solve on these plans. */
int pr_fista_workspace_size(pr_phi_plan phi, pr_psi_plan psi, size_t* bytes);

/* Run FISTA. y: complex[M], plan order; x: real[n*n], in: x_0, out: the last
 * x_k, in place (normalised-operator units, as for pr_admm_solve). rep: if
 * not NULL, filled on return (resid_norm = ||Phi xh / ||Phi|| - y|| of the last
 * gradient, rel_var = ||x_k - x_{k-1}|| / ||x_k||) and the call synchronises;
 * if NULL the call is asynchronous. Errors: PR_EINVAL for NULL arguments or
 * parameters out of range, PR_EWORKSPACE for a NULL or unaligned workspace. */
int pr_fista_solve(pr_phi_plan phi, pr_psi_plan psi, const void* y,
                   const pr_fista_params* params, void* x, void* workspace,
                   pr_admm_report* rep, void* stream);

/* ------------------------------------------------------------------------
 * Primal-Dual splitting (Section "Primal-Dual Splitting", Algorithm
 * "Primal-Dual Algorithm") for
 *   min f(Phi x / ||Phi||) + gamma ||Psi^dagger x||_1 + iota_{R+}(x),
 * f = iota of {v : ||v - y|| <= eps} (PR_PD_BALL, the constrained problem of
 * Algorithm 1) or f = 1/2 ||v - y||^2 (PR_PD_L2, the MAP problem):
 *   z' = prox_{sigma f*}(z + sigma Phi xh)   (Moreau's decomposition);
 *   x' = DualFB(x - tau Phi^dagger z', tau gamma) (d carried, as in Algorithm 1);
 *   xh = x' + theta (x' - x).
 * x_0 = xh_0 = x (input), z_0 = 0. tau sigma < 1 is the usual step
 * condition for the normalised operator. The kernels are those of
 * pr_admm_solve (the multiplier update reads kappa from the ball or, for
 * PR_PD_L2, uses sigma / (1 + sigma)), plus one extrapolation pass.
 * ---------------------------------------------------------------------- */
enum { PR_PD_BALL = 0, PR_PD_L2 = 1 };

typedef struct {
  int32_t iters;       /* iterations (>= 0)                                  */
  int32_t inner_iters; /* DualFB iterations per prox (>= 1)                  */
  int32_t misfit;      /* PR_PD_BALL or PR_PD_L2                             */
  double eps;          /* l2-ball radius (PR_PD_BALL, >= 0)                  */
  double gamma;        /* regularisation weight (> 0), or <= 0 with
                          gamma_factor > 0 (formed on the device as for
                          pr_admm_params)                                    */
  double tau;          /* primal step (> 0)                                  */
  double sigma;        /* dual step (> 0)                                    */
  double theta;        /* extrapolation, in [0, 1]                           */
  double eta;          /* DualFB step (> 0)                                  */
  double op_norm;      /* ||Phi||; <= 0: power method on the device          */
  double gamma_factor;
  int32_t norm_iters;  /* power-method steps when op_norm <= 0 (<= 0: 100)   */
} pr_pd_params;

/* Device workspace bytes for pr_pd_solve on these plans. */
int pr_pd_workspace_size(pr_phi_plan phi, pr_psi_plan psi, size_t* bytes);

/* Run the Primal-Dual algorithm. y: complex[M], plan order; x: real[n*n],
 * in: x_0, out: the last x_k, in place (normalised-operator units). rep: if
 * not NULL, filled on return (resid_norm = ||Phi xh / ||Phi|| - y|| of the
 * last iteration, rel_var = ||x_k - x_{k-1}|| / ||x_k||) and the call
 * synchronises; if NULL the call is asynchronous. Errors: PR_EINVAL for NULL
 * arguments or parameters out of range, PR_EWORKSPACE for a NULL or
 * unaligned workspace. */
int pr_pd_solve(pr_phi_plan phi, pr_psi_plan psi, const void* y,
                const pr_pd_params* params, void* x, void* workspace,
                pr_admm_report* rep, void* stream);

/* ------------------------------------------------------------------------
 * Batched solves: many independent solves of Algorithm 1 (frequency channels
 * or imaging jobs of different n and M) stepped together, each one the
 * problem above with its own data (the per-channel / per-node split of the
 * paper's Section "Distributed Images", kept on one GPU). A step runs one
 * outer iteration of every member; members run on the batch's own streams in
 * longest-first order and are joined back to the caller's stream. With
 * use_graph the step is captured once into a HIP graph and replayed (one
 * launch per step) until the membership changes. Each member needs its own
 * Phi and Psi plans and workspace; its kernels are those of pr_admm_solve,
 * so results are bitwise identical to the member solved alone.
 * Ownership: plans, data and workspaces stay the caller's and must outlive
 * the membership. The batch holds only host objects (streams, events, graph).
 * ---------------------------------------------------------------------- */
typedef struct pr_batch_t* pr_batch;

/* max_members in [1, 4096]; nstreams in [1, 64] streams of default priority. */
int pr_batch_create(int32_t max_members, int32_t nstreams, pr_batch* out);
/* Waits for the batch streams, then frees the host objects. */
int pr_batch_destroy(pr_batch b);
/* Add a member: y complex[M] in plan order, x real[n*n] (in: x0, out: the
 * iterate, updated in place), workspace of pr_admm_workspace_size bytes.
 * The member's state is cleared and 1 / ||Phi|| (and gamma when
 * params->gamma <= 0) formed on the device, asynchronously on `stream`.
 * params->iters and rel_tol are ignored (pr_batch_step sets the count).
 * Fails with PR_EINVAL if either plan is already used by a member. */
int pr_batch_add(pr_batch b, pr_phi_plan phi, pr_psi_plan psi, const void* y,
                 void* x, const pr_admm_params* params, void* workspace,
                 void* stream, int32_t* slot);
int pr_batch_remove(pr_batch b, int32_t slot);
int pr_batch_members(pr_batch b, int32_t* count);
/* iters outer iterations of every member, asynchronous on `stream`. */
int pr_batch_step(pr_batch b, int32_t iters, int32_t use_graph, void* stream);
/* Batched operators over the members' plans: for each slot i with both
 * pointers non-NULL, y[i] = Phi_i x[i] (plan order) or x[i] = Re Phi_i^dagger y[i].
 * x, y: HOST arrays of device pointers indexed by slot (max_members long). */
int pr_batch_phi_apply(pr_batch b, const void* const* x, void* const* y,
                       void* stream);
int pr_batch_phi_adjoint(pr_batch b, const void* const* y, void* const* x,
                         void* stream);
/* FP64 diagnostics of a member's current iterate (synchronises `stream`). */
int pr_batch_report(pr_batch b, int32_t slot, pr_admm_report* rep, void* stream);

/* Fused form of pr_batch_phi_apply / pr_batch_phi_adjoint (the per-channel
 * split of Section "Distributed Images" kept on one GPU): one launch per
 * operator stage for all current members instead of one per member. The
 * degridding, the gridding walk and the patch merge run once over every
 * member's work items or tiles (each item carries its member), and each FFT
 * pass once per image size; every item and line is computed as in the
 * member's own launch, so results are bitwise those of per-member calls.
 * pr_batch_fuse_bytes gives the device workspace the current members need;
 * pr_batch_fuse builds the schedules and member tables in the caller's
 * workspace (256-byte aligned, owned by the caller, kept until the batch is
 * destroyed or fused again) and synchronises the stream once. The two calls
 * then use the fused form when every member has both vectors; adding or
 * removing a member drops it (the calls launch per member again until
 * pr_batch_fuse). PR_EUNSUPPORTED if the members' plans differ in precision,
 * J, D, lookup or tile, or J > 4; PR_EWORKSPACE if ws is too small. Each call
 * uploads the members' vector pointers when they changed since the last call
 * (synchronising the stream then). */
int pr_batch_fuse_bytes(pr_batch b, size_t* bytes);
int pr_batch_fuse(pr_batch b, void* workspace, size_t bytes, void* stream);

/* ------------------------------------------------------------------------
 * Serving: a request loop over imaging solves with continuous batching.
 * Requests are admitted in arrival order as the active-job limit and the
 * caller's device arena allow (the footprint is exact: plans, workspace,
 * plan-ordered visibilities and image, see pr_server_job_bytes); admitted
 * jobs run one outer iteration per tick on a pool of streams, so jobs join
 * and leave while others run. A job's kernels are those of a solve alone:
 * its result is independent of the mix. The library allocates no device
 * memory: everything lives in the arena. Calls on one server must come from
 * one thread.
 * ---------------------------------------------------------------------- */
typedef struct pr_server_t* pr_server;

typedef struct {
  int32_t n;            /* image side (power of two)                          */
  int32_t J;            /* kernel support                                     */
  int32_t D;            /* table samples per grid cell; <= 0: 2000            */
  int32_t tile;         /* 0: default                                         */
  int32_t levels;       /* wavelet levels                                     */
  uint32_t basis_mask;  /* SARA bases: bit 0 Dirac, bit k db k (0x1FF: all)    */
  int32_t prec;         /* PR_F32 or PR_F64                                   */
  int64_t M;            /* visibilities (>= 1)                                */
  const void* uv;       /* device Real[M][2], user order                      */
  const void* w;        /* device Real[M] or NULL (ones)                      */
  const void* y;        /* device complex[M], user order                      */
  pr_admm_params params;/* iters = outer iterations; rel_tol ignored; x0 = 0  */
  int32_t interp;       /* kernel lookup, as pr_phi_desc.interp              */
} pr_job_desc;
/* uv, w and y must stay valid until the job is running (state >= 1). */

/* Arena bytes the job occupies from admission until it is fetched. */
int pr_server_job_bytes(const pr_job_desc* desc, size_t* bytes);
/* arena: device memory of arena_bytes (256-byte aligned), owned by the
 * caller, used by no one else while the server lives. */
int pr_server_create(void* arena, size_t arena_bytes, int32_t max_active,
                     int32_t nstreams, pr_server* out);
int pr_server_destroy(pr_server s);
/* Queue a request; fails with PR_EWORKSPACE if it can never fit the arena. */
int pr_server_submit(pr_server s, const pr_job_desc* desc, int64_t* job_id);
/* Retire finished jobs, admit queued ones, and queue outer iterations of
 * every running job until it has three in flight (each job's iterations are
 * ordered on its own stream). Blocks only while an admitted job's plan is
 * built. Counts are optional. */
int pr_server_tick(pr_server s, int32_t* queued, int32_t* running,
                   int32_t* finished);
/* state: 0 queued, 1 running, 2 finished, 3 failed. */
int pr_server_job_state(pr_server s, int64_t job_id, int32_t* state,
                        int32_t* iters_done);
/* For a finished job: copy the image (real[n*n], normalised-operator units)
 * to x_out (device, may be NULL), fill rep (may be NULL), synchronise
 * `stream` and release the job's arena memory. */
int pr_server_fetch(pr_server s, int64_t job_id, void* x_out,
                    pr_admm_report* rep, void* stream);
/* Cancel a job in any state: a queued job leaves the queue; a running job is
 * given no further iterations, the call waits for the ones in flight (on the
 * job's own stream) and releases its arena memory; a finished or failed job
 * is released without a fetch. The id is unknown afterwards. */
int pr_server_cancel(pr_server s, int64_t job_id);
int pr_server_free_bytes(pr_server s, size_t* free_bytes, size_t* largest);

#ifdef __cplusplus
}
#endif

#endif /* PURIMI_H */
