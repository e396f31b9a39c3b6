/*
 * ga.h -- C ABI of the MI355X hot path of the explicit order-2k
 * generalized-alpha method for isogeometric structural dynamics with
 * Kronecker-preconditioned conjugate-gradient mass solves.
 *
 * Problem (Sec. 2, eqs. pde and mp): M U'' + K U = 0 with homogeneous
 * Dirichlet data, unit density and wave speed (C = 0, F = 0), on one
 * single-patch spline domain (Sec. 5.2) of degree p with maximal smoothness.
 *
 * Conventions shared by every call:
 *  - Vectors are FP64, device-resident, and hold the free (Dirichlet-
 *    eliminated) coefficients in co-lexicographic order, x fastest
 *    (Sec. 5.2): index ix + mf_x*(iy + mf_y*iz), mf_a = n_a + p - 2.
 *    Several right-hand sides ("nrhs") are stored back to back.
 *  - The caller owns every vector it passes; the library never frees or
 *    retains them.  The library owns all handle internals (tables,
 *    geometric factors, preconditioner data, work buffers).
 *  - All work is ordered on the HIP stream passed as `stream` (a
 *    hipStream_t; NULL = the default stream).  Calls return once the work
 *    is enqueued unless they hand scalars back to the host (ga_mass_solve,
 *    ga_step, ga_init_state, ga_lambda_max, ga_patch_setup).
 *  - Every call returns GA_OK or a negative status; it never throws.
 *    ga_last_error() gives a message for the last failure of the calling
 *    thread.
 */
#ifndef GA_H
#define GA_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ga_patch ga_patch;
typedef struct ga_integrator ga_integrator;
typedef struct ga_gnet ga_gnet;
typedef struct ga_batch ga_batch;
typedef struct ga_mp ga_mp;
typedef struct ga_wave1d ga_wave1d;

enum {
  GA_OK = 0,
  GA_EINVAL = -1,     /* bad argument: sizes, degree, null pointer, k, rho */
  GA_ENOMEM = -2,     /* device allocation failed                         */
  GA_EDEVICE = -3,    /* a HIP call failed                                */
  GA_EGEOMETRY = -4,  /* det DF <= 0 at a quadrature point (Assumption 3) */
  GA_ENOCONV = -5,    /* PCG hit maxit; the last iterate is still written */
  GA_EUNSTABLE = -6   /* stepping diverged: a state norm became non-finite, or
                         |U| + tau |V| grew past the bound of a stable step (ga_step) */
};

/* Arithmetic (precision is an addition to the paper, which computes in FP64).
 *   GA_FP64  FP64 factors, vectors and arithmetic.
 *   GA_FP32  FP32 factors, vectors and arithmetic.
 *   GA_BF16  quadrature factors stored in BF16 (round to nearest even) and widened
 *            to FP32 for the FP32 sum-factorised contractions; the preconditioner's
 *            per-axis dense contractions on the matrix cores with BF16 operands and
 *            FP32 accumulation (FP32 vectors).
 * In the mass solves (ga_mass_solve, ga_integrator_create) GA_FP32 and GA_BF16 select
 * the inner arithmetic of an FP64 iterative refinement: the residual r = b - M x
 * with FP64 factors, the dot products and norms, the stopping test and the solution
 * are FP64; the correction M d = r comes from an inner flexible PCG in that
 * precision.  The stiffness apply and the state update of ga_step are FP64 in every
 * mode. */
enum { GA_FP64 = 0, GA_FP32 = 1, GA_BF16 = 2 };
/* Initial guess of the stage solves in ga_step, from the stage solutions of
 * the previous steps: zero (the paper's choice), the previous step's, or the
 * polynomial extrapolation through the last (up to 4) steps, or the learned
 * guess (a convolutional net attached per stage with ga_integrator_set_net;
 * stages without a net, and steps with fewer than 4 past solutions, use the
 * extrapolation).  A nonzero guess is kept only if its preconditioned
 * residual is smaller than that of the zero guess; otherwise the solve
 * restarts from zero (counted in ga_solve_stats). */
enum { GA_GUESS_ZERO = 0, GA_GUESS_PREV = 1, GA_GUESS_EXTRAP = 2, GA_GUESS_LEARNED = 3 };

/*
 * ga_setup_patch -- build one patch (Sec. 5.1-5.2, eq. mass_matrix and the
 * preconditioner definition of Sec. 5.4).
 *   dim        2 or 3.
 *   n_el[dim]  elements per direction (>= 1), uniform open knot vectors.
 *   p          spline degree, 1..4; p+1 Gauss points per element/direction.
 *   ctrl_host  host array [N_dof][dim] of control points C_i of the map
 *              F = sum_i C_i B_i, co-lex over the full grid of
 *              N_dof = prod (n_a + p) coefficients.  Read during the call only.
 * Builds, on the device: the quadrature factors w|det J| and
 * w|det J| J^{-1} J^{-T}, D = diag(M), the scaling s = (Dhat/D)^{1/2}, and for
 * each axis the univariate parametric mass matrix Mhat_a on the free coefficients
 * as its banded Cholesky factor (used by the default preconditioner) and as its
 * dense inverse (used by the dense preconditioner modes).  FP32 and BF16 copies
 * of the factors, and the inverses packed for the matrix cores, are built on
 * first use.  Returns GA_EGEOMETRY (and no handle) if det J <= 0 anywhere.
 */
int ga_setup_patch(int dim, const int* n_el, int p, const double* ctrl_host,
                   void* stream, ga_patch** out);
/*
 * ga_setup_patch_ex -- as ga_setup_patch with a choice of the faces that carry
 * the homogeneous Dirichlet data (3-D only): bit 2a of dirichlet_faces is the
 * face xi_a = 0, bit 2a+1 the face xi_a = 1 (0x3F = all six, ga_setup_patch).
 * Coefficients on the other faces stay free, as on an interface of a glued
 * multi-patch domain (Sec. 5.3): along axis a the free coefficients are
 * lo_a .. m_a - 1 - hi_a with lo_a, hi_a the two face bits, and every vector
 * of the patch holds them in co-lex order.  M-hat, its factors and the scaling
 * s are those of that index range.
 */
int ga_setup_patch_ex(int dim, const int* n_el, int p, const double* ctrl_host,
                      unsigned dirichlet_faces, void* stream, ga_patch** out);
int ga_destroy_patch(ga_patch* patch);

/* Sizes: free coefficients, quadrature points, free coefficients per axis. */
int ga_patch_info(const ga_patch* patch, long long* n_free, long long* n_quad,
                  int* mf /* [3]; mf[2] = 1 for dim 2 */);

/* Counters of the mass solves since the last reset: solves, solves started
 * from a nonzero guess, guesses rejected by the residual test, and the mean of
 * |r0|_P / |b|_P over the guessed solves (P-norm: sqrt(r^T P^{-1} r)). */
int ga_solve_stats(ga_patch* patch, long long* solves, long long* guessed, long long* fallbacks,
                   double* mean_guess_relres, int reset);

/* d_dev[N_free] <- diag(M) (the D of Sec. 5.4). */
int ga_diag_M(ga_patch* patch, double* d_dev, void* stream);

/*
 * ga_apply_MK -- y = alpha * Op x for nrhs vectors, Op = M (which = 'M', eq.
 * mass_matrix) or K (which = 'K', stiffness of eq. mp with omega = 1),
 * restricted to the free coefficients, applied matrix-free by sum
 * factorisation over the Gauss points.  x and y must not overlap.
 *   prec  GA_FP64; or (3-D patches) GA_FP32 / GA_BF16: x is rounded to FP32, the
 *         factors are the FP32 / BF16 copies (built on the first such call), the
 *         contractions run in FP32 and the FP32 result is widened into y.
 * The low-precision forms use the patch's work area (calls on one patch from
 * overlapping streams race).
 */
int ga_apply_MK(ga_patch* patch, char which, int nrhs, int prec, double alpha,
                const double* x_dev, double* y_dev, void* stream);

/*
 * ga_apply_Pinv -- z = P^{-1} r for nrhs vectors, with
 * P = D^{1/2} Dhat^{-1/2} Mhat Dhat^{-1/2} D^{1/2} (Sec. 5.4), applied as
 * z = s * (Mz^{-1} x My^{-1} x Mx^{-1})(s * r), one univariate solve along
 * each tensor axis.  r and z may be the same buffer.
 *   prec  GA_FP64: the patch's preconditioner mode (ga_patch_set_pinv): by default
 *         forward and backward substitution with the banded Cholesky factor of
 *         Mhat_a (where a z-plane fits the on-chip staging, 152 KiB), otherwise a
 *         product with the dense inverse of Mhat_a;
 *         GA_FP32 (3-D): the same in FP32 (r rounded to FP32, result widened);
 *         GA_BF16 (3-D, axes of at most 256 free coefficients): the dense inverse
 *         products on the matrix cores with BF16 operands and FP32 accumulation.
 */
int ga_apply_Pinv(ga_patch* patch, int nrhs, int prec, const double* r_dev, double* z_dev,
                  void* stream);
/*
 * ga_apply_Pinv_noalloc -- ga_apply_Pinv with prec = GA_FP64 for callers that
 * cannot allocate device memory (code under HIP stream or graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  It allocates nothing: its two
 * intermediate vectors live in a fixed device array that the library holds on every
 * GPU it runs on (2 * GA_NOALLOC_MAX_ENTRIES doubles, 72 MiB, from module load
 * until the process ends).
 *   nrhs * n_free must not exceed GA_NOALLOC_MAX_ENTRIES (GA_EINVAL otherwise).
 *   With GA_PINV_MFMA the packed inverses must have been built by an earlier
 *   ga_apply_Pinv or solve on the patch (GA_EINVAL otherwise).
 * All calls on one GPU share that array: calls that overlap on one GPU (other
 * streams, other threads) race and must be serialized by the caller.  Results
 * equal those of ga_apply_Pinv (the same kernels).
 */
#define GA_NOALLOC_MAX_ENTRIES 4718592
int ga_apply_Pinv_noalloc(ga_patch* patch, int nrhs, const double* r_dev, double* z_dev,
                          void* stream);

/* Preconditioner algorithm of a patch (all compute the same P^{-1}):
 * GA_PINV_AUTO (banded solves when they fit, the default), GA_PINV_DENSE (dense
 * inverse products on the vector ALU) or GA_PINV_MFMA (dense inverse products on
 * the matrix cores: v_mfma_f64_16x16x4 in FP64, v_mfma_f32_32x32x2 in FP32; axes
 * of at most 256 free coefficients).  Device-side PCG control (ga_patch_set_cg)
 * applies to GA_PINV_AUTO only. */
enum { GA_PINV_AUTO = 0, GA_PINV_DENSE = 1, GA_PINV_MFMA = 2 };
int ga_patch_set_pinv(ga_patch* patch, int mode);
/*
 * PCG control of a patch's FP64 solves (Sec. 5.6 PCG; the control is an
 * implementation choice and gives the same iterates):
 *   GA_CG_HOST    the host reads the convergence flags after every iteration;
 *   GA_CG_DEVICE  (default) the convergence test stays on the device: the mass apply,
 *                 the preconditioner, the fills and dots of every iteration are
 *                 gated by the per-system flags, so a converged system costs
 *                 nothing.  The host enqueues as many iterations as the
 *                 previous solve with the same number of right-hand sides
 *                 needed (the right-hand sides expected to be active share
 *                 one operator launch, the others get gated launches of their
 *                 own), then reads the flags once and continues per iteration
 *                 only if a system is still active.  2-D and 3-D patches with
 *                 the banded preconditioner; otherwise the host control is used.
 *   GA_CG_FUSED   single-reduction (Chronopoulos-Gear) PCG under the same device
 *                 control: six launches per iteration instead of eleven: the mass
 *                 apply w = M z, one reduction for z^T w, one kernel that completes
 *                 it in every workgroup, takes the alpha/beta step and updates p,
 *                 s = M p, x and r, and the three preconditioner passes, the last of
 *                 which sums r^T z and applies the stopping test (its last
 *                 workgroup completes the sum).  The same iterates as GA_CG_DEVICE
 *                 in exact arithmetic and the same stopping test.  3-D patches with
 *                 the banded preconditioner (otherwise GA_CG_DEVICE's rules apply).
 * ga_cg_stats: iterations enqueued ahead so far and host reads of the flags.
 */
enum { GA_CG_HOST = 0, GA_CG_DEVICE = 1, GA_CG_FUSED = 2 };
int ga_patch_set_cg(ga_patch* patch, int mode);
int ga_cg_stats(const ga_patch* patch, long long* spec_iters, long long* host_checks);
/*
 * ga_patch_tune -- autotuner for the operator launches of a 3-D patch: for the
 * mass and the stiffness apply with nrhs (1..3) right-hand sides, times `reps`
 * launches for each candidate number of element layers per workgroup along z
 * (whole columns, then halving down to 4) and keeps the fastest for the patch.
 * Results do not change (the same sums, in another tiling).  best_ms (may be
 * NULL): one tuned mass plus one tuned stiffness launch.  Allocates two scratch
 * vectors for the duration of the call and synchronizes `stream`.
 * ga_patch_tuned_layers: the layer counts the patch now uses (either may be NULL).
 */
int ga_patch_tune(ga_patch* patch, int nrhs, int reps, double* best_ms, void* stream);
int ga_patch_tuned_layers(const ga_patch* patch, int* ze_mass, int* ze_stiff);
/* ga_patch_set_layers -- sets the element layers per workgroup of the FP64 mass and
 * stiffness launches of a 3-D patch (1..n_el[2]; 0 = automatic), as the autotuner
 * would: the launch shapes change, the results do not.  GA_EINVAL out of range. */
int ga_patch_set_layers(ga_patch* patch, int ze_mass, int ze_stiff);
/* ga_patch_set_deterministic -- on != 0: the operator applies of a 3-D patch add the
 * contributions of neighbouring tiles in a fixed order, so every apply, solve and
 * step gives bitwise the same result on every run (an implementation choice: the
 * default adds shared coefficients with FP64 atomics, whose order changes from run
 * to run and moves the last bits).  The tiles are split into colour classes whose
 * tiles share no coefficient (4 classes in x-y for p <= 3, 9 for p = 4, times 2 or
 * more along z when a column is split into z ranges), launched one after the other:
 * slower (fewer tiles per launch).  Single-patch launches only (not the batch). */
int ga_patch_set_deterministic(ga_patch* patch, int on);


/*
 * ga_mass_solve -- PCG for M x_j = b_j, j < nrhs (Sec. 5.6; solver settings of
 * Sec. 6).  x_dev holds the initial guesses on entry (zero them for the
 * paper's null guess) and the solutions on return.  Each right-hand side
 * stops when sqrt(r^T P^{-1} r) <= rtol * sqrt(b^T P^{-1} b); converged
 * right-hand sides are frozen while the others continue.
 *   prec   GA_FP64, or GA_FP32 / GA_BF16 (3-D only; see above).  With GA_FP32
 *          and GA_BF16 the stopping test uses P^{-1} applied in that precision
 *          and iters_out counts the inner iterations.  Where rtol is at least 8
 *          times the inner arithmetic's accuracy floor (3e-7 for GA_FP32, 2e-3
 *          for GA_BF16), a refinement pass whose inner PCG reached half the
 *          tolerance, with a rounding error (about floor times the pass's
 *          starting residual) of at most an eighth of it, ends that right-hand
 *          side without a further FP64 residual; its relres_out is then the
 *          inner residual estimate.
 *   iters_out[nrhs], relres_out[nrhs]  host arrays or NULL.
 * Returns GA_ENOCONV if any right-hand side did not converge in maxit.
 */
int ga_mass_solve(ga_patch* patch, int nrhs, const double* b_dev, double* x_dev,
                  double rtol, int maxit, int prec, int* iters_out, double* relres_out,
                  void* stream);

/*
 * ga_lambda_max -- estimate of the largest eigenvalue of M^{-1} K by power
 * iteration (iters steps, each one K apply and one PCG mass solve).  Used to
 * choose tau below the stability limit tau^2 lambda_max <= Theta_s.
 */
int ga_lambda_max(ga_patch* patch, int iters, double* lambda_out, void* stream);

/* Theta_s(rho): stability limit on tau^2 lambda of the scheme (all k). */
double ga_stability_limit(double rho);
/* Theta_s of the two-parameter family rho_s <= rho_b (Remark in Sec. 3): the
 * lambda = -1 root of the type-k characteristic polynomial, the same for all k. */
double ga_stability_limit2(double rho_b, double rho_s);

/*
 * ga_integrator_create -- the order-2k scheme of Sec. 4 (k = 1, 2, 3, 4) with
 * rho_b = rho_s = rho in [0, 1), step tau > 0, PCG tolerance rtol and maxit,
 * mass-solve arithmetic prec (GA_FP64, GA_FP32 or GA_BF16; the last two on 3-D
 * patches).
 * State vectors are L^a, a = -2 .. 3k-3 (U, V, A, then time derivatives of A).
 */
int ga_integrator_create(ga_patch* patch, int k, double rho, double tau, double rtol,
                         int maxit, int prec, int guess_mode, ga_integrator** out);
int ga_integrator_destroy(ga_integrator* integ);

/*
 * ga_init_state -- initial data: L^{-2} = U0, L^{-1} = V0 and
 * L^a = M^{-1}(-K L^{a-2}) for a = 0..3k-3 (the initial solves of Sec. 3,
 * continued to general k).  state_dev[3k] are caller-owned vectors.
 */
int ga_init_state(ga_integrator* integ, const double* U0_dev, const double* V0_dev,
                  double* const* state_dev, void* stream);

/*
 * ga_step -- advance state_dev[3k] by nsteps steps.  Each step forms the
 * Taylor predictors, the k stage right-hand sides -K Y_j (eq. ho1), solves
 * the k mass systems together by PCG, and applies the updates of eq. ho2.
 *   iters_out  host array [nsteps][k] of PCG iterations, or NULL.
 * Returns GA_ENOCONV if a stage solve did not converge, GA_EUNSTABLE if U or V
 * became non-finite or N = |U| + tau |V| (Euclidean norms of the coefficient
 * vectors) grew by more than 10 * 1.05^nsteps over the call: a stable step keeps
 * the discrete energy bounded, and growth from a small start (U0 = 0: N grows
 * about like nsteps + 1 while nsteps * tau * omega << 1) stays within that bound
 * for every nsteps, while an unstable mode grows geometrically.  ga_step_forced
 * checks only for non-finite values (a load may make the state grow).
 */
int ga_step(ga_integrator* integ, double* const* state_dev, int nsteps,
            int* iters_out, void* stream);

/*
 * Damping and forcing (eq. ho1 with C and F; initial data of Sec. 3).
 * Stage j solves  M X_j = F^{(a_j)}(t_n + alpha_fj tau) - C Z_j - K Y_j,
 * a_j = 3j-3, with Y_j the stiffness argument of ga_step and Z_j its damping
 * counterpart: the Taylor predictor of L^{a_j-1} at t_{n+1} for j < k, L^{N-1}_n
 * for j = k (the reading that keeps order 2k; C on L^{a_j-1}_n gives order 1).
 * alpha_fj = 1 for j < k and 0 for j = k (ga_stage_times).
 *
 * ga_integrator_set_damping -- Rayleigh damping C = cM M + cK K (cM, cK >= 0;
 * both 0 = undamped, the default).  Applies to ga_init_state* and ga_step*.
 */
int ga_integrator_set_damping(ga_integrator* integ, double cM, double cK);
/* ga_stage_times -- t_n + alpha_fj tau for j = 1..k into out[k] (host). */
int ga_stage_times(const ga_integrator* integ, double t_n, double* out);
/*
 * ga_init_state_forced -- as ga_init_state with a load:
 * L^a = M^{-1}(F^{(a)}(0) - C L^{a-1} - K L^{a-2}), a = 0..3k-3.
 * F0_dev: 3k-2 device vectors F^{(a)}(0) (the a-th time derivative of the load
 * vector at t = 0), or NULL for no load.
 */
int ga_init_state_forced(ga_integrator* integ, const double* U0_dev, const double* V0_dev,
                         const double* const* F0_dev, double* const* state_dev, void* stream);
/*
 * ga_step_forced -- one step from t_n with the load: forcing_dev[j] (k device
 * vectors) = F^{(a_j)} at the stage time t_n + alpha_fj tau of ga_stage_times.
 * iters_out: host [k] or NULL.
 */
int ga_step_forced(ga_integrator* integ, double* const* state_dev, const double* const* forcing_dev,
                   int* iters_out, void* stream);

/*
 * ga_stage_solution -- copy the stage-j solution X_j of `age` steps ago
 * (age 0 = the last step; ages 1..3 need a guess mode other than
 * GA_GUESS_ZERO, which keeps the ring of past solutions) into out_dev
 * [n_free].  GA_EINVAL if that solution does not exist yet.
 */
int ga_stage_solution(ga_integrator* integ, int stage, int age, double* out_dev, void* stream);

/*
 * Checkpoint and resume (an addition).  The step state is the 3k state vectors
 * (caller-owned), tau and the integrator settings, plus, in a guess mode other
 * than GA_GUESS_ZERO, the ring of the last (up to 4) stage solutions that the
 * guesses are formed from.  A checkpoint saves the state vectors and, for ages
 * 0 .. nhist-1, ga_stage_solution of every stage; a resume creates an integrator
 * with the same settings, restores the ring with ga_integrator_set_history and
 * steps on from the saved state vectors.  With ga_patch_set_deterministic and
 * FP64 solves the resumed steps are bitwise those of an uninterrupted run (the
 * mixed solves' refinement passes also depend on the patch's adaptive inner
 * iteration counts, so they agree to the solver tolerance).
 *   ga_integrator_history: *nhist = number of stage solutions in the ring (0..4).
 *   ga_integrator_set_history: hist_dev[age * k + stage], age 0 the newest,
 *     nhist in 0..4 device vectors of n_free each (copied; the caller keeps
 *     ownership); replaces the ring.  GA_EINVAL for GA_GUESS_ZERO integrators
 *     when nhist > 0.
 */
int ga_integrator_history(const ga_integrator* integ, int* nhist);
int ga_integrator_set_history(ga_integrator* integ, int nhist, const double* const* hist_dev,
                              void* stream);

/*
 * Learned initial guess (not in the paper; an addition on top of its zero
 * initial guess).  From the last four solutions H1..H4 of stage j (newest
 * first) form the backward differences
 *   D0 = H1, D1 = H1 - H2, D2 = H1 - 2H2 + H3, D3 = H1 - 3H2 + 3H3 - H4,
 * their RMS values s_c (1 where D_c = 0) and the cubic extrapolation
 * E = D0 + D1 + D2 + D3; then
 *   guess_j = E + s_3 * net(D0/s_0, D1/s_1, D2/s_2, D3/s_3).
 * net: a 3-layer convolutional net on the free-coefficient grid, 3x3x3
 * kernels, channels 4 -> 32 -> 32 -> 1, ReLU after layers 1 and 2, zero
 * padding at the grid boundary (the homogeneous Dirichlet data).
 * Parameters: GA_GNET_NPARAM FP32 values, tap-major:
 *   W1[27][4][32] b1[32] W2[27][32][32] b2[32] W3[27][32][1] b3[1],
 *   tap t = 9 kz + 3 ky + kx; W[t][ci][co] multiplies input channel ci at
 *   offset (kx-1, ky-1, kz-1) in the output channel co.
 * Training runs on crops of S^3 points (the target is the interior (S-6)^3)
 * with FP32 master weights, activations and gradients; by default (GA_BF16)
 * layer 2's forward, backward-data and backward-weight convolutions, 55,296 of
 * the 63,936 flops per point in each pass, run on the matrix cores with BF16
 * operands and FP32 accumulation, the rest in FP32.  Inference runs in BF16
 * (weights and activations) with FP32 accumulation, all three layers on MFMA.
 * A net owns its parameters, Adam moments and work buffers; calls that use one
 * net on overlapping streams race.
 */
#define GA_GNET_NPARAM 32033
/* params_host: GA_GNET_NPARAM floats, or NULL for all-zero parameters. */
int ga_gnet_create(const float* params_host, ga_gnet** out);
int ga_gnet_destroy(ga_gnet* net);
int ga_gnet_set_params(ga_gnet* net, const float* params_host);  /* resets Adam */
int ga_gnet_get_params(ga_gnet* net, float* params_host);
/*
 * ga_gnet_set_train_prec -- arithmetic of ga_gnet_forward and ga_gnet_loss_grad:
 * GA_BF16 (the default; layer 2 on BF16 MFMA with FP32 accumulation) or GA_FP32
 * (every convolution in FP32 on the vector units).  Other values: GA_EINVAL.
 */
int ga_gnet_set_train_prec(ga_gnet* net, int prec);
/*
 * ga_gnet_make_batch -- training crops from one stage of a 3-D patch:
 *   in_dev  [nb][4][S^3]  D_c / s_c at grid points origin_b + (0..S-1)^3, zero
 *                          outside the grid (s_c over the whole grid);
 *   tgt_dev [nb][(S-6)^3] (X - E) / s_3 at origin_b + 3 + (0..S-7)^3.
 * hist_dev: 4 device vectors H1..H4 [n_free]; x_dev: the solution paired with
 * them.  origins_host [nb][3] (x, y, z); the target region must lie inside
 * the grid: -3 <= origin_a and origin_a + S - 3 <= mf_a.  S >= 7.
 */
int ga_gnet_make_batch(ga_gnet* net, ga_patch* patch, const double* const* hist_dev,
                       const double* x_dev, int nb, int S, const int* origins_host,
                       float* in_dev, float* tgt_dev, void* stream);
/*
 * ga_gnet_forward -- forward pass on crops: out_dev [nb][(S-6)^3] (FP32 output).
 * grid3 (host, 3 ints) and origins_host (as in ga_gnet_make_batch) place the
 * crops in the grid: layer-1 and layer-2 activations outside it are zero.
 */
int ga_gnet_forward(ga_gnet* net, int nb, int S, const int* grid3, const int* origins_host,
                    const float* in_dev, float* out_dev, void* stream);
/*
 * ga_gnet_loss_grad -- loss = mean over the nb (S-6)^3 targets of
 * (net - tgt)^2 and its gradient w.r.t. the parameters into grad_dev
 * [GA_GNET_NPARAM] (FP32).  loss_out (host) may be NULL; if given, the call
 * waits for the stream.
 */
int ga_gnet_loss_grad(ga_gnet* net, int nb, int S, const int* grid3, const int* origins_host,
                      const float* in_dev, const float* tgt_dev, float* grad_dev,
                      double* loss_out, void* stream);
/* ga_gnet_adam -- one Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with grad_dev. */
int ga_gnet_adam(ga_gnet* net, const float* grad_dev, float lr, void* stream);
/*
 * ga_gnet_infer -- the learned guess on the whole free grid of a 3-D patch:
 * x_dev [n_free] = E + s_3 * net(D / s) from hist_dev[4] (newest first), BF16
 * inference.
 */
int ga_gnet_infer(ga_gnet* net, ga_patch* patch, const double* const* hist_dev, double* x_dev,
                  void* stream);
/* ga_integrator_set_net -- net for stage j (0-based) in GA_GUESS_LEARNED mode;
 * NULL detaches.  The integrator does not own the net. */
int ga_integrator_set_net(ga_integrator* integ, int stage, ga_gnet* net);

/*
 * Batched independent patches (an addition, not in the paper: the patches are
 * not glued to each other).  One call advances R 3-D patches (p = 2..4, each
 * axis at most 256 free coefficients) by the order-2k scheme with a common
 * step tau, FP64 PCG with the zero initial guess.  Work on all patches shares
 * launches: one per spline degree for each mass or stiffness apply, one per
 * preconditioner pass and axis-length class, one for each vector operation.
 * Batched vectors hold patch r's free coefficients (in that patch's
 * co-lexicographic order) at entries off_r .. off_r + n_free_r - 1, with
 * N = sum n_free_r entries in all (ga_batch_info gives N and off_r).  The
 * patches are borrowed: they must outlive the batch.
 */
int ga_batch_create(int npatch, ga_patch* const* patches, int k, double rho, double tau,
                    double rtol, int maxit, ga_batch** out);
int ga_batch_destroy(ga_batch* batch);
/*
 * ga_batch_set_precision -- arithmetic of the batch's mass solves (an addition, not in the paper):
 * GA_FP64 (default) or GA_FP32 = FP32 flexible-PCG corrections (FP32 mass
 * factors, vectors and preconditioner, inner reduction 1e-4) inside an FP64
 * iterative refinement whose residual and stopping test are FP64.  The first
 * switch to GA_FP32 builds FP32 copies of every patch's factors (kept with the
 * patch) and the FP32 launch tables; it synchronizes `stream`.  Iteration
 * counts reported by ga_batch_step are then inner FP32 iterations.
 */
int ga_batch_set_precision(ga_batch* batch, int prec, void* stream);
/*
 * ga_batch_set_tau -- per-patch time steps: patch r advances by tau_host[r]
 * per step (the patches are independent, so each may run at its own stability
 * limit; a step of the batch is one step of every patch).  tau_host = NULL
 * returns to the common tau of ga_batch_create.  The scheme's parameters do
 * not depend on tau.
 */
int ga_batch_set_tau(ga_batch* batch, const double* tau_host);
/* n_total: N; offsets_out[npatch] (may be NULL); graph_replays: PCG iterations
 * run so far as replays of the captured iteration graph (may be NULL). */
int ga_batch_info(const ga_batch* batch, long long* n_total, long long* offsets_out,
                  long long* graph_replays);
/*
 * ga_batch_tune -- autotuner: for each operator launch (mass, stiffness; per
 * degree) time `reps` launches of each candidate tile shape (element layers
 * per tile along z) and workgroup count of the tile queue, keep the fastest.
 * best_ms (may be NULL): summed time of one launch of each tuned operator.
 */
int ga_batch_tune(ga_batch* batch, int reps, double* best_ms, void* stream);
/* L^{-2} = U0, L^{-1} = V0, L^a = M^{-1}(-K L^{a-2}) patch by patch; batched
 * vectors of N entries. */
int ga_batch_init_state(ga_batch* batch, const double* U0_dev, const double* V0_dev,
                        double* const* state_dev, void* stream);
/*
 * ga_batch_step -- nsteps steps of every patch.  use_graph != 0: each PCG
 * iteration is a replay of a captured hipGraph (run on a stream the batch
 * owns, ordered after `stream`).  iters_out: host [nsteps][k * npatch] PCG
 * iterations of system j * npatch + r (stage j, patch r), or NULL.  Waits for
 * the work before returning.
 */
int ga_batch_step(ga_batch* batch, double* const* state_dev, int nsteps, int use_graph,
                  int* iters_out, void* stream);

/*
 * Glued multi-patch domain (Sec. 5.3) with the additive Schwarz mass
 * preconditioner P_ad^{-1} = sum_r R^(r)T (P^(r))^{-1} R^(r) (Sec. 5.5), P^(r)
 * the preconditioner of Sec. 5.4 on patch r.  The domain is a brick: the unit
 * cube's parameter box split into P[0] x P[1] x P[2] boxes, patch r = box
 * (r % P0, (r / P0) % P1, r / (P0 P1)), each with n_el elements per direction
 * and degree p (2..4), glued with C^0 continuity: along axis a, coefficient i
 * (0..n_el+p-1) of box b_a is global coefficient b_a (n_el+p-1) + i, so
 * neighbouring boxes share the coefficients of their common face (their
 * control points must match there).  The outer boundary carries homogeneous
 * Dirichlet data; the unknowns are the interior global coefficients,
 * mfg_a = P_a (n_el+p-1) - 1 per axis, co-lex (x fastest), N = prod mfg_a.
 *   ctrl_host[r]  control points of patch r, as for ga_setup_patch.
 * The library owns the patches it builds.  Time stepping: the order-2k scheme
 * of ga_step on the global unknowns (C = F = 0), PCG with P_ad, zero guess.
 */
int ga_mp_create(const int* P, int n_el, int p, const double* const* ctrl_host, int k, double rho,
                 double tau, double rtol, int maxit, void* stream, ga_mp** out);
int ga_mp_destroy(ga_mp* mp);
/* n_global: N; mfg[3]: unknowns per axis; n_local: sum of the patches' free
 * coefficients (interface coefficients counted once per patch). */
int ga_mp_info(const ga_mp* mp, long long* n_global, int* mfg, long long* n_local);
/* y = M x, K x ('M', 'K') or P_ad^{-1} x ('P') on global vectors, nrhs <= k. */
int ga_mp_apply(ga_mp* mp, char which, int nrhs, const double* x_dev, double* y_dev, void* stream);
/* PCG with P_ad for M x_j = b_j, zero guess, the integrator's rtol and maxit. */
int ga_mp_mass_solve(ga_mp* mp, int nrhs, const double* b_dev, double* x_dev, int* iters_out,
                     void* stream);
int ga_mp_init_state(ga_mp* mp, const double* U0_dev, const double* V0_dev,
                     double* const* state_dev, void* stream);
/* iters_out: host [nsteps][k] or NULL. */
int ga_mp_step(ga_mp* mp, double* const* state_dev, int nsteps, int* iters_out, void* stream);

/*
 * ga_integrator_set_rho -- the two-parameter family (Remark in Sec. 3):
 * 0 <= rho_s <= rho_b < 1; blocks j < k take the printed type-j formulas at
 * (-rho_b, -rho_s), block k the type-k formulas at (rho_b, rho_s).  rho_s =
 * rho_b is the one-parameter scheme of ga_integrator_create.
 */
int ga_integrator_set_rho(ga_integrator* integ, double rho_b, double rho_s);

/*
 * Batched 1-D wave problems (the dispersion study of Sec. 6.2): nsys
 * independent systems M U_r'' + omega_r^2 K U_r = 0 on (0, 1), homogeneous
 * Dirichlet data, degree p (C^{p-1}) on n_el uniform elements (identity map),
 * stepped together by the order-2k scheme with (rho_b, rho_s) and one tau.
 * On the identity map the Kronecker preconditioner of Sec. 5.4 equals M, so
 * each stage solve is the first (and converged) PCG iterate M^{-1} b.
 * Vectors: FP64 device, system r at entries r*m .. r*m+m-1, m = n_el + p - 2
 * (ga_wave1d_info); the state is 3k such vectors (L^{-2} .. L^{3k-3}).
 * The caller keeps the stability condition tau^2 omega_r^2 lambda_max(M^{-1}K)
 * <= ga_stability_limit2(rho_b, rho_s); nothing is checked per step.
 */
int ga_wave1d_create(int n_el, int p, int nsys, const double* omega2_host, int k, double rho_b,
                     double rho_s, double tau, ga_wave1d** out);
int ga_wave1d_destroy(ga_wave1d* w);
int ga_wave1d_info(const ga_wave1d* w, int* n_free);
/* f[r][i] = int_0^1 b_i(x) sin(j_r pi x) dx (2p + 8 Gauss points per element),
 * wavenumbers_host[nsys]; synchronizes the stream. */
int ga_wave1d_load_sine(ga_wave1d* w, const double* wavenumbers_host, double* f_dev, void* stream);
/* y[r] = M x[r] ('M'), K x[r] ('K') or M^{-1} x[r] ('S') for every system. */
int ga_wave1d_apply(ga_wave1d* w, char which, const double* x_dev, double* y_dev, void* stream);
/* L^{-2} = U0, L^{-1} = V0, L^a = M^{-1}(-omega^2 K L^{a-2}), a = 0 .. 3k-3. */
int ga_wave1d_init_state(ga_wave1d* w, const double* U0_dev, const double* V0_dev,
                         double* const* state_dev, void* stream);
/* nsteps steps of every system; no host synchronization. */
int ga_wave1d_step(ga_wave1d* w, double* const* state_dev, int nsteps, void* stream);

/*
 * Launch timing (instrumentation, not part of the method): launches of the
 * timed kinds are bracketed by HIP events on the stream they run on.  Kinds:
 * 0 = mass apply (operator launch), 1 = stiffness apply, 2 = preconditioner
 * application, 3 = learned-guess inference in ga_step.  ga_profile(kinds)
 * clears the totals and times the kinds whose bit (1 << kind) is set in
 * `kinds` (0 turns timing off, GA_PROF_ALL times every kind; outside [0, 15]:
 * GA_EINVAL).  Each event pair costs the stream a few microseconds, so time
 * only the kinds that are needed.  ga_profile_query waits for the recorded
 * events and returns the summed duration in ms and the number of launches of
 * one kind.  Host-global state, not thread safe.
 */
#define GA_PROF_ALL 15
int ga_profile(int kinds);
int ga_profile_query(int kind, double* total_ms, long long* launches);

/* Message for the last non-GA_OK status returned on this thread. */
const char* ga_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* GA_H */
