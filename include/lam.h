/*
 * lam.h -- C ABI of the least-action TDSE relaxation library (liblam.so).
 *
 * Method: Z. B. Walters, "An efficient parallel method for relaxing to the
 * minimum action wavefunction".  One propagation step expands the
 * wavefunction as phi(x,t) = sum_{i,n} C_in chi_i(x) T_n(t) (Sec. "Review of
 * the Least Action Principle") and solves the stationarity conditions of the
 * action, Eq. (stationaryphase), with one Lagrange multiplier per spatial
 * function imposing the initial condition.  Instead of a direct solve, the
 * library relaxes many small independent subvolume problems (Sec. "Iterative
 * relaxation to the least action solution", correction form
 * Eq. (leastaction_correction)) inside a multigrid V-cycle (Sec. "Multigrid
 * Relaxation", Eqs. (residual_rough), (correction_fine)).
 *
 * Discretisation used by this library:
 *   - chi_i: one function per point of a 1D/2D/3D finite-difference grid,
 *     overlap O = identity, H0 = -(1/2m) Lap_h with the (2d+1)-point
 *     Laplacian; values one spacing outside the grid are zero, or the grid
 *     is periodic.  Point coordinates are cell centred,
 *     x_a(i) = (i - (n_a - 1)/2) h.
 *   - T_n: Legendre polynomial P_n mapped onto [t0, t0 + dt], n < n_t
 *     (Sec. "Implementation with Legendre Polynomials"), so that
 *     U = diag(dt/(2n+1)), Q_nm = 2 for n > m with n - m odd, T_n(t0) = (-1)^n
 *     and T_n(t0 + dt) = 1.
 *   - V(x,t) = V0(x) + z E(t), z the coordinate along field_axis.
 *
 * Unknowns of one step, per grid point j: c_j0 .. c_j,n_t-1 and lambda_j.
 * Row (j,m):  i sum_n Q_nm c_jn - U_mm ((T+V0) c)_jm - z_j sum_n W_mn c_jn
 *             + (-1)^m lambda_j = rhs_jm     (rhs = 0 for a forward step),
 * row j:      sum_n (-1)^n c_jn = psi0_j,
 * with W_nm = int T_n T_m E(t) dt over the step.
 *
 * Conventions for every call:
 *   - Device arrays are on the GPU the context was created on and are
 *     accessed on the context's stream only.  Complex arrays are interleaved
 *     (re, im) FP64 ("lam_c64"), i.e. the memory of a torch.complex128 tensor.
 *   - A grid array has one entry per point in C order over the axes (axis
 *     dim-1 contiguous).  A coefficient array c has n_t consecutive entries
 *     per point: c[j * n_t + n].
 *   - Caller memory is never freed or retained by the library.  The context
 *     owns all of its internal device buffers.
 *   - Calls that return a host scalar (a norm, statistics) synchronise the
 *     stream.  Other calls are asynchronous with respect to the host.
 *   - Return value: LAM_OK (0) or a negative LAM_E* code; lam_strerror()
 *     names it.  On error no output is guaranteed to be written.
 *   - A context is not thread safe; calls on one context must not overlap.
 */
#ifndef LAM_H
#define LAM_H

#ifdef __cplusplus
extern "C" {
#endif

#define LAM_OK          0
#define LAM_EINVAL     -1   /* invalid argument: shape, block, level count, n_t, null pointer */
#define LAM_ENOMEM     -2   /* device allocation failed */
#define LAM_EHIP       -3   /* a HIP runtime call failed */
#define LAM_ENOCONV    -4   /* tolerance not reached within max_cycles (outputs still written) */
#define LAM_EDIVERGED  -5   /* residual norm non-finite or grew by more than 1e6 */
#define LAM_ESTATE     -6   /* call needs a state that was never set (lam_set_state) */
#define LAM_ETOOBIG    -7   /* input larger than a no-allocation call's fixed scratch */

#define LAM_MAX_NT     8    /* largest number of Legendre time functions */
#define LAM_MAX_BLOCK  64   /* largest number of grid points in one subvolume */
#define LAM_MAX_INNER  32   /* largest n_inner (inner passes of one subvolume solve) */
#define LAM_MAX_SPLIT  8    /* largest max_split (sub-steps of dt / 256) */
#define LAM_NOALLOC_SCRATCH_BYTES (4u << 20)  /* fixed device scratch per GPU (4 MiB) */

#define LAM_PULSE_NONE          0
#define LAM_PULSE_SIN2          1  /* E = e0 sin^2(pi t/T) cos(omega t) on [0,T] */
#define LAM_PULSE_FOURIER       2  /* E = sum_q coef[q-1] sin(q pi t/T) on [0,T] */
#define LAM_PULSE_SIN2_FOURIER  3  /* sum of the two */

#define LAM_COARSE_REDISCRETISED 0
#define LAM_COARSE_GALERKIN      1

#define LAM_TF_SHARED 0
#define LAM_TF_STORED 1

#define LAM_FP64   0   /* every kernel in FP64 */
#define LAM_MIXED  1   /* subvolume solves in FP32, residuals/transfers/state in FP64 */

typedef struct lam_ctx lam_ctx;
typedef double lam_c64;   /* interleaved complex: element k is (p[2k], p[2k+1]) */

typedef struct {
    int dim;          /* 1, 2 or 3 */
    int n[3];         /* points per axis (entries >= dim ignored) */
    double h;         /* grid spacing of the finest level */
    int periodic;     /* 0: zero values outside the grid; 1: periodic wrap */
    int block[3];     /* subvolume points per axis; must divide n/2^l at every level l,
                         product <= LAM_MAX_BLOCK */
    int levels;       /* multigrid levels, >= 1 (1 = relaxation only); every axis
                         must be even at all levels but the coarsest */
    int nu_pre;       /* full sweeps before the coarse correction */
    int nu_post;      /* full sweeps after it */
    int nu_coarse;    /* full sweeps of the coarsest-level solve (its maximum when the
                         solver's coarse_reduction > 0) */
    int interp;       /* 0: cell-centred tensor-linear interpolation,
                         1: piecewise constant (projection * interpolation = identity) */
    int coarse_op;    /* LAM_COARSE_REDISCRETISED (0): each coarse level is the step
                         operator rediscretised on its grid (kinetic coefficient
                         1/(2 m H^2), H = 2^l h);
                         LAM_COARSE_GALERKIN (1): the Galerkin product R K I of the finer
                         level with piecewise-constant I (interp must be 1): the same
                         operator with the kinetic coefficient 1/(2 m h^2 2^l), halved
                         per level instead of quartered, the potential averaged over
                         children and the field at the coarse cell centres (exactly).
                         Required by the adaptive tree (lam_set_refinement) */
} lam_grid;

typedef struct {
    int n_t;          /* Legendre time functions per step, 1..LAM_MAX_NT */
    double dt;        /* step length */
} lam_time;

typedef struct {
    double mass;          /* particle mass (T = -(1/2m) Lap) */
    const double* v0;     /* device, one FP64 per finest grid point; copied at create */
    int field_axis;       /* axis of the dipole coordinate z (0..dim-1) */
    int pulse_kind;       /* LAM_PULSE_* */
    double e0, omega;     /* sin^2 pulse amplitude and carrier frequency */
    double t_total;       /* pulse length T */
    int n_coef;           /* Fourier sine amplitudes (may be 0) */
    const double* coef;   /* host, n_coef values; copied at create */
} lam_ham;

typedef struct {
    int precision;    /* LAM_FP64 or LAM_MIXED */
    double tol;       /* stop when sqrt(N / N0) <= tol (N: residual norm, N0: at the start) */
    int max_cycles;   /* V-cycle limit per solve */
    int n_inner;      /* most inner corrections of each subvolume solve when E(t) != 0,
                         0..LAM_MAX_INNER or -1 = automatic (16 with a field, 0 without).
                         The factor of a subvolume takes the field's full time matrix W
                         at one dipole coordinate zf, the centre of its slab of
                         subvolumes along the field axis; the corrections remove the
                         rest, (z - zf) W, point by point.  Each subvolume stops once its
                         own residual fell by inner_tol, or stops improving
                         (lam_pass_stats counts both) */
    int time_factor;  /* how each mode's time system is solved inside a sweep:
                         LAM_TF_SHARED (0): one factor shared by all modes (the n_t x n_t
                         system left after each point's continuity row eliminates c_0,
                         in the eigenbasis of its time operator; streams one eigenvalue
                         per mode);
                         LAM_TF_STORED (1): stored per-mode inverses ((n_t+1)^2 complex per
                         mode, refactored for every step with a field) */
    double coarse_reduction;  /* the coarsest-level solve of each V-cycle: 0 = exactly
                         grid.nu_coarse full sweeps; in (0, 1) = full sweeps until the
                         coarsest residual norm sqrt(N) has fallen by this factor from
                         its value at the start of the solve, at most grid.nu_coarse
                         (decided on the device; lam_stats counts sweeps and misses) */
    int max_split;    /* time-step splitting, 0..LAM_MAX_SPLIT (0 = off).  Halving the
                         step halves both dimensionless parameters of the least-action
                         equations (kappa = p_max^2 dt / 2, nu = V dt; Sec. "Implementation
                         with Legendre Polynomials", after Eq. (leastaction_dimensionless)),
                         which brings relaxation back into its convergent regime.  With
                         max_split > 0 a solve is abandoned as soon as its residual norm
                         grows (a checked V-cycle ends above N0, or above the one checked
                         before it while sqrt(N / N0) > 100 tol), diverges or misses tol
                         after max_cycles, and the
                         step is then done as two steps of half its length, each of which
                         may split again, down to dt / 2^max_split.  The result is the
                         state after the sub-steps; lam_stats reports how many were solved
                         and the deepest halving used.  Forward steps (lam_solve_step,
                         lam_propagate) and adjoint steps (lam_adjoint_step, which splits
                         the same way its forward recomputation does) */
    double inner_tol; /* the inner corrections of a subvolume stop once its own residual
                         norm fell by this factor; 0 = the default, 1e-2 in both precisions:
                         the V-cycles converge to the same step solution whatever the
                         tolerance (the relaxation is their smoother, the FP64 residual
                         decides when to stop), a field defect left below 1% of the local
                         residual does not change their rate, and each further correction
                         costs a whole block solve.  Exact subvolume solves, the
                         relaxation as the paper defines it (Sec. "Iterative relaxation to
                         the least action solution"): 1e-13 in FP64, 1e-5 in FP32 (exact to
                         its precision).  0 <= inner_tol < 1 */
} lam_solver;

typedef struct {
    int cycles;           /* V-cycles done */
    int sweeps_fine;      /* full sweeps (both colours) on the finest level */
    double resid0;        /* sqrt(N) of the initial guess */
    double resid;         /* sqrt(N) at the end */
    double t_factor_ms;   /* host time spent on time factors (field steps) this call */
    double t_solve_ms;    /* wall time of the call */
    double resid0_last;   /* sqrt(N) of the initial guess of the last step solved */
    double resid_last;    /* sqrt(N) at the end of the last step solved */
    int coarse_sweeps;    /* full sweeps of the coarsest-level solves (coarse_reduction > 0) */
    int coarse_unmet;     /* V-cycles whose coarsest solve stopped at nu_coarse sweeps before
                             reaching coarse_reduction */
    int substeps;         /* steps solved, counting each sub-step of a split step (1 per
                             unsplit step) */
    int split_depth;      /* the deepest halving used: sub-steps of dt / 2^split_depth */
} lam_stats;

/* Create a propagator context: builds the level hierarchy (coarse grids with
 * doubled spacing and the potential averaged over children) and factors every
 * subvolume operator of every level.  hip_stream: a hipStream_t (NULL = the
 * null stream).  Sec. "Review of the Least Action Principle" (problem
 * statement), Sec. "Multigrid Relaxation" (hierarchy).
 * Errors: LAM_EINVAL (shapes, blocks, levels, n_t, mass, h, dt, pointers),
 * LAM_ENOMEM, LAM_EHIP. */
int lam_create(const lam_grid* grid, const lam_time* time, const lam_ham* ham,
               const lam_solver* solver, void* hip_stream, lam_ctx** out);

/* Release every device buffer of the context.  Accepts NULL.  Resource
 * management only: no passage of the paper. */
int lam_destroy(lam_ctx* ctx);

/* Replace the Fourier pulse amplitudes (host array of n_coef values, n_coef
 * must equal the count given at create): the coefficients of the dipole
 * field E(t) in the time-dependent local potential V(x, t) of the action
 * (Sec. "Review of the Least Action Principle", the V_ijnm term of
 * Eq. (stationaryphase)).  Field matrices and factors are rebuilt on next use;
 * a loaded state keeps its step. */
int lam_set_pulse(lam_ctx* ctx, int n_coef, const double* coef);

/* Replace V0 (device, one FP64 per finest point) and refactor every level:
 * the static part of the local potential of the Hamiltonian (Sec. "Review of
 * the Least Action Principle"), averaged over children on coarser levels
 * (Sec. "Multigrid Relaxation"); every subvolume factor of Sec. "Iterative
 * relaxation to the least action solution" depends on it. */
int lam_set_potential(lam_ctx* ctx, const double* v0);

/* Action residual of a forward step at time t0, Eq. (actionresidual) extended
 * by the multiplier rows: rho = rhs - (stationarity rows applied to (c, lam)),
 * sigma = psi0 - sum_n (-1)^n c_n.  norm (host, may be NULL) receives
 * N = sum_jm U_mm |rho_jm|^2 + sum_j |sigma_j|^2 (Eq. (residnorm) with O = I).
 * psi0, c, lam: device inputs (P, P*n_t, P complex).  rho (P*n_t) and
 * sigma (P) are device outputs and may be NULL. */
int lam_residual_action(lam_ctx* ctx, double t0, const lam_c64* psi0, const lam_c64* c,
                        const lam_c64* lam, lam_c64* rho, lam_c64* sigma, double* norm);

/* Same for the adjoint system K^H mu = E^H g of a step at t0 (E: end-of-step
 * evaluation psi_j = sum_n c_jn, so E^H g puts g_j on every row (j, n)): the
 * conjugate transpose of the step system of Eq. (stationaryphase) and its
 * initial-condition rows (Sec. "Review of the Least Action Principle").
 * g: device (P); mu_c (P*n_t), mu_lam (P): device inputs. */
int lam_residual_adjoint(lam_ctx* ctx, double t0, const lam_c64* g, const lam_c64* mu_c,
                         const lam_c64* mu_lam, lam_c64* rho, lam_c64* sigma, double* norm);

/* Load a forward state into the context: step time t0, initial wavefunction
 * psi0 (P), coefficients c (P*n_t) and multipliers lam (P), all device.
 * Subsequent lam_relax_sweep / lam_vcycle act on the system K x = (0, psi0):
 * the stationarity rows of Eq. (stationaryphase) and the initial-condition
 * rows of one step (Sec. "Review of the Least Action Principle"). */
int lam_set_state(lam_ctx* ctx, double t0, const lam_c64* psi0, const lam_c64* c,
                  const lam_c64* lam);

/* Load an adjoint state: subsequent sweeps / V-cycles act on K^H mu = E^H g,
 * the conjugate-transposed step system (as for lam_residual_adjoint). */
int lam_set_adjoint_state(lam_ctx* ctx, double t0, const lam_c64* g, const lam_c64* mu_c,
                          const lam_c64* mu_lam);

/* Copy the finest-level state (c: P*n_t, lam: P; device) out of the context:
 * the time-expansion coefficients c_jn and multipliers of the step system
 * (Sec. "Review of the Least Action Principle"). */
int lam_get_state(lam_ctx* ctx, lam_c64* c, lam_c64* lam);

/* One colour of subvolume relaxation of the context state on the finest
 * level (level must be 0; a coarse level relaxes a correction problem whose
 * right-hand side only a V-cycle produces, so other levels are LAM_EINVAL):
 * every subvolume of that colour (parity of the sum of its box coordinates)
 * is replaced by x_U + K_UU^{-1} (b - K x)_U with the exterior held fixed
 * (Sec. "Iterative relaxation to the least action solution").  Subvolumes of
 * one colour do not share a face, so they run in parallel.  Acts on the step
 * of the loaded state (lam_set_state / lam_set_adjoint_state), whatever step a
 * residual call looked at since. */
int lam_relax_sweep(lam_ctx* ctx, int level, int colour);

/* One V-cycle on the context state (Eqs. (residual_rough), (correction_fine)):
 * nu_pre sweeps, residual, projection, recursive coarse correction (the
 * coarsest level does nu_coarse sweeps), interpolation, nu_post sweeps.
 * norm (host, may be NULL) receives N of the finest level afterwards. */
int lam_vcycle(lam_ctx* ctx, double* norm);

/* Propagate one step from t0 (Sec. "Review of the Least Action Principle":
 * the least-action solution of one step, continued from its initial value;
 * Sec. "Multigrid Relaxation" for the V-cycles): psi_in (device, P) ->
 * psi_out (device, P, psi_out_j = sum_n c_jn, every T_n being 1 at the end of
 * the step).  V-cycles from the initial guess c_j0 = psi_in_j,
 * c_jn = 0 (n >= 1), lambda = 0 until sqrt(N/N0) <= tol.  stats may be NULL.
 * Returns LAM_ENOCONV (psi_out written) if max_cycles is reached,
 * LAM_EDIVERGED if the norm becomes non-finite or grows by more than 1e6. */
int lam_solve_step(lam_ctx* ctx, double t0, const lam_c64* psi_in, lam_c64* psi_out,
                   lam_stats* stats);

/* Propagate n_steps consecutive steps, step k starting at t0 + k dt, each
 * solved as by lam_solve_step (the step-by-step propagation of Sec. "Review
 * of the Least Action Principle", each step's end value the next one's
 * initial condition): psi_in (device, P) -> psi_out (device, P); the
 * buffers may coincide.  The steps run back to back on the context stream;
 * the host waits only for each batch of norms.  The next step's initial state
 * and its N0 (with its field) are queued ahead of the wait for the current
 * step's last norms, into spare finest-level buffers (P (n_t + 2) complex
 * values, allocated by the context on first use and kept until lam_destroy;
 * if they cannot be allocated, the steps run without them), and the host
 * builds the next step's time factor records during that wait.  stats (may be NULL): cycles and
 * sweeps_fine summed over the steps, resid0/resid of the step with the
 * largest resid/resid0, resid0_last/resid_last of the last step solved,
 * t_factor_ms and t_solve_ms summed.  Stops at the first
 * step that does not return LAM_OK and returns its code (psi_out then holds
 * that step's result for LAM_ENOCONV); n_steps = 0 copies nothing and
 * returns LAM_OK. */
int lam_propagate(lam_ctx* ctx, double t0, int n_steps, const lam_c64* psi_in, lam_c64* psi_out,
                  lam_stats* stats);

/* Backward pass of one step for a real loss L: the adjoint of the step's
 * linear system (Sec. "Review of the Least Action Principle", Eqs.
 * (stationaryphase) and the initial-condition rows; the adjoint is the
 * conjugate-transposed system, solved by the relaxation of Sec. "Iterative
 * relaxation to the least action solution" and the V-cycles of Sec.
 * "Multigrid Relaxation").  psi_in: the step's initial
 * wavefunction (device checkpoint; the forward solve is recomputed from it).
 * g_out = dL/dpsi_out^* (device, P).  Solves K^H mu = E^H g_out with the same
 * relaxation and multigrid machinery, then
 *   g_in   = dL/dpsi_in^* = mu on the initial-condition rows (device, P, written),
 *   dL_dv0 += 2 Re sum_m conj(mu_jm) U_mm c_jm           (device, P, accumulated),
 *   dL_dcoef[q] += 2 Re sum_j z_j sum_mn conj(mu_jm) W^(q)_mn c_jn
 *                                            (host, n_coef, accumulated; may be NULL),
 * with W^(q) the time matrix of the q-th Fourier sine function.
 * stats (may be NULL) describe the adjoint solve. */
int lam_adjoint_step(lam_ctx* ctx, double t0, const lam_c64* psi_in, const lam_c64* g_out,
                     lam_c64* g_in, double* dL_dv0, double* dL_dcoef, lam_stats* stats);

/* Backward pass of one step from its stored forward solution: the adjoint solve
 * and gradients of lam_adjoint_step (the same conjugate-transposed step system
 * of Sec. "Review of the Least Action Principle", the same relaxation and
 * V-cycles), without recomputing the forward solve.  For callers that keep the
 * forward coefficients of every step instead of only the step-boundary
 * wavefunctions: P*n_t complex values per step (2.1 GB at 256^3 with n_t = 8),
 * which the HBM of one GPU holds for tens of steps.
 *   c_fwd: device (P*n_t), the converged coefficients of the forward step at
 *          t0 (lam_get_state after that step's lam_solve_step), read during the
 *          call only;
 *   g_out, g_in, dL_dv0, dL_dcoef, stats: as for lam_adjoint_step.
 * A step whose forward solve was split (lam_stats.substeps > 1) has no single
 * set of coefficients: its backward pass is lam_adjoint_step.  Synchronises
 * the stream.  Errors: LAM_EINVAL (pointers), LAM_ENOCONV (g_in and the
 * gradients written) or LAM_EDIVERGED from the adjoint solve, LAM_EHIP. */
int lam_adjoint_step_stored(lam_ctx* ctx, double t0, const lam_c64* c_fwd, const lam_c64* g_out,
                            lam_c64* g_in, double* dL_dv0, double* dL_dcoef, lam_stats* stats);

/* Grid transfers on caller buffers; `level` is the fine level (0..levels-2).
 * lam_restrict: coarse (rho, sigma) = average of the 2^d children of the fine
 * (rho, sigma) (projection of Eq. (residual_rough)).
 * lam_prolong_add: fine (c, lam) += interpolation of coarse (c, lam)
 * (Eq. (correction_fine)).  All pointers device; sizes follow each level's
 * point count (lam_level_shape). */
int lam_restrict(lam_ctx* ctx, int level, const lam_c64* rho_f, const lam_c64* sigma_f,
                 lam_c64* rho_c, lam_c64* sigma_c);
int lam_prolong_add(lam_ctx* ctx, int level, const lam_c64* c_c, const lam_c64* lam_c,
                    lam_c64* c_f, lam_c64* lam_f);

/* Points per axis of a level (n[3], host): each coarser level doubles the
 * spacing (Sec. "Multigrid Relaxation"). */
int lam_level_shape(const lam_ctx* ctx, int level, int* n);

/* Subvolume factor of block `block` on `level`: eigenvectors (host, bpts*bpts,
 * row-major [point][mode]) and eigenvalues (host, bpts) of the real symmetric
 * spatial block operator T_U + diag(V0_U), the factor that turns each
 * subvolume solve of Sec. "Iterative relaxation to the least action solution"
 * into independent time systems.  For tests of the block factor. */
int lam_block_factor(const lam_ctx* ctx, int level, int block, double* vecs, double* vals);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the residual
 * of lam_residual_action without a context and without any allocation or host
 * synchronisation.  grid, time, ham: as for lam_create (validated the same way;
 * ham->v0 is read by the kernels, so it must stay valid until the stream has
 * run them; ham->coef is read during the call); solver settings play no part.
 * psi0, c, lam: device inputs (P, P*n_t, P complex); rho, sigma: device outputs
 * (may be NULL).  norm (device, one double, may be NULL) receives N, computed
 * through a fixed device scratch array of LAM_NOALLOC_SCRATCH_BYTES per GPU
 * holding one FP64 partial sum per group of floor(256 / n_t) points: so
 * P <= 524288 * floor(256 / n_t) points (16,777,216 at n_t = 8); a larger grid
 * with norm != NULL is LAM_ETOOBIG and nothing runs.  All work is queued on hip_stream (a hipStream_t
 * of the current device; NULL = the null stream).  Every call on one GPU uses
 * that GPU's one scratch array, and every partial it reads is written by the
 * same call first: calls whose work overlaps on one GPU (different streams)
 * race and must be ordered by the caller. */
int lam_residual_action_noalloc(const lam_grid* grid, const lam_time* time, const lam_ham* ham, double t0,
                                const lam_c64* psi0, const lam_c64* c, const lam_c64* lam, lam_c64* rho,
                                lam_c64* sigma, double* norm, void* hip_stream);

/* The adaptive tree (Sec. "Multigrid Relaxation": the tree of elements need
 * not subdivide every volume equally; where the function has little detail a
 * coarse element stands for its children).  The finest level is refined only
 * on the subvolumes whose flag is nonzero; elsewhere the next level is the
 * leaf.  Solves then relax the finest level only on those subvolumes (every
 * coarser level in full) and converge to the composite state
 *     x = x0 + (corrections on the refined subvolumes) + I (coarse corrections),
 *     refined rows of b - K x = 0,   R (b - K x) = 0,
 * with N (the stopping norm, lam_stats resid*) the U-weighted residual norm on
 * the refined rows plus that of the projected residual on level 1.  With every
 * flag set it is the ordinary step solution.  Forward solves only (the adjoint
 * and lam_propagate's step-ahead pipeline run unrefined).
 *   active: host, one byte per finest-level subvolume, in C order of the
 *           subvolume coordinates; NULL clears the refinement (every subvolume).
 * LAM_EINVAL unless levels >= 2 and grid.coarse_op == LAM_COARSE_GALERKIN (with
 * the rediscretised coarse operator the unrefined region is corrected only
 * approximately each cycle and the composite iteration converges slowly). */
int lam_set_refinement(lam_ctx* ctx, const unsigned char* active);

/* Haar detail energy of psi per finest-level subvolume: sum over its points j of
 * |psi_j - (I R psi)_j|^2, where (I R psi)_j is the average of psi over the 2^d
 * children of j's parent cell (R: average over children, I: piecewise constant).
 * The parts I R psi and psi - I R psi are orthogonal (a Haar decomposition);
 * large details mark where the tree should be refined.
 *   psi: device, one complex per finest point; detail: host, one double per
 *   finest subvolume (C order of subvolume coordinates).  Synchronises. */
int lam_block_detail(lam_ctx* ctx, const lam_c64* psi, double* detail);

/* ---- The plane-wave relaxation experiment in the Legendre element basis ----
 * Sec. "Implementation with Legendre Polynomials" (element matrices O, U, Q, T,
 * transfers, continuity) and Sec. "Convergence" (the experiment).  A regime is
 * the dimensionless element operator of Eq. (leastaction_dimensionless),
 *   i O_ij Q_nm - 2 kappa T_ij U_nm - nu O_ij U_nm,
 * on n_x x n_t Legendre functions per element (1..8 each), and a relaxation mode:
 *   LAM_PW_ONE           one element [-1, 1];
 *   LAM_PW_SIMULTANEOUS  two elements [-1, 0], [0, 1] relaxed at once;
 *   LAM_PW_INTERGRID     two elements: the parent element's correction (Galerkin
 *                        problem of Eq. (residual_rough), Eq. (correction_fine)),
 *                        then each element with its interface held fixed.
 * (elements x n_x x n_t <= LAM_PW_MAX_UNKNOWNS).  T_ij is the closed form the
 * paper prints, (j(j+1) - i(i+1))/2 for i > j, i - j even, read as the entry of
 * trial i in test row j. */
#define LAM_PW_ONE           0
#define LAM_PW_SIMULTANEOUS  1
#define LAM_PW_INTERGRID     2
#define LAM_PW_MAX_UNKNOWNS  72

typedef struct {
    int n_x, n_t;        /* Legendre functions per element in space and in time */
    int mode;            /* LAM_PW_* */
    double kappa, nu;    /* kinetic and potential action parameters */
} lam_pw_regime;

/* For every trial f = exp(i(k x + w t)) of the grid (k[ik], w[iw]) (host arrays
 * of nk and nw values; x, t in [-1, 1]): project f onto the element(s) (L2,
 * continuous across the interface), relax once in the correction form with the
 * correction zero at the initial time and at both ends (and continuous inside),
 * and write sqrt(N_after / N_before) to resid_ratio[iw * nk + ik] and
 * |S_after| / |S_before| to action_ratio[iw * nk + ik] (device, FP64), where
 * N = r^H (O (x) U) r is the norm of the residual r = -A C (without multiplier
 * terms) and S = C^H A C the action.  A trial whose residual or action is zero
 * gives NaN.  The call builds the regime's matrices on the host, copies them to
 * a device buffer it allocates, runs the kernel on hip_stream (NULL = null
 * stream), synchronises it and frees the buffer.  Errors: LAM_EINVAL (sizes,
 * mode, pointers, a singular reduced system), LAM_ENOMEM, LAM_EHIP. */
int lam_plane_wave_map(const lam_pw_regime* regime, int nk, const double* k, int nw, const double* w,
                       double* resid_ratio, double* action_ratio, void* hip_stream);

/* Inner passes of the subvolume solves on `level`: hist (host, LAM_MAX_INNER
 * + 2 entries) receives in hist[p] the number of subvolumes whose last solve
 * took p inner corrections (0 without field) and in hist[LAM_MAX_INNER + 1]
 * the number whose last solve stopped with its local residual above the
 * tolerance (pass limit reached, or corrections that stopped improving).
 * The inner corrections take the time-dependent field term of the block
 * system (the V_ijnm term of Eq. (stationaryphase)) into account by repeated
 * solves with the field-free factor.
 * Synchronises the stream.  For measurements and tests. */
int lam_pass_stats(lam_ctx* ctx, int level, long long* hist);

/* Timing of finest-level sweep launches with HIP events on the context
 * stream (measurement only: no passage of the paper).  enable = k > 0 starts recording (clearing previous records) the
 * 1st, (k+1)-th, (2k+1)-th ... finest-level sweep launch: a sample, since each
 * event record costs a few microseconds of stream time; 0 stops; negative is
 * LAM_EINVAL.  lam_profile_read returns the number of recorded launches and
 * their summed kernel time (ms) since the last enable; it synchronises the
 * stream. */
int lam_profile(lam_ctx* ctx, int enable);
int lam_profile_read(lam_ctx* ctx, int* launches, double* total_ms);

/* Text of a LAM_* return code (static storage; unknown codes give a generic
 * text).  No passage of the paper. */
const char* lam_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* LAM_H */
