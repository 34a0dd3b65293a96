/*
 * stmg.h -- C ABI of the MI355X space-time multigrid library (libstmg.so).
 *
 * The library solves the all-at-once space-time system of a reaction-
 * diffusion problem discretized by finite differences in space and by
 * right-Radau collocation / DG in time (Benedusi, Minion, Krause: "An
 * experimental comparison of a space-time multigrid method with PFASST for a
 * reaction-diffusion problem").  The system is Eq. (st_system) of Sec. 3:
 * one block row per time step ("slab"), diagonal blocks
 * A = K_q (x) M_h + M_q (x) K_h and sub-diagonal blocks B = -J_q (x) M_h
 * (Eq. A_B_ops), here with the lumped mass divided out of every spatial row,
 * so that K_h becomes -nu Lap_h + lambda (2nd-order central differences).
 * With M_q = dt diag(b) and J_q = l(0) e_M^T (exact for right Radau nodes),
 * the operator acting on a space-time vector U is
 *
 *   (A U)_{n,i} = sum_j Kq[i,j] U_{n,j} + dt b_i (-nu Lap_h U_{n,i} + R(U_{n,i}))
 *                 - [n > 0] l_i(0) U_{n-1,M}
 *   b_{n,i}     = [n = 0] l_i(0) u0                     (Sec. 3, padding of u_0)
 *
 * with R(u) = lambda u (linear) or gamma (u^3 - u) (Allen-Cahn, Eq. model).
 *
 * Data layout.  Every space-time vector is a contiguous FP64 array
 * [N][M][ny][nx] (slab, node, then space with x fastest), the node-major,
 * space-minor ordering of Sec. 3.  A 1D problem has ny = 1.  Periodic grids
 * have nx points per dimension (h = length / nx); Neumann grids have nx + 1
 * points (h = length / nx, ghost reflection at both ends, which is the
 * lumped linear-FE operator of Sec. 3 divided by the lumped mass).
 *
 * Memory and streams.  The caller owns every device array, including one
 * workspace buffer whose size comes from stmg_workspace_bytes(); it must
 * stay allocated while the handle lives.  The library never allocates or
 * frees device memory.  All work is enqueued on the stream given at setup
 * (a hipStream_t passed as void*, NULL = the null stream).  Calls that
 * return host scalars (norms, statistics, d loss / d nu) synchronize that
 * stream before returning; all other calls are asynchronous.
 *
 * Errors.  Every int-returning function returns STMG_OK (0) or a negative
 * stmg_status.  No exception or abort crosses the ABI.  A description of the
 * last failure on the calling thread is returned by stmg_last_error().
 * Calls on one handle must not overlap (one host thread at a time).
 */
#ifndef STMG_H
#define STMG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STMG_OK = 0,
  STMG_EINVAL = -1,        /* invalid argument or problem description       */
  STMG_ENOMEM = -2,        /* workspace too small                             */
  STMG_EHIP = -3,          /* a HIP runtime call failed                       */
  STMG_ENOTCONV = -4,      /* max_cycles reached before rtol ("n.c.", Sec. 5.2) */
  STMG_EDIVERGED = -5,     /* residual grew by 1e3, or by > 10% per cycle for 5 cycles in a row */
  STMG_ENAN = -6,          /* a residual norm was NaN or Inf                  */
  STMG_EUNSUPPORTED = -7   /* valid but not supported (e.g. coarsest too big) */
} stmg_status;

enum { STMG_BC_PERIODIC = 0, STMG_BC_NEUMANN = 1 };
enum { STMG_REACT_LINEAR = 0, STMG_REACT_ALLEN_CAHN = 1 };
enum { STMG_PREC_FP64 = 0, STMG_PREC_MIXED = 1 };
enum { STMG_COARSEN_AUTO = 0, STMG_COARSEN_SPACE = 1, STMG_COARSEN_SPACETIME = 2,
       STMG_COARSEN_SMMG = 3 };
enum { STMG_FORM_DG = 0, STMG_FORM_COLLOC = 1 };
enum { STMG_SMOOTH_PBJ = 0, STMG_SMOOTH_SDC = 1 };
enum { STMG_COARSE_REDISC = 0, STMG_COARSE_GALERKIN = 1 };

/* The problem statement: Eq. (model) of Sec. 3 generalized to a diffusion
 * coefficient, 2D and periodic grids; uniform partitions of Sec. 3. */
typedef struct {
  int32_t dim;        /* 1 or 2                                              */
  int32_t nx[2];      /* elements per dimension (nx[1] ignored when dim = 1) */
  double length[2];   /* domain size X (and Y)                               */
  int32_t bc;         /* STMG_BC_PERIODIC or STMG_BC_NEUMANN                 */
  double nu;          /* diffusion coefficient (> 0)                         */
  int32_t reaction;   /* STMG_REACT_LINEAR: f = nu Lap u - lambda u
                         STMG_REACT_ALLEN_CAHN: f = nu Lap u + gamma (u - u^3) */
  double lambda;      /* linear reaction rate (>= 0)                         */
  double gamma;       /* Allen-Cahn reaction intensity                       */
  int32_t M;          /* right Radau nodes per step, 1..8 (Sec. 2.1)         */
  int32_t N;          /* time steps (slabs)                                  */
  double dt;          /* step size; T = N dt                                 */
} stmg_problem;

/* Solver options.  stmg_default_options() fills the defaults shown. */
typedef struct {
  int32_t precision;  /* STMG_PREC_FP64 (default) or STMG_PREC_MIXED: FP32
                         smoother and transfers inside FP64 refinement        */
  int32_t coarsen;    /* AUTO (default): space if mu_l = nu dt_l / h_l^2 >=
                         mu_crit, else time (Sec. 4.2); SPACE = SMG;
                         SPACETIME = STMG (both at once); SMMG = space
                         coarsening with M lowered by one per level until
                         M = 1 (Lagrange node transfer, R = P^T; linear
                         reaction only)                                       */
  double mu_crit;     /* 0.5                                                 */
  double omega;       /* smoother damping, 0.8                                */
  int32_t chunk;      /* smoother block length in slabs on the finest level,
                         16 (1 = point-block Jacobi over single slabs)        */
  int32_t chunk_coarse; /* the same on the coarser levels, 4                  */
  int32_t nu_pre;     /* pre-smoothing sweeps, 1                              */
  int32_t nu_post;    /* post-smoothing sweeps, 1                             */
  int32_t max_levels; /* 30                                                  */
  int32_t min_coarse; /* stop coarsening at <= this many unknowns, 64         */
  int32_t max_cycles; /* 200                                                 */
  double rtol;        /* stop at ||b - A U||_2 <= rtol ||b||_2, 1e-12          */
  double newton_rtol; /* Allen-Cahn: stop Newton at ||G(U)|| <= newton_rtol
                         ||b||, 1e-10                                          */
  int32_t max_newton; /* 30                                                  */
  size_t mem_budget;  /* adjoint: max bytes for the stored forward trajectory;
                         0 = unlimited (no checkpointing)                     */
  int32_t sdc;        /* 1: reserve workspace for stmg_sdc_sweep, 0 (default) */
  int32_t autotune;   /* 1: at setup (stmg_setup, stmg_batch_setup), time the
                         launch shape of the restriction kernels (slabs per
                         workgroup run) per level and keep the fastest
                         (results are bitwise identical for every shape);
                         choices are cached in the JSON file named by
                         $STMG_TUNE_CACHE, keyed by level shape, M, precision
                         and coarse smoother block.  0 (default): fixed
                         shapes                                               */
  int32_t inner_cycles; /* mixed precision: FP32 V-cycles on each correction
                         equation per FP64 refinement step (at most, with
                         inner_adapt; exactly, in batches), 1..64, 5          */
  int32_t fft_coarse; /* periodic grids with a linear reaction: coarsening
                         also stops at the first level below the finest whose
                         planes hold <= 1024 points (2D: or have power-of-two
                         sides of <= 64 points) and which holds <=
                         fft_coarse unknowns; that level is solved exactly by
                         Fourier diagonalization in space and the slab
                         recurrence per mode.  4194304; 0 = off               */
  int32_t krylov;     /* restart length m (1..32) of an outer flexible GMRES
                         around the cycles: one V-cycle from a zero guess is
                         the right preconditioner of each Krylov step (FP32
                         cycles with STMG_PREC_MIXED, the Krylov vectors stay
                         FP64).  The stop test is unchanged (true residual,
                         rtol), `cycles` counts V-cycles = Krylov steps and
                         max_cycles bounds them; 2 (m + 1) more level-0
                         vectors of workspace.  Ignored by batches.
                         0 (default): the plain V-cycle iteration             */
  int32_t krylov_left; /* with krylov > 0: 1 = left preconditioning, GMRES on
                         M^-1 A U = M^-1 b stopping when the preconditioned
                         residual ||M^-1 (b - A U)|| has fallen by rtol
                         against its value at the initial guess (PETSc's
                         default, the stop the paper reports, Sec. 5.2);
                         rel_res still reports the true residual and cycles
                         counts every V-cycle (one more per restart).  The
                         V-cycle must then be a fixed operator: FP64 or FP32
                         cycles alike.  0 (default): flexible GMRES, right
                         preconditioning, true-residual stop                 */
  int32_t inner_adapt; /* mixed precision: 1 (default) = from the second
                         refinement step on, run only as many of the
                         inner_cycles FP32 cycles as the previous step's
                         contraction per cycle says are needed to reach rtol
                         (at least 1); the stop test is unchanged.  0 = always
                         inner_cycles.  Ignored by batches.                    */
  int32_t form;       /* the form of the all-at-once system whose residuals
                         are reported and tested: STMG_FORM_DG (default), the
                         DG form Eq. (st_system) of Sec. 3, or
                         STMG_FORM_COLLOC, the collocation form of Sec. 2.1
                         (Eq. collocation), whose residual is G r_DG per slab
                         and grid point with G = Q diag(b)^-1 (the same
                         solution; G l(0) = 1, so ||b|| = sqrt(M) ||u0||).
                         Affects stmg_residual (r and its norm), rel_res and
                         the stop tests of stmg_solve / stmg_vcycle on the
                         forward problem; the correction equations, the
                         smoother (invariant under G) and the adjoint stay in
                         the DG form.  EUNSUPPORTED with krylov > 0; batches
                         use the DG form.                                      */
  int32_t smoother;   /* STMG_SMOOTH_PBJ (default): block-Jacobi over chunks of
                         slabs with point-block M x M solves (Sec. 4.2);
                         STMG_SMOOTH_SDC: on the finest level each smoothing
                         step is one SDC sweep (the implicit-Euler
                         preconditioned Richardson step of Sec. 2.1 and 4.1,
                         all slabs at once, as stmg_sdc_sweep) on the
                         collocation form; coarser levels keep block-Jacobi.
                         FP64 linear problems without Krylov or time windows
                         (EUNSUPPORTED otherwise)                              */
  int32_t coarse_op;  /* STMG_COARSE_REDISC (default): every coarse level
                         rediscretizes the problem with its own h and dt;
                         STMG_COARSE_GALERKIN: coarse levels A_{l+1} =
                         R A_l P (Sec. 4.2), i.e. K_q (x) Ms + diag(dt b) (x)
                         Ks on the slab blocks and -l(0) e_M^T (x) Ms below
                         them, with 3 x 3 mass and stiffness stencils Ms, Ks
                         (9 points in 2D).  Their point-block sweep uses
                         the stencils' centres, damped by omega m_0 / sum|m|.
                         Space coarsening only (coarsen = SPACE), periodic
                         grids, linear reaction, Fourier coarsest solve
                         (EUNSUPPORTED otherwise)                             */
  int32_t pfasst_levels; /* >= 2: the handle also runs PFASST
                         (stmg_pfasst_solve) with this many levels: the
                         problem's grid and M, then bisections in space with
                         M = 1 (Sec. 5.2, PFASST item).  0 (default): not set
                         up.  FP64 without Krylov or time windows; an
                         Allen-Cahn reaction is explicit in the sweeps (IMEX,
                         Sec. 5.4); every level's element counts even, the
                         coarsest grid at least 3 points per dimension
                         (EUNSUPPORTED or EINVAL otherwise)                  */
  int32_t pfasst_sweeps; /* SDC sweeps per level and PFASST iteration (nu of
                         PFASST^L_nu; default 1)                              */
  int32_t pfasst_inner_cycles; /* > 0: every inner solve of stmg_pfasst_solve
                         (the SDC node solves, the M = 1 level solves) stops
                         after at most this many V-cycles, warm-started where
                         the sweep allows (inexact spatial solves, as the
                         paper's few ILU(0)-PGMRES iterations); 0 (default):
                         to rtol.  0..100                                     */
} stmg_options;

typedef struct {
  int32_t cycles;       /* V-cycles done (all Newton steps together)         */
  int32_t newton_its;   /* Newton iterations (Allen-Cahn)                    */
  int32_t refinements;  /* FP64 refinement steps (mixed precision)           */
  int32_t status;       /* final status of the call                          */
  double rel_res;       /* final ||b - A U|| / ||b||                         */
  double seconds;       /* wall time of the call (host clock, synchronized)  */
} stmg_stats;

typedef struct stmg_handle stmg_handle;
typedef struct stmg_batch stmg_batch;

void stmg_default_options(stmg_options* opt);

/* Bytes of device workspace needed by stmg_setup for this problem/options,
 * or 0 if the description is invalid (see stmg_last_error). */
size_t stmg_workspace_bytes(const stmg_problem* prob, const stmg_options* opt);

/* Builds the Radau tables (Sec. 2.1/2.2), the level hierarchy and the
 * coarsest-level factors, and copies the device tables into d_ws.  d_ws must
 * be 256-byte aligned and at least stmg_workspace_bytes() long.  Returns the
 * handle in *out.  EINVAL: M outside 1..8, N < 1, dt <= 0, nu <= 0, fewer
 * than 3 points per dimension, dim not 1 or 2, or a NULL pointer.
 * EUNSUPPORTED: the coarsest level would have more than 1024 unknowns per
 * slab. */
int stmg_setup(const stmg_problem* prob, const stmg_options* opt, void* d_ws,
               size_t ws_bytes, void* stream, stmg_handle** out);

/* Number of levels and the shape of level l: out[0] = points in x, out[1] =
 * points in y, out[2] = slabs, out[3] = coarsening kind to level l+1
 * (bits: 1 space, 2 time, 4 collocation nodes; 0 none).  Host only. */
int stmg_num_levels(const stmg_handle* h);
int stmg_level_shape(const stmg_handle* h, int level, int32_t out[4], double* dt);
/* Collocation nodes M_l on level l (M on every level except under SMMG), or a
 * negative status.  Host only. */
int stmg_level_nodes(const stmg_handle* h, int level);

/* r = b - A(U) on the finest level (Eq. st_system), b built from u0.
 * d_u0: [ny][nx]; d_U: [N][M][ny][nx]; d_r may be NULL (norm only).
 * h_norm (may be NULL) receives ||r||_2 and synchronizes the stream. */
int stmg_residual(stmg_handle* h, const double* d_u0, const double* d_U,
                  double* d_r, double* h_norm);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * residual of stmg_residual without a handle or workspace.  The problem is
 * described as for stmg_setup (default options); d_u0, d_U, d_r and h_norm
 * are as in stmg_residual, and the work goes on `stream` (a hipStream_t of
 * the current device, NULL = null stream).  The per-block partial sums of
 * ||r||^2 live in a fixed device array of 1 MiB + 256 bytes inside the
 * library (one per GPU, kept until the process ends); no device or pinned
 * memory is allocated.  EINVAL when the problem needs more partial sums than
 * that array holds (ceil(nx ny / 256) * ceil(N / 8) must not exceed 131072,
 * e.g. 512 x 512 points with N <= 1024 slabs), and the errors of
 * stmg_setup's problem checks.  Every call on one GPU shares that array:
 * calls that overlap on one GPU (other host threads, or other streams
 * before the earlier call's stream has finished) race and must not be
 * issued.  With h_norm non-NULL the call synchronizes `stream`. */
int stmg_residual_noalloc(const stmg_problem* prob, const double* d_u0, const double* d_U,
                          double* d_r, double* h_norm, void* stream);

/* One V-cycle (Sec. 4.2) on A U = b, updating d_U in place.  h_rel (may be
 * NULL) receives ||b - A U|| / ||b|| after the cycle and synchronizes.
 * On an Allen-Cahn handle the cycle acts on the Jacobian at the last Newton
 * linearization point, with b the last Newton right-hand side; before the
 * first stmg_solve on the handle there is none and the call returns
 * STMG_EINVAL. */
int stmg_vcycle(stmg_handle* h, const double* d_u0, double* d_U, double* h_rel);

/* Solves the all-at-once system from the initial guess in d_U (zero is the
 * paper's choice, Sec. 5.2): V-cycles (FP64, or FP32 cycles inside FP64
 * refinement when precision = MIXED) until rel_res <= rtol, or with
 * options.krylov = m > 0 restarted flexible GMRES(m) preconditioned by one
 * V-cycle per step (the preconditioned Krylov iteration of Sec. 5.2), wrapped
 * in Newton for Allen-Cahn (Sec. 4.2).  d_U receives the solution (the last
 * iterate on ENOTCONV/EDIVERGED/ENAN).  stats may be NULL.  Synchronizes. */
int stmg_solve(stmg_handle* h, const double* d_u0, double* d_U, stmg_stats* stats);

/* Like stmg_solve but returns only the end value u(T) = U_{N,M} ([ny][nx])
 * in d_uT.  Only on a handle whose options' mem_budget is too small for the
 * trajectory (time windows, see stmg_num_windows): the solve runs window by
 * window and keeps the window start values as checkpoints in the workspace,
 * so the trajectory is never stored.  EUNSUPPORTED on other handles. */
int stmg_solve_end(stmg_handle* h, const double* d_u0, double* d_uT, stmg_stats* stats);

/* Slabs per workgroup run of the restriction from `level` to level + 1 (the
 * autotuned value with options.autotune, else the fixed default); 0 for the
 * coarsest level.  Host only. */
int stmg_tuned_shape(const stmg_handle* h, int level);

/* Number of time windows (0: the handle holds the whole trajectory).  A
 * positive mem_budget smaller than about five FP64 trajectories makes the
 * handle split the N slabs into windows of W = 2^k slabs, W the largest with
 * six window vectors within the budget.  stmg_solve then solves window after
 * window (exact: the system is block lower-triangular); stmg_vcycle,
 * stmg_residual, stmg_coarse_solve and the stmg_level_* calls return
 * EUNSUPPORTED.  Host only. */
int stmg_num_windows(const stmg_handle* h);

/* Gradients of L = || U_{N,M} - u_tgt ||^2 (linear problems, periodic grids).  d_U is the
 * converged forward solution; d_gT = dL/du(T) = 2 (U_{N,M} - u_tgt), [ny][nx].
 * Solves the transposed system A^T lam = g (backward in time, same V-cycle
 * kernels) and returns d_grad_u0 = sum_i l_i(0) lam_{0,i} ([ny][nx], device)
 * and *h_grad_nu = sum_{n,i,x} lam_{n,i} dt b_i (Lap_h U_{n,i})(x).  On a
 * windowed handle the windows are processed backward in time, each with its
 * trajectory taken from d_U or, when d_U is NULL, recomputed from its
 * checkpoint (d_u0 required then).  Without windows d_U is required and d_u0
 * may be NULL.  Synchronizes. */
int stmg_adjoint(stmg_handle* h, const double* d_u0, const double* d_U,
                 const double* d_gT, double* d_grad_u0, double* h_grad_nu,
                 stmg_stats* stats);

/* `sweeps` SDC sweeps (Sec. 2.1 and 4.1: preconditioned Richardson on the
 * collocation form U = 1 (x) u_{n-1} + dt (Q (x) I) F(U), with the
 * implicit-Euler lower-triangular Q_Delta) over all slabs at once, the
 * previous slab's end value lagged (Jacobi across slabs).  Per sweep and
 * node m the implicit solve (I - dt Q_Delta[m][m] L) delta_m = ... runs as
 * spatial V-cycles (the same kernels with M = 1, all slabs batched) to rtol.
 * d_U is updated in place; h_rel (may be NULL) receives ||b - A U|| / ||b||
 * (DG form) afterwards.  With the Allen-Cahn reaction the sweep is IMEX: the
 * reaction explicit with the explicit-Euler weights c_{j+1} - c_j on the
 * node intervals' left ends (Sec. 5.4).  Handles set up with options.sdc = 1
 * (EUNSUPPORTED otherwise). */
int stmg_sdc_sweep(stmg_handle* h, const double* d_u0, double* d_U,
                   int32_t sweeps, double* h_rel);

/* PFASST (Sec. 4.1; Sec. 5.2, PFASST item) on the collocation form of the
 * problem, for a handle set up with options.pfasst_levels = L >= 2.  One
 * iteration: on levels 0 .. L-2, pfasst_sweeps SDC sweeps (the sweep of
 * stmg_sdc_sweep on level 0; on the M = 1 levels an exact per-slab solve
 * with the previous slab's end value from the incoming iterate), then the
 * FAS restriction to the next level (space full weighting of the end-node
 * values; tau_{l+1} = R_s [tau_l + dt (Q L V)_M] - dt L_{l+1} R_s V_M); on
 * the coarsest level the serial sweep, which at M = 1 is the exact solve of
 * its block lower-bidiagonal system (done all slabs at once by that level's
 * own multigrid solver to rtol); going up, the coarse corrections e_n are
 * interpolated bilinearly in space and linearly in time between the slab's
 * start and end, V_{n,i} += P ((1 - c_i) e_{n-1} + c_i e_n), followed by
 * the sweeps on the M = 1 levels.  With the Allen-Cahn reaction every sweep
 * is IMEX (reaction explicit with the explicit-Euler weights, diffusion
 * implicit) and the coarsest serial sweep runs slab after slab.  d_U holds
 * the initial guess and receives
 * the iterate; stops at ||b - A U|| / ||b|| <= rtol (in the handle's form)
 * or after max_cycles iterations (stats.cycles = iterations; ENOTCONV,
 * EDIVERGED and ENAN as stmg_solve).  Inner solves stop at rtol: the SDC
 * node solves relative to their first residual, the M = 1 level solves
 * relative to (||f||^2 + ||u0||^2)^{1/2} of their right-hand side.
 * EUNSUPPORTED on a handle without PFASST levels. */
int stmg_pfasst_solve(stmg_handle* h, const double* d_u0, double* d_U, stmg_stats* stats);

/* Component entry points on level `level` of the hierarchy (FP64):
 *   smooth : U_out = U_in + omega D^{-1} (f - A_l U_in); the block-Jacobi
 *            sweep over chunks of slabs (Sec. 4.2); U_in may be NULL (zero)
 *   restrict_residual : f_coarse = R (f - A_l U)  (Eq. space_time_tran)
 *   prolong : U_out = U_in + P e_coarse            (transpose structure)
 *   coarse_solve : U = A_L^{-1} f on the coarsest level (exact, Sec. 4.2)
 * On level 0, f may be NULL, meaning the right-hand side built from d_u0. */
int stmg_level_smooth(stmg_handle* h, int level, const double* d_f,
                      const double* d_u0, const double* d_Uin, double* d_Uout);
int stmg_level_restrict_residual(stmg_handle* h, int level, const double* d_f,
                                 const double* d_u0, const double* d_U, double* d_fc);
int stmg_level_prolong(stmg_handle* h, int level, const double* d_Uin,
                       const double* d_ec, double* d_Uout);
int stmg_coarse_solve(stmg_handle* h, const double* d_f, double* d_U);
/* The V-cycle's way up on level `level` as one fused sweep: U' = U_in +
 * P e_coarse, then one block-Jacobi sweep U_out = U' + omega D^{-1} (f -
 * A_l U') (Sec. 4.2: prolongation followed by post-smoothing).  The same
 * result as stmg_level_prolong followed by stmg_level_smooth, without storing
 * U'.  U_in may be NULL (zero); on level 0 f may be NULL (built from d_u0).
 * EUNSUPPORTED on grids other than periodic ones with even point counts and
 * on windowed handles. */
int stmg_level_prolong_smooth(stmg_handle* h, int level, const double* d_f, const double* d_u0,
                              const double* d_Uin, const double* d_ec, double* d_Uout);
/* The V-cycle's way down on level 0 as one fused sweep (Sec. 4.2: the
 * pre-smoothing sweep, then the restriction of the new residual): U_out =
 * U_in + omega C^{-1} (f - A_0 U_in) (the block-Jacobi sweep of
 * stmg_level_smooth), d_fc = R (f - A_0 U_out) (as stmg_level_restrict_residual
 * of U_out), and when d_uc is not NULL the coarse level's first block-Jacobi
 * sweep from zero with d_fc as right-hand side.  The residual of U_out is
 * formed from the sweep's own residual and correction, so the result agrees
 * with the two separate calls up to rounding.  Arrays in the level layouts
 * [N][M][ny][nx] (d_fc, d_uc: level 1); U_in may be NULL (zero), f may be
 * NULL (built from d_u0).  EUNSUPPORTED unless the problem is 2D, periodic
 * and linear, level 0 coarsens in space only, nx is a multiple of 64, ny of
 * 16, M <= 4 and the level-0 smoother chunk a multiple of the level-1 one
 * (at most 8); EINVAL for a level other than 0. */
int stmg_level_smooth_restrict(stmg_handle* h, int level, const double* d_f, const double* d_u0,
                               const double* d_Uin, double* d_Uout, double* d_fc, double* d_uc);

void stmg_destroy(stmg_handle* h);

/* Batched independent linear problems (mixed precision to rtol): one
 * phase-kernel launch per multigrid phase for all problems at once, one
 * refinement step (FP64 residual, inner_cycles FP32 V-cycles, FP64 update)
 * captured in a HIP graph; stats report cycles = refinements x inner_cycles.
 * d_u0[p], d_U[p] are the per-problem device arrays.  Synchronizes in solve. */
size_t stmg_batch_workspace_bytes(int32_t n, const stmg_problem* probs,
                                  const stmg_options* opt);
int stmg_batch_setup(int32_t n, const stmg_problem* probs, const stmg_options* opt,
                     void* d_ws, size_t ws_bytes, void* stream, stmg_batch** out);
int stmg_batch_solve(stmg_batch* b, const double* const* d_u0, double* const* d_U,
                     stmg_stats* stats /* [n], may be NULL */);
void stmg_batch_destroy(stmg_batch* b);

const char* stmg_status_string(int status);
const char* stmg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* STMG_H */
