/*
 * dbs.h -- C ABI of the MI355X (gfx950) implementation of one PISO time step
 * of the two-phase micro-continuum Darcy-Brinkman-Stokes method of Carrillo,
 * Bourg and Soulaine (arXiv:2003.08374).
 *
 * The problem follows the paper's summary of the model, Eq.
 * (two-phase-microcontinuum) in Sec. 2.2: the saturation alpha (wetting
 * phase), the single-field (superficial) velocity U, the pressure p (solved
 * as p_rgh = p - rho g.x), the porosity phi and the permeability k go in;
 * advanced fields come out.  One call of dbs_step advances dt with the
 * sequence of Sec. 3.2: MULES saturation transport with the relative flux of
 * Sec. 2.3, property update (App. A closures, App. B capillary force),
 * momentum predictor with the Darcy drag of Eq. (single-field-kr) in its
 * Sec. 2.3 summary form, and n_corr pressure correctors (Eqs.
 * (corrected_velocity), (pressure_predictor)) whose pressure equation is
 * solved by conjugate gradients preconditioned with a geometric multigrid
 * V-cycle.
 *
 * Mesh: uniform Cartesian nx*ny*nz, cell-centred.  Cell arrays hold nx*ny*nz
 * doubles, index i + nx*(j + ny*k).  Face arrays are concatenated x|y|z:
 * (nx+1)*ny*nz x-faces (index i + (nx+1)*(j + ny*k)), then nx*(ny+1)*nz
 * y-faces (index i + nx*(j + (ny+1)*k)), then nx*ny*(nz+1) z-faces (index
 * i + nx*(j + ny*k)); a face value is a volumetric flux [m^3/s] oriented
 * along +axis.  Vector cell fields (U) are component-major: Ux | Uy | Uz.
 * Domain faces: 0 x-, 1 x+, 2 y-, 3 y+, 4 z-, 5 z+.
 *
 * Ownership: the caller owns every host buffer; calls copy in or out and
 * never keep caller pointers.  The library owns its device state from
 * dbs_create to dbs_destroy.  The *_dev calls borrow caller device buffers
 * only for the duration of the call.
 *
 * Errors: every int-returning call returns DBS_OK (0) or a negative DBS_E*
 * code and records a message readable with dbs_last_error.  No C++
 * exception crosses this boundary.  A handle is not thread-safe: calls on
 * one handle must not overlap.
 */
#ifndef DBS_H
#define DBS_H

#ifdef __cplusplus
extern "C" {
#endif

#define DBS_OK 0
#define DBS_EINVAL (-1)   /* invalid argument or input field */
#define DBS_ENOMEM (-2)   /* device allocation failed */
#define DBS_EHIP (-3)     /* HIP runtime error */
#define DBS_ENOCONV (-4)  /* pressure solve hit p_maxit; state = last iterate */
#define DBS_ENAN (-5)     /* non-finite value in the state after a step */
#define DBS_ECOURANT (-6) /* Courant number above max_courant; step not taken */
#define DBS_EBOUNDS (-7)  /* alpha left [-bounds_tol, 1 + bounds_tol] */

enum { DBS_BC_WALL = 0, DBS_BC_INLET = 1, DBS_BC_OUTLET = 2, DBS_BC_EMPTY = 3, DBS_BC_WAVE = 4 };
enum { DBS_BROOKS_COREY = 0, DBS_VAN_GENUCHTEN = 1 };
enum { DBS_FP64 = 0, DBS_MIXED = 1 };

typedef struct {
  int nx, ny, nz;       /* cells per axis; nz = 1 with EMPTY z faces is 2D */
  double dx, dy, dz;    /* cell size [m] */
} dbs_grid;

typedef struct {
  double rho_l, rho_g;  /* densities of the wetting (alpha) and other phase */
  double mu_l, mu_g;    /* viscosities [Pa s] */
  double g[3];          /* gravity [m/s^2] */
  double c_alpha;       /* interface compression coefficient (Sec. 2.3) */
  int kr_model;         /* DBS_BROOKS_COREY or DBS_VAN_GENUCHTEN (App. A.1) */
  double kr_m;          /* exponent m */
  double s_lirr, s_girr;/* irreducible saturations */
  int pc_model;         /* DBS_BROOKS_COREY or DBS_VAN_GENUCHTEN (App. A.2) */
  double pc0;           /* entry capillary pressure [Pa] */
  double pc_exp;        /* beta (Brooks-Corey) or m (Van Genuchten) */
  double a_pcirr, a_pcmax; /* saturation range of the p_c model */
  double eps_pc;        /* clamp of the normalised p_c saturation (>0) */
  double sigma;         /* interfacial tension [N/m], >= 0.  In solid-free cells
                           the continuum surface force of Sec. 2.2 (Brackbill's
                           CSF) adds sigma kappa grad(alpha) / phi, kappa =
                           div(n_lg) = -div(grad(alpha)/|grad(alpha)|), positive
                           for a liquid drop; porous cells keep the App. B
                           capillary force.  0 switches it off (no extra work).
                           */
  double contact_angle; /* penalized contact angle theta [rad] in [0, pi), measured
                           through the alpha = 1 phase, imposed on every face between
                           a clear and a porous cell (Sec. 2.3, locally modified
                           normal): that face's normal flux in the curvature becomes
                           -cos(theta) (n_w . e_axis) |n_f|, n_w pointing from the
                           porous into the clear cell.  0 = not imposed. */
} dbs_physics;

typedef struct {
  int kind;             /* DBS_BC_* */
  double U[3];          /* inlet velocity */
  double alpha;         /* inlet alpha; outlet backflow alpha */
  double p;             /* outlet static pressure p [Pa] */
  double wave[3];       /* DBS_BC_WAVE (x faces): amplitude A [m], period T [s] and
                           still-water depth d [m] above y = 0 of a linear wave:
                           surface d + A sin(w t), w = 2 pi / T, w^2 = |g| k tanh(k d);
                           below it alpha = 1, u = A w cosh(k y)/sinh(k d) sin(w t)
                           into the domain and v = A w sinh(k y)/sinh(k d) cos(w t);
                           above it alpha = 0 and U = 0.  Values of a step are taken
                           at its end time; outflowing faces carry the cell alpha.
                           The paper gives no formula for its coastal-barrier inlet
                           (Sec. 4.2); this is linear wave theory. */
} dbs_bc;

typedef struct {
  double dt;            /* time step [s] */
  int n_corr;           /* PISO correctors (>= 1, the paper uses >= 2) */
  int mom_maxit;        /* sweep cap of the momentum predictor solve (0: U* = U^n) */
  int transpose_visc;   /* 1: add div(mu grad(U)^T) explicitly */
  int mules_iter;       /* MULES limiter iterations (>= 1) */
  double p_tol;         /* pressure solve: ||b - A x||_2 <= p_tol ||b||_2 */
  int p_maxit;          /* PCG iteration limit */
  int precision;        /* DBS_FP64, or DBS_MIXED: FP32 multigrid inside FP64 PCG */
  int mg_pre, mg_post;  /* red-black Gauss-Seidel sweeps per level (0: default 2) */
  double max_courant;   /* > 0: refuse a step whose Courant number exceeds it */
  double bounds_tol;    /* > 0: report DBS_EBOUNDS when alpha leaves the band */
  double target_courant;/* > 0: CFL-adaptive time step (Sec. 3.2): before every step
                           dt <- min(dt_max, 1.2 dt, target_courant dt / Co), Co = dt
                           max over cells of sum_out max(F_f, 0) / (phi V) of the
                           current fluxes; dt above is the first step.  A batch
                           steps in lockstep with the smallest dt of its samples.
                           Not available in graph mode (DBS_EINVAL). */
  double dt_max;        /* cap of the adaptive time step (> 0 when adaptive) */
  double mom_tol;       /* momentum predictor (Sec. 3.2, Eq. (semi_discretised_bis), solved
                           implicitly): Jacobi sweeps from U^n, each forming the residual
                           B + sum a_N U_N - a_P U of the iterate it starts from; the solve
                           ends after the first sweep whose starting residual is at most
                           mom_tol ||B||_2 (three components), or after mom_maxit sweeps.
                           0: always mom_maxit sweeps. */
  int n_alpha_sub;      /* saturation sub-cycles per step (>= 1): the transport stage runs
                           n times with dt/n, F and p_rgh of the step start held fixed and
                           the closures following the current saturation; the momentum
                           equation takes the mean of the n limited fluxes. */
} dbs_controls;

typedef struct {
  long long steps;      /* steps taken since creation */
  int p_iters[16];      /* PCG iterations per corrector of the last step */
  double p_relres[16];  /* final relative residual per corrector */
  int mg_levels;        /* multigrid levels */
  double alpha_min, alpha_max;
  double phase_volume;  /* sum phi alpha V */
  double max_courant;   /* at the start of the last step */
  double time;          /* time reached (the sum of the steps from dbs_set_time's value) */
  double dt;            /* time step of the last step */
  int mom_sweeps;       /* momentum predictor sweeps of the last step */
  double mom_relres;    /* ||r|| / ||B|| of the iterate the last predictor sweep started from */
  double p_bnorm[16];   /* ||b||_2 of each corrector's pressure system (closed domains:
                           of the mean-free b) */
  double p_res0[16];    /* relative residual of each corrector's initial guess */
  double max_div;       /* max over cells of |sum_out F_f| after the last step (the
                           discrete divergence; at most p_tol p_bnorm[n_corr - 1] when the
                           last solve converged) */
  int p_guess_order;    /* time-extrapolation order of the next step's first pressure
                           guess (0: p_rgh itself, 1: linear, 2: quadratic, 3: cubic) */
  int p_guess_change[16]; /* per corrector c >= 1: the change its next guess adds to the
                           previous corrector's solution (0: none, 1: the change its solve
                           made in the last step, 2 and 3: the last two or three changes
                           extrapolated linearly or quadratically in time); [0] is 0 */
} dbs_stats;

typedef struct dbs_handle dbs_handle;

/* Validate the problem and allocate device state on the current HIP device.
   All inputs are copied.  Fails with DBS_EINVAL for non-positive sizes, an
   unpaired or misplaced EMPTY face, unknown models or non-positive dt. */
int dbs_create(const dbs_grid *grid, const dbs_physics *phys, const dbs_bc bc[6],
               const dbs_controls *ctl, dbs_handle **out);

/* Porosity phi in (0, 1] and inverse permeability k0^-1 >= 0 [m^-2]
   (0 marks a solid-free cell), host cell arrays (Sec. 2.2 porosity field).
   DBS_EINVAL if a value is out of range or not finite. */
int dbs_set_static(dbs_handle *h, const double *phi, const double *kinv);

/* Host cell arrays alpha, U (3 x cells), p_rgh and the face flux F (or NULL:
   F = linearly interpolated U . S with boundary values).  Resets the
   derived fields (closures) from alpha. */
int dbs_set_state(dbs_handle *h, const double *alpha, const double *U,
                  const double *p_rgh, const double *F);

/* Advance nsteps time steps (Sec. 3.2 sequence).  The first corrector's
   pressure solve starts from p_rgh extrapolated in time from the ends of
   the previous steps (per sample, the order from 0 to 3 that best
   predicted the last step) less the later correctors' predicted changes;
   each later corrector's starts from the previous corrector's solution plus
   its predicted change (none, the change its solve made in the previous
   step, or the last two or three changes extrapolated, whichever predicted
   the last change best).  The guesses
   change only the iteration counts; the first step after creation or a
   state reset starts from p_rgh itself.  Synchronises the library stream
   before returning. */
int dbs_step(dbs_handle *h, int nsteps);

/* Copy the state to host arrays; any pointer may be NULL.  p = p_rgh +
   rho g.x (cell centres measured from the minimum corner). */
int dbs_get_state(dbs_handle *h, double *alpha, double *U, double *p_rgh, double *p,
                  double *F);

/* Device-pointer forms: the same layouts in device memory, copied on
   `stream` (a hipStream_t, NULL = the library stream) and synchronised. */
int dbs_set_state_dev(dbs_handle *h, const double *alpha, const double *U,
                      const double *p_rgh, const double *F, void *stream);
int dbs_get_state_dev(dbs_handle *h, double *alpha, double *U, double *p_rgh, double *p,
                      double *F, void *stream);

/* Run subsequent work on a caller stream (hipStream_t; NULL restores the
   library's own stream, created with default priority). */
int dbs_set_stream(dbs_handle *h, void *stream);

int dbs_get_stats(dbs_handle *h, dbs_stats *out);
/* Time of the state of every sample (default 0); time-dependent boundary
   values (DBS_BC_WAVE) of the next step are taken at t + dt. */
int dbs_set_time(dbs_handle *h, double t);
/* Message of the last failed call on h; with h = NULL, of this thread's last
   failed handle-free call (dbs_pressure_solve_noalloc). */
const char *dbs_last_error(const dbs_handle *h);
void dbs_destroy(dbs_handle *h);

/* Kernel timing with HIP events on the library stream.  mask selects kernel
   classes (bit i = class i, see dbs_kernel_name); 0 turns timing off.
   dbs_kernel_time returns the launches and the summed milliseconds of one
   class since the last reset. */
int dbs_set_profiling(dbs_handle *h, unsigned long long mask);
int dbs_kernel_time(dbs_handle *h, int cls, long long *launches, double *ms);
const char *dbs_kernel_name(int cls);
int dbs_kernel_classes(void);
void dbs_reset_profiling(dbs_handle *h);

/* ------------------------------------------------------------- batches
 *
 * A batch advances n independent samples (meshes of uneven sizes, each with
 * its own porosity, permeability, boundary values and state) together: each
 * stage of the step is one launch over all samples, and each sample's
 * pressure solve runs its own CG iterations (converged samples are masked
 * off), so a sample's result does not depend on the rest of the batch.  The
 * batch is not in the paper; it serves many porous samples at once.
 *
 * grids[i] and bcs[6*i .. 6*i+5] describe sample i; physics and controls are
 * shared.  A handle from dbs_create is a batch of one; the single-sample
 * calls (dbs_set_static, dbs_set_state, dbs_get_state, dbs_get_stats and
 * their _dev forms) act on sample 0.  dbs_step advances every sample;
 * DBS_ENOCONV, DBS_ENAN and DBS_EBOUNDS are reported if any sample raises
 * them, DBS_ECOURANT names the sample in dbs_last_error.  Arrays per sample
 * have the single-mesh layouts above.  Errors: DBS_EINVAL for n < 1, a bad
 * sample or an index outside [0, n). */
int dbs_batch_create(int n, const dbs_grid *grids, const dbs_physics *phys, const dbs_bc *bcs,
                     const dbs_controls *ctl, dbs_handle **out);
int dbs_batch_size(const dbs_handle *h);
int dbs_batch_set_static(dbs_handle *h, int i, const double *phi, const double *kinv);
int dbs_batch_set_state(dbs_handle *h, int i, const double *alpha, const double *U,
                        const double *p_rgh, const double *F);
int dbs_batch_get_state(dbs_handle *h, int i, double *alpha, double *U, double *p_rgh,
                        double *p, double *F);
int dbs_batch_set_state_dev(dbs_handle *h, int i, const double *alpha, const double *U,
                            const double *p_rgh, const double *F, void *stream);
int dbs_batch_get_state_dev(dbs_handle *h, int i, double *alpha, double *U, double *p_rgh,
                            double *p, double *F, void *stream);
int dbs_batch_get_stats(dbs_handle *h, int i, dbs_stats *out);
/* Advance every sample of the batch nsteps time steps: the same call as
   dbs_step, under the batch's name. */
int dbs_batch_step(dbs_handle *h, int nsteps);

/* Graph mode (on != 0): each step is replayed from a captured HIP graph.
   The first step after switching runs eagerly and sets a budget of
   momentum predictor sweeps and of PCG iterations per corrector (the
   largest counts over the samples plus a margin); the captured step runs
   exactly that many with converged samples masked and no host
   synchronisation inside.  If a sample has not converged within a budget,
   the step is redone eagerly from a saved copy of the state and the
   budgets grow, so results equal eager stepping.  A step leaves the
   buffers of alpha^n, U^n and F^n untouched (their roles move), so only
   p_rgh is saved, one cell array of device memory.  on > 1 starts from
   budgets of on - 1 instead of measuring them (this exercises the recovery
   path when a budget is too small). */
int dbs_set_graph(dbs_handle *h, int on);

/* Autotuner: times the pressure solve of the current state's first
   corrector under candidate settings and keeps the fastest that converges:
   red-black sweeps on the finest level (1..3, pre = post) with the same
   count on the coarse levels and the depth at which the single work-group
   bottom takes over (bottom_shift 0 or 1 levels coarser than the first that
   fits in LDS), then 1..4 sweeps on the coarse levels, fused full sweeps
   on the finest level or two half-sweep launches, then the planes per
   fine-level tile (kz 2..16); block-local coarse smoothing is left as set
   (*coarse_block reports it).  The state is unchanged afterwards.  Outputs
   may be NULL; *ms receives the best solve time in milliseconds. */
int dbs_autotune(dbs_handle *h, int *kz, int *sweeps, int *coarse_sweeps, int *bottom_shift,
                 int *fused, int *coarse_block, double *ms);
/* Set the same knobs by hand (kz = 0: the launch-size heuristic), and the
   planes per coarse-level tile or thread column kz_coarse (0: the launch-size
   heuristic, which keeps enough blocks to fill the chip; the autotuner leaves
   it as set).  coarse_block picks the coarse-level smoother (with fused
   sweeps; fused = 0 takes red-black half sweeps everywhere): 0 (the
   default) exact red-black sweeps, on 8 x 8 x 4 tiles (16 x 16 x 1 where
   every sample is one cell deep) in one pass on levels of at most 2^20
   cycled cells and on levels less than 8 cells deep, as half sweeps on
   the larger levels whose rows fill less than half of a 128-cell tile row,
   and on the others walking planes of 2.5-D tiles of 128 x 8 cells (FP32)
   or as half sweeps (FP64); 2 the plane walk (FP32) or half sweeps (FP64)
   on every level deep enough for the plane walk and half sweeps on the
   others; 3 the small tiles on every level; 4 half sweeps on every level;
   1 (the FP64 V-cycle takes it as 0) block-local smoothing, where the coarse_sweeps sweeps of each
   grid-cycled coarse level run in one launch, each block smoothing a 16^3
   tile in LDS with the cells around it held fixed (Jacobi between tiles,
   Gauss-Seidel within; the post-sweeps transpose the pre-sweeps, so the
   preconditioner stays symmetric).  kz and kz_coarse in [0, 64], sweeps and
   coarse_sweeps in [1, 8], bottom_shift in [0, 4], coarse_block in [0, 4];
   else DBS_EINVAL. */
int dbs_set_tuning(dbs_handle *h, int kz, int kz_coarse, int sweeps, int coarse_sweeps,
                   int bottom_shift, int fused, int coarse_block);

/* Tests only (single-sample handles).  Solve the p_rgh pressure equation of
   this handle's mesh and boundary conditions, -div(rAU_f grad x) with outlet faces as Dirichlet
   faces (the operator of Eq. (pressure_predictor)), for host arrays rAU and
   b; x holds the initial guess and receives the solution. */
int dbs_debug_pressure_solve(dbs_handle *h, const double *rAU, const double *b, double *x,
                             int *iters, double *relres);

/* For callers that cannot allocate device memory (code under HIP graph
   capture, tight serving loops, harnesses that forbid hipMalloc): the solve
   of dbs_debug_pressure_solve without a handle and without any allocation.
   The mesh `grid` and the kinds of its six domain faces (DBS_BC_*; outlet
   faces are the Dirichlet faces of the operator, EMPTY faces pair on an
   axis of one cell, the other kinds are fixed-flux faces) define
   -div(rAU_f grad x); rAU, b and x are caller DEVICE arrays of nx*ny*nz
   doubles (x: initial guess in, solution out), solved on `stream`
   (hipStream_t, NULL: the default stream) to ||b - A x||_2 <= tol ||b||_2
   with at most maxit iterations, FP64 or DBS_MIXED (FP32 V-cycle);
   iters and relres may be NULL.  Every work array (CG vectors, multigrid
   levels, launch tables, partial sums) lives in one static device array of
   DBS_NOALLOC_BYTES per GPU, held from module load to process end and
   cleared at the start of each call; meshes above DBS_NOALLOC_MAX_CELLS
   cells, or whose hierarchy does not fit, return DBS_EINVAL.  Calls that
   overlap on one GPU race for that array.  The call synchronises `stream`
   before returning.  Errors: DBS_EINVAL (arguments, size), DBS_ENOCONV,
   DBS_EHIP; dbs_last_error(NULL) gives the message of this thread's last
   failed call. */
#define DBS_NOALLOC_BYTES (64u << 20)
#define DBS_NOALLOC_MAX_CELLS (1 << 19)
int dbs_pressure_solve_noalloc(const dbs_grid *grid, const int bc_kind[6], int precision,
                               const double *rAU, const double *b, double *x, double tol,
                               int maxit, int *iters, double *relres, void *stream);

/* Tests only (single-sample handles).  Run one step and copy intermediate fields to host arrays
   (any pointer may be NULL): the MULES antidiffusive flux A (faces), 1/a_P
   (cells), momentum source Shat and predicted U (3 x cells), and from the
   first corrector HbyA (3 x cells), phiHbyA (faces) and the pressure
   right-hand side b (cells); from the saturation stage (its last sub-cycle)
   the Zalesak cell factors R+ and R- of the last limiter iteration (cells)
   and the limited flux alpha_f F_f (faces; with sub-cycles the mean the
   momentum equation receives). */
int dbs_debug_step_trace(dbs_handle *h, double *A, double *rAU, double *Shat, double *Ustar,
                         double *HbyA, double *phiHbyA, double *b, double *Rp, double *Rm,
                         double *alphaPhi);

#ifdef __cplusplus
}
#endif
#endif /* DBS_H */
