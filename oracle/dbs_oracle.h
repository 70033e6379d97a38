/*
 * Plain FP64 CPU oracle for one PISO time step of the two-phase
 * micro-continuum Darcy-Brinkman-Stokes method (Carrillo, Bourg & Soulaine,
 * "A micro-continuum framework for multiphase flow in porous media",
 * arXiv:2003.08374) on a uniform Cartesian mesh.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path may include, link,
 * load or call this code: only the tests, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no source with the HIP library.
 *
 * Conventions (all readings are listed in the oracle source header):
 *   - cells (i,j,k), linear index c = i + nx*(j + ny*k), x fastest;
 *   - face arrays: Fx has (nx+1)*ny*nz entries, index i + (nx+1)*(j + ny*k);
 *     Fy nx*(ny+1)*nz, index i + nx*(j + (ny+1)*k); Fz nx*ny*(nz+1),
 *     index i + nx*(j + ny*k); face values are oriented along +axis;
 *   - domain faces are numbered 0:x-, 1:x+, 2:y-, 3:y+, 4:z-, 5:z+.
 */
#ifndef DBS_ORACLE_H
#define DBS_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

enum { DBSO_WALL = 0, DBSO_INLET = 1, DBSO_OUTLET = 2, DBSO_EMPTY = 3, DBSO_WAVE = 4 };
enum { DBSO_BROOKS_COREY = 0, DBSO_VAN_GENUCHTEN = 1 };

typedef struct {
  int nx, ny, nz;
  double hx, hy, hz;
  /* fluids: l = wetting (alpha), g = non-wetting */
  double rho_l, rho_g, mu_l, mu_g;
  double g[3];
  double c_alpha;           /* interface compression coefficient */
  int kr_model;             /* DBSO_BROOKS_COREY or DBSO_VAN_GENUCHTEN */
  double kr_m;              /* exponent m of the relative permeability model */
  int pc_model;             /* DBSO_BROOKS_COREY or DBSO_VAN_GENUCHTEN */
  double pc0;               /* entry capillary pressure p_c0 [Pa] */
  double pc_exp;            /* beta (Brooks-Corey) or m (Van Genuchten) */
  double s_lirr, s_girr;    /* irreducible saturations of the k_r model */
  double a_pcirr, a_pcmax;  /* saturation range of the p_c model */
  double eps_pc;            /* clamp of the normalised p_c saturation */
  int bc_kind[6];
  double bc_U[6][3];        /* inlet velocity */
  double bc_alpha[6];       /* inlet alpha; outlet backflow alpha */
  double bc_p[6];           /* outlet static pressure p */
  double dt;
  int n_corr;               /* PISO correctors */
  int mom_maxit;            /* sweep cap of the momentum predictor solve */
  int transpose_visc;       /* include div(mu grad(U)^T) */
  int mules_iter;           /* MULES limiter iterations */
  double p_tol;             /* relative residual of the pressure solve */
  int p_maxit;
  /* wave inlet (x faces only): amplitude A [m], period T [s], still-water
     depth d [m] measured from y = 0 */
  double bc_wave[6][3];
  double t0;                /* time at the start of the first step [s] */
  double sigma;             /* interfacial tension [N/m] (clear-fluid CSF) */
  double contact_angle;     /* at clear/porous faces [rad], 0 = not imposed */
  double target_courant;    /* > 0: CFL-adaptive time step (R19), dt is the first */
  double dt_max;            /* cap of the adaptive time step (> 0) */
  double mom_tol;           /* momentum predictor: Jacobi sweeps until the residual
                               of the iterate a sweep starts from is at most
                               mom_tol ||B||_2 (0: always mom_maxit sweeps) */
  int n_alpha_sub;          /* saturation sub-cycles per step (>= 1): the
                               transport runs n times with dt/n, F and p_rgh
                               frozen, and the momentum equation sees the mean
                               limited flux */
} dbso_case;

typedef struct {
  int p_iters[16];          /* pressure iterations per corrector (last step) */
  double p_relres[16];
  double alpha_min, alpha_max;
  double phase_volume;      /* sum phi*alpha*V after the last step */
  double max_div;           /* max |sum_out F| over cells after the last step */
  double dt_last;           /* time step of the last step */
  double t_end;             /* time reached */
  int mom_sweeps;           /* predictor sweeps of the last step */
  double mom_relres;        /* ||r|| / ||B|| of the iterate the last sweep started from */
  double p_bnorm[16];       /* ||b||_2 of each corrector's pressure system (last step) */
} dbso_info;

/* Optional intermediate arrays of the first step (any pointer may be NULL).
   Face arrays use the concatenated x|y|z face order. */
typedef struct {
  double *A;                /* MULES antidiffusive flux, faces */
  double *Rp, *Rm;          /* Zalesak limiter R+ / R-, cells */
  double *alphaPhi;         /* limited alpha flux, faces */
  double *alpha_new;        /* cells */
  double *rAU;              /* 1/a_P of the momentum equation, cells */
  double *Shat;             /* explicit momentum source, 3 x cells */
  double *Ustar;            /* predicted velocity, 3 x cells */
  double *HbyA;             /* first corrector, 3 x cells */
  double *phiHbyA;          /* first corrector, faces */
  double *b;                /* first corrector pressure right-hand side */
  double *aP;               /* momentum diagonal per unit volume, cells */
  double *aON, *aNO;        /* per face: coefficient of U_nbr in the owner's row and
                               of U_own in the neighbour's row (0 on domain faces) */
  double *B;                /* predictor right-hand side Shat + R(q), 3 x cells */
} dbso_trace;

/* Relative permeabilities, capillary pressure and dp_c/dalpha at one
   saturation (paper App. A). */
void dbso_closures(const dbso_case *cs, double alpha, double *krl, double *krg,
                   double *pc, double *dpc);

/* Interface curvature kappa = -div(grad(alpha)/|grad(alpha)|) of every cell
   (Brackbill's CSF, Sec. 2.2) for the given alpha and face fluxes (the
   fluxes pick the outlet backflow value of alpha); with a contact angle,
   faces between clear and porous cells (kinv > 0; kinv may be NULL: all
   clear) carry the penalized normal of Sec. 2.3.  Returns 0 or -1. */
int dbso_curvature(const dbso_case *cs, const double *alpha, const double *kinv,
                   const double *Fx, const double *Fy, const double *Fz, double *kappa);

/* Face fluxes F = (linear interpolate U) . S; boundary faces take the
   inlet velocity, zero at walls, the cell velocity at outlets. */
int dbso_init_flux(const dbso_case *cs, const double *Ux, const double *Uy,
                   const double *Uz, double *Fx, double *Fy, double *Fz);

/* Values an inlet boundary b (x-, x+, y-, ... = 0..5) prescribes at time t:
   out[4*l + 0..2] = U, out[4*l + 3] = alpha for the l-th face of that side
   (faces in the order of the side's face array).  Returns the face count, or
   -1 when b is not an inlet. */
int dbso_inlet_values(const dbso_case *cs, int b, double t, double *out);

/* Saturation transport alone (Eq. (phaseEq), the first stage of a step):
   nsteps transport stages of cs->dt, each of cs->n_alpha_sub sub-cycles,
   with the face fluxes F and p_rgh held fixed; alpha is advanced in place.
   alphaPhi (faces, may be NULL) receives the last stage's mean limited flux
   alpha_f F_f.  Boundary values are taken at t0 + (stage + 1) dt.  Returns 0
   or -1 (bad input). */
int dbso_alpha_advance(const dbso_case *cs, const double *phi, const double *kinv,
                       double *alpha, const double *Fx, const double *Fy, const double *Fz,
                       const double *p_rgh, int nsteps, double *alphaPhi);

/* Advance nsteps PISO steps in place.  p (out) may be NULL.  Returns 0, or a
   negative code: -1 bad input, -4 pressure solve did not converge. */
int dbso_step(const dbso_case *cs, const double *phi, const double *kinv,
              double *alpha, double *Ux, double *Uy, double *Uz, double *p_rgh,
              double *p, double *Fx, double *Fy, double *Fz, int nsteps,
              dbso_info *info, dbso_trace *trace);

/* y = A x for the pressure operator built from rAU and the case's boundary
   conditions (SPD form: -laplacian(rAU_f) with Dirichlet outlet faces). */
int dbso_pressure_apply(const dbso_case *cs, const double *rAU, const double *x,
                        double *y);

/* Solve A x = b (x holds the initial guess on entry).  Jacobi-preconditioned
   conjugate gradients to ||b - A x|| <= tol ||b||. */
int dbso_pressure_solve(const dbso_case *cs, const double *rAU, const double *b,
                        double *x, double tol, int maxit, int *iters,
                        double *relres);

#ifdef __cplusplus
}
#endif
#endif
