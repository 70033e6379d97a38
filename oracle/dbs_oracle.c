/*
 * dbs_oracle.c -- plain FP64 CPU oracle of one PISO step of the two-phase
 * micro-continuum Darcy-Brinkman-Stokes (DBS) method of Carrillo, Bourg and
 * Soulaine (arXiv:2003.08374).
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the HIP
 * product library and is written as a face-list finite-volume code: every
 * face is visited once, its flux is added to the owner and subtracted from
 * the neighbour.  Single thread, scalar loops, built with -O2
 * -ffp-contract=off.
 *
 * What it computes, in the order of the paper's solution algorithm (Sec. 3.2):
 *   1. explicit saturation transport, Eq. (phaseEq) as restated in
 *      Eq. (two-phase-microcontinuum): Van Leer high-order convection and a
 *      flux-corrected-transport (Zalesak) limiter (Sec. 3.1, 3.2).  The
 *      relative flux phi*alpha_l*alpha_g*v_r uses the closures summarised in
 *      Sec. 2.3: interface compression in clear regions and Eq. (vr_porous)
 *      in porous regions;
 *   2. property update from the new saturation: App. A relative permeability
 *      and capillary pressure, mu = alpha mu_l + (1-alpha) mu_g (Eq. Fc context),
 *      rho = alpha rho_l + (1-alpha) rho_g and the porous capillary force of
 *      App. B;
 *   3. momentum predictor, Eq. (semi_discretised_bis), with the Darcy drag
 *      coefficient mu k^-1 = k0^-1 (k_rl/mu_l + k_rg/mu_g)^-1 (Sec. 2.3 summary);
 *   4. n_corr pressure correctors, Eqs. (corrected_velocity) and
 *      (pressure_predictor), solved in the p_rgh = p - rho g.x form.
 *
 * Readings taken where the paper is silent, garbled or inconsistent:
 *   R1  compression velocity sign: +grad(alpha)/|grad(alpha)| (Sec. 2.3 summary),
 *       face-local |v| = |F_f|/A_f, upwinded alpha*(1-alpha) product;
 *   R2  drag coefficient in the k_rl/mu_l + k_rg/mu_g form (Sec. 2.3 summary);
 *       the form printed beside Eq. (single-field-kr) is read as a typo;
 *   R3  one density rho = alpha rho_l + (1-alpha) rho_g everywhere and the
 *       porous capillary force of App. B:
 *       F_c = (f_l - alpha)[(rho_l - rho_g) g + grad p_c] - p_c grad alpha,
 *       f_l = M_l/(M_l + M_g); F_c = 0 in clear cells (sigma = 0);
 *   R4  the 1/phi factors of the momentum PDE are kept on the time and
 *       convection terms (convective flux divided by the face porosity);
 *   R5  irreducible saturations 0, alpha_pc,max = 1 unless given; the
 *       normalised p_c saturation is clamped to [eps_pc, 1] (Brooks-Corey) or
 *       [eps_pc, 1 - eps_pc] (Van Genuchten) and dp_c/dalpha = 0 where clamped;
 *   R6  a cell is porous iff k0^-1 > 0; a face is porous iff either side is;
 *       face permeability is the harmonic mean 2/(k^-1_P + k^-1_N);
 *       p_c = 0 and f_l - alpha = 0 in clear cells;
 *   R7  porous relative flux phi a a_g v_r with the 1/alpha factors multiplied
 *       out: G_f = a_g,f u_l - a_f u_g, u_l = -M_l,f (dn p_l - rho_l g_n) A_f,
 *       u_g = -M_g,f (dn p_g - rho_g g_n) A_f, p_l = p - a_g p_c, p_g = p + a p_c,
 *       which expands to the bracket of Eq. (vr_porous); a_f arithmetic face
 *       mean; M_i,f = k0_f k_ri/mu_i of the cell upstream of phase i's
 *       potential (phase-potential upwinding); p = p_rgh + rho g.x of the
 *       previous step;
 *   R8  MULES limiter: Zalesak bounds from the face neighbours and inflow
 *       boundary values clipped to [0, 1], then mules_iter limiter iterations
 *       in which a cell's room to rise (fall) is its bound margin plus the
 *       limited antidiffusive flux leaving (entering) it; face factors never
 *       grow between iterations;
 *   R9  Van Leer ratio r = (a_U - a_UU)/(a_D - a_U); beyond a boundary a_UU = a_U;
 *   R10 momentum convection upwind; viscous term implicit mu_f grad(U) plus an
 *       explicit div(mu grad(U)^T) from U^n (switchable);
 *   R11 momentum predictor: Sec. 3.2 obtains v* by solving the momentum
 *       equation implicitly, Eq. (semi_discretised_bis), which leaves the
 *       linear solver open; Jacobi sweeps from U^n until the residual
 *       B + sum a_N U_N - a_P U of the iterate a sweep starts from is at
 *       most mom_tol ||B||_2 over the three components (the sweep is still
 *       applied), at most mom_maxit sweeps;
 *   R12 no Rhie-Chow / ddt flux correction; Cartesian reconstruct
 *       R(q)_x = (q_west + q_east)/(2 A_x); no body force on boundary faces;
 *       fixed-flux faces carry the p_rgh gradient that reproduces their
 *       prescribed flux in the correctors, and the opposite face's force
 *       density in the predictor;
 *   R13 boundary conditions: inlet = fixed U, alpha and flux (zero normal
 *       gradient of p_rgh); outlet = fixed static p (p_rgh_b = p_b - rho_P g.x_b),
 *       zero-gradient U, alpha zero-gradient on outflow and the given value on
 *       backflow; wall = no-slip, zero flux, zero-gradient alpha; empty = 2D;
 *   R14 closed domains: zero-mean p_rgh;
 *   R15 the pressure solve ends at ||b - A x||_2 <= tol ||b||_2;
 *   R16 wave inlet (the coastal-barrier configuration of Sec. 4; the paper
 *       gives no boundary formula): linear (Airy) wave theory on still water
 *       of depth d, surface elevation A sin(w t) at the inlet, w = 2 pi / T,
 *       wavenumber from w^2 = |g| k tanh(k d); below the surface the face
 *       carries alpha = 1 and the orbital velocity
 *       u = A w cosh(k y)/sinh(k d) sin(w t) (into the domain),
 *       v = A w sinh(k y)/sinh(k d) cos(w t) (so v = d eta/dt at y = d),
 *       above it alpha = 0 and U = 0; y is the face-centre height; all
 *       boundary values of a step are taken at its end time t^{n+1};
 *       outflowing wave faces carry the cell alpha;
 *   R17 clear-fluid surface tension (CSF, Brackbill et al. 1992), taken with
 *       the physical sign: F_c = phi^-1 sigma kappa grad(alpha), kappa =
 *       div(n_lg) = -div(grad(alpha)/|grad(alpha)|) (curvature as defined
 *       in Sec. 2.1, positive for a liquid drop).  The two printed forms
 *       (Sec. 2.2 and the Sec. 2.3 summary) carry the opposite overall sign,
 *       which would lower the pressure inside a drop; the Laplace jump pins
 *       the sign taken.  Discretely: Gauss cell gradients (face values as in
 *       the compression term), face gradient = mean of the two cells (the
 *       cell's own on a domain face), n_f = grad_f/(|grad_f| + dN), kappa_P
 *       = -(1/V) sum_f n_f.S_f; per cell s_P = sigma kappa_P / phi_P in clear
 *       cells and 0 in porous ones (where F_c is the App. B form), and the
 *       face force gains (s_P + s_N)/2 dn(alpha), alpha^{n+1} throughout.
 *   R18 penalized contact angle (Sec. 2.3, locally modified normal): on a
 *       face between a clear and a porous cell the wall normal n_w is the
 *       face axis pointing from the porous into the clear cell, and the
 *       interface normal n_lg = -grad(alpha)/|grad(alpha)| is replaced by
 *       cos(theta) n_w + sin(theta) t_w, t_w the unit wall tangent in the
 *       plane of n_w and the current normal.  On a Cartesian face only the
 *       normal component enters the divergence, so that face contributes
 *       n.S = -cos(theta) (n_w . e_axis) |n_f| A to the curvature of grad(alpha)
 *       normals, |n_f| = |grad_f|/(|grad_f| + dN) (no interface, no term).
 *       theta is measured through the liquid (alpha = 1) phase; the wall
 *       being the face between the two cells, the same angle holds at every
 *       clear/porous face; 0 means not imposed.  The same angle fixes
 *       the wall-normal derivative of alpha in the clear cell, as a wall
 *       contact-angle condition does: the curvature's Gauss gradient of a
 *       clear cell next to a porous cell along an axis takes, on that axis,
 *       the component that makes its normal meet the wall at theta given
 *       its other components (the solid's own saturation, frozen, would
 *       otherwise pin the contact line);
 *   R19 CFL-adaptive time step (Sec. 3.2: the march follows an imposed
 *       Courant number; no rule is printed): before every step
 *       dt <- min(dt_max, 1.2 dt, Co_target dt / Co), Co = dt max over cells
 *       of the outflow sum_f max(F_f, 0) / (phi V) of the current fluxes
 *       (the growth factor 1.2 is a choice); the first step starts from the
 *       given dt;
 *   R20 saturation sub-cycling (robustness for long runs; the paper marches
 *       the explicit saturation equation at the imposed Courant number): a
 *       step's transport may run in n sub-cycles of dt/n, each the whole
 *       transport stage above applied to the current saturation with F and
 *       p_rgh of the step start held fixed (closures follow the current
 *       saturation); the momentum equation takes the mean of the n limited
 *       fluxes, so that alpha^{n+1} - alpha^n = -dt/(phi V) sum_out of that
 *       mean exactly as for one stage, and rho^n from the step start.
 *
 * Pins (tests/test_oracle_pins.py) tie each function to what the paper and
 * the mathematics fix.  Parity unpinned: the values the eps_pc clamp of R5
 * gives in dry porous cells, which only the GPU path checks; pinned are the
 * clamp at the closure level, that it changes nothing while every porous
 * cell is inside the range, and that dry cells keep a step finite and
 * bounded.  Parity unpinned as well: the 1/phi factor of R17 (it acts only
 * in clear cells with phi < 1, which no workload has) and the equilibrium
 * angle a drop reaches under R18 (pinned: the imposed normal against a
 * static cap's geometry).
 */
#include "dbs_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ mesh */

typedef struct {
  int axis;
  int own, nbr;      /* cell on the minus / plus side, -1 outside the domain */
  int own2, nbr2;    /* cell beyond own (minus side) / beyond nbr (plus side) */
  int bnd;           /* domain face 0..5, -1 for interior faces */
  int kind;          /* boundary kind, -1 for interior faces */
  double area, dist; /* area; centre-to-centre or centre-to-face distance */
  double xf[3];      /* face centre */
} face_t;

typedef struct {
  const dbso_case *cs;
  int n[3], nc, nf, nfa[3];
  double h[3], V;
  face_t *f;
  int *cf; /* six face ids per cell: x-, x+, y-, y+, z-, z+ */
  double t; /* time at which boundary values are taken */
} mesh_t;

static double clampd(double x, double lo, double hi) {
  return x < lo ? lo : (x > hi ? hi : x);
}
static double maxd(double a, double b) { return a > b ? a : b; }
static double mind(double a, double b) { return a < b ? a : b; }

static int cell_id(const mesh_t *m, int i, int j, int k) {
  return i + m->n[0] * (j + m->n[1] * k);
}

static void cell_centre(const mesh_t *m, int c, double x[3]) {
  int i = c % m->n[0];
  int j = (c / m->n[0]) % m->n[1];
  int k = c / (m->n[0] * m->n[1]);
  x[0] = (i + 0.5) * m->h[0];
  x[1] = (j + 0.5) * m->h[1];
  x[2] = (k + 0.5) * m->h[2];
}

static int validate_case(const dbso_case *cs) {
  int n[3] = {cs->nx, cs->ny, cs->nz};
  double h[3] = {cs->hx, cs->hy, cs->hz};
  for (int a = 0; a < 3; a++) {
    if (n[a] < 1 || !(h[a] > 0.0)) return -1;
    int e0 = cs->bc_kind[2 * a] == DBSO_EMPTY, e1 = cs->bc_kind[2 * a + 1] == DBSO_EMPTY;
    if (e0 != e1) return -1;
    if (e0 && n[a] != 1) return -1;
  }
  for (int b = 0; b < 6; b++)
    if (cs->bc_kind[b] < DBSO_WALL || cs->bc_kind[b] > DBSO_WAVE) return -1;
  if (!(cs->sigma >= 0.0) || isinf(cs->sigma)) return -1;
  if (!(cs->contact_angle >= 0.0 && cs->contact_angle < 3.14159265358979323846)) return -1;
  for (int b = 2; b < 6; b++)
    if (cs->bc_kind[b] == DBSO_WAVE) return -1; /* wave inlets sit on x faces */
  for (int b = 0; b < 2; b++)
    if (cs->bc_kind[b] == DBSO_WAVE &&
        !(cs->bc_wave[b][1] > 0.0 && cs->bc_wave[b][2] > 0.0)) return -1;
  if (!(cs->dt > 0.0) || cs->n_corr < 1 || cs->n_corr > 16 || cs->mom_maxit < 0 ||
      !(cs->mom_tol >= 0.0) || cs->n_alpha_sub < 1)
    return -1;
  return 0;
}

static int build_mesh(const dbso_case *cs, mesh_t *m) {
  memset(m, 0, sizeof(*m));
  if (validate_case(cs)) return -1;
  m->cs = cs;
  m->n[0] = cs->nx; m->n[1] = cs->ny; m->n[2] = cs->nz;
  m->h[0] = cs->hx; m->h[1] = cs->hy; m->h[2] = cs->hz;
  m->V = cs->hx * cs->hy * cs->hz;
  m->nc = cs->nx * cs->ny * cs->nz;
  m->nfa[0] = (cs->nx + 1) * cs->ny * cs->nz;
  m->nfa[1] = cs->nx * (cs->ny + 1) * cs->nz;
  m->nfa[2] = cs->nx * cs->ny * (cs->nz + 1);
  m->nf = m->nfa[0] + m->nfa[1] + m->nfa[2];
  m->f = (face_t *)calloc((size_t)m->nf, sizeof(face_t));
  m->cf = (int *)calloc((size_t)m->nc * 6, sizeof(int));
  if (!m->f || !m->cf) return -2;
  int stride[3] = {1, m->n[0], m->n[0] * m->n[1]};
  int id = 0;
  for (int a = 0; a < 3; a++) {
    int fn[3] = {m->n[0], m->n[1], m->n[2]};
    fn[a] += 1;
    for (int k = 0; k < fn[2]; k++)
      for (int j = 0; j < fn[1]; j++)
        for (int i = 0; i < fn[0]; i++) {
          int idx[3] = {i, j, k};
          int s = idx[a];
          face_t *F = &m->f[id];
          F->axis = a;
          int lo[3] = {i, j, k};
          lo[a] = s - 1;
          F->own = s - 1 >= 0 ? cell_id(m, lo[0], lo[1], lo[2]) : -1;
          F->nbr = s < m->n[a] ? cell_id(m, i, j, k) : -1;
          F->own2 = s - 2 >= 0 ? F->own - stride[a] : -1;
          F->nbr2 = s + 1 < m->n[a] ? F->nbr + stride[a] : -1;
          F->bnd = s == 0 ? 2 * a : (s == m->n[a] ? 2 * a + 1 : -1);
          F->kind = F->bnd >= 0 ? cs->bc_kind[F->bnd] : -1;
          F->area = m->V / m->h[a];
          F->dist = F->bnd >= 0 ? 0.5 * m->h[a] : m->h[a];
          for (int b = 0; b < 3; b++)
            F->xf[b] = b == a ? s * m->h[a] : (idx[b] + 0.5) * m->h[b];
          if (F->own >= 0) m->cf[F->own * 6 + 2 * a + 1] = id;
          if (F->nbr >= 0) m->cf[F->nbr * 6 + 2 * a] = id;
          id++;
        }
  }
  return 0;
}

static void free_mesh(mesh_t *m) {
  free(m->f);
  free(m->cf);
}

/* inside cell and outward sign of a boundary face */
static int bnd_cell(const face_t *F, double *so) {
  if (F->bnd & 1) { *so = 1.0; return F->own; }
  *so = -1.0;
  return F->nbr;
}

/* ------------------------------------------------------------- closures */

/* App. A: relative permeability (A.1) and capillary pressure (A.2). */
void dbso_closures(const dbso_case *cs, double alpha, double *krl, double *krg,
                   double *pc, double *dpc) {
  double ae = clampd((alpha - cs->s_lirr) / (1.0 - cs->s_girr - cs->s_lirr), 0.0, 1.0);
  double m = cs->kr_m;
  if (cs->kr_model == DBSO_BROOKS_COREY) {
    *krl = pow(ae, m);
    *krg = pow(1.0 - ae, m);
  } else {
    double t = pow(ae, 1.0 / m);
    double u = 1.0 - pow(1.0 - t, m);
    *krl = sqrt(ae) * u * u;
    *krg = sqrt(1.0 - ae) * pow(1.0 - t, 2.0 * m);
  }
  double span = cs->a_pcmax - cs->a_pcirr;
  double s = (alpha - cs->a_pcirr) / span;
  double eps = cs->eps_pc;
  double top = cs->pc_model == DBSO_BROOKS_COREY ? 1.0 : 1.0 - eps;
  int clamped = s < eps || s > top;
  s = clampd(s, eps, top);
  if (cs->pc_model == DBSO_BROOKS_COREY) {
    double beta = cs->pc_exp;
    *pc = cs->pc0 * pow(s, -beta);
    *dpc = clamped ? 0.0 : -beta * cs->pc0 * pow(s, -beta - 1.0) / span;
  } else {
    double mv = cs->pc_exp;
    double t = pow(s, -1.0 / mv) - 1.0;
    *pc = cs->pc0 * pow(t, 1.0 - mv);
    *dpc = clamped ? 0.0
                   : cs->pc0 * (1.0 - mv) * pow(t, -mv) * (-1.0 / mv) *
                         pow(s, -1.0 / mv - 1.0) / span;
  }
}

typedef struct {
  double ml, mg; /* k_ri / mu_i */
  double pc;     /* capillary pressure, 0 in clear cells (R6) */
  double cf;     /* f_l - alpha in porous cells, 0 in clear cells (R3) */
  double K;      /* Darcy drag coefficient mu k^-1 (R2) */
  double rho, mu;
  double sk;     /* sigma kappa / phi in clear cells, 0 in porous cells (R17) */
} props_t;

static void cell_props(const dbso_case *cs, double a, double kinv, props_t *p) {
  double krl, krg, pc, dpc;
  dbso_closures(cs, a, &krl, &krg, &pc, &dpc);
  p->ml = krl / cs->mu_l;
  p->mg = krg / cs->mu_g;
  double mt = p->ml + p->mg;
  int porous = kinv > 0.0;
  p->pc = porous ? pc : 0.0;
  p->cf = porous ? p->ml / mt - a : 0.0;
  p->K = porous ? kinv / mt : 0.0;
  p->rho = a * cs->rho_l + (1.0 - a) * cs->rho_g;
  p->mu = a * cs->mu_l + (1.0 - a) * cs->mu_g;
  p->sk = 0.0;
}

static const double PI = 3.14159265358979323846;

static int is_inlet(int kind) { return kind == DBSO_INLET || kind == DBSO_WAVE; }

/* wavenumber of linear waves: the root of w^2 = gm k tanh(k d), by bisection */
static double wave_number(double w, double gm, double d) {
  double lo = 0.0, hi = 1.0;
  while (gm * hi * tanh(hi * d) < w * w) hi *= 2.0;
  for (int it = 0; it < 200; it++) {
    double mid = 0.5 * (lo + hi);
    if (gm * mid * tanh(mid * d) < w * w) lo = mid; else hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* velocity and alpha prescribed on an inlet face at time m->t (R13, R16) */
static void inlet_face(const mesh_t *m, const face_t *F, double U[3], double *alpha) {
  const dbso_case *cs = m->cs;
  if (F->kind != DBSO_WAVE) {
    for (int d = 0; d < 3; d++) U[d] = cs->bc_U[F->bnd][d];
    *alpha = cs->bc_alpha[F->bnd];
    return;
  }
  const double *wv = cs->bc_wave[F->bnd];
  double A = wv[0], w = 2.0 * PI / wv[1], d = wv[2];
  double gm = sqrt(cs->g[0] * cs->g[0] + cs->g[1] * cs->g[1] + cs->g[2] * cs->g[2]);
  double k = wave_number(w, gm, d);
  double y = F->xf[1], t = m->t;
  U[0] = U[1] = U[2] = 0.0;
  *alpha = 0.0;
  if (y < d + A * sin(w * t)) {
    double into = F->bnd == 0 ? 1.0 : -1.0;
    U[0] = into * A * w * cosh(k * y) / sinh(k * d) * sin(w * t);
    U[1] = A * w * sinh(k * y) / sinh(k * d) * cos(w * t);
    *alpha = 1.0;
  }
}

/* alpha on a boundary face (R13, R16) given the face flux along +axis */
static double bnd_alpha(const mesh_t *m, const face_t *F, const double *alpha, double flux) {
  const dbso_case *cs = m->cs;
  double so;
  int c = bnd_cell(F, &so);
  if (F->kind == DBSO_INLET) return cs->bc_alpha[F->bnd];
  if (F->kind == DBSO_WAVE && so * flux < 0.0) {
    double U[3], ab;
    inlet_face(m, F, U, &ab);
    return ab;
  }
  if (F->kind == DBSO_OUTLET && so * flux < 0.0) return cs->bc_alpha[F->bnd];
  return alpha[c];
}

/* ---------------------------------------------------- 1. alpha transport */

static double dot3(const double *a, const double *b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}

/* Gauss cell gradient of alpha (face values: mean inside, boundary value);
   grad holds 3 entries per cell and is overwritten */
static void gauss_grad(const mesh_t *m, const double *alpha, const double *F, double *grad) {
  memset(grad, 0, sizeof(double) * 3 * (size_t)m->nc);
  for (int f = 0; f < m->nf; f++) {
    const face_t *Fc = &m->f[f];
    if (Fc->kind == DBSO_EMPTY) continue;
    double af = Fc->bnd < 0 ? 0.5 * (alpha[Fc->own] + alpha[Fc->nbr])
                            : bnd_alpha(m, Fc, alpha, F[f]);
    if (Fc->own >= 0) grad[Fc->own * 3 + Fc->axis] += af * Fc->area / m->V;
    if (Fc->nbr >= 0) grad[Fc->nbr * 3 + Fc->axis] -= af * Fc->area / m->V;
  }
}

/* kappa_P = -(1/V) sum over the cell's faces of n_f . S_f (outward), with
   n_f the regularised unit face gradient of alpha (R17), penalized on
   clear/porous faces when a contact angle is imposed (R18) */
static void curvature(const mesh_t *m, const double *alpha, const double *kinv,
                      const double *F, double *kappa) {
  const double th = m->cs->contact_angle;
  double *grad = (double *)malloc(sizeof(double) * 3 * (size_t)m->nc);
  gauss_grad(m, alpha, F, grad);
  if (th > 0.0 && kinv) {
    /* the wall-normal component of a clear cell's gradient next to a porous
       cell: the one that makes the cell's normal meet the wall at theta
       (n.n_w = -cos(theta) for n = grad(alpha)/|grad(alpha)|), given the
       components along the other axes; a cell with porous cells on both
       sides of an axis keeps its Gauss value there */
    int *wall = (int *)calloc((size_t)m->nc * 3, sizeof(int));
    double *g0 = (double *)malloc(sizeof(double) * 3 * (size_t)m->nc);
    memcpy(g0, grad, sizeof(double) * 3 * (size_t)m->nc);
    for (int f = 0; f < m->nf; f++) {
      const face_t *Fc = &m->f[f];
      if (Fc->kind == DBSO_EMPTY || Fc->bnd >= 0) continue;
      const int po = kinv[Fc->own] > 0.0, pn = kinv[Fc->nbr] > 0.0;
      if (po == pn) continue;
      /* n_w . e_axis: +1 with the porous cell on the minus side */
      if (!po) wall[Fc->own * 3 + Fc->axis] -= 1;
      else wall[Fc->nbr * 3 + Fc->axis] += 1;
    }
    const double cot = cos(th) / sin(th);
    for (int c = 0; c < m->nc; c++)
      for (int a = 0; a < 3; a++) {
        const int w = wall[c * 3 + a];
        if (w != 1 && w != -1) continue;
        double t2 = 0.0;
        for (int b = 0; b < 3; b++)
          if (b != a) t2 += g0[c * 3 + b] * g0[c * 3 + b];
        grad[c * 3 + a] = -cot * sqrt(t2) * (double)w;
      }
    free(g0);
    free(wall);
  }
  double dN = 1e-8 / cbrt(m->V);
  for (int c = 0; c < m->nc; c++) kappa[c] = 0.0;
  for (int f = 0; f < m->nf; f++) {
    const face_t *Fc = &m->f[f];
    if (Fc->kind == DBSO_EMPTY) continue;
    double gf[3];
    for (int d = 0; d < 3; d++) {
      if (Fc->bnd < 0) gf[d] = 0.5 * (grad[Fc->own * 3 + d] + grad[Fc->nbr * 3 + d]);
      else gf[d] = grad[(Fc->own >= 0 ? Fc->own : Fc->nbr) * 3 + d];
    }
    double mag = sqrt(dot3(gf, gf));
    double nS = gf[Fc->axis] / (mag + dN) * Fc->area;
    if (th > 0.0 && kinv && Fc->bnd < 0 && (kinv[Fc->own] > 0.0) != (kinv[Fc->nbr] > 0.0)) {
      /* n_w . e_axis = +1 when the porous cell is on the minus side */
      double nw = kinv[Fc->own] > 0.0 ? 1.0 : -1.0;
      nS = -cos(th) * nw * (mag / (mag + dN)) * Fc->area;
    }
    if (Fc->own >= 0) kappa[Fc->own] -= nS / m->V;  /* +axis is outward of own */
    if (Fc->nbr >= 0) kappa[Fc->nbr] += nS / m->V;
  }
  free(grad);
}

static void alpha_stage(const mesh_t *m, const double *phi, const double *kinv,
                        const double *alpha, const double *F, const double *prgh, double dt,
                        double *alpha_new, double *alphaPhi, dbso_trace *tr) {
  const dbso_case *cs = m->cs;
  int nc = m->nc, nf = m->nf;
  double V = m->V;
  props_t *pr = (props_t *)malloc(sizeof(props_t) * nc);
  double *p = (double *)malloc(sizeof(double) * nc);
  double *grad = (double *)calloc((size_t)nc * 3, sizeof(double));
  double *FL = (double *)calloc((size_t)nf, sizeof(double));
  double *A = (double *)calloc((size_t)nf, sizeof(double));
  double *Rp = (double *)malloc(sizeof(double) * nc);
  double *Rm = (double *)malloc(sizeof(double) * nc);

  for (int c = 0; c < nc; c++) {
    double x[3];
    cell_props(cs, alpha[c], kinv[c], &pr[c]);
    cell_centre(m, c, x);
    p[c] = prgh[c] + pr[c].rho * (cs->g[0] * x[0] + cs->g[1] * x[1] + cs->g[2] * x[2]);
  }
  gauss_grad(m, alpha, F, grad);
  double dN = 1e-8 / cbrt(V);

  /* face fluxes: low order, high order, relative flux, antidiffusive part */
  for (int f = 0; f < nf; f++) {
    const face_t *Fc = &m->f[f];
    if (Fc->kind == DBSO_EMPTY) continue;
    double Ff = F[f];
    if (Fc->bnd >= 0) {
      FL[f] = Ff * bnd_alpha(m, Fc, alpha, Ff);
      A[f] = 0.0;
      continue;
    }
    int o = Fc->own, n = Fc->nbr;
    int up = Ff >= 0.0 ? o : n, dn = Ff >= 0.0 ? n : o;
    int uu = Ff >= 0.0 ? Fc->own2 : Fc->nbr2;
    double aU = alpha[up], aD = alpha[dn], aUU = uu >= 0 ? alpha[uu] : aU;
    FL[f] = Ff * aU;
    double avl = aU;
    if (aD != aU) {
      double r = (aU - aUU) / (aD - aU);
      double psi = (r + fabs(r)) / (1.0 + fabs(r));
      avl = aU + 0.5 * psi * (aD - aU);
    }
    double G;
    if (kinv[o] == 0.0 && kinv[n] == 0.0) {
      /* clear face: interface compression (R1) */
      double gf[3], mag = 0.0;
      for (int b = 0; b < 3; b++) {
        gf[b] = 0.5 * (grad[o * 3 + b] + grad[n * 3 + b]);
        mag += gf[b] * gf[b];
      }
      mag = sqrt(mag);
      double nfa = gf[Fc->axis] / (mag + dN);
      double Fr = cs->c_alpha * fabs(Ff) * nfa;
      G = Fr >= 0.0 ? Fr * alpha[o] * (1.0 - alpha[n]) : Fr * alpha[n] * (1.0 - alpha[o]);
    } else {
      /* porous face: Eq. (vr_porous) times phi alpha_l alpha_g (R7), written
         as alpha_g u_l - alpha u_g with the two phase Darcy fluxes of the
         pressure-gradient relations of Sec. 2.3; each phase's mobility is
         taken from the upstream cell of that phase's potential */
      double k0f = 2.0 / (kinv[o] + kinv[n]);
      double af = 0.5 * (alpha[o] + alpha[n]), agf = 1.0 - af;
      double d = Fc->dist;
      double ge = cs->g[Fc->axis];
      double dp = (p[n] - p[o]) / d;
      double dpl = dp - ((1.0 - alpha[n]) * pr[n].pc - (1.0 - alpha[o]) * pr[o].pc) / d -
                   cs->rho_l * ge;
      double dpg = dp + (alpha[n] * pr[n].pc - alpha[o] * pr[o].pc) / d - cs->rho_g * ge;
      double ml = dpl < 0.0 ? pr[o].ml : pr[n].ml;
      double mg = dpg < 0.0 ? pr[o].mg : pr[n].mg;
      double ul = -k0f * ml * dpl * Fc->area;
      double ug = -k0f * mg * dpg * Fc->area;
      G = agf * ul - af * ug;
    }
    A[f] = Ff * avl + G - FL[f];
  }

  /* MULES limiter (R8): Zalesak bounds, then limiter iterations in which the
     room left in a cell counts the already-limited counter-fluxes */
  double *Qp = (double *)malloc(sizeof(double) * nc), *Qm = (double *)malloc(sizeof(double) * nc);
  double *Pin = (double *)malloc(sizeof(double) * nc), *Pout = (double *)malloc(sizeof(double) * nc);
  double *lam = (double *)malloc(sizeof(double) * nf);
  for (int c = 0; c < nc; c++) {
    double vol = phi[c] * V / dt;
    double outL = 0.0, amax = alpha[c], amin = alpha[c], pin = 0.0, pout = 0.0;
    for (int s = 0; s < 6; s++) {
      int f = m->cf[c * 6 + s];
      const face_t *Fc = &m->f[f];
      if (Fc->kind == DBSO_EMPTY) continue;
      double so = (s & 1) ? 1.0 : -1.0;
      outL += so * FL[f];
      if (Fc->bnd < 0) {
        int nb = (s & 1) ? Fc->nbr : Fc->own;
        amax = maxd(amax, alpha[nb]);
        amin = mind(amin, alpha[nb]);
      } else if (so * F[f] < 0.0) {
        double ab = bnd_alpha(m, Fc, alpha, F[f]);
        amax = maxd(amax, ab);
        amin = mind(amin, ab);
      }
      pin += maxd(0.0, -so * A[f]);
      pout += maxd(0.0, so * A[f]);
    }
    amax = mind(1.0, amax);
    amin = maxd(0.0, amin);
    double aL = alpha[c] - outL / vol;
    Qp[c] = vol * maxd(0.0, amax - aL);
    Qm[c] = vol * maxd(0.0, aL - amin);
    Pin[c] = pin;
    Pout[c] = pout;
  }
  for (int f = 0; f < nf; f++) lam[f] = m->f[f].bnd < 0 ? 1.0 : 0.0;
  for (int it = 0; it < cs->mules_iter; it++) {
    for (int c = 0; c < nc; c++) {
      double lout = 0.0, lin = 0.0;
      for (int s = 0; s < 6; s++) {
        int f = m->cf[c * 6 + s];
        if (m->f[f].kind == DBSO_EMPTY) continue;
        double so = (s & 1) ? 1.0 : -1.0;
        lout += lam[f] * maxd(0.0, so * A[f]);
        lin += lam[f] * maxd(0.0, -so * A[f]);
      }
      Rp[c] = Pin[c] > 0.0 ? clampd((Qp[c] + lout) / Pin[c], 0.0, 1.0) : 1.0;
      Rm[c] = Pout[c] > 0.0 ? clampd((Qm[c] + lin) / Pout[c], 0.0, 1.0) : 1.0;
    }
    for (int f = 0; f < nf; f++) {
      const face_t *Fc = &m->f[f];
      if (Fc->bnd >= 0) continue;
      double l = A[f] >= 0.0 ? mind(Rm[Fc->own], Rp[Fc->nbr]) : mind(Rp[Fc->own], Rm[Fc->nbr]);
      lam[f] = mind(lam[f], l);
    }
  }
  for (int f = 0; f < nf; f++) {
    const face_t *Fc = &m->f[f];
    alphaPhi[f] = Fc->kind == DBSO_EMPTY ? 0.0 : FL[f] + lam[f] * A[f];
  }
  free(Qp); free(Qm); free(Pin); free(Pout); free(lam);
  /* forward Euler on d(phi alpha)/dt with static phi */
  for (int c = 0; c < nc; c++) {
    double out = 0.0;
    for (int s = 0; s < 6; s++) {
      int f = m->cf[c * 6 + s];
      if (m->f[f].kind == DBSO_EMPTY) continue;
      out += ((s & 1) ? 1.0 : -1.0) * alphaPhi[f];
    }
    alpha_new[c] = alpha[c] - dt * out / (phi[c] * V);
  }
  if (tr) {
    if (tr->A) memcpy(tr->A, A, sizeof(double) * nf);
    if (tr->Rp) memcpy(tr->Rp, Rp, sizeof(double) * nc);
    if (tr->Rm) memcpy(tr->Rm, Rm, sizeof(double) * nc);
  }
  free(pr); free(p); free(grad); free(FL); free(A); free(Rp); free(Rm);
}

/* The saturation stage of a step (R20): n_alpha_sub sub-cycles of dt/n, each
   the transport stage applied to the current saturation with F and p_rgh
   fixed.  alphaPhi receives the mean of the sub-cycles' limited fluxes and
   rhoPhi the mass flux built from it.  The trace keeps the last sub-cycle's
   A and R+-, the mean flux and the final saturation. */
static void alpha_transport(const mesh_t *m, const double *phi, const double *kinv,
                            const double *alpha, const double *F, const double *prgh,
                            double *alpha_new, double *alphaPhi, double *rhoPhi,
                            dbso_trace *tr) {
  const dbso_case *cs = m->cs;
  int nc = m->nc, nf = m->nf, n = cs->n_alpha_sub;
  double dts = cs->dt / n;
  double *cur = (double *)malloc(sizeof(double) * nc);
  double *sub = (double *)malloc(sizeof(double) * nf);
  memcpy(cur, alpha, sizeof(double) * nc);
  for (int f = 0; f < nf; f++) alphaPhi[f] = 0.0;
  for (int k = 0; k < n; k++) {
    alpha_stage(m, phi, kinv, cur, F, prgh, dts, alpha_new, sub, k == n - 1 ? tr : NULL);
    for (int f = 0; f < nf; f++) alphaPhi[f] += sub[f];
    memcpy(cur, alpha_new, sizeof(double) * nc);
  }
  for (int f = 0; f < nf; f++) {
    alphaPhi[f] /= n;
    rhoPhi[f] = m->f[f].kind == DBSO_EMPTY
                    ? 0.0
                    : (cs->rho_l - cs->rho_g) * alphaPhi[f] + cs->rho_g * F[f];
  }
  if (tr) {
    if (tr->alphaPhi) memcpy(tr->alphaPhi, alphaPhi, sizeof(double) * nf);
    if (tr->alpha_new) memcpy(tr->alpha_new, alpha_new, sizeof(double) * nc);
  }
  free(cur);
  free(sub);
}

/* ------------------------------------------------------- 3.-4. momentum */

typedef struct {
  double *aP;        /* diagonal per unit volume */
  double *aON, *aNO; /* per face: owner-row coefficient of U_nbr, nbr-row of U_own */
  double *Sh;        /* explicit source, 3 x nc (component-major) */
} momeq_t;


/* face force q_f = [F_c - (g.x_f) dn(rho) - dn(p_rgh)] A_f along +axis on
   interior and outlet faces (R3, R12).  Fixed-flux faces (walls, inlets) are
   filled by fixed_flux_forces. */
static double face_body_force(const mesh_t *m, const props_t *pr, const double *alpha, int f);

static void face_forces(const mesh_t *m, const props_t *pr, const double *alpha,
                        const double *prgh, double *q) {
  const dbso_case *cs = m->cs;
  for (int f = 0; f < m->nf; f++) {
    const face_t *Fc = &m->f[f];
    q[f] = 0.0;
    if (Fc->kind == DBSO_EMPTY) continue;
    if (Fc->bnd >= 0) {
      if (Fc->kind != DBSO_OUTLET) continue;
      double so;
      int c = bnd_cell(Fc, &so);
      double pb = cs->bc_p[Fc->bnd] - pr[c].rho * dot3(cs->g, Fc->xf);
      double sn = so > 0.0 ? (pb - prgh[c]) / Fc->dist : (prgh[c] - pb) / Fc->dist;
      q[f] = -sn * Fc->area;
      continue;
    }
    q[f] = (face_body_force(m, pr, alpha, f) - (prgh[Fc->nbr] - prgh[Fc->own]) / Fc->dist) *
           Fc->area;
  }
}

/* Fixed-flux faces (R12): in a corrector (HbyA != NULL) the boundary normal
   gradient of p_rgh is the one that makes the corrected flux equal the
   prescribed flux, so q_b = (F_b - HbyA_n A) / rAU_P; in the predictor the
   force density is extrapolated from the opposite face of the same cell. */
static void fixed_flux_forces(const mesh_t *m, const double *HbyA, const double *rAU,
                              double *q) {
  for (int f = 0; f < m->nf; f++) {
    const face_t *Fc = &m->f[f];
    if (Fc->bnd < 0 || (Fc->kind != DBSO_WALL && !is_inlet(Fc->kind))) continue;
    double so;
    int c = bnd_cell(Fc, &so);
    int a = Fc->axis;
    if (HbyA) {
      double Ub[3], ab;
      if (is_inlet(Fc->kind)) inlet_face(m, Fc, Ub, &ab);
      double Fb = is_inlet(Fc->kind) ? Ub[a] * Fc->area : 0.0;
      q[f] = (Fb - HbyA[a * m->nc + c] * Fc->area) / rAU[c];
    } else {
      int opp = m->cf[c * 6 + 2 * a + (so > 0.0 ? 0 : 1)];
      const face_t *Fo = &m->f[opp];
      q[f] = (Fo->bnd >= 0 && Fo->kind != DBSO_OUTLET) ? 0.0 : q[opp];
    }
  }
}

/* capillary + gravity part of the face force only (phig / rAU_f / A_f) */
static double face_body_force(const mesh_t *m, const props_t *pr, const double *alpha, int f) {
  const dbso_case *cs = m->cs;
  const face_t *Fc = &m->f[f];
  int o = Fc->own, n = Fc->nbr;
  double d = Fc->dist;
  double cff = 0.5 * (pr[o].cf + pr[n].cf), pcf = 0.5 * (pr[o].pc + pr[n].pc);
  double Fcap = cff * ((cs->rho_l - cs->rho_g) * cs->g[Fc->axis] + (pr[n].pc - pr[o].pc) / d) -
                pcf * (alpha[n] - alpha[o]) / d;
  if (cs->sigma != 0.0) Fcap += 0.5 * (pr[o].sk + pr[n].sk) * (alpha[n] - alpha[o]) / d;
  return Fcap - dot3(cs->g, Fc->xf) * (pr[n].rho - pr[o].rho) / d;
}

/* R(q)_P along each non-empty axis */
static void reconstruct(const mesh_t *m, const double *q, double *R) {
  for (int c = 0; c < m->nc; c++)
    for (int a = 0; a < 3; a++) {
      int fm = m->cf[c * 6 + 2 * a], fp = m->cf[c * 6 + 2 * a + 1];
      if (m->f[fm].kind == DBSO_EMPTY) { R[a * m->nc + c] = 0.0; continue; }
      R[a * m->nc + c] = (q[fm] + q[fp]) / (2.0 * m->f[fm].area);
    }
}

/* sum over neighbours of a_N U_N for component d */
static double nb_sum(const mesh_t *m, const momeq_t *eq, const double *U, int c) {
  double s = 0.0;
  for (int k = 0; k < 6; k++) {
    int f = m->cf[c * 6 + k];
    const face_t *Fc = &m->f[f];
    if (Fc->bnd >= 0) continue;
    if (k & 1) s += eq->aON[f] * U[Fc->nbr];
    else s += eq->aNO[f] * U[Fc->own];
  }
  return s;
}

static void momentum_assemble(const mesh_t *m, const double *phi, const props_t *po,
                              const props_t *pn, const double *alpha_new,
                              const double *U, const double *rhoPhi, const double *F,
                              momeq_t *eq) {
  const dbso_case *cs = m->cs;
  int nc = m->nc, nf = m->nf;
  double V = m->V, dt = cs->dt;
  for (int c = 0; c < nc; c++) {
    eq->aP[c] = pn[c].rho / (phi[c] * dt) + pn[c].K;
    for (int d = 0; d < 3; d++) eq->Sh[d * nc + c] = po[c].rho * U[d * nc + c] / (phi[c] * dt);
  }
  for (int f = 0; f < nf; f++) {
    const face_t *Fc = &m->f[f];
    eq->aON[f] = eq->aNO[f] = 0.0;
    if (Fc->kind == DBSO_EMPTY) continue;
    double rp = rhoPhi[f];
    if (Fc->bnd < 0) {
      int o = Fc->own, n = Fc->nbr;
      double phf = 0.5 * (phi[o] + phi[n]);
      double vis = 0.5 * (pn[o].mu + pn[n].mu) * Fc->area / (Fc->dist * V);
      eq->aP[o] += maxd(rp, 0.0) / (phf * phi[o] * V) + vis;
      eq->aON[f] = maxd(-rp, 0.0) / (phf * phi[o] * V) + vis;
      eq->aP[n] += maxd(-rp, 0.0) / (phf * phi[n] * V) + vis;
      eq->aNO[f] = maxd(rp, 0.0) / (phf * phi[n] * V) + vis;
      continue;
    }
    double so;
    int c = bnd_cell(Fc, &so);
    double out = so * rp;
    double conv = 1.0 / (phi[c] * phi[c] * V);
    if (Fc->kind == DBSO_WALL) {
      eq->aP[c] += pn[c].mu * Fc->area / (Fc->dist * V);
    } else if (is_inlet(Fc->kind)) {
      double Ub[3], ab;
      inlet_face(m, Fc, Ub, &ab);
      double vis = (ab * cs->mu_l + (1.0 - ab) * cs->mu_g) * Fc->area / (Fc->dist * V);
      if (out >= 0.0) eq->aP[c] += out * conv;
      else
        for (int d = 0; d < 3; d++) eq->Sh[d * nc + c] += -out * Ub[d] * conv;
      eq->aP[c] += vis;
      for (int d = 0; d < 3; d++) eq->Sh[d * nc + c] += vis * Ub[d];
    } else if (Fc->kind == DBSO_OUTLET) {
      eq->aP[c] += out * conv;
    }
  }
  if (cs->transpose_visc) {
    /* explicit div(mu grad(U)^T) from U^n (R10); gradU[c][i][d] = dU_d/dx_i */
    double *gU = (double *)calloc((size_t)nc * 9, sizeof(double));
    for (int f = 0; f < nf; f++) {
      const face_t *Fc = &m->f[f];
      if (Fc->kind == DBSO_EMPTY) continue;
      double Uf[3];
      if (Fc->bnd < 0) {
        for (int d = 0; d < 3; d++) Uf[d] = 0.5 * (U[d * nc + Fc->own] + U[d * nc + Fc->nbr]);
      } else {
        double so, Ub[3], ab;
        int c = bnd_cell(Fc, &so);
        if (is_inlet(Fc->kind)) inlet_face(m, Fc, Ub, &ab);
        for (int d = 0; d < 3; d++)
          Uf[d] = Fc->kind == DBSO_WALL ? 0.0 : is_inlet(Fc->kind) ? Ub[d] : U[d * nc + c];
      }
      for (int d = 0; d < 3; d++) {
        if (Fc->own >= 0) gU[Fc->own * 9 + Fc->axis * 3 + d] += Uf[d] * Fc->area / V;
        if (Fc->nbr >= 0) gU[Fc->nbr * 9 + Fc->axis * 3 + d] -= Uf[d] * Fc->area / V;
      }
    }
    for (int f = 0; f < nf; f++) {
      const face_t *Fc = &m->f[f];
      if (Fc->kind == DBSO_EMPTY) continue;
      int a = Fc->axis;
      for (int i = 0; i < 3; i++) {
        double gfi, muf;
        if (Fc->bnd < 0) {
          gfi = 0.5 * (gU[Fc->own * 9 + i * 3 + a] + gU[Fc->nbr * 9 + i * 3 + a]);
          muf = 0.5 * (pn[Fc->own].mu + pn[Fc->nbr].mu);
          double t = muf * Fc->area * gfi / V;
          eq->Sh[i * nc + Fc->own] += t;
          eq->Sh[i * nc + Fc->nbr] -= t;
        } else {
          double so;
          int c = bnd_cell(Fc, &so);
          gfi = gU[c * 9 + i * 3 + a];
          if (is_inlet(Fc->kind)) {
            double Ub[3], ab;
            inlet_face(m, Fc, Ub, &ab);
            muf = ab * cs->mu_l + (1.0 - ab) * cs->mu_g;
          } else {
            muf = pn[c].mu;
          }
          eq->Sh[i * nc + c] += so * muf * Fc->area * gfi / V;
        }
      }
    }
    free(gU);
  }
  (void)alpha_new;
  (void)F;
}

/* ---------------------------------------------------- pressure operator */

/* per-face coefficient of the SPD pressure operator (interior and outlet faces) */
static void pressure_coeffs(const mesh_t *m, const double *rAU, double *T) {
  for (int f = 0; f < m->nf; f++) {
    const face_t *Fc = &m->f[f];
    T[f] = 0.0;
    if (Fc->bnd < 0) {
      T[f] = 0.5 * (rAU[Fc->own] + rAU[Fc->nbr]) * Fc->area / Fc->dist;
    } else if (Fc->kind == DBSO_OUTLET) {
      double so;
      int c = bnd_cell(Fc, &so);
      T[f] = rAU[c] * Fc->area / Fc->dist;
    }
  }
}

static void apply_op(const mesh_t *m, const double *T, const double *x, double *y) {
  for (int c = 0; c < m->nc; c++) y[c] = 0.0;
  for (int f = 0; f < m->nf; f++) {
    const face_t *Fc = &m->f[f];
    if (T[f] == 0.0) continue;
    if (Fc->bnd < 0) {
      double t = T[f] * (x[Fc->own] - x[Fc->nbr]);
      y[Fc->own] += t;
      y[Fc->nbr] -= t;
    } else {
      double so;
      int c = bnd_cell(Fc, &so);
      y[c] += T[f] * x[c];
    }
  }
}

static int has_outlet(const dbso_case *cs) {
  for (int b = 0; b < 6; b++)
    if (cs->bc_kind[b] == DBSO_OUTLET) return 1;
  return 0;
}

static double vdot(int n, const double *a, const double *b) {
  double s = 0.0;
  for (int i = 0; i < n; i++) s += a[i] * b[i];
  return s;
}

static void remove_mean(int n, double *v) {
  double s = 0.0;
  for (int i = 0; i < n; i++) s += v[i];
  s /= n;
  for (int i = 0; i < n; i++) v[i] -= s;
}

/* Jacobi-preconditioned CG for A x = b (R14, R15) */
static int pcg(const mesh_t *m, const double *T, const double *b_in, double *x,
               double tol, int maxit, int *iters, double *relres) {
  int n = m->nc, closed = !has_outlet(m->cs);
  double *b = (double *)malloc(sizeof(double) * n);
  double *r = (double *)malloc(sizeof(double) * n);
  double *z = (double *)malloc(sizeof(double) * n);
  double *p = (double *)malloc(sizeof(double) * n);
  double *q = (double *)malloc(sizeof(double) * n);
  double *dg = (double *)calloc((size_t)n, sizeof(double));
  memcpy(b, b_in, sizeof(double) * n);
  if (closed) remove_mean(n, b);
  for (int f = 0; f < m->nf; f++) {
    const face_t *Fc = &m->f[f];
    if (T[f] == 0.0) continue;
    if (Fc->bnd < 0) { dg[Fc->own] += T[f]; dg[Fc->nbr] += T[f]; }
    else { double so; dg[bnd_cell(Fc, &so)] += T[f]; }
  }
  apply_op(m, T, x, q);
  for (int i = 0; i < n; i++) r[i] = b[i] - q[i];
  if (closed) remove_mean(n, r);
  double nb = sqrt(vdot(n, b, b)), nr = sqrt(vdot(n, r, r));
  double norm = nb > 0.0 ? nb : nr;
  int it = 0, rc = 0;
  if (norm > 0.0 && nr > tol * norm) {
    for (int i = 0; i < n; i++) { z[i] = dg[i] > 0.0 ? r[i] / dg[i] : 0.0; p[i] = z[i]; }
    double rz = vdot(n, r, z);
    for (;;) {
      if (it >= maxit) { rc = -4; break; }
      apply_op(m, T, p, q);
      double pq = vdot(n, p, q);
      if (pq <= 0.0) { rc = nr <= tol * norm ? 0 : -4; break; }
      double al = rz / pq;
      for (int i = 0; i < n; i++) { x[i] += al * p[i]; r[i] -= al * q[i]; }
      it++;
      nr = sqrt(vdot(n, r, r));
      if (nr <= tol * norm) break;
      for (int i = 0; i < n; i++) z[i] = dg[i] > 0.0 ? r[i] / dg[i] : 0.0;
      double rz1 = vdot(n, r, z);
      double be = rz1 / rz;
      rz = rz1;
      for (int i = 0; i < n; i++) p[i] = z[i] + be * p[i];
    }
  }
  if (closed) remove_mean(n, x);
  /* report the true residual */
  apply_op(m, T, x, q);
  for (int i = 0; i < n; i++) r[i] = b[i] - q[i];
  if (closed) remove_mean(n, r);
  if (iters) *iters = it;
  if (relres) *relres = norm > 0.0 ? sqrt(vdot(n, r, r)) / norm : 0.0;
  free(b); free(r); free(z); free(p); free(q); free(dg);
  return rc;
}

/* --------------------------------------------------------------- driver */

int dbso_init_flux(const dbso_case *cs, const double *Ux, const double *Uy,
                   const double *Uz, double *Fx, double *Fy, double *Fz) {
  mesh_t m;
  if (build_mesh(cs, &m)) { free_mesh(&m); return -1; }
  m.t = cs->t0;
  const double *U[3] = {Ux, Uy, Uz};
  double *Fo[3] = {Fx, Fy, Fz};
  int off = 0;
  for (int a = 0; a < 3; a++) {
    for (int l = 0; l < m.nfa[a]; l++) {
      const face_t *Fc = &m.f[off + l];
      double v = 0.0;
      if (Fc->bnd < 0) {
        v = 0.5 * (U[a][Fc->own] + U[a][Fc->nbr]) * Fc->area;
      } else if (is_inlet(Fc->kind)) {
        double Ub[3], ab;
        inlet_face(&m, Fc, Ub, &ab);
        v = Ub[a] * Fc->area;
      } else if (Fc->kind == DBSO_OUTLET) {
        double so;
        v = U[a][bnd_cell(Fc, &so)] * Fc->area;
      }
      Fo[a][l] = v;
    }
    off += m.nfa[a];
  }
  free_mesh(&m);
  return 0;
}

int dbso_inlet_values(const dbso_case *cs, int b, double t, double *out) {
  if (b < 0 || b > 5 || !is_inlet(cs->bc_kind[b])) return -1;
  mesh_t m;
  if (build_mesh(cs, &m)) { free_mesh(&m); return -1; }
  m.t = t;
  int n = 0, off = 0;
  for (int a = 0; a < 3; a++) {
    for (int l = 0; l < m.nfa[a]; l++) {
      const face_t *Fc = &m.f[off + l];
      if (Fc->bnd != b) continue;
      double Ub[3], ab;
      inlet_face(&m, Fc, Ub, &ab);
      for (int d = 0; d < 3; d++) out[4 * n + d] = Ub[d];
      out[4 * n + 3] = ab;
      n++;
    }
    off += m.nfa[a];
  }
  free_mesh(&m);
  return n;
}

int dbso_curvature(const dbso_case *cs, const double *alpha, const double *kinv,
                   const double *Fx, const double *Fy, const double *Fz, double *kappa) {
  mesh_t m;
  if (build_mesh(cs, &m)) { free_mesh(&m); return -1; }
  double *F = (double *)malloc(sizeof(double) * m.nf);
  memcpy(F, Fx, sizeof(double) * m.nfa[0]);
  memcpy(F + m.nfa[0], Fy, sizeof(double) * m.nfa[1]);
  memcpy(F + m.nfa[0] + m.nfa[1], Fz, sizeof(double) * m.nfa[2]);
  curvature(&m, alpha, kinv, F, kappa);
  free(F);
  free_mesh(&m);
  return 0;
}

int dbso_pressure_apply(const dbso_case *cs, const double *rAU, const double *x,
                        double *y) {
  mesh_t m;
  if (build_mesh(cs, &m)) { free_mesh(&m); return -1; }
  double *T = (double *)malloc(sizeof(double) * m.nf);
  pressure_coeffs(&m, rAU, T);
  apply_op(&m, T, x, y);
  free(T);
  free_mesh(&m);
  return 0;
}

int dbso_pressure_solve(const dbso_case *cs, const double *rAU, const double *b,
                        double *x, double tol, int maxit, int *iters, double *relres) {
  mesh_t m;
  if (build_mesh(cs, &m)) { free_mesh(&m); return -1; }
  double *T = (double *)malloc(sizeof(double) * m.nf);
  pressure_coeffs(&m, rAU, T);
  int rc = pcg(&m, T, b, x, tol, maxit, iters, relres);
  free(T);
  free_mesh(&m);
  return rc;
}

int dbso_alpha_advance(const dbso_case *cs, const double *phi, const double *kinv,
                       double *alpha, const double *Fx, const double *Fy, const double *Fz,
                       const double *p_rgh, int nsteps, double *alphaPhi) {
  mesh_t m;
  if (build_mesh(cs, &m)) { free_mesh(&m); return -1; }
  int nc = m.nc, nf = m.nf;
  for (int c = 0; c < nc; c++)
    if (!(phi[c] > 0.0 && phi[c] <= 1.0) || !(kinv[c] >= 0.0) ||
        (phi[c] == 1.0 && kinv[c] > 0.0)) { free_mesh(&m); return -1; }
  double *F = (double *)malloc(sizeof(double) * nf);
  double *an = (double *)malloc(sizeof(double) * nc);
  double *aPhi = (double *)malloc(sizeof(double) * nf);
  double *rPhi = (double *)malloc(sizeof(double) * nf);
  memcpy(F, Fx, sizeof(double) * m.nfa[0]);
  memcpy(F + m.nfa[0], Fy, sizeof(double) * m.nfa[1]);
  memcpy(F + m.nfa[0] + m.nfa[1], Fz, sizeof(double) * m.nfa[2]);
  for (int st = 0; st < nsteps; st++) {
    m.t = cs->t0 + (st + 1) * cs->dt;
    alpha_transport(&m, phi, kinv, alpha, F, p_rgh, an, aPhi, rPhi, NULL);
    memcpy(alpha, an, sizeof(double) * nc);
  }
  if (alphaPhi && nsteps > 0) memcpy(alphaPhi, aPhi, sizeof(double) * nf);
  free(F); free(an); free(aPhi); free(rPhi);
  free_mesh(&m);
  return 0;
}

int dbso_step(const dbso_case *cs, const double *phi, const double *kinv,
              double *alpha, double *Ux, double *Uy, double *Uz, double *p_rgh,
              double *p_out, double *Fx, double *Fy, double *Fz, int nsteps,
              dbso_info *info, dbso_trace *trace) {
  mesh_t m;
  /* working copy: the adaptive time step (R19) changes dt between steps */
  dbso_case cw = *cs;
  int rc = build_mesh(&cw, &m);
  if (rc) { free_mesh(&m); return rc; }
  cs = &cw;
  if (cw.target_courant > 0.0 && !(cw.dt_max > 0.0)) { free_mesh(&m); return -1; }
  int nc = m.nc, nf = m.nf;
  /* porosity in (0, 1], k^-1 >= 0, and no drag in a solid-free cell */
  for (int c = 0; c < nc; c++)
    if (!(phi[c] > 0.0 && phi[c] <= 1.0) || !(kinv[c] >= 0.0) ||
        (phi[c] == 1.0 && kinv[c] > 0.0)) { free_mesh(&m); return -1; }
  double tnow = cw.t0;
  double V = m.V;
  double *F = (double *)malloc(sizeof(double) * nf);
  double *U = (double *)malloc(sizeof(double) * 3 * nc);
  double *U2 = (double *)malloc(sizeof(double) * 3 * nc);
  double *an = (double *)malloc(sizeof(double) * nc);
  double *kap = (double *)malloc(sizeof(double) * nc);
  double *aPhi = (double *)malloc(sizeof(double) * nf);
  double *rPhi = (double *)malloc(sizeof(double) * nf);
  double *q = (double *)malloc(sizeof(double) * nf);
  double *R = (double *)malloc(sizeof(double) * 3 * nc);
  double *B = (double *)malloc(sizeof(double) * 3 * nc);
  double *rAU = (double *)malloc(sizeof(double) * nc);
  double *HbyA = (double *)malloc(sizeof(double) * 3 * nc);
  double *phiH = (double *)malloc(sizeof(double) * nf);
  double *T = (double *)malloc(sizeof(double) * nf);
  double *b = (double *)malloc(sizeof(double) * nc);
  props_t *po = (props_t *)malloc(sizeof(props_t) * nc);
  props_t *pn = (props_t *)malloc(sizeof(props_t) * nc);
  momeq_t eq;
  eq.aP = (double *)malloc(sizeof(double) * nc);
  eq.aON = (double *)malloc(sizeof(double) * nf);
  eq.aNO = (double *)malloc(sizeof(double) * nf);
  eq.Sh = (double *)malloc(sizeof(double) * 3 * nc);
  memcpy(F, Fx, sizeof(double) * m.nfa[0]);
  memcpy(F + m.nfa[0], Fy, sizeof(double) * m.nfa[1]);
  memcpy(F + m.nfa[0] + m.nfa[1], Fz, sizeof(double) * m.nfa[2]);
  memcpy(U, Ux, sizeof(double) * nc);
  memcpy(U + nc, Uy, sizeof(double) * nc);
  memcpy(U + 2 * nc, Uz, sizeof(double) * nc);
  if (info) memset(info, 0, sizeof(*info));

  for (int step = 0; step < nsteps && rc == 0; step++) {
    dbso_trace *tr = step == 0 ? trace : NULL;
    if (cw.target_courant > 0.0) {
      /* R19: Courant number of the current fluxes at the current dt */
      double rate = 0.0;
      for (int c = 0; c < nc; c++) {
        double out = 0.0;
        for (int k = 0; k < 6; k++) {
          const face_t *Fc = &m.f[m.cf[c * 6 + k]];
          if (Fc->kind == DBSO_EMPTY) continue;
          double fl = F[m.cf[c * 6 + k]];
          out += (k & 1) ? maxd(fl, 0.0) : maxd(-fl, 0.0);
        }
        rate = maxd(rate, out / (phi[c] * V));
      }
      double co = cw.dt * rate;
      double dtn = mind(cw.dt_max, 1.2 * cw.dt);
      if (co > 0.0) dtn = mind(dtn, cw.target_courant * cw.dt / co);
      cw.dt = dtn;
    }
    m.t = tnow + cw.dt;  /* boundary values at t^{n+1} (R16) */
    tnow = m.t;
    /* 1. saturation */
    for (int c = 0; c < nc; c++) cell_props(cs, alpha[c], kinv[c], &po[c]);
    alpha_transport(&m, phi, kinv, alpha, F, p_rgh, an, aPhi, rPhi, tr);
    /* 2. properties at alpha^{n+1}, with the clear-fluid CSF coefficient */
    for (int c = 0; c < nc; c++) cell_props(cs, an[c], kinv[c], &pn[c]);
    if (cs->sigma != 0.0) {
      curvature(&m, an, kinv, F, kap);
      for (int c = 0; c < nc; c++)
        pn[c].sk = kinv[c] > 0.0 ? 0.0 : cs->sigma * kap[c] / phi[c];
    }
    /* 3. momentum predictor */
    momentum_assemble(&m, phi, po, pn, an, U, rPhi, F, &eq);
    face_forces(&m, pn, an, p_rgh, q);
    fixed_flux_forces(&m, NULL, NULL, q);
    reconstruct(&m, q, R);
    for (int i = 0; i < 3 * nc; i++) B[i] = eq.Sh[i] + R[i];
    if (tr) {
      if (tr->aP) memcpy(tr->aP, eq.aP, sizeof(double) * nc);
      if (tr->aON) memcpy(tr->aON, eq.aON, sizeof(double) * nf);
      if (tr->aNO) memcpy(tr->aNO, eq.aNO, sizeof(double) * nf);
      if (tr->B) memcpy(tr->B, B, sizeof(double) * 3 * nc);
    }
    /* the implicit predictor system a_P U - sum a_N U_N = B (R11): Jacobi
       sweeps from U^n; each sweep also forms the residual of the iterate it
       starts from, and the solve ends after the sweep whose starting
       residual is at most mom_tol ||B|| */
    {
      double nB = sqrt(vdot(3 * nc, B, B));
      int sw = 0;
      double rel = 0.0;
      while (sw < cs->mom_maxit) {
        double r2 = 0.0;
        for (int d = 0; d < 3; d++)
          for (int c = 0; c < nc; c++) {
            double acc = nb_sum(&m, &eq, U + d * nc, c) + B[d * nc + c];
            double r = acc - eq.aP[c] * U[d * nc + c];
            r2 += r * r;
            U2[d * nc + c] = acc / eq.aP[c];
          }
        memcpy(U, U2, sizeof(double) * 3 * nc);
        sw++;
        rel = nB > 0.0 ? sqrt(r2) / nB : 0.0;
        if (sqrt(r2) <= cs->mom_tol * nB) break;
      }
      if (info) { info->mom_sweeps = sw; info->mom_relres = rel; }
    }
    if (tr) {
      if (tr->Shat) memcpy(tr->Shat, eq.Sh, sizeof(double) * 3 * nc);
      if (tr->Ustar) memcpy(tr->Ustar, U, sizeof(double) * 3 * nc);
    }
    /* 4. PISO correctors */
    for (int c = 0; c < nc; c++) rAU[c] = 1.0 / eq.aP[c];
    pressure_coeffs(&m, rAU, T);
    for (int corr = 0; corr < cs->n_corr; corr++) {
      for (int d = 0; d < 3; d++)
        for (int c = 0; c < nc; c++)
          HbyA[d * nc + c] = rAU[c] * (nb_sum(&m, &eq, U + d * nc, c) + eq.Sh[d * nc + c]);
      for (int f = 0; f < nf; f++) {
        const face_t *Fc = &m.f[f];
        int a = Fc->axis;
        phiH[f] = 0.0;
        if (Fc->kind == DBSO_EMPTY || Fc->kind == DBSO_WALL) continue;
        if (Fc->bnd < 0) {
          int o = Fc->own, n = Fc->nbr;
          double rAUf = 0.5 * (rAU[o] + rAU[n]);
          phiH[f] = 0.5 * (HbyA[a * nc + o] + HbyA[a * nc + n]) * Fc->area +
                    rAUf * face_body_force(&m, pn, an, f) * Fc->area;
        } else if (is_inlet(Fc->kind)) {
          double Ub[3], ab;
          inlet_face(&m, Fc, Ub, &ab);
          phiH[f] = Ub[a] * Fc->area;
        } else {
          double so;
          phiH[f] = HbyA[a * nc + bnd_cell(Fc, &so)] * Fc->area;
        }
      }
      for (int c = 0; c < nc; c++) {
        double div = 0.0, dir = 0.0;
        for (int s = 0; s < 6; s++) {
          int f = m.cf[c * 6 + s];
          const face_t *Fc = &m.f[f];
          div += ((s & 1) ? 1.0 : -1.0) * phiH[f];
          if (Fc->kind == DBSO_OUTLET) {
            double pb = cs->bc_p[Fc->bnd] - pn[c].rho * dot3(cs->g, Fc->xf);
            dir += T[f] * pb;
          }
        }
        b[c] = -div + dir;
      }
      if (tr && corr == 0) {
        if (tr->rAU) memcpy(tr->rAU, rAU, sizeof(double) * nc);
        if (tr->HbyA) memcpy(tr->HbyA, HbyA, sizeof(double) * 3 * nc);
        if (tr->phiHbyA) memcpy(tr->phiHbyA, phiH, sizeof(double) * nf);
        if (tr->b) memcpy(tr->b, b, sizeof(double) * nc);
      }
      int its = 0;
      double rr = 0.0;
      int src = pcg(&m, T, b, p_rgh, cs->p_tol, cs->p_maxit, &its, &rr);
      if (info && corr < 16) {
        info->p_iters[corr] = its;
        info->p_relres[corr] = rr;
        /* the norm the solve is relative to (closed domains: projected b) */
        double bb = 0.0, mb = 0.0;
        if (!has_outlet(cs)) {
          for (int c = 0; c < nc; c++) mb += b[c];
          mb /= nc;
        }
        for (int c = 0; c < nc; c++) bb += (b[c] - mb) * (b[c] - mb);
        info->p_bnorm[corr] = sqrt(bb);
      }
      if (src) rc = src;
      /* flux and velocity correction */
      for (int f = 0; f < nf; f++) {
        const face_t *Fc = &m.f[f];
        F[f] = phiH[f];
        if (Fc->bnd < 0) {
          F[f] -= T[f] * (p_rgh[Fc->nbr] - p_rgh[Fc->own]);
        } else if (Fc->kind == DBSO_OUTLET) {
          double so;
          int c = bnd_cell(Fc, &so);
          double pb = cs->bc_p[Fc->bnd] - pn[c].rho * dot3(cs->g, Fc->xf);
          F[f] -= so > 0.0 ? T[f] * (pb - p_rgh[c]) : T[f] * (p_rgh[c] - pb);
        }
      }
      face_forces(&m, pn, an, p_rgh, q);
      fixed_flux_forces(&m, HbyA, rAU, q);
      reconstruct(&m, q, R);
      for (int d = 0; d < 3; d++)
        for (int c = 0; c < nc; c++)
          U[d * nc + c] = HbyA[d * nc + c] + rAU[c] * R[d * nc + c];
    }
    memcpy(alpha, an, sizeof(double) * nc);
  }

  /* outputs */
  memcpy(Ux, U, sizeof(double) * nc);
  memcpy(Uy, U + nc, sizeof(double) * nc);
  memcpy(Uz, U + 2 * nc, sizeof(double) * nc);
  memcpy(Fx, F, sizeof(double) * m.nfa[0]);
  memcpy(Fy, F + m.nfa[0], sizeof(double) * m.nfa[1]);
  memcpy(Fz, F + m.nfa[0] + m.nfa[1], sizeof(double) * m.nfa[2]);
  if (p_out) {
    for (int c = 0; c < nc; c++) {
      double x[3];
      cell_centre(&m, c, x);
      double rho = alpha[c] * cs->rho_l + (1.0 - alpha[c]) * cs->rho_g;
      p_out[c] = p_rgh[c] + rho * dot3(cs->g, x);
    }
  }
  if (info) {
    info->alpha_min = 1e300;
    info->alpha_max = -1e300;
    info->phase_volume = 0.0;
    info->max_div = 0.0;
    info->dt_last = cw.dt;
    info->t_end = tnow;
    for (int c = 0; c < nc; c++) {
      info->alpha_min = mind(info->alpha_min, alpha[c]);
      info->alpha_max = maxd(info->alpha_max, alpha[c]);
      info->phase_volume += phi[c] * alpha[c] * V;
      double div = 0.0;
      for (int s = 0; s < 6; s++) div += ((s & 1) ? 1.0 : -1.0) * F[m.cf[c * 6 + s]];
      info->max_div = maxd(info->max_div, fabs(div));
    }
  }
  free(F); free(U); free(U2); free(an); free(kap); free(aPhi); free(rPhi); free(q); free(R);
  free(B); free(rAU); free(HbyA); free(phiH); free(T); free(b); free(po); free(pn);
  free(eq.aP); free(eq.aON); free(eq.aNO); free(eq.Sh);
  free_mesh(&m);
  return rc;
}
