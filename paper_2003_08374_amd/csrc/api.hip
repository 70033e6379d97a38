// C ABI of the DBS PISO step (declared in include/dbs.h): validation, device
// state, the step sequence of Sec. 3.2, state transfer, statistics and event
// timing.  No C++ exception leaves this file.
#include <math.h>
#include <string.h>

#include <new>
#include <string>

#include "dbs_internal.h"

using namespace dbs;

struct dbs_handle {
  Handle h;
};

namespace dbs {

static const char *kNames[KC_COUNT] = {
    "alpha_face", "alpha_bounds", "alpha_limit", "alpha_update", "mom_assemble",
    "mom_offdiag", "phihbya",     "correct",     "spmv",         "axpy",
    "dot",         "xpby",        "finalize",    "smooth_fine",  "restrict_fine",
    "prolong_fine", "smooth_coarse", "restrict_coarse", "prolong_coarse", "coarse_solve",
    "build_coarse", "stats",      "misc",        "smooth_fine_zero"};

void prof_begin(Handle *h, int cls) {
  Timer &t = h->tm;
  if (t.used + 2 > t.ev.size()) {
    for (int i = 0; i < 256; i++) {
      hipEvent_t e;
      hipEventCreate(&e);
      t.ev.push_back(e);
    }
    t.cls.resize(t.ev.size() / 2 + 1);
  }
  t.cls[t.used / 2] = cls;
  hipEventRecord(t.ev[t.used], h->stream);
}

void prof_end(Handle *h, int cls) {
  (void)cls;
  Timer &t = h->tm;
  hipEventRecord(t.ev[t.used + 1], h->stream);
  t.used += 2;
}

void prof_collect(Handle *h) {
  Timer &t = h->tm;
  if (t.used == 0) return;
  hipStreamSynchronize(h->stream);
  for (size_t i = 0; i < t.used; i += 2) {
    float ms = 0.f;
    hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]);
    int c = t.cls[i / 2];
    h->k_launches[c]++;
    h->k_ms[c] += ms;
  }
  t.used = 0;
}

// ------------------------------------------------------------- statistics

// per block: min alpha, max alpha, sum phi alpha V, max Courant, non-finite count
__global__ void __launch_bounds__(NTHREADS) k_stats(Geom G, const double *__restrict__ alpha,
                                                    const double *__restrict__ U,
                                                    const double *__restrict__ prgh,
                                                    const double *__restrict__ phi,
                                                    const double *__restrict__ F,
                                                    double *__restrict__ part, int nb) {
  __shared__ double lds[5][NTHREADS / 64];
  double amin = 1e300, amax = -1e300, vol = 0.0, co = 0.0, bad = 0.0;
  FOR_CELLS(G, P) {
    const double a = alpha[P.c];
    amin = fmin(amin, a);
    amax = fmax(amax, a);
    vol += phi[P.c] * a * G.V;
    double out = 0.0;
    for (int ax = 0; ax < 3; ax++) {
      const double fm = F[face_of(G, P, ax, 0)], fp = F[face_of(G, P, ax, 1)];
      out += fmax(fp, 0.0) + fmax(-fm, 0.0);
    }
    co = fmax(co, G.dt * out / (phi[P.c] * G.V));
    bool ok = isfinite(a) && isfinite(prgh[P.c]);
    for (int d = 0; d < 3; d++) ok = ok && isfinite(U[(size_t)d * G.nc + P.c]);
    bad += ok ? 0.0 : 1.0;
  }
  amin = wave_min(amin);
  amax = wave_max(amax);
  vol = wave_sum(vol);
  co = wave_max(co);
  bad = wave_sum(bad);
  const int t = threadIdx.x + BX * threadIdx.y;
  if ((t & 63) == 0) {
    lds[0][t >> 6] = amin; lds[1][t >> 6] = amax; lds[2][t >> 6] = vol;
    lds[3][t >> 6] = co;   lds[4][t >> 6] = bad;
  }
  __syncthreads();
  if (t == 0) {
    double r[5] = {1e300, -1e300, 0.0, 0.0, 0.0};
    for (int w = 0; w < NTHREADS / 64; w++) {
      r[0] = fmin(r[0], lds[0][w]); r[1] = fmax(r[1], lds[1][w]); r[2] += lds[2][w];
      r[3] = fmax(r[3], lds[3][w]); r[4] += lds[4][w];
    }
    for (int q = 0; q < 5; q++) part[q * nb + blockIdx.x] = r[q];
  }
}

__global__ void __launch_bounds__(1024) k_stats_final(const double *__restrict__ part, int nb,
                                                      double *__restrict__ out) {
  __shared__ double lds[5][16];
  const int t = threadIdx.x;
  double r[5] = {1e300, -1e300, 0.0, 0.0, 0.0};
  for (int i = t; i < nb; i += 1024) {
    r[0] = fmin(r[0], part[i]); r[1] = fmax(r[1], part[nb + i]); r[2] += part[2 * nb + i];
    r[3] = fmax(r[3], part[3 * nb + i]); r[4] += part[4 * nb + i];
  }
  r[0] = wave_min(r[0]); r[1] = wave_max(r[1]); r[2] = wave_sum(r[2]);
  r[3] = wave_max(r[3]); r[4] = wave_sum(r[4]);
  if ((t & 63) == 0)
    for (int q = 0; q < 5; q++) lds[q][t >> 6] = r[q];
  __syncthreads();
  if (t == 0) {
    double s[5] = {1e300, -1e300, 0.0, 0.0, 0.0};
    for (int w = 0; w < 16; w++) {
      s[0] = fmin(s[0], lds[0][w]); s[1] = fmax(s[1], lds[1][w]); s[2] += lds[2][w];
      s[3] = fmax(s[3], lds[3][w]); s[4] += lds[4][w];
    }
    for (int q = 0; q < 5; q++) out[q] = s[q];
  }
}

void cell_stats(Handle *h, double out[5]) {
  dim3 blk(BX, BY);
  // partials holds 2 x nblocks doubles; the statistics need 5 x nblocks
  DBS_LAUNCH(h, KC_STATS, k_stats, h->grid, blk, h->G, (const double *)h->alpha,
             (const double *)h->U, (const double *)h->prgh, (const double *)h->phi,
             (const double *)h->F, h->Qp, h->nblocks);
  DBS_LAUNCH(h, KC_STATS, k_stats_final, dim3(1), dim3(1024), (const double *)h->Qp,
             h->nblocks, h->scal + 16);
  hipMemcpyAsync(h->hscal + 16, h->scal + 16, 5 * sizeof(double), hipMemcpyDeviceToHost,
                 h->stream);
  hipStreamSynchronize(h->stream);
  for (int q = 0; q < 5; q++) out[q] = h->hscal[16 + q];
}

}  // namespace dbs

// ------------------------------------------------------------------ helpers

static int fail(Handle *h, int code, const std::string &msg) {
  if (h) h->err = msg;
  return code;
}

static int hip_check(Handle *h, hipError_t e, const char *what) {
  if (e == hipSuccess) return DBS_OK;
  return fail(h, DBS_EHIP, std::string(what) + ": " + hipGetErrorString(e));
}

static double *dmalloc(Handle *h, size_t n, int &rc) {
  void *p = nullptr;
  if (rc) return nullptr;
  if (hipMalloc(&p, (n ? n : 1) * sizeof(double)) != hipSuccess) {
    rc = DBS_ENOMEM;
    return nullptr;
  }
  hipMemsetAsync(p, 0, (n ? n : 1) * sizeof(double), h->stream);
  h->allocs.push_back(p);
  return (double *)p;
}

static bool all_finite(const double *a, size_t n) {
  for (size_t i = 0; i < n; i++)
    if (!isfinite(a[i])) return false;
  return true;
}

static int validate(const dbs_grid *g, const dbs_physics *p, const dbs_bc *bc,
                    const dbs_controls *c, std::string &msg) {
  if (!g || !p || !bc || !c) { msg = "null argument"; return DBS_EINVAL; }
  const int n[3] = {g->nx, g->ny, g->nz};
  const double hh[3] = {g->dx, g->dy, g->dz};
  long long nc = 1;
  for (int a = 0; a < 3; a++) {
    if (n[a] < 1 || !(hh[a] > 0.0) || !isfinite(hh[a])) { msg = "bad grid"; return DBS_EINVAL; }
    nc *= n[a];
    const bool e0 = bc[2 * a].kind == DBS_BC_EMPTY, e1 = bc[2 * a + 1].kind == DBS_BC_EMPTY;
    if (e0 != e1 || (e0 && n[a] != 1)) {
      msg = "EMPTY faces must pair on an axis of one cell";
      return DBS_EINVAL;
    }
  }
  if (nc * 4 > 2000000000LL) { msg = "mesh too large for 32-bit indices"; return DBS_EINVAL; }
  for (int b = 0; b < 6; b++)
    if (bc[b].kind < DBS_BC_WALL || bc[b].kind > DBS_BC_EMPTY) { msg = "bad bc kind"; return DBS_EINVAL; }
  if (p->kr_model != DBS_BROOKS_COREY && p->kr_model != DBS_VAN_GENUCHTEN) { msg = "kr_model"; return DBS_EINVAL; }
  if (p->pc_model != DBS_BROOKS_COREY && p->pc_model != DBS_VAN_GENUCHTEN) { msg = "pc_model"; return DBS_EINVAL; }
  if (!(p->kr_m > 0.0) || !(1.0 - p->s_girr - p->s_lirr > 0.0)) { msg = "kr parameters"; return DBS_EINVAL; }
  if (!(p->a_pcmax - p->a_pcirr > 0.0) || !(p->eps_pc > 0.0 && p->eps_pc < 0.5) || !(p->pc0 >= 0.0)) {
    msg = "pc parameters"; return DBS_EINVAL;
  }
  if (p->pc_model == DBS_VAN_GENUCHTEN && !(p->pc_exp > 0.0 && p->pc_exp < 1.0)) { msg = "VG m"; return DBS_EINVAL; }
  if (!(p->rho_l > 0.0 && p->rho_g > 0.0 && p->mu_l > 0.0 && p->mu_g > 0.0)) { msg = "fluid properties"; return DBS_EINVAL; }
  if (!(c->dt > 0.0) || c->n_corr < 1 || c->n_corr > 16 || c->mom_sweeps < 0 ||
      c->mules_iter < 1 || !(c->p_tol > 0.0) || c->p_maxit < 1 ||
      (c->precision != DBS_FP64 && c->precision != DBS_MIXED) || c->mg_pre < 0 || c->mg_post < 0) {
    msg = "bad controls";
    return DBS_EINVAL;
  }
  return DBS_OK;
}

// ----------------------------------------------------------------- the ABI

extern "C" {

int dbs_kernel_classes(void) { return KC_COUNT; }

const char *dbs_kernel_name(int cls) {
  return (cls >= 0 && cls < KC_COUNT) ? kNames[cls] : "";
}

int dbs_create(const dbs_grid *grid, const dbs_physics *phys, const dbs_bc bc[6],
               const dbs_controls *ctl, dbs_handle **out) {
  if (!out) return DBS_EINVAL;
  *out = nullptr;
  std::string msg;
  int rc = validate(grid, phys, bc, ctl, msg);
  if (rc) return rc;
  dbs_handle *H = new (std::nothrow) dbs_handle();
  if (!H) return DBS_ENOMEM;
  Handle *h = &H->h;
  Geom &G = h->G;
  memset(&G, 0, sizeof(G));
  G.n[0] = grid->nx; G.n[1] = grid->ny; G.n[2] = grid->nz;
  G.h[0] = grid->dx; G.h[1] = grid->dy; G.h[2] = grid->dz;
  G.nc = G.n[0] * G.n[1] * G.n[2];
  G.fo[0] = 0;
  G.fo[1] = (G.n[0] + 1) * G.n[1] * G.n[2];
  G.fo[2] = G.fo[1] + G.n[0] * (G.n[1] + 1) * G.n[2];
  G.nf = G.fo[2] + G.n[0] * G.n[1] * (G.n[2] + 1);
  G.V = G.h[0] * G.h[1] * G.h[2];
  G.iV = 1.0 / G.V;
  for (int a = 0; a < 3; a++) {
    G.ih[a] = 1.0 / G.h[a];
    G.area[a] = G.V / G.h[a];
  }
  G.dt = ctl->dt;
  G.has_outlet = 0;
  for (int b = 0; b < 6; b++) {
    G.bck[b] = bc[b].kind;
    for (int a = 0; a < 3; a++) G.bcU[b][a] = bc[b].U[a];
    G.bca[b] = bc[b].alpha;
    G.bcp[b] = bc[b].p;
    if (bc[b].kind == DBS_BC_OUTLET) G.has_outlet = 1;
  }
  G.dN = 1e-8 / cbrt(G.V);
  Phys &P = h->P;
  P.rho_l = phys->rho_l; P.rho_g = phys->rho_g; P.mu_l = phys->mu_l; P.mu_g = phys->mu_g;
  for (int a = 0; a < 3; a++) P.g[a] = phys->g[a];
  P.c_alpha = phys->c_alpha;
  P.kr_model = phys->kr_model;
  P.kr_m = phys->kr_m;
  P.inv_kr_m = 1.0 / phys->kr_m;
  P.s_lirr = phys->s_lirr;
  P.inv_span_kr = 1.0 / (1.0 - phys->s_girr - phys->s_lirr);
  P.pc_model = phys->pc_model;
  P.pc0 = phys->pc0;
  P.pc_exp = phys->pc_exp;
  P.a_pcirr = phys->a_pcirr;
  P.inv_span_pc = 1.0 / (phys->a_pcmax - phys->a_pcirr);
  P.eps_pc = phys->eps_pc;
  h->ctl = *ctl;
  h->mg_pre = ctl->mg_pre > 0 ? ctl->mg_pre : 2;
  h->mg_post = ctl->mg_post > 0 ? ctl->mg_post : 2;
  memset(&h->st, 0, sizeof(h->st));
  if ((rc = hip_check(h, hipStreamCreate(&h->own_stream), "hipStreamCreate"))) {
    delete H;
    return rc;
  }
  h->stream = h->own_stream;
  h->nblocks = cell_blocks(G);
  h->grid = dim3(h->nblocks);
  const size_t nc = G.nc, nf = G.nf;
  rc = DBS_OK;
  h->phi = dmalloc(h, nc, rc); h->kinv = dmalloc(h, nc, rc);
  h->alpha = dmalloc(h, nc, rc); h->alpha_old = dmalloc(h, nc, rc);
  h->U = dmalloc(h, 3 * nc, rc); h->U2 = dmalloc(h, 3 * nc, rc);
  h->prgh = dmalloc(h, nc, rc); h->p = dmalloc(h, nc, rc);
  h->F = dmalloc(h, nf, rc);
  h->ml = dmalloc(h, nc, rc); h->mg = dmalloc(h, nc, rc); h->pc = dmalloc(h, nc, rc);
  h->cf = dmalloc(h, nc, rc);
  h->A = dmalloc(h, nf, rc); h->lam = dmalloc(h, nf, rc); h->rhoPhi = dmalloc(h, nf, rc);
  h->Qp = dmalloc(h, nc > 5 * (size_t)h->nblocks ? nc : 5 * (size_t)h->nblocks, rc);
  h->Qm = dmalloc(h, nc, rc); h->Pin = dmalloc(h, nc, rc); h->Pout = dmalloc(h, nc, rc);
  h->Rp = dmalloc(h, nc, rc); h->Rm = dmalloc(h, nc, rc);
  h->rAU = dmalloc(h, nc, rc); h->Sh = dmalloc(h, 3 * nc, rc); h->B = dmalloc(h, 3 * nc, rc);
  h->HbyA = dmalloc(h, 3 * nc, rc); h->phiH = dmalloc(h, nf, rc); h->rhs = dmalloc(h, nc, rc);
  h->r = dmalloc(h, nc, rc); h->z = dmalloc(h, nc, rc); h->pv = dmalloc(h, nc, rc);
  h->q = dmalloc(h, nc, rc);
  h->partials = dmalloc(h, 2 * (size_t)h->nblocks, rc);
  h->scal = dmalloc(h, 32, rc);
  if (!rc && hipHostMalloc((void **)&h->hscal, 32 * sizeof(double), hipHostMallocDefault) !=
                 hipSuccess)
    rc = DBS_ENOMEM;
  if (!rc) rc = pressure_setup(h);
  if (!rc) rc = hip_check(h, hipStreamSynchronize(h->stream), "create");
  if (rc) {
    dbs_destroy(H);
    return rc;
  }
  *out = H;
  return DBS_OK;
}

void dbs_destroy(dbs_handle *H) {
  if (!H) return;
  Handle *h = &H->h;
  if (h->stream) hipStreamSynchronize(h->stream);
  for (void *p : h->allocs) hipFree(p);
  if (h->hscal) hipHostFree(h->hscal);
  for (hipEvent_t e : h->tm.ev) hipEventDestroy(e);
  pressure_free(h);
  if (h->own_stream) hipStreamDestroy(h->own_stream);
  delete H;
}

const char *dbs_last_error(const dbs_handle *H) { return H ? H->h.err.c_str() : "null handle"; }

int dbs_set_stream(dbs_handle *H, void *stream) {
  if (!H) return DBS_EINVAL;
  Handle *h = &H->h;
  hipStreamSynchronize(h->stream);
  h->stream = stream ? (hipStream_t)stream : h->own_stream;
  return DBS_OK;
}

int dbs_set_static(dbs_handle *H, const double *phi, const double *kinv) {
  if (!H || !phi || !kinv) return DBS_EINVAL;
  Handle *h = &H->h;
  const size_t nc = h->G.nc;
  for (size_t i = 0; i < nc; i++) {
    if (!(phi[i] > 0.0 && phi[i] <= 1.0)) return fail(h, DBS_EINVAL, "porosity outside (0,1]");
    if (!(kinv[i] >= 0.0) || !isfinite(kinv[i])) return fail(h, DBS_EINVAL, "bad k^-1");
  }
  int rc = hip_check(h, hipMemcpyAsync(h->phi, phi, nc * 8, hipMemcpyHostToDevice, h->stream), "copy phi");
  if (!rc) rc = hip_check(h, hipMemcpyAsync(h->kinv, kinv, nc * 8, hipMemcpyHostToDevice, h->stream), "copy kinv");
  if (!rc) update_closures(h);
  if (!rc) rc = hip_check(h, hipStreamSynchronize(h->stream), "set_static");
  return rc;
}

static int set_state_impl(Handle *h, const double *alpha, const double *U, const double *prgh,
                          const double *F, hipMemcpyKind kind, hipStream_t s) {
  const size_t nc = h->G.nc, nf = h->G.nf;
  int rc = DBS_OK;
  if (alpha) rc = hip_check(h, hipMemcpyAsync(h->alpha, alpha, nc * 8, kind, s), "copy alpha");
  if (!rc && U) rc = hip_check(h, hipMemcpyAsync(h->U, U, 3 * nc * 8, kind, s), "copy U");
  if (!rc && prgh) rc = hip_check(h, hipMemcpyAsync(h->prgh, prgh, nc * 8, kind, s), "copy p_rgh");
  if (!rc && F) rc = hip_check(h, hipMemcpyAsync(h->F, F, nf * 8, kind, s), "copy F");
  if (!rc) rc = hip_check(h, hipStreamSynchronize(s), "set_state");
  if (rc) return rc;
  if (!F) init_flux(h);
  update_closures(h);
  return hip_check(h, hipStreamSynchronize(h->stream), "set_state");
}

int dbs_set_state(dbs_handle *H, const double *alpha, const double *U, const double *prgh,
                  const double *F) {
  if (!H || !alpha || !U || !prgh) return DBS_EINVAL;
  Handle *h = &H->h;
  const size_t nc = h->G.nc;
  if (!all_finite(alpha, nc) || !all_finite(U, 3 * nc) || !all_finite(prgh, nc) ||
      (F && !all_finite(F, h->G.nf)))
    return fail(h, DBS_EINVAL, "non-finite input state");
  return set_state_impl(h, alpha, U, prgh, F, hipMemcpyHostToDevice, h->stream);
}

int dbs_set_state_dev(dbs_handle *H, const double *alpha, const double *U, const double *prgh,
                      const double *F, void *stream) {
  if (!H || !alpha || !U || !prgh) return DBS_EINVAL;
  Handle *h = &H->h;
  hipStream_t s = stream ? (hipStream_t)stream : h->stream;
  hipStreamSynchronize(h->stream);
  return set_state_impl(h, alpha, U, prgh, F, hipMemcpyDeviceToDevice, s);
}

static int get_state_impl(Handle *h, double *alpha, double *U, double *prgh, double *p, double *F,
                          hipMemcpyKind kind, hipStream_t s) {
  const size_t nc = h->G.nc, nf = h->G.nf;
  int rc = hip_check(h, hipStreamSynchronize(h->stream), "get_state");
  if (!rc && alpha) rc = hip_check(h, hipMemcpyAsync(alpha, h->alpha, nc * 8, kind, s), "copy alpha");
  if (!rc && U) rc = hip_check(h, hipMemcpyAsync(U, h->U, 3 * nc * 8, kind, s), "copy U");
  if (!rc && prgh) rc = hip_check(h, hipMemcpyAsync(prgh, h->prgh, nc * 8, kind, s), "copy p_rgh");
  if (!rc && p) rc = hip_check(h, hipMemcpyAsync(p, h->p, nc * 8, kind, s), "copy p");
  if (!rc && F) rc = hip_check(h, hipMemcpyAsync(F, h->F, nf * 8, kind, s), "copy F");
  if (!rc) rc = hip_check(h, hipStreamSynchronize(s), "get_state");
  return rc;
}

int dbs_get_state(dbs_handle *H, double *alpha, double *U, double *prgh, double *p, double *F) {
  if (!H) return DBS_EINVAL;
  Handle *h = &H->h;
  return get_state_impl(h, alpha, U, prgh, p, F, hipMemcpyDeviceToHost, h->stream);
}

int dbs_get_state_dev(dbs_handle *H, double *alpha, double *U, double *prgh, double *p,
                      double *F, void *stream) {
  if (!H) return DBS_EINVAL;
  Handle *h = &H->h;
  hipStream_t s = stream ? (hipStream_t)stream : h->stream;
  return get_state_impl(h, alpha, U, prgh, p, F, hipMemcpyDeviceToDevice, s);
}

struct TraceOut {
  double *A, *rAU, *Shat, *Ustar, *HbyA, *phiHbyA, *b;
};

static int copy_out(Handle *h, double *dst, const double *src, size_t n) {
  if (!dst) return DBS_OK;
  return hip_check(h, hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToHost, h->stream), "trace");
}

static int one_step(Handle *h, TraceOut *tr) {
  int rc = DBS_OK;
  if (h->ctl.max_courant > 0.0) {
    double s[5];
    cell_stats(h, s);
    h->st.max_courant = s[3];
    if (s[3] > h->ctl.max_courant)
      return fail(h, DBS_ECOURANT, "Courant number " + std::to_string(s[3]) + " above limit");
  }
  alpha_stage(h);
  if (tr) rc |= copy_out(h, tr->A, h->A, h->G.nf);
  momentum_predictor(h);
  if (tr) {
    rc |= copy_out(h, tr->rAU, h->rAU, h->G.nc);
    rc |= copy_out(h, tr->Shat, h->Sh, 3 * (size_t)h->G.nc);
    rc |= copy_out(h, tr->Ustar, h->U, 3 * (size_t)h->G.nc);
  }
  int solve_rc = DBS_OK;
  for (int c = 0; c < h->ctl.n_corr; c++) {
    corrector_assemble(h);
    if (tr && c == 0) {
      rc |= copy_out(h, tr->HbyA, h->HbyA, 3 * (size_t)h->G.nc);
      rc |= copy_out(h, tr->phiHbyA, h->phiH, h->G.nf);
      rc |= copy_out(h, tr->b, h->rhs, h->G.nc);
    }
    int its = 0;
    double rr = 0.0;
    int src = pressure_solve(h, h->rAU, h->rhs, h->prgh, &its, &rr);
    h->st.p_iters[c] = its;
    h->st.p_relres[c] = rr;
    if (src) solve_rc = src;
    corrector_update(h, c == h->ctl.n_corr - 1);
  }
  h->st.steps++;
  if (rc) return fail(h, DBS_EHIP, "trace copy failed");
  if (solve_rc) return fail(h, solve_rc, "pressure solve did not converge");
  return DBS_OK;
}

static int finish_steps(Handle *h, int rc) {
  int e = hip_check(h, hipStreamSynchronize(h->stream), "step");
  if (!e) e = hip_check(h, hipGetLastError(), "kernel launch");
  if (e) return e;
  prof_collect(h);
  double s[5];
  cell_stats(h, s);
  h->st.alpha_min = s[0];
  h->st.alpha_max = s[1];
  h->st.phase_volume = s[2];
  if (s[4] > 0.0) return fail(h, DBS_ENAN, "non-finite value in the state");
  if (rc) return rc;
  if (h->ctl.bounds_tol > 0.0 &&
      (s[0] < -h->ctl.bounds_tol || s[1] > 1.0 + h->ctl.bounds_tol))
    return fail(h, DBS_EBOUNDS, "alpha outside the admissible band");
  return DBS_OK;
}

int dbs_step(dbs_handle *H, int nsteps) {
  if (!H || nsteps < 0) return DBS_EINVAL;
  Handle *h = &H->h;
  int rc = DBS_OK;
  for (int s = 0; s < nsteps && !rc; s++) rc = one_step(h, nullptr);
  if (rc == DBS_ECOURANT) return rc;
  return finish_steps(h, rc);
}

int dbs_debug_step_trace(dbs_handle *H, double *A, double *rAU, double *Shat, double *Ustar,
                         double *HbyA, double *phiHbyA, double *b) {
  if (!H) return DBS_EINVAL;
  Handle *h = &H->h;
  TraceOut tr{A, rAU, Shat, Ustar, HbyA, phiHbyA, b};
  int rc = one_step(h, &tr);
  if (rc == DBS_ECOURANT) return rc;
  return finish_steps(h, rc);
}

int dbs_get_stats(dbs_handle *H, dbs_stats *out) {
  if (!H || !out) return DBS_EINVAL;
  *out = H->h.st;
  return DBS_OK;
}

int dbs_set_profiling(dbs_handle *H, unsigned long long mask) {
  if (!H) return DBS_EINVAL;
  H->h.prof_mask = mask;
  return DBS_OK;
}

void dbs_reset_profiling(dbs_handle *H) {
  if (!H) return;
  for (int i = 0; i < KC_COUNT; i++) {
    H->h.k_launches[i] = 0;
    H->h.k_ms[i] = 0.0;
  }
}

int dbs_kernel_time(dbs_handle *H, int cls, long long *launches, double *ms) {
  if (!H || cls < 0 || cls >= KC_COUNT) return DBS_EINVAL;
  prof_collect(&H->h);
  if (launches) *launches = H->h.k_launches[cls];
  if (ms) *ms = H->h.k_ms[cls];
  return DBS_OK;
}

int dbs_debug_pressure_solve(dbs_handle *H, const double *rAU, const double *b, double *x,
                             int *iters, double *relres) {
  if (!H || !rAU || !b || !x) return DBS_EINVAL;
  Handle *h = &H->h;
  const size_t nc = h->G.nc;
  int rc = hip_check(h, hipMemcpyAsync(h->rAU, rAU, nc * 8, hipMemcpyHostToDevice, h->stream), "copy");
  if (!rc) rc = hip_check(h, hipMemcpyAsync(h->rhs, b, nc * 8, hipMemcpyHostToDevice, h->stream), "copy");
  if (!rc) rc = hip_check(h, hipMemcpyAsync(h->Rp, x, nc * 8, hipMemcpyHostToDevice, h->stream), "copy");
  if (rc) return rc;
  int src = pressure_solve(h, h->rAU, h->rhs, h->Rp, iters, relres);
  rc = hip_check(h, hipMemcpyAsync(x, h->Rp, nc * 8, hipMemcpyDeviceToHost, h->stream), "copy");
  if (!rc) rc = hip_check(h, hipStreamSynchronize(h->stream), "solve");
  if (!rc) rc = hip_check(h, hipGetLastError(), "kernel launch");
  prof_collect(h);
  if (rc) return rc;
  if (src) return fail(h, src, "pressure solve did not converge");
  return DBS_OK;
}

}  // extern "C"
