// C ABI of the DBS PISO step (declared in include/dbs.h): validation, device
// state, the step sequence of Sec. 3.2 over a batch of samples, state
// transfer, statistics, graph-captured steps, the autotuner and event
// timing.  No C++ exception leaves this file.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <mutex>
#include <new>
#include <string>

#include "dbs_internal.h"

using namespace dbs;

struct dbs_handle {
  Handle h;
};

static int hip_check(Handle *h, hipError_t e, const char *what);

namespace dbs {

static const char *kNames[KC_COUNT] = {
    "alpha_face", "alpha_bounds", "alpha_limit", "alpha_update", "mom_assemble",
    "mom_offdiag", "phihbya",     "correct",     "spmv",         "axpy",
    "dot",         "finalize",    "smooth_fine",  "restrict_fine",
    "prolong_fine", "smooth_coarse", "restrict_coarse", "prolong_coarse", "coarse_solve",
    "build_coarse", "stats",      "misc",        "smooth_fine_zero", "residual",
    "smooth_fine_dot", "curvature"};

void prof_begin(Handle *h, int cls) {
  Timer &t = h->tm;
  if (t.used + 2 > t.ev.size()) {
    // timing only: no system-scope fence (cache write-back) at the
    // records, which would add its own cost to every bracketed launch
    for (int i = 0; i < 256; i++) {
      hipEvent_t e;
      if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) break;
      t.ev.push_back(e);
    }
    t.cls.resize(t.ev.size() / 2 + 1);
  }
  // no events to be had: this launch goes untimed (profiling is
  // instrumentation only; the launch itself reports its own errors)
  t.skip = t.used + 2 > t.ev.size();
  if (t.skip) return;
  t.cls[t.used / 2] = cls;
  t.ok = t.ok && hipEventRecord(t.ev[t.used], h->stream) == hipSuccess;
}

void prof_end(Handle *h, int cls) {
  (void)cls;
  Timer &t = h->tm;
  if (t.skip) return;
  t.ok = t.ok && hipEventRecord(t.ev[t.used + 1], h->stream) == hipSuccess;
  t.used += 2;
}

// called after the stream has been synchronised and checked: add the timed
// launches to the per-class totals (none if an event failed)
void prof_collect(Handle *h) {
  Timer &t = h->tm;
  if (t.used == 0) return;
  for (size_t i = 0; i < t.used && t.ok; i += 2) {
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, t.ev[i], t.ev[i + 1]) != hipSuccess) continue;
    int c = t.cls[i / 2];
    h->k_launches[c]++;
    h->k_ms[c] += ms;
  }
  t.used = 0;
  t.ok = true;
}

// ------------------------------------------------------------- statistics

// Per block: min alpha, max alpha, sum phi alpha V, max Courant number,
// non-finite count and max |sum_out F| (the discrete divergence).  Slots
// combine by min, max, sum, max, sum, max.
__device__ __forceinline__ double stat_comb(int q, double a, double b) {
  return q == 0 ? fmin(a, b) : (q == 2 || q == 4) ? a + b : fmax(a, b);
}
__device__ __forceinline__ double stat_wave(int q, double v) {
  return q == 0 ? wave_min(v) : (q == 2 || q == 4) ? wave_sum(v) : wave_max(v);
}

__global__ void __launch_bounds__(NTHREADS) k_stats(Segs SG, const double *__restrict__ alpha,
                                                    const double *__restrict__ U,
                                                    const double *__restrict__ prgh,
                                                    const double *__restrict__ phi,
                                                    const double *__restrict__ F,
                                                    double *__restrict__ part, int nb) {
  __shared__ double lds[NSTAT][NTHREADS / 64];
  double r[NSTAT] = {1e300, -1e300, 0.0, 0.0, 0.0, 0.0};
  FOR_CELLS(SG, G, P) {
    const double a = alpha[P.c];
    r[0] = fmin(r[0], a);
    r[1] = fmax(r[1], a);
    r[2] += phi[P.c] * a * G.V;
    double out = 0.0, div = 0.0;
    for (int ax = 0; ax < 3; ax++) {
      const double fm = F[face_of(G, P, ax, 0)], fp = F[face_of(G, P, ax, 1)];
      out += fmax(fp, 0.0) + fmax(-fm, 0.0);
      div += fp - fm;
    }
    r[3] = fmax(r[3], G.dt * out / (phi[P.c] * G.V));
    bool ok = isfinite(a) && isfinite(prgh[P.c]);
    for (int d = 0; d < 3; d++) ok = ok && isfinite(U[(size_t)d * G.vs + P.c]);
    r[4] += ok ? 0.0 : 1.0;
    r[5] = fmax(r[5], fabs(div));
  }
  const int t = threadIdx.x + BX * threadIdx.y;
#pragma unroll
  for (int q = 0; q < NSTAT; q++) {
    const double v = stat_wave(q, r[q]);
    if ((t & 63) == 0) lds[q][t >> 6] = v;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int q = 0; q < NSTAT; q++) {
      double v = lds[q][0];
      for (int w = 1; w < NTHREADS / 64; w++) v = stat_comb(q, v, lds[q][w]);
      part[q * nb + cell_gb] = v;
    }
  }
}

// one block per sample: reduce the sample's block partials into `out`
// (host-mapped memory), NSTAT values per sample
__global__ void __launch_bounds__(1024) k_stats_final(const double *__restrict__ part, int nb,
                                                      const int *__restrict__ bp,
                                                      double *__restrict__ out) {
  __shared__ double lds[NSTAT][16];
  const int t = threadIdx.x, s = blockIdx.x;
  double r[NSTAT] = {1e300, -1e300, 0.0, 0.0, 0.0, 0.0};
  for (int i = bp[s] + t; i < bp[s + 1]; i += 1024)
#pragma unroll
    for (int q = 0; q < NSTAT; q++) r[q] = stat_comb(q, r[q], part[q * nb + i]);
#pragma unroll
  for (int q = 0; q < NSTAT; q++) {
    const double v = stat_wave(q, r[q]);
    if ((t & 63) == 0) lds[q][t >> 6] = v;
  }
  __syncthreads();
  if (t == 0) {
#pragma unroll
    for (int q = 0; q < NSTAT; q++) {
      double v = lds[q][0];
      for (int w = 1; w < 16; w++) v = stat_comb(q, v, lds[q][w]);
      out[s * NSTAT + q] = v;
    }
  }
}

// the boundary-value time of every sample moves by dt (kept on the device
// so that captured steps replay correctly)
__global__ void k_add_time(Geom *__restrict__ g, int ns, double dt) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < ns) g[s].t += dt;
}

// the time step of every sample (adaptive stepping)
__global__ void k_set_dt(Geom *__restrict__ g, int ns, double dt) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < ns) g[s].dt = dt;
}

// Wave inlet values of every row at each sample's time (linear wave on
// still water of depth d, surface d + A sin(w t)): below the surface
// alpha = 1, u = A w cosh(k y)/sinh(k d) sin(w t) into the domain and
// v = A w sinh(k y)/sinh(k d) cos(w t); above it air at rest.  One block per
// sample, threads over the rows of both x faces.
__global__ void k_wave_profile(const Geom *__restrict__ g) {
  const Geom &G = g[blockIdx.x];
  const int ny = G.n[1];
  for (int r = threadIdx.x; r < 2 * ny; r += blockDim.x) {
    const int b = r / ny, j = r % ny;
    if (G.bck[b] != BC_WAVE) continue;
    const double y = (j + 0.5) * G.h[1];
    const double A = G.wA[b], w = G.wom[b], k = G.wk[b], d = G.wd[b];
    const double st = sin(w * G.t), ct = cos(w * G.t);
    double u = 0.0, v = 0.0, a = 0.0;
    if (y < d + A * st) {
      const double amp = A * w / sinh(k * d);
      u = (b == 0 ? 1.0 : -1.0) * amp * cosh(k * y) * st;
      v = amp * sinh(k * y) * ct;
      a = 1.0;
    }
    double *o = G.wprof + ((size_t)b * ny + j) * 3;
    o[0] = u;
    o[1] = v;
    o[2] = a;
  }
}

void wave_profile(Handle *h) {
  if (!h->has_wave) return;
  DBS_LAUNCH(h, KC_MISC, k_wave_profile, dim3(h->ns), dim3(256), (const Geom *)h->dG);
}

void add_time(Handle *h, double dt) {
  DBS_LAUNCH(h, KC_MISC, k_add_time, dim3((h->ns + 255) / 256), dim3(256), h->dG, h->ns, dt);
  h->tnow += dt;
  wave_profile(h);
}

int cell_stats(Handle *h) {
  dim3 blk(BX, BY);
  const int nb = h->cell.nblk;
  DBS_LAUNCH(h, KC_STATS, k_stats, h->cgrid, blk, h->seg, (const double *)h->alpha,
             (const double *)h->U, (const double *)h->prgh, (const double *)h->phi,
             (const double *)h->F, h->partials, nb);
  DBS_LAUNCH(h, KC_STATS, k_stats_final, dim3(h->ns), dim3(1024), (const double *)h->partials,
             nb, (const int *)h->cell.bp, h->dsstat_h);
  return hip_check(h, hipStreamSynchronize(h->stream), "cell statistics");
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

static void *dmalloc_bytes(Handle *h, size_t bytes, int &rc) {
  void *p = nullptr;
  if (rc) return nullptr;
  if (hipMalloc(&p, bytes ? bytes : 8) != hipSuccess) {
    rc = DBS_ENOMEM;
    return nullptr;
  }
  if (hipMemset(p, 0, bytes ? bytes : 8) != hipSuccess) rc = DBS_EHIP;
  h->allocs.push_back(p);
  return p;
}

static double *dmalloc(Handle *h, size_t n, int &rc) {
  return (double *)dmalloc_bytes(h, n * sizeof(double), rc);
}

// pinned host memory that kernels write directly (mapped, coherent): small
// per-sample flags and records the host reads after an event or a sync
static void *hmap(Handle *h, size_t bytes, void **dev, int &rc) {
  void *p = nullptr;
  if (rc) return nullptr;
  if (hipHostMalloc(&p, bytes ? bytes : 8, hipHostMallocMapped | hipHostMallocCoherent) !=
      hipSuccess) {
    rc = DBS_ENOMEM;
    return nullptr;
  }
  memset(p, 0, bytes ? bytes : 8);
  h->hallocs.push_back(p);
  if (hipHostGetDevicePointer(dev, p, 0) != hipSuccess) rc = DBS_EHIP;
  return p;
}

static bool all_finite(const double *a, size_t n) {
  for (size_t i = 0; i < n; i++)
    if (!isfinite(a[i])) return false;
  return true;
}

static int validate_shared(const dbs_physics *p, const dbs_controls *c, std::string &msg) {
  if (!p || !c) { msg = "null argument"; return DBS_EINVAL; }
  if (p->kr_model != DBS_BROOKS_COREY && p->kr_model != DBS_VAN_GENUCHTEN) { msg = "kr_model"; return DBS_EINVAL; }
  if (p->pc_model != DBS_BROOKS_COREY && p->pc_model != DBS_VAN_GENUCHTEN) { msg = "pc_model"; return DBS_EINVAL; }
  if (!(p->kr_m > 0.0) || !(1.0 - p->s_girr - p->s_lirr > 0.0)) { msg = "kr parameters"; return DBS_EINVAL; }
  if (!(p->a_pcmax - p->a_pcirr > 0.0) || !(p->eps_pc > 0.0 && p->eps_pc < 0.5) || !(p->pc0 >= 0.0)) {
    msg = "pc parameters"; return DBS_EINVAL;
  }
  if (p->pc_model == DBS_VAN_GENUCHTEN && !(p->pc_exp > 0.0 && p->pc_exp < 1.0)) { msg = "VG m"; return DBS_EINVAL; }
  if (!(p->rho_l > 0.0 && p->rho_g > 0.0 && p->mu_l > 0.0 && p->mu_g > 0.0)) { msg = "fluid properties"; return DBS_EINVAL; }
  if (!(p->sigma >= 0.0 && p->sigma < HUGE_VAL)) { msg = "sigma"; return DBS_EINVAL; }
  if (!(p->contact_angle >= 0.0 && p->contact_angle < M_PI)) { msg = "contact_angle"; return DBS_EINVAL; }
  if (c->target_courant > 0.0 && !(c->dt_max > 0.0)) { msg = "dt_max"; return DBS_EINVAL; }
  if (!(c->dt > 0.0) || c->n_corr < 1 || c->n_corr > 16 || c->mom_maxit < 0 ||
      !(c->mom_tol >= 0.0) || c->n_alpha_sub < 1 || c->n_alpha_sub > 64 ||
      c->mules_iter < 1 || !(c->p_tol > 0.0) || c->p_maxit < 1 ||
      (c->precision != DBS_FP64 && c->precision != DBS_MIXED) || c->mg_pre < 0 || c->mg_post < 0) {
    msg = "bad controls";
    return DBS_EINVAL;
  }
  return DBS_OK;
}

static int validate_sample(const dbs_grid *g, const dbs_bc *bc, std::string &msg) {
  if (!g || !bc) { msg = "null argument"; return DBS_EINVAL; }
  const int n[3] = {g->nx, g->ny, g->nz};
  const double hh[3] = {g->dx, g->dy, g->dz};
  for (int a = 0; a < 3; a++) {
    if (n[a] < 1 || !(hh[a] > 0.0) || !isfinite(hh[a])) { msg = "bad grid"; return DBS_EINVAL; }
    const bool e0 = bc[2 * a].kind == DBS_BC_EMPTY, e1 = bc[2 * a + 1].kind == DBS_BC_EMPTY;
    if (e0 != e1 || (e0 && n[a] != 1)) {
      msg = "EMPTY faces must pair on an axis of one cell";
      return DBS_EINVAL;
    }
  }
  if ((long long)n[0] * n[1] * n[2] * 4 > 2000000000LL) { msg = "mesh too large"; return DBS_EINVAL; }
  for (int b = 0; b < 6; b++) {
    if (bc[b].kind < DBS_BC_WALL || bc[b].kind > DBS_BC_WAVE) { msg = "bad bc kind"; return DBS_EINVAL; }
    if (bc[b].kind == DBS_BC_WAVE &&
        (b > 1 || !(bc[b].wave[1] > 0.0) || !(bc[b].wave[2] > 0.0) || !isfinite(bc[b].wave[0]))) {
      msg = "a wave inlet needs an x face, a positive period and a positive depth";
      return DBS_EINVAL;
    }
  }
  return DBS_OK;
}

// wavenumber of a linear wave of angular frequency w on depth d: Newton on
// f(k) = g k tanh(k d) - w^2 from the deep-water value
static double wavenumber(double w, double gm, double d) {
  double k = w * w / gm;
  for (int it = 0; it < 100; it++) {
    const double th = tanh(k * d);
    const double f = gm * k * th - w * w;
    const double df = gm * (th + k * d * (1.0 - th * th));
    const double dk = f / df;
    k -= dk;
    if (fabs(dk) <= 1e-15 * k) break;
  }
  return k;
}

static Geom make_geom(const dbs_grid *grid, const dbs_bc *bc, double dt, const double g[3]) {
  Geom G;
  memset(&G, 0, sizeof(G));
  G.n[0] = grid->nx; G.n[1] = grid->ny; G.n[2] = grid->nz;
  G.h[0] = grid->dx; G.h[1] = grid->dy; G.h[2] = grid->dz;
  G.nc = G.n[0] * G.n[1] * G.n[2];
  const int nfx = (G.n[0] + 1) * G.n[1] * G.n[2];
  const int nfy = G.n[0] * (G.n[1] + 1) * G.n[2];
  const int nfz = G.n[0] * G.n[1] * (G.n[2] + 1);
  G.fo[0] = 0;
  G.fo[1] = nfx;
  G.fo[2] = nfx + nfy;
  G.nf = nfx + nfy + nfz;
  G.V = G.h[0] * G.h[1] * G.h[2];
  G.iV = 1.0 / G.V;
  for (int a = 0; a < 3; a++) {
    G.ih[a] = 1.0 / G.h[a];
    G.area[a] = G.V / G.h[a];
  }
  G.dt = dt;
  G.has_outlet = 0;
  for (int b = 0; b < 6; b++) {
    G.bck[b] = bc[b].kind;
    for (int a = 0; a < 3; a++) G.bcU[b][a] = bc[b].U[a];
    G.bca[b] = bc[b].alpha;
    G.bcp[b] = bc[b].p;
    if (bc[b].kind == DBS_BC_OUTLET) G.has_outlet = 1;
  }
  G.dN = 1e-8 / cbrt(G.V);
  const double gm = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
  for (int b = 0; b < 2; b++) {
    if (bc[b].kind != DBS_BC_WAVE) continue;
    G.wA[b] = bc[b].wave[0];
    G.wom[b] = 2.0 * M_PI / bc[b].wave[1];
    G.wd[b] = bc[b].wave[2];
    G.wk[b] = gm > 0.0 ? wavenumber(G.wom[b], gm, G.wd[b]) : 0.0;
  }
  G.t = 0.0;
  return G;
}

static Phys make_phys(const dbs_physics *phys) {
  Phys P;
  memset(&P, 0, sizeof(P));
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
  P.sigma = phys->sigma;
  P.ca_on = phys->contact_angle > 0.0 ? 1 : 0;
  P.cos_ca = cos(phys->contact_angle);
  P.cot_ca = P.ca_on ? cos(phys->contact_angle) / sin(phys->contact_angle) : 0.0;
  return P;
}

static void clear_graphs(Handle *h) {
  for (auto &kv : h->graphs) {
    if (kv.second.front) (void)hipGraphExecDestroy(kv.second.front);
    if (kv.second.back) (void)hipGraphExecDestroy(kv.second.back);
  }
  h->graphs.clear();
}

extern "C" void dbs_destroy(dbs_handle *H);

static int create_impl(int n, const dbs_grid *grids, const dbs_physics *phys, const dbs_bc *bcs,
                       const dbs_controls *ctl, dbs_handle **out) {
  if (!out) return DBS_EINVAL;
  *out = nullptr;
  if (n < 1 || !grids || !bcs) return DBS_EINVAL;
  std::string msg;
  int rc = validate_shared(phys, ctl, msg);
  for (int s = 0; s < n && !rc; s++) rc = validate_sample(&grids[s], &bcs[6 * s], msg);
  if (rc) return rc;
  dbs_handle *H = new (std::nothrow) dbs_handle();
  if (!H) return DBS_ENOMEM;
  Handle *h = &H->h;
  h->ns = n;
  h->hG.resize(n);
  h->hrng.resize(n);
  h->st.assign(n, dbs_stats());
  for (auto &s : h->st) memset(&s, 0, sizeof(s));
  // arenas: cells padded per sample to whole vector-kernel blocks
  long long c0 = 0, f0 = 0;
  for (int s = 0; s < n; s++) {
    Geom G = make_geom(&grids[s], &bcs[6 * s], ctl->dt, phys->g);
    G.c0 = (int)c0;
    for (int a = 0; a < 3; a++) G.fo[a] += (int)f0;
    h->hrng[s] = Rng{(int)c0, G.nc, G.has_outlet ? 0 : 1, 0};
    c0 += ((long long)G.nc + FLAT_CELLS - 1) / FLAT_CELLS * FLAT_CELLS;
    f0 += G.nf;
    h->hG[s] = G;
  }
  h->NC = c0;
  h->NF = f0;
  if (3 * h->NC > 2000000000LL || h->NF > 2000000000LL) {
    delete H;
    return DBS_EINVAL;  // 32-bit cell and face indices
  }
  for (int s = 0; s < n; s++) h->hG[s].vs = (int)h->NC;
  h->P = make_phys(phys);
  h->ctl = *ctl;
  h->mg_pre = ctl->mg_pre > 0 ? ctl->mg_pre : 2;
  h->mg_post = ctl->mg_post > 0 ? ctl->mg_post : 2;
  if ((rc = hip_check(h, hipStreamCreate(&h->own_stream), "hipStreamCreate"))) {
    delete H;
    return rc;
  }
  h->stream = h->own_stream;
  if ((rc = hip_check(h, hipEventCreateWithFlags(&h->flag_ev, hipEventDisableTiming),
                      "hipEventCreateWithFlags"))) {
    (void)hipStreamDestroy(h->own_stream);
    delete H;
    return rc;
  }
  const size_t NC = (size_t)h->NC, NF = (size_t)h->NF;
  rc = DBS_OK;
  // per-cell launch shape and flat vector shape
  h->cell.hbp.assign(n + 1, 0);
  h->flat.hbp.assign(n + 1, 0);
  for (int s = 0; s < n; s++) {
    h->cell.hbp[s + 1] = h->cell.hbp[s] + cell_blocks(h->hG[s]);
    h->flat.hbp[s] = h->hG[s].c0 / FLAT_CELLS;
  }
  h->flat.hbp[n] = (int)(NC / FLAT_CELLS);
  h->cell.nblk = h->cell.hbp[n];
  h->flat.nblk = h->flat.hbp[n];
  // wave inlet tables: 2 faces x ny rows x (u, v, alpha) per sample
  {
    size_t np = 0;
    for (int s = 0; s < n; s++) {
      np += 6 * (size_t)h->hG[s].n[1];
      if (h->hG[s].bck[0] == BC_WAVE || h->hG[s].bck[1] == BC_WAVE) h->has_wave = 1;
    }
    double *wp = dmalloc(h, np, rc);
    size_t off = 0;
    for (int s = 0; s < n && wp; s++) {
      h->hG[s].wprof = wp + off;
      off += 6 * (size_t)h->hG[s].n[1];
    }
  }
  h->cell.bp = (int *)dmalloc_bytes(h, sizeof(int) * (n + 1), rc);
  h->flat.bp = (int *)dmalloc_bytes(h, sizeof(int) * (n + 1), rc);
  h->dG = (Geom *)dmalloc_bytes(h, sizeof(Geom) * n, rc);
  h->rng = (Rng *)dmalloc_bytes(h, sizeof(Rng) * n, rc);
  if (!rc) {
    int e = 0;
    e |= hip_check(h, hipMemcpy(h->cell.bp, h->cell.hbp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice), "upload");
    e |= hip_check(h, hipMemcpy(h->flat.bp, h->flat.hbp.data(), sizeof(int) * (n + 1), hipMemcpyHostToDevice), "upload");
    e |= hip_check(h, hipMemcpy(h->dG, h->hG.data(), sizeof(Geom) * n, hipMemcpyHostToDevice), "upload");
    e |= hip_check(h, hipMemcpy(h->rng, h->hrng.data(), sizeof(Rng) * n, hipMemcpyHostToDevice), "upload");
    if (e) rc = DBS_EHIP;
  }
  h->seg = Segs{h->dG, h->cell.bp, n};
  h->cgrid = dim3(h->cell.nblk);
  h->phi = dmalloc(h, NC, rc); h->kinv = dmalloc(h, NC, rc);
  h->alpha = dmalloc(h, NC, rc); h->alpha_old = dmalloc(h, NC, rc);
  if (ctl->n_alpha_sub > 1) h->alpha3 = dmalloc(h, NC, rc);
  h->U = dmalloc(h, 3 * NC, rc); h->U2 = dmalloc(h, 3 * NC, rc); h->U3 = dmalloc(h, 3 * NC, rc);
  h->prgh = dmalloc(h, NC, rc); h->p = dmalloc(h, NC, rc);
  h->pprev = dmalloc(h, NC, rc); h->pprev2 = dmalloc(h, NC, rc); h->pprev3 = dmalloc(h, NC, rc);
  h->pprev4 = dmalloc(h, NC, rc);
  h->gord = (int *)dmalloc_bytes(h, sizeof(int) * n, rc);
  if (ctl->n_corr > 1) {
    h->p1 = dmalloc(h, NC, rc);
    h->dcorr = dmalloc(h, (size_t)3 * (ctl->n_corr - 1) * NC, rc);
    h->gchg = (int *)dmalloc_bytes(h, sizeof(int) * n * (ctl->n_corr - 1), rc);
  }
  h->F = dmalloc(h, NF, rc); h->F2 = dmalloc(h, NF, rc);
  h->ml = dmalloc(h, NC, rc); h->mg = dmalloc(h, NC, rc); h->pc = dmalloc(h, NC, rc);
  h->cf = dmalloc(h, NC, rc);
  h->A = dmalloc(h, NF, rc); h->lam = dmalloc(h, NF, rc); h->rhoPhi = dmalloc(h, NF, rc);
  h->Qp = dmalloc(h, NC, rc); h->Qm = dmalloc(h, NC, rc); h->Pin = dmalloc(h, NC, rc);
  h->Pout = dmalloc(h, NC, rc); h->Rp = dmalloc(h, NC, rc); h->Rm = dmalloc(h, NC, rc);
  h->rAU = dmalloc(h, NC, rc); h->Sh = dmalloc(h, 3 * NC, rc); h->B = dmalloc(h, 3 * NC, rc);
  h->AN = dmalloc(h, 6 * NC, rc); h->FB = dmalloc(h, NF, rc);
  if (h->P.sigma != 0.0) h->SK = dmalloc(h, NC, rc);
  h->HbyA = dmalloc(h, 3 * NC, rc); h->phiH = dmalloc(h, NF, rc); h->rhs = dmalloc(h, NC, rc);
  h->r = dmalloc(h, NC, rc); h->z = dmalloc(h, NC, rc); h->pv = dmalloc(h, NC, rc);
  h->q = dmalloc(h, NC, rc); h->pv2 = dmalloc(h, NC, rc);
  h->scal = dmalloc(h, (size_t)NSC * n, rc);
  h->msc = dmalloc(h, (size_t)NMSC * n, rc);
  h->mact = (int *)dmalloc_bytes(h, sizeof(int) * n, rc);
  h->hscal = (double *)hmap(h, sizeof(double) * NSC * n, (void **)&h->dscal_h, rc);
  h->hpub = (int *)hmap(h, sizeof(int) * 2 * n, (void **)&h->dpub, rc);
  h->hmsc = (double *)hmap(h, sizeof(double) * NMSC * n, (void **)&h->dmsc, rc);
  h->hmflag = (int *)hmap(h, sizeof(int) * 2 * n, (void **)&h->dmflag, rc);
  h->hsstat = (double *)hmap(h, sizeof(double) * NSTAT * n, (void **)&h->dsstat_h, rc);
  h->hrec = (double *)hmap(h, sizeof(double) * 16 * NREC * n, (void **)&h->rec, rc);
  for (int e = 0; e < 2 && !rc; e++)
    rc = hip_check(h, hipEventCreateWithFlags(&h->mom_ev[e], hipEventDisableTiming), "event");
  if (!rc) rc = pressure_setup(h);
  if (!rc) rc = hip_check(h, hipDeviceSynchronize(), "create");
  if (rc) {
    dbs_destroy(H);
    return rc;
  }
  *out = H;
  return DBS_OK;
}

// ---------------------------------------------------------- sample access

static int check_sample(Handle *h, int i) {
  if (i < 0 || i >= h->ns) return fail(h, DBS_EINVAL, "sample index out of range");
  return DBS_OK;
}

static int set_static_impl(Handle *h, int i, const double *phi, const double *kinv) {
  if (int rc = check_sample(h, i)) return rc;
  const Geom &G = h->hG[i];
  const size_t nc = G.nc;
  for (size_t c = 0; c < nc; c++) {
    if (!(phi[c] > 0.0 && phi[c] <= 1.0)) return fail(h, DBS_EINVAL, "porosity outside (0,1]");
    if (!(kinv[c] >= 0.0) || !isfinite(kinv[c])) return fail(h, DBS_EINVAL, "bad k^-1");
    // a solid-free cell (phi = 1) has no Darcy drag: k^-1 > 0 there contradicts
    // the porosity field (Sec. 2.2: k tends to infinity as phi tends to 1)
    if (phi[c] == 1.0 && kinv[c] > 0.0)
      return fail(h, DBS_EINVAL, "phi = 1 (solid-free) with k^-1 > 0");
  }
  int rc = hip_check(h, hipMemcpyAsync(h->phi + G.c0, phi, nc * 8, hipMemcpyHostToDevice, h->stream), "copy phi");
  if (!rc) rc = hip_check(h, hipMemcpyAsync(h->kinv + G.c0, kinv, nc * 8, hipMemcpyHostToDevice, h->stream), "copy kinv");
  if (!rc) update_closures(h, i);
  if (!rc) rc = hip_check(h, hipStreamSynchronize(h->stream), "set_static");
  return rc;
}

static int set_state_impl(Handle *h, int i, const double *alpha, const double *U,
                          const double *prgh, const double *F, hipMemcpyKind kind,
                          hipStream_t s) {
  const Geom &G = h->hG[i];
  const size_t nc = G.nc, nf = G.nf;
  int rc = DBS_OK;
  if (alpha) rc = hip_check(h, hipMemcpyAsync(h->alpha + G.c0, alpha, nc * 8, kind, s), "copy alpha");
  for (int d = 0; d < 3 && !rc && U; d++)
    rc = hip_check(h, hipMemcpyAsync(h->U + (size_t)d * h->NC + G.c0, U + d * nc, nc * 8, kind, s), "copy U");
  if (!rc && prgh) rc = hip_check(h, hipMemcpyAsync(h->prgh + G.c0, prgh, nc * 8, kind, s), "copy p_rgh");
  if (!rc && F) rc = hip_check(h, hipMemcpyAsync(h->F + G.fo[0], F, nf * 8, kind, s), "copy F");
  if (!rc) rc = hip_check(h, hipStreamSynchronize(s), "set_state");
  if (rc) return rc;
  if (!F) {
    wave_profile(h);
    init_flux(h, i);
  }
  update_closures(h, i);
  h->hist = 0;  // no previous step for the extrapolated guess
  return hip_check(h, hipStreamSynchronize(h->stream), "set_state");
}

static int get_state_impl(Handle *h, int i, double *alpha, double *U, double *prgh, double *p,
                          double *F, hipMemcpyKind kind, hipStream_t s) {
  const Geom &G = h->hG[i];
  const size_t nc = G.nc, nf = G.nf;
  int rc = hip_check(h, hipStreamSynchronize(h->stream), "get_state");
  if (!rc && alpha) rc = hip_check(h, hipMemcpyAsync(alpha, h->alpha + G.c0, nc * 8, kind, s), "copy alpha");
  for (int d = 0; d < 3 && !rc && U; d++)
    rc = hip_check(h, hipMemcpyAsync(U + d * nc, h->U + (size_t)d * h->NC + G.c0, nc * 8, kind, s), "copy U");
  if (!rc && prgh) rc = hip_check(h, hipMemcpyAsync(prgh, h->prgh + G.c0, nc * 8, kind, s), "copy p_rgh");
  if (!rc && p) rc = hip_check(h, hipMemcpyAsync(p, h->p + G.c0, nc * 8, kind, s), "copy p");
  if (!rc && F) rc = hip_check(h, hipMemcpyAsync(F, h->F + G.fo[0], nf * 8, kind, s), "copy F");
  if (!rc) rc = hip_check(h, hipStreamSynchronize(s), "get_state");
  return rc;
}

// ----------------------------------------------------------------- stepping

struct TraceOut {
  double *A, *rAU, *Shat, *Ustar, *HbyA, *phiHbyA, *b, *Rp, *Rm, *alphaPhi;
};

static int copy_out(Handle *h, double *dst, const double *src, size_t n) {
  if (!dst) return DBS_OK;
  return hip_check(h, hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToHost, h->stream), "trace");
}

// copy the 3 components of a vector field of sample 0 (arena stride NC)
static int copy_out3(Handle *h, double *dst, const double *src) {
  if (!dst) return DBS_OK;
  const Geom &G = h->hG[0];
  int rc = DBS_OK;
  for (int d = 0; d < 3; d++)
    rc |= copy_out(h, dst + (size_t)d * G.nc, src + (size_t)d * h->NC + G.c0, G.nc);
  return rc;
}

// CFL-adaptive time step: dt <- min(dt_max, 1.2 dt, target dt / Co) from
// the Courant numbers of the current fluxes (one dt for the whole batch)
static int adapt_dt(Handle *h) {
  if (!(h->ctl.target_courant > 0.0)) return DBS_OK;
  const int e = cell_stats(h);
  if (e) return e;
  double co = 0.0;
  for (int s = 0; s < h->ns; s++) co = std::max(co, h->hsstat[NSTAT * s + 3]);
  double dt = std::min(h->ctl.dt_max, 1.2 * h->ctl.dt);
  if (co > 0.0) dt = std::min(dt, h->ctl.target_courant * h->ctl.dt / co);
  h->ctl.dt = dt;
  for (int s = 0; s < h->ns; s++) h->hG[s].dt = dt;
  DBS_LAUNCH(h, KC_MISC, k_set_dt, dim3((h->ns + 255) / 256), dim3(256), h->dG, h->ns, dt);
  return DBS_OK;
}

static int courant_check(Handle *h) {
  if (!(h->ctl.max_courant > 0.0)) return DBS_OK;
  const int e = cell_stats(h);
  if (e) return e;
  for (int s = 0; s < h->ns; s++) {
    const double co = h->hsstat[NSTAT * s + 3];
    h->st[s].max_courant = co;
    if (co > h->ctl.max_courant)
      return fail(h, DBS_ECOURANT, "Courant number " + std::to_string(co) +
                                       " above limit (sample " + std::to_string(s) + ")");
  }
  return DBS_OK;
}

// The step body.  budget > 0: the predictor runs h->mom_budget sweeps and
// every pressure solve the per-corrector iteration budget, with no host
// synchronisation (graph capture); per-sample results go to h->rec and the
// host-mapped predictor records.  Else results go to the statistics, the
// largest iteration count per corrector to its_out and the largest
// predictor sweep count to *sweeps_out.
// The step body runs in two parts (graph mode captures each on its own):
// the saturation stage and the predictor, then the correctors.
static int step_front(Handle *h, TraceOut *tr, int budget) {
  int rc = DBS_OK;
  add_time(h, h->ctl.dt);  // boundary values of this step are taken at its end
  // the trace's limited flux borrows phiH, which the correctors fill later
  alpha_stage(h, tr && tr->alphaPhi ? h->phiH : nullptr);
  if (tr) {
    rc |= copy_out(h, tr->A, h->A, h->hG[0].nf);
    double *Rp, *Rm;
    alpha_final_R(h, &Rp, &Rm);
    rc |= copy_out(h, tr->Rp, Rp, h->hG[0].nc);
    rc |= copy_out(h, tr->Rm, Rm, h->hG[0].nc);
    rc |= copy_out(h, tr->alphaPhi, h->phiH, h->hG[0].nf);
  }
  momentum_predictor(h, budget > 0 ? h->mom_budget : 0);
  if (tr) {
    rc |= copy_out(h, tr->rAU, h->rAU, h->hG[0].nc);
    rc |= copy_out3(h, tr->Shat, h->Sh);
    rc |= copy_out3(h, tr->Ustar, h->U);
  }
  return rc;
}

// ---------------------------------------------------- pressure initial guesses
//
// The first corrector's solve starts from p_rgh at the end of the coming
// step extrapolated in time from the ends of the previous steps, less the
// changes the later correctors' solves are predicted to make; each later
// corrector's solve starts from the previous corrector's solution plus its
// predicted change.  Every prediction is chosen per sample from how it would
// have fared one step back: the extrapolation order of p_rgh (0: p_rgh^n
// itself, 1 to 3: linear to cubic) whose prediction of p_rgh^n from the
// steps before came closest in the L2 norm, and for each later corrector
// the prediction of its change (0: none, 1: the previous step's change, 2
// and 3: the last two or three changes extrapolated linearly or
// quadratically) that came closest to this step's change.  (At 256^3, mixed, steps 13 to 22 from rest, the quadratic
// order and the linear change win; in the wave flume p_rgh and the changes
// alternate from step to step, so order 0 and no change win there.)

// one block per sample: the NQ block partials of the sample summed in a
// fixed order; the sums are valid in thread 0
template <int NQ>
__device__ __forceinline__ void sample_sums(const double *__restrict__ part, int nb,
                                            const int *__restrict__ bp, double *r) {
  __shared__ double lds[NQ][16];
  const int t = threadIdx.x, s = blockIdx.x;
  for (int q = 0; q < NQ; q++) r[q] = 0.0;
  strided_sums<NQ>(part, (size_t)nb, bp[s], bp[s + 1], r);
  for (int q = 0; q < NQ; q++) {
    const double v = wave_sum(r[q]);
    if ((t & 63) == 0) lds[q][t >> 6] = v;
  }
  __syncthreads();
  if (t == 0)
    for (int q = 0; q < NQ; q++) {
      double v = lds[q][0];
      for (int w = 1; w < 16; w++) v += lds[q][w];
      r[q] = v;
    }
}

// NQ per-thread values summed over the block into part[q * nb + block]
template <int NQ>
__device__ __forceinline__ void block_partials(const double *v, int gb, double *part, int nb) {
  __shared__ double lds[NQ][NTHREADS / 64];
  const int t = threadIdx.x + BX * threadIdx.y;
  for (int q = 0; q < NQ; q++) {
    const double w = wave_sum(v[q]);
    if ((t & 63) == 0) lds[q][t >> 6] = w;
  }
  __syncthreads();
  if (t == 0)
    for (int q = 0; q < NQ; q++) {
      double w = lds[q][0];
      for (int k = 1; k < NTHREADS / 64; k++) w += lds[q][k];
      part[(size_t)q * nb + gb] = w;
    }
}

// predicted change of a later corrector's solve, kind 1 to 3, from its last
// three changes d, d1, d2 (A: this step's coefficients, linear r and
// quadratic q1, q2 as for p_rgh)
__device__ __forceinline__ double predicted_change(int kind, double d, double d1, double d2,
                                                   const GuessArgs &A) {
  if (kind == 3) return fma(A.q2, d - d2, fma(A.q1, d - d1, d));
  return kind == 2 ? fma(A.r, d - d1, d) : d;
}

// The first corrector's guess in p (p_rgh^n on entry) with the sample's
// order ord[s] (at most A.use) less the later correctors' predicted changes
// (kind chg[s * nd + k] at most A.usec; slices k, k + nd and k + 2 nd of d
// hold the last three changes); the squared errors of the backtests as
// block partials; the history shifts (pr <- pq <- pb <- pa <- p_rgh^n).
__global__ void __launch_bounds__(NTHREADS) k_extrap(Segs SG, double *__restrict__ p,
                                                     double *__restrict__ pa,
                                                     double *__restrict__ pb,
                                                     double *__restrict__ pq,
                                                     double *__restrict__ pr,
                                                     const double *__restrict__ d, size_t nc,
                                                     const int *__restrict__ ord,
                                                     const int *__restrict__ chg, GuessArgs A,
                                                     double *__restrict__ part, int nb) {
  double e[4] = {0.0, 0.0, 0.0, 0.0};
  FOR_CELLS(SG, G, P) {
    const size_t c = P.c;
    const double t = p[c], a = pa[c], b = pb[c], q = pq[c];
    const int o = min(ord[cell_sg], A.use);
    double g = t;
    if (o == 1) g = fma(A.r, t - a, t);
    else if (o == 2) g = fma(A.q2, t - b, fma(A.q1, t - a, t));
    else if (o == 3) g = fma(A.k3, t - q, fma(A.k2, t - b, fma(A.k1, t - a, t)));
    for (int k = 0; k < A.nd; k++) {
      const int kind = min(chg[cell_sg * A.nd + k], A.usec);
      if (kind >= 1)
        g -= predicted_change(kind, d[(size_t)k * nc + c],
                              kind >= 2 ? d[(size_t)(k + A.nd) * nc + c] : 0.0,
                              kind == 3 ? d[(size_t)(k + 2 * A.nd) * nc + c] : 0.0, A);
    }
    if (A.nbt >= 1) e[0] = (t - a) * (t - a);
    if (A.nbt >= 2) {
      const double x = t - fma(A.b1, a - b, a);
      e[1] = x * x;
    }
    if (A.nbt >= 3) {
      const double x = t - fma(A.c2, a - q, fma(A.c1, a - b, a));
      e[2] = x * x;
    }
    if (A.nbt >= 4) {
      const double x = t - fma(A.m3, a - pr[c], fma(A.m2, a - q, fma(A.m1, a - b, a)));
      e[3] = x * x;
    }
    p[c] = g;
    pr[c] = q;
    pq[c] = b;
    pb[c] = a;
    pa[c] = t;
  }
  block_partials<4>(e, cell_gb, part, nb);
}

// one block per sample: the order of the next step's guess, the one whose
// backtest erred least (linear while fewer than two backtests exist)
__global__ void __launch_bounds__(1024) k_extrap_final(const double *__restrict__ part, int nb,
                                                       const int *__restrict__ bp, int nbt,
                                                       int *__restrict__ ord) {
  double r[4];
  sample_sums<4>(part, nb, bp, r);
  if (threadIdx.x != 0) return;
  int o = 1;
  if (nbt >= 2) {
    o = 0;
    for (int k = 1; k < nbt && k < 4; k++)
      if (r[k] < r[o]) o = k;
  }
  ord[blockIdx.x] = o;
}

// A later corrector's guess: the previous corrector's solution (kept in
// p1) plus the change predicted with the sample's kind (at most A.usec)
// from its last three changes d, d1, d2.
__global__ void __launch_bounds__(NTHREADS) k_corr_guess(Segs SG, double *__restrict__ p,
                                                         double *__restrict__ p1,
                                                         const double *__restrict__ d,
                                                         const double *__restrict__ d1,
                                                         const double *__restrict__ d2,
                                                         const int *__restrict__ chg, int nd,
                                                         int k, GuessArgs A) {
  FOR_CELLS(SG, G, P) {
    const size_t c = P.c;
    const double t = p[c];
    p1[c] = t;
    const int kind = min(chg[cell_sg * nd + k], A.usec);
    if (kind >= 1)
      p[c] = t + predicted_change(kind, d[c], kind >= 2 ? d1[c] : 0.0, kind == 3 ? d2[c] : 0.0,
                                  A);
  }
}

// The change of this step's solve x = p - p1; as block partials the squared
// errors of its predictions from the stored changes (kind 0, none; kind k
// >= 1 with A.usec >= k, i.e. once k steps are stored); the changes shift
// (d2 <- d1 <- d <- x).
__global__ void __launch_bounds__(NTHREADS) k_corr_record(Segs SG, const double *__restrict__ p,
                                                          const double *__restrict__ p1,
                                                          double *__restrict__ d,
                                                          double *__restrict__ d1,
                                                          double *__restrict__ d2, GuessArgs A,
                                                          double *__restrict__ part, int nb) {
  double e[4] = {0.0, 0.0, 0.0, 0.0};
  FOR_CELLS(SG, G, P) {
    const size_t c = P.c;
    const double x = p[c] - p1[c];
    e[0] = x * x;
    if (A.usec >= 1) {
      const double v0 = d[c];
      const double v1 = A.usec >= 2 ? d1[c] : 0.0;
      const double v2 = A.usec >= 3 ? d2[c] : 0.0;
      for (int kind = 1; kind <= A.usec; kind++) {
        const double y = x - predicted_change(kind, v0, v1, v2, A);
        e[kind] = y * y;
      }
      if (A.usec >= 2) d2[c] = v1;
      d1[c] = v0;
    }
    d[c] = x;
  }
  block_partials<4>(e, cell_gb, part, nb);
}

// one block per sample: the kind of the next step's change prediction, the
// one whose backtest erred least among the usec + 1 told (the last change
// while none can be told)
__global__ void __launch_bounds__(1024) k_record_final(const double *__restrict__ part, int nb,
                                                       const int *__restrict__ bp, int usec,
                                                       int *__restrict__ chg, int nd, int k) {
  double r[4];
  sample_sums<4>(part, nb, bp, r);
  if (threadIdx.x != 0) return;
  int o = 1;
  if (usec >= 1) {
    o = 0;
    for (int q = 1; q <= usec && q < 4; q++)
      if (r[q] < r[o]) o = q;
  }
  chg[blockIdx.x * nd + k] = o;
}

// Lagrange extrapolation to offset tau past node 0 from nodes 0, -h[0],
// -(h[0] + h[1]), ... (m nodes before node 0), in the difference form
// x0 + sum_k c[k - 1] (x0 - x_k): c[k - 1] = -w_k, with w_k the Lagrange
// weight of node k (the weights sum to 1).
static void lag_coef(double tau, const double *h, int m, double *c) {
  double x[4] = {0.0, 0.0, 0.0, 0.0};
  for (int k = 1; k <= m; k++) x[k] = x[k - 1] - h[k - 1];
  for (int k = 1; k <= m; k++) {
    double w = 1.0;
    for (int j = 0; j <= m; j++)
      if (j != k) w *= (tau - x[j]) / (x[k] - x[j]);
    c[k - 1] = -w;
  }
}

// the coming step's GuessArgs from the stored steps and their time steps
static GuessArgs guess_args(const Handle *h) {
  GuessArgs A{};
  const double tau = h->ctl.dt;
  const double hs[4] = {h->dt_prev, h->dt_prev2, h->dt_prev3, h->dt_prev4};
  A.use = std::min(h->hist, 3);
  A.usec = std::min(h->hist, 3);
  A.nbt = std::min(h->hist, 4);
  A.nd = h->hist >= 1 ? h->ctl.n_corr - 1 : 0;
  double c[3];
  if (A.use >= 1) { lag_coef(tau, hs, 1, c); A.r = c[0]; }
  if (A.use >= 2) { lag_coef(tau, hs, 2, c); A.q1 = c[0]; A.q2 = c[1]; }
  if (A.use >= 3) { lag_coef(tau, hs, 3, c); A.k1 = c[0]; A.k2 = c[1]; A.k3 = c[2]; }
  if (A.nbt >= 2) { lag_coef(hs[0], hs + 1, 1, c); A.b1 = c[0]; }
  if (A.nbt >= 3) { lag_coef(hs[0], hs + 1, 2, c); A.c1 = c[0]; A.c2 = c[1]; }
  if (A.nbt >= 4) { lag_coef(hs[0], hs + 1, 3, c); A.m1 = c[0]; A.m2 = c[1]; A.m3 = c[2]; }
  return A;
}

static bool same_args(const GuessArgs &x, const GuessArgs &y) {
  return x.r == y.r && x.q1 == y.q1 && x.q2 == y.q2 && x.b1 == y.b1 && x.c1 == y.c1 &&
         x.c2 == y.c2 && x.k1 == y.k1 && x.k2 == y.k2 && x.k3 == y.k3 && x.m1 == y.m1 &&
         x.m2 == y.m2 && x.m3 == y.m3 && x.use == y.use && x.usec == y.usec &&
         x.nbt == y.nbt && x.nd == y.nd;
}

static void extrapolate_guess(Handle *h) {
  const GuessArgs A = guess_args(h);
  const int nb = h->cell.nblk;
  DBS_LAUNCH(h, KC_MISC, k_extrap, h->cgrid, dim3(BX, BY), h->seg, h->prgh, h->pprev,
             h->pprev2, h->pprev3, h->pprev4, (const double *)h->dcorr, (size_t)h->NC,
             (const int *)h->gord, (const int *)h->gchg, A, h->partials, nb);
  DBS_LAUNCH(h, KC_MISC, k_extrap_final, dim3(h->ns), dim3(1024), (const double *)h->partials,
             nb, (const int *)h->cell.bp, A.nbt, h->gord);
  h->guess_used = A;
  h->hist = std::min(h->hist + 1, 4);
  h->dt_prev4 = h->dt_prev3;
  h->dt_prev3 = h->dt_prev2;
  h->dt_prev2 = h->dt_prev;
  h->dt_prev = h->ctl.dt;
}

// rc: the first part's trace copy status
static int step_back(Handle *h, TraceOut *tr, int budget, std::vector<int> *its_out,
                     int *sweeps_out, int rc) {
  int solve_rc = DBS_OK;
  const size_t NCs = (size_t)h->NC;
  const int nd = h->ctl.n_corr - 1, nb = h->cell.nblk;
  const dim3 blk(BX, BY);
  std::vector<int> its(h->ns);
  std::vector<double> rel(h->ns);
  for (int c = 0; c < h->ctl.n_corr; c++) {
    corrector_assemble(h);
    if (tr && c == 0) {
      rc |= copy_out3(h, tr->HbyA, h->HbyA);
      rc |= copy_out(h, tr->phiHbyA, h->phiH, h->hG[0].nf);
      rc |= copy_out(h, tr->b, h->rhs, h->hG[0].nc);
    }
    // this corrector's last change and the one before
    double *dc = c > 0 ? h->dcorr + (size_t)(c - 1) * NCs : nullptr;
    double *dc1 = c > 0 ? h->dcorr + (size_t)(c - 1 + nd) * NCs : nullptr;
    double *dc2 = c > 0 ? h->dcorr + (size_t)(c - 1 + 2 * nd) * NCs : nullptr;
    if (c == 0)
      extrapolate_guess(h);  // sets guess_used, this step's coefficients
    else
      DBS_LAUNCH(h, KC_MISC, k_corr_guess, h->cgrid, blk, h->seg, h->prgh, h->p1,
                 (const double *)dc, (const double *)dc1, (const double *)dc2,
                 (const int *)h->gchg, nd, c - 1, h->guess_used);
    const int b = budget > 0 ? h->graph_budget[c] : 0;
    h->keep_hierarchy = c > 0;  // rAU is the predictor's for every corrector
    const int src = pressure_solve(h, h->rAU, h->rhs, h->prgh, b, its.data(), rel.data());
    h->keep_hierarchy = false;
    if (c > 0) {
      DBS_LAUNCH(h, KC_MISC, k_corr_record, h->cgrid, blk, h->seg, (const double *)h->prgh,
                 (const double *)h->p1, dc, dc1, dc2, h->guess_used, h->partials, nb);
      DBS_LAUNCH(h, KC_MISC, k_record_final, dim3(h->ns), dim3(1024),
                 (const double *)h->partials, nb, (const int *)h->cell.bp, h->guess_used.usec,
                 h->gchg, nd, c - 1);
    }
    if (budget > 0) {
      pressure_record(h, h->rec, c);
    } else {
      std::vector<double> bn(h->ns), r0(h->ns);
      pressure_norms(h, bn.data(), r0.data());
      for (int s = 0; s < h->ns; s++) {
        h->st[s].p_iters[c] = its[s];
        h->st[s].p_relres[c] = rel[s];
        h->st[s].p_bnorm[c] = bn[s];
        h->st[s].p_res0[c] = r0[s];
        if (its_out) (*its_out)[c] = std::max((*its_out)[c], its[s]);
      }
    }
    if (src) solve_rc = src;
    corrector_update(h, c == h->ctl.n_corr - 1);
  }
  std::swap(h->F, h->F2);  // the corrected fluxes; F^n stays in F2
  if (budget <= 0) {
    // the pressure solves synchronised the stream: the predictor records
    // in host-mapped memory are final
    std::vector<int> sw(h->ns);
    std::vector<double> mr(h->ns);
    momentum_results(h, sw.data(), mr.data(), nullptr);
    for (int s = 0; s < h->ns; s++) {
      h->st[s].mom_sweeps = sw[s];
      h->st[s].mom_relres = mr[s];
      if (sweeps_out) *sweeps_out = std::max(*sweeps_out, sw[s]);
    }
  }
  if (rc) return fail(h, DBS_EHIP, "trace copy failed");
  if (solve_rc) return fail(h, solve_rc, "pressure solve did not converge");
  return DBS_OK;
}

static int step_body(Handle *h, TraceOut *tr, int budget, std::vector<int> *its_out,
                     int *sweeps_out = nullptr) {
  const int rc = step_front(h, tr, budget);
  return step_back(h, tr, budget, its_out, sweeps_out, rc);
}

static int eager_step(Handle *h, TraceOut *tr, std::vector<int> *its_out) {
  int rc = adapt_dt(h);
  if (rc) return rc;
  rc = courant_check(h);
  if (rc) return rc;
  rc = step_body(h, tr, 0, its_out);
  for (int s = 0; s < h->ns; s++) h->st[s].steps++;
  return rc;
}

// A step never overwrites the buffers of alpha^n, U^n and F^n (the roles
// below move instead); p_rgh is solved in place, so a step that may be
// redone saves it first.
static void snapshot(Handle *h, bool save) {
  if (save) copy_n(h, h->prgh, h->snap, (size_t)h->NC);
  else copy_n(h, h->snap, h->prgh, (size_t)h->NC);
}

// buffer roles of the state (the host side of a step permutes them)
struct Roles {
  double *alpha, *alpha_old, *alpha3, *U, *U2, *U3, *F, *F2;
};
static Roles roles(const Handle *h) {
  return Roles{h->alpha, h->alpha_old, h->alpha3, h->U, h->U2, h->U3, h->F, h->F2};
}
static void set_roles(Handle *h, const Roles &r) {
  h->alpha = r.alpha;
  h->alpha_old = r.alpha_old;
  h->alpha3 = r.alpha3;
  h->U = r.U;
  h->U2 = r.U2;
  h->U3 = r.U3;
  h->F = r.F;
  h->F2 = r.F2;
}

// the roles a captured step leaves: the saturation stage's permutation, the
// predictor's result in U2 (odd budget) or U3 (even) with U^n moved to U3,
// and the correctors' fluxes swapped into F
static void replay_roles(Handle *h) {
  alpha_roles(h);
  double *Un = h->U, *X = h->U2, *Y = h->U3;
  double *to = (h->mom_budget & 1) ? X : Y;
  if (h->ctl.mom_maxit <= 0) to = X;
  h->U = to;
  h->U2 = to == X ? Y : X;
  h->U3 = Un;
  std::swap(h->F, h->F2);
}

// One step in graph mode: the step is captured once per buffer-role
// combination with a fixed predictor sweep budget and a fixed PCG budget per
// corrector, then replayed.  A sample that does not converge within a
// budget makes the step run again eagerly from the state before it, and
// the budgets grow.
static int graph_step(Handle *h) {
  int rc = courant_check(h);
  if (rc) return rc;
  const int nc = h->ctl.n_corr;
  // The predictor's budget keeps the parity of the sweeps it expects (two
  // more), so a sample that converges on schedule needs no gather copy.
  auto set_budgets = [&](const std::vector<int> &its, int sweeps, bool grow) {
    for (int c = 0; c < nc; c++) {
      const int want = its[c] + std::max(2, its[c] / 4);
      h->graph_budget[c] = grow ? std::max(h->graph_budget[c] + 2, want) : want;
    }
    const int mw = std::min(h->ctl.mom_maxit, sweeps + 2);
    h->mom_budget = grow ? std::min(h->ctl.mom_maxit, std::max(h->mom_budget + 2, mw)) : mw;
    h->slack_steps = 0;
  };
  if (h->graph_budget[0] == 0) {
    std::vector<int> its(nc, 0);
    int sweeps = 0;
    rc = step_body(h, nullptr, 0, &its, &sweeps);
    for (int s = 0; s < h->ns; s++) h->st[s].steps++;
    if (rc) return rc;
    set_budgets(its, sweeps, false);
    return DBS_OK;
  }
  const Roles before = roles(h);
  // the captured steps bake in the coefficients of the first solve's guess:
  // capture again when they change (the first steps after a state reset, a
  // change of the time step)
  if (!same_args(guess_args(h), h->graph_guess)) {
    rc = hip_check(h, hipStreamSynchronize(h->stream), "graph step");  // a replay may run
    if (rc) return rc;
    clear_graphs(h);
  }
  const GraphKey key{h->alpha, h->U, h->F};
  auto it = h->graphs.find(key);
  if (it == h->graphs.end()) {
    const unsigned long long pm = h->prof_mask;
    h->prof_mask = 0;
    StepGraphs sg;
    for (int part = 0; part < 2 && !rc; part++) {
      hipGraph_t g = nullptr;
      rc = hip_check(h, hipStreamBeginCapture(h->stream, hipStreamCaptureModeThreadLocal),
                     "capture");
      if (rc) break;
      if (part == 0) {
        step_front(h, nullptr, 1);
      } else {
        step_back(h, nullptr, 1, nullptr, nullptr, DBS_OK);
      }
      rc = hip_check(h, hipStreamEndCapture(h->stream, &g), "capture");
      if (rc) break;
      hipGraphExec_t &ex = part == 0 ? sg.front : sg.back;
      rc = hip_check(h, hipGraphInstantiate(&ex, g, nullptr, nullptr, 0), "instantiate");
      (void)hipGraphDestroy(g);
    }
    h->prof_mask = pm;
    if (rc) {
      if (sg.front) (void)hipGraphExecDestroy(sg.front);
      if (sg.back) (void)hipGraphExecDestroy(sg.back);
      return rc;
    }
    it = h->graphs.emplace(key, sg).first;
    h->graph_guess = h->guess_used;
    // capturing ran the host side of the step: the roles are already set
    // and the host time moved
  } else {
    replay_roles(h);
    h->tnow += h->ctl.dt;
  }
  // The host waits for the ready tags of the last corrector's records, not
  // for the whole replay: the next step is then submitted while the last
  // kernels of this one still run, and the device does not idle while the
  // host wakes up and launches.  An event after the replay bounds the wait.
  const int ns = h->ns;
  volatile double *tag = h->hrec;
  auto tag_of = [&](int s) -> volatile double & {
    return tag[((size_t)s * 16 + (nc - 1)) * NREC + (NREC - 1)];
  };
  for (int s = 0; s < ns; s++) tag_of(s) = -1.0;
  rc = hip_check(h, hipGraphLaunch(it->second.front, h->stream), "graph launch");
  if (!rc) rc = hip_check(h, hipGraphLaunch(it->second.back, h->stream), "graph launch");
  if (!rc) rc = hip_check(h, hipEventRecord(h->flag_ev, h->stream), "graph step");
  if (rc) return rc;
  for (;;) {
    bool ready = true;
    for (int s = 0; s < ns && ready; s++) ready = tag_of(s) > 0.0;
    if (ready) break;
    const hipError_t q = hipEventQuery(h->flag_ev);
    if (q == hipSuccess) break;  // the replay has ended: the records are final
    if (q != hipErrorNotReady) return hip_check(h, q, "graph step");
  }
  std::atomic_thread_fence(std::memory_order_acquire);
  // the records were written to host-mapped memory by the replayed kernels
  bool ok = true;
  const int slot = (h->mom_budget - 1) & 1;
  for (int s = 0; s < ns; s++) {
    for (int c = 0; c < nc; c++) {
      const double *o = h->hrec + ((size_t)s * 16 + c) * NREC;
      h->st[s].p_iters[c] = (int)o[0];
      h->st[s].p_relres[c] = o[1];
      h->st[s].p_bnorm[c] = o[3];
      h->st[s].p_res0[c] = o[4];
      ok = ok && o[2] != 0.0;
    }
    if (h->ctl.mom_maxit > 0) ok = ok && h->hmflag[slot * ns + s] == 0;
  }
  {
    std::vector<int> sw(ns);
    std::vector<double> mr(ns);
    momentum_results(h, sw.data(), mr.data(), nullptr);
    for (int s = 0; s < ns; s++) {
      h->st[s].mom_sweeps = sw[s];
      h->st[s].mom_relres = mr[s];
    }
  }
  if (ok) {
    for (int s = 0; s < ns; s++) h->st[s].steps++;
    // Budgets only grow on a redo; when every corrector has kept a slack of
    // two or more iterations for two replays in a row, they shrink to the
    // largest count of those replays plus one (and the step is captured
    // again), so masked iterations do not accumulate as the solves speed up.
    bool slack = true;
    for (int c = 0; c < nc; c++) {
      int used = 0;
      for (int s = 0; s < ns; s++) used = std::max(used, h->st[s].p_iters[c]);
      h->used_max[c] = h->slack_steps == 0 ? used : std::max(h->used_max[c], used);
      slack = slack && h->graph_budget[c] - used >= 2;
    }
    h->slack_steps = slack ? h->slack_steps + 1 : 0;
    if (h->slack_steps >= 2) {
      for (int c = 0; c < nc; c++) h->graph_budget[c] = h->used_max[c] + 1;
      h->slack_steps = 0;
      rc = hip_check(h, hipStreamSynchronize(h->stream), "graph step");
      clear_graphs(h);
    }
    return rc;
  }
  // redo eagerly from the state before the step with the budgets raised: the
  // other buffers of the roles still hold it, and the first guess's history
  // holds p_rgh^n (the first corrector's guess stored it there)
  rc = hip_check(h, hipStreamSynchronize(h->stream), "graph step");
  if (rc) return rc;
  set_roles(h, before);
  copy_n(h, h->pprev, h->prgh, (size_t)h->NC);
  add_time(h, -h->ctl.dt);
  update_closures(h);
  h->hist = 0;  // the replay moved the guesses' histories on: start them again
  std::vector<int> its(nc, 0);
  int sweeps = 0;
  rc = step_body(h, nullptr, 0, &its, &sweeps);
  for (int s = 0; s < ns; s++) h->st[s].steps++;
  set_budgets(its, sweeps, true);
  clear_graphs(h);
  return rc;
}

// the per-sample choices of the next step's pressure guesses
static int guess_stats(Handle *h) {
  const int ns = h->ns, nd = h->ctl.n_corr - 1;
  std::vector<int> go(ns), gc((size_t)ns * std::max(nd, 0));
  int e = hip_check(h, hipMemcpyAsync(go.data(), h->gord, sizeof(int) * ns,
                                      hipMemcpyDeviceToHost, h->stream), "guess state");
  if (!e && nd > 0)
    e = hip_check(h, hipMemcpyAsync(gc.data(), h->gchg, sizeof(int) * gc.size(),
                                    hipMemcpyDeviceToHost, h->stream), "guess state");
  if (!e) e = hip_check(h, hipStreamSynchronize(h->stream), "guess state");
  if (e) return e;
  const int use = std::min(h->hist, 3), usec = std::min(h->hist, 3);
  for (int s = 0; s < ns; s++) {
    h->st[s].p_guess_order = std::min(go[s], use);
    h->st[s].p_guess_change[0] = 0;
    for (int k = 0; k < nd && k < 15; k++)
      h->st[s].p_guess_change[k + 1] = std::min(gc[(size_t)s * nd + k], usec);
  }
  return DBS_OK;
}

static int finish_steps(Handle *h, int rc) {
  int e = hip_check(h, hipStreamSynchronize(h->stream), "step");
  if (!e) e = hip_check(h, hipGetLastError(), "kernel launch");
  if (e) return e;
  prof_collect(h);
  e = cell_stats(h);
  if (e) return e;
  e = guess_stats(h);
  if (e) return e;
  bool bad = false, out = false;
  for (int s = 0; s < h->ns; s++) {
    const double *v = h->hsstat + NSTAT * s;
    h->st[s].alpha_min = v[0];
    h->st[s].alpha_max = v[1];
    h->st[s].phase_volume = v[2];
    h->st[s].max_div = v[5];
    bad = bad || v[4] > 0.0;
    out = out || v[0] < -h->ctl.bounds_tol || v[1] > 1.0 + h->ctl.bounds_tol;
  }
  if (bad) return fail(h, DBS_ENAN, "non-finite value in the state");
  if (rc) return rc;
  if (h->ctl.bounds_tol > 0.0 && out)
    return fail(h, DBS_EBOUNDS, "alpha outside the admissible band");
  return DBS_OK;
}

// time one pressure solve of the current system (from x0) under the present knobs
static double time_solve(Handle *h, const double *x0, int *ok) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  *ok = 0;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) (void)hipEventDestroy(e0);
    return 0.0;
  }
  copy_n(h, x0, h->prgh, (size_t)h->NC);
  std::vector<int> its(h->ns);
  std::vector<double> rel(h->ns);
  bool good = hipEventRecord(e0, h->stream) == hipSuccess;
  const int rc = pressure_solve(h, h->rAU, h->rhs, h->prgh, 0, its.data(), rel.data());
  good = good && hipEventRecord(e1, h->stream) == hipSuccess;
  good = good && hipEventSynchronize(e1) == hipSuccess;
  float ms = 0.f;
  good = good && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ok = good && rc == DBS_OK;
  return ms;
}

static void reset_graphs(Handle *h) {
  clear_graphs(h);
  for (int c = 0; c < 16; c++) h->graph_budget[c] = 0;
  h->mom_budget = 0;
}

// ------------------------------------------ pressure solve without allocation
//
// The no-alloc solve keeps every device array it needs (work vectors,
// multigrid levels, launch tables, reduction partials) in `scratch`, a
// file-scope device array that each GPU holds from module load until the
// process ends.  In host code the symbol is only a stand-in: its device
// address is taken once per device with hipGetSymbolAddress and that
// address (never the symbol) is what kernels and copies receive.  Calls on
// one GPU share the array and must not overlap.

static __device__ __align__(256) unsigned char scratch[DBS_NOALLOC_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned char *g_scratch_ptr[kMaxDevices] = {nullptr};
thread_local std::string g_noalloc_err;
}  // namespace

static const char *noalloc_error() {
  return g_noalloc_err.empty() ? "null handle" : g_noalloc_err.c_str();
}

__global__ void __launch_bounds__(256) k_zero16(uint4 *__restrict__ p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (size_t)gridDim.x * 256)
    p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// device address of this device's scratch array (taken once per device)
static unsigned char *scratch_of_device(int &rc) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    rc = DBS_EHIP;
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      rc = DBS_EHIP;
      return nullptr;
    }
    g_scratch_ptr[dev] = (unsigned char *)ptr;
  }
  return g_scratch_ptr[dev];
}

static int noalloc_fail(int code, const std::string &msg) {
  g_noalloc_err = msg;
  return code;
}

static int pressure_solve_noalloc(const dbs_grid *grid, const int *bc_kind, int precision,
                                  const double *rAU, const double *b, double *x, double tol,
                                  int maxit, int *iters, double *relres, hipStream_t stream) {
  if (!grid || !bc_kind || !rAU || !b || !x) return noalloc_fail(DBS_EINVAL, "null argument");
  if (precision != DBS_FP64 && precision != DBS_MIXED)
    return noalloc_fail(DBS_EINVAL, "precision");
  if (!(tol > 0.0) || maxit < 1) return noalloc_fail(DBS_EINVAL, "tolerance or iteration limit");
  dbs_bc bc[6];
  memset(bc, 0, sizeof(bc));
  for (int q = 0; q < 6; q++) {
    if (bc_kind[q] < DBS_BC_WALL || bc_kind[q] > DBS_BC_WAVE)
      return noalloc_fail(DBS_EINVAL, "bad bc kind");
    // only outlet (Dirichlet) and empty faces matter to the operator
    bc[q].kind = bc_kind[q] == DBS_BC_WAVE ? DBS_BC_INLET : bc_kind[q];
  }
  std::string msg;
  if (validate_sample(grid, bc, msg)) return noalloc_fail(DBS_EINVAL, msg);
  const long long nc = (long long)grid->nx * grid->ny * grid->nz;
  if (nc > DBS_NOALLOC_MAX_CELLS)
    return noalloc_fail(DBS_EINVAL, "mesh of " + std::to_string(nc) +
                                        " cells exceeds the no-alloc maximum of " +
                                        std::to_string(DBS_NOALLOC_MAX_CELLS));
  int rc = DBS_OK;
  unsigned char *base = scratch_of_device(rc);
  if (rc) return noalloc_fail(rc, "hipGetSymbolAddress failed");
  Handle hh;
  Handle *h = &hh;
  h->stream = stream;
  h->arena = base;
  h->arena_cap = DBS_NOALLOC_BYTES;
  h->hscal = h->hscal_own;
  h->hpub = h->hpub_own;
  // the array keeps the last call's contents: clear all of it
  const size_t n16 = DBS_NOALLOC_BYTES / 16;
  hipLaunchKernelGGL(k_zero16, dim3(2048), dim3(256), 0, h->stream, (uint4 *)base, n16);
  const double g0[3] = {0.0, 0.0, 0.0};
  Geom G = make_geom(grid, bc, 1.0, g0);
  G.c0 = 0;
  h->ns = 1;
  h->NC = ((long long)G.nc + FLAT_CELLS - 1) / FLAT_CELLS * FLAT_CELLS;
  G.vs = (int)h->NC;
  h->hG.assign(1, G);
  h->hrng.assign(1, Rng{0, G.nc, G.has_outlet ? 0 : 1, 0});
  h->st.assign(1, dbs_stats());
  memset(&h->ctl, 0, sizeof(h->ctl));
  h->ctl.p_tol = tol;
  h->ctl.p_maxit = maxit;
  h->ctl.precision = precision;
  h->cell.hbp = {0, cell_blocks(G)};
  h->cell.nblk = h->cell.hbp[1];
  h->flat.hbp = {0, (int)(h->NC / FLAT_CELLS)};
  h->flat.nblk = h->flat.hbp[1];
  const size_t NC = (size_t)h->NC;
  h->cell.bp = (int *)arena_take(h, sizeof(int) * 2, rc);
  h->flat.bp = (int *)arena_take(h, sizeof(int) * 2, rc);
  h->rng = (Rng *)arena_take(h, sizeof(Rng), rc);
  h->scal = (double *)arena_take(h, sizeof(double) * NSC, rc);
  double *vec[8];
  for (double *&v : vec) v = (double *)arena_take(h, sizeof(double) * NC, rc);
  h->r = vec[0]; h->z = vec[1]; h->pv = vec[2]; h->q = vec[3]; h->pv2 = vec[4];
  double *rA = vec[5], *bA = vec[6], *xA = vec[7];
  if (!rc) {
    const bool ok =
        hipMemcpyAsync(h->cell.bp, h->cell.hbp.data(), sizeof(int) * 2, hipMemcpyHostToDevice,
                       h->stream) == hipSuccess &&
        hipMemcpyAsync(h->flat.bp, h->flat.hbp.data(), sizeof(int) * 2, hipMemcpyHostToDevice,
                       h->stream) == hipSuccess &&
        hipMemcpyAsync(h->rng, h->hrng.data(), sizeof(Rng), hipMemcpyHostToDevice, h->stream) ==
            hipSuccess &&
        hipStreamSynchronize(h->stream) == hipSuccess;
    if (!ok) rc = DBS_EHIP;
  }
  if (!rc) rc = pressure_setup(h);
  if (rc == DBS_ENOMEM)
    return noalloc_fail(DBS_EINVAL, "the solve needs more than " +
                                        std::to_string(h->arena_used) + " bytes of scratch (has " +
                                        std::to_string((size_t)DBS_NOALLOC_BYTES) + ")");
  if (rc) return noalloc_fail(rc, h->err.empty() ? "set-up failed" : h->err);
  // the caller's arrays hold nc cells; the solve runs over the padded arena
  copy_n(h, rAU, rA, (size_t)G.nc);
  copy_n(h, b, bA, (size_t)G.nc);
  copy_n(h, x, xA, (size_t)G.nc);
  int its = 0;
  double rel = 0.0;
  const int src = pressure_solve(h, rA, bA, xA, 0, &its, &rel);
  copy_n(h, xA, x, (size_t)G.nc);
  if (hipStreamSynchronize(h->stream) != hipSuccess || hipGetLastError() != hipSuccess)
    return noalloc_fail(DBS_EHIP, "solve failed");
  if (iters) *iters = its;
  if (relres) *relres = rel;
  if (src) return noalloc_fail(src, "pressure solve did not converge");
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
  return create_impl(1, grid, phys, bc, ctl, out);
}

int dbs_batch_create(int n, const dbs_grid *grids, const dbs_physics *phys, const dbs_bc *bcs,
                     const dbs_controls *ctl, dbs_handle **out) {
  return create_impl(n, grids, phys, bcs, ctl, out);
}

int dbs_batch_size(const dbs_handle *H) { return H ? H->h.ns : 0; }

void dbs_destroy(dbs_handle *H) {
  if (!H) return;
  Handle *h = &H->h;
  // teardown: nothing is left to report an error to
  if (h->stream) (void)hipStreamSynchronize(h->stream);
  clear_graphs(h);
  for (void *p : h->allocs) (void)hipFree(p);
  for (void *p : h->hallocs) (void)hipHostFree(p);
  for (hipEvent_t e : h->tm.ev) (void)hipEventDestroy(e);
  if (h->flag_ev) (void)hipEventDestroy(h->flag_ev);
  for (hipEvent_t e : h->mom_ev)
    if (e) (void)hipEventDestroy(e);
  pressure_free(h);
  if (h->own_stream) (void)hipStreamDestroy(h->own_stream);
  delete H;
}

const char *dbs_last_error(const dbs_handle *H) {
  return H ? H->h.err.c_str() : noalloc_error();
}

int dbs_set_stream(dbs_handle *H, void *stream) {
  if (!H) return DBS_EINVAL;
  Handle *h = &H->h;
  if (int rc = hip_check(h, hipStreamSynchronize(h->stream), "set_stream")) return rc;
  h->stream = stream ? (hipStream_t)stream : h->own_stream;
  return DBS_OK;
}

int dbs_batch_set_static(dbs_handle *H, int i, const double *phi, const double *kinv) {
  if (!H || !phi || !kinv) return DBS_EINVAL;
  return set_static_impl(&H->h, i, phi, kinv);
}

int dbs_set_static(dbs_handle *H, const double *phi, const double *kinv) {
  return dbs_batch_set_static(H, 0, phi, kinv);
}

int dbs_batch_set_state(dbs_handle *H, int i, const double *alpha, const double *U,
                        const double *prgh, const double *F) {
  if (!H || !alpha || !U || !prgh) return DBS_EINVAL;
  Handle *h = &H->h;
  if (int rc = check_sample(h, i)) return rc;
  const size_t nc = h->hG[i].nc;
  if (!all_finite(alpha, nc) || !all_finite(U, 3 * nc) || !all_finite(prgh, nc) ||
      (F && !all_finite(F, h->hG[i].nf)))
    return fail(h, DBS_EINVAL, "non-finite input state");
  return set_state_impl(h, i, alpha, U, prgh, F, hipMemcpyHostToDevice, h->stream);
}

int dbs_set_state(dbs_handle *H, const double *alpha, const double *U, const double *prgh,
                  const double *F) {
  return dbs_batch_set_state(H, 0, alpha, U, prgh, F);
}

int dbs_batch_set_state_dev(dbs_handle *H, int i, const double *alpha, const double *U,
                            const double *prgh, const double *F, void *stream) {
  if (!H || !alpha || !U || !prgh) return DBS_EINVAL;
  Handle *h = &H->h;
  if (int rc = check_sample(h, i)) return rc;
  hipStream_t s = stream ? (hipStream_t)stream : h->stream;
  if (int rc = hip_check(h, hipStreamSynchronize(h->stream), "set_state")) return rc;
  return set_state_impl(h, i, alpha, U, prgh, F, hipMemcpyDeviceToDevice, s);
}

int dbs_set_state_dev(dbs_handle *H, const double *alpha, const double *U, const double *prgh,
                      const double *F, void *stream) {
  return dbs_batch_set_state_dev(H, 0, alpha, U, prgh, F, stream);
}

int dbs_batch_get_state(dbs_handle *H, int i, double *alpha, double *U, double *prgh, double *p,
                        double *F) {
  if (!H) return DBS_EINVAL;
  Handle *h = &H->h;
  if (int rc = check_sample(h, i)) return rc;
  return get_state_impl(h, i, alpha, U, prgh, p, F, hipMemcpyDeviceToHost, h->stream);
}

int dbs_get_state(dbs_handle *H, double *alpha, double *U, double *prgh, double *p, double *F) {
  return dbs_batch_get_state(H, 0, alpha, U, prgh, p, F);
}

int dbs_batch_get_state_dev(dbs_handle *H, int i, double *alpha, double *U, double *prgh,
                            double *p, double *F, void *stream) {
  if (!H) return DBS_EINVAL;
  Handle *h = &H->h;
  if (int rc = check_sample(h, i)) return rc;
  hipStream_t s = stream ? (hipStream_t)stream : h->stream;
  return get_state_impl(h, i, alpha, U, prgh, p, F, hipMemcpyDeviceToDevice, s);
}

int dbs_get_state_dev(dbs_handle *H, double *alpha, double *U, double *prgh, double *p,
                      double *F, void *stream) {
  return dbs_batch_get_state_dev(H, 0, alpha, U, prgh, p, F, stream);
}

int dbs_step(dbs_handle *H, int nsteps) {
  if (!H || nsteps < 0) return DBS_EINVAL;
  Handle *h = &H->h;
  int rc = DBS_OK;
  for (int s = 0; s < nsteps && !rc; s++)
    rc = h->graph_mode ? graph_step(h) : eager_step(h, nullptr, nullptr);
  if (rc == DBS_ECOURANT || rc == DBS_EHIP) return rc;
  return finish_steps(h, rc);
}

int dbs_batch_step(dbs_handle *H, int nsteps) { return dbs_step(H, nsteps); }

int dbs_set_graph(dbs_handle *H, int on) {
  if (!H) return DBS_EINVAL;
  Handle *h = &H->h;
  if (on && h->ctl.target_courant > 0.0) {
    h->err = "graph mode replays a fixed time step; adaptive stepping is eager only";
    return DBS_EINVAL;
  }
  if (int rc = hip_check(h, hipStreamSynchronize(h->stream), "set_graph")) return rc;
  h->graph_mode = on ? 1 : 0;
  reset_graphs(h);
  // on > 1: start from a budget of on - 1 iterations (and predictor sweeps)
  // instead of measuring it
  if (on > 1) {
    for (int c = 0; c < 16; c++) h->graph_budget[c] = on - 1;
    h->mom_budget = std::min(h->ctl.mom_maxit, on - 1);
  }
  return DBS_OK;
}

int dbs_autotune(dbs_handle *H, int *kz_out, int *sweeps_out, int *coarse_out, int *shift_out,
                 int *fused_out, int *cblock_out, double *ms_out) {
  if (!H) return DBS_EINVAL;
  Handle *h = &H->h;
  int rc = DBS_OK;
  if (!h->snap) {
    h->snap = dmalloc(h, (size_t)h->NC, rc);
    if (rc) return fail(h, rc, "snapshot allocation");
  }
  double *x0 = h->Rp;  // transport scratch, free once the transport is done
  const unsigned long long pm = h->prof_mask;
  h->prof_mask = 0;
  // the first corrector's system of the current state (p_rgh is untouched
  // until the solve)
  const Roles before = roles(h);
  snapshot(h, true);
  alpha_stage(h);
  momentum_predictor(h);
  corrector_assemble(h);
  copy_n(h, h->prgh, x0, (size_t)h->NC);
  struct Cand {
    int kz, sweeps, coarse, shift, fused, cblock;
  };
  Cand best{h->kz_fine, h->mg_pre, h->mgc, h->bottom_shift, h->fused_sweep, h->coarse_block};
  double best_ms = 1e300;
  auto trial = [&](const Cand &c) {
    h->kz_fine = c.kz;
    h->mg_pre = h->mg_post = c.sweeps;
    h->mgc = c.coarse;
    h->bottom_shift = c.shift;
    h->fused_sweep = c.fused;
    h->coarse_block = c.cblock;
    if (pressure_retune(h)) return;
    int ok = 0;
    time_solve(h, x0, &ok);  // first run: caches and clocks
    const double ms = time_solve(h, x0, &ok);
    if (ok && ms < best_ms) {
      best_ms = ms;
      best = c;
    }
  };
  for (int sw = 1; sw <= 3; sw++)
    for (int shf = 0; shf <= 1; shf++) trial(Cand{0, sw, sw, shf, 1, 0});
  {
    const Cand b0 = best;
    for (int cs = 1; cs <= 4; cs++)
      if (cs != b0.coarse) trial(Cand{0, b0.sweeps, cs, b0.shift, 1, 0});
  }
  trial(Cand{0, best.sweeps, best.coarse, best.shift, 0, best.cblock});
  const Cand mid = best;
  for (int kz : {2, 4, 8, 16})
    trial(Cand{kz, mid.sweeps, mid.coarse, mid.shift, mid.fused, mid.cblock});
  h->kz_fine = best.kz;
  h->mg_pre = h->mg_post = best.sweeps;
  h->mgc = best.coarse;
  h->bottom_shift = best.shift;
  h->fused_sweep = best.fused;
  h->coarse_block = best.cblock;
  rc = pressure_retune(h);
  // restore the state as it was before tuning
  set_roles(h, before);
  snapshot(h, false);
  update_closures(h);
  h->prof_mask = pm;
  reset_graphs(h);
  if (!rc) rc = hip_check(h, hipStreamSynchronize(h->stream), "autotune");
  if (kz_out) *kz_out = best.kz;
  if (sweeps_out) *sweeps_out = best.sweeps;
  if (coarse_out) *coarse_out = best.coarse;
  if (shift_out) *shift_out = best.shift;
  if (fused_out) *fused_out = best.fused;
  if (cblock_out) *cblock_out = best.cblock;
  if (ms_out) *ms_out = best_ms;
  return rc;
}

int dbs_set_tuning(dbs_handle *H, int kz, int kz_coarse, int sweeps, int coarse_sweeps,
                   int shift, int fused, int coarse_block) {
  if (!H || kz < 0 || kz > 64 || kz_coarse < 0 || kz_coarse > 64 || sweeps < 1 || sweeps > 8 ||
      coarse_sweeps < 1 || coarse_sweeps > 8 || shift < 0 || shift > 4 || coarse_block < 0 ||
      coarse_block > 4)
    return DBS_EINVAL;
  Handle *h = &H->h;
  if (int rc = hip_check(h, hipStreamSynchronize(h->stream), "set_tuning")) return rc;
  h->kz_fine = kz;
  h->kz_coarse = kz_coarse;
  h->coarse_block = coarse_block;
  h->mg_pre = h->mg_post = sweeps;
  h->mgc = coarse_sweeps;
  h->bottom_shift = shift;
  h->fused_sweep = fused ? 1 : 0;
  reset_graphs(h);
  return pressure_retune(h);
}

int dbs_debug_step_trace(dbs_handle *H, double *A, double *rAU, double *Shat, double *Ustar,
                         double *HbyA, double *phiHbyA, double *b, double *Rp, double *Rm,
                         double *alphaPhi) {
  if (!H) return DBS_EINVAL;
  Handle *h = &H->h;
  if (h->ns != 1) return fail(h, DBS_EINVAL, "trace needs a single-sample handle");
  TraceOut tr{A, rAU, Shat, Ustar, HbyA, phiHbyA, b, Rp, Rm, alphaPhi};
  int rc = eager_step(h, &tr, nullptr);
  if (rc == DBS_ECOURANT) return rc;
  return finish_steps(h, rc);
}

int dbs_batch_get_stats(dbs_handle *H, int i, dbs_stats *out) {
  if (!H || !out) return DBS_EINVAL;
  if (int rc = check_sample(&H->h, i)) return rc;
  *out = H->h.st[i];
  out->time = H->h.tnow;
  out->dt = H->h.ctl.dt;  // the step just taken (adaptive: chosen before it)
  return DBS_OK;
}

int dbs_set_time(dbs_handle *H, double t) {
  if (!H || !isfinite(t)) return DBS_EINVAL;
  Handle *h = &H->h;
  int rc = hip_check(h, hipStreamSynchronize(h->stream), "set_time");
  if (rc) return rc;
  for (auto &G : h->hG) G.t = t;
  h->tnow = t;
  rc = hip_check(h, hipMemcpy(h->dG, h->hG.data(), sizeof(Geom) * h->ns,
                              hipMemcpyHostToDevice), "set_time");
  if (!rc) wave_profile(h);
  if (!rc) rc = hip_check(h, hipStreamSynchronize(h->stream), "set_time");
  return rc;
}

int dbs_get_stats(dbs_handle *H, dbs_stats *out) { return dbs_batch_get_stats(H, 0, out); }

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

int dbs_pressure_solve_noalloc(const dbs_grid *grid, const int bc_kind[6], int precision,
                               const double *rAU, const double *b, double *x, double tol,
                               int maxit, int *iters, double *relres, void *stream) {
  return pressure_solve_noalloc(grid, bc_kind, precision, rAU, b, x, tol, maxit, iters, relres,
                                (hipStream_t)stream);
}

int dbs_debug_pressure_solve(dbs_handle *H, const double *rAU, const double *b, double *x,
                             int *iters, double *relres) {
  if (!H || !rAU || !b || !x) return DBS_EINVAL;
  Handle *h = &H->h;
  if (h->ns != 1) return fail(h, DBS_EINVAL, "debug solve needs a single-sample handle");
  const size_t nc = h->hG[0].nc;
  int rc = hip_check(h, hipMemcpyAsync(h->rAU, rAU, nc * 8, hipMemcpyHostToDevice, h->stream), "copy");
  if (!rc) rc = hip_check(h, hipMemcpyAsync(h->rhs, b, nc * 8, hipMemcpyHostToDevice, h->stream), "copy");
  if (!rc) rc = hip_check(h, hipMemcpyAsync(h->Rp, x, nc * 8, hipMemcpyHostToDevice, h->stream), "copy");
  if (rc) return rc;
  int its = 0;
  double rel = 0.0;
  const int src = pressure_solve(h, h->rAU, h->rhs, h->Rp, 0, &its, &rel);
  if (iters) *iters = its;
  if (relres) *relres = rel;
  rc = hip_check(h, hipMemcpyAsync(x, h->Rp, nc * 8, hipMemcpyDeviceToHost, h->stream), "copy");
  if (!rc) rc = hip_check(h, hipStreamSynchronize(h->stream), "solve");
  if (!rc) rc = hip_check(h, hipGetLastError(), "kernel launch");
  prof_collect(h);
  if (rc) return rc;
  if (src) return fail(h, src, "pressure solve did not converge");
  return DBS_OK;
}

}  // extern "C"
