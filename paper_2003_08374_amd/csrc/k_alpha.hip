// Saturation transport: Eq. (phaseEq) of Sec. 2.2 advanced explicitly with a
// Van Leer convection flux, the relative flux phi*alpha_l*alpha_g*v_r of the
// Sec. 2.3 summary (interface compression in clear regions, Eq. (vr_porous)
// in porous regions) and the MULES flux limiter (Sec. 3.2).
//
// One transport cycle is M + 3 passes over the cells for M limiter
// iterations:
//   alpha_grad     cell gradient of alpha (for the compression flux)
//   alpha_face     antidiffusive face flux A = F*alpha_VL + G - F*alpha_upwind
//   alpha_bounds   local extrema, low-order provisional alpha, Q+-, and the
//                  first iteration's R+- (face limiters all 1)
//   alpha_iter     (M - 1 times) face limiters of an iteration (min over the
//                  two cells, never increasing) and the next R+- (limited
//                  counter-fluxes counted)
//   alpha_update   the last iteration's face limiter, limited flux,
//                  alpha^{n+1}, mass flux rhoPhi, closures
// The passes are bound by FP64 arithmetic and load latency more than by
// bandwidth, and run one cell per thread at high occupancy: a tiled variant
// that kept A in LDS and formed the bounds in the same launch (one barrier
// per plane, half the occupancy) took 30% longer than the two passes.  Every face is owned by the cell on its plus side (plus
// the last face of each row, owned by the last cell), so all writes are
// race-free; R+- and the face limiters alternate between two buffers.
#include "dbs_internal.h"

namespace dbs {

struct AlphaArgs {
  const double *__restrict__ alpha, *__restrict__ F, *__restrict__ phi, *__restrict__ kinv;
  const double *__restrict__ prgh, *__restrict__ ml, *__restrict__ mg, *__restrict__ pc;
  const double *__restrict__ gx, *__restrict__ gy, *__restrict__ gz;  // cell grad(alpha)
};

__device__ inline Cell shifted(const Geom &G, const Cell &P, int a, int d) {
  Cell Q = P;
  Q.co[a] += d;
  Q.i = Q.co[0]; Q.j = Q.co[1]; Q.k = Q.co[2];
  Q.c = P.c + d * stride_of(G, a);
  return Q;
}

// Gauss gradient of alpha in cell P: face values are the mean with the
// neighbour, or the boundary alpha; empty axes contribute nothing.  Both
// neighbour loads of an axis are issued unconditionally (a domain side
// reads the cell itself), the boundary value replaces the face value after.
__device__ inline void grad_alpha(const Geom &G, const AlphaArgs &X, const Cell &P, double g[3]) {
  const double aP = X.alpha[P.c];
#pragma unroll
  for (int a = 0; a < 3; a++) {
    if (G.n[a] == 1 && G.bck[2 * a] == BC_EMPTY) { g[a] = 0.0; continue; }
    const bool bm = on_boundary(G, P, a, 0), bp = on_boundary(G, P, a, 1);
    const int st = stride_of(G, a);
    const double am = X.alpha[bm ? P.c : P.c - st], ap = X.alpha[bp ? P.c : P.c + st];
    double fv0 = 0.5 * (aP + am), fv1 = 0.5 * (aP + ap);
    if (bm) fv0 = bnd_alpha(G, 2 * a, P.j, aP, X.F[face_of(G, P, a, 0)]);
    if (bp) fv1 = bnd_alpha(G, 2 * a + 1, P.j, aP, X.F[face_of(G, P, a, 1)]);
    g[a] = (fv1 - fv0) * G.ih[a];
  }
}

// Antidiffusive flux of the face on the minus side of cell N along a
// (zero on a domain face).  Every load of the upwind stencil and of the
// porous form is issued before any branch; a domain face reads the cell
// itself and is discarded.  The axis is a compile-time constant, so the
// cell's coordinates are indexed statically.
template <int a>
__device__ inline double face_antidiffusive(const Geom &G, const Phys &Ph, const AlphaArgs &X,
                                            const Cell &N, int f) {
  const bool bnd = on_boundary(G, N, a, 0);
  const int sa = stride_of(G, a);
  const int o = bnd ? N.c : N.c - sa, n = N.c;
  const double Ff = X.F[f];
  const double ao = X.alpha[o], an = X.alpha[n];
  const double ko = X.kinv[o], kn = X.kinv[n];
  const bool fwd = Ff >= 0.0;
  // second upwind cell, or the upwind cell itself next to a domain face
  const int iuu = fwd ? (N.co[a] >= 2 ? o - sa : o) : (N.co[a] + 1 < G.n[a] ? n + sa : n);
  const double auu = X.alpha[iuu];
  const double pro = X.prgh[o], prn = X.prgh[n], pco = X.pc[o], pcn = X.pc[n];
  const double mlo = X.ml[o], mln = X.ml[n], mgo = X.mg[o], mgn = X.mg[n];
  const double aU = fwd ? ao : an, aD = fwd ? an : ao;
  const double aUU = auu;
  const double FL = Ff * aU;
  // Van Leer: aU + psi(r) (aD - aU) / 2 with psi(r) = (r + |r|) / (1 + |r|)
  // and r = d0 / d1 (d0 = aU - aUU, d1 = aD - aU) is aU + d0 d1 / (d0 + d1)
  // where d0 d1 > 0 and aU elsewhere: one division instead of two
  const double d0 = aU - aUU, d1 = aD - aU;
  const double avl = d0 * d1 > 0.0 ? aU + d0 * d1 / (d0 + d1) : aU;
  double Gr;
  Cell O = shifted(G, N, a, bnd ? 0 : -1);
  if (ko == 0.0 && kn == 0.0) {
    // clear face: compression flux along +grad(alpha), face-local |v|
    const double go[3] = {X.gx[O.c], X.gy[O.c], X.gz[O.c]};
    const double gn[3] = {X.gx[N.c], X.gy[N.c], X.gz[N.c]};
    double gf[3], mag2 = 0.0;
    for (int b = 0; b < 3; b++) {
      gf[b] = 0.5 * (go[b] + gn[b]);
      mag2 += gf[b] * gf[b];
    }
    double nfa = gf[a] / (sqrt(mag2) + G.dN);
    double Fr = Ph.c_alpha * fabs(Ff) * nfa;
    Gr = Fr >= 0.0 ? Fr * ao * (1.0 - an) : Fr * an * (1.0 - ao);
  } else {
    // porous face: alpha_g u_l - alpha u_g with phase-upwinded mobilities
    const double k0f = 2.0 / (ko + kn);
    const double af = 0.5 * (ao + an), agf = 1.0 - af;
    const double ga = Ph.g[a];
    const double po = pro + rho_of(Ph, ao) * gdotx_cell(G, Ph, O);
    const double pn = prn + rho_of(Ph, an) * gdotx_cell(G, Ph, N);
    const double dp = (pn - po) * G.ih[a];
    const double dpl = dp - ((1.0 - an) * pcn - (1.0 - ao) * pco) * G.ih[a] - Ph.rho_l * ga;
    const double dpg = dp + (an * pcn - ao * pco) * G.ih[a] - Ph.rho_g * ga;
    const double mlf = dpl < 0.0 ? mlo : mln;
    const double mgf = dpg < 0.0 ? mgo : mgn;
    const double ul = -k0f * mlf * dpl * G.area[a];
    const double ug = -k0f * mgf * dpg * G.area[a];
    Gr = agf * ul - af * ug;
  }
  return bnd ? 0.0 : Ff * avl + Gr - FL;
}

// grad(alpha) of every cell, read by the compression flux of clear faces
// and by the curvature.  ca (the curvature's gradient with a contact angle
// imposed): a clear cell next to a porous cell along an axis takes, on that
// axis, the component that makes its normal meet the wall at the angle
// (n.n_w = -cos(theta) for n = grad(alpha)/|grad(alpha)|, n_w from the
// porous into the clear cell) given its other Gauss components; with
// porous cells on both sides of an axis it keeps the Gauss value.
__global__ void __launch_bounds__(NTHREADS) k_alpha_grad(Segs SG, AlphaArgs X,
                                                         double *__restrict__ gx,
                                                         double *__restrict__ gy,
                                                         double *__restrict__ gz, int ca,
                                                         double cot) {
  FOR_CELLS(SG, G, P) {
  double g[3];
  grad_alpha(G, X, P, g);
  if (ca && X.kinv[P.c] == 0.0) {
    const double g0[3] = {g[0], g[1], g[2]};
#pragma unroll
    for (int a = 0; a < 3; a++) {
      if (G.n[a] == 1 && G.bck[2 * a] == BC_EMPTY) continue;
      const int st = stride_of(G, a);
      // n_w . e_axis summed over the porous neighbours along a
      int w = 0;
      if (!on_boundary(G, P, a, 0) && X.kinv[P.c - st] > 0.0) w += 1;
      if (!on_boundary(G, P, a, 1) && X.kinv[P.c + st] > 0.0) w -= 1;
      if (w == 0) continue;
      double t2 = 0.0;
#pragma unroll
      for (int b = 0; b < 3; b++)
        if (b != a) t2 += g0[b] * g0[b];
      g[a] = -cot * sqrt(t2) * (double)w;
    }
  }
  gx[P.c] = g[0];
  gy[P.c] = g[1];
  gz[P.c] = g[2];
  }
}

// low-order (upwind) flux of side s of cell P along a, oriented along +axis
// (both candidate upwind values are loaded with the flux, before any
// branch; a domain face reads the cell itself)
__device__ __forceinline__ double low_order_flux(const Geom &G, const double *__restrict__ alpha,
                                                 const double *__restrict__ F, const Cell &P,
                                                 int a, int s, int f, bool bnd) {
  const double Ff = F[f];
  const int nb = bnd ? P.c : P.c + (s ? 1 : -1) * stride_of(G, a);
  const double ac = alpha[P.c], anb = alpha[nb];
  if (bnd) return Ff * bnd_alpha(G, 2 * a + s, P.j, ac, Ff);
  const double aown = s ? ac : anb, anbr = s ? anb : ac;
  return Ff * (Ff >= 0.0 ? aown : anbr);
}

__global__ void __launch_bounds__(NTHREADS) k_alpha_face(Segs SG, Phys Ph, AlphaArgs X,
                                                         double *__restrict__ A) {
  FOR_CELLS(SG, G, P) {
  A[face_of(G, P, 0, 0)] = face_antidiffusive<0>(G, Ph, X, P, face_of(G, P, 0, 0));
  A[face_of(G, P, 1, 0)] = face_antidiffusive<1>(G, Ph, X, P, face_of(G, P, 1, 0));
  A[face_of(G, P, 2, 0)] = face_antidiffusive<2>(G, Ph, X, P, face_of(G, P, 2, 0));
#pragma unroll
  for (int a = 0; a < 3; a++)
    if (P.co[a] == G.n[a] - 1) A[face_of(G, P, a, 1)] = 0.0;
  }
}


// Local extrema, the low-order provisional alpha and Q+- of each cell, and
// the cell factors R+- of the first limiter iteration (all face limiters 1,
// so the limited sums equal P-+).  P+- are not kept: the later iterations
// form them again from A.
__global__ void __launch_bounds__(NTHREADS) k_alpha_bounds(Segs SG, const double *__restrict__ alpha,
    const double *__restrict__ F, const double *__restrict__ phi, const double *__restrict__ A,
    double *__restrict__ Qp, double *__restrict__ Qm, double *__restrict__ Rp,
    double *__restrict__ Rm, int nsub) {
  FOR_CELLS(SG, G, P) {
  const double aP = alpha[P.c];
  double outL = 0.0, amax = aP, amin = aP, pin = 0.0, pout = 0.0;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    if (G.n[a] == 1 && G.bck[2 * a] == BC_EMPTY) continue;
#pragma unroll
    for (int s = 0; s < 2; s++) {
      const double so = s ? 1.0 : -1.0;
      const int f = face_of(G, P, a, s);
      const bool bnd = on_boundary(G, P, a, s);
      outL += so * low_order_flux(G, alpha, F, P, a, s, f, bnd);
      if (!bnd) {
        double an = alpha[P.c + (s ? 1 : -1) * stride_of(G, a)];
        amax = fmax(amax, an);
        amin = fmin(amin, an);
      } else if (so * F[f] < 0.0) {
        double ab = bnd_alpha(G, 2 * a + s, P.j, aP, F[f]);
        amax = fmax(amax, ab);
        amin = fmin(amin, ab);
      }
      const double Af = A[f];
      pin += fmax(0.0, -so * Af);
      pout += fmax(0.0, so * Af);
    }
  }
  amax = fmin(1.0, amax);
  amin = fmax(0.0, amin);
  const double vol = phi[P.c] * G.V / (G.dt / nsub);
  const double aL = aP - outL / vol;
  const double qp = vol * fmax(0.0, amax - aL), qm = vol * fmax(0.0, aL - amin);
  Qp[P.c] = qp;
  Qm[P.c] = qm;
  Rp[P.c] = pin > 0.0 ? clamp01((qp + pout) / pin, 0.0, 1.0) : 1.0;
  Rm[P.c] = pout > 0.0 ? clamp01((qm + pin) / pout, 0.0, 1.0) : 1.0;
  }
}

// One further limiter iteration: the face limiters lam_k = min(lam_{k-1},
// the factor of R_k at the face's two cells) of the cell's six faces (each
// interior face formed by both its cells with the same arithmetic; the
// owned faces stored), and the cell's next R+- with the limited
// counter-fluxes counted.  first: lam_{k-1} is 1 everywhere (k = 1).
__global__ void __launch_bounds__(NTHREADS) k_alpha_iter(Segs SG, const double *__restrict__ A,
    const double *__restrict__ Rp, const double *__restrict__ Rm,
    const double *__restrict__ lam_in, int first, const double *__restrict__ Qp,
    const double *__restrict__ Qm, double *__restrict__ lam_out, double *__restrict__ Rp_out,
    double *__restrict__ Rm_out) {
  FOR_CELLS(SG, G, P) {
  double lout = 0.0, lin = 0.0, pin = 0.0, pout = 0.0;
  for (int a = 0; a < 3; a++) {
    for (int s = 0; s < 2; s++) {
      const int f = face_of(G, P, a, s);
      if (on_boundary(G, P, a, s)) {
        // A = 0 on domain faces (and on both faces of an empty axis)
        lam_out[f] = 0.0;
        continue;
      }
      const double so = s ? 1.0 : -1.0;
      const int nb = P.c + (s ? 1 : -1) * stride_of(G, a);
      const int o = s ? P.c : nb, n = s ? nb : P.c;
      const double Af = A[f];
      const double l = Af >= 0.0 ? fmin(Rm[o], Rp[n]) : fmin(Rp[o], Rm[n]);
      const double lf = first ? l : fmin(lam_in[f], l);
      if (s == 0) lam_out[f] = lf;
      lout += lf * fmax(0.0, so * Af);
      lin += lf * fmax(0.0, -so * Af);
      pin += fmax(0.0, -so * Af);
      pout += fmax(0.0, so * Af);
    }
  }
  Rp_out[P.c] = pin > 0.0 ? clamp01((Qp[P.c] + lout) / pin, 0.0, 1.0) : 1.0;
  Rm_out[P.c] = pout > 0.0 ? clamp01((Qm[P.c] + lin) / pout, 0.0, 1.0) : 1.0;
  }
}

// The last limiter iteration's face factor is formed here for each of the
// cell's faces (each interior face by both its cells, with the same
// arithmetic) from R+- and the previous factors lam (first: none).
// Sub-cycle `sub` of nsub (time step dt / nsub): the face's limited flux is
// summed into rhoPhi (and aphi) over the sub-cycles, and the last turns the
// sum into the mean and the mean into the mass flux.
__global__ void __launch_bounds__(NTHREADS) k_alpha_update(Segs SG, Phys Ph, const double *__restrict__ alpha, const double *__restrict__ F,
    const double *__restrict__ phi, const double *__restrict__ kinv, const double *__restrict__ A,
    const double *__restrict__ Rp, const double *__restrict__ Rm,
    const double *__restrict__ lam, int first, double *__restrict__ alpha_new,
    double *__restrict__ rhoPhi, double *__restrict__ ml, double *__restrict__ mg,
    double *__restrict__ pc, double *__restrict__ cf, int sub, int nsub,
    double *__restrict__ aphi) {
  FOR_CELLS(SG, G, P) {
  double out = 0.0;
  const double drho = Ph.rho_l - Ph.rho_g;
  const bool last = sub == nsub - 1;
  for (int a = 0; a < 3; a++) {
    const bool empty = G.n[a] == 1 && G.bck[2 * a] == BC_EMPTY;
    for (int s = 0; s < 2; s++) {
      const int f = face_of(G, P, a, s);
      if (empty) {
        if (s == 0 || P.co[a] == G.n[a] - 1) {
          rhoPhi[f] = 0.0;
          if (aphi) aphi[f] = 0.0;
        }
        continue;
      }
      const bool bnd = on_boundary(G, P, a, s);
      const double FL = low_order_flux(G, alpha, F, P, a, s, f, bnd);
      // face factor: minus-side cell o, plus-side cell n (a domain face
      // reads the cell itself and is not limited)
      const int nb = bnd ? P.c : P.c + (s ? 1 : -1) * stride_of(G, a);
      const int o = s ? P.c : nb, n = s ? nb : P.c;
      const double Af = A[f];
      const double l = Af >= 0.0 ? fmin(Rm[o], Rp[n]) : fmin(Rp[o], Rm[n]);
      const double lf = first ? l : fmin(lam[f], l);
      const double ap = bnd ? FL : fma(lf, Af, FL);
      out += s ? ap : -ap;
      if (s == 0 || bnd) {
        // the running sum of the sub-cycles' limited fluxes (one cycle: the flux)
        const double sum = (sub == 0 ? 0.0 : rhoPhi[f]) + ap;
        rhoPhi[f] = last ? drho * (sum / nsub) + Ph.rho_g * F[f] : sum;
        if (aphi) {
          const double sa = (sub == 0 ? 0.0 : aphi[f]) + ap;
          aphi[f] = last ? sa / nsub : sa;
        }
      }
    }
  }
  const double an = alpha[P.c] - (G.dt / nsub) * out / (phi[P.c] * G.V);
  alpha_new[P.c] = an;
  double l, g, p;
  closures(Ph, an, l, g, p);
  ml[P.c] = l;
  mg[P.c] = g;
  const bool porous = kinv[P.c] > 0.0;
  pc[P.c] = porous ? p : 0.0;
  cf[P.c] = porous ? l / (l + g) - an : 0.0;
  }
}

// Clear-fluid surface tension (Sec. 2.2, Brackbill's continuum surface
// force): SK = sigma kappa / phi in clear cells, 0 in porous cells, with
// kappa = div(n_lg) = -div(n_f), n_f = grad_f / (|grad_f| + dN) and grad_f
// the mean of the two cells' Gauss gradients of alpha^{n+1} (the cell's own
// on a domain face; empty axes carry no face).  With a contact angle, a
// face between a clear and a porous cell carries the penalized normal of
// Sec. 2.3 instead: only its component along the face axis enters the
// divergence, -cos(theta) (n_w . e_axis) |n_f|, n_w from the porous into the
// clear cell.
__global__ void __launch_bounds__(NTHREADS) k_curvature(Segs SG, Phys Ph,
                                                        const double *__restrict__ gx,
                                                        const double *__restrict__ gy,
                                                        const double *__restrict__ gz,
                                                        const double *__restrict__ phi,
                                                        const double *__restrict__ kinv,
                                                        double *__restrict__ SK) {
  FOR_CELLS(SG, G, P) {
  const double gP[3] = {gx[P.c], gy[P.c], gz[P.c]};
  const bool pP = kinv[P.c] > 0.0;
  double div = 0.0;
#pragma unroll
  for (int a = 0; a < 3; a++) {
    if (G.n[a] == 1 && G.bck[2 * a] == BC_EMPTY) continue;
    const int st = stride_of(G, a);
    const int cm = on_boundary(G, P, a, 0) ? P.c : P.c - st;
    const int cp = on_boundary(G, P, a, 1) ? P.c : P.c + st;
    const double fm[3] = {0.5 * (gP[0] + gx[cm]), 0.5 * (gP[1] + gy[cm]), 0.5 * (gP[2] + gz[cm])};
    const double fp[3] = {0.5 * (gP[0] + gx[cp]), 0.5 * (gP[1] + gy[cp]), 0.5 * (gP[2] + gz[cp])};
    const double mm = sqrt(fm[0] * fm[0] + fm[1] * fm[1] + fm[2] * fm[2]);
    const double mp = sqrt(fp[0] * fp[0] + fp[1] * fp[1] + fp[2] * fp[2]);
    double nm = fm[a] / (mm + G.dN);
    double np = fp[a] / (mp + G.dN);
    if (Ph.ca_on) {
      // a domain face reads the cell itself: same porosity, no wall
      const bool pm = kinv[cm] > 0.0, pp = kinv[cp] > 0.0;
      if (pm != pP) nm = -Ph.cos_ca * (pm ? 1.0 : -1.0) * (mm / (mm + G.dN));
      if (pp != pP) np = -Ph.cos_ca * (pP ? 1.0 : -1.0) * (mp / (mp + G.dN));
    }
    div += (np - nm) * G.ih[a];
  }
  SK[P.c] = kinv[P.c] > 0.0 ? 0.0 : Ph.sigma * -div / phi[P.c];
  }
}

// only >= 0: that sample alone
__global__ void __launch_bounds__(NTHREADS) k_closures(Segs SG, Phys Ph,
                                                       const double *__restrict__ alpha,
                                                       const double *__restrict__ kinv,
                                                       double *__restrict__ ml,
                                                       double *__restrict__ mg,
                                                       double *__restrict__ pc,
                                                       double *__restrict__ cf, int only,
                                                       int base) {
  FOR_CELLS_ONE(SG, G, P, only, base) {
  double l, g, p;
  const double a = alpha[P.c];
  closures(Ph, a, l, g, p);
  ml[P.c] = l;
  mg[P.c] = g;
  const bool porous = kinv[P.c] > 0.0;
  pc[P.c] = porous ? p : 0.0;
  cf[P.c] = porous ? l / (l + g) - a : 0.0;
  }
}

// F = (linearly interpolated U) . S, boundary: inlet velocity, 0 at walls,
// the cell velocity at outlets.
// only >= 0: that sample alone
__global__ void __launch_bounds__(NTHREADS) k_init_flux(Segs SG, const double *__restrict__ U,
                                                        double *__restrict__ F, int only,
                                                        int base) {
  FOR_CELLS_ONE(SG, G, P, only, base) {
  for (int a = 0; a < 3; a++) {
    const double *Ua = U + (size_t)a * G.vs;
    for (int s = 0; s < 2; s++) {
      const bool bnd = on_boundary(G, P, a, s);
      if (s == 1 && !bnd) continue;
      const int f = face_of(G, P, a, s);
      double v = 0.0;
      if (!bnd) {
        v = 0.5 * (Ua[P.c - stride_of(G, a)] + Ua[P.c]) * G.area[a];
      } else {
        int kind = G.bck[2 * a + s];
        if (is_inlet(kind)) v = inlet_u(G, 2 * a + s, P.j, a) * G.area[a];
        else if (kind == BC_OUTLET) v = Ua[P.c] * G.area[a];
      }
      F[f] = v;
    }
  }
  }
}

// R+- of limiter iteration k (k = 1..M) alternate between (Rp, Rm) and
// (Pin, Pout); the face limiters of iteration k between lam and FB (which
// the momentum stage fills later in the step)
static double *R_buf(Handle *h, int k, int sign) {
  return ((k - 1) & 1) ? (sign ? h->Pin : h->Pout) : (sign ? h->Rp : h->Rm);
}
static double *lam_buf(Handle *h, int k) { return ((k - 1) & 1) ? h->FB : h->lam; }

void alpha_final_R(Handle *h, double **Rp, double **Rm) {
  *Rp = R_buf(h, h->ctl.mules_iter, 1);
  *Rm = R_buf(h, h->ctl.mules_iter, 0);
}

// One transport sub-cycle: alpha_in -> alpha_out with dt / nsub.
static void alpha_cycle(Handle *h, const double *ain, double *aout, int sub, int nsub,
                        double *aphi) {
  dim3 blk(BX, BY);
  const int M = h->ctl.mules_iter;
  // the cell gradients borrow HbyA, which the correctors fill later
  double *gx = h->HbyA, *gy = h->HbyA + h->NC, *gz = h->HbyA + 2 * h->NC;
  AlphaArgs X{ain, h->F, h->phi, h->kinv, h->prgh, h->ml, h->mg, h->pc, gx, gy, gz};
  DBS_LAUNCH(h, KC_ALPHA_FACE, k_alpha_grad, h->cgrid, blk, h->seg, X, gx, gy, gz, 0, 0.0);
  DBS_LAUNCH(h, KC_ALPHA_FACE, k_alpha_face, h->cgrid, blk, h->seg, h->P, X, h->A);
  DBS_LAUNCH(h, KC_ALPHA_BOUNDS, k_alpha_bounds, h->cgrid, blk, h->seg, ain,
             (const double *)h->F, (const double *)h->phi, (const double *)h->A, h->Qp, h->Qm,
             R_buf(h, 1, 1), R_buf(h, 1, 0), nsub);
  for (int k = 1; k < M; k++)
    DBS_LAUNCH(h, KC_ALPHA_LIMIT, k_alpha_iter, h->cgrid, blk, h->seg, (const double *)h->A,
               (const double *)R_buf(h, k, 1), (const double *)R_buf(h, k, 0),
               (const double *)lam_buf(h, k - 1), k == 1 ? 1 : 0, (const double *)h->Qp,
               (const double *)h->Qm, lam_buf(h, k), R_buf(h, k + 1, 1), R_buf(h, k + 1, 0));
  // the last iteration's face limiters are formed inside the update
  DBS_LAUNCH(h, KC_ALPHA_UPDATE, k_alpha_update, h->cgrid, blk, h->seg, h->P, ain,
             (const double *)h->F, (const double *)h->phi, (const double *)h->kinv,
             (const double *)h->A, (const double *)R_buf(h, M, 1),
             (const double *)R_buf(h, M, 0), (const double *)lam_buf(h, M - 1), M == 1 ? 1 : 0,
             aout, h->rhoPhi, h->ml, h->mg, h->pc, h->cf, sub, nsub, aphi);
}

// Buffer roles after the stage: the cycles alternate between alpha_old and
// alpha3 starting with alpha_old, alpha^n stays where it was (for rho^n)
void alpha_roles(Handle *h) {
  const int n = h->ctl.n_alpha_sub;
  double *src = h->alpha, *x = h->alpha_old, *y = h->alpha3;
  double *fin = (n & 1) ? x : y;
  h->alpha_old = src;
  h->alpha = fin;
  if (n > 1) h->alpha3 = fin == x ? y : x;
}

void alpha_stage(Handle *h, double *aphi) {
  dim3 blk(BX, BY);
  const int n = h->ctl.n_alpha_sub;
  const double *cur = h->alpha;
  for (int k = 0; k < n; k++) {
    // alpha^{n+1} goes to the spare buffers; alpha^n stays for rho^n
    double *dst = (k & 1) ? h->alpha3 : h->alpha_old;
    alpha_cycle(h, cur, dst, k, n, aphi);
    cur = dst;
  }
  alpha_roles(h);
  AlphaArgs X{h->alpha, h->F, h->phi, h->kinv, h->prgh, h->ml, h->mg, h->pc,
              nullptr, nullptr, nullptr};
  if (h->SK) {
    // surface tension coefficient from alpha^{n+1}; the gradients borrow
    // HbyA again (R+- of the last limiter iteration stay for the trace)
    AlphaArgs Xn = X;
    Xn.alpha = h->alpha;
    double *gx = h->HbyA, *gy = h->HbyA + h->NC, *gz = h->HbyA + 2 * h->NC;
    DBS_LAUNCH(h, KC_CURV, k_alpha_grad, h->cgrid, blk, h->seg, Xn, gx, gy, gz, h->P.ca_on,
               h->P.cot_ca);
    DBS_LAUNCH(h, KC_CURV, k_curvature, h->cgrid, blk, h->seg, h->P, (const double *)gx,
               (const double *)gy, (const double *)gz, (const double *)h->phi,
               (const double *)h->kinv, h->SK);
  }
}

// launch over every sample, or (only >= 0) over that sample's blocks alone
static dim3 one_grid(const Handle *h, int only, int &base) {
  base = only >= 0 ? h->cell.hbp[only] : 0;
  return only >= 0 ? dim3((unsigned)(h->cell.hbp[only + 1] - h->cell.hbp[only])) : h->cgrid;
}

void update_closures(Handle *h, int only) {
  dim3 blk(BX, BY);
  int base;
  const dim3 g = one_grid(h, only, base);
  DBS_LAUNCH(h, KC_MISC, k_closures, g, blk, h->seg, h->P, (const double *)h->alpha,
             (const double *)h->kinv, h->ml, h->mg, h->pc, h->cf, only, base);
}

void init_flux(Handle *h, int only) {
  dim3 blk(BX, BY);
  int base;
  const dim3 g = one_grid(h, only, base);
  DBS_LAUNCH(h, KC_MISC, k_init_flux, g, blk, h->seg, (const double *)h->U, h->F, only, base);
}

}  // namespace dbs
