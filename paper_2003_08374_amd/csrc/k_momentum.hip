// Momentum predictor and PISO correctors (Sec. 3.2, Eqs. (semi_discretised_bis),
// (corrected_velocity), (pressure_predictor)) in the p_rgh = p - rho g.x form.
//
// Per unit volume, cell P (1/phi factors of the inertial terms kept):
//   a_P = rho^{n+1}/(phi dt) + K + sum_f [max(out_f,0)/(phi_f phi V) + mu_f A/(h V)]
//   a_N = max(-out_f,0)/(phi_f phi V) + mu_f A/(h V)       (upwind convection)
//   S   = rho^n U^n/(phi dt) + div(mu grad(U)^T)|_{U^n} + boundary sources
// with K = k0^-1 / (k_rl/mu_l + k_rg/mu_g) the Darcy drag (Sec. 2.3 summary),
// out_f the outward mass flux rhoPhi.  Face forces
//   q_f = [F_c,f - (g.x_f) dn(rho) - dn(p_rgh)] A_f,
//   F_c = (f_l - alpha)[(rho_l - rho_g) g + grad p_c] - p_c grad alpha   (App. B)
// are reconstructed to cells as R(q)_x = (q_west + q_east)/(2 A_x).
// Quantities fixed within a step are formed once and stored: the neighbour
// coefficients a_N (6 per cell, by the assembly) for the three Jacobi sweeps
// and the two H evaluations, and the face body force F_c - (g.x_f) dn(rho)
// (one per face) for the assembly and both correctors; the kernels then
// read them instead of gathering phi, alpha, p_c and f_l - alpha of every
// neighbour.
#include "dbs_internal.h"

namespace dbs {

struct MomArgs {
  const double *__restrict__ alpha;      // alpha^{n+1}
  const double *__restrict__ alpha_old;  // alpha^n
  const double *__restrict__ rhoPhi;
  const double *__restrict__ phi, *__restrict__ kinv;
  const double *__restrict__ ml, *__restrict__ mg, *__restrict__ pc;
  const double *__restrict__ cf;  // f_l - alpha (porous), 0 (clear)
  const double *__restrict__ prgh;
  const double *__restrict__ rAU;
  const double *__restrict__ FB;  // face_body of each interior face (k_face_body)
  const double *__restrict__ sk;  // sigma kappa / phi (clear cells), NULL when sigma = 0
};

__device__ __forceinline__ bool empty_axis(const Geom &G, int a) {
  return G.n[a] == 1 && G.bck[2 * a] == BC_EMPTY;
}

__device__ __forceinline__ int nbr_of(const Geom &G, const Cell &P, int a, int s) {
  return P.c + (s ? 1 : -1) * stride_of(G, a);
}

// f_l - alpha in porous cells, 0 in clear cells
__device__ __forceinline__ double cap_coef(const MomArgs &M, int c) { return M.cf[c]; }

// body force per unit volume on the interior face between own (minus side)
// and nbr (plus side) along a: F_c - (g.x_f) dn(rho)
__device__ inline double face_body(const Geom &G, const Phys &Ph, const MomArgs &M, int own,
                                   int nbr, int a, double gxf) {
  const double ih = G.ih[a];
  const double ao = M.alpha[own], an = M.alpha[nbr];
  const double cf = 0.5 * (cap_coef(M, own) + cap_coef(M, nbr));
  const double pco = M.pc[own], pcn = M.pc[nbr];
  const double pcf = 0.5 * (pco + pcn);
  double Fcap =
      cf * ((Ph.rho_l - Ph.rho_g) * Ph.g[a] + (pcn - pco) * ih) - pcf * (an - ao) * ih;
  // clear-fluid CSF force: the face mean of sigma kappa / phi times dn(alpha)
  if (M.sk) Fcap += 0.5 * (M.sk[own] + M.sk[nbr]) * (an - ao) * ih;
  return Fcap - gxf * (rho_of(Ph, an) - rho_of(Ph, ao)) * ih;
}

// q on side s of P along a for interior and outlet faces (fixed-flux faces
// are handled by the caller); p_rgh from `prgh`.  BF: both forms are
// evaluated and one selected, so that the neighbour loads need no branch (a
// boundary side reads the cell itself for the interior form); faster where
// little else hides the load latency (the corrector), slower in the
// assembly.
template <bool BF = false>
__device__ inline double face_force(const Geom &G, const Phys &Ph, const MomArgs &M,
                                    const double *__restrict__ prgh, const Cell &P, int a,
                                    int s) {
  const double gxf = gdotx_face(G, Ph, P, a, s);
  if constexpr (BF) {
    const bool bnd = on_boundary(G, P, a, s);
    const int nb = bnd ? P.c : nbr_of(G, P, a, s);
    const int own = s ? P.c : nb, nbr = s ? nb : P.c;
    const double vi =
        (M.FB[face_of(G, P, a, s)] - (prgh[nbr] - prgh[own]) * G.ih[a]) * G.area[a];
    const double pb = G.bcp[2 * a + s] - rho_of(Ph, M.alpha[P.c]) * gxf;
    const double sn = s ? (pb - prgh[P.c]) * 2.0 * G.ih[a] : (prgh[P.c] - pb) * 2.0 * G.ih[a];
    return bnd ? -sn * G.area[a] : vi;
  }
  if (on_boundary(G, P, a, s)) {
    // outlet: fixed static pressure, p_rgh_b = p_b - rho_P g.x_b
    const double pb = G.bcp[2 * a + s] - rho_of(Ph, M.alpha[P.c]) * gxf;
    const double sn = s ? (pb - prgh[P.c]) * 2.0 * G.ih[a] : (prgh[P.c] - pb) * 2.0 * G.ih[a];
    return -sn * G.area[a];
  }
  const int nb = nbr_of(G, P, a, s);
  const int own = s ? P.c : nb, nbr = s ? nb : P.c;
  return (M.FB[face_of(G, P, a, s)] - (prgh[nbr] - prgh[own]) * G.ih[a]) * G.area[a];
}

__device__ __forceinline__ bool fixed_flux(const Geom &G, int b) {
  return G.bck[b] == BC_WALL || is_inlet(G.bck[b]);
}

// R(q)_a of cell P.  hbya == nullptr: predictor (a fixed-flux face copies the
// opposite face's force); otherwise corrector (a fixed-flux face carries the
// p_rgh gradient that reproduces its prescribed flux).
template <bool BF = false>
__device__ inline double reconstruct_axis(const Geom &G, const Phys &Ph, const MomArgs &M,
                                          const double *__restrict__ prgh,
                                          const double *__restrict__ hbya, const Cell &P,
                                          int a) {
  if (empty_axis(G, a)) return 0.0;
  double q[2];
  bool ff[2];
  for (int s = 0; s < 2; s++) {
    ff[s] = on_boundary(G, P, a, s) && fixed_flux(G, 2 * a + s);
    if (BF || !ff[s]) q[s] = face_force<BF>(G, Ph, M, prgh, P, a, s);
  }
  for (int s = 0; s < 2; s++) {
    if (!ff[s]) continue;
    if (hbya) {
      const int b = 2 * a + s;
      const double Fb = is_inlet(G.bck[b]) ? inlet_u(G, b, P.j, a) * G.area[a] : 0.0;
      q[s] = (Fb - hbya[(size_t)a * G.vs + P.c] * G.area[a]) / M.rAU[P.c];
    } else {
      q[s] = ff[1 - s] ? 0.0 : q[1 - s];
    }
  }
  return (q[0] + q[1]) / (2.0 * G.area[a]);
}

// momentum coefficient of side s of P along a
struct FaceCoef {
  double aN;      // neighbour coefficient (interior faces)
  double diag;    // contribution to a_P
  double src;     // multiplies the boundary velocity (inlet/wall sources)
  int nb;         // neighbour cell or -1
};

__device__ inline FaceCoef mom_face(const Geom &G, const Phys &Ph, const MomArgs &M,
                                    const Cell &P, int a, int s) {
  FaceCoef r{0.0, 0.0, 0.0, -1};
  const int f = face_of(G, P, a, s);
  const double rp = M.rhoPhi[f];
  const double out = s ? rp : -rp;
  const double phP = M.phi[P.c];
  if (!on_boundary(G, P, a, s)) {
    const int nb = nbr_of(G, P, a, s);
    const double phf = 0.5 * (phP + M.phi[nb]);
    const double vis =
        0.5 * (mu_of(Ph, M.alpha[P.c]) + mu_of(Ph, M.alpha[nb])) * G.area[a] * G.ih[a] * G.iV;
    const double conv = 1.0 / (phf * phP * G.V);
    r.diag = fmax(out, 0.0) * conv + vis;
    r.aN = fmax(-out, 0.0) * conv + vis;
    r.nb = nb;
    return r;
  }
  const int b = 2 * a + s;
  const double conv = 1.0 / (phP * phP * G.V);
  const double d2 = 2.0 * G.ih[a];  // 1 / (h/2)
  if (G.bck[b] == BC_WALL) {
    r.diag = mu_of(Ph, M.alpha[P.c]) * G.area[a] * d2 * G.iV;
  } else if (is_inlet(G.bck[b])) {
    const double vis = mu_of(Ph, inlet_alpha(G, b, P.j)) * G.area[a] * d2 * G.iV;
    if (out >= 0.0) r.diag = out * conv;
    else r.src = -out * conv;
    r.diag += vis;
    r.src += vis;
  } else if (G.bck[b] == BC_OUTLET) {
    r.diag = out * conv;
  }
  return r;
}

// dU_comp/dx_axis at cell Q (Gauss; boundary: wall 0, inlet U_b, outlet U_Q).
// Both neighbour loads are issued unconditionally (a boundary side reads the
// cell itself); the boundary value replaces the face value afterwards.
__device__ inline double dU(const Geom &G, const double *__restrict__ U, int Qc,
                             const int Qco[3], int comp, int axis) {
  const double *Uc = U + (size_t)comp * G.vs;
  const int st = stride_of(G, axis);
  const bool bm = Qco[axis] == 0, bp = Qco[axis] == G.n[axis] - 1;
  const double uq = Uc[Qc];
  const double um = Uc[bm ? Qc : Qc - st], up = Uc[bp ? Qc : Qc + st];
  double f0 = 0.5 * (uq + um), f1 = 0.5 * (uq + up);
  auto bval = [&](int b) -> double {
    if (G.bck[b] == BC_WALL) return 0.0;
    if (is_inlet(G.bck[b])) return inlet_u(G, b, Qco[1], comp);
    return uq;
  };
  if (bm) f0 = bval(2 * axis);
  if (bp) f1 = bval(2 * axis + 1);
  return empty_axis(G, axis) ? 0.0 : (f1 - f0) * G.ih[axis];
}

// rAU = 1/a_P, Sh, B = Sh + R(q), and the neighbour coefficients a_N of the
// six faces (face 2a+s; zero on boundary and empty faces) into AN, which
// every Jacobi sweep and H evaluation of the step reads
__global__ void __launch_bounds__(NTHREADS) k_mom_assemble(Segs SG, Phys Ph, MomArgs M,
                                                           const double *__restrict__ U,
                                                           int transpose,
                                                           double *__restrict__ rAU,
                                                           double *__restrict__ Sh,
                                                           double *__restrict__ B,
                                                           double *__restrict__ AN) {
  FOR_CELLS(SG, G, P) {
  const int c = P.c;
  const double phP = M.phi[c];
  const double an = M.alpha[c];
  const double mt = M.ml[c] + M.mg[c];
  const double K = M.kinv[c] > 0.0 ? M.kinv[c] / mt : 0.0;
  double aP = rho_of(Ph, an) / (phP * G.dt) + K;
  const double rho_o = rho_of(Ph, M.alpha_old[c]);
  double S[3];
  for (int d = 0; d < 3; d++) S[d] = rho_o * U[(size_t)d * G.vs + c] / (phP * G.dt);
  for (int a = 0; a < 3; a++) {
    if (empty_axis(G, a)) {
      AN[(size_t)(2 * a) * G.vs + c] = 0.0;
      AN[(size_t)(2 * a + 1) * G.vs + c] = 0.0;
      continue;
    }
    for (int s = 0; s < 2; s++) {
      FaceCoef fc = mom_face(G, Ph, M, P, a, s);
      AN[(size_t)(2 * a + s) * G.vs + c] = fc.aN;
      aP += fc.diag;
      if (fc.src != 0.0) {
        S[0] += fc.src * inlet_u(G, 2 * a + s, P.j, 0);
        S[1] += fc.src * inlet_u(G, 2 * a + s, P.j, 1);
        S[2] += fc.src * inlet_u(G, 2 * a + s, P.j, 2);
      }
    }
  }
  if (transpose) {
    // explicit div(mu grad(U)^T): face flux mu_f A dU_a/dx_i, outward sign.
    // The cell's own gradient is formed once; a boundary face evaluates its
    // "neighbour" at the cell itself and discards it.
    double gP[3][3];
#pragma unroll
    for (int a = 0; a < 3; a++)
#pragma unroll
      for (int i = 0; i < 3; i++) gP[a][i] = dU(G, U, c, P.co, a, i);
    const double muP = mu_of(Ph, an);
#pragma unroll
    for (int a = 0; a < 3; a++) {
      if (empty_axis(G, a)) continue;
#pragma unroll
      for (int s = 0; s < 2; s++) {
        const double sg = s ? 1.0 : -1.0;
        const bool bnd = on_boundary(G, P, a, s);
        const int nb = bnd ? c : nbr_of(G, P, a, s);
        int nco[3] = {P.co[0], P.co[1], P.co[2]};
        if (!bnd) nco[a] += s ? 1 : -1;
        double muf = 0.5 * (muP + mu_of(Ph, M.alpha[nb]));
        if (bnd) {
          const int b = 2 * a + s;
          muf = is_inlet(G.bck[b]) ? mu_of(Ph, inlet_alpha(G, b, P.j)) : muP;
        }
#pragma unroll
        for (int i = 0; i < 3; i++) {
          const double gN = dU(G, U, nb, nco, a, i);
          const double gf = bnd ? gP[a][i] : 0.5 * (gP[a][i] + gN);
          S[i] += sg * muf * G.area[a] * gf * G.iV;
        }
      }
    }
  }
  const double r = 1.0 / aP;
  rAU[c] = r;
  for (int d = 0; d < 3; d++) {
    Sh[(size_t)d * G.vs + c] = S[d];
    B[(size_t)d * G.vs + c] =
        S[d] + reconstruct_axis(G, Ph, M, M.prgh, nullptr, P, d);
  }
  }
}

// Uout = rAU (sum_N a_N Uin_N + src): one Jacobi sweep (src = S + R(q)) or
// HbyA (src = S), with the step's a_N from the assembly
__global__ void __launch_bounds__(NTHREADS) k_mom_offdiag(Segs SG, Phys Ph, MomArgs M,
                                                          const double *__restrict__ AN,
                                                          const double *__restrict__ Uin,
                                                          const double *__restrict__ src,
                                                          double *__restrict__ Uout) {
  FOR_CELLS(SG, G, P) {
  const int c = P.c;
  const size_t vs = (size_t)G.vs;
  // All six faces without branches: a boundary face reads the cell itself
  // with a zero weight, so every load can be issued at once.
  double aN[6], un[6][3];
#pragma unroll
  for (int a = 0; a < 3; a++) {
#pragma unroll
    for (int s = 0; s < 2; s++) {
      const int q = 2 * a + s;
      const bool interior = !empty_axis(G, a) && !on_boundary(G, P, a, s);
      const int nb = interior ? nbr_of(G, P, a, s) : c;
      aN[q] = empty_axis(G, a) ? 0.0 : AN[(size_t)q * vs + c];  // zero on an empty axis
#pragma unroll
      for (int d = 0; d < 3; d++) un[q][d] = Uin[(size_t)d * vs + nb];
    }
  }
  double acc[3] = {src[c], src[vs + c], src[2 * vs + c]};
#pragma unroll
  for (int q = 0; q < 6; q++)
#pragma unroll
    for (int d = 0; d < 3; d++) acc[d] += aN[q] * un[q][d];
  const double r = M.rAU[c];
  for (int d = 0; d < 3; d++) Uout[(size_t)d * vs + c] = r * acc[d];
  }
}

// One Jacobi sweep of the implicit predictor system a_P U - sum a_N U_N = B
// (Eq. (semi_discretised_bis)) for the samples still iterating (mact != 0;
// the blocks of the others return at once): Uout = rAU (B + sum a_N Uin_N),
// and per block the sum over the three components of the squared residual
// B + sum a_N Uin_N - Uin / rAU of the iterate the sweep starts from (and of
// B^2 in the first sweep) for the sample's convergence test.
__global__ void __launch_bounds__(NTHREADS) k_mom_jacobi(Segs SG, MomArgs M,
                                                         const double *__restrict__ AN,
                                                         const double *__restrict__ Uin,
                                                         const double *__restrict__ B,
                                                         double *__restrict__ Uout,
                                                         const int *__restrict__ mact,
                                                         double *__restrict__ part, int nb,
                                                         int first) {
  __shared__ double lds[2][NTHREADS / 64];
  const int cell_gb = xcd_remap(blockIdx.x, gridDim.x);
  const int cell_sg = find_seg(SG.bp, SG.ns, cell_gb);
  if (!mact[cell_sg]) return;  // uniform over the block: one sample per block
  const Geom &G = SG.g[cell_sg];
  Cell P;
  double r2 = 0.0, b2 = 0.0;
  if (cell_of_thread(G, cell_gb - SG.bp[cell_sg], P)) {
    const int c = P.c;
    const size_t vs = (size_t)G.vs;
    double aN[6], un[6][3];
#pragma unroll
    for (int a = 0; a < 3; a++) {
#pragma unroll
      for (int s = 0; s < 2; s++) {
        const int q = 2 * a + s;
        const bool interior = !empty_axis(G, a) && !on_boundary(G, P, a, s);
        const int nbc = interior ? nbr_of(G, P, a, s) : c;
        aN[q] = empty_axis(G, a) ? 0.0 : AN[(size_t)q * vs + c];  // zero on an empty axis
#pragma unroll
        for (int d = 0; d < 3; d++) un[q][d] = Uin[(size_t)d * vs + nbc];
      }
    }
    const double rau = M.rAU[c];
#pragma unroll
    for (int d = 0; d < 3; d++) {
      const double bd = B[(size_t)d * vs + c];
      double acc = bd;
#pragma unroll
      for (int q = 0; q < 6; q++) acc += aN[q] * un[q][d];
      const double r = acc - Uin[(size_t)d * vs + c] / rau;
      r2 += r * r;
      b2 += bd * bd;
      Uout[(size_t)d * vs + c] = rau * acc;
    }
  }
  r2 = wave_sum(r2);
  b2 = wave_sum(b2);
  const int t = threadIdx.x + BX * threadIdx.y;
  if ((t & 63) == 0) {
    lds[0][t >> 6] = r2;
    lds[1][t >> 6] = b2;
  }
  __syncthreads();
  if (t == 0) {
    double sr = 0.0, sb = 0.0;
    for (int w = 0; w < NTHREADS / 64; w++) {
      sr += lds[0][w];
      sb += lds[1][w];
    }
    part[cell_gb] = sr;
    if (first) part[nb + cell_gb] = sb;
  }
}

// One block per sample after a predictor sweep: the sample's residual sum
// (and ||B||^2 after the first sweep) decides whether it iterates on.  The
// flags go to slot `slot` of host-mapped memory for the host's stopping test
// and the record {||B||^2, sweeps, relative residual, converged} to the
// device and host-mapped records.
__global__ void __launch_bounds__(1024) k_mom_final(const double *__restrict__ part, int nb,
                                                    const int *__restrict__ bp, int ns,
                                                    int *__restrict__ mact,
                                                    double *__restrict__ msc,
                                                    double *__restrict__ hmsc,
                                                    int *__restrict__ hflag, int slot,
                                                    double tol2, int maxit, int first) {
  __shared__ double lds[2][16];
  const int s = blockIdx.x, t = threadIdx.x;
  double *R = msc + (size_t)s * NMSC;
  if (!mact[s]) {
    if (t == 0) hflag[slot * ns + s] = 0;
    return;
  }
  double v2[2] = {0.0, 0.0};
  if (first) strided_sums<2>(part, (size_t)nb, bp[s], bp[s + 1], v2);
  else strided_sums<1>(part, (size_t)nb, bp[s], bp[s + 1], v2);
  double vr = v2[0], vb = v2[1];
  vr = wave_sum(vr);
  vb = wave_sum(vb);
  if ((t & 63) == 0) {
    lds[0][t >> 6] = vr;
    lds[1][t >> 6] = vb;
  }
  __syncthreads();
  if (t != 0) return;
  double r2 = 0.0, b2 = 0.0;
  for (int w = 0; w < 16; w++) {
    r2 += lds[0][w];
    b2 += lds[1][w];
  }
  if (first) R[0] = b2;
  b2 = R[0];
  const double sweeps = first ? 1.0 : R[1] + 1.0;
  R[1] = sweeps;
  R[2] = b2 > 0.0 ? sqrt(r2 / b2) : 0.0;
  const bool conv = r2 <= tol2 * b2;
  R[3] = conv ? 1.0 : 0.0;
  const int on = (conv || sweeps >= (double)maxit) ? 0 : 1;
  mact[s] = on;
  hflag[slot * ns + s] = on;
  for (int q = 0; q < NMSC; q++) hmsc[(size_t)s * NMSC + q] = R[q];
}

// before the sweeps: every sample iterates, its record is cleared
__global__ void k_mom_init(int *__restrict__ mact, double *__restrict__ msc, int ns, int on) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  mact[s] = on;
  for (int q = 0; q < NMSC; q++) msc[(size_t)s * NMSC + q] = 0.0;
}

// After the sweeps: a sample that made n sweeps ended in X (n odd), Y (n
// even) or, without sweeps, in Un; the samples whose buffer is not `to`
// copy their cells there, so that every sample's predicted velocity is in
// `to` (Un itself is never written).
__global__ void __launch_bounds__(NTHREADS) k_mom_gather(Segs SG, const double *__restrict__ msc,
                                                         const double *__restrict__ Un,
                                                         const double *__restrict__ X,
                                                         const double *__restrict__ Y,
                                                         double *__restrict__ to) {
  const int cell_gb = xcd_remap(blockIdx.x, gridDim.x);
  const int cell_sg = find_seg(SG.bp, SG.ns, cell_gb);
  const int n = (int)msc[(size_t)cell_sg * NMSC + 1];
  const double *src = n == 0 ? Un : ((n & 1) ? X : Y);
  if (src == to) return;
  const Geom &G = SG.g[cell_sg];
  Cell P;
  if (cell_of_thread(G, cell_gb - SG.bp[cell_sg], P))
    for (int d = 0; d < 3; d++) to[(size_t)d * G.vs + P.c] = src[(size_t)d * G.vs + P.c];
}

// phiHbyA on the cell's faces and the pressure right-hand side
// b = -sum_out phiHbyA + sum_outlet T_b p_rgh_b
__device__ inline double phi_hbya(const Geom &G, const Phys &Ph, const MomArgs &M,
                                  const double *__restrict__ H, const Cell &P, int a, int s) {
  if (on_boundary(G, P, a, s)) {
    const int b = 2 * a + s;
    if (is_inlet(G.bck[b])) return inlet_u(G, b, P.j, a) * G.area[a];
    if (G.bck[b] == BC_OUTLET) return H[(size_t)a * G.vs + P.c] * G.area[a];
    return 0.0;
  }
  const int nb = nbr_of(G, P, a, s);
  const int own = s ? P.c : nb, nbr = s ? nb : P.c;
  const double *Ha = H + (size_t)a * G.vs;
  const double rAUf = 0.5 * (M.rAU[own] + M.rAU[nbr]);
  return 0.5 * (Ha[own] + Ha[nbr]) * G.area[a] +
         rAUf * M.FB[face_of(G, P, a, s)] * G.area[a];
}

__global__ void __launch_bounds__(NTHREADS) k_phihbya(Segs SG, Phys Ph, MomArgs M,
                                                      const double *__restrict__ H,
                                                      double *__restrict__ phiH,
                                                      double *__restrict__ rhs) {
  FOR_CELLS(SG, G, P) {
  double div = 0.0, dir = 0.0;
  for (int a = 0; a < 3; a++) {
    const bool empty = empty_axis(G, a);
    for (int s = 0; s < 2; s++) {
      const int f = face_of(G, P, a, s);
      const bool bnd = on_boundary(G, P, a, s);
      const double v = empty ? 0.0 : phi_hbya(G, Ph, M, H, P, a, s);
      if (s == 0 || bnd) phiH[f] = v;
      div += s ? v : -v;
      if (bnd && !empty && G.bck[2 * a + s] == BC_OUTLET) {
        const double pb = G.bcp[2 * a + s] -
                          rho_of(Ph, M.alpha[P.c]) * gdotx_face(G, Ph, P, a, s);
        dir += M.rAU[P.c] * G.area[a] * 2.0 * G.ih[a] * pb;
      }
    }
  }
  rhs[P.c] = -div + dir;
  }
}

// flux and velocity correction; last corrector also writes p = p_rgh + rho g.x
__global__ void __launch_bounds__(NTHREADS) k_correct(Segs SG, Phys Ph, MomArgs M,
                                                      const double *__restrict__ H,
                                                      const double *__restrict__ phiH,
                                                      double *__restrict__ F,
                                                      double *__restrict__ U,
                                                      double *__restrict__ p, int last) {
  FOR_CELLS(SG, G, P) {
  const int c = P.c;
  const double *prgh = M.prgh;
  // the minus face of every axis (interior: the neighbour's loads are issued
  // without a branch), and the plus face where it is a domain boundary
  auto bflux = [&](int a, int s, double v) {
    if (G.bck[2 * a + s] == BC_OUTLET) {
      const double pb = G.bcp[2 * a + s] - rho_of(Ph, M.alpha[c]) * gdotx_face(G, Ph, P, a, s);
      const double Tb = M.rAU[c] * G.area[a] * 2.0 * G.ih[a];
      v -= s ? Tb * (pb - prgh[c]) : Tb * (prgh[c] - pb);
    }
    return v;
  };
  for (int a = 0; a < 3; a++) {
    const bool bnd = on_boundary(G, P, a, 0);
    const int own = bnd ? c : c - stride_of(G, a);
    const int f = face_of(G, P, a, 0);
    const double v = phiH[f];
    const double T = 0.5 * (M.rAU[own] + M.rAU[c]) * G.area[a] * G.ih[a];
    const double vi = v - T * (prgh[c] - prgh[own]);
    F[f] = bnd ? bflux(a, 0, v) : vi;
    if (on_boundary(G, P, a, 1)) {
      const int f1 = face_of(G, P, a, 1);
      F[f1] = bflux(a, 1, phiH[f1]);
    }
  }
  const double r = M.rAU[c];
  for (int d = 0; d < 3; d++)
    U[(size_t)d * G.vs + c] =
        H[(size_t)d * G.vs + c] + r * reconstruct_axis<true>(G, Ph, M, prgh, H, P, d);
  if (last) p[c] = prgh[c] + rho_of(Ph, M.alpha[c]) * gdotx_cell(G, Ph, P);
  }
}

static MomArgs mom_args(Handle *h) {
  return MomArgs{h->alpha, h->alpha_old, h->rhoPhi, h->phi,  h->kinv, h->ml,
                 h->mg,    h->pc,        h->cf,     h->prgh, h->rAU,  h->FB,
                 h->SK};
}

// FB = face_body on every interior face (each cell its minus faces), zero
// on domain faces: alpha, p_c and f_l - alpha are fixed within a step, so
// the assembly and both correctors read it instead of gathering them
__global__ void __launch_bounds__(NTHREADS) k_face_body(Segs SG, Phys Ph, MomArgs M,
                                                        double *__restrict__ FB) {
  FOR_CELLS(SG, G, P) {
  for (int a = 0; a < 3; a++) {
    const int f0 = face_of(G, P, a, 0);
    if (on_boundary(G, P, a, 0))
      FB[f0] = 0.0;
    else
      FB[f0] = face_body(G, Ph, M, P.c - stride_of(G, a), P.c, a, gdotx_face(G, Ph, P, a, 0));
    if (on_boundary(G, P, a, 1)) FB[face_of(G, P, a, 1)] = 0.0;
  }
  }
}

// The predictor: assembly, then Jacobi sweeps until every sample's starting
// residual is at most mom_tol ||B|| (or mom_maxit sweeps).  U^n stays
// untouched (a graph step redone eagerly starts from it again): sweep 0
// reads it and writes X = U2, later sweeps alternate between X and Y = U3.
// A sample that has converged skips the later sweeps, so its result sits in
// X or Y by the parity of its sweep count, and a last gather brings every
// sample into one of them, which becomes U; U^n becomes U3.  Eager: the
// flags of sweep k are read by the host (host-mapped memory, one event per
// sweep) while sweep k + 1 is already queued, so the device never drains;
// the sweep launched past the last convergence finds no sample iterating.
// Budgeted (graph capture): exactly `budget` sweeps, no host reads.
void momentum_predictor(Handle *h, int budget) {
  dim3 blk(BX, BY);
  MomArgs M = mom_args(h);
  DBS_LAUNCH(h, KC_MOM_ASSEMBLE, k_face_body, h->cgrid, blk, h->seg, h->P, M, h->FB);
  DBS_LAUNCH(h, KC_MOM_ASSEMBLE, k_mom_assemble, h->cgrid, blk, h->seg, h->P, M,
             (const double *)h->U, h->ctl.transpose_visc, h->rAU, h->Sh, h->B, h->AN);
  const int maxit = h->ctl.mom_maxit;
  const int ns = h->ns;
  DBS_LAUNCH(h, KC_MISC, k_mom_init, dim3((ns + 255) / 256), dim3(256), h->mact, h->msc, ns,
             maxit > 0 ? 1 : 0);
  h->mom_last = 0;
  if (maxit <= 0) {
    // U* = U^n, copied, so that U^n itself stays untouched
    DBS_LAUNCH(h, KC_MISC, k_mom_gather, h->cgrid, blk, h->seg, (const double *)h->msc,
               (const double *)h->U, (const double *)h->U2, (const double *)h->U3, h->U2);
    double *Un = h->U;
    h->U = h->U2;
    h->U2 = h->U3;
    h->U3 = Un;
    return;
  }
  const double tol2 = h->ctl.mom_tol * h->ctl.mom_tol;
  const int nb = h->cell.nblk;
  double *Un = h->U, *X = h->U2, *Y = h->U3;
  const bool graph = budget > 0;
  const int kmax = graph ? budget : maxit;
  int K = 0, par = -1;
  for (int k = 0; k < kmax; k++) {
    const double *in = k == 0 ? Un : ((k & 1) ? X : Y);
    double *out = (k & 1) ? Y : X;
    DBS_LAUNCH(h, KC_MOM_OFFDIAG, k_mom_jacobi, h->cgrid, blk, h->seg, M, (const double *)h->AN,
               in, (const double *)h->B, out, (const int *)h->mact, h->partials, nb,
               k == 0 ? 1 : 0);
    DBS_LAUNCH(h, KC_MISC, k_mom_final, dim3(ns), dim3(1024), (const double *)h->partials, nb,
               (const int *)h->cell.bp, ns, h->mact, h->msc, h->dmsc, h->dmflag, k & 1, tol2,
               maxit, k == 0 ? 1 : 0);
    K = k + 1;
    if (graph) continue;
    (void)hipEventRecord(h->mom_ev[k & 1], h->stream);
    if (k >= 1) {
      (void)hipEventSynchronize(h->mom_ev[(k - 1) & 1]);
      int on = 0;
      for (int s = 0; s < ns; s++) on += h->hmflag[((k - 1) & 1) * ns + s];
      if (!on) {
        // every sample stopped after sweep k - 1: the last one to stop made
        // k sweeps, and sweep k was a no-op
        par = k & 1;
        break;
      }
    }
  }
  if (par < 0) par = K & 1;
  h->mom_last = K;
  double *to = par ? X : Y;  // where a sample of K (resp. k) sweeps ended
  // single sample stopped by the host test: it already sits in `to`
  if (!(ns == 1 && !graph && K < kmax))
    DBS_LAUNCH(h, KC_MISC, k_mom_gather, h->cgrid, blk, h->seg, (const double *)h->msc,
               (const double *)Un, (const double *)X, (const double *)Y, to);
  h->U = to;
  h->U2 = to == X ? Y : X;
  h->U3 = Un;
}

void momentum_results(Handle *h, int *sweeps, double *relres, int *converged) {
  for (int s = 0; s < h->ns; s++) {
    const double *R = h->hmsc + (size_t)s * NMSC;
    if (sweeps) sweeps[s] = (int)R[1];
    if (relres) relres[s] = R[2];
    if (converged) converged[s] = R[3] != 0.0 || h->ctl.mom_maxit <= 0;
  }
}

void corrector_assemble(Handle *h) {
  dim3 blk(BX, BY);
  MomArgs M = mom_args(h);
  DBS_LAUNCH(h, KC_MOM_OFFDIAG, k_mom_offdiag, h->cgrid, blk, h->seg, h->P, M,
             (const double *)h->AN, (const double *)h->U, (const double *)h->Sh, h->HbyA);
  DBS_LAUNCH(h, KC_PHIHBYA, k_phihbya, h->cgrid, blk, h->seg, h->P, M, (const double *)h->HbyA,
             h->phiH, h->rhs);
}

// the corrected fluxes go to F2 (F^n stays for a redone graph step); the
// step swaps F and F2 after its last corrector
void corrector_update(Handle *h, bool last) {
  dim3 blk(BX, BY);
  MomArgs M = mom_args(h);
  DBS_LAUNCH(h, KC_CORRECT, k_correct, h->cgrid, blk, h->seg, h->P, M, (const double *)h->HbyA,
             (const double *)h->phiH, h->F2, h->U, h->p, (int)last);
}

}  // namespace dbs
