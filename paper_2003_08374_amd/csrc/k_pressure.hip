// Pressure solve of the PISO corrector: the SPD system
//   sum_f T_f (x_P - x_N) + sum_outlet T_b x_P = b,
//   T_f = mean(rAU) A_f / h (interior faces), T_b = rAU_P A / (h/2) (outlets),
// i.e. -div(rAU grad p_rgh) of Eq. (pressure_predictor), by conjugate gradients
// preconditioned with one geometric-multigrid V-cycle (the paper uses a
// geometric-algebraic multigrid solver, Sec. 3.2).
//
// Hierarchy: cell-centred 2x2x2 aggregation (ceil(n/2) per axis, ragged odd
// edges).  The fine operator is never stored: kernels rebuild T_f from rAU
// (8 B per cell instead of 32).  Coarse operators store the +x/+y/+z face
// coefficient of each cell, the outlet part of the diagonal and the diagonal;
// a coarse face coefficient is half the sum of the fine ones it covers (the
// h-doubling of a rediscretised operator).  Smoother: red-black Gauss-Seidel,
// red then black on the way down and black then red on the way up, so the
// V-cycle is a symmetric preconditioner.  Restriction sums the 8 children's
// residuals (transpose of piecewise-constant prolongation).
//
// Mixed precision (DBS_MIXED): the V-cycle runs in FP32 (rAU, coefficients,
// residual, correction); the CG vectors, dot products and the convergence
// test stay FP64; CG becomes flexible (Polak-Ribiere beta) and the true FP64
// residual b - A x replaces the recursive one every few iterations.
//
// Reductions are deterministic: each block writes one partial sum, a single
// block adds the partials in a fixed order.
#include <type_traits>

#include "dbs_internal.h"

namespace dbs {

enum { S_RZ = 0, S_PQ, S_RR, S_ALPHA, S_BETA, S_RZNEW, S_RZOLD, S_BB, S_SUM, S_NSCAL };

__device__ __forceinline__ bool red(int i, int j, int k) { return ((i + j + k) & 1) == 0; }

// ----------------------------------------------------------- fine level (0)

template <typename R>
struct Row0 {
  R D, T[6];
  int nb[6];
};

// row of the fine operator, rebuilt from rAU
template <typename R>
__device__ __forceinline__ void row0(const Geom &G, const R *__restrict__ rAU, const Cell &P,
                                     Row0<R> &w) {
  const R rP = rAU[P.c];
  R D = 0;
  for (int a = 0; a < 3; a++) {
    const R ca = (R)(G.area[a] * G.ih[a]);
    for (int s = 0; s < 2; s++) {
      const int q = 2 * a + s;
      if (on_boundary(G, P, a, s)) {
        w.nb[q] = -1;
        w.T[q] = 0;
        if (G.bck[q] == BC_OUTLET) D += rP * ca * (R)2;
      } else {
        const int nb = P.c + (s ? 1 : -1) * stride_of(G, a);
        w.nb[q] = nb;
        w.T[q] = (R)0.5 * (rP + rAU[nb]) * ca;
        D += w.T[q];
      }
    }
  }
  w.D = D;
}

template <typename R, typename X>
__device__ __forceinline__ R offsum(const Row0<R> &w, const X *__restrict__ x) {
  R s = 0;
  for (int q = 0; q < 6; q++)
    if (w.nb[q] >= 0) s += w.T[q] * (R)x[w.nb[q]];
  return s;
}

// q = A p, partial sum of p.q
__global__ void __launch_bounds__(NTHREADS) k_spmv0_dot(Geom G, const double *__restrict__ rAU,
                                                        const double *__restrict__ p,
                                                        double *__restrict__ q,
                                                        double *__restrict__ partials) {
  __shared__ double lds[NTHREADS / 64];
  Cell P;
  double v = 0.0;
  if (cell_from_thread(G, P)) {
    Row0<double> w;
    row0(G, rAU, P, w);
    const double pp = p[P.c];
    const double y = w.D * pp - offsum(w, p);
    q[P.c] = y;
    v = pp * y;
  }
  double s = block_sum(v, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    partials[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = s;
}

// r = b - A x, partial sum of r.r and of b.b
__global__ void __launch_bounds__(NTHREADS) k_resid0(Geom G, const double *__restrict__ rAU,
                                                     const double *__restrict__ b,
                                                     const double *__restrict__ x,
                                                     double *__restrict__ r,
                                                     double *__restrict__ partials, int nb2) {
  __shared__ double lds[NTHREADS / 64];
  Cell P;
  double v = 0.0, vb = 0.0;
  if (cell_from_thread(G, P)) {
    Row0<double> w;
    row0(G, rAU, P, w);
    const double rr = b[P.c] - (w.D * x[P.c] - offsum(w, x));
    r[P.c] = rr;
    v = rr * rr;
    vb = b[P.c] * b[P.c];
  }
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  double s = block_sum(v, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[bid] = s;
  __syncthreads();
  s = block_sum(vb, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[nb2 + bid] = s;
}

// x += alpha p, r -= alpha q, partial sum of r.r
__global__ void __launch_bounds__(NTHREADS) k_axpy_dot(Geom G, const double *__restrict__ scal,
                                                       const double *__restrict__ p,
                                                       const double *__restrict__ q,
                                                       double *__restrict__ x,
                                                       double *__restrict__ r,
                                                       double *__restrict__ partials) {
  __shared__ double lds[NTHREADS / 64];
  Cell P;
  double v = 0.0;
  if (cell_from_thread(G, P)) {
    const double al = scal[S_ALPHA];
    x[P.c] = fma(al, p[P.c], x[P.c]);
    const double rr = fma(-al, q[P.c], r[P.c]);
    r[P.c] = rr;
    v = rr * rr;
  }
  double s = block_sum(v, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    partials[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = s;
}

// partial sums of r.z and (flexible) r.zold
template <typename Z>
__global__ void __launch_bounds__(NTHREADS) k_dot_rz(Geom G, const double *__restrict__ r,
                                                     const Z *__restrict__ z,
                                                     const Z *__restrict__ zold,
                                                     double *__restrict__ partials, int nb2) {
  __shared__ double lds[NTHREADS / 64];
  Cell P;
  double v = 0.0, vo = 0.0;
  if (cell_from_thread(G, P)) {
    v = r[P.c] * (double)z[P.c];
    if (zold) vo = r[P.c] * (double)zold[P.c];
  }
  const int bid = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  double s = block_sum(v, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0) partials[bid] = s;
  if (zold) {
    __syncthreads();
    s = block_sum(vo, lds);
    if (threadIdx.x == 0 && threadIdx.y == 0) partials[nb2 + bid] = s;
  }
}

// p = z + beta p (first: p = z); flexible CG keeps zold = z
template <typename Z>
__global__ void __launch_bounds__(NTHREADS) k_xpby(Geom G, const double *__restrict__ scal,
                                                   const Z *__restrict__ z,
                                                   double *__restrict__ p, int first,
                                                   Z *__restrict__ zold) {
  Cell P;
  if (!cell_from_thread(G, P)) return;
  const double zz = (double)z[P.c];
  p[P.c] = first ? zz : fma(scal[S_BETA], p[P.c], zz);
  if (zold) zold[P.c] = z[P.c];
}

enum { FIN_STORE = 0, FIN_ALPHA = 1, FIN_BETA = 2, FIN_BETA_FLEX = 3 };

// one block: scal[slot] = sum(partials[0..n)) (and scal[slot2] from the
// second half); then derive alpha or beta on the device
__global__ void __launch_bounds__(1024) k_finalize(const double *__restrict__ partials, int n,
                                                   int two, double *__restrict__ scal, int slot,
                                                   int slot2, int op) {
  __shared__ double lds[16];
  const int t = threadIdx.x;
  for (int h = 0; h < (two ? 2 : 1); h++) {
    double v = 0.0;
    for (int i = t; i < n; i += 1024) v += partials[h * n + i];
    v = wave_sum(v);
    if ((t & 63) == 0) lds[t >> 6] = v;
    __syncthreads();
    if (t == 0) {
      double s = 0.0;
      for (int w = 0; w < 16; w++) s += lds[w];
      scal[h ? slot2 : slot] = s;
    }
    __syncthreads();
  }
  if (t == 0) {
    if (op == FIN_ALPHA) {
      const double pq = scal[S_PQ];
      scal[S_ALPHA] = pq != 0.0 ? scal[S_RZ] / pq : 0.0;
    } else if (op == FIN_BETA || op == FIN_BETA_FLEX) {
      const double num = op == FIN_BETA ? scal[S_RZNEW] : scal[S_RZNEW] - scal[S_RZOLD];
      scal[S_BETA] = scal[S_RZ] != 0.0 ? num / scal[S_RZ] : 0.0;
      scal[S_RZ] = scal[S_RZNEW];
    }
  }
}

// partial sums of x (mean removal in closed domains)
__global__ void __launch_bounds__(NTHREADS) k_sum(Geom G, const double *__restrict__ x,
                                                  double *__restrict__ partials) {
  __shared__ double lds[NTHREADS / 64];
  Cell P;
  double v = 0.0;
  if (cell_from_thread(G, P)) v = x[P.c];
  double s = block_sum(v, lds);
  if (threadIdx.x == 0 && threadIdx.y == 0)
    partials[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = s;
}

__global__ void __launch_bounds__(NTHREADS) k_sub_mean(Geom G, const double *__restrict__ scal,
                                                       double *__restrict__ x) {
  Cell P;
  if (!cell_from_thread(G, P)) return;
  x[P.c] -= scal[S_SUM] / (double)G.nc;
}

template <typename R>
__global__ void __launch_bounds__(NTHREADS) k_cast(Geom G, const double *__restrict__ in,
                                                   R *__restrict__ out) {
  Cell P;
  if (!cell_from_thread(G, P)) return;
  out[P.c] = (R)in[P.c];
}

// red-black Gauss-Seidel half sweep on the fine level; zero_init: x = b/D on
// this colour and 0 on the other (first half sweep from a zero guess)
template <typename R, typename B>
__global__ void __launch_bounds__(NTHREADS) k_smooth0(Geom G, const R *__restrict__ rAU,
                                                      const B *__restrict__ b,
                                                      R *__restrict__ x, int color,
                                                      int zero_init) {
  Cell P;
  if (!cell_from_thread(G, P)) return;
  const bool mine = red(P.i, P.j, P.k) == (color == 0);
  if (zero_init) {
    if (!mine) { x[P.c] = 0; return; }
    Row0<R> w;
    row0(G, rAU, P, w);
    x[P.c] = w.D > 0 ? (R)b[P.c] / w.D : (R)0;
    return;
  }
  if (!mine) return;
  Row0<R> w;
  row0(G, rAU, P, w);
  x[P.c] = w.D > 0 ? ((R)b[P.c] + offsum(w, x)) / w.D : (R)0;
}

// coarse right-hand side: sum over the 8 children of the fine residual
template <typename R, typename B>
__global__ void __launch_bounds__(NTHREADS) k_restrict0(Geom G, int cn0, int cn1, int cn2,
                                                        const R *__restrict__ rAU,
                                                        const B *__restrict__ b,
                                                        const R *__restrict__ x,
                                                        R *__restrict__ bc) {
  const int I = blockIdx.x * BX + threadIdx.x, J = blockIdx.y * BY + threadIdx.y,
            K = blockIdx.z;
  if (I >= cn0 || J >= cn1) return;
  R s = 0;
  for (int dk = 0; dk < 2; dk++)
    for (int dj = 0; dj < 2; dj++)
      for (int di = 0; di < 2; di++) {
        Cell P;
        P.i = 2 * I + di; P.j = 2 * J + dj; P.k = 2 * K + dk;
        if (P.i >= G.n[0] || P.j >= G.n[1] || P.k >= G.n[2]) continue;
        P.co[0] = P.i; P.co[1] = P.j; P.co[2] = P.k;
        P.c = cidx(G, P.i, P.j, P.k);
        Row0<R> w;
        row0(G, rAU, P, w);
        s += (R)b[P.c] - (w.D * x[P.c] - offsum(w, x));
      }
  bc[I + cn0 * (J + cn1 * K)] = s;
}

// ---------------------------------------------------------- coarse levels

template <typename R>
struct LV {
  int n0, n1, n2;
  const R *Tx, *Ty, *Tz, *D;
};

template <typename R>
__device__ __forceinline__ R coarse_off(const LV<R> &L, int i, int j, int k, int c,
                                        const R *__restrict__ x) {
  R s = 0;
  const int sy = L.n0, sz = L.n0 * L.n1;
  if (i + 1 < L.n0) s += L.Tx[c] * x[c + 1];
  if (i > 0) s += L.Tx[c - 1] * x[c - 1];
  if (j + 1 < L.n1) s += L.Ty[c] * x[c + sy];
  if (j > 0) s += L.Ty[c - sy] * x[c - sy];
  if (k + 1 < L.n2) s += L.Tz[c] * x[c + sz];
  if (k > 0) s += L.Tz[c - sz] * x[c - sz];
  return s;
}

template <typename R>
__global__ void __launch_bounds__(NTHREADS) k_smoothc(LV<R> L, const R *__restrict__ b,
                                                      R *__restrict__ x, int color,
                                                      int zero_init) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y,
            k = blockIdx.z;
  if (i >= L.n0 || j >= L.n1) return;
  const int c = i + L.n0 * (j + L.n1 * k);
  const bool mine = red(i, j, k) == (color == 0);
  const R D = L.D[c];
  if (zero_init) {
    x[c] = mine && D > 0 ? b[c] / D : (R)0;
    return;
  }
  if (!mine) return;
  x[c] = D > 0 ? (b[c] + coarse_off(L, i, j, k, c, x)) / D : (R)0;
}

template <typename R>
__global__ void __launch_bounds__(NTHREADS) k_restrictc(LV<R> L, int cn0, int cn1, int cn2,
                                                        const R *__restrict__ b,
                                                        const R *__restrict__ x,
                                                        R *__restrict__ bc) {
  const int I = blockIdx.x * BX + threadIdx.x, J = blockIdx.y * BY + threadIdx.y,
            K = blockIdx.z;
  if (I >= cn0 || J >= cn1) return;
  R s = 0;
  for (int dk = 0; dk < 2; dk++)
    for (int dj = 0; dj < 2; dj++)
      for (int di = 0; di < 2; di++) {
        const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
        if (i >= L.n0 || j >= L.n1 || k >= L.n2) continue;
        const int c = i + L.n0 * (j + L.n1 * k);
        s += b[c] - (L.D[c] * x[c] - coarse_off(L, i, j, k, c, x));
      }
  bc[I + cn0 * (J + cn1 * K)] = s;
}

// x_fine += x_coarse(parent)
template <typename R>
__global__ void __launch_bounds__(NTHREADS) k_prolong(int n0, int n1, int n2, int cn0, int cn1,
                                                      const R *__restrict__ xc,
                                                      R *__restrict__ x) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y,
            k = blockIdx.z;
  if (i >= n0 || j >= n1) return;
  x[i + n0 * (j + n1 * k)] += xc[(i >> 1) + cn0 * ((j >> 1) + cn1 * (k >> 1))];
}

// coarsest level: symmetric red-black sweeps by one block
template <typename R>
__global__ void __launch_bounds__(1024) k_coarse_solve(LV<R> L, const R *__restrict__ b,
                                                       R *__restrict__ x, int sweeps) {
  const int n = L.n0 * L.n1 * L.n2;
  for (int c = threadIdx.x; c < n; c += blockDim.x) x[c] = 0;
  __syncthreads();
  for (int sw = 0; sw < 2 * sweeps; sw++) {
    for (int h = 0; h < 2; h++) {
      // forward sweeps red,black; backward sweeps black,red
      const int color = (sw < sweeps) ? h : 1 - h;
      for (int c = threadIdx.x; c < n; c += blockDim.x) {
        const int i = c % L.n0, j = (c / L.n0) % L.n1, k = c / (L.n0 * L.n1);
        if (red(i, j, k) != (color == 0)) continue;
        const R D = L.D[c];
        x[c] = D > 0 ? (b[c] + coarse_off(L, i, j, k, c, x)) / D : (R)0;
      }
      __syncthreads();
    }
  }
}

// level-1 operator from the fine rAU
template <typename R>
__global__ void __launch_bounds__(NTHREADS) k_build_coarse0(Geom G, const double *__restrict__ rAU,
                                                            int cn0, int cn1, int cn2,
                                                            R *__restrict__ Tx, R *__restrict__ Ty,
                                                            R *__restrict__ Tz,
                                                            R *__restrict__ Db) {
  const int I = blockIdx.x * BX + threadIdx.x, J = blockIdx.y * BY + threadIdx.y,
            K = blockIdx.z;
  if (I >= cn0 || J >= cn1) return;
  double tx = 0, ty = 0, tz = 0, db = 0;
  for (int dk = 0; dk < 2; dk++)
    for (int dj = 0; dj < 2; dj++)
      for (int di = 0; di < 2; di++) {
        const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
        if (i >= G.n[0] || j >= G.n[1] || k >= G.n[2]) continue;
        const int c = cidx(G, i, j, k);
        const double r = rAU[c];
        // fine faces on the coarse cell's + side
        if (di == 1 && i + 1 < G.n[0]) tx += 0.5 * (r + rAU[c + 1]) * G.area[0] * G.ih[0];
        if (dj == 1 && j + 1 < G.n[1]) ty += 0.5 * (r + rAU[c + G.n[0]]) * G.area[1] * G.ih[1];
        if (dk == 1 && k + 1 < G.n[2])
          tz += 0.5 * (r + rAU[c + G.n[0] * G.n[1]]) * G.area[2] * G.ih[2];
        for (int a = 0; a < 3; a++) {
          const int co[3] = {i, j, k};
          if (co[a] == 0 && G.bck[2 * a] == BC_OUTLET) db += r * G.area[a] * 2.0 * G.ih[a];
          if (co[a] == G.n[a] - 1 && G.bck[2 * a + 1] == BC_OUTLET)
            db += r * G.area[a] * 2.0 * G.ih[a];
        }
      }
  const int C = I + cn0 * (J + cn1 * K);
  Tx[C] = (R)(0.5 * tx);
  Ty[C] = (R)(0.5 * ty);
  Tz[C] = (R)(0.5 * tz);
  Db[C] = (R)(0.5 * db);
}

template <typename R>
__global__ void __launch_bounds__(NTHREADS) k_build_coarsec(LV<R> L, const R *__restrict__ Dbf,
                                                            int cn0, int cn1, int cn2,
                                                            R *__restrict__ Tx, R *__restrict__ Ty,
                                                            R *__restrict__ Tz,
                                                            R *__restrict__ Db) {
  const int I = blockIdx.x * BX + threadIdx.x, J = blockIdx.y * BY + threadIdx.y,
            K = blockIdx.z;
  if (I >= cn0 || J >= cn1) return;
  R tx = 0, ty = 0, tz = 0, db = 0;
  for (int dk = 0; dk < 2; dk++)
    for (int dj = 0; dj < 2; dj++)
      for (int di = 0; di < 2; di++) {
        const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
        if (i >= L.n0 || j >= L.n1 || k >= L.n2) continue;
        const int c = i + L.n0 * (j + L.n1 * k);
        if (di == 1 && i + 1 < L.n0) tx += L.Tx[c];
        if (dj == 1 && j + 1 < L.n1) ty += L.Ty[c];
        if (dk == 1 && k + 1 < L.n2) tz += L.Tz[c];
        db += Dbf[c];
      }
  const int C = I + cn0 * (J + cn1 * K);
  Tx[C] = (R)0.5 * tx;
  Ty[C] = (R)0.5 * ty;
  Tz[C] = (R)0.5 * tz;
  Db[C] = (R)0.5 * db;
}

template <typename R>
__global__ void __launch_bounds__(NTHREADS) k_diag(LV<R> L, const R *__restrict__ Db,
                                                   R *__restrict__ D) {
  const int i = blockIdx.x * BX + threadIdx.x, j = blockIdx.y * BY + threadIdx.y,
            k = blockIdx.z;
  if (i >= L.n0 || j >= L.n1) return;
  const int c = i + L.n0 * (j + L.n1 * k);
  const int sy = L.n0, sz = L.n0 * L.n1;
  R d = Db[c] + L.Tx[c] + L.Ty[c] + L.Tz[c];
  if (i > 0) d += L.Tx[c - 1];
  if (j > 0) d += L.Ty[c - sy];
  if (k > 0) d += L.Tz[c - sz];
  D[c] = d;
}

// ------------------------------------------------------------------ host

static dim3 grid_of(int n0, int n1, int n2) {
  return dim3((n0 + BX - 1) / BX, (n1 + BY - 1) / BY, n2);
}

template <typename R>
static LV<R> view(const Level &L);
template <>
LV<double> view<double>(const Level &L) {
  return LV<double>{L.n[0], L.n[1], L.n[2], L.Tx, L.Ty, L.Tz, L.D};
}
template <>
LV<float> view<float>(const Level &L) {
  return LV<float>{L.n[0], L.n[1], L.n[2], L.Txf, L.Tyf, L.Tzf, L.Df};
}
template <typename R> static R *lx(Level &L);
template <> double *lx<double>(Level &L) { return L.x; }
template <> float *lx<float>(Level &L) { return L.xf; }
template <typename R> static R *lb(Level &L);
template <> double *lb<double>(Level &L) { return L.b; }
template <> float *lb<float>(Level &L) { return L.bf; }
template <typename R> static R *lTx(Level &L);
template <> double *lTx<double>(Level &L) { return L.Tx; }
template <> float *lTx<float>(Level &L) { return L.Txf; }
template <typename R> static R *lTy(Level &L);
template <> double *lTy<double>(Level &L) { return L.Ty; }
template <> float *lTy<float>(Level &L) { return L.Tyf; }
template <typename R> static R *lTz(Level &L);
template <> double *lTz<double>(Level &L) { return L.Tz; }
template <> float *lTz<float>(Level &L) { return L.Tzf; }
template <typename R> static R *lDb(Level &L);
template <> double *lDb<double>(Level &L) { return L.Db; }
template <> float *lDb<float>(Level &L) { return L.Dbf; }
template <typename R> static R *lD(Level &L);
template <> double *lD<double>(Level &L) { return L.D; }
template <> float *lD<float>(Level &L) { return L.Df; }

static void *dalloc(Handle *h, size_t bytes, int &rc) {
  void *p = nullptr;
  if (hipMalloc(&p, bytes < 256 ? 256 : bytes) != hipSuccess) {
    rc = DBS_ENOMEM;
    return nullptr;
  }
  h->allocs.push_back(p);
  return p;
}

int pressure_setup(Handle *h) {
  int rc = DBS_OK;
  const bool mixed = h->ctl.precision == DBS_MIXED;
  h->lv.clear();
  Level L0;
  for (int a = 0; a < 3; a++) L0.n[a] = h->G.n[a];
  L0.nc = h->G.nc;
  L0.grid = h->grid;
  h->lv.push_back(L0);
  // coarsen until the level is small enough for one block
  while (true) {
    const Level &F = h->lv.back();
    if (F.nc <= 64 || (F.n[0] == 1 && F.n[1] == 1 && F.n[2] == 1)) break;
    Level C;
    for (int a = 0; a < 3; a++) C.n[a] = (F.n[a] + 1) / 2;
    C.nc = C.n[0] * C.n[1] * C.n[2];
    C.grid = grid_of(C.n[0], C.n[1], C.n[2]);
    size_t n = (size_t)C.nc;
    if (mixed) {
      C.Txf = (float *)dalloc(h, n * 4, rc); C.Tyf = (float *)dalloc(h, n * 4, rc);
      C.Tzf = (float *)dalloc(h, n * 4, rc); C.Dbf = (float *)dalloc(h, n * 4, rc);
      C.Df = (float *)dalloc(h, n * 4, rc); C.xf = (float *)dalloc(h, n * 4, rc);
      C.bf = (float *)dalloc(h, n * 4, rc);
    } else {
      C.Tx = (double *)dalloc(h, n * 8, rc); C.Ty = (double *)dalloc(h, n * 8, rc);
      C.Tz = (double *)dalloc(h, n * 8, rc); C.Db = (double *)dalloc(h, n * 8, rc);
      C.D = (double *)dalloc(h, n * 8, rc); C.x = (double *)dalloc(h, n * 8, rc);
      C.b = (double *)dalloc(h, n * 8, rc);
    }
    if (rc) return rc;
    h->lv.push_back(C);
  }
  if (mixed) {
    h->lv[0].xf = (float *)dalloc(h, (size_t)h->G.nc * 4, rc);   // z (FP32)
    h->lv[0].bf = (float *)dalloc(h, (size_t)h->G.nc * 4, rc);   // rAU (FP32)
    h->rf = (float *)dalloc(h, (size_t)h->G.nc * 4, rc);         // r (FP32)
    h->zoldf = (float *)dalloc(h, (size_t)h->G.nc * 4, rc);      // previous z (FP32)
  }
  h->st.mg_levels = (int)h->lv.size();
  return rc;
}

void pressure_free(Handle *h) { h->lv.clear(); }

// build coarse operators for the current rAU (rAUr: rAU in the V-cycle type)
template <typename R>
static void build_hierarchy(Handle *h, const double *rAU) {
  dim3 blk(BX, BY);
  for (size_t l = 1; l < h->lv.size(); l++) {
    Level &C = h->lv[l];
    if (l == 1) {
      DBS_LAUNCH(h, KC_BUILD_COARSE, k_build_coarse0<R>, C.grid, blk, h->G, rAU, C.n[0], C.n[1],
                 C.n[2], lTx<R>(C), lTy<R>(C), lTz<R>(C), lDb<R>(C));
    } else {
      Level &F = h->lv[l - 1];
      DBS_LAUNCH(h, KC_BUILD_COARSE, k_build_coarsec<R>, C.grid, blk, view<R>(F),
                 (const R *)lDb<R>(F), C.n[0], C.n[1], C.n[2], lTx<R>(C), lTy<R>(C), lTz<R>(C),
                 lDb<R>(C));
    }
    DBS_LAUNCH(h, KC_BUILD_COARSE, k_diag<R>, C.grid, blk, view<R>(C), (const R *)lDb<R>(C),
               lD<R>(C));
  }
}

// z = M r: one V-cycle.  Level 0 uses the matrix-free operator of rAUr.
template <typename R, typename B>
static void vcycle(Handle *h, const R *rAUr, const B *b0, R *z0) {
  dim3 blk(BX, BY);
  const Geom &G = h->G;
  const int nl = (int)h->lv.size();
  if (nl == 1) {
    // single level: symmetric sweeps on the fine grid
    for (int s = 0; s < h->mg_pre; s++) {
      DBS_LAUNCH(h, KC_SMOOTH0, (k_smooth0<R, B>), h->grid, blk, G, rAUr, b0, z0, 0, s == 0);
      DBS_LAUNCH(h, KC_SMOOTH0, (k_smooth0<R, B>), h->grid, blk, G, rAUr, b0, z0, 1, 0);
    }
    for (int s = 0; s < h->mg_post; s++) {
      DBS_LAUNCH(h, KC_SMOOTH0, (k_smooth0<R, B>), h->grid, blk, G, rAUr, b0, z0, 1, 0);
      DBS_LAUNCH(h, KC_SMOOTH0, (k_smooth0<R, B>), h->grid, blk, G, rAUr, b0, z0, 0, 0);
    }
    return;
  }
  // down
  for (int s = 0; s < h->mg_pre; s++) {
    DBS_LAUNCH(h, KC_SMOOTH0, (k_smooth0<R, B>), h->grid, blk, G, rAUr, b0, z0, 0, s == 0);
    DBS_LAUNCH(h, KC_SMOOTH0, (k_smooth0<R, B>), h->grid, blk, G, rAUr, b0, z0, 1, 0);
  }
  {
    Level &C = h->lv[1];
    DBS_LAUNCH(h, KC_RESTRICT0, (k_restrict0<R, B>), C.grid, blk, G, C.n[0], C.n[1], C.n[2],
               rAUr, b0, (const R *)z0, lb<R>(C));
  }
  for (int l = 1; l < nl - 1; l++) {
    Level &L = h->lv[l];
    Level &C = h->lv[l + 1];
    for (int s = 0; s < h->mg_pre; s++) {
      DBS_LAUNCH(h, KC_SMOOTHC, k_smoothc<R>, L.grid, blk, view<R>(L), (const R *)lb<R>(L),
                 lx<R>(L), 0, s == 0);
      DBS_LAUNCH(h, KC_SMOOTHC, k_smoothc<R>, L.grid, blk, view<R>(L), (const R *)lb<R>(L),
                 lx<R>(L), 1, 0);
    }
    DBS_LAUNCH(h, KC_RESTRICTC, k_restrictc<R>, C.grid, blk, view<R>(L), C.n[0], C.n[1], C.n[2],
               (const R *)lb<R>(L), (const R *)lx<R>(L), lb<R>(C));
  }
  {
    Level &L = h->lv[nl - 1];
    DBS_LAUNCH(h, KC_COARSE, k_coarse_solve<R>, dim3(1), dim3(1024), view<R>(L),
               (const R *)lb<R>(L), lx<R>(L), h->coarse_sweeps);
  }
  // up
  for (int l = nl - 2; l >= 1; l--) {
    Level &L = h->lv[l];
    Level &C = h->lv[l + 1];
    DBS_LAUNCH(h, KC_PROLONGC, k_prolong<R>, L.grid, blk, L.n[0], L.n[1], L.n[2], C.n[0], C.n[1],
               (const R *)lx<R>(C), lx<R>(L));
    for (int s = 0; s < h->mg_post; s++) {
      DBS_LAUNCH(h, KC_SMOOTHC, k_smoothc<R>, L.grid, blk, view<R>(L), (const R *)lb<R>(L),
                 lx<R>(L), 1, 0);
      DBS_LAUNCH(h, KC_SMOOTHC, k_smoothc<R>, L.grid, blk, view<R>(L), (const R *)lb<R>(L),
                 lx<R>(L), 0, 0);
    }
  }
  {
    Level &C = h->lv[1];
    DBS_LAUNCH(h, KC_PROLONG0, k_prolong<R>, h->grid, blk, G.n[0], G.n[1], G.n[2], C.n[0], C.n[1],
               (const R *)lx<R>(C), z0);
  }
  for (int s = 0; s < h->mg_post; s++) {
    DBS_LAUNCH(h, KC_SMOOTH0, (k_smooth0<R, B>), h->grid, blk, G, rAUr, b0, z0, 1, 0);
    DBS_LAUNCH(h, KC_SMOOTH0, (k_smooth0<R, B>), h->grid, blk, G, rAUr, b0, z0, 0, 0);
  }
}

static void finalize(Handle *h, int two, int slot, int slot2, int op) {
  DBS_LAUNCH(h, KC_FINALIZE, k_finalize, dim3(1), dim3(1024), (const double *)h->partials,
             h->nblocks, two, h->scal, slot, slot2, op);
}

static double fetch(Handle *h, int slot) {
  hipMemcpyAsync(h->hscal, h->scal, sizeof(double) * S_NSCAL, hipMemcpyDeviceToHost, h->stream);
  hipStreamSynchronize(h->stream);
  return h->hscal[slot];
}

static void remove_mean(Handle *h, double *x) {
  dim3 blk(BX, BY);
  DBS_LAUNCH(h, KC_MISC, k_sum, h->grid, blk, h->G, (const double *)x, h->partials);
  finalize(h, 0, S_SUM, 0, FIN_STORE);
  DBS_LAUNCH(h, KC_MISC, k_sub_mean, h->grid, blk, h->G, (const double *)h->scal, x);
}

// true residual r = b - A x; returns ||r|| and sets ||b||
static double true_residual(Handle *h, const double *rAU, const double *b, const double *x,
                            double *nb) {
  dim3 blk(BX, BY);
  DBS_LAUNCH(h, KC_SPMV, k_resid0, h->grid, blk, h->G, rAU, b, x, h->r, h->partials, h->nblocks);
  finalize(h, 1, S_RR, S_BB, FIN_STORE);
  if (!h->G.has_outlet) {
    remove_mean(h, h->r);
    dim3 blk2(BX, BY);
    DBS_LAUNCH(h, KC_DOT, k_dot_rz<double>, h->grid, blk2, h->G, (const double *)h->r,
               (const double *)h->r, (const double *)nullptr, h->partials, h->nblocks);
    finalize(h, 0, S_RR, 0, FIN_STORE);
  }
  fetch(h, S_RR);
  *nb = sqrt(h->hscal[S_BB]);
  return sqrt(h->hscal[S_RR]);
}

// z = M r (FP32 V-cycle on an FP32 copy of r in the mixed form)
template <typename R>
static void precondition(Handle *h, const R *rAUr, R *zR) {
  dim3 blk(BX, BY);
  if (std::is_same<R, float>::value) {
    DBS_LAUNCH(h, KC_MISC, k_cast<float>, h->grid, blk, h->G, (const double *)h->r, h->rf);
    vcycle<R, R>(h, rAUr, (const R *)h->rf, zR);
  } else {
    vcycle<R, double>(h, rAUr, (const double *)h->r, zR);
  }
}

template <typename R>
static int pcg(Handle *h, const double *rAU, const double *b, double *x, int *iters,
               double *relres) {
  dim3 blk(BX, BY);
  const Geom &G = h->G;
  const bool flex = std::is_same<R, float>::value;
  const R *rAUr;
  if (flex) {
    float *rf = h->lv[0].bf;
    DBS_LAUNCH(h, KC_MISC, k_cast<float>, h->grid, blk, G, rAU, rf);
    rAUr = (const R *)rf;
  } else {
    rAUr = (const R *)rAU;
  }
  build_hierarchy<R>(h, rAU);
  // closed domains: the right-hand side must be compatible (zero mean)
  double nb;
  double nr = true_residual(h, rAU, b, x, &nb);
  if (!G.has_outlet) {
    // ||b|| of the projected right-hand side: project a copy into z
    hipMemcpyAsync(h->z, b, sizeof(double) * G.nc, hipMemcpyDeviceToDevice, h->stream);
    remove_mean(h, h->z);
    DBS_LAUNCH(h, KC_DOT, k_dot_rz<double>, h->grid, blk, G, (const double *)h->z,
               (const double *)h->z, (const double *)nullptr, h->partials, h->nblocks);
    finalize(h, 0, S_BB, 0, FIN_STORE);
    nb = sqrt(fetch(h, S_BB));
  }
  const double norm = nb > 0.0 ? nb : nr;
  const double tol = h->ctl.p_tol;
  int it = 0, rc = DBS_OK;
  R *zR = flex ? (R *)h->lv[0].xf : (R *)h->z;
  R *zold = flex ? (R *)h->zoldf : nullptr;
  if (norm > 0.0 && nr > tol * norm) {
    const int replace_every = flex ? 8 : 0;
    // z = M r, p = z, rz = r.z
    precondition<R>(h, rAUr, zR);
    DBS_LAUNCH(h, KC_DOT, k_dot_rz<R>, h->grid, blk, G, (const double *)h->r, (const R *)zR,
               (const R *)nullptr, h->partials, h->nblocks);
    finalize(h, 0, S_RZ, 0, FIN_STORE);
    DBS_LAUNCH(h, KC_XPBY, k_xpby<R>, h->grid, blk, G, (const double *)h->scal, (const R *)zR,
               h->pv, 1, zold);
    for (;;) {
      if (it >= h->ctl.p_maxit) { rc = DBS_ENOCONV; break; }
      DBS_LAUNCH(h, KC_SPMV, k_spmv0_dot, h->grid, blk, G, rAU, (const double *)h->pv, h->q,
                 h->partials);
      finalize(h, 0, S_PQ, 0, FIN_ALPHA);
      DBS_LAUNCH(h, KC_AXPY, k_axpy_dot, h->grid, blk, G, (const double *)h->scal,
                 (const double *)h->pv, (const double *)h->q, x, h->r, h->partials);
      it++;
      bool replaced = false;
      if (replace_every && it % replace_every == 0) {
        // residual replacement: the true FP64 residual takes the recursive one's place
        nr = true_residual(h, rAU, b, x, &nb);
        replaced = true;
      } else {
        finalize(h, 0, S_RR, 0, FIN_STORE);
        nr = sqrt(fetch(h, S_RR));
      }
      if (nr <= tol * norm) {
        // stop only when the true residual b - A x meets the tolerance; else
        // continue with it in place of the recursive one
        if (replaced) break;
        nr = true_residual(h, rAU, b, x, &nb);
        if (nr <= tol * norm) break;
      }
      precondition<R>(h, rAUr, zR);
      if (flex) {
        DBS_LAUNCH(h, KC_DOT, k_dot_rz<R>, h->grid, blk, G, (const double *)h->r, (const R *)zR,
                   (const R *)zold, h->partials, h->nblocks);
        finalize(h, 1, S_RZNEW, S_RZOLD, FIN_BETA_FLEX);
      } else {
        DBS_LAUNCH(h, KC_DOT, k_dot_rz<R>, h->grid, blk, G, (const double *)h->r, (const R *)zR,
                   (const R *)nullptr, h->partials, h->nblocks);
        finalize(h, 0, S_RZNEW, 0, FIN_BETA);
      }
      DBS_LAUNCH(h, KC_XPBY, k_xpby<R>, h->grid, blk, G, (const double *)h->scal, (const R *)zR,
                 h->pv, 0, zold);
    }
  }
  if (!G.has_outlet) remove_mean(h, x);
  // report the true residual
  nr = true_residual(h, rAU, b, x, &nb);
  if (iters) *iters = it;
  if (relres) *relres = norm > 0.0 ? nr / norm : 0.0;
  return rc;
}

int pressure_solve(Handle *h, const double *rAU, const double *b, double *x, int *iters,
                   double *relres) {
  if (h->ctl.precision == DBS_MIXED) return pcg<float>(h, rAU, b, x, iters, relres);
  return pcg<double>(h, rAU, b, x, iters, relres);
}

}  // namespace dbs
