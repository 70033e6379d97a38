// Pressure solve of the PISO corrector: the SPD system
//   sum_f T_f (x_P - x_N) + sum_outlet T_b x_P = b,
//   T_f = mean(rAU) A_f / h (interior faces), T_b = rAU_P A / (h/2) (outlets),
// i.e. -div(rAU grad p_rgh) of Eq. (pressure_predictor), by conjugate gradients
// preconditioned with one geometric-multigrid V-cycle (the paper uses a
// geometric-algebraic multigrid solver, Sec. 3.2).
//
// Hierarchy: cell-centred 2x2x2 aggregation (ceil(n/2) per axis, ragged odd
// edges).  The fine operator is never stored: kernels rebuild T_f from rAU
// (one array instead of four).  Coarse operators store the +x/+y/+z face
// coefficient of each cell and the diagonal; a coarse face coefficient is
// half the sum of the fine ones it covers (the h-doubling of a rediscretised
// operator).  Smoother: red-black Gauss-Seidel, red then black on the way
// down and black then red on the way up, so the V-cycle is a symmetric
// preconditioner.  Restriction sums the 8 children's residuals (transpose of
// piecewise-constant prolongation).  The smallest levels of a sample (from
// the first one whose remaining hierarchy fits in BOTTOM_LDS bytes) are
// cycled by one work-group in a single launch.
//
// Mixed precision (DBS_MIXED): the V-cycle runs in FP32 (rAU, coefficients,
// residual, correction); the CG vectors, dot products and the convergence
// test stay FP64; CG becomes flexible (Polak-Ribiere beta) and the true FP64
// residual b - A x replaces the recursive one every few iterations.
//
// Batches: every launch covers all samples; a block finds its sample in the
// block prefix of its launch shape.  CG runs per sample in lockstep: alpha,
// beta and the convergence test are per-sample device scalars, converged
// samples are masked off (their blocks return at once), so each sample
// follows the iterations it would follow alone.  With a fixed iteration
// budget the solve needs no host synchronisation and can be captured in a
// graph.
//
// Reductions are deterministic: each block writes one partial sum and one
// block per sample adds that sample's partials in a fixed order.
#include <algorithm>
#include <array>
#include <cstring>
#include <type_traits>

#include "dbs_internal.h"

namespace dbs {

enum {
  S_RZ = 0, S_PQ, S_RR, S_ALPHA, S_BETA, S_RZNEW, S_RZOLD, S_BB, S_SUM, S_NRM2, S_ITS,
  S_NOCONV, S_RRFIN, S_RESTART, S_RR0
};
static_assert(S_RR0 < NSC, "device scalars per sample");

constexpr int KZ = 8;               // planes per thread column (coarse levels)
constexpr int BOTTOM_LDS = 144000;  // bytes of LDS for the single work-group bottom
constexpr int MAXLV = 16;
constexpr int MIN_BLOCKS = 2048;

// ------------------------------------------------------------ launch shape

// device view of a Shape
struct SH {
  const int *bp;
  int ns;
  int kz;
};

// This block's global tile number (XCD order), sample and block within the
// sample; false when the sample is masked off.
__device__ __forceinline__ bool locate(const SH &S, const int *__restrict__ mask, int &g, int &s,
                                       int &lb) {
  g = xcd_remap(blockIdx.x, gridDim.x);
  s = find_seg(S.bp, S.ns, g);
  lb = g - S.bp[s];
  return !mask || mask[s];
}

// Column kernels give each thread a column of kz planes at one cell (or an
// x-pair of cells) of a plane, on 64 x 4 blocks tiling the plane.  Levels
// whose rows would leave more than a ninth of those lanes idle (rows of a
// few dozen cells, as on the coarse levels of a batch of small samples)
// take the plane's columns in order instead, 256 consecutive ones a block.
__host__ __device__ inline bool column_linear(int n0, int n1, bool pair) {
  const int cx = pair ? 2 * BX : BX;
  const long long units = pair ? (n0 + 1) / 2 : n0;  // columns per row
  const long long tiled = (long long)((n0 + cx - 1) / cx) * BX * ((n1 + BY - 1) / BY) * BY;
  return 8 * tiled > 9 * units * n1;
}

__host__ __device__ inline int column_blocks(int n0, int n1, int n2, int kz, bool pair) {
  const int chunks = (n2 + kz - 1) / kz;
  if (column_linear(n0, n1, pair)) {
    const long long cols = (long long)(pair ? (n0 + 1) / 2 : n0) * n1;
    return (int)((cols + BX * BY - 1) / (BX * BY)) * chunks;
  }
  const int cx = pair ? 2 * BX : BX;
  return ((n0 + cx - 1) / cx) * ((n1 + BY - 1) / BY) * chunks;
}

// column owned by this thread in block lb of a level of n0 x n1 x n2 cells:
// x index (first of the pair), y index, plane range
__device__ __forceinline__ bool column(int n0, int n1, int n2, int lb, int kz, bool pair, int &i,
                                       int &j, int &k0, int &k1) {
  if (column_linear(n0, n1, pair)) {
    const unsigned units = pair ? (unsigned)(n0 + 1) / 2 : (unsigned)n0;
    const unsigned cols = units * (unsigned)n1;
    const unsigned per = (cols + BX * BY - 1) / (BX * BY);  // blocks per chunk of planes
    const unsigned chunk = (unsigned)lb / per;
    const unsigned q = ((unsigned)lb - chunk * per) * (BX * BY) + threadIdx.x + BX * threadIdx.y;
    const unsigned jj = q / units;
    i = (int)(q - jj * units) * (pair ? 2 : 1);
    j = (int)jj;
    k0 = (int)chunk * kz;
    k1 = min(k0 + kz, n2);
    return q < cols;
  }
  const int cx = pair ? 2 * BX : BX;
  const int nbx = (n0 + cx - 1) / cx, nby = (n1 + BY - 1) / BY;
  const int bx = lb % nbx;
  const int L = lb / nbx;
  i = (bx * BX + threadIdx.x) * (pair ? 2 : 1);
  j = (L % nby) * BY + threadIdx.y;
  k0 = (L / nby) * kz;
  k1 = min(k0 + kz, n2);
  return i < n0 && j < n1;
}

// ------------------------------------------------------------------ operator

// one sample on one level; pointers start at the sample's first cell
template <typename R>
struct Op {
  int n0, n1, n2;
  int matfree;           // 1: coefficients rebuilt from rAU (fine level)
  const R *rAU;
  R c[3];                // area / h per axis
  R ob[6];               // outlet diagonal factor per domain face (2 c or 0)
  const R *Tx, *Ty, *Tz, *D;  // stored operator (coarse levels)
};

// one level over the batch
template <typename R>
struct OpB {
  const LvS *ls;
  int matfree;
  const R *rAU, *Tx, *Ty, *Tz, *D;
};

template <typename R>
__device__ __forceinline__ Op<R> op_at(const OpB<R> &B, int s) {
  const LvS &Q = B.ls[s];
  Op<R> o;
  o.n0 = Q.n0; o.n1 = Q.n1; o.n2 = Q.n2;
  o.matfree = B.matfree;
  const int c0 = Q.c0;
  for (int a = 0; a < 3; a++) o.c[a] = (R)Q.c[a];
  for (int b = 0; b < 6; b++) o.ob[b] = (R)Q.ob[b];
  if (B.matfree) {
    o.rAU = B.rAU + c0;
    o.Tx = o.Ty = o.Tz = o.D = nullptr;
  } else {
    o.rAU = nullptr;
    o.Tx = B.Tx + c0; o.Ty = B.Ty + c0; o.Tz = B.Tz + c0; o.D = B.D + c0;
  }
  return o;
}

// diagonal and the six neighbour coefficients of cell (i,j,k); neighbour
// order -x,+x,-y,+y,-z,+z; 0 where there is no neighbour
template <typename R>
__device__ __forceinline__ void op_row(const Op<R> &L, int i, int j, int k, int c, R &D,
                                       R T[6]) {
  const int sy = L.n0, sz = L.n0 * L.n1;
  if (L.matfree) {
    const R r = L.rAU[c];
    const R h = (R)0.5;
    T[0] = i > 0 ? h * (r + L.rAU[c - 1]) * L.c[0] : (R)0;
    T[1] = i + 1 < L.n0 ? h * (r + L.rAU[c + 1]) * L.c[0] : (R)0;
    T[2] = j > 0 ? h * (r + L.rAU[c - sy]) * L.c[1] : (R)0;
    T[3] = j + 1 < L.n1 ? h * (r + L.rAU[c + sy]) * L.c[1] : (R)0;
    T[4] = k > 0 ? h * (r + L.rAU[c - sz]) * L.c[2] : (R)0;
    T[5] = k + 1 < L.n2 ? h * (r + L.rAU[c + sz]) * L.c[2] : (R)0;
    R db = (i == 0 ? L.ob[0] : (R)0) + (i + 1 == L.n0 ? L.ob[1] : (R)0) +
           (j == 0 ? L.ob[2] : (R)0) + (j + 1 == L.n1 ? L.ob[3] : (R)0) +
           (k == 0 ? L.ob[4] : (R)0) + (k + 1 == L.n2 ? L.ob[5] : (R)0);
    D = T[0] + T[1] + T[2] + T[3] + T[4] + T[5] + r * db;
  } else {
    T[0] = i > 0 ? L.Tx[c - 1] : (R)0;
    T[1] = i + 1 < L.n0 ? L.Tx[c] : (R)0;
    T[2] = j > 0 ? L.Ty[c - sy] : (R)0;
    T[3] = j + 1 < L.n1 ? L.Ty[c] : (R)0;
    T[4] = k > 0 ? L.Tz[c - sz] : (R)0;
    T[5] = k + 1 < L.n2 ? L.Tz[c] : (R)0;
    D = L.D[c];
  }
}

// outlet (Dirichlet) part of the fine-level diagonal
template <typename R>
__device__ __forceinline__ R op_outlet(const Op<R> &L, int i, int j, int k, int c) {
  const R db = (i == 0 ? L.ob[0] : (R)0) + (i + 1 == L.n0 ? L.ob[1] : (R)0) +
               (j == 0 ? L.ob[2] : (R)0) + (j + 1 == L.n1 ? L.ob[3] : (R)0) +
               (k == 0 ? L.ob[4] : (R)0) + (k + 1 == L.n2 ? L.ob[5] : (R)0);
  return L.rAU[c] * db;
}

// sum of T_N x_N; a zero coefficient marks a missing neighbour
template <typename R, typename X>
__device__ __forceinline__ R op_off(const Op<R> &L, int c, const R T[6],
                                    const X *__restrict__ x) {
  const int sy = L.n0, sz = L.n0 * L.n1;
  R s = 0;
  if (T[0] != (R)0) s += T[0] * (R)x[c - 1];
  if (T[1] != (R)0) s += T[1] * (R)x[c + 1];
  if (T[2] != (R)0) s += T[2] * (R)x[c - sy];
  if (T[3] != (R)0) s += T[3] * (R)x[c + sy];
  if (T[4] != (R)0) s += T[4] * (R)x[c - sz];
  if (T[5] != (R)0) s += T[5] * (R)x[c + sz];
  return s;
}

// ------------------------------------------------ vector kernels (flat)
//
// FLAT_CELLS consecutive cells of the fine arena per block of FLAT_T
// threads; a sample's cells are padded to whole blocks and the padding is
// zero in every vector, so dot products and updates may run over it.

struct FL {
  const int *bp;   // first block of each sample
  int ns;
  const Rng *rng;
};

__device__ __forceinline__ void flat_partial(double v, double *lds, double *partials, int slot0) {
  v = wave_sum(v);
  const int t = threadIdx.x;
  if ((t & 63) == 0) lds[t >> 6] = v;
  __syncthreads();
  if (t == 0) partials[slot0 + blockIdx.x] = (lds[0] + lds[1]) + (lds[2] + lds[3]);
}

__device__ __forceinline__ size_t flat_cell(int m) {
  return (size_t)blockIdx.x * FLAT_CELLS + m * FLAT_T + threadIdx.x;
}

// x += alpha p, r -= alpha q (and its FP32 copy), partial sum of r.r
__global__ void __launch_bounds__(FLAT_T) k_axpy_dot(FL F, const double *__restrict__ scal,
                                                     const double *__restrict__ p,
                                                     const double *__restrict__ q,
                                                     double *__restrict__ x,
                                                     double *__restrict__ r,
                                                     float *__restrict__ rf,
                                                     double *__restrict__ partials,
                                                     const int *__restrict__ act) {
  __shared__ double lds[FLAT_T / 64];
  const int s = find_seg(F.bp, F.ns, blockIdx.x);
  if (!act[s]) return;
  const double al = scal[s * NSC + S_ALPHA];
  double v = 0.0;
#pragma unroll
  for (int m = 0; m < FLAT_CELLS / FLAT_T; m++) {
    const size_t c = flat_cell(m);
    x[c] = fma(al, p[c], x[c]);
    const double rr = fma(-al, q[c], r[c]);
    r[c] = rr;
    if (rf) rf[c] = (float)rr;
    v += rr * rr;
  }
  flat_partial(v, lds, partials, 0);
}

// partial sums of a.z and (flexible) a.zold
template <typename Z>
__global__ void __launch_bounds__(FLAT_T) k_dot2(FL F, const double *__restrict__ a,
                                                 const Z *__restrict__ zz,
                                                 const Z *__restrict__ zold,
                                                 double *__restrict__ partials, int off2,
                                                 const int *__restrict__ mask, int closed_only) {
  __shared__ double lds[FLAT_T / 64];
  const int s = find_seg(F.bp, F.ns, blockIdx.x);
  if ((mask && !mask[s]) || (closed_only && !F.rng[s].closed)) return;
  double v = 0.0, vo = 0.0;
#pragma unroll
  for (int m = 0; m < FLAT_CELLS / FLAT_T; m++) {
    const size_t c = flat_cell(m);
    const double ac = a[c];
    v += ac * (double)zz[c];
    if (zold) vo += ac * (double)zold[c];
  }
  flat_partial(v, lds, partials, 0);
  if (zold) {
    __syncthreads();
    flat_partial(vo, lds, partials, off2);
  }
}

template <typename R>
__global__ void __launch_bounds__(FLAT_T) k_cast(const double *__restrict__ in,
                                                 R *__restrict__ out) {
#pragma unroll
  for (int m = 0; m < FLAT_CELLS / FLAT_T; m++) {
    const size_t c = flat_cell(m);
    out[c] = (R)in[c];
  }
}

__global__ void __launch_bounds__(FLAT_T) k_copy(const double *__restrict__ in,
                                                 double *__restrict__ out) {
#pragma unroll
  for (int m = 0; m < FLAT_CELLS / FLAT_T; m++) {
    const size_t c = flat_cell(m);
    out[c] = in[c];
  }
}

// partial sums of x over closed samples
__global__ void __launch_bounds__(FLAT_T) k_sum(FL F, const double *__restrict__ x,
                                                double *__restrict__ partials,
                                                const int *__restrict__ mask) {
  __shared__ double lds[FLAT_T / 64];
  const int s = find_seg(F.bp, F.ns, blockIdx.x);
  if ((mask && !mask[s]) || !F.rng[s].closed) return;
  double v = 0.0;
#pragma unroll
  for (int m = 0; m < FLAT_CELLS / FLAT_T; m++) v += x[flat_cell(m)];
  flat_partial(v, lds, partials, 0);
}

// x -= mean(x) on the real cells of closed samples (and refresh an FP32 copy)
__global__ void __launch_bounds__(FLAT_T) k_sub_mean(FL F, const double *__restrict__ scal,
                                                     double *__restrict__ x,
                                                     float *__restrict__ xf,
                                                     const int *__restrict__ mask) {
  const int s = find_seg(F.bp, F.ns, blockIdx.x);
  const Rng g = F.rng[s];
  if ((mask && !mask[s]) || !g.closed) return;
  const double mean = scal[s * NSC + S_SUM] / (double)g.nc;
#pragma unroll
  for (int m = 0; m < FLAT_CELLS / FLAT_T; m++) {
    const size_t c = flat_cell(m);
    if ((long long)c - g.c0 < g.nc) {
      const double v = x[c] - mean;
      x[c] = v;
      if (xf) xf[c] = (float)v;
    }
  }
}

// a[s] = va (unless a is NULL), w[s] = vw
__global__ void k_flags(int *__restrict__ a, int va, int *__restrict__ w, int vw, int n) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) {
    if (a) a[t] = va;
    w[t] = vw;
  }
}

// after the CG loop: the samples whose last S_RR is not the true residual of
// the final x (still active, stopped by the iteration limit on the
// recursive residual, or closed: the mean was removed from x)
__global__ void k_want_final(const double *__restrict__ scal, const int *__restrict__ act,
                             const Rng *__restrict__ rng, int *__restrict__ want, int n) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) want[s] = (act[s] || scal[(size_t)s * NSC + S_NOCONV] != 0.0 || rng[s].closed) ? 1 : 0;
}

enum {
  FIN_STORE = 0, FIN_ALPHA, FIN_BETA, FIN_BETA_FLEX, FIN_RR, FIN_CHECK, FIN_INIT, FIN_RRFIN
};

struct FinArgs {
  const double *partials;
  const int *bp;        // block prefix of the producing launch (NULL: no sum)
  int off2;             // offset of the second partial array
  int two;              // 1: also reduce the second array into slot2
  int slot, slot2, op;
  const int *mask;      // samples taking part (NULL: all)
  const Rng *rng;
  int closed_only;
  int *act, *want;
  double tol2;          // p_tol^2
  int maxit;
};

// one block per sample: scal[slot] = sum of the sample's partials (and slot2
// from the second array), then the CG scalar and flag updates of `op`
constexpr int FIN_T = 1024;
__global__ void __launch_bounds__(FIN_T) k_finalize(FinArgs A, double *__restrict__ scal) {
  __shared__ double lds[FIN_T / 64];
  const int s = blockIdx.x;
  if ((A.mask && !A.mask[s]) || (A.closed_only && !A.rng[s].closed)) return;
  const int t = threadIdx.x;
  double *S = scal + (size_t)s * NSC;
  if (A.bp) {
    const int b0 = A.bp[s], b1 = A.bp[s + 1];
    for (int hh = 0; hh < (A.two ? 2 : 1); hh++) {
      const double *P = A.partials + (hh ? A.off2 : 0);
      double v0 = 0.0, v1 = 0.0;
      int i = b0 + t;
      for (; i + FIN_T < b1; i += 2 * FIN_T) {
        v0 += P[i];
        v1 += P[i + FIN_T];
      }
      if (i < b1) v0 += P[i];
      const double v = wave_sum(v0 + v1);
      if ((t & 63) == 0) lds[t >> 6] = v;
      __syncthreads();
      if (t == 0) {
        double sum = 0.0;
        for (int w = 0; w < FIN_T / 64; w++) sum += lds[w];
        S[hh ? A.slot2 : A.slot] = sum;
      }
      __syncthreads();
    }
  }
  if (t != 0) return;
  switch (A.op) {
    case FIN_ALPHA: {
      const double pq = S[S_PQ];
      S[S_ALPHA] = pq != 0.0 ? S[S_RZ] / pq : 0.0;
      break;
    }
    case FIN_BETA:
    case FIN_BETA_FLEX: {
      const double num = A.op == FIN_BETA ? S[S_RZNEW] : S[S_RZNEW] - S[S_RZOLD];
      double beta = S[S_RZ] != 0.0 ? num / S[S_RZ] : 0.0;
      // Flexible CG restarts (beta = 0) when r.z_old is not small against
      // r.z, Powell's test (1977) with its factor 0.2.  With r.z taken from
      // the FP32 copy of r, alpha carries an FP32 rounding error, so r is
      // orthogonal to the last direction only to that level; once the
      // residual falls to it (a sample the V-cycle solves almost exactly,
      // such as a single cell) r.z_old dominates, the Polak-Ribiere
      // direction would cancel to noise and alpha = r.z / p.q blow up.
      if (A.op == FIN_BETA_FLEX && !(fabs(S[S_RZOLD]) < 0.2 * S[S_RZNEW])) beta = 0.0;
      // after a residual replacement the new r is not orthogonal to the old
      // direction: restart, so that alpha = r.z / p.q is the exact line
      // minimum along p = z and the error cannot grow
      if (S[S_RESTART] != 0.0) beta = 0.0;
      S[S_RESTART] = 0.0;
      S[S_BETA] = beta;
      S[S_RZ] = S[S_RZNEW];
      break;
    }
    case FIN_RR: {
      const double its = S[S_ITS] + 1.0;
      S[S_ITS] = its;
      // the recursive residual is updated in FP64 in both forms (only z
      // comes from the FP32 V-cycle); once it reports convergence, the true
      // residual decides (and replaces it if it is not small)
      const bool small = S[S_RR] <= A.tol2 * S[S_NRM2];
      A.want[s] = small ? 1 : 0;
      if (!small && its >= A.maxit) {
        A.act[s] = 0;
        S[S_NOCONV] = 1.0;
      }
      break;
    }
    case FIN_CHECK: {
      if (S[S_RR] <= A.tol2 * S[S_NRM2]) {
        A.act[s] = 0;
      } else if (S[S_ITS] >= A.maxit) {
        A.act[s] = 0;
        S[S_NOCONV] = 1.0;
      } else {
        S[S_RESTART] = 1.0;  // the true residual replaced the recursive one
      }
      A.want[s] = 0;
      break;
    }
    case FIN_INIT: {
      const double n2 = S[S_BB] > 0.0 ? S[S_BB] : S[S_RR];
      S[S_NRM2] = n2;
      S[S_RR0] = S[S_RR];
      S[S_ITS] = 0.0;
      S[S_NOCONV] = 0.0;
      S[S_RESTART] = 0.0;
      A.act[s] = (n2 > 0.0 && S[S_RR] > A.tol2 * n2) ? 1 : 0;
      A.want[s] = 0;
      break;
    }
    case FIN_RRFIN:
      S[S_RRFIN] = S[S_RR];
      break;
    default:
      break;
  }
}

// ------------------------------------------------------ multigrid kernels

// red-black Gauss-Seidel half sweep of colour `color` (0 = red: i+j+k even)
// on a coarse level.  Each thread owns the x-pair (i, i+1) and updates the
// one of this colour in every plane.  zero_init: x = b/D on this colour and
// 0 on the other.
template <typename R, typename B>
__global__ void __launch_bounds__(NTHREADS) k_smooth(OpB<R> LB, SH S, const B *__restrict__ b,
                                                     R *__restrict__ x, int color, int zero_init,
                                                     const int *__restrict__ mask) {
  int g, s, lb;
  if (!locate(S, mask, g, s, lb)) return;
  const Op<R> L = op_at(LB, s);
  const int c0 = LB.ls[s].c0;
  b += c0;
  x += c0;
  int i0, j, k0, k1;
  if (!column(L.n0, L.n1, L.n2, lb, S.kz, true, i0, j, k0, k1)) return;
  const int sz = L.n0 * L.n1;
  int base = i0 + L.n0 * (j + L.n1 * k0);
  for (int k = k0; k < k1; k++, base += sz) {
    const int off = ((j + k) & 1) == color ? 0 : 1;  // i0 is even
    const int i = i0 + off;
    if (zero_init && i0 + 1 - off < L.n0) x[base + 1 - off] = (R)0;
    if (i >= L.n0) continue;
    const int c = base + off;
    R D, T[6];
    op_row(L, i, j, k, c, D, T);
    if (zero_init)
      x[c] = D > (R)0 ? (R)b[c] / D : (R)0;
    else
      x[c] = D > (R)0 ? ((R)b[c] + op_off(L, c, T, x)) / D : (R)0;
  }
}

// coarse right-hand side: sum over the 8 children of the fine residual; the
// launch covers the coarse cells of the samples cycled on the fine level.
// red: the smoothing ended with a black half sweep, so only the red
// children (even i + j + k) have a residual to add.
template <typename R, typename B>
__global__ void __launch_bounds__(NTHREADS) k_restrict(OpB<R> LB, SH S, const B *__restrict__ b,
                                                       const R *__restrict__ x,
                                                       R *__restrict__ bc,
                                                       const int *__restrict__ mask, int red) {
  int g, s, lb;
  if (!locate(S, mask, g, s, lb)) return;
  const Op<R> L = op_at(LB, s);
  const LvS &Q = LB.ls[s];
  b += Q.c0;
  x += Q.c0;
  bc += Q.cc0;
  const int cn0 = Q.cn0, cn1 = Q.cn1, cn2 = Q.cn2;
  int I, J, K0, K1;
  if (!column(cn0, cn1, cn2, lb, S.kz, false, I, J, K0, K1)) return;
  for (int K = K0; K < K1; K++) {
    R sum = 0;
    for (int dk = 0; dk < 2; dk++) {
      const int k = 2 * K + dk;
      if (k >= L.n2) continue;
      for (int dj = 0; dj < 2; dj++) {
        const int j = 2 * J + dj;
        if (j >= L.n1) continue;
        for (int di = 0; di < 2; di++) {
          const int i = 2 * I + di;
          if (i >= L.n0 || (red && ((di + dj + dk) & 1))) continue;
          const int c = i + L.n0 * (j + L.n1 * k);
          R D, T[6];
          op_row(L, i, j, k, c, D, T);
          sum += (R)b[c] - (D * x[c] - op_off(L, c, T, x));
        }
      }
    }
    bc[I + cn0 * (J + cn1 * K)] = sum;
  }
}

// x_fine += x_coarse(parent) on a coarse level
template <typename R>
__global__ void __launch_bounds__(NTHREADS) k_prolong(const LvS *__restrict__ ls, SH S,
                                                      const R *__restrict__ xc,
                                                      R *__restrict__ x,
                                                      const int *__restrict__ mask) {
  int g, s, lb;
  if (!locate(S, mask, g, s, lb)) return;
  const LvS &Q = ls[s];
  const int n0 = Q.n0, n1 = Q.n1, n2 = Q.n2, cn0 = Q.cn0, cn1 = Q.cn1;
  x += Q.c0;
  xc += Q.cc0;
  int i, j, k0, k1;
  if (!column(n0, n1, n2, lb, S.kz, false, i, j, k0, k1)) return;
  int c = i + n0 * (j + n1 * k0);
  for (int k = k0; k < k1; k++, c += n0 * n1)
    x[c] += xc[(i >> 1) + cn0 * ((j >> 1) + cn1 * (k >> 1))];
}

// coarse operator of the next level from this level's operator; the launch
// covers the coarse cells of every sample that has the coarse level
template <typename R>
__global__ void __launch_bounds__(NTHREADS) k_build_coarse(OpB<R> LB, const R *__restrict__ Dbf,
                                                           SH S, R *__restrict__ Tx,
                                                           R *__restrict__ Ty,
                                                           R *__restrict__ Tz,
                                                           R *__restrict__ Db) {
  int g, s, lb;
  if (!locate(S, nullptr, g, s, lb)) return;
  const Op<R> L = op_at(LB, s);
  const LvS &Q = LB.ls[s];
  if (Dbf) Dbf += Q.c0;
  Tx += Q.cc0; Ty += Q.cc0; Tz += Q.cc0; Db += Q.cc0;
  const int cn0 = Q.cn0, cn1 = Q.cn1, cn2 = Q.cn2;
  int I, J, K0, K1;
  if (!column(cn0, cn1, cn2, lb, S.kz, false, I, J, K0, K1)) return;
  for (int K = K0; K < K1; K++) {
    R tx = 0, ty = 0, tz = 0, db = 0;
    for (int dk = 0; dk < 2; dk++)
      for (int dj = 0; dj < 2; dj++)
        for (int di = 0; di < 2; di++) {
          const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
          if (i >= L.n0 || j >= L.n1 || k >= L.n2) continue;
          const int c = i + L.n0 * (j + L.n1 * k);
          R D, T[6];
          op_row(L, i, j, k, c, D, T);
          if (di == 1) tx += T[1];
          if (dj == 1) ty += T[3];
          if (dk == 1) tz += T[5];
          db += L.matfree ? op_outlet(L, i, j, k, c) : Dbf[c];
        }
    const int C = I + cn0 * (J + cn1 * K);
    Tx[C] = (R)0.5 * tx;
    Ty[C] = (R)0.5 * ty;
    Tz[C] = (R)0.5 * tz;
    Db[C] = (R)0.5 * db;
  }
}

template <typename R>
__global__ void __launch_bounds__(NTHREADS) k_diag(const LvS *__restrict__ ls, SH S,
                                                   const R *__restrict__ Tx,
                                                   const R *__restrict__ Ty,
                                                   const R *__restrict__ Tz,
                                                   const R *__restrict__ Db,
                                                   R *__restrict__ D) {
  int g, s, lb;
  if (!locate(S, nullptr, g, s, lb)) return;
  const LvS &Q = ls[s];
  const int n0 = Q.n0, n1 = Q.n1, n2 = Q.n2;
  Tx += Q.c0; Ty += Q.c0; Tz += Q.c0; Db += Q.c0; D += Q.c0;
  int i, j, k0, k1;
  if (!column(n0, n1, n2, lb, S.kz, false, i, j, k0, k1)) return;
  const int sy = n0, sz = n0 * n1;
  int c = i + n0 * (j + n1 * k0);
  for (int k = k0; k < k1; k++, c += sz) {
    R d = Db[c] + Tx[c] + Ty[c] + Tz[c];
    if (i > 0) d += Tx[c - 1];
    if (j > 0) d += Ty[c - sy];
    if (k > 0) d += Tz[c - sz];
    D[c] = d;
  }
}

// 1/D for the smoother: the hardware reciprocal in FP32 (the V-cycle is a
// preconditioner; the outer FP64 CG is unaffected), exact in FP64
__device__ __forceinline__ float sw_rcp(float d) { return __builtin_amdgcn_rcpf(d); }
__device__ __forceinline__ double sw_rcp(double d) { return 1.0 / d; }

// ----------------------------------------------- single work-group bottom
//
// The smallest levels of a sample (from the first one whose whole
// sub-hierarchy fits in BOTTOM_LDS bytes) are cycled by one work-group of
// 1024 threads with every array in LDS: coefficients and b of the top bottom
// level are loaded once, the V-cycle runs with LDS-latency barriers, and x
// goes back to memory.  One work-group per sample.

template <typename R>
struct BLevel {
  int n0, n1, n2, off;  // off: first cell of the level in the LDS arrays
  const R *Tx, *Ty, *Tz, *D;
  R *x, *b;             // global x and b (b read and x written for the top level)
};

// Each LDS array is preceded by `pad` zero cells (pad >= one plane of the
// top level).  Face coefficients are zero on domain faces, so every
// neighbour term is formed without a test: an index past a level's edge
// lands on a zero coefficient of the same level, on a domain face of the
// previous (larger) level or in a pad, and multiplies a finite x (all of x
// starts at zero).
template <typename R>
struct Bottom {
  int s;                // sample
  int nl, ntot, pad;
  int pre, post, coarse_sweeps;
  BLevel<R> L[MAXLV];
};

template <typename R>
struct LdsView {
  R *tx, *ty, *tz, *d, *x, *b;
};

// q / d for 0 <= q < 2^22 and d >= 1: a float reciprocal and one
// correction (the float product is within 1/2 of q/d), no integer division
__device__ __forceinline__ int sdiv(int q, int d, float invd) {
  int t = (int)((float)q * invd);
  t -= (t * d > q) ? 1 : 0;
  t += ((t + 1) * d <= q) ? 1 : 0;
  return t;
}

// s plus the six neighbour terms of LDS cell g (row stride sy, plane sz)
template <typename R>
__device__ __forceinline__ R bl_nsum(const LdsView<R> &S, int g, int sy, int sz, R s) {
  s += S.tx[g - 1] * S.x[g - 1];
  s += S.tx[g] * S.x[g + 1];
  s += S.ty[g - sy] * S.x[g - sy];
  s += S.ty[g] * S.x[g + sy];
  s += S.tz[g - sz] * S.x[g - sz];
  s += S.tz[g] * S.x[g + sz];
  return s;
}

// (A x) at LDS cell g
template <typename R>
__device__ __forceinline__ R bl_ax(const LdsView<R> &S, int g, int sy, int sz) {
  R ax = S.d[g] * S.x[g];
  ax -= S.tx[g - 1] * S.x[g - 1];
  ax -= S.tx[g] * S.x[g + 1];
  ax -= S.ty[g - sy] * S.x[g - sy];
  ax -= S.ty[g] * S.x[g + sy];
  ax -= S.tz[g - sz] * S.x[g - sz];
  ax -= S.tz[g] * S.x[g + sz];
  return ax;
}

// one red-black half sweep of a bottom level over pairs of cells along x,
// two pairs per thread iteration with both pairs' loads issued before
// either store; the pair's cell of this colour is relaxed (zero: x = b/D on
// this colour and 0 on the other)
template <typename R>
__device__ inline void bl_sweep(const LdsView<R> &S, const BLevel<R> &L, int color, bool zero) {
  const int n0 = L.n0, n1 = L.n1;
  const int hx = (n0 + 1) >> 1, np = hx * n1 * L.n2;
  const int sy = n0, sz = n0 * n1;
  const float ihx = 1.0f / (float)hx, in1 = 1.0f / (float)n1;
  const int bs = blockDim.x;
  for (int q0 = threadIdx.x; q0 < np; q0 += 2 * bs) {
    int g[2], io[2];
    bool on[2];
    R v[2];
#pragma unroll
    for (int u = 0; u < 2; u++) {
      // a second pair past the end repeats the first (same value, same place)
      const int q = q0 + u * bs < np ? q0 + u * bs : q0;
      const int row = sdiv(q, hx, ihx), iq = q - row * hx;
      const int k = sdiv(row, n1, in1), j = row - k * n1;
      const int off = (j + k + color) & 1;  // (i + j + k) & 1 == color
      const int i = 2 * iq + off;
      g[u] = L.off + i + n0 * row;
      on[u] = i < n0;
      io[u] = 2 * iq + 1 - off < n0 ? 1 - 2 * off : 0;  // other cell of the pair
      const R d = S.d[g[u]];
      const R s = zero ? S.b[g[u]] : bl_nsum(S, g[u], sy, sz, S.b[g[u]]);
      v[u] = d > (R)0 ? s * sw_rcp(d) : (R)0;
    }
#pragma unroll
    for (int u = 0; u < 2; u++) {
      if (on[u]) S.x[g[u]] = v[u];
      if (zero && io[u] != 0) S.x[g[u] + io[u]] = (R)0;
    }
  }
  __syncthreads();
}

// The pairs of a level that one thread relaxes when the level has at most
// NP x 1024 pairs (pair q = threadIdx.x + 1024 u): first LDS cell, x index
// and parity of j + k, computed once per visit of the level.  A missing
// pair points at the level's first cell and stores nothing.
template <int NP>
struct BPairs {
  int g[NP], i2[NP], par[NP];
  bool ok[NP];
};

template <typename R, int NP>
__device__ inline BPairs<NP> bl_pairs(const BLevel<R> &L) {
  const int n0 = L.n0, n1 = L.n1;
  const int hx = (n0 + 1) >> 1, np = hx * n1 * L.n2;
  const float ihx = 1.0f / (float)hx, in1 = 1.0f / (float)n1;
  BPairs<NP> P;
#pragma unroll
  for (int u = 0; u < NP; u++) {
    const int q = (int)threadIdx.x + 1024 * u;
    P.ok[u] = q < np;
    const int qq = P.ok[u] ? q : 0;
    const int row = sdiv(qq, hx, ihx), iq = qq - row * hx;
    const int k = sdiv(row, n1, in1), j = row - k * n1;
    P.g[u] = L.off + 2 * iq + n0 * row;
    P.i2[u] = 2 * iq;
    P.par[u] = (j + k) & 1;
  }
  return P;
}

// half sweep of colour `color` over planned pairs; the loads of all pairs
// are issued before any store
template <typename R, int NP>
__device__ inline void bl_sweep_p(const LdsView<R> &S, const BLevel<R> &L, const BPairs<NP> &P,
                                  int color, bool zero) {
  const int n0 = L.n0, sy = n0, sz = n0 * L.n1;
  int g[NP], o[NP];
  R v[NP];
#pragma unroll
  for (int u = 0; u < NP; u++) {
    o[u] = (P.par[u] + color) & 1;  // (i + j + k) & 1 == color
    g[u] = P.g[u] + (P.ok[u] ? o[u] : 0);
    const R d = S.d[g[u]];
    const R sum = zero ? S.b[g[u]] : bl_nsum(S, g[u], sy, sz, S.b[g[u]]);
    v[u] = d > (R)0 ? sum * sw_rcp(d) : (R)0;
  }
#pragma unroll
  for (int u = 0; u < NP; u++) {
    if (P.ok[u] && P.i2[u] + o[u] < n0) S.x[g[u]] = v[u];
    if (zero && P.ok[u] && P.i2[u] + 1 - o[u] < n0) S.x[g[u] + 1 - 2 * o[u]] = (R)0;
  }
  __syncthreads();
}

// ns sweeps of a bottom level, each colour c0 then 1 - c0 (zero: the first
// starts from x = 0)
template <typename R>
__device__ inline void bl_smooth(const LdsView<R> &S, const BLevel<R> &L, int ns, int c0,
                                 bool zero) {
  const int np = ((L.n0 + 1) >> 1) * L.n1 * L.n2;
  if (np <= 1024) {
    const BPairs<1> P = bl_pairs<R, 1>(L);
    for (int s = 0; s < ns; s++) {
      bl_sweep_p<R, 1>(S, L, P, c0, zero && s == 0);
      bl_sweep_p<R, 1>(S, L, P, 1 - c0, false);
    }
  } else if (np <= 2048) {
    const BPairs<2> P = bl_pairs<R, 2>(L);
    for (int s = 0; s < ns; s++) {
      bl_sweep_p<R, 2>(S, L, P, c0, zero && s == 0);
      bl_sweep_p<R, 2>(S, L, P, 1 - c0, false);
    }
  } else {
    for (int s = 0; s < ns; s++) {
      bl_sweep(S, L, c0, zero && s == 0);
      bl_sweep(S, L, 1 - c0, false);
    }
  }
}

// b of the coarser level: the sum of the residuals of a cell's (up to 8)
// children; a missing child (odd size) reads the first child and adds zero.
// red: the smoothing ended with a black half sweep, whose cells have zero
// residual, so only the red children (even i + j + k) are summed.
template <typename R>
__device__ inline void bl_restrict(const LdsView<R> &S, const BLevel<R> &F, const BLevel<R> &C,
                                   bool red) {
  const int n = C.n0 * C.n1 * C.n2;
  const int sy = F.n0, sz = F.n0 * F.n1;
  const float cin0 = 1.0f / (float)C.n0, cin1 = 1.0f / (float)C.n1;
  for (int cc = threadIdx.x; cc < n; cc += blockDim.x) {
    const int crow = sdiv(cc, C.n0, cin0), I = cc - crow * C.n0;
    const int K = sdiv(crow, C.n1, cin1), J = crow - K * C.n1;
    const int g0 = F.off + 2 * I + F.n0 * (2 * J + F.n1 * 2 * K);
    R s = 0;
#pragma unroll
    for (int dk = 0; dk < 2; dk++)
#pragma unroll
      for (int dj = 0; dj < 2; dj++)
#pragma unroll
        for (int di = 0; di < 2; di++) {
          if (red && ((di + dj + dk) & 1)) continue;
          const bool ok = 2 * I + di < F.n0 && 2 * J + dj < F.n1 && 2 * K + dk < F.n2;
          const int g = ok ? g0 + di + sy * dj + sz * dk : g0;
          const R r = S.b[g] - bl_ax(S, g, sy, sz);
          s += ok ? r : (R)0;
        }
    S.b[C.off + cc] = s;
  }
  __syncthreads();
}

template <typename R>
__device__ inline void bl_prolong(const LdsView<R> &S, const BLevel<R> &F, const BLevel<R> &C) {
  const int n = F.n0 * F.n1 * F.n2;
  const float in0 = 1.0f / (float)F.n0, in1 = 1.0f / (float)F.n1;
  for (int c = threadIdx.x; c < n; c += blockDim.x) {
    const int row = sdiv(c, F.n0, in0), i = c - row * F.n0;
    const int k = sdiv(row, F.n1, in1), j = row - k * F.n1;
    S.x[F.off + c] += S.x[C.off + (i >> 1) + C.n0 * ((j >> 1) + C.n1 * (k >> 1))];
  }
  __syncthreads();
}

// cells of the bottom hierarchy one thread loads (coefficients and b)
template <typename R>
constexpr int bottom_cells_per_thread() {
  return (int)((BOTTOM_LDS / (6 * sizeof(R)) + 1023) / 1024);
}

template <typename R>
__global__ void __launch_bounds__(1024) k_bottom(const Bottom<R> *__restrict__ tab,
                                                 const int *__restrict__ mask) {
  __shared__ __align__(16) R lds[BOTTOM_LDS / sizeof(R)];
  __shared__ const R *ptab[MAXLV][5];  // per level: Tx, Ty, Tz, D, b
  const Bottom<R> &A = tab[blockIdx.x];
  if (mask && !mask[A.s]) return;
  const int N = A.ntot, P = A.pad, ST = N + P, nl = A.nl;
  if ((int)threadIdx.x < nl) {
    const BLevel<R> &L = A.L[threadIdx.x];
    ptab[threadIdx.x][0] = L.Tx;
    ptab[threadIdx.x][1] = L.Ty;
    ptab[threadIdx.x][2] = L.Tz;
    ptab[threadIdx.x][3] = L.D;
    ptab[threadIdx.x][4] = L.b;
  }
  LdsView<R> S{lds + P, lds + P + ST, lds + P + 2 * ST, lds + P + 3 * ST, lds + P + 4 * ST,
               lds + P + 5 * ST};
  // zero every array and pad (x starts at zero; pads stay zero)
  {
    constexpr int V = 16 / sizeof(R);
    const int nv = (6 * ST + V - 1) / V;
    static_assert(BOTTOM_LDS % 16 == 0, "whole vectors");
    float4 *l4 = reinterpret_cast<float4 *>(lds);
    for (int e = threadIdx.x; e < nv; e += 1024) l4[e] = make_float4(0.f, 0.f, 0.f, 0.f);
  }
  __syncthreads();
  // coefficients and b of every level, all loads in flight before the
  // stores (b of the levels below the top is loaded and later overwritten)
  {
    constexpr int U = bottom_cells_per_thread<R>();
    R v[U][5];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int e0 = threadIdx.x + u * 1024;
      const int e = e0 < N ? e0 : N - 1;
      int m = 0, off = 0;
      for (int q = 1; q < nl; q++) {
        const int oq = A.L[q].off;
        m += e >= oq ? 1 : 0;
        off = e >= oq ? oq : off;
      }
      const int c = e - off;
#pragma unroll
      for (int a = 0; a < 5; a++) v[u][a] = ptab[m][a][c];
    }
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int e = threadIdx.x + u * 1024;
      if (e < N) {
        S.tx[e] = v[u][0];
        S.ty[e] = v[u][1];
        S.tz[e] = v[u][2];
        S.d[e] = v[u][3];
        S.b[e] = v[u][4];
      }
    }
  }
  __syncthreads();
  for (int l = 0; l < nl - 1; l++) {
    bl_smooth(S, A.L[l], A.pre, 0, true);
    bl_restrict(S, A.L[l], A.L[l + 1], A.pre > 0);
  }
  // coarsest level; a single cell is solved by its first half sweep
  const BLevel<R> &C = A.L[nl - 1];
  const bool one = C.n0 * C.n1 * C.n2 == 1;
  bl_smooth(S, C, A.coarse_sweeps, 0, true);
  if (!one) bl_smooth(S, C, A.coarse_sweeps, 1, false);
  for (int l = nl - 2; l >= 0; l--) {
    bl_prolong(S, A.L[l], A.L[l + 1]);
    bl_smooth(S, A.L[l], A.post, 1, false);
  }
  const BLevel<R> &T = A.L[0];
  const int n = T.n0 * T.n1 * T.n2;
  for (int c = threadIdx.x; c < n; c += 1024) T.x[c] = S.x[T.off + c];
}

// ------------------------------------------------ fine level, 2.5-D tiles
//
// A block of 64 x TY2 threads owns a tile of W x TY2 cells (W = 64 one cell
// per thread, or 128 with an x-pair per thread) and walks kz planes.  Each
// plane of x (or p) and rAU is staged with a one-cell halo in LDS; the z
// neighbours of a thread's own cells stay in registers, so each array is
// read from memory about once per pass (plus the halo and the chunk ends).

constexpr int TY2 = 8;
constexpr int KZ2 = 16;
constexpr int NT2 = 64 * TY2;
constexpr int MIN_BLOCKS2 = 1024;
constexpr int MIN_BLOCKS_CSW = 256;  // fused coarse sweeps (one block per CU)
constexpr int CSW_MIN_DEPTH = 8;     // planes a level needs for fused coarse sweeps

__host__ __device__ inline int tiles25(int n0, int n1, int n2, int W, int kz) {
  return ((n0 + W - 1) / W) * ((n1 + TY2 - 1) / TY2) * ((n2 + kz - 1) / kz);
}

__device__ __forceinline__ void tile_of(int lb, int n0, int n1, int n2, int W, int kz, int &x0b,
                                        int &y0, int &k0, int &k1) {
  const int nbx = (n0 + W - 1) / W, nby = (n1 + TY2 - 1) / TY2;
  x0b = lb % nbx;
  const int L = lb / nbx;
  y0 = (L % nby) * TY2;
  k0 = (L / nby) * kz;
  k1 = min(k0 + kz, n2);
}

#define LIX(W, lx, ly) (((ly) + 1) * ((W) + 2) + (lx) + 1)

template <int NW>
__device__ __forceinline__ double block_sum_n(double v, double *lds) {
  v = wave_sum(v);
  const int t = threadIdx.x + 64 * threadIdx.y;
  if ((t & 63) == 0) lds[t >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (t == 0)
    for (int q = 0; q < NW; q++) s += lds[q];
  __syncthreads();
  return s;
}

template <typename R>
__device__ __forceinline__ R ld_or0(const R *__restrict__ a, int i, int j, int k, int n0, int n1,
                                    int n2) {
  return (i >= 0 && i < n0 && j >= 0 && j < n1 && k >= 0 && k < n2) ? a[i + n0 * (j + n1 * k)]
                                                                     : (R)0;
}

// two cells of one thread, selected without dynamic register indexing
template <typename R>
struct P2 {
  R v0, v1;
  __device__ __forceinline__ R get(int off) const { return off ? v1 : v0; }
  __device__ __forceinline__ void set(int off, R v) {
    if (off) v1 = v; else v0 = v;
  }
};

template <typename R> struct Vec16;
template <> struct Vec16<float> { using T = float4; using T2 = float2; };
template <> struct Vec16<double> { using T = double2; using T2 = double2; };

// component access and arithmetic on the 16-byte vectors (indices are
// compile-time constants after unrolling, so these stay in registers)
template <typename VT> __device__ __forceinline__ VT vzero();
template <> __device__ __forceinline__ float4 vzero<float4>() { return make_float4(0.f, 0.f, 0.f, 0.f); }
template <> __device__ __forceinline__ double2 vzero<double2>() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ void vset(float4 &v, int u, float a) {
  if (u == 0) v.x = a; else if (u == 1) v.y = a; else if (u == 2) v.z = a; else v.w = a;
}
__device__ __forceinline__ void vset(double2 &v, int u, double a) {
  if (u == 0) v.x = a; else v.y = a;
}
// packed parents (one per two cells) spread over the vector's cells
__device__ __forceinline__ float4 vspread(float4 a) { return make_float4(a.x, a.x, a.y, a.y); }
__device__ __forceinline__ double2 vspread(double2 a) { return make_double2(a.x, a.x); }
__device__ __forceinline__ float4 vadd(float4 a, float4 b) {
  return make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
}
__device__ __forceinline__ double2 vadd(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}


// row of the fine operator at (i,j,k) from the seven rAU values around it
template <typename R>
__device__ __forceinline__ void coef7(const Op<R> &L, int i, int j, int k, R rc, R rxm, R rxp,
                                      R rym, R ryp, R rzm, R rzp, R T[6], R &D) {
  const R h = (R)0.5;
  T[0] = i > 0 ? h * (rc + rxm) * L.c[0] : (R)0;
  T[1] = i + 1 < L.n0 ? h * (rc + rxp) * L.c[0] : (R)0;
  T[2] = j > 0 ? h * (rc + rym) * L.c[1] : (R)0;
  T[3] = j + 1 < L.n1 ? h * (rc + ryp) * L.c[1] : (R)0;
  T[4] = k > 0 ? h * (rc + rzm) * L.c[2] : (R)0;
  T[5] = k + 1 < L.n2 ? h * (rc + rzp) * L.c[2] : (R)0;
  const R db = (i == 0 ? L.ob[0] : (R)0) + (i + 1 == L.n0 ? L.ob[1] : (R)0) +
               (j == 0 ? L.ob[2] : (R)0) + (j + 1 == L.n1 ? L.ob[3] : (R)0) +
               (k == 0 ? L.ob[4] : (R)0) + (k + 1 == L.n2 ? L.ob[5] : (R)0);
  D = T[0] + T[1] + T[2] + T[3] + T[4] + T[5] + rc * db;
}

// The FP64 operator row in difference form: (A x)_P = sum_f T_f (x_P - x_N)
// + Dirichlet part x_P.  Same value as D x_P - sum_f T_f x_N, but the
// rounding error scales with the differences instead of |x|, so the
// attainable residual of a pressure field far from zero mean (closed boxes,
// large hydrostatic levels) does not stall above the oracle's.
__device__ __forceinline__ double row_diff(const Op<double> &L, int i, int j, int k, double rc,
                                           double rxm, double rxp, double rym, double ryp,
                                           double rzm, double rzp, double pc, double pxm,
                                           double pxp, double pym, double pyp, double pzm,
                                           double pzp) {
  double T[6], D;
  coef7(L, i, j, k, rc, rxm, rxp, rym, ryp, rzm, rzp, T, D);
  const double db = (i == 0 ? L.ob[0] : 0.0) + (i + 1 == L.n0 ? L.ob[1] : 0.0) +
                    (j == 0 ? L.ob[2] : 0.0) + (j + 1 == L.n1 ? L.ob[3] : 0.0) +
                    (k == 0 ? L.ob[4] : 0.0) + (k + 1 == L.n2 ? L.ob[5] : 0.0);
  return T[0] * (pc - pxm) + T[1] * (pc - pxp) + T[2] * (pc - pym) + T[3] * (pc - pyp) +
         T[4] * (pc - pzm) + T[5] * (pc - pzp) + rc * db * pc;
}

// The same row when the neighbour values outside the mesh are zero (as in
// the LDS planes): T = (rc + rn) hc needs no mask, since its product with a
// zero iterate vanishes, and D removes the spurious rc hc of each face to
// the outside again while adding the outlet's Dirichlet part: e = ob - hc
// per domain side.  hc = c/2 is exact, so T is the same number as h (rc +
// rn) c; D differs from the masked sum in rounding only.
template <typename R>
struct RowK {
  R hc[3];
  R e[6];
};
template <typename R>
__device__ __forceinline__ RowK<R> rowk(const Op<R> &L) {
  RowK<R> K;
  for (int a = 0; a < 3; a++) K.hc[a] = (R)0.5 * L.c[a];
  for (int q = 0; q < 6; q++) K.e[q] = L.ob[q] - K.hc[q >> 1];
  return K;
}
template <typename R>
__device__ __forceinline__ void coefu(const RowK<R> &K, int i, int j, int k, int n0, int n1,
                                      int n2, R rc, R rxm, R rxp, R rym, R ryp, R rzm, R rzp,
                                      R T[6], R &D) {
  T[0] = (rc + rxm) * K.hc[0];
  T[1] = (rc + rxp) * K.hc[0];
  T[2] = (rc + rym) * K.hc[1];
  T[3] = (rc + ryp) * K.hc[1];
  T[4] = (rc + rzm) * K.hc[2];
  T[5] = (rc + rzp) * K.hc[2];
  const R db = (i == 0 ? K.e[0] : (R)0) + (i + 1 == n0 ? K.e[1] : (R)0) +
               (j == 0 ? K.e[2] : (R)0) + (j + 1 == n1 ? K.e[3] : (R)0) +
               (k == 0 ? K.e[4] : (R)0) + (k + 1 == n2 ? K.e[5] : (R)0);
  D = T[0] + T[1] + T[2] + T[3] + T[4] + T[5] + rc * db;
}

// Planes of a W x TY2 tile staged in LDS with a ring of one 16-byte vector
// in x and RY rows in y (zero outside the mesh).  Thread t loads vectors t,
// t + NT2, ... of a plane into registers one plane step before it stores
// them, so the loads are in flight while the current plane is computed.
// With four slots per array one barrier per plane suffices: the slot
// written at plane k+1 held plane k-3, which no thread still reads.
template <typename R, int W, int RY>
struct PlG {
  static constexpr int VEC = 16 / sizeof(R);
  static constexpr int RX = VEC;                // x-ring width (cells)
  static constexpr int FXR = W + 2 * RX;        // row stride
  static constexpr int NX = FXR * (TY2 + 2 * RY);  // elements per plane
  static constexpr int NV = NX / VEC;           // vectors per plane
  static constexpr int MV = (NV + NT2 - 1) / NT2;
  __device__ static constexpr int at(int lx, int ly) { return (ly + RY) * FXR + lx + RX; }
};
template <typename R, int W>
using Pl1 = PlG<R, W, 1>;

template <int NS>
__device__ __forceinline__ int slot_of(int k) { return (k + NS) % NS; }  // k >= -NS

// vector handled by thread t in pass m of a plane of NV vectors: threads past
// the end repeat a vector of the last pass (same value to the same place),
// so every thread stores unconditionally and no load is left pending on a
// path that skipped its store
template <int NV, int MV>
__device__ __forceinline__ int pl_vec(int t, int m) {
  static_assert(2 * NV >= MV * NT2 && NV <= MV * NT2, "plane vectors per pass");
  const int e = t + m * NT2;
  return e < NV ? e : e - (MV * NT2 - NV);
}

// A sample's array as a buffer resource: loads at byte offsets at or past
// its end return zero, so cells outside the mesh need no branch (and no
// load waits on a path that skipped it).
struct Buf {
  __amdgpu_buffer_rsrc_t r;
  unsigned oob;  // an offset past the end
};
template <typename R>
__device__ __forceinline__ Buf mkbuf(const R *base, int n) {
  const unsigned bytes = (unsigned)n * (unsigned)sizeof(R);
  // 0x00020000: 32-bit data format of a raw (unstructured) buffer on CDNA
  return Buf{__builtin_amdgcn_make_buffer_rsrc((void *)base, (short)0, (int)bytes, 0x00020000),
             bytes};
}
__device__ __forceinline__ float4 bld_vec(const Buf &B, unsigned off, float4) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(B.r, off, 0, 0);
  return make_float4(__uint_as_float(v[0]), __uint_as_float(v[1]), __uint_as_float(v[2]),
                     __uint_as_float(v[3]));
}
__device__ __forceinline__ double2 bld_vec(const Buf &B, unsigned off, double2) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b128(B.r, off, 0, 0);
  return make_double2(__hiloint2double((int)v[1], (int)v[0]),
                      __hiloint2double((int)v[3], (int)v[2]));
}
__device__ __forceinline__ float bld1(const Buf &B, unsigned off, float) {
  return __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(B.r, off, 0, 0));
}
__device__ __forceinline__ double bld1(const Buf &B, unsigned off, double) {
  const auto v = __builtin_amdgcn_raw_buffer_load_b64(B.r, off, 0, 0);
  return __hiloint2double((int)v[1], (int)v[0]);
}

// vector m of thread t of plane k of a sample's array B (zero outside the
// mesh).  VOK: n0 is a multiple of the vector length, so rows start on
// 16-byte boundaries and a vector is wholly inside or outside; otherwise
// cells are loaded one by one.
template <typename PL, bool VOK, typename R>
__device__ __forceinline__ typename Vec16<R>::T pl_load(const Buf &B, int t, int m, int x0,
                                                        int y0, int k, int n0, int n1, int n2) {
  using VT = typename Vec16<R>::T;
  constexpr int VEC = PL::VEC, RV = PL::FXR / VEC, RY = (PL::NX / PL::FXR - TY2) / 2;
  const int e = pl_vec<PL::NV, PL::MV>(t, m);
  const int ia = x0 - PL::RX + (e % RV) * VEC, jj = y0 - RY + e / RV;
  const bool in = jj >= 0 && jj < n1 && k >= 0 && k < n2 && ia + VEC > 0 && ia < n0;
  const int c = ia + n0 * (jj + n1 * k);
  if (VOK) return bld_vec(B, in ? (unsigned)c * (unsigned)sizeof(R) : B.oob, VT{});
  VT v;
#pragma unroll
  for (int u = 0; u < VEC; u++) {
    const bool ok = in && ia + u >= 0 && ia + u < n0;
    vset(v, u, bld1(B, ok ? (unsigned)(c + u) * (unsigned)sizeof(R) : B.oob, R{}));
  }
  return v;
}

template <typename PL, typename R>
__device__ __forceinline__ void pl_store(R *s, int t, int m, typename Vec16<R>::T v) {
  const int e = pl_vec<PL::NV, PL::MV>(t, m);
  *reinterpret_cast<typename Vec16<R>::T *>(s + e * PL::VEC) = v;
}

// Halo of one plane for a thread: the cell left of the tile (tx == 0), right
// of it (tx == 63), and below / above its two cells (ty == 0 / ty == TY2-1),
// for the iterate and rAU.  Loaded one plane ahead, so the loads are in
// flight while the current plane is computed.  Plain scalars (no arrays):
// they must stay in registers.
template <typename R>
struct Halo {
  R xl, xr, rl, rr, xs0, xs1, xn0, xn1, rs0, rs1, rn0, rn1;
};

template <typename R, int CPT, int W, typename FX>
__device__ __forceinline__ Halo<R> halo_load(const FX &X, const R *__restrict__ rA, int x0, int y0,
                                             int i0, int j, int k, int n0, int n1, int n2) {
  const int tx = threadIdx.x, ty = threadIdx.y;
  Halo<R> h;
  const bool L = tx == 0, Rt = tx == 63, S = ty == 0, N = ty == TY2 - 1;
  h.xl = L ? X(x0 - 1, j, k) : (R)0;
  h.rl = L ? ld_or0(rA, x0 - 1, j, k, n0, n1, n2) : (R)0;
  h.xr = Rt ? X(x0 + W, j, k) : (R)0;
  h.rr = Rt ? ld_or0(rA, x0 + W, j, k, n0, n1, n2) : (R)0;
  h.xs0 = S ? X(i0, y0 - 1, k) : (R)0;
  h.rs0 = S ? ld_or0(rA, i0, y0 - 1, k, n0, n1, n2) : (R)0;
  h.xn0 = N ? X(i0, y0 + TY2, k) : (R)0;
  h.rn0 = N ? ld_or0(rA, i0, y0 + TY2, k, n0, n1, n2) : (R)0;
  h.xs1 = (S && CPT == 2) ? X(i0 + 1, y0 - 1, k) : (R)0;
  h.rs1 = (S && CPT == 2) ? ld_or0(rA, i0 + 1, y0 - 1, k, n0, n1, n2) : (R)0;
  h.xn1 = (N && CPT == 2) ? X(i0 + 1, y0 + TY2, k) : (R)0;
  h.rn1 = (N && CPT == 2) ? ld_or0(rA, i0 + 1, y0 + TY2, k, n0, n1, n2) : (R)0;
  return h;
}

template <typename R, int CPT, int W>
__device__ __forceinline__ void halo_store(const Halo<R> &h, R *sx, R *sr) {
  const int tx = threadIdx.x, ty = threadIdx.y;
  if (tx == 0) { sx[LIX(W, -1, ty)] = h.xl; sr[LIX(W, -1, ty)] = h.rl; }
  if (tx == 63) { sx[LIX(W, W, ty)] = h.xr; sr[LIX(W, W, ty)] = h.rr; }
  if (ty == 0) {
    sx[LIX(W, CPT * tx, -1)] = h.xs0;
    sr[LIX(W, CPT * tx, -1)] = h.rs0;
    if (CPT == 2) { sx[LIX(W, CPT * tx + 1, -1)] = h.xs1; sr[LIX(W, CPT * tx + 1, -1)] = h.rs1; }
  }
  if (ty == TY2 - 1) {
    sx[LIX(W, CPT * tx, TY2)] = h.xn0;
    sr[LIX(W, CPT * tx, TY2)] = h.rn0;
    if (CPT == 2) { sx[LIX(W, CPT * tx + 1, TY2)] = h.xn1; sr[LIX(W, CPT * tx + 1, TY2)] = h.rn1; }
  }
}

// row of the fine operator at (i,j,k), lx/ty its LDS position; z
// neighbours' rAU from registers
template <typename R, int W>
__device__ __forceinline__ void row25(const Op<R> &L, int i, int j, int k, int lx, int ty,
                                      const R *sr, R rc, R rm, R rp, R T[6], R &D) {
  const R h = (R)0.5;
  T[0] = i > 0 ? h * (rc + sr[LIX(W, lx - 1, ty)]) * L.c[0] : (R)0;
  T[1] = i + 1 < L.n0 ? h * (rc + sr[LIX(W, lx + 1, ty)]) * L.c[0] : (R)0;
  T[2] = j > 0 ? h * (rc + sr[LIX(W, lx, ty - 1)]) * L.c[1] : (R)0;
  T[3] = j + 1 < L.n1 ? h * (rc + sr[LIX(W, lx, ty + 1)]) * L.c[1] : (R)0;
  T[4] = k > 0 ? h * (rc + rm) * L.c[2] : (R)0;
  T[5] = k + 1 < L.n2 ? h * (rc + rp) * L.c[2] : (R)0;
  const R db = (i == 0 ? L.ob[0] : (R)0) + (i + 1 == L.n0 ? L.ob[1] : (R)0) +
               (j == 0 ? L.ob[2] : (R)0) + (j + 1 == L.n1 ? L.ob[3] : (R)0) +
               (k == 0 ? L.ob[4] : (R)0) + (k + 1 == L.n2 ? L.ob[5] : (R)0);
  D = T[0] + T[1] + T[2] + T[3] + T[4] + T[5] + rc * db;
}

template <typename R, int W>
__device__ __forceinline__ R off25(const R T[6], int lx, int ty, const R *sx, R xm, R xp) {
  return T[0] * sx[LIX(W, lx - 1, ty)] + T[1] * sx[LIX(W, lx + 1, ty)] +
         T[2] * sx[LIX(W, lx, ty - 1)] + T[3] * sx[LIX(W, lx, ty + 1)] + T[4] * xm + T[5] * xp;
}

// two cells of the preconditioned residual z in the raw loaded form (kept
// unconverted until the plane is stored)
template <typename Z> struct ZPair;
template <> struct ZPair<float> {
  using T = unsigned __attribute__((ext_vector_type(2)));
  __device__ static T ld(const Buf &B, unsigned off) {
    return __builtin_amdgcn_raw_buffer_load_b64(B.r, off, 0, 0);
  }
  __device__ static double get(const T &v, int u) { return (double)__uint_as_float(v[u]); }
  __device__ static T one(const Buf &B, unsigned off, T v, int u) {
    v[u] = __builtin_amdgcn_raw_buffer_load_b32(B.r, off, 0, 0);
    return v;
  }
};
template <> struct ZPair<double> {
  using T = unsigned __attribute__((ext_vector_type(4)));
  __device__ static T ld(const Buf &B, unsigned off) {
    return __builtin_amdgcn_raw_buffer_load_b128(B.r, off, 0, 0);
  }
  __device__ static double get(const T &v, int u) {
    return __hiloint2double((int)v[2 * u + 1], (int)v[2 * u]);
  }
  __device__ static T one(const Buf &B, unsigned off, T v, int u) {
    const auto w = __builtin_amdgcn_raw_buffer_load_b64(B.r, off, 0, 0);
    v[2 * u] = w[0];
    v[2 * u + 1] = w[1];
    return v;
  }
};

// MODE 0: q = A p and partial p.q.  MODE 1: r = b - A p (and its FP32 copy)
// and partials r.r, b.b.  MODE 2: the CG direction update fused in front of
// MODE 0: p_new = z + beta p (p_new = z when first) is formed while the
// planes are staged (ring cells included, from z and the old p, which no
// block writes), written for the tile's own cells to a second buffer (with
// the copy z_old = z of flexible CG when zold is given), and q = A p_new,
// p_new.q follow.
// 64 x 8 tiles walk up to kz planes; the inputs are staged in LDS slots,
// two planes in flight (one cell per thread).
template <int MODE, typename Z = double>
__global__ void __launch_bounds__(NT2) k_stencil25(OpB<double> LB, SH S,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ b,
                                                   double *__restrict__ out,
                                                   float *__restrict__ outf,
                                                   double *__restrict__ partials, int off2,
                                                   const int *__restrict__ mask,
                                                   const Z *__restrict__ z = nullptr,
                                                   double *__restrict__ pnew = nullptr,
                                                   Z *__restrict__ zold = nullptr,
                                                   const double *__restrict__ scal = nullptr,
                                                   int first = 0) {
  constexpr int W = 64, NS = 4, NSB = 3;
  using PL = Pl1<double, W>;
  using VT = typename Vec16<double>::T;
  using ZP = ZPair<Z>;
  using ZT = typename ZP::T;
  constexpr int NX = PL::NX, FXR = PL::FXR, RV = FXR / PL::VEC;
  static_assert(PL::VEC == 2, "two cells per staged vector");
  __shared__ __align__(16) double sp[NS * NX], sr[NS * NX];
  __shared__ __align__(16) double sb[MODE == 1 ? NSB * NX : 2];
  __shared__ double lred[NT2 / 64];
  int g, s, lb;
  if (!locate(S, mask, g, s, lb)) return;
  const Op<double> L = op_at(LB, s);
  const int c0 = LB.ls[s].c0;
  p += c0;
  if (MODE == 1) b += c0;
  out += c0;
  if (outf) outf += c0;
  if (MODE == 2) {
    z += c0;
    pnew += c0;
    if (zold) zold += c0;
  }
  const double beta = (MODE == 2 && !first) ? scal[s * NSC + S_BETA] : 0.0;
  const int n0 = L.n0, n1 = L.n1, n2 = L.n2;
  int xb, y0, k0, k1;
  tile_of(lb, n0, n1, n2, W, S.kz, xb, y0, k0, k1);
  const int x0 = xb * W;
  const int tx = threadIdx.x, ty = threadIdx.y, t = tx + 64 * ty;
  const int i = x0 + tx, j = y0 + ty;
  const bool in = i < n0 && j < n1;
  const int ncs = n0 * n1 * n2;
  const Buf Bp = mkbuf(p, ncs), Br = mkbuf(L.rAU, ncs), Bb = mkbuf(MODE == 1 ? b : p, ncs);
  const Buf Bz = mkbuf(MODE == 2 ? z : (const Z *)p, MODE == 2 ? ncs : 0);
  const bool vec_ok = (n0 % PL::VEC) == 0;
  double v1 = 0.0, v2 = 0.0;
  // the body is instantiated for aligned rows (16-byte loads) and not,
  // so that each copy issues a fixed number of loads per plane
  auto run = [&](auto vok) {
    constexpr bool VOK = decltype(vok)::value;
    // two register sets alternate: plane k+2 is in flight in one while plane
    // k+1 is stored from the other and plane k computed
    struct Regs {
      VT p[PL::MV], r[PL::MV], b[PL::MV];
      ZT z[PL::MV];
    } RA, RB;
    auto load = [&](Regs &G, int k) {
#pragma unroll
      for (int m = 0; m < PL::MV; m++) {
        G.r[m] = pl_load<PL, VOK, double>(Br, t, m, x0, y0, k, n0, n1, n2);
        if (MODE == 1) G.b[m] = pl_load<PL, VOK, double>(Bb, t, m, x0, y0, k, n0, n1, n2);
        if (MODE == 2) {
          // z of the same two cells as the p vector (zero outside the mesh)
          const int e = pl_vec<PL::NV, PL::MV>(t, m);
          const int ia = x0 - PL::RX + (e % RV) * 2, jj = y0 - 1 + e / RV;
          const bool inz = jj >= 0 && jj < n1 && k >= 0 && k < n2 && ia + 2 > 0 && ia < n0;
          const int c = ia + n0 * (jj + n1 * k);
          if (VOK) {
            G.z[m] = ZP::ld(Bz, inz ? (unsigned)c * (unsigned)sizeof(Z) : Bz.oob);
          } else {
            ZT v = ZT{};
#pragma unroll
            for (int u = 0; u < 2; u++) {
              const bool ok = inz && ia + u >= 0 && ia + u < n0;
              v = ZP::one(Bz, ok ? (unsigned)(c + u) * (unsigned)sizeof(Z) : Bz.oob, v, u);
            }
            G.z[m] = v;
          }
        }
        // (the old p is loaded when first as well, so that every path issues
        // the same loads; first discards it)
        G.p[m] = pl_load<PL, VOK, double>(Bp, t, m, x0, y0, k, n0, n1, n2);
      }
    };
    auto store = [&](Regs &G, int k) {
#pragma unroll
      for (int m = 0; m < PL::MV; m++) {
        if (MODE == 2) {
          // p_new of the vector's two cells; the tile's own cells also go to
          // memory (planes k0..k1-1, rows y0.., columns x0..x0+63)
          const double z0 = ZP::get(G.z[m], 0), z1 = ZP::get(G.z[m], 1);
          VT pn;
          pn.x = first ? z0 : fma(beta, G.p[m].x, z0);
          pn.y = first ? z1 : fma(beta, G.p[m].y, z1);
          G.p[m] = pn;
          const int e = pl_vec<PL::NV, PL::MV>(t, m);
          const int lx = (e % RV) * 2 - PL::RX, ly = e / RV - 1;
          const int ia = x0 + lx, jj = y0 + ly;
          const bool own = k >= k0 && k < k1 && lx >= 0 && lx < W && ly >= 0 && ly < TY2 &&
                           jj < n1 && ia < n0 && e == t + m * NT2;
          if (own) {
            const int c = ia + n0 * (jj + n1 * k);
            if (VOK) {
              *reinterpret_cast<VT *>(pnew + c) = pn;
              if (zold) {
                zold[c] = (Z)z0;
                zold[c + 1] = (Z)z1;
              }
            } else {
              pnew[c] = pn.x;
              if (zold) zold[c] = (Z)z0;
              if (ia + 1 < n0) {
                pnew[c + 1] = pn.y;
                if (zold) zold[c + 1] = (Z)z1;
              }
            }
          }
        }
        pl_store<PL>(sp + slot_of<NS>(k) * NX, t, m, G.p[m]);
        pl_store<PL>(sr + slot_of<NS>(k) * NX, t, m, G.r[m]);
        if (MODE == 1) pl_store<PL>(sb + slot_of<NSB>(k) * NX, t, m, G.b[m]);
      }
    };
    const int c2 = PL::at(tx, ty);
    auto compute = [&](int k) {
      if (!in) return;
      const double *Pm = sp + slot_of<NS>(k - 1) * NX, *Pc = sp + slot_of<NS>(k) * NX,
                   *Pp = sp + slot_of<NS>(k + 1) * NX;
      const double *Rm = sr + slot_of<NS>(k - 1) * NX, *Rc = sr + slot_of<NS>(k) * NX,
                   *Rp = sr + slot_of<NS>(k + 1) * NX;
      const double pc = Pc[c2];
      const double y = row_diff(L, i, j, k, Rc[c2], Rc[c2 - 1], Rc[c2 + 1], Rc[c2 - FXR],
                                Rc[c2 + FXR], Rm[c2], Rp[c2], pc, Pc[c2 - 1], Pc[c2 + 1],
                                Pc[c2 - FXR], Pc[c2 + FXR], Pm[c2], Pp[c2]);
      const int c = i + n0 * (j + n1 * k);
      if (MODE != 1) {
        out[c] = y;
        v1 += pc * y;
      } else {
        const double bb = sb[slot_of<NSB>(k) * NX + c2];
        const double res = bb - y;
        out[c] = res;
        if (outf) outf[c] = (float)res;
        v1 += res * res;
        v2 += bb * bb;
      }
    };
    // G holds plane k+1 on entry and plane k+3 in flight on exit
    auto step = [&](Regs &G, int k) {
      store(G, k + 1);
      __syncthreads();
      load(G, k + 3 <= k1 ? k + 3 : n2);  // plane n2: no memory access
      if (k < k1) compute(k);
    };
    load(RA, k0 - 1);
    store(RA, k0 - 1);
    load(RA, k0);
    store(RA, k0);
    load(RA, k0 + 1);
    load(RB, k0 + 2 <= k1 ? k0 + 2 : n2);
    // planes in pairs; an odd count ends with a step that only stores and
    // loads, so that both steps issue the same loads on every path
    for (int k = k0; k < k1; k += 2) {
      step(RA, k);
      step(RB, k + 1);
    }
  };
  if (vec_ok) run(std::true_type{});
  else run(std::false_type{});
  const double s1 = block_sum_n<NT2 / 64>(v1, lred);
  if (tx == 0 && ty == 0) partials[g] = s1;
  if (MODE == 1) {
    const double s2 = block_sum_n<NT2 / 64>(v2, lred);
    if (tx == 0 && ty == 0) partials[off2 + g] = s2;
  }
}

enum { SM_NORMAL = 0, SM_ZERO = 1, SM_PROLONG = 2 };

// Red-black Gauss-Seidel half sweep on the fine level, one x-pair per thread.
// SM_ZERO: x = b/D on this colour, 0 on the other (zero initial guess).
// SM_PROLONG: x_in + (coarse correction of the parent, if the sample has a
// coarse level) is the current iterate; this colour is relaxed and both
// colours go to x_out.  Otherwise x_out == x_in and only this colour is
// written.
template <typename R, typename B, int MODE>
__global__ void __launch_bounds__(NT2) k_smooth25(OpB<R> LB, SH S, const B *__restrict__ b,
                                                  const R *xin, R *xout, int color,
                                                  const R *__restrict__ xc,
                                                  const int *__restrict__ mask) {
  constexpr int W = 128;
  __shared__ R sx[(TY2 + 2) * (W + 2)], sr[(TY2 + 2) * (W + 2)];
  int g, s, lb;
  if (!locate(S, mask, g, s, lb)) return;
  const Op<R> L = op_at(LB, s);
  const LvS &Q = LB.ls[s];
  b += Q.c0;
  xin += Q.c0;
  xout += Q.c0;
  const R *xcs = (MODE == SM_PROLONG && Q.cn0 > 0) ? xc + Q.cc0 : nullptr;
  const int cn0 = Q.cn0, cn1 = Q.cn1;
  const int n0 = L.n0, n1 = L.n1, n2 = L.n2;
  int xb, y0, k0, k1;
  tile_of(lb, n0, n1, n2, W, S.kz, xb, y0, k0, k1);
  const int x0 = xb * W;
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i0 = x0 + 2 * tx, j = y0 + ty;
  const R *rA = L.rAU;
  auto X = [&](int ii, int jj, int kk) -> R {
    if (MODE == SM_ZERO) return (R)0;
    R v = ld_or0(xin, ii, jj, kk, n0, n1, n2);
    if (MODE == SM_PROLONG && xcs && ii >= 0 && ii < n0 && jj >= 0 && jj < n1 && kk >= 0 &&
        kk < n2)
      v += xcs[(ii >> 1) + cn0 * ((jj >> 1) + cn1 * (kk >> 1))];
    return v;
  };
  auto XP = [&](int kk) -> P2<R> { return P2<R>{X(i0, j, kk), X(i0 + 1, j, kk)}; };
  auto RP = [&](int kk) -> P2<R> {
    return P2<R>{ld_or0(rA, i0, j, kk, n0, n1, n2), ld_or0(rA, i0 + 1, j, kk, n0, n1, n2)};
  };
  P2<R> xm = XP(k0 - 1), xk = XP(k0), xp = XP(k0 + 1), xq = XP(k0 + 2);
  P2<R> rm = RP(k0 - 1), rk = RP(k0), rp = RP(k0 + 1), rq = RP(k0 + 2);
  Halo<R> hc = halo_load<R, 2, W>(X, rA, x0, y0, i0, j, k0, n0, n1, n2), hn = hc;
  for (int k = k0; k < k1; k++) {
    sx[LIX(W, 2 * tx, ty)] = xk.v0;
    sx[LIX(W, 2 * tx + 1, ty)] = xk.v1;
    sr[LIX(W, 2 * tx, ty)] = rk.v0;
    sr[LIX(W, 2 * tx + 1, ty)] = rk.v1;
    halo_store<R, 2, W>(hc, sx, sr);
    __syncthreads();
    if (k + 1 < k1) hn = halo_load<R, 2, W>(X, rA, x0, y0, i0, j, k + 1, n0, n1, n2);
    const P2<R> xr = XP(k + 3), rr = RP(k + 3);
    const int off = ((j + k) & 1) == color ? 0 : 1;
    const int i = i0 + off;
    const int c = i + n0 * (j + n1 * k);
    const bool act = j < n1 && i < n0;
    const R bc = act ? (R)b[c] : (R)0;
    if (act) {
      const int lx = 2 * tx + off;
      R T[6], D;
      row25<R, W>(L, i, j, k, lx, ty, sr, rk.get(off), rm.get(off), rp.get(off), T, D);
      R xn;
      if (MODE == SM_ZERO)
        xn = D > (R)0 ? bc / D : (R)0;
      else
        xn = D > (R)0 ? (bc + off25<R, W>(T, lx, ty, sx, xm.get(off), xp.get(off))) / D : (R)0;
      xout[c] = xn;
      xk.set(off, xn);
    }
    if (MODE != SM_NORMAL && j < n1 && i0 + 1 - off < n0)
      xout[i0 + 1 - off + n0 * (j + n1 * k)] = MODE == SM_ZERO ? (R)0 : xk.get(1 - off);
    __syncthreads();
    xm = xk; xk = xp; xp = xq; xq = xr;
    rm = rk; rk = rp; rp = rq; rq = rr;
    hc = hn;
  }
}

// ------------------------------------------------ fused full sweep (fine level)
//
// One red-black Gauss-Seidel sweep (colour A then colour B) in a single pass
// over memory.  An A cell's six neighbours are all B cells, so its update
// needs only old values; a B cell's update needs the new A values around
// it.  A block owns a 128 x 8 tile and walks its planes as a wavefront: at
// step k it relaxes the A cells of plane k on the tile and on a one-cell
// ring around it (the ring values are recomputed, bit for bit, by the
// blocks owning them), then the B cells of plane k-1 on the tile, and writes
// both colours of plane k-1.  x is read from one buffer and written to
// another, so neighbours' old values are never overwritten under a block.
// Each thread owns an x-pair: it relaxes the A cell of its pair in every
// plane (138 threads also take one ring cell) and the B cell one plane
// behind, keeping its own column's new A values, rAU and b in registers.
// LDS holds three planes of old x and rAU (rows widened to whole 16-byte
// vectors, two rows of ring above and below) and two planes of new A
// values, 50 KB in FP32.  Planes are fetched one step ahead with 16-byte
// loads.  Per sweep each of x, b and rAU is read once and x written once,
// where two half sweeps read and write every cache line twice.

constexpr int FW = 128;              // tile width (cells), one x-pair per thread
constexpr int FX1 = FW + 2;          // row stride of planes with a 1-cell ring
constexpr int FY1 = TY2 + 2;
constexpr int NX1 = FX1 * FY1;
constexpr int NRING = FX1 + TY2;     // A cells on the 1-ring of a plane
#define I1(lx, ly) (((ly) + 1) * FX1 + (lx) + 1)

enum { SW_NORMAL = 0, SW_ZERO = 1, SW_PROLONG = 2 };

// plane geometry of the fused sweep: 128 x TY2 tiles with a two-row ring
template <typename R>
using SwPlane = PlG<R, FW, 2>;

// position (lx, ly) of ring A cell r (0 <= r < NRING) of plane k: rows above
// and below the tile (65 each), then the columns left and right (4 each)
__device__ __forceinline__ void ring_cell(int r, int x0, int y0, int k, int colA, int &lx,
                                          int &ly) {
  if (r < 2 * (FX1 / 2)) {
    ly = r < FX1 / 2 ? -1 : TY2;
    const int q = r < FX1 / 2 ? r : r - FX1 / 2;
    lx = 2 * q - 1 + ((colA - (x0 - 1 + y0 + ly + k)) & 1);
  } else {
    const int q = r - 2 * (FX1 / 2);
    lx = q < TY2 / 2 ? -1 : FW;
    const int qq = q < TY2 / 2 ? q : q - TY2 / 2;
    ly = 2 * qq + ((colA - (x0 + lx + y0 + k)) & 1);
  }
}

// MODE SW_ZERO: the iterate starts at zero (xin unused).  SW_PROLONG: the
// iterate is xin plus the coarse correction of each cell's parent (when the
// sample has a coarse level).  colA: colour relaxed first.  xout != xin.
// OPK 0: the fine level (rows rebuilt from rAU); OPK 1: a coarse level with
// stored face coefficients Tx, Ty, Tz (zero on domain faces) and diagonal D,
// staged like rAU.  DOT: the block's partial sums of b.xout and b.zold
// (zold may be null) go to partials[g] and partials[off2 + g].
template <typename R, typename B, int MODE, int OPK = 0, int DOT = 0>
__global__ void __launch_bounds__(NT2) k_sweep25(OpB<R> LB, SH S, const B *__restrict__ b,
                                                 const R *__restrict__ xin,
                                                 R *__restrict__ xout, int colA,
                                                 const R *__restrict__ xc,
                                                 const int *__restrict__ mask,
                                                 const R *__restrict__ zold,
                                                 double *__restrict__ partials, int off2) {
  using PL = SwPlane<R>;
  using VT = typename Vec16<R>::T;
  constexpr int VEC = PL::VEC, NX = PL::NX, FXR = PL::FXR;
  __shared__ __align__(16) R sX[3 * NX];   // old x, planes k-1, k, k+1 (slot k mod 3)
  constexpr int NR = OPK ? 4 : 1;          // coefficient arrays: rAU, or Tx Ty Tz D
  __shared__ __align__(16) R sR[3 * NR * NX];  // array q, plane k at slot 3 q + k mod 3
  __shared__ __align__(16) R sB[3 * NX];   // right-hand side, planes k-1, k, k+1
  static_assert(std::is_same<R, B>::value, "the right-hand side is staged as R");
  __shared__ R sA[2 * NX1];                // new A values, planes k-1, k (slot k mod 2)
  __shared__ double lred[DOT ? NT2 / 64 : 1];
  int g, s, lb;
  if (!locate(S, mask, g, s, lb)) return;
  const Op<R> L = op_at(LB, s);
  const LvS &Q = LB.ls[s];
  b += Q.c0;
  if (MODE != SW_ZERO) xin += Q.c0;
  xout += Q.c0;
  const R *xcs = (MODE == SW_PROLONG && Q.cn0 > 0) ? xc + Q.cc0 : nullptr;
  const int cn0 = Q.cn0, cn1 = Q.cn1;
  const int n0 = L.n0, n1 = L.n1, n2 = L.n2;
  int xb, y0, k0, k1;
  tile_of(lb, n0, n1, n2, FW, S.kz, xb, y0, k0, k1);
  const int x0 = xb * FW;
  const int tx = threadIdx.x, ty = threadIdx.y, t = tx + 64 * ty;
  const int i0 = x0 + 2 * tx, j = y0 + ty;
  const R *rA = OPK ? L.D : L.rAU;
  // rows start on 16-byte boundaries
  const bool vec_ok = n0 % VEC == 0 && Q.c0 % VEC == 0;
  auto inside = [&](int i, int jj, int k) {
    return i >= 0 && i < n0 && jj >= 0 && jj < n1 && k >= 0 && k < n2;
  };
  auto xs = [](int k) { return (k + 3) % 3; };
  // Registers of the plane in flight: x, rAU, b and (SW_PROLONG) the coarse
  // correction, kept apart from x until the LDS store so that nothing reads
  // a loaded value before the next plane step (the loads stay in flight
  // while the current plane is relaxed).
  const int ncs = n0 * n1 * n2;
  const Buf Bx = mkbuf(MODE == SW_ZERO ? rA : xin, ncs), Bb = mkbuf(b, ncs);
  Buf Br[NR];
  if constexpr (OPK) {
    Br[0] = mkbuf(L.Tx, ncs);
    Br[1] = mkbuf(L.Ty, ncs);
    Br[2] = mkbuf(L.Tz, ncs);
    Br[3] = mkbuf(L.D, ncs);
  } else {
    Br[0] = mkbuf(rA, ncs);
  }
  auto sr = [&](int q, int k) -> R * { return sR + (3 * q + xs(k)) * NX; };
  const Buf Bc = mkbuf(xcs ? xcs : rA, xcs ? cn0 * cn1 * Q.cn2 : 0);
  // DOT: sums over the cells this thread stores, and zold of its pair of
  // plane k-1 (loaded before the plane loads of the step, used at the store)
  double dz = 0.0, dzo = 0.0;
  const Buf Bz = mkbuf(DOT && zold ? zold + Q.c0 : rA, DOT && zold ? ncs : 0);
  R zo0 = (R)0, zo1 = (R)0;
  auto zpre = [&](int k) {
    const int kb = k - 1;
    const bool ok = kb >= k0 && kb < k1 && j < n1;
    const unsigned cp = (unsigned)(i0 + n0 * (j + n1 * kb)) * (unsigned)sizeof(R);
    zo0 = bld1(Bz, ok && i0 < n0 ? cp : Bz.oob, R{});
    zo1 = bld1(Bz, ok && i0 + 1 < n0 ? cp + (unsigned)sizeof(R) : Bz.oob, R{});
  };
  // coarse correction of the parents of vector m of plane k
  auto parent = [&](int m, int k, auto vok) -> VT {
    constexpr bool VOK = decltype(vok)::value;
    constexpr int RV = FXR / VEC;
    const int e = pl_vec<PL::NV, PL::MV>(t, m);
    const int ia = x0 - PL::RX + (e % RV) * VEC, jj = y0 - 2 + e / RV;
    const bool in = jj >= 0 && jj < n1 && k >= 0 && k < n2 && ia + VEC > 0 && ia < n0;
    const int pidx = (ia >> 1) + cn0 * ((jj >> 1) + cn1 * (k >> 1));
    VT v = vzero<VT>();
    if (VOK) {
      // ia is a multiple of VEC (even): the vector has VEC/2 parents, and
      // cn0 = n0/2 is even, so they are one aligned 8-byte load.  They are
      // kept packed in the leading components (no use of the loaded values
      // until the LDS store, which spreads them with vspread).
      const unsigned off = in ? (unsigned)pidx * (unsigned)sizeof(R) : Bc.oob;
      if constexpr (VEC == 4) {
        const auto w = __builtin_amdgcn_raw_buffer_load_b64(Bc.r, off, 0, 0);
        vset(v, 0, __uint_as_float(w[0]));
        vset(v, 1, __uint_as_float(w[1]));
      } else {
        vset(v, 0, bld1(Bc, off, R{}));
      }
    } else {
#pragma unroll
      for (int u = 0; u < VEC; u++) {
        const bool ok = in && ia + u >= 0 && ia + u < n0;
        const int q = ((ia + u) >> 1) + cn0 * ((jj >> 1) + cn1 * (k >> 1));
        vset(v, u, bld1(Bc, ok ? (unsigned)q * (unsigned)sizeof(R) : Bc.oob, R{}));
      }
    }
    return v;
  };
  const bool ringer = t < NRING;
  // new A value at (lx, ly) of plane k from LDS neighbours
  const RowK<R> K = rowk(L);
  // new A value at (lx, ly) of plane k from LDS neighbours (zero outside
  // the mesh; computed without a branch and selected)
  auto relax_a = [&](int lx, int ly, int k) -> R {
    const int i = x0 + lx, jj = y0 + ly;
    const R bb = sB[xs(k) * NX + PL::at(lx, ly)];
    const R *Xm = sX + xs(k - 1) * NX, *Xc = sX + xs(k) * NX, *Xp = sX + xs(k + 1) * NX;
    const int c2 = PL::at(lx, ly);
    R T[6], D;
    if constexpr (OPK) {
      const R *Tx = sr(0, k), *Ty = sr(1, k);
      T[0] = Tx[c2 - 1];
      T[1] = Tx[c2];
      T[2] = Ty[c2 - FXR];
      T[3] = Ty[c2];
      T[4] = sr(2, k - 1)[c2];
      T[5] = sr(2, k)[c2];
      D = sr(3, k)[c2];
    } else {
      const R *Rm = sr(0, k - 1), *Rc = sr(0, k), *Rp = sr(0, k + 1);
      coefu(K, i, jj, k, n0, n1, n2, Rc[c2], Rc[c2 - 1], Rc[c2 + 1], Rc[c2 - FXR],
            Rc[c2 + FXR], Rm[c2], Rp[c2], T, D);
    }
    R v;
    if (MODE == SW_ZERO) {
      v = bb * sw_rcp(D);
    } else {
      const R off = T[0] * Xc[c2 - 1] + T[1] * Xc[c2 + 1] + T[2] * Xc[c2 - FXR] +
                    T[3] * Xc[c2 + FXR] + T[4] * Xm[c2] + T[5] * Xp[c2];
      v = (bb + off) * sw_rcp(D);
    }
    return inside(i, jj, k) && D > (R)0 ? v : (R)0;
  };
  P2<R> r_m2 = {(R)0, (R)0}, r_m1 = {(R)0, (R)0}, r_0;
  R a_m2 = (R)0, a_m1 = (R)0, a_0;
  // relax the A cells of plane k and the B cells of plane k-1 (planes k-1,
  // k, k+1 in LDS)
  auto relax_planes = [&](int k) {
    const int offA = ((j + k) & 1) == colA ? 0 : 1;  // x0 and 2 tx are even
    // own column: rAU (OPK 1: Tz) of plane k; the coefficients around the
    // own B cell of plane k-1
    const R *Rk = sr(OPK ? 2 : 0, k);
    r_0 = P2<R>{Rk[PL::at(2 * tx, ty)], Rk[PL::at(2 * tx + 1, ty)]};
    const int lxB = 2 * tx + offA;  // B cell of plane k-1 = A position of plane k
    const int cb = PL::at(lxB, ty);
    R rbc, rbxm, rbxp, rbym, rbyp;
    if constexpr (OPK) {
      rbxm = sr(0, k - 1)[cb - 1];
      rbxp = sr(0, k - 1)[cb];
      rbym = sr(1, k - 1)[cb - FXR];
      rbyp = sr(1, k - 1)[cb];
      rbc = sr(3, k - 1)[cb];
    } else {
      const R *Rb = sr(0, k - 1);
      rbc = Rb[cb];
      rbxm = Rb[cb - 1];
      rbxp = Rb[cb + 1];
      rbym = Rb[cb - FXR];
      rbyp = Rb[cb + FXR];
    }
    // (read before the barrier: the next plane step overwrites plane k-1's slot)
    const R bB = sB[xs(k - 1) * NX + cb];
    const R bA = DOT ? sB[xs(k - 1) * NX + PL::at(2 * tx + 1 - offA, ty)] : (R)0;
    // A cells of plane k: own, then one ring cell
    R *An = sA + (k & 1) * NX1;
    a_0 = j < n1 ? relax_a(2 * tx + offA, ty, k) : (R)0;
    An[I1(2 * tx + offA, ty)] = a_0;
    if (ringer) {
      int lx, ly;
      ring_cell(t, x0, y0, k, colA, lx, ly);
      An[I1(lx, ly)] = relax_a(lx, ly, k);
    }
    __syncthreads();
    // B cell of plane k-1; write both colours of plane k-1
    const int kb = k - 1;
    if (kb >= k0 && kb < k1 && j < n1) {
      const int iB = i0 + offA;
      R vB = (R)0;
      if (iB < n0) {
        const R *Ac = sA + (kb & 1) * NX1;
        const int c1 = I1(lxB, ty);
        R T[6], D;
        if constexpr (OPK) {
          T[0] = rbxm;
          T[1] = rbxp;
          T[2] = rbym;
          T[3] = rbyp;
          T[4] = r_m2.get(offA);  // Tz of plane k-2: the face below plane k-1
          T[5] = r_m1.get(offA);
          D = rbc;
        } else {
          coefu(K, iB, j, kb, n0, n1, n2, rbc, rbxm, rbxp, rbym, rbyp, r_m2.get(offA),
                r_0.get(offA), T, D);
        }
        const R off = T[0] * Ac[c1 - 1] + T[1] * Ac[c1 + 1] + T[2] * Ac[c1 - FX1] +
                      T[3] * Ac[c1 + FX1] + T[4] * a_m2 + T[5] * a_0;
        vB = D > (R)0 ? (bB + off) * sw_rcp(D) : (R)0;
      }
      // the pair in memory order: offset 0 first
      const R v0 = offA == 0 ? vB : a_m1, v1 = offA == 0 ? a_m1 : vB;
      if constexpr (DOT) {
        // b and the new x are zero outside the mesh
        const R b0 = offA == 0 ? bB : bA, b1 = offA == 0 ? bA : bB;
        dz += (double)b0 * (double)v0 + (double)b1 * (double)v1;
        dzo += (double)b0 * (double)zo0 + (double)b1 * (double)zo1;
      }
      R *row = xout + n0 * (j + n1 * kb);
      if ((n0 & 1) == 0 && i0 + 1 < n0) {
        using V2 = typename Vec16<R>::T2;
        R pv[2] = {v0, v1};
        V2 w;
        memcpy(&w, pv, sizeof(R) * 2);
        if (sizeof(V2) == 2 * sizeof(R)) {
          *reinterpret_cast<V2 *>(row + i0) = w;
        } else {
          row[i0] = v0;
          row[i0 + 1] = v1;
        }
      } else {
        if (i0 < n0) row[i0] = v0;
        if (i0 + 1 < n0) row[i0 + 1] = v1;
      }
    }
    r_m2 = r_m1;
    r_m1 = r_0;
    a_m2 = a_m1;
    a_m1 = a_0;
  };
  // Registers of the planes in flight: x, rAU, b and (SW_PROLONG) the coarse
  // correction, kept apart from x until the LDS store so that nothing reads
  // a loaded value before its plane step.  Two sets alternate: plane k+2 is
  // in flight in one while plane k+1 is stored from the other.  The body is
  // instantiated for aligned rows (16-byte loads) and not, so that each copy
  // issues a fixed number of loads per plane.
  auto run = [&](auto vok) {
    constexpr bool VOK = decltype(vok)::value;
    struct Regs {
      VT x[PL::MV], r[NR][PL::MV], b[PL::MV], c[PL::MV];
    } RA, RB;
    auto load_planes = [&](Regs &G, int k) {
#pragma unroll
      for (int m = 0; m < PL::MV; m++) {
        if (MODE != SW_ZERO) G.x[m] = pl_load<PL, VOK, R>(Bx, t, m, x0, y0, k, n0, n1, n2);
#pragma unroll
        for (int q = 0; q < NR; q++)
          G.r[q][m] = pl_load<PL, VOK, R>(Br[q], t, m, x0, y0, k, n0, n1, n2);
        G.b[m] = pl_load<PL, VOK, R>(Bb, t, m, x0, y0, k, n0, n1, n2);
        if (MODE == SW_PROLONG) G.c[m] = parent(m, k, vok);
      }
    };
    auto store_planes = [&](const Regs &G, int k) {
#pragma unroll
      for (int m = 0; m < PL::MV; m++) {
        const int e = pl_vec<PL::NV, PL::MV>(t, m);
        if (MODE == SW_PROLONG)
          *reinterpret_cast<VT *>(sX + xs(k) * NX + e * VEC) =
              vadd(G.x[m], VOK ? vspread(G.c[m]) : G.c[m]);
        else if (MODE != SW_ZERO)
          *reinterpret_cast<VT *>(sX + xs(k) * NX + e * VEC) = G.x[m];
#pragma unroll
        for (int q = 0; q < NR; q++) *reinterpret_cast<VT *>(sr(q, k) + e * VEC) = G.r[q][m];
        *reinterpret_cast<VT *>(sB + xs(k) * NX + e * VEC) = G.b[m];
      }
    };
    // G holds plane k+1 on entry and plane k+3 in flight on exit
    auto step = [&](Regs &G, int k) {
      store_planes(G, k + 1);  // its slot (plane k-2) is free
      __syncthreads();
      if constexpr (DOT) zpre(k);
      load_planes(G, k + 3 <= k1 + 1 ? k + 3 : n2);  // plane n2: no memory access
      if (k <= k1) relax_planes(k);
    };
    // The A cells of plane k0-1 are relaxed only for the B cells of plane
    // k0-1, which belong to the tile below; at the bottom of the mesh there
    // is none, so the walk starts at k0 (a 2D tile then takes two steps).
    // Prologue: planes k0-2 .. ks in LDS, ks+1 and ks+2 in flight.
    const int ks = k0 > 0 ? k0 - 1 : k0;
    for (int q = k0 - 2; q <= ks; q++) {
      load_planes(RA, q);
      store_planes(RA, q);
    }
    load_planes(RA, ks + 1);
    load_planes(RB, ks + 2 <= k1 + 1 ? ks + 2 : n2);
    // planes in pairs; an odd count ends with a step that only stores and
    // loads, so that both steps issue the same loads on every path
    for (int k = ks; k <= k1; k += 2) {
      step(RA, k);
      step(RB, k + 1);
    }
  };
  if (vec_ok) run(std::true_type{});
  else run(std::false_type{});
  if constexpr (DOT) {
    const double s1 = block_sum_n<NT2 / 64>(dz, lred);
    if (t == 0) partials[g] = s1;
    if (zold) {
      const double s2 = block_sum_n<NT2 / 64>(dzo, lred);
      if (t == 0) partials[off2 + g] = s2;
    }
  }
}

// ------------------------------------------ block-local coarse smoothing
//
// All sweeps of a coarse level in one launch (FP32 V-cycle, stored
// operator): a block owns a CB^3 tile and makes `sweeps` red-black
// Gauss-Seidel sweeps over it in LDS, the cells around the tile held at
// their values when the launch starts (Jacobi between tiles, Gauss-Seidel
// within).  CB_ZERO (pre-smoothing): from x = 0, red then black.
// CB_PROLONG (post-smoothing): from x = xin plus the parent's coarse
// correction on the tile and its halo, black then red.  The post-smoother
// is the transpose of the pre-smoother, so the V-cycle stays symmetric.
// Each thread owns a column of 8 cells (4 of each colour) and keeps their
// coefficients in registers; LDS holds the iterate with a one-cell halo.
constexpr int CB = 16;                   // tile edge (cells)
constexpr int CBT = 512;                 // threads per block
constexpr int CBH = CB + 2;              // tile edge with the halo
constexpr int CBQ = CB * CB * CB / CBT;  // cells per thread (a column in z)
enum { CB_ZERO = 0, CB_PROLONG = 1 };

__host__ __device__ inline int cb_tiles(int n0, int n1, int n2) {
  return ((n0 + CB - 1) / CB) * ((n1 + CB - 1) / CB) * ((n2 + CB - 1) / CB);
}

template <int MODE>
__global__ void __launch_bounds__(CBT) k_cblock(OpB<float> LB, SH S, const float *__restrict__ b,
                                                const float *__restrict__ xin,
                                                float *__restrict__ xout,
                                                const float *__restrict__ xc, int sweeps,
                                                const int *__restrict__ mask) {
  static_assert(CB * CB * CB == CBT * CBQ && CBQ % 2 == 0, "tile columns");
  __shared__ float sx[CBH * CBH * CBH];
  int g, s, lb;
  if (!locate(S, mask, g, s, lb)) return;
  const Op<float> L = op_at(LB, s);
  const LvS &Q = LB.ls[s];
  const int n0 = L.n0, n1 = L.n1, n2 = L.n2;
  b += Q.c0;
  xout += Q.c0;
  if (MODE == CB_PROLONG) xin += Q.c0;
  const float *xcs = (MODE == CB_PROLONG && Q.cn0 > 0) ? xc + Q.cc0 : nullptr;
  const int ntx = (n0 + CB - 1) / CB, nty = (n1 + CB - 1) / CB;
  const int x0 = (lb % ntx) * CB, y0 = ((lb / ntx) % nty) * CB, z0 = (lb / (ntx * nty)) * CB;
  const int t = threadIdx.x;
  // the iterate on the tile and its halo (zero outside the mesh)
  for (int e = t; e < CBH * CBH * CBH; e += CBT) {
    const int i = x0 + e % CBH - 1, j = y0 + (e / CBH) % CBH - 1, k = z0 + e / (CBH * CBH) - 1;
    float v = 0.f;
    if (MODE == CB_PROLONG && i >= 0 && i < n0 && j >= 0 && j < n1 && k >= 0 && k < n2) {
      v = xin[i + n0 * (j + n1 * k)];
      if (xcs) v += xcs[(i >> 1) + Q.cn0 * ((j >> 1) + Q.cn1 * (k >> 1))];
    }
    sx[e] = v;
  }
  // own column: (i, j) and CBQ planes from kq
  const int li = t % CB, lj = (t / CB) % CB, lk = (t / (CB * CB)) * CBQ;
  const int i = x0 + li, j = y0 + lj;
  float D[CBQ], Bv[CBQ], Txm[CBQ], Txp[CBQ], Tym[CBQ], Typ[CBQ], Tzm[CBQ], Tzp[CBQ];
#pragma unroll
  for (int q = 0; q < CBQ; q++) {
    const int k = z0 + lk + q;
    const bool in = i < n0 && j < n1 && k < n2;
    const int c = in ? i + n0 * (j + n1 * k) : 0;
    D[q] = in ? L.D[c] : 0.f;
    Bv[q] = in ? b[c] : 0.f;
    Txp[q] = in ? L.Tx[c] : 0.f;
    Txm[q] = (in && i > 0) ? L.Tx[c - 1] : 0.f;
    Typ[q] = in ? L.Ty[c] : 0.f;
    Tym[q] = (in && j > 0) ? L.Ty[c - n0] : 0.f;
    Tzp[q] = in ? L.Tz[c] : 0.f;
    Tzm[q] = (in && k > 0) ? L.Tz[c - n0 * n1] : 0.f;
  }
  __syncthreads();
  const int par0 = (i + j + z0 + lk) & 1;  // colour of the column's first cell
  for (int sw = 0; sw < sweeps; sw++) {
#pragma unroll
    for (int hh = 0; hh < 2; hh++) {
      const int color = MODE == CB_ZERO ? hh : 1 - hh;  // 0 = red (i + j + k even)
#pragma unroll
      for (int q = 0; q < CBQ; q++) {
        if (((par0 + q) & 1) != color || !(D[q] > 0.f)) continue;
        const int e = (li + 1) + CBH * ((lj + 1) + CBH * (lk + q + 1));
        const float off = Txm[q] * sx[e - 1] + Txp[q] * sx[e + 1] + Tym[q] * sx[e - CBH] +
                          Typ[q] * sx[e + CBH] + Tzm[q] * sx[e - CBH * CBH] +
                          Tzp[q] * sx[e + CBH * CBH];
        sx[e] = (Bv[q] + off) * sw_rcp(D[q]);
      }
      __syncthreads();
    }
  }
#pragma unroll
  for (int q = 0; q < CBQ; q++) {
    const int k = z0 + lk + q;
    if (i < n0 && j < n1 && k < n2)
      xout[i + n0 * (j + n1 * k)] = sx[(li + 1) + CBH * ((lj + 1) + CBH * (lk + q + 1))];
  }
}

// ------------------------------------------ small-tile coarse sweeps
//
// One fused red-black Gauss-Seidel sweep of a coarse level (FP32, stored
// operator) on small tiles, one cell per thread, with no plane pipeline:
// the smaller coarse levels are too small for the 2.5-D walk to pay for its
// prologue, their launches are latency-bound, and short rows would idle
// most lanes of the 128-wide plane-walk tiles.  The sweep is exact, with
// the plane-walking sweep's arithmetic (each update reads the same
// neighbours in the same order): the block loads the old iterate on the
// tile with a two-cell ring and the coefficients and b on a one-cell ring,
// relaxes the colour colA on the tile and its ring (the values the other
// colour's update of the tile reads), then the other colour on the tile.
// Tiles are 8 x 8 x 4 cells, or 16 x 16 x 1 on levels whose samples are
// all one cell deep (no z ring, no z terms: their z coefficients are the
// zeros of domain faces).  MODE as k_sweep25 (SW_ZERO: from zero;
// SW_PROLONG: xin plus the parent's coarse correction).
template <int TX, int TY, int TZ>
struct CsTile {
  static constexpr int X = TX, Y = TY, Z = TZ, T = TX * TY * TZ;  // cells = threads
  static constexpr int RZ2 = TZ > 1 ? 2 : 0, RZ1 = TZ > 1 ? 1 : 0;  // z rings
  static constexpr int XW = TX + 4, XH = TY + 4, XD = TZ + 2 * RZ2;  // iterate, 2-cell ring
  static constexpr int RW = TX + 2, RH = TY + 2, RD = TZ + 2 * RZ1;  // coefficients, 1-cell ring
  static constexpr int XN = XW * XH * XD, RN = RW * RH * RD;
};
using Cs3 = CsTile<8, 8, 4>;
using Cs2 = CsTile<16, 16, 1>;
constexpr int CST = 256;  // threads per block
static_assert(Cs3::T == CST && Cs2::T == CST, "one cell per thread");

template <typename TL>
__host__ __device__ inline int cs_tiles(int n0, int n1, int n2) {
  return ((n0 + TL::X - 1) / TL::X) * ((n1 + TL::Y - 1) / TL::Y) * ((n2 + TL::Z - 1) / TL::Z);
}

template <int MODE, typename TL, typename R = float>
__global__ void __launch_bounds__(CST) k_csweep(OpB<R> LB, SH S, const R *__restrict__ b,
                                                const R *__restrict__ xin,
                                                R *__restrict__ xout, int colA,
                                                const R *__restrict__ xc,
                                                const int *__restrict__ mask) {
  constexpr bool Z3 = TL::Z > 1;
  constexpr int XW = TL::XW, XH = TL::XH, RW = TL::RW, RH = TL::RH;
  __shared__ R sx[TL::XN];          // old iterate (0 outside the mesh)
  __shared__ R sc[8][TL::RN];       // b, D, T[0..5] of the ring-1 region
  __shared__ R sa[TL::RN];          // new colour-A values of the region
  int g, s, lb;
  if (!locate(S, mask, g, s, lb)) return;
  const Op<R> L = op_at(LB, s);
  const LvS &Q = LB.ls[s];
  const int n0 = L.n0, n1 = L.n1, n2 = L.n2;
  const int sy = n0, sz = n0 * n1;
  b += Q.c0;
  if (MODE != SW_ZERO) xin += Q.c0;
  xout += Q.c0;
  const R *xcs = (MODE == SW_PROLONG && Q.cn0 > 0) ? xc + Q.cc0 : nullptr;
  const int nbx = (n0 + TL::X - 1) / TL::X, nby = (n1 + TL::Y - 1) / TL::Y;
  const int i0 = (lb % nbx) * TL::X, j0 = ((lb / nbx) % nby) * TL::Y;
  const int k0 = (lb / (nbx * nby)) * TL::Z;
  const int t = threadIdx.x;
  // old iterate on the tile and its two-cell ring
  if (MODE != SW_ZERO) {
#pragma unroll
    for (int e = t; e < TL::XN; e += CST) {
      const int i = i0 - 2 + e % XW, j = j0 - 2 + (e / XW) % XH;
      const int k = k0 - TL::RZ2 + e / (XW * XH);
      R v = (R)0;
      if (i >= 0 && i < n0 && j >= 0 && j < n1 && k >= 0 && k < n2) {
        v = xin[i + sy * j + sz * k];
        if (MODE == SW_PROLONG && xcs)
          v += xcs[(i >> 1) + Q.cn0 * ((j >> 1) + Q.cn1 * (k >> 1))];
      }
      sx[e] = v;
    }
  }
  // b, diagonal and the six neighbour coefficients (0 on domain faces and
  // outside the mesh) on the tile and its one-cell ring
#pragma unroll
  for (int e = t; e < TL::RN; e += CST) {
    const int i = i0 - 1 + e % RW, j = j0 - 1 + (e / RW) % RH;
    const int k = k0 - TL::RZ1 + e / (RW * RH);
    R v[8] = {(R)0, (R)0, (R)0, (R)0, (R)0, (R)0, (R)0, (R)0};
    if (i >= 0 && i < n0 && j >= 0 && j < n1 && k >= 0 && k < n2) {
      const int c = i + sy * j + sz * k;
      v[0] = b[c];
      v[1] = L.D[c];
      v[2] = i > 0 ? L.Tx[c - 1] : (R)0;
      v[3] = i + 1 < n0 ? L.Tx[c] : (R)0;
      v[4] = j > 0 ? L.Ty[c - sy] : (R)0;
      v[5] = j + 1 < n1 ? L.Ty[c] : (R)0;
      if constexpr (Z3) {
        v[6] = k > 0 ? L.Tz[c - sz] : (R)0;
        v[7] = k + 1 < n2 ? L.Tz[c] : (R)0;
      }
    }
#pragma unroll
    for (int q = 0; q < 8; q++) sc[q][e] = v[q];
  }
  __syncthreads();
  // colour A on the tile and its ring, from the old iterate
  for (int e = t; e < TL::RN; e += CST) {
    const int li = e % RW, lj = (e / RW) % RH, lk = e / (RW * RH);
    const int i = i0 - 1 + li, j = j0 - 1 + lj, k = k0 - TL::RZ1 + lk;
    R v = (R)0;
    const R D = sc[1][e];
    if (((i + j + k) & 1) == colA && i >= 0 && i < n0 && j >= 0 && j < n1 && k >= 0 &&
        k < n2 && D > (R)0) {
      if (MODE == SW_ZERO) {
        v = sc[0][e] * sw_rcp(D);
      } else {
        const int x = (li + 1) + XW * ((lj + 1) + XH * (lk + TL::RZ2 - TL::RZ1));
        R off;
        if constexpr (Z3)
          off = sc[2][e] * sx[x - 1] + sc[3][e] * sx[x + 1] + sc[4][e] * sx[x - XW] +
                sc[5][e] * sx[x + XW] + sc[6][e] * sx[x - XW * XH] + sc[7][e] * sx[x + XW * XH];
        else
          off = sc[2][e] * sx[x - 1] + sc[3][e] * sx[x + 1] + sc[4][e] * sx[x - XW] +
                sc[5][e] * sx[x + XW];
        v = (sc[0][e] + off) * sw_rcp(D);
      }
    }
    sa[e] = v;
  }
  __syncthreads();
  // the tile: colour A as relaxed, the other colour from the new A values
  const int li = t % TL::X + 1, lj = (t / TL::X) % TL::Y + 1, lk = t / (TL::X * TL::Y) + TL::RZ1;
  const int i = i0 + li - 1, j = j0 + lj - 1, k = k0 + lk - TL::RZ1;
  if (i < n0 && j < n1 && k < n2) {
    const int e = li + RW * (lj + RH * lk);
    R v = sa[e];
    if (((i + j + k) & 1) != colA) {
      const R D = sc[1][e];
      R off;
      if constexpr (Z3)
        off = sc[2][e] * sa[e - 1] + sc[3][e] * sa[e + 1] + sc[4][e] * sa[e - RW] +
              sc[5][e] * sa[e + RW] + sc[6][e] * sa[e - RW * RH] + sc[7][e] * sa[e + RW * RH];
      else
        off = sc[2][e] * sa[e - 1] + sc[3][e] * sa[e + 1] + sc[4][e] * sa[e - RW] +
              sc[5][e] * sa[e + RW];
      v = D > (R)0 ? (sc[0][e] + off) * sw_rcp(D) : (R)0;
    }
    xout[i + sy * j + sz * k] = v;
  }
}

// Restriction after a pre-smoothing that ended with a black half sweep: the
// black residual is zero, so the coarse right-hand side is the sum of the
// red children's residuals.  Block tiles are 128 x 8 fine cells and walk
// plane pairs; rows 2J and 2J+1 are combined through LDS.
template <typename R, typename B>
__global__ void __launch_bounds__(NT2) k_restrict25(OpB<R> LB, SH S, const B *__restrict__ b,
                                                    const R *__restrict__ x, R *__restrict__ bc,
                                                    const int *__restrict__ mask) {
  constexpr int W = 128, NS = 4, NSB = 3;
  using PL = Pl1<R, W>;
  using VT = typename Vec16<R>::T;
  constexpr int NX = PL::NX, FXR = PL::FXR;
  static_assert(std::is_same<R, B>::value, "the right-hand side is staged as R");
  __shared__ __align__(16) R sx[NS * NX], sr[NS * NX], sb[NSB * NX];
  __shared__ R part[TY2 / 2][64];
  int g, s, lb;
  if (!locate(S, mask, g, s, lb)) return;
  const Op<R> L = op_at(LB, s);
  const LvS &Q = LB.ls[s];
  b += Q.c0;
  x += Q.c0;
  bc += Q.cc0;
  const int cn0 = Q.cn0, cn1 = Q.cn1;
  const int n0 = L.n0, n1 = L.n1, n2 = L.n2;
  int xb, y0, k0, k1;
  tile_of(lb, n0, n1, n2, W, S.kz, xb, y0, k0, k1);
  const int x0 = xb * W;
  const int tx = threadIdx.x, ty = threadIdx.y, t = tx + 64 * ty;
  const int i0 = x0 + 2 * tx, j = y0 + ty;
  const int ncs = n0 * n1 * n2;
  const Buf Bx = mkbuf(x, ncs), Br = mkbuf(L.rAU, ncs), Bb = mkbuf(b, ncs);
  const bool vec_ok = (n0 % PL::VEC) == 0;
  // the body is instantiated for aligned rows (16-byte loads) and not,
  // so that each copy issues a fixed number of loads per plane
  auto run = [&](auto vok) {
    constexpr bool VOK = decltype(vok)::value;
    // two register sets alternate: plane k+2 is in flight in one while plane
    // k+1 is stored from the other and plane k computed
    struct Regs {
      VT x[PL::MV], r[PL::MV], b[PL::MV];
    } RA, RB;
    auto load = [&](Regs &G, int k) {
#pragma unroll
      for (int m = 0; m < PL::MV; m++) {
        G.x[m] = pl_load<PL, VOK, R>(Bx, t, m, x0, y0, k, n0, n1, n2);
        G.r[m] = pl_load<PL, VOK, R>(Br, t, m, x0, y0, k, n0, n1, n2);
        G.b[m] = pl_load<PL, VOK, R>(Bb, t, m, x0, y0, k, n0, n1, n2);
      }
    };
    auto store = [&](const Regs &G, int k) {
#pragma unroll
      for (int m = 0; m < PL::MV; m++) {
        pl_store<PL>(sx + slot_of<NS>(k) * NX, t, m, G.x[m]);
        pl_store<PL>(sr + slot_of<NS>(k) * NX, t, m, G.r[m]);
        pl_store<PL>(sb + slot_of<NSB>(k) * NX, t, m, G.b[m]);
      }
    };
    R acc = 0;
    auto compute = [&](int k) {
      const int off = ((j + k) & 1) == 0 ? 0 : 1;  // the red cell of the pair
      const int i = i0 + off;
      if (j < n1 && i < n0) {
        const int c2 = PL::at(2 * tx + off, ty);
        const R *Xm = sx + slot_of<NS>(k - 1) * NX, *Xc = sx + slot_of<NS>(k) * NX,
                *Xp = sx + slot_of<NS>(k + 1) * NX;
        const R *Rm = sr + slot_of<NS>(k - 1) * NX, *Rc = sr + slot_of<NS>(k) * NX,
                *Rp = sr + slot_of<NS>(k + 1) * NX;
        R T[6], D;
        coef7(L, i, j, k, Rc[c2], Rc[c2 - 1], Rc[c2 + 1], Rc[c2 - FXR], Rc[c2 + FXR], Rm[c2],
              Rp[c2], T, D);
        const R sm = T[0] * Xc[c2 - 1] + T[1] * Xc[c2 + 1] + T[2] * Xc[c2 - FXR] +
                     T[3] * Xc[c2 + FXR] + T[4] * Xm[c2] + T[5] * Xp[c2];
        acc += sb[slot_of<NSB>(k) * NX + c2] - (D * Xc[c2] - sm);
      }
      const bool flush = (k & 1) == 1 || k + 1 == n2;
      if (flush && (ty & 1)) part[ty >> 1][tx] = acc;
      __syncthreads();
      if (flush) {
        if (!(ty & 1)) {
          const int I = i0 >> 1, J = j >> 1, K = k >> 1;
          const R other = (j + 1 < n1) ? part[ty >> 1][tx] : (R)0;
          if (i0 < n0 && j < n1) bc[I + cn0 * (J + cn1 * K)] = acc + other;
        }
        acc = 0;
      }
    };
    auto step = [&](Regs &G, int k) {
      store(G, k + 1);
      __syncthreads();
      load(G, k + 3 <= k1 ? k + 3 : n2);  // plane n2: no memory access
      if (k < k1) compute(k);
    };
    load(RA, k0 - 1);
    store(RA, k0 - 1);
    load(RA, k0);
    store(RA, k0);
    load(RA, k0 + 1);
    load(RB, k0 + 2 <= k1 ? k0 + 2 : n2);
    // planes in pairs; an odd count ends with a step that only stores and
    // loads, so that both steps issue the same loads on every path
    for (int k = k0; k < k1; k += 2) {
      step(RA, k);
      step(RB, k + 1);
    }
  };
  if (vec_ok) run(std::true_type{});
  else run(std::false_type{});
}

// ------------------------------------------ fine level, one-cell-deep meshes
//
// On a 2D mesh (one cell deep) the plane walk of the 2.5-D kernels has one
// plane per tile, and its prologue, staging and barriers cost more than the
// plane itself (the SpMV, sweeps and restriction of a 2048 x 512 flume ran
// 2.8 times slower per cell than at 256^3).  These kernels take the same
// tiles and launch shapes with no pipeline: the tile and its ring are
// staged in LDS once (zero outside the mesh), one barrier, then the cells
// are computed.  Same operator rows as the plane walk (coef7 / row_diff,
// coefu with zero outside the mesh); the z terms vanish.

template <typename R>
__device__ __forceinline__ R at2(const R *__restrict__ a, int i, int j, int n0, int n1) {
  return (i >= 0 && i < n0 && j >= 0 && j < n1) ? a[i + n0 * j] : (R)0;
}

// MODE 1: r = b - A p (and its FP32 copy), partials r.r and b.b.  MODE 2:
// p_new = z + beta p (z when first) on the tile and its ring, written for
// the tile's cells (with the copy z_old = z when zold is given), q = A p_new
// and the partial p_new.q.  Tiles of 64 x 8 cells, one cell per thread (the
// SpMV shape of the 2.5-D kernel).
template <int MODE, typename Z = double>
__global__ void __launch_bounds__(NT2) k_stencil2d(OpB<double> LB, SH S,
                                                   const double *__restrict__ p,
                                                   const double *__restrict__ b,
                                                   double *__restrict__ out,
                                                   float *__restrict__ outf,
                                                   double *__restrict__ partials, int off2,
                                                   const int *__restrict__ mask,
                                                   const Z *__restrict__ z = nullptr,
                                                   double *__restrict__ pnew = nullptr,
                                                   Z *__restrict__ zold = nullptr,
                                                   const double *__restrict__ scal = nullptr,
                                                   int first = 0) {
  static_assert(MODE == 1 || MODE == 2, "residual or direction update + SpMV");
  constexpr int W = 64, AW = W + 2, AH = TY2 + 2, AN = AW * AH;
  __shared__ double sP[AN], sR[AN];  // iterate and rAU, tile and one-cell ring
  __shared__ double lred[NT2 / 64];
  int g, s, lb;
  if (!locate(S, mask, g, s, lb)) return;
  const Op<double> L = op_at(LB, s);
  const int c0 = LB.ls[s].c0;
  p += c0;
  if (MODE == 1) b += c0;
  out += c0;
  if (outf) outf += c0;
  if (MODE == 2) {
    z += c0;
    pnew += c0;
    if (zold) zold += c0;
  }
  const double beta = (MODE == 2 && !first) ? scal[s * NSC + S_BETA] : 0.0;
  const int n0 = L.n0, n1 = L.n1;
  int xb, y0, k0, k1;
  tile_of(lb, n0, n1, 1, W, S.kz, xb, y0, k0, k1);
  const int x0 = xb * W;
  const int tx = threadIdx.x, ty = threadIdx.y, t = tx + 64 * ty;
  const double *rA = L.rAU;
  for (int e = t; e < AN; e += NT2) {
    const int ii = x0 + e % AW - 1, jj = y0 + e / AW - 1;
    double pv = 0.0, rv = 0.0;
    if (ii >= 0 && ii < n0 && jj >= 0 && jj < n1) {
      const int c = ii + n0 * jj;
      rv = rA[c];
      if constexpr (MODE == 2) {
        const double zc = (double)z[c];
        pv = first ? zc : fma(beta, p[c], zc);
      } else {
        pv = p[c];
      }
    }
    sP[e] = pv;
    sR[e] = rv;
  }
  __syncthreads();
  const int i = x0 + tx, j = y0 + ty;
  double v1 = 0.0, v2 = 0.0;
  if (i < n0 && j < n1) {
    const int c = i + n0 * j, e = (ty + 1) * AW + tx + 1;
    const double pc = sP[e];
    const double y = row_diff(L, i, j, 0, sR[e], sR[e - 1], sR[e + 1], sR[e - AW], sR[e + AW],
                              0.0, 0.0, pc, sP[e - 1], sP[e + 1], sP[e - AW], sP[e + AW], 0.0,
                              0.0);
    if constexpr (MODE == 2) {
      pnew[c] = pc;
      if (zold) zold[c] = z[c];
      out[c] = y;
      v1 += pc * y;
    } else {
      const double bb = b[c];
      const double res = bb - y;
      out[c] = res;
      if (outf) outf[c] = (float)res;
      v1 += res * res;
      v2 += bb * bb;
    }
  }
  const double s1 = block_sum_n<NT2 / 64>(v1, lred);
  if (t == 0) partials[g] = s1;
  if (MODE == 1) {
    const double s2 = block_sum_n<NT2 / 64>(v2, lred);
    if (t == 0) partials[off2 + g] = s2;
  }
}

// One fused red-black sweep of the fine level of a 2D mesh, colour colA
// first, xin -> xout: tiles of 128 x 8 cells, one x-pair per thread (the
// shape of the 2.5-D sweep).  The old iterate (with the parent's coarse
// correction) and rAU are staged with a two-cell ring, b with a one-cell
// ring; each thread relaxes the colA cell of its pair, threads t < 138 also
// one colA cell of the one-cell ring, into LDS (zero outside the mesh), and
// after a barrier the other cell of its pair from them, and writes both.
// MODE and DOT as k_sweep25.
template <typename R, typename B, int MODE, int DOT = 0>
__global__ void __launch_bounds__(NT2) k_sweep2d(OpB<R> LB, SH S, const B *__restrict__ b,
                                                 const R *__restrict__ xin,
                                                 R *__restrict__ xout, int colA,
                                                 const R *__restrict__ xc,
                                                 const int *__restrict__ mask,
                                                 const R *__restrict__ zold,
                                                 double *__restrict__ partials, int off2) {
  static_assert(std::is_same<R, B>::value, "one precision per level");
  constexpr int W = 128;
  constexpr int XW = W + 4, XH = TY2 + 4, XN = XW * XH;  // two-cell ring
  constexpr int AW = W + 2, AH = TY2 + 2, AN = AW * AH;  // one-cell ring
  __shared__ R sX[MODE == SW_ZERO ? 1 : XN], sR[XN], sB[AN];
  __shared__ R sA[AN];  // new colA values of the tile and its ring
  __shared__ double lred[DOT ? NT2 / 64 : 1];
  int g, s, lb;
  if (!locate(S, mask, g, s, lb)) return;
  const Op<R> L = op_at(LB, s);
  const LvS &Q = LB.ls[s];
  b += Q.c0;
  if (MODE != SW_ZERO) xin += Q.c0;
  xout += Q.c0;
  const R *xcs = (MODE == SW_PROLONG && Q.cn0 > 0) ? xc + Q.cc0 : nullptr;
  const int cn0 = Q.cn0;
  const int n0 = L.n0, n1 = L.n1;
  int xb, y0, k0, k1;
  tile_of(lb, n0, n1, 1, W, S.kz, xb, y0, k0, k1);
  const int x0 = xb * W;
  const int tx = threadIdx.x, ty = threadIdx.y, t = tx + 64 * ty;
  const int i0 = x0 + 2 * tx, j = y0 + ty;
  const R *rA = L.rAU;
  const RowK<R> K = rowk(L);
  auto inside = [&](int ii, int jj) { return ii >= 0 && ii < n0 && jj >= 0 && jj < n1; };
  for (int e = t; e < XN; e += NT2) {
    const int ii = x0 + e % XW - 2, jj = y0 + e / XW - 2;
    R xv = (R)0, rv = (R)0;
    if (inside(ii, jj)) {
      const int c = ii + n0 * jj;
      rv = rA[c];
      if (MODE != SW_ZERO) {
        xv = xin[c];
        if (MODE == SW_PROLONG && xcs) xv += xcs[(ii >> 1) + cn0 * (jj >> 1)];
      }
    }
    if (MODE != SW_ZERO) sX[e] = xv;
    sR[e] = rv;
  }
  for (int e = t; e < AN; e += NT2) {
    const int ii = x0 + e % AW - 1, jj = y0 + e / AW - 1;
    sB[e] = inside(ii, jj) ? (R)b[ii + n0 * jj] : (R)0;
  }
  __syncthreads();
  auto xi = [](int lx, int ly) { return (ly + 2) * XW + lx + 2; };
  auto ai = [](int lx, int ly) { return (ly + 1) * AW + lx + 1; };
  // new value of the colA cell at (lx, ly) of the tile or its ring
  auto relax_a = [&](int lx, int ly) -> R {
    const int ii = x0 + lx, jj = y0 + ly;
    if (!inside(ii, jj)) return (R)0;
    const int q = xi(lx, ly);
    R T[6], D;
    coefu(K, ii, jj, 0, n0, n1, 1, sR[q], sR[q - 1], sR[q + 1], sR[q - XW], sR[q + XW], (R)0,
          (R)0, T, D);
    const R bb = sB[ai(lx, ly)];
    R v;
    if (MODE == SW_ZERO) {
      v = bb * sw_rcp(D);
    } else {
      const R off = T[0] * sX[q - 1] + T[1] * sX[q + 1] + T[2] * sX[q - XW] +
                    T[3] * sX[q + XW] + T[4] * (R)0 + T[5] * (R)0;
      v = (bb + off) * sw_rcp(D);
    }
    return D > (R)0 ? v : (R)0;
  };
  // own colA cell
  const int offA = ((i0 + j) & 1) == colA ? 0 : 1;  // i0 is even
  const R aOwn = relax_a(2 * tx + offA, ty);
  sA[ai(2 * tx + offA, ty)] = aOwn;
  // colA cells of the ring: rows above and below (65 each), then the
  // columns left and right (4 each)
  constexpr int NR = 2 * (AW / 2) + TY2;
  if (t < NR) {
    int lx, ly;
    if (t < 2 * (AW / 2)) {
      ly = t < AW / 2 ? -1 : TY2;
      const int q = t < AW / 2 ? t : t - AW / 2;
      lx = 2 * q - 1 + ((colA - (x0 - 1 + y0 + ly)) & 1);
    } else {
      const int q = t - 2 * (AW / 2);
      lx = q < TY2 / 2 ? -1 : W;
      const int qq = q < TY2 / 2 ? q : q - TY2 / 2;
      ly = 2 * qq + ((colA - (x0 + lx + y0)) & 1);
    }
    sA[ai(lx, ly)] = relax_a(lx, ly);
  }
  __syncthreads();
  // the other cell of the pair, from the new colA values; both are written
  double dz = 0.0, dzo = 0.0;
  if (j < n1) {
    const int lxB = 2 * tx + (1 - offA), iB = i0 + 1 - offA;
    const R bB = sB[ai(lxB, ty)];
    R vB = (R)0;
    if (iB < n0) {
      const int q = xi(lxB, ty);
      R T[6], D;
      coefu(K, iB, j, 0, n0, n1, 1, sR[q], sR[q - 1], sR[q + 1], sR[q - XW], sR[q + XW], (R)0,
            (R)0, T, D);
      const int a = ai(lxB, ty);
      const R off = T[0] * sA[a - 1] + T[1] * sA[a + 1] + T[2] * sA[a - AW] +
                    T[3] * sA[a + AW] + T[4] * (R)0 + T[5] * (R)0;
      vB = D > (R)0 ? (bB + off) * sw_rcp(D) : (R)0;
    }
    const R v0 = offA == 0 ? aOwn : vB, v1 = offA == 0 ? vB : aOwn;
    R *row = xout + n0 * j;
    if (i0 < n0) row[i0] = v0;
    if (i0 + 1 < n0) row[i0 + 1] = v1;
    if constexpr (DOT) {
      // b and the new x are zero outside the mesh
      const R b0 = sB[ai(2 * tx, ty)], b1 = sB[ai(2 * tx + 1, ty)];
      dz += (double)b0 * (double)v0 + (double)b1 * (double)v1;
      if (zold) {
        const R z0 = i0 < n0 ? zold[Q.c0 + i0 + n0 * j] : (R)0;
        const R z1 = i0 + 1 < n0 ? zold[Q.c0 + i0 + 1 + n0 * j] : (R)0;
        dzo += (double)b0 * (double)z0 + (double)b1 * (double)z1;
      }
    }
  }
  if constexpr (DOT) {
    const double s1 = block_sum_n<NT2 / 64>(dz, lred);
    if (t == 0) partials[g] = s1;
    if (zold) {
      const double s2 = block_sum_n<NT2 / 64>(dzo, lred);
      if (t == 0) partials[off2 + g] = s2;
    }
  }
}

// Restriction of a 2D fine level after a pre-smoothing that ended with a
// black half sweep: the coarse right-hand side is the sum of the red
// children's residuals.  Tiles of 128 x 8 fine cells (the shape of the
// 2.5-D restriction), one x-pair (one red cell) per thread; rows 2J and
// 2J+1 are combined through LDS.
template <typename R, typename B>
__global__ void __launch_bounds__(NT2) k_restrict2d(OpB<R> LB, SH S, const B *__restrict__ b,
                                                    const R *__restrict__ x, R *__restrict__ bc,
                                                    const int *__restrict__ mask) {
  static_assert(std::is_same<R, B>::value, "one precision per level");
  __shared__ R part[TY2 / 2][64];
  int g, s, lb;
  if (!locate(S, mask, g, s, lb)) return;
  const Op<R> L = op_at(LB, s);
  const LvS &Q = LB.ls[s];
  b += Q.c0;
  x += Q.c0;
  bc += Q.cc0;
  const int cn0 = Q.cn0;
  const int n0 = L.n0, n1 = L.n1;
  int xb, y0, k0, k1;
  tile_of(lb, n0, n1, 1, 128, S.kz, xb, y0, k0, k1);
  const int tx = threadIdx.x, ty = threadIdx.y;
  const int i0 = xb * 128 + 2 * tx, j = y0 + ty;
  const R *rA = L.rAU;
  R acc = 0;
  const int off = (j & 1) == 0 ? 0 : 1;  // the red cell of the pair
  const int i = i0 + off;
  if (j < n1 && i < n0) {
    const int c = i + n0 * j;
    R T[6], D;
    coef7(L, i, j, 0, rA[c], at2(rA, i - 1, j, n0, n1), at2(rA, i + 1, j, n0, n1),
          at2(rA, i, j - 1, n0, n1), at2(rA, i, j + 1, n0, n1), (R)0, (R)0, T, D);
    const R sm = T[0] * at2(x, i - 1, j, n0, n1) + T[1] * at2(x, i + 1, j, n0, n1) +
                 T[2] * at2(x, i, j - 1, n0, n1) + T[3] * at2(x, i, j + 1, n0, n1) +
                 T[4] * (R)0 + T[5] * (R)0;
    acc = (R)b[c] - (D * x[c] - sm);
  }
  if (ty & 1) part[ty >> 1][tx] = acc;
  __syncthreads();
  if (!(ty & 1) && i0 < n0 && j < n1) {
    const R other = (j + 1 < n1) ? part[ty >> 1][tx] : (R)0;
    bc[(i0 >> 1) + cn0 * (j >> 1)] = acc + other;
  }
}

// ------------------------------------------------------------------ host

template <typename R> static R *lx(Level &L);
template <> double *lx<double>(Level &L) { return L.x; }
template <> float *lx<float>(Level &L) { return L.xf; }
template <typename R> static R *lx2(Level &L);
template <> double *lx2<double>(Level &L) { return L.x2; }
template <> float *lx2<float>(Level &L) { return L.xf2; }
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

static SH sh(const Handle *h, const Shape &S) { return SH{S.bp, h->ns, S.kz}; }
static FL fl(const Handle *h) { return FL{h->flat.bp, h->ns, h->rng}; }

template <typename R>
static OpB<R> opb(Handle *h, int l, const R *rAU) {
  Level &L = h->lv[l];
  OpB<R> o;
  o.ls = L.ds;
  o.matfree = l == 0;
  o.rAU = rAU;
  o.Tx = lTx<R>(L); o.Ty = lTy<R>(L); o.Tz = lTz<R>(L); o.D = lD<R>(L);
  return o;
}

static void *dalloc(Handle *h, size_t bytes, int &rc) {
  void *p = nullptr;
  if (rc) return nullptr;
  const size_t n = bytes < 256 ? 256 : bytes;
  if (h->arena) return arena_take(h, n, rc);  // zeroed by the caller of the solve
  if (hipMalloc(&p, n) != hipSuccess) {
    rc = DBS_ENOMEM;
    return nullptr;
  }
  if (hipMemset(p, 0, n) != hipSuccess) rc = DBS_EHIP;
  h->allocs.push_back(p);
  return p;
}

// host table -> device; with a scratch arena on the handle's stream
static int upload(Handle *h, void *dst, const void *src, size_t bytes) {
  if (h->arena)
    return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, h->stream) == hipSuccess &&
                   hipStreamSynchronize(h->stream) == hipSuccess
               ? DBS_OK
               : DBS_EHIP;
  return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) == hipSuccess ? DBS_OK : DBS_EHIP;
}

// fill a shape from per-sample block counts
static void set_shape(Handle *h, Shape &S, const std::vector<int> &blocks, int kz, int &rc) {
  if (rc) return;
  S.kz = kz;
  S.hbp.assign(h->ns + 1, 0);
  for (int s = 0; s < h->ns; s++) S.hbp[s + 1] = S.hbp[s] + blocks[s];
  S.nblk = S.hbp[h->ns];
  if (!S.bp) S.bp = (int *)dalloc(h, sizeof(int) * (h->ns + 1), rc);
  if (!rc) rc = upload(h, S.bp, S.hbp.data(), sizeof(int) * (h->ns + 1));
}

static dim3 blk() { return dim3(BX, BY); }
static dim3 blk2() { return dim3(64, TY2); }

// planes per block: as many as kzmax while the launch keeps at least
// minblocks blocks
template <typename F>
static int pick_kz(int start, int kzmax, long long minblocks, F total_blocks) {
  int kz = start;
  while (kz < kzmax && total_blocks(2 * kz) >= minblocks) kz *= 2;
  return kz;
}

// launch shapes of every level and the bottom table; depends on the tuning
// knobs kz_fine, kz_coarse and bottom_shift
int pressure_retune(Handle *h) {
  int rc = DBS_OK;
  const int ns = h->ns;
  const bool mixed = h->ctl.precision == DBS_MIXED;
  const size_t rs = mixed ? 4 : 8;
  auto nlev = [&](int s) { return h->nlev[s]; };
  // bottom level per sample
  h->maxbottom = 0;
  h->nbt = 0;
  h->bottom.assign(ns, 0);
  for (int s = 0; s < ns; s++) {
    const int nl = nlev(s);
    if (nl < 2) continue;
    int bl = nl - 1;
    for (int l = 1; l < nl; l++) {
      size_t cells = 0;
      for (int m = l; m < nl; m++) {
        const LvS &Q = h->lv[m].hs[s];
        cells += (size_t)Q.n0 * Q.n1 * Q.n2;
      }
      const size_t pad = (size_t)h->lv[l].hs[s].n0 * h->lv[l].hs[s].n1;
      if ((cells + pad) * 6 * rs + 16 <= (size_t)BOTTOM_LDS) { bl = l; break; }
    }
    bl = std::min(bl + h->bottom_shift, nl - 1);
    h->bottom[s] = bl;
    h->maxbottom = std::max(h->maxbottom, bl);
    h->nbt++;
  }
  // fine level shapes
  Level &F = h->lv[0];
  std::vector<int> blocks(ns);
  auto fine_total = [&](int W, int kz, bool need_coarse) {
    long long t = 0;
    for (int s = 0; s < ns; s++)
      if (!need_coarse || nlev(s) > 1) t += tiles25(F.hs[s].n0, F.hs[s].n1, F.hs[s].n2, W, kz);
    return t;
  };
  const int kst = h->kz_fine > 0 ? h->kz_fine : pick_kz(1, KZ2, MIN_BLOCKS2, [&](int kz) {
    return fine_total(64, kz, false);
  });
  const int ksm = h->kz_fine > 0 ? h->kz_fine : pick_kz(1, KZ2, MIN_BLOCKS2, [&](int kz) {
    return fine_total(128, kz, false);
  });
  int krs = h->kz_fine > 1 ? h->kz_fine : pick_kz(2, KZ2, MIN_BLOCKS2, [&](int kz) {
    return fine_total(128, kz, true);
  });
  if (krs & 1) krs++;
  for (int s = 0; s < ns; s++) blocks[s] = tiles25(F.hs[s].n0, F.hs[s].n1, F.hs[s].n2, 64, kst);
  set_shape(h, F.st, blocks, kst, rc);
  for (int s = 0; s < ns; s++) blocks[s] = tiles25(F.hs[s].n0, F.hs[s].n1, F.hs[s].n2, 128, ksm);
  set_shape(h, F.sm, blocks, ksm, rc);
  for (int s = 0; s < ns; s++)
    blocks[s] = nlev(s) > 1 ? tiles25(F.hs[s].n0, F.hs[s].n1, F.hs[s].n2, 128, krs) : 0;
  set_shape(h, F.rs, blocks, krs, rc);
  F.flat = 1;
  for (int s = 0; s < ns; s++)
    if (F.hs[s].n2 != 1) F.flat = 0;
  // coarse levels
  for (int l = 1; l < (int)h->lv.size() && !rc; l++) {
    Level &L = h->lv[l];
    auto shape_of = [&](Shape &S, bool pair, auto member) {
      auto total = [&](int kz) {
        long long t = 0;
        for (int s = 0; s < ns; s++)
          if (member(s)) t += column_blocks(L.hs[s].n0, L.hs[s].n1, L.hs[s].n2, kz, pair);
        return t;
      };
      const int kz = h->kz_coarse > 0 ? h->kz_coarse : pick_kz(1, KZ, MIN_BLOCKS, total);
      for (int s = 0; s < ns; s++)
        blocks[s] = member(s) ? column_blocks(L.hs[s].n0, L.hs[s].n1, L.hs[s].n2, kz, pair) : 0;
      set_shape(h, S, blocks, kz, rc);
    };
    shape_of(L.one_all, false, [&](int s) { return nlev(s) > l; });
    shape_of(L.pair_cyc, true, [&](int s) { return nlev(s) > l && h->bottom[s] > l; });
    shape_of(L.one_cyc, false, [&](int s) { return nlev(s) > l && h->bottom[s] > l; });
    shape_of(L.one_rc, false, [&](int s) { return l >= 2 && nlev(s) > l && h->bottom[s] >= l; });
    // fused coarse sweeps: about a block per CU (the kernel's LDS holds one)
    {
      auto cyc = [&](int s) { return nlev(s) > l && h->bottom[s] > l; };
      auto total = [&](int kz) {
        long long t = 0;
        for (int s = 0; s < ns; s++)
          if (cyc(s)) t += tiles25(L.hs[s].n0, L.hs[s].n1, L.hs[s].n2, 128, kz);
        return t;
      };
      const int kz = h->kz_coarse > 0 ? h->kz_coarse : pick_kz(1, KZ2, MIN_BLOCKS_CSW, total);
      L.sw_lanes = 0;
      for (int s = 0; s < ns; s++) {
        blocks[s] = cyc(s) ? tiles25(L.hs[s].n0, L.hs[s].n1, L.hs[s].n2, 128, kz) : 0;
        if (cyc(s))
          L.sw_lanes += (long long)((L.hs[s].n0 + 127) / 128 * 128) *
                        ((L.hs[s].n1 + TY2 - 1) / TY2 * TY2) * L.hs[s].n2;
      }
      set_shape(h, L.sw, blocks, kz, rc);
      // the plane wavefront stages three planes beyond a tile's own: thin
      // (2D or nearly) levels take the small tiles (or half sweeps)
      L.sw_ok = 1;
      for (int s = 0; s < ns; s++)
        if (cyc(s) && L.hs[s].n2 < CSW_MIN_DEPTH) L.sw_ok = 0;
      // block-local smoothing: one block per CB^3 tile
      for (int s = 0; s < ns; s++)
        blocks[s] = cyc(s) ? cb_tiles(L.hs[s].n0, L.hs[s].n1, L.hs[s].n2) : 0;
      set_shape(h, L.cb, blocks, 1, rc);
      // small-tile sweeps: one block per 8 x 8 x 4 tile, or per 16 x 16 x 1
      // tile where every cycled sample is one cell deep
      L.cyc_cells = 0;
      L.cs2d = 1;
      for (int s = 0; s < ns; s++)
        if (cyc(s) && L.hs[s].n2 != 1) L.cs2d = 0;
      for (int s = 0; s < ns; s++) {
        const LvS &Q = L.hs[s];
        blocks[s] = !cyc(s) ? 0
                    : L.cs2d ? cs_tiles<Cs2>(Q.n0, Q.n1, Q.n2)
                             : cs_tiles<Cs3>(Q.n0, Q.n1, Q.n2);
        if (cyc(s)) L.cyc_cells += (long long)Q.n0 * Q.n1 * Q.n2;
      }
      set_shape(h, L.cs, blocks, 1, rc);
    }
  }
  if (rc) return rc;
  // bottom table (one work-group per sample with a coarse level)
  auto build = [&](auto tag) -> int {
    using R = decltype(tag);
    std::vector<Bottom<R>> tab;
    for (int s = 0; s < ns; s++) {
      const int nl = nlev(s);
      if (nl < 2) continue;
      Bottom<R> A;
      memset(&A, 0, sizeof(A));
      A.s = s;
      A.nl = nl - h->bottom[s];
      A.pre = h->mgc;
      A.post = h->mgc;
      int off = 0;
      for (int m = 0; m < A.nl; m++) {
        Level &L = h->lv[h->bottom[s] + m];
        const LvS &Q = L.hs[s];
        A.L[m] = BLevel<R>{Q.n0, Q.n1, Q.n2, off, lTx<R>(L) + Q.c0, lTy<R>(L) + Q.c0,
                           lTz<R>(L) + Q.c0, lD<R>(L) + Q.c0, lx<R>(L) + Q.c0, lb<R>(L) + Q.c0};
        off += Q.n0 * Q.n1 * Q.n2;
      }
      A.ntot = off;
      A.pad = std::max(1, A.L[0].n0 * A.L[0].n1);  // one plane of the top level
      if ((size_t)6 * (A.ntot + A.pad) * sizeof(R) + 16 > (size_t)BOTTOM_LDS) {
        h->err = "bottom levels exceed the work-group's LDS";
        return DBS_EINVAL;
      }
      // a one-cell coarsest level is solved exactly by one sweep
      const LvS &Cq = h->lv[nl - 1].hs[s];
      A.coarse_sweeps = Cq.n0 * Cq.n1 * Cq.n2 == 1 ? 1 : h->coarse_sweeps;
      tab.push_back(A);
    }
    if (tab.empty()) return DBS_OK;
    int r2 = DBS_OK;
    if (!h->btab) h->btab = dalloc(h, sizeof(Bottom<R>) * tab.size(), r2);
    if (r2) return r2;
    return upload(h, h->btab, tab.data(), sizeof(Bottom<R>) * tab.size());
  };
  rc = mixed ? build(0.0f) : build(0.0);
  return rc;
}

int pressure_setup(Handle *h) {
  int rc = DBS_OK;
  const int ns = h->ns;
  const bool mixed = h->ctl.precision == DBS_MIXED;
  // per-sample level dimensions
  std::vector<std::vector<std::array<int, 3>>> dims(ns);
  int nlmax = 0;
  h->nlev.assign(ns, 0);
  for (int s = 0; s < ns; s++) {
    std::array<int, 3> d = {h->hG[s].n[0], h->hG[s].n[1], h->hG[s].n[2]};
    dims[s].push_back(d);
    while ((int)dims[s].size() < MAXLV && (long long)d[0] * d[1] * d[2] > 1) {
      for (int a = 0; a < 3; a++) d[a] = (d[a] + 1) / 2;
      dims[s].push_back(d);
    }
    h->nlev[s] = (int)dims[s].size();
    nlmax = std::max(nlmax, h->nlev[s]);
  }
  h->lv.assign(nlmax, Level());
  // arenas: level 0 is the fine cell arena; coarse levels are packed
  for (int l = 0; l < nlmax; l++) {
    Level &L = h->lv[l];
    L.hs.assign(ns, LvS());
    long long off = 0;
    for (int s = 0; s < ns; s++) {
      LvS &Q = L.hs[s];
      memset(&Q, 0, sizeof(Q));
      const Geom &G = h->hG[s];
      for (int a = 0; a < 3; a++) Q.c[a] = G.area[a] * G.ih[a];
      for (int b = 0; b < 6; b++) Q.ob[b] = G.bck[b] == BC_OUTLET ? 2.0 * Q.c[b / 2] : 0.0;
      Q.outlet = G.has_outlet;
      if (l >= h->nlev[s]) continue;
      Q.n0 = dims[s][l][0]; Q.n1 = dims[s][l][1]; Q.n2 = dims[s][l][2];
      if (l == 0) {
        Q.c0 = G.c0;
      } else {
        Q.c0 = (int)off;
        // next sample on a 4-cell boundary: its rows may use 16-byte loads
        off += ((long long)Q.n0 * Q.n1 * Q.n2 + 3) & ~3LL;
      }
    }
    L.nc = l == 0 ? h->NC : off;
  }
  for (int l = 0; l + 1 < nlmax; l++)
    for (int s = 0; s < ns; s++) {
      if (l + 1 >= h->nlev[s]) continue;
      LvS &Q = h->lv[l].hs[s];
      const LvS &C = h->lv[l + 1].hs[s];
      Q.cn0 = C.n0; Q.cn1 = C.n1; Q.cn2 = C.n2; Q.cc0 = C.c0;
    }
  for (int l = 0; l < nlmax && !rc; l++) {
    Level &L = h->lv[l];
    L.ds = (LvS *)dalloc(h, sizeof(LvS) * ns, rc);
    if (!rc) rc = upload(h, L.ds, L.hs.data(), sizeof(LvS) * ns);
    if (l == 0 || rc) continue;
    const size_t n = (size_t)L.nc;
    const size_t s = mixed ? 4 : 8;
    void *Tx = dalloc(h, n * s, rc), *Ty = dalloc(h, n * s, rc), *Tz = dalloc(h, n * s, rc);
    void *Db = dalloc(h, n * s, rc), *D = dalloc(h, n * s, rc), *x = dalloc(h, n * s, rc);
    void *b = dalloc(h, n * s, rc);
    if (rc) return rc;
    if (mixed) {
      L.Txf = (float *)Tx; L.Tyf = (float *)Ty; L.Tzf = (float *)Tz; L.Dbf = (float *)Db;
      L.Df = (float *)D; L.xf = (float *)x; L.bf = (float *)b;
      L.xf2 = (float *)dalloc(h, n * s, rc);
    } else {
      L.Tx = (double *)Tx; L.Ty = (double *)Ty; L.Tz = (double *)Tz; L.Db = (double *)Db;
      L.D = (double *)D; L.x = (double *)x; L.b = (double *)b;
      L.x2 = (double *)dalloc(h, n * s, rc);
    }
  }
  if (rc) return rc;
  const size_t NC = (size_t)h->NC;
  if (mixed) {
    h->lv[0].xf = (float *)dalloc(h, NC * 4, rc);   // z (FP32)
    h->lv[0].bf = (float *)dalloc(h, NC * 4, rc);   // rAU (FP32)
    h->rf = (float *)dalloc(h, NC * 4, rc);         // r (FP32)
    h->zoldf = (float *)dalloc(h, NC * 4, rc);      // previous z (FP32)
    h->zf2 = (float *)dalloc(h, NC * 4, rc);        // second z buffer (FP32)
  } else {
    h->z2 = (double *)dalloc(h, NC * 8, rc);        // second z buffer
  }
  h->act = (int *)dalloc(h, sizeof(int) * ns, rc);
  h->want = (int *)dalloc(h, sizeof(int) * ns, rc);
  if (rc) return rc;
  // partial sums: the largest launch (fine tiles at one plane per block)
  size_t np = 2 * (size_t)(NC / FLAT_CELLS);
  size_t t1 = 0;
  for (int s = 0; s < ns; s++)
    t1 += (size_t)tiles25(h->hG[s].n[0], h->hG[s].n[1], h->hG[s].n[2], 64, 1);
  np = std::max(np, 2 * t1);
  np = std::max(np, (size_t)NSTAT * h->cell.nblk);
  h->partials = (double *)dalloc(h, np * 8, rc);
  h->npartials = np;
  if (rc) return rc;
  for (int s = 0; s < ns; s++) h->st[s].mg_levels = h->nlev[s];
  return pressure_retune(h);
}

void pressure_free(Handle *h) { h->lv.clear(); }

template <typename R>
static void build_hierarchy(Handle *h, const R *rAUr) {
  for (size_t l = 1; l < h->lv.size(); l++) {
    Level &C = h->lv[l];
    Level &F = h->lv[l - 1];
    if (!C.one_all.nblk) continue;
    OpB<R> opF = opb<R>(h, (int)l - 1, rAUr);
    DBS_LAUNCH(h, KC_BUILD_COARSE, k_build_coarse<R>, dim3(C.one_all.nblk), blk(), opF,
               (const R *)(l == 1 ? nullptr : lDb<R>(F)), sh(h, C.one_all), lTx<R>(C),
               lTy<R>(C), lTz<R>(C), lDb<R>(C));
    DBS_LAUNCH(h, KC_BUILD_COARSE, k_diag<R>, dim3(C.one_all.nblk), blk(), (const LvS *)C.ds,
               sh(h, C.one_all), (const R *)lTx<R>(C), (const R *)lTy<R>(C),
               (const R *)lTz<R>(C), (const R *)lDb<R>(C), lD<R>(C));
  }
}

template <typename R, typename B>
static void smooth_level(Handle *h, int l, const OpB<R> &o, const B *b, R *x, bool down) {
  Level &L = h->lv[l];
  if (!L.pair_cyc.nblk) return;
  const SH S = sh(h, L.pair_cyc);
  const dim3 g(L.pair_cyc.nblk);
  const int n = h->mgc;
  const int first = down ? 0 : 1;
  for (int s = 0; s < n; s++) {
    DBS_LAUNCH(h, KC_SMOOTHC, (k_smooth<R, B>), g, blk(), o, S, b, x, first,
               (int)(down && s == 0), (const int *)h->act);
    DBS_LAUNCH(h, KC_SMOOTHC, (k_smooth<R, B>), g, blk(), o, S, b, x, 1 - first, 0,
               (const int *)h->act);
  }
}

// fine-level half sweep with the 2.5-D kernel
template <typename R, typename B>
static void smooth_fine(Handle *h, const OpB<R> &o, const B *b, const R *xin, R *xout, int color,
                        int mode, const R *xc) {
  const Shape &Z = h->lv[0].sm;
  const dim3 g(Z.nblk);
  const SH S = sh(h, Z);
  const int *m = h->act;
  if (mode == SM_ZERO)
    DBS_LAUNCH(h, KC_SMOOTH0_ZERO, (k_smooth25<R, B, SM_ZERO>), g, blk2(), o, S, b, xin, xout,
               color, xc, m);
  else if (mode == SM_PROLONG)
    DBS_LAUNCH(h, KC_PROLONG0, (k_smooth25<R, B, SM_PROLONG>), g, blk2(), o, S, b, xin, xout,
               color, xc, m);
  else
    DBS_LAUNCH(h, KC_SMOOTH0, (k_smooth25<R, B, SM_NORMAL>), g, blk2(), o, S, b, xin, xout,
               color, xc, m);
}

// one fused fine-level sweep (colour colA first), xin -> xout
template <typename R, typename B>
static void sweep_fine(Handle *h, const OpB<R> &o, const B *b, const R *xin, R *xout, int colA,
                       int mode, const R *xc) {
  const Shape &Z = h->lv[0].sm;
  const dim3 g(Z.nblk);
  const SH S = sh(h, Z);
  const int *m = h->act;
  const R *nz = nullptr;
  double *np = nullptr;
  if (h->lv[0].flat) {
    if (mode == SW_ZERO)
      DBS_LAUNCH(h, KC_SMOOTH0_ZERO, (k_sweep2d<R, B, SW_ZERO>), g, blk2(), o, S, b, xin, xout,
                 colA, xc, m, nz, np, 0);
    else if (mode == SW_PROLONG)
      DBS_LAUNCH(h, KC_PROLONG0, (k_sweep2d<R, B, SW_PROLONG>), g, blk2(), o, S, b, xin, xout,
                 colA, xc, m, nz, np, 0);
    else
      DBS_LAUNCH(h, KC_SMOOTH0, (k_sweep2d<R, B, SW_NORMAL>), g, blk2(), o, S, b, xin, xout,
                 colA, xc, m, nz, np, 0);
    return;
  }
  if (mode == SW_ZERO)
    DBS_LAUNCH(h, KC_SMOOTH0_ZERO, (k_sweep25<R, B, SW_ZERO>), g, blk2(), o, S, b, xin, xout,
               colA, xc, m, nz, np, 0);
  else if (mode == SW_PROLONG)
    DBS_LAUNCH(h, KC_PROLONG0, (k_sweep25<R, B, SW_PROLONG>), g, blk2(), o, S, b, xin, xout,
               colA, xc, m, nz, np, 0);
  else
    DBS_LAUNCH(h, KC_SMOOTH0, (k_sweep25<R, B, SW_NORMAL>), g, blk2(), o, S, b, xin, xout,
               colA, xc, m, nz, np, 0);
}

// the same sweep (FP32, SW_PROLONG or SW_NORMAL) also forming the partial
// sums of b.xout and b.zold per block of the fine smoothing shape
static void sweep_fine_dot(Handle *h, const OpB<float> &o, const float *b, const float *xin,
                           float *xout, int colA, int mode, const float *xc,
                           const float *zold) {
  const Shape &Z = h->lv[0].sm;
  const dim3 g(Z.nblk);
  const SH S = sh(h, Z);
  const int *m = h->act;
  if (h->lv[0].flat) {
    if (mode == SW_PROLONG)
      DBS_LAUNCH(h, KC_PROLONG0, (k_sweep2d<float, float, SW_PROLONG, 1>), g, blk2(), o, S, b,
                 xin, xout, colA, xc, m, zold, h->partials, (int)Z.nblk);
    else
      DBS_LAUNCH(h, KC_SMOOTH0_DOT, (k_sweep2d<float, float, SW_NORMAL, 1>), g, blk2(), o, S,
                 b, xin, xout, colA, xc, m, zold, h->partials, (int)Z.nblk);
    return;
  }
  if (mode == SW_PROLONG)
    DBS_LAUNCH(h, KC_PROLONG0, (k_sweep25<float, float, SW_PROLONG, 0, 1>), g, blk2(), o, S,
               b, xin, xout, colA, xc, m, zold, h->partials, (int)Z.nblk);
  else
    DBS_LAUNCH(h, KC_SMOOTH0_DOT, (k_sweep25<float, float, SW_NORMAL, 0, 1>), g, blk2(), o, S,
               b, xin, xout, colA, xc, m, zold, h->partials, (int)Z.nblk);
}

// The coarse-level smoother of the V-cycle with fused sweeps (coarse_block
// 0): small tiles on levels of at most CS_MAX_CELLS cycled cells (launch-
// and latency-bound) and on levels too thin for the plane walk; half sweeps
// on the larger levels whose rows would leave more than half of the
// 128-wide plane-walk tiles' lanes idle (a batch of small samples: there the
// half sweeps, walking the columns in order, beat the small tiles, 243
// against 257 ms per step of the 512-sample batch); the plane walk on the
// others.  The FP64 V-cycle has no plane walk (its planes would not fit in
// LDS) and takes half sweeps there (its small tiles, with a third of the
// blocks per CU, were slower).  coarse_block 2: the plane walk where deep
// enough, else half sweeps; 3: small tiles everywhere; 4: half sweeps
// everywhere.
constexpr long long CS_MAX_CELLS = 1LL << 20;
enum { CS_HALF = 0, CS_TILES = 1, CS_WALK = 2 };
template <typename R>
static int coarse_smoother(const Handle *h, const Level &L) {
  constexpr bool fp32 = std::is_same<R, float>::value;
  if (!h->fused_sweep || h->coarse_block == 4) return CS_HALF;
  if (h->coarse_block == 3) return CS_TILES;
  if (h->coarse_block == 2) return fp32 && L.sw_ok ? CS_WALK : CS_HALF;
  if (!L.sw_ok || L.cyc_cells <= CS_MAX_CELLS) return CS_TILES;
  if (!fp32 || 2 * L.cyc_cells < L.sw_lanes) return CS_HALF;
  return CS_WALK;
}

// the V-cycle smooths coarse level L with fused sweeps (plane walk or small
// tiles) rather than half sweeps
template <typename R>
static bool fused_coarse(const Handle *h, const Level &L) {
  return coarse_smoother<R>(h, L) != CS_HALF;
}

// one fused sweep on coarse level l (stored coefficients), xin -> xout
template <typename R>
static void sweep_coarse(Handle *h, int l, const OpB<R> &o, const R *b, const R *xin, R *xout,
                         int colA, int mode, const R *xc) {
  const int *m = h->act;
  if (coarse_smoother<R>(h, h->lv[l]) == CS_TILES) {
    const Shape &C = h->lv[l].cs;
    if (!C.nblk) return;
    const dim3 g(C.nblk);
    const SH S = sh(h, C);
    auto go = [&](auto tile) {
      using TL = decltype(tile);
      if (mode == SW_ZERO)
        DBS_LAUNCH(h, KC_SMOOTHC, (k_csweep<SW_ZERO, TL, R>), g, dim3(CST), o, S, b, xin, xout,
                   colA, xc, m);
      else if (mode == SW_PROLONG)
        DBS_LAUNCH(h, KC_SMOOTHC, (k_csweep<SW_PROLONG, TL, R>), g, dim3(CST), o, S, b, xin,
                   xout, colA, xc, m);
      else
        DBS_LAUNCH(h, KC_SMOOTHC, (k_csweep<SW_NORMAL, TL, R>), g, dim3(CST), o, S, b, xin,
                   xout, colA, xc, m);
    };
    if (h->lv[l].cs2d)
      go(Cs2{});
    else
      go(Cs3{});
    return;
  }
  if constexpr (std::is_same<R, float>::value) {
  const Shape &Z = h->lv[l].sw;
  if (!Z.nblk) return;
  const dim3 g(Z.nblk);
  const SH S = sh(h, Z);
  const float *nz = nullptr;
  double *np = nullptr;
  if (mode == SW_ZERO)
    DBS_LAUNCH(h, KC_SMOOTHC, (k_sweep25<float, float, SW_ZERO, 1>), g, blk2(), o, S, b, xin,
               xout, colA, xc, m, nz, np, 0);
  else if (mode == SW_PROLONG)
    DBS_LAUNCH(h, KC_SMOOTHC, (k_sweep25<float, float, SW_PROLONG, 1>), g, blk2(), o, S, b,
               xin, xout, colA, xc, m, nz, np, 0);
  else
    DBS_LAUNCH(h, KC_SMOOTHC, (k_sweep25<float, float, SW_NORMAL, 1>), g, blk2(), o, S, b,
               xin, xout, colA, xc, m, nz, np, 0);
  }
}

// z = M r: one V-cycle over the active samples.  b0 is the fine right-hand
// side (r); z0 and z1 are the two fine correction buffers; returns the one
// holding the result.  dot (FP32 fused sweeps): the last sweep also leaves
// the per-block partial sums of b0.z and b0.zold (zold may be null) for a
// finalize over the fine smoothing shape.
template <typename R, typename B>
static R *vcycle(Handle *h, const R *rAUr, const B *b0, R *z0, R *z1, bool dot = false,
                 const R *zold = nullptr) {
  const int *act = h->act;
  const int nl = (int)h->lv.size();
  OpB<R> o0 = opb<R>(h, 0, rAUr);
  const R *xc1 = nl > 1 ? (const R *)lx<R>(h->lv[1]) : nullptr;
  // fine level down: red (zero guess), black, ...; red-only restriction.
  // Fused sweeps alternate between the two buffers; cur holds the iterate.
  R *cur = z0, *oth = z1;
  for (int s = 0; s < h->mg_pre; s++) {
    if (h->fused_sweep) {
      if (s == 0) {
        sweep_fine<R, B>(h, o0, b0, (const R *)nullptr, cur, 0, SW_ZERO, (const R *)nullptr);
      } else {
        sweep_fine<R, B>(h, o0, b0, cur, oth, 0, SW_NORMAL, (const R *)nullptr);
        std::swap(cur, oth);
      }
    } else {
      smooth_fine<R, B>(h, o0, b0, z0, z0, 0, s == 0 ? SM_ZERO : SM_NORMAL, (const R *)nullptr);
      smooth_fine<R, B>(h, o0, b0, z0, z0, 1, SM_NORMAL, (const R *)nullptr);
    }
  }
  if (nl > 1 && h->lv[0].rs.nblk) {
    const Shape &Z = h->lv[0].rs;
    if (h->lv[0].flat)
      DBS_LAUNCH(h, KC_RESTRICT0, (k_restrict2d<R, B>), dim3(Z.nblk), blk2(), o0, sh(h, Z), b0,
                 (const R *)cur, lb<R>(h->lv[1]), act);
    else
      DBS_LAUNCH(h, KC_RESTRICT0, (k_restrict25<R, B>), dim3(Z.nblk), blk2(), o0, sh(h, Z), b0,
                 (const R *)cur, lb<R>(h->lv[1]), act);
  }
  // Coarse levels.  With fused sweeps, a level's sweeps alternate between
  // its two correction buffers; the first (zero guess) writes the second
  // buffer (xf2, x2), so the 2 mgc sweeps of a cycle end in the first (xf,
  // x), where the bottom also leaves its result.  ccur[l] holds the
  // pre-smoothed iterate.
  constexpr bool flexr = std::is_same<R, float>::value;
  const bool cblock = flexr && h->coarse_block == 1;
  std::vector<R *> ccur(h->lv.size(), nullptr), coth(h->lv.size(), nullptr);
  for (int l = 1; l < h->maxbottom; l++) {
    OpB<R> o = opb<R>(h, l, rAUr);
    Level &L = h->lv[l];
    Level &C = h->lv[l + 1];
    ccur[l] = lx<R>(L);
    const bool cbl = cblock && L.cb.nblk;
    const bool lf = !cbl && fused_coarse<R>(h, L);
    if constexpr (flexr) {
      if (cbl) {
        // all pre-sweeps of the level in one launch, into xf2
        DBS_LAUNCH(h, KC_SMOOTHC, k_cblock<CB_ZERO>, dim3(L.cb.nblk), dim3(CBT), o,
                   sh(h, L.cb), (const float *)lb<R>(L), (const float *)nullptr, (float *)L.xf2,
                   (const float *)nullptr, h->mgc, act);
        ccur[l] = (R *)L.xf2;
      }
    }
    if (lf) {
      R *a = lx2<R>(L), *b2 = lx<R>(L);
      sweep_coarse<R>(h, l, o, (const R *)lb<R>(L), (const R *)nullptr, a, 0, SW_ZERO,
                      (const R *)nullptr);
      for (int s = 1; s < h->mgc; s++) {
        sweep_coarse<R>(h, l, o, (const R *)lb<R>(L), (const R *)a, b2, 0, SW_NORMAL,
                        (const R *)nullptr);
        std::swap(a, b2);
      }
      ccur[l] = a;
      coth[l] = b2;
    }
    if (!lf && !cbl) smooth_level<R, R>(h, l, o, (const R *)lb<R>(L), lx<R>(L), true);
    if (C.one_rc.nblk)
      DBS_LAUNCH(h, KC_RESTRICTC, (k_restrict<R, R>), dim3(C.one_rc.nblk), blk(), o,
                 sh(h, C.one_rc), (const R *)lb<R>(L), (const R *)ccur[l], lb<R>(C), act,
                 h->mgc > 0 ? 1 : 0);
  }
  if (h->nbt)
    DBS_LAUNCH(h, KC_COARSE, k_bottom<R>, dim3(h->nbt), dim3(1024),
               (const Bottom<R> *)h->btab, act);
  for (int l = h->maxbottom - 1; l >= 1; l--) {
    OpB<R> o = opb<R>(h, l, rAUr);
    Level &L = h->lv[l];
    Level &C = h->lv[l + 1];
    if constexpr (flexr) {
      if (cblock && L.cb.nblk) {
        // the prolongation and all post-sweeps in one launch: xf2 -> xf,
        // where the finer level's prolongation reads the correction
        DBS_LAUNCH(h, KC_SMOOTHC, k_cblock<CB_PROLONG>, dim3(L.cb.nblk), dim3(CBT), o,
                   sh(h, L.cb), (const float *)lb<R>(L), (const float *)L.xf2, (float *)lx<R>(L),
                   (const float *)lx<R>(C), h->mgc, act);
        continue;
      }
    }
    if (fused_coarse<R>(h, L)) {
      // the prolongation rides on the first (black) sweep
      R *a = ccur[l], *b2 = coth[l];
      for (int s = 0; s < h->mgc; s++) {
        sweep_coarse<R>(h, l, o, (const R *)lb<R>(L), (const R *)a, b2, 1,
                        s == 0 ? SW_PROLONG : SW_NORMAL, (const R *)lx<R>(C));
        std::swap(a, b2);
      }
      continue;
    }
    if (L.one_cyc.nblk)
      DBS_LAUNCH(h, KC_PROLONGC, k_prolong<R>, dim3(L.one_cyc.nblk), blk(), (const LvS *)L.ds,
                 sh(h, L.one_cyc), (const R *)lx<R>(C), lx<R>(L), act);
    smooth_level<R, R>(h, l, o, (const R *)lb<R>(L), lx<R>(L), false);
  }
  // fine level up: the prolongation rides on the first (black) half sweep
  if (h->fused_sweep) {
    for (int s = 0; s < h->mg_post; s++) {
      const int mode = s == 0 ? SW_PROLONG : SW_NORMAL;
      if constexpr (std::is_same<R, float>::value && std::is_same<B, float>::value) {
        if (dot && s + 1 == h->mg_post) {
          sweep_fine_dot(h, o0, b0, cur, oth, 1, mode, xc1, zold);
          std::swap(cur, oth);
          continue;
        }
      }
      sweep_fine<R, B>(h, o0, b0, cur, oth, 1, mode, xc1);
      std::swap(cur, oth);
    }
    return cur;
  }
  for (int s = 0; s < h->mg_post; s++) {
    if (s == 0)
      smooth_fine<R, B>(h, o0, b0, z0, z1, 1, SM_PROLONG, xc1);
    else
      smooth_fine<R, B>(h, o0, b0, z1, z1, 1, SM_NORMAL, (const R *)nullptr);
    smooth_fine<R, B>(h, o0, b0, z1, z1, 0, SM_NORMAL, (const R *)nullptr);
  }
  return z1;
}

// ---------------------------------------------------------------- CG

static FinArgs fin_args(Handle *h, const Shape *S, int two, int slot, int slot2, int op,
                        const int *mask, int closed_only = 0) {
  FinArgs A;
  A.partials = h->partials;
  A.bp = S ? S->bp : nullptr;
  A.off2 = S ? S->nblk : 0;
  A.two = two;
  A.slot = slot;
  A.slot2 = slot2;
  A.op = op;
  A.mask = mask;
  A.rng = h->rng;
  A.closed_only = closed_only;
  A.act = h->act;
  A.want = h->want;
  A.tol2 = h->ctl.p_tol * h->ctl.p_tol;
  A.maxit = h->ctl.p_maxit;
  return A;
}

static void finalize(Handle *h, const FinArgs &A) {
  DBS_LAUNCH(h, KC_FINALIZE, k_finalize, dim3(h->ns), dim3(FIN_T), A, h->scal);
}

static bool any_closed(const Handle *h) {
  for (const Rng &g : h->hrng)
    if (g.closed) return true;
  return false;
}

static dim3 flat_grid(const Handle *h) { return dim3((unsigned)(h->NC / FLAT_CELLS)); }

void arena_copy(Handle *h, const double *src, double *dst, int narrays) {
  DBS_LAUNCH(h, KC_MISC, k_copy, dim3((unsigned)(narrays * (h->NC / FLAT_CELLS))),
             dim3(FLAT_T), src, dst);
}

// x -= mean(x) on the closed samples selected by mask (FP32 copy refreshed)
static void remove_mean(Handle *h, double *x, float *xf, const int *mask) {
  DBS_LAUNCH(h, KC_MISC, k_sum, flat_grid(h), dim3(FLAT_T), fl(h), (const double *)x,
             h->partials, mask);
  finalize(h, fin_args(h, &h->flat, 0, S_SUM, 0, FIN_STORE, mask, 1));
  DBS_LAUNCH(h, KC_MISC, k_sub_mean, flat_grid(h), dim3(FLAT_T), fl(h), (const double *)h->scal,
             x, xf, mask);
}

// slot = a.a over the closed samples selected by mask
static void dot_self_closed(Handle *h, const double *a, int slot, const int *mask) {
  DBS_LAUNCH(h, KC_DOT, k_dot2<double>, flat_grid(h), dim3(FLAT_T), fl(h), a, a,
             (const double *)nullptr, h->partials, (int)h->flat.nblk, mask, 1);
  finalize(h, fin_args(h, &h->flat, 0, slot, 0, FIN_STORE, mask, 1));
}

// true residual r = b - A x (and its FP32 copy) of the samples selected by
// mask; S_RR = r.r (projected on closed samples) and S_BB = b.b; then the
// finalize op `then` on the same samples (in the same launch as the sums
// when no sample is closed)
static void true_residual(Handle *h, const double *rAU, const double *b, const double *x,
                          float *rf, const int *mask, int then = FIN_STORE) {
  const Shape &Z = h->lv[0].st;
  OpB<double> o = opb<double>(h, 0, rAU);
  if (h->lv[0].flat)
    DBS_LAUNCH(h, KC_RESIDUAL, k_stencil2d<1>, dim3(Z.nblk), blk2(), o, sh(h, Z), x, b, h->r, rf,
               h->partials, (int)Z.nblk, mask);
  else
    DBS_LAUNCH(h, KC_RESIDUAL, k_stencil25<1>, dim3(Z.nblk), blk2(), o, sh(h, Z), x, b, h->r, rf,
               h->partials, (int)Z.nblk, mask);
  const bool closed = any_closed(h);
  finalize(h, fin_args(h, &Z, 1, S_RR, S_BB, closed ? FIN_STORE : then, mask));
  if (closed) {
    remove_mean(h, h->r, rf, mask);
    dot_self_closed(h, h->r, S_RR, mask);
    if (then != FIN_STORE) finalize(h, fin_args(h, nullptr, 0, 0, 0, then, mask));
  }
}

// the active flags into host-mapped memory (a kernel store, where a
// device-to-host copy would launch a blit of about 25 us)
__global__ void k_publish(const int *__restrict__ act, int *__restrict__ pub, int n) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) pub[s] = act[s];
}
__global__ void k_publish2(const int *__restrict__ act, const int *__restrict__ want,
                           int *__restrict__ pub, int n) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) {
    pub[s] = act[s];
    pub[n + s] = want[s];
  }
}

// copies the CG flags to the host; returns the number of active samples and
// sets *nwant to the number asking for a true residual
static int fetch_flags(Handle *h, int *nwant) {
  if (h->dpub) {
    DBS_LAUNCH(h, KC_MISC, k_publish2, dim3((h->ns + 255) / 256), dim3(256),
               (const int *)h->act, (const int *)h->want, h->dpub, h->ns);
  } else {
    // no host-mapped memory (scratch-arena solve): plain copies
    (void)hipMemcpyAsync(h->hpub, h->act, sizeof(int) * h->ns, hipMemcpyDeviceToHost, h->stream);
    (void)hipMemcpyAsync(h->hpub + h->ns, h->want, sizeof(int) * h->ns, hipMemcpyDeviceToHost,
                         h->stream);
  }
  (void)hipStreamSynchronize(h->stream);
  int na = 0, nw = 0;
  for (int s = 0; s < h->ns; s++) {
    na += h->hpub[s] != 0;
    nw += h->hpub[h->ns + s] != 0;
  }
  if (nwant) *nwant = nw;
  return na;
}

// eager CG: the active flags are published to host-mapped memory and an
// event marks their arrival; the host waits on the event while later work
// is queued
static void post_flags(Handle *h) {
  if (!h->dpub) {
    (void)hipMemcpyAsync(h->hpub, h->act, sizeof(int) * h->ns, hipMemcpyDeviceToHost, h->stream);
    return;
  }
  DBS_LAUNCH(h, KC_MISC, k_publish, dim3((h->ns + 255) / 256), dim3(256), (const int *)h->act,
             h->dpub, h->ns);
  (void)hipEventRecord(h->flag_ev, h->stream);
}
static int wait_flags(Handle *h) {
  if (h->dpub) (void)hipEventSynchronize(h->flag_ev);
  else (void)hipStreamSynchronize(h->stream);
  int na = 0;
  for (int s = 0; s < h->ns; s++) na += h->hpub[s] != 0;
  return na;
}

// act[s] = va (va < 0: unchanged), want[s] = vw
static void set_flags(Handle *h, int va, int vw) {
  DBS_LAUNCH(h, KC_MISC, k_flags, dim3((h->ns + 255) / 256), dim3(256), va < 0 ? nullptr : h->act,
             va, h->want, vw, h->ns);
}

template <typename R>
static int pcg(Handle *h, const double *rAU, const double *b, double *x, int budget,
               int *iters, double *relres) {
  const bool flex = std::is_same<R, float>::value;
  const bool graph = budget > 0;
  float *rf = flex ? h->rf : nullptr;
  // the operator's FP32 coefficients and the coarse levels' operators; a
  // later corrector of the same step solves with the same rAU and keeps them
  const R *rAUr = flex ? (const R *)h->lv[0].bf : (const R *)rAU;
  if (!h->keep_hierarchy) {
    if (flex)
      DBS_LAUNCH(h, KC_MISC, k_cast<float>, flat_grid(h), dim3(FLAT_T), rAU, h->lv[0].bf);
    build_hierarchy<R>(h, rAUr);
  }
  // initial residual and norms of every sample
  set_flags(h, 1, 1);
  true_residual(h, rAU, b, x, rf, h->want);
  if (any_closed(h)) {
    // closed domain: norm of the projected (compatible) right-hand side
    arena_copy(h, b, h->z, 1);
    remove_mean(h, h->z, nullptr, nullptr);
    dot_self_closed(h, h->z, S_BB, nullptr);
  }
  finalize(h, fin_args(h, nullptr, 0, 0, 0, FIN_INIT, nullptr));
  const FL F = fl(h);
  const dim3 fg = flat_grid(h), ft(FLAT_T);
  const int *act = h->act;
  R *zold = flex ? (R *)h->zoldf : nullptr;  // written by the SpMV unless z rotates
  const Shape &ST = h->lv[0].st;
  OpB<double> o = opb<double>(h, 0, rAU);
  // FP32 fused sweeps: r.z and r.zold come from the last sweep of the
  // V-cycle, with the FP32 copy of r that the V-cycle reads (products and
  // sums in FP64); otherwise from a separate pass with r in FP64
  const bool fdot = flex && h->fused_sweep && h->mg_post >= 1;
  const Shape *SM = &h->lv[0].sm;
  // With fdot, z rotates through three FP32 buffers: each V-cycle works in
  // the two that do not hold the previous z, which stays as z_old (no copy).
  float *zb[3] = {h->lv[0].xf, h->zf2, h->zoldf};
  int zi = 2;  // buffer of the previous z
  auto precondition = [&](const R *zo) -> R * {
    if (flex) {
      float *w0 = zb[zi == 0 ? 1 : 0], *w1 = zb[zi == 2 ? 1 : 2];
      float *zn = vcycle<float, float>(h, (const float *)rAUr, (const float *)h->rf, w0, w1,
                                       fdot, (const float *)zo);
      if (fdot) zi = zn == zb[0] ? 0 : zn == zb[1] ? 1 : 2;
      return (R *)zn;
    }
    return (R *)vcycle<double, double>(h, (const double *)rAUr, (const double *)h->r, h->z,
                                       h->z2);
  };
  int nact = graph ? 1 : fetch_flags(h, nullptr);
  if (nact > 0) {
    R *zR = precondition(nullptr);
    if (fdot) {
      finalize(h, fin_args(h, SM, 0, S_RZ, 0, FIN_STORE, act));
    } else {
      DBS_LAUNCH(h, KC_DOT, k_dot2<R>, fg, ft, F, (const double *)h->r, (const R *)zR,
                 (const R *)nullptr, h->partials, (int)h->flat.nblk, act, 0);
      finalize(h, fin_args(h, &h->flat, 0, S_RZ, 0, FIN_STORE, act));
    }
    // the direction update p = z + beta p rides on the SpMV, which reads the
    // old direction from pc and writes the new one to pn
    double *pc = h->pv, *pn = h->pv2;
    const R *zc = zR;
    for (int it = 0;; it++) {
      if (graph && it >= budget) break;
      if (h->lv[0].flat)
        DBS_LAUNCH(h, KC_SPMV, (k_stencil2d<2, R>), dim3(ST.nblk), blk2(), o, sh(h, ST),
                   (const double *)pc, (const double *)nullptr, h->q, (float *)nullptr,
                   h->partials, 0, act, zc, pn, fdot ? (R *)nullptr : zold,
                   (const double *)h->scal, it == 0 ? 1 : 0);
      else
        DBS_LAUNCH(h, KC_SPMV, (k_stencil25<2, R>), dim3(ST.nblk), blk2(), o, sh(h, ST),
                   (const double *)pc, (const double *)nullptr, h->q, (float *)nullptr,
                   h->partials, 0, act, zc, pn, fdot ? (R *)nullptr : zold,
                   (const double *)h->scal, it == 0 ? 1 : 0);
      std::swap(pc, pn);
      finalize(h, fin_args(h, &ST, 0, S_PQ, 0, FIN_ALPHA, act));
      DBS_LAUNCH(h, KC_AXPY, k_axpy_dot, fg, ft, F, (const double *)h->scal,
                 (const double *)pc, (const double *)h->q, x, h->r, rf, h->partials, act);
      finalize(h, fin_args(h, &h->flat, 0, S_RR, 0, FIN_RR, act));
      // the true residual of the samples that ask for it decides convergence
      // (and replaces the recursive one); launched every iteration, its
      // blocks skip the other samples
      true_residual(h, rAU, b, x, rf, h->want, FIN_CHECK);
      // Eager: the flags of this iteration travel to the host while the
      // V-cycle is queued behind them, so the device does not drain; when
      // no sample is left active, that V-cycle was skipped block by block.
      if (!graph) post_flags(h);
      R *zn = precondition(fdot ? zc : zold);
      if (fdot) {
        finalize(h, fin_args(h, SM, 1, S_RZNEW, S_RZOLD, FIN_BETA_FLEX, act));
      } else if (flex) {
        DBS_LAUNCH(h, KC_DOT, k_dot2<R>, fg, ft, F, (const double *)h->r, (const R *)zn,
                   (const R *)zold, h->partials, (int)h->flat.nblk, act, 0);
        finalize(h, fin_args(h, &h->flat, 1, S_RZNEW, S_RZOLD, FIN_BETA_FLEX, act));
      } else {
        DBS_LAUNCH(h, KC_DOT, k_dot2<R>, fg, ft, F, (const double *)h->r, (const R *)zn,
                   (const R *)nullptr, h->partials, (int)h->flat.nblk, act, 0);
        finalize(h, fin_args(h, &h->flat, 0, S_RZNEW, 0, FIN_BETA, act));
      }
      zc = zn;
      if (!graph && wait_flags(h) == 0) break;
    }
  }
  if (any_closed(h)) remove_mean(h, x, nullptr, nullptr);
  // final true residual (act is kept: a sample still active here did not
  // converge within the budget); a sample that converged holds it already
  DBS_LAUNCH(h, KC_MISC, k_want_final, dim3((h->ns + 255) / 256), dim3(256),
             (const double *)h->scal, (const int *)h->act, (const Rng *)h->rng, h->want, h->ns);
  true_residual(h, rAU, b, x, nullptr, h->want);
  finalize(h, fin_args(h, nullptr, 0, 0, 0, FIN_RRFIN, nullptr));
  if (graph) return DBS_OK;
  std::vector<int> conv(h->ns);
  pressure_results(h, iters, relres, conv.data());
  for (int s = 0; s < h->ns; s++)
    if (!conv[s]) return DBS_ENOCONV;
  return DBS_OK;
}

void pressure_results(Handle *h, int *iters, double *relres, int *converged) {
  const int ns = h->ns;
  if (h->dpub) {
    host_copy(h, h->scal, h->dscal_h, (size_t)NSC * ns);
    DBS_LAUNCH(h, KC_MISC, k_publish, dim3((ns + 255) / 256), dim3(256), (const int *)h->act,
               h->dpub, ns);
  } else {
    (void)hipMemcpyAsync(h->hscal, h->scal, sizeof(double) * NSC * ns, hipMemcpyDeviceToHost,
                         h->stream);
    (void)hipMemcpyAsync(h->hpub, h->act, sizeof(int) * ns, hipMemcpyDeviceToHost, h->stream);
  }
  (void)hipStreamSynchronize(h->stream);
  for (int s = 0; s < ns; s++) {
    const double *S = h->hscal + (size_t)s * NSC;
    if (iters) iters[s] = (int)S[S_ITS];
    if (relres) relres[s] = S[S_NRM2] > 0.0 ? sqrt(S[S_RRFIN] / S[S_NRM2]) : 0.0;
    if (converged) converged[s] = S[S_NOCONV] == 0.0 && h->hpub[s] == 0;
  }
}

int pressure_solve(Handle *h, const double *rAU, const double *b, double *x, int budget,
                   int *iters, double *relres) {
  if (h->ctl.precision == DBS_MIXED) return pcg<float>(h, rAU, b, x, budget, iters, relres);
  return pcg<double>(h, rAU, b, x, budget, iters, relres);
}

}  // namespace dbs

namespace dbs {

// per-sample results of the last solve, stored for corrector c (graph mode:
// read back by the host after the replayed step, or as soon as the last
// corrector's records are ready).  The ready tag o[5] = 1 is written after
// the other fields are visible to the host (the host clears it to -1 before
// each replay).
__global__ void k_record(const double *__restrict__ scal, const int *__restrict__ act, int ns,
                         double *__restrict__ rec, int c) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= ns) return;
  const double *S = scal + (size_t)s * NSC;
  double *o = rec + ((size_t)s * 16 + c) * NREC;
  o[0] = S[S_ITS];
  o[1] = S[S_NRM2] > 0.0 ? sqrt(S[S_RRFIN] / S[S_NRM2]) : 0.0;
  o[2] = (S[S_NOCONV] == 0.0 && act[s] == 0) ? 1.0 : 0.0;
  o[3] = sqrt(S[S_NRM2]);
  o[4] = S[S_NRM2] > 0.0 ? sqrt(S[S_RR0] / S[S_NRM2]) : 0.0;
  __threadfence_system();
  o[5] = 1.0;
}

__global__ void __launch_bounds__(FLAT_T) k_copyn(const double *__restrict__ in,
                                                  double *__restrict__ out, size_t n) {
  const size_t c = (size_t)blockIdx.x * FLAT_T + threadIdx.x;
  if (c < n) out[c] = in[c];
}

void pressure_norms(Handle *h, double *bnorm, double *res0) {
  // valid after pressure_results (which copies the scalars to the host)
  for (int s = 0; s < h->ns; s++) {
    const double *S = h->hscal + (size_t)s * NSC;
    if (bnorm) bnorm[s] = sqrt(S[S_NRM2]);
    if (res0) res0[s] = S[S_NRM2] > 0.0 ? sqrt(S[S_RR0] / S[S_NRM2]) : 0.0;
  }
}

void pressure_record(Handle *h, double *rec, int c) {
  DBS_LAUNCH(h, KC_MISC, k_record, dim3((h->ns + 255) / 256), dim3(256),
             (const double *)h->scal, (const int *)h->act, h->ns, rec, c);
}

void host_copy(Handle *h, const double *src, double *dst_mapped, size_t n) {
  if (!n) return;
  DBS_LAUNCH(h, KC_MISC, k_copyn, dim3((unsigned)((n + FLAT_T - 1) / FLAT_T)), dim3(FLAT_T), src,
             dst_mapped, n);
}

void copy_n(Handle *h, const double *src, double *dst, size_t n) {
  if (!n) return;
  DBS_LAUNCH(h, KC_MISC, k_copyn, dim3((unsigned)((n + FLAT_T - 1) / FLAT_T)), dim3(FLAT_T), src,
             dst, n);
}

}  // namespace dbs
