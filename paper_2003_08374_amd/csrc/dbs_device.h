// Internal device-side definitions shared by the HIP translation units.
//
// Layout: structure-of-arrays FP64 fields, x fastest (c = i + nx*(j + ny*k)).
// Face arrays keep (n+1) entries along their own axis; a face value is
// oriented along +axis.  Kernels run one thread per cell on 64 x 4 blocks
// (one wavefront per 64-cell x-row segment, coalesced 512-byte loads).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

namespace dbs {

enum { BC_WALL = 0, BC_INLET = 1, BC_OUTLET = 2, BC_EMPTY = 3, BC_WAVE = 4 };
enum { M_BROOKS_COREY = 0, M_VAN_GENUCHTEN = 1 };

constexpr int BX = 64;
constexpr int BY = 4;
constexpr int NTHREADS = BX * BY;

struct Phys {
  double rho_l, rho_g, mu_l, mu_g;
  double g[3];
  double c_alpha;
  int kr_model;
  double kr_m, inv_kr_m, s_lirr, inv_span_kr;
  int pc_model;
  double pc0, pc_exp, a_pcirr, inv_span_pc, eps_pc;
  double sigma;  // interfacial tension of the clear-fluid CSF force (0: off)
  int ca_on;     // a contact angle is imposed on clear/porous faces
  double cos_ca; // its cosine
  double cot_ca; // and cotangent
};

// One sample (one mesh) of a batch.  Cell and face indices are absolute in
// the batch arenas: a sample's cells start at c0, its x|y|z face blocks at
// fo[0..2]; vector fields are component-major over the whole cell arena
// (component stride vs).
struct Geom {
  int n[3];
  int nc;           // cells of this sample
  int c0;           // first cell of this sample in the cell arena
  int vs;           // component stride of vector fields (cells in the arena)
  int fo[3];        // first x|y|z face of this sample in the face arena
  int nf;           // faces of this sample
  double h[3], ih[3], area[3], V, iV;
  double dt;
  int bck[6];
  double bcU[6][3];
  double bca[6];
  double bcp[6];
  int has_outlet;
  double dN;        // interface-normal regularisation 1e-8 / V^(1/3)
  // wave inlet on x face b: amplitude, angular frequency, wavenumber and
  // still-water depth of a linear (Airy) wave
  double wA[2], wom[2], wk[2], wd[2];
  double t;         // time of the boundary values: the end of the current step
  double *wprof;    // wave inlet values at time t: [face 0|1][row j][u, v, alpha]
};

// ---------------------------------------------------------------- indexing

__device__ __forceinline__ int cidx(const Geom &G, int i, int j, int k) {
  return G.c0 + i + G.n[0] * (j + G.n[1] * k);
}

// face on the minus side of cell coordinate (i,j,k) along axis a (the
// coordinate along a may equal n[a]: the last face)
__device__ __forceinline__ int fidx(const Geom &G, int a, int i, int j, int k) {
  if (a == 0) return G.fo[0] + i + (G.n[0] + 1) * (j + G.n[1] * k);
  if (a == 1) return G.fo[1] + i + G.n[0] * (j + (G.n[1] + 1) * k);
  return G.fo[2] + i + G.n[0] * (j + G.n[1] * k);
}

__device__ __forceinline__ int stride_of(const Geom &G, int a) {
  return a == 0 ? 1 : (a == 1 ? G.n[0] : G.n[0] * G.n[1]);
}

struct Cell {
  int i, j, k, c;
  int co[3];
};

// Launches cover a whole batch: the blocks of all samples are concatenated
// and bp[s] is the first block of sample s (bp has ns + 1 entries).  Global
// block numbers are first renumbered so that each of the 8 XCDs receives a
// contiguous run (a slab of planes of one sample, or whole small samples):
// the y and z neighbours of a tile then sit in the same L2.
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  const int full = nb & ~7;
  return b < full ? (b & 7) * (full >> 3) + (b >> 3) : b;
}

// the sample owning global block b: the last s with bp[s] <= b
__device__ __forceinline__ int find_seg(const int *__restrict__ bp, int ns, int b) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (bp[mid] <= b) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// per-cell launch over a batch: sample table and block prefix
struct Segs {
  const Geom *g;
  const int *bp;
  int ns;
};

// Per-cell kernels run one cell per thread on 64x4 blocks; blocks of one
// sample walk its x-row segments, rows and planes.  (Walking several planes
// per thread was tried: the heavy per-cell kernels then hold more registers
// and lose occupancy.)  A sample whose rows would leave more than a ninth
// of those lanes idle (x rows of a few dozen cells, as in a batch of small
// samples) is instead walked in cell order, 256 consecutive cells a block.
__host__ __device__ inline bool cell_linear(const Geom &G) {
  const long long tiled =
      (long long)((G.n[0] + BX - 1) / BX * BX) * ((G.n[1] + BY - 1) / BY * BY);
  return 8 * tiled > 9 * (long long)G.n[0] * G.n[1];
}

__host__ __device__ inline int cell_blocks(const Geom &G) {
  if (cell_linear(G)) return (G.nc + BX * BY - 1) / (BX * BY);
  return ((G.n[0] + BX - 1) / BX) * ((G.n[1] + BY - 1) / BY) * G.n[2];
}

// Blocks of a sample are ordered in bands of CELL_BAND block rows: a band
// runs through all planes before the next band starts.  The blocks in
// flight on one XCD then cover a few consecutive planes of one band, so the
// z neighbours of a cell (read again one and two planes later) are still in
// that XCD's L2; plane-by-plane order over the whole cross-section evicts
// them first when a kernel touches many arrays.
constexpr int CELL_BAND = 4;

__device__ __forceinline__ bool cell_of_thread(const Geom &G, int lb, Cell &P) {
  if (cell_linear(G)) {
    const unsigned n0 = (unsigned)G.n[0], n01 = n0 * (unsigned)G.n[1];
    const unsigned e = (unsigned)lb * (BX * BY) + threadIdx.x + BX * threadIdx.y;
    const unsigned k = e / n01, r = e - k * n01, j = r / n0;
    P.i = (int)(r - j * n0);
    P.j = (int)j;
    P.k = (int)k;
    P.co[0] = P.i; P.co[1] = P.j; P.co[2] = P.k;
    P.c = G.c0 + (int)e;
    return e < (unsigned)G.nc;
  }
  const int nbx = (G.n[0] + BX - 1) / BX, nby = (G.n[1] + BY - 1) / BY, n2 = G.n[2];
  const int full = nby / CELL_BAND;               // bands of CELL_BAND block rows
  const int full_blocks = full * nbx * CELL_BAND * n2;
  int band, rows, r;
  if (lb < full_blocks) {
    band = lb / (nbx * CELL_BAND * n2);
    r = lb - band * (nbx * CELL_BAND * n2);
    rows = CELL_BAND;
  } else {
    band = full;
    r = lb - full_blocks;
    rows = nby - full * CELL_BAND;
  }
  const int per_plane = nbx * rows;
  P.k = r / per_plane;
  r -= P.k * per_plane;
  const int byl = r / nbx;
  P.i = (r - byl * nbx) * BX + threadIdx.x;
  P.j = (band * CELL_BAND + byl) * BY + threadIdx.y;
  P.co[0] = P.i; P.co[1] = P.j; P.co[2] = P.k;
  P.c = cidx(G, P.i, P.j, P.k);
  return P.i < G.n[0] && P.j < G.n[1];
}

// Body executed for this thread's cell; G names the cell's sample and
// cell_gb the block's global number in the concatenated order.
#define FOR_CELLS(S, G, P)                                         \
  const int cell_gb = xcd_remap(blockIdx.x, gridDim.x);            \
  const int cell_sg = find_seg((S).bp, (S).ns, cell_gb);           \
  const Geom &G = (S).g[cell_sg];                                  \
  Cell P;                                                          \
  if (cell_of_thread(G, cell_gb - (S).bp[cell_sg], P))

// FOR_CELLS for a launch over all samples (only < 0) or over the blocks of
// sample `only` alone, which start at block `base` of the shape
#define FOR_CELLS_ONE(S, G, P, only, base)                                      \
  const int cell_gb = (only) >= 0 ? (base) + (int)blockIdx.x                    \
                                  : xcd_remap(blockIdx.x, gridDim.x);           \
  const int cell_sg = (only) >= 0 ? (only) : find_seg((S).bp, (S).ns, cell_gb); \
  const Geom &G = (S).g[cell_sg];                                               \
  Cell P;                                                                       \
  if (cell_of_thread(G, cell_gb - (S).bp[cell_sg], P))

// face index of side s (0 = minus, 1 = plus) of cell P along axis a
__device__ __forceinline__ int face_of(const Geom &G, const Cell &P, int a, int s) {
  int ii = P.i + (a == 0 ? s : 0), jj = P.j + (a == 1 ? s : 0), kk = P.k + (a == 2 ? s : 0);
  return fidx(G, a, ii, jj, kk);
}

// is side s of cell P along axis a a domain boundary face?
__device__ __forceinline__ bool on_boundary(const Geom &G, const Cell &P, int a, int s) {
  return s == 0 ? P.co[a] == 0 : P.co[a] == G.n[a] - 1;
}

__device__ __forceinline__ double gdotx_cell(const Geom &G, const Phys &Ph, const Cell &P) {
  return Ph.g[0] * (P.i + 0.5) * G.h[0] + Ph.g[1] * (P.j + 0.5) * G.h[1] +
         Ph.g[2] * (P.k + 0.5) * G.h[2];
}

// g . x at the centre of side s of cell P along axis a
__device__ __forceinline__ double gdotx_face(const Geom &G, const Phys &Ph, const Cell &P, int a,
                                             int s) {
  double x[3] = {(P.i + 0.5) * G.h[0], (P.j + 0.5) * G.h[1], (P.k + 0.5) * G.h[2]};
  x[a] = (P.co[a] + s) * G.h[a];
  return Ph.g[0] * x[0] + Ph.g[1] * x[1] + Ph.g[2] * x[2];
}

// ---------------------------------------------------------------- physics

__device__ __forceinline__ double rho_of(const Phys &Ph, double a) {
  return a * Ph.rho_l + (1.0 - a) * Ph.rho_g;
}
__device__ __forceinline__ double mu_of(const Phys &Ph, double a) {
  return a * Ph.mu_l + (1.0 - a) * Ph.mu_g;
}

__device__ __forceinline__ double clamp01(double x, double lo, double hi) {
  return fmin(fmax(x, lo), hi);
}

// x^e for x >= 0.  The exponents of the usual closures (1, 2, 3, 1/2,
// -1/2) are taken by multiplication or the square root, whose results are
// within an ulp or two of the correctly rounded power; any other exponent
// goes to pow.  The exponent is the same for the whole launch, so the
// choice does not diverge.
__device__ __forceinline__ double powc(double x, double e) {
  if (e == 2.0) return x * x;
  if (e == 1.0) return x;
  if (e == 0.5) return sqrt(x);
  if (e == 3.0) return x * x * x;
  if (e == -0.5) return 1.0 / sqrt(x);
  return pow(x, e);
}

// App. A.1 relative permeabilities divided by the viscosities (mobility per
// unit permeability) and App. A.2 capillary pressure of one cell.
__device__ inline void closures(const Phys &Ph, double a, double &ml, double &mg, double &pc) {
  double ae = clamp01((a - Ph.s_lirr) * Ph.inv_span_kr, 0.0, 1.0);
  double krl, krg;
  if (Ph.kr_model == M_BROOKS_COREY) {
    krl = powc(ae, Ph.kr_m);
    krg = powc(1.0 - ae, Ph.kr_m);
  } else {
    double t = powc(ae, Ph.inv_kr_m);
    double u = 1.0 - powc(1.0 - t, Ph.kr_m);
    krl = sqrt(ae) * u * u;
    krg = sqrt(1.0 - ae) * powc(1.0 - t, 2.0 * Ph.kr_m);
  }
  ml = krl / Ph.mu_l;
  mg = krg / Ph.mu_g;
  double s = (a - Ph.a_pcirr) * Ph.inv_span_pc;
  if (Ph.pc_model == M_BROOKS_COREY) {
    s = clamp01(s, Ph.eps_pc, 1.0);
    pc = Ph.pc0 * powc(s, -Ph.pc_exp);
  } else {
    s = clamp01(s, Ph.eps_pc, 1.0 - Ph.eps_pc);
    pc = Ph.pc0 * powc(powc(s, -1.0 / Ph.pc_exp) - 1.0, 1.0 - Ph.pc_exp);
  }
}

__device__ __forceinline__ bool is_inlet(int kind) { return kind == BC_INLET || kind == BC_WAVE; }

// Velocity component comp and alpha of inlet face b in row j.  Wave inlet
// values are tabulated once per step (wave_profile), so the heavy kernels
// only read them.
__device__ __forceinline__ double inlet_u(const Geom &G, int b, int j, int comp) {
  if (G.bck[b] != BC_WAVE) return G.bcU[b][comp];
  if (comp == 2) return 0.0;  // the wave moves in the x-y plane
  return G.wprof[((size_t)b * G.n[1] + j) * 3 + comp];
}

__device__ __forceinline__ double inlet_alpha(const Geom &G, int b, int j) {
  if (G.bck[b] != BC_WAVE) return G.bca[b];
  return G.wprof[((size_t)b * G.n[1] + j) * 3 + 2];
}

// boundary alpha at a face in row j: inlet value; wave or outlet value on
// inflow; else the cell value
__device__ __forceinline__ double bnd_alpha(const Geom &G, int b, int j, double a_cell,
                                            double Fb) {
  const int kind = G.bck[b];
  const double so = (b & 1) ? 1.0 : -1.0;
  if (kind == BC_INLET) return G.bca[b];
  if (kind == BC_WAVE && so * Fb < 0.0) return inlet_alpha(G, b, j);
  if (kind == BC_OUTLET && so * Fb < 0.0) return G.bca[b];
  return a_cell;
}

// ---------------------------------------------------------- reductions

__device__ __forceinline__ double wave_sum(double v) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
__device__ __forceinline__ double wave_min(double v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// Thread t of a 1024-thread block adds part[q * nb + i] for i = lo + t,
// lo + t + 1024, ... below hi into r[q], in that order, with eight loads in
// flight (the sums equal those of the plain strided loop bit for bit).
template <int NQ>
__device__ __forceinline__ void strided_sums(const double *__restrict__ part, size_t nb, int lo,
                                             int hi, double *r) {
  for (int i = lo + (int)threadIdx.x; i < hi; i += 8 * 1024) {
    double v[NQ][8];
#pragma unroll
    for (int u = 0; u < 8; u++) {
      const int j = i + u * 1024;
#pragma unroll
      for (int q = 0; q < NQ; q++) v[q][u] = j < hi ? part[(size_t)q * nb + j] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 8; u++)
#pragma unroll
      for (int q = 0; q < NQ; q++)
        if (i + u * 1024 < hi) r[q] += v[q][u];
  }
}

// block-wide sum over NTHREADS threads (4 wavefronts); result valid in thread 0
__device__ __forceinline__ double block_sum(double v, double *lds) {
  v = wave_sum(v);
  int t = threadIdx.x + BX * threadIdx.y;
  int w = t >> 6;
  if ((t & 63) == 0) lds[w] = v;
  __syncthreads();
  double s = 0.0;
  if (t == 0)
    for (int q = 0; q < NTHREADS / 64; q++) s += lds[q];
  return s;
}

}  // namespace dbs
