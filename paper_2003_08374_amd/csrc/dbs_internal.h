// Host-side state of a dbs_handle and the launchers each translation unit
// provides.  Not part of the public ABI.
//
// A handle holds a batch of ns independent samples (ns = 1 for dbs_create).
// Every field lives in one arena per kind: cell fields hold the samples one
// after the other (each padded to a multiple of FLAT_CELLS cells, padding
// kept at zero), face fields likewise without padding, and each multigrid
// level has its own arena.  Every kernel is one launch over all samples.
#pragma once
#include <map>
#include <string>
#include <vector>

#include "../../include/dbs.h"
#include "dbs_device.h"

namespace dbs {

// kernel classes for event timing (order = dbs_kernel_name)
enum KClass {
  KC_ALPHA_FACE = 0, KC_ALPHA_BOUNDS, KC_ALPHA_LIMIT, KC_ALPHA_UPDATE,
  KC_MOM_ASSEMBLE, KC_MOM_OFFDIAG, KC_PHIHBYA, KC_CORRECT,
  KC_SPMV, KC_AXPY, KC_DOT, KC_FINALIZE,
  KC_SMOOTH0, KC_RESTRICT0, KC_PROLONG0,
  KC_SMOOTHC, KC_RESTRICTC, KC_PROLONGC, KC_COARSE, KC_BUILD_COARSE,
  KC_STATS, KC_MISC, KC_SMOOTH0_ZERO, KC_RESIDUAL, KC_SMOOTH0_DOT, KC_CURV, KC_COUNT
};

constexpr int FLAT_T = 256;               // threads of a vector-kernel block
constexpr int FLAT_CELLS = 4 * FLAT_T;    // cells of a vector-kernel block
constexpr int NSC = 16;                   // device scalars per sample
constexpr int NSTAT = 6;                  // cell statistics per sample
constexpr int NREC = 6;                   // graph-mode solve record per corrector (last: ready tag)
constexpr int NMSC = 4;                   // predictor record per sample

// first cell, cell count and closed-domain flag of a sample's fine cells
struct Rng {
  int c0, nc, closed, pad;
};

// one sample on one multigrid level (device table entry)
struct LvS {
  int n0, n1, n2;     // cells per axis (0: the sample has no such level)
  int c0;             // first cell in the level's arena
  int cn0, cn1, cn2;  // the sample's next coarser level (0: none)
  int cc0;            // its first cell in the coarser arena
  int outlet;         // the sample has an outlet (Dirichlet) face
  int pad;
  double c[3];        // area / h per axis
  double ob[6];       // outlet diagonal factor per domain face (2 c or 0)
};

// a launch over (a subset of) the batch: block prefix per sample
struct Shape {
  int *bp = nullptr;       // device, ns + 1 entries
  std::vector<int> hbp;
  int nblk = 0;
  int kz = 1;
};

struct Level {
  long long nc = 0;        // cells in this level's arena
  std::vector<LvS> hs;     // per sample
  LvS *ds = nullptr;
  // coarse-level operator (level >= 1): coefficient of the +x/+y/+z face of
  // each cell, Dirichlet diagonal part and full diagonal
  double *Tx = nullptr, *Ty = nullptr, *Tz = nullptr, *Db = nullptr, *D = nullptr;
  float *Txf = nullptr, *Tyf = nullptr, *Tzf = nullptr, *Dbf = nullptr, *Df = nullptr;
  double *x = nullptr, *b = nullptr;  // correction and right-hand side
  float *xf = nullptr, *bf = nullptr;
  float *xf2 = nullptr;  // second FP32 correction buffer (fused coarse sweeps)
  double *x2 = nullptr;  // second FP64 correction buffer (small-tile coarse sweeps)
  // launch shapes: fine level
  Shape st, sm, rs;
  // coarse levels: every sample holding the level; samples cycled on it by
  // grid kernels (pairs and single cells); samples restricted into it
  Shape one_all, pair_cyc, one_cyc, one_rc;
  Shape sw;  // coarse levels: 2.5-D tiles of the cycled samples (fused sweeps)
  Shape cb;  // coarse levels: CB^3 tiles of the cycled samples (block-local smoothing)
  Shape cs;  // coarse levels: 8 x 8 x 4 tiles of the cycled samples (small-tile sweeps)
  long long cyc_cells = 0;  // cells of the cycled samples on this level
  long long sw_lanes = 0;   // cells the 2.5-D tiles of `sw` span (idle lanes included)
  int sw_ok = 0;  // every cycled sample is deep enough in z for fused sweeps
  int cs2d = 0;   // every cycled sample is one cell deep: small tiles are 16 x 16 x 1
  int flat = 0;   // fine level: every sample is one cell deep (the 2D kernels)
};

struct Timer {
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  std::vector<int> cls;
  size_t used = 0;
  bool skip = false;  // the current launch is untimed (no event to be had)
  bool ok = true;     // every record since the last collection succeeded
};

// one captured step (graph mode), keyed by the buffer roles it was captured with
// a captured step in two parts, launched back to back: the small first
// part (saturation stage and momentum predictor) starts on the device while
// the host is still submitting the second (the correctors' solves)
struct StepGraphs {
  hipGraphExec_t front = nullptr, back = nullptr;
};

struct GraphKey {
  const void *alpha, *U, *F;
  bool operator<(const GraphKey &o) const {
    if (alpha != o.alpha) return alpha < o.alpha;
    if (U != o.U) return U < o.U;
    return F < o.F;
  }
};

// Coefficients of the first corrector's initial guess (k_extrap), in the
// difference form t + sum_k c_k (t - x_k) of Lagrange extrapolation in time
// from p_rgh at the ends of this step (t) and the steps before (x_1 = a,
// x_2 = b, x_3 = q): order 1 r; order 2 q1, q2; order 3 k1, k2, k3.  The
// backtests predict t from a and the steps before in the same forms: b1;
// c1, c2; m1, m2, m3.
struct GuessArgs {
  double r, q1, q2, b1, c1, c2, k1, k2, k3, m1, m2, m3;
  int use;  // highest order the stored steps allow (0 to 3)
  int usec; // highest kind of change prediction they allow (0 to 3)
  int nbt;  // orders whose backtest the stored steps allow (0 to 4)
  int nd;   // later correctors' changes recorded (0 or n_corr - 1)
};

struct Handle {
  int ns = 1;
  std::vector<Geom> hG;   // per sample, absolute arena offsets
  Geom *dG = nullptr;
  long long NC = 0, NF = 0;  // cell arena (padded) and face arena sizes
  Phys P;
  dbs_controls ctl;
  std::string err;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;

  Shape cell;           // per-cell kernels (64 x 4 blocks)
  Segs seg;             // device view of cell
  dim3 cgrid;
  Shape flat;           // vector kernels (FLAT_CELLS cells per block)
  Rng *rng = nullptr;   // per sample
  std::vector<Rng> hrng;

  // static fields
  double *phi = nullptr, *kinv = nullptr;
  // state (alpha is double-buffered: alpha holds n+1 after the transport;
  // with sub-cycles a third buffer keeps alpha^n while the cycles alternate)
  double *alpha = nullptr, *alpha_old = nullptr, *alpha3 = nullptr;
  // U: the current velocity; U2, U3: the predictor's sweep buffers (the
  // step leaves U^n in U3).  3 x NC each
  double *U = nullptr, *U2 = nullptr, *U3 = nullptr;
  double *prgh = nullptr, *p = nullptr;
  // p_rgh at the ends of the previous four steps (pprev .. pprev4),
  // for the extrapolated initial guess of the first corrector's solve; hist
  // of them are valid (0 to 4: steps run since the state was last set), with
  // time steps dt_prev .. dt_prev4.
  double *pprev = nullptr, *pprev2 = nullptr, *pprev3 = nullptr, *pprev4 = nullptr;
  // the solution of the corrector before (p1) and, per later corrector, the
  // changes its solve made in the previous three steps (dcorr: n_corr - 1
  // slices of the last changes, then of the ones before, then of the ones
  // before those, NC each)
  double *p1 = nullptr, *dcorr = nullptr;
  // per sample: the extrapolation order of the next first guess (gord) and,
  // per later corrector, the kind of its change prediction (gchg, ns x
  // (n_corr - 1): 0 none, 1 the last change, 2 linear in the last two, 3
  // quadratic in the last three); set
  // on the device after every step
  int *gord = nullptr, *gchg = nullptr;
  int hist = 0;
  double dt_prev = 0.0, dt_prev2 = 0.0, dt_prev3 = 0.0, dt_prev4 = 0.0;
  // the first guess's coefficients as the last step used them and as the
  // captured steps use them
  GuessArgs guess_used{}, graph_guess{0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, -1, -1, -1, -1};
  double *F = nullptr;                 // faces
  double *F2 = nullptr;                // the correctors' fluxes (swapped with F per step)
  // closures of the current alpha: k_rl/mu_l, k_rg/mu_g, p_c (0 in clear cells)
  double *ml = nullptr, *mg = nullptr, *pc = nullptr;
  double *cf = nullptr;  // f_l - alpha in porous cells, 0 in clear cells
  // transport work arrays
  double *A = nullptr, *lam = nullptr, *rhoPhi = nullptr;  // faces
  double *Qp = nullptr, *Qm = nullptr, *Pin = nullptr, *Pout = nullptr, *Rp = nullptr,
         *Rm = nullptr;
  // momentum / pressure work arrays
  double *rAU = nullptr, *Sh = nullptr, *B = nullptr, *HbyA = nullptr;  // Sh,B,HbyA 3 x NC
  double *AN = nullptr;  // momentum neighbour coefficients of the step, 6 x NC
  double *FB = nullptr;  // body force F_c - (g.x_f) dn(rho) of each face, for the step
  double *SK = nullptr;  // sigma kappa / phi (clear cells), 0 (porous); only when sigma > 0
  double *phiH = nullptr;  // faces
  double *rhs = nullptr;
  // PCG vectors
  double *r = nullptr, *z = nullptr, *pv = nullptr, *q = nullptr;
  double *pv2 = nullptr;  // CG directions alternate between pv and pv2
  float *rf = nullptr;     // FP32 residual (mixed precision)
  float *zoldf = nullptr;  // third FP32 z buffer (z rotation), or z_old with half sweeps
  float *zf2 = nullptr;    // second fine correction buffer (FP32 V-cycle)
  double *z2 = nullptr;    // second fine correction buffer (FP64 V-cycle)
  double *partials = nullptr;  // per-block partial sums
  size_t npartials = 0;
  double *scal = nullptr;      // NSC device scalars per sample
  double *hscal = nullptr, *dscal_h = nullptr;  // host-mapped mirror (host, device view)
  int *act = nullptr, *want = nullptr;  // per-sample CG flags
  hipEvent_t flag_ev = nullptr;  // eager CG: the flags of an iteration have landed
  // pinned host memory written by kernels (mapped): the active flags of the
  // eager CG iteration, and the predictor's flags (two slots) and records
  int *hpub = nullptr, *dpub = nullptr;
  // momentum predictor solve: per sample an iterate flag and a record
  // {||B||^2, sweeps, relative residual, converged}; host-mapped mirrors
  int *mact = nullptr;
  double *msc = nullptr, *hmsc = nullptr, *dmsc = nullptr;
  int *hmflag = nullptr, *dmflag = nullptr;
  hipEvent_t mom_ev[2] = {nullptr, nullptr};
  int mom_budget = 0;          // graph mode: predictor sweeps in a captured step
  int mom_last = 0;            // sweeps launched by the last predictor solve
  // per-sample statistics (NSTAT each): host-mapped, written by the kernel
  double *hsstat = nullptr, *dsstat_h = nullptr;

  std::vector<Level> lv;
  std::vector<int> nlev;     // levels per sample
  std::vector<int> bottom;   // per sample: first level cycled by one work-group
  int maxbottom = 0;         // largest bottom level over the samples
  void *btab = nullptr;      // device table of bottom descriptors
  int nbt = 0;               // samples with a bottom (>= 2 levels)
  int mg_pre = 2, mg_post = 2, coarse_sweeps = 16;
  int mgc = 3;  // sweeps per coarse level (pre = post), bottom levels included
  // tuning knobs (autotuner): fine tile depth (0 = heuristic), bottom shift,
  // fused full sweeps on the fine level (else two half-sweep launches)
  int kz_fine = 0, bottom_shift = 0, fused_sweep = 1;
  int kz_coarse = 0;  // planes per coarse-level tile or thread column (0 = heuristic)
  // FP32 V-cycle: the sweeps of a grid-cycled coarse level in one launch of
  // block-local smoothing (Jacobi between CB^3 tiles) instead of global
  // red-black sweeps
  int coarse_block = 0;
  // the coming solve uses the rAU of the previous one (a later corrector of
  // the same step): the FP32 coefficients and coarse operators are kept
  bool keep_hierarchy = false;

  std::vector<dbs_stats> st;  // per sample
  double tnow = 0.0;          // time reached by the samples
  int has_wave = 0;           // some sample has a wave inlet

  // graph mode
  int graph_mode = 0;
  int graph_budget[16] = {0};  // PCG iterations per corrector in a captured step
  int used_max[16] = {0};      // largest count per corrector over the slack run
  int slack_steps = 0;         // replays in a row that left a slack of two or more
  std::map<GraphKey, StepGraphs> graphs;
  double *snap = nullptr;      // p_rgh saved for a step redone eagerly (the other
                               // fields keep their step-start buffers)
  // per-sample solve records (ns x 16 x NREC), host-mapped (host, device view)
  double *hrec = nullptr, *rec = nullptr;

  // profiling
  unsigned long long prof_mask = 0;
  Timer tm;
  long long k_launches[KC_COUNT] = {0};
  double k_ms[KC_COUNT] = {0};
  std::vector<void *> allocs;   // device allocations
  // Scratch-arena mode (the no-alloc pressure solve): device arrays are
  // carved from a caller-provided zeroed region instead of hipMalloc, and
  // flags and scalars travel by plain copies into these host arrays.
  unsigned char *arena = nullptr;
  size_t arena_cap = 0, arena_used = 0;
  double hscal_own[NSC] = {0};
  int hpub_own[2] = {0, 0};
  std::vector<void *> hallocs;  // host-mapped allocations
};

// bytes from the scratch arena (256-byte aligned); DBS_ENOMEM when it is full
inline void *arena_take(Handle *h, size_t bytes, int &rc) {
  if (rc) return nullptr;
  const size_t off = (h->arena_used + 255) & ~(size_t)255;
  if (off + bytes > h->arena_cap) {
    rc = DBS_ENOMEM;
    h->arena_used = off + bytes;  // the size that was asked for, for the message
    return nullptr;
  }
  h->arena_used = off + bytes;
  return h->arena + off;
}

// launch-time event bracketing
void prof_begin(Handle *h, int cls);
void prof_end(Handle *h, int cls);
void prof_collect(Handle *h);

#define DBS_LAUNCH(h, cls, kernel, grid, block, ...)                         \
  do {                                                                        \
    bool _p = ((h)->prof_mask >> (cls)) & 1ull;                               \
    if (_p) prof_begin((h), (cls));                                          \
    hipLaunchKernelGGL(kernel, grid, block, 0, (h)->stream, __VA_ARGS__);     \
    if (_p) prof_end((h), (cls));                                            \
  } while (0)

// k_alpha.hip
// the saturation stage (n_alpha_sub sub-cycles); aphi (faces, may be NULL)
// receives the mean limited flux
void alpha_stage(Handle *h, double *aphi = nullptr);
// the buffer roles the stage leaves: alpha^{n+1} current, alpha^n kept
void alpha_roles(Handle *h);
// R+- of the last limiter iteration of the last transport cycle
void alpha_final_R(Handle *h, double **Rp, double **Rm);
void update_closures(Handle *h, int only = -1);  // pc/ml/mg/cf from the current alpha
void init_flux(Handle *h, int only = -1);  // F from U (linear interpolation)
// k_momentum.hip
// budget > 0: exactly that many sweeps (graph capture), samples that have
// converged skipped; else sweeps until every sample has converged
void momentum_predictor(Handle *h, int budget = 0);
// after a budgeted predictor: per-sample sweeps and convergence (host-mapped)
void momentum_results(Handle *h, int *sweeps, double *relres, int *converged);
void corrector_assemble(Handle *h);
void corrector_update(Handle *h, bool last);
// k_pressure.hip
int pressure_setup(Handle *h);    // multigrid hierarchy and launch shapes
int pressure_retune(Handle *h);   // rebuild launch shapes after a knob changed
void pressure_free(Handle *h);
// Solve every sample's system; budget > 0: exactly that many iterations with
// converged samples masked and no host synchronisation (graph capture).
// Per-sample iterations and relative residuals go to iters[s], relres[s] (or
// are left on the device when budget > 0).  Returns DBS_ENOCONV if a sample
// hit p_maxit.
int pressure_solve(Handle *h, const double *rAU, const double *b, double *x, int budget,
                   int *iters, double *relres);
// after a budgeted solve: per-sample iterations, relative residuals and
// whether the sample converged
void pressure_results(Handle *h, int *iters, double *relres, int *converged);
// k_pressure.hip: flat copy kernel over the cell arena (n arrays of NC)
void arena_copy(Handle *h, const double *src, double *dst, int narrays);
// copy n doubles with a kernel (safe under graph capture)
void copy_n(Handle *h, const double *src, double *dst, size_t n);
// the same into host-mapped memory (its device address), no blit
void host_copy(Handle *h, const double *src, double *dst_mapped, size_t n);
// store the last solve's per-sample iterations, relative residual,
// convergence flag, ||b|| and initial relative residual for corrector c in
// rec (ns x 16 x NREC doubles)
void pressure_record(Handle *h, double *rec, int c);
// per sample of the last solve: ||b||_2 and the initial relative residual
void pressure_norms(Handle *h, double *bnorm, double *res0);
// api.hip
void add_time(Handle *h, double dt);  // move the boundary-value time
// per sample: min a, max a, sum phi a V, max Co, nonfinite count, max |div F|
int cell_stats(Handle *h);

}  // namespace dbs
