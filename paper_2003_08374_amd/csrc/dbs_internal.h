// Host-side state of a dbs_handle and the launchers each translation unit
// provides.  Not part of the public ABI.
#pragma once
#include <string>
#include <vector>

#include "../../include/dbs.h"
#include "dbs_device.h"

namespace dbs {

// kernel classes for event timing (order = dbs_kernel_name)
enum KClass {
  KC_ALPHA_FACE = 0, KC_ALPHA_BOUNDS, KC_ALPHA_LIMIT, KC_ALPHA_UPDATE,
  KC_MOM_ASSEMBLE, KC_MOM_OFFDIAG, KC_PHIHBYA, KC_CORRECT,
  KC_SPMV, KC_AXPY, KC_DOT, KC_XPBY, KC_FINALIZE,
  KC_SMOOTH0, KC_RESTRICT0, KC_PROLONG0,
  KC_SMOOTHC, KC_RESTRICTC, KC_PROLONGC, KC_COARSE, KC_BUILD_COARSE,
  KC_STATS, KC_MISC, KC_SMOOTH0_ZERO, KC_COUNT
};

struct Level {
  int n[3] = {0, 0, 0};
  int nc = 0;
  // coarse-level operator (level >= 1): coefficient of the +x/+y/+z face of
  // each cell, Dirichlet diagonal part and full diagonal
  double *Tx = nullptr, *Ty = nullptr, *Tz = nullptr, *Db = nullptr, *D = nullptr;
  float *Txf = nullptr, *Tyf = nullptr, *Tzf = nullptr, *Dbf = nullptr, *Df = nullptr;
  double *x = nullptr, *b = nullptr;  // correction and right-hand side
  float *xf = nullptr, *bf = nullptr;
  dim3 grid;
};

struct Timer {
  std::vector<hipEvent_t> ev;  // pairs (start, stop)
  std::vector<int> cls;
  size_t used = 0;
};

struct Handle {
  Geom G;
  Phys P;
  dbs_controls ctl;
  std::string err;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  dim3 grid;  // cell launch grid of the fine mesh
  int nblocks = 0;

  // static fields
  double *phi = nullptr, *kinv = nullptr;
  // state (alpha is double-buffered: alpha holds n+1 after the transport)
  double *alpha = nullptr, *alpha_old = nullptr;
  double *U = nullptr, *U2 = nullptr;  // 3 x nc each
  double *prgh = nullptr, *p = nullptr;
  double *F = nullptr;                 // faces
  // closures of the current alpha: k_rl/mu_l, k_rg/mu_g, p_c (0 in clear cells)
  double *ml = nullptr, *mg = nullptr, *pc = nullptr;
  double *cf = nullptr;  // f_l - alpha in porous cells, 0 in clear cells
  // transport work arrays
  double *A = nullptr, *lam = nullptr, *rhoPhi = nullptr;  // faces
  double *Qp = nullptr, *Qm = nullptr, *Pin = nullptr, *Pout = nullptr, *Rp = nullptr,
         *Rm = nullptr;
  // momentum / pressure work arrays
  double *rAU = nullptr, *Sh = nullptr, *B = nullptr, *HbyA = nullptr;  // Sh,B,HbyA 3 x nc
  double *phiH = nullptr;  // faces
  double *rhs = nullptr;
  // PCG vectors
  double *r = nullptr, *z = nullptr, *pv = nullptr, *q = nullptr;
  float *rf = nullptr;  // FP32 residual (mixed precision)
  float *zoldf = nullptr;  // previous preconditioned residual (flexible CG)
  float *zf2 = nullptr;    // second fine correction buffer (FP32 V-cycle)
  double *z2 = nullptr;    // second fine correction buffer (FP64 V-cycle)
  double *partials = nullptr;  // per-block partial sums
  double *scal = nullptr;      // device scalars
  double *hscal = nullptr;     // pinned host mirror
  std::vector<Level> lv;
  void *lvshape = nullptr;  // launch shapes per level (owned by k_pressure.hip)
  int bottom = 0;           // first level cycled by one work-group
  int red_blocks = 0;       // blocks of the fine-level reduction kernels
  int mg_pre = 2, mg_post = 2, coarse_sweeps = 16;

  dbs_stats st;
  // profiling
  unsigned long long prof_mask = 0;
  Timer tm;
  long long k_launches[KC_COUNT] = {0};
  double k_ms[KC_COUNT] = {0};
  std::vector<void *> allocs;
};

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
void alpha_stage(Handle *h);
void update_closures(Handle *h);  // pc/ml/mg from the current alpha
void init_flux(Handle *h);        // F from U (linear interpolation)
// k_momentum.hip
void momentum_predictor(Handle *h);
void corrector_assemble(Handle *h);
void corrector_update(Handle *h, bool last);
// k_pressure.hip
int pressure_setup(Handle *h);    // allocate the multigrid hierarchy
void pressure_free(Handle *h);
int pressure_solve(Handle *h, const double *rAU, const double *b, double *x, int *iters,
                   double *relres);
// api.hip
void cell_stats(Handle *h, double out[5]);  // min a, max a, sum phi a V, max Co, nonfinite

}  // namespace dbs
