// Structured grids: 5-point / 7-point stencils with constant or variable
// coefficients, batched along z.  Messages live in six direction-major
// arrays; see kernels_grid.hip.
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "engine.h"

namespace gabp {

int check_grid(const gabp_grid *A, GridGeom *g) {
  if (!A || A->nx < 1 || A->ny < 1 || A->nz < 1 || A->batch < 1) return GABP_ERR_ARG;
  const int64_t N = (int64_t)A->nx * A->ny * A->nz * A->batch;
  if (N >= (int64_t)INT32_MAX / 8) return GABP_ERR_UNSUPPORTED;  // 6 N message slots in int32 range
  const bool any = A->cx || A->cy || A->cz;
  if (any && (!A->cx || !A->cy || (A->nz > 1 && !A->cz))) return GABP_ERR_ARG;
  if (!A->diag && (A->diag_value == 0.0)) return GABP_ERR_ZERO_DIAG;
  if (!A->diag && !std::isfinite(A->diag_value)) return GABP_ERR_ARG;
  if (!any && !std::isfinite(A->off_value)) return GABP_ERR_ARG;
  g->nx = A->nx; g->ny = A->ny; g->nz = A->nz; g->batch = A->batch;
  geom_finish(*g);
  return GABP_OK;
}

namespace {

bool grid_varc(const gabp_grid *A) { return A->cx || A->diag; }

// With variable coefficients every array must exist: constants the caller
// left NULL are expanded into device arrays owned by `owned`.
int expand_coefficients(const gabp_grid *A, int64_t N, GridCoef<double> *k,
                        std::vector<double *> *owned) {
  k->diag = A->diag; k->cx = A->cx; k->cy = A->cy; k->cz = A->cz;
  k->dconst = A->diag_value; k->aconst = A->off_value;
  if (!grid_varc(A)) return GABP_OK;
  const double *const *src[4] = {&k->diag, &k->cx, &k->cy, &k->cz};
  const double fill[4] = {A->diag_value, A->off_value, A->off_value, A->nz > 1 ? A->off_value : 0.0};
  for (int q = 0; q < 4; ++q) {
    if (*src[q]) continue;
    std::vector<double> h((size_t)N, fill[q]);
    double *d = nullptr;
    int st;
    if ((st = from_hip(dalloc(&d, N, sizeof(double))))) return st;
    owned->push_back(d);
    if ((st = from_hip(hipMemcpy(d, h.data(), (size_t)N * sizeof(double), hipMemcpyHostToDevice))))
      return st;
    *const_cast<const double **>(src[q]) = d;
  }
  return GABP_OK;
}

int64_t grid_edges(const gabp_grid *A) {
  const int64_t per = (int64_t)(A->nx - 1) * A->ny * A->nz + (int64_t)A->nx * (A->ny - 1) * A->nz +
                      (int64_t)A->nx * A->ny * (A->nz - 1);
  return 2 * per * A->batch;
}

}  // namespace

struct GridEngine : Engine {
  gabp_grid A{};
  GridGeom g{};
  bool varc = false;
  int grid = 1;
  GridCoef<double> k64{};          // caller's FP64 coefficients (residual)
  void *wdiag = nullptr, *wcx = nullptr, *wcy = nullptr, *wcz = nullptr;  // working copies
  std::vector<double *> owned;     // expanded constant coefficients
  void *rhs = nullptr;
  void *msg[2] = {nullptr, nullptr};  // (P, h)[6][N]
  void *coef = nullptr, *hh[2] = {nullptr, nullptr}, *Sfix = nullptr;  // frozen
  bool hzero = false;  // a restart left to the next sweep (restart_lazy)

  ~GridEngine() override {
    void *bufs[] = {wdiag, wcx, wcy, wcz, rhs, msg[0], msg[1], coef, hh[0], hh[1], Sfix};
    for (void *b : bufs)
      if (b) dfree(b);
    for (double *b : owned) dfree(b);
  }

  int64_t slots() const { return 6 * (int64_t)g.N; }

  GridArgs args(int mode, const Ctl *c) const {
    GridArgs a{};
    a.g = g; a.grid = grid; a.fp32 = fp32; a.varc = varc; a.damp = o.damping > 0.0 && mode != 2;
    a.frozen = frozen; a.mode = mode;
    a.diag = wdiag; a.cx = wcx; a.cy = wcy; a.cz = wcz;
    a.dconst = A.diag_value; a.aconst = A.off_value;
    a.rhs = rhs; a.coef = coef; a.Sfix = Sfix; a.alpha = o.damping; a.xprev = xprev;
    a.part = part; a.sticky = sticky; a.ctl = c;
    return a;
  }

  // the working right-hand side, for kernels that produce the FP64 one
  virtual WorkRhs work_rhs() const {
    WorkRhs w;
    w.p = rhs;
    w.fp32 = fp32;
    return w;
  }

  // a pending restart, carried out before anything but a sweep reads messages
  hipError_t settle_restart(hipStream_t s) { return hzero ? restart(s) : hipSuccess; }

  hipError_t restart_lazy(hipStream_t) override {
    hzero = true;
    return hipSuccess;
  }

  hipError_t sweep(int mode, const Ctl *c, hipStream_t s) override {
    GridArgs a = args(mode, c);
    a.msg_in = frozen ? hh[cur] : msg[cur];
    a.msg_out = frozen ? hh[cur ^ 1] : msg[cur ^ 1];
    // both the in-messages and a node's previous out-messages are in msg_in
    a.fl = hzero ? (SWEEP_ZIN | SWEEP_ZOWN) : 0;
    hzero = false;
    hipError_t err = launch_grid_sweep(a, s);
    cur ^= 1;
    return err;
  }

  hipError_t infer(double *xacc, double *marg, void *means, hipStream_t s) override {
    TRY_HIP_E(settle_restart(s));
    GridArgs a = args(2, nullptr);
    a.msg_in = frozen ? hh[cur] : msg[cur];
    a.xacc = xacc;
    a.marg = marg;
    a.xprev = means;
    return launch_grid_sweep(a, s);
  }

  hipError_t infer_set(double *x, hipStream_t s) override {
    TRY_HIP_E(settle_restart(s));
    GridArgs a = args(2, nullptr);
    a.msg_in = frozen ? hh[cur] : msg[cur];
    a.xacc = x;
    a.fl = SWEEP_XSET;
    return launch_grid_sweep(a, s);
  }

  hipError_t restart(hipStream_t s) override {
    hzero = false;
    if (frozen) return fp32 ? launch_fill_zero4(hh[cur], slots(), s) : launch_fill_zero(hh[cur], slots(), s);
    return launch_grid_zero_h(fp32, slots(), msg[cur], s);
  }

  hipError_t reset(const double *b, hipStream_t s) override {
    cur = 0;
    frozen = false;
    hzero = false;
    const int64_t words = slots() * (int64_t)(2 * tsz) / 8;
    hipError_t err;
    if ((err = launch_fill_zero(msg[0], words, s)) != hipSuccess) return err;
    if ((err = launch_fill_zero(msg[1], words, s)) != hipSuccess) return err;
    return launch_grid_residual(g, k64, varc, nsum, b, nullptr, rhs, fp32, nullptr, sumpart, s, 0, nseg);
  }

  hipError_t residual(const double *b, const double *x, double *r64, hipStream_t s) override {
    return launch_grid_residual(g, k64, varc, nsum, b, x, rhs, fp32, r64, sumpart, s, 0, nseg);
  }

  bool has_warm_start() const override { return true; }
  hipError_t warm_start(const uint16_t *w, hipStream_t s) override {
    cur = 0;
    frozen = false;
    hzero = false;
    return launch_grid_warm(fp32, g, varc ? wdiag : nullptr, varc ? wcx : nullptr,
                            varc ? wcy : nullptr, varc ? wcz : nullptr, A.diag_value, A.off_value,
                            rhs, w, msg[0], s);
  }

  bool can_freeze() const override { return true; }

  hipError_t ensure_frozen_buffers() override {
    struct { void **p; size_t count; } need[] = {
        {&coef, (size_t)slots()}, {&hh[0], (size_t)slots()}, {&hh[1], (size_t)slots()},
        {&Sfix, (size_t)g.N}};
    for (auto &b : need)
      if (!*b.p) {
        hipError_t err = dalloc(b.p, b.count, tsz);
        if (err != hipSuccess) return err;
      }
    return hipSuccess;
  }

  bool frozen_ready() const override { return coef && hh[0] && hh[1] && Sfix; }

  hipError_t freeze(hipStream_t s) override {
    TRY_HIP_E(settle_restart(s));
    GridArgs a = args(0, nullptr);
    a.msg_in = msg[cur];
    a.msg_out = hh[cur];
    hipError_t err = launch_grid_freeze(a, s);
    frozen = true;
    return err;
  }

  hipError_t freeze_restart(hipStream_t s) override {
    GridArgs a = args(0, nullptr);
    a.msg_in = msg[cur];
    a.msg_out = nullptr;  // informations not copied: the next sweep takes them as zero
    hipError_t err = launch_grid_freeze(a, s);
    frozen = true;
    hzero = true;
    return err;
  }

  int get_messages(double *P, double *h, hipStream_t s) override {
    if (!P || !h) return GABP_ERR_ARG;
    TRY_HIP(settle_restart(s));
    TRY_HIP(launch_grid_io(fp32, true, slots(), msg[cur], P, h, s));
    TRY_HIP(hipStreamSynchronize(s));
    return GABP_OK;
  }

  int set_messages(const double *P, const double *h, hipStream_t s) override {
    if (!P || !h) return GABP_ERR_ARG;
    hzero = false;
    TRY_HIP(launch_grid_io(fp32, false, slots(), msg[cur], (double *)P, (double *)h, s));
    TRY_HIP(hipStreamSynchronize(s));
    return GABP_OK;
  }

  // validate coefficients, build working-precision copies
  int build(hipStream_t s) {
    varc = grid_varc(&A);
    const int64_t N = g.N;
    int st;
    if ((st = expand_coefficients(&A, N, &k64, &owned))) return st;
    uint32_t *flags = nullptr;
    if ((st = from_hip(dalloc(&flags, 1, sizeof(uint32_t))))) return st;
    uint32_t hflags = 0;
    hipError_t e1 = launch_fill_zero4(flags, 1, s);
    if (e1 == hipSuccess) e1 = launch_grid_check(g, k64, varc, nsum, flags, s);
    if (e1 == hipSuccess) e1 = hipMemcpyAsync(&hflags, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
    if (e1 == hipSuccess) e1 = hipStreamSynchronize(s);
    dfree(flags);
    if (e1 != hipSuccess) return from_hip(e1);
    if (hflags & FLAG_ARG) return GABP_ERR_ARG;
    if (hflags & FLAG_ZERO_DIAG) return GABP_ERR_ZERO_DIAG;
    if (varc) {
      if ((st = from_hip(dalloc(&wdiag, N, tsz))) || (st = from_hip(dalloc(&wcx, N, tsz))) ||
          (st = from_hip(dalloc(&wcy, N, tsz))) || (st = from_hip(dalloc(&wcz, N, tsz))))
        return st;
      if ((st = from_hip(launch_to_working(fp32, N, k64.diag, wdiag, s))) ||
          (st = from_hip(launch_to_working(fp32, N, k64.cx, wcx, s))) ||
          (st = from_hip(launch_to_working(fp32, N, k64.cy, wcy, s))) ||
          (st = from_hip(launch_to_working(fp32, N, k64.cz, wcz, s))))  // NULL cz -> zeros
        return st;
    }
    return GABP_OK;
  }
};

// Two-colour schedule: one message buffer, colour-major storage
// (kernels_grid_rb.hip); a sweep is a launch per colour.
struct RbGridEngine : GridEngine {
  int hx = 1, Nc = 0;
  int rgrid = 1;  // blocks of a one-colour launch

  int64_t means_slots() const override { return 2 * (int64_t)Nc; }
  int sweep_launches() const override { return 2; }

  WorkRhs work_rhs() const override {
    WorkRhs w = GridEngine::work_rhs();
    w.hx = hx;
    w.nc = Nc;
    return w;
  }
  int64_t rb_slots() const { return 12 * (int64_t)Nc; }

  RbArgs rargs(int mode, int colour, const Ctl *c) const {
    RbArgs a{};
    a.g = g; a.hx = hx; a.Nc = Nc; a.grid = rgrid; a.colour = colour;
    a.fp32 = fp32; a.varc = varc; a.damp = o.damping > 0.0 && mode != 2;
    a.frozen = frozen; a.mode = mode;
    a.diag = wdiag; a.cx = wcx; a.cy = wcy; a.cz = wcz;
    a.dconst = A.diag_value; a.aconst = A.off_value;
    a.rhs = rhs; a.msg = frozen ? hh[0] : msg[0]; a.coef = coef; a.Sfix = Sfix;
    a.alpha = o.damping; a.xprev = xprev;
    // a stack's grids stop one by one: their check maxima go to one entry per grid
    a.part = part + (size_t)colour * (segctl ? nparts / 2 : rgrid); a.sticky = sticky; a.ctl = c;
    // segments only inside a solve: sweeps under the controller, and the
    // pass's x update; trajectory sweeps and marginals cover every grid
    const bool segs = segctl && ((mode < 2 && c) || (mode == 2 && infer_skips));
    a.nseg = nseg; a.seg = segs ? segctl : nullptr; a.act = segs ? segact : nullptr;
    return a;
  }

  hipError_t sweep(int mode, const Ctl *c, hipStream_t s) override {
    // after a pending restart colour 0 reads zero informations of colour 1;
    // colour 1 then reads colour 0's new ones; neither has old ones to damp with
    const bool z = hzero;
    hzero = false;
    for (int colour = 0; colour < 2; ++colour) {
      RbArgs a = rargs(mode, colour, c);
      a.fl = z ? (colour == 0 ? SWEEP_ZIN | SWEEP_ZOWN : SWEEP_ZOWN) : 0;
      hipError_t err = launch_rb_sweep(a, s);
      if (err != hipSuccess) return err;
    }
    return hipSuccess;
  }

  // Colour 1's nodes have their final in-messages once colour 0 has sent, so
  // colour 1's sweep launch also writes their means; colour 0's means follow
  // in a launch of their own (three launches instead of four, bitwise the
  // same x)
  hipError_t sweep_means(double *x, bool set, hipStream_t s) override {
    const bool z = hzero;
    hzero = false;
    RbArgs a = rargs(0, 0, nullptr);
    a.fl = z ? SWEEP_ZIN | SWEEP_ZOWN : 0;
    TRY_HIP_E(launch_rb_sweep(a, s));
    a = rargs(3, 1, nullptr);
    a.fl = (z ? SWEEP_ZOWN : 0) | (set ? SWEEP_XSET : 0);
    a.xacc = x;
    TRY_HIP_E(launch_rb_sweep(a, s));
    a = rargs(2, 0, nullptr);
    a.fl = set ? SWEEP_XSET : 0;
    a.xacc = x;
    return launch_rb_sweep(a, s);
  }

  hipError_t infer_set(double *x, hipStream_t s) override {
    TRY_HIP_E(settle_restart(s));
    for (int colour = 0; colour < 2; ++colour) {
      RbArgs a = rargs(2, colour, nullptr);
      a.xacc = x;
      a.fl = SWEEP_XSET;
      hipError_t err = launch_rb_sweep(a, s);
      if (err != hipSuccess) return err;
    }
    return hipSuccess;
  }

  hipError_t infer(double *xacc, double *marg, void *means, hipStream_t s) override {
    TRY_HIP_E(settle_restart(s));
    for (int colour = 0; colour < 2; ++colour) {
      RbArgs a = rargs(2, colour, nullptr);
      a.xacc = xacc;
      a.marg = marg;
      a.xprev = means;
      hipError_t err = launch_rb_sweep(a, s);
      if (err != hipSuccess) return err;
    }
    return hipSuccess;
  }

  hipError_t restart(hipStream_t s) override {
    hzero = false;
    if (frozen) return fp32 ? launch_fill_zero4(hh[0], rb_slots(), s) : launch_fill_zero(hh[0], rb_slots(), s);
    return launch_grid_zero_h(fp32, rb_slots(), msg[0], s);
  }

  hipError_t reset(const double *b, hipStream_t s) override {
    frozen = false;
    hzero = false;
    hipError_t err = launch_fill_zero(msg[0], rb_slots() * (int64_t)(2 * tsz) / 8, s);
    if (err != hipSuccess) return err;
    return launch_grid_residual(g, k64, varc, nsum, b, nullptr, rhs, fp32, nullptr, sumpart, s, hx, nseg);
  }

  hipError_t residual(const double *b, const double *x, double *r64, hipStream_t s) override {
    return launch_grid_residual(g, k64, varc, nsum, b, x, rhs, fp32, r64, sumpart, s, hx, nseg);
  }

  hipError_t warm_start(const uint16_t *w, hipStream_t s) override {
    frozen = false;
    hzero = false;
    // slots of unused positions and of faces without a coupling stay zero
    hipError_t err = launch_fill_zero(msg[0], rb_slots() * (int64_t)(2 * tsz) / 8, s);
    if (err != hipSuccess) return err;
    return launch_grid_warm(fp32, g, varc ? wdiag : nullptr, varc ? wcx : nullptr,
                            varc ? wcy : nullptr, varc ? wcz : nullptr, A.diag_value, A.off_value,
                            rhs, w, msg[0], s, hx);
  }

  hipError_t ensure_frozen_buffers() override {
    struct { void **p; size_t count; } need[] = {
        {&coef, (size_t)rb_slots()}, {&hh[0], (size_t)rb_slots()}, {&Sfix, 2 * (size_t)Nc}};
    for (auto &b : need)
      if (!*b.p) {
        hipError_t err = dalloc(b.p, b.count, tsz);
        if (err != hipSuccess) return err;
      }
    return hipSuccess;
  }

  bool frozen_ready() const override { return coef && hh[0] && Sfix; }

  hipError_t freeze(hipStream_t s) override {
    TRY_HIP_E(settle_restart(s));
    RbArgs a = rargs(0, 0, nullptr);
    a.msg = msg[0];
    hipError_t err = launch_rb_freeze(a, hh[0], s);
    frozen = true;
    return err;
  }

  hipError_t freeze_restart(hipStream_t s) override {
    RbArgs a = rargs(0, 0, nullptr);
    a.msg = msg[0];
    hipError_t err = launch_rb_freeze(a, nullptr, s);  // informations not copied
    frozen = true;
    hzero = true;
    return err;
  }

  int get_messages(double *P, double *h, hipStream_t s) override {
    if (!P || !h) return GABP_ERR_ARG;
    TRY_HIP(settle_restart(s));
    TRY_HIP(launch_rb_io(fp32, true, g, hx, Nc, msg[0], P, h, s));
    TRY_HIP(hipStreamSynchronize(s));
    return GABP_OK;
  }

  int set_messages(const double *P, const double *h, hipStream_t s) override {
    if (!P || !h) return GABP_ERR_ARG;
    hzero = false;
    TRY_HIP(launch_rb_io(fp32, false, g, hx, Nc, msg[0], (double *)P, (double *)h, s));
    TRY_HIP(hipStreamSynchronize(s));
    return GABP_OK;
  }
};

// ---------------------------------------------------------------------------
// Coarse-grid predicted corrections.  GaBP removes the smooth part of the
// error slowly (it behaves like a relaxation on the low modes of a Poisson
// operator), and no initial messages computed from a node's own neighbourhood
// can supply it.  Here every correction d of A d = r (r = b - A x) is
// predicted on coarser grids: a few GaBP sweeps on r (zero information
// messages, precisions of the level's previous sweeps kept) give d; the
// residual of d, summed over 2 x 2 x 2 blocks, is the right-hand side of the
// same procedure on the Galerkin operator of the next coarser grid, down to a
// grid of at most 64 cells, where the correction is the exact solution of the
// Galerkin system (its dense inverse per grid, built once); the coarse
// correction, injected back and scaled, is added; a few more GaBP sweeps on
// the remaining residual finish d.  Then x += d, until every grid of the
// stack meets the tolerance.  (A grid that is itself at most 64 cells is
// corrected by kCoarseSweeps GaBP sweeps alone.)
// ---------------------------------------------------------------------------
// Sweeps per visit of a level: 3 before and 3 after the coarse prediction
// (4 + 4 took the same number of corrections in the FP64 oracle on 32^3 to
// 64^3 variable-coefficient stacks and damped synchronous grids, one more
// on a few, at a quarter more sweeps).
constexpr int kCoarsePre = 3, kCoarsePost = 3, kCoarseSweeps = 24;
// The coarsest level is the first below the finest with at most
// kCoarsestCellsMax cells per grid, solved exactly by its dense inverses
// when those take at most kCoarseInverseBytes (one mat-vec per visit
// replaces a launch of the LDS tail, which on a single grid takes one
// workgroup about 50 us); otherwise the first with at most kCoarsestCells,
// the LDS tail running the levels between.  A finest grid of at most
// kCoarsestCells cells is its own coarsest level.  GABP_COARSE_EXACT=64 at
// plan time takes the small coarsest level.
constexpr int64_t kCoarseInverseBytes = (int64_t)1 << 30;
// A level whose grids have at most kCoarseVCells cells is cycled once by the
// level above (a V-cycle into it), a larger one twice (a W-cycle): the small
// levels are a handful of short launches per visit, and in the FP64 oracle
// their second visits saved no correction (64^3 variable-coefficient grids
// 6, 256^3 damped Poisson 8, with or without them; 128^3 damped Poisson 9
// instead of 8).  GABP_COARSE_WCYCLE=1 at plan time cycles every level twice.
constexpr int64_t kCoarseVCells = 4096;
// Synchronous sweeps on a grid (a bipartite graph) do not damp the error mode
// that alternates between the two colours, so as a smoother they need
// damping: an undamped synchronous plan smooths with this factor (the FP64
// oracle diverges without it and takes 11-13 corrections with it on
// 16^3 - 24^3 grids); the coloured schedule smooths with the plan's own.
constexpr double kCoarseSyncDamping = 0.3;
// The precision messages do not depend on the right-hand side; once a level
// has swept this many times in one solve (with opts.freeze on: from its
// second smoothing on) it keeps them fixed and sweeps the information
// messages only (the settled-precision sweeps of the plain solve).  The
// smoother is then GaBP with precisions of a few sweeps, and the FP64
// residual of every correction absorbs the difference.  Measured with 3 + 3
// sweeps (freeze after 16 / 9 / 6 / 3 sweeps of a level): 64 grids of 64^3
// 37.8 / 35.0 / 33.6 / 32.7 ms, 7 corrections each; 256^3 damped 80.2 /
// 78.4 / 78.1 / 72.3 ms, 14 corrections, 13 with the last.
constexpr int kCoarseFreezeAfter = 2;
// Injection of a block's correction into its cells under-corrects smooth
// error (the coarse operator of piecewise constants is too stiff by about a
// factor of two); the scale was chosen with the FP64 oracle on
// variable-coefficient grids of 16^3 to 64^3.
constexpr double kCoarseScale = 1.8;
// Cycles of the next level per coarse correction: 2 (a W-cycle).  With one
// (a V-cycle) the correction loses accuracy with every level: in the FP64
// oracle the shifted 64^3 Laplacian (5 levels) stalls near 3e-3 under damped
// synchronous smoothing, while with two every tested grid (16^3 to 64^3,
// constant and variable coefficients, both schedules) needs 7 to 13.
constexpr int kCoarseGamma = 2;

struct CoarseHierarchy {
  struct Level {
    gabp_plan *plan = nullptr;  // levels >= 1 (level 0 is the caller's plan)
    Engine *eng = nullptr;
    GridEngine *ge = nullptr;   // the same engine as a grid plan's
    GridGeom g{};
    double *dg = nullptr, *cx = nullptr, *cy = nullptr, *cz = nullptr;  // levels >= 1
    double *v = nullptr, *d = nullptr;  // right-hand side, correction
    double *e = nullptr;  // levels >= 1: the first cycle's correction (a tail level: the tail's sum)
    double *Pt = nullptr; // tail levels: precision messages kept between tail launches
    double *inv = nullptr;  // the coarsest level (below the finest): inverse per grid
    GridCoef<double> k{};   // the level's FP64 operator
    bool varc = true;
    bool fresh = true;  // messages not yet set in this solve
    int swept = 0;      // sweeps of this level in this solve
  };
  std::vector<Level> lv;
  // Levels tail.. (when tail > 0) have at most kTailThreads cells per grid
  // and run inside one k_coarse_tail launch per visit of level tail - 1
  // instead of a few hundred launches of their own; they have no plans.
  // GABP_COARSE_TAIL=0 at plan time runs them as plans too.
  int tail = 0;
  int max_cells = kCoarsestCellsMax;  // of the coarsest level below the finest
  int64_t vcells = kCoarseVCells;     // levels of at most this many cells per grid: one visit
  bool tail_fresh = true;  // the tail's precision messages not yet set in this solve
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  // Once every level has been set up in a solve and (with opts.freeze) has
  // settled its precisions, a correction is the same sequence of launches on
  // the same buffers every time (each visit of a level runs an even number of
  // sweeps, so double-buffered engines start every correction from the same
  // buffer): it is captured once into a graph and replayed, one launch per
  // correction instead of a few hundred (most of them on the small grids,
  // where the launches, not the sweeps, set the time).  GABP_COARSE_GRAPH=0
  // at plan time keeps every correction eager.
  bool use_graph = true;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t cs = nullptr;  // capture stream (the caller's may be the legacy NULL stream)
  // The solve combines each grid's corrections by GCR(1): the new one made
  // orthogonal, through its image under A, to the previous step's, and
  // taken with the step that minimises the residual along it (the oracle's
  // convergence tests: 13 -> 8 corrections on a 128^3 shifted Poisson grid,
  // 7 -> 6 on a variable-coefficient one).  GABP_COARSE_GCR=0 at plan time
  // adds the corrections as they come.
  bool gcr = true;
  int gseg = 1, gsegb = 1;  // grids of the stack, blocks per grid of the inner products
  double *gw = nullptr, *gpc = nullptr, *gpw = nullptr, *gpart = nullptr, *gpp = nullptr;
  double2 *gab = nullptr;

  ~CoarseHierarchy() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cs) (void)hipStreamDestroy(cs);
    for (Level &L : lv) {
      if (L.plan) gabp_plan_destroy(L.plan);
      double *bufs[] = {L.dg, L.cx, L.cy, L.cz, L.v, L.d, L.e, L.Pt, L.inv};
      for (double *b : bufs)
        if (b) dfree(b);
    }
    double *gbufs[] = {gw, gpc, gpw, gpart, gpp, (double *)gab};
    for (double *b : gbufs)
      if (b) dfree(b);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }

  double damping = 0.0;  // of every level's sweeps
  bool freeze = true;    // settle the precisions after kCoarseFreezeAfter sweeps

  TailArgs tail_args(const Level &top) const {
    TailArgs a{};
    a.nlev = (int)lv.size() - tail;
    a.batch = top.g.batch;
    for (int l = 0; l < a.nlev; ++l) {
      const Level &L = lv[tail + l];
      a.lv[l] = TailLevel{L.g.nx, L.g.ny, L.g.nz, L.dg, L.cx, L.cy, L.cz, L.Pt};
    }
    a.inv = lv.back().inv;
    a.rc = top.v;
    a.e = top.e;
    a.damping = damping;
    a.scale = kCoarseScale;
    a.colored = colored ? 1 : 0;
    a.pre = kCoarsePre;
    a.post = kCoarsePost;
    // every tail level has at most kTailThreads cells per grid
    a.gamma = vcells >= kTailThreads ? 1 : kCoarseGamma;
    return a;
  }

  // the first level the tail kernel can take with every level below it
  // (0: none)
  static int tail_start(const std::vector<GridGeom> &shapes) {
    const int nl = (int)shapes.size();
    for (int l = 1; l < nl; ++l) {
      if (nl - l > kTailMaxLevels) continue;
      TailArgs a{};
      a.nlev = nl - l;
      bool fits = true;
      for (int m = l; m < nl; ++m) {
        const GridGeom &g = shapes[m];
        fits = fits && (int64_t)g.nx * g.ny * g.nz <= kTailThreads;
        a.lv[m - l].nx = g.nx; a.lv[m - l].ny = g.ny; a.lv[m - l].nz = g.nz;
      }
      if (fits && coarse_tail_lds(a) <= (size_t)max_lds_per_block()) return l;
    }
    return 0;
  }

  bool colored = false;

  int build(GridEngine *e0, hipStream_t s) {
    damping = e0->o.damping;
    freeze = e0->o.freeze != 0;
    colored = e0->o.schedule == GABP_SCHEDULE_COLORED;
    if (const char *g = std::getenv("GABP_COARSE_GRAPH")) use_graph = std::strcmp(g, "0") != 0;
    if (const char *g = std::getenv("GABP_COARSE_GCR")) gcr = std::strcmp(g, "0") != 0;
    if (const char *g = std::getenv("GABP_COARSE_WCYCLE"); g && std::strcmp(g, "1") == 0)
      vcells = 0;
    if (gcr) {
      gseg = e0->nseg > 1 ? e0->nseg : 1;
      gsegb = e0->nseg > 1 ? e0->segb : std::max(e0->nsum, 1);
      TRY_HIP(dalloc(&gw, e0->g.N, sizeof(double)));
      TRY_HIP(dalloc(&gpc, e0->g.N, sizeof(double)));
      TRY_HIP(dalloc(&gpw, e0->g.N, sizeof(double)));
      TRY_HIP(dalloc(&gpart, (size_t)gseg * gsegb * 4, sizeof(double)));
      TRY_HIP(dalloc(&gpp, gseg, sizeof(double)));
      TRY_HIP(dalloc(&gab, gseg, sizeof(double2)));
    }
    if (e0->o.schedule == GABP_SCHEDULE_SYNC && damping == 0.0) damping = kCoarseSyncDamping;
    TRY_HIP(hipEventCreate(&ev0));
    TRY_HIP(hipEventCreate(&ev1));
    auto cells_of = [](const GridGeom &g) { return (int64_t)g.nx * g.ny * g.nz; };
    auto shapes_for = [&](int mc) {
      std::vector<GridGeom> sh{e0->g};
      while (cells_of(sh.back()) > (sh.size() == 1 ? kCoarsestCells : mc))
        sh.push_back(coarse_geom(sh.back()));
      return sh;
    };
    const char *xe = std::getenv("GABP_COARSE_EXACT");
    if (xe && std::strcmp(xe, "64") == 0) {
      max_cells = kCoarsestCells;
    } else {
      const std::vector<GridGeom> big = shapes_for(kCoarsestCellsMax);
      const int64_t nc = cells_of(big.back());
      if (big.size() > 1 && (int64_t)big.back().batch * nc * nc * 8 > kCoarseInverseBytes)
        max_cells = kCoarsestCells;
    }
    const std::vector<GridGeom> shapes = shapes_for(max_cells);
    const char *te = std::getenv("GABP_COARSE_TAIL");
    tail = (te && std::strcmp(te, "0") == 0) || max_cells > kCoarsestCells ? 0 : tail_start(shapes);
    Level L0;
    L0.eng = e0;
    L0.ge = e0;
    L0.g = e0->g;
    L0.k = e0->k64;
    L0.varc = e0->varc;
    lv.push_back(L0);
    GridCoef<double> k = e0->k64;
    bool varc = e0->varc;
    for (;;) {
      Level &F = lv.back();
      TRY_HIP(dalloc(&F.v, F.g.N, sizeof(double)));
      TRY_HIP(dalloc(&F.d, F.g.N, sizeof(double)));
      if (lv.size() > 1) TRY_HIP(dalloc(&F.e, F.g.N, sizeof(double)));
      if (cells_of(F.g) <= (lv.size() == 1 ? kCoarsestCells : max_cells)) break;
      Level C;
      C.g = coarse_geom(F.g);
      const GridGeom fg = F.g;  // F may move when lv grows
      TRY_HIP(dalloc(&C.dg, C.g.N, sizeof(double)));
      TRY_HIP(dalloc(&C.cx, C.g.N, sizeof(double)));
      TRY_HIP(dalloc(&C.cy, C.g.N, sizeof(double)));
      TRY_HIP(dalloc(&C.cz, C.g.N, sizeof(double)));
      TRY_HIP(launch_coarse_coef(fg, k, varc, C.g, C.dg, C.cx, C.cy, C.cz, s));
      gabp_grid Ag{};
      Ag.nx = C.g.nx; Ag.ny = C.g.ny; Ag.nz = C.g.nz; Ag.batch = C.g.batch;
      Ag.diag = C.dg; Ag.cx = C.cx; Ag.cy = C.cy; Ag.cz = C.cz;
      gabp_opts o = e0->o;
      o.damping = damping;
      C.k = GridCoef<double>{C.dg, C.cx, C.cy, C.cz, 0.0, 0.0};
      C.varc = true;
      lv.push_back(C);  // owned from here on (freed by the destructor)
      const int64_t cells = (int64_t)C.g.nx * C.g.ny * C.g.nz;
      if (cells <= max_cells) {
        // the coarsest level: its inverse per grid, no messages
        Level &Z = lv.back();
        uint32_t *bad = nullptr;
        double *work = nullptr;  // [M | I] per grid for the larger inverses
        TRY_HIP(dalloc(&Z.inv, (size_t)cells * cells * C.g.batch, sizeof(double)));
        TRY_HIP(dalloc(&bad, 1, sizeof(uint32_t)));
        hipError_t e = cells > kCoarsestCells
                           ? dalloc(&work, (size_t)(2 * cells + 1) * cells * C.g.batch,
                                    sizeof(double))
                           : hipSuccess;
        uint32_t hb = 0;
        if (e == hipSuccess) e = launch_fill_zero4(bad, 1, s);
        if (e == hipSuccess)
          e = launch_coarse_inverse(C.g, C.dg, C.cx, C.cy, C.cz, Z.inv, work, bad, s);
        if (e == hipSuccess) e = hipMemcpyAsync(&hb, bad, sizeof(hb), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        dfree(bad);
        if (work) dfree(work);
        TRY_HIP(e);
        if (hb & FLAG_BREAKDOWN) return GABP_ERR_BREAKDOWN;  // a singular coarse system
      } else if (tail > 0 && (int)lv.size() - 1 >= tail) {
        TRY_HIP(dalloc(&lv.back().Pt, (size_t)6 * C.g.N, sizeof(double)));
      } else {
        const int rc = gabp_plan_create_grid(&Ag, &o, &lv.back().plan, s);
        if (rc) return rc;
        lv.back().eng = lv.back().plan->eng;
        lv.back().ge = dynamic_cast<GridEngine *>(lv.back().eng);
        if (!lv.back().ge) return GABP_ERR_UNSUPPORTED;
      }
      k = GridCoef<double>{C.dg, C.cx, C.cy, C.cz, 0.0, 0.0};
      varc = true;
    }
    TRY_HIP(hipStreamSynchronize(s));
    return GABP_OK;
  }

  // d_l (set: =, else +=) the means of `sweeps` GaBP sweeps on the level's
  // right-hand side, from zero information messages (zeroed by the first
  // sweep itself).  The kernel that produced the FP64 right-hand side v has
  // also written it into the engine's working right-hand side: the solve's
  // residual on level 0, the level above's restriction or copy-residual
  // below; v is needed only by a level's first smoothing in a solve, which
  // resets the engine from it.
  int smooth(int l, const double *v, int sweeps, bool set, hipStream_t s) {
    Level &L = lv[l];
    if (v && L.fresh) {
      TRY_HIP(L.eng->reset(v, s));
      L.fresh = false;
      L.swept = 0;
    } else {
      TRY_HIP(L.eng->restart_lazy(s));  // zero informations (after a freeze: the settled ones)
    }
    if (freeze && !L.eng->frozen && L.swept >= kCoarseFreezeAfter) {
      TRY_HIP(L.eng->ensure_frozen_buffers());
      TRY_HIP(L.eng->freeze_restart(s));
    }
    static_assert(kCoarsePre > 0 && kCoarseSweeps > 0, "every smoothing sweeps");
    for (int k = 0; k + 1 < sweeps; ++k) TRY_HIP(L.eng->sweep(0, nullptr, s));
    TRY_HIP(L.eng->sweep_means(L.d, set, s));
    L.swept += sweeps;
    return GABP_OK;
  }

  int correction(hipStream_t s);


  // d_l from v_l: smoothing, coarse prediction, smoothing
  int cycle(int l, hipStream_t s) {
    Level &L = lv[l];
    if (l + 1 == (int)lv.size()) {
      if (l == 0) return smooth(l, L.v, kCoarseSweeps, true, s);  // its own coarsest level
      TRY_HIP(launch_coarse_dense_solve(L.g, L.inv, L.v, L.d, s));
      return GABP_OK;
    }
    int rc = smooth(l, L.v, kCoarsePre, true, s);
    if (rc) return rc;
    Level &C = lv[l + 1];
    const WorkRhs cw = C.ge ? C.ge->work_rhs() : WorkRhs{};
    // the next level's right-hand side P^T (v - A d)
    TRY_HIP(launch_coarse_residual_restrict(L.g, L.k, L.varc, C.g, L.v, L.d, C.v, cw, s));
    // the coarse system: kCoarseGamma cycles of the next level (one of a
    // small level), each on the residual the previous ones left; two
    // cycles' corrections summed in C.e
    if (tail > 0 && l + 1 == tail) {
      TailArgs a = tail_args(C);
      a.sticky = lv[0].eng->sticky;
      a.fresh = tail_fresh ? 1 : 0;
      TRY_HIP(launch_coarse_tail(a, s));
      tail_fresh = false;
      TRY_HIP(launch_coarse_prolong(L.g, C.g, C.e, nullptr, kCoarseScale, L.d, s));
    } else if (l + 2 == (int)lv.size() || (int64_t)C.g.nx * C.g.ny * C.g.nz <= vcells) {
      // one cycle: the next level is the coarsest (its exact solution) or small
      if ((rc = cycle(l + 1, s))) return rc;
      TRY_HIP(launch_coarse_prolong(L.g, C.g, C.d, nullptr, kCoarseScale, L.d, s));
    } else {
      static_assert(kCoarseGamma == 2, "the second cycle's right-hand side below assumes two");
      if ((rc = cycle(l + 1, s))) return rc;
      // e = d, and the second cycle on what the first left: v_c = rc - A_c e
      TRY_HIP(launch_coarse_copy_residual(C.g, C.k, C.varc, C.d, C.e, C.v, cw, s));
      if ((rc = cycle(l + 1, s))) return rc;
      // the two cycles' corrections summed (e + d) inside the prolongation
      TRY_HIP(launch_coarse_prolong(L.g, C.g, C.e, C.d, kCoarseScale, L.d, s));
    }
    if (kCoarsePost > 0) {
      TRY_HIP(L.eng->residual(L.v, L.d, nullptr, s));  // the engine's right-hand side only
      if ((rc = smooth(l, nullptr, kCoarsePost, false, s))) return rc;
    }
    return GABP_OK;
  }
};

// One correction d_0 = cycle(0): eager until the hierarchy is in its steady
// state, then from the captured graph.
int CoarseHierarchy::correction(hipStream_t s) {
  bool steady = use_graph && !(tail > 0 && tail_fresh);
  for (const Level &L : lv)
    if (L.eng) steady = steady && !L.fresh && (!freeze || L.eng->frozen);
  if (!steady) return cycle(0, s);
  if (!exec) {
    // record on a stream of our own (nothing runs while capturing); the
    // steady state's host bookkeeping (sweep counts, buffer parity) ends where
    // it began, so a failed capture only means running this correction eagerly
    hipGraph_t g = nullptr;
    bool ok = (cs || hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess) &&
              hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
    if (ok) {
      const int rc = cycle(0, cs);
      ok = hipStreamEndCapture(cs, &g) == hipSuccess && rc == GABP_OK && g &&
           hipGraphInstantiate(&exec, g, nullptr, nullptr, 0) == hipSuccess;
    }
    if (!ok) {
      (void)hipGetLastError();
      if (g) (void)hipGraphDestroy(g);
      exec = nullptr;
      use_graph = false;
      if (std::getenv("GABP_VERBOSE")) std::fprintf(stderr, "gabp: coarse cycle not captured\n");
      return cycle(0, s);
    }
    graph = g;
  }
  TRY_HIP(hipGraphLaunch(exec, s));
  return GABP_OK;
}

void coarse_destroy(CoarseHierarchy *h) { delete h; }

int64_t coarse_bytes(const CoarseHierarchy *h) {
  int64_t b = 0;
  for (const auto &L : h->lv)
    if (L.plan && L.plan->acct) b += L.plan->acct->bytes.load();
  return b;
}

int coarse_solve(gabp_plan *p, const double *b, double *x, double *marg_prec, gabp_stats *st,
                 hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  GridEngine *e0 = p ? dynamic_cast<GridEngine *>(p->eng) : nullptr;
  if (!e0) return GABP_ERR_UNSUPPORTED;
  if (e0->n > 0 && (!b || !x)) return GABP_ERR_ARG;
  gabp_stats stats{};
  stats.edges = e0->E;
  stats.sweep_launches = e0->sweep_launches();
  stats.damping = e0->o.damping;
  auto finish = [&](int status) {
    stats.status = status;
    stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats.mean_sweeps = stats.sweeps;
    stats.edge_updates_per_s =
        stats.seconds > 0 ? (double)stats.edges * stats.sweeps / stats.seconds : 0.0;
    if (st) *st = stats;
    return status;
  };
  if (!p->coarse) {
    auto *h = new (std::nothrow) CoarseHierarchy();
    if (!h) return GABP_ERR_NOMEM;
    const int rc = h->build(e0, s);
    if (rc) {
      delete h;
      return finish(rc);
    }
    p->coarse = h;
  }
  CoarseHierarchy &H = *p->coarse;
  for (auto &L : H.lv) L.fresh = true;
  H.tail_fresh = true;
  // the plan's own sweeps smooth with the hierarchy's damping for this call
  struct Restore {
    GridEngine *e;
    double d;
    ~Restore() { e->o.damping = d; }
  } restore{e0, e0->o.damping};
  e0->o.damping = H.damping;
  stats.damping = H.damping;
  TRY_HIP(launch_fill_zero4(e0->sticky, 1, s));
  TRY_HIP(launch_fill_zero(x, e0->n, s));
  // ||b_t|| of every grid of the stack (kept by the engine for the norms below)
  TRY_HIP(e0->reset(b, s));
  HostReadout r0;
  int rc = e0->read_sum(s, &r0, 1);
  if (rc) return finish(rc);
  if (!std::isfinite(r0.sum)) return finish(GABP_ERR_ARG);
  const double bn = std::sqrt(r0.sum);
  if (bn == 0.0) {
    stats.rel_residual = 0.0;
    return finish(GABP_OK);
  }
  int status = GABP_NOT_CONVERGED;
  // With the GCR step the residual in lv[0].v (and the working right-hand
  // side and the norms' partial sums) follows x through the step itself, as
  // r - alpha A c'; b - A x is formed at the start and again, to confirm, when
  // the recursive residual meets the tolerance or the budget ends the loop.
  bool recur = false;
  TRY_HIP(hipEventRecord(H.ev0, s));
  for (int cyc = 0;;) {
    double rel = 1.0;
    if (cyc == 0 && !recur && e0->o.tol < 1.0) {
      // x = 0: r = b, whose working copy and norms the reset above produced
      TRY_HIP(hipMemcpyAsync(H.lv[0].v, b, (size_t)e0->n * sizeof(double),
                             hipMemcpyDeviceToDevice, s));
      stats.rel_residual = 1.0;
      stats.residual_per_eq = bn / e0->n;
    } else {
      // r = b - A x (FP64) and the worst grid's relative residual
      if (!recur) TRY_HIP(e0->residual(b, x, H.lv[0].v, s));
      HostReadout rr;
      if ((rc = e0->read_sum(s, &rr, 2, bn))) return finish(rc);
      const double rel_all = std::sqrt(rr.sum) / bn;
      rel = (e0->nseg > 1 && std::isfinite(rel_all)) ? rr.segrel : rel_all;
      stats.rel_residual = rel;
      stats.residual_per_eq = std::sqrt(rr.sum) / e0->n;
      if (rr.flags & FLAG_BREAKDOWN) { status = GABP_ERR_BREAKDOWN; break; }
      if ((rr.flags & FLAG_NONFINITE) || !std::isfinite(rel) || rel > 1e6) {
        status = GABP_ERR_DIVERGED;
        break;
      }
    }
    const bool done = rel <= e0->o.tol;
    const bool spent = cyc >= e0->o.max_restarts || stats.sweeps >= e0->o.max_sweeps;
    if ((done || spent) && recur) {
      recur = false;  // confirm on b - A x
      continue;
    }
    if (done) { status = GABP_OK; break; }
    if (spent) break;
    if ((rc = H.correction(s))) return finish(rc);
    if (H.gcr) {
      // lv[0].v still holds this iteration's residual r
      TRY_HIP(launch_gcr_step(e0->g, e0->k64, e0->varc, H.gseg, H.gsegb, H.lv[0].d, H.lv[0].v,
                              H.gw, H.gpc, H.gpw, H.gpart, H.gpp, H.gab, cyc == 0, x,
                              e0->work_rhs(), e0->sumpart, s));
      recur = true;
    } else {
      TRY_HIP(launch_axpy(e0->n, H.lv[0].d, x, s));
    }
    stats.sweeps += kCoarsePre + kCoarsePost;
    stats.restarts = ++cyc;
  }
  TRY_HIP(hipEventRecord(H.ev1, s));
  if (marg_prec) TRY_HIP(e0->infer(nullptr, marg_prec, nullptr, s));
  TRY_HIP(hipStreamSynchronize(s));
  float ms = 0.f;
  TRY_HIP(hipEventElapsedTime(&ms, H.ev0, H.ev1));
  stats.sweep_ms = ms;
  return finish(status);
}

}  // namespace gabp

using namespace gabp;

extern "C" {

static int plan_create_grid_impl(const gabp_grid *A, const gabp_opts *o, gabp_plan **plan, hipStream_t s) {
  clear_stale_error();
  if (!plan) return GABP_ERR_ARG;
  *plan = nullptr;
  gabp_opts opts;
  if (o) opts = *o;
  else gabp_default_opts(&opts);
  int st;
  if ((st = check_opts(&opts))) return st;
  if (opts.accel != GABP_ACCEL_NONE) return GABP_ERR_UNSUPPORTED;  // small CSR batches only
  GridGeom g{};
  if ((st = check_grid(A, &g))) return st;
  const bool coloured = opts.schedule == GABP_SCHEDULE_COLORED;
  RbGridEngine *rb = coloured ? new (std::nothrow) RbGridEngine() : nullptr;
  GridEngine *e = coloured ? rb : new (std::nothrow) GridEngine();
  if (!e) return GABP_ERR_NOMEM;
  e->A = *A;
  e->g = g;
  e->o = opts;
  e->n = g.N;
  e->E = grid_edges(A);
  e->fp32 = opts.msg_fp32 != 0;
  e->tsz = e->fp32 ? sizeof(float) : sizeof(double);
  const int cap = opts.grid_blocks > 0 ? opts.grid_blocks : kMaxSweepBlocks;
  const int need = (g.N + kBlock - 1) / kBlock;
  e->grid = need < cap ? need : cap;
  e->nparts = e->grid;
  e->nsum = e->grid;
  if (g.batch > 1) {
    // the grids of a stack are independent systems: each must meet the tolerance
    const int per = (g.N / g.batch + kBlock - 1) / kBlock;
    const int share = std::max(1, kMaxSweepBlocks / g.batch);
    e->nseg = g.batch;
    e->segb = std::min(per, share);
    e->nsum = e->nseg * e->segb;
  }
  if (rb) {
    rb->hx = rb_row_slots(g);
    rb->Nc = rb->hx * (g.N / g.nx);
    const int rneed = (rb->Nc + kBlock - 1) / kBlock;
    rb->rgrid = rneed < cap ? rneed : cap;
    e->nparts = 2 * rb->rgrid;  // a check sweep publishes one partial per block and colour
    const int widest = std::min(cap, kMaxSweepBlocks);
    if (e->nseg > 1 && e->nseg <= widest) {
      // each grid of the stack leaves the sweeps once it meets its own
      // target; the segment sweeps need a block per grid at least, and the
      // readout's per-grid reduction bounds the launch
      rb->rgrid = std::min(std::max(rb->rgrid, e->nseg), widest);
      e->segctl_wanted = true;
      e->seg_grid = rb->rgrid;
      e->nparts = 2 * rb->rgrid;
    }
  }
  auto fail = [&](int code) {
    delete e;
    return code;
  };
  if ((st = e->init_common(s))) return fail(st);
  if ((st = e->build(s))) return fail(st);
  if (rb) {
    if ((st = from_hip(dalloc(&e->msg[0], rb->rb_slots(), 2 * e->tsz))) ||
        (st = from_hip(dalloc(&e->rhs, 2 * (size_t)rb->Nc, e->tsz))))
      return fail(st);
  } else if ((st = from_hip(dalloc(&e->msg[0], e->slots(), 2 * e->tsz))) ||
             (st = from_hip(dalloc(&e->msg[1], e->slots(), 2 * e->tsz))) ||
             (st = from_hip(dalloc(&e->rhs, g.N, e->tsz))))
    return fail(st);
  gabp_plan *p = new (std::nothrow) gabp_plan();
  if (!p) return fail(GABP_ERR_NOMEM);
  p->eng = e;
  *plan = p;
  return GABP_OK;
}

int gabp_plan_create_grid(const gabp_grid *A, const gabp_opts *o, gabp_plan **plan, hipStream_t s) {
  return with_account(plan, [&] { return plan_create_grid_impl(A, o, plan, s); });
}

int gabp_solve_grid(const gabp_grid *A, const double *b, double *x, double *marg_prec,
                    const gabp_opts *o, gabp_stats *st, hipStream_t s) {
  clear_stale_error();
  gabp_plan *p = nullptr;
  int rc = gabp_plan_create_grid(A, o, &p, s);
  if (rc) {
    if (st) { std::memset(st, 0, sizeof(*st)); st->status = rc; }
    return rc;
  }
  rc = gabp_plan_solve(p, b, x, marg_prec, st, s);
  gabp_plan_destroy(p);
  return rc;
}

int gabp_residual_grid(const gabp_grid *A, const double *b, const double *x, double *r,
                       double *rel_norm, hipStream_t s) {
  clear_stale_error();
  GridGeom g{};
  int rc = check_grid(A, &g);
  if (rc) return rc;
  if (!rel_norm || !b || !x) return GABP_ERR_ARG;
  const bool varc = grid_varc(A);
  GridCoef<double> k{};
  std::vector<double *> owned;
  if ((rc = expand_coefficients(A, g.N, &k, &owned))) {
    for (double *d : owned) dfree(d);
    return rc;
  }
  const int need = (g.N + kBlock - 1) / kBlock;
  const int nb = need < kMaxSweepBlocks ? need : kMaxSweepBlocks;
  double *sum = nullptr;
  HostReadout *host = nullptr;
  hipEvent_t ev = nullptr;
  auto cleanup = [&](int code) {
    if (sum) dfree(sum);
    for (double *d : owned) dfree(d);
    if (host) (void)hipHostFree(host);
    if (ev) (void)hipEventDestroy(ev);
    return code;
  };
  if ((rc = from_hip(dalloc(&sum, nb, sizeof(double)))) ||
      (rc = from_hip(hipHostMalloc((void **)&host, 2 * sizeof(HostReadout), hipHostMallocDefault))) ||
      (rc = from_hip(hipEventCreateWithFlags(&ev, hipEventDisableTiming))))
    return cleanup(rc);
  if ((rc = from_hip(launch_grid_residual(g, k, varc, nb, b, nullptr, nullptr, false, nullptr, sum, s))) ||
      (rc = from_hip(launch_readout(nullptr, 0, sum, nb, nullptr, nullptr, 0, 0, &host[0], s))) ||
      (rc = from_hip(launch_grid_residual(g, k, varc, nb, b, x, nullptr, false, r, sum, s))) ||
      (rc = from_hip(launch_readout(nullptr, 0, sum, nb, nullptr, nullptr, 0, 1, &host[1], s))) ||
      (rc = from_hip(hipEventRecord(ev, s))) || (rc = from_hip(hipEventSynchronize(ev))))
    return cleanup(rc);
  const double bn = std::sqrt(host[0].sum), rn = std::sqrt(host[1].sum);
  *rel_norm = bn > 0 ? rn / bn : rn;
  return cleanup(std::isfinite(*rel_norm) ? GABP_OK : GABP_ERR_ARG);
}

int gabp_plan_solve_coarse(gabp_plan *p, const double *b, double *x, double *marg_prec,
                           gabp_stats *st, hipStream_t s) {
  GABP_PLAN_SCOPE(p);
  clear_stale_error();
  if (!p || !p->eng) return GABP_ERR_ARG;
  return coarse_solve(p, b, x, marg_prec, st, s);
}

}  // extern "C"
