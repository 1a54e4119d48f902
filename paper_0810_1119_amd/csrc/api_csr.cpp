// Host side of the C ABI for general sparse matrices (include/gabp.h).
//
// A solve is a sequence of inner GaBP solves with FP64 refinement between
// them:
//   x = 0, r = b
//   repeat: sweeps from the current messages with right-hand side r until the
//           marginal means settle (device-side controller), then
//           x += H/S (FP64), r = b - A x (FP64), stop when ||r||/||b|| <= tol,
//           else zero every h (mean) message and keep every P message -- the
//           precision messages do not depend on the right-hand side
//           (Algorithm 1 never reads b in the P update).
// Sweeps are issued in chunks of `check_every` (even) launches, the last one
// also checking the means; a single-thread readout kernel decides on the
// device whether the inner solve is done and publishes its state to pinned
// host memory.  The host keeps two chunks in flight, so the GPU never waits
// for the host; chunks queued after the device decided to stop return at
// once.  In the pair layout, once the controller reports that every
// precision message has settled, the host switches to information-only
// sweeps (one freeze launch, then frozen chunks).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "gabp_internal.h"

using namespace gabp;

namespace {

constexpr int kRing = 4;       // readout slots / events in flight
constexpr int kLookahead = 2;  // chunks queued ahead of the one being read

int from_hip(hipError_t e) {
  if (e == hipSuccess) return GABP_OK;
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return GABP_ERR_NOMEM;
  return GABP_ERR_HIP;
}

#define TRY_HIP(expr)                          \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) return from_hip(_e); \
  } while (0)

template <typename P>
hipError_t dalloc(P **p, size_t count, size_t elem) {
  *p = nullptr;
  return hipMalloc((void **)p, std::max<size_t>(1, count) * elem);
}

// Lanes per row: about two lanes per edge of an average row (measured best on
// random graphs of mean degree 8: 16 lanes), at least 4, at most a wave.
int choose_group(int64_t n, int64_t E) {
  const double d = n > 0 ? (double)E / (double)n : 0.0;
  if (d < 3) return 4;
  if (d < 6) return 8;
  if (d < 12) return 16;
  if (d < 24) return 32;
  return 64;
}

bool valid_group(int g) { return g == 4 || g == 8 || g == 16 || g == 32 || g == 64; }

}  // namespace

struct gabp_plan {
  gabp_csr A{};
  gabp_opts o{};
  int32_t n = 0;
  int64_t E = 0;
  bool fp32 = true;
  bool pair = true;
  int group = 8;
  size_t tsz = 4;
  // graph
  int32_t *oprt = nullptr, *ocol = nullptr, *rev = nullptr;
  int64_t *diagpos = nullptr;
  void *acoef = nullptr, *diag = nullptr, *rhs = nullptr, *xprev = nullptr;
  // gather layout: (P, h) out-message per slot; pair layout: (P_ij, h_ij, P_ji, h_ji)
  void *msg[2] = {nullptr, nullptr};
  void *sums[2] = {nullptr, nullptr};  // pair: (S, H) per node
  // frozen phase (pair layout, allocated on first use)
  void *coef = nullptr, *hp[2] = {nullptr, nullptr}, *Sfix = nullptr, *Hfz[2] = {nullptr, nullptr};
  bool frozen = false;
  int cur = 0;
  double *sumpart = nullptr;
  int nres_blocks = 0;
  BlockPartial *part = nullptr;
  int nsweep_blocks = 0;
  uint32_t *sticky = nullptr;
  Ctl *ctl = nullptr;
  HostReadout *host = nullptr;
  hipEvent_t ev_beg[kRing] = {}, ev_end[kRing] = {}, ev_done[kRing] = {};
  bool events = false;
  int seq = 0;

  void release() {
    void *bufs[] = {oprt, ocol, rev, diagpos, acoef, diag, rhs, xprev, msg[0], msg[1],
                    sums[0], sums[1], coef, hp[0], hp[1], Sfix, Hfz[0], Hfz[1], sumpart,
                    part, sticky, ctl};
    for (void *b : bufs)
      if (b) (void)hipFree(b);
    if (host) (void)hipHostFree(host);
    if (events)
      for (int k = 0; k < kRing; ++k) {
        (void)hipEventDestroy(ev_beg[k]);
        (void)hipEventDestroy(ev_end[k]);
        (void)hipEventDestroy(ev_done[k]);
      }
  }

  size_t msg_bytes() const { return (pair ? 4 : 2) * tsz; }

  // one synchronous sweep from buffer cur into cur ^ 1
  hipError_t sweep(int mode, const Ctl *c, hipStream_t s) {
    hipError_t err;
    if (!pair) {
      SweepArgs a{};
      a.grid = nsweep_blocks;
      a.fp32 = fp32; a.group = group; a.mode = mode; a.damp = o.damping > 0.0; a.n = n;
      a.oprt = oprt; a.rev = rev; a.acoef = acoef; a.diag = diag; a.rhs = rhs;
      a.msg_in = msg[cur]; a.msg_out = msg[cur ^ 1]; a.alpha = o.damping; a.xprev = xprev;
      a.part = part; a.sticky = sticky; a.ctl = c;
      err = launch_sweep(a, s);
    } else {
      PairArgs a{};
      a.grid = nsweep_blocks;
      a.fp32 = fp32; a.group = group; a.mode = mode; a.damp = o.damping > 0.0; a.frozen = frozen;
      a.n = n; a.oprt = oprt; a.ocol = ocol; a.acoef = acoef; a.diag = diag; a.rhs = rhs;
      a.alpha = o.damping; a.xprev = xprev; a.part = part; a.sticky = sticky; a.ctl = c;
      if (frozen) {
        a.coef = coef; a.Sfix = Sfix;
        a.msg_in = hp[cur]; a.msg_out = hp[cur ^ 1]; a.sums_in = Hfz[cur]; a.sums_out = Hfz[cur ^ 1];
      } else {
        a.msg_in = msg[cur]; a.msg_out = msg[cur ^ 1]; a.sums_in = sums[cur]; a.sums_out = sums[cur ^ 1];
      }
      err = launch_pair_sweep(a, s);
    }
    cur ^= 1;
    return err;
  }

  // x += H/S and/or marginal precisions from the current state
  hipError_t infer(double *xacc, double *marg, hipStream_t s) {
    if (!pair) {
      SweepArgs a{};
      a.grid = nsweep_blocks;
      a.fp32 = fp32; a.group = group; a.mode = 2; a.n = n; a.oprt = oprt; a.rev = rev;
      a.acoef = acoef; a.diag = diag; a.rhs = rhs; a.msg_in = msg[cur]; a.xacc = xacc;
      a.marg = marg; a.sticky = sticky;
      return launch_sweep(a, s);
    }
    if (frozen) return launch_pair_infer(fp32, n, nullptr, Sfix, Hfz[cur], xacc, marg, sticky, s);
    return launch_pair_infer(fp32, n, sums[cur], nullptr, nullptr, xacc, marg, sticky, s);
  }

  // zero every mean message, keep the precisions; rhs must already hold r
  hipError_t restart(hipStream_t s) {
    if (!pair) return launch_zero_h(fp32, E, msg[cur], s);
    if (frozen) return launch_frozen_restart(fp32, E, n, hp[cur], rhs, Hfz[cur], s);
    hipError_t err = launch_pair_zero_h(fp32, E, msg[cur], s);
    if (err != hipSuccess) return err;
    return launch_pair_aggregate(fp32, group, nsweep_blocks, n, oprt, diag, rhs, msg[cur], sums[cur], s);
  }

  // zero messages, rhs = b (and ||b||^2 into the residual partials), full state
  hipError_t reset(const double *b, hipStream_t s) {
    cur = 0;
    frozen = false;
    const int64_t words = E * (int64_t)msg_bytes() / 8;
    hipError_t err;
    if ((err = launch_fill_zero(msg[0], words, s)) != hipSuccess) return err;
    if ((err = launch_fill_zero(msg[1], words, s)) != hipSuccess) return err;
    if ((err = launch_fill_zero4(sticky, 1, s)) != hipSuccess) return err;
    if ((err = launch_residual(fp32, group, nres_blocks, n, A.row_ptr, A.col, A.val, b, nullptr, rhs, nullptr,
                               sumpart, s)) != hipSuccess)
      return err;
    if (pair) return launch_pair_aggregate(fp32, group, nsweep_blocks, n, oprt, diag, rhs, msg[0], sums[0], s);
    return hipSuccess;
  }

  // allocates whichever frozen-phase buffer is still missing
  hipError_t ensure_frozen_buffers() {
    struct { void **p; size_t count, elem; } need[] = {
        {&coef, (size_t)E, 2 * tsz}, {&hp[0], (size_t)E, 2 * tsz}, {&hp[1], (size_t)E, 2 * tsz},
        {&Sfix, (size_t)n, tsz},     {&Hfz[0], (size_t)n, tsz},    {&Hfz[1], (size_t)n, tsz}};
    for (auto &b : need)
      if (!*b.p) {
        hipError_t err = dalloc(b.p, b.count, b.elem);
        if (err != hipSuccess) return err;
      }
    return hipSuccess;
  }
  bool frozen_ready() const { return coef && hp[0] && hp[1] && Sfix && Hfz[0] && Hfz[1]; }

  hipError_t freeze(hipStream_t s) {
    hipError_t err = launch_pair_freeze(fp32, group, nsweep_blocks, n, oprt, ocol, acoef, msg[cur], sums[cur],
                                        coef, hp[cur], Sfix, Hfz[cur], s);
    frozen = true;
    return err;
  }

  // readout without a check: residual sums only; waits
  int read_sum(hipStream_t s, HostReadout *outv) {
    const int slot = 0;
    TRY_HIP(launch_readout(nullptr, 0, sumpart, nres_blocks, sticky, ctl, 0, ++seq, &host[slot], s));
    TRY_HIP(hipEventRecord(ev_done[slot], s));
    TRY_HIP(hipEventSynchronize(ev_done[slot]));
    *outv = host[slot];
    return GABP_OK;
  }
};

extern "C" {

const char *gabp_version(void) { return "gabp-mi355x 0.2 (gfx950)"; }

void gabp_default_opts(gabp_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->msg_fp32 = 1;
  o->tol = 1e-8;
  o->max_sweeps = 20000;
  o->check_every = 2;
  o->damping = 0.0;
  o->inner_tol = 0.0;
  o->max_restarts = 30;
  o->group = 0;
  o->layout = GABP_LAYOUT_PAIR;
  o->freeze = 1;
}

static int check_csr(const gabp_csr *A) {
  if (!A || A->n < 0 || A->nnz < 0) return GABP_ERR_ARG;
  if (A->n > 0 && (!A->row_ptr || !A->col || !A->val)) return GABP_ERR_ARG;
  if (A->n == 0) return GABP_OK;
  int64_t ends[2];
  if (hipMemcpy(&ends[0], A->row_ptr, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&ends[1], A->row_ptr + A->n, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
    return GABP_ERR_ARG;
  if (ends[0] != 0 || ends[1] != A->nnz) return GABP_ERR_ARG;
  return GABP_OK;
}

static int check_opts(const gabp_opts *o) {
  if (!(o->tol >= 0.0) || o->max_sweeps < 0 || o->check_every < 1 || !(o->damping >= 0.0) ||
      !(o->damping < 1.0) || !(o->inner_tol >= 0.0) || o->max_restarts < 0 ||
      (o->group != 0 && !valid_group(o->group)) || o->grid_blocks < 0 ||
      (o->layout != GABP_LAYOUT_PAIR && o->layout != GABP_LAYOUT_GATHER))
    return GABP_ERR_ARG;
  return GABP_OK;
}

static int plan_build(gabp_plan *p, hipStream_t s) {
  const int n = p->n;
  const gabp_csr &A = p->A;
  int64_t *deg = nullptr, *oprt64 = nullptr, *tmp = nullptr;
  uint32_t *flags = nullptr;
  int st = GABP_OK;
  auto fail = [&](int code) {
    void *bufs[] = {deg, oprt64, tmp, flags};
    for (void *b : bufs)
      if (b) (void)hipFree(b);
    return code;
  };
  if ((st = from_hip(dalloc(&deg, n, sizeof(int64_t)))) ||
      (st = from_hip(dalloc(&p->diagpos, n, sizeof(int64_t)))) ||
      (st = from_hip(dalloc(&oprt64, n + 1, sizeof(int64_t)))) ||
      (st = from_hip(dalloc(&tmp, scan_tmp_elems(n), sizeof(int64_t)))) ||
      (st = from_hip(dalloc(&flags, 1, sizeof(uint32_t)))))
    return fail(st);
  if ((st = from_hip(launch_fill_zero4(flags, 1, s))) ||
      (st = from_hip(launch_plan_rows(n, A.nnz, A.row_ptr, A.col, A.val, deg, p->diagpos, flags, s))))
    return fail(st);
  uint32_t hflags = 0;
  if ((st = from_hip(hipMemcpyAsync(&hflags, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s))) ||
      (st = from_hip(hipStreamSynchronize(s))))
    return fail(st);
  if (hflags & FLAG_ARG) return fail(GABP_ERR_ARG);
  if (hflags & FLAG_ZERO_DIAG) return fail(GABP_ERR_ZERO_DIAG);
  if ((st = from_hip(launch_scan(deg, oprt64, n, tmp, s)))) return fail(st);
  int64_t E = 0;
  if ((st = from_hip(hipMemcpyAsync(&E, oprt64 + n, sizeof(int64_t), hipMemcpyDeviceToHost, s))) ||
      (st = from_hip(hipStreamSynchronize(s))))
    return fail(st);
  if (E >= (int64_t)INT32_MAX) return fail(GABP_ERR_UNSUPPORTED);
  p->E = E;
  if ((st = from_hip(dalloc(&p->oprt, n + 1, sizeof(int32_t)))) ||
      (st = from_hip(dalloc(&p->ocol, E, sizeof(int32_t)))) ||
      (st = from_hip(dalloc(&p->rev, E, sizeof(int32_t)))) ||
      (st = from_hip(dalloc(&p->acoef, E, p->tsz))) ||
      (st = from_hip(dalloc(&p->diag, n, p->tsz))))
    return fail(st);
  if ((st = from_hip(launch_plan_edges(p->fp32, n, A.row_ptr, A.col, A.val, p->diagpos, oprt64,
                                       p->oprt, p->ocol, p->rev, p->acoef, p->diag, flags, s))))
    return fail(st);
  if ((st = from_hip(hipMemcpyAsync(&hflags, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s))) ||
      (st = from_hip(hipStreamSynchronize(s))))
    return fail(st);
  if (hflags & FLAG_ASYM) return fail(GABP_ERR_NOT_SYMMETRIC);
  return fail(GABP_OK);
}

int gabp_plan_create(const gabp_csr *A, const gabp_opts *o, gabp_plan **plan, hipStream_t s) {
  if (!plan) return GABP_ERR_ARG;
  *plan = nullptr;
  gabp_opts opts;
  if (o) opts = *o;
  else gabp_default_opts(&opts);
  int st = check_csr(A);
  if (st) return st;
  if ((st = check_opts(&opts))) return st;
  gabp_plan *p = new (std::nothrow) gabp_plan();
  if (!p) return GABP_ERR_NOMEM;
  p->A = *A;
  p->o = opts;
  p->n = A->n;
  p->fp32 = opts.msg_fp32 != 0;
  p->pair = opts.layout == GABP_LAYOUT_PAIR;
  p->tsz = p->fp32 ? sizeof(float) : sizeof(double);
  auto fail = [&](int code) {
    p->release();
    delete p;
    return code;
  };
  if (p->n > 0 && (st = plan_build(p, s))) return fail(st);
  p->group = opts.group ? opts.group : choose_group(p->n, p->E);
  const int cap = opts.grid_blocks > 0 ? opts.grid_blocks : kMaxSweepBlocks;
  p->nres_blocks = residual_blocks(std::max(p->n, 1), p->group, cap);
  p->nsweep_blocks = sweep_blocks(std::max(p->n, 1), p->group, cap);
  if ((st = from_hip(dalloc(&p->msg[0], p->E, p->msg_bytes()))) ||
      (st = from_hip(dalloc(&p->msg[1], p->E, p->msg_bytes()))) ||
      (st = from_hip(dalloc(&p->rhs, p->n, p->tsz))) ||
      (st = from_hip(dalloc(&p->xprev, p->n, p->tsz))) ||
      (st = from_hip(dalloc(&p->sumpart, p->nres_blocks, sizeof(double)))) ||
      (st = from_hip(dalloc(&p->part, p->nsweep_blocks, sizeof(BlockPartial)))) ||
      (st = from_hip(dalloc(&p->sticky, 1, sizeof(uint32_t)))) ||
      (st = from_hip(dalloc(&p->ctl, 1, sizeof(Ctl)))))
    return fail(st);
  if (p->pair && ((st = from_hip(dalloc(&p->sums[0], p->n, 2 * p->tsz))) ||
                  (st = from_hip(dalloc(&p->sums[1], p->n, 2 * p->tsz)))))
    return fail(st);
  if ((st = from_hip(hipHostMalloc((void **)&p->host, kRing * sizeof(HostReadout), hipHostMallocDefault))))
    return fail(st);
  for (int k = 0; k < kRing; ++k) {
    if ((st = from_hip(hipEventCreate(&p->ev_beg[k]))) || (st = from_hip(hipEventCreate(&p->ev_end[k]))) ||
        (st = from_hip(hipEventCreateWithFlags(&p->ev_done[k], hipEventDisableTiming)))) {
      for (int j = 0; j <= k; ++j) {
        if (p->ev_beg[j]) (void)hipEventDestroy(p->ev_beg[j]);
        if (p->ev_end[j]) (void)hipEventDestroy(p->ev_end[j]);
        if (p->ev_done[j]) (void)hipEventDestroy(p->ev_done[j]);
      }
      return fail(st);
    }
  }
  p->events = true;
  *plan = p;
  return GABP_OK;
}

int gabp_plan_destroy(gabp_plan *p) {
  if (!p) return GABP_ERR_ARG;
  (void)hipDeviceSynchronize();
  p->release();
  delete p;
  return GABP_OK;
}

int gabp_plan_reset(gabp_plan *p, const double *b, hipStream_t s) {
  if (!p || (p->n > 0 && !b)) return GABP_ERR_ARG;
  if (p->n == 0) return GABP_OK;
  TRY_HIP(p->reset(b, s));
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int gabp_plan_sweeps(gabp_plan *p, int32_t count, hipStream_t s) {
  if (!p || count < 0) return GABP_ERR_ARG;
  if (p->frozen) return GABP_ERR_ARG;  // trajectory access needs the full state (reset first)
  for (int k = 0; k < count && p->n > 0; ++k) TRY_HIP(p->sweep(0, nullptr, s));
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int gabp_plan_marginals(gabp_plan *p, double *mean, double *prec, hipStream_t s) {
  if (!p || (p->n > 0 && !mean)) return GABP_ERR_ARG;
  if (p->n == 0) return GABP_OK;
  TRY_HIP(launch_fill_zero(mean, p->n, s));
  TRY_HIP(p->infer(mean, prec, s));
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int gabp_plan_get_messages(gabp_plan *p, double *P, double *h, hipStream_t s) {
  if (!p || (p->A.nnz > 0 && (!P || !h)) || p->frozen) return GABP_ERR_ARG;
  if (p->pair)
    TRY_HIP(launch_pair_io(p->fp32, true, p->n, p->A.row_ptr, p->diagpos, p->oprt, p->rev,
                           p->msg[p->cur], P, h, s));
  else
    TRY_HIP(launch_get_msgs(p->fp32, p->n, p->A.row_ptr, p->diagpos, p->oprt, p->msg[p->cur], P, h, s));
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int gabp_plan_set_messages(gabp_plan *p, const double *P, const double *h, hipStream_t s) {
  if (!p || (p->A.nnz > 0 && (!P || !h)) || p->frozen) return GABP_ERR_ARG;
  if (p->pair) {
    TRY_HIP(launch_pair_io(p->fp32, false, p->n, p->A.row_ptr, p->diagpos, p->oprt, p->rev,
                           p->msg[p->cur], (double *)P, (double *)h, s));
    TRY_HIP(launch_pair_aggregate(p->fp32, p->group, p->nsweep_blocks, p->n, p->oprt, p->diag, p->rhs,
                                  p->msg[p->cur], p->sums[p->cur], s));
  } else {
    TRY_HIP(launch_set_msgs(p->fp32, p->n, p->A.row_ptr, p->diagpos, p->oprt, p->msg[p->cur], P, h, s));
  }
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int gabp_plan_solve(gabp_plan *p, const double *b, double *x, double *marg_prec, gabp_stats *st,
                    hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!p || (p->n > 0 && (!b || !x))) return GABP_ERR_ARG;
  gabp_stats stats{};
  stats.edges = p->E;
  stats.status = GABP_OK;
  const gabp_opts &o = p->o;
  auto finish = [&](int status) {
    stats.status = status;
    stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats.edge_updates_per_s =
        stats.seconds > 0 ? (double)stats.edges * stats.sweeps / stats.seconds : 0.0;
    if (st) *st = stats;
    return status;
  };
  if (p->n == 0) return finish(GABP_OK);

  const int c = std::max(2, o.check_every + (o.check_every & 1));  // even: buffer parity kept
  // Inner targets: the first pass runs to the message precision's floor (or
  // to 0.3 tol if that is coarser); later passes only need the remaining
  // factor tol / rel, with the same margin.  inner_tol > 0 fixes the target.
  const double floor = p->fp32 ? 1e-6 : 1e-14;
  // The freeze takes effect a few sweeps after the check that allows it (the
  // chunks already queued still run full sweeps), so the precisions keep
  // settling in between; 1e-6 leaves them at FP32 resolution by then on the
  // workloads measured, and the FP64 refinement absorbs any remainder.
  const double freeze_tol = (p->pair && o.freeze) ? (p->fp32 ? 1e-6 : 1e-14) : -1.0;
  auto target_for = [&](double rel) {
    if (o.inner_tol > 0) return o.inner_tol;
    return std::min(0.5, std::max(0.3 * o.tol / rel, p->fp32 ? 1e-7 : 1e-15));
  };
  if (freeze_tol > 0) TRY_HIP(p->ensure_frozen_buffers());
  TRY_HIP(p->reset(b, s));  // also computes ||b||^2 into the residual partials
  if (p->fp32) TRY_HIP(launch_fill_zero4(p->xprev, p->n, s));
  else TRY_HIP(launch_fill_zero(p->xprev, p->n, s));
  TRY_HIP(launch_fill_zero(x, p->n, s));
  TRY_HIP(launch_ctl_reset(p->ctl, target_for(1.0), floor, freeze_tol, true, s));
  HostReadout r0;
  int rc = p->read_sum(s, &r0);
  if (rc) return finish(rc);
  if (!std::isfinite(r0.sum)) return finish(GABP_ERR_ARG);
  const double bn = std::sqrt(r0.sum);
  if (bn == 0.0) {
    stats.rel_residual = 0.0;
    if (marg_prec) {
      TRY_HIP(p->infer(nullptr, marg_prec, s));
      TRY_HIP(hipStreamSynchronize(s));
    }
    return finish(GABP_OK);
  }

  int status = GABP_NOT_CONVERGED;
  int sweeps_done = 0;
  double rel_prev = 1.0;
  for (int pass = 0;; ++pass) {
    if (pass > 0) TRY_HIP(launch_ctl_reset(p->ctl, target_for(rel_prev), floor, freeze_tol, false, s));
    // ---- inner solve: chunks of c sweeps, lookahead, device-side stop ----
    const int budget = o.max_sweeps - sweeps_done;
    int enq = 0, rd = 0, enq_sweeps = 0, last_sweeps = sweeps_done;
    bool stopped = false, want_freeze = false;
    bool chunk_frozen[kRing] = {};
    while (true) {
      while (!stopped && enq - rd < kLookahead && enq_sweeps < budget) {
        const int slot = enq % kRing;
        if (want_freeze && !p->frozen && freeze_tol > 0 && p->pair && p->frozen_ready())
          TRY_HIP(p->freeze(s));
        chunk_frozen[slot] = p->frozen;
        for (int k = 0; k < c; ++k) {
          if (k == 0) TRY_HIP(hipEventRecord(p->ev_beg[slot], s));
          TRY_HIP(p->sweep(k == c - 1 ? 1 : 0, p->ctl, s));
        }
        TRY_HIP(hipEventRecord(p->ev_end[slot], s));
        TRY_HIP(launch_readout(p->part, p->nsweep_blocks, nullptr, 0, p->sticky, p->ctl, c, enq,
                               &p->host[slot], s));
        TRY_HIP(hipEventRecord(p->ev_done[slot], s));
        ++enq;
        enq_sweeps += c;
      }
      if (rd == enq) break;
      const int slot = rd % kRing;
      TRY_HIP(hipEventSynchronize(p->ev_done[slot]));
      const HostReadout h = p->host[slot];
      if (h.seq != rd) return finish(GABP_ERR_HIP);
      stats.checks += 1;
      if (h.sweeps > last_sweeps) {  // this chunk ran (not skipped)
        float ms = 0.f;
        TRY_HIP(hipEventElapsedTime(&ms, p->ev_beg[slot], p->ev_end[slot]));
        stats.sweep_ms += ms;
        if (chunk_frozen[slot]) {
          stats.frozen_sweeps += h.sweeps - last_sweeps;
          stats.frozen_sweep_ms += ms;
        }
        last_sweeps = h.sweeps;
      }
      if (h.freeze) want_freeze = true;
      ++rd;
      if (h.stop != STOP_NONE) stopped = true;
      if (stopped && rd < enq) {
        // drain: the remaining queued chunks are no-ops on the device
        TRY_HIP(hipEventSynchronize(p->ev_done[(enq - 1) % kRing]));
        rd = enq;
      }
    }
    sweeps_done = last_sweeps;
    stats.sweeps = sweeps_done;
    // ---- x += H/S, r = b - A x (FP64), ||r|| ----
    TRY_HIP(p->infer(x, nullptr, s));
    TRY_HIP(launch_residual(p->fp32, p->group, p->nres_blocks, p->n, p->A.row_ptr, p->A.col, p->A.val, b, x,
                            p->rhs, nullptr, p->sumpart, s));
    HostReadout rr;
    if ((rc = p->read_sum(s, &rr))) return finish(rc);
    const double rel = std::sqrt(rr.sum) / bn;
    rel_prev = rel;
    stats.rel_residual = rel;
    stats.residual_per_eq = std::sqrt(rr.sum) / p->n;
    if (rr.flags & FLAG_BREAKDOWN) { status = GABP_ERR_BREAKDOWN; break; }
    if ((rr.flags & FLAG_NONFINITE) || !std::isfinite(rel) || rel > 1e6) {
      status = GABP_ERR_DIVERGED;
      break;
    }
    if (rel <= o.tol) { status = GABP_OK; break; }
    if (stats.restarts >= o.max_restarts || sweeps_done >= o.max_sweeps) {
      status = GABP_NOT_CONVERGED;
      break;
    }
    // restart: zero the mean messages, keep the precision messages
    TRY_HIP(p->restart(s));
    stats.restarts += 1;
  }
  if (marg_prec) TRY_HIP(p->infer(nullptr, marg_prec, s));
  TRY_HIP(hipStreamSynchronize(s));
  return finish(status);
}

int gabp_solve(const gabp_csr *A, const double *b, double *x, double *marg_prec,
               const gabp_opts *o, gabp_stats *st, hipStream_t s) {
  gabp_plan *p = nullptr;
  int rc = gabp_plan_create(A, o, &p, s);
  if (rc) {
    if (st) { std::memset(st, 0, sizeof(*st)); st->status = rc; }
    return rc;
  }
  rc = gabp_plan_solve(p, b, x, marg_prec, st, s);
  gabp_plan_destroy(p);
  return rc;
}

int gabp_residual(const gabp_csr *A, const double *b, const double *x, double *r,
                  double *rel_norm, hipStream_t s) {
  int rc = check_csr(A);
  if (rc) return rc;
  if (!rel_norm || (A->n > 0 && (!b || !x))) return GABP_ERR_ARG;
  if (A->n == 0) { *rel_norm = 0.0; return GABP_OK; }
  const int64_t nnzE = A->nnz - A->n;
  const int g = choose_group(A->n, std::max<int64_t>(0, nnzE));
  const int nb = residual_blocks(A->n, g);
  double *sum = nullptr;
  int64_t *deg = nullptr, *dpos = nullptr;
  uint32_t *flags = nullptr;
  HostReadout *host = nullptr;
  hipEvent_t ev = nullptr;
  auto cleanup = [&](int code) {
    void *bufs[] = {sum, deg, dpos, flags};
    for (void *b : bufs)
      if (b) (void)hipFree(b);
    if (host) (void)hipHostFree(host);
    if (ev) (void)hipEventDestroy(ev);
    return code;
  };
  if ((rc = from_hip(dalloc(&sum, nb, sizeof(double)))) ||
      (rc = from_hip(hipHostMalloc((void **)&host, 2 * sizeof(HostReadout), hipHostMallocDefault))) ||
      (rc = from_hip(hipEventCreateWithFlags(&ev, hipEventDisableTiming))) ||
      (rc = from_hip(dalloc(&deg, A->n, sizeof(int64_t)))) ||
      (rc = from_hip(dalloc(&dpos, A->n, sizeof(int64_t)))) ||
      (rc = from_hip(dalloc(&flags, 1, sizeof(uint32_t)))))
    return cleanup(rc);
  // column range and ordering are validated before any x[col] gather
  uint32_t hflags = 0;
  if ((rc = from_hip(launch_fill_zero4(flags, 1, s))) ||
      (rc = from_hip(launch_plan_rows(A->n, A->nnz, A->row_ptr, A->col, A->val, deg, dpos, flags, s))) ||
      (rc = from_hip(hipMemcpyAsync(&hflags, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s))) ||
      (rc = from_hip(hipStreamSynchronize(s))))
    return cleanup(rc);
  if (hflags & FLAG_ARG) return cleanup(GABP_ERR_ARG);
  if ((rc = from_hip(launch_residual(false, g, nb, A->n, A->row_ptr, A->col, A->val, b, nullptr,
                                     nullptr, nullptr, sum, s))) ||
      (rc = from_hip(launch_readout(nullptr, 0, sum, nb, nullptr, nullptr, 0, 0, &host[0], s))) ||
      (rc = from_hip(launch_residual(false, g, nb, A->n, A->row_ptr, A->col, A->val, b, x, nullptr, r,
                                     sum, s))) ||
      (rc = from_hip(launch_readout(nullptr, 0, sum, nb, nullptr, nullptr, 0, 1, &host[1], s))) ||
      (rc = from_hip(hipEventRecord(ev, s))) || (rc = from_hip(hipEventSynchronize(ev))))
    return cleanup(rc);
  const double bn = std::sqrt(host[0].sum), rn = std::sqrt(host[1].sum);
  *rel_norm = bn > 0 ? rn / bn : rn;
  return cleanup(std::isfinite(*rel_norm) ? GABP_OK : GABP_ERR_ARG);
}

}  // extern "C"
