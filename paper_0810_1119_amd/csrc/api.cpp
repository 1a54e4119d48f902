// C ABI entry points shared by every matrix kind, and the solve loop.
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
// Sweeps are issued in chunks of `check_every` (even) sweeps, or of a length
// that grows with the pass (check_every = 0), the last one also checking the
// means; a single-thread readout kernel decides on the
// device whether the inner solve is done and publishes its state to pinned
// host memory.  The host keeps two chunks in flight, so the GPU never waits
// for the host; chunks queued after the device decided to stop return at
// once.  When the engine supports it and the controller reports that every
// precision message has settled, the host switches to information-only
// sweeps (one freeze launch, then frozen chunks).
#include <chrono>
#include <cmath>
#include <cstring>

#include "engine.h"

#include <cstdio>
#include <cstdlib>

namespace gabp {

void report_hip(hipError_t e, const char *file, int line) {
  static const bool on = std::getenv("GABP_VERBOSE") != nullptr;
  if (on) std::fprintf(stderr, "gabp: %s (%d) at %s:%d\n", hipGetErrorName(e), (int)e, file, line);
}

Engine::~Engine() {
  void *bufs[] = {part, sumpart, sticky, ctl, xprev, segb2, segctl, segact};
  for (void *b : bufs)
    if (b) dfree(b);
  if (host) (void)hipHostFree(host);
  if (events)
    for (int k = 0; k < kRing; ++k) {
      (void)hipEventDestroy(ev_beg[k]);
      (void)hipEventDestroy(ev_end[k]);
    }
  if (ev_sum) (void)hipEventDestroy(ev_sum);
}

int Engine::init_common(hipStream_t s) {
  int st;
  // check partials start cleared (slot_publish raises them atomically; the
  // readout clears them again)
  if ((st = from_hip(dalloc(&part, nparts, sizeof(BlockPartial)))) ||
      (st = from_hip(launch_fill_zero(part, (int64_t)std::max(nparts, 1) * 4, s))) ||
      (st = from_hip(dalloc(&sumpart, nsum, sizeof(double)))) ||
      (st = from_hip(dalloc(&sticky, 1, sizeof(uint32_t)))) ||
      (st = from_hip(dalloc(&ctl, 1, sizeof(Ctl)))) ||
      (st = from_hip(dalloc(&xprev, means_slots(), tsz))))
    return st;
  if (nseg > 1 && (st = from_hip(dalloc(&segb2, nseg, sizeof(double))))) return st;
  // zeroed: an empty list of sweeping segments until a solve fills it
  if (segctl_wanted && ((st = from_hip(dalloc(&segctl, nseg, sizeof(SegCtl)))) ||
                        (st = from_hip(dalloc(&segact, nseg + 1, sizeof(int32_t)))) ||
                        (st = from_hip(launch_fill_zero(segctl, nseg * (int64_t)sizeof(SegCtl) / 8, s))) ||
                        (st = from_hip(launch_fill_zero4(segact, nseg + 1, s)))))
    return st;
  // kRing chunk readouts and one slot for the residual sums
  // coherent, so that the host can watch a readout's sequence number arrive
  if ((st = from_hip(hipHostMalloc((void **)&host, (kRing + 1) * sizeof(HostReadout),
                                   hipHostMallocCoherent))) ||
      (st = from_hip(hipEventCreateWithFlags(&ev_sum, hipEventDisableTiming))))
    return st;
  for (int k = 0; k < kRing; ++k) {
    // timing only: no system-scope fence (cache writeback and invalidation)
    // when these are recorded between the sweeps and the readout
    if ((st = from_hip(hipEventCreateWithFlags(&ev_beg[k], hipEventDisableSystemFence))) ||
        (st = from_hip(hipEventCreateWithFlags(&ev_end[k], hipEventDisableSystemFence)))) {
      for (int j = 0; j <= k; ++j) {
        if (ev_beg[j]) (void)hipEventDestroy(ev_beg[j]);
        if (ev_end[j]) (void)hipEventDestroy(ev_end[j]);
        ev_beg[j] = ev_end[j] = nullptr;
      }
      return st;
    }
  }
  events = true;
  return GABP_OK;
}

int Engine::post_sum(hipStream_t s, int seg_mode, double bnorm) {
  TRY_HIP(launch_readout(nullptr, 0, sumpart, nsum, sticky, ctl, 0, ++seq, &host[kRing], s));
  if (nseg > 1 && seg_mode > 0)
    TRY_HIP(launch_seg_norms(sumpart, nseg, segb, segb2, seg_mode == 1, bnorm, &host[kRing], s,
                             segctl, segact, o.tol, inner_floor(), o.inner_tol));
  TRY_HIP(hipEventRecord(ev_sum, s));
  return GABP_OK;
}

int Engine::wait_sum(HostReadout *outv) {
  TRY_HIP(hipEventSynchronize(ev_sum));
  *outv = host[kRing];
  return GABP_OK;
}

// Wait until the readout with sequence number `want` has arrived in slot h:
// watch its sequence number (written last by the readout kernel), asking the
// stream now and then whether it failed or went idle without delivering it.
static int wait_readout(const HostReadout *h, int want, hipStream_t s) {
  for (uint32_t k = 1;; ++k) {
    if (__atomic_load_n(&h->seq, __ATOMIC_ACQUIRE) == want) return GABP_OK;
    if ((k & 1023u) == 0) {
      const hipError_t e = hipStreamQuery(s);
      if (e == hipSuccess) {  // idle: the readout has run
        return __atomic_load_n(&h->seq, __ATOMIC_ACQUIRE) == want ? GABP_OK : GABP_ERR_HIP;
      }
      if (e != hipErrorNotReady) return from_hip(e);
    }
  }
}

int Engine::read_sum(hipStream_t s, HostReadout *outv, int seg_mode, double bnorm) {
  const int rc = post_sum(s, seg_mode, bnorm);
  return rc ? rc : wait_sum(outv);
}

int engine_solve(Engine *p, const double *b, double *x, double *marg_prec, gabp_stats *st,
                 hipStream_t s, const uint16_t *warm) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!p || (p->n > 0 && (!b || !x))) return GABP_ERR_ARG;
  gabp_stats stats{};
  int64_t seg_sweeps = 0, frozen_seg_sweeps = 0;  // sweeps summed over the segments that ran them
  stats.edges = p->E;
  stats.sweep_launches = p->sweep_launches();
  stats.damping = p->o.damping;
  stats.status = GABP_OK;
  const gabp_opts &o = p->o;
  auto finish = [&](int status) {
    stats.status = status;
    stats.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    stats.mean_sweeps = p->segctl ? (double)seg_sweeps / p->nseg : (double)stats.sweeps;
    stats.mean_frozen_sweeps =
        p->segctl ? (double)frozen_seg_sweeps / p->nseg : (double)stats.frozen_sweeps;
    stats.edge_updates_per_s =
        stats.seconds > 0 ? (double)stats.edges * stats.mean_sweeps / stats.seconds : 0.0;
    if (st) *st = stats;
    return status;
  };
  if (p->n == 0) return finish(GABP_OK);

  // Sweeps per chunk, even (the double buffers' parity is kept): the option
  // rounded up, or with 0 a length that grows with the pass's sweeps: a check
  // sweep costs more than a plain one (the previous means are read and
  // written, the check maxima published) and each chunk adds a readout, so
  // long passes check less often; 8 sweeps later than needed is little next
  // to hundreds, while short passes keep checking every 2.
  auto chunk_len = [&](int pass_sweeps) {
    if (o.check_every > 0) return std::max(2, o.check_every + (o.check_every & 1));
    return pass_sweeps < 64 ? 2 : pass_sweeps < 256 ? 4 : 8;
  };
  // Inner targets: the first pass runs to the message precision's floor (or
  // to 0.3 tol if that is coarser); later passes only need the remaining
  // factor tol / rel, with the same margin.  inner_tol > 0 fixes the target.
  const double floor = p->fp32 ? 1e-6 : 1e-14;
  // The freeze takes effect a few sweeps after the check that allows it (the
  // chunks already queued still run full sweeps), so the precisions keep
  // settling in between; 1e-6 leaves them at FP32 resolution by then on the
  // workloads measured, and the FP64 refinement absorbs any remainder.
  const bool freezing = o.freeze && p->can_freeze();
  const double freeze_tol =
      freezing ? (o.freeze_tol > 0.0 ? o.freeze_tol : (p->fp32 ? 1e-6 : 1e-14)) : -1.0;
  auto target_for = [&](double rel) {
    if (o.inner_tol > 0) return o.inner_tol;
    return std::min(0.5, std::max(0.3 * o.tol / rel, p->inner_floor()));
  };
  if (freezing) TRY_HIP(p->ensure_frozen_buffers());
  TRY_HIP(launch_fill_zero4(p->sticky, 1, s));
  TRY_HIP(launch_fill_zero(p->part, (int64_t)std::max(p->nparts, 1) * 4, s));  // no stale check maxima
  TRY_HIP(p->reset(b, s));  // also computes ||b||^2 into the residual partials
  if (p->fp32) TRY_HIP(launch_fill_zero4(p->xprev, p->means_slots(), s));
  else TRY_HIP(launch_fill_zero(p->xprev, p->means_slots(), s));
  TRY_HIP(launch_fill_zero(x, p->n, s));
  TRY_HIP(launch_ctl_reset(p->ctl, target_for(1.0), floor, freeze_tol, true, 0, s));
  // ||b||: a plain solve reads it back after the first pass's sweeps, which
  // then need not wait for it (x is untouched until then; a zero b converges
  // at the first check, a non-finite one stops it); a warm start and the
  // marginals of a zero b need it now
  int rc = p->post_sum(s, 1);
  if (rc) return finish(rc);
  double bn = -1.0;
  auto take_bn = [&]() -> int {
    HostReadout r0;
    const int e = p->wait_sum(&r0);
    if (e) return e;
    if (!std::isfinite(r0.sum)) return GABP_ERR_ARG;
    bn = std::sqrt(r0.sum);
    return GABP_OK;
  };
  auto zero_b = [&]() {
    stats.rel_residual = 0.0;
    if (marg_prec) {
      TRY_HIP(p->infer(nullptr, marg_prec, nullptr, s));
      TRY_HIP(hipStreamSynchronize(s));
    }
    return finish(GABP_OK);
  };
  if (warm || marg_prec) {
    if ((rc = take_bn())) return finish(rc);
    if (bn == 0.0) return zero_b();
  }

  if (warm) {
    // Messages from the warm-start network.  They are kept only if the means
    // they imply fit b better than x = 0 does; otherwise the solve starts
    // from zero messages as Algorithm 1 does.
    TRY_HIP(p->warm_start(warm, s));
    TRY_HIP(p->infer(x, nullptr, nullptr, s));
    TRY_HIP(p->residual(b, x, nullptr, s));
    HostReadout rw;
    if ((rc = p->read_sum(s, &rw))) return finish(rc);
    const double rel0 = std::sqrt(rw.sum) / bn;
    TRY_HIP(launch_fill_zero(x, p->n, s));
    if (rel0 <= 1.0 && !(rw.flags & (FLAG_NONFINITE | FLAG_BREAKDOWN))) {
      TRY_HIP(p->residual(b, x, nullptr, s));  // right-hand side back to b (x = 0)
      stats.warm_start = 1;
    } else {
      TRY_HIP(launch_fill_zero4(p->sticky, 1, s));
      TRY_HIP(p->reset(b, s));
      stats.warm_start = -1;
    }
    stats.warm_rel0 = rel0;
  }

  int status = GABP_NOT_CONVERGED;
  int sweeps_done = 0;
  double rel_prev = 1.0;
  for (int pass = 0;; ++pass) {
    if (pass > 0) TRY_HIP(launch_ctl_reset(p->ctl, target_for(rel_prev), floor, freeze_tol, false, 0, s));
    // the first check of the pass measures its change from these means (the
    // messages the pass starts from), not from those of another right-hand side
    TRY_HIP(p->infer(nullptr, nullptr, p->xprev, s));
    // ---- inner solve: chunks of c sweeps, lookahead, device-side stop ----
    const int budget = o.max_sweeps - sweeps_done;
    int enq = 0, rd = 0, enq_sweeps = 0, last_sweeps = sweeps_done;
    bool stopped = false, want_freeze = false;
    bool chunk_frozen[kRing] = {};
    int slot_seq[kRing] = {};
    while (true) {
      while (!stopped && enq - rd < kLookahead && enq_sweeps < budget) {
        const int slot = enq % kRing;
        const int c = chunk_len(enq_sweeps);
        if (want_freeze && !p->frozen && freezing && p->frozen_ready()) TRY_HIP(p->freeze(s));
        chunk_frozen[slot] = p->frozen;
        for (int k = 0; k < c; ++k) {
          if (k == 0) TRY_HIP(hipEventRecord(p->ev_beg[slot], s));
          TRY_HIP(p->sweep(k == c - 1 ? 1 : 0, p->ctl, s));
        }
        TRY_HIP(hipEventRecord(p->ev_end[slot], s));
        // a pinned buffer may come back from the allocator with an earlier
        // plan's readouts in it: mark the slot unwritten before the readout
        __atomic_store_n(&p->host[slot].seq, -1, __ATOMIC_RELEASE);
        slot_seq[slot] = ++p->seq;
        TRY_HIP(launch_readout(p->part, p->nparts, nullptr, 0, p->sticky, p->ctl, c,
                               slot_seq[slot], &p->host[slot], s, p->segctl, p->segact,
                               p->nseg, p->seg_grid));
        ++enq;
        enq_sweeps += c;
      }
      if (rd == enq) break;
      const int slot = rd % kRing;
      if ((rc = wait_readout(&p->host[slot], slot_seq[slot], s))) return finish(rc);
      const HostReadout h = p->host[slot];
      if (h.sweeps > last_sweeps) {  // this chunk ran (not skipped)
        stats.checks += 1;
        if (chunk_frozen[slot]) frozen_seg_sweeps += h.seg_sweeps - seg_sweeps;
        seg_sweeps = h.seg_sweeps;
        float ms = 0.f;
        TRY_HIP(hipEventSynchronize(p->ev_end[slot]));  // done: the readout after it has run
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
        // the remaining queued chunks are no-ops on the device; the work
        // enqueued next runs after them in stream order, and the host's next
        // wait covers them, so there is nothing to wait for here
        rd = enq;
      }
    }
    sweeps_done = last_sweeps;
    stats.sweeps = sweeps_done;
    if (bn < 0.0) {
      if ((rc = take_bn())) return finish(rc);
      if (bn == 0.0) return zero_b();
    }
    // ---- x += H/S, r = b - A x (FP64), ||r|| ----
    p->infer_skips = true;  // segments that sat the pass out add nothing
    const hipError_t ie = p->infer(x, nullptr, nullptr, s);
    p->infer_skips = false;
    TRY_HIP(ie);
    TRY_HIP(p->residual(b, x, nullptr, s));
    HostReadout rr;
    if ((rc = p->read_sum(s, &rr, 2, bn))) return finish(rc);
    // independent systems: the worst one decides (the whole-system norm still
    // catches non-finite values)
    const double rel_all = std::sqrt(rr.sum) / bn;
    const double rel = (p->nseg > 1 && std::isfinite(rel_all)) ? rr.segrel : rel_all;
    if (std::getenv("GABP_VERBOSE"))
      std::fprintf(stderr, "gabp: pass %d: %d sweeps (%d settled), rel. residual %.3e\n", pass,
                   sweeps_done, stats.frozen_sweeps, rel);
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
  if (marg_prec) TRY_HIP(p->infer(nullptr, marg_prec, nullptr, s));
  TRY_HIP(hipStreamSynchronize(s));
  return finish(status);
}

}  // namespace gabp

using namespace gabp;

extern "C" {

const char *gabp_version(void) { return "gabp-mi355x 0.3 (gfx950)"; }

void gabp_default_opts(gabp_opts *o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->msg_fp32 = 1;
  o->tol = 1e-8;
  o->max_sweeps = 20000;
  o->check_every = 0;
  o->damping = 0.0;
  o->inner_tol = 0.0;
  o->max_restarts = 30;
  o->group = 0;
  o->layout = GABP_LAYOUT_PAIR;
  o->grid_blocks = 0;
  o->freeze = 1;
  o->batch_waves = 0;
  o->adapt_damping = 1;
  o->schedule = GABP_SCHEDULE_SYNC;
  o->col_blocks = 0;
  o->accel = GABP_ACCEL_NONE;
  o->accel_stride = 0;
  o->accel_cycle = 0;
}

int gabp_plan_workspace_bytes(const gabp_plan *p, size_t *bytes) {
  clear_stale_error();
  if (!p || !bytes) return GABP_ERR_ARG;
  int64_t b = p->acct ? p->acct->bytes.load() : 0;
  if (p->coarse) b += coarse_bytes(p->coarse);
  *bytes = (size_t)std::max<int64_t>(b, 0);
  return GABP_OK;
}

int gabp_plan_destroy(gabp_plan *p) {
  clear_stale_error();
  if (!p) return GABP_ERR_ARG;
  (void)hipDeviceSynchronize();
  if (p->coarse) coarse_destroy(p->coarse);  // its levels refer to the engine
  delete p->eng;
  if (p->bat) batch_destroy(p->bat);
  if (p->small) small_destroy(p->small);
  if (p->lsq) lsq_destroy(p->lsq);  // after the engine that reads its matrix
  if (p->perm) perm_destroy(p->perm);
  delete p;
  return GABP_OK;
}

int gabp_plan_solve(gabp_plan *p, const double *b, double *x, double *marg_prec, gabp_stats *st,
                    hipStream_t s) {
  clear_stale_error();
  GABP_PLAN_SCOPE(p);
  if (p && p->bat) return batch_solve(p->bat, b, x, marg_prec, nullptr, st, s);
  if (p && p->small) return small_solve(p->small, b, x, marg_prec, nullptr, st, s);
  if (!p || !p->eng) return GABP_ERR_ARG;
  if (p->perm) return perm_solve(p->perm, p->eng, b, x, marg_prec, st, s);
  return engine_solve(p->eng, b, x, marg_prec, st, s);
}

int gabp_plan_reset(gabp_plan *p, const double *b, hipStream_t s) {
  clear_stale_error();
  GABP_PLAN_SCOPE(p);
  if (p && p->bat) return batch_reset(p->bat, b, s);
  if (p && p->small) return small_reset(p->small, b, s);
  if (!p || !p->eng || (p->eng->n > 0 && !b)) return GABP_ERR_ARG;
  if (p->eng->n == 0) return GABP_OK;
  if (p->perm && !(b = perm_in(p->perm, b, s))) return GABP_ERR_HIP;
  TRY_HIP(launch_fill_zero4(p->eng->sticky, 1, s));
  TRY_HIP(p->eng->reset(b, s));
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int gabp_plan_sweeps(gabp_plan *p, int32_t count, hipStream_t s) {
  GABP_PLAN_SCOPE(p);
  clear_stale_error();
  if (p && p->bat) return batch_sweeps(p->bat, count, s);
  if (p && p->small) return small_sweeps(p->small, count, s);
  if (!p || !p->eng || count < 0) return GABP_ERR_ARG;
  Engine *e = p->eng;
  if (e->frozen) return GABP_ERR_ARG;  // trajectory access needs the full state (reset first)
  for (int k = 0; k < count && e->n > 0; ++k) TRY_HIP(e->sweep(0, nullptr, s));
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int gabp_plan_marginals(gabp_plan *p, double *mean, double *prec, hipStream_t s) {
  GABP_PLAN_SCOPE(p);
  clear_stale_error();
  if (p && p->bat) return batch_marginals(p->bat, mean, prec, s);
  if (p && p->small) return small_marginals(p->small, mean, prec, s);
  if (!p || !p->eng || (p->eng->n > 0 && !mean)) return GABP_ERR_ARG;
  if (p->eng->n == 0) return GABP_OK;
  if (p->perm) return perm_marginals(p->perm, p->eng, mean, prec, s);
  TRY_HIP(launch_fill_zero(mean, p->eng->n, s));
  TRY_HIP(p->eng->infer(mean, prec, nullptr, s));
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int gabp_plan_get_messages(gabp_plan *p, double *P, double *h, hipStream_t s) {
  GABP_PLAN_SCOPE(p);
  clear_stale_error();
  if (p && p->small) return small_messages(p->small, P, h, false, s);
  if (p && p->bat) return GABP_ERR_UNSUPPORTED;
  if (!p || !p->eng || p->eng->frozen) return GABP_ERR_ARG;
  if (p->perm) return perm_messages(p->perm, p->eng, P, h, false, s);
  return p->eng->get_messages(P, h, s);
}

int gabp_plan_set_messages(gabp_plan *p, const double *P, const double *h, hipStream_t s) {
  GABP_PLAN_SCOPE(p);
  clear_stale_error();
  if (p && p->small)
    return small_messages(p->small, const_cast<double *>(P), const_cast<double *>(h), true, s);
  if (p && p->bat) return GABP_ERR_UNSUPPORTED;
  if (!p || !p->eng || p->eng->frozen) return GABP_ERR_ARG;
  if (p->perm)
    return perm_messages(p->perm, p->eng, const_cast<double *>(P), const_cast<double *>(h), true,
                         s);
  return p->eng->set_messages(P, h, s);
}

int gabp_plan_colors(gabp_plan *p, int32_t *colors, int32_t *ncolors, hipStream_t s) {
  GABP_PLAN_SCOPE(p);
  clear_stale_error();
  if (p && p->small) return small_colors(p->small, colors, ncolors, s);
  if (!p || !p->eng) return GABP_ERR_ARG;
  if (p->perm) return perm_colors(p->perm, colors, ncolors, s);
  if (p->lsq && lsq_coloured(p->lsq)) return lsq_colors(p->lsq, colors, ncolors, s);
  return GABP_ERR_UNSUPPORTED;
}

}  // extern "C"
