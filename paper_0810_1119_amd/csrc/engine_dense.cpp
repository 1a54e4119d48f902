// Batched dense instances: plan creation (validation, packing, queue order,
// workgroup shape), the persistent solve and trajectory access.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <map>
#include <memory>
#include <mutex>
#include <numeric>
#include <tuple>
#include <vector>

#include "engine.h"

namespace gabp {

struct BatchEngine {
  gabp_opts o{};
  int kind = GABP_BATCH_BIPARTITE;
  int count = 0;
  bool fp32 = true;
  size_t tsz = 4;
  const double *mat64 = nullptr;
  std::vector<DenseInst> hinst;
  DenseInst *inst = nullptr;
  int32_t *order = nullptr;
  uint32_t *queue = nullptr;
  void *matT = nullptr;          // FP32 couplings (FP64 messages read mat64)
  void *state = nullptr, *fcoef = nullptr, *fh = nullptr;
  void *tot = nullptr, *nb = nullptr;
  DenseStat *dstat = nullptr;
  uint32_t *vflags = nullptr;
  int64_t entries = 0, nodes = 0, xlen = 0, rhslen = 0, edges = 0;
  int nr = 0, nc = 0, maxm = 1, waves = 8, grid = 1;
  bool traj = false, fresh = true;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  ~BatchEngine() {
    void *bufs[] = {inst, order, queue, matT, state, fcoef, fh, tot, nb, dstat, vflags};
    for (void *b : bufs)
      if (b) dfree(b);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }

  DenseArgs args(int mode) const {
    DenseArgs a{};
    a.kind = kind;
    a.fp32 = fp32;
    a.waves = waves;
    a.grid = grid;
    a.nr = nr;
    a.nc = nc;
    a.maxm = maxm;
    a.mode = mode;
    a.count = count;
    a.inst = inst;
    a.order = order;
    a.queue = queue;
    a.mat64 = mat64;
    a.matT = fp32 ? matT : (const void *)mat64;
    a.state = state;
    a.fcoef = fcoef;
    a.fh = fh;
    a.colored = o.schedule == GABP_SCHEDULE_COLORED;
    a.tot = tot;
    a.nb = nb;
    a.stat = dstat;
    a.tol = o.tol;
    a.alpha = o.damping;
    a.inner_tol = o.inner_tol;
    a.freeze = o.freeze != 0 && fcoef != nullptr;
    a.freeze_tol = a.freeze ? (o.freeze_tol > 0.0 ? o.freeze_tol : (fp32 ? 1e-6 : 1e-14)) : -1.0;
    a.floor = fp32 ? 1e-6 : 1e-14;
    a.max_sweeps = o.max_sweeps;
    a.max_restarts = o.max_restarts;
    a.check_every = std::max(2, o.check_every + (o.check_every & 1));
    a.adapt = o.adapt_damping != 0;
    return a;
  }
};

namespace {

int cu_count() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 1;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 1;
  return std::max(1, v);
}

// wavefronts per workgroup must cover the widest row (residual column pass)
bool waves_fit(const BatchEngine *e, int w) {
  if (w * 64 < e->nc) return false;
  const int lds = dense_lds(e->nr, e->nc, w, (int)e->tsz).total + 64;
  return lds <= max_lds_per_block();
}

int grid_for(BatchEngine *e) {
  DenseArgs a = e->args(DENSE_SOLVE);
  const int occ = dense_batch_occupancy(a);
  if (occ <= 0) return 0;
  int g = occ * cu_count();
  if (e->o.grid_blocks > 0) g = std::min(g, e->o.grid_blocks);
  return std::max(1, std::min(g, e->count));
}

// Autotuner of the workgroup shape: time two full sweeps of the whole batch
// for each shape that fits and keep the fastest.  The choice is remembered per
// shape class (kind and schedule, precision, largest instance, batch size,
// entries) in the persistent tuning cache (and so across processes).
int autotune(BatchEngine *e, hipStream_t s) {
  const int64_t bucket = e->entries > 0 ? (int64_t)std::log2((double)e->entries) : 0;
  char shape[160];
  std::snprintf(shape, sizeof shape, "kind=%d,colored=%d,fp32=%d,rows=%d,cols=%d,count=%d,log2e=%lld",
                e->kind, e->o.schedule == GABP_SCHEDULE_COLORED ? 1 : 0, (int)e->fp32, e->nr,
                e->nc, e->count, (long long)bucket);
  const std::string key = tune_key("k_dense_batch.waves", shape);
  {
    int w = 0;
    if (tune_lookup(key, &w) && (w == 4 || w == 8 || w == 16) && waves_fit(e, w)) return w;
  }
  const int cands[] = {4, 8, 16};
  int best = 0;
  float best_ms = 0.f;
  for (int w : cands) {
    if (!waves_fit(e, w)) continue;
    if (best == 0) best = w;
    if (e->entries < (int64_t)1 << 20) break;  // small batches: first shape that fits
    e->waves = w;
    e->grid = grid_for(e);
    if (e->grid <= 0) continue;
    float total = 0.f;
    bool ok = true;
    for (int rep = 0; rep < 2 && ok; ++rep) {
      DenseArgs a = e->args(DENSE_RESET);  // b = NULL: zero right-hand side
      ok = launch_fill_zero4(e->queue, 1, s) == hipSuccess && launch_dense_batch(a, s) == hipSuccess;
      a = e->args(DENSE_SWEEPS);
      a.nsweeps = 2;
      a.fresh = true;
      ok = ok && launch_fill_zero4(e->queue, 1, s) == hipSuccess &&
           hipEventRecord(e->ev0, s) == hipSuccess && launch_dense_batch(a, s) == hipSuccess &&
           hipEventRecord(e->ev1, s) == hipSuccess && hipEventSynchronize(e->ev1) == hipSuccess;
      float ms = 0.f;
      ok = ok && hipEventElapsedTime(&ms, e->ev0, e->ev1) == hipSuccess;
      if (rep == 1) total = ms;  // the first repetition warms caches and code
    }
    if (!ok) {
      (void)hipGetLastError();
      continue;
    }
    if (best_ms == 0.f || total < best_ms) {
      best_ms = total;
      best = w;
    }
  }
  if (best != 0) tune_store(key, best);
  return best;
}

int check_batch(const gabp_batch *B) {
  if (!B || B->count < 0) return GABP_ERR_ARG;
  if (B->kind != GABP_BATCH_BIPARTITE && B->kind != GABP_BATCH_DENSE) return GABP_ERR_ARG;
  if (B->count == 0) return GABP_OK;
  if (!B->k) return GABP_ERR_ARG;
  if (B->kind == GABP_BATCH_BIPARTITE && (!B->m || !B->sigma2)) return GABP_ERR_ARG;
  for (int t = 0; t < B->count; ++t) {
    if (B->k[t] < 0) return GABP_ERR_ARG;
    if (B->k[t] > 512) return GABP_ERR_UNSUPPORTED;
    if (B->kind == GABP_BATCH_BIPARTITE) {
      if (B->m[t] < 0) return GABP_ERR_ARG;
      if (!std::isfinite(B->sigma2[t]) || !(B->sigma2[t] > 0.0)) return GABP_ERR_ARG;
    }
  }
  return GABP_OK;
}

}  // namespace

int batch_create(const gabp_batch *B, const gabp_opts *o, BatchEngine **out, hipStream_t s) {
  *out = nullptr;
  int st = check_batch(B);
  if (st) return st;
  if (o && (st = check_opts(o))) return st;
  if (o && o->accel != GABP_ACCEL_NONE) return GABP_ERR_UNSUPPORTED;  // small CSR batches only
  // the two-colour schedule needs a two-colourable graph: the bipartite kind
  if (o && o->schedule != GABP_SCHEDULE_SYNC && B->kind != GABP_BATCH_BIPARTITE)
    return GABP_ERR_UNSUPPORTED;
  if (o && o->batch_waves != 0 && o->batch_waves != 4 && o->batch_waves != 8 &&
      o->batch_waves != 16)
    return GABP_ERR_ARG;
  auto *e = new BatchEngine();
  std::unique_ptr<BatchEngine> guard(e);
  if (o) e->o = *o;
  else gabp_default_opts(&e->o);
  e->kind = B->kind;
  e->count = B->count;
  e->fp32 = e->o.msg_fp32 != 0;
  e->tsz = e->fp32 ? 4 : 8;
  e->mat64 = B->mat;
  // packing and queue order (largest block first, ties by index)
  e->hinst.resize(e->count);
  int64_t mo = 0, ro = 0, xo = 0, no = 0;
  for (int t = 0; t < e->count; ++t) {
    DenseInst &I = e->hinst[t];
    I.cols = B->k[t];
    I.rows = B->kind == GABP_BATCH_BIPARTITE ? B->m[t] : B->k[t];
    I.sigma2 = B->kind == GABP_BATCH_BIPARTITE ? B->sigma2[t] : 0.0;
    I.mat = mo;
    I.rhs = ro;
    I.xoff = xo;
    I.node = no;
    I.edges = 0;
    mo += (int64_t)I.rows * I.cols;
    ro += B->kind == GABP_BATCH_BIPARTITE ? I.rows : I.cols;
    xo += I.cols;
    no += I.cols + (B->kind == GABP_BATCH_BIPARTITE ? I.rows : 0);
    e->nr = std::max(e->nr, I.rows);
    e->nc = std::max(e->nc, I.cols);
  }
  e->entries = mo;
  e->rhslen = ro;
  e->xlen = xo;
  e->nodes = no;
  if (e->entries > 0 && !B->mat) return GABP_ERR_ARG;
  std::vector<int32_t> ord(e->count);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
    return (int64_t)e->hinst[a].rows * e->hinst[a].cols > (int64_t)e->hinst[b].rows * e->hinst[b].cols;
  });
  e->maxm = 1;
  while (e->maxm * 64 < e->nc) e->maxm *= 2;
  if (e->maxm > 8) return GABP_ERR_UNSUPPORTED;
  TRY_HIP(hipEventCreate(&e->ev0));
  TRY_HIP(hipEventCreate(&e->ev1));
  if (e->count == 0) {
    *out = guard.release();
    return GABP_OK;
  }
  TRY_HIP(dalloc(&e->inst, e->count, sizeof(DenseInst)));
  TRY_HIP(dalloc(&e->order, e->count, sizeof(int32_t)));
  TRY_HIP(dalloc(&e->queue, 1, sizeof(uint32_t)));
  TRY_HIP(dalloc(&e->dstat, e->count, sizeof(DenseStat)));
  TRY_HIP(dalloc(&e->vflags, e->count, sizeof(uint32_t)));
  if (e->fp32) TRY_HIP(dalloc((char **)&e->matT, e->entries, sizeof(float)));
  TRY_HIP(dalloc((char **)&e->state, e->entries, 4 * e->tsz));
  TRY_HIP(dalloc((char **)&e->tot, e->nodes, 2 * e->tsz));
  TRY_HIP(dalloc((char **)&e->nb, e->nodes, e->tsz));
  if (e->o.freeze) {
    TRY_HIP(dalloc((char **)&e->fcoef, e->entries, 2 * e->tsz));
    TRY_HIP(dalloc((char **)&e->fh, e->entries, 2 * e->tsz));
  }
  TRY_HIP(hipMemcpyAsync(e->inst, e->hinst.data(), e->count * sizeof(DenseInst),
                         hipMemcpyHostToDevice, s));
  TRY_HIP(hipMemcpyAsync(e->order, ord.data(), e->count * sizeof(int32_t), hipMemcpyHostToDevice, s));
  // validation, FP32 copy, message counts
  TRY_HIP(launch_dense_prepare(e->args(DENSE_SOLVE), e->vflags, s));
  std::vector<uint32_t> fl(e->count);
  TRY_HIP(hipMemcpyAsync(fl.data(), e->vflags, e->count * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TRY_HIP(hipMemcpyAsync(e->hinst.data(), e->inst, e->count * sizeof(DenseInst),
                         hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  uint32_t all = 0;
  for (uint32_t f : fl) all |= f;
  if (all & FLAG_ARG) return GABP_ERR_ARG;
  if (all & FLAG_ASYM) return GABP_ERR_NOT_SYMMETRIC;
  if (all & FLAG_ZERO_DIAG) return GABP_ERR_ZERO_DIAG;
  for (const DenseInst &I : e->hinst) e->edges += I.edges;
  // workgroup shape
  if (e->o.batch_waves != 0) {
    // the requested shape, or the next larger one that covers the widest row
    e->waves = 0;
    for (int w = e->o.batch_waves; w <= 16 && e->waves == 0; w *= 2)
      if (waves_fit(e, w)) e->waves = w;
    if (e->waves == 0) return GABP_ERR_UNSUPPORTED;
  } else {
    e->waves = autotune(e, s);
    if (e->waves == 0) return GABP_ERR_UNSUPPORTED;
  }
  e->grid = grid_for(e);
  if (e->grid <= 0) return GABP_ERR_UNSUPPORTED;
  *out = guard.release();
  return GABP_OK;
}

void batch_destroy(BatchEngine *e) { delete e; }

static void merge_status(int &worst, int st) {
  if (st < 0) {
    if (worst >= 0 || st < worst) worst = st;
  } else if (worst >= 0 && st > worst) {
    worst = st;
  }
}

int batch_solve(BatchEngine *e, const double *b, double *x, double *marg_prec,
                gabp_stats *per, gabp_stats *summary, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!e) return GABP_ERR_ARG;
  if ((e->rhslen > 0 && !b) || (e->xlen > 0 && !x)) return GABP_ERR_ARG;
  gabp_stats sum{};
  sum.edges = e->edges;
  sum.batch_waves = e->waves;
  sum.batch_groups = e->grid;
  int worst = GABP_OK;
  if (e->count > 0) {
    TRY_HIP(launch_fill_zero4(e->queue, 1, s));
    DenseArgs a = e->args(DENSE_SOLVE);
    a.b = b;
    a.x = x;
    TRY_HIP(hipEventRecord(e->ev0, s));
    TRY_HIP(launch_dense_batch(a, s));
    TRY_HIP(hipEventRecord(e->ev1, s));
    if (marg_prec) TRY_HIP(launch_dense_marginals(a, nullptr, marg_prec, false, s));
    std::vector<DenseStat> hs(e->count);
    TRY_HIP(hipMemcpyAsync(hs.data(), e->dstat, e->count * sizeof(DenseStat), hipMemcpyDeviceToHost, s));
    TRY_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    TRY_HIP(hipEventElapsedTime(&ms, e->ev0, e->ev1));
    sum.sweep_ms = ms;
    double work = 0.0;
    for (int t = 0; t < e->count; ++t) {
      const DenseStat &d = hs[t];
      const DenseInst &I = e->hinst[t];
      merge_status(worst, d.status);
      sum.sweeps = std::max(sum.sweeps, d.sweeps);
      sum.frozen_sweeps = std::max(sum.frozen_sweeps, d.frozen_sweeps);
      sum.restarts = std::max(sum.restarts, d.restarts);
      sum.checks += d.checks;
      sum.rel_residual = std::max(sum.rel_residual, d.rel);
      work += (double)I.edges * d.sweeps;
      if (per) {
        gabp_stats &p = per[t];
        p = gabp_stats{};
        p.status = d.status;
        p.sweeps = d.sweeps;
        p.frozen_sweeps = d.frozen_sweeps;
        p.restarts = d.restarts;
        p.checks = d.checks;
        p.rel_residual = d.rel;
        p.residual_per_eq = I.cols > 0 ? d.rnorm / I.cols : 0.0;
        p.edges = I.edges;
        p.mean_sweeps = d.sweeps;
        p.mean_frozen_sweeps = d.frozen_sweeps;
        p.damping = d.damping;
        p.batch_waves = e->waves;
        p.batch_groups = e->grid;
      }
      sum.damping = std::max(sum.damping, d.damping);
    }
    sum.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    sum.edge_updates_per_s = sum.seconds > 0 ? work / sum.seconds : 0.0;
    double swept = 0.0;
    for (int t = 0; t < e->count; ++t) swept += hs[t].sweeps;
    sum.mean_sweeps = swept / e->count;
    double settled = 0.0;
    for (int t = 0; t < e->count; ++t) settled += hs[t].frozen_sweeps;
    sum.mean_frozen_sweeps = settled / e->count;
    if (per)
      for (int t = 0; t < e->count; ++t) {
        per[t].seconds = sum.seconds;
        per[t].sweep_ms = sum.sweep_ms;
      }
  } else {
    sum.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  sum.status = worst;
  if (summary) *summary = sum;
  e->traj = false;
  return worst;
}

int batch_reset(BatchEngine *e, const double *b, hipStream_t s) {
  if (!e || (e->rhslen > 0 && !b)) return GABP_ERR_ARG;
  if (e->count > 0) {
    TRY_HIP(launch_fill_zero4(e->queue, 1, s));
    DenseArgs a = e->args(DENSE_RESET);
    a.b = b;
    TRY_HIP(launch_dense_batch(a, s));
    TRY_HIP(hipStreamSynchronize(s));
  }
  e->traj = true;
  e->fresh = true;
  return GABP_OK;
}

int batch_sweeps(BatchEngine *e, int count, hipStream_t s) {
  if (!e || count < 0 || !e->traj) return GABP_ERR_ARG;
  if (e->count > 0 && count > 0) {
    TRY_HIP(launch_fill_zero4(e->queue, 1, s));
    DenseArgs a = e->args(DENSE_SWEEPS);
    a.nsweeps = count;
    a.fresh = e->fresh;
    TRY_HIP(launch_dense_batch(a, s));
    TRY_HIP(hipStreamSynchronize(s));
    e->fresh = false;
  }
  return GABP_OK;
}

int batch_marginals(BatchEngine *e, double *mean, double *prec, hipStream_t s) {
  if (!e || (e->nodes > 0 && !mean)) return GABP_ERR_ARG;
  if (e->count > 0) {
    TRY_HIP(launch_dense_marginals(e->args(DENSE_SOLVE), mean, prec, true, s));
    TRY_HIP(hipStreamSynchronize(s));
  }
  return GABP_OK;
}

}  // namespace gabp

using namespace gabp;

extern "C" {

static int plan_create_batched_impl(const gabp_batch *B, const gabp_opts *o, gabp_plan **plan,
                             hipStream_t s) {
  clear_stale_error();
  if (!plan) return GABP_ERR_ARG;
  *plan = nullptr;
  if (B && B->kind == GABP_BATCH_CSR) {
    SmallEngine *q = nullptr;
    const int st = small_create(B, o, &q, s);
    if (st) return st;
    auto *p = new gabp_plan();
    p->small = q;
    *plan = p;
    return GABP_OK;
  }
  BatchEngine *e = nullptr;
  const int st = batch_create(B, o, &e, s);
  if (st) return st;
  auto *p = new gabp_plan();
  p->bat = e;
  *plan = p;
  return GABP_OK;
}

int gabp_plan_create_batched(const gabp_batch *B, const gabp_opts *o, gabp_plan **plan,
                             hipStream_t s) {
  return with_account(plan, [&] { return plan_create_batched_impl(B, o, plan, s); });
}

int gabp_plan_solve_batched(gabp_plan *p, const double *b, double *x, gabp_stats *per,
                            gabp_stats *summary, hipStream_t s) {
  GABP_PLAN_SCOPE(p);
  clear_stale_error();
  if (p && p->small) return small_solve(p->small, b, x, nullptr, per, summary, s);
  if (!p || !p->bat) return GABP_ERR_ARG;
  return batch_solve(p->bat, b, x, nullptr, per, summary, s);
}

int gabp_solve_batched(const gabp_batch *B, const double *b, double *x, const gabp_opts *o,
                       gabp_stats *per, gabp_stats *summary, hipStream_t s) {
  clear_stale_error();
  if (B && B->kind == GABP_BATCH_CSR) {
    SmallEngine *q = nullptr;
    int st = small_create(B, o, &q, s);
    if (st) return st;
    st = small_solve(q, b, x, nullptr, per, summary, s);
    small_destroy(q);
    return st;
  }
  BatchEngine *e = nullptr;
  int st = batch_create(B, o, &e, s);
  if (st) return st;
  st = batch_solve(e, b, x, nullptr, per, summary, s);
  delete e;
  return st;
}

}  // extern "C"
