// Batches of small sparse instances (GABP_BATCH_CSR): plan creation
// (validation, in-slot arrays, colouring, queue order, launch shape), the
// persistent solve and trajectory access.  The instances are the diagonal
// blocks of one CSR matrix; every instance is solved by one workgroup with its
// messages in LDS (kernels_small.hip).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <memory>
#include <numeric>
#include <vector>

#include "engine.h"

namespace gabp {

struct SmallEngine {
  gabp_opts o{};
  bool fp32 = true;
  size_t tsz = 4;
  int count = 0, N = 0;
  int64_t nnz = 0, E = 0;
  const int64_t *rp = nullptr;
  const int32_t *col = nullptr;
  const double *val = nullptr;
  std::vector<SmallInst> hinst;
  std::vector<int32_t> hcolor;
  SmallInst *inst = nullptr;
  int32_t *order = nullptr;
  uint32_t *queue = nullptr;
  int32_t *soff = nullptr, *rev = nullptr, *color = nullptr;
  void *acoef = nullptr, *diagT = nullptr, *msg = nullptr, *rhsT = nullptr;
  double *hist = nullptr;
  SmallStat *stat = nullptr;
  int emax = 0, nmax = 0, maxdeg = 0, ncolors = 1;
  int rpt = 1, threads = 64, grid = 0;
  bool cache = false, traj = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;

  ~SmallEngine() {
    void *bufs[] = {inst, order, queue, soff, rev, color, acoef, diagT, msg, rhsT, hist, stat};
    for (void *b : bufs)
      if (b) dfree(b);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
  }

  SmallArgs args(int mode) const {
    SmallArgs a{};
    a.mode = mode;
    a.fp32 = fp32;
    a.colored = o.schedule == GABP_SCHEDULE_COLORED;
    a.rows_per_thread = rpt;
    a.cache = cache;
    a.maxdeg = maxdeg;
    a.threads = threads;
    a.grid = grid;
    a.count = count;
    a.inst = inst;
    a.order = order;
    a.queue = queue;
    a.emax = emax;
    a.nmax = nmax;
    a.rp = rp;
    a.col = col;
    a.val = val;
    a.soff = soff;
    a.rev = rev;
    a.acoef = acoef;
    a.diagT = diagT;
    a.color = a.colored ? color : nullptr;
    a.msg = msg;
    a.rhsT = rhsT;
    a.stat = stat;
    a.hist = hist;
    a.nodes = N;
    a.tol = o.tol;
    a.alpha = o.damping;
    a.inner_tol = o.inner_tol;
    a.floor = fp32 ? 1e-6 : 1e-14;
    a.max_sweeps = o.max_sweeps;
    a.max_restarts = o.max_restarts;
    a.check_every = o.check_every > 0 ? o.check_every : 2;
    a.accel = o.accel;
    a.stride = o.accel_stride > 0 ? o.accel_stride : 2;
    a.cycle = o.accel_cycle > 0 ? o.accel_cycle : 100;
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

// Colour of every row, per instance: two colours (breadth-first search) where
// the instance's graph is bipartite, else greedy first-fit in row order.
// adj: in-slot neighbours (global rows) of row g at [off[g], off[g + 1]).
void colour_instances(const std::vector<SmallInst> &inst, const std::vector<int32_t> &off,
                      const std::vector<int32_t> &adj, std::vector<int32_t> &colour,
                      std::vector<int32_t> &ncol) {
  colour.assign(off.size() - 1, -1);
  ncol.assign(inst.size(), 1);
  std::vector<int32_t> queue;
  std::vector<char> used;
  for (size_t t = 0; t < inst.size(); ++t) {
    const int b = inst[t].node0, e = b + inst[t].n;
    bool bip = true;
    for (int s = b; s < e && bip; ++s) {
      if (colour[s] >= 0) continue;
      colour[s] = 0;
      queue.assign(1, s);
      for (size_t h = 0; h < queue.size() && bip; ++h) {
        const int u = queue[h];
        for (int k = off[u]; k < off[u + 1]; ++k) {
          const int v = adj[k];
          if (colour[v] < 0) {
            colour[v] = colour[u] ^ 1;
            queue.push_back(v);
          } else if (colour[v] == colour[u]) {
            bip = false;
            break;
          }
        }
      }
    }
    int nc = 1;
    if (bip) {
      for (int g = b; g < e; ++g) nc = std::max(nc, colour[g] + 1);
    } else {
      for (int g = b; g < e; ++g) colour[g] = -1;
      for (int g = b; g < e; ++g) {
        used.assign(off[g + 1] - off[g] + 2, 0);
        for (int k = off[g]; k < off[g + 1]; ++k) {
          const int c = colour[adj[k]];
          if (c >= 0 && c < (int)used.size()) used[c] = 1;
        }
        int c = 0;
        while (used[c]) ++c;
        colour[g] = c;
        nc = std::max(nc, c + 1);
      }
    }
    ncol[t] = nc;
  }
}

// device buffers of plan creation only, freed on every return path
struct Scratch {
  std::vector<void *> p;
  ~Scratch() {
    for (void *q : p) dfree(q);
  }
  template <typename P>
  hipError_t alloc(P **q, size_t count, size_t elem) {
    hipError_t r = dalloc(q, count, elem);
    if (r == hipSuccess) p.push_back((void *)*q);
    return r;
  }
};

int check_small_batch(const gabp_batch *B) {
  if (!B || B->kind != GABP_BATCH_CSR || B->count < 0 || !B->csr) return GABP_ERR_ARG;
  int st = check_csr(B->csr);
  if (st) return st;
  if (B->count > 0 && !B->k) return GABP_ERR_ARG;
  int64_t tot = 0;
  for (int t = 0; t < B->count; ++t) {
    if (B->k[t] < 0) return GABP_ERR_ARG;
    if (B->k[t] > 4096) return GABP_ERR_UNSUPPORTED;
    tot += B->k[t];
  }
  if (tot != B->csr->n) return GABP_ERR_ARG;
  return GABP_OK;
}

}  // namespace

int small_create(const gabp_batch *B, const gabp_opts *o, SmallEngine **out, hipStream_t s) {
  *out = nullptr;
  int st = check_small_batch(B);
  if (st) return st;
  auto *e = new SmallEngine();
  std::unique_ptr<SmallEngine> guard(e);
  if (o) e->o = *o;
  else gabp_default_opts(&e->o);
  if ((st = check_opts(&e->o))) return st;
  e->fp32 = e->o.msg_fp32 != 0;
  e->tsz = e->fp32 ? 4 : 8;
  e->count = B->count;
  e->N = B->csr->n;
  e->nnz = B->csr->nnz;
  e->rp = B->csr->row_ptr;
  e->col = B->csr->col;
  e->val = B->csr->val;
  TRY_HIP(hipEventCreate(&e->ev0));
  TRY_HIP(hipEventCreate(&e->ev1));
  // instances in row order
  e->hinst.resize(e->count);
  std::vector<int32_t> node_off(e->count + 1, 0);
  for (int t = 0; t < e->count; ++t) {
    node_off[t + 1] = node_off[t] + B->k[t];
    e->hinst[t] = SmallInst{B->k[t], node_off[t], 0, 0, 1, 0};
    e->nmax = std::max(e->nmax, B->k[t]);
  }
  const int N = e->N;
  // validation and in-slot arrays (the CSR plan's builders, one column range)
  Scratch w;
  int64_t *deg = nullptr, *dpos = nullptr, *vo = nullptr, *scan = nullptr;
  uint32_t *flags = nullptr;
  int32_t *ocol = nullptr, *noff = nullptr;
  TRY_HIP(w.alloc(&deg, N, sizeof(int64_t)));
  TRY_HIP(w.alloc(&dpos, N, sizeof(int64_t)));
  TRY_HIP(w.alloc(&vo, (size_t)N + 1, sizeof(int64_t)));
  TRY_HIP(w.alloc(&scan, scan_tmp_elems(N), sizeof(int64_t)));
  TRY_HIP(w.alloc(&flags, 1, sizeof(uint32_t)));
  TRY_HIP(w.alloc(&noff, (size_t)e->count + 1, sizeof(int32_t)));
  uint32_t hf = 0;
  TRY_HIP(launch_fill_zero4(flags, 1, s));
  TRY_HIP(launch_plan_rows(N, e->nnz, e->rp, e->col, e->val, deg, dpos, flags, s));
  TRY_HIP(hipMemcpyAsync(&hf, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  if (hf & FLAG_ARG) return GABP_ERR_ARG;
  if (hf & FLAG_ZERO_DIAG) return GABP_ERR_ZERO_DIAG;
  if (e->count > 0) {
    TRY_HIP(hipMemcpyAsync(noff, node_off.data(), node_off.size() * sizeof(int32_t),
                           hipMemcpyHostToDevice, s));
    TRY_HIP(launch_small_blocks(N, e->count, noff, e->rp, e->col, flags, s));
  }
  TRY_HIP(launch_scan(deg, vo, N, scan, s));
  int64_t Et = 0;
  TRY_HIP(hipMemcpyAsync(&Et, vo + N, sizeof(int64_t), hipMemcpyDeviceToHost, s));
  TRY_HIP(hipMemcpyAsync(&hf, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  if (hf & FLAG_ARG) return GABP_ERR_ARG;  // an entry joins two instances
  if (Et > INT32_MAX) return GABP_ERR_UNSUPPORTED;
  e->E = Et;
  TRY_HIP(dalloc(&e->soff, (size_t)N + 1, sizeof(int32_t)));
  TRY_HIP(dalloc(&e->rev, Et, sizeof(int32_t)));
  TRY_HIP(w.alloc(&ocol, Et, sizeof(int32_t)));
  TRY_HIP(dalloc((char **)&e->acoef, Et, e->tsz));
  TRY_HIP(dalloc((char **)&e->diagT, N, e->tsz));
  TRY_HIP(launch_plan_edges(e->fp32, N, 1, e->rp, e->col, e->val, dpos, vo, e->soff, ocol, e->rev,
                            e->acoef, e->diagT, flags, s));
  std::vector<int32_t> hoff((size_t)N + 1, 0), hadj;
  TRY_HIP(hipMemcpyAsync(hoff.data(), e->soff, hoff.size() * sizeof(int32_t),
                         hipMemcpyDeviceToHost, s));
  TRY_HIP(hipMemcpyAsync(&hf, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  const bool coloured = e->o.schedule == GABP_SCHEDULE_COLORED;
  if (coloured) {
    hadj.resize((size_t)Et);
    TRY_HIP(hipMemcpyAsync(hadj.data(), ocol, (size_t)Et * sizeof(int32_t), hipMemcpyDeviceToHost,
                           s));
  }
  TRY_HIP(hipStreamSynchronize(s));
  if (hf & FLAG_ASYM) return GABP_ERR_NOT_SYMMETRIC;
  if (hf & FLAG_ARG) return GABP_ERR_ARG;
  for (int g = 0; g < N; ++g) e->maxdeg = std::max(e->maxdeg, hoff[g + 1] - hoff[g]);
  for (SmallInst &I : e->hinst) {
    I.slot0 = hoff[I.node0];
    I.E = hoff[I.node0 + I.n] - I.slot0;
    e->emax = std::max(e->emax, I.E);
  }
  // colouring (serial scheme in colour order)
  if (coloured) {
    std::vector<int32_t> nc;
    colour_instances(e->hinst, hoff, hadj, e->hcolor, nc);
    for (int t = 0; t < e->count; ++t) {
      e->hinst[t].ncol = nc[t];
      e->ncolors = std::max(e->ncolors, nc[t]);
    }
    TRY_HIP(dalloc(&e->color, N, sizeof(int32_t)));
    TRY_HIP(hipMemcpyAsync(e->color, e->hcolor.data(), (size_t)N * sizeof(int32_t),
                           hipMemcpyHostToDevice, s));
  }
  // launch shape: one row per thread up to 1024 rows, else up to 4 per thread
  e->threads = std::min(1024, std::max(64, (e->nmax + 63) / 64 * 64));
  e->rpt = (e->nmax + e->threads - 1) / e->threads;
  if (e->rpt > 4) return GABP_ERR_UNSUPPORTED;
  e->rpt = e->rpt <= 1 ? 1 : 4;
  e->cache = e->rpt == 1 && e->maxdeg <= 8;
  if (small_lds(e->args(SMALL_SOLVE)) > (size_t)max_lds_per_block()) return GABP_ERR_UNSUPPORTED;
  // queue: most in-slots first, ties by index
  std::vector<int32_t> ord(e->count);
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
    return (int64_t)e->hinst[a].E + e->hinst[a].n > (int64_t)e->hinst[b].E + e->hinst[b].n;
  });
  TRY_HIP(dalloc(&e->inst, e->count, sizeof(SmallInst)));
  TRY_HIP(dalloc(&e->order, e->count, sizeof(int32_t)));
  TRY_HIP(dalloc(&e->queue, 1, sizeof(uint32_t)));
  TRY_HIP(dalloc(&e->stat, e->count, sizeof(SmallStat)));
  TRY_HIP(dalloc((char **)&e->msg, Et, 2 * e->tsz));
  TRY_HIP(dalloc((char **)&e->rhsT, ((size_t)N * e->tsz + 7) / 8, 8));  // whole 8-byte words
  TRY_HIP(dalloc(&e->hist, (size_t)6 * N, sizeof(double)));
  if (e->count > 0) {
    TRY_HIP(hipMemcpyAsync(e->inst, e->hinst.data(), e->count * sizeof(SmallInst),
                           hipMemcpyHostToDevice, s));
    TRY_HIP(hipMemcpyAsync(e->order, ord.data(), e->count * sizeof(int32_t), hipMemcpyHostToDevice,
                           s));
  }
  TRY_HIP(launch_fill_zero(e->msg, Et * 2 * (int64_t)e->tsz / 8, s));
  TRY_HIP(launch_fill_zero(e->rhsT, ((int64_t)N * (int64_t)e->tsz + 7) / 8, s));
  TRY_HIP(hipStreamSynchronize(s));
  if (e->count > 0) {
    const int occ = small_occupancy(e->args(SMALL_SOLVE));
    if (occ <= 0) return GABP_ERR_UNSUPPORTED;
    e->grid = std::max(1, std::min(occ * cu_count(), e->count));
    if (e->o.grid_blocks > 0) e->grid = std::min(e->grid, e->o.grid_blocks);
  }
  *out = guard.release();
  return GABP_OK;
}

void small_destroy(SmallEngine *e) { delete e; }

int small_solve(SmallEngine *e, const double *b, double *x, double *marg_prec, gabp_stats *per,
                gabp_stats *summary, hipStream_t s) {
  const auto t0 = std::chrono::steady_clock::now();
  if (!e) return GABP_ERR_ARG;
  if (e->N > 0 && (!b || !x)) return GABP_ERR_ARG;
  gabp_stats sum{};
  sum.edges = e->E;
  sum.batch_waves = e->threads / 64;
  sum.batch_groups = e->grid;
  sum.sweep_launches = 0;
  int worst = GABP_OK;
  if (e->count > 0) {
    TRY_HIP(launch_fill_zero4(e->queue, 1, s));
    SmallArgs a = e->args(SMALL_SOLVE);
    a.b = b;
    a.x = x;
    TRY_HIP(hipEventRecord(e->ev0, s));
    TRY_HIP(launch_small_batch(a, s));
    TRY_HIP(hipEventRecord(e->ev1, s));
    if (marg_prec) TRY_HIP(launch_small_marginals(a, e->N, nullptr, marg_prec, s));
    std::vector<SmallStat> hs(e->count);
    TRY_HIP(hipMemcpyAsync(hs.data(), e->stat, e->count * sizeof(SmallStat), hipMemcpyDeviceToHost,
                           s));
    TRY_HIP(hipStreamSynchronize(s));
    float ms = 0.f;
    TRY_HIP(hipEventElapsedTime(&ms, e->ev0, e->ev1));
    sum.sweep_ms = ms;
    double work = 0.0, swept = 0.0;
    for (int t = 0; t < e->count; ++t) {
      const SmallStat &d = hs[t];
      const SmallInst &I = e->hinst[t];
      if (d.status < 0) {
        if (worst >= 0 || d.status < worst) worst = d.status;
      } else if (worst >= 0 && d.status > worst) {
        worst = d.status;
      }
      sum.sweeps = std::max(sum.sweeps, d.sweeps);
      sum.restarts = std::max(sum.restarts, d.restarts);
      sum.checks += d.checks;
      sum.rel_residual = std::max(sum.rel_residual, d.rel);
      work += (double)I.E * d.sweeps;
      swept += d.sweeps;
      if (per) {
        gabp_stats &p = per[t];
        p = gabp_stats{};
        p.status = d.status;
        p.sweeps = d.sweeps;
        p.restarts = d.restarts;
        p.checks = d.checks;
        p.rel_residual = d.rel;
        p.residual_per_eq = I.n > 0 ? d.rnorm / I.n : 0.0;
        p.edges = I.E;
        p.mean_sweeps = d.sweeps;
        p.damping = e->o.damping;
        p.batch_waves = e->threads / 64;
        p.batch_groups = e->grid;
      }
    }
    sum.damping = e->o.damping;
    sum.mean_sweeps = swept / e->count;
    sum.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    sum.edge_updates_per_s = sum.seconds > 0 ? work / sum.seconds : 0.0;
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

int small_reset(SmallEngine *e, const double *b, hipStream_t s) {
  if (!e || (e->N > 0 && !b)) return GABP_ERR_ARG;
  if (e->count > 0) {
    TRY_HIP(launch_fill_zero4(e->queue, 1, s));
    SmallArgs a = e->args(SMALL_RESET);
    a.b = b;
    TRY_HIP(launch_small_batch(a, s));
    TRY_HIP(hipStreamSynchronize(s));
  }
  e->traj = true;
  return GABP_OK;
}

int small_sweeps(SmallEngine *e, int count, hipStream_t s) {
  if (!e || count < 0 || !e->traj) return GABP_ERR_ARG;
  if (e->count > 0 && count > 0) {
    TRY_HIP(launch_fill_zero4(e->queue, 1, s));
    SmallArgs a = e->args(SMALL_SWEEPS);
    a.nsweeps = count;
    TRY_HIP(launch_small_batch(a, s));
    TRY_HIP(hipStreamSynchronize(s));
  }
  return GABP_OK;
}

int small_marginals(SmallEngine *e, double *mean, double *prec, hipStream_t s) {
  if (!e || (e->N > 0 && !mean)) return GABP_ERR_ARG;
  TRY_HIP(launch_small_marginals(e->args(SMALL_SOLVE), e->N, mean, prec, s));
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int small_messages(SmallEngine *e, double *P, double *h, bool set, hipStream_t s) {
  if (!e || (e->nnz > 0 && (!P || !h))) return GABP_ERR_ARG;
  TRY_HIP(launch_small_messages(e->args(SMALL_SOLVE), e->N, P, h, set, s));
  TRY_HIP(hipStreamSynchronize(s));
  if (set) e->traj = true;
  return GABP_OK;
}

int small_colors(const SmallEngine *e, int32_t *colors, int32_t *ncolors, hipStream_t s) {
  if (!e || !ncolors || (e->N > 0 && !colors)) return GABP_ERR_ARG;
  if (e->o.schedule != GABP_SCHEDULE_COLORED) return GABP_ERR_UNSUPPORTED;
  if (e->N > 0) {
    TRY_HIP(hipMemcpyAsync(colors, e->color, (size_t)e->N * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, s));
    TRY_HIP(hipStreamSynchronize(s));
  }
  *ncolors = e->ncolors;
  return GABP_OK;
}

}  // namespace gabp
