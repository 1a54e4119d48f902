// The warm-start network object of the C ABI: FP32 master parameters, Adam
// moments and the bfloat16 copy the kernels read, plus training scratch
// grown to the largest batch seen.
#include <cmath>
#include <cstring>
#include <vector>

#include "engine.h"

using namespace gabp;

struct gabp_model {
  float *master = nullptr, *m1 = nullptr, *m2 = nullptr;
  uint16_t *wbf = nullptr;
  int64_t step = 0;
  // training scratch
  int64_t cap = 0;
  float *H1 = nullptr, *H2 = nullptr, *R = nullptr, *D1 = nullptr, *D2 = nullptr;
  double *part = nullptr;
  float *gpart = nullptr;
  double *lossv = nullptr;

  void free_scratch() {
    void *bufs[] = {H1, H2, R, D1, D2, part, gpart};
    for (void *b : bufs)
      if (b) dfree(b);
    H1 = H2 = R = D1 = D2 = nullptr;
    part = nullptr;
    gpart = nullptr;
    cap = 0;
  }
  ~gabp_model() {
    free_scratch();
    void *bufs[] = {master, m1, m2, wbf, lossv};
    for (void *b : bufs)
      if (b) dfree(b);
  }
  int ensure(int64_t S) {
    if (S <= cap) return GABP_OK;
    free_scratch();
    const int64_t fb = mlp_fwd_blocks(S), gb = (S + mlp_chunk() - 1) / mlp_chunk();
    int st;
    if ((st = from_hip(dalloc(&H1, 64 * S, sizeof(float)))) ||
        (st = from_hip(dalloc(&H2, 64 * S, sizeof(float)))) ||
        (st = from_hip(dalloc(&D1, 64 * S, sizeof(float)))) ||
        (st = from_hip(dalloc(&D2, 64 * S, sizeof(float)))) ||
        (st = from_hip(dalloc(&R, 12 * S, sizeof(float)))) ||
        (st = from_hip(dalloc(&part, 2 * fb, sizeof(double)))) ||
        (st = from_hip(dalloc(&gpart, gb * mlp_params(), sizeof(float)))))
      return st;
    cap = S;
    return GABP_OK;
  }
};

namespace {

// splitmix64 (Steele, Lea, Flood), uniform in [0, 1) from the top 53 bits
struct SplitMix {
  uint64_t x;
  uint64_t next() {
    uint64_t z = (x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

int set_params(gabp_model *m, const float *host, hipStream_t s) {
  float *tmp = nullptr;
  TRY_HIP(dalloc(&tmp, mlp_params(), sizeof(float)));
  hipError_t e = hipMemcpyAsync(tmp, host, mlp_params() * sizeof(float), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = launch_mlp_set(tmp, m->master, m->wbf, m->m1, m->m2, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dfree(tmp);
  m->step = 0;
  return from_hip(e);
}

int run(gabp_model *m, const float *U, const float *T, int64_t count, float *grad, bool update,
        double lr, double *loss, hipStream_t s) {
  if (!m || !U || !T || count <= 0) return GABP_ERR_ARG;
  if (update && !(lr > 0.0 && std::isfinite(lr))) return GABP_ERR_ARG;
  int st;
  if ((st = m->ensure(count))) return st;
  MlpTrainArgs a{};
  a.w = m->wbf;
  a.U = U;
  a.T = T;
  a.S = count;
  a.H1 = m->H1; a.H2 = m->H2; a.R = m->R; a.D1 = m->D1; a.D2 = m->D2;
  a.part = m->part;
  a.gpart = m->gpart;
  a.lossv = m->lossv;
  a.grad = grad;
  a.update = update;
  a.master = m->master; a.m1 = m->m1; a.m2 = m->m2; a.wbf = m->wbf;
  const int64_t t = m->step + 1;
  a.lr = (float)lr;
  a.c1 = (float)(1.0 - std::pow(0.9, (double)t));
  a.c2 = (float)(1.0 - std::pow(0.999, (double)t));
  TRY_HIP(launch_mlp_train(a, s));
  double lv[2] = {0.0, 0.0};
  TRY_HIP(hipMemcpyAsync(lv, m->lossv, sizeof(lv), hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  if (update) m->step = t;
  if (loss) *loss = lv[0];
  return GABP_OK;
}

}  // namespace

const uint16_t *model_weights(const gabp_model *m) { return m ? m->wbf : nullptr; }

extern "C" {

int gabp_model_create(uint64_t seed, gabp_model **out, hipStream_t s) {
  clear_stale_error();
  if (!out) return GABP_ERR_ARG;
  *out = nullptr;
  auto *m = new (std::nothrow) gabp_model();
  if (!m) return GABP_ERR_NOMEM;
  const int P = mlp_params();
  int st;
  if ((st = from_hip(dalloc(&m->master, P, sizeof(float)))) ||
      (st = from_hip(dalloc(&m->m1, P, sizeof(float)))) ||
      (st = from_hip(dalloc(&m->m2, P, sizeof(float)))) ||
      (st = from_hip(dalloc(&m->wbf, P, sizeof(uint16_t)))) ||
      (st = from_hip(dalloc(&m->lossv, 2, sizeof(double))))) {
    delete m;
    return st;
  }
  // He-uniform weights (bound sqrt(6 / fan_in)), zero biases
  std::vector<float> h(P, 0.f);
  SplitMix rng{seed};
  const int layers[3][3] = {{0, 64, 8}, {576, 64, 64}, {4736, 12, 64}};  // offset, rows, cols
  for (const auto &L : layers) {
    const double bound = std::sqrt(6.0 / L[2]);
    for (int e = 0; e < L[1] * L[2]; ++e) h[L[0] + e] = (float)((2.0 * rng.uniform() - 1.0) * bound);
  }
  if ((st = set_params(m, h.data(), s))) {
    delete m;
    return st;
  }
  *out = m;
  return GABP_OK;
}

int gabp_model_destroy(gabp_model *m) {
  clear_stale_error();
  if (!m) return GABP_ERR_ARG;
  (void)hipDeviceSynchronize();
  delete m;
  return GABP_OK;
}

int gabp_model_get_params(const gabp_model *m, float *params, hipStream_t s) {
  clear_stale_error();
  if (!m || !params) return GABP_ERR_ARG;
  float *tmp = nullptr;
  TRY_HIP(dalloc(&tmp, mlp_params(), sizeof(float)));
  hipError_t e = launch_mlp_get(m->wbf, tmp, s);
  if (e == hipSuccess)
    e = hipMemcpyAsync(params, tmp, mlp_params() * sizeof(float), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  dfree(tmp);
  return from_hip(e);
}

int gabp_model_set_params(gabp_model *m, const float *params, hipStream_t s) {
  clear_stale_error();
  if (!m || !params) return GABP_ERR_ARG;
  for (int p = 0; p < mlp_params(); ++p)
    if (!std::isfinite(params[p])) return GABP_ERR_ARG;
  return set_params(m, params, s);
}

int gabp_model_forward(const gabp_model *m, const float *U, int64_t count, float *out,
                       hipStream_t s) {
  clear_stale_error();
  if (!m || count < 0 || (count > 0 && (!U || !out))) return GABP_ERR_ARG;
  TRY_HIP(launch_mlp_forward(m->wbf, U, count, out, s));
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int gabp_model_grad(gabp_model *m, const float *U, const float *T, int64_t count, float *grad,
                    double *loss, hipStream_t s) {
  clear_stale_error();
  return run(m, U, T, count, grad, false, 0.0, loss, s);
}

int gabp_model_train_step(gabp_model *m, const float *U, const float *T, int64_t count,
                          double lr, double *loss, hipStream_t s) {
  clear_stale_error();
  return run(m, U, T, count, nullptr, true, lr, loss, s);
}

int gabp_model_grid_features(const gabp_grid *A, const double *b, const int64_t *nodes,
                             int64_t count, float *U, hipStream_t s) {
  clear_stale_error();
  GridGeom g{};
  int st;
  if ((st = check_grid(A, &g))) return st;
  if (count < 0 || (count > 0 && (!b || !U)) || (!nodes && count > g.N)) return GABP_ERR_ARG;
  GridCoef<double> k{A->diag, A->cx, A->cy, A->cz, A->diag_value, A->off_value};
  TRY_HIP(launch_grid_features(g, k, b, nodes, count, U, s));
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int gabp_model_grid_targets(const gabp_grid *A, const double *P, const double *h,
                            const int64_t *nodes, int64_t count, float *T, hipStream_t s) {
  clear_stale_error();
  GridGeom g{};
  int st;
  if ((st = check_grid(A, &g))) return st;
  if (count < 0 || (count > 0 && (!P || !h || !T)) || (!nodes && count > g.N)) return GABP_ERR_ARG;
  GridCoef<double> k{A->diag, A->cx, A->cy, A->cz, A->diag_value, A->off_value};
  TRY_HIP(launch_grid_targets(g, k, P, h, nodes, count, T, s));
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

int gabp_plan_solve_warm(gabp_plan *p, const gabp_model *m, const double *b, double *x,
                         double *marg_prec, gabp_stats *st, hipStream_t s) {
  GABP_PLAN_SCOPE(p);
  clear_stale_error();
  if (!p || !m) return GABP_ERR_ARG;
  if (!p->eng || !p->eng->has_warm_start()) return GABP_ERR_UNSUPPORTED;  // grid plans only
  gabp_stats a{};
  int rc = engine_solve(p->eng, b, x, marg_prec, &a, s, m->wbf);
  const bool failed = rc == GABP_NOT_CONVERGED || rc == GABP_ERR_BREAKDOWN || rc == GABP_ERR_DIVERGED;
  if (failed && a.warm_start == 1) {
    // the warm-started solve failed: plain GaBP from zero messages decides
    gabp_stats z{};
    rc = engine_solve(p->eng, b, x, marg_prec, &z, s, nullptr);
    z.sweeps += a.sweeps;
    z.frozen_sweeps += a.frozen_sweeps;
    z.restarts += a.restarts;
    z.checks += a.checks;
    z.seconds += a.seconds;
    z.sweep_ms += a.sweep_ms;
    z.frozen_sweep_ms += a.frozen_sweep_ms;
    z.mean_sweeps += a.mean_sweeps;
    z.mean_frozen_sweeps += a.mean_frozen_sweeps;
    z.edge_updates_per_s = z.seconds > 0 ? (double)z.edges * z.mean_sweeps / z.seconds : 0.0;
    z.warm_start = -2;
    z.warm_rel0 = a.warm_rel0;
    a = z;
  }
  if (st) *st = a;
  return rc;
}

}  // extern "C"
