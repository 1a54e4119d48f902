// Section VII for any sparse matrix: the plan assembles the symmetric
// bipartite system R = [[I_k, S^T], [S, -psi I_m]] on the device
// (kernels_lsq.hip) and solves R [x; z] = [0; y] as an ordinary CSR plan.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "engine.h"

namespace gabp {

struct LsqSystem {
  int m = 0, k = 0;
  double psi = 0.0;
  int64_t nnzA = 0;
  int64_t *Arp = nullptr;
  int32_t *Acol = nullptr;
  double *Aval = nullptr;
  double *bt = nullptr, *xt = nullptr;  // [0; y] and [x; z] of a solve
  double *u = nullptr, *part = nullptr; // normal-equations residual scratch
  int nparts = 1;
  bool coloured = false;

  ~LsqSystem() {
    void *bufs[] = {Arp, Acol, Aval, bt, xt, u, part};
    for (void *b : bufs)
      if (b) dfree(b);
  }
};

void lsq_destroy(LsqSystem *q) { delete q; }

bool lsq_coloured(const LsqSystem *q) { return q->coloured; }

// x rows colour 0, z rows colour 1
int lsq_colors(const LsqSystem *q, int32_t *colors, int32_t *ncolors, hipStream_t s) {
  if (ncolors) *ncolors = (q->k > 0) + (q->m > 0);
  const int64_t n = (int64_t)q->k + q->m;
  if (colors && n > 0) {
    std::vector<int32_t> h((size_t)n, 1);
    std::fill(h.begin(), h.begin() + q->k, 0);
    TRY_HIP(hipMemcpyAsync(colors, h.data(), h.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    TRY_HIP(hipStreamSynchronize(s));
  }
  return GABP_OK;
}

namespace {

// Scratch of the assembly, freed on every path.
struct LsqScratch {
  uint32_t *colcnt = nullptr, *keys = nullptr, *flags = nullptr;
  int64_t *rowlen = nullptr, *scan = nullptr;
  int32_t *rowof = nullptr, *idx = nullptr, *perm = nullptr;
  void *sort = nullptr;
  ~LsqScratch() {
    void *bufs[] = {colcnt, keys, flags, rowlen, scan, rowof, idx, perm, sort};
    for (void *b : bufs)
      if (b) dfree(b);
  }
};

int assemble(const gabp_rect *S, LsqSystem *q, hipStream_t s) {
  const int m = S->m, k = S->k;
  const int64_t nnz = S->nnz, n = (int64_t)k + m;
  LsqScratch w;
  TRY_HIP(dalloc(&q->Arp, n + 1, sizeof(int64_t)));
  TRY_HIP(dalloc(&q->Acol, q->nnzA, sizeof(int32_t)));
  TRY_HIP(dalloc(&q->Aval, q->nnzA, sizeof(double)));
  TRY_HIP(dalloc(&w.colcnt, k, sizeof(uint32_t)));
  TRY_HIP(dalloc(&w.flags, 1, sizeof(uint32_t)));
  TRY_HIP(dalloc(&w.rowlen, n, sizeof(int64_t)));
  TRY_HIP(dalloc(&w.scan, scan_tmp_elems(n), sizeof(int64_t)));
  TRY_HIP(dalloc(&w.rowof, nnz, sizeof(int32_t)));
  TRY_HIP(dalloc(&w.idx, nnz, sizeof(int32_t)));
  TRY_HIP(dalloc(&w.perm, nnz, sizeof(int32_t)));
  TRY_HIP(dalloc(&w.keys, nnz, sizeof(uint32_t)));
  TRY_HIP(launch_fill_zero4(w.colcnt, k, s));
  TRY_HIP(launch_fill_zero4(w.flags, 1, s));
  TRY_HIP(launch_lsq_rows(m, k, nnz, S->row_ptr, S->col, S->val, w.colcnt, w.rowlen, w.rowof,
                          w.idx, w.flags, s));
  uint32_t hflags = 0;
  TRY_HIP(hipMemcpyAsync(&hflags, w.flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  if (hflags & FLAG_ARG) return GABP_ERR_ARG;
  TRY_HIP(launch_scan(w.rowlen, q->Arp, n, w.scan, s));
  if (nnz > 0) {
    size_t bytes = 0;
    TRY_HIP(launch_lsq_sort(k, nnz, S->col, w.keys, w.idx, w.perm, nullptr, &bytes, s));
    TRY_HIP(dalloc((char **)&w.sort, bytes, 1));
    TRY_HIP(launch_lsq_sort(k, nnz, S->col, w.keys, w.idx, w.perm, w.sort, &bytes, s));
  }
  TRY_HIP(launch_lsq_fill(m, k, q->psi, S->row_ptr, S->col, S->val, q->Arp, w.perm, w.rowof,
                          q->Acol, q->Aval, s));
  TRY_HIP(hipStreamSynchronize(s));  // the scratch is freed on return
  return GABP_OK;
}

int check_rect(const gabp_rect *S, double psi) {
  if (!S || S->m < 0 || S->k < 0 || S->nnz < 0) return GABP_ERR_ARG;
  if (!(psi > 0.0) || !std::isfinite(psi)) return GABP_ERR_ARG;
  if (!S->row_ptr || (S->nnz > 0 && (!S->col || !S->val))) return GABP_ERR_ARG;
  const int64_t n = (int64_t)S->k + S->m;
  if (2 * S->nnz + n >= (int64_t)INT32_MAX) return GABP_ERR_UNSUPPORTED;
  int64_t ends[2] = {0, 0};
  if (hipMemcpy(&ends[0], S->row_ptr, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess ||
      hipMemcpy(&ends[1], S->row_ptr + S->m, sizeof(int64_t), hipMemcpyDeviceToHost) != hipSuccess)
    return GABP_ERR_ARG;
  if (ends[0] != 0 || ends[1] != S->nnz) return GABP_ERR_ARG;
  return GABP_OK;
}

// ||S^T (y - S x) - psi x||^2 (x == NULL: ||S^T y||^2), summed on the host in
// block order
int normal_sq(LsqSystem *q, const double *y, const double *x, double *r, double *out,
              hipStream_t s) {
  TRY_HIP(launch_lsq_normal(q->m, q->k, q->psi, q->Arp, q->Acol, q->Aval, y, x, q->u, r, q->part, s));
  std::vector<double> h((size_t)q->nparts);
  TRY_HIP(hipMemcpyAsync(h.data(), q->part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  double t = 0.0;
  for (double v : h) t += v;
  *out = t;
  return GABP_OK;
}

}  // namespace
}  // namespace gabp

using namespace gabp;

extern "C" {

static int plan_create_lsq_impl(const gabp_rect *S, double psi, const gabp_opts *o, gabp_plan **plan,
                         hipStream_t s) {
  clear_stale_error();
  if (!plan) return GABP_ERR_ARG;
  *plan = nullptr;
  int rc = check_rect(S, psi);
  if (rc) return rc;
  LsqSystem *q = new (std::nothrow) LsqSystem();
  if (!q) return GABP_ERR_NOMEM;
  q->m = S->m;
  q->k = S->k;
  q->psi = psi;
  q->nnzA = 2 * S->nnz + S->k + S->m;
  q->nparts = lsq_normal_blocks(S->k);
  const int64_t n = (int64_t)S->k + S->m;
  if ((rc = assemble(S, q, s)) || (rc = from_hip(dalloc(&q->bt, n, sizeof(double)))) ||
      (rc = from_hip(dalloc(&q->xt, n, sizeof(double)))) ||
      (rc = from_hip(dalloc(&q->u, S->m, sizeof(double)))) ||
      (rc = from_hip(dalloc(&q->part, q->nparts, sizeof(double))))) {
    delete q;
    return rc;
  }
  gabp_csr A{};
  A.n = (int32_t)n;
  A.nnz = q->nnzA;
  A.row_ptr = q->Arp;
  A.col = q->Acol;
  A.val = q->Aval;
  // the two classes of the bipartite graph: the x rows, then the z rows
  const std::vector<int> classes = {0, S->k, (int)n};
  const bool coloured = o && o->schedule == GABP_SCHEDULE_COLORED;
  gabp_plan *p = nullptr;
  if ((rc = csr_plan_create(&A, o, coloured ? &classes : nullptr, &p, s))) {
    delete q;
    return rc;
  }
  q->coloured = coloured;
  p->lsq = q;
  *plan = p;
  return GABP_OK;
}

int gabp_plan_create_lsq(const gabp_rect *S, double psi, const gabp_opts *o, gabp_plan **plan,
                         hipStream_t s) {
  return with_account(plan, [&] { return plan_create_lsq_impl(S, psi, o, plan, s); });
}

int gabp_plan_solve_lsq(gabp_plan *p, const double *y, double *x, gabp_stats *st, hipStream_t s) {
  GABP_PLAN_SCOPE(p);
  clear_stale_error();
  if (!p || !p->eng || !p->lsq) return GABP_ERR_ARG;
  LsqSystem *q = p->lsq;
  if ((q->m > 0 && !y) || (q->k > 0 && !x)) return GABP_ERR_ARG;
  TRY_HIP(launch_lsq_embed(q->k, q->m, y, q->bt, s));
  const int rc = engine_solve(p->eng, q->bt, q->xt, nullptr, st, s);
  if (rc < 0 && rc != GABP_ERR_DIVERGED && rc != GABP_ERR_BREAKDOWN) return rc;
  // x: the first k unknowns (also after a failed or unconverged solve)
  if (q->k > 0) {
    TRY_HIP(hipMemcpyAsync(x, q->xt, (size_t)q->k * sizeof(double), hipMemcpyDeviceToDevice, s));
    TRY_HIP(hipStreamSynchronize(s));
  }
  return rc;
}

int gabp_solve_lsq(const gabp_rect *S, double psi, const double *y, double *x,
                   const gabp_opts *o, gabp_stats *st, hipStream_t s) {
  clear_stale_error();
  gabp_plan *p = nullptr;
  int rc = gabp_plan_create_lsq(S, psi, o, &p, s);
  if (rc) {
    if (st) { std::memset(st, 0, sizeof(*st)); st->status = rc; }
    return rc;
  }
  rc = gabp_plan_solve_lsq(p, y, x, st, s);
  gabp_plan_destroy(p);
  return rc;
}

int gabp_plan_residual_lsq(gabp_plan *p, const double *y, const double *x, double *r,
                           double *rel_norm, hipStream_t s) {
  GABP_PLAN_SCOPE(p);
  clear_stale_error();
  if (!p || !p->lsq || !rel_norm) return GABP_ERR_ARG;
  LsqSystem *q = p->lsq;
  if ((q->m > 0 && !y) || (q->k > 0 && !x)) return GABP_ERR_ARG;
  double bn2 = 0.0, rn2 = 0.0;
  int rc;
  if ((rc = normal_sq(q, y, nullptr, nullptr, &bn2, s)) || (rc = normal_sq(q, y, x, r, &rn2, s)))
    return rc;
  const double bn = std::sqrt(bn2), rn = std::sqrt(rn2);
  *rel_norm = bn > 0.0 ? rn / bn : rn;
  return std::isfinite(*rel_norm) ? GABP_OK : GABP_ERR_ARG;
}

}  // extern "C"
