// Coloured CSR plans: the caller's matrix is coloured on the device
// (kernels_color.hip), renumbered so that each colour class is a contiguous
// range of rows, and solved as a CSR plan whose sweep sends one class per
// launch.  Vectors cross the boundary through the permutation.
#include <cstring>
#include <new>
#include <vector>

#include "engine.h"

namespace gabp {

struct CsrPerm {
  int n = 0, ncolors = 0;
  int32_t *new2old = nullptr, *old2new = nullptr, *color = nullptr;  // color: caller's order
  int64_t *rp = nullptr;
  int32_t *col = nullptr;
  double *val = nullptr;
  int64_t nnz = 0;
  int32_t *slot = nullptr;  // the caller's CSR slot of each renumbered slot
  double *bp = nullptr, *xp = nullptr, *mp = nullptr;  // renumbered b, x, marginals

  ~CsrPerm() {
    void *bufs[] = {new2old, old2new, color, rp, col, val, slot, bp, xp, mp};
    for (void *b : bufs)
      if (b) dfree(b);
  }
};

void perm_destroy(CsrPerm *q) { delete q; }

namespace {

struct Scratch {
  std::vector<void *> bufs;
  template <typename P>
  hipError_t alloc(P **p, size_t count, size_t elem) {
    hipError_t e = dalloc(p, count, elem);
    if (e == hipSuccess) bufs.push_back(*p);
    return e;
  }
  ~Scratch() {
    for (void *b : bufs) dfree(b);
  }
};

// validation of the rows, colouring, renumbering, renumbered matrix
int build_perm(const gabp_csr *A, CsrPerm *q, std::vector<int> *classes, hipStream_t s) {
  const int n = A->n;
  const int64_t nnz = A->nnz;
  Scratch w;
  int64_t *deg = nullptr, *dpos = nullptr, *len = nullptr, *scan = nullptr;
  uint32_t *flags = nullptr, *left = nullptr, *keys = nullptr;
  int32_t *idx = nullptr, *first = nullptr, *cmax = nullptr, *col_tmp = nullptr;
  int32_t *slot_tmp = nullptr;
  if (nnz > (int64_t)INT32_MAX) return GABP_ERR_UNSUPPORTED;  // slots are int32
  TRY_HIP(w.alloc(&deg, n, sizeof(int64_t)));
  TRY_HIP(w.alloc(&dpos, n, sizeof(int64_t)));
  TRY_HIP(w.alloc(&flags, 1, sizeof(uint32_t)));
  TRY_HIP(w.alloc(&left, 1, sizeof(uint32_t)));
  TRY_HIP(w.alloc(&cmax, 1, sizeof(int32_t)));
  // the rows are validated before the colouring reads them
  uint32_t hflags = 0;
  TRY_HIP(launch_fill_zero4(flags, 1, s));
  TRY_HIP(launch_plan_rows(n, nnz, A->row_ptr, A->col, A->val, deg, dpos, flags, s));
  TRY_HIP(hipMemcpyAsync(&hflags, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  if (hflags & FLAG_ARG) return GABP_ERR_ARG;
  if (hflags & FLAG_ZERO_DIAG) return GABP_ERR_ZERO_DIAG;
  // Jones-Plassmann rounds until every node is coloured
  TRY_HIP(dalloc(&q->color, n, sizeof(int32_t)));
  TRY_HIP(hipMemsetAsync(q->color, 0xFF, (size_t)n * sizeof(int32_t), s));  // -1: uncoloured
  for (int round = 0;; ++round) {
    uint32_t hleft = 0;
    TRY_HIP(launch_fill_zero4(left, 1, s));
    TRY_HIP(launch_jp_round(n, A->row_ptr, A->col, q->color, left, flags, s));
    TRY_HIP(hipMemcpyAsync(&hleft, left, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
    TRY_HIP(hipStreamSynchronize(s));
    if (hleft == 0) break;
    if (round > n) return GABP_ERR_HIP;  // each round colours at least one node
  }
  TRY_HIP(hipMemcpyAsync(&hflags, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
  TRY_HIP(hipMemsetAsync(cmax, 0xFF, sizeof(int32_t), s));
  TRY_HIP(launch_color_max(n, q->color, cmax, s));
  int32_t hmax = -1;
  TRY_HIP(hipMemcpyAsync(&hmax, cmax, sizeof(int32_t), hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  if (hflags & FLAG_UNSUPPORTED) return GABP_ERR_UNSUPPORTED;
  q->ncolors = hmax + 1;
  // renumbering: stable sort by colour
  TRY_HIP(dalloc(&q->new2old, n, sizeof(int32_t)));
  TRY_HIP(dalloc(&q->old2new, n, sizeof(int32_t)));
  TRY_HIP(w.alloc(&idx, n, sizeof(int32_t)));
  TRY_HIP(w.alloc(&keys, n, sizeof(uint32_t)));
  TRY_HIP(w.alloc(&first, q->ncolors, sizeof(int32_t)));
  TRY_HIP(launch_iota(n, idx, s));
  size_t bytes = 0;
  void *tmp = nullptr;
  TRY_HIP(launch_color_sort(n, q->ncolors, q->color, keys, idx, q->new2old, nullptr, &bytes, s));
  TRY_HIP(w.alloc((char **)&tmp, bytes, 1));
  TRY_HIP(launch_color_sort(n, q->ncolors, q->color, keys, idx, q->new2old, tmp, &bytes, s));
  TRY_HIP(hipMemsetAsync(first, 0xFF, (size_t)q->ncolors * sizeof(int32_t), s));
  TRY_HIP(launch_perm_finish(n, keys, q->new2old, q->old2new, first, s));
  std::vector<int32_t> hfirst((size_t)q->ncolors);
  TRY_HIP(hipMemcpyAsync(hfirst.data(), first, hfirst.size() * sizeof(int32_t),
                         hipMemcpyDeviceToHost, s));
  TRY_HIP(hipStreamSynchronize(s));
  classes->clear();
  for (int32_t f : hfirst)
    if (f >= 0) classes->push_back(f);  // colours present, in colour order
  classes->push_back(n);
  // the renumbered matrix, each row's columns sorted, and the caller's slot
  // of each of its slots (the values gathered through it; messages cross
  // the boundary the same way)
  TRY_HIP(w.alloc(&len, n, sizeof(int64_t)));
  TRY_HIP(w.alloc(&scan, scan_tmp_elems(n), sizeof(int64_t)));
  TRY_HIP(dalloc(&q->rp, (size_t)n + 1, sizeof(int64_t)));
  TRY_HIP(dalloc(&q->col, nnz, sizeof(int32_t)));
  TRY_HIP(dalloc(&q->val, nnz, sizeof(double)));
  TRY_HIP(dalloc(&q->slot, nnz, sizeof(int32_t)));
  q->nnz = nnz;
  TRY_HIP(w.alloc(&col_tmp, nnz, sizeof(int32_t)));
  TRY_HIP(w.alloc(&slot_tmp, nnz, sizeof(int32_t)));
  TRY_HIP(launch_perm_rowlen(n, A->row_ptr, q->new2old, len, s));
  TRY_HIP(launch_scan(len, q->rp, n, scan, s));
  TRY_HIP(launch_perm_fill(n, A->row_ptr, A->col, q->new2old, q->old2new, q->rp, col_tmp,
                           slot_tmp, s));
  if (nnz > 0) {
    size_t sb = 0;
    void *stmp = nullptr;
    TRY_HIP(launch_rows_sort(n, nnz, q->rp, col_tmp, q->col, slot_tmp, q->slot, nullptr, &sb, s));
    TRY_HIP(w.alloc((char **)&stmp, sb, 1));
    TRY_HIP(launch_rows_sort(n, nnz, q->rp, col_tmp, q->col, slot_tmp, q->slot, stmp, &sb, s));
  }
  TRY_HIP(launch_slot_move(nnz, q->slot, A->val, q->val, true, s));
  TRY_HIP(dalloc(&q->bp, n, sizeof(double)));
  TRY_HIP(dalloc(&q->xp, n, sizeof(double)));
  TRY_HIP(dalloc(&q->mp, n, sizeof(double)));
  TRY_HIP(hipStreamSynchronize(s));  // the scratch is freed on return
  return GABP_OK;
}

}  // namespace

int coloured_csr_plan(const gabp_csr *A, const gabp_opts *o, gabp_plan **plan, hipStream_t s) {
  *plan = nullptr;
  int rc = check_csr(A);
  if (rc) return rc;
  CsrPerm *q = new (std::nothrow) CsrPerm();
  if (!q) return GABP_ERR_NOMEM;
  q->n = A->n;
  std::vector<int> classes;
  if (A->n > 0 && (rc = build_perm(A, q, &classes, s))) {
    delete q;
    return rc;
  }
  if (A->n == 0) classes = {0, 0};
  gabp_csr B = *A;
  B.row_ptr = q->rp;
  B.col = q->col;
  B.val = q->val;
  if (A->n == 0) B = *A;
  gabp_plan *p = nullptr;
  if ((rc = csr_plan_create(&B, o, &classes, &p, s))) {
    delete q;
    return rc;
  }
  p->perm = q;
  *plan = p;
  return GABP_OK;
}

const double *perm_in(CsrPerm *q, const double *b, hipStream_t s) {
  if (launch_permute(q->n, q->new2old, b, q->bp, true, s) != hipSuccess) return nullptr;
  return q->bp;
}

int perm_solve(CsrPerm *q, Engine *e, const double *b, double *x, double *marg, gabp_stats *st,
               hipStream_t s) {
  if (q->n > 0 && (!b || !x)) return GABP_ERR_ARG;
  const double *bp = perm_in(q, b, s);
  if (q->n > 0 && !bp) return GABP_ERR_HIP;
  const int rc = engine_solve(e, bp, q->xp, marg ? q->mp : nullptr, st, s);
  if (q->n > 0) {
    TRY_HIP(launch_permute(q->n, q->new2old, q->xp, x, false, s));
    if (marg) TRY_HIP(launch_permute(q->n, q->new2old, q->mp, marg, false, s));
    TRY_HIP(hipStreamSynchronize(s));
  }
  return rc;
}

int perm_marginals(CsrPerm *q, Engine *e, double *mean, double *prec, hipStream_t s) {
  if (q->n == 0) return GABP_OK;
  TRY_HIP(launch_fill_zero(q->xp, q->n, s));
  TRY_HIP(e->infer(q->xp, prec ? q->mp : nullptr, nullptr, s));
  TRY_HIP(launch_permute(q->n, q->new2old, q->xp, mean, false, s));
  if (prec) TRY_HIP(launch_permute(q->n, q->new2old, q->mp, prec, false, s));
  TRY_HIP(hipStreamSynchronize(s));
  return GABP_OK;
}

// Messages in the caller's CSR order: the plan's own (renumbered) slots moved
// through the slot map, by way of two FP64 buffers of nnz held for the call.
int perm_messages(CsrPerm *q, Engine *e, double *P, double *h, bool set, hipStream_t s) {
  if (q->nnz == 0) return set ? e->set_messages(P, h, s) : e->get_messages(P, h, s);
  if (!P || !h) return GABP_ERR_ARG;
  double *Pn = nullptr, *hn = nullptr;
  hipError_t err = dalloc(&Pn, q->nnz, sizeof(double));
  if (err == hipSuccess) err = dalloc(&hn, q->nnz, sizeof(double));
  int rc = from_hip(err);
  if (!rc && set) {
    err = launch_slot_move(q->nnz, q->slot, P, Pn, true, s);
    if (err == hipSuccess) err = launch_slot_move(q->nnz, q->slot, h, hn, true, s);
    rc = err == hipSuccess ? e->set_messages(Pn, hn, s) : from_hip(err);
  } else if (!rc) {
    rc = e->get_messages(Pn, hn, s);
    if (!rc) {
      err = launch_slot_move(q->nnz, q->slot, Pn, P, false, s);
      if (err == hipSuccess) err = launch_slot_move(q->nnz, q->slot, hn, h, false, s);
      if (err == hipSuccess) err = hipStreamSynchronize(s);
      rc = from_hip(err);
    }
  }
  (void)hipStreamSynchronize(s);  // the buffers are free only after their last reader
  if (Pn) dfree(Pn);
  if (hn) dfree(hn);
  return rc;
}

int perm_colors(const CsrPerm *q, int32_t *colors, int32_t *ncolors, hipStream_t s) {
  if (ncolors) *ncolors = q->ncolors;
  if (colors && q->n > 0) {
    TRY_HIP(hipMemcpyAsync(colors, q->color, (size_t)q->n * sizeof(int32_t),
                           hipMemcpyDeviceToDevice, s));
    TRY_HIP(hipStreamSynchronize(s));
  }
  return GABP_OK;
}

}  // namespace gabp
