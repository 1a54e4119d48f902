/*
 * FP64 CPU oracle for Gaussian belief propagation (GaBP) on A x = b.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links or calls
 * this file; only the tests, the smoke check and the benchmark's CPU-baseline
 * leg do.  It shares no code, header or constant with the HIP path.
 *
 * Follows Shental, Bickson, Siegel, Wolf, Dolev, "Gaussian Belief Propagation
 * for Solving Systems of Linear Equations: Theory and Application":
 *   - graph and scalar fixes: section III-C, eq. (prec), (mean), (PhiGauss);
 *   - message rule: eq. (prec_message), (mean_message), written out in
 *     Algorithm 1 step 2 (naive GaBP);
 *   - broadcast form: Algorithm 2 (aggregate per node, then subtract the
 *     reverse message), section V;
 *   - marginals: Algorithm 1 step 4 (the marginal-mean equation of III-C is
 *     read with P_i^{-1}, as Algorithm 1 step 4 writes it);
 *   - parallel (synchronous) schedule: section III-C, two message buffers;
 *   - Jacobi special case: Proposition GaBPJ (section VI-C);
 *   - residual r = b - A x: section II-A, Definition (Residual) (sign flipped,
 *     the norm is unchanged).
 * Messages are kept in the paper's (P, mu) parametrisation.
 *
 * Matrix: CSR with the full symmetric pattern including the diagonal,
 * int64 row pointers, int32 columns sorted within each row, double values.
 * Directed message i->j is stored at the CSR slot of entry (i, j), i != j;
 * diagonal slots hold no message.  rev[slot(i,j)] = slot(j,i).
 *
 * Determinism: every round reads only the previous round's buffers, so the
 * OpenMP loops over rows give bitwise-identical results for any thread count;
 * all norms and maxima are taken in a fixed serial order.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum {
  ORC_OK = 0,
  ORC_NOT_CONVERGED = 1,
  ORC_ERR_ARG = -1,
  ORC_ERR_NOT_SYMMETRIC = -2,
  ORC_ERR_ZERO_DIAG = -3,
  ORC_ERR_BREAKDOWN = -4,
  ORC_ERR_DIVERGED = -5,
};

enum { ORC_STOP_RESIDUAL = 0, ORC_STOP_MESSAGES = 1, ORC_STOP_MEANS = 2 };

typedef struct {
  int32_t n;
  const int64_t *row_ptr;
  const int32_t *col;
  const double *val;
} orc_csr;

typedef struct {
  int32_t algorithm;  /* 1: naive (Algorithm 1), 2: broadcast (Algorithm 2) */
  int32_t stop;       /* ORC_STOP_* */
  double tol;         /* threshold of the stop rule */
  int32_t max_rounds;
  double damping;     /* alpha in [0, 1): m <- alpha m_old + (1 - alpha) m_new */
  int32_t nthreads;   /* OpenMP threads, 0 = runtime default */
} orc_opts;

static void set_threads(int nt) {
#ifdef _OPENMP
  if (nt > 0) omp_set_num_threads(nt);
#else
  (void)nt;
#endif
}

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Slot of entry (i, j) by a linear scan of row i; -1 if absent. */
static int64_t slot_of(const orc_csr *A, int32_t i, int32_t j) {
  for (int64_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e)
    if (A->col[e] == j) return e;
  return -1;
}

/* Reverse-slot table and input validation (Assumption 1: A square symmetric;
 * A_ii != 0 so that mu_ii = b_i / A_ii exists). */
int orc_build_reverse(const orc_csr *A, int64_t *rev, double *diag) {
  if (A->n < 0) return ORC_ERR_ARG;
  for (int32_t i = 0; i < A->n; ++i) {
    diag[i] = 0.0;
    for (int64_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e) {
      int32_t j = A->col[e];
      if (j < 0 || j >= A->n) return ORC_ERR_ARG;
      if (j == i) { diag[i] = A->val[e]; rev[e] = -1; continue; }
      int64_t f = slot_of(A, j, i);
      if (f < 0 || A->val[f] != A->val[e]) return ORC_ERR_NOT_SYMMETRIC;
      rev[e] = f;
    }
    if (diag[i] == 0.0) return ORC_ERR_ZERO_DIAG;
  }
  return ORC_OK;
}

/* One synchronous round of Algorithm 1 (naive GaBP).  For every directed
 * edge i->j, using only round t-1 messages:
 *   P_ij = -A_ij^2 / (P_ii + sum_{k in N(i)\j} P_ki)
 *   mu_ij = (P_ii mu_ii + sum_{k in N(i)\j} P_ki mu_ki) / A_ij
 * with P_ii = A_ii, mu_ii = b_i / A_ii.  Damping (section VI-D: a moving
 * average of successive iterates) is applied to P and to P*mu.  Returns the
 * number of zero cavity precisions met (a breakdown of the rule). */
int64_t orc_alg1_round(const orc_csr *A, const double *b, const int64_t *rev,
                       const double *diag, const double *Pold, const double *Mold,
                       double *Pnew, double *Mnew, double damping, int nthreads) {
  int64_t zeros = 0;
  set_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+ : zeros)
  for (int32_t i = 0; i < A->n; ++i) {
    const double Pii = diag[i];
    const double muii = b[i] / diag[i];
    for (int64_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e) {
      const int32_t j = A->col[e];
      if (j == i) { Pnew[e] = 0.0; Mnew[e] = 0.0; continue; }
      double prec = Pii;
      double num = Pii * muii;
      for (int64_t f = A->row_ptr[i]; f < A->row_ptr[i + 1]; ++f) {
        const int32_t k = A->col[f];
        if (k == i || k == j) continue;
        const int64_t in = rev[f]; /* message k -> i */
        prec += Pold[in];
        num += Pold[in] * Mold[in];
      }
      if (prec == 0.0) ++zeros;
      const double Aij = A->val[e];
      double P = -Aij * Aij / prec;
      double mu = num / Aij;
      if (damping > 0.0) {
        const double Pd = damping * Pold[e] + (1.0 - damping) * P;
        const double hd = damping * Pold[e] * Mold[e] + (1.0 - damping) * P * mu;
        P = Pd;
        mu = hd / Pd;
      }
      Pnew[e] = P;
      Mnew[e] = mu;
    }
  }
  return zeros;
}

/* One synchronous round of Algorithm 2 (broadcast GaBP): every node forms
 *   Pt_i = P_ii + sum_{k in N(i)} P_ki,
 *   mut_i = Pt_i^{-1} (P_ii mu_ii + sum_{k in N(i)} P_ki mu_ki),
 * and each directed message subtracts the reverse one:
 *   P_ij = -A_ij^2 / (Pt_i - P_ji),   mu_ij = (Pt_i mut_i - P_ji mu_ji) / A_ij. */
int64_t orc_alg2_round(const orc_csr *A, const double *b, const int64_t *rev,
                       const double *diag, const double *Pold, const double *Mold,
                       double *Pnew, double *Mnew, double damping, int nthreads) {
  int64_t zeros = 0;
  set_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+ : zeros)
  for (int32_t i = 0; i < A->n; ++i) {
    const double Pii = diag[i];
    const double muii = b[i] / diag[i];
    double Pt = Pii;
    double num = Pii * muii;
    for (int64_t f = A->row_ptr[i]; f < A->row_ptr[i + 1]; ++f) {
      if (A->col[f] == i) continue;
      const int64_t in = rev[f];
      Pt += Pold[in];
      num += Pold[in] * Mold[in];
    }
    const double mut = num / Pt;
    for (int64_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e) {
      if (A->col[e] == i) { Pnew[e] = 0.0; Mnew[e] = 0.0; continue; }
      const int64_t in = rev[e]; /* message j -> i */
      const double cav = Pt - Pold[in];
      if (cav == 0.0) ++zeros;
      const double Aij = A->val[e];
      double P = -Aij * Aij / cav;
      double mu = (Pt * mut - Pold[in] * Mold[in]) / Aij;
      if (damping > 0.0) {
        const double Pd = damping * Pold[e] + (1.0 - damping) * P;
        const double hd = damping * Pold[e] * Mold[e] + (1.0 - damping) * P * mu;
        P = Pd;
        mu = hd / Pd;
      }
      Pnew[e] = P;
      Mnew[e] = mu;
    }
  }
  return zeros;
}

/* A coloured (serial-like) schedule, section III-C's serial scheme in an
 * order fixed by a proper node colouring: one class sends all of its
 * messages, computed as in Algorithm 2 from the messages as they are now,
 * and the classes take turns within a sweep.  The update is in
 * place: with a proper colouring no edge joins two nodes of the class, so
 * none of the messages a node of the class reads is written in its round.
 * Damping mixes in the node's own previous message, as in the synchronous
 * round.  Returns the number of zero cavity precisions met. */
int64_t orc_alg2_color_round(const orc_csr *A, const double *b, const int64_t *rev,
                             const double *diag, double *P, double *M, const int8_t *color,
                             int c, double damping, int nthreads) {
  int64_t zeros = 0;
  set_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+ : zeros)
  for (int32_t i = 0; i < A->n; ++i) {
    if (color[i] != c) continue;
    const double Pii = diag[i];
    const double muii = b[i] / diag[i];
    double Pt = Pii;
    double num = Pii * muii;
    for (int64_t f = A->row_ptr[i]; f < A->row_ptr[i + 1]; ++f) {
      if (A->col[f] == i) continue;
      const int64_t in = rev[f];
      Pt += P[in];
      num += P[in] * M[in];
    }
    const double mut = num / Pt;
    for (int64_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e) {
      if (A->col[e] == i) continue;
      const int64_t in = rev[e]; /* message j -> i, not written in this round */
      const double cav = Pt - P[in];
      if (cav == 0.0) ++zeros;
      const double Aij = A->val[e];
      double Pn = -Aij * Aij / cav;
      double mu = (Pt * mut - P[in] * M[in]) / Aij;
      if (damping > 0.0) {
        const double Pd = damping * P[e] + (1.0 - damping) * Pn;
        const double hd = damping * P[e] * M[e] + (1.0 - damping) * Pn * mu;
        Pn = Pd;
        mu = hd / Pd;
      }
      P[e] = Pn;
      M[e] = mu;
    }
  }
  return zeros;
}

/* Algorithm 1 step 4: marginal means and (optionally) marginal precisions
 *   P_i = P_ii + sum_{k in N(i)} P_ki,
 *   mu_i = (P_ii mu_ii + sum_{k in N(i)} P_ki mu_ki) / P_i. */
void orc_marginals(const orc_csr *A, const double *b, const int64_t *rev,
                   const double *diag, const double *P, const double *M,
                   double *mean, double *prec, int nthreads) {
  set_threads(nthreads);
#pragma omp parallel for schedule(static)
  for (int32_t i = 0; i < A->n; ++i) {
    double Pi = diag[i];
    double num = diag[i] * (b[i] / diag[i]);
    for (int64_t f = A->row_ptr[i]; f < A->row_ptr[i + 1]; ++f) {
      if (A->col[f] == i) continue;
      Pi += P[rev[f]];
      num += P[rev[f]] * M[rev[f]];
    }
    mean[i] = num / Pi;
    if (prec) prec[i] = Pi;
  }
}

/* r = b - A x (r nullable); returns the Euclidean norm of r. */
double orc_residual(const orc_csr *A, const double *b, const double *x, double *r) {
  double ss = 0.0;
  for (int32_t i = 0; i < A->n; ++i) {
    double ax = 0.0;
    for (int64_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e)
      ax += A->val[e] * x[A->col[e]];
    const double ri = b[i] - ax;
    if (r) r[i] = ri;
    ss += ri * ri;
  }
  return sqrt(ss);
}

/* Proposition GaBPJ: Algorithm 1 with (1) every precision message forced to
 * zero and (2) the target's own message included in the cavity sum.  Only the
 * mean part survives, carried as P_ij mu_ij = -A_ij mu_{i\j} with
 * mu_{i\j} = A_ii^{-1} (b_i + sum_{k in N(i)} P_ki mu_ki).  h holds P*mu per
 * directed edge.  Writes the marginal means mu_i (which then equal mu_{i\j}). */
void orc_jacobi_variant_round(const orc_csr *A, const double *b, const int64_t *rev,
                              const double *diag, const double *hold, double *hnew,
                              double *mean) {
  for (int32_t i = 0; i < A->n; ++i) {
    double num = b[i];
    for (int64_t f = A->row_ptr[i]; f < A->row_ptr[i + 1]; ++f)
      if (A->col[f] != i) num += hold[rev[f]];
    const double mu_cav = num / diag[i];
    mean[i] = mu_cav;
    for (int64_t e = A->row_ptr[i]; e < A->row_ptr[i + 1]; ++e)
      hnew[e] = (A->col[e] == i) ? 0.0 : -A->val[e] * mu_cav;
  }
}

static int all_finite(const double *v, int64_t m) {
  for (int64_t k = 0; k < m; ++k)
    if (!isfinite(v[k])) return 0;
  return 1;
}

/* Synchronous GaBP from the messages in P, M (zeros = Algorithm 1's start).
 * Stops when the chosen rule drops below opts->tol:
 *   ORC_STOP_RESIDUAL: ||b - A x||_2 / ||b||_2,
 *   ORC_STOP_MESSAGES: max over directed messages of |P_new - P_old| and
 *                      |mu_new - mu_old| (the criterion of section VIII),
 *   ORC_STOP_MEANS:    max_i |x_i^t - x_i^{t-1}|.
 * On return P, M hold the last messages; x the marginal means; prec (nullable)
 * the marginal precisions; *rounds the rounds run; trace[t] (nullable, length
 * max_rounds + 1) the relative residual after round t (trace[0]: zero messages).
 */
int orc_solve(const orc_csr *A, const double *b, const orc_opts *o, double *P,
              double *M, double *x, double *prec, int32_t *rounds, double *trace) {
  const int32_t n = A->n;
  const int64_t nnz = A->row_ptr[n];
  if (!o || (o->algorithm != 1 && o->algorithm != 2) || o->max_rounds < 0 ||
      !(o->damping >= 0.0 && o->damping < 1.0))
    return ORC_ERR_ARG;
  int64_t *rev = (int64_t *)malloc(sizeof(int64_t) * (nnz ? nnz : 1));
  double *diag = (double *)malloc(sizeof(double) * (n ? n : 1));
  double *P2 = (double *)malloc(sizeof(double) * (nnz ? nnz : 1));
  double *M2 = (double *)malloc(sizeof(double) * (nnz ? nnz : 1));
  double *xprev = (double *)malloc(sizeof(double) * (n ? n : 1));
  double *pbuf = prec ? prec : (double *)malloc(sizeof(double) * (n ? n : 1));
  int status = orc_build_reverse(A, rev, diag);
  if (status != ORC_OK) goto done;
  double bn = 0.0;
  for (int32_t i = 0; i < n; ++i) bn += b[i] * b[i];
  bn = sqrt(bn);
  if (bn == 0.0) bn = 1.0;

  orc_marginals(A, b, rev, diag, P, M, x, pbuf, o->nthreads);
  if (trace) trace[0] = orc_residual(A, b, x, NULL) / bn;
  status = ORC_NOT_CONVERGED;
  int32_t t = 0;
  int zero_marg = 0;
  while (t < o->max_rounds) {
    memcpy(xprev, x, sizeof(double) * n);
    const int64_t zeros =
        (o->algorithm == 1)
            ? orc_alg1_round(A, b, rev, diag, P, M, P2, M2, o->damping, o->nthreads)
            : orc_alg2_round(A, b, rev, diag, P, M, P2, M2, o->damping, o->nthreads);
    ++t;
    double dmsg = 0.0;
    if (o->stop == ORC_STOP_MESSAGES)
      for (int64_t e = 0; e < nnz; ++e) {
        const double dp = fabs(P2[e] - P[e]), dm = fabs(M2[e] - M[e]);
        if (dp > dmsg) dmsg = dp;
        if (dm > dmsg) dmsg = dm;
      }
    memcpy(P, P2, sizeof(double) * nnz);
    memcpy(M, M2, sizeof(double) * nnz);
    if (zeros) { status = ORC_ERR_BREAKDOWN; break; }
    orc_marginals(A, b, rev, diag, P, M, x, pbuf, o->nthreads);
    /* a zero marginal precision leaves the mean undefined: also a breakdown */
    for (int32_t i = 0; i < n; ++i)
      if (pbuf[i] == 0.0) zero_marg = 1;
    if (zero_marg) { status = ORC_ERR_BREAKDOWN; break; }
    if (!all_finite(P, nnz) || !all_finite(M, nnz) || !all_finite(x, n)) {
      status = ORC_ERR_DIVERGED;
      break;
    }
    const double rr = orc_residual(A, b, x, NULL) / bn;
    if (trace) trace[t] = rr;
    double crit;
    if (o->stop == ORC_STOP_RESIDUAL) crit = rr;
    else if (o->stop == ORC_STOP_MESSAGES) crit = dmsg;
    else {
      crit = 0.0;
      for (int32_t i = 0; i < n; ++i) {
        const double d = fabs(x[i] - xprev[i]);
        if (d > crit) crit = d;
      }
    }
    if (crit < o->tol || (o->stop == ORC_STOP_RESIDUAL && crit <= o->tol)) {
      status = ORC_OK;
      break;
    }
  }
  *rounds = t;
done:
  free(rev); free(diag); free(P2); free(M2); free(xprev);
  if (!prec) free(pbuf);
  return status;
}

/* Iterative refinement around GaBP (not in the paper; its definition is
 * stated here in full).  x = 0, r = b.  Repeat: run GaBP on A d = r from the
 * current messages until max_i |d_i^t - d_i^{t-1}| <= inner_tol * max_i |d_i^t|
 * (or inner_max rounds); x += d; r = b - A x; stop when ||r||/||b|| <= tol;
 * otherwise zero every mean message and keep the precision messages (the
 * precisions do not depend on the right-hand side: Algorithm 1 never reads b
 * in the P update).  Uses Algorithm 2.  Outputs the totals in *rounds and
 * *restarts and the final relative residual in *rel. */
int orc_refine_solve(const orc_csr *A, const double *b, double tol, double inner_tol,
                     int32_t inner_max, int32_t max_restarts, double damping,
                     int32_t nthreads, double *x, double *P, double *M,
                     int32_t *rounds, int32_t *restarts, double *rel) {
  const int32_t n = A->n;
  const int64_t nnz = A->row_ptr[n];
  int64_t *rev = (int64_t *)malloc(sizeof(int64_t) * (nnz ? nnz : 1));
  double *diag = (double *)malloc(sizeof(double) * (n ? n : 1));
  double *P2 = (double *)malloc(sizeof(double) * (nnz ? nnz : 1));
  double *M2 = (double *)malloc(sizeof(double) * (nnz ? nnz : 1));
  double *r = (double *)malloc(sizeof(double) * (n ? n : 1));
  double *d = (double *)malloc(sizeof(double) * (n ? n : 1));
  double *dprev = (double *)malloc(sizeof(double) * (n ? n : 1));
  int status = orc_build_reverse(A, rev, diag);
  *rounds = 0; *restarts = 0; *rel = NAN;
  if (status != ORC_OK) goto done;
  double bn = 0.0;
  for (int32_t i = 0; i < n; ++i) { bn += b[i] * b[i]; x[i] = 0.0; r[i] = b[i]; }
  bn = sqrt(bn);
  if (bn == 0.0) { *rel = 0.0; status = ORC_OK; goto done; }
  status = ORC_NOT_CONVERGED;
  for (int32_t pass = 0; pass <= max_restarts; ++pass) {
    orc_marginals(A, r, rev, diag, P, M, d, NULL, nthreads);
    for (int32_t t = 0; t < inner_max; ++t) {
      memcpy(dprev, d, sizeof(double) * n);
      const int64_t zeros = orc_alg2_round(A, r, rev, diag, P, M, P2, M2, damping, nthreads);
      memcpy(P, P2, sizeof(double) * nnz);
      memcpy(M, M2, sizeof(double) * nnz);
      ++*rounds;
      if (zeros) { status = ORC_ERR_BREAKDOWN; goto done; }
      orc_marginals(A, r, rev, diag, P, M, d, NULL, nthreads);
      if (!all_finite(d, n)) { status = ORC_ERR_DIVERGED; goto done; }
      double dd = 0.0, dm = 0.0;
      for (int32_t i = 0; i < n; ++i) {
        const double c = fabs(d[i] - dprev[i]);
        if (c > dd) dd = c;
        if (fabs(d[i]) > dm) dm = fabs(d[i]);
      }
      if (dd <= inner_tol * dm) break;
    }
    for (int32_t i = 0; i < n; ++i) x[i] += d[i];
    *rel = orc_residual(A, b, x, r) / bn;
    if (*rel <= tol) { status = ORC_OK; break; }
    if (pass == max_restarts) break;
    ++*restarts;
    for (int64_t e = 0; e < nnz; ++e) M[e] = 0.0;
  }
done:
  free(rev); free(diag); free(P2); free(M2); free(r); free(d); free(dprev);
  return status;
}

/* r = b - A x for a stack of `batch` grids nx x ny x nz (node x + nx (y + ny z)
 * per grid) with the 5/7-point operator: diag[i] (or dval everywhere) on the
 * diagonal and, between node i and its +x / +y / +z neighbour inside the same
 * grid, cx[i] / cy[i] / cz[i] (or off everywhere when cx is NULL).  Returns
 * ||r||_2; r nullable.  Same residual definition as orc_residual, written
 * for the structured case so that full-size grids need no CSR. */
double orc_residual_grid(int32_t nx, int32_t ny, int32_t nz, int32_t batch, const double *diag,
                         double dval, const double *cx, const double *cy, const double *cz,
                         double off, const double *b, const double *x, double *r) {
  const int64_t nxy = (int64_t)nx * ny, n = nxy * nz;
  double ss = 0.0;
  for (int64_t t = 0; t < batch; ++t)
    for (int64_t z = 0; z < nz; ++z)
      for (int64_t y = 0; y < ny; ++y)
        for (int64_t xx = 0; xx < nx; ++xx) {
          const int64_t i = t * n + xx + nx * (y + ny * z);
          double ax = (diag ? diag[i] : dval) * x[i];
          if (xx + 1 < nx) ax += (cx ? cx[i] : off) * x[i + 1];
          if (xx > 0) ax += (cx ? cx[i - 1] : off) * x[i - 1];
          if (y + 1 < ny) ax += (cy ? cy[i] : off) * x[i + nx];
          if (y > 0) ax += (cy ? cy[i - nx] : off) * x[i - nx];
          if (z + 1 < nz) ax += (cz ? cz[i] : off) * x[i + nxy];
          if (z > 0) ax += (cz ? cz[i - nxy] : off) * x[i - nxy];
          const double ri = b[i] - ax;
          if (r) r[i] = ri;
          ss += ri * ri;
        }
  return sqrt(ss);
}

/* Section IV-A, Aitken's method, per node on its own history: for three
 * consecutive members x0 = x_n, x1 = x_{n+1}, x2 = x_{n+2} of a sequence
 *   y_n = x_n - (x_{n+1} - x_n)^2 / (x_{n+2} - 2 x_{n+1} + x_n).
 * The paper leaves a vanishing second difference open; then y = x_{n+2} (the
 * sequence is already at rest or moves linearly, and nothing is extrapolated). */
void orc_aitken(int64_t n, const double *x0, const double *x1, const double *x2, double *y) {
  for (int64_t i = 0; i < n; ++i) {
    const double d1 = x1[i] - x0[i];
    const double d2 = x2[i] - 2.0 * x1[i] + x0[i];
    y[i] = (d2 != 0.0) ? x0[i] - d1 * d1 / d2 : x2[i];
  }
}

/* Parallel GaBP + Aitken (section IV-A): synchronous Algorithm 2 rounds from
 * zero messages, unchanged by the extrapolation; the tentative means are
 * sampled every `stride` rounds (x_0 = the means of the zero messages,
 * b_i / A_ii) and, at sample k >= 2, every node extrapolates its own last
 * three samples x_{(k-2)s}, x_{(k-1)s}, x_{ks} to y; at sample 1, y = x_s.
 * The run stops at the first sample whose y has ||b - A y||_2 / ||b||_2 <= tol.
 * y receives that extrapolated vector, *rounds the rounds run.  A stride of 2
 * pairs rounds of equal parity, which matters where the iteration has
 * eigenvalues of both signs (bipartite graphs under the parallel schedule). */
int orc_solve_aitken(const orc_csr *A, const double *b, int32_t stride, double tol,
                     int32_t max_rounds, double damping, int32_t nthreads, double *y,
                     int32_t *rounds) {
  const int32_t n = A->n;
  const int64_t nnz = A->row_ptr[n];
  *rounds = 0;
  if (stride < 1 || max_rounds < 0 || !(damping >= 0.0 && damping < 1.0)) return ORC_ERR_ARG;
  const size_t nb = sizeof(double) * (n ? n : 1), eb = sizeof(double) * (nnz ? nnz : 1);
  int64_t *rev = (int64_t *)malloc(sizeof(int64_t) * (nnz ? nnz : 1));
  double *diag = (double *)malloc(nb), *prec = (double *)malloc(nb);
  double *P = (double *)calloc(nnz ? nnz : 1, sizeof(double));
  double *M = (double *)calloc(nnz ? nnz : 1, sizeof(double));
  double *P2 = (double *)malloc(eb), *M2 = (double *)malloc(eb);
  double *h0 = (double *)malloc(nb), *h1 = (double *)malloc(nb), *h2 = (double *)malloc(nb);
  int status = orc_build_reverse(A, rev, diag);
  if (status != ORC_OK) goto done;
  double bn = 0.0;
  for (int32_t i = 0; i < n; ++i) bn += b[i] * b[i];
  bn = sqrt(bn);
  if (bn == 0.0) bn = 1.0;
  orc_marginals(A, b, rev, diag, P, M, h2, prec, nthreads);  /* x_0 */
  status = ORC_NOT_CONVERGED;
  int32_t k = 0;
  for (int32_t t = 1; t <= max_rounds; ++t) {
    const int64_t zeros = orc_alg2_round(A, b, rev, diag, P, M, P2, M2, damping, nthreads);
    memcpy(P, P2, eb);
    memcpy(M, M2, eb);
    *rounds = t;
    if (zeros) { status = ORC_ERR_BREAKDOWN; break; }
    if (t % stride) continue;
    ++k;
    double *tmp = h0; h0 = h1; h1 = h2; h2 = tmp;  /* h0 <- x_{(k-2)s}, h1 <- x_{(k-1)s} */
    orc_marginals(A, b, rev, diag, P, M, h2, prec, nthreads);
    int zero_marg = 0;
    for (int32_t i = 0; i < n; ++i)
      if (prec[i] == 0.0) zero_marg = 1;
    if (zero_marg) { status = ORC_ERR_BREAKDOWN; break; }
    if (k >= 2) orc_aitken(n, h0, h1, h2, y);
    else memcpy(y, h2, nb);
    if (!all_finite(y, n) || !all_finite(h2, n)) { status = ORC_ERR_DIVERGED; break; }
    if (orc_residual(A, b, y, NULL) / bn <= tol) { status = ORC_OK; break; }
  }
done:
  free(rev); free(diag); free(prec); free(P); free(M); free(P2); free(M2);
  free(h0); free(h1); free(h2);
  return status;
}

/* GaBP + Steffensen (section IV-A): a cycle runs `cycle` synchronous rounds,
 * Aitken extrapolates every node's tentative means from rounds cycle - 2s,
 * cycle - s and cycle (s = stride), and the extrapolated value replaces the
 * iterate before GaBP runs again.  The paper does not say how a vector of
 * means is put back into message form; here GaBP "runs again from y" on the
 * correction system: x <- x + y_d (x = 0 before the first cycle, y_d the
 * extrapolated correction), then the next cycle solves A d = b - A x starting
 * from zero information messages P mu while keeping every precision message
 * (they do not depend on the right-hand side: Algorithm 1 never reads b in the
 * P update).  Stops after the first cycle with ||b - A x||_2 / ||b||_2 <= tol.
 * Outputs x, the rounds and cycles run and the final relative residual. */
int orc_solve_steffensen(const orc_csr *A, const double *b, int32_t stride, int32_t cycle,
                         double tol, int32_t max_cycles, double damping, int32_t nthreads,
                         double *x, int32_t *rounds, int32_t *cycles, double *rel) {
  const int32_t n = A->n;
  const int64_t nnz = A->row_ptr[n];
  *rounds = 0; *cycles = 0; *rel = NAN;
  if (stride < 1 || cycle < 2 * stride || max_cycles < 1 || !(damping >= 0.0 && damping < 1.0))
    return ORC_ERR_ARG;
  const size_t nb = sizeof(double) * (n ? n : 1), eb = sizeof(double) * (nnz ? nnz : 1);
  int64_t *rev = (int64_t *)malloc(sizeof(int64_t) * (nnz ? nnz : 1));
  double *diag = (double *)malloc(nb), *prec = (double *)malloc(nb);
  double *P = (double *)calloc(nnz ? nnz : 1, sizeof(double));
  double *M = (double *)calloc(nnz ? nnz : 1, sizeof(double));
  double *P2 = (double *)malloc(eb), *M2 = (double *)malloc(eb);
  double *r = (double *)malloc(nb), *yd = (double *)malloc(nb);
  double *d0 = (double *)malloc(nb), *d1 = (double *)malloc(nb), *d2 = (double *)malloc(nb);
  int status = orc_build_reverse(A, rev, diag);
  if (status != ORC_OK) goto done;
  double bn = 0.0;
  for (int32_t i = 0; i < n; ++i) { bn += b[i] * b[i]; x[i] = 0.0; r[i] = b[i]; }
  bn = sqrt(bn);
  if (bn == 0.0) { *rel = 0.0; status = ORC_OK; goto done; }
  status = ORC_NOT_CONVERGED;
  for (int32_t c = 0; c < max_cycles; ++c) {
    for (int64_t e = 0; e < nnz; ++e) M[e] = 0.0;  /* information restarts, precisions kept */
    if (cycle == 2 * stride)  /* the first sample is the cycle's starting state */
      orc_marginals(A, r, rev, diag, P, M, d0, prec, nthreads);
    for (int32_t t = 1; t <= cycle; ++t) {
      const int64_t zeros = orc_alg2_round(A, r, rev, diag, P, M, P2, M2, damping, nthreads);
      memcpy(P, P2, eb);
      memcpy(M, M2, eb);
      ++*rounds;
      if (zeros) { status = ORC_ERR_BREAKDOWN; goto done; }
      double *dst = (t == cycle - 2 * stride) ? d0 : (t == cycle - stride) ? d1
                  : (t == cycle) ? d2 : NULL;
      if (!dst) continue;
      orc_marginals(A, r, rev, diag, P, M, dst, prec, nthreads);
      for (int32_t i = 0; i < n; ++i)
        if (prec[i] == 0.0) { status = ORC_ERR_BREAKDOWN; goto done; }
    }
    orc_aitken(n, d0, d1, d2, yd);
    for (int32_t i = 0; i < n; ++i) x[i] += yd[i];
    ++*cycles;
    if (!all_finite(x, n)) { status = ORC_ERR_DIVERGED; break; }
    *rel = orc_residual(A, b, x, r) / bn;
    if (*rel <= tol) { status = ORC_OK; break; }
  }
done:
  free(rev); free(diag); free(prec); free(P); free(M); free(P2); free(M2);
  free(r); free(yd); free(d0); free(d1); free(d2);
  return status;
}
