// General sparse matrices (CSR): plan construction on the device, the two
// message layouts (pair: both directions per edge slot with node broadcasts;
// gather: out-messages per slot with in-messages through the reverse-edge
// index) and the settled-precision phase of the pair layout.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "engine.h"

namespace gabp {
namespace {

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

int check_csr(const gabp_csr *A) {
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

int check_opts(const gabp_opts *o) {
  if (!(o->tol >= 0.0) || o->max_sweeps < 0 || o->check_every < 0 || !(o->damping >= 0.0) ||
      !(o->damping < 1.0) || !(o->inner_tol >= 0.0) || o->max_restarts < 0 ||
      !(o->freeze_tol >= 0.0) || !(o->freeze_tol < 1.0) ||
      (o->group != 0 && !valid_group(o->group)) || o->grid_blocks < 0 ||
      (o->layout != GABP_LAYOUT_PAIR && o->layout != GABP_LAYOUT_GATHER) ||
      (o->schedule != GABP_SCHEDULE_SYNC && o->schedule != GABP_SCHEDULE_COLORED) ||
      o->col_blocks < 0 || o->col_blocks > 2 || o->accel < GABP_ACCEL_NONE ||
      o->accel > GABP_ACCEL_STEFFENSEN || o->accel_stride < 0 || o->accel_cycle < 0)
    return GABP_ERR_ARG;
  if (o->accel == GABP_ACCEL_STEFFENSEN) {
    const int stride = o->accel_stride ? o->accel_stride : 2;
    const int cycle = o->accel_cycle ? o->accel_cycle : 100;
    if (cycle < 2 * stride) return GABP_ERR_ARG;
  }
  return GABP_OK;
}

struct CsrEngine : Engine {
  gabp_csr A{};
  bool pair = true;
  int group = 8;
  int grid = 1;       // blocks of a row-kernel launch
  // pair sweeps: row blocks (offsets rblk, pair_row_blocks), the first block
  // of every colour class (or of the one range) and the workgroups a sweep
  // launch walks them with
  int32_t *rblk = nullptr;
  std::vector<int> bfirst;
  int sgrid = 1;
  // column ranges of the synchronous pair layout (1 or 2): range p of row i
  // is virtual row p * n + i (oprt has nb * n + 1 offsets); with 2, a sweep's
  // first launch leaves the first range's node sums in `carry` and the second
  // continues from them
  int nb = 1;
  void *carry = nullptr;
  int32_t *oprt = nullptr, *ocol = nullptr, *rev = nullptr;
  int64_t *diagpos = nullptr;
  void *acoef = nullptr, *diag = nullptr, *rhs = nullptr;
  // gather layout: (P, h) out-message per slot; pair layout: (P_ij, h_ij, P_ji, h_ji)
  void *msg[2] = {nullptr, nullptr};
  void *sums[2] = {nullptr, nullptr};  // pair: (S, H) per node
  // settled-precision phase (pair layout, allocated on first use)
  void *coef = nullptr, *hp[2] = {nullptr, nullptr}, *Sfix = nullptr, *Hfz[2] = {nullptr, nullptr};
  // coloured schedule (pair layout): class c is rows [cls[c], cls[c + 1]);
  // one buffer (index 0), updated in place by one launch per class
  std::vector<int> cls;
  bool first = true;  // no sweep since the messages were set (reset, restart, import)
  // synchronous pair plans after a reset: every message is zero and msg[cur]
  // has not been written (the first sweep reads no slot state)
  bool zero_msgs = false;

  ~CsrEngine() override {
    void *bufs[] = {oprt, ocol, rev, diagpos, acoef, diag, rhs, msg[0], msg[1], sums[0],
                    sums[1], coef, hp[0], hp[1], Sfix, Hfz[0], Hfz[1], rblk, carry};
    for (void *b : bufs)
      if (b) dfree(b);
  }

  size_t msg_bytes() const { return (pair ? 4 : 2) * tsz; }

  bool colored() const { return !cls.empty(); }

  int sweep_launches() const override { return colored() ? (int)cls.size() - 1 : (pair ? nb : 1); }

  // workgroups of a launch over all row blocks
  int bgrid() const { return std::max(1, std::min(bfirst.back(), pair_max_blocks())); }

  // node sums from the stored in-messages, range by range as the sweeps add
  // them (one range: every row block, colour classes included)
  hipError_t aggregate(const void *m, void *out, hipStream_t s) {
    if (nb == 1)
      return launch_pair_aggregate(fp32, bgrid(), rblk, 0, bfirst.back(), 0, oprt, diag, rhs, m,
                                   nullptr, out, true, s);
    for (int p = 0; p < nb; ++p) {
      const bool last = p == nb - 1;
      hipError_t err = launch_pair_aggregate(fp32, sgrid, rblk, bfirst[p], bfirst[p + 1], p * n,
                                             oprt, diag, rhs, m, p > 0 ? carry : nullptr,
                                             last ? out : carry, last, s);
      if (err != hipSuccess) return err;
    }
    return hipSuccess;
  }

  hipError_t sweep(int mode, const Ctl *c, hipStream_t s) override {
    hipError_t err;
    if (colored()) {
      for (size_t k = 0; k + 1 < cls.size(); ++k) {
        PairArgs a{};
        a.grid = sgrid; a.fp32 = fp32; a.group = group; a.mode = mode; a.damp = o.damping > 0.0;
        a.frozen = frozen; a.n = n; a.oprt = oprt; a.ocol = ocol; a.acoef = acoef; a.diag = diag;
        a.rhs = rhs; a.alpha = o.damping; a.xprev = xprev; a.part = part; a.sticky = sticky;
        a.ctl = c; a.colored = true; a.nslots = nparts; a.row0 = cls[k]; a.row1 = cls[k + 1];
        a.rb = rblk; a.b0 = bfirst[k]; a.b1 = bfirst[k + 1];
        a.first = first;
        if (frozen) {
          a.coef = coef; a.Sfix = Sfix; a.msg_out = hp[0]; a.sums_out = Hfz[0];
        } else {
          a.msg_out = msg[0]; a.sums_out = sums[0];
        }
        a.msg_in = a.msg_out; a.sums_in = a.sums_out;
        if ((err = launch_pair_sweep(a, s)) != hipSuccess) return err;
      }
      first = false;
      return hipSuccess;
    }
    if (!pair) {
      SweepArgs a{};
      a.grid = grid; a.fp32 = fp32; a.group = group; a.mode = mode; a.damp = o.damping > 0.0;
      a.n = n; a.oprt = oprt; a.rev = rev; a.acoef = acoef; a.diag = diag; a.rhs = rhs;
      a.msg_in = msg[cur]; a.msg_out = msg[cur ^ 1]; a.alpha = o.damping; a.xprev = xprev;
      a.part = part; a.sticky = sticky; a.ctl = c;
      err = launch_sweep(a, s);
    } else {
      PairArgs a{};
      a.grid = sgrid; a.fp32 = fp32; a.group = group; a.mode = mode; a.damp = o.damping > 0.0;
      a.frozen = frozen; a.n = n; a.rb = rblk; a.nslots = nparts;
      a.oprt = oprt; a.ocol = ocol; a.acoef = acoef; a.diag = diag;
      a.rhs = rhs; a.alpha = o.damping; a.xprev = xprev; a.part = part; a.sticky = sticky;
      a.ctl = c;
      if (frozen) {
        a.coef = coef; a.Sfix = Sfix;
        a.msg_in = hp[cur]; a.msg_out = hp[cur ^ 1]; a.sums_in = Hfz[cur]; a.sums_out = Hfz[cur ^ 1];
      } else {
        a.msg_in = zero_msgs ? nullptr : msg[cur]; a.msg_out = msg[cur ^ 1];
        a.sums_in = sums[cur]; a.sums_out = sums[cur ^ 1];
        zero_msgs = false;
      }
      void *final_out = a.sums_out;
      err = hipSuccess;
      for (int p = 0; p < nb && err == hipSuccess; ++p) {
        a.b0 = bfirst[p];
        a.b1 = bfirst[p + 1];
        a.vbase = p * n;
        a.carry = p > 0 ? carry : nullptr;
        a.last = p == nb - 1;
        a.sums_out = a.last ? final_out : carry;
        err = launch_pair_sweep(a, s);
      }
    }
    cur ^= 1;
    return err;
  }

  hipError_t infer(double *xacc, double *marg, void *means, hipStream_t s) override {
    if (!pair) {
      SweepArgs a{};
      a.grid = grid; a.fp32 = fp32; a.group = group; a.mode = 2; a.n = n; a.oprt = oprt;
      a.rev = rev; a.acoef = acoef; a.diag = diag; a.rhs = rhs; a.msg_in = msg[cur];
      a.xacc = xacc; a.marg = marg; a.xprev = means; a.sticky = sticky;
      return launch_sweep(a, s);
    }
    if (colored() && !first) {
      // the broadcasts of earlier classes predate the later classes' messages
      PairArgs a{};
      a.grid = grid; a.fp32 = fp32; a.group = group; a.damp = o.damping > 0.0; a.frozen = frozen;
      a.n = n; a.oprt = oprt; a.ocol = ocol; a.acoef = acoef; a.diag = diag; a.rhs = rhs;
      a.alpha = o.damping; a.sticky = sticky; a.coef = coef; a.Sfix = Sfix;
      a.msg_in = frozen ? hp[0] : msg[0];
      a.sums_in = frozen ? Hfz[0] : sums[0];
      for (size_t k = 0; k + 1 < cls.size(); ++k) {
        a.row0 = cls[k];
        a.row1 = cls[k + 1];
        a.rb = rblk;
        a.b0 = bfirst[k];
        a.b1 = bfirst[k + 1];
        a.grid = std::max(1, std::min(a.b1 - a.b0, pair_max_blocks()));
        hipError_t err = launch_pair_col_infer(a, xacc, marg, means, s);
        if (err != hipSuccess) return err;
      }
      return hipSuccess;
    }
    if (frozen)
      return launch_pair_infer(fp32, n, nullptr, Sfix, Hfz[cur], xacc, marg, means, sticky, s);
    return launch_pair_infer(fp32, n, sums[cur], nullptr, nullptr, xacc, marg, means, sticky, s);
  }

  hipError_t restart(hipStream_t s) override {
    first = true;
    if (!pair) return launch_zero_h(fp32, E, msg[cur], s);
    if (frozen) return launch_frozen_restart(fp32, E, n, hp[cur], rhs, Hfz[cur], s);
    if (zero_msgs) return aggregate(nullptr, sums[cur], s);  // nothing sent yet
    hipError_t err = launch_pair_zero_h(fp32, E, msg[cur], s);
    if (err != hipSuccess) return err;
    // coloured: a row's stored copy of a later class's precision message is
    // one half sweep old; make every copy the sender's current message
    if (colored() && (err = launch_pair_sync_in(fp32, E, rev, msg[cur], s)) != hipSuccess)
      return err;
    return aggregate(msg[cur], sums[cur], s);
  }

  hipError_t reset(const double *b, hipStream_t s) override {
    cur = 0;
    frozen = false;
    first = true;
    const int64_t words = E * (int64_t)msg_bytes() / 8;
    hipError_t err;
    // No slot state needs clearing for a synchronous pair plan: its first
    // sweep takes every message as zero and writes every slot of msg[1].
    // Coloured sweeps work in msg[0] and the gather layout reads it.
    zero_msgs = pair && !colored();
    if (!zero_msgs && (err = launch_fill_zero(msg[0], words, s)) != hipSuccess) return err;
    if ((err = launch_residual(fp32, nsum, n, A.row_ptr, A.col, A.val, b, nullptr, rhs,
                               nullptr, sumpart, s)) != hipSuccess)
      return err;
    if (pair) return aggregate(zero_msgs ? nullptr : msg[0], sums[0], s);
    return hipSuccess;
  }

  hipError_t residual(const double *b, const double *x, double *r64, hipStream_t s) override {
    return launch_residual(fp32, nsum, n, A.row_ptr, A.col, A.val, b, x, rhs, r64,
                           sumpart, s);
  }

  bool can_freeze() const override { return pair; }

  hipError_t ensure_frozen_buffers() override {
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

  bool frozen_ready() const override {
    return coef && hp[0] && hp[1] && Sfix && Hfz[0] && Hfz[1];
  }

  hipError_t freeze(hipStream_t s) override {
    if (zero_msgs) {  // not reached by a solve (it freezes after sweeps); kept well defined
      hipError_t err = launch_fill_zero(msg[cur], E * (int64_t)msg_bytes() / 8, s);
      if (err != hipSuccess) return err;
      zero_msgs = false;
    }
    hipError_t err = launch_pair_freeze(fp32, bgrid(), rblk, bfirst.back(), n, oprt, ocol, rev,
                                        colored(), acoef, msg[cur], sums[cur], coef, hp[cur], Sfix,
                                        Hfz[cur], s);
    frozen = true;
    return err;
  }

  int get_messages(double *P, double *h, hipStream_t s) override {
    if (A.nnz > 0 && (!P || !h)) return GABP_ERR_ARG;
    if (zero_msgs) {
      TRY_HIP(launch_fill_zero(P, A.nnz, s));
      TRY_HIP(launch_fill_zero(h, A.nnz, s));
    } else if (pair)
      TRY_HIP(launch_pair_io(fp32, true, n, nb, A.row_ptr, diagpos, oprt, rev, msg[cur], P, h, s));
    else
      TRY_HIP(launch_get_msgs(fp32, n, A.row_ptr, diagpos, oprt, msg[cur], P, h, s));
    TRY_HIP(hipStreamSynchronize(s));
    return GABP_OK;
  }

  int set_messages(const double *P, const double *h, hipStream_t s) override {
    if (A.nnz > 0 && (!P || !h)) return GABP_ERR_ARG;
    first = true;
    zero_msgs = false;  // every slot is written
    if (pair) {
      TRY_HIP(launch_pair_io(fp32, false, n, nb, A.row_ptr, diagpos, oprt, rev, msg[cur], (double *)P,
                             (double *)h, s));
      TRY_HIP(aggregate(msg[cur], sums[cur], s));
    } else {
      TRY_HIP(launch_set_msgs(fp32, n, A.row_ptr, diagpos, oprt, msg[cur], P, h, s));
    }
    TRY_HIP(hipStreamSynchronize(s));
    return GABP_OK;
  }

  // Row blocks of the pair sweeps from a host copy of the slot offsets; every
  // class launch of a coloured sweep has the same workgroups, so a check's
  // partials line up.
  int row_blocks(int cap, hipStream_t s) {
    std::vector<int32_t> hrp((size_t)nb * n + 1, 0);
    if (n > 0) {
      TRY_HIP(hipMemcpyAsync(hrp.data(), oprt, hrp.size() * sizeof(int32_t),
                             hipMemcpyDeviceToHost, s));
      TRY_HIP(hipStreamSynchronize(s));
    }
    std::vector<int> bounds = colored() ? cls : std::vector<int>{0, n};
    if (nb == 2) bounds.push_back(2 * n);
    const std::vector<int32_t> rb = pair_row_blocks(hrp.data(), bounds, &bfirst);
    int most = 1;
    for (size_t k = 0; k + 1 < bfirst.size(); ++k) most = std::max(most, bfirst[k + 1] - bfirst[k]);
    sgrid = std::min(most, cap);
    nparts = std::min(sgrid, 1024);  // check partial slots (slot_publish)
    TRY_HIP(dalloc(&rblk, rb.size(), sizeof(int32_t)));
    if (nb > 1) TRY_HIP(dalloc(&carry, n, 2 * tsz));
    TRY_HIP(hipMemcpyAsync(rblk, rb.data(), rb.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    TRY_HIP(hipStreamSynchronize(s));
    return GABP_OK;
  }

  // validate A on the device and build the edge arrays and reverse index
  int build(hipStream_t s) {
    int64_t *deg = nullptr, *vo = nullptr, *tmp = nullptr, *L = nullptr;
    uint32_t *flags = nullptr;
    unsigned long long *far = nullptr;
    int st = GABP_OK;
    auto fail = [&](int code) {
      void *bufs[] = {deg, vo, tmp, L, flags, far};
      for (void *b : bufs)
        if (b) dfree(b);
      return code;
    };
    if ((st = from_hip(dalloc(&deg, n, sizeof(int64_t)))) ||
        (st = from_hip(dalloc(&diagpos, n, sizeof(int64_t)))) ||
        (st = from_hip(dalloc(&flags, 1, sizeof(uint32_t)))))
      return fail(st);
    if ((st = from_hip(launch_fill_zero4(flags, 1, s))) ||
        (st = from_hip(launch_plan_rows(n, A.nnz, A.row_ptr, A.col, A.val, deg, diagpos, flags, s))))
      return fail(st);
    uint32_t hflags = 0;
    if ((st = from_hip(hipMemcpyAsync(&hflags, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s))) ||
        (st = from_hip(hipStreamSynchronize(s))))
      return fail(st);
    if (hflags & FLAG_ARG) return fail(GABP_ERR_ARG);
    if (hflags & FLAG_ZERO_DIAG) return fail(GABP_ERR_ZERO_DIAG);
    // column ranges (pair layout, synchronous schedule)
    nb = 1;
    if (pair && !colored() && o.col_blocks != 1) {
      const int split = (n + 1) / 2;
      if ((st = from_hip(dalloc(&L, 2 * (size_t)n, sizeof(int64_t)))) ||
          (st = from_hip(dalloc(&far, 1, sizeof(unsigned long long)))) ||
          (st = from_hip(hipMemsetAsync(far, 0, sizeof(unsigned long long), s))) ||
          (st = from_hip(launch_plan_split(n, A.row_ptr, A.col, diagpos, split, L, far, s))))
        return fail(st);
      unsigned long long hfar = 0;
      if ((st = from_hip(hipMemcpyAsync(&hfar, far, sizeof(hfar), hipMemcpyDeviceToHost, s))) ||
          (st = from_hip(hipStreamSynchronize(s))))
        return fail(st);
      const int64_t offdiag = A.nnz - n;
      const bool big = (int64_t)n * 2 * (int64_t)tsz > ((int64_t)4 << 20);
      nb = (o.col_blocks == 2 || (big && offdiag > 0 && 2 * (int64_t)hfar >= offdiag)) ? 2 : 1;
    }
    const int64_t vrows = (int64_t)nb * n;
    if ((st = from_hip(dalloc(&vo, vrows + 1, sizeof(int64_t)))) ||
        (st = from_hip(dalloc(&tmp, scan_tmp_elems(vrows), sizeof(int64_t)))) ||
        (st = from_hip(launch_scan(nb == 2 ? L : deg, vo, vrows, tmp, s))))
      return fail(st);
    int64_t e = 0;
    if ((st = from_hip(hipMemcpyAsync(&e, vo + vrows, sizeof(int64_t), hipMemcpyDeviceToHost, s))) ||
        (st = from_hip(hipStreamSynchronize(s))))
      return fail(st);
    // slot indices stay in int32 with a chunk of headroom
    if (e >= (int64_t)INT32_MAX - 4096) return fail(GABP_ERR_UNSUPPORTED);
    E = e;
    if ((st = from_hip(dalloc(&oprt, vrows + 1, sizeof(int32_t)))) ||
        (st = from_hip(dalloc(&ocol, E, sizeof(int32_t)))) ||
        (st = from_hip(dalloc(&rev, E, sizeof(int32_t)))) ||
        (st = from_hip(dalloc(&acoef, E, tsz))) || (st = from_hip(dalloc(&diag, n, tsz))))
      return fail(st);
    if ((st = from_hip(launch_plan_edges(fp32, n, nb, A.row_ptr, A.col, A.val, diagpos, vo, oprt,
                                         ocol, rev, acoef, diag, flags, s))))
      return fail(st);
    if ((st = from_hip(hipMemcpyAsync(&hflags, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s))) ||
        (st = from_hip(hipStreamSynchronize(s))))
      return fail(st);
    if (hflags & FLAG_ASYM) return fail(GABP_ERR_NOT_SYMMETRIC);
    return fail(GABP_OK);
  }
};

// A CSR plan; `classes` (row offsets of the colour classes, classes[0] = 0,
// last = n) selects the coloured schedule, NULL the synchronous one.
int csr_plan_create(const gabp_csr *A, const gabp_opts *o, const std::vector<int> *classes,
                    gabp_plan **plan, hipStream_t s) {
  if (!plan) return GABP_ERR_ARG;
  *plan = nullptr;
  gabp_opts opts;
  if (o) opts = *o;
  else gabp_default_opts(&opts);
  int st = check_csr(A);
  if (st) return st;
  if ((st = check_opts(&opts))) return st;
  if (opts.accel != GABP_ACCEL_NONE) return GABP_ERR_UNSUPPORTED;  // small CSR batches only
  if ((opts.schedule != GABP_SCHEDULE_SYNC) != (classes != nullptr)) return GABP_ERR_UNSUPPORTED;
  if (classes && opts.layout != GABP_LAYOUT_PAIR) return GABP_ERR_UNSUPPORTED;
  if (opts.col_blocks == 2 && (classes || opts.layout != GABP_LAYOUT_PAIR))
    return GABP_ERR_UNSUPPORTED;
  CsrEngine *e = new (std::nothrow) CsrEngine();
  if (!e) return GABP_ERR_NOMEM;
  e->A = *A;
  e->o = opts;
  e->n = A->n;
  e->fp32 = opts.msg_fp32 != 0;
  e->pair = opts.layout == GABP_LAYOUT_PAIR;
  e->tsz = e->fp32 ? sizeof(float) : sizeof(double);
  auto fail = [&](int code) {
    delete e;
    return code;
  };
  if (classes) e->cls = *classes;
  if (e->n > 0 && (st = e->build(s))) return fail(st);
  e->group = opts.group ? opts.group : choose_group(e->n, e->E);
  const int cap = opts.grid_blocks > 0 ? opts.grid_blocks : kMaxSweepBlocks;
  e->grid = sweep_blocks(std::max(e->n, 1), e->group, cap);
  e->nparts = e->grid;
  if (e->pair && (st = e->row_blocks(opts.grid_blocks > 0 ? opts.grid_blocks : pair_max_blocks(), s)))
    return fail(st);
  e->nsum = residual_blocks(std::max(e->n, 1), cap);
  if ((st = e->init_common(s))) return fail(st);
  if ((st = from_hip(dalloc(&e->msg[0], e->E, e->msg_bytes()))) ||
      (st = from_hip(dalloc(&e->msg[1], e->E, e->msg_bytes()))) ||
      (st = from_hip(dalloc(&e->rhs, e->n, e->tsz))))
    return fail(st);
  if (e->pair && ((st = from_hip(dalloc(&e->sums[0], e->n, 2 * e->tsz))) ||
                  (st = from_hip(dalloc(&e->sums[1], e->n, 2 * e->tsz)))))
    return fail(st);
  gabp_plan *p = new (std::nothrow) gabp_plan();
  if (!p) return fail(GABP_ERR_NOMEM);
  p->eng = e;
  *plan = p;
  return GABP_OK;
}

}  // namespace gabp

using namespace gabp;

extern "C" {

static int plan_create_impl(const gabp_csr *A, const gabp_opts *o, gabp_plan **plan, hipStream_t s) {
  clear_stale_error();
  if (!plan) return GABP_ERR_ARG;
  if (o && o->schedule == GABP_SCHEDULE_COLORED) {
    if (o->layout != GABP_LAYOUT_PAIR) return GABP_ERR_UNSUPPORTED;
    int st = check_opts(o);
    if (!st && o->col_blocks == 2) st = GABP_ERR_UNSUPPORTED;
    return st ? st : coloured_csr_plan(A, o, plan, s);
  }
  return csr_plan_create(A, o, nullptr, plan, s);
}

int gabp_plan_create(const gabp_csr *A, const gabp_opts *o, gabp_plan **plan, hipStream_t s) {
  return with_account(plan, [&] { return plan_create_impl(A, o, plan, s); });
}

int gabp_solve(const gabp_csr *A, const double *b, double *x, double *marg_prec,
               const gabp_opts *o, gabp_stats *st, hipStream_t s) {
  clear_stale_error();
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
  clear_stale_error();
  int rc = check_csr(A);
  if (rc) return rc;
  if (!rel_norm || (A->n > 0 && (!b || !x))) return GABP_ERR_ARG;
  if (A->n == 0) { *rel_norm = 0.0; return GABP_OK; }
  const int nb = residual_blocks(A->n);
  double *sum = nullptr;
  int64_t *deg = nullptr, *dpos = nullptr;
  uint32_t *flags = nullptr;
  HostReadout *host = nullptr;
  hipEvent_t ev = nullptr;
  auto cleanup = [&](int code) {
    void *bufs[] = {sum, deg, dpos, flags};
    for (void *b : bufs)
      if (b) dfree(b);
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
  if ((rc = from_hip(launch_residual(false, nb, A->n, A->row_ptr, A->col, A->val, b, nullptr,
                                     nullptr, nullptr, sum, s))) ||
      (rc = from_hip(launch_readout(nullptr, 0, sum, nb, nullptr, nullptr, 0, 0, &host[0], s))) ||
      (rc = from_hip(launch_residual(false, nb, A->n, A->row_ptr, A->col, A->val, b, x, nullptr,
                                     r, sum, s))) ||
      (rc = from_hip(launch_readout(nullptr, 0, sum, nb, nullptr, nullptr, 0, 1, &host[1], s))) ||
      (rc = from_hip(hipEventRecord(ev, s))) || (rc = from_hip(hipEventSynchronize(ev))))
    return cleanup(rc);
  const double bn = std::sqrt(host[0].sum), rn = std::sqrt(host[1].sum);
  *rel_norm = bn > 0 ? rn / bn : rn;
  return cleanup(std::isfinite(*rel_norm) ? GABP_OK : GABP_ERR_ARG);
}

}  // extern "C"
