// Host-side solver engine shared by every matrix kind.  An engine owns the
// device state of one system (graph arrays, message buffers, right-hand side)
// and knows how to launch its kernels; the refinement loop, the chunked
// sweep schedule and the device-side controller are written once in
// engine_solve() (api.cpp) on top of this interface.
#pragma once

#include <algorithm>
#include <atomic>
#include <memory>
#include <string>
#include <vector>

#include "gabp_internal.h"

namespace gabp {

constexpr int kRing = 4;       // readout slots / events in flight
constexpr int kLookahead = 2;  // chunks queued ahead of the one being read

// With GABP_VERBOSE set in the environment, every HIP failure the library
// turns into a status is reported on stderr with its source line.
void report_hip(hipError_t e, const char *file, int line);

inline int from_hip_at(hipError_t e, const char *file, int line) {
  if (e == hipSuccess) return GABP_OK;
  report_hip(e, file, line);
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) return GABP_ERR_NOMEM;
  return GABP_ERR_HIP;
}
#define from_hip(e) from_hip_at((e), __FILE__, __LINE__)

// The launch helpers report hipGetLastError(); an error some earlier,
// unrelated HIP call left behind (the caller's, or an optional attribute
// query of ours) must not be taken for ours, so every entry point of the C
// ABI starts by clearing it.
inline void clear_stale_error() { (void)hipGetLastError(); }

// inside functions that return hipError_t
#define TRY_HIP_E(expr)                \
  do {                                 \
    hipError_t _e = (expr);            \
    if (_e != hipSuccess) return _e;   \
  } while (0)

#define TRY_HIP(expr)                          \
  do {                                         \
    hipError_t _e = (expr);                    \
    if (_e != hipSuccess) return from_hip(_e); \
  } while (0)

// the most LDS one workgroup may use on the current device
inline int max_lds_per_block() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 65536;
  return v;
}

// Device memory held by a plan (memory.cpp): every allocation made while an
// AccountScope of the plan is open on the thread counts until it is freed.
struct DevAccount {
  std::atomic<int64_t> bytes{0};
};
struct AccountScope {
  explicit AccountScope(DevAccount *a);
  ~AccountScope();
  AccountScope(const AccountScope &) = delete;
  AccountScope &operator=(const AccountScope &) = delete;
  DevAccount *prev;
};
hipError_t dalloc_bytes(void **p, size_t bytes);  // hipMalloc, recorded
void dfree(void *p);                               // hipFree, unrecorded (NULL: nothing)

// the plan's account for the duration of an entry point on an existing plan
#define GABP_PLAN_SCOPE(p) gabp::AccountScope gabp_scope_((p) && (p)->acct ? (p)->acct.get() : nullptr)

template <typename P>
hipError_t dalloc(P **p, size_t count, size_t elem) {
  void *q = nullptr;
  const hipError_t e = dalloc_bytes(&q, std::max<size_t>(1, count) * elem);
  *p = (P *)q;
  return e;
}

struct Engine {
  gabp_opts o{};
  int32_t n = 0;      // unknowns
  int64_t E = 0;      // directed edges (messages per sweep)
  bool fp32 = true;
  size_t tsz = 4;
  int cur = 0;        // buffer holding the latest messages
  bool frozen = false;
  // controller plumbing
  BlockPartial *part = nullptr;
  int nparts = 0;     // blocks of a check launch
  double *sumpart = nullptr;
  int nsum = 0;       // blocks of a residual launch
  uint32_t *sticky = nullptr;
  Ctl *ctl = nullptr;
  void *xprev = nullptr;
  // independent systems in one plan (a stack of grids): the residual
  // partials come in nseg runs of segb, and a solve stops when every
  // segment's relative residual meets the tolerance
  int nseg = 1, segb = 0;
  double *segb2 = nullptr;  // ||b_t||^2 per segment
  // per-segment control (engines whose sweeps can skip segments): the check
  // partials are then laid out per segment (launch_readout)
  SegCtl *segctl = nullptr;
  int32_t *segact = nullptr;  // [nseg + 1]: count, then the segments still sweeping
  bool segctl_wanted = false;  // set before init_common
  int seg_grid = 0;            // blocks of a segment sweep launch
  // set by the solve around the pass's x update only: x of a segment with
  // done == 2 stays as it is
  bool infer_skips = false;
  HostReadout *host = nullptr;
  // per chunk: the sweeps' timing events; the readout itself is watched in
  // its host slot (sequence number); ev_sum marks the residual sums' readout
  hipEvent_t ev_beg[kRing] = {}, ev_end[kRing] = {}, ev_sum = nullptr;
  bool events = false;
  int seq = 0;

  virtual ~Engine();
  // allocate the controller plumbing (after n, nparts, nsum are known)
  int init_common(hipStream_t s);
  // entries of xprev (the means of the last check, in the engine's order)
  virtual int64_t means_slots() const { return n; }
  // kernel launches of one sweep
  virtual int sweep_launches() const { return 1; }
  // lowest automatic inner target: the message precision's resolution
  double inner_floor() const { return fp32 ? 1e-7 : 1e-15; }

  // one sweep (mode 0: sweep, 1: sweep + check of the means); c = controller
  // or NULL.  Synchronous: from buffer cur into cur ^ 1; coloured: every
  // colour class in turn, in place.
  virtual hipError_t sweep(int mode, const Ctl *c, hipStream_t s) = 0;
  // x += H/S (FP64), marginal precisions and/or the means in working
  // precision (into `means`, means_slots() entries), from the current messages
  virtual hipError_t infer(double *xacc, double *marg, void *means, hipStream_t s) = 0;
  // zero every information message, keep the precisions (rhs already holds r)
  virtual hipError_t restart(hipStream_t s) = 0;
  // the same, left to the next sweep where the engine can (that sweep takes
  // the informations as zero); anything else that reads messages first
  // carries the restart out
  virtual hipError_t restart_lazy(hipStream_t s) { return restart(s); }
  // x = H/S (FP64) from the current messages
  virtual hipError_t infer_set(double *x, hipStream_t s) {
    hipError_t e = launch_fill_zero(x, n, s);
    return e != hipSuccess ? e : infer(x, nullptr, nullptr, s);
  }
  // the last sweep of a smoothing (mode 0), then x (set: =, else +=) H/S of
  // the messages it leaves; an engine may fuse the two
  virtual hipError_t sweep_means(double *x, bool set, hipStream_t s) {
    hipError_t e = sweep(0, nullptr, s);
    if (e != hipSuccess) return e;
    return set ? infer_set(x, s) : infer(x, nullptr, nullptr, s);
  }
  // zero all messages, rhs = b, full state; ||b||^2 into the residual partials
  virtual hipError_t reset(const double *b, hipStream_t s) = 0;
  // rhs = b - A x (FP64, optionally r64 = the same), ||.||^2 into the partials
  virtual hipError_t residual(const double *b, const double *x, double *r64, hipStream_t s) = 0;
  // settled-precision phase
  virtual bool can_freeze() const { return false; }
  virtual hipError_t ensure_frozen_buffers() { return hipSuccess; }
  virtual bool frozen_ready() const { return false; }
  virtual hipError_t freeze(hipStream_t) { return hipErrorNotSupported; }
  // freeze, then a (lazy) restart: the informations are discarded, so an
  // engine need not carry a pending restart out or copy them
  virtual hipError_t freeze_restart(hipStream_t s) {
    hipError_t e = freeze(s);
    return e != hipSuccess ? e : restart_lazy(s);
  }
  // initial messages from the warm-start network (bfloat16 parameters)
  virtual bool has_warm_start() const { return false; }
  virtual hipError_t warm_start(const uint16_t *, hipStream_t) { return hipErrorNotSupported; }
  // trajectory access (full state only)
  virtual int get_messages(double *P, double *h, hipStream_t s) = 0;
  virtual int set_messages(const double *P, const double *h, hipStream_t s) = 0;

  // readout of the residual partials only; waits for it.  seg_mode (nseg > 1):
  // 1 keeps the per-segment squared norms as ||b_t||^2, 2 reports the largest
  // per-segment relative residual in outv->segrel (bnorm = ||b||)
  int read_sum(hipStream_t s, HostReadout *outv, int seg_mode = 0, double bnorm = 0.0);
  // read_sum in two halves: post_sum enqueues the reduction into its own host
  // slot, wait_sum waits for it and copies the readout
  int post_sum(hipStream_t s, int seg_mode = 0, double bnorm = 0.0);
  int wait_sum(HostReadout *outv);
};

// refinement loop around chunked sweeps (api.cpp)
int engine_solve(Engine *e, const double *b, double *x, double *marg, gabp_stats *st,
                 hipStream_t s, const uint16_t *warm = nullptr);

// persistent autotuning cache (tune_cache.cpp): key = arch | version | kernel | shape class
std::string tune_key(const std::string &kernel, const std::string &shape);
bool tune_lookup(const std::string &key, int *value);
void tune_store(const std::string &key, int value);

int check_opts(const gabp_opts *o);  // engine_csr.cpp
int check_csr(const gabp_csr *A);    // engine_csr.cpp: sizes, pointers, row_ptr ends
// a CSR plan; classes = row offsets of colour classes (coloured schedule) or
// NULL (engine_csr.cpp)
int csr_plan_create(const gabp_csr *A, const gabp_opts *o, const std::vector<int> *classes,
                    gabp_plan **plan, hipStream_t s);
int check_grid(const gabp_grid *A, GridGeom *g);  // engine_grid.cpp

// batches of dense instances (engine_dense.cpp)
struct BatchEngine;
int batch_create(const gabp_batch *B, const gabp_opts *o, BatchEngine **out, hipStream_t s);
void batch_destroy(BatchEngine *e);
int batch_solve(BatchEngine *e, const double *b, double *x, double *marg_prec, gabp_stats *per,
                gabp_stats *summary, hipStream_t s);
int batch_reset(BatchEngine *e, const double *b, hipStream_t s);
int batch_sweeps(BatchEngine *e, int count, hipStream_t s);
int batch_marginals(BatchEngine *e, double *mean, double *prec, hipStream_t s);

// coarse-grid predicted corrections of grid plans (engine_grid.cpp)
struct CoarseHierarchy;
void coarse_destroy(CoarseHierarchy *h);
int coarse_solve(gabp_plan *p, const double *b, double *x, double *marg_prec, gabp_stats *st,
                 hipStream_t s);

// batches of small sparse instances, one workgroup each (engine_small.cpp)
struct SmallEngine;
int small_create(const gabp_batch *B, const gabp_opts *o, SmallEngine **out, hipStream_t s);
void small_destroy(SmallEngine *e);
int small_solve(SmallEngine *e, const double *b, double *x, double *marg_prec, gabp_stats *per,
                gabp_stats *summary, hipStream_t s);
int small_reset(SmallEngine *e, const double *b, hipStream_t s);
int small_sweeps(SmallEngine *e, int count, hipStream_t s);
int small_marginals(SmallEngine *e, double *mean, double *prec, hipStream_t s);
int small_messages(SmallEngine *e, double *P, double *h, bool set, hipStream_t s);
int small_colors(const SmallEngine *e, int32_t *colors, int32_t *ncolors, hipStream_t s);

}  // namespace gabp

namespace gabp {
// the assembled section VII system of an lsq plan (engine_lsq.cpp)
struct LsqSystem;
void lsq_destroy(LsqSystem *q);
bool lsq_coloured(const LsqSystem *q);
int lsq_colors(const LsqSystem *q, int32_t *colors, int32_t *ncolors, hipStream_t s);
// the colour-sorted renumbering of a coloured CSR plan (engine_color.cpp)
struct CsrPerm;
void perm_destroy(CsrPerm *q);
int coloured_csr_plan(const gabp_csr *A, const gabp_opts *o, gabp_plan **plan, hipStream_t s);
// a coloured CSR plan's vectors in and out of its renumbered order
// (engine_color.cpp): b into the plan's own buffer (returned), and x / the
// marginal precisions back from them
const double *perm_in(CsrPerm *q, const double *b, hipStream_t s);
int perm_solve(CsrPerm *q, Engine *e, const double *b, double *x, double *marg, gabp_stats *st,
               hipStream_t s);
int perm_marginals(CsrPerm *q, Engine *e, double *mean, double *prec, hipStream_t s);
int perm_colors(const CsrPerm *q, int32_t *colors, int32_t *ncolors, hipStream_t s);
// get (set = false) or set messages in the caller's CSR slot order
int perm_messages(CsrPerm *q, Engine *e, double *P, double *h, bool set, hipStream_t s);
}  // namespace gabp

// the opaque plan of the C ABI: one system (eng), a batch of dense instances
// (bat), a batch of small sparse instances (small); an lsq plan is a CSR system (eng) over its own assembled matrix (lsq);
// a coloured CSR plan runs on a colour-sorted renumbering of the caller's
// matrix (perm)
struct gabp_plan {
  // the account its device allocations count against
  std::shared_ptr<gabp::DevAccount> acct;
  gabp::Engine *eng = nullptr;
  gabp::BatchEngine *bat = nullptr;
  gabp::SmallEngine *small = nullptr;
  gabp::CoarseHierarchy *coarse = nullptr;  // grid plans: coarse levels, built on first use
  gabp::LsqSystem *lsq = nullptr;
  gabp::CsrPerm *perm = nullptr;
};

namespace gabp {
// Runs a plan constructor f (which stores the new plan in *plan) with a fresh
// account open, so that everything it allocates counts for the new plan.
template <typename F>
int with_account(gabp_plan **plan, F f) {
  auto acct = std::make_shared<DevAccount>();
  int rc;
  {
    AccountScope scope(acct.get());
    rc = f();
  }
  if (rc == GABP_OK && plan && *plan) (*plan)->acct = acct;
  return rc;
}
int64_t coarse_bytes(const CoarseHierarchy *h);  // the coarse levels' own plans
}  // namespace gabp
