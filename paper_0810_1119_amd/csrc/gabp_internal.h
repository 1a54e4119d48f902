// Internal declarations shared by the HIP kernels and the host side of the
// C ABI.  Nothing here is part of the public interface (include/gabp.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "gabp.h"

namespace gabp {

// Sticky error bits raised by kernels (atomicOr, only when the event occurs).
enum : uint32_t {
  FLAG_BREAKDOWN = 1u,   // zero cavity or marginal precision
  FLAG_NONFINITE = 2u,   // non-finite mean seen at a check
  FLAG_ASYM = 4u,        // pattern or value asymmetry (plan build)
  FLAG_ZERO_DIAG = 8u,   // missing or zero diagonal (plan build)
  FLAG_ARG = 16u,        // malformed CSR or non-finite value (plan build)
};

// Why an inner solve stopped (written by the device-side controller).
enum : uint32_t {
  STOP_NONE = 0, STOP_CONVERGED = 1, STOP_STALLED = 2, STOP_NONFINITE = 3,
};

// Per-block result of a check sweep: largest change of a marginal mean over
// the check interval and largest |mean|.
struct BlockPartial {
  double dmax;
  double xmax;
};

// Device-resident controller of an inner solve.  Only the single-thread
// readout kernel writes it, in stream order, so no atomics are needed; the
// sweep kernels read `stop` once at entry and skip all work when it is set.
struct Ctl {
  uint32_t stop;       // STOP_*
  int32_t sweeps;      // sweeps actually executed in this solve
  int32_t checks;      // checks evaluated
  int32_t stall;       // consecutive checks without progress
  double best;         // best relative change seen in this inner solve
  double inner_tol;    // stop threshold on max|dx| / max|x|
  double stall_floor;  // below this level 8 checks without a 1% gain = stall
  double last_d;       // last max|dx|
  double last_x;       // last max|x|
};

// What the host reads back (pinned, written by the readout kernel).
struct HostReadout {
  double dmax;
  double xmax;
  double sum;          // sum of the residual partials (||r||^2)
  uint32_t flags;      // sticky flags at readout time
  uint32_t stop;       // controller state
  int32_t sweeps;
  int32_t seq;         // chunk sequence number (sanity check)
};

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

constexpr int kBlock = 256;  // threads per block of the row kernels

// ---- launchers (kernels_csr.hip) ----
hipError_t launch_plan_rows(int n, int64_t nnz, const int64_t *rp, const int32_t *col,
                            const double *val, int64_t *deg, int64_t *diagpos, uint32_t *flags,
                            hipStream_t s);
// Exclusive scan of in[0..n) into out[0..n] (out[n] = total).  tmp must hold
// scan_tmp_elems(n) int64 values.
size_t scan_tmp_elems(int64_t n);
hipError_t launch_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s);
hipError_t launch_plan_edges(bool fp32, int n, const int64_t *rp, const int32_t *col,
                             const double *val, const int64_t *diagpos, const int64_t *oprt64,
                             int32_t *oprt, int32_t *rev, void *acoef, void *diag,
                             uint32_t *flags, hipStream_t s);

struct SweepArgs {
  bool fp32;
  int group;           // lanes per row
  int mode;            // 0 sweep, 1 sweep + check, 2 infer (means/precisions only)
  bool damp;
  int n;
  const int32_t *oprt, *rev;
  const void *acoef, *diag, *rhs;
  const void *msg_in;
  void *msg_out;
  double alpha;
  void *xprev;         // mode 1
  double *xacc;        // mode 2: x += H/S (nullable)
  double *marg;        // mode 2: marginal precision S (nullable)
  BlockPartial *part;  // mode 1
  uint32_t *sticky;
  const Ctl *ctl;      // nullable: when set and ctl->stop != 0 the launch is a no-op
};
int sweep_blocks(int n, int group);
hipError_t launch_sweep(const SweepArgs &a, hipStream_t s);

hipError_t launch_residual(bool fp32, int group, int n, const int64_t *rp, const int32_t *col,
                           const double *val, const double *b, const double *x, void *rT,
                           double *r64, double *sumpart, hipStream_t s);
int residual_blocks(int n, int group);

// Reduce check partials and residual partials, update the controller, write
// the host readout slot.  Either count may be 0.
hipError_t launch_readout(const BlockPartial *part, int nparts, const double *sumpart, int nsum,
                          const uint32_t *sticky, Ctl *ctl, int sweeps_in_chunk, int seq,
                          HostReadout *host, hipStream_t s);
hipError_t launch_ctl_reset(Ctl *ctl, double inner_tol, double stall_floor, bool full,
                            hipStream_t s);

hipError_t launch_zero_h(bool fp32, int64_t E, void *msg, hipStream_t s);
hipError_t launch_fill_zero(void *p, int64_t bytes8, hipStream_t s);  // bytes8: count of 8-byte words
hipError_t launch_fill_zero4(void *p, int64_t words4, hipStream_t s);
hipError_t launch_get_msgs(bool fp32, int n, const int64_t *rp, const int64_t *diagpos,
                           const int32_t *oprt, const void *msg, double *P, double *h,
                           hipStream_t s);
hipError_t launch_set_msgs(bool fp32, int n, const int64_t *rp, const int64_t *diagpos,
                           const int32_t *oprt, void *msg, const double *P, const double *h,
                           hipStream_t s);

}  // namespace gabp
