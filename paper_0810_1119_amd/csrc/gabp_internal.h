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

// Per-block maxima of a check sweep: the largest change of a marginal mean
// over the check interval, the largest |mean|, the largest change of a
// precision message over the last sweep and the largest |precision message|.
// The readout kernel reduces them in a fixed order (no atomics).
struct BlockPartial {
  double dmax, xmax, dpmax, pmax;
};

// Device-resident controller of an inner solve.  Only the single-thread
// readout kernel writes it, in stream order, so no atomics are needed; the
// sweep kernels read `stop` once at entry and skip all work when it is set.
//
// Stop rule of an inner solve: with d_k = max_i |x_i - x_i(previous check)|
// over one check interval and q = d_k / d_{k-1}, a linearly convergent
// sequence has error about d_k q / (1 - q).  The solve stops when that
// estimate, relative to max|x|, drops to `target`; or when the change is
// already below `floor` (the arithmetic's resolution) and q shows no more
// contraction (q > 0.7 twice), i.e. the iteration has reached rounding noise.
struct Ctl {
  uint32_t stop;       // STOP_*
  int32_t sweeps;      // sweeps actually executed in this solve
  int32_t checks;      // checks evaluated
  int32_t stall;       // consecutive stagnant checks below the floor
  double target;       // stop when estimated relative error <= target
  double floor;        // relative change below which stagnation means done
  double last_d;       // d of the previous check (0 before the first)
  double last_x;       // max|x| at the last check
  double est;          // last error estimate (relative)
  double freeze_tol;   // precision messages count as settled when their
                       // largest change <= freeze_tol * largest |P|
  int32_t freeze;      // set once the precision messages have settled
  int32_t pad;
};

// What the host reads back (pinned, written by the readout kernel).
struct HostReadout {
  double dmax;
  double xmax;
  double sum;          // sum of the residual partials (||r||^2)
  double dpmax;        // largest change of a precision message (last check)
  double pmax;         // largest |precision message| (last check)
  uint32_t flags;      // sticky flags at readout time
  uint32_t stop;       // controller state
  int32_t sweeps;
  int32_t seq;         // chunk sequence number (sanity check)
  int32_t freeze;      // precision messages settled
  int32_t pad;
};

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

constexpr int kBlock = 256;       // threads per block of the row kernels
constexpr int kMaxSweepBlocks = 2048;  // row kernels loop over row groups beyond this

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
                             int32_t *oprt, int32_t *ocol, int32_t *rev, void *acoef, void *diag,
                             uint32_t *flags, hipStream_t s);

struct SweepArgs {
  int grid;            // blocks of the launch (sweep_blocks)
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
  BlockPartial *part;  // mode 1: one entry per block of the launch
  uint32_t *sticky;
  const Ctl *ctl;      // nullable: when set and ctl->stop != 0 the launch is a no-op
};
// blocks of a sweep launch: one row group per block, capped at `cap` blocks
// (kernels loop over the remaining row groups)
int sweep_blocks(int n, int group, int cap = kMaxSweepBlocks);
hipError_t launch_sweep(const SweepArgs &a, hipStream_t s);

hipError_t launch_residual(bool fp32, int group, int grid, int n, const int64_t *rp, const int32_t *col,
                           const double *val, const double *b, const double *x, void *rT,
                           double *r64, double *sumpart, hipStream_t s);
int residual_blocks(int n, int group, int cap = kMaxSweepBlocks);

// Reduce residual partials and (nparts > 0) the check partials, update the
// controller, write the host readout slot.
hipError_t launch_readout(const BlockPartial *part, int nparts, const double *sumpart, int nsum,
                          const uint32_t *sticky, Ctl *ctl, int sweeps_in_chunk, int seq,
                          HostReadout *host, hipStream_t s);
hipError_t launch_ctl_reset(Ctl *ctl, double target, double floor, double freeze_tol, bool full,
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

// ---- pair layout (kernels_pair.hip) ----
struct PairArgs {
  int grid;            // blocks of the launch (sweep_blocks)
  bool fp32;
  int group;
  int mode;            // 0 sweep, 1 sweep + check
  bool damp;
  bool frozen;         // information-only sweep with fixed coefficients
  int n;
  const int32_t *oprt, *ocol;
  const void *acoef, *diag, *rhs;
  const void *coef, *Sfix;        // frozen
  const void *msg_in;             // full: (P_ij, h_ij, P_ji, h_ji); frozen: (h_ij, h_ji)
  void *msg_out;
  const void *sums_in;            // full: (S, H) per node; frozen: H per node
  void *sums_out;
  double alpha;
  void *xprev;
  BlockPartial *part;
  uint32_t *sticky;
  const Ctl *ctl;
};
hipError_t launch_pair_sweep(const PairArgs &a, hipStream_t s);
hipError_t launch_pair_aggregate(bool fp32, int group, int grid, int n, const int32_t *oprt, const void *diag,
                                 const void *rhs, const void *msg, void *sums, hipStream_t s);
hipError_t launch_pair_zero_h(bool fp32, int64_t E, void *msg, hipStream_t s);
hipError_t launch_pair_infer(bool fp32, int n, const void *sums, const void *Sfix, const void *Hfz,
                             double *xacc, double *marg, uint32_t *sticky, hipStream_t s);
hipError_t launch_pair_freeze(bool fp32, int group, int grid, int n, const int32_t *oprt, const int32_t *ocol,
                              const void *acoef, const void *msg, const void *sums, void *coef,
                              void *hp, void *Sfix, void *Hfz, hipStream_t s);
hipError_t launch_frozen_restart(bool fp32, int64_t E, int n, void *hp, const void *rhs, void *Hfz,
                                 hipStream_t s);
hipError_t launch_pair_io(bool fp32, bool get, int n, const int64_t *rp, const int64_t *diagpos,
                          const int32_t *oprt, const int32_t *rev, void *msg, double *P, double *h,
                          hipStream_t s);

// ---- structured grids (kernels_grid.hip) ----
struct GridGeom {
  int nx, ny, nz, batch;
  int N;  // nx * ny * nz * batch
};
template <typename T> struct GridCoef {
  const T *diag, *cx, *cy, *cz;  // per node / per face (NULL when constant)
  T dconst, aconst;              // constant diagonal and coupling
};
struct GridArgs {
  GridGeom g;
  int grid;            // blocks of the launch
  bool fp32, varc, damp, frozen;
  int mode;            // 0 sweep, 1 sweep + check, 2 means / precisions only
  const void *diag, *cx, *cy, *cz;  // working-precision coefficient arrays (varc)
  double dconst, aconst;
  const void *rhs;
  const void *msg_in;  // full: (P, h)[6][N]; frozen: h[6][N]
  void *msg_out;
  const void *coef, *Sfix;  // frozen coefficients c[6][N] and S
  double alpha;
  void *xprev;
  double *xacc, *marg;
  BlockPartial *part;
  uint32_t *sticky;
  const Ctl *ctl;
};
hipError_t launch_grid_sweep(const GridArgs &a, hipStream_t s);
hipError_t launch_grid_freeze(const GridArgs &a, hipStream_t s);
hipError_t launch_grid_residual(const GridGeom &g, const GridCoef<double> &k, bool varc, int grid,
                                const double *b, const double *x, void *rT, bool rT32, double *r64,
                                double *sumpart, hipStream_t s);
hipError_t launch_grid_check(const GridGeom &g, const GridCoef<double> &k, bool varc, int grid,
                             uint32_t *flags, hipStream_t s);
hipError_t launch_to_working(bool fp32, int64_t m, const double *in, void *out, hipStream_t s);
hipError_t launch_grid_zero_h(bool fp32, int64_t m, void *msg, hipStream_t s);
hipError_t launch_grid_io(bool fp32, bool get, int64_t m, void *msg, double *P, double *h,
                          hipStream_t s);

}  // namespace gabp
