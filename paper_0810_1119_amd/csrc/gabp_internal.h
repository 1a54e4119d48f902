// Internal declarations shared by the HIP kernels and the host side of the
// C ABI.  Nothing here is part of the public interface (include/gabp.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "gabp.h"

namespace gabp {

// Sticky error bits raised by kernels (atomicOr, only when the event occurs).
enum : uint32_t {
  FLAG_BREAKDOWN = 1u,   // zero cavity or marginal precision
  FLAG_NONFINITE = 2u,   // non-finite mean seen at a check
  FLAG_ASYM = 4u,        // pattern or value asymmetry (plan build)
  FLAG_ZERO_DIAG = 8u,   // missing or zero diagonal (plan build)
  FLAG_ARG = 16u,        // malformed CSR or non-finite value (plan build)
  FLAG_UNSUPPORTED = 32u, // a limit of the implementation (plan build)
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
  int32_t warmup;      // checks left that only refresh the previous means: the
                       // first check of a pass compares against means of
                       // another right-hand side (or zeros), so its change is
                       // no measure of this pass's convergence
  int32_t pad;
  int64_t seg_sweeps;  // sweeps summed over the segments that ran them
};

// Per-segment control of a plan made of independent systems (a stack of
// grids under the two-colour schedule): each segment applies the stop rule
// above to its own maxima and leaves the sweeps once it meets its own target;
// the inner solve ends when no segment is left.  The readout and the
// segment-norm kernels (one block each) write these, in stream order, and
// keep the list of segments still sweeping: act[0] = count, act[1..] = their
// indices in increasing order.
struct SegCtl {
  double last_d;       // the segment's d at its previous check (0 before the first)
  double target;       // the segment's inner target (0: the controller's)
  int32_t done;        // 0 sweeping; 1 met its target in this pass; 2 sits the
                       // pass out (its residual already met the tolerance), so
                       // the pass adds nothing to its x
  int32_t stall;       // consecutive stagnant checks below the floor
  double rel;          // relative residual after the previous pass
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
  double segrel;       // largest relative residual of a segment (independent systems)
  int64_t seg_sweeps;  // Ctl::seg_sweeps
};

template <typename T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

constexpr int kBlock = 256;       // threads per block of the row kernels
constexpr int kMaxSweepBlocks = 2048;  // row kernels loop over row groups beyond this

// ---- launchers (kernels_csr.hip) ----
// deg and diagpos may both be NULL: the rows are then only validated (flags)
hipError_t launch_plan_rows(int n, int64_t nnz, const int64_t *rp, const int32_t *col,
                            const double *val, int64_t *deg, int64_t *diagpos, uint32_t *flags,
                            hipStream_t s);
// Exclusive scan of in[0..n) into out[0..n] (out[n] = total).  tmp must hold
// scan_tmp_elems(n) int64 values.
size_t scan_tmp_elems(int64_t n);
hipError_t launch_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s);
// L[i] / L[n + i]: off-diagonal entries of row i with column below / at or
// above split; *far += the entries joining nodes n / 4 or more apart
hipError_t launch_plan_split(int n, const int64_t *rp, const int32_t *col, const int64_t *diagpos,
                             int split, int64_t *L, unsigned long long *far, hipStream_t s);
// Edge arrays of the pair / gather layouts with nb (1 or 2) column ranges: vo
// holds the nb * n + 1 slot offsets of the virtual rows (range p of row i is
// virtual row p * n + i), copied to oprt; ocol, rev, acoef per slot
hipError_t launch_plan_edges(bool fp32, int n, int nb, const int64_t *rp, const int32_t *col,
                             const double *val, const int64_t *diagpos, const int64_t *vo,
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

// FP64 r = b - A x (x == NULL: r = b) over a CSR matrix, optionally rounded
// to the message type (rT), and one partial sum of r^2 per workgroup (grid =
// residual_blocks(n))
hipError_t launch_residual(bool fp32, int grid, int n, const int64_t *rp, const int32_t *col,
                           const double *val, const double *b, const double *x, void *rT,
                           double *r64, double *sumpart, hipStream_t s);
int residual_blocks(int n, int cap = kMaxSweepBlocks);

// Reduce residual partials and (nparts > 0) the check partials, update the
// controller, write the host readout slot.
// With seg (nseg segments, sweeps of nseg <= seg_grid <= kMaxSweepBlocks
// blocks): part holds two colour halves of nparts / 2 >= seg_grid entries in
// the layout of the segment sweeps (kernels_grid_rb.hip); each segment swept
// runs the stop rule on its own maxima and act is rebuilt.
hipError_t launch_readout(BlockPartial *part, int nparts, const double *sumpart, int nsum,
                          const uint32_t *sticky, Ctl *ctl, int sweeps_in_chunk, int seq,
                          HostReadout *host, hipStream_t s, SegCtl *seg = nullptr,
                          int32_t *act = nullptr, int nseg = 0, int seg_grid = 0);
hipError_t launch_ctl_reset(Ctl *ctl, double target, double floor, double freeze_tol, bool full,
                            int warmup, hipStream_t s);

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
  int grid;            // workgroups of the launch (each walks row blocks b0 + k * grid)
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
  // sweeps: the row blocks [b0, b1) of rb (pair_row_blocks)
  const int32_t *rb;
  int b0, b1;
  // synchronous sweeps with column ranges: the blocks are virtual rows
  // [vbase, vbase + n) of one range; carry (nullable) holds the earlier
  // ranges' node sums; last: the final range (adds A_ii, b_i, checks; sums_out
  // is the broadcast array, else the carry)
  int vbase;
  const void *carry;
  bool last;
  // check partials: nslots slots raised with atomics (slot_publish), so the
  // launches of one check (colour classes, column ranges) add up
  int nslots;
  // coloured schedule: one colour class, rows [row0, row1), updated in place
  // (msg_in == msg_out, sums_in == sums_out)
  bool colored;
  int row0, row1;
  bool first;  // first sweep since the messages were set, not sent
};
hipError_t launch_pair_sweep(const PairArgs &a, hipStream_t s);
// Row blocks of the pair sweeps for the row ranges [bounds[k], bounds[k+1])
// (colour classes, or one range): consecutive rows, at most 256 rows and 1024
// slots per block unless one row has more; rp is the slot offset of every row
// (host copy).  Returns the block offsets (rows); first_block[k] is the first
// block of range k (first_block.back() = the number of blocks).
std::vector<int32_t> pair_row_blocks(const int32_t *rp, const std::vector<int> &bounds,
                                     std::vector<int> *first_block);
// workgroups of a pair-layout launch at most: one per row block up to this
// many, so that blocks overlap through the hardware scheduler rather than
// queue inside a workgroup
int pair_max_blocks();
// marginals of one class (rows [row0, row1), row blocks [b0, b1) of rb) of a
// coloured pair plan from its current messages after a complete sweep
// (msg_in / sums_in: the full state, or in the settled state the information
// pairs and H broadcasts, with coef and Sfix)
hipError_t launch_pair_col_infer(const PairArgs &a, double *xacc, double *marg, void *means,
                                 hipStream_t s);
// msg[e].P_ji := msg[rev[e]].P_ij for every slot (pair layout)
hipError_t launch_pair_sync_in(bool fp32, int64_t E, const int32_t *rev, void *msg, hipStream_t s);
// (S, H) from the stored in-messages over the row blocks [b0, b1) of rb (one
// column range, virtual rows from vbase), a row's added in slot order after
// carry (nullable) as the sweeps add them; last: add A_ii and b_i.  msg ==
// NULL: every message is zero (S = A_ii, H = b_i)
hipError_t launch_pair_aggregate(bool fp32, int grid, const int32_t *rb, int b0, int b1,
                                 int vbase, const int32_t *oprt, const void *diag, const void *rhs,
                                 const void *msg, const void *carry, void *sums, bool last,
                                 hipStream_t s);
hipError_t launch_pair_zero_h(bool fp32, int64_t E, void *msg, hipStream_t s);
hipError_t launch_pair_infer(bool fp32, int n, const void *sums, const void *Sfix, const void *Hfz,
                             double *xacc, double *marg, void *means, uint32_t *sticky,
                             hipStream_t s);
// Settled-precision coefficients over the row blocks [0, nblk) of rb (n nodes;
// with two column ranges the blocks span both).  scatter (coloured plans):
// every slot stores its out-coefficient and, through rev, the in-coefficient
// of its reverse slot; otherwise each slot recomputes its in-coefficient from
// its copy of the message and the gathered total (ocol)
hipError_t launch_pair_freeze(bool fp32, int grid, const int32_t *rb, int nblk, int n,
                              const int32_t *oprt, const int32_t *ocol, const int32_t *rev,
                              bool scatter, const void *acoef, const void *msg, const void *sums,
                              void *coef, void *hp, void *Sfix, void *Hfz, hipStream_t s);
hipError_t launch_frozen_restart(bool fp32, int64_t E, int n, void *hp, const void *rhs, void *Hfz,
                                 hipStream_t s);
// messages in CSR entry order (get) or into the slots (set); nb column ranges
hipError_t launch_pair_io(bool fp32, bool get, int n, int nb, const int64_t *rp,
                          const int64_t *diagpos, const int32_t *oprt, const int32_t *rev,
                          void *msg, double *P, double *h, hipStream_t s);

// ---- structured grids (kernels_grid.hip) ----
// n / d for 0 <= n < 2^31 and 1 <= d < 2^31 as a multiply and a shift
// (division by invariant integers, Granlund and Montgomery, PLDI 1994): with
// l = ceil(log2 d) and m = floor(2^32 (2^l - d) / d) + 1, the quotient is
// (mulhi(m, n) + n) >> l, where the sum stays below 2^32 because n < 2^31.
// The index arithmetic of the grid kernels divides by the grid's extents; a
// divisor known only at run time otherwise costs a few dozen instructions.
struct FastDiv {
  uint32_t m = 0, l = 0;
  int d = 0;  // the divisor (0: not set up)
};
inline FastDiv fast_div(int d) {
  FastDiv f;
  uint32_t l = 0;
  while ((1ull << l) < (uint64_t)d) ++l;
  f.l = l;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << l) - (uint64_t)d)) / (uint64_t)d + 1);
  f.d = d;
  return f;
}
__host__ __device__ inline int fdiv(int n, const FastDiv &f) {
  const uint32_t t = (uint32_t)(((uint64_t)f.m * (uint32_t)n) >> 32);
  return (int)((t + (uint32_t)n) >> f.l);
}

struct GridGeom {
  int nx, ny, nz, batch;
  int N;  // nx * ny * nz * batch
  // divisions by nx, ny, nz and by the red-black row length (nx + 1) / 2
  FastDiv fx, fy, fz, fh;
};
// sets N and the divisors from nx, ny, nz, batch
inline void geom_finish(GridGeom &g) {
  g.N = g.nx * g.ny * g.nz * g.batch;
  g.fx = fast_div(g.nx);
  g.fy = fast_div(g.ny);
  g.fz = fast_div(g.nz);
  g.fh = fast_div((g.nx + 1) / 2);
}
inline bool geom_ok(const GridGeom &g) {
  return g.nx >= 1 && g.ny >= 1 && g.nz >= 1 && g.batch >= 1 && g.fx.d == g.nx &&
         g.fy.d == g.ny && g.fz.d == g.nz && g.fh.d == (g.nx + 1) / 2;
}
template <typename T> struct GridCoef {
  const T *diag, *cx, *cy, *cz;  // per node / per face (NULL when constant)
  T dconst, aconst;              // constant diagonal and coupling
};
// Per-launch options of the grid sweeps (GridArgs::fl, RbArgs::fl)
enum : int {
  SWEEP_ZIN = 1,   // the in-messages' informations count as zero (a pending restart)
  SWEEP_ZOWN = 2,  // the launch's own previous informations count as zero (damping)
  SWEEP_XSET = 4,  // means pass: xacc = H / S instead of xacc += H / S
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
  int fl;              // SWEEP_*
};
hipError_t launch_grid_sweep(const GridArgs &a, hipStream_t s);
// a.msg_out receives the information messages (NULL: not copied)
hipError_t launch_grid_freeze(const GridArgs &a, hipStream_t s);
// rT (the working-precision right-hand side) in natural order when hx == 0,
// else in the two-colour order of a red-black plan with hx slots per row.
// With nseg > 1 the stack is cut into nseg equal segments (its grids) and
// block k covers segment k / (grid / nseg) only, so the partials of a grid are
// contiguous (grid must be a multiple of nseg).
hipError_t launch_grid_residual(const GridGeom &g, const GridCoef<double> &k, bool varc, int grid,
                                const double *b, const double *x, void *rT, bool rT32, double *r64,
                                double *sumpart, hipStream_t s, int hx = 0, int nseg = 1);
// Per-segment norms from residual partials (segb consecutive partials per
// segment): store != 0 keeps the squared norms in segb2 (||b_t||^2);
// otherwise host->segrel = max_t ||r_t|| / ||b_t|| (||b|| of the whole system
// where ||b_t|| = 0, given as bnorm).
// With seg: store != 0 also starts every segment sweeping (a new solve);
// otherwise a segment whose residual meets tol sits the next pass out and the
// others get the inner target of their own residual (inner_tol if > 0, else
// 0.3 tol / rel clamped to [tfloor, 0.5], and then at most a tenth of the
// previous target, not below tfloor, where the residual grew over the pass);
// act is rebuilt either way.
hipError_t launch_seg_norms(const double *sumpart, int nseg, int segb, double *segb2, int store,
                            double bnorm, HostReadout *host, hipStream_t s, SegCtl *seg = nullptr,
                            int32_t *act = nullptr, double tol = 0.0, double tfloor = 0.0,
                            double inner_tol = 0.0);

// ---- two-colour (red-black) schedule on grids (kernels_grid_rb.hip) ----
// Node (x, y, z) of a stack (z counted over the whole stack) has colour
// (x + y + z) & 1; row r = y + ny z holds hx = (nx + 1) / 2 slots of each
// colour and the node sits in slot r hx + x / 2 of its colour's arrays (with
// nx odd, one slot per row and colour is never used).  Every per-node and
// per-direction array of such a plan is colour-major: [2][Nc] or [2][6][Nc],
// Nc = hx * ny * nz * batch.
__host__ __device__ inline int rb_row_slots(const GridGeom &g) { return (g.nx + 1) / 2; }
__host__ __device__ inline void rb_place(const GridGeom &g, int hx, int i, int &colour, int &slot) {
  const int r = fdiv(i, g.fx), x = i - r * g.nx;
  const int z = fdiv(r, g.fy), y = r - z * g.ny;
  colour = (x + y + z) & 1;
  slot = r * hx + (x >> 1);
}
struct RbArgs {
  GridGeom g;
  int hx, Nc;          // slots per row and colour, slots per colour
  int grid;            // blocks of a one-colour launch
  int colour;          // the class a sweep launch updates
  bool fp32, varc, damp, frozen;
  int mode;            // 0 sweep, 1 sweep + check, 2 means / precisions only,
                       // 3 sweep + the colour's means into xacc (no segments)
  const void *diag, *cx, *cy, *cz;  // working-precision coefficients, natural order (varc)
  double dconst, aconst;
  const void *rhs;     // [2][Nc]
  void *msg;           // full: (P, h)[2][6][Nc]; frozen: h[2][6][Nc]
  const void *coef, *Sfix;  // frozen: c[2][6][Nc], S[2][Nc]
  double alpha;
  void *xprev;         // [2][Nc]
  double *xacc, *marg; // natural order
  BlockPartial *part;  // this launch's partials (grid entries; with seg one per segment)
  uint32_t *sticky;
  const Ctl *ctl;
  // segments (1 < nseg <= grid, the grids of a stack, Nc / nseg slots each):
  // sweeps cover the segments listed in act only; infer adds nothing to xacc
  // for a segment with done == 2
  int nseg;
  const SegCtl *seg;
  const int32_t *act;
  int fl;              // SWEEP_*
};
hipError_t launch_rb_sweep(const RbArgs &a, hipStream_t s);
// coefficients, information messages and S of the settled phase from the
// full state (both colours); hh receives the information messages (NULL:
// not copied, for a restart that follows)
hipError_t launch_rb_freeze(const RbArgs &a, void *hh, hipStream_t s);
// export (get) / import of the messages in the natural direction-major FP64
// order [6][N] of the synchronous plans
hipError_t launch_rb_io(bool fp32, bool get, const GridGeom &g, int hx, int Nc, void *msg,
                        double *P, double *h, hipStream_t s);
hipError_t launch_grid_check(const GridGeom &g, const GridCoef<double> &k, bool varc, int grid,
                             uint32_t *flags, hipStream_t s);
hipError_t launch_to_working(bool fp32, int64_t m, const double *in, void *out, hipStream_t s);
hipError_t launch_grid_zero_h(bool fp32, int64_t m, void *msg, hipStream_t s);
hipError_t launch_grid_io(bool fp32, bool get, int64_t m, void *msg, double *P, double *h,
                          hipStream_t s);

// ---- colouring and renumbering for coloured CSR plans (kernels_color.hip) ----
constexpr int kMaxColors = 256;
// one Jones-Plassmann round (color < 0: not yet coloured); *left += nodes
// still uncoloured after it; FLAG_UNSUPPORTED if a node needs more colours
hipError_t launch_jp_round(int n, const int64_t *rp, const int32_t *col, int32_t *color,
                           uint32_t *left, uint32_t *flags, hipStream_t s);
hipError_t launch_color_max(int n, const int32_t *color, int32_t *out, hipStream_t s);
hipError_t launch_iota(int n, int32_t *v, hipStream_t s);
// stable sort of the nodes by colour: new2old (tmp == NULL: only *bytes)
hipError_t launch_color_sort(int n, int ncolors, const int32_t *color, uint32_t *keys_out,
                             const int32_t *idx, int32_t *new2old, void *tmp, size_t *bytes,
                             hipStream_t s);
// old2new and the first new row of each colour present (first[] preset to -1)
hipError_t launch_perm_finish(int n, const uint32_t *keys, const int32_t *new2old,
                              int32_t *old2new, int32_t *first, hipStream_t s);
hipError_t launch_perm_rowlen(int n, const int64_t *rp, const int32_t *new2old, int64_t *len,
                              hipStream_t s);
// the renumbered rows' columns and, for each of their slots, the caller's slot
hipError_t launch_perm_fill(int n, const int64_t *rp, const int32_t *col, const int32_t *new2old,
                            const int32_t *old2new, const int64_t *rp2, int32_t *col2,
                            int32_t *slot2, hipStream_t s);
// to_new: out[d] = in[slot[d]]; else out[slot[d]] = in[d] (d < nnz)
hipError_t launch_slot_move(int64_t nnz, const int32_t *slot, const double *in, double *out,
                            bool to_new, hipStream_t s);
// every row's (column, slot) pairs sorted by column
hipError_t launch_rows_sort(int n, int64_t nnz, const int64_t *rp, const int32_t *col_in,
                            int32_t *col_out, const int32_t *val_in, int32_t *val_out, void *tmp,
                            size_t *bytes, hipStream_t s);
// to_new: out[r] = in[new2old[r]]; else out[new2old[r]] = in[r]
hipError_t launch_permute(int n, const int32_t *new2old, const double *in, double *out,
                          bool to_new, hipStream_t s);

// ---- section VII for any sparse S (kernels_lsq.hip) ----
// validation of S, row lengths of R (k + m, int64), column counts, the row
// of each nonzero and the identity permutation
hipError_t launch_lsq_rows(int m, int k, int64_t nnz, const int64_t *rp, const int32_t *col,
                           const double *val, uint32_t *colcnt, int64_t *rowlen, int32_t *rowof,
                           int32_t *idx, uint32_t *flags, hipStream_t s);
hipError_t launch_lsq_sort(int k, int64_t nnz, const int32_t *col, uint32_t *keys_out,
                           const int32_t *idx, int32_t *perm, void *tmp, size_t *tmp_bytes,
                           hipStream_t s);
hipError_t launch_lsq_fill(int m, int k, double psi, const int64_t *rp, const int32_t *col,
                           const double *val, const int64_t *Arp, const int32_t *perm,
                           const int32_t *rowof, int32_t *Acol, double *Aval, hipStream_t s);
hipError_t launch_lsq_embed(int k, int m, const double *y, double *bt, hipStream_t s);
// r = S^T (y - S x) - psi x (x == NULL: S^T y) with the assembled R, u scratch
// [m]; ||r||^2 as lsq_normal_blocks(k) block partials
int lsq_normal_blocks(int k);
hipError_t launch_lsq_normal(int m, int k, double psi, const int64_t *Arp, const int32_t *Acol,
                             const double *Aval, const double *y, const double *x, double *u,
                             double *r, double *part, hipStream_t s);

// ---- batches of dense instances (kernels_dense.hip) ----
// One instance of a batch.  Its couplings form a rows x cols row-major block
// of the packed matrix array; entry (r, c) is one undirected edge between the
// row node r and the column node c (bipartite: chip r, user c; dense: nodes
// r < c of the upper triangle, the diagonal entries are A_ii).
struct DenseInst {
  int64_t mat;     // first entry of the block (also of its message state)
  int64_t rhs;     // first right-hand-side entry (bipartite: rows; dense: cols)
  int64_t xoff;    // first unknown of x (cols entries)
  int64_t node;    // first node of the per-node arrays (bipartite: cols users
                   // then rows chips; dense: cols nodes)
  int64_t edges;   // directed messages per sweep (filled by the validation)
  double sigma2;   // bipartite: -A_rr of every chip node
  int32_t rows, cols;
};

// Per-instance outcome written by the persistent kernel.
struct DenseStat {
  int32_t status, sweeps, frozen_sweeps, restarts, checks, pad;
  double rel;      // final relative residual (FP64)
  double rnorm;    // final ||r||_2
  double damping;  // damping factor in use at the end
};

enum { DENSE_SOLVE = 0, DENSE_RESET = 1, DENSE_SWEEPS = 2 };

struct DenseArgs {
  int kind;              // GABP_BATCH_BIPARTITE / GABP_BATCH_DENSE
  bool fp32;
  int waves;             // wavefronts per workgroup
  int grid;              // workgroups of the persistent launch
  int nr, nc;            // LDS capacity: largest rows and cols of the batch
  int maxm;              // column chunks of 64 lanes per row (1, 2, 4, 8)
  int mode;              // DENSE_*
  int nsweeps;           // DENSE_SWEEPS: sweeps to run
  bool fresh;            // the stored messages are all zero (read none)
  int count;
  const DenseInst *inst;
  const int32_t *order;  // queue: instance indices, largest first
  uint32_t *queue;       // next queue position (zeroed before the launch)
  const double *mat64;   // the caller's FP64 matrices
  const void *matT;      // couplings in the message precision
  const double *b;
  double *x;
  void *state;           // (P_rc, h_rc, P_cr, h_cr) per entry; coloured: per
                         // instance all (P_rc, h_rc), then all (P_cr, h_cr)
  void *fcoef, *fh;      // settled phase: (c_rc, c_cr) and (h_rc, h_cr) per entry;
                         // coloured: all c_rc then all c_cr, the same for h
  bool colored;          // bipartite: two-colour schedule (rows send, then columns)
  void *tot, *nb;        // per node: (S, H) totals and right-hand side
  DenseStat *stat;
  double tol, alpha, inner_tol, freeze_tol, floor;
  int max_sweeps, max_restarts, check_every;
  bool freeze;           // settled phase allowed (buffers allocated)
  bool adapt;            // raise the damping of instances that stop contracting
};

// Byte offsets of the dynamic LDS arrays of the persistent kernel.
struct DenseLds {
  int tot_row, tot_col, uni, b_row, b_col, xprev, diag, red, total;
};
__host__ __device__ inline DenseLds dense_lds(int nr, int nc, int waves, int tsz) {
  auto al = [](int v) { return (v + 15) & ~15; };
  DenseLds L{};
  int o = 0;
  L.tot_row = o; o = al(o + nr * 2 * tsz);
  L.tot_col = o; o = al(o + nc * 2 * tsz);
  L.uni = o;
  const int colpart = waves * nc * 2 * tsz;           // per-wave column partials
  const int resid = 8 * (2 * nc + nr + waves * 64);   // FP64 residual scratch
  o = al(o + (colpart > resid ? colpart : resid));
  L.b_row = o; o = al(o + nr * tsz);
  L.b_col = o; o = al(o + nc * tsz);
  L.xprev = o; o = al(o + nc * tsz);
  L.diag = o; o = al(o + nc * tsz);
  L.red = o; o = al(o + waves * 8 * 8);
  L.total = o;
  return L;
}
hipError_t launch_dense_batch(const DenseArgs &a, hipStream_t s);
// occupancy of the persistent kernel: workgroups per compute unit (0 = cannot launch)
int dense_batch_occupancy(const DenseArgs &a);
hipError_t launch_dense_prepare(const DenseArgs &a, uint32_t *flags, hipStream_t s);
// Means H/S and precisions S from the stored node totals: every node of each
// instance (all = true, node packing) or its unknowns only (packed like x).
hipError_t launch_dense_marginals(const DenseArgs &a, double *mean, double *prec, bool all,
                                  hipStream_t s);

// ---- small sparse systems, one workgroup each (kernels_small.hip) ----
struct SmallInst {
  int32_t n;      // rows of the instance
  int32_t node0;  // its first row in the block-diagonal matrix
  int32_t slot0;  // its first in-slot
  int32_t E;      // in-slots (directed edges)
  int32_t ncol;   // colours (coloured schedule)
  int32_t pad;
};
struct SmallStat {
  int32_t status, sweeps, restarts, checks;
  double rel;    // final relative residual (FP64)
  double rnorm;  // final ||r||_2
};
enum { SMALL_SOLVE = 0, SMALL_RESET = 1, SMALL_SWEEPS = 2 };
struct SmallArgs {
  int mode;              // SMALL_*
  bool fp32;
  bool colored;          // serial scheme in colour order
  int rows_per_thread;   // 1 or 4
  bool cache;            // rows_per_thread == 1 and degree <= 8: slot data in registers
  int maxdeg;            // largest row degree of the batch
  int threads, grid;     // workgroup size and workgroups of the persistent launch
  int count;
  const SmallInst *inst;
  const int32_t *order;  // queue: instance indices, largest first
  uint32_t *queue;       // next queue position (zeroed before the launch)
  int emax, nmax;        // LDS capacity: largest in-slot and row counts
  const int64_t *rp;     // the caller's block-diagonal CSR (FP64 residual)
  const int32_t *col;
  const double *val;
  const int32_t *soff;   // [N + 1] in-slot offsets of the rows
  const int32_t *rev;    // [E] in-slot of the reverse message
  const void *acoef;     // [E] coupling A_ij of in-slot (i <- j), message precision
  const void *diagT;     // [N] A_ii, message precision
  const int32_t *color;  // [N] colour of each row (coloured schedule) or NULL
  const double *b;
  double *x;
  void *msg;             // [E] (P, h) per in-slot: the state after a kernel run
  void *rhsT;            // [N] right-hand side of the current pass
  SmallStat *stat;
  double *hist;          // [6][nodes] FP64 sample history of the solve
  int nodes;             // rows of the whole batch
  double tol, alpha, inner_tol, floor;
  int max_sweeps, max_restarts, check_every;
  int accel, stride, cycle;  // GABP_ACCEL_*, samples every stride sweeps, Steffensen cycle
  int nsweeps;           // SMALL_SWEEPS
};
size_t small_lds(const SmallArgs &a);
int small_occupancy(const SmallArgs &a);  // workgroups per compute unit (0: cannot launch)
hipError_t launch_small_batch(const SmallArgs &a, hipStream_t s);
hipError_t launch_small_marginals(const SmallArgs &a, int N, double *mean, double *prec,
                                  hipStream_t s);
// P, h per CSR position of the caller's matrix (diagonal: 0); set: store them
hipError_t launch_small_messages(const SmallArgs &a, int N, double *P, double *h, bool set,
                                 hipStream_t s);
// FLAG_ARG if a row has a column outside its instance (node_off: count + 1)
hipError_t launch_small_blocks(int N, int count, const int32_t *node_off, const int64_t *rp,
                               const int32_t *col, uint32_t *flags, hipStream_t s);

// ---- coarse grids of a grid stack (kernels_coarse.hip) ----
GridGeom coarse_geom(const GridGeom &f);  // 2 x 2 x 2 blocks (an axis of extent 1 stays)
// Galerkin operator P^T A P of the aggregation, FP64 arrays in the grid layout
hipError_t launch_coarse_coef(const GridGeom &f, const GridCoef<double> &k, bool varc,
                              const GridGeom &c, double *dg, double *cx, double *cy, double *cz,
                              hipStream_t s);
hipError_t launch_coarse_restrict(const GridGeom &f, const GridGeom &c, const double *r, double *rc,
                                  hipStream_t s);
// d += scale * P (dc + dc2) (dc2 NULL: d += scale * P dc)
hipError_t launch_coarse_prolong(const GridGeom &f, const GridGeom &c, const double *dc,
                                 const double *dc2, double scale, double *d, hipStream_t s);
hipError_t launch_axpy(int n, const double *d, double *x, hipStream_t s);  // x += d
// A grid plan's working right-hand side, which a kernel producing the level's
// FP64 right-hand side may write as well: natural order (hx == 0) or the
// red-black colour-major order (hx slots per row and colour, nc slots per
// colour); p == NULL: none
struct WorkRhs {
  void *p = nullptr;
  bool fp32 = true;
  int hx = 0, nc = 0;
};
// One GCR(1) step per grid of a stack (nseg = g.batch grids, segb blocks each) that
// adds the correction c to x: w = A c (the grid's FP64 operator k), then
// per grid beta = (w, pw) / (pw, pw) and alpha = (r, w') / (w', w') with
// w' = w - beta pw, x += alpha (c - beta pc), and (pc, pw) = (c', w') for the
// next step.  first: no previous step (pc, pw, pp not read).  part: nseg *
// segb * 4 doubles; pp, ab: nseg entries kept between steps.  The residual r
// follows x: r -= alpha w' (w' = A c', so r stays b - A x up to rounding),
// also written to wr, with one partial sum of r^2 per block into sumpart
// (nseg * segb entries, the grid residual's layout).
constexpr double kGcrParallel = 1e-10;
hipError_t launch_gcr_step(const GridGeom &g, const GridCoef<double> &k, bool varc, int nseg,
                           int segb, const double *c, double *r, double *w, double *pc,
                           double *pw, double *part, double *pp, double2 *ab, bool first,
                           double *x, const WorkRhs &wr, double *sumpart, hipStream_t s);
// rc = P^T (v - A d) in one pass (A: the fine level's FP64 coefficients);
// w: the coarse level's working right-hand side, set to rc as well
hipError_t launch_coarse_residual_restrict(const GridGeom &f, const GridCoef<double> &k, bool varc,
                                           const GridGeom &c, const double *v, const double *d,
                                           double *rc, const WorkRhs &w, hipStream_t s);
// e = d, v = v - A d in one pass; w set to the new v as well
hipError_t launch_coarse_copy_residual(const GridGeom &g, const GridCoef<double> &k, bool varc,
                                       const double *d, double *e, double *v, const WorkRhs &w,
                                       hipStream_t s);

// The coarsest levels of a hierarchy in one launch (one workgroup of
// kTailThreads per grid of the stack, every vector and message of those
// levels in LDS, FP64 throughout): what the level above asks of them --
// `gamma` cycles on the restricted residual rc, each on the residual the
// previous ones left -- summed into e.
constexpr int kTailThreads = 512;   // also the most cells per grid of a tail level
constexpr int kTailMaxLevels = 8;
struct TailLevel {
  int nx, ny, nz;                    // per grid
  const double *dg, *cx, *cy, *cz;   // Galerkin operator, grid layout of the stack
  double *P;                         // precision messages kept between calls, [batch][6][n]
};
struct TailArgs {
  int nlev, batch;
  TailLevel lv[kTailMaxLevels];  // the last one is the coarsest level
  const double *inv;  // the coarsest level's inverse per grid, [batch][n][n]
  const double *rc;   // the first tail level's right-hand side (grid layout of the stack)
  double *e;          // its correction summed over the gamma cycles
  uint32_t *sticky;   // FLAG_* bits
  double damping, scale;
  int colored, fresh, pre, post, gamma;
};
size_t coarse_tail_lds(const TailArgs &a);  // bytes of LDS per workgroup
hipError_t launch_coarse_tail(const TailArgs &a, hipStream_t s);
// The coarsest level (at most kCoarsestCellsMax cells per grid; at most
// kCoarsestCells when the LDS tail runs the levels above it) is solved
// exactly: its dense inverse per grid by Gauss-Jordan elimination with
// partial pivoting (once per hierarchy; FLAG_BREAKDOWN on a zero pivot; in
// LDS up to kCoarsestCells cells, else on [M | I] in `work`, 2 n^2 + n
// doubles per grid, one pivot step per pair of launches), and
// d = inverse * v per grid.
constexpr int kCoarsestCells = 64;
constexpr int kCoarsestCellsMax = kTailThreads;
hipError_t launch_coarse_inverse(const GridGeom &c, const double *dg, const double *cx,
                                 const double *cy, const double *cz, double *inv, double *work,
                                 uint32_t *flags, hipStream_t s);
hipError_t launch_coarse_dense_solve(const GridGeom &c, const double *inv, const double *v,
                                     double *d, hipStream_t s);

// ---- warm-start network (kernels_mlp.hip) ----
struct MlpTrainArgs {
  const uint16_t *w;            // bfloat16 parameters used by the passes
  const float *U, *T;           // [S][8] features, [S][12] targets
  int64_t S;
  float *H1, *H2, *R, *D1, *D2; // activations and errors, feature-major [width][S]
  double *part;                 // forward partials, 2 per block
  float *gpart;                 // weight-gradient partials [blocks][params]
  double *lossv;                // [loss, unmasked outputs]
  float *grad;                  // nullable: the gradient
  bool update;                  // Adam step
  float *master, *m1, *m2;      // FP32 masters and moments
  uint16_t *wbf;                // bfloat16 copy written by the update
  float lr, c1, c2;             // step size, bias corrections 1 - beta^t
};
int mlp_params();
int mlp_chunk();
int mlp_fwd_blocks(int64_t S);
hipError_t launch_mlp_set(const float *src, float *master, uint16_t *wbf, float *m1, float *m2,
                          hipStream_t s);
hipError_t launch_mlp_get(const uint16_t *wbf, float *dst, hipStream_t s);
hipError_t launch_mlp_forward(const uint16_t *w, const float *U, int64_t S, float *out,
                              hipStream_t s);
hipError_t launch_mlp_train(const MlpTrainArgs &a, hipStream_t s);
hipError_t launch_grid_features(const GridGeom &g, const GridCoef<double> &k, const double *b,
                                const int64_t *nodes, int64_t count, float *U, hipStream_t s);
hipError_t launch_grid_targets(const GridGeom &g, const GridCoef<double> &k, const double *P,
                               const double *h, const int64_t *nodes, int64_t count, float *T,
                               hipStream_t s);
// msg and rhs in natural order when hx == 0, else in the two-colour order
hipError_t launch_grid_warm(bool fp32, const GridGeom &g, const void *diag, const void *cx,
                            const void *cy, const void *cz, double dconst, double aconst,
                            const void *rhs, const uint16_t *w, void *msg, hipStream_t s,
                            int hx = 0);

}  // namespace gabp
