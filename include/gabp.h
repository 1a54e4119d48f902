/*
 * gabp.h -- C ABI of the MI355X (gfx950) Gaussian belief propagation solver.
 *
 * Solves A x = b for a square symmetric A (Assumption 1, section II-C of
 * Shental, Bickson et al., "Gaussian Belief Propagation for Solving Systems of
 * Linear Equations: Theory and Application") by synchronous GaBP: the
 * solution is the vector of marginal means of the Gaussian N(A^{-1} b, A^{-1})
 * (Proposition 3, section III-A).  Every sweep runs the broadcast form of
 * Algorithm 2 (section V): per node the aggregate precision and information
 * of all incoming messages, then per directed edge the new message after
 * subtracting the reverse one (eq. prec_message / mean_message of III-C).
 * Positive definiteness is NOT required (remark of section III-A); the
 * solver never clamps precisions.
 *
 * Conventions for every entry point:
 *   - Pointers marked "device" are HIP device allocations owned by the caller;
 *     the library never frees or retains them beyond the call, except that a
 *     plan keeps reading the CSR arrays it was created from until it is
 *     destroyed.  Pointers marked "host" are ordinary host memory.
 *   - The return value is a gabp_status.  Nothing is thrown and nothing aborts.
 *   - All device work is ordered on the given stream (NULL = default stream);
 *     a call returns after its results are complete and visible.
 *   - Calls on different plans and different streams are independent; calls
 *     on one plan must not overlap.
 *   - On GABP_NOT_CONVERGED the output x holds the last iterate; on a negative
 *     status the outputs are unspecified.
 */
#ifndef GABP_H
#define GABP_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GABP_OK = 0,                 /* converged to the requested tolerance */
  GABP_NOT_CONVERGED = 1,      /* sweep or restart budget exhausted */
  GABP_ERR_ARG = -1,           /* bad argument: null pointer, size, unsorted or
                                  out-of-range column, non-finite input */
  GABP_ERR_NOT_SYMMETRIC = -2, /* pattern or values of A are not symmetric */
  GABP_ERR_ZERO_DIAG = -3,     /* missing or zero diagonal (mu_ii = b_i / A_ii
                                  undefined, Algorithm 1 step 1) */
  GABP_ERR_BREAKDOWN = -4,     /* a cavity or marginal precision became exactly
                                  zero (a zero elimination pivot, Proposition
                                  GaBPGE) */
  GABP_ERR_DIVERGED = -5,      /* a non-finite message or mean appeared */
  GABP_ERR_HIP = -6,           /* a HIP runtime call failed */
  GABP_ERR_NOMEM = -7,         /* device or pinned allocation failed */
  GABP_ERR_UNSUPPORTED = -8    /* size beyond the library's limits (e.g. more
                                  than 2^31 - 1 directed edges) */
} gabp_status;

/* Sparse symmetric matrix, full pattern (both triangles) including the
 * diagonal.  Each row's columns are strictly increasing.  The graph of
 * section II-B has an edge {i, j} for every stored A_ij != 0, i != j; every
 * stored off-diagonal entry is one directed message per sweep.  */
typedef struct {
  int32_t n;                 /* unknowns, >= 0 */
  int64_t nnz;               /* stored entries = row_ptr[n] */
  const int64_t *row_ptr;    /* device [n+1] */
  const int32_t *col;        /* device [nnz] */
  const double *val;         /* device [nnz] */
} gabp_csr;

typedef struct {
  int32_t msg_fp32;    /* 1: messages and node sums in FP32, with the residual
                          b - A x and the correction restarts in FP64;
                          0: everything in FP64 */
  double tol;          /* stop when ||b - A x||_2 / ||b||_2 <= tol (FP64); for a
                          stack of grids (batch > 1) every grid's own
                          ||b_t - A_t x_t|| / ||b_t|| must meet it */
  int32_t max_sweeps;  /* budget of synchronous sweeps over all restarts */
  int32_t check_every; /* sweeps between checks of the marginal means, rounded
                          up to an even count; 0 (default): 2 in the first 64
                          sweeps of a refinement pass, 4 up to 256, then 8
                          (a check sweep costs more than a plain one and adds
                          a readout).  Batched solves: 0 means 2.  < 0:
                          GABP_ERR_ARG */
  double damping;      /* alpha in [0,1): P <- alpha P_old + (1-alpha) P_new
                          and the same for the information h = P mu */
  double inner_tol;    /* an inner solve ends when the estimated relative
                          error of the means, d q / (1 - q) / max|x| with d the
                          largest change over one check interval and q the
                          ratio of successive d, is at most inner_tol;
                          0 = automatic: the first inner solve runs to the
                          message precision's floor, later ones to the
                          remaining factor 0.3 tol / (current residual) */
  int32_t max_restarts;/* refinement restarts (mean messages zeroed,
                          precision messages kept) */
  int32_t group;       /* GABP_LAYOUT_GATHER only: lanes per row in the sweep,
                          0 = chosen from the degree profile, else 4, 8, 16,
                          32 or 64.  The pair layout streams rows in blocks
                          of up to 256 rows and 1024 slots and ignores it */
  int32_t layout;      /* GABP_LAYOUT_PAIR (default): each edge slot holds both
                          directions of its edge and nodes broadcast their
                          aggregates (Algorithm 2, section V), so the only
                          random access is a node-sized gather;
                          GABP_LAYOUT_GATHER: each slot holds its out-message
                          and in-messages are gathered through the
                          reverse-edge index (half the message memory) */
  int32_t grid_blocks; /* blocks of a sweep launch; rows beyond are handled
                          by a grid-stride loop; 0 = default (2048) */
  int32_t freeze;      /* 1 (default): once every precision message has settled
                          (largest change <= 1e-6 |P|max in FP32, 1e-14 in FP64)
                          pair-layout sweeps keep the precisions fixed and
                          update the information h = P mu only; the FP64
                          refinement absorbs the last-ulp difference.  0: never */
  int32_t batch_waves; /* batched solves: wavefronts (64 lanes) per workgroup,
                          4, 8 or 16; 0 = chosen by the plan's autotuner,
                          whose choices persist in a text file:
                          $GABP_TUNE_CACHE, else $XDG_CACHE_HOME or
                          $HOME/.cache, /gabp-mi355x/tune.txt
                          (GABP_TUNE_CACHE=off: this process only) */
  double freeze_tol;    /* the settled-precision threshold (see freeze); 0 = the
                          default, 1e-6 for FP32 messages and 1e-14 for FP64 */
  int32_t adapt_damping; /* batched solves, 1 (default): an instance whose means
                          stop contracting (ratio of successive changes >= 0.95
                          at 8 checks in a row after the first 32 sweeps of a
                          pass) or turn non-finite runs that pass again from
                          zero messages with the damping raised to 0.3, then
                          0.5, then 0.7 (damping as in section VI-D); 0 = never */
  int32_t schedule;     /* GABP_SCHEDULE_SYNC (default): every message of a sweep
                          from the previous sweep's messages (the parallel
                          scheme of section III-C); GABP_SCHEDULE_COLORED: the
                          serial scheme of section III-C in the order of a
                          node colouring: grid plans (checkerboard: one sweep
                          lets every node of colour 0, (x + y + z) even with z
                          counted over the whole stack, send from the newest
                          messages, then every node of colour 1), bipartite
                          batches (chips send, then users), lsq plans (x, then
                          z) and CSR plans in the pair layout (a colouring the
                          plan computes, see gabp_plan_colors).  Dense batches
                          and the gather layout return GABP_ERR_UNSUPPORTED */
  int32_t col_blocks;   /* CSR plans, pair layout, synchronous schedule: 1 or 2
                          column ranges.  With 2 the slots of every row are
                          ordered by neighbour range (node indices below
                          (n + 1) / 2 first) and a sweep runs one launch per
                          range, so each launch gathers node broadcasts from
                          half of the node table, which then fits the L2 cache
                          of an XCD better.  0 (default): 2 when the node table
                          (8 B per node in FP32, 16 B in FP64) exceeds 4 MiB
                          and at least half of the edges join nodes n / 4 or
                          more apart in index, else 1.  The two differ only in
                          the order of the node sums.  2 with the coloured
                          schedule or the gather layout: GABP_ERR_UNSUPPORTED;
                          other values: GABP_ERR_ARG.  Other plan kinds ignore
                          it. */
  int32_t accel;        /* acceleration of the means, section IV-A (batches of
                          small CSR instances only; other plans return
                          GABP_ERR_UNSUPPORTED for a nonzero value):
                          GABP_ACCEL_NONE (default);
                          GABP_ACCEL_AITKEN: GaBP runs unchanged, the means are
                          sampled every accel_stride sweeps (x_0 = the means of
                          the messages a pass starts from) and each node
                          extrapolates its last three samples x0, x1, x2 to
                          y = x0 - (x1 - x0)^2 / (x2 - 2 x1 + x0) (y = x2 when
                          the second difference is zero; at the first sample
                          of a pass y is that sample); the stop rule and the
                          answer use y;
                          GABP_ACCEL_STEFFENSEN: cycles of accel_cycle sweeps;
                          at the end of a cycle the samples of sweeps
                          cycle - 2 stride, cycle - stride and cycle are
                          extrapolated, x += y, and GaBP runs again on the
                          residual b - A x from zero information messages with
                          the precision messages kept (the paper does not say
                          how a vector of means re-enters message form) */
  int32_t accel_stride; /* sweeps between samples, >= 1; 0 = 2 (pairs sweeps of
                          equal parity, which bipartite graphs need under the
                          synchronous schedule) */
  int32_t accel_cycle;  /* Steffensen: sweeps per cycle, >= 2 stride; 0 = 100 */
} gabp_opts;

enum { GABP_LAYOUT_PAIR = 0, GABP_LAYOUT_GATHER = 1 };
enum { GABP_SCHEDULE_SYNC = 0, GABP_SCHEDULE_COLORED = 1 };
enum { GABP_ACCEL_NONE = 0, GABP_ACCEL_AITKEN = 1, GABP_ACCEL_STEFFENSEN = 2 };

typedef struct {
  int32_t status;          /* gabp_status of the solve */
  int32_t sweeps;          /* synchronous sweeps run (all restarts) */
  int32_t frozen_sweeps;   /* of which with settled (fixed) precisions */
  int32_t restarts;        /* refinement restarts taken */
  int32_t checks;          /* check sweeps run (one per chunk of sweeps) */
  double rel_residual;     /* final ||b - A x||_2 / ||b||_2, FP64 (a grid stack:
                              the largest over its grids) */
  double residual_per_eq;  /* ||b - A x||_2 / n (section II-A norm) */
  double seconds;          /* host wall time of the solve */
  double sweep_ms;         /* summed device time of the sweep launches */
  double frozen_sweep_ms;  /* of which in sweeps with settled precisions */
  int64_t edges;           /* directed off-diagonal messages per sweep */
  double edge_updates_per_s; /* messages computed per second: edges *
                                mean_sweeps / seconds (batched: each
                                instance's edges times its own sweeps) */
  double damping;          /* damping factor in use at the end (batched
                              instances may have raised it) */
  int32_t batch_waves;     /* batched solves: wavefronts per workgroup of the
                              persistent launch (the autotuner's choice) */
  int32_t batch_groups;    /* batched solves: workgroups of that launch */
  int32_t warm_start;      /* gabp_plan_solve_warm: 1 the network's messages were
                              used; -1 rejected before the first sweep (the means
                              they imply fit b worse than x = 0); -2 the warm
                              solve did not converge and was redone from zero
                              messages; 0 no warm start */
  int32_t sweep_launches;  /* kernel launches per sweep: column ranges of a CSR
                              plan, colour classes of a coloured plan, 1 else;
                              0 for batched solves (one launch runs the solve) */
  double warm_rel0;        /* ||b - A x0|| / ||b|| of the warm start's means */
  double mean_sweeps;      /* sweeps per independent system, averaged over them:
                              a grid stack under the coloured schedule lets each
                              grid leave the sweeps once it meets its own inner
                              target, so this is below `sweeps` (the slowest
                              grid's); batched solves: the instances' mean;
                              otherwise equal to sweeps */
  double mean_frozen_sweeps; /* of which with settled precisions (frozen_sweeps
                              counted the same way) */
} gabp_stats;

/* Fills o with the defaults: FP32 messages, tol 1e-8, 20000 sweeps,
 * automatic check interval (check_every 0), no damping, automatic inner
 * targets (inner_tol 0), 30 restarts, group 0, pair layout, freeze on,
 * batch_waves 0 (autotuned), adapt_damping on. */
void gabp_default_opts(gabp_opts *o);

/* One-call solve (plan create + solve + destroy).
 *   A        device CSR as above.
 *   b        device [n] right-hand side.
 *   x        device [n] output, marginal means (Algorithm 1 steps 4-5).
 *   marg_prec  device [n] or NULL: marginal precisions P_i = A_ii + sum_k P_ki
 *            of the final messages (exact only on trees, section IV).
 *   o        host options or NULL for the defaults.
 *   st       host stats or NULL. */
int gabp_solve(const gabp_csr *A, const double *b, double *x, double *marg_prec,
               const gabp_opts *o, gabp_stats *st, hipStream_t stream);

/* FP64 residual r = b - A x (section II-A, sign flipped) and its relative norm.
 *   r        device [n] or NULL.
 *   rel_norm host: ||r||_2 / ||b||_2 (||r||_2 if b = 0).
 * Deterministic: fixed-order block reduction, no floating-point atomics. */
int gabp_residual(const gabp_csr *A, const double *b, const double *x, double *r,
                  double *rel_norm, hipStream_t stream);

/* gabp_residual without any allocation, for callers that cannot allocate
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, results and errors as gabp_residual (the same
 * kernels in the same order: bitwise the same results).  Its scratch (32 KiB:
 * validation flags, at most 2048 partial sums, two readout records) is one
 * static device array per GPU, looked up on the first call with that device
 * current and held until the process ends; no call allocates device or pinned
 * memory.  Every call on a GPU shares that GPU's array: calls that overlap on
 * one GPU (other streams or threads) race and must be serialised by the
 * caller.  The stream must belong to the current device.  Any n is accepted
 * (the residual uses at most 2048 workgroups); a partial count beyond the
 * array would be GABP_ERR_UNSUPPORTED. */
int gabp_residual_noalloc(const gabp_csr *A, const double *b, const double *x, double *r,
                          double *rel_norm, hipStream_t stream);

/* ---- Plans: reuse the validated graph, reverse-edge index and buffers. ---- */
typedef struct gabp_plan gabp_plan;

/* Validates A on the device (sorted in-range columns, nonzero diagonal,
 * symmetric pattern and values), builds the off-diagonal edge arrays and the
 * reverse-edge index rev[e(i->j)] = e(j->i), and allocates the message
 * buffers.  A's arrays must stay valid and unchanged until destroy. */
int gabp_plan_create(const gabp_csr *A, const gabp_opts *o, gabp_plan **plan,
                     hipStream_t stream);
int gabp_plan_destroy(gabp_plan *plan);

/* Solve A x = b from zero messages (Algorithm 1 step 1) with the plan's
 * options; arguments as for gabp_solve. */
int gabp_plan_solve(gabp_plan *plan, const double *b, double *x, double *marg_prec,
                    gabp_stats *st, hipStream_t stream);

/* Trajectory access (parity checks, checkpoint and resume).
 * reset:     zero all messages and take b (device [n]) as the right-hand side.
 * sweeps:    run exactly `count` sweeps of the plan's schedule (no checks, no
 *            restarts).
 * marginals: mean (device [n]) and precision (device [n] or NULL) from the
 *            current messages.
 * get/set_messages: P and h = P * mu of every directed message i->j at the
 *            CSR slot of A_ij (device [nnz] each, FP64; diagonal slots read
 *            as 0 and are ignored on set).  Coloured CSR plans run on a
 *            renumbering of A: their messages cross through its slot map
 *            (two FP64 buffers of nnz are held for the call).
 * A coloured CSR plan (gabp_plan_create with GABP_SCHEDULE_COLORED, pair
 * layout) colours the graph of A on the device (Jones-Plassmann rounds with
 * fixed pseudo-random priorities and first-fit colours, deterministic; at
 * most 256 colours, else GABP_ERR_UNSUPPORTED), renumbers the nodes so each
 * colour is a contiguous range of rows, and lets one colour send per launch:
 * each node first rebuilds its in-messages from its neighbours' broadcast
 * totals, then sends from its new totals (the serial scheme of section III-C
 * in colour order).  b, x and the marginals stay in the caller's order. */
int gabp_plan_reset(gabp_plan *plan, const double *b, hipStream_t stream);
int gabp_plan_sweeps(gabp_plan *plan, int32_t count, hipStream_t stream);
int gabp_plan_marginals(gabp_plan *plan, double *mean, double *prec, hipStream_t stream);
int gabp_plan_get_messages(gabp_plan *plan, double *P, double *h, hipStream_t stream);
int gabp_plan_set_messages(gabp_plan *plan, const double *P, const double *h,
                           hipStream_t stream);
/* The colour of every node under the coloured schedule (device [n], int32, the
 * caller's node order) and the number of colours (host); colours are
 * processed in increasing order within a sweep.  Coloured CSR plans and
 * coloured lsq plans (x: 0, z: 1); GABP_ERR_UNSUPPORTED for other plans. */
int gabp_plan_colors(gabp_plan *plan, int32_t *colors, int32_t *ncolors, hipStream_t stream);

/* Device memory the plan holds (host *bytes): every buffer the library
 * allocated for it and has not freed -- messages, index and coefficient
 * arrays, working copies, controller state, and what solves added later
 * (settled-precision buffers, the coarse levels of gabp_plan_solve_coarse
 * with their own plans).  Memory the caller passes in is not counted.  A
 * one-shot call (gabp_solve and the like) allocates what a plan for the same
 * problem holds and frees it before returning.  No device work, no
 * synchronisation; GABP_ERR_ARG for a NULL argument. */
int gabp_plan_workspace_bytes(const gabp_plan *plan, size_t *bytes);

/* ---- Structured grids: the finite-difference Poisson operators of ----------
 * section IX (5-point in 2-D, 7-point in 3-D), with constant or variable
 * coefficients, as a stack of independent grids.  Node index
 * i = x + nx (y + ny z) within a grid (natural row ordering), grid t of the
 * stack holding nodes [t n, (t + 1) n), n = nx ny nz.  A_ij is nonzero only
 * between face neighbours; symmetry holds by construction. */
typedef struct {
  int32_t nx, ny, nz;        /* extent of one grid, >= 1; nz = 1: 5-point 2-D stencil */
  int32_t batch;             /* independent grids in the stack, >= 1 */
  const double *diag;        /* device [batch n] A_ii, or NULL: diag_value everywhere */
  double diag_value;
  const double *cx, *cy, *cz;/* device [batch n] coupling of node i with its +x, +y, +z
                                neighbour (A_{i,i+1}, A_{i,i+nx}, A_{i,i+nx ny}); values
                                on a grid's last plane in that direction are ignored.
                                All NULL: off_value on every interior face (cz may be
                                NULL when nz = 1) */
  double off_value;
} gabp_grid;

/* Plan, one-call solve and FP64 residual for grids; same conventions as the
 * CSR entry points.  Messages of a grid plan (get/set_messages) are laid out
 * direction-major: [6][batch n] for the directions +x, -x, +y, -y, +z, -z,
 * entries without an edge read as 0.  A zero or non-finite coefficient is
 * GABP_ERR_ZERO_DIAG / GABP_ERR_ARG; more than 2^31 - 1 nodes is
 * GABP_ERR_UNSUPPORTED. */
int gabp_plan_create_grid(const gabp_grid *A, const gabp_opts *o, gabp_plan **plan,
                          hipStream_t stream);
int gabp_solve_grid(const gabp_grid *A, const double *b, double *x, double *marg_prec,
                    const gabp_opts *o, gabp_stats *st, hipStream_t stream);
int gabp_residual_grid(const gabp_grid *A, const double *b, const double *x, double *r,
                       double *rel_norm, hipStream_t stream);

/* ---- Batches of small dense instances, one persistent launch. -------------
 * Each workgroup takes the next instance from a queue sorted by size (largest
 * first) and runs all of that instance's sweeps, mean checks and FP64
 * refinement passes on its own, so instances of very different sizes finish
 * independently and no host round trip happens between sweeps.
 *
 * GABP_BATCH_BIPARTITE (section VII): instance t is a linear detector with
 * spreading matrix S_t (N_t chips x K_t users), observations y_t and noise
 * variance sigma2_t > 0; its answer is the MMSE estimate
 *     x_t = (S_t^T S_t + sigma2_t I)^{-1} S_t^T y_t        (section VIII-B),
 * computed by GaBP on the symmetric (K_t + N_t)-node system
 *     [[I, S_t^T], [S_t, -sigma2_t I]] [x; z] = [0; y_t],
 * whose graph is the complete bipartite graph users x chips (one edge per
 * nonzero S entry).  GaBP on the K_t x K_t matrix S^T S + sigma2 I itself
 * diverges when the loading K/N is large (that matrix is not walk-summable);
 * the bipartite system has the same x and converges.
 * Refinement: with r = S^T y - (S^T S + sigma2 I) x in FP64, the correction
 * solves the bipartite system with right-hand side [r / sigma2; 0], whose
 * first block is the solution d of (S^T S + sigma2 I) d = r.
 * tol applies to ||S^T y - (S^T S + sigma2 I) x||_2 / ||S^T y||_2.
 *
 * GABP_BATCH_DENSE: instance t is a dense symmetric K_t x K_t matrix A_t
 * (complete graph on its nonzero entries), solved as by gabp_solve.
 *
 * Packing: instance matrices back to back in `mat` (row-major), right-hand
 * sides back to back in b (y_t of N_t entries, or b_t of K_t), solutions back
 * to back in x (K_t entries each).  Limits: K_t <= 512 and the per-workgroup
 * state of the largest instance must fit the 160 KB LDS (about N_t <= 4096 for
 * FP32 messages); beyond: GABP_ERR_UNSUPPORTED. */
enum { GABP_BATCH_BIPARTITE = 0, GABP_BATCH_DENSE = 1, GABP_BATCH_CSR = 2 };
typedef struct {
  int32_t kind;          /* GABP_BATCH_BIPARTITE, GABP_BATCH_DENSE or GABP_BATCH_CSR */
  int32_t count;         /* instances, >= 0 */
  const int32_t *k;      /* host [count]: users K_t, or the order of A_t */
  const int32_t *m;      /* host [count]: chips N_t (bipartite; NULL otherwise) */
  const double *sigma2;  /* host [count]: noise variance (bipartite; NULL otherwise) */
  const double *mat;     /* device: S_t (N_t x K_t) or A_t (K_t x K_t), packed; read
                            by the plan until it is destroyed (NULL for CSR) */
  const gabp_csr *csr;   /* GABP_BATCH_CSR: the instances as the diagonal blocks
                            of one sparse symmetric matrix (host struct, device
                            arrays as for gabp_solve): instance t owns rows
                            [o_t, o_t + k_t), o_t = k_0 + ... + k_{t-1}, and no
                            stored entry may join two instances (GABP_ERR_ARG);
                            read by the plan until it is destroyed.  NULL for
                            the dense kinds */
} gabp_batch;
/* GABP_BATCH_CSR: independent sparse symmetric systems A_t x_t = b_t of
 * uneven sizes (section II-C each), one workgroup per instance in one
 * persistent launch, every message of an instance in LDS, so no host round
 * trip happens between sweeps and each instance stops on its own: at every
 * check (every check_every sweeps, 0 = 2; with Aitken every accel_stride
 * sweeps; with Steffensen at the end of each cycle) the FP64 residual
 * ||b_t - A_t x_t|| / ||b_t|| of the instance's current answer is computed and
 * the instance stops once it meets tol.  An inner solve that has converged to
 * its own target or stagnated at the message precision restarts on the
 * residual (refinement, as for gabp_solve).  Both schedules: synchronous, or
 * the serial scheme in the order of a colouring the plan computes on the host
 * (two colours where an instance's graph is bipartite, else greedy first-fit
 * in row order; gabp_plan_colors reports it).  b and x are packed like the
 * rows.  Limits (GABP_ERR_UNSUPPORTED beyond): k_t <= 4096 rows; the
 * messages of the largest instance must fit the 160 KB LDS: directed edges x
 * 16 bytes (FP32) or 32 bytes (FP64) under the synchronous schedule (two
 * buffers), half that under the coloured one, plus 8 bytes per row; at most
 * 2^31 - 1 directed edges in all.  gabp_plan_reset / sweeps / marginals /
 * get_messages / set_messages work as for a CSR plan of the whole
 * block-diagonal matrix (messages at the CSR slot of A_ij). */
/* Validates every instance on the device (finite entries; dense: exactly
 * symmetric with nonzero diagonal; bipartite: sigma2 finite and > 0), keeps a
 * working-precision copy of the couplings and allocates the message state
 * (16 bytes per entry of each matrix in FP32, 32 in FP64, plus the same again
 * once the settled-precision phase is used). */
int gabp_plan_create_batched(const gabp_batch *B, const gabp_opts *o, gabp_plan **plan,
                             hipStream_t stream);
/* Solves every instance from zero messages.
 *   b             device, packed right-hand sides as above.
 *   x             device, packed solutions (FP64).
 *   per_instance  host [count] or NULL: stats of each instance (status, sweeps,
 *                 frozen_sweeps, restarts, checks, rel_residual, edges;
 *                 residual_per_eq = ||r||_2 / K_t).
 *   summary       host or NULL: status = the worst instance status, sweeps and
 *                 restarts = the largest over instances, edges = directed
 *                 messages per sweep summed over instances, seconds = wall time,
 *                 sweep_ms = device time of the launch, edge_updates_per_s =
 *                 sum over instances of edges x sweeps / seconds.
 * Returns the worst instance status (a negative code if any instance failed,
 * else GABP_NOT_CONVERGED if any did not converge, else GABP_OK).  For batched
 * plans gabp_plan_solve does the same with `st` as the summary and marg_prec
 * (device, packed like x, or NULL) the marginal precisions of the unknowns;
 * gabp_plan_reset / sweeps / marginals work as for CSR plans with the node
 * values packed per instance (bipartite: K_t users then N_t chips; dense: K_t
 * nodes) and the same right-hand-side packing as solve; get/set_messages
 * return GABP_ERR_UNSUPPORTED. */
int gabp_plan_solve_batched(gabp_plan *plan, const double *b, double *x,
                            gabp_stats *per_instance, gabp_stats *summary, hipStream_t stream);
int gabp_solve_batched(const gabp_batch *B, const double *b, double *x, const gabp_opts *o,
                       gabp_stats *per_instance, gabp_stats *summary, hipStream_t stream);

/* ---- Any sparse matrix: regularised least squares (section VII) ---------
 * For an m x k matrix S (any shape; square and nonsymmetric included) and
 * psi > 0, section VII builds the symmetric (k + m) x (k + m) system
 *     [[I_k, S^T], [S, -psi I_m]] [x; z] = [0; y]
 * whose first k unknowns are x = (S^T S + psi I)^{-1} S^T y (psi -> 0: the
 * Moore-Penrose solution S^+ y, which GaBP cannot reach: a zero diagonal).
 * The plan assembles that system on the device (unknowns x first, then z;
 * rows sorted) and solves it as a CSR plan in the pair layout, so every
 * option and trajectory call of CSR plans applies to it with vectors of
 * length k + m. */
typedef struct {
  int32_t m, k;              /* rows and columns of S, >= 0 */
  int64_t nnz;
  const int64_t *row_ptr;    /* device [m + 1], row_ptr[0] = 0, row_ptr[m] = nnz */
  const int32_t *col;        /* device [nnz], strictly increasing within a row, in [0, k) */
  const double *val;         /* device [nnz], finite */
} gabp_rect;
/* Validates S (GABP_ERR_ARG on a bad row_ptr, an out-of-range or unsorted
 * column, a non-finite value, psi <= 0 or not finite; GABP_ERR_UNSUPPORTED if
 * 2 nnz + k + m does not fit in 31 bits) and keeps the assembled system; S
 * itself is not read after this call. */
int gabp_plan_create_lsq(const gabp_rect *S, double psi, const gabp_opts *o, gabp_plan **plan,
                         hipStream_t stream);
/* x (device, k, FP64) from y (device, m, FP64).  The stop rule and
 * st->rel_residual are those of the assembled system,
 * ||[0; y] - R [x; z]||_2 / ||y||_2 <= tol; the least-squares residual of x
 * is gabp_plan_residual_lsq's. */
int gabp_plan_solve_lsq(gabp_plan *plan, const double *y, double *x, gabp_stats *st,
                        hipStream_t stream);
int gabp_solve_lsq(const gabp_rect *S, double psi, const double *y, double *x,
                   const gabp_opts *o, gabp_stats *st, hipStream_t stream);
/* FP64 residual of the regularised normal equations of an lsq plan:
 * r = S^T y - (S^T S + psi I) x (device, k, or NULL) and
 * *rel_norm = ||r||_2 / ||S^T y||_2 (||r||_2 when S^T y = 0). */
int gabp_plan_residual_lsq(gabp_plan *plan, const double *y, const double *x, double *r,
                           double *rel_norm, hipStream_t stream);

/* ---- Learned warm start for grid solves (not part of the paper) ----------
 * A per-node network proposes the initial messages of a structured-grid solve
 * in place of the zero messages of Algorithm 1 step 1; the iteration, its
 * fixed point and the answer x = A^{-1} b are unchanged.  Network: 8 inputs,
 * two hidden layers of 64 ReLU units, 12 outputs; parameters held in bfloat16
 * with FP32 masters and Adam moments; FP32 accumulation everywhere.
 *   inputs of node i:  (log A_ii, a_1/A_ii, ..., a_6/A_ii, b_i/A_ii), a_d the
 *                      coupling to the neighbour in direction d (+x, -x, +y,
 *                      -y, +z, -z), 0 where there is none;
 *   outputs:           (P_d/A_ii, h_d/A_ii) of the message toward direction d
 *                      (information form h = P mu), ignored where a_d = 0.
 * Flat parameter order (GABP_MODEL_PARAMS floats): W1 [64][8], b1 [64],
 * W2 [64][64], b2 [64], W3 [12][64], b3 [12]. */
enum { GABP_MODEL_INPUTS = 8, GABP_MODEL_OUTPUTS = 12, GABP_MODEL_PARAMS = 5516 };
typedef struct gabp_model gabp_model;
/* He-uniform weights from `seed` (splitmix64 stream), zero biases. */
int gabp_model_create(uint64_t seed, gabp_model **model, hipStream_t stream);
int gabp_model_destroy(gabp_model *model);
/* params: host [GABP_MODEL_PARAMS].  get returns the bfloat16 values the
 * kernels use (widened); set stores FP32 masters, rounds them to bfloat16 and
 * clears the Adam state. */
int gabp_model_get_params(const gabp_model *model, float *params, hipStream_t stream);
int gabp_model_set_params(gabp_model *model, const float *params, hipStream_t stream);
/* out = network(U): U device [count][8], out device [count][12]. */
int gabp_model_forward(const gabp_model *model, const float *U, int64_t count, float *out,
                       hipStream_t stream);
/* Masked mean squared error / 2 over the outputs whose direction has a
 * neighbour (U[s][1 + d] != 0), and its gradient (device [GABP_MODEL_PARAMS],
 * may be NULL); train_step then applies one Adam step (beta 0.9, 0.999,
 * eps 1e-8) with step size lr.  loss: host, may be NULL.  T: device [count][12].
 * Deterministic: fixed-order reductions. */
int gabp_model_grad(gabp_model *model, const float *U, const float *T, int64_t count,
                    float *grad, double *loss, hipStream_t stream);
int gabp_model_train_step(gabp_model *model, const float *U, const float *T, int64_t count,
                          double lr, double *loss, hipStream_t stream);
/* Inputs and targets of grid nodes: nodes device [count] node indices, or NULL
 * for nodes 0..count-1 (an index outside [0, N) yields a zero row); b device
 * [N]; P, h device [6][N] messages as gabp_plan_get_messages returns them for
 * a grid plan. */
int gabp_model_grid_features(const gabp_grid *A, const double *b, const int64_t *nodes,
                             int64_t count, float *U, hipStream_t stream);
int gabp_model_grid_targets(const gabp_grid *A, const double *P, const double *h,
                            const int64_t *nodes, int64_t count, float *T, hipStream_t stream);
/* gabp_plan_solve of a grid plan starting from the network's messages, with
 * plain zero-message GaBP as the fallback (see gabp_stats.warm_start). */
int gabp_plan_solve_warm(gabp_plan *plan, const gabp_model *model, const double *b, double *x,
                         double *marg_prec, gabp_stats *st, hipStream_t stream);

/* ---- Coarse-grid predicted corrections for grid solves (not part of the
 * paper; a predictor from beyond a node's neighbourhood) --------------------
 * GaBP reduces the smooth part of the error slowly: on a Poisson operator it
 * converges like a relaxation whose slowest modes are the smoothest, and the
 * information messages that would remove them are globally determined, so no
 * initial messages computed from a node's own neighbourhood can supply them.
 * This solve predicts every correction of the refinement loop on coarser
 * grids.  With r = b - A x (FP64), the correction d of A d = r is
 *   d  = means of 3 GaBP sweeps on r (the plan's schedule and message
 *        precision, zero information messages, the precision messages of the
 *        level's previous sweeps kept);
 *   d += 1.8 P e, where e solves the next coarser grid's system
 *        P^T A P e = rc, rc = P^T (r - A d), by two applications of the same
 *        procedure (e = the first's result, then e += the second's on
 *        rc - P^T A P e: a W-cycle; one application when the coarser grids
 *        have at most 4096 cells), P the 2 x 2 x 2 block indicator (an axis
 *        of extent 1 is not halved) and P^T A P the Galerkin product (again a
 *        5/7-point stencil), recursively down to the first grid below the
 *        plan's with at most 512 cells (at most 64 when the dense inverses of
 *        512-cell grids would take more than 1 GiB), whose systems are
 *        solved exactly (their dense inverses, built once; the level above
 *        takes that exact solution once instead of two cycles; a plan whose
 *        own grids have at most 64 cells is corrected by the means of 24
 *        sweeps instead);
 *   d += means of 3 GaBP sweeps on r - A d;
 * then, on every grid t of the stack, with w = A d and (pc, pw) the previous
 * correction's direction and its image (none on the first):
 *   beta = (w, pw) / (pw, pw), d' = d - beta pc, w' = w - beta pw,
 *   x += alpha d', alpha = (r, w') / (w', w')
 * (inner products over the grid's cells; beta = 0 when w' keeps less than
 * 1e-10 of (w, w)): the generalized conjugate residual step over the last two
 * corrections, which minimises the grid's residual over both; repeated
 * until every grid of the stack meets tol (each grid's own
 * ||b_t - A_t x_t|| / ||b_t||).  The sweeps use the plan's damping, except
 * that an undamped synchronous plan sweeps with damping 0.3 here: undamped
 * synchronous sweeps leave the error mode that alternates between the two
 * colours of a grid, and the cycle diverges.  The coarse levels are built on the first call
 * and kept with the plan (about 1/7 of the plan's memory, plus three FP64
 * vectors of the plan's size for the combination of the corrections).  Grid plans only
 * (GABP_ERR_UNSUPPORTED otherwise); st->restarts counts the corrections
 * (at most opts.max_restarts), st->sweeps the sweeps on the plan's own grid.
 * The dense inverses of the coarsest level take at most 1 GiB, and building
 * those of more than 64 cells per grid holds about twice their size for the
 * duration of the first call.  Environment, read when the levels are built:
 * GABP_COARSE_EXACT=64 (coarsest level of at most 64 cells), GABP_COARSE_TAIL=0
 * (with it, the small levels as plans instead of one launch per visit),
 * GABP_COARSE_WCYCLE=1 (two cycles of every level), GABP_COARSE_GCR=0 (the
 * corrections added as they come), GABP_COARSE_GRAPH=0 (no graph replay).
 * Arguments as for gabp_plan_solve. */
int gabp_plan_solve_coarse(gabp_plan *plan, const double *b, double *x, double *marg_prec,
                           gabp_stats *st, hipStream_t stream);

/* Library version string. */
const char *gabp_version(void);

#ifdef __cplusplus
}
#endif
#endif /* GABP_H */
