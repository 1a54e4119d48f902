// Coarse grids of a stack of grids (coarse-grid predicted corrections of
// grid solves): the Galerkin operator of 2 x 2 x 2 aggregation, restriction
// (block sums) and prolongation (injection) of FP64 vectors.
//
// Cell (x, y, z) of a grid belongs to the coarse cell (x / 2, y / 2, z / 2),
// an axis of extent 1 is not halved.  With P the indicator matrix of that map
// the coarse operator is A_c = P^T A P: (A_c)_IJ is the sum of A_ij over i in
// I and j in J.  For a 5/7-point stencil that is again a 5/7-point stencil:
// the diagonal of I collects the fine diagonals of its cells and twice every
// coupling inside the block; the coupling of I with its +x neighbour collects
// the fine +x couplings that cross the block's +x face.
#include "device_common.h"

namespace gabp {
namespace {

__device__ __forceinline__ int half_up(int n) { return n > 1 ? (n + 1) / 2 : 1; }

// (x, y, z) of cell i of a stack and its grid t
__device__ __forceinline__ void grid_coords(const GridGeom &g, int i, int &x, int &y, int &z,
                                            int &t) {
  const int r = fdiv(i, g.fx);
  x = i - r * g.nx;
  const int q = fdiv(r, g.fy);
  y = r - q * g.ny;
  t = fdiv(q, g.fz);
  z = q - t * g.nz;
}

__global__ void k_coarse_coef(GridGeom f, GridCoef<double> k, int varc, GridGeom c,
                              double *__restrict__ dg, double *__restrict__ cx,
                              double *__restrict__ cy, double *__restrict__ cz) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= c.N) return;
  const int nf = f.nx * f.ny * f.nz;
  int t, X, Y, Z;
  grid_coords(c, I, X, Y, Z, t);
  const int sx = f.nx > 1 ? 2 : 1, sy = f.ny > 1 ? 2 : 1, sz = f.nz > 1 ? 2 : 1;
  const int x0 = X * sx, y0 = Y * sy, z0 = Z * sz;
  const int x1 = min(x0 + sx, f.nx), y1 = min(y0 + sy, f.ny), z1 = min(z0 + sz, f.nz);
  double d = 0.0, ax = 0.0, ay = 0.0, az = 0.0;
  for (int z = z0; z < z1; ++z)
    for (int y = y0; y < y1; ++y)
      for (int x = x0; x < x1; ++x) {
        const int i = t * nf + x + f.nx * (y + f.ny * z);
        d += varc ? k.diag[i] : k.dconst;
        if (x < f.nx - 1) {  // the +x face of cell i is a coupling
          const double a = varc ? k.cx[i] : k.aconst;
          if (x + 1 < x1) d += 2.0 * a;  // both cells in the block: A_ij + A_ji
          else ax += a;                  // crosses into block X + 1
        }
        if (y < f.ny - 1) {
          const double a = varc ? k.cy[i] : k.aconst;
          if (y + 1 < y1) d += 2.0 * a;
          else ay += a;
        }
        if (z < f.nz - 1) {
          const double a = varc ? k.cz[i] : k.aconst;
          if (z + 1 < z1) d += 2.0 * a;
          else az += a;
        }
      }
  dg[I] = d;
  cx[I] = ax;
  cy[I] = ay;
  cz[I] = az;
}

// rc[I] = sum of r over the cells of block I (fixed order: z, y, x)
__global__ void k_coarse_restrict(GridGeom f, GridGeom c, const double *__restrict__ r,
                                  double *__restrict__ rc) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= c.N) return;
  const int nf = f.nx * f.ny * f.nz;
  int t, X, Y, Z;
  grid_coords(c, I, X, Y, Z, t);
  const int sx = f.nx > 1 ? 2 : 1, sy = f.ny > 1 ? 2 : 1, sz = f.nz > 1 ? 2 : 1;
  const int x0 = X * sx, y0 = Y * sy, z0 = Z * sz;
  const int x1 = min(x0 + sx, f.nx), y1 = min(y0 + sy, f.ny), z1 = min(z0 + sz, f.nz);
  double s = 0.0;
  for (int z = z0; z < z1; ++z)
    for (int y = y0; y < y1; ++y)
      for (int x = x0; x < x1; ++x) s += r[t * nf + x + f.nx * (y + f.ny * z)];
  rc[I] = s;
}

// d[i] += scale * (dc + dc2)[block of i] (the sum formed as e = e + d
// would form it)
__global__ void k_coarse_prolong(GridGeom f, GridGeom c, const double *__restrict__ dc,
                                 const double *__restrict__ dc2, double scale,
                                 double *__restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= f.N) return;
  const int nc = c.nx * c.ny * c.nz;
  int t, x, y, z;
  grid_coords(f, i, x, y, z, t);
  // an axis of extent 1 is not halved
  const int hx = f.nx > 1, hy = f.ny > 1, hz = f.nz > 1;
  const int I = t * nc + (x >> hx) + c.nx * ((y >> hy) + c.ny * (z >> hz));
  double e = dc[I];
  if (dc2) e += dc2[I];
  d[i] += scale * e;
}

// the working right-hand side of cell i (WorkRhs)
__device__ __forceinline__ void put_work_rhs(const GridGeom &g, const WorkRhs &w, int i,
                                             double r) {
  if (!w.p) return;
  int at = i;
  if (w.hx > 0) {
    int c, slot;
    rb_place(g, w.hx, i, c, slot);
    at = c * w.nc + slot;
  }
  if (w.fp32) ((float *)w.p)[at] = (float)r;
  else ((double *)w.p)[at] = r;
}

// (A x)_i of a 5/7-point stack in FP64, terms in the order of the grid
// residual (diagonal first, then +x, -x, +y, -y, +z, -z), so that the fused
// kernels below give bitwise the results of residual + restriction
template <bool VARC>
__device__ __forceinline__ double stencil_ax(const GridGeom &g, const GridCoef<double> &k,
                                             const double *__restrict__ x, int i, int xx, int y,
                                             int zl) {
  const int nxy = g.nx * g.ny;
  const bool ok[6] = {xx < g.nx - 1, xx > 0, y < g.ny - 1, y > 0, zl < g.nz - 1, zl > 0};
  const int j[6] = {i + 1, i - 1, i + g.nx, i - g.nx, i + nxy, i - nxy};
  double a[6];
  if (VARC) {
    a[0] = ok[0] ? k.cx[i] : 0.0;
    a[1] = ok[1] ? k.cx[i - 1] : 0.0;
    a[2] = ok[2] ? k.cy[i] : 0.0;
    a[3] = ok[3] ? k.cy[i - g.nx] : 0.0;
    a[4] = ok[4] ? k.cz[i] : 0.0;
    a[5] = ok[5] ? k.cz[i - nxy] : 0.0;
  } else {
#pragma unroll
    for (int d = 0; d < 6; ++d) a[d] = ok[d] ? k.aconst : 0.0;
  }
  double xn[6];  // loaded on the geometry alone, not after the couplings
#pragma unroll
  for (int d = 0; d < 6; ++d) xn[d] = ok[d] ? x[j[d]] : 0.0;
  double ax = (VARC ? k.diag[i] : k.dconst) * x[i];
#pragma unroll
  for (int d = 0; d < 6; ++d)
    if (a[d] != 0.0) ax += a[d] * xn[d];
  return ax;
}
template <bool VARC>
__device__ __forceinline__ double stencil_ax(const GridGeom &g, const GridCoef<double> &k,
                                             const double *__restrict__ x, int i) {
  int xx, y, zl, t;
  grid_coords(g, i, xx, y, zl, t);
  return stencil_ax<VARC>(g, k, x, i, xx, y, zl);
}

// rc[I] = sum over the cells i of block I of (v - A d)_i.  Eight lanes per
// coarse cell, lane k on the child (k & 1, (k >> 1) & 1, k >> 2) of the
// 2 x 2 x 2 block (absent children add 0), summed by a fixed butterfly over
// the eight lanes, so every lane holds the same sum; consecutive coarse
// cells on consecutive lane groups keep the fine reads in runs along x.
template <bool VARC>
__global__ __launch_bounds__(kBlock) void k_coarse_residual_restrict(
    GridGeom f, GridCoef<double> k, GridGeom c, const double *__restrict__ v,
    const double *__restrict__ d, double *__restrict__ rc, WorkRhs w) {
  const int64_t t8 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int I = (int)(t8 >> 3), kid = threadIdx.x & 7;
  double r = 0.0;
  if (I < c.N) {
    const int nf = f.nx * f.ny * f.nz;
    int t, X, Y, Z;
    grid_coords(c, I, X, Y, Z, t);
    const int sx = f.nx > 1 ? 2 : 1, sy = f.ny > 1 ? 2 : 1, sz = f.nz > 1 ? 2 : 1;
    const int dx = kid & 1, dy = (kid >> 1) & 1, dz = kid >> 2;
    const int x = X * sx + dx, y = Y * sy + dy, z = Z * sz + dz;
    if (dx < sx && dy < sy && dz < sz && x < f.nx && y < f.ny && z < f.nz) {
      const int i = t * nf + x + f.nx * (y + f.ny * z);
      r = v[i];
      r -= stencil_ax<VARC>(f, k, d, i, x, y, z);
    }
  }
  r += __shfl_xor(r, 1, 8);
  r += __shfl_xor(r, 2, 8);
  r += __shfl_xor(r, 4, 8);
  if (I < c.N && kid == 0) {
    rc[I] = r;
    put_work_rhs(c, w, I, r);
  }
}

// e = d and v = v - A d: the right-hand side of a level's next cycle
template <bool VARC>
__global__ void k_coarse_copy_residual(GridGeom g, GridCoef<double> k, const double *__restrict__ d,
                                       double *__restrict__ e, double *__restrict__ v, WorkRhs w) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  e[i] = d[i];
  double r = v[i];
  r -= stencil_ax<VARC>(g, k, d, i);
  v[i] = r;
  put_work_rhs(g, w, i, r);
}

// GCR(1) combination of the coarse-grid corrections, one step per grid of
// the stack.  Partial sums per block over one grid's cells (the blocks of a
// segment, as in the grid residual): (r, w), (w, w), (w, pw), (r, pw) with
// w = A c written out; pw is the previous step's direction image (not read
// on the first step).
template <bool VARC>
__global__ __launch_bounds__(kBlock) void k_gcr_dots(GridGeom g, GridCoef<double> k,
                                                     const double *__restrict__ c,
                                                     const double *__restrict__ r,
                                                     const double *__restrict__ pw,
                                                     double *__restrict__ w,
                                                     double *__restrict__ part, int nseg,
                                                     int first) {
  const int segb = gridDim.x / nseg;
  const int seg = blockIdx.x / segb;
  const int len = g.N / nseg;
  const int hi = (seg + 1) * len;
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  for (int i = seg * len + (blockIdx.x - seg * segb) * kBlock + threadIdx.x; i < hi;
       i += segb * kBlock) {
    int xx, y, zl, t;
    grid_coords(g, i, xx, y, zl, t);
    const double wi = stencil_ax<VARC>(g, k, c, i, xx, y, zl);
    w[i] = wi;
    const double ri = r[i];
    s[0] += ri * wi;
    s[1] += wi * wi;
    if (!first) {
      const double p = pw[i];
      s[2] += wi * p;
      s[3] += ri * p;
    }
  }
  __shared__ double sh[4][kBlock / 64];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double v = wave_sum(s[q]);
    if ((threadIdx.x & 63) == 0) sh[q][threadIdx.x / 64] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double v = 0.0;
    for (int wv = 0; wv < kBlock / 64; ++wv) v += sh[threadIdx.x][wv];
    part[(size_t)blockIdx.x * 4 + threadIdx.x] = v;
  }
}

// alpha and beta of each grid's step from its blocks' partial sums, one
// workgroup per grid (thread k adds the partials of blocks k, k + kBlock, ...,
// then a fixed-order reduction: the same sums on every run):
// beta = (w, pw) / (pw, pw), so that w' = w - beta pw is orthogonal to pw, and
// alpha = (r, w') / (w', w'); (w', w') and (r, w') expanded from the sums.  A
// w' keeping less than kGcrParallel of (w, w) takes beta = 0.  pp: (w', w')
// of each grid's last step, kept for the next.
__global__ __launch_bounds__(kBlock) void k_gcr_coef(const double *__restrict__ part, int segb,
                                                     int first, double *__restrict__ pp,
                                                     double2 *__restrict__ ab) {
  const int t = blockIdx.x;
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = threadIdx.x; b < segb; b += kBlock) {
    const double *q = part + ((size_t)t * segb + b) * 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] += q[j];
  }
  __shared__ double sh[4][kBlock / 64];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const double u = wave_sum(v[j]);
    if ((threadIdx.x & 63) == 0) sh[j][threadIdx.x / 64] = u;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double rw = 0.0, ww = 0.0, wp = 0.0, rp = 0.0;
  for (int wv = 0; wv < kBlock / 64; ++wv) {
    rw += sh[0][wv];
    ww += sh[1][wv];
    wp += sh[2][wv];
    rp += sh[3][wv];
  }
  double beta = 0.0, w2 = ww, rw2 = rw;
  const double ppt = first ? 0.0 : pp[t];
  if (ppt > 0.0) {
    const double bt = wp / ppt;
    const double wo = ww - 2.0 * bt * wp + bt * bt * ppt;
    if (wo > kGcrParallel * ww) {
      beta = bt;
      w2 = wo;
      rw2 = rw - bt * rp;
    }
  }
  pp[t] = w2;
  ab[t] = make_double2(w2 > 0.0 ? rw2 / w2 : 0.0, beta);
}

// c' = c - beta pc, w' = w - beta pw, x += alpha c', then (pc, pw) = (c', w');
// the residual follows: r -= alpha w', into wr as well, and one partial sum
// of r^2 per block (the blocks of a segment, as in k_gcr_dots)
__global__ __launch_bounds__(kBlock) void k_gcr_update(GridGeom g, const double *__restrict__ c,
                                                       const double *__restrict__ w,
                                                       const double2 *__restrict__ ab, int first,
                                                       double *__restrict__ pc,
                                                       double *__restrict__ pw,
                                                       double *__restrict__ x,
                                                       double *__restrict__ r, WorkRhs wr,
                                                       double *__restrict__ sumpart, int nseg) {
  const int segb = gridDim.x / nseg;
  const int seg = blockIdx.x / segb;
  const int len = g.N / nseg;
  const int hi = (seg + 1) * len;
  double sq = 0.0;
  for (int i = seg * len + (blockIdx.x - seg * segb) * kBlock + threadIdx.x; i < hi;
       i += segb * kBlock) {
    const double2 q = ab[seg];  // a segment is one grid of the stack
    double ci = c[i], wi = w[i];
    if (!first && q.y != 0.0) {
      ci -= q.y * pc[i];
      wi -= q.y * pw[i];
    }
    x[i] += q.x * ci;
    pc[i] = ci;
    pw[i] = wi;
    const double ri = r[i] - q.x * wi;
    r[i] = ri;
    put_work_rhs(g, wr, i, ri);
    sq += ri * ri;
  }
  __shared__ double sh[kBlock / 64];
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x / 64] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = sh[0];
    for (int wv = 1; wv < kBlock / 64; ++wv) v += sh[wv];
    sumpart[blockIdx.x] = v;
  }
}

__global__ void k_axpy(int n, const double *__restrict__ d, double *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += d[i];
}

dim3 blocks_for(int n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

// ---------------------------------------------------------------------------
// The coarsest levels in one launch
// ---------------------------------------------------------------------------
// Below a few hundred cells per grid a level's launches last a few
// microseconds each and the W-cycle visits the coarsest level 2^(levels - 1)
// times per correction, so the small levels' launches, not their sweeps, set
// the time of a correction.  k_coarse_tail does everything the level above
// asks of them in one workgroup per grid: each thread owns one cell of every
// tail level; the GaBP messages are kept per receiving cell (slot d of cell i:
// the message from its neighbour in direction d = +x, -x, +y, -y, +z, -z), so
// a sending cell reads its own in-slots and writes the in-slot d ^ 1 of each
// neighbour.  Arithmetic is FP64 whatever the plan's message precision.

// Dynamic LDS of the tail kernel; a level is a set of offsets into it, 21
// doubles per cell (so that every access is an LDS access).
extern __shared__ double tail_sm[];
constexpr int kTailDoublesPerCell = 21;

struct TL {
  int nx, ny, nz, n, zpar;  // zpar: parity of the grid's first plane in the stack
  int P, h;                 // in-messages [6][n]
  int dg, cx, cy, cz;
  int V, D, T, RC, E;  // rhs, cycle result, work, restricted residual, summed result
};

__device__ __forceinline__ int tail_cells(const TailLevel &L) { return L.nx * L.ny * L.nz; }

__device__ __forceinline__ TL tail_level(const TailArgs &a, int l, int t) {
  int p = 0;
  for (int m = 0; m < l; ++m) p += kTailDoublesPerCell * tail_cells(a.lv[m]);
  TL L;
  L.nx = a.lv[l].nx; L.ny = a.lv[l].ny; L.nz = a.lv[l].nz;
  const int n = L.nx * L.ny * L.nz;
  L.n = n;
  L.zpar = (t * L.nz) & 1;  // the checkerboard counts z over the whole stack
  L.P = p; L.h = p + 6 * n;
  p += 12 * n;
  L.dg = p; L.cx = p + n; L.cy = p + 2 * n; L.cz = p + 3 * n;
  p += 4 * n;
  L.V = p; L.D = p + n; L.T = p + 2 * n; L.RC = p + 3 * n; L.E = p + 4 * n;
  return L;
}

// the coarsest level's inverse follows every level's arrays
__device__ __forceinline__ int tail_inverse_offset(const TailArgs &a) {
  int p = 0;
  for (int m = 0; m < a.nlev; ++m) p += kTailDoublesPerCell * tail_cells(a.lv[m]);
  return p;
}

// neighbour of cell i in direction d and their coupling (0: no edge)
__device__ __forceinline__ void tail_edges(const TL &L, int i, int j[6], double a[6]) {
  const double *S = tail_sm;
  const int x = i % L.nx, y = (i / L.nx) % L.ny, z = i / (L.nx * L.ny);
  const int sy = L.nx, sz = L.nx * L.ny;
  j[0] = i + 1;  a[0] = x < L.nx - 1 ? S[L.cx + i] : 0.0;
  j[1] = i - 1;  a[1] = x > 0 ? S[L.cx + i - 1] : 0.0;
  j[2] = i + sy; a[2] = y < L.ny - 1 ? S[L.cy + i] : 0.0;
  j[3] = i - sy; a[3] = y > 0 ? S[L.cy + i - sy] : 0.0;
  j[4] = i + sz; a[4] = z < L.nz - 1 ? S[L.cz + i] : 0.0;
  j[5] = i - sz; a[5] = z > 0 ? S[L.cz + i - sz] : 0.0;
}

// the k-th cell of colour c (in the order of the grid layout; -1: none):
// row r = (y, z) holds the cells x = 2 kx + ((c + y + z + zpar) & 1)
__device__ __forceinline__ int tail_colour_cell(const TL &L, int c, int k) {
  const int hx = (L.nx + 1) >> 1;
  const int r = k / hx;
  if (r >= L.ny * L.nz) return -1;
  const int kx = k - r * hx, y = r % L.ny, z = r / L.ny;
  const int x = 2 * kx + ((c + y + z + L.zpar) & 1);
  return x < L.nx ? x + L.nx * r : -1;
}

// The out-messages of cell i from its in-slots (slots of absent edges hold
// zeros: no one writes them); av: its couplings (0: no edge).
__device__ __forceinline__ void tail_out(const TL &L, int i, const double av[6], int R,
                                         double Pn[6], double hn[6], uint32_t &flags) {
  const double *S_ = tail_sm;
  const int n = L.n;
  double Pi[6], hi[6], S = S_[L.dg + i], H = S_[R + i];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    Pi[d] = S_[L.P + d * n + i];
    hi[d] = S_[L.h + d * n + i];
    S += Pi[d];
    H += hi[d];
  }
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const double cav = S - Pi[d];
    if (av[d] != 0.0 && cav == 0.0) flags |= FLAG_BREAKDOWN;
    const double inv = 1.0 / cav;
    Pn[d] = -(av[d] * av[d]) * inv;
    hn[d] = -(av[d] * (H - hi[d])) * inv;
  }
}

// the out-messages into the neighbours' in-slots d ^ 1, damped with the old
// message of the same directed edge
__device__ __forceinline__ void tail_put(const TL &L, int i, const double av[6], double al,
                                         const double Pn[6], const double hn[6]) {
  double *S_ = tail_sm;
  const int n = L.n;
  const int step[6] = {1, -1, L.nx, -L.nx, L.nx * L.ny, -L.nx * L.ny};
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    if (av[d] == 0.0) continue;
    const int o = (d ^ 1) * n + i + step[d];
    double P = Pn[d], h = hn[d];
    if (al > 0.0) {
      P = al * S_[L.P + o] + (1.0 - al) * P;
      h = al * S_[L.h + o] + (1.0 - al) * h;
    }
    S_[L.P + o] = P;
    S_[L.h + o] = h;
  }
}

// D (= or +=) the means of `sweeps` GaBP sweeps on right-hand side R (an
// offset) from zero information messages, the level's precision messages
// kept.  Coloured: a thread takes the k-th cell of each colour, so that only
// as many waves as a class has cells do the work of a half sweep.
__device__ __forceinline__ void tail_smooth(const TL &L, int R, int sweeps, bool add,
                                            const TailArgs &a, uint32_t &flags) {
  double *S_ = tail_sm;
  const int t = threadIdx.x, n = L.n;
  int i0, i1;
  if (a.colored) {
    i0 = tail_colour_cell(L, 0, t);
    i1 = tail_colour_cell(L, 1, t);
  } else {
    i0 = t < n ? t : -1;
    i1 = -1;
  }
  double a0[6], a1[6];
  int jj[6];
  if (i0 >= 0) tail_edges(L, i0, jj, a0);
  if (i1 >= 0) tail_edges(L, i1, jj, a1);
  if (t < n) {
#pragma unroll
    for (int d = 0; d < 6; ++d) S_[L.h + d * n + t] = 0.0;
  }
  __syncthreads();
  const double al = a.damping;
  double Pn[6], hn[6];
  for (int s = 0; s < sweeps; ++s) {
    if (a.colored) {
      // a class writes only the other class's in-slots
      if (i0 >= 0) {
        tail_out(L, i0, a0, R, Pn, hn, flags);
        tail_put(L, i0, a0, al, Pn, hn);
      }
      __syncthreads();
      if (i1 >= 0) {
        tail_out(L, i1, a1, R, Pn, hn, flags);
        tail_put(L, i1, a1, al, Pn, hn);
      }
      __syncthreads();
    } else {
      // every cell reads its in-slots before any is written
      if (i0 >= 0) tail_out(L, i0, a0, R, Pn, hn, flags);
      __syncthreads();
      if (i0 >= 0) tail_put(L, i0, a0, al, Pn, hn);
      __syncthreads();
    }
  }
  if (t < n) {
    double S = S_[L.dg + t], H = S_[R + t];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      S += S_[L.P + d * n + t];
      H += S_[L.h + d * n + t];
    }
    if (S == 0.0) flags |= FLAG_BREAKDOWN;
    const double m = H / S;
    if (!isfinite(m)) flags |= FLAG_NONFINITE;
    S_[L.D + t] = add ? S_[L.D + t] + m : m;
  }
  __syncthreads();
}

// out = R - A X (offsets)
__device__ __forceinline__ void tail_residual(const TL &L, int R, int X, int out) {
  double *S_ = tail_sm;
  const int i = threadIdx.x;
  if (i < L.n) {
    int j[6];
    double av[6];
    tail_edges(L, i, j, av);
    double s = S_[L.dg + i] * S_[X + i];
#pragma unroll
    for (int d = 0; d < 6; ++d)
      if (av[d] != 0.0) s += av[d] * S_[X + j[d]];
    S_[out + i] = S_[R + i] - s;
  }
  __syncthreads();
}

// C.RC = C.V = block sums of F.T (fixed order: z, y, x)
__device__ __forceinline__ void tail_restrict(const TL &F, const TL &C) {
  double *S_ = tail_sm;
  const int I = threadIdx.x;
  if (I < C.n) {
    const int X = I % C.nx, Y = (I / C.nx) % C.ny, Z = I / (C.nx * C.ny);
    const int sx = F.nx > 1 ? 2 : 1, sy = F.ny > 1 ? 2 : 1, sz = F.nz > 1 ? 2 : 1;
    const int x0 = X * sx, y0 = Y * sy, z0 = Z * sz;
    const int x1 = min(x0 + sx, F.nx), y1 = min(y0 + sy, F.ny), z1 = min(z0 + sz, F.nz);
    double s = 0.0;
    for (int z = z0; z < z1; ++z)
      for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) s += S_[F.T + x + F.nx * (y + F.ny * z)];
    S_[C.RC + I] = s;
    S_[C.V + I] = s;
  }
  __syncthreads();
}

// F.D += scale * C.E[block of the cell]
__device__ __forceinline__ void tail_prolong(const TL &F, const TL &C, double scale) {
  double *S_ = tail_sm;
  const int i = threadIdx.x;
  if (i < F.n) {
    const int x = i % F.nx, y = (i / F.nx) % F.ny, z = i / (F.nx * F.ny);
    const int sx = F.nx > 1 ? 2 : 1, sy = F.ny > 1 ? 2 : 1, sz = F.nz > 1 ? 2 : 1;
    S_[F.D + i] += scale * S_[C.E + x / sx + C.nx * (y / sy + C.ny * (z / sz))];
  }
  __syncthreads();
}

__global__ __launch_bounds__(kTailThreads) void k_coarse_tail(TailArgs a) {
  double *S_ = tail_sm;
  const int t = blockIdx.x, i = threadIdx.x;
  // the operators, the kept precision messages (zero at the start of a
  // solve), the coarsest inverse and the right-hand side
  for (int l = 0; l < a.nlev; ++l) {
    const TL L = tail_level(a, l, t);
    const TailLevel &G = a.lv[l];
    const int n = L.n;
    if (i < n) {
      const size_t g = (size_t)t * n + i;
      S_[L.dg + i] = G.dg[g];
      S_[L.cx + i] = G.cx[g];
      S_[L.cy + i] = G.cy[g];
      S_[L.cz + i] = G.cz[g];
      if (l < a.nlev - 1) {
#pragma unroll
        for (int d = 0; d < 6; ++d)
          S_[L.P + d * n + i] = a.fresh ? 0.0 : G.P[((size_t)t * 6 + d) * n + i];
      }
      if (l == 0) {
        const double r = a.rc[g];
        S_[L.RC + i] = r;
        S_[L.V + i] = r;
      }
    }
  }
  const TL Lc = tail_level(a, a.nlev - 1, t);
  const int inv = tail_inverse_offset(a);
  for (int k = i; k < Lc.n * Lc.n; k += kTailThreads)
    S_[inv + k] = a.inv[(size_t)t * Lc.n * Lc.n + k];
  __syncthreads();
  uint32_t flags = 0;
  // The W-cycle without recursion: l is the level being worked on (uniform
  // over the workgroup); cnt holds, 4 bits per level, how many cycles of that
  // level its parent has started; `entering`: a cycle of l begins.  Level 0
  // is driven by the caller's level: gamma cycles, then done.
  uint32_t cnt = 1u;
  int l = 0;
  bool entering = true;
  for (;;) {
    const TL L = tail_level(a, l, t);
    if (entering) {
      if (l == a.nlev - 1) {
        // the coarsest level: its exact solution
        if (i < L.n) {
          double d = 0.0;
          for (int j = 0; j < L.n; ++j) d += S_[inv + i * L.n + j] * S_[L.V + j];
          if (!isfinite(d)) flags |= FLAG_NONFINITE;
          S_[L.D + i] = d;
        }
        __syncthreads();
        entering = false;
        continue;
      }
      tail_smooth(L, L.V, a.pre, false, a, flags);
      tail_residual(L, L.V, L.D, L.T);
      tail_restrict(L, tail_level(a, l + 1, t));
      cnt = (cnt & ~(15u << (4 * (l + 1)))) | (1u << (4 * (l + 1)));
      ++l;
      continue;
    }
    // a cycle of level l is done (its result in D): sum it for the parent
    const int k = (int)((cnt >> (4 * l)) & 15u);
    if (i < L.n) S_[L.E + i] = k == 1 ? S_[L.D + i] : S_[L.E + i] + S_[L.D + i];
    __syncthreads();
    // the coarsest level's first cycle is already its exact solution
    if (k < (l == a.nlev - 1 ? 1 : a.gamma)) {
      tail_residual(L, L.RC, L.E, L.V);  // the next cycle's right-hand side
      cnt += 1u << (4 * l);
      entering = true;
      continue;
    }
    if (l == 0) break;
    --l;
    const TL F = tail_level(a, l, t);
    tail_prolong(F, L, a.scale);
    if (a.post > 0) {
      tail_residual(F, F.V, F.D, F.T);
      tail_smooth(F, F.T, a.post, true, a, flags);
    }
  }
  // the result and the precision messages for the next call
  for (int m = 0; m < a.nlev; ++m) {
    const TL L = tail_level(a, m, t);
    const int n = L.n;
    if (i < n) {
      if (m == 0) a.e[(size_t)t * n + i] = S_[L.E + i];
      if (m < a.nlev - 1) {
#pragma unroll
        for (int d = 0; d < 6; ++d) a.lv[m].P[((size_t)t * 6 + d) * n + i] = S_[L.P + d * n + i];
      }
    }
  }
  if (flags) atomicOr(a.sticky, flags);
}

// The coarsest level's dense matrix per grid, inverted by Gauss-Jordan
// elimination with partial pivoting on [M | I] in LDS: one workgroup per
// grid, thread r owns row r.
__global__ __launch_bounds__(kCoarsestCells) void k_coarse_inverse(
    GridGeom c, const double *__restrict__ dg, const double *__restrict__ cx,
    const double *__restrict__ cy, const double *__restrict__ cz, double *__restrict__ inv,
    uint32_t *__restrict__ flags) {
  extern __shared__ double gj[];
  __shared__ int piv;
  __shared__ double pval;
  const int n = c.nx * c.ny * c.nz, w = 2 * n + 1;  // row stride (padded)
  const int t = blockIdx.x, r = threadIdx.x;
  if (r < n) {
    for (int j = 0; j < 2 * n; ++j) gj[r * w + j] = 0.0;
    const size_t g = (size_t)t * n + r;
    const int x = r % c.nx, y = (r / c.nx) % c.ny, z = r / (c.nx * c.ny);
    const int sy = c.nx, sz = c.nx * c.ny;
    gj[r * w + r] = dg[g];
    if (x < c.nx - 1) gj[r * w + r + 1] = cx[g];
    if (x > 0) gj[r * w + r - 1] = cx[g - 1];
    if (y < c.ny - 1) gj[r * w + r + sy] = cy[g];
    if (y > 0) gj[r * w + r - sy] = cy[g - sy];
    if (z < c.nz - 1) gj[r * w + r + sz] = cz[g];
    if (z > 0) gj[r * w + r - sz] = cz[g - sz];
    gj[r * w + n + r] = 1.0;
  }
  __syncthreads();
  bool ok = true;
  for (int k = 0; k < n; ++k) {
    if (r == 0) {
      int p = k;
      double best = fabs(gj[k * w + k]);
      for (int q = k + 1; q < n; ++q)
        if (fabs(gj[q * w + k]) > best) {
          best = fabs(gj[q * w + k]);
          p = q;
        }
      piv = p;
      pval = gj[p * w + k];
    }
    __syncthreads();
    const int p = piv;
    const double pv = pval;
    if (pv == 0.0) {  // singular: the coarse system has no solution
      ok = false;
      break;
    }
    // swap rows k and p, scale the pivot row
    for (int j = r; j < 2 * n; j += blockDim.x) {
      const double a = gj[k * w + j], b = gj[p * w + j];
      gj[k * w + j] = b / pv;
      if (p != k) gj[p * w + j] = a;
    }
    __syncthreads();
    if (r < n && r != k) {
      const double f = gj[r * w + k];
      if (f != 0.0)
        for (int j = 0; j < 2 * n; ++j) gj[r * w + j] -= f * gj[k * w + j];
    }
    __syncthreads();
  }
  if (!ok) {
    if (r == 0) atomicOr(flags, (uint32_t)FLAG_BREAKDOWN);
    return;
  }
  for (int k = r; k < n * n; k += blockDim.x)
    inv[(size_t)t * n * n + k] = gj[(k / n) * w + n + k % n];
}

// The same elimination for coarsest levels of up to kCoarsestCellsMax cells,
// on [M | I] in global memory (`work`, n x 2n doubles per grid, row-major),
// one pivot step per pair of launches so that every grid's elimination is
// spread over the whole device: k_gj_setup writes [M | I]; k_gj_pivot (one
// workgroup per grid) finds the pivot row of column k (the largest |M[q][k]|
// over q >= k, ties to the lower row, by a tree reduction), swaps it into
// row k, divides it by the pivot and saves column k in F; k_gj_elim
// subtracts F[q] times row k from every other row q (one workgroup per row,
// the threads on consecutive columns).  Columns left of k are zero in the
// pivot row and are skipped.  A zero pivot flags the breakdown (the hierarchy
// is then not built) and skips that step's swap and elimination.
__global__ void k_gj_setup(GridGeom c, const double *__restrict__ dg,
                           const double *__restrict__ cx, const double *__restrict__ cy,
                           const double *__restrict__ cz, double *__restrict__ work) {
  const int n = c.nx * c.ny * c.nz, w = 2 * n;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)n * c.batch) return;
  const int t = (int)(q / n), r = (int)(q - (int64_t)t * n);
  double *row = work + q * w;
  for (int j = 0; j < w; ++j) row[j] = 0.0;
  const size_t g = (size_t)q;
  const int x = r % c.nx, y = (r / c.nx) % c.ny, z = r / (c.nx * c.ny);
  const int sy = c.nx, sz = c.nx * c.ny;
  row[r] = dg[g];
  if (x < c.nx - 1) row[r + 1] = cx[g];
  if (x > 0) row[r - 1] = cx[g - 1];
  if (y < c.ny - 1) row[r + sy] = cy[g];
  if (y > 0) row[r - sy] = cy[g - sy];
  if (z < c.nz - 1) row[r + sz] = cz[g];
  if (z > 0) row[r - sz] = cz[g - sz];
  row[n + r] = 1.0;
}

__global__ __launch_bounds__(kCoarsestCellsMax) void k_gj_pivot(int n, int k,
                                                                 double *__restrict__ work,
                                                                 double *__restrict__ F,
                                                                 uint32_t *__restrict__ flags) {
  __shared__ double best[kCoarsestCellsMax];
  __shared__ int arg[kCoarsestCellsMax];
  const int w = 2 * n, t = blockIdx.x, r = threadIdx.x;
  double *M = work + (size_t)t * n * w;
  double *Ft = F + (size_t)t * n;
  best[r] = (r >= k && r < n) ? fabs(M[(size_t)r * w + k]) : -1.0;
  arg[r] = r;
  __syncthreads();
  for (int h = kCoarsestCellsMax / 2; h > 0; h >>= 1) {
    if (r < h && (best[r + h] > best[r] || (best[r + h] == best[r] && arg[r + h] < arg[r]))) {
      best[r] = best[r + h];
      arg[r] = arg[r + h];
    }
    __syncthreads();
  }
  const int p = arg[0];
  const double pv = M[(size_t)p * w + k];
  if (pv == 0.0) {  // singular: no swap, and F = 0 makes the elimination a no-op
    if (r < n) Ft[r] = 0.0;
    if (r == 0) atomicOr(flags, (uint32_t)FLAG_BREAKDOWN);
    return;
  }
  __syncthreads();
  for (int j = k + r; j < w; j += blockDim.x) {
    const double a = M[(size_t)k * w + j], b = M[(size_t)p * w + j];
    M[(size_t)k * w + j] = b / pv;
    if (p != k) M[(size_t)p * w + j] = a;
  }
  __syncthreads();
  if (r < n) Ft[r] = r == k ? 0.0 : M[(size_t)r * w + k];
}

__global__ __launch_bounds__(kBlock) void k_gj_elim(int n, int k, double *__restrict__ work,
                                                    const double *__restrict__ F) {
  const int w = 2 * n;
  const int64_t q = blockIdx.x;  // grid t, row r
  const int64_t t = q / n;
  const double f = F[q];
  if (f == 0.0) return;  // uniform over the workgroup (the pivot row has f = 0)
  double *row = work + q * w;
  const double *prow = work + (t * n + k) * w;
  for (int j = k + threadIdx.x; j < w; j += blockDim.x) row[j] -= f * prow[j];
}

__global__ void k_gj_store(int n, int batch, const double *__restrict__ work,
                           double *__restrict__ inv) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (q >= nn * batch) return;
  const int64_t t = q / nn, e = q - t * nn;
  const int r = (int)(e / n), j = (int)(e - (int64_t)r * n);
  inv[q] = work[(t * n + r) * (2 * n) + n + j];
}

// d = inverse * v on every grid of the coarsest level: one wave per row (the
// lanes on consecutive columns, a fixed-order wave sum)
__global__ __launch_bounds__(kBlock) void k_coarse_dense_solve(
    GridGeom c, const double *__restrict__ inv, const double *__restrict__ v,
    double *__restrict__ d) {
  const int n = c.nx * c.ny * c.nz;
  const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (row >= (int64_t)n * c.batch) return;  // uniform over the wave
  const int64_t t = row / n;
  const double *a = inv + row * n;
  const double *vt = v + t * n;
  double s = 0.0;
  for (int j = lane; j < n; j += 64) s += a[j] * vt[j];
  s = wave_sum(s);
  if (lane == 0) d[row] = s;
}

}  // namespace

size_t coarse_tail_lds(const TailArgs &a) {
  size_t cells = 0;
  for (int l = 0; l < a.nlev; ++l) cells += (size_t)a.lv[l].nx * a.lv[l].ny * a.lv[l].nz;
  const size_t nc = (size_t)a.lv[a.nlev - 1].nx * a.lv[a.nlev - 1].ny * a.lv[a.nlev - 1].nz;
  return (cells * kTailDoublesPerCell + nc * nc) * sizeof(double);
}

hipError_t launch_coarse_inverse(const GridGeom &c, const double *dg, const double *cx,
                                 const double *cy, const double *cz, double *inv, double *work,
                                 uint32_t *flags, hipStream_t s) {
  const int n = c.nx * c.ny * c.nz;
  if (c.batch <= 0 || n <= 0) return hipSuccess;
  if (n > kCoarsestCellsMax) return hipErrorInvalidValue;
  if (n > kCoarsestCells) {
    if (!work) return hipErrorInvalidValue;
    const int64_t rows = (int64_t)n * c.batch;
    double *F = work + rows * 2 * n;  // column k of every grid (work holds 2 n^2 + n per grid)
    hipLaunchKernelGGL(k_gj_setup, dim3((unsigned)((rows + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, c, dg, cx, cy, cz, work);
    for (int k = 0; k < n; ++k) {
      hipLaunchKernelGGL(k_gj_pivot, dim3((unsigned)c.batch), dim3(kCoarsestCellsMax), 0, s, n, k,
                         work, F, flags);
      hipLaunchKernelGGL(k_gj_elim, dim3((unsigned)rows), dim3(kBlock), 0, s, n, k, work, F);
    }
    const int64_t all = rows * n;
    hipLaunchKernelGGL(k_gj_store, dim3((unsigned)((all + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                       s, n, c.batch, work, inv);
    return hipGetLastError();
  }
  const size_t lds = (size_t)n * (2 * n + 1) * sizeof(double);
  hipError_t e = hipFuncSetAttribute((const void *)k_coarse_inverse,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_coarse_inverse, dim3((unsigned)c.batch), dim3(kCoarsestCells), lds, s, c,
                     dg, cx, cy, cz, inv, flags);
  return hipGetLastError();
}

hipError_t launch_coarse_dense_solve(const GridGeom &c, const double *inv, const double *v,
                                     double *d, hipStream_t s) {
  const int n = c.nx * c.ny * c.nz;
  if (c.batch <= 0 || n <= 0) return hipSuccess;
  if (n > kCoarsestCellsMax) return hipErrorInvalidValue;
  const int64_t threads = (int64_t)n * c.batch * 64;
  hipLaunchKernelGGL(k_coarse_dense_solve, dim3((unsigned)((threads + kBlock - 1) / kBlock)),
                     dim3(kBlock), 0, s, c, inv, v, d);
  return hipGetLastError();
}

hipError_t launch_coarse_tail(const TailArgs &a, hipStream_t s) {
  if (a.batch <= 0) return hipSuccess;
  if (a.nlev < 1 || a.nlev > kTailMaxLevels || a.gamma < 1 || a.gamma > 15 || !a.inv)
    return hipErrorInvalidValue;
  if ((int64_t)a.lv[a.nlev - 1].nx * a.lv[a.nlev - 1].ny * a.lv[a.nlev - 1].nz > kCoarsestCells)
    return hipErrorInvalidValue;
  for (int l = 0; l < a.nlev; ++l)
    if ((int64_t)a.lv[l].nx * a.lv[l].ny * a.lv[l].nz > kTailThreads) return hipErrorInvalidValue;
  const size_t lds = coarse_tail_lds(a);
  hipError_t e = hipFuncSetAttribute((const void *)k_coarse_tail,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_coarse_tail, dim3((unsigned)a.batch), dim3(kTailThreads), lds, s, a);
  return hipGetLastError();
}

GridGeom coarse_geom(const GridGeom &f) {
  GridGeom c{};
  c.nx = f.nx > 1 ? (f.nx + 1) / 2 : 1;
  c.ny = f.ny > 1 ? (f.ny + 1) / 2 : 1;
  c.nz = f.nz > 1 ? (f.nz + 1) / 2 : 1;
  c.batch = f.batch;
  geom_finish(c);
  return c;
}

hipError_t launch_coarse_coef(const GridGeom &f, const GridCoef<double> &k, bool varc,
                              const GridGeom &c, double *dg, double *cx, double *cy, double *cz,
                              hipStream_t s) {
  if (c.N <= 0) return hipSuccess;
  if (!geom_ok(f) || !geom_ok(c)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_coarse_coef, blocks_for(c.N), dim3(kBlock), 0, s, f, k, varc ? 1 : 0, c, dg,
                     cx, cy, cz);
  return hipGetLastError();
}

hipError_t launch_coarse_restrict(const GridGeom &f, const GridGeom &c, const double *r, double *rc,
                                  hipStream_t s) {
  if (c.N <= 0) return hipSuccess;
  if (!geom_ok(f) || !geom_ok(c)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_coarse_restrict, blocks_for(c.N), dim3(kBlock), 0, s, f, c, r, rc);
  return hipGetLastError();
}

hipError_t launch_coarse_prolong(const GridGeom &f, const GridGeom &c, const double *dc,
                                 const double *dc2, double scale, double *d, hipStream_t s) {
  if (f.N <= 0) return hipSuccess;
  if (!geom_ok(f) || !geom_ok(c)) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_coarse_prolong, blocks_for(f.N), dim3(kBlock), 0, s, f, c, dc, dc2, scale,
                     d);
  return hipGetLastError();
}

static bool work_rhs_ok(const GridGeom &g, const WorkRhs &w) {
  return !w.p || w.hx == 0 || (w.hx == g.fh.d && w.nc == w.hx * (g.N / g.nx));
}

hipError_t launch_coarse_residual_restrict(const GridGeom &f, const GridCoef<double> &k, bool varc,
                                           const GridGeom &c, const double *v, const double *d,
                                           double *rc, const WorkRhs &w, hipStream_t s) {
  if (c.N <= 0) return hipSuccess;
  if (!geom_ok(f) || !geom_ok(c) || !work_rhs_ok(c, w)) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((8 * (int64_t)c.N + kBlock - 1) / kBlock));
  if (varc)
    hipLaunchKernelGGL(k_coarse_residual_restrict<true>, grid, dim3(kBlock), 0, s, f, k, c, v, d,
                       rc, w);
  else
    hipLaunchKernelGGL(k_coarse_residual_restrict<false>, grid, dim3(kBlock), 0, s, f, k, c, v, d,
                       rc, w);
  return hipGetLastError();
}

hipError_t launch_coarse_copy_residual(const GridGeom &g, const GridCoef<double> &k, bool varc,
                                       const double *d, double *e, double *v, const WorkRhs &w,
                                       hipStream_t s) {
  if (g.N <= 0) return hipSuccess;
  if (!geom_ok(g) || !work_rhs_ok(g, w)) return hipErrorInvalidValue;
  if (varc)
    hipLaunchKernelGGL(k_coarse_copy_residual<true>, blocks_for(g.N), dim3(kBlock), 0, s, g, k, d,
                       e, v, w);
  else
    hipLaunchKernelGGL(k_coarse_copy_residual<false>, blocks_for(g.N), dim3(kBlock), 0, s, g, k, d,
                       e, v, w);
  return hipGetLastError();
}

hipError_t launch_gcr_step(const GridGeom &g, const GridCoef<double> &k, bool varc, int nseg,
                           int segb, const double *c, double *r, double *w, double *pc,
                           double *pw, double *part, double *pp, double2 *ab, bool first,
                           double *x, const WorkRhs &wr, double *sumpart, hipStream_t s) {
  if (g.N <= 0) return hipSuccess;
  if (!geom_ok(g) || nseg != g.batch || segb < 1 || !work_rhs_ok(g, wr) || !sumpart)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)(nseg * segb));
  if (varc)
    hipLaunchKernelGGL(k_gcr_dots<true>, grid, dim3(kBlock), 0, s, g, k, c, r, pw, w, part, nseg,
                       first ? 1 : 0);
  else
    hipLaunchKernelGGL(k_gcr_dots<false>, grid, dim3(kBlock), 0, s, g, k, c, r, pw, w, part, nseg,
                       first ? 1 : 0);
  hipLaunchKernelGGL(k_gcr_coef, dim3((unsigned)nseg), dim3(kBlock), 0, s, part, segb,
                     first ? 1 : 0, pp, ab);
  hipLaunchKernelGGL(k_gcr_update, grid, dim3(kBlock), 0, s, g, c, w, ab, first ? 1 : 0, pc, pw,
                     x, r, wr, sumpart, nseg);
  return hipGetLastError();
}

hipError_t launch_axpy(int n, const double *d, double *x, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, blocks_for(n), dim3(kBlock), 0, s, n, d, x);
  return hipGetLastError();
}

}  // namespace gabp
