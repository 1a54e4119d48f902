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
#include "gabp_internal.h"

namespace gabp {
namespace {

__device__ __forceinline__ int half_up(int n) { return n > 1 ? (n + 1) / 2 : 1; }

__global__ void k_coarse_coef(GridGeom f, GridCoef<double> k, int varc, GridGeom c,
                              double *__restrict__ dg, double *__restrict__ cx,
                              double *__restrict__ cy, double *__restrict__ cz) {
  const int I = blockIdx.x * blockDim.x + threadIdx.x;
  if (I >= c.N) return;
  const int nc = c.nx * c.ny * c.nz, nf = f.nx * f.ny * f.nz;
  const int t = I / nc, j = I - t * nc;
  const int X = j % c.nx, Y = (j / c.nx) % c.ny, Z = j / (c.nx * c.ny);
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
  const int nc = c.nx * c.ny * c.nz, nf = f.nx * f.ny * f.nz;
  const int t = I / nc, j = I - t * nc;
  const int X = j % c.nx, Y = (j / c.nx) % c.ny, Z = j / (c.nx * c.ny);
  const int sx = f.nx > 1 ? 2 : 1, sy = f.ny > 1 ? 2 : 1, sz = f.nz > 1 ? 2 : 1;
  const int x0 = X * sx, y0 = Y * sy, z0 = Z * sz;
  const int x1 = min(x0 + sx, f.nx), y1 = min(y0 + sy, f.ny), z1 = min(z0 + sz, f.nz);
  double s = 0.0;
  for (int z = z0; z < z1; ++z)
    for (int y = y0; y < y1; ++y)
      for (int x = x0; x < x1; ++x) s += r[t * nf + x + f.nx * (y + f.ny * z)];
  rc[I] = s;
}

// d[i] += scale * dc[block of i]
__global__ void k_coarse_prolong(GridGeom f, GridGeom c, const double *__restrict__ dc,
                                 double scale, double *__restrict__ d) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= f.N) return;
  const int nf = f.nx * f.ny * f.nz, nc = c.nx * c.ny * c.nz;
  const int t = i / nf, j = i - t * nf;
  const int x = j % f.nx, y = (j / f.nx) % f.ny, z = j / (f.nx * f.ny);
  const int sx = f.nx > 1 ? 2 : 1, sy = f.ny > 1 ? 2 : 1, sz = f.nz > 1 ? 2 : 1;
  d[i] += scale * dc[t * nc + x / sx + c.nx * (y / sy + c.ny * (z / sz))];
}

__global__ void k_axpy(int n, const double *__restrict__ d, double *__restrict__ x) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += d[i];
}

dim3 blocks_for(int n) { return dim3((unsigned)((n + kBlock - 1) / kBlock)); }

}  // namespace

GridGeom coarse_geom(const GridGeom &f) {
  GridGeom c{};
  c.nx = f.nx > 1 ? (f.nx + 1) / 2 : 1;
  c.ny = f.ny > 1 ? (f.ny + 1) / 2 : 1;
  c.nz = f.nz > 1 ? (f.nz + 1) / 2 : 1;
  c.batch = f.batch;
  c.N = c.nx * c.ny * c.nz * c.batch;
  return c;
}

hipError_t launch_coarse_coef(const GridGeom &f, const GridCoef<double> &k, bool varc,
                              const GridGeom &c, double *dg, double *cx, double *cy, double *cz,
                              hipStream_t s) {
  if (c.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarse_coef, blocks_for(c.N), dim3(kBlock), 0, s, f, k, varc ? 1 : 0, c, dg,
                     cx, cy, cz);
  return hipGetLastError();
}

hipError_t launch_coarse_restrict(const GridGeom &f, const GridGeom &c, const double *r, double *rc,
                                  hipStream_t s) {
  if (c.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarse_restrict, blocks_for(c.N), dim3(kBlock), 0, s, f, c, r, rc);
  return hipGetLastError();
}

hipError_t launch_coarse_prolong(const GridGeom &f, const GridGeom &c, const double *dc,
                                 double scale, double *d, hipStream_t s) {
  if (f.N <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_coarse_prolong, blocks_for(f.N), dim3(kBlock), 0, s, f, c, dc, scale, d);
  return hipGetLastError();
}

hipError_t launch_axpy(int n, const double *d, double *x, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_axpy, blocks_for(n), dim3(kBlock), 0, s, n, d, x);
  return hipGetLastError();
}

}  // namespace gabp
