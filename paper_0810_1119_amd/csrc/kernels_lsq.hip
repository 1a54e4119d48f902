// Section VII on the device: assembly of the symmetric bipartite system
//     R = [[I_k, S^T], [S, -psi I_m]]
// of any sparse m x k matrix S, the embedding of its right-hand side [0; y],
// and the FP64 residual of the regularised normal equations.
//
// Node order of R: the k unknowns x first, then the m auxiliary z.  Row i < k
// holds the diagonal 1 followed by column i of S at columns k + j (j
// increasing); row k + j holds row j of S followed by the diagonal -psi.  S^T
// is formed by a stable radix sort of the nonzeros by column, so the rows of
// R come out sorted and the assembly is deterministic.
#include <hipcub/hipcub.hpp>

#include "device_common.h"

namespace gabp {

namespace {

// Row j of S: bounds, strictly increasing columns in [0, k), finite values;
// the row length of R's row k + j and the column counts (integer atomics).
__global__ void k_lsq_rows(int m, int k, int64_t nnz, const int64_t *__restrict__ rp,
                           const int32_t *__restrict__ col, const double *__restrict__ val,
                           uint32_t *__restrict__ colcnt, int64_t *__restrict__ rowlen,
                           int32_t *__restrict__ rowof, int32_t *__restrict__ idx,
                           uint32_t *__restrict__ flags) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t b = rp[j], e = rp[j + 1];
  if (b < 0 || e < b || e > nnz) {
    atomicOr(flags, FLAG_ARG);
    rowlen[k + j] = 1;
    return;
  }
  uint32_t f = 0;
  int prev = -1;
  for (int64_t t = b; t < e; ++t) {
    const int c = col[t];
    if (c < 0 || c >= k || c <= prev) {
      f |= FLAG_ARG;
      break;
    }
    prev = c;
    if (!isfinite(val[t])) f |= FLAG_ARG;
    atomicAdd(&colcnt[c], 1u);
    rowof[t] = j;
    idx[t] = (int32_t)t;
  }
  if (f) atomicOr(flags, f);
  rowlen[k + j] = (e - b) + 1;
}

__global__ void k_lsq_collen(int k, const uint32_t *__restrict__ colcnt,
                             int64_t *__restrict__ rowlen) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < k) rowlen[i] = 1 + (int64_t)colcnt[i];
}

// rows k + j of R: row j of S, then the diagonal -psi
__global__ void k_lsq_fill_z(int m, int k, double psi, const int64_t *__restrict__ rp,
                             const int32_t *__restrict__ col, const double *__restrict__ val,
                             const int64_t *__restrict__ Arp, int32_t *__restrict__ Acol,
                             double *__restrict__ Aval) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  const int64_t b = rp[j], e = rp[j + 1];
  int64_t o = Arp[k + j];
  for (int64_t t = b; t < e; ++t, ++o) {
    Acol[o] = col[t];
    Aval[o] = val[t];
  }
  Acol[o] = k + j;
  Aval[o] = -psi;
}

// rows i < k of R: the diagonal 1, then column i of S (sorted nonzeros
// perm[Arp[i] - i ..], in increasing row order)
__global__ void k_lsq_fill_x(int k, const int64_t *__restrict__ Arp,
                             const int32_t *__restrict__ perm, const int32_t *__restrict__ rowof,
                             const double *__restrict__ val, int32_t *__restrict__ Acol,
                             double *__restrict__ Aval) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= k) return;
  const int64_t b = Arp[i], e = Arp[i + 1];
  const int64_t first = b - i;  // sorted position of the column's first nonzero
  Acol[b] = i;
  Aval[b] = 1.0;
  for (int64_t t = 1; t < e - b; ++t) {
    const int32_t src = perm[first + t - 1];
    Acol[b + t] = k + rowof[src];
    Aval[b + t] = val[src];
  }
}

__global__ void k_lsq_embed(int k, int m, const double *__restrict__ y, double *__restrict__ bt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < k) bt[t] = 0.0;
  else if (t < k + m) bt[t] = y[t - k];
}

// u_j = y_j - (S x)_j from row k + j of R (its last entry is the diagonal)
__global__ void k_lsq_u(int m, int k, const int64_t *__restrict__ Arp,
                        const int32_t *__restrict__ Acol, const double *__restrict__ Aval,
                        const double *__restrict__ y, const double *__restrict__ x,
                        double *__restrict__ u) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  double acc = y[j];
  if (x != nullptr)
    for (int64_t t = Arp[k + j]; t < Arp[k + j + 1] - 1; ++t) acc -= Aval[t] * x[Acol[t]];
  u[j] = acc;
}

// r_i = (S^T u)_i - psi x_i from row i of R (its first entry is the
// diagonal); block partial sums of r_i^2
__global__ __launch_bounds__(kBlock) void k_lsq_normal(int k, double psi,
                                                       const int64_t *__restrict__ Arp,
                                                       const int32_t *__restrict__ Acol,
                                                       const double *__restrict__ Aval,
                                                       const double *__restrict__ u,
                                                       const double *__restrict__ x,
                                                       double *__restrict__ r,
                                                       double *__restrict__ part) {
  __shared__ double sh[kBlock / 64];
  double sq = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < k; i += gridDim.x * kBlock) {
    double acc = 0.0;
    for (int64_t t = Arp[i] + 1; t < Arp[i + 1]; ++t) acc += Aval[t] * u[Acol[t] - k];
    if (x != nullptr) acc -= psi * x[i];
    if (r != nullptr) r[i] = acc;
    sq += acc * acc;
  }
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x / 64] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0];
    for (int w = 1; w < kBlock / 64; ++w) t += sh[w];
    part[blockIdx.x] = t;
  }
}

unsigned blocks(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_lsq_rows(int m, int k, int64_t nnz, const int64_t *rp, const int32_t *col,
                           const double *val, uint32_t *colcnt, int64_t *rowlen, int32_t *rowof,
                           int32_t *idx, uint32_t *flags, hipStream_t s) {
  if (m > 0)
    hipLaunchKernelGGL(k_lsq_rows, dim3(blocks(m)), dim3(kBlock), 0, s, m, k, nnz, rp, col, val,
                       colcnt, rowlen, rowof, idx, flags);
  if (k > 0)
    hipLaunchKernelGGL(k_lsq_collen, dim3(blocks(k)), dim3(kBlock), 0, s, k, colcnt, rowlen);
  return hipGetLastError();
}

// stable sort of the nonzero indices by column: perm lists column 0's
// nonzeros first, each column in increasing nonzero (= row) order
// (tmp == NULL: only *tmp_bytes is set).  Columns are validated nonnegative,
// so they sort as unsigned keys over their low bits.
hipError_t launch_lsq_sort(int k, int64_t nnz, const int32_t *col, uint32_t *keys_out,
                           const int32_t *idx, int32_t *perm, void *tmp, size_t *tmp_bytes,
                           hipStream_t s) {
  int bits = 1;
  while (bits < 31 && (1 << bits) < k) ++bits;
  return hipcub::DeviceRadixSort::SortPairs(tmp, *tmp_bytes, (const uint32_t *)col, keys_out, idx,
                                            perm, (int)nnz, 0, bits, s);
}

hipError_t launch_lsq_fill(int m, int k, double psi, const int64_t *rp, const int32_t *col,
                           const double *val, const int64_t *Arp, const int32_t *perm,
                           const int32_t *rowof, int32_t *Acol, double *Aval, hipStream_t s) {
  if (m > 0)
    hipLaunchKernelGGL(k_lsq_fill_z, dim3(blocks(m)), dim3(kBlock), 0, s, m, k, psi, rp, col, val,
                       Arp, Acol, Aval);
  if (k > 0)
    hipLaunchKernelGGL(k_lsq_fill_x, dim3(blocks(k)), dim3(kBlock), 0, s, k, Arp, perm, rowof, val,
                       Acol, Aval);
  return hipGetLastError();
}

hipError_t launch_lsq_embed(int k, int m, const double *y, double *bt, hipStream_t s) {
  if (k + m > 0)
    hipLaunchKernelGGL(k_lsq_embed, dim3(blocks((int64_t)k + m)), dim3(kBlock), 0, s, k, m, y, bt);
  return hipGetLastError();
}

int lsq_normal_blocks(int k) {
  const int64_t b = blocks(k);
  return (int)(b < 1 ? 1 : (b > kMaxSweepBlocks ? kMaxSweepBlocks : b));
}

hipError_t launch_lsq_normal(int m, int k, double psi, const int64_t *Arp, const int32_t *Acol,
                             const double *Aval, const double *y, const double *x, double *u,
                             double *r, double *part, hipStream_t s) {
  if (m > 0)
    hipLaunchKernelGGL(k_lsq_u, dim3(blocks(m)), dim3(kBlock), 0, s, m, k, Arp, Acol, Aval, y, x, u);
  hipLaunchKernelGGL(k_lsq_normal, dim3(lsq_normal_blocks(k)), dim3(kBlock), 0, s, k, psi, Arp,
                     Acol, Aval, u, x, r, part);
  return hipGetLastError();
}

}  // namespace gabp
