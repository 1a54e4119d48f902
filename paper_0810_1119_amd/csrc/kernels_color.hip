// Graph colouring and renumbering for the coloured schedule of general sparse
// plans (gfx950).
//
// Colouring: Jones-Plassmann rounds with first-fit colours.  Every node has a
// fixed pseudo-random priority (a bijective mix of its index, ties broken by
// the index); in a round, each uncoloured node whose priority beats every
// uncoloured neighbour takes the smallest colour none of its coloured
// neighbours has.  Two neighbours are never both local maxima, so no node
// reads a colour written in the same round: the result is deterministic.
// Colours are limited to kMaxColors (a node with more coloured neighbours of
// distinct colours is reported).
//
// Renumbering: nodes sorted by colour (stable), so each colour class is a
// contiguous range of rows; the matrix is rebuilt in that order with every
// row's columns sorted.
#include <hipcub/hipcub.hpp>

#include "device_common.h"

namespace gabp {

namespace {

__device__ __forceinline__ uint32_t priority(uint32_t i) {
  // MurmurHash3's 32-bit finaliser: a bijection, so priorities are distinct
  i ^= i >> 16;
  i *= 0x85ebca6bu;
  i ^= i >> 13;
  i *= 0xc2b2ae35u;
  i ^= i >> 16;
  return i;
}

__global__ __launch_bounds__(kBlock) void k_jp_round(int n, const int64_t *__restrict__ rp,
                                                     const int32_t *__restrict__ col,
                                                     int32_t *__restrict__ color,
                                                     uint32_t *__restrict__ left,
                                                     uint32_t *__restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  bool waiting = false;
  if (i < n && color[i] < 0) {
    const uint32_t pi = priority((uint32_t)i);
    uint64_t used[kMaxColors / 64] = {};
    bool top = true;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const int j = col[e];
      if (j == i) continue;
      const int cj = color[j];
      if (cj < 0) {
        const uint32_t pj = priority((uint32_t)j);
        if (pj > pi || (pj == pi && j > i)) {
          top = false;
          break;
        }
      } else {
        used[cj >> 6] |= 1ull << (cj & 63);
      }
    }
    if (top) {
      int c = -1;
#pragma unroll
      for (int w = 0; w < kMaxColors / 64; ++w)
        if (c < 0 && ~used[w] != 0ull) c = w * 64 + __builtin_ctzll(~used[w]);
      if (c < 0) {
        atomicOr(flags, FLAG_UNSUPPORTED);
        c = kMaxColors - 1;  // the plan is refused; any value ends the loop
      }
      color[i] = c;
    } else {
      waiting = true;
    }
  }
  // nodes still uncoloured: one atomic per wavefront
  const unsigned long long b = __ballot(waiting);
  if ((threadIdx.x & 63) == 0 && b) atomicAdd(left, (uint32_t)__popcll(b));
}

__global__ void k_color_max(int n, const int32_t *__restrict__ color, int32_t *__restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  int c = i < n ? color[i] : -1;
  for (int o = 32; o > 0; o >>= 1) c = max(c, __shfl_xor(c, o, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, c);
}

__global__ void k_iota(int n, int32_t *__restrict__ v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = i;
}

// old2new, the first row of each colour (classes sorted by colour)
__global__ void k_perm_finish(int n, const uint32_t *__restrict__ keys,
                              const int32_t *__restrict__ new2old, int32_t *__restrict__ old2new,
                              int32_t *__restrict__ first) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  old2new[new2old[r]] = r;
  if (r == 0 || keys[r] != keys[r - 1]) first[keys[r]] = r;
}

__global__ void k_perm_rowlen(int n, const int64_t *__restrict__ rp,
                              const int32_t *__restrict__ new2old, int64_t *__restrict__ len) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < n) len[r] = rp[new2old[r] + 1] - rp[new2old[r]];
}

__global__ void k_perm_fill(int n, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                            const int32_t *__restrict__ new2old, const int32_t *__restrict__ old2new,
                            const int64_t *__restrict__ rp2, int32_t *__restrict__ col2,
                            int32_t *__restrict__ slot2) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  const int o = new2old[r];
  int64_t d = rp2[r];
  for (int64_t e = rp[o]; e < rp[o + 1]; ++e, ++d) {
    col2[d] = old2new[col[e]];
    slot2[d] = (int32_t)e;  // the caller's slot (nnz < 2^31, checked by the host)
  }
}

// per slot: v2[d] = v[slot[d]] (gather) or v[slot[d]] = v2[d] (scatter), FP64
__global__ void k_slot_move(int64_t nnz, const int32_t *__restrict__ slot,
                            const double *__restrict__ in, double *__restrict__ out, bool to_new) {
  const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= nnz) return;
  if (to_new) out[d] = in[slot[d]];
  else out[slot[d]] = in[d];
}

// v2[new] = v[old] (gather) or v[old] = v2[new] (scatter), FP64
__global__ void k_permute(int n, const int32_t *__restrict__ new2old, const double *__restrict__ in,
                          double *__restrict__ out, bool to_new) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= n) return;
  if (to_new) out[r] = in[new2old[r]];
  else out[new2old[r]] = in[r];
}

unsigned nblk(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_jp_round(int n, const int64_t *rp, const int32_t *col, int32_t *color,
                           uint32_t *left, uint32_t *flags, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_jp_round, dim3(nblk(n)), dim3(kBlock), 0, s, n, rp, col, color, left, flags);
  return hipGetLastError();
}

hipError_t launch_color_max(int n, const int32_t *color, int32_t *out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_color_max, dim3(nblk(n)), dim3(kBlock), 0, s, n, color, out);
  return hipGetLastError();
}

hipError_t launch_iota(int n, int32_t *v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_iota, dim3(nblk(n)), dim3(kBlock), 0, s, n, v);
  return hipGetLastError();
}

hipError_t launch_color_sort(int n, int ncolors, const int32_t *color, uint32_t *keys_out,
                             const int32_t *idx, int32_t *new2old, void *tmp, size_t *bytes,
                             hipStream_t s) {
  int bits = 1;
  while ((1 << bits) < ncolors) ++bits;
  return hipcub::DeviceRadixSort::SortPairs(tmp, *bytes, (const uint32_t *)color, keys_out, idx,
                                            new2old, n, 0, bits, s);
}

hipError_t launch_perm_finish(int n, const uint32_t *keys, const int32_t *new2old,
                              int32_t *old2new, int32_t *first, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_perm_finish, dim3(nblk(n)), dim3(kBlock), 0, s, n, keys, new2old, old2new,
                     first);
  return hipGetLastError();
}

hipError_t launch_perm_rowlen(int n, const int64_t *rp, const int32_t *new2old, int64_t *len,
                              hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_perm_rowlen, dim3(nblk(n)), dim3(kBlock), 0, s, n, rp, new2old, len);
  return hipGetLastError();
}

hipError_t launch_perm_fill(int n, const int64_t *rp, const int32_t *col, const int32_t *new2old,
                            const int32_t *old2new, const int64_t *rp2, int32_t *col2,
                            int32_t *slot2, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_perm_fill, dim3(nblk(n)), dim3(kBlock), 0, s, n, rp, col, new2old, old2new,
                     rp2, col2, slot2);
  return hipGetLastError();
}

hipError_t launch_slot_move(int64_t nnz, const int32_t *slot, const double *in, double *out,
                            bool to_new, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_slot_move, dim3(nblk(nnz)), dim3(kBlock), 0, s, nnz, slot, in, out, to_new);
  return hipGetLastError();
}

// every row's entries sorted by column (tmp == NULL: only *bytes is set)
hipError_t launch_rows_sort(int n, int64_t nnz, const int64_t *rp, const int32_t *col_in,
                            int32_t *col_out, const int32_t *val_in, int32_t *val_out, void *tmp,
                            size_t *bytes, hipStream_t s) {
  return hipcub::DeviceSegmentedRadixSort::SortPairs(tmp, *bytes, col_in, col_out, val_in, val_out,
                                                     (int)nnz, n, rp, rp + 1, 0, 32, s);
}

hipError_t launch_permute(int n, const int32_t *new2old, const double *in, double *out,
                          bool to_new, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_permute, dim3(nblk(n)), dim3(kBlock), 0, s, n, new2old, in, out, to_new);
  return hipGetLastError();
}

}  // namespace gabp
