// GaBP on a general sparse symmetric matrix (CSR), gfx950.
//
// Edge layout: the off-diagonal entries of row i occupy slots
// oprt[i] .. oprt[i+1]-1 in column order; slot e = (i -> j) holds the message
// node i sends to node j as a (P, h) pair, h = P * mu, and rev[e] is the slot
// of (j -> i).  A sweep is Algorithm 2 of the paper (section V) in the
// information parametrisation:
//   S_i = A_ii + sum_k P_ki,   H_i = b_i + sum_k h_ki          (node aggregate)
//   P_ij = -A_ij^2 / (S_i - P_ji)                              (eq. prec_message)
//   h_ij = -A_ij (H_i - h_ji) / (S_i - P_ji)                   (eq. mean_message times P_ij)
// because P_ii mu_ii = b_i (eq. PhiGauss) and mu_ij = h_ij / P_ij; the
// marginal mean is x_i = H_i / S_i (Algorithm 1 step 4).  In-messages are
// gathered through rev[] (8 or 16 bytes each); out-messages are written
// coalesced in the row's own slots.  Two buffers give the synchronous
// (flooding) schedule of section III-C.
#include "device_common.h"

namespace gabp {

// ---------------------------------------------------------------------------
// plan build
// ---------------------------------------------------------------------------
__global__ void k_plan_rows(int n, int64_t nnz, const int64_t *__restrict__ rp,
                            const int32_t *__restrict__ col, const double *__restrict__ val,
                            int64_t *__restrict__ deg, int64_t *__restrict__ diagpos,
                            uint32_t *__restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = rp[i], e = rp[i + 1];
  if (b < 0 || e < b || e > nnz) {
    if (deg) {
      deg[i] = 0;
      diagpos[i] = -1;
    }
    atomicOr(flags, FLAG_ARG);
    return;
  }
  uint32_t f = 0;
  int64_t dp = -1, d = 0;
  int32_t prev = -1;
  for (int64_t k = b; k < e; ++k) {
    const int32_t j = col[k];
    if (j < 0 || j >= n || j <= prev) f |= FLAG_ARG;
    prev = j;
    if (!isfinite(val[k])) f |= FLAG_ARG;
    if (j == i) dp = k;
    else ++d;
  }
  if (dp < 0 || val[dp] == 0.0) f |= FLAG_ZERO_DIAG;
  if (deg) {  // NULL: validation only
    deg[i] = d;
    diagpos[i] = dp;
  }
  if (f) atomicOr(flags, f);
}

hipError_t launch_plan_rows(int n, int64_t nnz, const int64_t *rp, const int32_t *col,
                            const double *val, int64_t *deg, int64_t *diagpos, uint32_t *flags,
                            hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan_rows, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, nnz,
                     rp, col, val, deg, diagpos, flags);
  return hipGetLastError();
}

// Exclusive scan, 1024 items per block (256 threads x 4), block totals scanned
// recursively.
constexpr int kScanItems = 4;
constexpr int kScanTile = kBlock * kScanItems;

__global__ void k_scan_tile(const int64_t *__restrict__ in, int64_t *__restrict__ out, int64_t n,
                            int64_t *__restrict__ tile_sum) {
  __shared__ int64_t sh[kBlock];
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
  int64_t v[kScanItems];
  int64_t run = 0;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    v[k] = (idx < n) ? in[idx] : 0;
    run += v[k];
  }
  sh[threadIdx.x] = run;
  __syncthreads();
  // Hillis-Steele inclusive scan of the per-thread sums
  for (int off = 1; off < kBlock; off <<= 1) {
    const int64_t add = (threadIdx.x >= (unsigned)off) ? sh[threadIdx.x - off] : 0;
    __syncthreads();
    sh[threadIdx.x] += add;
    __syncthreads();
  }
  int64_t pre = sh[threadIdx.x] - run;
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t idx = base + k;
    if (idx < n) out[idx] = pre;
    pre += v[k];
  }
  if (threadIdx.x == kBlock - 1) tile_sum[blockIdx.x] = sh[kBlock - 1];
}

__global__ void k_scan_add(int64_t *__restrict__ out, int64_t n, const int64_t *__restrict__ off) {
  const int64_t idx = (int64_t)blockIdx.x * kScanTile + threadIdx.x;
  const int64_t add = off[blockIdx.x];
#pragma unroll
  for (int k = 0; k < kScanItems; ++k) {
    const int64_t j = idx + (int64_t)k * kBlock;
    if (j < n) out[j] += add;
  }
}

// Scratch of launch_scan: the padded copy of the input (n + 1 values), then
// per recursion level the tile sums and their scan (2 * tiles + 1 values).
size_t scan_tmp_elems(int64_t n) {
  size_t total = (size_t)(n + 1);
  int64_t m = n + 1;
  while (true) {
    const int64_t tiles = (m + kScanTile - 1) / kScanTile;
    total += 2 * (size_t)tiles + 1;
    if (tiles <= 1) break;
    m = tiles;
  }
  return total + 4;
}

// out[0..m) = exclusive scan of in[0..m); tmp holds the tile sums, their scan
// and the scratch of the deeper levels.
static hipError_t scan_rec(const int64_t *in, int64_t *out, int64_t m, int64_t *tmp,
                           hipStream_t s) {
  const int64_t tiles = (m + kScanTile - 1) / kScanTile;
  int64_t *tsum = tmp;
  int64_t *tscan = tmp + tiles;
  hipLaunchKernelGGL(k_scan_tile, dim3((unsigned)tiles), dim3(kBlock), 0, s, in, out, m, tsum);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess || tiles == 1) return err;
  err = scan_rec(tsum, tscan, tiles, tmp + 2 * tiles + 1, s);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)tiles), dim3(kBlock), 0, s, out, m, tscan);
  return hipGetLastError();
}

__global__ void k_copy_pad(const int64_t *__restrict__ in, int64_t *__restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = in[i];
  else if (i == n) out[i] = 0;
}

hipError_t launch_scan(const int64_t *in, int64_t *out, int64_t n, int64_t *tmp, hipStream_t s) {
  // scan n+1 values (the last one zero) so that out[n] is the total; the
  // padded input is staged in `out` itself, then scanned out of place into tmp
  // and copied back.
  int64_t *pad = tmp;
  int64_t *work = tmp + (n + 1);
  hipLaunchKernelGGL(k_copy_pad, dim3((unsigned)((n + 1 + kBlock - 1) / kBlock)), dim3(kBlock),
                     0, s, in, pad, n);
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  return scan_rec(pad, out, n + 1, work, s);
}

// Column ranges of the pair layout: L[i] = off-diagonal entries of row i with
// column < split, L[n + i] = the others; far += the entries joining nodes n / 4
// or more apart in index (one atomic per wavefront).
__global__ __launch_bounds__(kBlock) void k_plan_split(int n, const int64_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col,
                                                       const int64_t *__restrict__ diagpos,
                                                       int split, int64_t *__restrict__ L,
                                                       unsigned long long *__restrict__ far) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  double fr = 0.0;
  if (i < n) {
    const int64_t dp = diagpos[i];
    const int64_t q = n / 4;
    int64_t c0 = 0, d = 0;
    for (int64_t k = rp[i]; k < rp[i + 1]; ++k) {
      if (k == dp) continue;
      const int32_t j = col[k];
      ++d;
      c0 += j < split;
      const int64_t gap = j > i ? (int64_t)j - i : (int64_t)i - j;
      fr += gap >= q ? 1.0 : 0.0;
    }
    L[i] = c0;
    L[n + i] = d - c0;
  }
  fr = wave_sum(fr);
  if ((threadIdx.x & 63) == 0 && fr > 0.0) atomicAdd(far, (unsigned long long)fr);
}

hipError_t launch_plan_split(int n, const int64_t *rp, const int32_t *col, const int64_t *diagpos,
                             int split, int64_t *L, unsigned long long *far, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_plan_split, dim3((n + kBlock - 1) / kBlock), dim3(kBlock), 0, s, n, rp, col,
                     diagpos, split, L, far);
  return hipGetLastError();
}

// Slot of the off-diagonal entry of rank `rank` in row i.  One column range:
// vo[i] + rank.  Two: row i's entries below the split (its first
// vo[i + 1] - vo[i]) at vo[i] + rank, the others at vo[n + i] + the rest.
__device__ __forceinline__ int64_t pair_slot(const int64_t *vo, int n, int nb, int i,
                                             int64_t rank) {
  if (nb == 2) {
    const int64_t c0 = vo[i + 1] - vo[i];
    if (rank >= c0) return vo[n + i] + (rank - c0);
  }
  return vo[i] + rank;
}

template <typename T>
__global__ void k_plan_edges(int n, int nb, const int64_t *__restrict__ rp,
                             const int32_t *__restrict__ col, const double *__restrict__ val,
                             const int64_t *__restrict__ diagpos, const int64_t *__restrict__ vo,
                             int32_t *__restrict__ ocol, int32_t *__restrict__ rev,
                             T *__restrict__ acoef, T *__restrict__ diag,
                             uint32_t *__restrict__ flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = rp[i], e = rp[i + 1], dp = diagpos[i];
  diag[i] = (T)val[dp];
  uint32_t f = 0;
  for (int64_t k = b; k < e; ++k) {
    if (k == dp) continue;
    const int32_t j = col[k];
    const int64_t o = pair_slot(vo, n, nb, i, (k - b) - (k > dp ? 1 : 0));
    // binary search for column i in row j (columns sorted)
    int64_t lo = rp[j], hi = rp[j + 1] - 1, found = -1;
    while (lo <= hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      const int32_t c = col[mid];
      if (c == i) { found = mid; break; }
      if (c < i) lo = mid + 1;
      else hi = mid - 1;
    }
    int32_t r = 0;
    if (found < 0 || val[found] != val[k]) {
      f |= FLAG_ASYM;
    } else {
      r = (int32_t)pair_slot(vo, n, nb, j, (found - rp[j]) - (found > diagpos[j] ? 1 : 0));
    }
    rev[o] = r;
    ocol[o] = j;
    acoef[o] = (T)val[k];
  }
  if (f) atomicOr(flags, f);
}

__global__ void k_narrow_offsets(int64_t m, const int64_t *__restrict__ in, int32_t *__restrict__ out) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v < m) out[v] = (int32_t)in[v];
}

hipError_t launch_plan_edges(bool fp32, int n, int nb, const int64_t *rp, const int32_t *col,
                             const double *val, const int64_t *diagpos, const int64_t *vo,
                             int32_t *oprt, int32_t *ocol, int32_t *rev, void *acoef, void *diag,
                             uint32_t *flags, hipStream_t s) {
  const int64_t m = (int64_t)nb * n + 1;
  hipLaunchKernelGGL(k_narrow_offsets, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                     s, m, vo, oprt);
  if (n <= 0) return hipGetLastError();
  const dim3 grid((n + kBlock - 1) / kBlock);
  if (fp32)
    hipLaunchKernelGGL(k_plan_edges<float>, grid, dim3(kBlock), 0, s, n, nb, rp, col, val, diagpos,
                       vo, ocol, rev, (float *)acoef, (float *)diag, flags);
  else
    hipLaunchKernelGGL(k_plan_edges<double>, grid, dim3(kBlock), 0, s, n, nb, rp, col, val, diagpos,
                       vo, ocol, rev, (double *)acoef, (double *)diag, flags);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the sweep
// ---------------------------------------------------------------------------
// G lanes cooperate on one row; each lane keeps up to R gathered in-messages
// in registers so the edge update does not gather them twice.  Rows longer
// than G*R re-gather the tail (normally an L2 hit).
// MODE 0: sweep.  MODE 1: sweep + check of the means x_i = H_i / S_i formed
// from the input messages.  MODE 2: means / precisions only (no messages).
template <typename T, int G, int MODE, bool DAMP>
__global__ __launch_bounds__(kBlock) void k_csr_sweep(
    int n, const int32_t *__restrict__ oprt, const int32_t *__restrict__ rev,
    const T *__restrict__ acoef, const T *__restrict__ diag, const T *__restrict__ rhs,
    const typename Vec2<T>::type *__restrict__ min, typename Vec2<T>::type *__restrict__ mout,
    T alpha, T *__restrict__ xprev, double *__restrict__ xacc, double *__restrict__ marg,
    BlockPartial *__restrict__ part, uint32_t *__restrict__ sticky, const Ctl *__restrict__ ctl) {
  using V = typename Vec2<T>::type;
  constexpr int R = 4;
  constexpr int RPB = kBlock / G;
  if (ctl != nullptr && ctl->stop != STOP_NONE) return;  // uniform: inner solve already stopped
  const int lane = threadIdx.x % G;
  double d = 0.0, ax = 0.0;
  uint32_t f = 0;
  bool zero = false;
  for (int base = blockIdx.x * RPB; base < n; base += gridDim.x * RPB) {
    const int row = base + threadIdx.x / G;
    const bool active = row < n;
    int beg = 0, end = 0;
    if (active) {
      beg = oprt[row];
      end = oprt[row + 1];
    }
    // A1: aggregate the in-messages P_ki, h_ki (gathered through rev)
    T pin[R], hin[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      const int e = beg + lane + r * G;
      pin[r] = T(0);
      hin[r] = T(0);
      if (e < end) {
        const V m = min[rev[e]];
        pin[r] = m.x;
        hin[r] = m.y;
      }
    }
    T S = T(0), H = T(0);
#pragma unroll
    for (int r = 0; r < R; ++r) {
      S += pin[r];
      H += hin[r];
    }
    for (int e = beg + lane + R * G; e < end; e += G) {
      const V m = min[rev[e]];
      S += m.x;
      H += m.y;
    }
    S = gsum<G>(S);
    H = gsum<G>(H);
    if (active) {
      S += diag[row];
      H += rhs[row];
    }

    // A2: every out-message subtracts the reverse (in-)message
    if (MODE != 2) {
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const int e = beg + lane + r * G;
        if (e < end) {
          const T cav = S - pin[r];
          const T cavh = H - hin[r];
          const T a = acoef[e];
          zero |= (cav == T(0));
          const T inv = T(1) / cav;
          T P = -(a * a) * inv;
          T h = -(a * cavh) * inv;
          if (DAMP) {
            const V o = min[e];
            P = alpha * o.x + (T(1) - alpha) * P;
            h = alpha * o.y + (T(1) - alpha) * h;
          }
          V out;
          out.x = P;
          out.y = h;
          mout[e] = out;
        }
      }
      for (int e = beg + lane + R * G; e < end; e += G) {
        const V m = min[rev[e]];
        const T cav = S - m.x;
        const T cavh = H - m.y;
        const T a = acoef[e];
        zero |= (cav == T(0));
        const T inv = T(1) / cav;
        T P = -(a * a) * inv;
        T h = -(a * cavh) * inv;
        if (DAMP) {
          const V o = min[e];
          P = alpha * o.x + (T(1) - alpha) * P;
          h = alpha * o.y + (T(1) - alpha) * h;
        }
        V out;
        out.x = P;
        out.y = h;
        mout[e] = out;
      }
    }

    // A3: marginal means (check) or final inference
    if (MODE >= 1 && active && lane == 0) {
      if (S == T(0)) f |= FLAG_BREAKDOWN;
      const T x = H / S;
      if (!isfinite(x)) f |= FLAG_NONFINITE;
      if (MODE == 1) {
        d = fmax(d, (double)fabs(x - xprev[row]));
        xprev[row] = x;
      } else {
        if (xacc) xacc[row] += (double)H / (double)S;
        if (marg) marg[row] = (double)S;
        if (xprev) xprev[row] = x;  // means of the current messages
      }
      ax = fmax(ax, (double)fabs(x));
    }
  }
  if (zero) f |= FLAG_BREAKDOWN;
  if (f) atomicOr(sticky, f);
  if (MODE == 1) block_publish(d, ax, 0.0, 0.0, part);
}

int sweep_blocks(int n, int group, int cap) {
  const int need = (n + (kBlock / group) - 1) / (kBlock / group);
  return need < cap ? (need > 0 ? need : 1) : cap;
}

template <typename T, int G, int MODE, bool DAMP>
static void launch_one(const SweepArgs &a, hipStream_t s) {
  using V = typename Vec2<T>::type;
  hipLaunchKernelGGL((k_csr_sweep<T, G, MODE, DAMP>), dim3(a.grid), dim3(kBlock),
                     0, s, a.n, a.oprt, a.rev, (const T *)a.acoef, (const T *)a.diag,
                     (const T *)a.rhs, (const V *)a.msg_in, (V *)a.msg_out, (T)a.alpha,
                     (T *)a.xprev, a.xacc, a.marg, a.part, a.sticky, a.ctl);
}

template <typename T, int G>
static void dispatch_mode(const SweepArgs &a, hipStream_t s) {
  switch (a.mode) {
    case 0: a.damp ? launch_one<T, G, 0, true>(a, s) : launch_one<T, G, 0, false>(a, s); break;
    case 1: a.damp ? launch_one<T, G, 1, true>(a, s) : launch_one<T, G, 1, false>(a, s); break;
    default: launch_one<T, G, 2, false>(a, s); break;
  }
}

template <typename T>
static hipError_t dispatch_group(const SweepArgs &a, hipStream_t s) {
  switch (a.group) {
    case 4: dispatch_mode<T, 4>(a, s); break;
    case 8: dispatch_mode<T, 8>(a, s); break;
    case 16: dispatch_mode<T, 16>(a, s); break;
    case 32: dispatch_mode<T, 32>(a, s); break;
    case 64: dispatch_mode<T, 64>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sweep(const SweepArgs &a, hipStream_t s) {
  if (a.n <= 0) return hipSuccess;
  return a.fp32 ? dispatch_group<float>(a, s) : dispatch_group<double>(a, s);
}

// ---------------------------------------------------------------------------
// FP64 residual r = b - A x over the caller's CSR, with per-block sums of r^2
// ---------------------------------------------------------------------------
// A workgroup takes kResRows consecutive rows and streams their entries in
// chunks of kResChunk (thread t: entries c + t, c + t + kBlock, ...; all lanes
// busy, four gathers of x in flight per thread); the products go to LDS and
// the row's own thread adds them in entry order.
constexpr int kResRows = 64;
constexpr int kResK = 4;
constexpr int kResChunk = kBlock * kResK;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_csr_residual(
    int n, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
    const double *__restrict__ val, const double *__restrict__ b, const double *__restrict__ x,
    T *__restrict__ rT, double *__restrict__ r64, double *__restrict__ sumpart) {
  __shared__ int64_t rps[kResRows + 1];
  __shared__ double prod[kResChunk];
  __shared__ double sh[kBlock / 64];
  const int t = threadIdx.x;
  double sq = 0.0;
  for (int r0 = blockIdx.x * kResRows; r0 < n; r0 += gridDim.x * kResRows) {
    const int nr = min(kResRows, n - r0);
    __syncthreads();
    for (int k = t; k <= nr; k += kBlock) rps[k] = rp[r0 + k];
    __syncthreads();
    const int64_t e0 = rps[0], e1 = rps[nr];
    double acc = 0.0;
    if (x != nullptr) {
      for (int64_t c = e0; c < e1; c += kResChunk) {
        int j[kResK];
        double v[kResK], xv[kResK];
#pragma unroll
        for (int k = 0; k < kResK; ++k) {
          const int64_t e = c + k * kBlock + t;
          j[k] = 0;
          v[k] = 0.0;
          if (e < e1) {  // streamed once: kept out of the L2 that the x gather uses
            j[k] = __builtin_nontemporal_load(&col[e]);
            v[k] = __builtin_nontemporal_load(&val[e]);
          }
        }
#pragma unroll
        for (int k = 0; k < kResK; ++k) {
          xv[k] = 0.0;
          if (c + k * kBlock + t < e1) xv[k] = x[j[k]];
        }
#pragma unroll
        for (int k = 0; k < kResK; ++k)
          if (c + k * kBlock + t < e1) prod[k * kBlock + t] = v[k] * xv[k];
        __syncthreads();
        if (t < nr) {
          const int64_t lo = rps[t] > c ? rps[t] : c;
          const int64_t hi = rps[t + 1] < c + kResChunk ? rps[t + 1] : c + kResChunk;
          for (int64_t e = lo; e < hi; ++e) acc += prod[e - c];
        }
        __syncthreads();
      }
    }
    if (t < nr) {
      const int row = r0 + t;
      const double ri = b[row] - acc;
      if (rT) rT[row] = (T)ri;
      if (r64) r64[row] = ri;
      sq += ri * ri;
    }
  }
  sq = wave_sum(sq);
  if ((t & 63) == 0) sh[t / 64] = sq;
  __syncthreads();
  if (t == 0) {
    double tot = sh[0];
#pragma unroll
    for (int k = 1; k < kBlock / 64; ++k) tot += sh[k];
    sumpart[blockIdx.x] = tot;
  }
}

int residual_blocks(int n, int cap) {
  const int need = (n + kResRows - 1) / kResRows;
  return need < cap ? (need > 0 ? need : 1) : cap;
}

hipError_t launch_residual(bool fp32, int grid, int n, const int64_t *rp, const int32_t *col,
                           const double *val, const double *b, const double *x, void *rT,
                           double *r64, double *sumpart, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_csr_residual<float>, dim3(grid), dim3(kBlock), 0, s, n, rp, col, val, b,
                       x, (float *)rT, r64, sumpart);
  else
    hipLaunchKernelGGL(k_csr_residual<double>, dim3(grid), dim3(kBlock), 0, s, n, rp, col, val, b,
                       x, (double *)rT, r64, sumpart);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// readout: reduce partials in a fixed order, run the inner-solve controller,
// publish to pinned host memory
// ---------------------------------------------------------------------------
// The stop rule of the controller on one segment's own maxima (d, x).
__device__ __forceinline__ void seg_check(SegCtl &q, double d, double x, const Ctl *ctl,
                                          double &e) {
  const double rel = d / fmax(x, 1e-300);
  const double r = q.last_d > 0.0 ? d / q.last_d : 1.0;
  const double est = (r < 1.0) ? rel * r / (1.0 - r) : 1e300;
  q.last_d = d;
  e = fmax(e, est);
  if (rel == 0.0 || est <= (q.target > 0.0 ? q.target : ctl->target)) {
    q.done = 1;
  } else {
    q.stall = (rel < ctl->floor && r > 0.7) ? q.stall + 1 : 0;
    if (q.stall >= 2) q.done = 1;
  }
}

__device__ __forceinline__ unsigned long long max_bits(double v) {
  return (unsigned long long)__double_as_longlong(v > 0.0 ? v : 0.0);
}

// Without seg: part holds nparts block entries.  With seg: two colour halves
// of nparts / 2 entries, laid out as the segment sweeps publish them (see
// rb_cover): with nact <= seg_grid segments swept by seg_grid blocks,
// B = seg_grid / nact consecutive entries per segment.
__global__ __launch_bounds__(kBlock) void k_readout(
    BlockPartial *__restrict__ part, int nparts, const double *__restrict__ sumpart, int nsum,
    const uint32_t *__restrict__ sticky, Ctl *__restrict__ ctl, int sweeps_in_chunk, int seq,
    HostReadout *__restrict__ host, SegCtl *__restrict__ seg, int32_t *__restrict__ act,
    int nseg, int seg_grid) {
  __shared__ double sh[6][kBlock / 64];
  __shared__ unsigned long long accd[kMaxSweepBlocks / 2], accx[kMaxSweepBlocks / 2];
  // every thread takes these before thread 0 updates the controller below
  const bool live = nparts > 0 && ctl != nullptr && ctl->stop == STOP_NONE;
  const bool segs = live && seg != nullptr;
  const int swept = segs ? act[0] : 0;  // segments the chunk's sweeps covered
  const bool warm = live && ctl->warmup > 0;
  double s = 0.0, d = 0.0, x = 0.0, dp = 0.0, pm = 0.0, e = 0.0;
  for (int k = threadIdx.x; k < nsum; k += kBlock) s += sumpart[k];
  if (segs && swept > 0) {
    const int half = nparts / 2;
    const int B = seg_grid / swept;  // >= 1: swept <= nseg <= seg_grid
    const int ne = swept * B;
    if (B > 1) {
      for (int a = threadIdx.x; a < swept; a += kBlock) accd[a] = accx[a] = 0ull;
      __syncthreads();
    }
    for (int k = threadIdx.x; k < ne; k += kBlock) {
      const BlockPartial b0 = part[k], b1 = part[half + k];
      part[k] = BlockPartial{};
      part[half + k] = BlockPartial{};
      const double dk = fmax(b0.dmax, b1.dmax), xk = fmax(b0.xmax, b1.xmax);
      d = fmax(d, dk);
      x = fmax(x, xk);
      dp = fmax(dp, fmax(b0.dpmax, b1.dpmax));
      pm = fmax(pm, fmax(b0.pmax, b1.pmax));
      if (B > 1) {
        atomicMax(&accd[k / B], max_bits(dk));
        atomicMax(&accx[k / B], max_bits(xk));
      } else {
        SegCtl &q = seg[act[1 + k]];
        if (warm) q.last_d = 0.0;
        else seg_check(q, dk, xk, ctl, e);
      }
    }
    if (B > 1) {
      __syncthreads();
      for (int a = threadIdx.x; a < swept; a += kBlock) {
        SegCtl &q = seg[act[1 + a]];
        if (warm) q.last_d = 0.0;
        else seg_check(q, __longlong_as_double((long long)accd[a]),
                       __longlong_as_double((long long)accx[a]), ctl, e);
      }
    }
  } else if (!segs) {
    for (int k = threadIdx.x; k < nparts; k += kBlock) {
      const BlockPartial b = part[k];
      d = fmax(d, b.dmax);
      x = fmax(x, b.xmax);
      dp = fmax(dp, b.dpmax);
      pm = fmax(pm, b.pmax);
      part[k] = BlockPartial{};  // cleared for atomically raised slots (slot_publish)
    }
  }
  s = wave_sum(s);
  d = wave_max(d);
  x = wave_max(x);
  dp = wave_max(dp);
  pm = wave_max(pm);
  e = wave_max(e);
  const int w = threadIdx.x / 64;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = s; sh[1][w] = d; sh[2][w] = x; sh[3][w] = dp; sh[4][w] = pm; sh[5][w] = e;
  }
  __syncthreads();  // also orders the segment updates above before the compaction
  if (segs) seg_compact(seg, nseg, act);
  if (threadIdx.x != 0) return;
  s = sh[0][0]; d = sh[1][0]; x = sh[2][0]; dp = sh[3][0]; pm = sh[4][0]; e = sh[5][0];
  for (int k = 1; k < kBlock / 64; ++k) {
    s += sh[0][k];
    d = fmax(d, sh[1][k]);
    x = fmax(x, sh[2][k]);
    dp = fmax(dp, sh[3][k]);
    pm = fmax(pm, sh[4][k]);
    e = fmax(e, sh[5][k]);
  }
  const uint32_t flags = sticky ? *sticky : 0u;
  if (live) {
    ctl->sweeps += sweeps_in_chunk;
    ctl->checks += 1;
    ctl->seg_sweeps += (int64_t)sweeps_in_chunk * (segs ? swept : 1);
  }
  if (warm) {
    ctl->warmup -= 1;
    ctl->last_d = 0.0;
    if (flags & (FLAG_NONFINITE | FLAG_BREAKDOWN)) ctl->stop = STOP_NONFINITE;
  } else if (segs) {
    ctl->est = e;
    ctl->last_d = d;
    ctl->last_x = x;
    if (ctl->freeze_tol > 0.0 && dp <= ctl->freeze_tol * pm) ctl->freeze = 1;
    if (flags & (FLAG_NONFINITE | FLAG_BREAKDOWN)) ctl->stop = STOP_NONFINITE;
    else if (act[0] == 0) ctl->stop = STOP_CONVERGED;
  } else if (live) {
    const double rel = d / fmax(x, 1e-300);
    const double q = ctl->last_d > 0.0 ? d / ctl->last_d : 1.0;
    const double est = (q < 1.0) ? rel * q / (1.0 - q) : 1e300;
    ctl->est = est;
    ctl->last_d = d;
    ctl->last_x = x;
    if (ctl->freeze_tol > 0.0 && dp <= ctl->freeze_tol * pm) ctl->freeze = 1;
    if (flags & (FLAG_NONFINITE | FLAG_BREAKDOWN)) {
      ctl->stop = STOP_NONFINITE;
    } else if (rel == 0.0 || est <= ctl->target) {
      ctl->stop = STOP_CONVERGED;
    } else {
      ctl->stall = (rel < ctl->floor && q > 0.7) ? ctl->stall + 1 : 0;
      if (ctl->stall >= 2) ctl->stop = STOP_STALLED;
    }
  }
  host->dmax = d;
  host->xmax = x;
  host->sum = s;
  host->dpmax = dp;
  host->pmax = pm;
  host->flags = flags;
  host->stop = ctl ? ctl->stop : 0u;
  host->sweeps = ctl ? ctl->sweeps : 0;
  host->freeze = ctl ? ctl->freeze : 0;
  host->seg_sweeps = ctl ? ctl->seg_sweeps : 0;
  host->segrel = -1.0;  // set by the per-segment norms when a plan has segments
  // the sequence number last: a host that sees it sees the fields
  __threadfence_system();
  __hip_atomic_store(&host->seq, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  __threadfence_system();
}

hipError_t launch_readout(BlockPartial *part, int nparts, const double *sumpart, int nsum,
                          const uint32_t *sticky, Ctl *ctl, int sweeps_in_chunk, int seq,
                          HostReadout *host, hipStream_t s, SegCtl *seg, int32_t *act, int nseg,
                          int seg_grid) {
  if (seg && (nseg < 1 || seg_grid < nseg || seg_grid > kMaxSweepBlocks || nparts < 2 * seg_grid))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_readout, dim3(1), dim3(kBlock), 0, s, part, nparts, sumpart, nsum, sticky,
                     ctl, sweeps_in_chunk, seq, host, seg, act, nseg, seg_grid);
  return hipGetLastError();
}

__global__ void k_ctl_reset(Ctl *ctl, double target, double floor, double freeze_tol, int full,
                            int warmup) {
  if (threadIdx.x != 0) return;
  ctl->freeze_tol = freeze_tol;
  ctl->stop = STOP_NONE;
  ctl->stall = 0;
  ctl->target = target;
  ctl->floor = floor;
  ctl->last_d = 0.0;
  ctl->last_x = 0.0;
  ctl->est = 1e300;
  ctl->warmup = warmup;
  if (full) {
    ctl->seg_sweeps = 0;
    ctl->sweeps = 0;
    ctl->checks = 0;
    ctl->freeze = 0;
  }
}

hipError_t launch_ctl_reset(Ctl *ctl, double target, double floor, double freeze_tol, bool full,
                            int warmup, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl_reset, dim3(1), dim3(64), 0, s, ctl, target, floor, freeze_tol,
                     full ? 1 : 0, warmup);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// fills, restarts, message export / import
// ---------------------------------------------------------------------------
template <typename V>
__global__ void k_zero_h(int64_t E, V *__restrict__ msg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E) msg[e].y = 0;
}

hipError_t launch_zero_h(bool fp32, int64_t E, void *msg, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  const dim3 grid((unsigned)((E + kBlock - 1) / kBlock));
  if (fp32) hipLaunchKernelGGL(k_zero_h<float2>, grid, dim3(kBlock), 0, s, E, (float2 *)msg);
  else hipLaunchKernelGGL(k_zero_h<double2>, grid, dim3(kBlock), 0, s, E, (double2 *)msg);
  return hipGetLastError();
}

__global__ void k_fill_zero8(uint64_t *__restrict__ p, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) p[i] = 0;
}
__global__ void k_fill_zero4(uint32_t *__restrict__ p, int64_t m) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) p[i] = 0;
}

hipError_t launch_fill_zero(void *p, int64_t m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero8, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     (uint64_t *)p, m);
  return hipGetLastError();
}
hipError_t launch_fill_zero4(void *p, int64_t m, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero4, dim3((unsigned)((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                     (uint32_t *)p, m);
  return hipGetLastError();
}

template <typename V, bool GET>
__global__ void k_msgs_io(int n, const int64_t *__restrict__ rp, const int64_t *__restrict__ diagpos,
                          const int32_t *__restrict__ oprt, V *__restrict__ msg, double *__restrict__ P,
                          double *__restrict__ h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = rp[i], e = rp[i + 1], dp = diagpos[i];
  for (int64_t k = b; k < e; ++k) {
    if (k == dp) {
      if (GET) { P[k] = 0.0; h[k] = 0.0; }
      continue;
    }
    const int64_t o = oprt[i] + (k - b) - (k > dp ? 1 : 0);
    if (GET) {
      P[k] = (double)msg[o].x;
      h[k] = (double)msg[o].y;
    } else {
      msg[o].x = P[k];
      msg[o].y = h[k];
    }
  }
}

hipError_t launch_get_msgs(bool fp32, int n, const int64_t *rp, const int64_t *diagpos,
                           const int32_t *oprt, const void *msg, double *P, double *h,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((n + kBlock - 1) / kBlock);
  if (fp32) hipLaunchKernelGGL((k_msgs_io<float2, true>), grid, dim3(kBlock), 0, s, n, rp, diagpos, oprt, (float2 *)msg, P, h);
  else hipLaunchKernelGGL((k_msgs_io<double2, true>), grid, dim3(kBlock), 0, s, n, rp, diagpos, oprt, (double2 *)msg, P, h);
  return hipGetLastError();
}

hipError_t launch_set_msgs(bool fp32, int n, const int64_t *rp, const int64_t *diagpos,
                           const int32_t *oprt, void *msg, const double *P, const double *h,
                           hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((n + kBlock - 1) / kBlock);
  if (fp32) hipLaunchKernelGGL((k_msgs_io<float2, false>), grid, dim3(kBlock), 0, s, n, rp, diagpos, oprt, (float2 *)msg, (double *)P, (double *)h);
  else hipLaunchKernelGGL((k_msgs_io<double2, false>), grid, dim3(kBlock), 0, s, n, rp, diagpos, oprt, (double2 *)msg, (double *)P, (double *)h);
  return hipGetLastError();
}

}  // namespace gabp
