// GaBP on structured grids (5-point 2-D / 7-point 3-D stencils), gfx950.
//
// Node i = x + nx (y + ny z) of a stack of `batch` grids (z runs over the
// stack; grids are not coupled to each other).  Direction d in
// {+x, -x, +y, -y, +z, -z} = {0..5}, opposite direction d ^ 1.  The message
// node i sends toward direction d is stored at msg[d * N + i] as (P, h), h = P mu.
// The in-message that node i receives from its neighbour j = i + off(d) is
// j's out-message toward d ^ 1: msg[(d ^ 1) * N + j], a shifted coalesced
// read.  Each sweep is Algorithm 2 of the paper (section V) in information
// form:
//   S_i = A_ii + sum_d P_in(d),  H_i = b_i + sum_d h_in(d)
//   P_out(d) = -a_d^2 / (S_i - P_in(d)),  h_out(d) = -a_d (H_i - h_in(d)) / (S_i - P_in(d))
// (eq. prec_message / mean_message), a_d the coupling A_ij toward d; an edge
// with a_d = 0 (or outside the grid) carries no message.  Every message array
// is read once as in-messages, once as the previous out-messages (damping
// only) and written once: 16 bytes per edge undamped, 24 damped (FP32).
//
// Settled-precision ("frozen") sweeps keep c_d = -a_d / (S_i - P_in(d)) fixed
// and update h_out(d) = c_d (H_i - h_in(d)) only (h in separate FP32 arrays).
#include "device_common.h"

namespace gabp {

namespace {

struct Nbr {
  int j[6];      // neighbour index toward d (valid when ok[d])
  bool ok[6];    // edge exists (inside the grid)
};

// FAST: the divisions by the extents as multiply and shift (GridGeom's
// divisors).  The sweeps keep the compiler's division: with the shorter
// index arithmetic their check launches ran slower (300 -> 400 us on the
// 64-grid stack), the FP64 residual runs faster.
template <bool FAST = false>
__device__ __forceinline__ void neighbours(const GridGeom &g, int i, Nbr &nb) {
  const int nxy = g.nx * g.ny;
  int x, y, zl;
  if (FAST) {
    const int r = fdiv(i, g.fx), z = fdiv(r, g.fy);
    x = i - r * g.nx;
    y = r - z * g.ny;
    zl = z - fdiv(z, g.fz) * g.nz;
  } else {
    x = i % g.nx;
    y = (i / g.nx) % g.ny;
    zl = (i / nxy) % g.nz;
  }
  nb.ok[0] = x < g.nx - 1; nb.j[0] = i + 1;
  nb.ok[1] = x > 0;        nb.j[1] = i - 1;
  nb.ok[2] = y < g.ny - 1; nb.j[2] = i + g.nx;
  nb.ok[3] = y > 0;        nb.j[3] = i - g.nx;
  nb.ok[4] = zl < g.nz - 1; nb.j[4] = i + nxy;
  nb.ok[5] = zl > 0;        nb.j[5] = i - nxy;
}

// coupling toward each direction (0 where there is no edge)
template <typename T, bool VARC>
__device__ __forceinline__ void couplings(const GridGeom &g, const GridCoef<T> &k, int i,
                                          const Nbr &nb, T a[6]) {
  if (VARC) {
    a[0] = nb.ok[0] ? k.cx[i] : T(0);
    a[1] = nb.ok[1] ? k.cx[i - 1] : T(0);
    a[2] = nb.ok[2] ? k.cy[i] : T(0);
    a[3] = nb.ok[3] ? k.cy[i - g.nx] : T(0);
    a[4] = nb.ok[4] ? k.cz[i] : T(0);
    a[5] = nb.ok[5] ? k.cz[i - g.nx * g.ny] : T(0);
  } else {
#pragma unroll
    for (int d = 0; d < 6; ++d) a[d] = nb.ok[d] ? k.aconst : T(0);
  }
}

// XCD-aware tile order: dispatch sends consecutive blocks to different XCDs
// (round robin over 8); renumbering so that each XCD walks a contiguous range
// of tiles keeps the cache lines shared by neighbouring tiles in one L2.
__device__ __forceinline__ int tile_of_block() {
  const int nb = gridDim.x;
  if (nb % 8 != 0) return blockIdx.x;
  return (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
}

}  // namespace

// MODE 0 sweep, 1 sweep + check, 2 means / precisions only (no messages)
template <typename T, int MODE, bool DAMP, bool VARC>
__global__ __launch_bounds__(kBlock) void k_grid_sweep(
    GridGeom g, GridCoef<T> k, const typename Vec2<T>::type *__restrict__ min,
    typename Vec2<T>::type *__restrict__ mout, const T *__restrict__ rhs, T alpha,
    T *__restrict__ xprev, double *__restrict__ xacc, double *__restrict__ marg,
    BlockPartial *__restrict__ part, uint32_t *__restrict__ sticky, const Ctl *__restrict__ ctl,
    int fl) {
  using V = typename Vec2<T>::type;
  if (ctl != nullptr && ctl->stop != STOP_NONE) return;
  const int N = g.N;
  double dmax = 0.0, xmax = 0.0, dpb = 0.0, pmb = 0.0;
  uint32_t f = 0;
  const int tile0 = tile_of_block();
  for (int base = tile0 * kBlock; base < N; base += gridDim.x * kBlock) {
    const int i = base + threadIdx.x;
    if (i >= N) continue;
    Nbr nb;
    neighbours(g, i, nb);
    T a[6];
    couplings<T, VARC>(g, k, i, nb, a);
    T Pin[6], hin[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      Pin[d] = T(0);
      hin[d] = T(0);
      if (a[d] != T(0)) {
        const V m = min[(size_t)(d ^ 1) * N + nb.j[d]];
        Pin[d] = m.x;
        hin[d] = (fl & SWEEP_ZIN) ? T(0) : m.y;
      }
    }
    T S = VARC ? k.diag[i] : k.dconst, H = rhs[i];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      S += Pin[d];
      H += hin[d];
    }
    if (MODE != 2) {
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        if (a[d] == T(0)) continue;
        const T cav = S - Pin[d];
        if (cav == T(0)) f |= FLAG_BREAKDOWN;
        const T inv = T(1) / cav;
        T P = -(a[d] * a[d]) * inv;
        T h = -(a[d] * (H - hin[d])) * inv;
        if (DAMP || MODE == 1) {
          const V o = min[(size_t)d * N + i];
          if (DAMP) {
            P = alpha * o.x + (T(1) - alpha) * P;
            h = alpha * ((fl & SWEEP_ZOWN) ? T(0) : o.y) + (T(1) - alpha) * h;
          }
          if (MODE == 1) {
            dpb = fmax(dpb, (double)fabs(P - o.x));
            pmb = fmax(pmb, (double)fabs(P));
          }
        }
        V out;
        out.x = P;
        out.y = h;
        nt_store(&mout[(size_t)d * N + i], out);
      }
    }
    if (MODE >= 1) {
      if (S == T(0)) f |= FLAG_BREAKDOWN;
      const T x = H / S;
      if (!isfinite(x)) f |= FLAG_NONFINITE;
      if (MODE == 1) {
        dmax = fmax(dmax, (double)fabs(x - xprev[i]));
        xprev[i] = x;
      } else {
        if (xacc) {
          const double m = (double)H / (double)S;
          xacc[i] = (fl & SWEEP_XSET) ? m : xacc[i] + m;
        }
        if (marg) marg[i] = (double)S;
        if (xprev) xprev[i] = x;  // means of the current messages
      }
      xmax = fmax(xmax, (double)fabs(x));
    }
  }
  if (f) atomicOr(sticky, f);
  if (MODE == 1) block_publish(dmax, xmax, dpb, pmb, part);
}

// frozen: information only, fixed coefficients coef[d * N + i] = c_d(i)
template <typename T, int MODE, bool DAMP, bool VARC>
__global__ __launch_bounds__(kBlock) void k_grid_frozen(
    GridGeom g, GridCoef<T> k, const T *__restrict__ coef, const T *__restrict__ Sfix,
    const T *__restrict__ hin_arr, T *__restrict__ hout_arr, const T *__restrict__ rhs, T alpha,
    T *__restrict__ xprev, double *__restrict__ xacc, double *__restrict__ marg,
    BlockPartial *__restrict__ part, uint32_t *__restrict__ sticky, const Ctl *__restrict__ ctl,
    int fl) {
  if (ctl != nullptr && ctl->stop != STOP_NONE) return;
  const int N = g.N;
  double dmax = 0.0, xmax = 0.0;
  uint32_t f = 0;
  const int tile0 = tile_of_block();
  for (int base = tile0 * kBlock; base < N; base += gridDim.x * kBlock) {
    const int i = base + threadIdx.x;
    if (i >= N) continue;
    // Edges from the geometry alone: the freeze stored zero coefficients and
    // zero informations on faces whose coupling is zero, so those carry zeros
    // both ways and the couplings need not be read in this phase.
    Nbr nb;
    neighbours(g, i, nb);
    T hin[6];
    T H = rhs[i];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      hin[d] = T(0);
      if (nb.ok[d] && !(fl & SWEEP_ZIN)) hin[d] = hin_arr[(size_t)(d ^ 1) * N + nb.j[d]];
      H += hin[d];
    }
    if (MODE != 2) {
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        if (!nb.ok[d]) continue;
        T h = coef[(size_t)d * N + i] * (H - hin[d]);
        if (DAMP)
          h = alpha * ((fl & SWEEP_ZOWN) ? T(0) : hin_arr[(size_t)d * N + i]) + (T(1) - alpha) * h;
        __builtin_nontemporal_store(h, &hout_arr[(size_t)d * N + i]);
      }
    }
    if (MODE >= 1) {
      const T S = Sfix[i];
      const T x = H / S;
      if (!isfinite(x)) f |= FLAG_NONFINITE;
      if (MODE == 1) {
        dmax = fmax(dmax, (double)fabs(x - xprev[i]));
        xprev[i] = x;
      } else {
        if (xacc) {
          const double m = (double)H / (double)S;
          xacc[i] = (fl & SWEEP_XSET) ? m : xacc[i] + m;
        }
        if (marg) marg[i] = (double)S;
        if (xprev) xprev[i] = x;  // means of the current messages
      }
      xmax = fmax(xmax, (double)fabs(x));
    }
  }
  if (f) atomicOr(sticky, f);
  if (MODE == 1) block_publish(dmax, xmax, 0.0, 0.0, part);
}

// freeze: coefficients and information arrays from the current full state
// (hh NULL: the informations are discarded, a restart follows)
template <typename T, bool VARC>
__global__ __launch_bounds__(kBlock) void k_grid_freeze(
    GridGeom g, GridCoef<T> k, const typename Vec2<T>::type *__restrict__ msg,
    T *__restrict__ coef, T *__restrict__ hh, T *__restrict__ Sfix) {
  const int N = g.N;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    Nbr nb;
    neighbours(g, i, nb);
    T a[6];
    couplings<T, VARC>(g, k, i, nb, a);
    T Pin[6];
    T S = VARC ? k.diag[i] : k.dconst;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const T p = nb.ok[d] ? msg[(size_t)(d ^ 1) * N + nb.j[d]].x : T(0);
      Pin[d] = a[d] != T(0) ? p : T(0);
      S += Pin[d];
    }
    Sfix[i] = S;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const size_t o = (size_t)d * N + i;
      coef[o] = a[d] != T(0) ? -a[d] / (S - Pin[d]) : T(0);
      if (hh) hh[o] = a[d] != T(0) ? msg[o].y : T(0);
    }
  }
}

// FP64 residual r = b - A x with the caller's FP64 coefficients
template <bool VARC>
__global__ __launch_bounds__(kBlock) void k_grid_residual(
    GridGeom g, GridCoef<double> k, const double *__restrict__ b, const double *__restrict__ x,
    void *__restrict__ rT, bool rT32, double *__restrict__ r64, double *__restrict__ sumpart, int hx,
    int nseg) {
  const int N = g.N;
  const int Nc = hx * (N / g.nx);
  const int segb = gridDim.x / nseg;          // blocks per segment
  const int seg = blockIdx.x / segb;
  const int len = N / nseg;
  const int hi = (seg + 1) * len;
  double sq = 0.0;
  for (int i = seg * len + (blockIdx.x - seg * segb) * kBlock + threadIdx.x; i < hi;
       i += segb * kBlock) {
    double ri = b[i];
    if (x != nullptr) {
      Nbr nb;
      neighbours<true>(g, i, nb);
      double a[6];
      couplings<double, VARC>(g, k, i, nb, a);
      double xn[6];  // loaded on the geometry alone, not after the couplings
#pragma unroll
      for (int d = 0; d < 6; ++d) xn[d] = nb.ok[d] ? x[nb.j[d]] : 0.0;
      double ax = (VARC ? k.diag[i] : k.dconst) * x[i];
#pragma unroll
      for (int d = 0; d < 6; ++d)
        if (a[d] != 0.0) ax += a[d] * xn[d];
      ri -= ax;
    }
    if (rT) {
      int at = i;
      if (hx > 0) {
        int c, slot;
        rb_place(g, hx, i, c, slot);
        at = c * Nc + slot;
      }
      if (rT32) ((float *)rT)[at] = (float)ri;
      else ((double *)rT)[at] = ri;
    }
    if (r64) r64[i] = ri;
    sq += ri * ri;
  }
  __shared__ double sh[kBlock / 64];
  sq = wave_sum(sq);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x / 64] = sq;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0];
    for (int w = 1; w < kBlock / 64; ++w) t += sh[w];
    sumpart[blockIdx.x] = t;
  }
}

// validation of the coefficients: non-finite values or a zero diagonal
template <bool VARC>
__global__ void k_grid_check(GridGeom g, GridCoef<double> k, uint32_t *__restrict__ flags) {
  const int N = g.N;
  uint32_t f = 0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < N; i += gridDim.x * kBlock) {
    const double dv = VARC ? k.diag[i] : k.dconst;
    if (dv == 0.0) f |= FLAG_ZERO_DIAG;
    if (!isfinite(dv)) f |= FLAG_ARG;
    if (VARC) {
      if (!isfinite(k.cx[i]) || !isfinite(k.cy[i]) || (k.cz && !isfinite(k.cz[i]))) f |= FLAG_ARG;
    }
  }
  if (f) atomicOr(flags, f);
}

// FP64 coefficient arrays -> working precision
template <typename T>
__global__ void k_to_working(int64_t m, const double *__restrict__ in, T *__restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) out[i] = in ? (T)in[i] : T(0);
}

template <typename T>
__global__ void k_grid_zero_h(int64_t m, typename Vec2<T>::type *__restrict__ msg) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < m) msg[i].y = T(0);
}

// export / import in direction-major order [6][N] (FP64 P and h)
template <typename T, bool GET>
__global__ void k_grid_io(int64_t m, typename Vec2<T>::type *__restrict__ msg, double *__restrict__ P,
                          double *__restrict__ h) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= m) return;
  if (GET) {
    P[i] = (double)msg[i].x;
    h[i] = (double)msg[i].y;
  } else {
    msg[i].x = (T)P[i];
    msg[i].y = (T)h[i];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int MODE, bool DAMP, bool VARC>
static void grid_one(const GridArgs &a, hipStream_t s) {
  using V = typename Vec2<T>::type;
  GridCoef<T> k;
  k.diag = (const T *)a.diag; k.cx = (const T *)a.cx; k.cy = (const T *)a.cy; k.cz = (const T *)a.cz;
  k.dconst = (T)a.dconst; k.aconst = (T)a.aconst;
  if (a.frozen)
    hipLaunchKernelGGL((k_grid_frozen<T, MODE, DAMP, VARC>), dim3(a.grid), dim3(kBlock), 0, s,
                       a.g, k, (const T *)a.coef, (const T *)a.Sfix, (const T *)a.msg_in,
                       (T *)a.msg_out, (const T *)a.rhs, (T)a.alpha, (T *)a.xprev, a.xacc,
                       a.marg, a.part, a.sticky, a.ctl, a.fl);
  else
    hipLaunchKernelGGL((k_grid_sweep<T, MODE, DAMP, VARC>), dim3(a.grid), dim3(kBlock), 0, s, a.g,
                       k, (const V *)a.msg_in, (V *)a.msg_out, (const T *)a.rhs, (T)a.alpha,
                       (T *)a.xprev, a.xacc, a.marg, a.part, a.sticky, a.ctl, a.fl);
}

template <typename T, bool VARC>
static void grid_mode(const GridArgs &a, hipStream_t s) {
  switch (a.mode) {
    case 0: a.damp ? grid_one<T, 0, true, VARC>(a, s) : grid_one<T, 0, false, VARC>(a, s); break;
    case 1: a.damp ? grid_one<T, 1, true, VARC>(a, s) : grid_one<T, 1, false, VARC>(a, s); break;
    default: grid_one<T, 2, false, VARC>(a, s); break;
  }
}

hipError_t launch_grid_sweep(const GridArgs &a, hipStream_t s) {
  if (a.g.N <= 0) return hipSuccess;
  if (!geom_ok(a.g)) return hipErrorInvalidValue;
  if (a.fp32) a.varc ? grid_mode<float, true>(a, s) : grid_mode<float, false>(a, s);
  else a.varc ? grid_mode<double, true>(a, s) : grid_mode<double, false>(a, s);
  return hipGetLastError();
}

hipError_t launch_grid_freeze(const GridArgs &a, hipStream_t s) {
  if (a.g.N <= 0) return hipSuccess;
  if (!geom_ok(a.g)) return hipErrorInvalidValue;
  if (a.fp32) {
    GridCoef<float> k{(const float *)a.diag, (const float *)a.cx, (const float *)a.cy,
                      (const float *)a.cz, (float)a.dconst, (float)a.aconst};
    if (a.varc)
      hipLaunchKernelGGL((k_grid_freeze<float, true>), dim3(a.grid), dim3(kBlock), 0, s, a.g, k,
                         (const float2 *)a.msg_in, (float *)a.coef, (float *)a.msg_out, (float *)a.Sfix);
    else
      hipLaunchKernelGGL((k_grid_freeze<float, false>), dim3(a.grid), dim3(kBlock), 0, s, a.g, k,
                         (const float2 *)a.msg_in, (float *)a.coef, (float *)a.msg_out, (float *)a.Sfix);
  } else {
    GridCoef<double> k{(const double *)a.diag, (const double *)a.cx, (const double *)a.cy,
                       (const double *)a.cz, a.dconst, a.aconst};
    if (a.varc)
      hipLaunchKernelGGL((k_grid_freeze<double, true>), dim3(a.grid), dim3(kBlock), 0, s, a.g, k,
                         (const double2 *)a.msg_in, (double *)a.coef, (double *)a.msg_out, (double *)a.Sfix);
    else
      hipLaunchKernelGGL((k_grid_freeze<double, false>), dim3(a.grid), dim3(kBlock), 0, s, a.g, k,
                         (const double2 *)a.msg_in, (double *)a.coef, (double *)a.msg_out, (double *)a.Sfix);
  }
  return hipGetLastError();
}

hipError_t launch_grid_residual(const GridGeom &g, const GridCoef<double> &k, bool varc, int grid,
                                const double *b, const double *x, void *rT, bool rT32, double *r64,
                                double *sumpart, hipStream_t s, int hx, int nseg) {
  if (g.N <= 0) return hipSuccess;
  if (nseg < 1 || grid % nseg != 0 || g.N % nseg != 0 || !geom_ok(g)) return hipErrorInvalidValue;
  if (hx > 0 && hx != g.fh.d) return hipErrorInvalidValue;
  if (varc)
    hipLaunchKernelGGL((k_grid_residual<true>), dim3(grid), dim3(kBlock), 0, s, g, k, b, x, rT, rT32, r64, sumpart, hx, nseg);
  else
    hipLaunchKernelGGL((k_grid_residual<false>), dim3(grid), dim3(kBlock), 0, s, g, k, b, x, rT, rT32, r64, sumpart, hx, nseg);
  return hipGetLastError();
}

// one thread per segment: sums its partials in a fixed order
__global__ __launch_bounds__(kBlock) void k_seg_norms(
    const double *__restrict__ sumpart, int nseg, int segb, double *__restrict__ segb2, int store,
    double bnorm, HostReadout *__restrict__ host, SegCtl *__restrict__ seg,
    int32_t *__restrict__ act, double tol, double tfloor, double inner_tol) {
  __shared__ double sh[kBlock / 64];
  double worst = 0.0;
  for (int t = threadIdx.x; t < nseg; t += kBlock) {
    double sq = 0.0;
    for (int k = 0; k < segb; ++k) sq += sumpart[(size_t)t * segb + k];
    if (store) {
      segb2[t] = sq;
      if (seg) seg[t] = SegCtl{0.0, 0.0, 0, 0, HUGE_VAL};
    } else {
      const double bn = segb2[t] > 0.0 ? sqrt(segb2[t]) : bnorm;
      const double rel = bn > 0.0 ? sqrt(sq) / bn : sqrt(sq);
      worst = fmax(worst, rel);  // non-finite sums are caught by the whole-system norm
      if (seg) {
        // the next pass: a segment within the tolerance sits it out, the
        // others aim at the factor their own residual still needs.  A pass
        // stopped on an estimate made right after the restart can leave
        // high-frequency error that raises the residual; a segment whose
        // residual grew gets a ten times tighter target than it had.
        double tg = inner_tol > 0.0 ? inner_tol : fmin(0.5, fmax(0.3 * tol / rel, tfloor));
        if (inner_tol <= 0.0 && rel > seg[t].rel && seg[t].target > 0.0)
          tg = fmax(tfloor, fmin(tg, 0.1 * seg[t].target));
        seg[t] = SegCtl{0.0, tg, rel <= tol ? 2 : 0, 0, rel};
      }
    }
  }
  if (seg) seg_compact(seg, nseg, act);
  if (store) return;
  worst = wave_max(worst);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x / 64] = worst;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kBlock / 64; ++w) worst = fmax(worst, sh[w]);
    host->segrel = worst;
    __threadfence_system();
  }
}

hipError_t launch_seg_norms(const double *sumpart, int nseg, int segb, double *segb2, int store,
                            double bnorm, HostReadout *host, hipStream_t s, SegCtl *seg,
                            int32_t *act, double tol, double tfloor, double inner_tol) {
  hipLaunchKernelGGL(k_seg_norms, dim3(1), dim3(kBlock), 0, s, sumpart, nseg, segb, segb2, store,
                     bnorm, host, seg, act, tol, tfloor, inner_tol);
  return hipGetLastError();
}

hipError_t launch_grid_check(const GridGeom &g, const GridCoef<double> &k, bool varc, int grid,
                             uint32_t *flags, hipStream_t s) {
  if (g.N <= 0) return hipSuccess;
  if (varc) hipLaunchKernelGGL((k_grid_check<true>), dim3(grid), dim3(kBlock), 0, s, g, k, flags);
  else hipLaunchKernelGGL((k_grid_check<false>), dim3(grid), dim3(kBlock), 0, s, g, k, flags);
  return hipGetLastError();
}

hipError_t launch_to_working(bool fp32, int64_t m, const double *in, void *out, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((m + kBlock - 1) / kBlock));
  if (fp32) hipLaunchKernelGGL(k_to_working<float>, grid, dim3(kBlock), 0, s, m, in, (float *)out);
  else hipLaunchKernelGGL(k_to_working<double>, grid, dim3(kBlock), 0, s, m, in, (double *)out);
  return hipGetLastError();
}

hipError_t launch_grid_zero_h(bool fp32, int64_t m, void *msg, hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((m + kBlock - 1) / kBlock));
  if (fp32) hipLaunchKernelGGL(k_grid_zero_h<float>, grid, dim3(kBlock), 0, s, m, (float2 *)msg);
  else hipLaunchKernelGGL(k_grid_zero_h<double>, grid, dim3(kBlock), 0, s, m, (double2 *)msg);
  return hipGetLastError();
}

hipError_t launch_grid_io(bool fp32, bool get, int64_t m, void *msg, double *P, double *h,
                          hipStream_t s) {
  if (m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((m + kBlock - 1) / kBlock));
  if (fp32) {
    if (get) hipLaunchKernelGGL((k_grid_io<float, true>), grid, dim3(kBlock), 0, s, m, (float2 *)msg, P, h);
    else hipLaunchKernelGGL((k_grid_io<float, false>), grid, dim3(kBlock), 0, s, m, (float2 *)msg, P, h);
  } else {
    if (get) hipLaunchKernelGGL((k_grid_io<double, true>), grid, dim3(kBlock), 0, s, m, (double2 *)msg, P, h);
    else hipLaunchKernelGGL((k_grid_io<double, false>), grid, dim3(kBlock), 0, s, m, (double2 *)msg, P, h);
  }
  return hipGetLastError();
}

}  // namespace gabp
