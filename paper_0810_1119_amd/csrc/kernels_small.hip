// Small sparse systems in one persistent launch.  A batch of independent
// instances is given as the diagonal blocks of one CSR matrix; each workgroup
// takes the next instance from a queue sorted by size and solves it alone
// with every message in LDS: sweeps of Algorithm 2 (section V) in the
// synchronous or the serial scheme in colour order (section III-C), the FP64
// residual at every check, refinement restarts, and optionally Aitken's or
// Steffensen's acceleration of the means (section IV-A).  No host round trip
// happens between sweeps, so a single small system (a 32 x 32 Poisson grid)
// costs the sweeps themselves and nothing else.
//
// Message storage ("push" form).  In-slot e of row i, in the order of row i's
// off-diagonal CSR entries, holds the message j -> i that row i receives from
// its neighbour j, as (P_ji, h_ji) with h = P mu.  A row reads its in-slots
// (contiguous) to form its totals
//     S_i = A_ii + sum_k P_ki,     H_i = rhs_i + sum_k h_ki,
// and sends, for each in-slot e = (i <- j) with coupling a = A_ij,
//     P_ij = -a^2 / (S_i - P_ji),  h_ij = -a (H_i - h_ji) / (S_i - P_ji)
// (eq. prec_message / mean_message with the reverse message subtracted) into
// in-slot rev[e] of row j.  Synchronous: from one buffer into the other, one
// barrier per sweep.  Coloured: one colour class after the other, in place: no
// edge joins two rows of a class, so the in-slots a class reads are written
// only by other classes, and the in-slots it writes belong to idle rows.
#include <cmath>

#include "gabp_internal.h"

namespace gabp {
namespace {

// Wavefront reductions by a fixed butterfly: the result is the same in every
// lane and independent of timing.
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}

// One sum, two maxima and two flags over the workgroup, in a fixed order;
// every thread receives the results.  red holds 8 doubles per wavefront.
__device__ void block_reduce(double &sum, double &m0, double &m1, bool &f0, bool &f1,
                             double *red) {
  const int W = blockDim.x >> 6;
  sum = wave_sum(sum);
  m0 = wave_max(m0);
  m1 = wave_max(m1);
  const bool a0 = __any(f0), a1 = __any(f1);
  if ((threadIdx.x & 63) == 0) {
    double *o = red + (threadIdx.x >> 6) * 8;
    o[0] = sum; o[1] = m0; o[2] = m1; o[3] = a0 ? 1.0 : 0.0; o[4] = a1 ? 1.0 : 0.0;
  }
  __syncthreads();
  sum = 0.0; m0 = 0.0; m1 = 0.0;
  bool g0 = false, g1 = false;
  for (int w = 0; w < W; ++w) {
    const double *o = red + w * 8;
    sum += o[0];
    m0 = fmax(m0, o[1]);
    m1 = fmax(m1, o[2]);
    g0 = g0 || o[3] != 0.0;
    g1 = g1 || o[4] != 0.0;
  }
  f0 = g0;
  f1 = g1;
  __syncthreads();
}

// Section IV-A: y = x0 - (x1 - x0)^2 / (x2 - 2 x1 + x0) from three
// consecutive samples; a vanishing second difference keeps the newest.
__device__ __forceinline__ double aitken(double x0, double x1, double x2) {
  const double d1 = x1 - x0;
  const double d2 = x2 - 2.0 * x1 + x0;
  return d2 != 0.0 ? x0 - d1 * d1 / d2 : x2;
}

// The rows a thread owns (row tid + r * blockDim.x of the instance, r < RM)
// and, with CACHE > 0 (RM == 1), the reverse index and coupling of the slots
// of a row of degree <= CACHE in registers for the whole solve (longer rows
// read them from memory at every sweep).  In-messages are read from LDS
// where they are used (a register copy across the send would cost more
// registers than the second LDS read costs time).
template <typename T, int RM, int CACHE>
struct Rows {
  using T2 = typename Vec2<T>::type;
  static constexpr int CS = CACHE > 0 ? CACHE : 1;
  int slot0 = 0, node0 = 0;
  bool ok[RM];
  int s0[RM], deg[RM], colr[RM];
  T dg[RM], rhs[RM], S[RM], H[RM];
  int rv[CS];
  T av[CS];

  __device__ void load(const SmallArgs &a, const SmallInst &I) {
    slot0 = I.slot0;
    node0 = I.node0;
    const T *diag = (const T *)a.diagT;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      const int i = threadIdx.x + r * blockDim.x;
      ok[r] = i < I.n;
      s0[r] = 0; deg[r] = 0; colr[r] = 0;
      dg[r] = T(1); rhs[r] = T(0); S[r] = T(1); H[r] = T(0);
      if (ok[r]) {
        const int g = I.node0 + i;
        s0[r] = a.soff[g] - I.slot0;
        deg[r] = a.soff[g + 1] - a.soff[g];
        dg[r] = diag[g];
        colr[r] = a.color ? a.color[g] : 0;
      }
    }
    if (CACHE > 0) {
      const T *ac = (const T *)a.acoef;
#pragma unroll
      for (int k = 0; k < CS; ++k) {
        rv[k] = 0;
        av[k] = T(0);
        if (ok[0] && deg[0] <= CACHE && k < deg[0]) {
          const int e = I.slot0 + s0[0] + k;
          rv[k] = a.rev[e] - I.slot0;
          av[k] = ac[e];
        }
      }
    }
  }

  // totals of the rows (of colour c when c >= 0) from the messages in B
  __device__ void sums(const T2 *B, int c) {
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      if (!ok[r] || (c >= 0 && colr[r] != c)) continue;
      T s = dg[r], h = rhs[r];
      if (CACHE > 0 && deg[0] <= CACHE) {
#pragma unroll
        for (int k = 0; k < CS; ++k)
          if (k < deg[0]) {
            const T2 m = B[s0[0] + k];
            s += m.x;
            h += m.y;
          }
      } else {
        for (int k = 0; k < deg[r]; ++k) {
          const T2 m = B[s0[r] + k];
          s += m.x;
          h += m.y;
        }
      }
      S[r] = s;
      H[r] = h;
    }
  }

  // one outgoing message from the cavity of in-message (pin, hin)
  __device__ __forceinline__ void emit(const T2 *B, T2 *O, int rr, T aa, T pin, T hin, T Sr,
                                       T Hr, bool damp, T alpha, bool &brk) const {
    const T cav = Sr - pin;
    if (cav == T(0)) brk = true;
    const T f = -aa / cav;
    T P = f * aa;
    T h = f * (Hr - hin);
    if (damp) {
      const T2 old = B[rr];  // this message as last sent (same slot)
      P = alpha * old.x + (T(1) - alpha) * P;
      h = alpha * old.y + (T(1) - alpha) * h;
    }
    O[rr] = T2{P, h};
  }

  // send every message of the rows (of colour c when c >= 0): in-messages from
  // B (cached ones for CACHE > 0), out-messages into O
  __device__ void send(const SmallArgs &a, const T2 *B, T2 *O, int c, bool damp, T alpha,
                       bool &brk) const {
    const T *ac = (const T *)a.acoef;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      if (!ok[r] || (c >= 0 && colr[r] != c)) continue;
      if (CACHE > 0 && CACHE <= 4 && deg[0] <= CACHE) {
        // all cavities and factors first, without branches, so the divisions
        // of the row's slots overlap instead of running one after another
        // (a slot beyond the row's degree divides 0 by 1 and stores nothing;
        // with eight slots the three arrays would not fit the registers)
        T pin[CS], hin[CS], f[CS];
#pragma unroll
        for (int k = 0; k < CS; ++k) {
          const bool on = k < deg[0];
          const T2 m = on ? B[s0[0] + k] : T2{T(0), T(0)};
          pin[k] = m.x;
          hin[k] = m.y;
          const T cav = on ? S[0] - m.x : T(1);
          if (on && cav == T(0)) brk = true;
          f[k] = -av[k] / cav;
        }
#pragma unroll
        for (int k = 0; k < CS; ++k)
          if (k < deg[0]) {
            T P = f[k] * av[k];
            T h = f[k] * (H[0] - hin[k]);
            if (damp) {
              const T2 old = B[rv[k]];
              P = alpha * old.x + (T(1) - alpha) * P;
              h = alpha * old.y + (T(1) - alpha) * h;
            }
            O[rv[k]] = T2{P, h};
          }
      } else if (CACHE > 0 && deg[0] <= CACHE) {
#pragma unroll
        for (int k = 0; k < CS; ++k)
          if (k < deg[0]) {
            const T2 m = B[s0[0] + k];
            emit(B, O, rv[k], av[k], m.x, m.y, S[0], H[0], damp, alpha, brk);
          }
      } else {
        for (int k = 0; k < deg[r]; ++k) {
          const int e = slot0 + s0[r] + k;
          const T2 m = B[s0[r] + k];
          emit(B, O, a.rev[e] - slot0, ac[e], m.x, m.y, S[r], H[r], damp, alpha, brk);
        }
      }
    }
  }
};

// Largest instance state the launch must hold in LDS.
__host__ __device__ inline size_t small_lds_bytes(int emax, int nmax, int tsz, bool col) {
  const size_t msg = (size_t)(col ? 1 : 2) * (size_t)emax * 2 * (size_t)tsz;
  return ((msg + 15) & ~(size_t)15) + (size_t)nmax * 8;
}

template <typename T, int RM, int CACHE, bool COL>
__global__ __launch_bounds__(1024) void k_small_batch(SmallArgs a) {
  using T2 = typename Vec2<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sh_q;
  __shared__ double red[16 * 8];
  const size_t mbytes = (size_t)(COL ? 1 : 2) * a.emax * sizeof(T2);
  T2 *buf0 = (T2 *)smem;
  T2 *buf1 = COL ? buf0 : buf0 + a.emax;
  double *xs = (double *)(smem + ((mbytes + 15) & ~(size_t)15));
  const int NT = blockDim.x, tid = threadIdx.x;
  T2 *gmsg = (T2 *)a.msg;
  T *grhs = (T *)a.rhsT;
  const T alpha = (T)a.alpha;
  const bool damp = a.alpha > 0.0;

  for (;;) {
    if (tid == 0) sh_q = (int)atomicAdd(a.queue, 1u);
    __syncthreads();
    const int q = sh_q;
    __syncthreads();
    if (q >= a.count) break;
    const int t = a.order[q];
    const SmallInst I = a.inst[t];
    Rows<T, RM, CACHE> R;
    R.load(a, I);
    const int ncol = COL ? I.ncol : 1;

    if (a.mode == SMALL_RESET) {
      for (int e = tid; e < I.E; e += NT) gmsg[I.slot0 + e] = T2{T(0), T(0)};
      for (int i = tid; i < I.n; i += NT) grhs[I.node0 + i] = (T)a.b[I.node0 + i];
      continue;
    }

    // messages into LDS (trajectory: the stored state; solve: zeros)
    for (int e = tid; e < I.E; e += NT)
      buf0[e] = a.mode == SMALL_SWEEPS ? gmsg[I.slot0 + e] : T2{T(0), T(0)};
    int cur = 0;
    auto bufp = [&](int k) { return k ? buf1 : buf0; };

    if (a.mode == SMALL_SWEEPS) {
#pragma unroll
      for (int r = 0; r < RM; ++r)
        if (R.ok[r]) R.rhs[r] = grhs[I.node0 + tid + r * NT];
      __syncthreads();
      bool brk = false;
      for (int sw = 0; sw < a.nsweeps; ++sw) {
        if (!COL) {
          R.sums(bufp(cur), -1);
          R.send(a, bufp(cur), bufp(cur ^ 1), -1, damp, alpha, brk);
          __syncthreads();
          cur ^= 1;
        } else {
          for (int c = 0; c < ncol; ++c) {
            R.sums(buf0, c);
            R.send(a, buf0, buf0, c, damp, alpha, brk);
            __syncthreads();
          }
        }
      }
      for (int e = tid; e < I.E; e += NT) gmsg[I.slot0 + e] = bufp(cur)[e];
      continue;
    }

    // ---- SMALL_SOLVE ----
    SmallStat st{};
    st.status = GABP_NOT_CONVERGED;
    double bq = 0.0;
    // per row: the candidate means y and residual res of the last check in
    // registers; the accumulated corrections in x and the sample history
    // (previous means, Aitken's two older samples, Steffensen's three) in the
    // plan's FP64 history arrays, touched only at checks
    double y[RM], res[RM];
    const int Nall = a.nodes;
    double *hx = a.hist, *ha = a.hist + Nall, *hb = a.hist + 2 * (size_t)Nall;
    double *s0h = a.hist + 3 * (size_t)Nall, *s1h = a.hist + 4 * (size_t)Nall,
           *s2h = a.hist + 5 * (size_t)Nall;
#pragma unroll
    for (int r = 0; r < RM; ++r) {
      const int g = I.node0 + tid + r * NT;
      const double bv = R.ok[r] ? a.b[g] : 0.0;
      R.rhs[r] = (T)bv;
      bq += bv * bv;
      y[r] = res[r] = 0.0;
      if (R.ok[r]) a.x[g] = 0.0;
    }
    {
      double m0 = 0.0, m1 = 0.0;
      bool f0 = false, f1 = false;
      block_reduce(bq, m0, m1, f0, f1, red);  // also orders the LDS zeroing above
    }
    const double bn = sqrt(bq);
    if (I.n == 0 || bn == 0.0 || !isfinite(bn)) {
      st.status = (I.n == 0 || bn == 0.0) ? GABP_OK : GABP_ERR_ARG;
#pragma unroll
      for (int r = 0; r < RM; ++r)
        if (R.ok[r]) a.x[I.node0 + tid + r * NT] = 0.0;
    } else {
      const int ce = a.accel == GABP_ACCEL_AITKEN ? a.stride : a.check_every;
      const int s2 = a.cycle - 2 * a.stride, s1 = a.cycle - a.stride;
      double rel_prev = 1.0, last_d = 0.0;
      double target = fmin(0.5, fmax(0.3 * a.tol, a.floor));
      int in_pass = 0, nsamp = 0, stall = 0;
      bool brk = false;
      for (;;) {
        const bool steff = a.accel == GABP_ACCEL_STEFFENSEN;
        const bool seed = in_pass == 0;
        const bool chk = steff ? in_pass == a.cycle : (!seed && in_pass % ce == 0);
        const int sidx = !steff ? -1
                         : (in_pass == s2 ? 0 : in_pass == s1 ? 1 : in_pass == a.cycle ? 2 : -1);
        const bool need = seed || chk || sidx >= 0;
        if (!COL || need) R.sums(bufp(cur), -1);
        if (need) {
          // means of the current messages (FP64 from the working precision)
          double d = 0.0, xm = 0.0;
          bool nf = false, zs = false;
          double xv[RM];
#pragma unroll
          for (int r = 0; r < RM; ++r) {
            xv[r] = 0.0;
            if (!R.ok[r]) continue;
            if (R.S[r] == T(0)) zs = true;
            xv[r] = (double)R.H[r] / (double)R.S[r];
            if (!isfinite(xv[r])) nf = true;
          }
          if (seed) {
#pragma unroll
            for (int r = 0; r < RM; ++r)
              if (R.ok[r]) {
                const int g = I.node0 + tid + r * NT;
                hx[g] = xv[r];
                hb[g] = xv[r];
              }
            nsamp = 0;
          }
          // Steffensen's three samples of the cycle
          if (sidx >= 0) {
            double *dst = sidx == 0 ? s0h : sidx == 1 ? s1h : s2h;
#pragma unroll
            for (int r = 0; r < RM; ++r)
              if (R.ok[r]) dst[I.node0 + tid + r * NT] = xv[r];
          }
          if (chk) {
            // candidate means of this pass: x, or Aitken's extrapolation
#pragma unroll
            for (int r = 0; r < RM; ++r) {
              if (!R.ok[r]) continue;
              const int g = I.node0 + tid + r * NT;
              d = fmax(d, fabs(xv[r] - hx[g]));
              xm = fmax(xm, fabs(xv[r]));
              hx[g] = xv[r];
              if (a.accel == GABP_ACCEL_AITKEN) {
                const double x0 = ha[g], x1 = hb[g];
                y[r] = nsamp >= 1 ? aitken(x0, x1, xv[r]) : xv[r];
                ha[g] = x1;
                hb[g] = xv[r];
              } else if (steff) {
                y[r] = aitken(s0h[g], s1h[g], s2h[g]);
              } else {
                y[r] = xv[r];
              }
              if (!isfinite(y[r])) nf = true;
              xs[tid + r * NT] = a.x[g] + y[r];
            }
            ++nsamp;
            __syncthreads();
            // FP64 residual of x + y over the caller's CSR rows
            double sq = 0.0;
#pragma unroll
            for (int r = 0; r < RM; ++r) {
              if (!R.ok[r]) continue;
              const int g = I.node0 + tid + r * NT;
              double acc = a.b[g];
              for (int64_t k = a.rp[g]; k < a.rp[g + 1]; ++k)
                acc -= a.val[k] * xs[a.col[k] - I.node0];
              res[r] = acc;
              sq += acc * acc;
            }
            bool bad = nf, zz = zs || brk;
            block_reduce(sq, d, xm, bad, zz, red);
            ++st.checks;
            const double rel = sqrt(sq) / bn;
            st.rel = rel;
            st.rnorm = sqrt(sq);
            if (zz) { st.status = GABP_ERR_BREAKDOWN; break; }
            if (bad || !isfinite(rel) || rel > 1e6) { st.status = GABP_ERR_DIVERGED; break; }
            if (rel <= a.tol) { st.status = GABP_OK; break; }
            // end of an inner solve (a refinement pass)?
            const double relc = d / fmax(xm, 1e-300);
            const double qr = last_d > 0.0 ? d / last_d : 1.0;
            const double est = qr < 1.0 ? relc * qr / (1.0 - qr) : 1e300;
            last_d = d;
            bool end = false;
            if (steff) {
              end = true;
            } else if (a.inner_tol >= 0.0) {
              if (relc == 0.0 || est <= target) end = true;
              stall = (relc < a.floor && qr > 0.7) ? stall + 1 : 0;
              if (stall >= 2) end = true;
            }
            if (end) {
              if (st.restarts >= a.max_restarts) break;
              // x += the pass's candidate; its residual is the next right-hand
              // side; information messages restart from zero, precisions kept
#pragma unroll
              for (int r = 0; r < RM; ++r) {
                if (R.ok[r]) a.x[I.node0 + tid + r * NT] += y[r];
                y[r] = 0.0;  // the new pass has no candidate yet
                R.rhs[r] = (T)res[r];
              }
              T2 *B = bufp(cur);
#pragma unroll
              for (int r = 0; r < RM; ++r)
                if (R.ok[r])
                  for (int k = 0; k < R.deg[r]; ++k) B[R.s0[r] + k].y = T(0);
              ++st.restarts;
              rel_prev = rel;
              target = a.inner_tol > 0.0 ? a.inner_tol
                                         : fmin(0.5, fmax(0.3 * a.tol / rel_prev, a.floor));
              in_pass = 0;
              last_d = 0.0;
              stall = 0;
              __syncthreads();
              continue;
            }
          }
        }
        if (st.sweeps >= a.max_sweeps) break;
        // one sweep
        if (!COL) {
          R.send(a, bufp(cur), bufp(cur ^ 1), -1, damp, alpha, brk);
          __syncthreads();
          cur ^= 1;
        } else {
          for (int c = 0; c < ncol; ++c) {
            R.sums(buf0, c);
            R.send(a, buf0, buf0, c, damp, alpha, brk);
            __syncthreads();
          }
        }
        ++st.sweeps;
        ++in_pass;
      }
      // x = the accumulated corrections plus the last candidate
#pragma unroll
      for (int r = 0; r < RM; ++r)
        if (R.ok[r]) a.x[I.node0 + tid + r * NT] += y[r];
#pragma unroll
      for (int r = 0; r < RM; ++r)
        if (R.ok[r]) grhs[I.node0 + tid + r * NT] = R.rhs[r];
    }
    __syncthreads();
    for (int e = tid; e < I.E; e += NT) gmsg[I.slot0 + e] = bufp(cur)[e];
    if (tid == 0) a.stat[t] = st;
    __syncthreads();
  }
}

template <typename T>
__global__ void k_small_marginals(int N, const int32_t *__restrict__ soff, const T *__restrict__ diag,
                                  const T *__restrict__ rhs,
                                  const typename Vec2<T>::type *__restrict__ msg,
                                  double *__restrict__ mean, double *__restrict__ prec) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  T s = diag[g], h = rhs[g];
  for (int e = soff[g]; e < soff[g + 1]; ++e) {
    s += msg[e].x;
    h += msg[e].y;
  }
  if (mean) mean[g] = (double)h / (double)s;
  if (prec) prec[g] = (double)s;
}

// CSR position k of row g (off-diagonal) <-> the in-slot holding the message
// g -> col[k]: the reverse of g's own in-slot for that neighbour.
template <typename T>
__global__ void k_small_messages(int N, const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                                 const int32_t *__restrict__ soff, const int32_t *__restrict__ rev,
                                 typename Vec2<T>::type *__restrict__ msg, double *__restrict__ P,
                                 double *__restrict__ h, int set) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  int o = soff[g];
  for (int64_t k = rp[g]; k < rp[g + 1]; ++k) {
    if (col[k] == g) {
      if (!set) { P[k] = 0.0; h[k] = 0.0; }
      continue;
    }
    const int dst = rev[o++];
    if (set) {
      msg[dst].x = (T)P[k];
      msg[dst].y = (T)h[k];
    } else {
      P[k] = (double)msg[dst].x;
      h[k] = (double)msg[dst].y;
    }
  }
}

// Every row's columns stay inside its own instance (block-diagonal matrix).
__global__ void k_small_blocks(int N, int count, const int32_t *__restrict__ node_off,
                               const int64_t *__restrict__ rp, const int32_t *__restrict__ col,
                               uint32_t *__restrict__ flags) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= N) return;
  int lo = 0, hi = count - 1;  // last instance whose first node is <= g
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (node_off[mid] <= g) lo = mid;
    else hi = mid - 1;
  }
  const int b = node_off[lo], e = node_off[lo + 1];
  for (int64_t k = rp[g]; k < rp[g + 1]; ++k)
    if (col[k] < b || col[k] >= e) {
      atomicOr(flags, FLAG_ARG);
      return;
    }
}

template <typename T, int RM, int CACHE, bool COL>
const void *small_kernel() {
  return (const void *)&k_small_batch<T, RM, CACHE, COL>;
}

const void *pick_small(const SmallArgs &a) {
  const bool c = a.colored;
  const bool d4 = a.cache && a.maxdeg <= 4;  // rows of degree <= 4: four slots in registers
  if (a.fp32) {
    if (a.rows_per_thread == 1 && d4)
      return c ? small_kernel<float, 1, 4, true>() : small_kernel<float, 1, 4, false>();
    if (a.rows_per_thread == 1)
      return c ? small_kernel<float, 1, 8, true>() : small_kernel<float, 1, 8, false>();
    return c ? small_kernel<float, 4, 0, true>() : small_kernel<float, 4, 0, false>();
  }
  if (a.rows_per_thread == 1 && d4)
    return c ? small_kernel<double, 1, 4, true>() : small_kernel<double, 1, 4, false>();
  if (a.rows_per_thread == 1)
    return c ? small_kernel<double, 1, 8, true>() : small_kernel<double, 1, 8, false>();
  return c ? small_kernel<double, 4, 0, true>() : small_kernel<double, 4, 0, false>();
}

}  // namespace

size_t small_lds(const SmallArgs &a) {
  return small_lds_bytes(a.emax, a.nmax, a.fp32 ? 4 : 8, a.colored);
}

int small_occupancy(const SmallArgs &a) {
  const void *k = pick_small(a);
  const size_t lds = small_lds(a);
  if (lds > 65536) {
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, a.threads, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

hipError_t launch_small_batch(const SmallArgs &a, hipStream_t s) {
  if (a.count <= 0 || a.grid <= 0) return hipSuccess;
  const void *k = pick_small(a);
  const size_t lds = small_lds(a);
  if (lds > 65536) {
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();  // optional: the launch below reports what matters
  }
  SmallArgs arg = a;
  void *params[] = {&arg};
  return hipLaunchKernel(k, dim3(a.grid), dim3(a.threads), params, lds, s);
}

hipError_t launch_small_marginals(const SmallArgs &a, int N, double *mean, double *prec,
                                  hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const dim3 grid((N + kBlock - 1) / kBlock);
  if (a.fp32)
    hipLaunchKernelGGL(k_small_marginals<float>, grid, dim3(kBlock), 0, s, N, a.soff,
                       (const float *)a.diagT, (const float *)a.rhsT, (const float2 *)a.msg, mean,
                       prec);
  else
    hipLaunchKernelGGL(k_small_marginals<double>, grid, dim3(kBlock), 0, s, N, a.soff,
                       (const double *)a.diagT, (const double *)a.rhsT, (const double2 *)a.msg,
                       mean, prec);
  return hipGetLastError();
}

hipError_t launch_small_messages(const SmallArgs &a, int N, double *P, double *h, bool set,
                                 hipStream_t s) {
  if (N <= 0) return hipSuccess;
  const dim3 grid((N + kBlock - 1) / kBlock);
  if (a.fp32)
    hipLaunchKernelGGL(k_small_messages<float>, grid, dim3(kBlock), 0, s, N, a.rp, a.col, a.soff,
                       a.rev, (float2 *)a.msg, P, h, set ? 1 : 0);
  else
    hipLaunchKernelGGL(k_small_messages<double>, grid, dim3(kBlock), 0, s, N, a.rp, a.col, a.soff,
                       a.rev, (double2 *)a.msg, P, h, set ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_small_blocks(int N, int count, const int32_t *node_off, const int64_t *rp,
                               const int32_t *col, uint32_t *flags, hipStream_t s) {
  if (N <= 0 || count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_small_blocks, dim3((N + kBlock - 1) / kBlock), dim3(kBlock), 0, s, N,
                     count, node_off, rp, col, flags);
  return hipGetLastError();
}

}  // namespace gabp
