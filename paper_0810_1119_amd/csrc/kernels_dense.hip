// Batches of small dense instances in one persistent launch: the section VII
// bipartite detector and dense symmetric matrices.
//
// Each workgroup repeatedly takes the next instance from a queue sorted by
// size (largest first) and solves it alone: every sweep, mean check, the
// switch to settled precisions and the FP64 refinement passes run inside the
// workgroup, with the node totals in LDS and the per-entry message state
// streamed from memory.  No host round trip happens between sweeps and
// instances of very different sizes finish independently.
//
// One instance is a rows x cols block of couplings a_rc.  Entry (r, c) is the
// undirected edge between row node r and column node c and holds both of its
// messages in the information form (P, h = P mu):
//     (P_rc, h_rc)  row -> column          (P_cr, h_cr)  column -> row.
// Bipartite: rows are chips (A_rr = -sigma2), columns users (A_cc = 1).
// Dense: rows and columns are the same nodes and only entries r < c (the
// upper triangle) carry edges; the diagonal entries are A_ii.
//
// A sweep is Algorithm 2 (section V) in this form: from the totals of the
// previous sweep, S_i = A_ii + sum of in-precisions and H_i = b_i + sum of
// in-informations, each entry computes
//     P_rc = -a^2 / (S_r - P_cr),  h_rc = -a (H_r - h_cr) / (S_r - P_cr)
// (eq. prec_message / mean_message with the reverse message subtracted) and
// the same for c -> r; the new totals are the sums of the new in-messages.
// Lane l of a wavefront handles columns l, l + 64, ... of one row at a time:
// row sums are wavefront reductions, column sums stay in registers across the
// wavefront's rows and are then added over the wavefronts in a fixed order,
// so every sum, and therefore every result, is deterministic.
#include "device_common.h"
#include "gabp_internal.h"

namespace gabp {
namespace {

template <typename T> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };

enum { SK_FULL = 0, SK_FREEZE = 1, SK_FROZEN = 2 };

// Wavefront reductions with DPP row moves (no lane-index registers, unlike
// lane shuffles, which matters in a kernel this long): within each 16-lane row
// swap neighbours (quad_perm [1,0,3,2], [2,3,0,1]), then mirror half rows and
// rows, so every lane of a row holds the row's total; the four row totals are
// read as scalars and added in a fixed order.  The result is uniform and
// independent of timing.  All 64 lanes must be active.
enum : int { DPP_XOR1 = 0xB1, DPP_XOR2 = 0x4E, DPP_ROW_MIRROR = 0x140, DPP_HALF_MIRROR = 0x141 };

template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)b, CTRL, 0xF, 0xF, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_mov_dpp((int)(unsigned)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float lane_value(float v, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ __forceinline__ double lane_value(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <typename T>
__device__ __forceinline__ T wsum64(T v) {
  v += dpp<DPP_XOR1>(v);
  v += dpp<DPP_XOR2>(v);
  v += dpp<DPP_HALF_MIRROR>(v);
  v += dpp<DPP_ROW_MIRROR>(v);
  return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

template <typename T>
__device__ __forceinline__ T wmax64(T v) {
  v = fmax(v, dpp<DPP_XOR1>(v));
  v = fmax(v, dpp<DPP_XOR2>(v));
  v = fmax(v, dpp<DPP_HALF_MIRROR>(v));
  v = fmax(v, dpp<DPP_ROW_MIRROR>(v));
  return fmax(fmax(lane_value(v, 0), lane_value(v, 16)), fmax(lane_value(v, 32), lane_value(v, 48)));
}

// threadIdx.x, hidden from the optimizer.  Per-thread addresses derived from
// it are then recomputed at each loop instead of being hoisted to the start of
// the persistent kernel, where dozens of them would stay live (in vector
// registers) across every sweep.  The empty asm emits no instruction.
__device__ __forceinline__ int thread_id() {
  int v = (int)threadIdx.x;
  asm volatile("" : "+v"(v));
  return v;
}

template <typename T>
struct Inst {
  int R, C;                             // rows, cols
  const T *M;                           // couplings, message precision
  const double *M64;                    // couplings, FP64
  typename V4<T>::type *st;             // full state per entry
  typename Vec2<T>::type *fc, *fh;      // settled phase: coefficients, informations
  T rdiag;                              // bipartite: A_rr of a chip (-sigma2)
};

template <typename T>
struct Lds {
  typename Vec2<T>::type *tot_row;      // bipartite: chip totals; dense: row sums
  typename Vec2<T>::type *tot_col;      // column-node totals (dense: every node)
  typename Vec2<T>::type *colpart;      // [waves][cols] column partial sums
  T *b_row, *b_col, *xprev, *diag;
  double *red;                          // [waves][8] reduction scratch
  double *xs, *u, *part, *rk;           // FP64 residual scratch (aliases colpart)
};

// One synchronous sweep over an instance (all threads of the workgroup call).
//   SK_FULL:   recompute precisions and informations.
//   SK_FREEZE: store c_rc = -a / (S_r - P_cr), c_cr likewise, and the new
//              informations; the precision totals S stay as they are.
//   SK_FROZEN: informations only, h_rc = c_rc (H_r - h_cr).
// dp / pm: largest change and size of a precision message (SK_FULL only);
// brk: a cavity precision was exactly zero.
template <typename T, int MAXM, int KIND, int SK>
__device__ void sweep(const Inst<T> &in, const Lds<T> &L, bool fresh, bool zero_h, bool damp,
                      T alpha, T &dp, T &pm, bool &brk, int W) {
  using T2 = typename Vec2<T>::type;
  using T4 = typename V4<T>::type;
  // the wavefront index is uniform: keeping it scalar puts the row addressing
  // in scalar registers and leaves each lane a 32-bit column offset
  const int lane = thread_id() & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int R = in.R, C = in.C;
  T cS[MAXM], cH[MAXM], aP[MAXM], aH[MAXM];
#pragma unroll
  for (int m = 0; m < MAXM; ++m) {
    const int c = lane + 64 * m;
    const T2 v = c < C ? L.tot_col[c] : T2{T(0), T(0)};
    cS[m] = v.x;
    cH[m] = v.y;
    aP[m] = T(0);
    aH[m] = T(0);
  }
  const T beta = T(1) - alpha;
#pragma unroll 1
  for (int r = wave; r < R; r += W) {
    const T2 rt = KIND == GABP_BATCH_BIPARTITE ? L.tot_row[r] : L.tot_col[r];
    const size_t base = (size_t)r * (size_t)C;
    T av[MAXM];
    T4 sv[MAXM];
    T2 cv[MAXM], hv[MAXM];
    // issue every load of the row before any arithmetic
#pragma unroll
    for (int m = 0; m < MAXM; ++m) {
      const int c = lane + 64 * m;
      const bool act = c < C && (KIND == GABP_BATCH_BIPARTITE || c > r);
      if (SK == SK_FROZEN) {
        cv[m] = act ? in.fc[base + c] : T2{T(0), T(0)};
        hv[m] = (act && !zero_h) ? in.fh[base + c] : T2{T(0), T(0)};
      } else {
        av[m] = act ? in.M[base + c] : T(0);
        sv[m] = (act && !fresh) ? in.st[base + c] : T4{T(0), T(0), T(0), T(0)};
      }
    }
    T sP = T(0), sH = T(0);
#pragma unroll
    for (int m = 0; m < MAXM; ++m) {
      const int c = lane + 64 * m;
      const bool act = c < C && (KIND == GABP_BATCH_BIPARTITE || c > r);
      if (!act) continue;
      if (SK == SK_FROZEN) {
        const T2 k = cv[m], h = hv[m];
        T hrc = k.x * (rt.y - h.y);
        T hcr = k.y * (cH[m] - h.x);
        if (damp) {
          hrc = alpha * h.x + beta * hrc;
          hcr = alpha * h.y + beta * hcr;
        }
        aH[m] += hrc;
        sH += hcr;
        in.fh[base + c] = T2{hrc, hcr};
        continue;
      }
      const T a = av[m];
      T4 o = sv[m];
      if (zero_h) {
        o.y = T(0);
        o.w = T(0);
      }
      if (a == T(0)) {  // no edge: nothing is sent either way
        if (SK == SK_FREEZE) {
          in.fc[base + c] = T2{T(0), T(0)};
          in.fh[base + c] = T2{T(0), T(0)};
        }
        continue;
      }
      const T dr = rt.x - o.z;     // precision of r without c's message
      const T dc = cS[m] - o.x;    // precision of c without r's message
      if (dr == T(0) || dc == T(0)) brk = true;
      const T ir = T(1) / dr, ic = T(1) / dc;
      if (SK == SK_FREEZE) {
        const T krc = -a * ir, kcr = -a * ic;
        T hrc = krc * (rt.y - o.w);
        T hcr = kcr * (cH[m] - o.y);
        if (damp) {
          hrc = alpha * o.y + beta * hrc;
          hcr = alpha * o.w + beta * hcr;
        }
        in.fc[base + c] = T2{krc, kcr};
        in.fh[base + c] = T2{hrc, hcr};
        aH[m] += hrc;
        sH += hcr;
      } else {
        const T aa = a * a;
        T4 nw;
        nw.x = -aa * ir;
        nw.y = -a * (rt.y - o.w) * ir;
        nw.z = -aa * ic;
        nw.w = -a * (cH[m] - o.y) * ic;
        if (damp) {
          nw.x = alpha * o.x + beta * nw.x;
          nw.y = alpha * o.y + beta * nw.y;
          nw.z = alpha * o.z + beta * nw.z;
          nw.w = alpha * o.w + beta * nw.w;
        }
        dp = fmax(dp, fmax(fabs(nw.x - o.x), fabs(nw.z - o.z)));
        pm = fmax(pm, fmax(fabs(nw.x), fabs(nw.z)));
        aP[m] += nw.x;
        aH[m] += nw.y;
        sP += nw.z;
        sH += nw.w;
        in.st[base + c] = nw;
      }
    }
    sH = wsum64(sH);
    if (SK == SK_FULL) sP = wsum64(sP);
    if (lane == 0) {
      if (KIND == GABP_BATCH_BIPARTITE) {
        if (SK == SK_FULL) L.tot_row[r] = T2{in.rdiag + sP, L.b_row[r] + sH};
        else L.tot_row[r].y = L.b_row[r] + sH;
      } else {
        L.tot_row[r] = T2{sP, sH};
      }
    }
  }
#pragma unroll
  for (int m = 0; m < MAXM; ++m) {
    const int c = lane + 64 * m;
    if (c < C) L.colpart[wave * C + c] = T2{aP[m], aH[m]};
  }
  __syncthreads();
  for (int c = thread_id(); c < C; c += blockDim.x) {
    T P = T(0), H = T(0);
    for (int w = 0; w < W; ++w) {
      const T2 v = L.colpart[w * C + c];
      P += v.x;
      H += v.y;
    }
    if (KIND == GABP_BATCH_BIPARTITE) {
      if (SK == SK_FULL) L.tot_col[c] = T2{T(1) + P, L.b_col[c] + H};
      else L.tot_col[c].y = L.b_col[c] + H;
    } else {
      const T2 ra = L.tot_row[c];
      if (SK == SK_FULL) L.tot_col[c] = T2{L.diag[c] + ra.x + P, L.b_col[c] + ra.y + H};
      else L.tot_col[c].y = L.b_col[c] + ra.y + H;
    }
  }
  __syncthreads();
}

// One half of a coloured sweep of a bipartite instance (all threads call).
// Rows (chips) and columns (users) are the two colour classes of the
// section VII graph: PH 1 lets every row send, PH 2 every column, each from
// the newest messages of the other class, so one sweep (PH 1 then PH 2) is
// the serial scheme of section III-C in this order.  Storage of an instance
// with entry e = r C + c in the coloured layout:
//   full state:  rc[e] = (P_rc, h_rc), then cr[e] = (P_cr, h_cr)  (T2 arrays)
//   settled:     k_rc[e], then k_cr[e] (coefficients); h_rc[e], then h_cr[e]
// PH 1 rebuilds the column totals from the new row -> column messages and
// PH 2 the row totals from the new column -> row messages.  want_dp: track
// the largest precision change (a check sweep).
template <typename T, int MAXM, int SK, int PH>
__device__ void sweep_rb(const Inst<T> &in, const Lds<T> &L, bool fresh, bool zero_h, bool damp,
                         bool want_dp, T alpha, T &dp, T &pm, bool &brk, int W) {
  using T2 = typename Vec2<T>::type;
  const int lane = thread_id() & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int R = in.R, C = in.C;
  const size_t RC = (size_t)R * (size_t)C;
  T2 *own2 = nullptr, *rev2 = nullptr;  // full state: the sent and the received direction
  T *kown = nullptr, *hown = nullptr, *hrev = nullptr;
  if constexpr (SK == SK_FULL || SK == SK_FREEZE) {
    T2 *const rc = (T2 *)in.st;
    own2 = PH == 1 ? rc : rc + RC;
    rev2 = PH == 1 ? rc + RC : rc;
  }
  if constexpr (SK != SK_FULL) {
    T *const k = (T *)in.fc;
    T *const h = (T *)in.fh;
    kown = PH == 1 ? k : k + RC;
    hown = PH == 1 ? h : h + RC;
    hrev = PH == 1 ? h + RC : h;
  }
  T cS[MAXM], cH[MAXM], aP[MAXM], aH[MAXM];
#pragma unroll
  for (int m = 0; m < MAXM; ++m) {
    const int c = lane + 64 * m;
    cS[m] = T(0);
    cH[m] = T(0);
    if (PH == 2 && c < C) {
      const T2 v = L.tot_col[c];
      cS[m] = v.x;
      cH[m] = v.y;
    }
    aP[m] = T(0);
    aH[m] = T(0);
  }
  const T beta = T(1) - alpha;
  const bool read_old = damp || (SK == SK_FULL && want_dp);
  // Two rows per wavefront and iteration, with the loads of both in flight
  // together: a half sweep moves half the bytes per entry of a synchronous
  // sweep, and one row at a time would leave the memory pipeline half idle.
  // Wavefront w still visits rows w, w + W, w + 2W, ... in that order, so
  // every sum keeps its order.  Wide rows hold enough loads in flight alone
  // (and two of them would not fit the registers).
  constexpr int NR = MAXM * (int)sizeof(T) > 16 ? 1 : (SK == SK_FROZEN ? 4 : 2);
#pragma unroll 1
  for (int r0 = wave; r0 < R; r0 += NR * W) {
    T2 rt[NR];
    T av[NR][MAXM];
    T2 rv[NR][MAXM], ov[NR][MAXM];  // received (reverse) message, own previous message
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int r = r0 + q * W;
      const bool rok = r < R;  // uniform
      const size_t base = (size_t)r * (size_t)C;
      rt[q] = T2{T(0), T(0)};
      if (PH == 1 && rok) rt[q] = L.tot_row[r];
#pragma unroll
      for (int m = 0; m < MAXM; ++m) {
        const int c = lane + 64 * m;
        const bool act = rok && c < C;
        rv[q][m] = T2{T(0), T(0)};
        ov[q][m] = T2{T(0), T(0)};
        if constexpr (SK == SK_FROZEN) {
          av[q][m] = act ? kown[base + c] : T(0);  // the settled coefficient
          // informations zeroed by a restart are those not rewritten since:
          // the received ones in PH 1, the own ones in both halves
          if (act && !(PH == 1 && zero_h)) rv[q][m].y = hrev[base + c];
          if (act && damp && !zero_h) ov[q][m].y = hown[base + c];
        } else {
          av[q][m] = act ? in.M[base + c] : T(0);
          if (act && (PH == 2 || !fresh)) rv[q][m] = rev2[base + c];
          if (SK == SK_FREEZE && PH == 2 && act) rv[q][m].y = hrev[base + c];  // new, settled array
          if (PH == 1 && zero_h) rv[q][m].y = T(0);
          if (act && read_old && !fresh) ov[q][m] = own2[base + c];
          if (zero_h) ov[q][m].y = T(0);
        }
      }
    }
#pragma unroll
    for (int q = 0; q < NR; ++q) {
      const int r = r0 + q * W;
      if (r >= R) break;  // uniform
      const size_t base = (size_t)r * (size_t)C;
      T sP = T(0), sH = T(0);
#pragma unroll
      for (int m = 0; m < MAXM; ++m) {
        const int c = lane + 64 * m;
        if (c >= C) continue;
        const T tS = PH == 1 ? rt[q].x : cS[m];
        const T tH = PH == 1 ? rt[q].y : cH[m];
        if constexpr (SK == SK_FROZEN) {
          T h = av[q][m] * (tH - rv[q][m].y);
          if (damp) h = alpha * ov[q][m].y + beta * h;
          hown[base + c] = h;
          if (PH == 1) aH[m] += h;
          else sH += h;
          continue;
        }
        const T a = av[q][m];
        if (a == T(0)) {  // no edge: nothing is sent
          if constexpr (SK == SK_FREEZE) {
            kown[base + c] = T(0);
            hown[base + c] = T(0);
          }
          continue;
        }
        const T cav = tS - rv[q][m].x;  // precision of the sender without the receiver's message
        if (cav == T(0)) brk = true;
        const T inv = T(1) / cav;
        if constexpr (SK == SK_FREEZE) {
          const T k = -a * inv;
          T h = k * (tH - rv[q][m].y);
          if (damp) h = alpha * ov[q][m].y + beta * h;
          kown[base + c] = k;
          hown[base + c] = h;
          if (PH == 1) aH[m] += h;
          else sH += h;
        } else {
          T P = -(a * a) * inv;
          T h = -(a * (tH - rv[q][m].y)) * inv;
          if (damp) {
            P = alpha * ov[q][m].x + beta * P;
            h = alpha * ov[q][m].y + beta * h;
          }
          if (want_dp) {
            dp = fmax(dp, fabs(P - ov[q][m].x));
            pm = fmax(pm, fabs(P));
          }
          own2[base + c] = T2{P, h};
          if (PH == 1) {
            aP[m] += P;
            aH[m] += h;
          } else {
            sP += P;
            sH += h;
          }
        }
      }
      if (PH == 2) {
        sH = wsum64(sH);
        if (SK == SK_FULL) sP = wsum64(sP);
        if (lane == 0) {
          if (SK == SK_FULL) L.tot_row[r] = T2{in.rdiag + sP, L.b_row[r] + sH};
          else L.tot_row[r].y = L.b_row[r] + sH;
        }
      }
    }
  }
  if (PH == 1) {
#pragma unroll
    for (int m = 0; m < MAXM; ++m) {
      const int c = lane + 64 * m;
      if (c < C) L.colpart[wave * C + c] = T2{aP[m], aH[m]};
    }
    __syncthreads();
    for (int c = thread_id(); c < C; c += blockDim.x) {
      T P = T(0), H = T(0);
      for (int w = 0; w < W; ++w) {
        const T2 v = L.colpart[w * C + c];
        P += v.x;
        H += v.y;
      }
      if (SK == SK_FULL) L.tot_col[c] = T2{T(1) + P, L.b_col[c] + H};
      else L.tot_col[c].y = L.b_col[c] + H;
    }
  }
  __syncthreads();
}

// One sweep of either schedule.
template <typename T, int MAXM, int KIND, bool RB, int SK>
__device__ __forceinline__ void any_sweep(const Inst<T> &in, const Lds<T> &L, bool fresh,
                                          bool zero_h, bool damp, bool want_dp, T alpha, T &dp,
                                          T &pm, bool &brk, int W) {
  if constexpr (RB) {
    sweep_rb<T, MAXM, SK, 1>(in, L, fresh, zero_h, damp, want_dp, alpha, dp, pm, brk, W);
    sweep_rb<T, MAXM, SK, 2>(in, L, fresh, zero_h, damp, want_dp, alpha, dp, pm, brk, W);
  } else {
    sweep<T, MAXM, KIND, SK>(in, L, fresh, zero_h, damp, alpha, dp, pm, brk, W);
  }
}

// A value every lane holds identically, moved to scalar registers so the
// compiler treats it (and the control flow it decides) as uniform.
__device__ __forceinline__ double uniform(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Fixed-order sum over the workgroup; every thread returns the same value.
__device__ double block_sum(double v, double *red, int W) {
  v = wsum64(v);
  if ((threadIdx.x & 63) == 0) red[(threadIdx.x >> 6) * 8] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < W; ++w) s += red[w * 8];
  __syncthreads();
  return uniform(s);
}

// Workgroup maxima of v[0..3] and OR of `flag`; every thread gets the result.
__device__ void block_max4(double v[4], bool &flag, double *red, int W) {
#pragma unroll
  for (int j = 0; j < 4; ++j) v[j] = wmax64(v[j]);
  const bool f = __any(flag);
  if ((threadIdx.x & 63) == 0) {
    double *o = red + (threadIdx.x >> 6) * 8;
    o[0] = v[0]; o[1] = v[1]; o[2] = v[2]; o[3] = v[3];
    o[4] = f ? 1.0 : 0.0;
  }
  __syncthreads();
  bool any = false;
  for (int j = 0; j < 4; ++j) v[j] = 0.0;
  for (int w = 0; w < W; ++w) {
    const double *o = red + w * 8;
    for (int j = 0; j < 4; ++j) v[j] = fmax(v[j], o[j]);
    any = any || o[4] != 0.0;
  }
  for (int j = 0; j < 4; ++j) v[j] = uniform(v[j]);
  flag = __builtin_amdgcn_readfirstlane(any ? 1 : 0) != 0;
  __syncthreads();
}

// FP64 residual of the problem the instance solves, at x (FP64, global) or
// at x = 0 (x == NULL).  Bipartite: r = S^T (y - S x) - sigma2 x, the residual
// of (S^T S + sigma2 I) x = S^T y; dense: r = b - A x.  Leaves r in L.rk and
// returns ||r||^2 (the same in every thread).
template <typename T, int KIND>
__device__ double residual64(const Inst<T> &in, const Lds<T> &L, const double *x, const double *b,
                             double sigma2, int W) {
  const int NT = blockDim.x, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int R = in.R, C = in.C;
  const double *M = in.M64;
  if (C == 0) return 0.0;  // no unknowns: nothing to reduce (uniform exit)
  for (int c = thread_id(); c < C; c += NT) L.xs[c] = x ? x[c] : 0.0;
  __syncthreads();
  double sq = 0.0;
  if (KIND == GABP_BATCH_BIPARTITE) {
    for (int r = wave; r < R; r += W) {  // u = y - S x, one row per wavefront
      double acc = 0.0;
      for (int c = thread_id() & 63; c < C; c += 64) acc += M[(size_t)r * C + c] * L.xs[c];
      acc = wsum64(acc);
      if ((threadIdx.x & 63) == 0) L.u[r] = b[r] - acc;
    }
    __syncthreads();
    const int G = NT / C;  // row groups; the plan guarantees C <= NT
    {
      const int tid = thread_id(), g = tid / C, c = tid - g * C;
      if (g < G) {
        double acc = 0.0;
        for (int r = g; r < R; r += G) acc += M[(size_t)r * C + c] * L.u[r];
        L.part[g * C + c] = acc;
      }
    }
    __syncthreads();
    for (int c = thread_id(); c < C; c += NT) {
      double v = 0.0;
      for (int g = 0; g < G; ++g) v += L.part[g * C + c];
      v -= sigma2 * L.xs[c];
      L.rk[c] = v;
      sq += v * v;
    }
  } else {
    for (int r = wave; r < C; r += W) {
      double acc = 0.0;
      for (int c = thread_id() & 63; c < C; c += 64) acc += M[(size_t)r * C + c] * L.xs[c];
      acc = wsum64(acc);
      if ((threadIdx.x & 63) == 0) L.rk[r] = b[r] - acc;
    }
    __syncthreads();
    for (int c = thread_id(); c < C; c += NT) sq += L.rk[c] * L.rk[c];
  }
  return block_sum(sq, L.red, W);
}

// Whether any thread saw a zero cavity precision (uniform result).
__device__ __forceinline__ bool brk_any(bool brk, double *red, int W) {
  double v[4] = {0.0, 0.0, 0.0, 0.0};
  block_max4(v, brk, red, W);
  return brk;
}

// Node totals of all-zero messages: S = A_ii, H = b_i (Algorithm 1 step 1).
template <typename T, int KIND>
__device__ void init_totals(const Inst<T> &in, const Lds<T> &L) {
  using T2 = typename Vec2<T>::type;
  const int NT = blockDim.x;
  if (KIND == GABP_BATCH_BIPARTITE) {
    for (int r = thread_id(); r < in.R; r += NT) L.tot_row[r] = T2{in.rdiag, L.b_row[r]};
    for (int c = thread_id(); c < in.C; c += NT) L.tot_col[c] = T2{T(1), L.b_col[c]};
  } else {
    for (int c = thread_id(); c < in.C; c += NT) L.tot_col[c] = T2{L.diag[c], L.b_col[c]};
  }
  __syncthreads();
}

// The whole solve of one instance: refinement passes of inner GaBP solves
// (same rules as the single-system solver: stop on the estimated error of the
// means or on stagnation at the arithmetic's floor, switch to settled
// precisions, FP64 residual, restart with zeroed informations and kept
// precisions).
template <typename T, int MAXM, int KIND, bool RB>
__device__ DenseStat solve_instance(const DenseArgs &a, const DenseInst &I, const Inst<T> &in,
                                    const Lds<T> &L, int W) {
  using T2 = typename Vec2<T>::type;
  const int NT = blockDim.x;
  const int R = in.R, C = in.C;
  DenseStat s{};
  s.status = GABP_NOT_CONVERGED;
  double *xg = a.x + I.xoff;
  const double *bg = a.b + I.rhs;
  const double bn = sqrt(residual64<T, KIND>(in, L, nullptr, bg, I.sigma2, W));
  for (int c = thread_id(); c < C; c += NT) xg[c] = 0.0;
  if (C == 0 || bn == 0.0) {
    s.status = GABP_OK;
    return s;
  }
  if (!isfinite(bn)) {
    s.status = GABP_ERR_ARG;
    return s;
  }
  double alpha_d = a.alpha;
  bool damp = alpha_d > 0.0;
  T alpha = (T)alpha_d;
  int level = 0;  // damping escalations taken
  const int ce = a.check_every;
  bool fresh = true, zero_h = false, frozen = false, want_freeze = false;
  double rel_prev = 1.0;
  for (;;) {
    const double target = a.inner_tol > 0.0
                              ? a.inner_tol
                              : fmin(0.5, fmax(0.3 * a.tol / rel_prev, a.fp32 ? 1e-7 : 1e-15));
    double last_d = 0.0;
    int stall = 0, slow = 0, in_pass = 0;
    bool brk = false, nf = false, escalate = false;
    // the first check of the pass measures its change from the means of the
    // messages it starts from (not from zeros or another right-hand side)
    for (int c = thread_id(); c < C; c += NT) {
      const T2 t = L.tot_col[c];
      L.xprev[c] = t.x != T(0) ? t.y / t.x : T(0);
    }
    while (s.sweeps < a.max_sweeps) {
      T dp = T(0), pm = T(0);
      const bool check = (in_pass + 1) % ce == 0;
      if (frozen) {
        any_sweep<T, MAXM, KIND, RB, SK_FROZEN>(in, L, fresh, zero_h, damp, check, alpha, dp, pm,
                                                brk, W);
        ++s.frozen_sweeps;
      } else if (want_freeze && a.freeze) {
        any_sweep<T, MAXM, KIND, RB, SK_FREEZE>(in, L, fresh, zero_h, damp, check, alpha, dp, pm,
                                                brk, W);
        frozen = true;
        ++s.frozen_sweeps;
      } else {
        any_sweep<T, MAXM, KIND, RB, SK_FULL>(in, L, fresh, zero_h, damp, check, alpha, dp, pm,
                                              brk, W);
      }
      fresh = false;
      zero_h = false;
      ++s.sweeps;
      if (++in_pass % ce != 0) continue;
      // check of the means x = H / S of the unknowns
      double v[4] = {0.0, 0.0, (double)dp, (double)pm};  // d, max|x|, dp, pm
      for (int c = thread_id(); c < C; c += NT) {
        const T2 t = L.tot_col[c];
        if (t.x == T(0)) brk = true;
        const T xv = t.y / t.x;
        if (!isfinite(xv)) nf = true;
        v[0] = fmax(v[0], (double)fabs(xv - L.xprev[c]));
        v[1] = fmax(v[1], (double)fabs(xv));
        L.xprev[c] = xv;
      }
      bool bad = brk || nf;
      block_max4(v, bad, L.red, W);
      ++s.checks;
      const double d = v[0];
      const double relc = d / fmax(v[1], 1e-300);
      const double q = last_d > 0.0 ? d / last_d : 1.0;
      const double est = q < 1.0 ? relc * q / (1.0 - q) : 1e300;
      last_d = d;
      if (!frozen && a.freeze_tol > 0.0 && v[2] <= a.freeze_tol * v[3]) want_freeze = true;
      // an instance whose means turn non-finite or stop contracting runs the
      // pass again with more damping (the pass has not touched x yet)
      const bool can_raise = a.adapt && level < 3;
      if (bad) {
        escalate = can_raise && !brk_any(brk, L.red, W);
        break;
      }
      if (relc == 0.0 || est <= target) break;
      if (can_raise && in_pass >= 32) {
        slow = q >= 0.95 ? slow + 1 : 0;
        if (slow >= 8) {
          escalate = true;
          break;
        }
      }
      stall = (relc < a.floor && q > 0.7) ? stall + 1 : 0;
      if (stall >= 2) break;
    }
    if (escalate) {
      const double lv[3] = {0.3, 0.5, 0.7};
      alpha_d = fmax(a.alpha, lv[level]);
      ++level;
      damp = true;
      alpha = (T)alpha_d;
      fresh = true;
      zero_h = false;
      frozen = false;
      want_freeze = false;
      init_totals<T, KIND>(in, L);
      continue;
    }
    // flags of the whole pass, then x += H / S in FP64
    {
      double v[4] = {0.0, 0.0, 0.0, 0.0};
      bool f = brk;
      block_max4(v, f, L.red, W);
      brk = f;
      for (int c = thread_id(); c < C; c += NT) {
        const T2 t = L.tot_col[c];
        if (t.x == T(0)) nf = true;
        const double xv = (double)t.y / (double)t.x;
        if (!isfinite(xv)) nf = true;
        xg[c] += xv;
      }
      f = nf;
      block_max4(v, f, L.red, W);
      nf = f;
    }
    const double r2 = residual64<T, KIND>(in, L, xg, bg, I.sigma2, W);
    s.rnorm = sqrt(r2);
    s.rel = s.rnorm / bn;
    rel_prev = s.rel;
    if (brk) { s.status = GABP_ERR_BREAKDOWN; break; }
    if (nf || !isfinite(s.rel) || s.rel > 1e6) { s.status = GABP_ERR_DIVERGED; break; }
    if (s.rel <= a.tol) { s.status = GABP_OK; break; }
    if (s.restarts >= a.max_restarts || s.sweeps >= a.max_sweeps) {
      s.status = GABP_NOT_CONVERGED;
      break;
    }
    // restart: right-hand side from the residual, informations zeroed,
    // precisions (or settled coefficients) kept
    if (KIND == GABP_BATCH_BIPARTITE) {
      const double is2 = 1.0 / I.sigma2;
      for (int c = thread_id(); c < C; c += NT) {
        L.b_col[c] = (T)(L.rk[c] * is2);
        L.tot_col[c].y = L.b_col[c];
      }
      for (int r = thread_id(); r < R; r += NT) {
        L.b_row[r] = T(0);
        L.tot_row[r].y = T(0);
      }
    } else {
      for (int c = thread_id(); c < C; c += NT) {
        L.b_col[c] = (T)L.rk[c];
        L.tot_col[c].y = L.b_col[c];
      }
    }
    zero_h = true;
    ++s.restarts;
    __syncthreads();
  }
  s.damping = alpha_d;
  return s;
}

template <typename T, int MAXM, int KIND, bool RB>
__global__ __launch_bounds__(1024) void k_dense_batch(DenseArgs a) {
  using T2 = typename Vec2<T>::type;
  using T4 = typename V4<T>::type;
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ int sh_q;
  const DenseLds D = dense_lds(a.nr, a.nc, a.waves, (int)sizeof(T));
  Lds<T> L;
  L.tot_row = (T2 *)(smem + D.tot_row);
  L.tot_col = (T2 *)(smem + D.tot_col);
  L.colpart = (T2 *)(smem + D.uni);
  L.b_row = (T *)(smem + D.b_row);
  L.b_col = (T *)(smem + D.b_col);
  L.xprev = (T *)(smem + D.xprev);
  L.diag = (T *)(smem + D.diag);
  L.red = (double *)(smem + D.red);
  L.xs = (double *)(smem + D.uni);
  L.u = L.xs + a.nc;
  L.part = L.u + a.nr;
  L.rk = L.part + blockDim.x;
  const int NT = blockDim.x, W = a.waves;

  for (;;) {
    if (threadIdx.x == 0) sh_q = (int)atomicAdd(a.queue, 1u);
    __syncthreads();
    // uniform: instance fields then live in scalar registers
    const int q = __builtin_amdgcn_readfirstlane(sh_q);
    __syncthreads();
    if (q >= a.count) break;
    const int t = a.order[q];
    const DenseInst I = a.inst[t];
    Inst<T> in;
    in.R = I.rows;
    in.C = I.cols;
    in.M = (const T *)a.matT + I.mat;
    in.M64 = a.mat64 + I.mat;
    in.st = (T4 *)a.state + I.mat;
    in.fc = a.fcoef ? (T2 *)a.fcoef + I.mat : nullptr;
    in.fh = a.fh ? (T2 *)a.fh + I.mat : nullptr;
    in.rdiag = (T)(-I.sigma2);
    const int R = I.rows, C = I.cols;
    T2 *gtot = (T2 *)a.tot + I.node;
    T *gnb = (T *)a.nb + I.node;

    // node totals and right-hand side (reset without b: zero right-hand side)
    if (a.mode == DENSE_SWEEPS) {
      for (int c = thread_id(); c < C; c += NT) {
        L.tot_col[c] = gtot[c];
        L.b_col[c] = gnb[c];
        if (KIND == GABP_BATCH_DENSE) L.diag[c] = (T)in.M64[(size_t)c * C + c];
      }
      if (KIND == GABP_BATCH_BIPARTITE)
        for (int r = thread_id(); r < R; r += NT) {
          L.tot_row[r] = gtot[C + r];
          L.b_row[r] = gnb[C + r];
        }
    } else {
      if (KIND == GABP_BATCH_BIPARTITE) {
        for (int r = thread_id(); r < R; r += NT) {
          L.b_row[r] = a.b ? (T)a.b[I.rhs + r] : T(0);
          L.tot_row[r] = T2{in.rdiag, L.b_row[r]};
        }
        for (int c = thread_id(); c < C; c += NT) {
          L.b_col[c] = T(0);
          L.tot_col[c] = T2{T(1), T(0)};
        }
      } else {
        for (int c = thread_id(); c < C; c += NT) {
          L.diag[c] = (T)in.M64[(size_t)c * C + c];
          L.b_col[c] = a.b ? (T)a.b[I.rhs + c] : T(0);
          L.tot_col[c] = T2{L.diag[c], L.b_col[c]};
        }
      }
    }
    __syncthreads();

    if (a.mode == DENSE_SWEEPS) {
      T dp = T(0), pm = T(0);
      bool brk = false;
      for (int k = 0; k < a.nsweeps; ++k)
        any_sweep<T, MAXM, KIND, RB, SK_FULL>(in, L, a.fresh && k == 0, false, a.alpha > 0.0, false,
                                              (T)a.alpha, dp, pm, brk, W);
    } else if (a.mode == DENSE_SOLVE) {
      const DenseStat s = solve_instance<T, MAXM, KIND, RB>(a, I, in, L, W);
      if (threadIdx.x == 0) a.stat[t] = s;
    }

    // keep the node totals for marginals and trajectory access
    for (int c = thread_id(); c < C; c += NT) {
      gtot[c] = L.tot_col[c];
      gnb[c] = L.b_col[c];
    }
    if (KIND == GABP_BATCH_BIPARTITE)
      for (int r = thread_id(); r < R; r += NT) {
        gtot[C + r] = L.tot_row[r];
        gnb[C + r] = L.b_row[r];
      }
    __syncthreads();
  }
}

// Validation of every instance, the working-precision copy of the couplings
// and the count of directed messages per sweep.  One workgroup per instance.
template <int KIND>
__global__ __launch_bounds__(256) void k_dense_prepare(int count, DenseInst *inst,
                                                       const double *m64, float *m32,
                                                       uint32_t *flags) {
  __shared__ double red[4];
  for (int t = blockIdx.x; t < count; t += gridDim.x) {
    const DenseInst I = inst[t];
    const int R = I.rows, C = I.cols;
    const double *M = m64 + I.mat;
    const int64_t total = (int64_t)R * C;
    double cnt = 0.0;
    uint32_t f = 0;
    for (int64_t e = threadIdx.x; e < total; e += blockDim.x) {
      const double v = M[e];
      if (!isfinite(v)) f |= FLAG_ARG;
      if (m32) {
        const float w = (float)v;
        if (!isfinite(w)) f |= FLAG_ARG;
        m32[I.mat + e] = w;
      }
      const int r = (int)(e / C), c = (int)(e - (int64_t)r * C);
      if (KIND == GABP_BATCH_BIPARTITE) {
        if (v != 0.0) cnt += 2.0;
      } else if (r == c) {
        if (v == 0.0) f |= FLAG_ZERO_DIAG;
      } else {
        if (v != M[(int64_t)c * C + r]) f |= FLAG_ASYM;
        if (v != 0.0) cnt += 1.0;
      }
    }
    cnt = wsum64(cnt);
    const uint32_t any_arg = __any(f & FLAG_ARG) ? FLAG_ARG : 0u;
    const uint32_t any_zd = __any(f & FLAG_ZERO_DIAG) ? FLAG_ZERO_DIAG : 0u;
    const uint32_t any_as = __any(f & FLAG_ASYM) ? FLAG_ASYM : 0u;
    const int w = threadIdx.x >> 6;
    __shared__ uint32_t fl[4];
    if ((threadIdx.x & 63) == 0) {
      red[w] = cnt;
      fl[w] = any_arg | any_zd | any_as;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double s = 0.0;
      uint32_t ff = 0;
      for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
        s += red[k];
        ff |= fl[k];
      }
      inst[t].edges = (int64_t)s;
      flags[t] = ff;
    }
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_dense_marginals(int count, int kind,
                                                         const DenseInst *inst, const void *tot_,
                                                         double *mean, double *prec, int all) {
  using T2 = typename Vec2<T>::type;
  const T2 *tot = (const T2 *)tot_;
  for (int t = blockIdx.x; t < count; t += gridDim.x) {
    const DenseInst I = inst[t];
    const int64_t nodes = all ? (int64_t)I.cols + (kind == GABP_BATCH_BIPARTITE ? I.rows : 0)
                              : (int64_t)I.cols;
    const int64_t out = all ? I.node : I.xoff;
    for (int64_t i = threadIdx.x; i < nodes; i += blockDim.x) {
      const T2 v = tot[I.node + i];
      if (mean) mean[out + i] = (double)v.y / (double)v.x;
      if (prec) prec[out + i] = (double)v.x;
    }
  }
}

template <typename T, int KIND, bool RB>
const void *pick_m(int maxm) {
  switch (maxm) {
    case 1: return (const void *)k_dense_batch<T, 1, KIND, RB>;
    case 2: return (const void *)k_dense_batch<T, 2, KIND, RB>;
    case 4: return (const void *)k_dense_batch<T, 4, KIND, RB>;
    case 8: return (const void *)k_dense_batch<T, 8, KIND, RB>;
    default: return nullptr;
  }
}

template <typename T>
const void *pick_t(const DenseArgs &a) {
  if (a.kind == GABP_BATCH_DENSE)  // not two-colourable: synchronous only
    return a.colored ? nullptr : pick_m<T, GABP_BATCH_DENSE, false>(a.maxm);
  return a.colored ? pick_m<T, GABP_BATCH_BIPARTITE, true>(a.maxm)
                   : pick_m<T, GABP_BATCH_BIPARTITE, false>(a.maxm);
}

const void *pick(const DenseArgs &a) { return a.fp32 ? pick_t<float>(a) : pick_t<double>(a); }

size_t lds_bytes(const DenseArgs &a) {
  return (size_t)dense_lds(a.nr, a.nc, a.waves, a.fp32 ? 4 : 8).total;
}

}  // namespace

int dense_batch_occupancy(const DenseArgs &a) {
  const void *k = pick(a);
  if (!k) return 0;
  const size_t lds = lds_bytes(a);
  if (lds > 65536) {
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();  // optional: the occupancy query below decides
  }
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, a.waves * 64, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return nb;
}

hipError_t launch_dense_batch(const DenseArgs &a, hipStream_t s) {
  if (a.count <= 0 || a.grid <= 0) return hipSuccess;
  const void *k = pick(a);
  if (!k) return hipErrorInvalidValue;
  const size_t lds = lds_bytes(a);
  if (lds > 65536) {
    (void)hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipGetLastError();  // optional: the launch below reports what matters
  }
  DenseArgs arg = a;
  void *params[] = {&arg};
  return hipLaunchKernel(k, dim3(a.grid), dim3(a.waves * 64), params, lds, s);
}

hipError_t launch_dense_prepare(const DenseArgs &a, uint32_t *flags, hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  const dim3 grid((unsigned)std::min(a.count, 4096));
  DenseInst *inst = const_cast<DenseInst *>(a.inst);
  float *m32 = a.fp32 ? (float *)const_cast<void *>(a.matT) : nullptr;
  if (a.kind == GABP_BATCH_BIPARTITE)
    hipLaunchKernelGGL(k_dense_prepare<GABP_BATCH_BIPARTITE>, grid, dim3(256), 0, s, a.count, inst,
                       a.mat64, m32, flags);
  else
    hipLaunchKernelGGL(k_dense_prepare<GABP_BATCH_DENSE>, grid, dim3(256), 0, s, a.count, inst,
                       a.mat64, m32, flags);
  return hipGetLastError();
}

hipError_t launch_dense_marginals(const DenseArgs &a, double *mean, double *prec, bool all,
                                  hipStream_t s) {
  if (a.count <= 0) return hipSuccess;
  const dim3 grid((unsigned)std::min(a.count, 4096));
  if (a.fp32)
    hipLaunchKernelGGL(k_dense_marginals<float>, grid, dim3(256), 0, s, a.count, a.kind, a.inst,
                       a.tot, mean, prec, all ? 1 : 0);
  else
    hipLaunchKernelGGL(k_dense_marginals<double>, grid, dim3(256), 0, s, a.count, a.kind, a.inst,
                       a.tot, mean, prec, all ? 1 : 0);
  return hipGetLastError();
}

}  // namespace gabp
