// GaBP sweeps in the "pair" layout, gfx950: the broadcast form of the paper's
// Algorithm 2 (section V) mapped to memory.
//
// Every node i broadcasts its aggregate S_i = A_ii + sum_k P_ki and
// H_i = b_i + sum_k h_ki (h = P mu).  Slot e = (i, j) of row i keeps both
// directions of the edge: the message i -> j (P_ij, h_ij) that i sends and the
// message j -> i (P_ji, h_ji) that i receives.  From the neighbour's broadcast
// node i recomputes locally what j sends it, subtracting the message it sent j
// (the retrieval "by means of a subtraction" of section V):
//   P_ji' = -A_ij^2 / (S_j - P_ij),  h_ji' = -A_ij (H_j - h_ij) / (S_j - P_ij)
// and what it sends j:
//   P_ij' = -A_ij^2 / (S_i - P_ji),  h_ij' = -A_ij (H_i - h_ji) / (S_i - P_ji)
// (eq. prec_message / mean_message times P).  Both copies of a message are
// computed from bitwise-identical operands with FP contraction disabled, so
// they stay bitwise identical.  The only
// random access is the gather of (S_j, H_j) from an n-sized array; all slot
// traffic is coalesced.
//
// Once every precision message has stopped changing (it never depends on b),
// the "frozen" kernels keep P fixed and iterate the information only, with
// per-slot coefficients c_ij = -A_ij / (S_i - P_ji) (formed as -A_ij times the
// reciprocal, exactly as the full sweeps form the factor of h, so that a
// message computed before and after the switch rounds the same way):
//   h_ij' = c_ij (H_i - h_ji),  h_ji' = c_ji (H_j - h_ij),  H_i' = b_i + sum h_ji'.
// The gather then reads H_j alone (4 bytes per node).
#include <vector>

#include "device_common.h"

namespace gabp {

template <typename T> struct Vec4;
template <> struct Vec4<float> { using type = float4; };
template <> struct Vec4<double> { using type = double4; };

// ---------------------------------------------------------------------------
// row blocks: the unit of work of every sweep kernel
// ---------------------------------------------------------------------------
// The plan cuts the rows into blocks of consecutive rows, at most kSegRows rows
// and kSegChunk slots each (a longer row forms a block of its own), never
// across a colour class.  A workgroup takes a block: it loads the rows'
// offsets into LDS and streams their slots in chunks of kSegChunk, thread t
// handling slots c + t, c + t + kBlock, ... (coalesced, every lane busy
// whatever the row lengths, kSegK independent gathers in flight per thread);
// it finds each slot's row by a binary search of the offsets, leaves the
// slot's in-message in LDS, and the row's own thread then adds its
// in-messages in slot order.
constexpr int kSegRows = 256;    // rows of a block at most
constexpr int kSegChunk = 1024;  // slots of a block (a longer row alone), streamed per chunk
constexpr int kMaxPairBlocks = 16384;  // a random graph of 2^20 rows has 8192 blocks
constexpr int kSegK = kSegChunk / kBlock;
static_assert(kSegChunk % kBlock == 0 && kSegRows <= kBlock, "row block shape");


// the row of slot e: the last r with rp[r] <= e (rp[0] <= e < rp[nr])
__device__ __forceinline__ int seg_row(const int *rp, int nr, int e) {
  int lo = 0, hi = nr;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (rp[mid] <= e) lo = mid;
    else hi = mid;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// synchronous full sweep (P and h), MODE 0 = sweep, 1 = sweep + check
// ---------------------------------------------------------------------------
// Rows are the virtual rows [vbase, vbase + n) of one column range (node
// v - vbase); carry (nullable) holds the node sums of the ranges before it.
// mi == NULL: every message of round t is zero (the first sweep after a
// reset, which then reads no slot state).
// The last range adds A_ii and b_i, writes the broadcasts and checks the
// means; an earlier one writes its partial sums to sout (the carry).
template <typename T, int MODE, bool DAMP>
__global__ __launch_bounds__(kBlock) void k_pair_sweep(
    const int32_t *__restrict__ rb, int b0, int b1, int vbase, const int32_t *__restrict__ oprt,
    const int32_t *__restrict__ ocol, const T *__restrict__ acoef, const T *__restrict__ diag,
    const T *__restrict__ rhs, const typename Vec4<T>::type *__restrict__ mi,
    typename Vec4<T>::type *__restrict__ mo, const typename Vec2<T>::type *__restrict__ sin,
    const typename Vec2<T>::type *__restrict__ carry, typename Vec2<T>::type *__restrict__ sout,
    bool last, T alpha, T *__restrict__ xprev, BlockPartial *__restrict__ part, int nslots,
    uint32_t *__restrict__ sticky, const Ctl *__restrict__ ctl) {
  // no FMA contraction: both stored copies of a message, and the node sums
  // rebuilt from stored values, must round exactly like this sweep does
#pragma clang fp contract(off)
  using V4 = typename Vec4<T>::type;
  using V2 = typename Vec2<T>::type;
  __shared__ int rp[kSegRows + 1];
  __shared__ V2 own[kSegRows];   // the block's rows' broadcasts of round t
  __shared__ V2 in[kSegChunk];   // the chunk's new in-messages (P_ji, h_ji)
  if (ctl != nullptr && ctl->stop != STOP_NONE) return;
  const int t = threadIdx.x;
  const T b1m = T(1) - alpha;
  double d = 0.0, ax = 0.0;
  T dp = T(0), pm = T(0);
  bool zero = false;
  uint32_t f = 0;
  for (int b = b0 + blockIdx.x; b < b1; b += gridDim.x) {
    const int r0 = rb[b], nr = rb[b + 1] - r0;
    const int n0 = r0 - vbase;  // node of the block's first row
    __syncthreads();  // the previous block's readers are done with the LDS
    for (int k = t; k <= nr; k += kBlock) rp[k] = oprt[r0 + k];
    for (int k = t; k < nr; k += kBlock) own[k] = sin[n0 + k];
    __syncthreads();
    const int e0 = rp[0], e1 = rp[nr];
    T S = T(0), H = T(0);
    if (carry != nullptr && t < nr) {
      S = carry[n0 + t].x;
      H = carry[n0 + t].y;
    }
    for (int c = e0; c < e1; c += kSegChunk) {
      int j[kSegK];
      T a[kSegK];
      V4 m[kSegK];
      V2 sj[kSegK];
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        const int e = c + k * kBlock + t;
        j[k] = 0;
        a[k] = T(0);
        m[k] = V4{};
        if (e < e1) {
          j[k] = __builtin_nontemporal_load(&ocol[e]);
          a[k] = __builtin_nontemporal_load(&acoef[e]);
          if (mi != nullptr) m[k] = nt_load(&mi[e]);  // (P_ij, h_ij, P_ji, h_ji) of round t
        }
      }
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        sj[k] = V2{};
        if (c + k * kBlock + t < e1) sj[k] = sin[j[k]];  // broadcast of node j, round t
      }
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        const int e = c + k * kBlock + t;
        if (e >= e1) continue;
        const V2 si = own[seg_row(rp, nr, e)];
        const T cj = sj[k].x - m[k].x;  // S_j - P_ij: cavity of j toward i
        const T ci = si.x - m[k].z;     // S_i - P_ji: cavity of i toward j
        zero |= (cj == T(0)) | (ci == T(0));
        const T ij = T(1) / cj, ii = T(1) / ci;
        const T aa = a[k];
        T Pin = -(aa * aa) * ij, hin = (-aa * ij) * (sj[k].y - m[k].y);
        T Pout = -(aa * aa) * ii, hout = (-aa * ii) * (si.y - m[k].w);
        if (DAMP) {
          Pin = alpha * m[k].z + b1m * Pin;
          hin = alpha * m[k].w + b1m * hin;
          Pout = alpha * m[k].x + b1m * Pout;
          hout = alpha * m[k].y + b1m * hout;
        }
        if (MODE == 1) {
          dp = fmax(dp, fabs(Pout - m[k].x));
          pm = fmax(pm, fabs(Pout));
        }
        V4 o;
        o.x = Pout; o.y = hout; o.z = Pin; o.w = hin;
        nt_store(&mo[e], o);
        V2 v;
        v.x = Pin;
        v.y = hin;
        in[e - c] = v;
      }
      __syncthreads();
      if (t < nr) {
        const int lo = max(rp[t], c), hi = min(rp[t + 1], c + kSegChunk);
        for (int e = lo; e < hi; ++e) {
          S += in[e - c].x;
          H += in[e - c].y;
        }
      }
      __syncthreads();
    }
    if (t < nr) {
      const int row = n0 + t;
      if (last) {
        S += diag[row];
        H += rhs[row];
      }
      V2 o;
      o.x = S;
      o.y = H;
      sout[row] = o;
      if (MODE == 1 && last) {
        if (S == T(0)) f |= FLAG_BREAKDOWN;
        const T x = H / S;
        if (!isfinite(x)) f |= FLAG_NONFINITE;
        d = fmax(d, (double)fabs(x - xprev[row]));
        xprev[row] = x;
        ax = fmax(ax, (double)fabs(x));
      }
    }
  }
  if (zero) f |= FLAG_BREAKDOWN;
  if (f) atomicOr(sticky, f);
  if (MODE == 1) slot_publish(d, ax, (double)dp, (double)pm, part, nslots);
}

// Aggregate (S, H) from the slots' incoming messages: used after reset,
// message import and restarts.  Row blocks as in the sweeps; a row's
// in-messages are added in slot order, exactly as the sweeps add them, so that
// imported messages resume a solve bit for bit.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_pair_aggregate(
    const int32_t *__restrict__ rb, int b0, int b1, int vbase, const int32_t *__restrict__ oprt,
    const T *__restrict__ diag, const T *__restrict__ rhs,
    const typename Vec4<T>::type *__restrict__ msg, const typename Vec2<T>::type *__restrict__ carry,
    typename Vec2<T>::type *__restrict__ sums, bool last) {
#pragma clang fp contract(off)
  using V2 = typename Vec2<T>::type;
  __shared__ int rp[kSegRows + 1];
  __shared__ V2 in[kSegChunk];
  const int t = threadIdx.x;
  for (int b = b0 + blockIdx.x; b < b1; b += gridDim.x) {
    const int r0 = rb[b], nr = rb[b + 1] - r0;
    const int n0 = r0 - vbase;
    __syncthreads();
    for (int k = t; k <= nr; k += kBlock) rp[k] = oprt[r0 + k];
    __syncthreads();
    const int e0 = rp[0], e1 = rp[nr];
    T S = T(0), H = T(0);
    if (carry != nullptr && t < nr) {
      S = carry[n0 + t].x;
      H = carry[n0 + t].y;
    }
    for (int c = msg != nullptr ? e0 : e1; c < e1; c += kSegChunk) {  // NULL: no messages yet
      for (int e = c + t; e < e1 && e < c + kSegChunk; e += kBlock) {
        const auto m = msg[e];
        V2 v;
        v.x = m.z;
        v.y = m.w;
        in[e - c] = v;
      }
      __syncthreads();
      if (t < nr) {
        const int lo = max(rp[t], c), hi = min(rp[t + 1], c + kSegChunk);
        for (int e = lo; e < hi; ++e) {
          S += in[e - c].x;
          H += in[e - c].y;
        }
      }
      __syncthreads();
    }
    if (t < nr) {
      V2 o;
      o.x = last ? S + diag[n0 + t] : S;
      o.y = last ? H + rhs[n0 + t] : H;
      sums[n0 + t] = o;
    }
  }
}

// Zero every information field (restart) and re-aggregate H = rhs.
template <typename T>
__global__ void k_pair_zero_h(int64_t E, typename Vec4<T>::type *__restrict__ msg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E) {
    msg[e].y = T(0);
    msg[e].w = T(0);
  }
}

// x += H / S (FP64 accumulate) and/or marginal precisions from the broadcast
// array (full layout) or from the frozen (S, H) arrays.
template <typename T>
__global__ void k_pair_infer(int n, const typename Vec2<T>::type *__restrict__ sums,
                             const T *__restrict__ Sfix, const T *__restrict__ Hfz,
                             double *__restrict__ xacc, double *__restrict__ marg,
                             T *__restrict__ means, uint32_t *__restrict__ sticky) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  T S, H;
  if (sums) {
    S = sums[i].x;
    H = sums[i].y;
  } else {
    S = Sfix[i];
    H = Hfz[i];
  }
  if (S == T(0)) atomicOr(sticky, FLAG_BREAKDOWN);
  if (xacc) xacc[i] += (double)H / (double)S;
  if (marg) marg[i] = (double)S;
  if (means) means[i] = H / S;
}

// ---------------------------------------------------------------------------
// freeze: P has stopped changing; derive the fixed coefficients
// ---------------------------------------------------------------------------
// Each slot (i, j) computes its out-message coefficient c_ij = -A_ij / (S_i -
// P_ji) and the in-message coefficient c_ji of the message it receives.  The
// two copies of every coefficient (the sender's and the receiver's) must be
// the same number.  In a synchronous state both copies of every message are
// equal, so the receiver recomputes c_ji = -A_ij / (S_j - P_ij) from its own
// copy of P_ij and the gathered S_j.  In a coloured state a row that sent
// after j holds a newer P_ij than the one j used, so the receiver's copy would
// not match: there (SCATTER) each slot stores its c_ij twice instead, as its
// own out-coefficient and, through the reverse-slot index, as the
// in-coefficient of slot (j, i).  A scattered 4-byte store costs more than the
// gather on the random graph (180 against 117 us) but less than the two
// gathers a coloured receiver would need (374 against 607 us on the
// least-squares system).
template <typename T, bool SCATTER>
__global__ __launch_bounds__(kBlock) void k_pair_freeze(
    const int32_t *__restrict__ rb, int nblk, int n, const int32_t *__restrict__ oprt,
    const int32_t *__restrict__ ocol, const int32_t *__restrict__ rev, const T *__restrict__ acoef,
    const typename Vec4<T>::type *__restrict__ msg,
    const typename Vec2<T>::type *__restrict__ sums, typename Vec2<T>::type *__restrict__ coef,
    typename Vec2<T>::type *__restrict__ hp, T *__restrict__ Sfix, T *__restrict__ Hfz) {
#pragma clang fp contract(off)
  using V2 = typename Vec2<T>::type;
  __shared__ int rp[kSegRows + 1];
  __shared__ T own[kSegRows];
  const int t = threadIdx.x;
  for (int b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int r0 = rb[b], nr = rb[b + 1] - r0;
    // virtual rows of the second column range are nodes r0 - n, ...; the
    // first range lists every node once
    const int n0 = r0 >= n ? r0 - n : r0;
    __syncthreads();
    for (int k = t; k <= nr; k += kBlock) rp[k] = oprt[r0 + k];
    for (int k = t; k < nr; k += kBlock) {
      const V2 si = sums[n0 + k];
      own[k] = si.x;
      if (r0 < n) {
        Sfix[n0 + k] = si.x;
        Hfz[n0 + k] = si.y;
      }
    }
    __syncthreads();
    const int e1 = rp[nr];
    for (int e = rp[0] + t; e < e1; e += kBlock) {
      const T a = __builtin_nontemporal_load(&acoef[e]);
      const auto m = nt_load(&msg[e]);
      const T Si = own[seg_row(rp, nr, e)];
      const T cij = -a * (T(1) / (Si - m.z));  // out-message coefficient
      if (SCATTER) {
        const int r = __builtin_nontemporal_load(&rev[e]);
        coef[e].x = cij;
        coef[r].y = cij;  // in-message coefficient of (j, i)
      } else {
        const int j = __builtin_nontemporal_load(&ocol[e]);
        V2 c;
        c.x = cij;
        c.y = -a * (T(1) / (sums[j].x - m.x));  // c_ji from this slot's copy of P_ij
        nt_store(&coef[e], c);
      }
      V2 h;
      h.x = m.y;
      h.y = m.w;
      nt_store(&hp[e], h);
    }
  }
}

// synchronous settled-precision sweep: information only.
// MODE 0 = sweep, 1 = sweep + check.
// Column ranges as in k_pair_sweep (carry: the earlier ranges' H sums).
template <typename T, int MODE, bool DAMP>
__global__ __launch_bounds__(kBlock) void k_pair_frozen(
    const int32_t *__restrict__ rb, int b0, int b1, int vbase, const int32_t *__restrict__ oprt,
    const int32_t *__restrict__ ocol, const typename Vec2<T>::type *__restrict__ coef,
    const T *__restrict__ rhs, const T *__restrict__ Sfix,
    const typename Vec2<T>::type *__restrict__ hin, typename Vec2<T>::type *__restrict__ hout,
    const T *__restrict__ Hin, const T *__restrict__ carry, T *__restrict__ Hout, bool last,
    T alpha, T *__restrict__ xprev, BlockPartial *__restrict__ part, int nslots,
    uint32_t *__restrict__ sticky, const Ctl *__restrict__ ctl) {
#pragma clang fp contract(off)
  using V2 = typename Vec2<T>::type;
  __shared__ int rp[kSegRows + 1];
  __shared__ T own[kSegRows];
  __shared__ T in[kSegChunk];
  if (ctl != nullptr && ctl->stop != STOP_NONE) return;
  const int t = threadIdx.x;
  const T b1m = T(1) - alpha;
  double d = 0.0, ax = 0.0;
  uint32_t f = 0;
  for (int b = b0 + blockIdx.x; b < b1; b += gridDim.x) {
    const int r0 = rb[b], nr = rb[b + 1] - r0;
    const int n0 = r0 - vbase;
    __syncthreads();
    for (int k = t; k <= nr; k += kBlock) rp[k] = oprt[r0 + k];
    for (int k = t; k < nr; k += kBlock) own[k] = Hin[n0 + k];
    __syncthreads();
    const int e0 = rp[0], e1 = rp[nr];
    T H = (carry != nullptr && t < nr) ? carry[n0 + t] : T(0);
    for (int c = e0; c < e1; c += kSegChunk) {
      int j[kSegK];
      V2 cf[kSegK], h[kSegK];
      T Hj[kSegK];
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        const int e = c + k * kBlock + t;
        j[k] = 0;
        cf[k] = V2{};
        h[k] = V2{};
        if (e < e1) {
          j[k] = ocol[e];
          cf[k] = coef[e];
          h[k] = hin[e];  // (h_ij, h_ji)
        }
      }
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        Hj[k] = T(0);
        if (c + k * kBlock + t < e1) Hj[k] = Hin[j[k]];
      }
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        const int e = c + k * kBlock + t;
        if (e >= e1) continue;
        const T Hi = own[seg_row(rp, nr, e)];
        T ho = cf[k].x * (Hi - h[k].y);
        T hi = cf[k].y * (Hj[k] - h[k].x);
        if (DAMP) {
          ho = alpha * h[k].x + b1m * ho;
          hi = alpha * h[k].y + b1m * hi;
        }
        V2 o;
        o.x = ho;
        o.y = hi;
        nt_store(&hout[e], o);
        in[e - c] = hi;
      }
      __syncthreads();
      if (t < nr) {
        const int lo = max(rp[t], c), hi = min(rp[t + 1], c + kSegChunk);
        for (int e = lo; e < hi; ++e) H += in[e - c];
      }
      __syncthreads();
    }
    if (t < nr) {
      const int row = n0 + t;
      if (last) H += rhs[row];
      Hout[row] = H;
      if (MODE == 1 && last) {
        const T x = H / Sfix[row];
        if (!isfinite(x)) f |= FLAG_NONFINITE;
        d = fmax(d, (double)fabs(x - xprev[row]));
        xprev[row] = x;
        ax = fmax(ax, (double)fabs(x));
      }
    }
  }
  if (f) atomicOr(sticky, f);
  if (MODE == 1) slot_publish(d, ax, 0.0, 0.0, part, nslots);
}

// restart in the frozen state: h = 0, H = rhs
template <typename T>
__global__ void k_frozen_restart(int64_t E, int n, typename Vec2<T>::type *__restrict__ hp,
                                 const T *__restrict__ rhs, T *__restrict__ Hfz) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E) {
    hp[e].x = T(0);
    hp[e].y = T(0);
  }
  if (e < n) Hfz[e] = rhs[e];
}

// ---------------------------------------------------------------------------
// coloured schedule: the rows of one colour class send, in place
// ---------------------------------------------------------------------------
// Row i of the class first rebuilds its in-messages from the neighbours'
// current broadcasts (every neighbour is of another class, so these are the
// newest messages it sent, recomputed from the same operands it used), sums
// them into its new totals (S_i, H_i), and only then computes its
// out-messages from those totals: the serial scheme of section III-C, one
// colour class at a time.  No row of the class reads a slot or broadcast
// another row of the class writes, so one buffer suffices.  The launch walks
// the class's row blocks [b0, b1); a block within one chunk keeps its slots in
// registers between the two steps, a longer one (a single long row) reads
// them again and recomputes its in-messages with the same operands.
//
// The rebuilt in-message equals the stored one only if its sender computed it
// from its broadcast.  Messages that were set rather than sent (zeroed by a
// reset or a restart, or imported) are not; `first` marks the first sweep
// after such a change, in which the classes that have not sent yet (rows at
// or beyond row1: classes run in row order) pass their stored in-messages
// instead, which the engine keeps equal to the senders' out-messages.
template <typename T, bool DAMP>
__device__ __forceinline__ void col_in(bool rebuild, T a, const typename Vec4<T>::type &m,
                                       const typename Vec2<T>::type &sj, T alpha, T b1m, T &Pin,
                                       T &hin, bool &zero) {
#pragma clang fp contract(off)
  Pin = m.z;
  hin = m.w;
  if (rebuild) {
    const T cj = sj.x - m.x;
    zero |= cj == T(0);
    const T ij = T(1) / cj;
    Pin = -(a * a) * ij;
    hin = (-a * ij) * (sj.y - m.y);
    if (DAMP) {
      Pin = alpha * m.z + b1m * Pin;
      hin = alpha * m.w + b1m * hin;
    }
  }
}

template <typename T, int MODE, bool DAMP>
__global__ __launch_bounds__(kBlock) void k_pair_col(
    const int32_t *__restrict__ rb, int b0, int b1, int row1, bool first,
    const int32_t *__restrict__ oprt, const int32_t *__restrict__ ocol,
    const T *__restrict__ acoef, const T *__restrict__ diag, const T *__restrict__ rhs,
    typename Vec4<T>::type *msg, typename Vec2<T>::type *sums, T alpha, T *__restrict__ xprev,
    BlockPartial *__restrict__ part, int nslots, uint32_t *__restrict__ sticky,
    const Ctl *__restrict__ ctl) {
#pragma clang fp contract(off)
  using V4 = typename Vec4<T>::type;
  using V2 = typename Vec2<T>::type;
  __shared__ int rp[kSegRows + 1];
  __shared__ V2 tot[kSegRows];  // the rows' new totals (S_i, H_i)
  __shared__ V2 in[kSegChunk];
  if (ctl != nullptr && ctl->stop != STOP_NONE) return;
  const int t = threadIdx.x;
  const T b1m = T(1) - alpha;
  double d = 0.0, ax = 0.0;
  T dp = T(0), pm = T(0);
  bool zero = false;
  uint32_t f = 0;
  for (int b = b0 + blockIdx.x; b < b1; b += gridDim.x) {
    const int r0 = rb[b], nr = rb[b + 1] - r0;
    __syncthreads();
    for (int k = t; k <= nr; k += kBlock) rp[k] = oprt[r0 + k];
    __syncthreads();
    const int e0 = rp[0], e1 = rp[nr];
    const bool one = e1 - e0 <= kSegChunk;  // uniform over the workgroup
    T a[kSegK], Pin[kSegK], hin[kSegK];
    V4 m[kSegK];
    // step 1: the in-messages j -> i from j's broadcast, and the new totals
    T S = T(0), H = T(0);
    for (int c = e0; c < e1; c += kSegChunk) {
      int j[kSegK];
      V2 sj[kSegK];
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        const int e = c + k * kBlock + t;
        j[k] = 0;
        a[k] = T(0);
        m[k] = V4{};
        if (e < e1) {
          j[k] = ocol[e];
          a[k] = acoef[e];
          m[k] = nt_load(&msg[e]);  // (P_ij, h_ij, P_ji, h_ji) as last written
        }
      }
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        sj[k] = V2{};
        if (c + k * kBlock + t < e1 && !(first && j[k] >= row1)) sj[k] = sums[j[k]];
      }
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        const int e = c + k * kBlock + t;
        Pin[k] = T(0);
        hin[k] = T(0);
        if (e >= e1) continue;
        col_in<T, DAMP>(!(first && j[k] >= row1), a[k], m[k], sj[k], alpha, b1m, Pin[k], hin[k],
                        zero);
        V2 v;
        v.x = Pin[k];
        v.y = hin[k];
        in[e - c] = v;
      }
      __syncthreads();
      if (t < nr) {
        const int lo = max(rp[t], c), hi = min(rp[t + 1], c + kSegChunk);
        for (int e = lo; e < hi; ++e) {
          S += in[e - c].x;
          H += in[e - c].y;
        }
      }
      __syncthreads();
    }
    if (t < nr) {
      const int row = r0 + t;
      S += diag[row];
      H += rhs[row];
      V2 o;
      o.x = S;
      o.y = H;
      tot[t] = o;
      sums[row] = o;
      if (MODE == 1) {
        if (S == T(0)) f |= FLAG_BREAKDOWN;
        const T x = H / S;
        if (!isfinite(x)) f |= FLAG_NONFINITE;
        d = fmax(d, (double)fabs(x - xprev[row]));
        xprev[row] = x;
        ax = fmax(ax, (double)fabs(x));
      }
    }
    __syncthreads();
    // step 2: the out-messages i -> j from the new totals
    for (int c = e0; c < e1; c += kSegChunk) {
      if (!one) {  // recompute this chunk's in-messages exactly as in step 1
        int j[kSegK];
        V2 sj[kSegK];
#pragma unroll
        for (int k = 0; k < kSegK; ++k) {
          const int e = c + k * kBlock + t;
          j[k] = 0;
          a[k] = T(0);
          m[k] = V4{};
          if (e < e1) {
            j[k] = ocol[e];
            a[k] = acoef[e];
            m[k] = msg[e];
          }
        }
#pragma unroll
        for (int k = 0; k < kSegK; ++k) {
          sj[k] = V2{};
          if (c + k * kBlock + t < e1 && !(first && j[k] >= row1)) sj[k] = sums[j[k]];
        }
#pragma unroll
        for (int k = 0; k < kSegK; ++k) {
          Pin[k] = T(0);
          hin[k] = T(0);
          if (c + k * kBlock + t < e1)
            col_in<T, DAMP>(!(first && j[k] >= row1), a[k], m[k], sj[k], alpha, b1m, Pin[k],
                            hin[k], zero);
        }
      }
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        const int e = c + k * kBlock + t;
        if (e >= e1) continue;
        const V2 ti = tot[seg_row(rp, nr, e)];
        const T ci = ti.x - Pin[k];
        zero |= ci == T(0);
        const T ii = T(1) / ci;
        const T aa = a[k];
        T Pout = -(aa * aa) * ii, hout = (-aa * ii) * (ti.y - hin[k]);
        if (DAMP) {
          Pout = alpha * m[k].x + b1m * Pout;
          hout = alpha * m[k].y + b1m * hout;
        }
        if (MODE == 1) {
          dp = fmax(dp, fabs(Pout - m[k].x));
          pm = fmax(pm, fabs(Pout));
        }
        V4 o;
        o.x = Pout; o.y = hout; o.z = Pin[k]; o.w = hin[k];
        nt_store(&msg[e], o);
      }
    }
  }
  if (zero) f |= FLAG_BREAKDOWN;
  if (f) atomicOr(sticky, f);
  if (MODE == 1) slot_publish(d, ax, (double)dp, (double)pm, part, nslots);
}

// settled precisions, coloured: h_ji from H_j's broadcast, then H_i, then h_ij
template <typename T, bool DAMP>
__device__ __forceinline__ T col_hin(bool rebuild, const typename Vec2<T>::type &c,
                                     const typename Vec2<T>::type &h, T Hj, T alpha, T b1m) {
#pragma clang fp contract(off)
  T hin = h.y;
  if (rebuild) {
    hin = c.y * (Hj - h.x);
    if (DAMP) hin = alpha * h.y + b1m * hin;
  }
  return hin;
}

template <typename T, int MODE, bool DAMP>
__global__ __launch_bounds__(kBlock) void k_pair_frozen_col(
    const int32_t *__restrict__ rb, int b0, int b1, int row1, bool first,
    const int32_t *__restrict__ oprt, const int32_t *__restrict__ ocol,
    const typename Vec2<T>::type *__restrict__ coef, const T *__restrict__ rhs,
    const T *__restrict__ Sfix, typename Vec2<T>::type *hp, T *Hb, T alpha,
    T *__restrict__ xprev, BlockPartial *__restrict__ part, int nslots,
    uint32_t *__restrict__ sticky, const Ctl *__restrict__ ctl) {
#pragma clang fp contract(off)
  using V2 = typename Vec2<T>::type;
  __shared__ int rp[kSegRows + 1];
  __shared__ T tot[kSegRows];
  __shared__ T in[kSegChunk];
  if (ctl != nullptr && ctl->stop != STOP_NONE) return;
  const int t = threadIdx.x;
  const T b1m = T(1) - alpha;
  double d = 0.0, ax = 0.0;
  uint32_t f = 0;
  for (int b = b0 + blockIdx.x; b < b1; b += gridDim.x) {
    const int r0 = rb[b], nr = rb[b + 1] - r0;
    __syncthreads();
    for (int k = t; k <= nr; k += kBlock) rp[k] = oprt[r0 + k];
    __syncthreads();
    const int e0 = rp[0], e1 = rp[nr];
    const bool one = e1 - e0 <= kSegChunk;
    V2 cf[kSegK], h[kSegK];
    T hin[kSegK];
    T H = T(0);
    for (int c = e0; c < e1; c += kSegChunk) {
      int j[kSegK];
      T Hj[kSegK];
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        const int e = c + k * kBlock + t;
        j[k] = 0;
        cf[k] = V2{};
        h[k] = V2{};
        if (e < e1) {
          j[k] = ocol[e];
          cf[k] = coef[e];
          h[k] = hp[e];  // (h_ij, h_ji) as last written
        }
      }
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        Hj[k] = T(0);
        if (c + k * kBlock + t < e1 && !(first && j[k] >= row1)) Hj[k] = Hb[j[k]];
      }
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        const int e = c + k * kBlock + t;
        hin[k] = T(0);
        if (e >= e1) continue;
        hin[k] = col_hin<T, DAMP>(!(first && j[k] >= row1), cf[k], h[k], Hj[k], alpha, b1m);
        in[e - c] = hin[k];
      }
      __syncthreads();
      if (t < nr) {
        const int lo = max(rp[t], c), hi = min(rp[t + 1], c + kSegChunk);
        for (int e = lo; e < hi; ++e) H += in[e - c];
      }
      __syncthreads();
    }
    if (t < nr) {
      const int row = r0 + t;
      H += rhs[row];
      tot[t] = H;
      Hb[row] = H;
      if (MODE == 1) {
        const T x = H / Sfix[row];
        if (!isfinite(x)) f |= FLAG_NONFINITE;
        d = fmax(d, (double)fabs(x - xprev[row]));
        xprev[row] = x;
        ax = fmax(ax, (double)fabs(x));
      }
    }
    __syncthreads();
    for (int c = e0; c < e1; c += kSegChunk) {
      if (!one) {
        int j[kSegK];
        T Hj[kSegK];
#pragma unroll
        for (int k = 0; k < kSegK; ++k) {
          const int e = c + k * kBlock + t;
          j[k] = 0;
          cf[k] = V2{};
          h[k] = V2{};
          if (e < e1) {
            j[k] = ocol[e];
            cf[k] = coef[e];
            h[k] = hp[e];
          }
        }
#pragma unroll
        for (int k = 0; k < kSegK; ++k) {
          Hj[k] = T(0);
          if (c + k * kBlock + t < e1 && !(first && j[k] >= row1)) Hj[k] = Hb[j[k]];
        }
#pragma unroll
        for (int k = 0; k < kSegK; ++k) {
          hin[k] = T(0);
          if (c + k * kBlock + t < e1)
            hin[k] = col_hin<T, DAMP>(!(first && j[k] >= row1), cf[k], h[k], Hj[k], alpha, b1m);
        }
      }
#pragma unroll
      for (int k = 0; k < kSegK; ++k) {
        const int e = c + k * kBlock + t;
        if (e >= e1) continue;
        const T Hi = tot[seg_row(rp, nr, e)];
        T hout = cf[k].x * (Hi - hin[k]);
        if (DAMP) hout = alpha * h[k].x + b1m * hout;
        V2 o;
        o.x = hout;
        o.y = hin[k];
        nt_store(&hp[e], o);
      }
    }
  }
  if (f) atomicOr(sticky, f);
  if (MODE == 1) slot_publish(d, ax, 0.0, 0.0, part, nslots);
}

// Marginals of a coloured plan from its current messages, one class (rows
// [row0, row1)) per launch, after a complete sweep.  A row's broadcast
// predates the messages of the classes that sent after it, so the totals are
// rebuilt: in-messages from earlier classes are the stored copies (made in
// this row's phase, and their senders have not sent since), those from later
// classes are rebuilt from the senders' broadcasts (they were computed from
// this row's current out-messages).  Full state: (S, H) from the in-messages;
// settled: S fixed, H rebuilt.
template <typename T, bool DAMP, bool FROZEN>
__global__ __launch_bounds__(kBlock) void k_pair_col_infer(
    const int32_t *__restrict__ rb, int b0, int b1, int row1, const int32_t *__restrict__ oprt,
    const int32_t *__restrict__ ocol, const T *__restrict__ acoef, const T *__restrict__ diag,
    const T *__restrict__ rhs, const typename Vec4<T>::type *__restrict__ msg,
    const typename Vec2<T>::type *__restrict__ sums, const typename Vec2<T>::type *__restrict__ coef,
    const typename Vec2<T>::type *__restrict__ hp, const T *__restrict__ Sfix,
    const T *__restrict__ Hb, T alpha, double *__restrict__ xacc, double *__restrict__ marg,
    T *__restrict__ means, uint32_t *__restrict__ sticky) {
#pragma clang fp contract(off)
  using V2 = typename Vec2<T>::type;
  __shared__ int rp[kSegRows + 1];
  __shared__ V2 in[kSegChunk];
  const int t = threadIdx.x;
  const T b1m = T(1) - alpha;
  uint32_t f = 0;
  for (int b = b0 + blockIdx.x; b < b1; b += gridDim.x) {
    const int r0 = rb[b], nr = rb[b + 1] - r0;
    __syncthreads();
    for (int k = t; k <= nr; k += kBlock) rp[k] = oprt[r0 + k];
    __syncthreads();
    const int e0 = rp[0], e1 = rp[nr];
    T S = T(0), H = T(0);
    for (int c = e0; c < e1; c += kSegChunk) {
      for (int e = c + t; e < e1 && e < c + kSegChunk; e += kBlock) {
        const int j = ocol[e];
        V2 v;
        if (FROZEN) {
          const V2 h = hp[e];
          T hin = h.y;
          if (j >= row1) {
            hin = coef[e].y * (Hb[j] - h.x);
            if (DAMP) hin = alpha * h.y + b1m * hin;
          }
          v.x = T(0);
          v.y = hin;
        } else {
          const auto m = msg[e];
          T Pin = m.z, hin = m.w;
          if (j >= row1) {
            const T a = acoef[e];
            const V2 sj = sums[j];
            const T ij = T(1) / (sj.x - m.x);
            Pin = -(a * a) * ij;
            hin = (-a * ij) * (sj.y - m.y);
            if (DAMP) {
              Pin = alpha * m.z + b1m * Pin;
              hin = alpha * m.w + b1m * hin;
            }
          }
          v.x = Pin;
          v.y = hin;
        }
        in[e - c] = v;
      }
      __syncthreads();
      if (t < nr) {
        const int lo = max(rp[t], c), hi = min(rp[t + 1], c + kSegChunk);
        for (int e = lo; e < hi; ++e) {
          S += in[e - c].x;
          H += in[e - c].y;
        }
      }
      __syncthreads();
    }
    if (t < nr) {
      const int row = r0 + t;
      S = FROZEN ? Sfix[row] : S + diag[row];
      H += rhs[row];
      if (S == T(0)) f |= FLAG_BREAKDOWN;
      if (xacc) xacc[row] += (double)H / (double)S;
      if (marg) marg[row] = (double)S;
      if (means) means[row] = H / S;
    }
  }
  if (f) atomicOr(sticky, f);
}

// Stored in-messages := the senders' out-messages (P only; the coloured
// schedule's restart, after the informations were zeroed).
template <typename T>
__global__ void k_pair_sync_in(int64_t E, const int32_t *__restrict__ rev,
                               typename Vec4<T>::type *__restrict__ msg) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E) msg[e].z = msg[rev[e]].x;
}

// ---------------------------------------------------------------------------
// export / import in CSR slot order (pair layout holds the out-message at .xy)
// ---------------------------------------------------------------------------
// nb column ranges: row i's entries below the split sit at oprt[i] + rank,
// the others (nb == 2) at oprt[n + i] + the rest
template <typename T, bool GET>
__global__ void k_pair_io(int n, int nb, const int64_t *__restrict__ rp,
                          const int64_t *__restrict__ diagpos, const int32_t *__restrict__ oprt,
                          const int32_t *__restrict__ rev, typename Vec4<T>::type *__restrict__ msg,
                          double *__restrict__ P, double *__restrict__ h) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t b = rp[i], e = rp[i + 1], dp = diagpos[i];
  const int64_t c0 = oprt[i + 1] - oprt[i];
  for (int64_t k = b; k < e; ++k) {
    if (k == dp) {
      if (GET) { P[k] = 0.0; h[k] = 0.0; }
      continue;
    }
    const int64_t rank = (k - b) - (k > dp ? 1 : 0);
    const int64_t o = (nb == 2 && rank >= c0) ? oprt[n + i] + (rank - c0) : oprt[i] + rank;
    if (GET) {
      P[k] = (double)msg[o].x;
      h[k] = (double)msg[o].y;
    } else {
      // i -> j goes to this slot's out fields and to the in fields of (j, i)
      msg[o].x = (T)P[k];
      msg[o].y = (T)h[k];
      msg[rev[o]].z = (T)P[k];
      msg[rev[o]].w = (T)h[k];
    }
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
template <typename T, int MODE, bool DAMP>
static void pair_one(const PairArgs &a, hipStream_t s) {
  using V4 = typename Vec4<T>::type;
  using V2 = typename Vec2<T>::type;
  const dim3 grid(a.grid);
  if (a.colored) {
    if (a.frozen)
      hipLaunchKernelGGL((k_pair_frozen_col<T, MODE, DAMP>), grid, dim3(kBlock), 0, s, a.rb, a.b0,
                         a.b1, a.row1, a.first, a.oprt, a.ocol, (const V2 *)a.coef,
                         (const T *)a.rhs, (const T *)a.Sfix, (V2 *)a.msg_out, (T *)a.sums_out,
                         (T)a.alpha, (T *)a.xprev, a.part, a.nslots, a.sticky, a.ctl);
    else
      hipLaunchKernelGGL((k_pair_col<T, MODE, DAMP>), grid, dim3(kBlock), 0, s, a.rb, a.b0, a.b1,
                         a.row1, a.first, a.oprt, a.ocol, (const T *)a.acoef, (const T *)a.diag,
                         (const T *)a.rhs, (V4 *)a.msg_out, (V2 *)a.sums_out, (T)a.alpha,
                         (T *)a.xprev, a.part, a.nslots, a.sticky, a.ctl);
    return;
  }
  if (a.frozen)
    hipLaunchKernelGGL((k_pair_frozen<T, MODE, DAMP>), grid, dim3(kBlock), 0, s, a.rb, a.b0, a.b1,
                       a.vbase, a.oprt, a.ocol, (const V2 *)a.coef, (const T *)a.rhs,
                       (const T *)a.Sfix, (const V2 *)a.msg_in, (V2 *)a.msg_out,
                       (const T *)a.sums_in, (const T *)a.carry, (T *)a.sums_out, a.last,
                       (T)a.alpha, (T *)a.xprev, a.part, a.nslots, a.sticky, a.ctl);
  else
    hipLaunchKernelGGL((k_pair_sweep<T, MODE, DAMP>), grid, dim3(kBlock), 0, s, a.rb, a.b0, a.b1,
                       a.vbase, a.oprt, a.ocol, (const T *)a.acoef, (const T *)a.diag,
                       (const T *)a.rhs, (const V4 *)a.msg_in, (V4 *)a.msg_out,
                       (const V2 *)a.sums_in, (const V2 *)a.carry, (V2 *)a.sums_out, a.last,
                       (T)a.alpha, (T *)a.xprev, a.part, a.nslots, a.sticky, a.ctl);
}

template <typename T>
static hipError_t pair_t(const PairArgs &a, hipStream_t s) {
  if (a.mode == 1) a.damp ? pair_one<T, 1, true>(a, s) : pair_one<T, 1, false>(a, s);
  else a.damp ? pair_one<T, 0, true>(a, s) : pair_one<T, 0, false>(a, s);
  return hipGetLastError();
}

hipError_t launch_pair_sweep(const PairArgs &a, hipStream_t s) {
  if (a.b1 <= a.b0 && !(a.colored && a.mode == 1)) return hipSuccess;
  return a.fp32 ? pair_t<float>(a, s) : pair_t<double>(a, s);
}

int pair_max_blocks() { return kMaxPairBlocks; }

std::vector<int32_t> pair_row_blocks(const int32_t *rp, const std::vector<int> &bounds,
                                     std::vector<int> *first_block) {
  std::vector<int32_t> rb;
  first_block->clear();
  rb.push_back(bounds.empty() ? 0 : bounds[0]);
  for (size_t k = 0; k + 1 < bounds.size(); ++k) {
    first_block->push_back((int)rb.size() - 1);
    int r = bounds[k];
    while (r < bounds[k + 1]) {
      const int start = r;
      int64_t slots = 0;
      while (r < bounds[k + 1] && r - start < kSegRows) {
        const int64_t len = (int64_t)rp[r + 1] - rp[r];
        if (r > start && slots + len > kSegChunk) break;
        slots += len;
        ++r;
      }
      rb.push_back(r);
    }
  }
  first_block->push_back((int)rb.size() - 1);
  return rb;
}

hipError_t launch_pair_aggregate(bool fp32, int grid, const int32_t *rb, int b0, int b1,
                                 int vbase, const int32_t *oprt, const void *diag, const void *rhs,
                                 const void *msg, const void *carry, void *sums, bool last,
                                 hipStream_t s) {
  if (b1 <= b0) return hipSuccess;
  if (fp32)
    hipLaunchKernelGGL(k_pair_aggregate<float>, dim3(grid), dim3(kBlock), 0, s, rb, b0, b1, vbase,
                       oprt, (const float *)diag, (const float *)rhs, (const float4 *)msg,
                       (const float2 *)carry, (float2 *)sums, last);
  else
    hipLaunchKernelGGL(k_pair_aggregate<double>, dim3(grid), dim3(kBlock), 0, s, rb, b0, b1, vbase,
                       oprt, (const double *)diag, (const double *)rhs, (const double4 *)msg,
                       (const double2 *)carry, (double2 *)sums, last);
  return hipGetLastError();
}

hipError_t launch_pair_zero_h(bool fp32, int64_t E, void *msg, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  const dim3 grid((unsigned)((E + kBlock - 1) / kBlock));
  if (fp32) hipLaunchKernelGGL(k_pair_zero_h<float>, grid, dim3(kBlock), 0, s, E, (float4 *)msg);
  else hipLaunchKernelGGL(k_pair_zero_h<double>, grid, dim3(kBlock), 0, s, E, (double4 *)msg);
  return hipGetLastError();
}

hipError_t launch_pair_infer(bool fp32, int n, const void *sums, const void *Sfix, const void *Hfz,
                             double *xacc, double *marg, void *means, uint32_t *sticky,
                             hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((n + kBlock - 1) / kBlock);
  if (fp32)
    hipLaunchKernelGGL(k_pair_infer<float>, grid, dim3(kBlock), 0, s, n, (const float2 *)sums,
                       (const float *)Sfix, (const float *)Hfz, xacc, marg, (float *)means, sticky);
  else
    hipLaunchKernelGGL(k_pair_infer<double>, grid, dim3(kBlock), 0, s, n, (const double2 *)sums,
                       (const double *)Sfix, (const double *)Hfz, xacc, marg, (double *)means,
                       sticky);
  return hipGetLastError();
}

hipError_t launch_pair_freeze(bool fp32, int grid, const int32_t *rb, int nblk, int n,
                              const int32_t *oprt, const int32_t *ocol, const int32_t *rev,
                              bool scatter, const void *acoef, const void *msg, const void *sums,
                              void *coef, void *hp, void *Sfix, void *Hfz, hipStream_t s) {
  if (nblk <= 0) return hipSuccess;
#define FREEZE_LAUNCH(T, V4, V2, SC)                                                             \
  hipLaunchKernelGGL((k_pair_freeze<T, SC>), dim3(grid), dim3(kBlock), 0, s, rb, nblk, n, oprt,   \
                     ocol, rev, (const T *)acoef, (const V4 *)msg, (const V2 *)sums, (V2 *)coef, \
                     (V2 *)hp, (T *)Sfix, (T *)Hfz)
  if (fp32) {
    if (scatter) FREEZE_LAUNCH(float, float4, float2, true);
    else FREEZE_LAUNCH(float, float4, float2, false);
  } else {
    if (scatter) FREEZE_LAUNCH(double, double4, double2, true);
    else FREEZE_LAUNCH(double, double4, double2, false);
  }
#undef FREEZE_LAUNCH
  return hipGetLastError();
}

hipError_t launch_frozen_restart(bool fp32, int64_t E, int n, void *hp, const void *rhs, void *Hfz,
                                 hipStream_t s) {
  const int64_t m = E > n ? E : n;
  if (m <= 0) return hipSuccess;
  const dim3 grid((unsigned)((m + kBlock - 1) / kBlock));
  if (fp32)
    hipLaunchKernelGGL(k_frozen_restart<float>, grid, dim3(kBlock), 0, s, E, n, (float2 *)hp,
                       (const float *)rhs, (float *)Hfz);
  else
    hipLaunchKernelGGL(k_frozen_restart<double>, grid, dim3(kBlock), 0, s, E, n, (double2 *)hp,
                       (const double *)rhs, (double *)Hfz);
  return hipGetLastError();
}

hipError_t launch_pair_io(bool fp32, bool get, int n, int nb, const int64_t *rp,
                          const int64_t *diagpos, const int32_t *oprt, const int32_t *rev,
                          void *msg, double *P, double *h, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const dim3 grid((n + kBlock - 1) / kBlock);
  if (fp32) {
    if (get) hipLaunchKernelGGL((k_pair_io<float, true>), grid, dim3(kBlock), 0, s, n, nb, rp, diagpos, oprt, rev, (float4 *)msg, P, h);
    else hipLaunchKernelGGL((k_pair_io<float, false>), grid, dim3(kBlock), 0, s, n, nb, rp, diagpos, oprt, rev, (float4 *)msg, P, h);
  } else {
    if (get) hipLaunchKernelGGL((k_pair_io<double, true>), grid, dim3(kBlock), 0, s, n, nb, rp, diagpos, oprt, rev, (double4 *)msg, P, h);
    else hipLaunchKernelGGL((k_pair_io<double, false>), grid, dim3(kBlock), 0, s, n, nb, rp, diagpos, oprt, rev, (double4 *)msg, P, h);
  }
  return hipGetLastError();
}

}  // namespace gabp

namespace gabp {
hipError_t launch_pair_sync_in(bool fp32, int64_t E, const int32_t *rev, void *msg, hipStream_t s) {
  if (E <= 0) return hipSuccess;
  const dim3 grid((unsigned)((E + kBlock - 1) / kBlock));
  if (fp32) hipLaunchKernelGGL(k_pair_sync_in<float>, grid, dim3(kBlock), 0, s, E, rev, (float4 *)msg);
  else hipLaunchKernelGGL(k_pair_sync_in<double>, grid, dim3(kBlock), 0, s, E, rev, (double4 *)msg);
  return hipGetLastError();
}
}  // namespace gabp

namespace gabp {
template <typename T, bool DAMP, bool FROZEN>
static void col_infer_one(const PairArgs &a, double *xacc, double *marg, void *means,
                          hipStream_t s) {
  using V4 = typename Vec4<T>::type;
  using V2 = typename Vec2<T>::type;
  hipLaunchKernelGGL((k_pair_col_infer<T, DAMP, FROZEN>), dim3(a.grid), dim3(kBlock), 0, s, a.rb,
                     a.b0, a.b1, a.row1, a.oprt, a.ocol, (const T *)a.acoef, (const T *)a.diag,
                     (const T *)a.rhs, (const V4 *)a.msg_in, (const V2 *)a.sums_in,
                     (const V2 *)a.coef, (const V2 *)a.msg_in, (const T *)a.Sfix,
                     (const T *)a.sums_in, (T)a.alpha, xacc, marg, (T *)means, a.sticky);
}

template <typename T>
static hipError_t col_infer_t(const PairArgs &a, double *xacc, double *marg, void *means,
                              hipStream_t s) {
  if (a.frozen) a.damp ? col_infer_one<T, true, true>(a, xacc, marg, means, s)
                       : col_infer_one<T, false, true>(a, xacc, marg, means, s);
  else a.damp ? col_infer_one<T, true, false>(a, xacc, marg, means, s)
              : col_infer_one<T, false, false>(a, xacc, marg, means, s);
  return hipGetLastError();
}

hipError_t launch_pair_col_infer(const PairArgs &a, double *xacc, double *marg, void *means,
                                 hipStream_t s) {
  if (a.b1 <= a.b0) return hipSuccess;
  return a.fp32 ? col_infer_t<float>(a, xacc, marg, means, s)
                : col_infer_t<double>(a, xacc, marg, means, s);
}
}  // namespace gabp
