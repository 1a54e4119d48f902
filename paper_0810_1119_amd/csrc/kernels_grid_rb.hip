// Two-colour (red-black) schedule of GaBP on structured grids, gfx950.
//
// The serial scheme of section III-C updates messages one node at a time
// from the newest messages; on a grid, whose graph is bipartite, the nodes of
// one colour of the checkerboard colouring share no edge, so all of them can
// send at once from the messages the other colour sent last.  One sweep is
// two launches: colour 0 sends, then colour 1.  On a bipartite graph the
// synchronous schedule runs two independent copies of this recursion (one
// per parity of the round number) at twice the work; the coloured sweep runs
// one of them, so it reaches a given accuracy in about half the sweeps at the
// same bytes per sweep.
//
// Storage is colour-major (layout in gabp_internal.h): a launch for colour c
// reads the in-messages of its nodes from colour 1 - c's arrays at shifted,
// coalesced slots and updates its own out-messages in place (only one
// message buffer exists).  No edge joins two nodes of colour c, so no thread
// reads a message that another thread of the launch writes.  Per node and
// colour-launch: six (P, h) in-messages read, six written, and the
// right-hand side: the 16 bytes per edge of the synchronous sweep, in two
// halves.  The update itself is the synchronous one (information form of
// eq. prec_message / mean_message); damping mixes in the node's own previous
// message, read from the slot it overwrites.
#include "device_common.h"

namespace gabp {

namespace {

// The node a thread of a colour-c launch owns and its neighbours' slots in
// the other colour's arrays.
struct RbNode {
  int i;         // natural index (coefficients, x, marginals)
  int x;         // x coordinate
  int j[6];      // slot of the neighbour toward d (valid when ok[d])
  bool ok[6];
};

__device__ __forceinline__ bool rb_node(const GridGeom &g, int hx, int c, int s, RbNode &n) {
  // the compiler's divisions: with GridGeom's multiply-and-shift divisors
  // the check launches of the 64-grid stack ran 300 -> 400 us
  const int r = s / hx;
  const int kx = s - r * hx;
  const int y = r % g.ny;
  const int z = r / g.ny;  // over the whole stack
  const int zl = z % g.nz;
  const int x = 2 * kx + ((c + y + z) & 1);
  if (x >= g.nx) return false;  // unused slot (nx odd)
  n.i = r * g.nx + x;
  n.x = x;
  const int row = r * hx;
  const int plane = g.ny * hx;
  n.ok[0] = x < g.nx - 1;  n.j[0] = row + ((x + 1) >> 1);
  n.ok[1] = x > 0;         n.j[1] = row + ((x - 1) >> 1);
  n.ok[2] = y < g.ny - 1;  n.j[2] = s + hx;
  n.ok[3] = y > 0;         n.j[3] = s - hx;
  n.ok[4] = zl < g.nz - 1; n.j[4] = s + plane;
  n.ok[5] = zl > 0;        n.j[5] = s - plane;
  return true;
}

template <typename T, bool VARC>
__device__ __forceinline__ void rb_couplings(const GridGeom &g, const GridCoef<T> &k, const RbNode &n,
                                             T a[6]) {
  const int i = n.i;
  if (VARC) {
    a[0] = n.ok[0] ? k.cx[i] : T(0);
    a[1] = n.ok[1] ? k.cx[i - 1] : T(0);
    a[2] = n.ok[2] ? k.cy[i] : T(0);
    a[3] = n.ok[3] ? k.cy[i - g.nx] : T(0);
    a[4] = n.ok[4] ? k.cz[i] : T(0);
    a[5] = n.ok[5] ? k.cz[i - g.nx * g.ny] : T(0);
  } else {
#pragma unroll
    for (int d = 0; d < 6; ++d) a[d] = n.ok[d] ? k.aconst : T(0);
  }
}

// XCD-aware tile order, as in the synchronous grid sweep
__device__ __forceinline__ int rb_tile_of_block() {
  const int nb = gridDim.x;
  if (nb % 8 != 0) return blockIdx.x;
  return (blockIdx.x % 8) * (nb / 8) + blockIdx.x / 8;
}

}  // namespace

// Check maxima and flags of one block's slots.
struct RbAcc {
  double dmax = 0.0, xmax = 0.0, dpb = 0.0, pmb = 0.0;
  uint32_t f = 0;
};

// The slots a block of a colour launch covers.  Without segments (and for
// MODE 2): tiles of kBlock slots, strided by the grid; a check publishes one
// entry per block.  With segments (the grids of a stack, ncs = Nc / nseg
// slots each, nseg <= grid) only the nact segments listed in act are covered:
// B = grid / nact consecutive blocks share a segment, each taking every B-th
// of its tiles, so that the B blocks sweep it as one window of B consecutive
// tiles (few DRAM streams, the neighbouring planes in the XCD's L2) and a
// block's check maxima belong to one segment: block L publishes entry L
// without atomics, and the readout maps entry L to segment act[1 + L / B].
// (A second loop for more segments than blocks, even unused, made the
// compiled sweep about a third slower; such stacks run without segments.)
// fn(s, acc) updates slot s.
template <int MODE, bool SEG, typename F>
__device__ __forceinline__ void rb_cover(int Nc, int nseg, const int32_t *__restrict__ act,
                                         BlockPartial *__restrict__ part, RbAcc &acc, F fn) {
  const int tile0 = rb_tile_of_block();
  // one loop for both cases, which differ in its bounds only
  int first = tile0 * kBlock, stride = gridDim.x * kBlock, end = Nc;
  if (SEG && MODE != 2) {
    const int nact = act[0];
    const int B = nact > 0 ? gridDim.x / nact : 0;  // >= 1: nact <= nseg <= grid
    const int a = B > 0 ? tile0 / B : 0;
    if (B == 0 || a >= nact) {
      end = 0;
    } else {
      const int ncs = Nc / nseg;
      first = act[1 + a] * ncs + (tile0 - a * B) * kBlock;
      stride = B * kBlock;
      end = (act[1 + a] + 1) * ncs;
    }
  }
  for (int base = first; base < end; base += stride) {
    const int s = base + threadIdx.x;
    if (s < end) fn(s, acc);
  }
  if (MODE == 1) {
    if (SEG) {
      if (end > 0) entry_store(acc.dmax, acc.xmax, acc.dpb, acc.pmb, part + tile0);
    } else {
      block_publish(acc.dmax, acc.xmax, acc.dpb, acc.pmb, part);
    }
  }
}

// MODE 0 sweep, 1 sweep + check, 2 means / precisions only (no messages),
// 3 sweep + means of the launch's colour into xacc (its nodes' in-messages
// are final once the other colour has sent; not with segments)
template <typename T, int MODE, bool DAMP, bool VARC, bool SEG>
__global__ __launch_bounds__(kBlock) void k_rb_sweep(
    GridGeom g, int hx, int Nc, int c, GridCoef<T> k, typename Vec2<T>::type *__restrict__ msg,
    const T *__restrict__ rhs, T alpha, T *__restrict__ xprev, double *__restrict__ xacc,
    double *__restrict__ marg, BlockPartial *__restrict__ part, uint32_t *__restrict__ sticky,
    const Ctl *__restrict__ ctl, int nseg, const SegCtl *__restrict__ seg,
    const int32_t *__restrict__ act, int fl) {
  using V = typename Vec2<T>::type;
  if (ctl != nullptr && ctl->stop != STOP_NONE) return;
  const V *__restrict__ other = msg + (size_t)(1 - c) * 6 * Nc;
  V *__restrict__ own = msg + (size_t)c * 6 * Nc;
  RbAcc acc;
  rb_cover<MODE, SEG>(Nc, nseg, act, part, acc, [&](int s, RbAcc &q) {
    RbNode nd;
    if (!rb_node(g, hx, c, s, nd)) return;
    T a[6];
    rb_couplings<T, VARC>(g, k, nd, a);
    // In-messages behind the couplings: loading them on the geometry alone,
    // without waiting for the couplings, made these launches slower (the
    // whole-grid launches by 10%, check launches by 14%).
    T Pin[6], hin[6];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      Pin[d] = T(0);
      hin[d] = T(0);
      if (a[d] != T(0)) {
        const V m = other[(size_t)(d ^ 1) * Nc + nd.j[d]];
        Pin[d] = m.x;
        hin[d] = (fl & SWEEP_ZIN) ? T(0) : m.y;
      }
    }
    T S = VARC ? k.diag[nd.i] : k.dconst, H = rhs[(size_t)c * Nc + s];
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      S += Pin[d];
      H += hin[d];
    }
    // MODE 3: xacc's previous value loaded before the stores
    double xa = 0.0;
    if (MODE == 3 && xacc && !(fl & SWEEP_XSET)) xa = xacc[nd.i];
    if (MODE != 2) {
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        if (a[d] == T(0)) continue;
        const T cav = S - Pin[d];
        if (cav == T(0)) q.f |= FLAG_BREAKDOWN;
        const T inv = T(1) / cav;
        T P = -(a[d] * a[d]) * inv;
        T h = -(a[d] * (H - hin[d])) * inv;
        V *slot = own + (size_t)d * Nc + s;
        if (DAMP || MODE == 1) {
          const V o = *slot;
          if (DAMP) {
            P = alpha * o.x + (T(1) - alpha) * P;
            h = alpha * ((fl & SWEEP_ZOWN) ? T(0) : o.y) + (T(1) - alpha) * h;
          }
          if (MODE == 1) {
            q.dpb = fmax(q.dpb, (double)fabs(P - o.x));
            q.pmb = fmax(q.pmb, (double)fabs(P));
          }
        }
        V out;
        out.x = P;
        out.y = h;
        nt_store(slot, out);  // read by the other colour's next launch, not this one
      }
    }
    if (MODE >= 1) {
      if (S == T(0)) q.f |= FLAG_BREAKDOWN;
      const T x = H / S;
      if (!isfinite(x)) q.f |= FLAG_NONFINITE;
      T *xp = xprev ? xprev + (size_t)c * Nc + s : nullptr;
      if (MODE == 1) {
        q.dmax = fmax(q.dmax, (double)fabs(x - *xp));
        *xp = x;
      } else {
        // a segment sitting the pass out gets no correction
        if (xacc && !(SEG && seg[s / (Nc / nseg)].done == 2)) {
          const double m = (double)H / (double)S;
          xacc[nd.i] = (fl & SWEEP_XSET) ? m : (MODE == 3 ? xa : xacc[nd.i]) + m;
        }
        if (marg) marg[nd.i] = (double)S;
        if (xp) *xp = x;  // means of the current messages
      }
      q.xmax = fmax(q.xmax, (double)fabs(x));
    }
  });
  if (acc.f) atomicOr(sticky, acc.f);
}

// settled phase: information only, fixed coefficients coef[(6 c + d) Nc + s];
// MODE as in k_rb_sweep
template <typename T, int MODE, bool DAMP, bool SEG>
__global__ __launch_bounds__(kBlock) void k_rb_frozen(
    GridGeom g, int hx, int Nc, int c, const T *__restrict__ coef, const T *__restrict__ Sfix,
    T *__restrict__ hh, const T *__restrict__ rhs, T alpha, T *__restrict__ xprev,
    double *__restrict__ xacc, double *__restrict__ marg, BlockPartial *__restrict__ part,
    uint32_t *__restrict__ sticky, const Ctl *__restrict__ ctl, int nseg,
    const SegCtl *__restrict__ seg, const int32_t *__restrict__ act, int fl) {
  if (ctl != nullptr && ctl->stop != STOP_NONE) return;
  const T *__restrict__ other = hh + (size_t)(1 - c) * 6 * Nc;
  T *__restrict__ own = hh + (size_t)c * 6 * Nc;
  const T *__restrict__ cf = coef + (size_t)c * 6 * Nc;
  RbAcc acc;
  rb_cover<MODE, SEG>(Nc, nseg, act, part, acc, [&](int s, RbAcc &q) {
    RbNode nd;
    if (!rb_node(g, hx, c, s, nd)) return;
    // Faces with a zero coupling hold zero coefficients and zero
    // informations on both sides since the freeze, so the geometry decides.
    // Load order, as measured: with segments (a stack whose grids stop one
    // by one) every load before the first store; without, each direction's
    // coefficient (and old information) next to its store.
    T hin[6], kf[6], ho[6];
#pragma unroll
    for (int d = 0; d < 6; ++d)
      hin[d] = nd.ok[d] && !(fl & SWEEP_ZIN) ? other[(size_t)(d ^ 1) * Nc + nd.j[d]] : T(0);
    if (SEG && MODE != 2) {
#pragma unroll
      for (int d = 0; d < 6; ++d) kf[d] = nd.ok[d] ? cf[(size_t)d * Nc + s] : T(0);
      if (DAMP) {
#pragma unroll
        for (int d = 0; d < 6; ++d)
          ho[d] = nd.ok[d] && !(fl & SWEEP_ZOWN) ? own[(size_t)d * Nc + s] : T(0);
      }
    }
    T H = rhs[(size_t)c * Nc + s];
    T *xp = xprev ? xprev + (size_t)c * Nc + s : nullptr;
    T S = T(1), xold = T(0);
    if (SEG) {
      if (MODE >= 1) S = Sfix[(size_t)c * Nc + s];
      if (MODE == 1) xold = *xp;
    }
    // MODE 3: the means' operands with the messages, not after the stores
    double xa = 0.0;
    if (MODE == 3) {
      S = Sfix[(size_t)c * Nc + s];
      if (xacc && !(fl & SWEEP_XSET)) xa = xacc[nd.i];
    }
#pragma unroll
    for (int d = 0; d < 6; ++d) H += hin[d];
    if (MODE != 2) {
#pragma unroll
      for (int d = 0; d < 6; ++d) {
        if (!nd.ok[d]) continue;
        const size_t o = (size_t)d * Nc + s;
        T h = (SEG ? kf[d] : cf[o]) * (H - hin[d]);
        if (DAMP) {
          const T old = SEG ? ho[d] : ((fl & SWEEP_ZOWN) ? T(0) : own[o]);
          h = alpha * old + (T(1) - alpha) * h;
        }
        __builtin_nontemporal_store(h, &own[o]);
      }
    }
    if (MODE >= 1) {
      if (!SEG && MODE != 3) {
        S = Sfix[(size_t)c * Nc + s];
        if (MODE == 1) xold = *xp;
      }
      const T x = H / S;
      if (!isfinite(x)) q.f |= FLAG_NONFINITE;
      if (MODE == 1) {
        q.dmax = fmax(q.dmax, (double)fabs(x - xold));
        *xp = x;
      } else {
        if (xacc && !(SEG && seg[s / (Nc / nseg)].done == 2)) {
          const double m = (double)H / (double)S;
          xacc[nd.i] = (fl & SWEEP_XSET) ? m : (MODE == 3 ? xa : xacc[nd.i]) + m;
        }
        if (marg) marg[nd.i] = (double)S;
        if (xp) *xp = x;
      }
      q.xmax = fmax(q.xmax, (double)fabs(x));
    }
  });
  if (acc.f) atomicOr(sticky, acc.f);
}

// freeze: coefficients, S and information messages of both colours (hh NULL:
// the informations are discarded, a restart follows)
template <typename T, bool VARC>
__global__ __launch_bounds__(kBlock) void k_rb_freeze(GridGeom g, int hx, int Nc, GridCoef<T> k,
                                                      const typename Vec2<T>::type *__restrict__ msg,
                                                      T *__restrict__ coef, T *__restrict__ hh,
                                                      T *__restrict__ Sfix) {
  const int total = 2 * Nc;
  for (int t = blockIdx.x * kBlock + threadIdx.x; t < total; t += gridDim.x * kBlock) {
    const int c = t >= Nc ? 1 : 0;
    const int s = t - c * Nc;
    RbNode nd;
    if (!rb_node(g, hx, c, s, nd)) continue;
    T a[6];
    rb_couplings<T, VARC>(g, k, nd, a);
    const auto *other = msg + (size_t)(1 - c) * 6 * Nc;
    const size_t own = (size_t)c * 6 * Nc;
    T Pin[6];
    T S = VARC ? k.diag[nd.i] : k.dconst;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const T p = nd.ok[d] ? other[(size_t)(d ^ 1) * Nc + nd.j[d]].x : T(0);
      Pin[d] = a[d] != T(0) ? p : T(0);
      S += Pin[d];
    }
    Sfix[(size_t)c * Nc + s] = S;
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const size_t o = own + (size_t)d * Nc + s;
      coef[o] = a[d] != T(0) ? -a[d] / (S - Pin[d]) : T(0);
      if (hh) hh[o] = a[d] != T(0) ? msg[o].y : T(0);
    }
  }
}

// natural direction-major FP64 [6][N] <-> colour-major working precision
template <typename T, bool GET>
__global__ void k_rb_io(GridGeom g, int hx, int Nc, typename Vec2<T>::type *__restrict__ msg,
                        double *__restrict__ P, double *__restrict__ h) {
  const int64_t m = 6 * (int64_t)g.N;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= m) return;
  const int d = (int)(t / g.N);
  const int i = (int)(t - (int64_t)d * g.N);
  int c, slot;
  rb_place(g, hx, i, c, slot);
  const size_t at = ((size_t)c * 6 + d) * Nc + slot;
  if (GET) {
    P[t] = (double)msg[at].x;
    h[t] = (double)msg[at].y;
  } else {
    msg[at].x = (T)P[t];
    msg[at].y = (T)h[t];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
namespace {

template <typename T, int MODE, bool DAMP, bool VARC, bool SEG>
void rb_one(const RbArgs &a, hipStream_t s) {
  using V = typename Vec2<T>::type;
  GridCoef<T> k;
  k.diag = (const T *)a.diag; k.cx = (const T *)a.cx; k.cy = (const T *)a.cy; k.cz = (const T *)a.cz;
  k.dconst = (T)a.dconst; k.aconst = (T)a.aconst;
  const int nseg = a.seg ? a.nseg : 1;
  if (a.frozen)
    hipLaunchKernelGGL((k_rb_frozen<T, MODE, DAMP, SEG>), dim3(a.grid), dim3(kBlock), 0, s, a.g,
                       a.hx, a.Nc, a.colour, (const T *)a.coef, (const T *)a.Sfix, (T *)a.msg,
                       (const T *)a.rhs, (T)a.alpha, (T *)a.xprev, a.xacc, a.marg, a.part,
                       a.sticky, a.ctl, nseg, a.seg, a.act, a.fl);
  else
    hipLaunchKernelGGL((k_rb_sweep<T, MODE, DAMP, VARC, SEG>), dim3(a.grid), dim3(kBlock), 0, s,
                       a.g, a.hx, a.Nc, a.colour, k, (V *)a.msg, (const T *)a.rhs, (T)a.alpha,
                       (T *)a.xprev, a.xacc, a.marg, a.part, a.sticky, a.ctl, nseg, a.seg, a.act,
                       a.fl);
}

template <typename T, bool VARC, bool SEG>
void rb_mode_seg(const RbArgs &a, hipStream_t s) {
  switch (a.mode) {
    case 0: a.damp ? rb_one<T, 0, true, VARC, SEG>(a, s) : rb_one<T, 0, false, VARC, SEG>(a, s); break;
    case 1: a.damp ? rb_one<T, 1, true, VARC, SEG>(a, s) : rb_one<T, 1, false, VARC, SEG>(a, s); break;
    case 3:
      if constexpr (!SEG) {
        a.damp ? rb_one<T, 3, true, VARC, false>(a, s) : rb_one<T, 3, false, VARC, false>(a, s);
      }
      break;
    default: rb_one<T, 2, false, VARC, SEG>(a, s); break;
  }
}

template <typename T, bool VARC>
void rb_mode(const RbArgs &a, hipStream_t s) {
  a.seg ? rb_mode_seg<T, VARC, true>(a, s) : rb_mode_seg<T, VARC, false>(a, s);
}

template <typename T, bool VARC>
void rb_freeze(const RbArgs &a, void *hh, hipStream_t s) {
  GridCoef<T> k{(const T *)a.diag, (const T *)a.cx, (const T *)a.cy, (const T *)a.cz,
                (T)a.dconst, (T)a.aconst};
  hipLaunchKernelGGL((k_rb_freeze<T, VARC>), dim3(a.grid), dim3(kBlock), 0, s, a.g, a.hx, a.Nc, k,
                     (const typename Vec2<T>::type *)a.msg, (T *)a.coef, (T *)hh, (T *)a.Sfix);
}

}  // namespace

hipError_t launch_rb_sweep(const RbArgs &a, hipStream_t s) {
  if (a.Nc <= 0) return hipSuccess;
  if (a.seg && (a.nseg < 1 || a.nseg > a.grid || a.Nc % a.nseg != 0 || !a.act))
    return hipErrorInvalidValue;
  if (a.mode < 0 || a.mode > 3 || (a.mode == 3 && a.seg)) return hipErrorInvalidValue;
  if (!geom_ok(a.g) || a.hx != a.g.fh.d) return hipErrorInvalidValue;
  if (a.fp32) a.varc ? rb_mode<float, true>(a, s) : rb_mode<float, false>(a, s);
  else a.varc ? rb_mode<double, true>(a, s) : rb_mode<double, false>(a, s);
  return hipGetLastError();
}

hipError_t launch_rb_freeze(const RbArgs &a, void *hh, hipStream_t s) {
  if (a.Nc <= 0) return hipSuccess;
  if (!geom_ok(a.g) || a.hx != a.g.fh.d) return hipErrorInvalidValue;
  if (a.fp32) a.varc ? rb_freeze<float, true>(a, hh, s) : rb_freeze<float, false>(a, hh, s);
  else a.varc ? rb_freeze<double, true>(a, hh, s) : rb_freeze<double, false>(a, hh, s);
  return hipGetLastError();
}

hipError_t launch_rb_io(bool fp32, bool get, const GridGeom &g, int hx, int Nc, void *msg,
                        double *P, double *h, hipStream_t s) {
  const int64_t m = 6 * (int64_t)g.N;
  if (m <= 0) return hipSuccess;
  if (!geom_ok(g) || hx != g.fh.d) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((m + kBlock - 1) / kBlock));
  if (fp32) {
    if (get) hipLaunchKernelGGL((k_rb_io<float, true>), grid, dim3(kBlock), 0, s, g, hx, Nc, (float2 *)msg, P, h);
    else hipLaunchKernelGGL((k_rb_io<float, false>), grid, dim3(kBlock), 0, s, g, hx, Nc, (float2 *)msg, P, h);
  } else {
    if (get) hipLaunchKernelGGL((k_rb_io<double, true>), grid, dim3(kBlock), 0, s, g, hx, Nc, (double2 *)msg, P, h);
    else hipLaunchKernelGGL((k_rb_io<double, false>), grid, dim3(kBlock), 0, s, g, hx, Nc, (double2 *)msg, P, h);
  }
  return hipGetLastError();
}

}  // namespace gabp
