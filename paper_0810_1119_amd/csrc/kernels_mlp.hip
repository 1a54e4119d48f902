// Warm-start network: a per-node MLP 8 -> 64 -> 64 -> 12 (ReLU) that proposes
// the initial messages of a structured-grid solve.  Parameters are held in
// bfloat16 for inference and training arithmetic, with FP32 master copies
// and Adam moments for the updates; every multiply-add accumulates in FP32.
//
// Inputs of node i (directions +x, -x, +y, -y, +z, -z; a_d = A_{i, j(d)}, 0
// where there is no neighbour):
//     u = (log A_ii, a_1 / A_ii, ..., a_6 / A_ii, b_i / A_ii)
// Outputs: for each direction d, (P_d / A_ii, h_d / A_ii) of the message from
// i toward its neighbour, in the information form h = P mu; directions
// without a neighbour send nothing.  The network only chooses where the
// iteration starts: GaBP's fixed point, and the answer, do not depend on it.
//
// Parameter order (flat, 5516 values): W1 [64][8], b1 [64], W2 [64][64],
// b2 [64], W3 [12][64], b3 [12].
//
// Training works on a batch of S samples with activations stored
// feature-major ([64][S]) so that the per-sample threads write coalesced
// rows; the weight gradients are sums over samples, formed per block of
// samples and added in a fixed order, so a training step is deterministic.
#include "gabp_internal.h"

namespace gabp {
namespace {

constexpr int kIn = 8, kHid = 64, kOut = 12;
constexpr int oW1 = 0, oB1 = 512, oW2 = 576, oB2 = 4672, oW3 = 4736, oB3 = 5504;
constexpr int kParams = 5516;
constexpr int kThreads = 256;
constexpr int kChunk = 2048;   // samples per weight-gradient block
constexpr int kTile = 16;      // samples staged in LDS at a time

__device__ __forceinline__ float bf16_to_f32(uint16_t v) {
  return __uint_as_float((uint32_t)v << 16);
}

// round to nearest, ties to even (NaN kept quiet)
__device__ __forceinline__ uint16_t f32_to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

// all parameters into LDS as FP32 (22 KB)
__device__ void stage_params(const uint16_t *__restrict__ w, float *sp) {
  for (int i = threadIdx.x; i < kParams; i += blockDim.x) sp[i] = bf16_to_f32(w[i]);
  __syncthreads();
}

// Forward pass of one sample.  STORE: keep h1 and h2 for the backward pass.
template <bool STORE>
__device__ __forceinline__ void forward(const float *sp, const float u[kIn], float o[kOut],
                                        float *H1, float *H2, int64_t S, int64_t s) {
  float h1[kHid];
#pragma unroll
  for (int j = 0; j < kHid; ++j) {
    float z = sp[oB1 + j];
#pragma unroll
    for (int c = 0; c < kIn; ++c) z = fmaf(sp[oW1 + j * kIn + c], u[c], z);
    h1[j] = fmaxf(z, 0.f);
    if (STORE) H1[(int64_t)j * S + s] = h1[j];
  }
#pragma unroll
  for (int i = 0; i < kOut; ++i) o[i] = sp[oB3 + i];
#pragma unroll 1
  for (int j = 0; j < kHid; ++j) {
    float z = sp[oB2 + j];
#pragma unroll
    for (int k = 0; k < kHid; ++k) z = fmaf(sp[oW2 + j * kHid + k], h1[k], z);
    const float h2 = fmaxf(z, 0.f);
    if (STORE) H2[(int64_t)j * S + s] = h2;
#pragma unroll
    for (int i = 0; i < kOut; ++i) o[i] = fmaf(sp[oW3 + i * kHid + j], h2, o[i]);
  }
}

// fixed-order block sum of two doubles into part[blockIdx.x * 2 + {0,1}]
__device__ void block_sum2(double a, double b, double *part) {
  __shared__ double sh[2][kThreads / 64];
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    sh[0][w] = a;
    sh[1][w] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0.0, y = 0.0;
    for (int k = 0; k < (int)(blockDim.x >> 6); ++k) {
      x += sh[0][k];
      y += sh[1][k];
    }
    part[2 * blockIdx.x] = x;
    part[2 * blockIdx.x + 1] = y;
  }
}

__global__ __launch_bounds__(kThreads) void k_mlp_forward(const uint16_t *__restrict__ w,
                                                          const float *__restrict__ U, int64_t S,
                                                          float *__restrict__ out) {
  __shared__ float sp[kParams];
  stage_params(w, sp);
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S;
       s += (int64_t)gridDim.x * blockDim.x) {
    float u[kIn], o[kOut];
#pragma unroll
    for (int c = 0; c < kIn; ++c) u[c] = U[s * kIn + c];
    forward<false>(sp, u, o, nullptr, nullptr, S, s);
#pragma unroll
    for (int i = 0; i < kOut; ++i) out[s * kOut + i] = o[i];
  }
}

// Training forward: activations, masked output errors r = m (o - t) stored
// feature-major, and per-block (sum r^2, count of unmasked outputs).
__global__ __launch_bounds__(kThreads) void k_mlp_train_fwd(
    const uint16_t *__restrict__ w, const float *__restrict__ U, const float *__restrict__ T,
    int64_t S, float *__restrict__ H1, float *__restrict__ H2, float *__restrict__ R,
    double *__restrict__ part) {
  __shared__ float sp[kParams];
  stage_params(w, sp);
  double l2 = 0.0, cnt = 0.0;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S;
       s += (int64_t)gridDim.x * blockDim.x) {
    float u[kIn], o[kOut];
#pragma unroll
    for (int c = 0; c < kIn; ++c) u[c] = U[s * kIn + c];
    forward<true>(sp, u, o, H1, H2, S, s);
#pragma unroll
    for (int i = 0; i < kOut; ++i) {
      const bool on = u[1 + i / 2] != 0.f;  // the direction has a neighbour
      const float r = on ? o[i] - T[s * kOut + i] : 0.f;
      R[(int64_t)i * S + s] = r;
      l2 += (double)r * r;
      cnt += on ? 1.0 : 0.0;
    }
  }
  block_sum2(l2, cnt, part);
}

// Training backward through the layers: D2 = dL/dz2, D1 = dL/dz1 (up to the
// common factor 1 / count applied to the gradients at the end).
__global__ __launch_bounds__(kThreads) void k_mlp_train_bwd(
    const uint16_t *__restrict__ w, const float *__restrict__ H1, const float *__restrict__ H2,
    const float *__restrict__ R, int64_t S, float *__restrict__ D1, float *__restrict__ D2) {
  __shared__ float sp[kParams];
  stage_params(w, sp);
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < S;
       s += (int64_t)gridDim.x * blockDim.x) {
    float r[kOut], g1[kHid];
#pragma unroll
    for (int i = 0; i < kOut; ++i) r[i] = R[(int64_t)i * S + s];
#pragma unroll
    for (int k = 0; k < kHid; ++k) g1[k] = 0.f;
#pragma unroll 2
    for (int j = 0; j < kHid; ++j) {
      float g = 0.f;
#pragma unroll
      for (int i = 0; i < kOut; ++i) g = fmaf(sp[oW3 + i * kHid + j], r[i], g);
      const float d2 = H2[(int64_t)j * S + s] > 0.f ? g : 0.f;
      D2[(int64_t)j * S + s] = d2;
#pragma unroll
      for (int k = 0; k < kHid; ++k) g1[k] = fmaf(sp[oW2 + j * kHid + k], d2, g1[k]);
    }
#pragma unroll
    for (int k = 0; k < kHid; ++k) D1[(int64_t)k * S + s] = H1[(int64_t)k * S + s] > 0.f ? g1[k] : 0.f;
  }
}

// Weight gradients of one block of samples (unscaled):
//   W1[k][c] += D1[k] U[c], b1[k] += D1[k]; W2[j][k] += D2[j] H1[k],
//   b2[j] += D2[j]; W3[i][j] += R[i] H2[j], b3[i] += R[i].
// Sample tiles are staged in LDS; each thread owns a fixed set of
// parameters and adds the samples in order.
__global__ __launch_bounds__(kThreads) void k_mlp_wgrad(
    const float *__restrict__ U, const float *__restrict__ H1, const float *__restrict__ H2,
    const float *__restrict__ R, const float *__restrict__ D1, const float *__restrict__ D2,
    int64_t S, float *__restrict__ gpart) {
  __shared__ float tU[kTile][kIn], tH1[kHid][kTile], tH2[kHid][kTile], tR[kOut][kTile],
      tD1[kHid][kTile], tD2[kHid][kTile];
  constexpr int kPer = (kParams + kThreads - 1) / kThreads;  // 22 parameters per thread
  float acc[kPer];
#pragma unroll
  for (int q = 0; q < kPer; ++q) acc[q] = 0.f;
  const int64_t s0 = (int64_t)blockIdx.x * kChunk;
  const int64_t s1 = s0 + kChunk < S ? s0 + kChunk : S;
  for (int64_t t0 = s0; t0 < s1; t0 += kTile) {
    const int n = (int)(s1 - t0 < kTile ? s1 - t0 : kTile);
    for (int e = threadIdx.x; e < kHid * kTile; e += blockDim.x) {
      const int f = e / kTile, q = e % kTile;
      const bool in = q < n;
      const int64_t s = t0 + q;
      tH1[f][q] = in ? H1[(int64_t)f * S + s] : 0.f;
      tH2[f][q] = in ? H2[(int64_t)f * S + s] : 0.f;
      tD1[f][q] = in ? D1[(int64_t)f * S + s] : 0.f;
      tD2[f][q] = in ? D2[(int64_t)f * S + s] : 0.f;
      if (f < kOut) tR[f][q] = in ? R[(int64_t)f * S + s] : 0.f;
      if (f < kIn) tU[q][f] = in ? U[s * kIn + f] : 0.f;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kPer; ++q) {
      const int p = threadIdx.x + q * kThreads;
      if (p >= kParams) continue;
      float a = acc[q];
      if (p < oB1) {
        const int k = p / kIn, c = p % kIn;
        for (int t = 0; t < kTile; ++t) a = fmaf(tD1[k][t], tU[t][c], a);
      } else if (p < oW2) {
        const int k = p - oB1;
        for (int t = 0; t < kTile; ++t) a += tD1[k][t];
      } else if (p < oB2) {
        const int j = (p - oW2) / kHid, k = (p - oW2) % kHid;
        for (int t = 0; t < kTile; ++t) a = fmaf(tD2[j][t], tH1[k][t], a);
      } else if (p < oW3) {
        const int j = p - oB2;
        for (int t = 0; t < kTile; ++t) a += tD2[j][t];
      } else if (p < oB3) {
        const int i = (p - oW3) / kHid, j = (p - oW3) % kHid;
        for (int t = 0; t < kTile; ++t) a = fmaf(tR[i][t], tH2[j][t], a);
      } else {
        const int i = p - oB3;
        for (int t = 0; t < kTile; ++t) a += tR[i][t];
      }
      acc[q] = a;
    }
    __syncthreads();
  }
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int p = threadIdx.x + q * kThreads;
    if (p < kParams) gpart[(int64_t)blockIdx.x * kParams + p] = acc[q];
  }
}

// loss and count from the forward partials (one block)
__global__ __launch_bounds__(kThreads) void k_mlp_loss(const double *__restrict__ part, int nparts,
                                                       double *__restrict__ out) {
  __shared__ double sh[2][kThreads / 64];
  double a = 0.0, b = 0.0;
  for (int k = threadIdx.x; k < nparts; k += blockDim.x) {
    a += part[2 * k];
    b += part[2 * k + 1];
  }
  for (int o = 32; o > 0; o >>= 1) {
    a += __shfl_xor(a, o, 64);
    b += __shfl_xor(b, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = a;
    sh[1][threadIdx.x >> 6] = b;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double x = 0.0, y = 0.0;
    for (int k = 0; k < kThreads / 64; ++k) {
      x += sh[0][k];
      y += sh[1][k];
    }
    out[0] = 0.5 * x / (y > 0.0 ? y : 1.0);  // the loss
    out[1] = y;                               // unmasked outputs
  }
}

// Gradient = (sum of block partials in order) / count; optionally the Adam
// step on the FP32 masters and the bfloat16 copy used by the kernels.
__global__ __launch_bounds__(kThreads) void k_mlp_adam(
    const float *__restrict__ gpart, int nblk, const double *__restrict__ lossv,
    float *__restrict__ grad, int update, float *__restrict__ master, float *__restrict__ m1,
    float *__restrict__ m2, uint16_t *__restrict__ wbf, float lr, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  float g = 0.f;
  for (int b = 0; b < nblk; ++b) g += gpart[(int64_t)b * kParams + p];
  const double n = lossv[1];
  g = (float)((double)g / (n > 0.0 ? n : 1.0));
  if (grad) grad[p] = g;
  if (!update) return;
  const float a = 0.9f * m1[p] + 0.1f * g;
  const float v = 0.999f * m2[p] + 0.001f * g * g;
  m1[p] = a;
  m2[p] = v;
  const float mh = a / c1, vh = v / c2;  // bias corrections 1 - beta^t
  const float th = master[p] - lr * mh / (sqrtf(vh) + 1e-8f);
  master[p] = th;
  wbf[p] = f32_to_bf16(th);
}

__global__ void k_mlp_set(const float *__restrict__ src, float *__restrict__ master,
                          uint16_t *__restrict__ wbf, float *__restrict__ m1,
                          float *__restrict__ m2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kParams) return;
  master[p] = src[p];
  wbf[p] = f32_to_bf16(src[p]);
  m1[p] = 0.f;
  m2[p] = 0.f;
}

__global__ void k_mlp_get(const uint16_t *__restrict__ wbf, float *__restrict__ dst) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kParams) dst[p] = bf16_to_f32(wbf[p]);
}

// ---- grid features, targets and the warm start itself ----
struct GridNode {
  int64_t i;
  int x, y, z;
};

__device__ __forceinline__ GridNode grid_node(const GridGeom &g, int64_t i) {
  const int64_t n = (int64_t)g.nx * g.ny * g.nz;
  const int64_t loc = i % n;
  GridNode q;
  q.i = i;
  q.x = (int)(loc % g.nx);
  q.y = (int)((loc / g.nx) % g.ny);
  q.z = (int)(loc / ((int64_t)g.nx * g.ny));
  return q;
}

// diagonal and the six couplings of node i (0 where no neighbour); arrays
// NULL mean the constant
template <typename T>
__device__ __forceinline__ void node_couplings(const GridGeom &g, const GridCoef<T> &k,
                                               const GridNode &q, T &diag, T a[6]) {
  const int64_t i = q.i, sx = 1, sy = g.nx, sz = (int64_t)g.nx * g.ny;
  diag = k.diag ? k.diag[i] : k.dconst;
  auto c = [&](const T *arr, int64_t j) { return arr ? arr[j] : k.aconst; };
  a[0] = q.x + 1 < g.nx ? c(k.cx, i) : T(0);
  a[1] = q.x > 0 ? c(k.cx, i - sx) : T(0);
  a[2] = q.y + 1 < g.ny ? c(k.cy, i) : T(0);
  a[3] = q.y > 0 ? c(k.cy, i - sy) : T(0);
  a[4] = q.z + 1 < g.nz ? c(k.cz, i) : T(0);
  a[5] = q.z > 0 ? c(k.cz, i - sz) : T(0);
}

template <typename T>
__device__ __forceinline__ void node_features(T diag, const T a[6], T b, float u[kIn]) {
  const float d = (float)diag;
  u[0] = logf(d);
#pragma unroll
  for (int e = 0; e < 6; ++e) u[1 + e] = (float)a[e] / d;
  u[7] = (float)b / d;
}

__global__ __launch_bounds__(kThreads) void k_grid_features(GridGeom g, GridCoef<double> k,
                                                            const double *__restrict__ b,
                                                            const int64_t *__restrict__ nodes,
                                                            int64_t count, float *__restrict__ U) {
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < count;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = nodes ? nodes[s] : s;
    if (i < 0 || i >= (int64_t)g.N) {  // not a node: zero row
#pragma unroll
      for (int c = 0; c < kIn; ++c) U[s * kIn + c] = 0.f;
      continue;
    }
    double diag, a[6];
    node_couplings(g, k, grid_node(g, i), diag, a);
    float u[kIn];
    node_features(diag, a, b[i], u);
#pragma unroll
    for (int c = 0; c < kIn; ++c) U[s * kIn + c] = u[c];
  }
}

__global__ __launch_bounds__(kThreads) void k_grid_targets(GridGeom g, GridCoef<double> k,
                                                           const double *__restrict__ P,
                                                           const double *__restrict__ h,
                                                           const int64_t *__restrict__ nodes,
                                                           int64_t count, float *__restrict__ T) {
  const int64_t N = g.N;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < count;
       s += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = nodes ? nodes[s] : s;
    if (i < 0 || i >= N) {  // not a node: zero row
#pragma unroll
      for (int c = 0; c < kOut; ++c) T[s * kOut + c] = 0.f;
      continue;
    }
    double diag, a[6];
    node_couplings(g, k, grid_node(g, i), diag, a);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const bool on = a[d] != 0.0;
      T[s * kOut + 2 * d] = on ? (float)(P[d * N + i] / diag) : 0.f;
      T[s * kOut + 2 * d + 1] = on ? (float)(h[d * N + i] / diag) : 0.f;
    }
  }
}

// Initial messages of a grid plan from the network: msg[d][i] = (P, h).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_grid_warm(GridGeom g, GridCoef<T> k,
                                                        const T *__restrict__ rhs,
                                                        const uint16_t *__restrict__ w,
                                                        typename Vec2<T>::type *__restrict__ msg,
                                                        int hx) {
  using T2 = typename Vec2<T>::type;
  __shared__ float sp[kParams];
  stage_params(w, sp);
  const int64_t N = g.N;
  // natural order: node i, direction d at d N + i; two-colour order (hx > 0):
  // rhs at c Nc + slot, direction d at (6 c + d) Nc + slot
  const int64_t Nc = hx > 0 ? (int64_t)hx * (N / g.nx) : 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    int64_t at = i, bat = i, stride = N;
    if (hx > 0) {
      int c, slot;
      rb_place(g, hx, (int)i, c, slot);
      at = 6 * c * Nc + slot;
      bat = c * Nc + slot;
      stride = Nc;
    }
    T diag, a[6];
    node_couplings(g, k, grid_node(g, i), diag, a);
    float u[kIn], o[kOut];
    node_features(diag, a, rhs[bat], u);
    forward<false>(sp, u, o, nullptr, nullptr, 0, 0);
#pragma unroll
    for (int d = 0; d < 6; ++d) {
      const bool on = a[d] != T(0);
      msg[d * stride + at] = on ? T2{(T)o[2 * d] * diag, (T)o[2 * d + 1] * diag} : T2{T(0), T(0)};
    }
  }
}

unsigned blocks_for(int64_t n, int cap = 4096) {
  const int64_t b = (n + kThreads - 1) / kThreads;
  return (unsigned)(b < cap ? (b > 0 ? b : 1) : cap);
}

}  // namespace

int mlp_params() { return kParams; }
int mlp_chunk() { return kChunk; }

hipError_t launch_mlp_set(const float *src, float *master, uint16_t *wbf, float *m1, float *m2,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_set, dim3((kParams + 255) / 256), dim3(256), 0, s, src, master, wbf, m1, m2);
  return hipGetLastError();
}

hipError_t launch_mlp_get(const uint16_t *wbf, float *dst, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_get, dim3((kParams + 255) / 256), dim3(256), 0, s, wbf, dst);
  return hipGetLastError();
}

hipError_t launch_mlp_forward(const uint16_t *w, const float *U, int64_t S, float *out,
                              hipStream_t s) {
  if (S <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mlp_forward, dim3(blocks_for(S)), dim3(kThreads), 0, s, w, U, S, out);
  return hipGetLastError();
}

int mlp_fwd_blocks(int64_t S) { return (int)blocks_for(S); }

hipError_t launch_mlp_train(const MlpTrainArgs &a, hipStream_t s) {
  if (a.S <= 0) return hipErrorInvalidValue;
  const unsigned fb = blocks_for(a.S);
  hipLaunchKernelGGL(k_mlp_train_fwd, dim3(fb), dim3(kThreads), 0, s, a.w, a.U, a.T, a.S, a.H1,
                     a.H2, a.R, a.part);
  hipLaunchKernelGGL(k_mlp_train_bwd, dim3(fb), dim3(kThreads), 0, s, a.w, a.H1, a.H2, a.R, a.S,
                     a.D1, a.D2);
  const unsigned gb = (unsigned)((a.S + kChunk - 1) / kChunk);
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(gb), dim3(kThreads), 0, s, a.U, a.H1, a.H2, a.R, a.D1,
                     a.D2, a.S, a.gpart);
  hipLaunchKernelGGL(k_mlp_loss, dim3(1), dim3(kThreads), 0, s, a.part, (int)fb, a.lossv);
  hipLaunchKernelGGL(k_mlp_adam, dim3((kParams + kThreads - 1) / kThreads), dim3(kThreads), 0, s,
                     a.gpart, (int)gb, a.lossv, a.grad, a.update ? 1 : 0, a.master, a.m1, a.m2,
                     a.wbf, a.lr, a.c1, a.c2);
  return hipGetLastError();
}

hipError_t launch_grid_features(const GridGeom &g, const GridCoef<double> &k, const double *b,
                                const int64_t *nodes, int64_t count, float *U, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grid_features, dim3(blocks_for(count)), dim3(kThreads), 0, s, g, k, b,
                     nodes, count, U);
  return hipGetLastError();
}

hipError_t launch_grid_targets(const GridGeom &g, const GridCoef<double> &k, const double *P,
                               const double *h, const int64_t *nodes, int64_t count, float *T,
                               hipStream_t s) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_grid_targets, dim3(blocks_for(count)), dim3(kThreads), 0, s, g, k, P, h,
                     nodes, count, T);
  return hipGetLastError();
}

hipError_t launch_grid_warm(bool fp32, const GridGeom &g, const void *diag, const void *cx,
                            const void *cy, const void *cz, double dconst, double aconst,
                            const void *rhs, const uint16_t *w, void *msg, hipStream_t s, int hx) {
  if (g.N <= 0) return hipSuccess;
  if (!geom_ok(g) || (hx > 0 && hx != g.fh.d)) return hipErrorInvalidValue;
  const dim3 grid(blocks_for(g.N, 2048));
  if (fp32) {
    GridCoef<float> k{(const float *)diag, (const float *)cx, (const float *)cy, (const float *)cz,
                      (float)dconst, (float)aconst};
    hipLaunchKernelGGL(k_grid_warm<float>, grid, dim3(kThreads), 0, s, g, k, (const float *)rhs, w,
                       (float2 *)msg, hx);
  } else {
    GridCoef<double> k{(const double *)diag, (const double *)cx, (const double *)cy,
                       (const double *)cz, dconst, aconst};
    hipLaunchKernelGGL(k_grid_warm<double>, grid, dim3(kThreads), 0, s, g, k, (const double *)rhs,
                       w, (double2 *)msg, hx);
  }
  return hipGetLastError();
}

}  // namespace gabp
