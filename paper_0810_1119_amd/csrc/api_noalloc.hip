// Allocation-free FP64 residual: gabp_residual's kernels with their scratch
// (validation flags, per-workgroup partial sums of r^2 and the two readout
// records) in one static device array per GPU instead of buffers allocated
// per call.  For callers that cannot allocate: code under stream capture,
// tight serving loops, harnesses that forbid hipMalloc.
#include <cmath>
#include <mutex>
#include <vector>

#include "engine.h"

namespace gabp {
namespace {

// Scratch layout (bytes): [0, 256) validation flags, [256, 1024) two readout
// records, [1024, 32768) residual partial sums.  The residual never launches
// more than kMaxSweepBlocks workgroups, so any n fits.
constexpr size_t kScratchBytes = 32768;
constexpr size_t kOffFlags = 0;
constexpr size_t kOffReadout = 256;
constexpr size_t kOffPartials = 1024;
constexpr int kScratchPartials = (int)((kScratchBytes - kOffPartials) / sizeof(double));
static_assert(2 * sizeof(HostReadout) <= kOffPartials - kOffReadout, "readout records overflow");
static_assert(kScratchPartials >= kMaxSweepBlocks, "partials do not fit the scratch array");

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

std::mutex g_scratch_mu;
std::vector<unsigned char *> g_scratch_ptr;  // per device, set once

// Device address of this device's copy of `scratch` (the array's name is a
// host-side stand-in and must never reach a kernel or a copy).  Looked up once
// per device, with that device current.
int scratch_of_current_device(unsigned char **out) {
  int dev = 0;
  int rc = from_hip(hipGetDevice(&dev));
  if (rc) return rc;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if ((size_t)dev >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    if ((rc = from_hip(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))))) return rc;
    if (!p) return GABP_ERR_HIP;
    g_scratch_ptr[dev] = (unsigned char *)p;
  }
  *out = g_scratch_ptr[dev];
  return GABP_OK;
}

}  // namespace
}  // namespace gabp

using namespace gabp;

extern "C" {

int gabp_residual_noalloc(const gabp_csr *A, const double *b, const double *x, double *r,
                          double *rel_norm, hipStream_t s) {
  clear_stale_error();
  int rc = check_csr(A);
  if (rc) return rc;
  if (!rel_norm || (A->n > 0 && (!b || !x))) return GABP_ERR_ARG;
  if (A->n == 0) { *rel_norm = 0.0; return GABP_OK; }
  const int nb = residual_blocks(A->n);
  if (nb > kScratchPartials) return GABP_ERR_UNSUPPORTED;
  unsigned char *base = nullptr;
  if ((rc = scratch_of_current_device(&base))) return rc;
  uint32_t *flags = (uint32_t *)(base + kOffFlags);
  HostReadout *ro = (HostReadout *)(base + kOffReadout);
  double *sum = (double *)(base + kOffPartials);
  // the flags start at zero (a fill kernel, not a memset node under capture);
  // the partials and readout records are written whole by every call
  uint32_t hflags = 0;
  if ((rc = from_hip(launch_fill_zero4(flags, 1, s))) ||
      (rc = from_hip(launch_plan_rows(A->n, A->nnz, A->row_ptr, A->col, A->val, nullptr, nullptr,
                                      flags, s))) ||
      (rc = from_hip(hipMemcpyAsync(&hflags, flags, sizeof(uint32_t), hipMemcpyDeviceToHost, s))) ||
      (rc = from_hip(hipStreamSynchronize(s))))
    return rc;
  if (hflags & FLAG_ARG) return GABP_ERR_ARG;
  HostReadout h[2];
  if ((rc = from_hip(launch_residual(false, nb, A->n, A->row_ptr, A->col, A->val, b, nullptr,
                                     nullptr, nullptr, sum, s))) ||
      (rc = from_hip(launch_readout(nullptr, 0, sum, nb, nullptr, nullptr, 0, 0, &ro[0], s))) ||
      (rc = from_hip(launch_residual(false, nb, A->n, A->row_ptr, A->col, A->val, b, x, nullptr,
                                     r, sum, s))) ||
      (rc = from_hip(launch_readout(nullptr, 0, sum, nb, nullptr, nullptr, 0, 1, &ro[1], s))) ||
      (rc = from_hip(hipMemcpyAsync(h, ro, sizeof(h), hipMemcpyDeviceToHost, s))) ||
      (rc = from_hip(hipStreamSynchronize(s))))
    return rc;
  const double bn = std::sqrt(h[0].sum), rn = std::sqrt(h[1].sum);
  *rel_norm = bn > 0 ? rn / bn : rn;
  return std::isfinite(*rel_norm) ? GABP_OK : GABP_ERR_ARG;
}

}  // extern "C"
