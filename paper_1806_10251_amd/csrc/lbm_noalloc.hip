// lbm_fields_noalloc: lbm_fields for callers that may not allocate device
// memory.  The FP64 staging rows live in a file-scope device array instead of
// a per-call allocation; the lattice is exported through it in chunks of whole
// rows, each chunk copied to the caller's host arrays.
//
// The array is one per GPU, shared by every call on that GPU and holding the
// last call's contents; calls that overlap on one GPU race for it.  Nothing
// in it has to start at zero: every chunk's export writes each element that
// its copy reads.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/lbm.h"
#include "lbm_ctx.h"
#include "lbm_host.h"

namespace {

constexpr long long kStageNodes = 1LL << 17;                   // nodes per chunk
constexpr long long kStageDoubles = 3 * kStageNodes;            // rho, ux, uy: 3 MiB
constexpr int kMaxDevices = 64;

__device__ __align__(256) double scratch[kStageDoubles];

std::mutex g_mu;
double* g_scratch[kMaxDevices] = {};   // device address of `scratch`, per device

// Address of this device's copy of `scratch`, looked up once per device with
// that device current (the caller's current device is restored).
int scratch_for(int dev, double** out) {
  if (dev < 0 || dev >= kMaxDevices)
    return lbmh::fail(LBM_EDEVICE, "lbm_fields_noalloc: device index out of range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    int cur = -1;
    HIPCHECK(hipGetDevice(&cur));
    if (cur != dev) HIPCHECK(hipSetDevice(dev));
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (cur != dev) HIPCHECK(hipSetDevice(cur));
    if (e != hipSuccess || !ptr)
      return lbmh::fail(LBM_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") +
                                         hipGetErrorString(e));
    g_scratch[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch[dev];
  return LBM_OK;
}

}  // namespace

extern "C" int lbm_fields_noalloc(lbm_ctx* c, double* rho, double* ux, double* uy) {
  if (!c) return lbmh::fail(LBM_EINVAL, "null context");
  const long long nx = c->grid.nx, ny = c->grid.ny;
  if (nx > kStageNodes)
    return lbmh::fail(LBM_EINVAL, "lbm_fields_noalloc: rows longer than 131072 nodes do not fit "
                                  "its staging buffer");
  double* stage = nullptr;
  int rc = scratch_for(c->device, &stage);
  if (rc) return rc;
  double* host[3] = {rho, ux, uy};
  const long long rows_per_chunk = kStageNodes / nx;
  for (long long y0 = 0; y0 < ny; y0 += rows_per_chunk) {
    const long long rows = y0 + rows_per_chunk <= ny ? rows_per_chunk : ny - y0;
    const long long first = y0 * nx, count = rows * nx;
    rc = lbmh::export_range(c, first, count, nullptr, nullptr, nullptr, nullptr,
                            rho ? stage : nullptr, ux ? stage + kStageNodes : nullptr,
                            uy ? stage + 2 * kStageNodes : nullptr);
    if (rc) return rc;
    for (int i = 0; i < 3; ++i)
      if (host[i])
        HIPCHECK(hipMemcpyAsync(host[i] + first, stage + i * kStageNodes,
                                size_t(count) * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHECK(hipStreamSynchronize(c->stream));
  }
  return LBM_OK;
}
