// Host-side state of one lattice (the opaque lbm_ctx of the C ABI), shared
// by the translation units that implement its entry points.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_device.h"

struct lbm_ctx {
  lbm_grid grid{};
  lbm_params p{};
  int device = 0;
  hipStream_t own_stream = nullptr;
  hipStream_t stream = nullptr;
  size_t esize = 4;   // bytes per stored population
  size_t csize = 4;   // bytes per compute value
  void* lat[2] = {nullptr, nullptr};
  uint8_t* d_solid = nullptr;  // nullptr when no solid node
  std::vector<uint8_t> h_solid;
  std::vector<double> h_force;  // per-node body force [2][ny][nx]; empty: uniform
  void* d_force = nullptr;      // the same in the compute type

  void* hist[2] = {nullptr, nullptr};
  void* ubuf = nullptr;
  double* partials = nullptr;
  double* result = nullptr;
  // step counter of the stochastic rounding (two slots, see StepArgs::rng)
  // and the host copy it is written from
  unsigned* rng = nullptr;
  unsigned rng_host[2] = {0u, 0u};
  int cur = 0;
  int64_t t = 0;
  bool checked = false;
  int by = 4, rows = 1;
  int tiles_x = 0, tiles_y = 0, ntiles = 0, out_rows = 0;
  size_t partial_cap = 0;
  lbmk::Consts<double> kd{};
  lbmk::Consts<float> kf{};
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  bool timing = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  double last_ms = -1.0;
};

namespace lbmh {
// Decode the current lattice of c for the nodes first .. first + count - 1
// (row-major) into the given device arrays (any may be null; see
// export_kernel), queued on the context's stream.
int export_range(lbm_ctx* c, long long first, long long count, double* pops, float* ro,
                 float* uxo, float* uyo, double* rd, double* uxd, double* uyd);
}  // namespace lbmh
