// Host side of the single-lattice C ABI declared in include/lbm.h, plus the
// small auxiliary kernels (partial-sum finalisation, equilibrium
// initialisation, export).  The fused step kernels live in lbm_kernels.h and
// are instantiated per storage type and flavour in lbm_step.hip.

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_aux.h"
#include "lbm_ctx.h"
#include "lbm_host.h"
#include "lbm_kernels.h"

using namespace lbmk;
using namespace lbmh;

namespace lbmh {
namespace {
thread_local std::string g_err;
}
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

int export_range(lbm_ctx* c, long long first, long long count, double* pops, float* ro,
                 float* uxo, float* uyo, double* rd, double* uxd, double* uyd) {
  const Geom g = make_geom_for(c->grid.nx, c->grid.ny, c->grid.side, c->esize);
  if (count <= 0) return LBM_OK;
  const int blocks = int((count + 255) / 256);
  const void* src = c->lat[c->cur];
  switch (c->p.storage) {
    case LBM_STORE_F64:
      hipLaunchKernelGGL(export_kernel<StoreF64>, dim3(blocks), dim3(256), 0, c->stream,
                         (const double*)src, g, c->kd, c->d_solid, (const double*)c->d_force,
                         first, count, pops, ro, uxo, uyo, rd, uxd, uyd);
      break;
    case LBM_STORE_F32:
      hipLaunchKernelGGL(export_kernel<StoreF32>, dim3(blocks), dim3(256), 0, c->stream,
                         (const float*)src, g, c->kf, c->d_solid, (const float*)c->d_force,
                         first, count, pops, ro, uxo, uyo, rd, uxd, uyd);
      break;
    case LBM_STORE_BF16:
      hipLaunchKernelGGL(export_kernel<StoreBF16>, dim3(blocks), dim3(256), 0, c->stream,
                         (const uint16_t*)src, g, c->kf, c->d_solid, (const float*)c->d_force,
                         first, count, pops, ro, uxo, uyo, rd, uxd, uyd);
      break;
    default:
      hipLaunchKernelGGL(export_kernel<StoreF16>, dim3(blocks), dim3(256), 0, c->stream,
                         (const _Float16*)src, g, c->kf, c->d_solid, (const float*)c->d_force,
                         first, count, pops, ro, uxo, uyo, rd, uxd, uyd);
      break;
  }
  HIPCHECK(hipGetLastError());
  return LBM_OK;
}
}  // namespace lbmh

namespace {

// ---------------------------------------------------------------------------
// Host side
// ---------------------------------------------------------------------------

struct Shape {
  int by, rows;
};
constexpr Shape kShapes[] = {{16, 1}, {8, 1}, {4, 1}, {4, 2}, {8, 2}, {4, 4}, {8, 4}};
constexpr int kNumShapes = sizeof(kShapes) / sizeof(kShapes[0]);


}  // namespace


namespace {

template <class C>
const Consts<C>& consts_for(const lbm_ctx* c);
template <>
const Consts<double>& consts_for<double>(const lbm_ctx* c) { return c->kd; }
template <>
const Consts<float>& consts_for<float>(const lbm_ctx* c) { return c->kf; }



Geom make_geom(const lbm_ctx* c) { return make_geom_for(c->grid.nx, c->grid.ny, c->grid.side, c->esize); }


int configure_tiles(lbm_ctx* c) {
  c->out_rows = c->by * c->rows;
  c->tiles_x = (c->grid.nx + kLanes - 1) / kLanes;
  c->tiles_y = (c->grid.ny + c->out_rows - 1) / c->out_rows;
  c->ntiles = c->tiles_x * c->tiles_y;
  if ((size_t)c->ntiles > c->partial_cap) {
    if (c->partials) HIPCHECK(hipFree(c->partials));
    c->partials = nullptr;
    HIPCHECK(hipMalloc(&c->partials, (size_t)c->ntiles * 4 * sizeof(double)));
    c->partial_cap = c->ntiles;
  }
  for (int i = 0; i < 2; ++i)
    if (c->graph[i]) {
      hipGraphExecDestroy(c->graph[i]);
      c->graph[i] = nullptr;
    }
  return LBM_OK;
}

constexpr size_t kLastLevelCacheBytes = size_t(256) << 20;

// Queue one step (flavor by its 1-based index), then swap lattices.
void enqueue_step(lbm_ctx* c, hipStream_t st) {
  const int64_t idx = c->t + 1;
  const int K = c->p.check_every;
  int flavor = kPlain;
  if (idx % K == 0) flavor = kCheck;
  else if (K >= 2 && idx % K == K - 1) flavor = kStore;
  StepArgs a{};
  a.g = make_geom(c);
  a.tiles_x = c->tiles_x;
  a.ntiles = c->ntiles;
  a.out_rows = c->out_rows;
  a.solid = c->d_solid;
  a.hist_in = c->hist[c->cur];
  a.hist_out = c->hist[c->cur ^ 1];
  a.ubuf = c->ubuf;
  a.partials = c->partials;
  a.force = c->d_force ? c->d_force : c->ubuf;
  a.has_force = c->d_force != nullptr;
  a.rng = c->rng;
  a.rng_slot = c->cur;
  const void* src = c->lat[c->cur];
  void* dst = c->lat[c->cur ^ 1];
  int var = (c->p.strain_fd ? kVarFds : 0) | (c->p.mrt ? kVarMrt : 0);
  // When the two lattices together outgrow MI355X's 256 MiB Infinity Cache
  // the default kernel stores non-temporally: measured 6 % faster at 4096^2
  // (F32), while at 1024^2 (75 MB, cache resident) ordinary stores are 24 %
  // faster.
  const size_t elem = c->p.storage == LBM_STORE_F64 ? 8 : c->p.storage == LBM_STORE_F32 ? 4 : 2;
  if (var == 0 && 2 * 9 * (size_t)a.g.plane * elem > kLastLevelCacheBytes) var = kVarNts;
  const void* k = c->p.storage == LBM_STORE_F64 ? static_cast<const void*>(&c->kd)
                                                 : static_cast<const void*>(&c->kf);
  switch (c->p.storage * 3 + flavor) {
    case 0: launch_step<0, kPlain>(c->by, c->rows, var, src, dst, a, k, st); break;
    case 1: launch_step<0, kStore>(c->by, c->rows, var, src, dst, a, k, st); break;
    case 2: launch_step<0, kCheck>(c->by, c->rows, var, src, dst, a, k, st); break;
    case 3: launch_step<1, kPlain>(c->by, c->rows, var, src, dst, a, k, st); break;
    case 4: launch_step<1, kStore>(c->by, c->rows, var, src, dst, a, k, st); break;
    case 5: launch_step<1, kCheck>(c->by, c->rows, var, src, dst, a, k, st); break;
    case 6: launch_step<2, kPlain>(c->by, c->rows, var, src, dst, a, k, st); break;
    case 7: launch_step<2, kStore>(c->by, c->rows, var, src, dst, a, k, st); break;
    case 8: launch_step<2, kCheck>(c->by, c->rows, var, src, dst, a, k, st); break;
    case 9: launch_step<3, kPlain>(c->by, c->rows, var, src, dst, a, k, st); break;
    case 10: launch_step<3, kStore>(c->by, c->rows, var, src, dst, a, k, st); break;
    default: launch_step<3, kCheck>(c->by, c->rows, var, src, dst, a, k, st); break;
  }
  if (flavor == kCheck) {
    hipLaunchKernelGGL(finalize_kernel<256>, dim3(1), dim3(256), 0, st, c->partials, c->ntiles,
                       c->result);
    c->checked = true;
  }
  c->cur ^= 1;
  c->t = idx;
}

template <class S, class FT>
void launch_init(lbm_ctx* c, const FT* rho, const FT* ux, const FT* uy) {
  using C = typename S::C;
  using T = typename S::T;
  Geom g = make_geom(c);
  const int blocks = int(((long long)g.nx * g.ny + 255) / 256);
  hipLaunchKernelGGL((init_kernel<S, FT>), dim3(blocks), dim3(256), 0, c->stream, (T*)c->lat[0],
                     (T*)c->lat[1], g, consts_for<C>(c), c->d_solid, rho, ux, uy, (C*)c->ubuf,
                     (C*)c->hist[0], (C*)c->hist[1]);
  hipLaunchKernelGGL((ghost_fill_kernel<S>), dim3(blocks), dim3(256), 0, c->stream, (T*)c->lat[0],
                     g, consts_for<C>(c), c->d_solid);
}

template <class S>
void launch_ghost_fill(lbm_ctx* c, int which) {
  using C = typename S::C;
  using T = typename S::T;
  Geom g = make_geom(c);
  const int blocks = int(((long long)g.nx * g.ny + 255) / 256);
  hipLaunchKernelGGL((ghost_fill_kernel<S>), dim3(blocks), dim3(256), 0, c->stream,
                     (T*)c->lat[which], g, consts_for<C>(c), c->d_solid);
}

// The step counter of the stochastic rounding equals the step index: set it
// wherever the state's step index is set (initialisation, checkpoint load),
// in the slot the next step reads.
int set_rng_counter(lbm_ctx* c) {
  c->rng_host[c->cur] = unsigned(c->t);
  HIPCHECK(hipMemcpyAsync(c->rng + c->cur, &c->rng_host[c->cur], sizeof(unsigned),
                          hipMemcpyHostToDevice, c->stream));
  return LBM_OK;
}

template <class FT>
int init_common(lbm_ctx* c, const FT* rho, const FT* ux, const FT* uy) {
  switch (c->p.storage) {
    case LBM_STORE_F64: launch_init<StoreF64, FT>(c, rho, ux, uy); break;
    case LBM_STORE_F32: launch_init<StoreF32, FT>(c, rho, ux, uy); break;
    case LBM_STORE_BF16: launch_init<StoreBF16, FT>(c, rho, ux, uy); break;
    default: launch_init<StoreF16, FT>(c, rho, ux, uy); break;
  }
  HIPCHECK(hipGetLastError());
  c->cur = 0;
  c->t = 0;
  c->checked = false;
  for (int i = 0; i < 2; ++i)
    if (c->graph[i]) {
      hipGraphExecDestroy(c->graph[i]);
      c->graph[i] = nullptr;
    }
  return set_rng_counter(c);
}

int export_common(lbm_ctx* c, double* pops, float* ro, float* uxo, float* uyo, double* rd,
                  double* uxd, double* uyd) {
  return lbmh::export_range(c, 0, (long long)c->grid.nx * c->grid.ny, pops, ro, uxo, uyo, rd,
                            uxd, uyd);
}

// Device copy of the per-node force field in the current compute type and the
// force flag of the constants (a field replaces the uniform force).
int apply_force(lbm_ctx* c) {
  if (c->d_force) HIPCHECK(hipFree(c->d_force));
  c->d_force = nullptr;
  const bool uniform = c->p.fx != 0.0 || c->p.fy != 0.0;
  c->kd.force = c->kf.force = uniform ? 1 : 0;
  if (c->h_force.empty()) return LBM_OK;
  const size_t m = c->h_force.size();
  std::vector<char> buf(m * c->csize);
  if (c->csize == 8) {
    std::memcpy(buf.data(), c->h_force.data(), m * sizeof(double));
  } else {
    float* f = reinterpret_cast<float*>(buf.data());
    for (size_t i = 0; i < m; ++i) f[i] = float(c->h_force[i]);
  }
  HIPCHECK(hipMalloc(&c->d_force, buf.size()));
  HIPCHECK(hipMemcpy(c->d_force, buf.data(), buf.size(), hipMemcpyHostToDevice));
  c->kd.force = c->kf.force = 1;
  return LBM_OK;
}

void free_ctx(lbm_ctx* c) {
  if (!c) return;
  for (int i = 0; i < 2; ++i) {
    if (c->graph[i]) hipGraphExecDestroy(c->graph[i]);
    if (c->lat[i]) hipFree(c->lat[i]);
    if (c->hist[i]) hipFree(c->hist[i]);
  }
  if (c->d_solid) hipFree(c->d_solid);
  if (c->d_force) hipFree(c->d_force);
  if (c->ubuf) hipFree(c->ubuf);
  if (c->partials) hipFree(c->partials);
  if (c->result) hipFree(c->result);
  if (c->rng) hipFree(c->rng);
  if (c->ev0) hipEventDestroy(c->ev0);
  if (c->ev1) hipEventDestroy(c->ev1);
  if (c->own_stream) hipStreamDestroy(c->own_stream);
  delete c;
}

}  // namespace

extern "C" {

const char* lbm_last_error(void) { return lbmh::g_err.c_str(); }

int lbm_launch_shapes(int32_t* shapes, int32_t cap) {
  for (int i = 0; i < kNumShapes && i < cap; ++i) {
    shapes[2 * i] = kShapes[i].by;
    shapes[2 * i + 1] = kShapes[i].rows;
  }
  return kNumShapes;
}

int lbm_create(const lbm_grid* grid, const uint8_t* solid_mask, const lbm_params* params,
               lbm_ctx** out) {
  if (!out) return fail(LBM_EINVAL, "null output pointer");
  *out = nullptr;
  int rc = validate(grid, solid_mask, params);
  if (rc) return rc;
  lbm_ctx* c = new (std::nothrow) lbm_ctx();
  if (!c) return fail(LBM_ENOMEM, "host allocation failed");
  c->grid = *grid;
  c->p = *params;
  if (c->p.omega3 == 0) c->p.omega3 = 1.0;
  if (c->p.omega6 == 0) c->p.omega6 = 1.0;
  if (c->p.omega7 == 0) c->p.omega7 = 1.0;
  if (c->p.omega8 == 0) c->p.omega8 = 1.0;
  if (c->p.rho0 == 0) c->p.rho0 = 1.0;
  double scale = 1.0;
  if (c->p.storage == LBM_STORE_BF16 || c->p.storage == LBM_STORE_F16) {
    scale = c->p.storage_scale > 0 ? c->p.storage_scale
                                   : (c->p.storage == LBM_STORE_F16 ? 4096.0 : 1.0);
    int e;
    if (std::frexp(scale, &e) != 0.5) {
      free_ctx(c);
      return fail(LBM_EINVAL, "storage_scale must be a power of two");
    }
  }
  c->kd = make_consts<double>(c->p, scale);
  c->kf = make_consts<float>(c->p, scale);
  c->esize = storage_bytes(c->p.storage);
  c->csize = c->p.storage == LBM_STORE_F64 ? 8 : 4;
  c->by = 4;
  c->rows = 1;
  auto dev = [&](hipError_t e, const char* what) {
    if (e != hipSuccess) {
      g_err = std::string(what) + ": " + hipGetErrorString(e);
      return false;
    }
    return true;
  };
  const size_t n = (size_t)grid->nx * grid->ny;
  bool ok = dev(hipGetDevice(&c->device), "hipGetDevice") &&
            dev(hipStreamCreateWithFlags(&c->own_stream, hipStreamNonBlocking), "hipStreamCreate");
  c->stream = c->own_stream;
  const Geom g0 = make_geom(c);
  for (int i = 0; ok && i < 2; ++i) {
    ok = dev(hipMalloc(&c->lat[i], 9 * (size_t)g0.plane * c->esize), "hipMalloc lattice") &&
         dev(hipMemset(c->lat[i], 0, 9 * (size_t)g0.plane * c->esize), "hipMemset lattice") &&
         dev(hipMalloc(&c->hist[i], 2 * (size_t)grid->ny * c->csize), "hipMalloc history");
  }
  ok = ok && dev(hipMalloc(&c->ubuf, 2 * n * c->csize), "hipMalloc velocity") &&
       dev(hipMalloc(&c->result, 4 * sizeof(double)), "hipMalloc result") &&
       dev(hipMalloc(&c->rng, 2 * sizeof(unsigned)), "hipMalloc step counter") &&
       dev(hipMemset(c->rng, 0, 2 * sizeof(unsigned)), "hipMemset step counter") &&
       dev(hipEventCreate(&c->ev0), "hipEventCreate") &&
       dev(hipEventCreate(&c->ev1), "hipEventCreate");
  if (ok && solid_mask) {
    bool any = false;
    for (size_t i = 0; i < n; ++i) any |= solid_mask[i] != 0;
    if (any) {
      c->h_solid.assign(solid_mask, solid_mask + n);
      for (auto& v : c->h_solid) v = v ? 1 : 0;
      ok = dev(hipMalloc(&c->d_solid, n), "hipMalloc mask") &&
           dev(hipMemcpy(c->d_solid, c->h_solid.data(), n, hipMemcpyHostToDevice), "copy mask");
    }
  }
  if (!ok) {
    free_ctx(c);
    return LBM_EDEVICE;
  }
  rc = configure_tiles(c);
  if (!rc) rc = init_common<double>(c, nullptr, nullptr, nullptr);
  if (!rc) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) rc = fail(LBM_EDEVICE, hipGetErrorString(e));
  }
  if (rc) {
    free_ctx(c);
    return rc;
  }
  *out = c;
  return LBM_OK;
}

void lbm_destroy(lbm_ctx* c) {
  if (!c) return;
  if (c->stream) hipStreamSynchronize(c->stream);
  free_ctx(c);
}

int lbm_set_stream(lbm_ctx* c, void* s) {
  if (!c) return fail(LBM_EINVAL, "null context");
  HIPCHECK(hipStreamSynchronize(c->stream));
  c->stream = s ? (hipStream_t)s : c->own_stream;
  return LBM_OK;
}

int lbm_init_fields(lbm_ctx* c, const double* rho, const double* ux, const double* uy) {
  if (!c) return fail(LBM_EINVAL, "null context");
  const size_t n = (size_t)c->grid.nx * c->grid.ny;
  double* tmp[3] = {nullptr, nullptr, nullptr};
  const double* src[3] = {rho, ux, uy};
  int rc = LBM_OK;
  for (int i = 0; i < 3 && rc == LBM_OK; ++i) {
    if (!src[i]) continue;
    if (hipMalloc(&tmp[i], n * sizeof(double)) != hipSuccess ||
        hipMemcpy(tmp[i], src[i], n * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      rc = fail(LBM_EDEVICE, "upload of initial fields failed");
  }
  if (rc == LBM_OK) rc = init_common<double>(c, tmp[0], tmp[1], tmp[2]);
  hipError_t e = hipStreamSynchronize(c->stream);
  if (rc == LBM_OK && e != hipSuccess) rc = fail(LBM_EDEVICE, hipGetErrorString(e));
  for (int i = 0; i < 3; ++i)
    if (tmp[i]) hipFree(tmp[i]);
  return rc;
}

int lbm_init_fields_device(lbm_ctx* c, const float* rho, const float* ux, const float* uy) {
  if (!c) return fail(LBM_EINVAL, "null context");
  const int rc = init_common<float>(c, rho, ux, uy);
  if (rc) return rc;
  // the caller may release the arrays as soon as this returns
  HIPCHECK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int lbm_step(lbm_ctx* c, int64_t n) {
  if (!c) return fail(LBM_EINVAL, "null context");
  if (n < 0) return fail(LBM_EINVAL, "n must be >= 0");
  if (n == 0) return LBM_OK;
  const int K = c->p.check_every;
  hipStream_t st = c->stream;
  if (c->timing) HIPCHECK(hipEventRecord(c->ev0, st));
  int64_t left = n;
  // replay a captured graph of K steps for every aligned block of K steps
  while (left > 0) {
    if (c->t % K == 0 && left >= K && K >= 4) {
      const int par = c->cur;
      if (!c->graph[par]) {
        hipGraph_t gr = nullptr;
        const int64_t t0 = c->t;
        const int cur0 = c->cur;
        const bool chk0 = c->checked;
        HIPCHECK(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
        for (int i = 0; i < K; ++i) enqueue_step(c, st);
        hipError_t e = hipStreamEndCapture(st, &gr);
        c->t = t0;
        c->cur = cur0;
        c->checked = chk0;
        if (e != hipSuccess) return fail(LBM_EDEVICE, hipGetErrorString(e));
        e = hipGraphInstantiate(&c->graph[par], gr, nullptr, nullptr, 0);
        hipGraphDestroy(gr);
        if (e != hipSuccess) {
          c->graph[par] = nullptr;
          return fail(LBM_EDEVICE, hipGetErrorString(e));
        }
      }
      HIPCHECK(hipGraphLaunch(c->graph[par], st));
      c->t += K;
      if (K % 2) c->cur ^= 1;
      c->checked = true;
      left -= K;
    } else {
      enqueue_step(c, st);
      --left;
    }
  }
  HIPCHECK(hipGetLastError());
  if (c->timing) {
    HIPCHECK(hipEventRecord(c->ev1, st));
    HIPCHECK(hipEventSynchronize(c->ev1));
    float ms = 0.f;
    HIPCHECK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    c->last_ms = double(ms) / double(n);
  }
  return LBM_OK;
}

int lbm_set_timing(lbm_ctx* c, int32_t timing) {
  if (!c) return fail(LBM_EINVAL, "null context");
  c->timing = timing != 0;
  return LBM_OK;
}

int lbm_last_step_ms(lbm_ctx* c, double* ms) {
  if (!c || !ms) return fail(LBM_EINVAL, "null argument");
  if (c->last_ms < 0) return fail(LBM_ESTATE, "no timed step yet");
  *ms = c->last_ms;
  return LBM_OK;
}

static int read_result(lbm_ctx* c, double r[4]) {
  if (!c->checked) return fail(LBM_ESTATE, "no check step has run yet");
  HIPCHECK(hipStreamSynchronize(c->stream));
  HIPCHECK(hipMemcpy(r, c->result, 4 * sizeof(double), hipMemcpyDeviceToHost));
  return LBM_OK;
}

int lbm_average_last_two(lbm_ctx* c) {
  if (!c) return fail(LBM_EINVAL, "null context");
  const Geom g = make_geom(c);
  const long long n = 9LL * g.plane;
  HIPCHECK(launch_average(c->p.storage, c->lat[c->cur], c->lat[c->cur ^ 1], n,
                          (double)c->kf.scale, c->hist[c->cur], c->hist[c->cur ^ 1],
                          c->hist[0] ? 2LL * c->grid.ny : 0, c->stream));
  return LBM_OK;
}

int lbm_residual(lbm_ctx* c, double* r) {
  if (!c || !r) return fail(LBM_EINVAL, "null argument");
  double v[4];
  int rc = read_result(c, v);
  if (rc) return rc;
  if (!std::isfinite(v[0]) || !std::isfinite(v[1])) {
    *r = NAN;
    return fail(LBM_EUNSTABLE, "residual is not finite");
  }
  *r = v[1] > 0 ? std::sqrt(v[0] / v[1]) : (v[0] > 0 ? INFINITY : 0.0);
  return LBM_OK;
}

int lbm_mass(lbm_ctx* c, double* m) {
  if (!c || !m) return fail(LBM_EINVAL, "null argument");
  double v[4];
  int rc = read_result(c, v);
  if (rc) return rc;
  size_t fluid = (size_t)c->grid.nx * c->grid.ny;
  if (!c->h_solid.empty()) {
    fluid = 0;
    for (auto s : c->h_solid) fluid += s == 0;
  }
  *m = double(fluid) * c->p.rho0 + v[2];
  if (!std::isfinite(*m)) return fail(LBM_EUNSTABLE, "mass is not finite");
  return LBM_OK;
}

int lbm_guard_count(lbm_ctx* c, int64_t* n) {
  if (!c || !n) return fail(LBM_EINVAL, "null argument");
  double v[4];
  int rc = read_result(c, v);
  if (rc) return rc;
  *n = (int64_t)v[3];
  return LBM_OK;
}

int lbm_steps(lbm_ctx* c, int64_t* n) {
  if (!c || !n) return fail(LBM_EINVAL, "null argument");
  *n = c->t;
  return LBM_OK;
}

int lbm_fields(lbm_ctx* c, double* rho, double* ux, double* uy) {
  if (!c) return fail(LBM_EINVAL, "null context");
  const size_t n = (size_t)c->grid.nx * c->grid.ny;
  double* d = nullptr;
  HIPCHECK(hipMalloc(&d, 3 * n * sizeof(double)));
  int rc = export_common(c, nullptr, nullptr, nullptr, nullptr, d, d + n, d + 2 * n);
  if (rc == LBM_OK) {
    hipError_t e = hipStreamSynchronize(c->stream);
    double* h[3] = {rho, ux, uy};
    for (int i = 0; i < 3 && e == hipSuccess; ++i)
      if (h[i]) e = hipMemcpy(h[i], d + i * n, n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = fail(LBM_EDEVICE, hipGetErrorString(e));
  }
  hipFree(d);
  return rc;
}

int lbm_fields_device(lbm_ctx* c, float* rho, float* ux, float* uy) {
  if (!c) return fail(LBM_EINVAL, "null context");
  const int rc = export_common(c, nullptr, rho, ux, uy, nullptr, nullptr, nullptr);
  if (rc) return rc;
  HIPCHECK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}

int lbm_populations(lbm_ctx* c, double* f) {
  if (!c || !f) return fail(LBM_EINVAL, "null argument");
  const size_t n = (size_t)c->grid.nx * c->grid.ny;
  double* d = nullptr;
  HIPCHECK(hipMalloc(&d, 9 * n * sizeof(double)));
  int rc = export_common(c, d, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr);
  if (rc == LBM_OK) {
    hipError_t e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess) e = hipMemcpy(f, d, 9 * n * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) rc = fail(LBM_EDEVICE, hipGetErrorString(e));
  }
  hipFree(d);
  return rc;
}

static const char kMagic[8] = {'L', 'B', 'M', 'C', 'K', 'P', 'T', '1'};

int lbm_save(lbm_ctx* c, const char* path) {
  if (!c || !path) return fail(LBM_EINVAL, "null argument");
  HIPCHECK(hipStreamSynchronize(c->stream));
  const size_t n = (size_t)c->grid.nx * c->grid.ny;
  const Geom g = make_geom(c);
  std::vector<char> lat(9 * (size_t)g.plane * c->esize), hist(2 * (size_t)c->grid.ny * c->csize);
  HIPCHECK(hipMemcpy(lat.data(), c->lat[c->cur], lat.size(), hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(hist.data(), c->hist[c->cur], hist.size(), hipMemcpyDeviceToHost));
  std::vector<char> ub(2 * n * c->csize);
  HIPCHECK(hipMemcpy(ub.data(), c->ubuf, ub.size(), hipMemcpyDeviceToHost));
  FILE* fp = std::fopen(path, "wb");
  if (!fp) return fail(LBM_EINVAL, std::string("cannot open ") + path);
  int32_t hdr[8] = {c->grid.nx, c->grid.ny, c->p.storage, (int32_t)c->esize, 0, 0, 0, 0};
  int64_t t = c->t;
  bool ok = std::fwrite(kMagic, 1, 8, fp) == 8 && std::fwrite(hdr, sizeof hdr, 1, fp) == 1 &&
            std::fwrite(&t, sizeof t, 1, fp) == 1 &&
            std::fwrite(lat.data(), 1, lat.size(), fp) == lat.size() &&
            std::fwrite(hist.data(), 1, hist.size(), fp) == hist.size() &&
            std::fwrite(ub.data(), 1, ub.size(), fp) == ub.size();
  ok = (std::fclose(fp) == 0) && ok;
  return ok ? LBM_OK : fail(LBM_EDEVICE, "write failed");
}

int lbm_load(lbm_ctx* c, const char* path) {
  if (!c || !path) return fail(LBM_EINVAL, "null argument");
  FILE* fp = std::fopen(path, "rb");
  if (!fp) return fail(LBM_EINVAL, std::string("cannot open ") + path);
  char mg[8];
  int32_t hdr[8];
  int64_t t;
  const size_t n = (size_t)c->grid.nx * c->grid.ny;
  const Geom g = make_geom(c);
  std::vector<char> lat(9 * (size_t)g.plane * c->esize), hist(2 * (size_t)c->grid.ny * c->csize),
      ub(2 * n * c->csize);
  bool ok = std::fread(mg, 1, 8, fp) == 8 && std::memcmp(mg, kMagic, 8) == 0 &&
            std::fread(hdr, sizeof hdr, 1, fp) == 1 && hdr[0] == c->grid.nx &&
            hdr[1] == c->grid.ny && hdr[2] == c->p.storage && std::fread(&t, sizeof t, 1, fp) == 1 &&
            std::fread(lat.data(), 1, lat.size(), fp) == lat.size() &&
            std::fread(hist.data(), 1, hist.size(), fp) == hist.size() &&
            std::fread(ub.data(), 1, ub.size(), fp) == ub.size();
  std::fclose(fp);
  if (!ok) return fail(LBM_EINVAL, "checkpoint does not match this lattice");
  HIPCHECK(hipStreamSynchronize(c->stream));
  HIPCHECK(hipMemcpy(c->lat[0], lat.data(), lat.size(), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(c->lat[1], lat.data(), lat.size(), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(c->hist[0], hist.data(), hist.size(), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(c->hist[1], hist.data(), hist.size(), hipMemcpyHostToDevice));
  HIPCHECK(hipMemcpy(c->ubuf, ub.data(), ub.size(), hipMemcpyHostToDevice));
  c->cur = 0;
  c->t = t;
  c->checked = false;
  for (int i = 0; i < 2; ++i)
    if (c->graph[i]) {
      hipGraphExecDestroy(c->graph[i]);
      c->graph[i] = nullptr;
    }
  const int rc = set_rng_counter(c);
  if (rc) return rc;
  HIPCHECK(hipStreamSynchronize(c->stream));
  return LBM_OK;
}


int lbm_set_storage(lbm_ctx* c, int32_t storage, double storage_scale) {
  if (!c) return fail(LBM_EINVAL, "null context");
  if (storage < LBM_STORE_F64 || storage > LBM_STORE_F16) return fail(LBM_EINVAL, "unknown storage");
  double scale = 1.0;
  if (storage == LBM_STORE_BF16 || storage == LBM_STORE_F16) {
    scale = storage_scale > 0 ? storage_scale : (storage == LBM_STORE_F16 ? 4096.0 : 1.0);
    int e;
    if (std::frexp(scale, &e) != 0.5) return fail(LBM_EINVAL, "storage_scale must be a power of two");
  }
  HIPCHECK(hipStreamSynchronize(c->stream));
  const Geom g1 = make_geom(c);
  const int s1 = c->p.storage;
  const double inv1 = s1 == LBM_STORE_F64 ? double(c->kd.inv_scale) : double(c->kf.inv_scale);
  const size_t esize2 = storage_bytes(storage), csize2 = storage == LBM_STORE_F64 ? 8 : 4;
  {
    const int rc = check_lattice_bytes(c->grid.nx, c->grid.ny, esize2);
    if (rc) return rc;
  }
  const Geom g2 = make_geom_for(c->grid.nx, c->grid.ny, c->grid.side, esize2);
  const size_t np = (size_t)c->grid.nx * c->grid.ny;
  void* lat2[2] = {nullptr, nullptr};
  void* hist2[2] = {nullptr, nullptr};
  void* ubuf2 = nullptr;
  bool ok = true;
  for (int i = 0; ok && i < 2; ++i)
    ok = hipMalloc(&lat2[i], 9 * (size_t)g2.plane * esize2) == hipSuccess &&
         hipMemset(lat2[i], 0, 9 * (size_t)g2.plane * esize2) == hipSuccess &&
         hipMalloc(&hist2[i], 2 * (size_t)c->grid.ny * csize2) == hipSuccess;
  ok = ok && hipMalloc(&ubuf2, 2 * np * csize2) == hipSuccess;
  if (!ok) {
    for (int i = 0; i < 2; ++i) {
      hipFree(lat2[i]);
      hipFree(hist2[i]);
    }
    hipFree(ubuf2);
    return fail(LBM_ENOMEM, "allocation for the new storage failed");
  }
  const long long nf = (long long)(c->grid.nx + 2) * (c->grid.ny + 2);
  for (int i = 0; i < 2; ++i) {
    hipLaunchKernelGGL(convert_lattice_kernel, dim3(int((nf + 255) / 256)), dim3(256), 0, c->stream,
                       c->lat[i], s1, g1, inv1, lat2[i], (int)storage, g2, scale);
    const long long nh = 2LL * c->grid.ny;
    hipLaunchKernelGGL(convert_values_kernel, dim3(int((nh + 255) / 256)), dim3(256), 0, c->stream,
                       c->hist[i], int(c->csize == 8), hist2[i], int(csize2 == 8), nh);
  }
  hipLaunchKernelGGL(convert_values_kernel, dim3(int((2 * np + 255) / 256)), dim3(256), 0,
                     c->stream, c->ubuf, int(c->csize == 8), ubuf2, int(csize2 == 8),
                     (long long)(2 * np));
  HIPCHECK(hipGetLastError());
  HIPCHECK(hipStreamSynchronize(c->stream));
  for (int i = 0; i < 2; ++i) {
    hipFree(c->lat[i]);
    hipFree(c->hist[i]);
    c->lat[i] = lat2[i];
    c->hist[i] = hist2[i];
  }
  hipFree(c->ubuf);
  c->ubuf = ubuf2;
  c->p.storage = storage;
  c->p.storage_scale = storage_scale;
  c->esize = esize2;
  c->csize = csize2;
  c->kd = make_consts<double>(c->p, scale);
  c->kf = make_consts<float>(c->p, scale);
  for (int i = 0; i < 2; ++i)
    if (c->graph[i]) {
      hipGraphExecDestroy(c->graph[i]);
      c->graph[i] = nullptr;
    }
  return apply_force(c);
}

int lbm_set_force_field(lbm_ctx* c, const double* fx, const double* fy) {
  if (!c) return fail(LBM_EINVAL, "null context");
  if ((fx == nullptr) != (fy == nullptr))
    return fail(LBM_EINVAL, "force field: give both components or neither");
  const size_t n = (size_t)c->grid.nx * c->grid.ny;
  if (fx)
    for (size_t i = 0; i < n; ++i)
      if (!std::isfinite(fx[i]) || !std::isfinite(fy[i]))
        return fail(LBM_EINVAL, "force field holds a non-finite value");
  HIPCHECK(hipStreamSynchronize(c->stream));
  c->h_force.clear();
  if (fx) {
    c->h_force.assign(fx, fx + n);
    c->h_force.insert(c->h_force.end(), fy, fy + n);
  }
  for (int i = 0; i < 2; ++i)
    if (c->graph[i]) {
      hipGraphExecDestroy(c->graph[i]);
      c->graph[i] = nullptr;
    }
  return apply_force(c);
}

int lbm_set_launch(lbm_ctx* c, int32_t by, int32_t rows) {
  if (!c) return fail(LBM_EINVAL, "null context");
  bool known = false;
  for (int i = 0; i < kNumShapes; ++i) known |= kShapes[i].by == by && kShapes[i].rows == rows;
  if (!known) return fail(LBM_EINVAL, "unsupported launch shape");
  HIPCHECK(hipStreamSynchronize(c->stream));
  c->by = by;
  c->rows = rows;
  return configure_tiles(c);
}

int lbm_get_launch(lbm_ctx* c, int32_t* by, int32_t* rows) {
  if (!c || !by || !rows) return fail(LBM_EINVAL, "null argument");
  *by = c->by;
  *rows = c->rows;
  return LBM_OK;
}

}  // extern "C"
