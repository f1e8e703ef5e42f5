// Batched steady solver: many independent lattices (cases of different size,
// Re, gamma and geometry) advanced together by one persistent kernel.
//
// Work items are (case, tile) pairs over all active cases.  The grid is
// co-resident (cooperative launch); in every time step each block takes a
// contiguous chunk of the item list (chunks handed out XCD by XCD, so that a
// case's neighbouring tiles share an L2), runs the same fused step body as the
// single-lattice kernel, then all blocks meet at a grid barrier.  On check
// steps each block then reduces, in a fixed order, the residual partials of
// some cases and retires the ones whose residual fell below the tolerance
// (or became non-finite); a second barrier makes the retirement visible.
// The barrier waits are bounded: a block that waits too long raises an error
// flag and leaves, so the grid always drains.
//
// All cases share one step counter and one storage type (FP32 deviations).

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/lbm.h"
#include "lbm_aux.h"
#include "lbm_host.h"
#include "lbm_kernels.h"

using namespace lbmk;
using namespace lbmh;

namespace {

using BS = StoreF32;  // batch storage
using BC = float;     // batch compute type

// Per-case descriptor (device).
struct CaseDev {
  StepArgs a[2];       // per lattice parity: geometry, tiling, mask, ubuf,
                       // partials (case base), outlet history in/out
  Consts<BC> k;
  void* lat[2];
  int outlet;
  int ntiles;
};

struct BatchArgs {
  const CaseDev* cases;
  int ncases;
  const int* item_case;   // active work items
  const int* item_tile;
  int n_items;
  int schedule;           // 0: contiguous chunks per block (XCD-local), 1: round-robin
  long long t0;           // steps done before this launch
  int nsteps;
  int K;                  // check cadence
  double tol;
  long long min_steps;    // no retirement before this many steps
  int* active;            // [ncases]
  long long* done_step;   // [ncases]
  double* case_res;       // [ncases][4]
  unsigned* bar;          // [2] grid-barrier count and generation
  int* err;               // set when a barrier wait timed out
  long long spin_limit;
};

__device__ __forceinline__ int load_flag(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid-wide barrier (sense by generation counter).  Release before the
// arrival, acquire after the wait; bounded spin.
__device__ void grid_sync(unsigned* bar, unsigned nblocks, int* err, long long spin_limit) {
  __syncthreads();
  if (threadIdx.x == 0 && threadIdx.y == 0) {
    const unsigned gen = __hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __atomic_thread_fence(__ATOMIC_RELEASE);
    const unsigned arrived =
        __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    if (arrived == nblocks - 1) {
      __hip_atomic_store(&bar[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_fetch_add(&bar[1], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      long long spins = 0;
      while (__hip_atomic_load(&bar[1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > spin_limit) {
          __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
    }
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
  }
  __syncthreads();
}

template <int BY, int R, int FL>
__device__ __forceinline__ void run_item(const CaseDev& cd, int par, int tile, BC (*s_rho)[kLanes + 2],
                                         double (*s_red)[4]) {
  const float* fa = static_cast<const float*>(cd.lat[par]);
  float* fb = static_cast<float*>(cd.lat[par ^ 1]);
  if (cd.outlet)
    step_tile<BS, BY, R, FL, true, true>(fa, fb, cd.a[par], cd.k, tile, s_rho, s_red);
  else
    step_tile<BS, BY, R, FL, true, false>(fa, fb, cd.a[par], cd.k, tile, s_rho, s_red);
}

template <int BY, int R>
__global__ __launch_bounds__(kLanes* BY) void batch_kernel(BatchArgs b) {
  __shared__ BC s_rho[BY * R + 2][kLanes + 2];
  __shared__ double s_red[BY][4];
  __shared__ double s_sum[4][kLanes];
  const int G = gridDim.x;
  // logical block: XCD x = blockIdx % 8 gets the logical range [x*G/8, (x+1)*G/8)
  const int lb = xcd_tile(blockIdx.x, G);
  for (int s = 0; s < b.nsteps; ++s) {
    const long long t = b.t0 + s;   // steps done before this one
    const int par = int(t & 1);
    const long long idx = (t + 1) % b.K;
    const int flavor = idx == 0 ? kCheck : ((b.K >= 2 && idx == b.K - 1) ? kStore : kPlain);
    int it0, it1, istep;
    if (b.schedule == 0) {
      it0 = int((long long)b.n_items * lb / G);
      it1 = int((long long)b.n_items * (lb + 1) / G);
      istep = 1;
    } else {
      it0 = blockIdx.x;
      it1 = b.n_items;
      istep = G;
    }
    for (int it = it0; it < it1; it += istep) {
      const int c = b.item_case[it];
      if (!load_flag(&b.active[c])) continue;
      const CaseDev& cd = b.cases[c];
      const int tile = b.item_tile[it];
      if (flavor == kCheck) run_item<BY, R, kCheck>(cd, par, tile, s_rho, s_red);
      else if (flavor == kStore) run_item<BY, R, kStore>(cd, par, tile, s_rho, s_red);
      else run_item<BY, R, kPlain>(cd, par, tile, s_rho, s_red);
      __syncthreads();  // LDS is reused by the next item
    }
    grid_sync(b.bar, G, b.err, b.spin_limit);
    if (flavor == kCheck) {
      // per-case residual and retirement (fixed-order sums)
      for (int c = blockIdx.x; c < b.ncases; c += G) {
        if (!load_flag(&b.active[c])) continue;
        const CaseDev& cd = b.cases[c];
        const int lane = threadIdx.x, w = threadIdx.y;
        if (w == 0) {
          double acc[4] = {0.0, 0.0, 0.0, 0.0};
          for (int i = lane; i < cd.ntiles; i += kLanes)
            for (int q = 0; q < 4; ++q) acc[q] += cd.a[0].partials[(long long)i * 4 + q];
          for (int q = 0; q < 4; ++q) s_sum[q][lane] = acc[q];
        }
        __syncthreads();
        if (w == 0 && lane == 0) {
          double v[4] = {0.0, 0.0, 0.0, 0.0};
          for (int i = 0; i < kLanes; ++i)
            for (int q = 0; q < 4; ++q) v[q] += s_sum[q][i];
          for (int q = 0; q < 4; ++q) b.case_res[(long long)c * 4 + q] = v[q];
          const bool finite = isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]);
          const double r = v[1] > 0.0 ? sqrt(v[0] / v[1]) : (v[0] > 0.0 ? INFINITY : 0.0);
          if (!finite) {
            b.done_step[c] = -(t + 1);
            __hip_atomic_store(&b.active[c], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          } else if (t + 1 >= b.min_steps && r < b.tol) {
            b.done_step[c] = t + 1;
            __hip_atomic_store(&b.active[c], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          }
        }
        __syncthreads();
      }
      grid_sync(b.bar, G, b.err, b.spin_limit);
    }
    if (load_flag(b.err)) return;
  }
}

struct Shape {
  int by, rows;
};
constexpr Shape kBatchShapes[] = {{4, 1}, {8, 1}, {16, 1}};

template <int BY, int R>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&batch_kernel<BY, R>);
}

const void* batch_kernel_for(int by, int rows) {
  switch (by * 100 + rows) {
    case 801: return kernel_ptr<8, 1>();
    case 1601: return kernel_ptr<16, 1>();
    default: return kernel_ptr<4, 1>();
  }
}

struct HostCase {
  lbm_grid grid;
  lbm_params p;
  Geom g;
  Consts<BC> k;
  void* lat[2] = {nullptr, nullptr};
  void* hist[2] = {nullptr, nullptr};
  float* ubuf = nullptr;
  uint8_t* solid = nullptr;
  int tiles_x = 0, ntiles = 0, tile_base = 0;
  size_t fluid = 0;
};

}  // namespace

struct lbm_batch {
  std::vector<HostCase> cs;
  int n = 0;
  int K = 100;
  int by = 4, rows = 1;
  int blocks = 0;    // 0 = all co-resident blocks
  int schedule = 0;
  int device = 0;
  hipStream_t own_stream = nullptr, stream = nullptr;
  CaseDev* d_cases = nullptr;
  int* d_item_case = nullptr;
  int* d_item_tile = nullptr;
  int n_items = 0, item_cap = 0;
  double* d_partials = nullptr;
  double* d_case_res = nullptr;
  int* d_active = nullptr;
  long long* d_done = nullptr;
  unsigned* d_bar = nullptr;
  int* d_err = nullptr;
  int64_t t = 0;
  std::vector<int> h_active;
};

namespace {

void free_batch(lbm_batch* b) {
  if (!b) return;
  for (auto& c : b->cs) {
    for (int i = 0; i < 2; ++i) {
      if (c.lat[i]) hipFree(c.lat[i]);
      if (c.hist[i]) hipFree(c.hist[i]);
    }
    if (c.ubuf) hipFree(c.ubuf);
    if (c.solid) hipFree(c.solid);
  }
  hipFree(b->d_cases);
  hipFree(b->d_item_case);
  hipFree(b->d_item_tile);
  hipFree(b->d_partials);
  hipFree(b->d_case_res);
  hipFree(b->d_active);
  hipFree(b->d_done);
  hipFree(b->d_bar);
  hipFree(b->d_err);
  if (b->own_stream) hipStreamDestroy(b->own_stream);
  delete b;
}

// (Re)build the tiling of every case for the current launch shape, the
// descriptors and the active item list.
int configure(lbm_batch* b) {
  const int ro = b->by * b->rows;
  int total = 0;
  for (auto& c : b->cs) {
    c.tiles_x = (c.grid.nx + kLanes - 1) / kLanes;
    c.ntiles = c.tiles_x * ((c.grid.ny + ro - 1) / ro);
    c.tile_base = total;
    total += c.ntiles;
  }
  hipFree(b->d_partials);
  b->d_partials = nullptr;
  HIPCHECK(hipMalloc(&b->d_partials, (size_t)std::max(total, 1) * 4 * sizeof(double)));
  std::vector<CaseDev> desc(b->n);
  for (int i = 0; i < b->n; ++i) {
    const HostCase& c = b->cs[i];
    CaseDev d{};
    for (int par = 0; par < 2; ++par) {
      StepArgs& a = d.a[par];
      a.g = c.g;
      a.tiles_x = c.tiles_x;
      a.ntiles = c.ntiles;
      a.out_rows = ro;
      a.solid = c.solid;
      a.ubuf = c.ubuf;
      a.partials = b->d_partials + (long long)c.tile_base * 4;
      a.hist_in = c.hist[par];
      a.hist_out = c.hist[par ^ 1];
    }
    d.k = c.k;
    d.lat[0] = c.lat[0];
    d.lat[1] = c.lat[1];
    d.outlet = c.grid.side[1] == LBM_SIDE_OUTLET;
    d.ntiles = c.ntiles;
    desc[i] = d;
  }
  if (!b->d_cases) HIPCHECK(hipMalloc(&b->d_cases, sizeof(CaseDev) * b->n));
  HIPCHECK(hipMemcpy(b->d_cases, desc.data(), sizeof(CaseDev) * b->n, hipMemcpyHostToDevice));
  b->item_cap = 0;  // force the item list to be rebuilt
  return LBM_OK;
}

int rebuild_items(lbm_batch* b) {
  std::vector<int> ic, itl;
  for (int i = 0; i < b->n; ++i) {
    if (!b->h_active[i]) continue;
    for (int t = 0; t < b->cs[i].ntiles; ++t) {
      ic.push_back(i);
      itl.push_back(t);
    }
  }
  b->n_items = (int)ic.size();
  if (b->n_items > b->item_cap) {
    hipFree(b->d_item_case);
    hipFree(b->d_item_tile);
    b->d_item_case = b->d_item_tile = nullptr;
    HIPCHECK(hipMalloc(&b->d_item_case, sizeof(int) * b->n_items));
    HIPCHECK(hipMalloc(&b->d_item_tile, sizeof(int) * b->n_items));
    b->item_cap = b->n_items;
  }
  if (b->n_items) {
    HIPCHECK(hipMemcpy(b->d_item_case, ic.data(), sizeof(int) * b->n_items, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(b->d_item_tile, itl.data(), sizeof(int) * b->n_items, hipMemcpyHostToDevice));
  }
  return LBM_OK;
}

template <class FT>
int init_case(lbm_batch* b, int ci, const FT* rho, const FT* ux, const FT* uy) {
  HostCase& c = b->cs[ci];
  const int blocks = int(((long long)c.grid.nx * c.grid.ny + 255) / 256);
  hipLaunchKernelGGL((init_kernel<BS, FT>), dim3(blocks), dim3(256), 0, b->stream,
                     (float*)c.lat[0], (float*)c.lat[1], c.g, c.k, c.solid, rho, ux, uy, c.ubuf,
                     (float*)c.hist[0], (float*)c.hist[1]);
  hipLaunchKernelGGL((ghost_fill_kernel<BS>), dim3(blocks), dim3(256), 0, b->stream,
                     (float*)c.lat[0], c.g, c.k, c.solid);
  HIPCHECK(hipGetLastError());
  // lattice parity of the batch: state lives in lat[t & 1]; copy when t is odd
  if (b->t & 1) {
    const size_t bytes = 9 * (size_t)c.g.plane * sizeof(float);
    HIPCHECK(hipMemcpyAsync(c.lat[1], c.lat[0], bytes, hipMemcpyDeviceToDevice, b->stream));
    HIPCHECK(hipMemcpyAsync(c.hist[1], c.hist[0], 2 * sizeof(float) * c.grid.ny,
                            hipMemcpyDeviceToDevice, b->stream));
  }
  return LBM_OK;
}

}  // namespace

extern "C" {

int lbm_batch_create(int32_t n, const lbm_grid* grids, const uint8_t* const* masks,
                     const lbm_params* params, lbm_batch** out) {
  if (!out) return fail(LBM_EINVAL, "null output pointer");
  *out = nullptr;
  if (n < 1 || !grids || !params) return fail(LBM_EINVAL, "need n >= 1 cases");
  const int K = params[0].check_every;
  for (int i = 0; i < n; ++i) {
    int rc = validate(&grids[i], masks ? masks[i] : nullptr, &params[i]);
    if (rc) return fail(rc, "case " + std::to_string(i) + ": " + lbm_last_error());
    if (params[i].storage != LBM_STORE_F32)
      return fail(LBM_EINVAL, "batch cases must use LBM_STORE_F32");
    if (params[i].check_every != K) return fail(LBM_EINVAL, "batch cases must share check_every");
  }
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return fail(LBM_ENOMEM, "host allocation failed");
  b->n = n;
  b->K = K;
  b->cs.resize(n);
  auto dev = [&](hipError_t e, const char* what) {
    if (e != hipSuccess) {
      fail(LBM_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
      return false;
    }
    return true;
  };
  bool ok = dev(hipGetDevice(&b->device), "hipGetDevice") &&
            dev(hipStreamCreateWithFlags(&b->own_stream, hipStreamNonBlocking), "hipStreamCreate");
  b->stream = b->own_stream;
  for (int i = 0; ok && i < n; ++i) {
    HostCase& c = b->cs[i];
    c.grid = grids[i];
    c.p = params[i];
    if (c.p.omega3 == 0) c.p.omega3 = 1.0;
    if (c.p.omega6 == 0) c.p.omega6 = 1.0;
    if (c.p.omega7 == 0) c.p.omega7 = 1.0;
    if (c.p.omega8 == 0) c.p.omega8 = 1.0;
    if (c.p.rho0 == 0) c.p.rho0 = 1.0;
    c.k = make_consts<BC>(c.p, 1.0);
    c.g = make_geom_for(c.grid.nx, c.grid.ny, c.grid.side, sizeof(float));
    const size_t np = (size_t)c.grid.nx * c.grid.ny;
    for (int j = 0; ok && j < 2; ++j)
      ok = dev(hipMalloc(&c.lat[j], 9 * (size_t)c.g.plane * sizeof(float)), "hipMalloc lattice") &&
           dev(hipMemset(c.lat[j], 0, 9 * (size_t)c.g.plane * sizeof(float)), "hipMemset") &&
           dev(hipMalloc(&c.hist[j], 2 * sizeof(float) * c.grid.ny), "hipMalloc history");
    ok = ok && dev(hipMalloc(&c.ubuf, 2 * np * sizeof(float)), "hipMalloc velocity");
    // the batch kernel always runs the obstacle path: every case has a mask
    // (all fluid when none was given)
    const uint8_t* m = masks ? masks[i] : nullptr;
    std::vector<uint8_t> hm(np, 0);
    size_t solid = 0;
    if (m)
      for (size_t q = 0; q < np; ++q) {
        hm[q] = m[q] ? 1 : 0;
        solid += hm[q];
      }
    c.fluid = np - solid;
    ok = ok && dev(hipMalloc(&c.solid, np), "hipMalloc mask") &&
         dev(hipMemcpy(c.solid, hm.data(), np, hipMemcpyHostToDevice), "copy mask");
  }
  ok = ok && dev(hipMalloc(&b->d_case_res, sizeof(double) * 4 * n), "hipMalloc") &&
       dev(hipMemset(b->d_case_res, 0, sizeof(double) * 4 * n), "hipMemset") &&
       dev(hipMalloc(&b->d_active, sizeof(int) * n), "hipMalloc") &&
       dev(hipMalloc(&b->d_done, sizeof(long long) * n), "hipMalloc") &&
       dev(hipMalloc(&b->d_bar, 2 * sizeof(unsigned)), "hipMalloc") &&
       dev(hipMemset(b->d_bar, 0, 2 * sizeof(unsigned)), "hipMemset") &&
       dev(hipMalloc(&b->d_err, sizeof(int)), "hipMalloc") &&
       dev(hipMemset(b->d_err, 0, sizeof(int)), "hipMemset");
  if (!ok) {
    free_batch(b);
    return LBM_EDEVICE;
  }
  int rc = configure(b);
  for (int i = 0; rc == LBM_OK && i < n; ++i) rc = init_case<double>(b, i, nullptr, nullptr, nullptr);
  if (rc == LBM_OK && hipStreamSynchronize(b->stream) != hipSuccess)
    rc = fail(LBM_EDEVICE, "initialisation failed");
  if (rc) {
    free_batch(b);
    return rc;
  }
  *out = b;
  return LBM_OK;
}

void lbm_batch_destroy(lbm_batch* b) {
  if (!b) return;
  if (b->stream) hipStreamSynchronize(b->stream);
  free_batch(b);
}

int lbm_batch_set_stream(lbm_batch* b, void* s) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  HIPCHECK(hipStreamSynchronize(b->stream));
  b->stream = s ? (hipStream_t)s : b->own_stream;
  return LBM_OK;
}

int lbm_batch_set_launch(lbm_batch* b, int32_t rows_per_item, int32_t blocks) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  // rows_per_item selects the block height: 4, 8 or 16 wavefronts of one row
  // each (0 = 4); blocks: persistent grid size (0 = all co-resident blocks;
  // a negative value selects the round-robin schedule with |blocks| blocks).
  int by = rows_per_item == 0 ? 4 : rows_per_item;
  bool known = false;
  for (auto& s : kBatchShapes) known |= s.by == by;
  if (!known) return fail(LBM_EINVAL, "rows_per_item must be 4, 8 or 16");
  HIPCHECK(hipStreamSynchronize(b->stream));
  b->by = by;
  b->rows = 1;
  b->schedule = blocks < 0 ? 1 : 0;
  b->blocks = blocks < 0 ? -blocks : blocks;
  return configure(b);
}

int lbm_batch_init_fields(lbm_batch* b, int32_t ci, const double* rho, const double* ux,
                          const double* uy) {
  if (!b || ci < 0 || ci >= b->n) return fail(LBM_EINVAL, "bad batch or case index");
  const size_t np = (size_t)b->cs[ci].grid.nx * b->cs[ci].grid.ny;
  double* tmp[3] = {nullptr, nullptr, nullptr};
  const double* src[3] = {rho, ux, uy};
  int rc = LBM_OK;
  for (int i = 0; i < 3 && rc == LBM_OK; ++i) {
    if (!src[i]) continue;
    if (hipMalloc(&tmp[i], np * sizeof(double)) != hipSuccess ||
        hipMemcpy(tmp[i], src[i], np * sizeof(double), hipMemcpyHostToDevice) != hipSuccess)
      rc = fail(LBM_EDEVICE, "upload of initial fields failed");
  }
  if (rc == LBM_OK) rc = init_case<double>(b, ci, tmp[0], tmp[1], tmp[2]);
  if (hipStreamSynchronize(b->stream) != hipSuccess && rc == LBM_OK)
    rc = fail(LBM_EDEVICE, "initialisation failed");
  for (auto p : tmp)
    if (p) hipFree(p);
  return rc;
}

int lbm_batch_init_fields_device(lbm_batch* b, int32_t ci, const float* rho, const float* ux,
                                 const float* uy) {
  if (!b || ci < 0 || ci >= b->n) return fail(LBM_EINVAL, "bad batch or case index");
  return init_case<float>(b, ci, rho, ux, uy);
}

int lbm_batch_run(lbm_batch* b, double tol, int64_t max_steps, int64_t* steps_per_case) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  if (max_steps < 0 || !(tol >= 0)) return fail(LBM_EINVAL, "bad tol or max_steps");
  const int n = b->n;
  // every case starts active; steps count from the batch's current step
  b->h_active.assign(n, 1);
  std::vector<long long> done(n, 0);
  HIPCHECK(hipMemcpyAsync(b->d_active, b->h_active.data(), sizeof(int) * n,
                          hipMemcpyHostToDevice, b->stream));
  HIPCHECK(hipMemcpyAsync(b->d_done, done.data(), sizeof(long long) * n, hipMemcpyHostToDevice,
                          b->stream));
  HIPCHECK(hipMemsetAsync(b->d_err, 0, sizeof(int), b->stream));
  HIPCHECK(hipMemsetAsync(b->d_bar, 0, 2 * sizeof(unsigned), b->stream));
  const void* kfn = batch_kernel_for(b->by, b->rows);
  int per_cu = 0;
  HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kLanes * b->by, 0));
  hipDeviceProp_t prop;
  HIPCHECK(hipGetDeviceProperties(&prop, b->device));
  const int max_blocks = per_cu * prop.multiProcessorCount;
  if (max_blocks < 1) return fail(LBM_EDEVICE, "batch kernel cannot be resident");
  const int G = b->blocks > 0 ? std::min(b->blocks, max_blocks) : max_blocks;
  const int64_t t_start = b->t;
  const int64_t chunk = (int64_t)b->K * std::max<int64_t>(1, 2000 / b->K);  // steps per launch
  int rc = rebuild_items(b);
  if (rc) return rc;
  int64_t left = max_steps;
  int active_n = n;
  while (left > 0 && active_n > 0) {
    const int64_t ns = std::min(left, chunk);
    BatchArgs a{};
    a.cases = b->d_cases;
    a.ncases = n;
    a.item_case = b->d_item_case;
    a.item_tile = b->d_item_tile;
    a.n_items = b->n_items;
    a.schedule = b->schedule;
    a.t0 = b->t;
    a.nsteps = (int)ns;
    a.K = b->K;
    a.tol = tol;
    a.min_steps = t_start + 2LL * b->K;
    a.active = b->d_active;
    a.done_step = b->d_done;
    a.case_res = b->d_case_res;
    a.bar = b->d_bar;
    a.err = b->d_err;
    a.spin_limit = 1LL << 26;
    void* kargs[] = {&a};
    HIPCHECK(hipLaunchCooperativeKernel(kfn, dim3(G), dim3(kLanes, b->by), kargs, 0, b->stream));
    HIPCHECK(hipStreamSynchronize(b->stream));
    int err = 0;
    HIPCHECK(hipMemcpy(&err, b->d_err, sizeof(int), hipMemcpyDeviceToHost));
    if (err) return fail(LBM_EDEVICE, "batch grid barrier timed out");
    b->t += ns;
    left -= ns;
    std::vector<int> act(n);
    HIPCHECK(hipMemcpy(act.data(), b->d_active, sizeof(int) * n, hipMemcpyDeviceToHost));
    int now = 0;
    for (int v : act) now += v;
    if (now < active_n) {  // drop retired cases from the item list
      b->h_active = act;
      rc = rebuild_items(b);
      if (rc) return rc;
    }
    active_n = now;
  }
  HIPCHECK(hipMemcpy(done.data(), b->d_done, sizeof(long long) * n, hipMemcpyDeviceToHost));
  bool diverged = false;
  for (int i = 0; i < n; ++i) {
    long long v = done[i];
    if (v == 0) v = b->t - t_start;         // not converged within max_steps
    else if (v < 0) {
      diverged = true;
      v = -(-v - t_start);
    } else {
      v -= t_start;
    }
    if (steps_per_case) steps_per_case[i] = v;
  }
  if (diverged) return fail(LBM_EUNSTABLE, "some cases diverged (negative step counts)");
  return LBM_OK;
}

int lbm_batch_residual(lbm_batch* b, int32_t ci, double* r) {
  if (!b || !r || ci < 0 || ci >= b->n) return fail(LBM_EINVAL, "bad argument");
  double v[4];
  HIPCHECK(hipStreamSynchronize(b->stream));
  HIPCHECK(hipMemcpy(v, b->d_case_res + 4 * ci, sizeof v, hipMemcpyDeviceToHost));
  if (!std::isfinite(v[0]) || !std::isfinite(v[1])) {
    *r = NAN;
    return fail(LBM_EUNSTABLE, "residual is not finite");
  }
  *r = v[1] > 0 ? std::sqrt(v[0] / v[1]) : (v[0] > 0 ? INFINITY : 0.0);
  return LBM_OK;
}

int lbm_batch_fields(lbm_batch* b, int32_t ci, double* rho, double* ux, double* uy) {
  if (!b || ci < 0 || ci >= b->n) return fail(LBM_EINVAL, "bad batch or case index");
  HostCase& c = b->cs[ci];
  const size_t np = (size_t)c.grid.nx * c.grid.ny;
  double* d = nullptr;
  HIPCHECK(hipMalloc(&d, 3 * np * sizeof(double)));
  const int blocks = int((np + 255) / 256);
  hipLaunchKernelGGL((export_kernel<BS>), dim3(blocks), dim3(256), 0, b->stream,
                     (const float*)c.lat[b->t & 1], c.g, c.k, c.solid, (double*)nullptr,
                     (float*)nullptr, (float*)nullptr, (float*)nullptr, d, d + np, d + 2 * np);
  hipError_t e = hipStreamSynchronize(b->stream);
  double* h[3] = {rho, ux, uy};
  for (int i = 0; i < 3 && e == hipSuccess; ++i)
    if (h[i]) e = hipMemcpy(h[i], d + i * np, np * sizeof(double), hipMemcpyDeviceToHost);
  hipFree(d);
  if (e != hipSuccess) return fail(LBM_EDEVICE, hipGetErrorString(e));
  return LBM_OK;
}

}  // extern "C"
