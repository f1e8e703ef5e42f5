// Batched steady solver: many independent lattices (cases of different size,
// Re, gamma and geometry) advanced together by one persistent kernel per
// window of check_every steps.
//
// Work is a stream of tickets (step, case, tile) taken in order from one
// atomic counter; the order is step-major, so while the last tiles of one
// step run, the first tiles of the next are already handed out.  A tile of
// case c at step s may start once all tiles of case c at step s-1 are done
// (a per-case completion counter): cases advance independently, with no
// grid-wide barrier.  A block only ever waits for tickets that running blocks
// already hold, so progress does not depend on co-residency; the wait is
// bounded anyway (an error flag ends the launch).  The block that completes
// a case's last tile of the window reduces, in a fixed order, that case's
// residual partials and retires it when converged, stalled or diverged; the
// host drops retired cases from the next window's ticket list.
//
// All cases share one step counter and one storage type: FP32 or FP64
// deviations.

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


// Per-case descriptor (device).
struct CaseDev {
  StepArgs a[2];       // per lattice parity: geometry, tiling, mask, ubuf,
                       // partials (case base), outlet history in/out
  Consts<float> kf;
  Consts<double> kd;
  void* lat[2];
  int outlet;
  int ntiles;
};

template <class C>
__device__ __forceinline__ const Consts<C>& case_consts(const CaseDev& cd);
template <>
__device__ __forceinline__ const Consts<float>& case_consts<float>(const CaseDev& cd) {
  return cd.kf;
}
template <>
__device__ __forceinline__ const Consts<double>& case_consts<double>(const CaseDev& cd) {
  return cd.kd;
}


__device__ __forceinline__ int load_flag(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Work items carry the tile index and, in bit kInteriorBit, whether the
// tile's region (the tile with its one-node ring) is all fluid and keeps away
// from every side: such tiles take the path without boundary, mask and outlet
// logic.
constexpr int kInteriorBit = 30;
constexpr int kTileMask = (1 << kInteriorBit) - 1;

// Below this many active items the graph schedule launches one kernel per
// step for all classes (kClsAny).
constexpr long long kSplitMinItems = 2048;

// Item classes of the graph schedule: each class is one launch per step, so
// that each gets the registers of its own path (the interior path and the
// closed-lattice boundary path fit eight blocks per compute unit; the outlet
// path needs more).  kClsAny decides per item (the dataflow kernel).
enum ItemClass : int { kClsInt = 0, kClsClosed = 1, kClsOutlet = 2, kClsOther = 3, kClsAny = 4 };
constexpr int kNumClasses = 4;

template <class S, int BY, int R, int FL, int VAR = 0, int CLS = kClsAny>
__device__ __forceinline__ void run_item(const CaseDev& cd, int par, int item_tile,
                                         typename S::C (*s_rho)[kLanes + 2], double (*s_red)[4]) {
  using T = typename S::T;
  using C = typename S::C;
  const T* fa = static_cast<const T*>(cd.lat[par]);
  T* fb = static_cast<T*>(cd.lat[par ^ 1]);
  const int tile = item_tile & kTileMask;
  // the case's step arguments and constants as local (scalar) copies, read
  // before the first population load: read where used, a field needed for
  // an address after the population loads are issued costs a second round
  // trip (its load waits for every load before it)
  const StepArgs args = cd.a[par];
  const Consts<C> k = case_consts<C>(cd);
  if constexpr (CLS == kClsInt) {
    step_tile<S, BY, R, FL, false, false, VAR, true>(fa, fb, args, k, tile, s_rho, s_red);
    return;
  } else if constexpr (CLS == kClsClosed) {
    step_tile<S, BY, R, FL, true, false, VAR, false, true>(fa, fb, args, k, tile, s_rho, s_red);
    return;
  } else if constexpr (CLS == kClsOutlet) {
    step_tile<S, BY, R, FL, true, true, VAR>(fa, fb, args, k, tile, s_rho, s_red);
    return;
  } else if constexpr (CLS == kClsOther) {
    step_tile<S, BY, R, FL, true, false, VAR>(fa, fb, args, k, tile, s_rho, s_red);
    return;
  }
  if (item_tile >> kInteriorBit)
    step_tile<S, BY, R, FL, false, false, VAR, true>(fa, fb, cd.a[par], case_consts<C>(cd), tile,
                                                     s_rho, s_red);
  else if (cd.outlet)
    step_tile<S, BY, R, FL, true, true, VAR>(fa, fb, cd.a[par], case_consts<C>(cd), tile, s_rho,
                                             s_red);
  else
    step_tile<S, BY, R, FL, true, false, VAR>(fa, fb, cd.a[par], case_consts<C>(cd), tile, s_rho,
                                              s_red);
}

// Retirement state shared by both batch schedules.
struct RetireArgs {
  const CaseDev* cases;
  double tol;
  long long min_steps;
  int* active;
  long long* done_step;
  int* status;
  double* best;
  int* stall;
  double* case_res;
  int plateau_checks;
  double plateau_factor;
};

// Residual of case c from its per-tile partials (fixed order: lane-strided
// sums, then lane 0 adds the 64 lane sums in order) and the retirement rule.
// t: steps done before the check step.  Uses threads (lane, 0) of the block.
__device__ void retire_check(const RetireArgs& b, int c, long long t, double (*s_sum)[kLanes]) {
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
    int st = 0;
    if (!finite) {
      st = 3;
    } else if (t + 1 >= b.min_steps) {
      if (r < b.tol) {
        st = 1;
      } else if (b.plateau_checks > 0) {
        // plateau: no improvement by plateau_factor for plateau_checks checks
        if (r < b.best[c] * b.plateau_factor) {
          b.best[c] = r;
          b.stall[c] = 0;
        } else if (++b.stall[c] >= b.plateau_checks) {
          st = 2;
        }
      }
    }
    if (st) {
      b.status[c] = st;
      b.done_step[c] = st == 3 ? -(t + 1) : t + 1;
      __hip_atomic_store(&b.active[c], 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __syncthreads();
}

// Arguments of the persistent dataflow kernel (one launch per window).
struct BatchArgs {
  const CaseDev* cases;
  int ncases;
  const int* item_case;   // work items of the window: (case, tile)
  const int* item_tile;
  int n_items;
  long long t0;           // steps done before this window
  int nsteps;             // steps in this window
  int K;                  // check cadence
  unsigned* ticket;       // ticket counter (zero at launch)
  unsigned* done;         // [ncases] tiles finished in this window (zero at launch)
  RetireArgs ret;
  int* err;               // set when a wait timed out
  long long spin_limit;
};

// ---- schedule "graph": one multi-case step kernel per time step (one block
// per active tile of any case, tiles handed out XCD by XCD), then a per-case
// reduction kernel on check steps; a window of check_every steps is captured
// once into a graph and replayed while the set of active cases is unchanged.
struct StepLaunch {
  const CaseDev* cases;
  const int* item_case;
  const int* item_tile;
  int n_items;
  const int* active;
  int par;
};

// NTS: non-temporal population stores (the active lattices together exceed
// the last-level cache).
template <class S, int BY, int R, int FL, bool NTS, int CLS>
__global__ __launch_bounds__(kLanes* BY) void batch_step_kernel(StepLaunch L) {
  __shared__ typename S::C s_rho[BY * R + 2][kLanes + 2];
  __shared__ double s_red[BY][4];
  const int it = xcd_tile(blockIdx.x, L.n_items);
  const int c = L.item_case[it];
  if (!L.active[c]) return;
  run_item<S, BY, R, FL, NTS ? kVarNts : 0, CLS>(L.cases[c], L.par, L.item_tile[it], s_rho,
                                                 s_red);
}

// one block per case: residual of the check step that ends the window
__global__ __launch_bounds__(kLanes) void batch_reduce_kernel(RetireArgs r, int ncases,
                                                              const long long* tnow, int nsteps) {
  __shared__ double s_sum[4][kLanes];
  const int c = blockIdx.x;
  if (c >= ncases || !r.active[c]) return;
  retire_check(r, c, *tnow + nsteps - 1, s_sum);
}

__global__ void batch_tick_kernel(long long* tnow, int nsteps) {
  if (threadIdx.x == 0) *tnow += nsteps;
}

// ---- schedule "dataflow": one persistent kernel per window.
template <class S, int BY, int R>
__global__ __launch_bounds__(kLanes* BY) void batch_kernel(BatchArgs b) {
  __shared__ typename S::C s_rho[BY * R + 2][kLanes + 2];
  __shared__ double s_red[BY][4];
  __shared__ double s_sum[4][kLanes];
  __shared__ unsigned s_ticket;
  __shared__ int s_last;
  const bool lead = threadIdx.x == 0 && threadIdx.y == 0;
  const unsigned total = unsigned(b.nsteps) * unsigned(b.n_items);
  for (;;) {
    if (lead) s_ticket = atomicAdd(b.ticket, 1u);
    __syncthreads();
    // uniform across the block: scalar registers (buffer resources and
    // offsets derived from the case must be wave-uniform)
    const unsigned tk = __builtin_amdgcn_readfirstlane(s_ticket);
    if (tk >= total) break;
    const int s = int(tk / unsigned(b.n_items));
    const int it = int(tk % unsigned(b.n_items));
    const int c = b.item_case[it];
    const int tile = b.item_tile[it];   // tile index and interior bit
    const CaseDev& cd = b.cases[c];
    // wait until case c has finished step s - 1 of this window
    if (lead) {
      const unsigned need = unsigned(s) * unsigned(cd.ntiles);
      long long spins = 0;
      while (__hip_atomic_load(&b.done[c], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
        __builtin_amdgcn_s_sleep(1);
        if (++spins > b.spin_limit) {
          __hip_atomic_store(b.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          break;
        }
      }
      __atomic_thread_fence(__ATOMIC_ACQUIRE);
    }
    __syncthreads();
    if (__hip_atomic_load(b.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
    const long long t = b.t0 + s;   // steps done before this one
    const int par = int(t & 1);
    const long long idx = (t + 1) % b.K;
    const int flavor = idx == 0 ? kCheck : ((b.K >= 2 && idx == b.K - 1) ? kStore : kPlain);
    if (flavor == kCheck) run_item<S, BY, R, kCheck>(cd, par, tile, s_rho, s_red);
    else if (flavor == kStore) run_item<S, BY, R, kStore>(cd, par, tile, s_rho, s_red);
    else run_item<S, BY, R, kPlain>(cd, par, tile, s_rho, s_red);
    __syncthreads();
    if (lead) {
      __atomic_thread_fence(__ATOMIC_RELEASE);
      const unsigned prev =
          __hip_atomic_fetch_add(&b.done[c], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      s_last = (prev + 1 == unsigned(b.nsteps) * unsigned(cd.ntiles)) && flavor == kCheck;
      if (s_last) __atomic_thread_fence(__ATOMIC_ACQUIRE);
    }
    __syncthreads();
    if (s_last) retire_check(b.ret, c, t, s_sum);
  }
}

struct Shape {
  int by, rows;
};
constexpr Shape kBatchShapes[] = {{4, 1}, {8, 1}, {16, 1}};

template <class S, int BY, int R>
const void* kernel_ptr() {
  return reinterpret_cast<const void*>(&batch_kernel<S, BY, R>);
}

template <class S>
const void* kernel_for_storage(int by) {
  switch (by) {
    case 8: return kernel_ptr<S, 8, 1>();
    case 16: return kernel_ptr<S, 16, 1>();
    default: return kernel_ptr<S, 4, 1>();
  }
}

const void* batch_kernel_for(int storage, int by) {
  return storage == LBM_STORE_F64 ? kernel_for_storage<StoreF64>(by)
                                  : kernel_for_storage<StoreF32>(by);
}

struct HostCase {
  lbm_grid grid;
  lbm_params p;
  Geom g;
  Consts<float> kf;
  Consts<double> kd;
  void* lat[2] = {nullptr, nullptr};
  void* hist[2] = {nullptr, nullptr};
  float* ubuf = nullptr;
  uint8_t* solid = nullptr;
  int tiles_x = 0, ntiles = 0, tile_base = 0;
  size_t fluid = 0;
  std::vector<uint8_t> h_mask;      // [ny][nx], 1 = solid
  std::vector<uint8_t> tile_int;    // per tile: region all fluid, away from the sides
  int state_par = 0;  // which lattice holds the case's current state
};

}  // namespace

struct lbm_batch {
  std::vector<HostCase> cs;
  int n = 0;
  int K = 100;
  int by = 4, rows = 1;
  int blocks = 0;    // 0 = all co-resident blocks
  int schedule = 0;
  int storage = LBM_STORE_F32;
  int plateau_checks = 0;
  double plateau_factor = 0.9;
  int device = 0;
  hipStream_t own_stream = nullptr, stream = nullptr;
  CaseDev* d_cases = nullptr;
  int* d_item_case = nullptr;
  int* d_item_tile = nullptr;
  int n_items = 0, item_cap = 0;
  int cls_off[kNumClasses + 1] = {0, 0, 0, 0, 0};  // graph schedule: items of class k
                                                   // are [cls_off[k], cls_off[k + 1])
  bool merged = false;  // graph schedule with few items: one launch per step
  double* d_partials = nullptr;
  double* d_case_res = nullptr;
  int* d_active = nullptr;
  long long* d_done = nullptr;
  int* d_status = nullptr;
  double* d_best = nullptr;
  int* d_stall = nullptr;
  unsigned* d_sync = nullptr;  // [1 + n]: ticket counter, per-case completion counters
  int* d_err = nullptr;
  long long* d_tnow = nullptr; // step counter read by the reduction kernel
  hipGraphExec_t graph[2] = {nullptr, nullptr};  // window graphs by start parity
  int64_t t = 0;
  std::vector<int> h_active;
  std::vector<int> enabled;     // cases a run advances
  std::vector<int> h_status;    // status of the last run
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
  hipFree(b->d_status);
  hipFree(b->d_best);
  hipFree(b->d_stall);
  hipFree(b->d_sync);
  hipFree(b->d_tnow);
  for (int i = 0; i < 2; ++i)
    if (b->graph[i]) hipGraphExecDestroy(b->graph[i]);
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
    // interior tiles: the same margins as the single-lattice kernel, and no
    // solid node in the tile or its ring
    c.tile_int.assign(c.ntiles, 0);
    const int nx = c.grid.nx, ny = c.grid.ny;
    for (int t = 0; t < c.ntiles; ++t) {
      const int x0 = (t % c.tiles_x) * kLanes, y0 = (t / c.tiles_x) * ro;
      if (!(x0 >= 2 && x0 + kLanes + 1 <= nx - 2 && y0 >= 2 && y0 + ro + 1 <= ny - 2)) continue;
      bool fluid = true;
      for (int y = y0 - 1; fluid && y <= y0 + ro; ++y)
        for (int x = x0 - 1; x <= x0 + kLanes; ++x)
          if (c.h_mask[(size_t)y * nx + x]) {
            fluid = false;
            break;
          }
      c.tile_int[t] = fluid ? 1 : 0;
    }
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
      a.force = c.ubuf;  // batch cases take the uniform force; any readable buffer
      a.has_force = 0;
      a.partials = b->d_partials + (long long)c.tile_base * 4;
      a.hist_in = c.hist[par];
      a.hist_out = c.hist[par ^ 1];
    }
    d.kf = c.kf;
    d.kd = c.kd;
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

void drop_graphs(lbm_batch* b) {
  for (int i = 0; i < 2; ++i)
    if (b->graph[i]) {
      hipGraphExecDestroy(b->graph[i]);
      b->graph[i] = nullptr;
    }
}

int rebuild_items(lbm_batch* b) {
  drop_graphs(b);
  // ticket order within a step: schedule 0 = case by case (a case's tiles
  // contiguous), 1 = tiles interleaved across cases
  // the graph schedules group the items by class (one launch per class and
  // step); the dataflow schedule keeps one list
  std::vector<int> ic, itl;
  auto item_class = [&](int i, int t) {
    if (b->cs[i].tile_int[t]) return int(kClsInt);
    const int32_t* sd = b->cs[i].grid.side;
    if (sd[1] == LBM_SIDE_OUTLET) return int(kClsOutlet);
    bool closed = true;
    for (int q = 0; q < 4; ++q)
      closed = closed && (sd[q] == LBM_SIDE_WALL || sd[q] == LBM_SIDE_LID);
    return int(closed ? kClsClosed : kClsOther);
  };
  // Few items (less than about two rounds of resident blocks): one launch
  // per step that decides the path per item.  Each launch then runs for
  // little more than its start-up latency, and one launch instead of up to
  // four per step is what counts (the tail of a steady run, where a few
  // cases remain).
  long long active_items = 0;
  for (int i = 0; i < b->n; ++i)
    if (b->h_active[i]) active_items += b->cs[i].ntiles;
  b->merged = b->schedule != 2 && active_items < kSplitMinItems;
  const int ncls = (b->schedule == 2 || b->merged) ? 1 : kNumClasses;
  for (int k = 0; k < ncls; ++k) {
    b->cls_off[k] = (int)ic.size();
    auto take = [&](int i, int t) {
      if (ncls > 1 && item_class(i, t) != k) return;
      ic.push_back(i);
      itl.push_back(t | (int(b->cs[i].tile_int[t]) << kInteriorBit));
    };
    if (b->schedule != 1) {
      for (int i = 0; i < b->n; ++i) {
        if (!b->h_active[i]) continue;
        for (int t = 0; t < b->cs[i].ntiles; ++t) take(i, t);
      }
    } else {
      int maxt = 0;
      for (int i = 0; i < b->n; ++i)
        if (b->h_active[i]) maxt = std::max(maxt, b->cs[i].ntiles);
      for (int t = 0; t < maxt; ++t)
        for (int i = 0; i < b->n; ++i)
          if (b->h_active[i] && t < b->cs[i].ntiles) take(i, t);
    }
  }
  for (int k = ncls; k <= kNumClasses; ++k) b->cls_off[k] = (int)ic.size();
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

template <class S, class FT>
void launch_case_init(lbm_batch* b, HostCase& c, const FT* rho, const FT* ux, const FT* uy) {
  using T = typename S::T;
  using C = typename S::C;
  const Consts<C>& k = *reinterpret_cast<const Consts<C>*>(
      sizeof(C) == 8 ? static_cast<const void*>(&c.kd) : static_cast<const void*>(&c.kf));
  const int blocks = int(((long long)c.grid.nx * c.grid.ny + 255) / 256);
  hipLaunchKernelGGL((init_kernel<S, FT>), dim3(blocks), dim3(256), 0, b->stream, (T*)c.lat[0],
                     (T*)c.lat[1], c.g, k, c.solid, rho, ux, uy, (C*)c.ubuf, (C*)c.hist[0],
                     (C*)c.hist[1]);
  hipLaunchKernelGGL((ghost_fill_kernel<S>), dim3(blocks), dim3(256), 0, b->stream, (T*)c.lat[0],
                     c.g, k, c.solid);
}

template <class FT>
int init_case(lbm_batch* b, int ci, const FT* rho, const FT* ux, const FT* uy) {
  HostCase& c = b->cs[ci];
  if (b->storage == LBM_STORE_F64) launch_case_init<StoreF64, FT>(b, c, rho, ux, uy);
  else launch_case_init<StoreF32, FT>(b, c, rho, ux, uy);
  HIPCHECK(hipGetLastError());
  // lattice parity of the batch: state lives in lat[t & 1]; copy when t is odd
  if (b->t & 1) {
    const size_t es = b->storage == LBM_STORE_F64 ? 8 : 4;
    const size_t bytes = 9 * (size_t)c.g.plane * es;
    HIPCHECK(hipMemcpyAsync(c.lat[1], c.lat[0], bytes, hipMemcpyDeviceToDevice, b->stream));
    HIPCHECK(hipMemcpyAsync(c.hist[1], c.hist[0], 2 * es * c.grid.ny, hipMemcpyDeviceToDevice,
                            b->stream));
  }
  c.state_par = int(b->t & 1);
  return LBM_OK;
}

// Before a run: every enabled case must hold its state in lat[t & 1].
int align_parity(lbm_batch* b) {
  const int par = int(b->t & 1);
  const size_t es = b->storage == LBM_STORE_F64 ? 8 : 4;
  for (int i = 0; i < b->n; ++i) {
    HostCase& c = b->cs[i];
    if (!b->enabled[i] || c.state_par == par) continue;
    HIPCHECK(hipMemcpyAsync(c.lat[par], c.lat[c.state_par], 9 * (size_t)c.g.plane * es,
                            hipMemcpyDeviceToDevice, b->stream));
    HIPCHECK(hipMemcpyAsync(c.hist[par], c.hist[c.state_par], 2 * es * c.grid.ny,
                            hipMemcpyDeviceToDevice, b->stream));
    c.state_par = par;
  }
  return LBM_OK;
}


template <class S, int BY, bool NTS, int CLS>
void launch_step_cls(int flavor, const StepLaunch& L, hipStream_t st) {
  dim3 grid(L.n_items), block(kLanes, BY);
  if (flavor == kCheck)
    hipLaunchKernelGGL((batch_step_kernel<S, BY, 1, kCheck, NTS, CLS>), grid, block, 0, st, L);
  else if (flavor == kStore)
    hipLaunchKernelGGL((batch_step_kernel<S, BY, 1, kStore, NTS, CLS>), grid, block, 0, st, L);
  else
    hipLaunchKernelGGL((batch_step_kernel<S, BY, 1, kPlain, NTS, CLS>), grid, block, 0, st, L);
}

template <class S, int BY, bool NTS>
void launch_step_nts(int flavor, int cls, const StepLaunch& L, hipStream_t st) {
  switch (cls) {
    case kClsInt: launch_step_cls<S, BY, NTS, kClsInt>(flavor, L, st); break;
    case kClsClosed: launch_step_cls<S, BY, NTS, kClsClosed>(flavor, L, st); break;
    case kClsOutlet: launch_step_cls<S, BY, NTS, kClsOutlet>(flavor, L, st); break;
    case kClsOther: launch_step_cls<S, BY, NTS, kClsOther>(flavor, L, st); break;
    default: launch_step_cls<S, BY, NTS, kClsAny>(flavor, L, st); break;
  }
}

template <class S, int BY>
void launch_step_by(int flavor, int cls, bool nts, const StepLaunch& L, hipStream_t st) {
  if (nts) launch_step_nts<S, BY, true>(flavor, cls, L, st);
  else launch_step_nts<S, BY, false>(flavor, cls, L, st);
}

template <class S>
void launch_step_storage(int by, int flavor, int cls, bool nts, const StepLaunch& L,
                         hipStream_t st) {
  if (by == 8) launch_step_by<S, 8>(flavor, cls, nts, L, st);
  else if (by == 16) launch_step_by<S, 16>(flavor, cls, nts, L, st);
  else launch_step_by<S, 4>(flavor, cls, nts, L, st);
}

// Bytes of the two lattices of every active case.  Beyond the 256 MiB
// Infinity Cache a written lattice is evicted before the next step reads it,
// so the step stores it non-temporally (as the single-lattice path does).
constexpr size_t kLastLevelCacheBytes = size_t(256) << 20;
size_t active_lattice_bytes(const lbm_batch* b) {
  const size_t es = b->storage == LBM_STORE_F64 ? 8 : 4;
  size_t bytes = 0;
  for (int i = 0; i < b->n; ++i)
    if (b->h_active[i]) bytes += 2 * 9 * (size_t)b->cs[i].g.plane * es;
  return bytes;
}

RetireArgs retire_args(lbm_batch* b, double tol, long long min_steps) {
  RetireArgs r{};
  r.cases = b->d_cases;
  r.tol = tol;
  r.min_steps = min_steps;
  r.active = b->d_active;
  r.done_step = b->d_done;
  r.status = b->d_status;
  r.best = b->d_best;
  r.stall = b->d_stall;
  r.case_res = b->d_case_res;
  r.plateau_checks = b->plateau_checks;
  r.plateau_factor = b->plateau_factor;
  return r;
}

// Enqueue nsteps steps starting at step counter t (graph schedule): the step
// kernels, and when the last one is a check step, the per-case reduction and
// the step-counter tick.
void enqueue_window(lbm_batch* b, long long t, int nsteps, const RetireArgs& r, hipStream_t st) {
  StepLaunch L{};
  L.cases = b->d_cases;
  L.item_case = b->d_item_case;
  L.item_tile = b->d_item_tile;
  L.n_items = b->n_items;
  L.active = b->d_active;
  int last_flavor = kPlain;
  const bool nts = active_lattice_bytes(b) > kLastLevelCacheBytes;
  for (int i = 0; i < nsteps; ++i) {
    const long long tt = t + i;
    const long long idx = (tt + 1) % b->K;
    const int flavor = idx == 0 ? kCheck : ((b->K >= 2 && idx == b->K - 1) ? kStore : kPlain);
    L.par = int(tt & 1);
    if (b->merged) {
      if (b->n_items > 0) {
        if (b->storage == LBM_STORE_F64)
          launch_step_storage<StoreF64>(b->by, flavor, kClsAny, nts, L, st);
        else
          launch_step_storage<StoreF32>(b->by, flavor, kClsAny, nts, L, st);
      }
      last_flavor = flavor;
      continue;
    }
    for (int k = 0; k < kNumClasses; ++k) {
      StepLaunch Lk = L;
      Lk.item_case = b->d_item_case + b->cls_off[k];
      Lk.item_tile = b->d_item_tile + b->cls_off[k];
      Lk.n_items = b->cls_off[k + 1] - b->cls_off[k];
      if (Lk.n_items <= 0) continue;
      if (b->storage == LBM_STORE_F64)
        launch_step_storage<StoreF64>(b->by, flavor, k, nts, Lk, st);
      else
        launch_step_storage<StoreF32>(b->by, flavor, k, nts, Lk, st);
    }
    last_flavor = flavor;
  }
  if (last_flavor == kCheck)
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(b->n), dim3(kLanes), 0, st, r, b->n,
                       (const long long*)b->d_tnow, nsteps);
  hipLaunchKernelGGL(batch_tick_kernel, dim3(1), dim3(64), 0, st, b->d_tnow, nsteps);
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
    if (!rc && (params[i].strain_fd || params[i].mrt))
      rc = fail(LBM_EINVAL, "batch cases use the default kernel (strain_fd 0, mrt 0)");
    if (rc) return fail(rc, "case " + std::to_string(i) + ": " + lbm_last_error());
    if (params[i].storage != params[0].storage ||
        (params[i].storage != LBM_STORE_F32 && params[i].storage != LBM_STORE_F64))
      return fail(LBM_EINVAL, "batch cases must all use LBM_STORE_F32 or all LBM_STORE_F64");
    if (params[i].check_every != K) return fail(LBM_EINVAL, "batch cases must share check_every");
  }
  lbm_batch* b = new (std::nothrow) lbm_batch();
  if (!b) return fail(LBM_ENOMEM, "host allocation failed");
  b->n = n;
  b->K = K;
  b->storage = params[0].storage;
  b->cs.resize(n);
  b->enabled.assign(n, 1);
  b->h_status.assign(n, 0);
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
    c.kf = make_consts<float>(c.p, 1.0);
    c.kd = make_consts<double>(c.p, 1.0);
    const size_t es = b->storage == LBM_STORE_F64 ? 8 : 4;
    c.g = make_geom_for(c.grid.nx, c.grid.ny, c.grid.side, es);
    const size_t np = (size_t)c.grid.nx * c.grid.ny;
    for (int j = 0; ok && j < 2; ++j)
      ok = dev(hipMalloc(&c.lat[j], 9 * (size_t)c.g.plane * es), "hipMalloc lattice") &&
           dev(hipMemset(c.lat[j], 0, 9 * (size_t)c.g.plane * es), "hipMemset") &&
           dev(hipMalloc(&c.hist[j], 2 * es * c.grid.ny), "hipMalloc history");
    ok = ok && dev(hipMalloc(&c.ubuf, 2 * np * es), "hipMalloc velocity");
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
    c.h_mask = hm;
    ok = ok && dev(hipMalloc(&c.solid, np), "hipMalloc mask") &&
         dev(hipMemcpy(c.solid, hm.data(), np, hipMemcpyHostToDevice), "copy mask");
  }
  ok = ok && dev(hipMalloc(&b->d_case_res, sizeof(double) * 4 * n), "hipMalloc") &&
       dev(hipMemset(b->d_case_res, 0, sizeof(double) * 4 * n), "hipMemset") &&
       dev(hipMalloc(&b->d_active, sizeof(int) * n), "hipMalloc") &&
       dev(hipMalloc(&b->d_done, sizeof(long long) * n), "hipMalloc") &&
       dev(hipMalloc(&b->d_status, sizeof(int) * n), "hipMalloc") &&
       dev(hipMalloc(&b->d_best, sizeof(double) * n), "hipMalloc") &&
       dev(hipMalloc(&b->d_stall, sizeof(int) * n), "hipMalloc") &&
       dev(hipMalloc(&b->d_sync, sizeof(unsigned) * (1 + n)), "hipMalloc") &&
       dev(hipMalloc(&b->d_tnow, sizeof(long long)), "hipMalloc") &&
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

int lbm_batch_set_launch(lbm_batch* b, int32_t rows_per_item, int32_t schedule) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  // rows_per_item: block height of 4, 8 or 16 wavefronts of one row (0 = 4).
  // schedule: 0 graph of per-step kernels, work case by case; 1 the same
  // with tiles interleaved across cases; 2 persistent dataflow kernel.
  int by = rows_per_item == 0 ? 4 : rows_per_item;
  bool known = false;
  for (auto& s : kBatchShapes) known |= s.by == by;
  if (!known) return fail(LBM_EINVAL, "rows_per_item must be 4, 8 or 16");
  if (schedule < 0 || schedule > 2) return fail(LBM_EINVAL, "schedule must be 0, 1 or 2");
  HIPCHECK(hipStreamSynchronize(b->stream));
  b->by = by;
  b->rows = 1;
  b->schedule = schedule;
  b->blocks = 0;
  drop_graphs(b);
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
                                 const float* uy) {  // NOLINT
  if (!b || ci < 0 || ci >= b->n) return fail(LBM_EINVAL, "bad batch or case index");
  const int rc = init_case<float>(b, ci, rho, ux, uy);
  if (rc) return rc;
  // the caller may release the arrays as soon as this returns
  HIPCHECK(hipStreamSynchronize(b->stream));
  return LBM_OK;
}

int lbm_batch_run(lbm_batch* b, double tol, int64_t max_steps, int64_t* steps_per_case) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  if (max_steps < 0 || !(tol >= 0)) return fail(LBM_EINVAL, "bad tol or max_steps");
  const int n = b->n;
  // enabled cases start active; steps count from the batch's current step
  {
    int rc0 = align_parity(b);
    if (rc0) return rc0;
  }
  b->h_active = b->enabled;
  std::vector<long long> done(n, 0);
  std::vector<int> zeros(n, 0);
  std::vector<double> inf(n, INFINITY);
  HIPCHECK(hipMemcpyAsync(b->d_status, zeros.data(), sizeof(int) * n, hipMemcpyHostToDevice,
                          b->stream));
  HIPCHECK(hipMemcpyAsync(b->d_stall, zeros.data(), sizeof(int) * n, hipMemcpyHostToDevice,
                          b->stream));
  HIPCHECK(hipMemcpyAsync(b->d_best, inf.data(), sizeof(double) * n, hipMemcpyHostToDevice,
                          b->stream));
  HIPCHECK(hipMemcpyAsync(b->d_active, b->h_active.data(), sizeof(int) * n,
                          hipMemcpyHostToDevice, b->stream));
  HIPCHECK(hipMemcpyAsync(b->d_done, done.data(), sizeof(long long) * n, hipMemcpyHostToDevice,
                          b->stream));
  HIPCHECK(hipMemsetAsync(b->d_err, 0, sizeof(int), b->stream));
  const int64_t t_start = b->t;
  int rc = rebuild_items(b);
  if (rc) return rc;
  const RetireArgs ret = retire_args(b, tol, t_start + 2LL * b->K);
  {
    long long tn = b->t;
    HIPCHECK(hipMemcpyAsync(b->d_tnow, &tn, sizeof tn, hipMemcpyHostToDevice, b->stream));
    HIPCHECK(hipStreamSynchronize(b->stream));
  }
  // dataflow schedule: resident grid size
  const void* kfn = batch_kernel_for(b->storage, b->by);
  int G = 1;
  if (b->schedule == 2) {
    int per_cu = 0;
    HIPCHECK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, kLanes * b->by, 0));
    hipDeviceProp_t prop;
    HIPCHECK(hipGetDeviceProperties(&prop, b->device));
    G = std::max(1, per_cu) * prop.multiProcessorCount;
    if (b->blocks > 0) G = std::min(G, b->blocks);
  }
  int64_t left = max_steps;
  int active_n = 0;
  for (int v : b->h_active) active_n += v;
  while (left > 0 && active_n > 0) {
    // one window per launch sequence, ending at the next check step
    const int64_t to_check = b->K - (b->t % b->K);
    const int64_t ns = std::min(left, to_check);
    if (b->schedule == 2) {
      BatchArgs a{};
      a.cases = b->d_cases;
      a.ncases = n;
      a.item_case = b->d_item_case;
      a.item_tile = b->d_item_tile;
      a.n_items = b->n_items;
      a.t0 = b->t;
      a.nsteps = (int)ns;
      a.K = b->K;
      a.ticket = b->d_sync;
      a.done = b->d_sync + 1;
      a.ret = ret;
      a.err = b->d_err;
      a.spin_limit = 1LL << 26;
      HIPCHECK(hipMemsetAsync(b->d_sync, 0, sizeof(unsigned) * (1 + n), b->stream));
      void* kargs[] = {&a};
      HIPCHECK(hipLaunchKernel(kfn, dim3(G), dim3(kLanes, b->by), kargs, 0, b->stream));
      hipLaunchKernelGGL(batch_tick_kernel, dim3(1), dim3(64), 0, b->stream, b->d_tnow, (int)ns);
    } else if (ns == b->K && b->K >= 4) {
      // full window: captured once per start parity, replayed
      const int par = int(b->t & 1);
      if (!b->graph[par]) {
        hipGraph_t gr = nullptr;
        HIPCHECK(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
        enqueue_window(b, b->t, (int)ns, ret, b->stream);
        hipError_t e = hipStreamEndCapture(b->stream, &gr);
        if (e != hipSuccess) return fail(LBM_EDEVICE, hipGetErrorString(e));
        e = hipGraphInstantiate(&b->graph[par], gr, nullptr, nullptr, 0);
        hipGraphDestroy(gr);
        if (e != hipSuccess) {
          b->graph[par] = nullptr;
          return fail(LBM_EDEVICE, hipGetErrorString(e));
        }
      }
      HIPCHECK(hipGraphLaunch(b->graph[par], b->stream));
    } else {
      enqueue_window(b, b->t, (int)ns, ret, b->stream);
    }
    HIPCHECK(hipGetLastError());
    b->t += ns;
    left -= ns;
    if (b->t % b->K == 0) {
      HIPCHECK(hipStreamSynchronize(b->stream));
      int err = 0;
      HIPCHECK(hipMemcpy(&err, b->d_err, sizeof(int), hipMemcpyDeviceToHost));
      if (err) return fail(LBM_EDEVICE, "batch dependency wait timed out");
      std::vector<int> act(n);
      HIPCHECK(hipMemcpy(act.data(), b->d_active, sizeof(int) * n, hipMemcpyDeviceToHost));
      int now = 0;
      for (int v : act) now += v;
      if (now < active_n) {  // drop retired cases from the work list
        b->h_active = act;
        rc = rebuild_items(b);
        if (rc) return rc;
      }
      active_n = now;
    }
  }
  HIPCHECK(hipStreamSynchronize(b->stream));
  HIPCHECK(hipMemcpy(done.data(), b->d_done, sizeof(long long) * n, hipMemcpyDeviceToHost));
  HIPCHECK(hipMemcpy(b->h_status.data(), b->d_status, sizeof(int) * n, hipMemcpyDeviceToHost));
  for (int i = 0; i < n; ++i) {
    if (!b->enabled[i]) continue;
    // retired at step |done|: state in lat[|done| & 1]; else in lat[t & 1]
    b->cs[i].state_par = done[i] != 0 ? int((done[i] < 0 ? -done[i] : done[i]) & 1) : int(b->t & 1);
  }
  bool diverged = false;
  for (int i = 0; i < n; ++i) {
    long long v = done[i];
    if (!b->enabled[i]) v = 0;              // not advanced by this run
    else if (v == 0) v = b->t - t_start;    // not converged within max_steps
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


int lbm_batch_set_plateau(lbm_batch* b, int32_t checks, double factor) {
  if (!b || checks < 0 || !(factor > 0 && factor <= 1))
    return fail(LBM_EINVAL, "checks >= 0 and 0 < factor <= 1");
  b->plateau_checks = checks;
  b->plateau_factor = factor;
  return LBM_OK;
}

int lbm_batch_status(lbm_batch* b, int32_t* status) {
  if (!b || !status) return fail(LBM_EINVAL, "null argument");
  for (int i = 0; i < b->n; ++i) status[i] = b->h_status[i];
  return LBM_OK;
}

int lbm_batch_set_enabled(lbm_batch* b, const int32_t* enabled) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  for (int i = 0; i < b->n; ++i) b->enabled[i] = enabled ? (enabled[i] != 0) : 1;
  return LBM_OK;
}

int lbm_batch_set_storage(lbm_batch* b, int32_t storage) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  if (storage != LBM_STORE_F32 && storage != LBM_STORE_F64)
    return fail(LBM_EINVAL, "batch storage must be LBM_STORE_F32 or LBM_STORE_F64");
  if (storage == b->storage) return LBM_OK;
  HIPCHECK(hipStreamSynchronize(b->stream));
  const size_t es2 = storage == LBM_STORE_F64 ? 8 : 4, es1 = b->storage == LBM_STORE_F64 ? 8 : 4;
  for (auto& c : b->cs) {
    const int rc = check_lattice_bytes(c.grid.nx, c.grid.ny, es2);
    if (rc) return rc;
  }
  for (auto& c : b->cs) {
    const Geom g2 = make_geom_for(c.grid.nx, c.grid.ny, c.grid.side, es2);
    const size_t np = (size_t)c.grid.nx * c.grid.ny;
    void* lat2[2] = {nullptr, nullptr};
    void* hist2[2] = {nullptr, nullptr};
    void* ub2 = nullptr;
    bool ok = true;
    for (int i = 0; ok && i < 2; ++i)
      ok = hipMalloc(&lat2[i], 9 * (size_t)g2.plane * es2) == hipSuccess &&
           hipMemset(lat2[i], 0, 9 * (size_t)g2.plane * es2) == hipSuccess &&
           hipMalloc(&hist2[i], 2 * es2 * c.grid.ny) == hipSuccess;
    ok = ok && hipMalloc(&ub2, 2 * np * es2) == hipSuccess;
    if (!ok) {
      for (int i = 0; i < 2; ++i) {
        hipFree(lat2[i]);
        hipFree(hist2[i]);
      }
      hipFree(ub2);
      return fail(LBM_ENOMEM, "allocation for the new storage failed");
    }
    const long long nf = (long long)(c.grid.nx + 2) * (c.grid.ny + 2);
    for (int i = 0; i < 2; ++i) {
      hipLaunchKernelGGL(convert_lattice_kernel, dim3(int((nf + 255) / 256)), dim3(256), 0,
                         b->stream, c.lat[i], b->storage, c.g, 1.0, lat2[i], (int)storage, g2, 1.0);
      const long long nh = 2LL * c.grid.ny;
      hipLaunchKernelGGL(convert_values_kernel, dim3(int((nh + 255) / 256)), dim3(256), 0,
                         b->stream, c.hist[i], int(es1 == 8), hist2[i], int(es2 == 8), nh);
    }
    hipLaunchKernelGGL(convert_values_kernel, dim3(int((2 * np + 255) / 256)), dim3(256), 0,
                       b->stream, (const void*)c.ubuf, int(es1 == 8), ub2, int(es2 == 8),
                       (long long)(2 * np));
    HIPCHECK(hipGetLastError());
    HIPCHECK(hipStreamSynchronize(b->stream));
    for (int i = 0; i < 2; ++i) {
      hipFree(c.lat[i]);
      hipFree(c.hist[i]);
      c.lat[i] = lat2[i];
      c.hist[i] = hist2[i];
    }
    hipFree(c.ubuf);
    c.ubuf = static_cast<float*>(ub2);
    c.g = g2;
    c.p.storage = storage;
  }
  b->storage = storage;
  drop_graphs(b);
  return configure(b);
}

int lbm_batch_average_last_two(lbm_batch* b) {
  if (!b) return fail(LBM_EINVAL, "null batch");
  for (int i = 0; i < b->n; ++i) {
    if (!b->enabled[i]) continue;
    HostCase& h = b->cs[i];
    const int cur = h.state_par;
    const long long n = 9LL * h.g.plane;
    HIPCHECK(launch_average(b->storage, h.lat[cur], h.lat[cur ^ 1], n, (double)h.kf.scale,
                            h.hist[cur], h.hist[cur ^ 1], h.hist[0] ? 2LL * h.grid.ny : 0,
                            b->stream));
  }
  HIPCHECK(hipStreamSynchronize(b->stream));
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
  if (b->storage == LBM_STORE_F64)
    hipLaunchKernelGGL((export_kernel<StoreF64>), dim3(blocks), dim3(256), 0, b->stream,
                       (const double*)c.lat[c.state_par], c.g, c.kd, c.solid,
                       (const double*)nullptr, 0LL, (long long)np, (double*)nullptr, (float*)nullptr,
                       (float*)nullptr,
                       (float*)nullptr, d, d + np, d + 2 * np);
  else
    hipLaunchKernelGGL((export_kernel<StoreF32>), dim3(blocks), dim3(256), 0, b->stream,
                       (const float*)c.lat[c.state_par], c.g, c.kf, c.solid,
                       (const float*)nullptr, 0LL, (long long)np, (double*)nullptr, (float*)nullptr,
                       (float*)nullptr,
                       (float*)nullptr, d, d + np, d + 2 * np);
  hipError_t e = hipStreamSynchronize(b->stream);
  double* h[3] = {rho, ux, uy};
  for (int i = 0; i < 3 && e == hipSuccess; ++i)
    if (h[i]) e = hipMemcpy(h[i], d + i * np, np * sizeof(double), hipMemcpyDeviceToHost);
  hipFree(d);
  if (e != hipSuccess) return fail(LBM_EDEVICE, hipGetErrorString(e));
  return LBM_OK;
}

}  // extern "C"
