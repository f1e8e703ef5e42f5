// Fused-step kernels of one storage type and one flavour.  The build compiles
// this file once per (storage, flavour) pair, with LBM_STEP_STORAGE set to an
// LBM_STORE_* code and LBM_STEP_FLAVOR to a Flavor, so the many template
// instantiations (launch shapes x variants x obstacle/outlet) spread over
// parallel compiler runs.
#include "lbm_kernels.h"

#if !defined(LBM_STEP_STORAGE) || !defined(LBM_STEP_FLAVOR)
#error "compile with -DLBM_STEP_STORAGE=<0..3> -DLBM_STEP_FLAVOR=<0..2>"
#endif

namespace lbmk {

namespace {

template <int ST>
struct StorageOf;
template <>
struct StorageOf<0> { using type = StoreF64; };
template <>
struct StorageOf<1> { using type = StoreF32; };
template <>
struct StorageOf<2> { using type = StoreBF16; };
template <>
struct StorageOf<3> { using type = StoreF16; };

using S = StorageOf<LBM_STEP_STORAGE>::type;
using T = S::T;
using C = S::C;
constexpr int FL = LBM_STEP_FLAVOR;

template <int BY, int R, int VAR>
void go_var(bool obst, bool outl, bool closed, const void* src, void* dst, const StepArgs& a,
            const Consts<C>& k, hipStream_t st) {
  dim3 block(kLanes, BY), grid(a.ntiles);
  // closed lattices (walls and lids only) take an instantiation without the
  // periodic, inlet and outlet code (fewer scalar registers, so more blocks
  // fit on a compute unit); default kernel only
  if constexpr ((VAR & ~kVarNts) == 0) {
    if (closed && obst) {
      hipLaunchKernelGGL((step_kernel<S, BY, R, FL, true, false, VAR, true>), grid, block, 0, st,
                         (const T*)src, (T*)dst, a, k);
      return;
    }
    if (closed) {
      hipLaunchKernelGGL((step_kernel<S, BY, R, FL, false, false, VAR, true>), grid, block, 0, st,
                         (const T*)src, (T*)dst, a, k);
      return;
    }
  }
  if (obst && outl)
    hipLaunchKernelGGL((step_kernel<S, BY, R, FL, true, true, VAR>), grid, block, 0, st,
                       (const T*)src, (T*)dst, a, k);
  else if (obst)
    hipLaunchKernelGGL((step_kernel<S, BY, R, FL, true, false, VAR>), grid, block, 0, st,
                       (const T*)src, (T*)dst, a, k);
  else if (outl)
    hipLaunchKernelGGL((step_kernel<S, BY, R, FL, false, true, VAR>), grid, block, 0, st,
                       (const T*)src, (T*)dst, a, k);
  else
    hipLaunchKernelGGL((step_kernel<S, BY, R, FL, false, false, VAR>), grid, block, 0, st,
                       (const T*)src, (T*)dst, a, k);
}

template <int BY, int R>
void go(bool obst, bool outl, bool closed, int var, const void* src, void* dst, const StepArgs& a,
        const Consts<C>& k, hipStream_t st) {
  switch (var) {
    case 0: go_var<BY, R, 0>(obst, outl, closed, src, dst, a, k, st); break;
    case kVarFds: go_var<BY, R, kVarFds>(obst, outl, closed, src, dst, a, k, st); break;
    case kVarMrt: go_var<BY, R, kVarMrt>(obst, outl, closed, src, dst, a, k, st); break;
    case kVarNts: go_var<BY, R, kVarNts>(obst, outl, closed, src, dst, a, k, st); break;
    default: go_var<BY, R, kVarFds | kVarMrt>(obst, outl, closed, src, dst, a, k, st); break;
  }
}

}  // namespace

template <>
void launch_step<LBM_STEP_STORAGE, LBM_STEP_FLAVOR>(int by, int rows, int var, const void* src,
                                                    void* dst, const StepArgs& a,
                                                    const void* consts, hipStream_t st) {
  const Consts<C>& k = *static_cast<const Consts<C>*>(consts);
  const bool obst = a.solid != nullptr;
  const bool outl = side_of(a.g, kE) == kOutlet;
  bool closed = true;
  for (int sd = 0; sd < 4; ++sd)
    closed = closed && (side_of(a.g, sd) == kWall || side_of(a.g, sd) == kLid);
  switch (by * 100 + rows) {
    case 1601: go<16, 1>(obst, outl, closed, var, src, dst, a, k, st); break;
    case 801: go<8, 1>(obst, outl, closed, var, src, dst, a, k, st); break;
    case 401: go<4, 1>(obst, outl, closed, var, src, dst, a, k, st); break;
    case 402: go<4, 2>(obst, outl, closed, var, src, dst, a, k, st); break;
    case 802: go<8, 2>(obst, outl, closed, var, src, dst, a, k, st); break;
    case 404: go<4, 4>(obst, outl, closed, var, src, dst, a, k, st); break;
    default: go<8, 4>(obst, outl, closed, var, src, dst, a, k, st); break;
  }
}

}  // namespace lbmk
