// Fused-step kernels instantiated for scaled FP16 deviation storage.
#include "lbm_kernels.h"

namespace lbmk {

namespace {
template <int BY, int R, int FL, int VAR>
void go4f(bool obst, bool outl, const void* src, void* dst, const StepArgs& a,
          const Consts<float>& k, hipStream_t st) {
  using S = StoreF16;
  using T = S::T;
  dim3 block(kLanes, BY), grid(a.ntiles);
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

template <int BY, int R, int FL>
void go4(bool obst, bool outl, int var, const void* src, void* dst, const StepArgs& a,
         const Consts<float>& k, hipStream_t st) {
  switch (var) {
    case 0: go4f<BY, R, FL, 0>(obst, outl, src, dst, a, k, st); break;
    case kVarFds: go4f<BY, R, FL, kVarFds>(obst, outl, src, dst, a, k, st); break;
    case kVarMrt: go4f<BY, R, FL, kVarMrt>(obst, outl, src, dst, a, k, st); break;
    case kVarNts: go4f<BY, R, FL, kVarNts>(obst, outl, src, dst, a, k, st); break;
    default: go4f<BY, R, FL, kVarFds | kVarMrt>(obst, outl, src, dst, a, k, st); break;
  }
}

template <int BY, int R>
void go(int flavor, bool obst, bool outl, int var, const void* src, void* dst,
        const StepArgs& a, const Consts<float>& k, hipStream_t st) {
  if (flavor == kPlain) go4<BY, R, kPlain>(obst, outl, var, src, dst, a, k, st);
  else if (flavor == kStore) go4<BY, R, kStore>(obst, outl, var, src, dst, a, k, st);
  else go4<BY, R, kCheck>(obst, outl, var, src, dst, a, k, st);
}
}  // namespace

void launch_step_f16(int by, int rows, int flavor, int var, const void* src,
                     void* dst, const StepArgs& a, const Consts<float>& k,
                     hipStream_t st) {
  const bool obst = a.solid != nullptr;
  const bool outl = a.g.side[kE] == kOutlet;
  switch (by * 100 + rows) {
    case 1601: go<16, 1>(flavor, obst, outl, var, src, dst, a, k, st); break;
    case 801: go<8, 1>(flavor, obst, outl, var, src, dst, a, k, st); break;
    case 401: go<4, 1>(flavor, obst, outl, var, src, dst, a, k, st); break;
    case 402: go<4, 2>(flavor, obst, outl, var, src, dst, a, k, st); break;
    case 802: go<8, 2>(flavor, obst, outl, var, src, dst, a, k, st); break;
    case 404: go<4, 4>(flavor, obst, outl, var, src, dst, a, k, st); break;
    default: go<8, 4>(flavor, obst, outl, var, src, dst, a, k, st); break;
  }
}

}  // namespace lbmk
