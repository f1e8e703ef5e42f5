// Fused-step kernels instantiated for FP64 storage.
#include "lbm_kernels.h"

namespace lbmk {

namespace {
template <int BY, int R>
void go(int flavor, const void* src, void* dst, const StepArgs& a, const Consts<double>& k,
        int ntiles, hipStream_t st) {
  using S = StoreF64;
  using T = S::T;
  dim3 block(kLanes, BY), grid(ntiles);
  if (flavor == kPlain)
    hipLaunchKernelGGL((step_kernel<S, BY, R, kPlain>), grid, block, 0, st, (const T*)src,
                       (T*)dst, a, k);
  else if (flavor == kStore)
    hipLaunchKernelGGL((step_kernel<S, BY, R, kStore>), grid, block, 0, st, (const T*)src,
                       (T*)dst, a, k);
  else
    hipLaunchKernelGGL((step_kernel<S, BY, R, kCheck>), grid, block, 0, st, (const T*)src,
                       (T*)dst, a, k);
}
}  // namespace

void launch_step_f64(int by, int rows, int flavor, const void* src, void* dst,
                     const StepArgs& a, const Consts<double>& k, int ntiles, hipStream_t st) {
  switch (by * 100 + rows) {
    case 404: go<4, 4>(flavor, src, dst, a, k, ntiles, st); break;
    case 802: go<8, 2>(flavor, src, dst, a, k, ntiles, st); break;
    case 804: go<8, 4>(flavor, src, dst, a, k, ntiles, st); break;
    case 1601: go<16, 1>(flavor, src, dst, a, k, ntiles, st); break;
    case 1602: go<16, 2>(flavor, src, dst, a, k, ntiles, st); break;
    default: go<4, 2>(flavor, src, dst, a, k, ntiles, st); break;
  }
}

}  // namespace lbmk
