// Adjoint kernel variants for trees and free-floating roots with the reverse
// passes in the handle's own type (FP32 or FP64), and the adjoint's
// launcher.  FP32 handles whose reverse passes run in FP64 go to
// abadj_kernels_bwd64.hip; serial chains to abadj_kernels_chain.hip.
#include "abadj_device.h"

namespace aba {

template <typename S>
hipError_t launch_backward(const BwdArgs<S>& a, const Shape& sh, const Tiling& tl, hipStream_t st) {
  if constexpr (sizeof(S) == sizeof(float)) {
    if (a.adj64) return launch_backward_adj64(a, sh, tl, st);
  }
  ABADJ_DISPATCH(launch_backward_v, launch_backward_chain, S, S)
}

template hipError_t launch_backward<float>(const BwdArgs<float>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_backward<double>(const BwdArgs<double>&, const Shape&, const Tiling&, hipStream_t);

}  // namespace aba
