// Adjoint kernel variants for trees and free-floating roots of FP32 handles
// whose backward pass runs in FP64: inputs, outputs, checkpoints and replays
// stay FP32, each step is recomputed and reversed in FP64 (BwdArgs::adj64).
#include "abadj_device.h"

namespace aba {

hipError_t launch_backward_adj64(const BwdArgs<float>& a, const Shape& sh, const Tiling& tl, hipStream_t st) {
  using S = float;
  ABADJ_DISPATCH(launch_backward_v, launch_backward_chain, float, double)
}

}  // namespace aba
