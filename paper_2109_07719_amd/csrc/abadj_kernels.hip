// Kernel variants for trees and free-floating roots of the forward rollout,
// single forward-dynamics evaluations and the tangent rollout, and the
// launchers that pick a variant for a handle's shape.  The adjoint lives in
// abadj_kernels_bwd.hip / abadj_kernels_bwd64.hip, the serial-chain variants
// in abadj_kernels_chain.hip.
#include "abadj_device.h"

namespace aba {

template <typename S>
hipError_t launch_aba(const AbaArgs<S>& a, const Shape& sh, const Tiling& tl, hipStream_t st) {
  ABADJ_DISPATCH(launch_aba_v, launch_aba_chain, S)
}
template <typename S>
hipError_t launch_forward(const FwdArgs<S>& a, const Shape& sh, const Tiling& tl, hipStream_t st) {
  ABADJ_DISPATCH(launch_forward_v, launch_forward_chain, S)
}
template <typename S>
hipError_t launch_forward_jvp(const JvpArgs<S>& a, const Shape& sh, const Tiling& tl, hipStream_t st) {
  ABADJ_DISPATCH(launch_forward_jvp_v, launch_forward_jvp_chain, S)
}

template hipError_t launch_aba<float>(const AbaArgs<float>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_aba<double>(const AbaArgs<double>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_forward<float>(const FwdArgs<float>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_forward<double>(const FwdArgs<double>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_forward_jvp<float>(const JvpArgs<float>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_forward_jvp<double>(const JvpArgs<double>&, const Shape&, const Tiling&, hipStream_t);

}  // namespace aba
