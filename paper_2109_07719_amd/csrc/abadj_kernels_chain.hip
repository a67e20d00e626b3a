// Kernel variants for batches of fixed-base serial chains of revolute
// joints (parent/child exchange between neighbouring lanes' registers),
// in a translation unit of their own so that the build compiles them in
// parallel with the other variants.
#include "abadj_device.h"

namespace aba {

template <typename S, int FR>
hipError_t launch_aba_chain(const AbaArgs<S>& a, const Tiling& tl, hipStream_t st) {
  return launch_aba_v<S, false, FR, true>(a, tl, st);
}
template <typename S, int FR>
hipError_t launch_forward_chain(const FwdArgs<S>& a, const Tiling& tl, hipStream_t st) {
  return launch_forward_v<S, false, FR, true>(a, tl, st);
}
template <typename S, int FR>
hipError_t launch_backward_chain(const BwdArgs<S>& a, const Tiling& tl, hipStream_t st) {
  if constexpr (sizeof(S) == sizeof(float)) {
    if (a.adj64) return launch_backward_v<S, double, false, FR, true>(a, tl, st);
  }
  return launch_backward_v<S, S, false, FR, true>(a, tl, st);
}
template <typename S, int FR>
hipError_t launch_forward_jvp_chain(const JvpArgs<S>& a, const Tiling& tl, hipStream_t st) {
  return launch_forward_jvp_v<S, false, FR, true>(a, tl, st);
}

#define ABADJ_CHAIN(S, FR)                                                                            \
  template hipError_t launch_aba_chain<S, FR>(const AbaArgs<S>&, const Tiling&, hipStream_t);         \
  template hipError_t launch_forward_chain<S, FR>(const FwdArgs<S>&, const Tiling&, hipStream_t);     \
  template hipError_t launch_backward_chain<S, FR>(const BwdArgs<S>&, const Tiling&, hipStream_t);    \
  template hipError_t launch_forward_jvp_chain<S, FR>(const JvpArgs<S>&, const Tiling&, hipStream_t);
ABADJ_CHAIN(float, kFrIdentity)
ABADJ_CHAIN(float, kFrGeneral)
ABADJ_CHAIN(double, kFrIdentity)
ABADJ_CHAIN(double, kFrGeneral)
#undef ABADJ_CHAIN

}  // namespace aba
