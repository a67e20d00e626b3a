// Kernel variants for trees and free-floating roots, and the launchers
// that pick a variant for a handle's shape.  The serial-chain variants are
// instantiated in abadj_kernels_chain.hip.
#include "abadj_device.h"

namespace aba {

namespace {

// Kernel variants: FREE (some system has a free-floating root), the
// link-frame kind FR (kFrIdentity: every joint frame the identity after
// canonicalisation; kFrGeneralJoints: prismatic joints or joint limits),
// CHAIN (every system is a fixed-base serial chain of revolute joints;
// register exchange between lanes).  Batches with prismatic joints or
// joint limits take the one general variant (FREE, kFrGeneralJoints),
// which handles every joint type and the limits.
enum class Variant { kFree, kFreeEti, kTree, kTreeEti, kChain, kChainEti, kGeneral };

Variant variant(const Shape& sh) {
  if (sh.has_prism || sh.has_limits) return Variant::kGeneral;
  if (sh.has_free) return sh.eti ? Variant::kFreeEti : Variant::kFree;
  if (sh.chain) return sh.eti ? Variant::kChainEti : Variant::kChain;
  return sh.eti ? Variant::kTreeEti : Variant::kTree;
}

}  // namespace

// One switch per entry: L<FREE, FR, CHAIN> is the per-variant launcher of
// this translation unit, LC<FR> the chain launcher of the other one.
#define ABADJ_DISPATCH(L, LC)                                            \
  switch (variant(sh)) {                                                 \
    case Variant::kFree: return L<S, true, kFrGeneral, false>(a, tl, st);     \
    case Variant::kFreeEti: return L<S, true, kFrIdentity, false>(a, tl, st); \
    case Variant::kTree: return L<S, false, kFrGeneral, false>(a, tl, st);    \
    case Variant::kTreeEti: return L<S, false, kFrIdentity, false>(a, tl, st); \
    case Variant::kChain: return LC<S, kFrGeneral>(a, tl, st);                \
    case Variant::kChainEti: return LC<S, kFrIdentity>(a, tl, st);            \
    case Variant::kGeneral: return L<S, true, kFrGeneralJoints, false>(a, tl, st); \
  }                                                                      \
  return hipErrorInvalidValue;

template <typename S>
hipError_t launch_aba(const AbaArgs<S>& a, const Shape& sh, const Tiling& tl, hipStream_t st) {
  ABADJ_DISPATCH(launch_aba_v, launch_aba_chain)
}
template <typename S>
hipError_t launch_forward(const FwdArgs<S>& a, const Shape& sh, const Tiling& tl, hipStream_t st) {
  ABADJ_DISPATCH(launch_forward_v, launch_forward_chain)
}
template <typename S>
hipError_t launch_backward(const BwdArgs<S>& a, const Shape& sh, const Tiling& tl, hipStream_t st) {
  ABADJ_DISPATCH(launch_backward_v, launch_backward_chain)
}
template <typename S>
hipError_t launch_forward_jvp(const JvpArgs<S>& a, const Shape& sh, const Tiling& tl, hipStream_t st) {
  ABADJ_DISPATCH(launch_forward_jvp_v, launch_forward_jvp_chain)
}
#undef ABADJ_DISPATCH

template hipError_t launch_aba<float>(const AbaArgs<float>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_aba<double>(const AbaArgs<double>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_forward<float>(const FwdArgs<float>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_forward<double>(const FwdArgs<double>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_backward<float>(const BwdArgs<float>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_backward<double>(const BwdArgs<double>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_forward_jvp<float>(const JvpArgs<float>&, const Shape&, const Tiling&, hipStream_t);
template hipError_t launch_forward_jvp<double>(const JvpArgs<double>&, const Shape&, const Tiling&, hipStream_t);

}  // namespace aba
