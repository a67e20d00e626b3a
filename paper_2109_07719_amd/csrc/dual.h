// Dual numbers (value, directional derivative) for the forward-mode
// (tangent) rollout.  The per-link ABA, integrator and spatial-algebra code
// is templated on its scalar type; instantiated with Dual<S> it carries one
// tangent direction alongside every value, so d(x^T)/d(x^0, u) . v comes out
// of the same statements as x^T itself.  Constants (link parameters,
// gravity, dt) enter with a zero tangent, which the device build's
// finite-math folding removes from the arithmetic.
#pragma once

#include <type_traits>

#include "spatial.h"

namespace aba {

template <typename S>
struct Dual {
  S v, d;
  Dual() = default;
  template <typename T, typename = std::enable_if_t<std::is_arithmetic_v<T>>>
  ABA_HD Dual(T x) : v(S(x)), d(S(0)) {}
  ABA_HD Dual(S x, S dx) : v(x), d(dx) {}
};

template <typename S>
ABA_HD Dual<S> operator+(const Dual<S>& a, const Dual<S>& b) {
  return Dual<S>(a.v + b.v, a.d + b.d);
}
template <typename S>
ABA_HD Dual<S> operator-(const Dual<S>& a, const Dual<S>& b) {
  return Dual<S>(a.v - b.v, a.d - b.d);
}
template <typename S>
ABA_HD Dual<S> operator-(const Dual<S>& a) {
  return Dual<S>(-a.v, -a.d);
}
template <typename S>
ABA_HD Dual<S> operator*(const Dual<S>& a, const Dual<S>& b) {
  return Dual<S>(a.v * b.v, a.d * b.v + a.v * b.d);
}
// the value parts use the same operations as the plain-valued code (a true
// division here, the reciprocal instruction in rcp), so the value part of a
// tangent rollout repeats the plain rollout's arithmetic
template <typename S>
ABA_HD Dual<S> operator/(const Dual<S>& a, const Dual<S>& b) {
  const S q = a.v / b.v;
  return Dual<S>(q, (a.d - q * b.d) / b.v);
}
template <typename S>
ABA_HD Dual<S>& operator+=(Dual<S>& a, const Dual<S>& b) {
  a = a + b;
  return a;
}
template <typename S>
ABA_HD Dual<S> rcp(const Dual<S>& a) {
  const S r = rcp(a.v);
  return Dual<S>(r, -a.d * r * r);
}
template <typename S>
ABA_HD Dual<S> sqrt(const Dual<S>& a) {
  using std::sqrt;
  const S s = sqrt(a.v);
  return Dual<S>(s, a.d * (S(0.5) * rcp(s)));
}

}  // namespace aba
