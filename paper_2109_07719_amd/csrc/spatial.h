// Structured spatial algebra for one link, written for registers.
//
// Motion vectors are [w; v] (angular first), force vectors [n; f].  A
// Plucker transform from parent to link coordinates is kept as (E, r):
// X = [E 0; -E[r]x E]; only E depends on the joint angle.  Symmetric 6x6
// spatial inertias are kept as [A B; B^T C] with A, C symmetric 3x3
// (21 numbers).  All functions are __host__ __device__ templates on the
// scalar type so the same code runs in the kernels and in host-side
// operation counting.
//
// Operators follow the spatial-algebra operator set of App. G
// (st_apply, st_apply_trans, st_multiply, sm_crossm, sm_crossf, dyad
// products, shift); their adjoints are re-derived here from the forward
// definitions (several printed adjoints in App. G are transposed or
// garbled, so none is transcribed).
#pragma once

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define ABA_HD __host__ __device__ __forceinline__
#else
#include <cmath>
#define ABA_HD inline
#endif

namespace aba {

template <typename S>
struct V3 {
  S x, y, z;
};
template <typename S>
struct V6 {
  V3<S> a, l;  // angular / moment part, linear / force part
};
template <typename S>
struct M3 {
  S m[9];  // row-major
};
template <typename S>
struct Sy3 {
  S xx, yy, zz, xy, xz, yz;
};
template <typename S>
struct SySp {  // [A B; B^T C]
  Sy3<S> A;
  M3<S> B;
  Sy3<S> C;
};

// reciprocal: one v_rcp_f32 (1 ulp) on the GPU in single precision, an exact
// division otherwise
ABA_HD float rcp(float x) {
#if defined(__HIP_DEVICE_COMPILE__)
  return __builtin_amdgcn_rcpf(x);
#else
  return 1.0f / x;
#endif
}
ABA_HD double rcp(double x) { return 1.0 / x; }
template <typename S>
ABA_HD S rcp(S x) {
  return S(1) / x;
}

// ---------------------------------------------------------------- 3-vectors
template <typename S>
ABA_HD V3<S> v3(S x, S y, S z) {
  V3<S> r;
  r.x = x;
  r.y = y;
  r.z = z;
  return r;
}
template <typename S>
ABA_HD V3<S> zero3() {
  return v3<S>(S(0), S(0), S(0));
}
template <typename S>
ABA_HD V3<S> operator+(const V3<S>& a, const V3<S>& b) {
  return v3<S>(a.x + b.x, a.y + b.y, a.z + b.z);
}
template <typename S>
ABA_HD V3<S> operator-(const V3<S>& a, const V3<S>& b) {
  return v3<S>(a.x - b.x, a.y - b.y, a.z - b.z);
}
template <typename S>
ABA_HD V3<S> operator-(const V3<S>& a) {
  return v3<S>(-a.x, -a.y, -a.z);
}
template <typename S>
ABA_HD V3<S> operator*(S s, const V3<S>& a) {
  return v3<S>(s * a.x, s * a.y, s * a.z);
}
template <typename S>
ABA_HD S dot(const V3<S>& a, const V3<S>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename S>
ABA_HD V3<S> cross(const V3<S>& a, const V3<S>& b) {
  return v3<S>(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
// a + s*b
template <typename S>
ABA_HD V3<S> axpy(const V3<S>& a, S s, const V3<S>& b) {
  return v3<S>(a.x + s * b.x, a.y + s * b.y, a.z + s * b.z);
}

// ---------------------------------------------------------------- 6-vectors
template <typename S>
ABA_HD V6<S> v6(const V3<S>& a, const V3<S>& l) {
  V6<S> r;
  r.a = a;
  r.l = l;
  return r;
}
template <typename S>
ABA_HD V6<S> zero6() {
  return v6<S>(zero3<S>(), zero3<S>());
}
template <typename S>
ABA_HD V6<S> operator+(const V6<S>& a, const V6<S>& b) {
  return v6<S>(a.a + b.a, a.l + b.l);
}
template <typename S>
ABA_HD V6<S> operator-(const V6<S>& a, const V6<S>& b) {
  return v6<S>(a.a - b.a, a.l - b.l);
}
template <typename S>
ABA_HD V6<S> operator*(S s, const V6<S>& a) {
  return v6<S>(s * a.a, s * a.l);
}
template <typename S>
ABA_HD S dot(const V6<S>& a, const V6<S>& b) {
  return dot(a.a, b.a) + dot(a.l, b.l);
}
// motion cross product  a x b = [wa x wb; wa x vb + va x wb]   (sm_crossm)
template <typename S>
ABA_HD V6<S> crm(const V6<S>& a, const V6<S>& b) {
  return v6<S>(cross(a.a, b.a), cross(a.a, b.l) + cross(a.l, b.a));
}
// force cross product  a x* f = [wa x n + va x f; wa x f]   (sm_crossf)
template <typename S>
ABA_HD V6<S> crf(const V6<S>& a, const V6<S>& f) {
  return v6<S>(cross(a.a, f.a) + cross(a.l, f.l), cross(a.a, f.l));
}
// crm(a)^T x = [x1 x wa + x2 x va; x2 x wa]
template <typename S>
ABA_HD V6<S> crmT(const V6<S>& a, const V6<S>& x) {
  return v6<S>(cross(x.a, a.a) + cross(x.l, a.l), cross(x.l, a.a));
}

// ---------------------------------------------------------------- 3x3
template <typename S>
ABA_HD V3<S> mul(const M3<S>& E, const V3<S>& v) {
  return v3<S>(E.m[0] * v.x + E.m[1] * v.y + E.m[2] * v.z,
               E.m[3] * v.x + E.m[4] * v.y + E.m[5] * v.z,
               E.m[6] * v.x + E.m[7] * v.y + E.m[8] * v.z);
}
template <typename S>
ABA_HD V3<S> mulT(const M3<S>& E, const V3<S>& v) {
  return v3<S>(E.m[0] * v.x + E.m[3] * v.y + E.m[6] * v.z,
               E.m[1] * v.x + E.m[4] * v.y + E.m[7] * v.z,
               E.m[2] * v.x + E.m[5] * v.y + E.m[8] * v.z);
}
template <typename S>
ABA_HD M3<S> mul(const M3<S>& A, const M3<S>& B) {
  M3<S> C;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      C.m[3 * i + j] = A.m[3 * i] * B.m[j] + A.m[3 * i + 1] * B.m[3 + j] + A.m[3 * i + 2] * B.m[6 + j];
  return C;
}
template <typename S>
ABA_HD V3<S> row(const M3<S>& A, int i) {
  return v3<S>(A.m[3 * i], A.m[3 * i + 1], A.m[3 * i + 2]);
}
template <typename S>
ABA_HD V3<S> col(const M3<S>& A, int j) {
  return v3<S>(A.m[j], A.m[3 + j], A.m[6 + j]);
}
template <typename S>
ABA_HD V3<S> mul(const Sy3<S>& A, const V3<S>& v) {
  return v3<S>(A.xx * v.x + A.xy * v.y + A.xz * v.z, A.xy * v.x + A.yy * v.y + A.yz * v.z,
               A.xz * v.x + A.yz * v.y + A.zz * v.z);
}
template <typename S>
ABA_HD Sy3<S> sy3(S xx, S yy, S zz, S xy, S xz, S yz) {
  Sy3<S> r;
  r.xx = xx;
  r.yy = yy;
  r.zz = zz;
  r.xy = xy;
  r.xz = xz;
  r.yz = yz;
  return r;
}
template <typename S>
ABA_HD Sy3<S> operator+(const Sy3<S>& a, const Sy3<S>& b) {
  return sy3<S>(a.xx + b.xx, a.yy + b.yy, a.zz + b.zz, a.xy + b.xy, a.xz + b.xz, a.yz + b.yz);
}
template <typename S>
ABA_HD Sy3<S> operator-(const Sy3<S>& a, const Sy3<S>& b) {
  return sy3<S>(a.xx - b.xx, a.yy - b.yy, a.zz - b.zz, a.xy - b.xy, a.xz - b.xz, a.yz - b.yz);
}
template <typename S>
ABA_HD M3<S> operator+(const M3<S>& a, const M3<S>& b) {
  M3<S> r;
#pragma unroll
  for (int k = 0; k < 9; ++k) r.m[k] = a.m[k] + b.m[k];
  return r;
}
// sym(u v^T + v u^T) * s   (symmetric rank-2 update, s scalar)
template <typename S>
ABA_HD Sy3<S> sym_outer(const V3<S>& u, const V3<S>& v, S s) {
  return sy3<S>(S(2) * s * u.x * v.x, S(2) * s * u.y * v.y, S(2) * s * u.z * v.z,
                s * (u.x * v.y + v.x * u.y), s * (u.x * v.z + v.x * u.z), s * (u.y * v.z + v.y * u.z));
}
// s * u u^T
template <typename S>
ABA_HD Sy3<S> self_outer(const V3<S>& u, S s) {
  return sy3<S>(s * u.x * u.x, s * u.y * u.y, s * u.z * u.z, s * u.x * u.y, s * u.x * u.z, s * u.y * u.z);
}
// s * u v^T
template <typename S>
ABA_HD M3<S> outer(const V3<S>& u, const V3<S>& v, S s) {
  M3<S> r;
  const S us[3] = {s * u.x, s * u.y, s * u.z};
  const S vv[3] = {v.x, v.y, v.z};
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) r.m[3 * i + j] = us[i] * vv[j];
  return r;
}

// E^T A E for symmetric A (symmetric result)
template <typename S>
ABA_HD Sy3<S> congT(const M3<S>& E, const Sy3<S>& A) {
  // T = A E (columns j: A * E[:,j])
  const V3<S> t0 = mul(A, col(E, 0)), t1 = mul(A, col(E, 1)), t2 = mul(A, col(E, 2));
  const V3<S> e0 = col(E, 0), e1 = col(E, 1), e2 = col(E, 2);
  return sy3<S>(dot(e0, t0), dot(e1, t1), dot(e2, t2), dot(e0, t1), dot(e0, t2), dot(e1, t2));
}
// E A E^T for symmetric A
template <typename S>
ABA_HD Sy3<S> cong(const M3<S>& E, const Sy3<S>& A) {
  const V3<S> r0 = row(E, 0), r1 = row(E, 1), r2 = row(E, 2);
  const V3<S> t0 = mul(A, r0), t1 = mul(A, r1), t2 = mul(A, r2);
  return sy3<S>(dot(r0, t0), dot(r1, t1), dot(r2, t2), dot(r0, t1), dot(r0, t2), dot(r1, t2));
}
// E^T B E for general B
template <typename S>
ABA_HD M3<S> congT(const M3<S>& E, const M3<S>& B) {
  M3<S> R;
  const V3<S> e[3] = {col(E, 0), col(E, 1), col(E, 2)};
  V3<S> t[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) t[j] = mul(B, e[j]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) R.m[3 * i + j] = dot(e[i], t[j]);
  return R;
}
// E B E^T for general B
template <typename S>
ABA_HD M3<S> cong(const M3<S>& E, const M3<S>& B) {
  M3<S> R;
  const V3<S> e[3] = {row(E, 0), row(E, 1), row(E, 2)};
  V3<S> t[3];
#pragma unroll
  for (int j = 0; j < 3; ++j) t[j] = mul(B, e[j]);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) R.m[3 * i + j] = dot(e[i], t[j]);
  return R;
}

// ---------------------------------------------------------------- transforms
// X m = [E w; E (v - r x w)]              (st_apply)
template <typename S>
ABA_HD V6<S> xform(const M3<S>& E, const V3<S>& r, const V6<S>& m) {
  return v6<S>(mul(E, m.a), mul(E, m.l - cross(r, m.a)));
}
// X^T f = [E^T n + r x (E^T f); E^T f]    (st_apply_trans)
template <typename S>
ABA_HD V6<S> xformT(const M3<S>& E, const V3<S>& r, const V6<S>& f) {
  const V3<S> g = mulT(E, f.l);
  return v6<S>(mulT(E, f.a) + cross(r, g), g);
}

// rows of B crossed with r: returns matrix whose row i is  B_i x r
template <typename S>
ABA_HD M3<S> rows_cross(const M3<S>& B, const V3<S>& r) {
  M3<S> R;
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    const V3<S> c = cross(row(B, i), r);
    R.m[3 * i] = c.x;
    R.m[3 * i + 1] = c.y;
    R.m[3 * i + 2] = c.z;
  }
  return R;
}
// [r]x M  (column j = r x M[:,j])
template <typename S>
ABA_HD M3<S> rx_mul(const V3<S>& r, const M3<S>& M) {
  M3<S> R;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const V3<S> c = cross(r, col(M, j));
    R.m[j] = c.x;
    R.m[3 + j] = c.y;
    R.m[6 + j] = c.z;
  }
  return R;
}
template <typename S>
ABA_HD M3<S> sy_to_m3(const Sy3<S>& A) {
  M3<S> R;
  R.m[0] = A.xx; R.m[1] = A.xy; R.m[2] = A.xz;
  R.m[3] = A.xy; R.m[4] = A.yy; R.m[5] = A.yz;
  R.m[6] = A.xz; R.m[7] = A.yz; R.m[8] = A.zz;
  return R;
}

// Congruence X^T M X (the "shift" of a spatial dyad from link to parent
// coordinates).  With X = rot(E) xlt(r):
//   A' = E^T A E, B' = E^T B E, C' = E^T C E,
//   C'' = C', B'' = B' + [r]x C', A'' = A' + [r]x B'^T - B'' [r]x.
template <typename S>
ABA_HD SySp<S> congruence_XT(const M3<S>& E, const V3<S>& r, const SySp<S>& M) {
  const Sy3<S> Ap = congT(E, M.A);
  const M3<S> Bp = congT(E, M.B);
  const Sy3<S> Cp = congT(E, M.C);
  SySp<S> R;
  R.C = Cp;
  R.B = Bp + rx_mul(r, sy_to_m3(Cp));
  // (r x B'^T)_{ij} = (r x B'_j)_i ;  (B'' [r]x)_{ij} = (B''_i x r)_j
  const V3<S> pb[3] = {cross(r, row(Bp, 0)), cross(r, row(Bp, 1)), cross(r, row(Bp, 2))};
  const V3<S> qb[3] = {cross(row(R.B, 0), r), cross(row(R.B, 1), r), cross(row(R.B, 2), r)};
  R.A = sy3<S>(Ap.xx + pb[0].x - qb[0].x, Ap.yy + pb[1].y - qb[1].y, Ap.zz + pb[2].z - qb[2].z,
               Ap.xy + pb[1].x - qb[0].y, Ap.xz + pb[2].x - qb[0].z, Ap.yz + pb[2].y - qb[1].z);
  return R;
}

// Congruence X N X^T of a symmetric spatial dyad (used by the adjoint of the
// shift: the child's share of the parent's inertia adjoint).  With
// X = rot(E) xlt(r), xlt N xlt^T = [A, A[r]x + B; ., C - [r]x B - ([r]x B)^T - [r]x A [r]x]
// then every block is rotated by E (.) E^T.
template <typename S>
ABA_HD SySp<S> congruence_X(const M3<S>& E, const V3<S>& r, const SySp<S>& N) {
  const M3<S> A = sy_to_m3(N.A);
  // A [r]x : row i = A_i x r ... (A [r]x)_{ij} = A_i . (r x e_j) = (A_i x r)_j
  const M3<S> Arx = rows_cross(A, r);
  const M3<S> Bo = Arx + N.B;
  // [r]x B
  const M3<S> rxB = rx_mul(r, N.B);
  // [r]x A [r]x = [r]x (A [r]x)
  const M3<S> rxArx = rx_mul(r, Arx);
  Sy3<S> Co;
  Co.xx = N.C.xx - S(2) * rxB.m[0] - rxArx.m[0];
  Co.yy = N.C.yy - S(2) * rxB.m[4] - rxArx.m[4];
  Co.zz = N.C.zz - S(2) * rxB.m[8] - rxArx.m[8];
  Co.xy = N.C.xy - rxB.m[1] - rxB.m[3] - rxArx.m[1];
  Co.xz = N.C.xz - rxB.m[2] - rxB.m[6] - rxArx.m[2];
  Co.yz = N.C.yz - rxB.m[5] - rxB.m[7] - rxArx.m[5];
  SySp<S> R;
  R.A = cong(E, N.A);
  R.B = cong(E, Bo);
  R.C = cong(E, Co);
  return R;
}

// M v for a symmetric spatial dyad
template <typename S>
ABA_HD V6<S> mul(const SySp<S>& M, const V6<S>& v) {
  return v6<S>(mul(M.A, v.a) + mul(M.B, v.l), mulT(M.B, v.a) + mul(M.C, v.l));
}
template <typename S>
ABA_HD SySp<S> operator+(const SySp<S>& a, const SySp<S>& b) {
  SySp<S> r;
  r.A = a.A + b.A;
  r.B = a.B + b.B;
  r.C = a.C + b.C;
  return r;
}
// M - s u u^T
template <typename S>
ABA_HD SySp<S> rank1_down(const SySp<S>& M, const V6<S>& u, S s) {
  SySp<S> r;
  r.A = M.A - self_outer(u.a, s);
  const M3<S> o = outer(u.a, u.l, s);
#pragma unroll
  for (int k = 0; k < 9; ++k) r.B.m[k] = M.B.m[k] - o.m[k];
  r.C = M.C - self_outer(u.l, s);
  return r;
}
// M + s * sym(x y^T) = M + s/2 (x y^T + y x^T)
template <typename S>
ABA_HD SySp<S> add_sym_outer(const SySp<S>& M, const V6<S>& x, const V6<S>& y, S s) {
  const S h = S(0.5) * s;
  SySp<S> r;
  r.A = M.A + sym_outer(x.a, y.a, h);
  const M3<S> o1 = outer(x.a, y.l, h), o2 = outer(y.a, x.l, h);
#pragma unroll
  for (int k = 0; k < 9; ++k) r.B.m[k] = M.B.m[k] + o1.m[k] + o2.m[k];
  r.C = M.C + sym_outer(x.l, y.l, h);
  return r;
}
template <typename S>
ABA_HD SySp<S> zero_sysp() {
  SySp<S> r;
  r.A = sy3<S>(S(0), S(0), S(0), S(0), S(0), S(0));
#pragma unroll
  for (int k = 0; k < 9; ++k) r.B.m[k] = S(0);
  r.C = r.A;
  return r;
}

// antisymmetric-part vector of a 3x3 product X Y:  avec(W) with
// <W, [a]x> = a . avec(W),  avec(W) = (W21 - W12, W02 - W20, W10 - W01)
template <typename S>
ABA_HD V3<S> avec_prod(const M3<S>& X, const M3<S>& Y) {
  const V3<S> x0 = row(X, 0), x1 = row(X, 1), x2 = row(X, 2);
  const V3<S> y0 = col(Y, 0), y1 = col(Y, 1), y2 = col(Y, 2);
  return v3<S>(dot(x2, y1) - dot(x1, y2), dot(x0, y2) - dot(x2, y0), dot(x1, y0) - dot(x0, y1));
}
template <typename S>
ABA_HD M3<S> transpose(const M3<S>& A) {
  M3<S> R;
  R.m[0] = A.m[0]; R.m[1] = A.m[3]; R.m[2] = A.m[6];
  R.m[3] = A.m[1]; R.m[4] = A.m[4]; R.m[5] = A.m[7];
  R.m[6] = A.m[2]; R.m[7] = A.m[5]; R.m[8] = A.m[8];
  return R;
}

// <M N, crm([a; l])> for symmetric spatial dyads M, N.  crm([a; l]) has
// [a]x in both diagonal blocks and [l]x in the lower-left one, so
//   = a . avec(M_A N_A + M_B N_B^T + M_B^T N_B + M_C N_C)
//   + l . avec(M_B^T N_A + M_C N_B^T)
// crmS_vec(M, N) is the vector [w; wl] of those two avec terms, so that the
// pairing is linear in s: <M N, crm(s)> = s . crmS_vec(M, N).
template <typename S>
ABA_HD V6<S> crmS_vec(const SySp<S>& M, const SySp<S>& N) {
  const M3<S> MA = sy_to_m3(M.A), NA = sy_to_m3(N.A), MC = sy_to_m3(M.C), NC = sy_to_m3(N.C);
  const M3<S> MBt = transpose(M.B), NBt = transpose(N.B);
  const V3<S> w = avec_prod(MA, NA) + avec_prod(M.B, NBt) + avec_prod(MBt, N.B) + avec_prod(MC, NC);
  const V3<S> wl = avec_prod(MBt, NA) + avec_prod(MC, NBt);
  return v6<S>(w, wl);
}
template <typename S>
ABA_HD S pair_crmS(const SySp<S>& M, const SySp<S>& N, const V6<S>& s) {
  return dot(s, crmS_vec(M, N));
}

// ---------------------------------------------------------------- quaternions (x, y, z, w)
template <typename S>
struct Q4 {
  S x, y, z, w;
};
// R(q) v with R = (w^2 - u.u) I + 2 u u^T + 2 w [u]x  (body -> world)
template <typename S>
ABA_HD V3<S> quat_rotate(const Q4<S>& q, const V3<S>& v) {
  const V3<S> u = v3<S>(q.x, q.y, q.z);
  return axpy(axpy((q.w * q.w - dot(u, u)) * v, S(2) * dot(u, v), u), S(2) * q.w, cross(u, v));
}
// R(q)^T v
template <typename S>
ABA_HD V3<S> quat_rotate_T(const Q4<S>& q, const V3<S>& v) {
  const V3<S> u = v3<S>(q.x, q.y, q.z);
  return axpy(axpy((q.w * q.w - dot(u, u)) * v, S(2) * dot(u, v), u), S(-2) * q.w, cross(u, v));
}
// gradient of x^T R(q) y with respect to (u, w)
template <typename S>
ABA_HD Q4<S> quat_rot_grad(const Q4<S>& q, const V3<S>& x, const V3<S>& y) {
  const V3<S> u = v3<S>(q.x, q.y, q.z);
  const S xy = dot(x, y);
  const V3<S> gu = axpy(axpy(axpy(S(-2) * xy * u, S(2) * dot(u, y), x), S(2) * dot(x, u), y), S(2) * q.w,
                        cross(y, x));
  Q4<S> g;
  g.x = gu.x;
  g.y = gu.y;
  g.z = gu.z;
  g.w = S(2) * q.w * xy + S(2) * dot(x, cross(u, y));
  return g;
}

}  // namespace aba
