// Per-link (per-lane) steps of the Articulated Body Algorithm, one
// semi-implicit Euler step, and the adjoint of each, in structured spatial
// algebra.  The kernels call these with one lane per link and exchange the
// parent/child quantities between lanes; a sequential host driver calls the
// same functions link by link to count algorithmic operations.
//
// Method (Sec. 3 "Articulated body dynamics"; Fig. 1; Sec. 4.1, five
// modules): pass 1 root->leaves (kinematics, velocities, bias forces), pass
// 2 leaves->root (articulated inertias and bias forces), pass 3
// root->leaves (accelerations), then time integration.  The adjoint runs the
// modules in reverse order (Sec. 4.1) after recomputing the step's
// intermediates from the stored initial state (Sec. 4.2, Eq. intermediate).
//
// Joint-coordinate derivatives use dX/dq = -crm(S) X, which holds for a
// revolute and a prismatic joint alike (X = X_J(q) X_T, X_J = exp(-q crm(S))),
// so every statement that applies X contributes a cross-product pairing to
// q_bar instead of a full X_bar.
#pragma once

#include "spatial.h"

namespace aba {

// per-link constants
template <typename S>
struct LinkC {
  M3<S> ET;   // fixed rotation parent -> joint frame
  V3<S> rT;   // joint origin in parent coordinates
  V6<S> sm;   // motion subspace of the 1-dof joint: [e_z; 0] revolute, [0; e_z]
              // prismatic (link coordinates, after canonicalisation)
  bool prism; // prismatic joint: the link slides along e_z instead of turning
  S m;        // mass
  V3<S> mc;   // mass * centre of mass
  Sy3<S> Ib;  // rotational inertia about the link origin: Ic - m [c]x^2
};

// spatial inertia applied to a motion vector: [Ib w + mc x v; m v - mc x w]
template <typename S>
ABA_HD V6<S> inertia_mul(const LinkC<S>& L, const V6<S>& v) {
  return v6<S>(mul(L.Ib, v.a) + cross(L.mc, v.l), L.m * v.l - cross(L.mc, v.a));
}
template <typename S>
ABA_HD SySp<S> inertia_sysp(const LinkC<S>& L) {
  SySp<S> I;
  I.A = L.Ib;
  const V3<S>& c = L.mc;
  I.B.m[0] = S(0); I.B.m[1] = -c.z; I.B.m[2] = c.y;
  I.B.m[3] = c.z;  I.B.m[4] = S(0); I.B.m[5] = -c.x;
  I.B.m[6] = -c.y; I.B.m[7] = c.x;  I.B.m[8] = S(0);
  I.C = sy3<S>(L.m, L.m, L.m, S(0), S(0), S(0));
  return I;
}

// ----------------------------------------------------------------- forward
// Intermediates of one link kept for the reverse sweep.
template <typename S>
struct Tape {
  S sq, cq;    // joint coordinate as X_J needs it: sin q, cos q (revolute); q, 1 (prismatic)
  M3<S> E;     // rotation of X = X_J(q) X_T (its translation: joint_r)
  V6<S> v, c;
  SySp<S> IA;  // final articulated inertia (children included)
  V6<S> pA;    // final articulated bias force
  V6<S> U;
  S Dinv, u;
  V6<S> pa;    // bias force handed to the parent
  V6<S> ap;    // X a_parent + c
  S qdd;
  // ball joint only: the joint-space blocks of pass 2 (ball_p2_local; not
  // carried by widen or the stored tapes: the reverse pass rebuilds them)
  Sy3<S> Ai;   // A^-1, A the angular block of IA
  M3<S> W;     // A^-1 B
  V3<S> y;     // A^-1 u
};

// Exact conversion of a link's constants and step intermediates to a wider
// scalar type, for an adjoint that runs in FP64 from an FP32 forward: the
// reverse passes then see exactly the numbers the forward computed.
template <typename R, typename S>
ABA_HD V3<R> widen(const V3<S>& v) {
  return v3<R>(R(v.x), R(v.y), R(v.z));
}
template <typename R, typename S>
ABA_HD V6<R> widen(const V6<S>& v) {
  return v6<R>(widen<R>(v.a), widen<R>(v.l));
}
template <typename R, typename S>
ABA_HD M3<R> widen(const M3<S>& M) {
  M3<R> W;
#pragma unroll
  for (int k = 0; k < 9; ++k) W.m[k] = R(M.m[k]);
  return W;
}
template <typename R, typename S>
ABA_HD Sy3<R> widen(const Sy3<S>& M) {
  return sy3<R>(R(M.xx), R(M.yy), R(M.zz), R(M.xy), R(M.xz), R(M.yz));
}
template <typename R, typename S>
ABA_HD SySp<R> widen(const SySp<S>& M) {
  SySp<R> W;
  W.A = widen<R>(M.A);
  W.B = widen<R>(M.B);
  W.C = widen<R>(M.C);
  return W;
}
template <typename R, typename S>
ABA_HD LinkC<R> widen(const LinkC<S>& L) {
  LinkC<R> W;
  W.ET = widen<R>(L.ET);
  W.rT = widen<R>(L.rT);
  W.sm = widen<R>(L.sm);
  W.prism = L.prism;
  W.m = R(L.m);
  W.mc = widen<R>(L.mc);
  W.Ib = widen<R>(L.Ib);
  return W;
}
template <typename R, typename S>
ABA_HD Tape<R> widen(const Tape<S>& t) {
  Tape<R> W;
  W.sq = R(t.sq);
  W.cq = R(t.cq);
  W.E = widen<R>(t.E);
  W.v = widen<R>(t.v);
  W.c = widen<R>(t.c);
  W.IA = widen<R>(t.IA);
  W.pA = widen<R>(t.pA);
  W.U = widen<R>(t.U);
  W.Dinv = R(t.Dinv);
  W.u = R(t.u);
  W.pa = widen<R>(t.pa);
  W.ap = widen<R>(t.ap);
  W.qdd = R(t.qdd);
  return W;
}

// X = X_J(q) X_T = (E, r) for a joint about or along the link's z axis
// (the host rotates every link frame so that its joint axis is e_z), from
// the tape's joint coordinate.
// Revolute: E = E_J(q) E_T with E_J = I - sin q [e_z]x + (1 - cos q)[e_z]x^2
// = [[c, s, 0], [-s, c, 0], [0, 0, 1]], r = r_T.  Prismatic: X_J is the
// translation by q e_z, so E = E_T and r = r_T + q E_T^T e_z.
// joint_X sets E; joint_r gives r where it is used, so that the revolute
// kernels keep r_T as the link constant it is.
template <typename S>
ABA_HD void joint_X(const LinkC<S>& L, Tape<S>& t) {
  if (L.prism) {
    t.E = L.ET;
  } else {
    M3<S> J;
    J.m[0] = t.cq;  J.m[1] = t.sq; J.m[2] = S(0);
    J.m[3] = -t.sq; J.m[4] = t.cq; J.m[5] = S(0);
    J.m[6] = S(0);  J.m[7] = S(0); J.m[8] = S(1);
    t.E = mul(J, L.ET);
  }
}
template <typename S>
ABA_HD V3<S> joint_r(const LinkC<S>& L, const Tape<S>& t) {
  return L.prism ? axpy(L.rT, t.sq, row(L.ET, 2)) : L.rT;
}

// pass 1 (1-dof joint): v = X v_parent + S qd
template <typename S>
ABA_HD V6<S> p1_velocity(const LinkC<S>& L, const Tape<S>& t, S qd, const V6<S>& vpar) {
  return xform(t.E, joint_r(L, t), vpar) + qd * L.sm;
}
// pass 1 (all links): c = v x S qd, h = I v, pA = v x* h, IA = I
template <typename S>
ABA_HD void p1_bias(const LinkC<S>& L, const V6<S>& v, S qd, bool onedof, V6<S>& c, V6<S>& pA,
                    SySp<S>& IA) {
  c = onedof ? crm(v, qd * L.sm) : zero6<S>();
  const V6<S> h = inertia_mul(L, v);
  pA = crf(v, h);
  IA = inertia_sysp(L);
}
// pass 2 (1-dof joint): U = IA S, D = S^T U, u = tau - S^T pA
template <typename S>
ABA_HD void p2_local(const LinkC<S>& L, Tape<S>& t, S tau) {
  t.U = mul(t.IA, L.sm);
  t.Dinv = rcp(dot(L.sm, t.U));
  t.u = tau - dot(L.sm, t.pA);
}
// pass 2 (1-dof joint with a parent link): Ia = IA - U U^T / D,
// pa = pA + Ia c + U u / D; the parent receives X^T Ia X and X^T pa.
template <typename S>
ABA_HD void p2_push(const LinkC<S>& L, Tape<S>& t, SySp<S>& IA_up, V6<S>& pA_up) {
  const SySp<S> Ia = rank1_down(t.IA, t.U, t.Dinv);
  t.pa = t.pA + mul(Ia, t.c) + (t.u * t.Dinv) * t.U;
  IA_up = congruence_XT(t.E, joint_r(L, t), Ia);
  pA_up = xformT(t.E, joint_r(L, t), t.pa);
}
// pass 3 (1-dof joint): a' = X a_parent + c, qdd = (u - U^T a') / D, a = a' + S qdd
template <typename S>
ABA_HD V6<S> p3_accel(const LinkC<S>& L, Tape<S>& t, const V6<S>& apar) {
  t.ap = xform(t.E, joint_r(L, t), apar) + t.c;
  t.qdd = (t.u - dot(t.U, t.ap)) * t.Dinv;
  return t.ap + t.qdd * L.sm;
}

// ------------------------------------------------------- free-floating root
// 6x6 SPD factorisation (lower Cholesky, packed rows)
template <typename S>
struct Chol6 {
  S L[21];
};
template <typename S>
ABA_HD void sysp_dense(const SySp<S>& M, S A[36]) {
  const M3<S> a = sy_to_m3(M.A), c = sy_to_m3(M.C);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      A[6 * i + j] = a.m[3 * i + j];
      A[6 * i + j + 3] = M.B.m[3 * i + j];
      A[6 * (i + 3) + j] = M.B.m[3 * j + i];
      A[6 * (i + 3) + j + 3] = c.m[3 * i + j];
    }
}
template <typename S>
ABA_HD Chol6<S> chol6(const SySp<S>& M) {
  S A[36];
  sysp_dense(M, A);
  Chol6<S> f;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
#pragma unroll
    for (int j = 0; j <= i; ++j) {
      S s = A[6 * i + j];
#pragma unroll
      for (int k = 0; k < j; ++k) s = s - f.L[i * (i + 1) / 2 + k] * f.L[j * (j + 1) / 2 + k];
      if (i == j)
        f.L[i * (i + 1) / 2 + i] = sqrt(s);
      else
        f.L[i * (i + 1) / 2 + j] = s / f.L[j * (j + 1) / 2 + j];
    }
  }
  return f;
}
template <typename S>
ABA_HD V6<S> chol6_solve(const Chol6<S>& f, const V6<S>& b) {
  S x[6] = {b.a.x, b.a.y, b.a.z, b.l.x, b.l.y, b.l.z};
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    S s = x[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s = s - f.L[i * (i + 1) / 2 + k] * x[k];
    x[i] = s / f.L[i * (i + 1) / 2 + i];
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    S s = x[i];
#pragma unroll
    for (int k = i + 1; k < 6; ++k) s = s - f.L[k * (k + 1) / 2 + i] * x[k];
    x[i] = s / f.L[i * (i + 1) / 2 + i];
  }
  return v6<S>(v3<S>(x[0], x[1], x[2]), v3<S>(x[3], x[4], x[5]));
}
// root acceleration in the gravity-free frame a' = -IA^{-1} pA, and the true
// body-frame acceleration a' + [0; R^T g]
template <typename S>
ABA_HD void root_accel(const SySp<S>& IA, const V6<S>& pA, const Q4<S>& quat, const V3<S>& g, V6<S>& ap,
                       V6<S>& abase) {
  const Chol6<S> f = chol6(IA);
  const V6<S> x = chol6_solve(f, pA);
  ap = v6<S>(-x.a, -x.l);
  abase = v6<S>(ap.a, ap.l + quat_rotate_T(quat, g));
}

// ------------------------------------------------------------- ball joint
// A spherical joint: X_J = rot(R(quat)^T) (a rotation, no translation),
// S = [1; 0] (the three angular unit vectors of the link frame), state
// (quat, w) with w the joint's angular velocity in link coordinates, three
// torques; R(quat) = (w^2 - u.u) 1 + 2 u u^T + 2 w [u]x for quat = (u, w),
// so a quaternion off the unit sphere scales X_J by |quat|^2 (the joint
// model of Sec. 2 and the quaternion operators of App. G).  With S = [1; 0]
// the 3x3 joint-space blocks of pass 2 are blocks of IA = [A B; B^T C]:
// U = IA S = [A; B^T] and D = S^T U = A, hence
//   Ia = IA - U D^-1 U^T = [0 0; 0 C - B^T W],   W = A^-1 B,
//   pa = pA + Ia c + U D^-1 u = [tau; pA_l + Ia_C c_l + B^T y],  y = A^-1 u,
// and pass 3's qdd = D^-1 (u - U^T a') = y - a'_a - W a'_l with
// a = a' + S qdd = [y - W a'_l; a'_l].
template <typename S>
ABA_HD M3<S> ball_E(const Q4<S>& q, const M3<S>& ET) {
  M3<S> E;
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const V3<S> c = quat_rotate_T(q, col(ET, j));
    E.m[j] = c.x;
    E.m[3 + j] = c.y;
    E.m[6 + j] = c.z;
  }
  return E;
}
// inverse of a symmetric 3x3 matrix (adjugate over the determinant)
template <typename S>
ABA_HD Sy3<S> sy3_inv(const Sy3<S>& A) {
  const S c00 = A.yy * A.zz - A.yz * A.yz;
  const S c01 = A.xz * A.yz - A.xy * A.zz;
  const S c02 = A.xy * A.yz - A.xz * A.yy;
  const S c11 = A.xx * A.zz - A.xz * A.xz;
  const S c12 = A.xy * A.xz - A.xx * A.yz;
  const S c22 = A.xx * A.yy - A.xy * A.xy;
  const S id = rcp(A.xx * c00 + A.xy * c01 + A.xz * c02);
  return sy3<S>(c00 * id, c11 * id, c22 * id, c01 * id, c02 * id, c12 * id);
}
// Ia_C = C - B^T W
template <typename S>
ABA_HD Sy3<S> ball_IaC(const Tape<S>& t) {
  const M3<S>& B = t.IA.B;
  const V3<S> b0 = col(B, 0), b1 = col(B, 1), b2 = col(B, 2);
  const V3<S> w0 = col(t.W, 0), w1 = col(t.W, 1), w2 = col(t.W, 2);
  const Sy3<S>& C = t.IA.C;
  return sy3<S>(C.xx - dot(b0, w0), C.yy - dot(b1, w1), C.zz - dot(b2, w2), C.xy - dot(b0, w1),
                C.xz - dot(b0, w2), C.yz - dot(b1, w2));
}
// pass 1 (ball): E from the quaternion; v = X v_parent + [w; 0]; c = v x [w; 0]
template <typename S>
ABA_HD void ball_p1(const LinkC<S>& L, Tape<S>& t, const Q4<S>& quat, const V3<S>& w, const V6<S>& vpar) {
  t.E = ball_E(quat, L.ET);
  const V6<S> vJ = v6<S>(w, zero3<S>());
  t.v = xform(t.E, L.rT, vpar) + vJ;
}
// pass 2 (ball): the joint-space blocks; returns u = tau - pA_a
template <typename S>
ABA_HD V3<S> ball_p2_local(Tape<S>& t, const V3<S>& tau) {
  const V3<S> u = tau - t.pA.a;
  t.Ai = sy3_inv(t.IA.A);
  t.y = mul(t.Ai, u);
  t.W = mul(sy_to_m3(t.Ai), t.IA.B);
  return u;
}
// pass 2 (ball with a parent link): pa, and the parent's shares X^T Ia X, X^T pa
template <typename S>
ABA_HD void ball_p2_push(const LinkC<S>& L, Tape<S>& t, const V3<S>& tau, SySp<S>& IA_up, V6<S>& pA_up) {
  const Sy3<S> IaC = ball_IaC(t);
  t.pa = v6<S>(tau, t.pA.l + mul(IaC, t.c.l) + mulT(t.IA.B, t.y));
  SySp<S> Ia = zero_sysp<S>();
  Ia.C = IaC;
  IA_up = congruence_XT(t.E, L.rT, Ia);
  pA_up = xformT(t.E, L.rT, t.pa);
}
// pass 3 (ball): a' = X a_parent + c; qdd = y - a'_a - W a'_l; returns a
template <typename S>
ABA_HD V6<S> ball_p3(const LinkC<S>& L, Tape<S>& t, const V6<S>& apar, V3<S>& qdd) {
  t.ap = xform(t.E, L.rT, apar) + t.c;
  const V3<S> Wl = mul(t.W, t.ap.l);
  qdd = t.y - t.ap.a - Wl;
  return v6<S>(t.y - Wl, t.ap.l);
}

// ----------------------------------------------------------------- integrator
// 1-dof joint: qd1 = qd + dt qdd; q1 = q + dt qd1
template <typename S>
ABA_HD void integrate_joint(S& q, S& qd, S qdd, S dt) {
  qd = qd + dt * qdd;
  q = q + dt * qd;
}
// quaternion step of a free root or ball joint with the new angular
// velocity w1 (body frame): normalize(quat + dt/2 quat (x) (w1, 0))
template <typename S>
ABA_HD Q4<S> quat_step(const Q4<S>& quat, const V3<S>& w1, S dt) {
  const V3<S> u = v3<S>(quat.x, quat.y, quat.z);
  const V3<S> ov = axpy(cross(u, w1), quat.w, w1);
  const S ow = -dot(u, w1);
  const S h = S(0.5) * dt;
  Q4<S> r;
  r.x = quat.x + h * ov.x;
  r.y = quat.y + h * ov.y;
  r.z = quat.z + h * ov.z;
  r.w = quat.w + h * ow;
  const S inv = S(1) / sqrt(r.x * r.x + r.y * r.y + r.z * r.z + r.w * r.w);
  Q4<S> o;
  o.x = r.x * inv;
  o.y = r.y * inv;
  o.z = r.z * inv;
  o.w = r.w * inv;
  return o;
}
// free root: v1 = v + dt a; p1 = p + dt R(quat) v1_lin;
// quat1 = normalize(quat + dt/2 quat (x) (w1, 0))
template <typename S>
ABA_HD void integrate_root(V3<S>& p, Q4<S>& quat, V6<S>& v, const V6<S>& abase, S dt) {
  v = v + dt * abase;
  p = axpy(p, dt, quat_rotate(quat, v.l));
  quat = quat_step(quat, v.a, dt);
}

// ----------------------------------------------------------------- adjoint
// Per-link adjoint accumulators that live across the three reverse passes.
template <typename S>
struct Bar {
  V6<S> c;     // c_bar
  V6<S> U;     // U_bar
  S D, u;      // D_bar, u_bar
  S q, qd;     // contributions to the joint angle / rate adjoints
  // Model-parameter adjoints of the step, formed only when params is set
  // (a compile-time constant in the kernels):
  bool params;
  V6<S> G;     // the link transform's: X -> exp(-crm(z)) X changes the loss by G . z
  V6<S> Sb;    // the motion subspace's
};
template <typename S>
ABA_HD void bar_zero(Bar<S>& b, bool params = false) {
  b.params = params;
  b.c = zero6<S>();
  b.U = zero6<S>();
  b.D = S(0);
  b.u = S(0);
  b.q = S(0);
  b.qd = S(0);
  b.G = zero6<S>();
  b.Sb = zero6<S>();
}

// The pairing of a statement y = X m (x = y_bar) or y = X^T f (x = f,
// y = X y_bar) with a change X -> exp(-crm(z)) X is -x^T crm(z) y = z . qvec(x, y),
// qvec(x, y) = [x_ang x y_ang + x_lin x y_lin; x_lin x y_ang].  With
// dX/dq = -crm(S) X the joint-coordinate pairing is S . qvec(x, y).
template <typename S>
ABA_HD V6<S> qvec(const V6<S>& x, const V6<S>& y) {
  return v6<S>(cross(x.a, y.a) + cross(x.l, y.l), cross(x.l, y.a));
}
template <typename S>
ABA_HD S qpair(const V6<S>& sm, const V6<S>& x, const V6<S>& y) {
  return dot(sm, qvec(x, y));
}

// reverse of pass 3 (1-dof joint), in two parts for the level sweep.  The
// serial part needs abar, the link's acceleration adjoint with all
// children's shares added, and qddbar, the integrator's seed; it returns
// ap_bar (the parent receives X^T ap_bar) and g = qdd_bar / D.  The local
// part updates the link's own accumulators once the sweep is done.
template <typename S>
ABA_HD V6<S> r3_path(const LinkC<S>& L, const Tape<S>& t, const V6<S>& abar, S qddbar, S& g) {
  // a = ap + S qdd;  qdd = (u - U^T ap) / D
  g = (qddbar + dot(L.sm, abar)) * t.Dinv;
  return abar - g * t.U;
}
template <typename S>
ABA_HD void r3_local(const LinkC<S>& L, const Tape<S>& t, Bar<S>& b, const V6<S>& apb, S g) {
  b.u = b.u + g;
  b.U = b.U - g * t.ap;
  b.D = b.D - g * t.qdd;
  // ap = X a_parent + c
  const V6<S> xv = qvec(apb, t.ap - t.c);
  b.q = b.q + dot(L.sm, xv);
  b.c = b.c + apb;
  if (b.params) {
    b.G = b.G + xv;
    // a = ap + S qdd, with a_bar = ap_bar + g U
    b.Sb = b.Sb + t.qdd * (apb + g * t.U);
  }
}
template <typename S>
ABA_HD V6<S> r3_link(const LinkC<S>& L, const Tape<S>& t, Bar<S>& b, const V6<S>& abar, S qddbar) {
  S g;
  const V6<S> apb = r3_path(L, t, abar, qddbar, g);
  r3_local(L, t, b, apb, g);
  return apb;
}

// reverse of pass 2 (1-dof joint), in two parts.  The serial part takes the
// parent's adjoints IAbp / pAbp (used only when has_parent), completes
// U_bar, u_bar and D_bar, and produces this link's IA_bar / pA_bar (handed
// to the children) and tau_bar; it also returns N = X IAbp X^T and
// pab = X pAbp for the local part, which adds the joint-angle pairings of
// the shift and the Ia c term's share of c_bar.
template <typename S>
ABA_HD S r2_path(const LinkC<S>& L, const Tape<S>& t, Bar<S>& b, bool has_parent, const SySp<S>& IAbp,
                 const V6<S>& pAbp, SySp<S>& N, V6<S>& pab, SySp<S>& IAb, V6<S>& pAb) {
  IAb = zero_sysp<S>();
  pAb = zero6<S>();
  if (has_parent) {
    // pA_parent += X^T pa;  IA_parent += X^T Ia X
    pab = xform(t.E, joint_r(L, t), pAbp);
    N = congruence_X(t.E, joint_r(L, t), IAbp);
    // pa = pA + Ia c + U u / D
    pAb = pAb + pab;
    const SySp<S> Iab = add_sym_outer(N, pab, t.c, S(1));
    b.U = b.U + (t.u * t.Dinv) * pab;
    const S Upa = dot(t.U, pab);
    b.u = b.u + Upa * t.Dinv;
    b.D = b.D - Upa * t.u * t.Dinv * t.Dinv;
    // Ia = IA - U U^T / D
    IAb = IAb + Iab;
    const V6<S> IU = mul(Iab, t.U);
    b.U = b.U - (S(2) * t.Dinv) * IU;
    b.D = b.D + dot(t.U, IU) * t.Dinv * t.Dinv;
  }
  // u = tau - S^T pA
  const S taub = b.u;
  pAb = pAb - b.u * L.sm;
  // D = S^T U
  b.U = b.U + b.D * L.sm;
  // U = IA S   (symmetric part of U_bar S^T)
  IAb = add_sym_outer(IAb, b.U, L.sm, S(1));
  return taub;
}
template <typename S>
ABA_HD void r2_local(const LinkC<S>& L, const Tape<S>& t, Bar<S>& b, const SySp<S>& N, const V6<S>& pab) {
  const SySp<S> Ia = rank1_down(t.IA, t.U, t.Dinv);
  const V6<S> xv = qvec(t.pa, pab) - S(2) * crmS_vec(Ia, N);
  b.q = b.q + dot(L.sm, xv);
  if (b.params) b.G = b.G + xv;
  b.c = b.c + mul(Ia, pab);
}
// motion-subspace adjoint of pass 2 (every 1-dof link, once its U_bar,
// D_bar and u_bar are final): u = tau - S^T pA, D = S^T U, U = IA S
template <typename S>
ABA_HD void r2_sbar(const Tape<S>& t, Bar<S>& b) {
  b.Sb = b.Sb - b.u * t.pA + b.D * t.U + mul(t.IA, b.U);
}
template <typename S>
ABA_HD S r2_link(const LinkC<S>& L, const Tape<S>& t, Bar<S>& b, bool has_parent, const SySp<S>& IAbp,
                 const V6<S>& pAbp, SySp<S>& IAb, V6<S>& pAb) {
  SySp<S> N;
  V6<S> pab;
  const S taub = r2_path(L, t, b, has_parent, IAbp, pAbp, N, pab, IAb, pAb);
  if (has_parent) r2_local(L, t, b, N, pab);
  return taub;
}

// reverse of pass 1, in three parts.  r1_own: the link's own share of its
// velocity adjoint (from pA = v x* I v and, for a 1-dof joint,
// c = v x S qd), which needs only the link's final pA_bar and c_bar.  The
// serial part adds the children's shares and hands X^T v_bar to the parent.
// r1_local: qd_bar and q_bar from the complete v_bar.
template <typename S>
ABA_HD V6<S> r1_own(const LinkC<S>& L, const V6<S>& v, const Bar<S>& b, const V6<S>& pAb, S qd, bool onedof) {
  // pA(initial) = v x* h, h = I v
  const V6<S> h = inertia_mul(L, v);
  const V6<S> hb = v6<S>(-cross(v.a, pAb.a), -(cross(v.a, pAb.l) + cross(v.l, pAb.a)));
  V6<S> own = crmT(pAb, h) + inertia_mul(L, hb);
  if (onedof) {
    // c = v x vJ = -crm(vJ) v, vJ = S qd
    own = own - crmT(qd * L.sm, b.c);
  }
  return own;
}
template <typename S>
ABA_HD void r1_local(const LinkC<S>& L, const Tape<S>& t, Bar<S>& b, const V6<S>& vbar, S qd) {
  const V6<S> vJb = crmT(t.v, b.c) + vbar;
  b.qd = b.qd + dot(L.sm, vJb);
  // v = X v_parent + vJ
  const V6<S> Xv = t.v - qd * L.sm;
  const V6<S> xv = qvec(vbar, Xv);
  b.q = b.q + dot(L.sm, xv);
  if (b.params) {
    b.G = b.G + xv;
    // vJ = S qd
    b.Sb = b.Sb + qd * vJb;
  }
}
// 1-dof joint: vbar holds the children's shares; returns X^T v_bar
template <typename S>
ABA_HD V6<S> r1_link(const LinkC<S>& L, const Tape<S>& t, Bar<S>& b, V6<S> vbar, const V6<S>& pAb, S qd) {
  vbar = vbar + r1_own(L, t.v, b, pAb, qd, true);
  r1_local(L, t, b, vbar, qd);
  return xformT(t.E, joint_r(L, t), vbar);
}

// Adjoint of a link's ten inertial parameters: mass m, first moment
// mc (m times the centre of mass) and rotational inertia about the link
// origin Ib (unique entries xx yy zz xy xz yz; an off-diagonal parameter
// stands for both of its matrix entries), in the kernels' link frame.  The
// spatial inertia I = [Ib, [mc]x; [mc]x^T, m 1] enters a step twice: as the
// start of the articulated inertia (IA = I + children's shares, so its
// adjoint is the link's final IA_bar) and in h = I v of the bias force (h_bar
// follows from pA_bar as in r1_own).  IAb is a symmetric adjoint: the
// pairing with a symmetric change counts the B block twice.
// (Sec. 4.1, after Eq. adj_r: other parameters follow from the same
// per-step adjoints as the controls.)
template <typename S>
struct ParamBar {
  S m;
  V3<S> mc;
  Sy3<S> Ib;
  // placement and axis of a 1-dof joint (frame_bar_add)
  V6<S> xi;  // joint-frame perturbation of X_T
  V3<S> w;   // axis rotation, beyond xi's angular part
};
template <typename S>
ABA_HD void param_bar_zero(ParamBar<S>& g) {
  g.m = S(0);
  g.mc = zero3<S>();
  g.Ib = sy3<S>(S(0), S(0), S(0), S(0), S(0), S(0));
  g.xi = zero6<S>();
  g.w = zero3<S>();
}

// X_J^T f for the joint transform of the tape (revolute: rot(E_J) with
// E_J = [[c, s, 0], [-s, c, 0], [0, 0, 1]]; prismatic: xlt(q e_z), whose
// transpose is [1 [q e_z]x; 0 1]).
template <typename S>
ABA_HD V6<S> joint_XT_mul(const LinkC<S>& L, const Tape<S>& t, const V6<S>& f) {
  if (L.prism) {
    const V3<S> r = v3<S>(S(0), S(0), t.sq);
    return v6<S>(f.a + cross(r, f.l), f.l);
  }
  auto rotT = [&](const V3<S>& x) {
    return v3<S>(t.cq * x.x - t.sq * x.y, t.sq * x.x + t.cq * x.y, x.z);
  };
  return v6<S>(rotT(f.a), rotT(f.l));
}

// Adds one step's placement and axis adjoint of a 1-dof link, in the
// kernels' joint frame (axis e_z), from the step's transform adjoint G and
// motion-subspace adjoint Sb (Bar).  With X = X_J(q) X_T:
//   X_T -> exp(-crm(xi)) X_T moves X by -crm(X_J xi) X, so xi_bar += X_J^T G;
//   rotating the axis by w (a -> exp([w]x) a) turns X_J into
//   rot(R) X_J rot(R)^T, which moves X by -crm(X_J w - w) X (w = [w; 0]),
//   and S by [w x a; 0] (revolute) or [0; w x a] (prismatic):
//   w_bar += (X_J^T G)_ang - G_ang + a x Sb_(ang or lin).
// The first term is xi_bar's angular part, so only the rest is kept in w.
template <typename S>
ABA_HD void frame_bar_add(ParamBar<S>& g, const LinkC<S>& L, const Tape<S>& t, const Bar<S>& b) {
  g.xi = g.xi + joint_XT_mul(L, t, b.G);
  const V3<S> sb = L.prism ? b.Sb.l : b.Sb.a;
  g.w = g.w - b.G.a + v3<S>(-sb.y, sb.x, S(0));
}
template <typename S>
ABA_HD void param_bar_add(ParamBar<S>& g, const SySp<S>& IAb, const V6<S>& v, const V6<S>& pAb) {
  const M3<S>& B = IAb.B;
  g.m = g.m + (IAb.C.xx + IAb.C.yy + IAb.C.zz);
  g.mc = g.mc + S(2) * v3<S>(B.m[7] - B.m[5], B.m[2] - B.m[6], B.m[3] - B.m[1]);
  g.Ib = g.Ib + sy3<S>(IAb.A.xx, IAb.A.yy, IAb.A.zz, S(2) * IAb.A.xy, S(2) * IAb.A.xz, S(2) * IAb.A.yz);
  // h = I v = [Ib w + mc x vl; m vl - mc x w]
  const V6<S> hb = v6<S>(-cross(v.a, pAb.a), -(cross(v.a, pAb.l) + cross(v.l, pAb.a)));
  const V3<S>& w = v.a;
  g.m = g.m + dot(hb.l, v.l);
  g.mc = g.mc + (cross(v.l, hb.a) - cross(w, hb.l));
  g.Ib = g.Ib + sy3<S>(hb.a.x * w.x, hb.a.y * w.y, hb.a.z * w.z, hb.a.x * w.y + hb.a.y * w.x,
                       hb.a.x * w.z + hb.a.z * w.x, hb.a.y * w.z + hb.a.z * w.y);
}

// free root, reverse of pass 3 and of the root solve.  abar: children's
// shares; qddbar: base-acceleration seed from the integrator.  Adds the
// gravity term's quaternion adjoint into quatb; returns pA_bar and IA_bar.
template <typename S>
ABA_HD void r3_root(const SySp<S>& IA, const V6<S>& ap, const Q4<S>& quat, const V3<S>& g, const V6<S>& abar,
                    const V6<S>& qddbar, Q4<S>& quatb, SySp<S>& IAb, V6<S>& pAb) {
  // abase = ap + [0; R^T g]:  <qddbar_lin, R^T g> = g^T R qddbar_lin
  const Q4<S> gq = quat_rot_grad(quat, g, qddbar.l);
  quatb.x = quatb.x + gq.x;
  quatb.y = quatb.y + gq.y;
  quatb.z = quatb.z + gq.z;
  quatb.w = quatb.w + gq.w;
  const V6<S> apb = abar + qddbar;
  // ap = -IA^{-1} pA
  const V6<S> w = chol6_solve(chol6(IA), apb);
  pAb = v6<S>(-w.a, -w.l);
  IAb = add_sym_outer(zero_sysp<S>(), w, ap, S(-1));
}
// free root, reverse of pass 1: returns the body-velocity adjoint
template <typename S>
ABA_HD V6<S> r1_root(const LinkC<S>& L, const V6<S>& v, const V6<S>& vbar, const V6<S>& pAb) {
  Bar<S> b;
  bar_zero(b);
  return vbar + r1_own(L, v, b, pAb, S(0), false);
}

// ----------------------------------------------------- ball joint adjoint
// Accumulators of a ball lane beyond Bar (whose c, G it shares: G collects
// the pairings of X with rotations, X -> exp(-crm([d; 0])) X changing the
// loss by G_a . d, for every step, as the joint's quaternion needs them).
template <typename S>
struct BallBar {
  V3<S> y;  // y_bar
  M3<S> W;  // W_bar (all nine entries)
};
template <typename S>
ABA_HD void ball_bar_zero(BallBar<S>& bb) {
  bb.y = zero3<S>();
#pragma unroll
  for (int k = 0; k < 9; ++k) bb.W.m[k] = S(0);
}
// reverse of pass 3 (ball), serial part: abar with the children's shares,
// qddb the integrator's seed; returns ap_bar and sets s = a_bar_a + qdd_bar.
template <typename S>
ABA_HD V6<S> ball_r3_path(const Tape<S>& t, const V6<S>& abar, const V3<S>& qddb, V3<S>& s) {
  // a = [y - W a'_l; a'_l], qdd = y - a'_a - W a'_l
  s = abar.a + qddb;
  return v6<S>(-qddb, abar.l - mulT(t.W, s));
}
template <typename S>
ABA_HD void ball_r3_local(const Tape<S>& t, Bar<S>& b, BallBar<S>& bb, const V6<S>& apb, const V3<S>& s) {
  bb.y = bb.y + s;
  bb.W = bb.W + outer(s, t.ap.l, S(-1));
  // ap = X a_parent + c
  b.G = b.G + qvec(apb, t.ap - t.c);
  b.c = b.c + apb;
}
// reverse of pass 2 (ball), serial part: as r2_path for a 1-dof joint; u is
// the forward's tau - pA_a.  Returns tau_bar.  IAb follows the symmetric
// convention of IA's adjoints (its B block is half of the adjoint of B as
// one matrix that appears as B and B^T).
template <typename S>
ABA_HD V3<S> ball_r2_path(const LinkC<S>& L, const Tape<S>& t, BallBar<S>& bb, const V3<S>& u, bool has_parent,
                          const SySp<S>& IAbp, const V6<S>& pAbp, SySp<S>& N, V6<S>& pab, SySp<S>& IAb,
                          V6<S>& pAb) {
  V3<S> taub = zero3<S>();
  pAb = zero6<S>();
  M3<S> Bb;  // adjoint of B (all nine entries, B and B^T counted once each)
  Sy3<S> Cb = sy3<S>(S(0), S(0), S(0), S(0), S(0), S(0));
#pragma unroll
  for (int k = 0; k < 9; ++k) Bb.m[k] = S(0);
  if (has_parent) {
    pab = xform(t.E, L.rT, pAbp);
    N = congruence_X(t.E, L.rT, IAbp);
    // pa = [tau; pA_l + Ia_C c_l + B^T y]
    taub = pab.a;
    pAb.l = pab.l;
    const Sy3<S> IaCb = N.C + sym_outer(pab.l, t.c.l, S(0.5));
    Bb = outer(t.y, pab.l, S(1));
    bb.y = bb.y + mul(t.IA.B, pab.l);
    // Ia_C = C - B^T W
    Cb = IaCb;
    const M3<S> Ic = sy_to_m3(IaCb);
    const M3<S> WI = mul(t.W, Ic), BI = mul(t.IA.B, Ic);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      Bb.m[k] = Bb.m[k] - WI.m[k];
      bb.W.m[k] = bb.W.m[k] - BI.m[k];
    }
  }
  // W = A^-1 B, y = A^-1 u
  const M3<S> Aim = sy_to_m3(t.Ai);
  const M3<S> AiW = mul(Aim, bb.W);
#pragma unroll
  for (int k = 0; k < 9; ++k) Bb.m[k] = Bb.m[k] + AiW.m[k];
  const V3<S> ub = mul(t.Ai, bb.y);
  // A^-1 bar = W_bar B^T + y_bar u^T, symmetric part
  const M3<S> WBt = mul(bb.W, transpose(t.IA.B));
  const Sy3<S> Aib = sy3<S>(WBt.m[0] + bb.y.x * u.x, WBt.m[4] + bb.y.y * u.y, WBt.m[8] + bb.y.z * u.z,
                            S(0.5) * (WBt.m[1] + WBt.m[3] + bb.y.x * u.y + bb.y.y * u.x),
                            S(0.5) * (WBt.m[2] + WBt.m[6] + bb.y.x * u.z + bb.y.z * u.x),
                            S(0.5) * (WBt.m[5] + WBt.m[7] + bb.y.y * u.z + bb.y.z * u.y));
  // u = tau - pA_a
  taub = taub + ub;
  pAb.a = -ub;
  // A^-1 = inv(A): A_bar = -A^-1 sym(A^-1 bar) A^-1
  const Sy3<S> Ab = cong(Aim, Aib);
  IAb.A = sy3<S>(-Ab.xx, -Ab.yy, -Ab.zz, -Ab.xy, -Ab.xz, -Ab.yz);
#pragma unroll
  for (int k = 0; k < 9; ++k) IAb.B.m[k] = S(0.5) * Bb.m[k];
  IAb.C = Cb;
  return taub;
}
// reverse of pass 2 (ball with a parent), local part: the pairings of the
// shift statements and the Ia c term's share of c_bar
template <typename S>
ABA_HD void ball_r2_local(const Tape<S>& t, Bar<S>& b, const SySp<S>& N, const V6<S>& pab) {
  SySp<S> Ia = zero_sysp<S>();
  Ia.C = ball_IaC(t);
  b.G = b.G + qvec(t.pa, pab) - S(2) * crmS_vec(Ia, N);
  b.c = b.c + mul(Ia, pab);
}
// reverse of pass 1 (ball): the link's own share of its velocity adjoint
template <typename S>
ABA_HD V6<S> ball_r1_own(const LinkC<S>& L, const V6<S>& v, const Bar<S>& b, const V6<S>& pAb, const V3<S>& w) {
  // c = v x vJ = -crm(vJ) v, vJ = [w; 0]
  return r1_own(L, v, b, pAb, S(0), false) - crmT(v6<S>(w, zero3<S>()), b.c);
}
// local part: returns the joint-rate adjoint; v_bar is complete
template <typename S>
ABA_HD V3<S> ball_r1_local(const Tape<S>& t, Bar<S>& b, const V6<S>& vbar, const V3<S>& w) {
  const V6<S> vJ = v6<S>(w, zero3<S>());
  const V6<S> vJb = crmT(t.v, b.c) + vbar;
  // v = X v_parent + vJ
  b.G = b.G + qvec(vbar, t.v - vJ);
  return vJb.a;
}
// The quaternion's adjoint from the rotation pairings, along the unit
// sphere.  A change dq = q (x) (d/2, 0) turns E_J = R(q)^T into
// (1 - [d]x) E_J, i.e. X into X - crm([d; 0]) X, so dL = G_a . d with
// d/2 = vec(q^-1 (x) dq), hence q_bar = 2 / |q|^2 q (x) (G_a, 0), which is
// orthogonal to q.  The radial part is left out on purpose: it depends only
// on how the step is continued off the unit sphere (where R(q) is scaled,
// and the free root's Galilean shift no longer leaves the dynamics
// unchanged), the integrator's normalisation removes it from every earlier
// step's adjoint, and the integrator's own share is tangent as well.
template <typename S>
ABA_HD Q4<S> ball_quat_bar(const Q4<S>& q, const V3<S>& Ga) {
  const S k = S(2) / (q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
  const V3<S> u = v3<S>(q.x, q.y, q.z);
  const V3<S> rv = axpy(cross(u, Ga), q.w, Ga);
  Q4<S> o;
  o.x = k * rv.x;
  o.y = k * rv.y;
  o.z = k * rv.z;
  o.w = -k * dot(u, Ga);
  return o;
}
// Placement adjoint of a ball link (no axis): X_T -> exp(-crm(xi)) X_T
// moves X by -crm(Xh_J xi) X with Xh_J = X_J / |q|^2 the joint's rotation,
// so xi_bar += Xh_J^T G = [R G_a; R G_l] / |q|^2.
template <typename S>
ABA_HD void ball_frame_bar_add(ParamBar<S>& g, const Q4<S>& q, const Bar<S>& b) {
  const S k = S(1) / (q.x * q.x + q.y * q.y + q.z * q.z + q.w * q.w);
  g.xi = g.xi + v6<S>(k * quat_rotate(q, b.G.a), k * quat_rotate(q, b.G.l));
}

// adjoint of quat_step: from the adjoint q1b of the new quaternion, returns
// the quaternion's share of the adjoint of quat and adds w1's to w1b.
template <typename S>
ABA_HD Q4<S> quat_step_adj(const Q4<S>& quat, const V3<S>& w1, S dt, const Q4<S>& q1b, V3<S>& w1b) {
  const V3<S> u = v3<S>(quat.x, quat.y, quat.z);
  const V3<S> ov = axpy(cross(u, w1), quat.w, w1);
  const S ow = -dot(u, w1);
  const S h = S(0.5) * dt;
  Q4<S> r;
  r.x = quat.x + h * ov.x;
  r.y = quat.y + h * ov.y;
  r.z = quat.z + h * ov.z;
  r.w = quat.w + h * ow;
  const S inv = S(1) / sqrt(r.x * r.x + r.y * r.y + r.z * r.z + r.w * r.w);
  const Q4<S> q1 = {r.x * inv, r.y * inv, r.z * inv, r.w * inv};
  // quat1 = r / |r|
  const S d = q1.x * q1b.x + q1.y * q1b.y + q1.z * q1b.z + q1.w * q1b.w;
  const V3<S> rbv = v3<S>((q1b.x - q1.x * d) * inv, (q1b.y - q1.y * d) * inv, (q1b.z - q1.z * d) * inv);
  const S rbw = (q1b.w - q1.w * d) * inv;
  // r = quat + h * quat (x) (w1, 0):  o_v = qw w1 + u x w1, o_w = -u . w1
  const V3<S> qvb = rbv + h * (cross(w1, rbv) - rbw * w1);
  const S qwb = rbw + h * dot(w1, rbv);
  w1b = w1b + h * (quat.w * rbv - cross(u, rbv) - rbw * u);
  Q4<S> o;
  o.x = qvb.x;
  o.y = qvb.y;
  o.z = qvb.z;
  o.w = qwb;
  return o;
}

// adjoint of integrate_root.  Inputs: state at the start of the step (p,
// quat, v), the base acceleration, and the adjoints of the new state (pb,
// quatb, vb: overwritten with the adjoints of the old state's integrator
// share).  Returns the base-acceleration seed dt * v1_bar.
template <typename S>
ABA_HD V6<S> integrate_root_adj(const Q4<S>& quat, const V6<S>& v, const V6<S>& abase, S dt, V3<S>& pb,
                                Q4<S>& quatb, V6<S>& vb) {
  (void)pb;  // p1 = p + ...: the position adjoint passes through unchanged
  const V6<S> v1 = v + dt * abase;
  V6<S> v1b = vb;
  const Q4<S> qs = quat_step_adj(quat, v1.a, dt, quatb, v1b.a);
  // p1 = p + dt R(quat) v1_lin
  const Q4<S> gq = quat_rot_grad(quat, dt * pb, v1.l);
  quatb.x = qs.x + gq.x;
  quatb.y = qs.y + gq.y;
  quatb.z = qs.z + gq.z;
  quatb.w = qs.w + gq.w;
  v1b.l = v1b.l + quat_rotate_T(quat, dt * pb);
  // v1 = v + dt abase
  vb = v1b;
  return dt * v1b;
}

}  // namespace aba
