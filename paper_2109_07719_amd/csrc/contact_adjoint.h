// Adjoint of one time step with contact (Sec. 4.1 "Collision resolution";
// App. C; Sec. 3, Eq. adj_back and Sec. 4.1, Eq. adj_r for the recursion
// through time): the statements of contact_step run backwards, each through
// its own adjoint.  Host and device code, one system per call, scalar S.
//
// The step, as contact_step computes it, in the order the adjoint reverses:
//   qdd = FD(q, qd, u)                                  ABA (passes 1-3)
//   qd_minus = qd + dt qdd
//   J(q), phi(q)                                        detection, contact rows
//   MJ = M(q)^-1 J^T                                    unit-impulse responses
//   A = J MJ,  b = J qd_minus + (beta/dt) phi_n
//   lambda_n = PGS(A_nn, b_n, [0, inf))                 first solve
//   lambda = PGS(A, b, normal [0, inf), tangent +-mu lambda_n)  second solve
//   qd1 = qd_minus + MJ lambda
//   q1 = integrate(q, qd1)
// Reverse: the integrator; the impulse update; the second and the first
// Gauss-Seidel solve swept backwards from their stored sweep vectors (the
// row adjoint of the batched solver); A and b; MJ = M^-1 J^T through
// W = M^-1 MJ_bar (J_bar += W^T, and the q-derivative of the inertia
// matrix as the q-adjoint of an inverse-dynamics pass with accelerations
// MJ and seed W); the contact rows and gaps through the world poses of the
// links; then the smooth step by tau_bar = M^-1 qdd_bar and the q- and
// qd-adjoints of the inverse dynamics at the step's accelerations (the
// derivative of M qdd + C(q, qd) = u, solved for qdd, at fixed qdd).
// Clamp, detection and row-dropping decisions are taken as in the forward
// step, so the result is the gradient of the step map as computed.
//
// Joint-coordinate derivatives: X = X_J(q) X_T with X_J = exp(-q crm(S)),
// so dX/dq = -crm(S) X for a revolute (S = [a; 0]) and a prismatic
// (S = [0; a]) joint alike; a statement y = X m (adjoint x = y_bar) or
// y = X^T f (x = f, y = X y_bar) contributes S . qvec(x, y) to q_bar, with
// qvec(x, y) = [x_ang x y_ang + x_lin x y_lin; x_lin x y_ang].
#pragma once

#include "contact_step.h"

namespace aba_contact {

// ---- small helpers on raw arrays ------------------------------------------

template <typename S>
ABA_HD S dot3(const S* a, const S* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
// crm(x) y = [x_a x y_a; x_l x y_a + x_a x y_l]
template <typename S>
ABA_HD void crm6(const S* x, const S* y, S* o) {
  S t1[3], t2[3], t3[3];
  cross3(x, y, t1);
  cross3(x + 3, y, t2);
  cross3(x, y + 3, t3);
  for (int k = 0; k < 3; ++k) {
    o[k] = t1[k];
    o[3 + k] = t2[k] + t3[k];
  }
}
// crm(x)^T y = [y_a x x_a + y_l x x_l; y_l x x_a]
template <typename S>
ABA_HD void crmT6(const S* x, const S* y, S* o) {
  S t1[3], t2[3], t3[3];
  cross3(y, x, t1);
  cross3(y + 3, x + 3, t2);
  cross3(y + 3, x, t3);
  for (int k = 0; k < 3; ++k) {
    o[k] = t1[k] + t2[k];
    o[3 + k] = t3[k];
  }
}
// x ^* h = -crm(x)^T h = [x_a x h_a + x_l x h_l; x_a x h_l]
template <typename S>
ABA_HD void crf6(const S* x, const S* h, S* o) {
  S t1[3], t2[3], t3[3];
  cross3(x, h, t1);
  cross3(x + 3, h + 3, t2);
  cross3(x, h + 3, t3);
  for (int k = 0; k < 3; ++k) {
    o[k] = t1[k] + t2[k];
    o[3 + k] = t3[k];
  }
}
// S . qvec(x, y) for the link's motion subspace (revolute [a; 0], prismatic [0; a])
template <typename S>
ABA_HD S spair(bool prism, const S* a, const S* x, const S* y) {
  S t1[3], t2[3];
  if (prism) {
    cross3(x + 3, y, t1);
    return dot3(a, t1);
  }
  cross3(x, y, t1);
  cross3(x + 3, y + 3, t2);
  return a[0] * (t1[0] + t2[0]) + a[1] * (t1[1] + t2[1]) + a[2] * (t1[2] + t2[2]);
}
// the link's motion subspace column S = [a; 0] or [0; a]
template <typename S>
ABA_HD void scol(bool prism, const S* a, S* s6) {
  for (int k = 0; k < 3; ++k) {
    s6[k] = prism ? S(0) : a[k];
    s6[3 + k] = prism ? a[k] : S(0);
  }
}
// gradient of x^T R(quat) y with respect to the raw quaternion (x, y, z, w),
// R = (w^2 - u.u) I + 2 u u^T + 2 w [u]x
template <typename S>
ABA_HD void quat_rot_grad4(const S* qt, const S* x, const S* y, S* g) {
  const S* u = qt;
  const S w = qt[3];
  const S xy = dot3(x, y), uy = dot3(u, y), xu = dot3(x, u);
  S yx[3], uy_[3];
  cross3(y, x, yx);
  cross3(u, y, uy_);
  for (int k = 0; k < 3; ++k) g[k] = S(-2) * xy * u[k] + S(2) * uy * x[k] + S(2) * xu * y[k] + S(2) * w * yx[k];
  g[3] = S(2) * w * xy + S(2) * dot3(x, uy_);
}

// The spatial inertia of link i about its origin applied to a motion vector
template <typename S, typename R>
ABA_HD void inertia_apply(const Par<R>& P, int i, const S* v, S* o) {
  const int pb = kParLink * i;
  const S m = S(P(pb + 15));
  const S cm[3] = {S(P(pb + 16)), S(P(pb + 17)), S(P(pb + 18))};
  const S Ic[9] = {S(P(pb + 19)), S(P(pb + 22)), S(P(pb + 23)), S(P(pb + 22)), S(P(pb + 20)),
                   S(P(pb + 24)), S(P(pb + 23)), S(P(pb + 24)), S(P(pb + 21))};
  // I = [Ic + m [c]x [c]x^T, m [c]x; m [c]x^T, m 1]
  S cxv[3], t[3];
  cross3(cm, v + 3, cxv);          // c x v_lin
  cross3(v, cm, t);                // w x c
  S wc[3];
  for (int k = 0; k < 3; ++k) wc[k] = v[3 + k] + t[k];  // v_lin + w x c (velocity of the com)
  S cwc[3];
  cross3(cm, wc, cwc);
  for (int a = 0; a < 3; ++a) {
    o[a] = Ic[3 * a] * v[0] + Ic[3 * a + 1] * v[1] + Ic[3 * a + 2] * v[2] + m * cwc[a];
    o[3 + a] = m * wc[a];
  }
}

// The same from the link's inertial parameters as stored in an Art copy
// (mass, centre of mass, inertia about it: the values inertia_apply reads).
template <typename S>
ABA_HD void inertia_apply_ib(const S* ib, const S* v, S* o) {
  const S m = ib[0];
  const S cm[3] = {ib[1], ib[2], ib[3]};
  const S Ic[9] = {ib[4], ib[7], ib[8], ib[7], ib[5], ib[9], ib[8], ib[9], ib[6]};
  S cxv[3], t[3];
  cross3(cm, v + 3, cxv);
  cross3(v, cm, t);
  S wc[3];
  for (int k = 0; k < 3; ++k) wc[k] = v[3 + k] + t[k];
  S cwc[3];
  cross3(cm, wc, cwc);
  for (int a = 0; a < 3; ++a) {
    o[a] = Ic[3 * a] * v[0] + Ic[3 * a + 1] * v[1] + Ic[3 * a + 2] * v[2] + m * cwc[a];
    o[3 + a] = m * wc[a];
  }
}

// M^-1 rhs at the step's configuration (zero velocity, no gravity), from
// the articulated inertias of the step's pass 2 kept in w (U, 1/D, the
// free root's LDL^T; an Art copy, whose scratch pA, a, u it uses).  rhs and
// out: [nv].
template <typename S>
ABA_HD void minv_apply(const CTopo& tp, Art<S>& w, const S* rhs, S* out) {
  const int n = tp.n;
  S (&pA)[kNL][6] = w.pA;
  S (&a)[kNL][6] = w.a;
  S (&uu)[kNL] = w.u;
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < 6; ++k) pA[i][k] = S(0);
  for (int i = n - 1; i >= 0; --i) {
    if (tp.jtype[i] == SIM_JOINT_FREE) continue;
    const bool pr = tp.jtype[i] == SIM_JOINT_PRISMATIC;
    const int off = pr ? 3 : 0, p = tp.parent[i];
    uu[i] = rhs[tp.vi[i]] - (pA[i][off] * w.ax[i][0] + pA[i][off + 1] * w.ax[i][1] + pA[i][off + 2] * w.ax[i][2]);
    if (p >= 0) {
      const S y = w.Dinv[i] * uu[i];
      S pa[6], f[6];
      for (int k = 0; k < 6; ++k) pa[k] = pA[i][k] + w.U[i][k] * y;
      xt_force(w.E[i], w.r[i], pa, f);
      for (int k = 0; k < 6; ++k) pA[p][k] = pA[p][k] + f[k];
    }
  }
  for (int i = 0; i < n; ++i) {
    if (tp.jtype[i] == SIM_JOINT_FREE) {
      S r6[6];
      for (int k = 0; k < 6; ++k) r6[k] = rhs[tp.vi[i] + k] - pA[i][k];
      ldl6_solve(w.L0, w.D0, r6, a[i]);
      for (int k = 0; k < 6; ++k) out[tp.vi[i] + k] = a[i][k];
    } else {
      const int p = tp.parent[i], off = tp.jtype[i] == SIM_JOINT_PRISMATIC ? 3 : 0;
      S ap[6];
      if (p < 0) {
        for (int k = 0; k < 6; ++k) ap[k] = S(0);
      } else {
        x_motion(w.E[i], w.r[i], a[p], ap);
      }
      S Uap = S(0);
      for (int k = 0; k < 6; ++k) Uap = Uap + w.U[i][k] * ap[k];
      const S qdd = w.Dinv[i] * (uu[i] - Uap);
      for (int k = 0; k < 6; ++k) a[i][k] = ap[k];
      for (int k = 0; k < 3; ++k) a[i][off + k] = a[i][off + k] + w.ax[i][k] * qdd;
      out[tp.vi[i]] = qdd;
    }
  }
}

// Adds the q- and qd-adjoints of <wv, ID(q, qd, acc)> (inverse dynamics by
// the recursive Newton-Euler statements, gravity as a fictitious base
// acceleration; a free root's acc is its true body-frame acceleration and
// its row of ID the wrench on it) to gq [nq] and gqd [nv] (gqd nullable when
// qd is: then velocities are zero).  with_gravity selects the gravity term.
// Link transforms, axes and the free root's rotation come from the step's
// pass 1 in w.
template <typename S, typename R>
ABA_HD void id_vjp(const CTopo& tp, const Par<R>& P, const Work<S>& w, const S* q, const S* qd, const S* acc,
                   bool with_gravity, const S* wv, S* gq, S* gqd) {
  const int n = tp.n;
  S V[kNL][6], A[kNL][6], F[kNL][6], Ap[kNL][6], Vp[kNL][6];
  const S g[3] = {S(tp.g[0]), S(tp.g[1]), S(tp.g[2])};
  // forward: velocities, accelerations, link forces
  for (int i = 0; i < n; ++i) {
    const int p = tp.parent[i];
    if (tp.jtype[i] == SIM_JOINT_FREE) {
      for (int k = 0; k < 6; ++k) {
        V[i][k] = qd ? qd[tp.vi[i] + k] : S(0);
        A[i][k] = acc[tp.vi[i] + k];
        Vp[i][k] = Ap[i][k] = S(0);
      }
      if (with_gravity)  // a' = a - [0; E g]
        for (int a = 0; a < 3; ++a)
          A[i][3 + a] = A[i][3 + a] - (w.E[i][3 * a] * g[0] + w.E[i][3 * a + 1] * g[1] + w.E[i][3 * a + 2] * g[2]);
    } else {
      const bool pr = tp.jtype[i] == SIM_JOINT_PRISMATIC;
      S s6[6], vJ[6], c[6];
      scol(pr, w.ax[i], s6);
      const S qdj = qd ? qd[tp.vi[i]] : S(0);
      for (int k = 0; k < 6; ++k) vJ[k] = s6[k] * qdj;
      S vpar[6], apar[6];
      if (p < 0) {
        for (int k = 0; k < 6; ++k) vpar[k] = S(0);
        for (int k = 0; k < 3; ++k) {
          apar[k] = S(0);
          apar[3 + k] = with_gravity ? -g[k] : S(0);
        }
      } else {
        for (int k = 0; k < 6; ++k) {
          vpar[k] = V[p][k];
          apar[k] = A[p][k];
        }
      }
      x_motion(w.E[i], w.r[i], vpar, Vp[i]);
      x_motion(w.E[i], w.r[i], apar, Ap[i]);
      for (int k = 0; k < 6; ++k) V[i][k] = Vp[i][k] + vJ[k];
      crm6(V[i], vJ, c);
      for (int k = 0; k < 6; ++k) A[i][k] = Ap[i][k] + s6[k] * acc[tp.vi[i]] + c[k];
    }
    S h[6], Ia[6], b[6];
    inertia_apply(P, i, V[i], h);
    inertia_apply(P, i, A[i], Ia);
    crf6(V[i], h, b);
    for (int k = 0; k < 6; ++k) F[i][k] = Ia[k] + b[k];
  }
  for (int i = n - 1; i >= 0; --i) {
    const int p = tp.parent[i];
    if (p >= 0) {
      S f[6];
      xt_force(w.E[i], w.r[i], F[i], f);
      for (int k = 0; k < 6; ++k) F[p][k] = F[p][k] + f[k];
    }
  }
  // reverse: force adjoints root -> leaves (F[p] += X^T F[i])
  S Fb[kNL][6], Ab[kNL][6], Vb[kNL][6];
  for (int i = 0; i < n; ++i) {
    const int p = tp.parent[i];
    if (tp.jtype[i] == SIM_JOINT_FREE) {
      for (int k = 0; k < 6; ++k) Fb[i][k] = wv[tp.vi[i] + k];
    } else {
      const bool pr = tp.jtype[i] == SIM_JOINT_PRISMATIC;
      S s6[6];
      scol(pr, w.ax[i], s6);
      for (int k = 0; k < 6; ++k) Fb[i][k] = s6[k] * wv[tp.vi[i]];
      if (p >= 0) {
        S y[6];
        x_motion(w.E[i], w.r[i], Fb[p], y);
        gq[tp.qi[i]] = gq[tp.qi[i]] + spair(pr, w.ax[i], F[i], y);
        for (int k = 0; k < 6; ++k) Fb[i][k] = Fb[i][k] + y[k];
      }
    }
  }
  // local: F = I A + V x* (I V)
  for (int i = 0; i < n; ++i) {
    S h[6], hb[6], t[6], Ih[6];
    inertia_apply(P, i, Fb[i], Ab[i]);
    inertia_apply(P, i, V[i], h);
    crm6(V[i], Fb[i], hb);
    for (int k = 0; k < 6; ++k) hb[k] = -hb[k];
    crmT6(Fb[i], h, t);
    inertia_apply(P, i, hb, Ih);
    for (int k = 0; k < 6; ++k) Vb[i][k] = t[k] + Ih[k];
  }
  // reverse of the acceleration and velocity recursions, leaves -> root
  for (int i = n - 1; i >= 0; --i) {
    const int p = tp.parent[i];
    if (tp.jtype[i] == SIM_JOINT_FREE) {
      if (gqd)
        for (int k = 0; k < 6; ++k) gqd[tp.vi[i] + k] = gqd[tp.vi[i] + k] + Vb[i][k];
      if (with_gravity) {
        // a' = a - [0; R^T g]: <Ab_lin, -R^T g> = -g^T R Ab_lin
        S gr[4];
        quat_rot_grad4(q + tp.qi[i] + 3, g, Ab[i] + 3, gr);
        for (int k = 0; k < 4; ++k) gq[tp.qi[i] + 3 + k] = gq[tp.qi[i] + 3 + k] - gr[k];
      }
      continue;
    }
    const bool pr = tp.jtype[i] == SIM_JOINT_PRISMATIC;
    S s6[6], vJ[6];
    scol(pr, w.ax[i], s6);
    const S qdj = qd ? qd[tp.vi[i]] : S(0);
    for (int k = 0; k < 6; ++k) vJ[k] = s6[k] * qdj;
    // A = X A_p + S acc + V x vJ
    gq[tp.qi[i]] = gq[tp.qi[i]] + spair(pr, w.ax[i], Ab[i], Ap[i]);
    if (p >= 0) {
      S f[6];
      xt_force(w.E[i], w.r[i], Ab[i], f);
      for (int k = 0; k < 6; ++k) Ab[p][k] = Ab[p][k] + f[k];
    }
    {
      // c = V x vJ = -crm(vJ) V: V_bar -= crm(vJ)^T c_bar; vJ_bar = crm(V)^T c_bar
      S t[6], tj[6];
      crmT6(vJ, Ab[i], t);
      for (int k = 0; k < 6; ++k) Vb[i][k] = Vb[i][k] - t[k];
      crmT6(V[i], Ab[i], tj);
      if (gqd) {
        S sv = S(0);
        for (int k = 0; k < 6; ++k) sv = sv + s6[k] * (tj[k] + Vb[i][k]);
        gqd[tp.vi[i]] = gqd[tp.vi[i]] + sv;
      }
    }
    // V = X V_p + S qd
    gq[tp.qi[i]] = gq[tp.qi[i]] + spair(pr, w.ax[i], Vb[i], Vp[i]);
    if (p >= 0) {
      S f[6];
      xt_force(w.E[i], w.r[i], Vb[i], f);
      for (int k = 0; k < 6; ++k) Vb[p][k] = Vb[p][k] + f[k];
    }
  }
}

// The q-adjoint of <wv, M(q) acc>: id_vjp at zero velocity without gravity,
// where every velocity-product and gravity term of the recursive
// Newton-Euler statements vanishes, written without them (A = X A_parent +
// S acc, F = I A, F_parent += X^T F, and the reverse of those).  The free
// root's row is body-frame, so M does not depend on its pose.
template <typename S>
ABA_HD void id_vjp_static(const CTopo& tp, Art<S>& w, const S* acc, const S* wv, S* gq) {
  const int n = tp.n;
  // the copy's scratch (free once minv_apply has returned)
  S (&A)[kNL][6] = w.pA;
  S (&F)[kNL][6] = w.a;
  S (&Ap)[kNL][6] = w.s3;
  for (int i = 0; i < n; ++i) {
    const int p = tp.parent[i];
    if (tp.jtype[i] == SIM_JOINT_FREE) {
      for (int k = 0; k < 6; ++k) {
        A[i][k] = acc[tp.vi[i] + k];
        Ap[i][k] = S(0);
      }
    } else {
      S s6[6];
      scol(tp.jtype[i] == SIM_JOINT_PRISMATIC, w.ax[i], s6);
      if (p < 0) {
        for (int k = 0; k < 6; ++k) Ap[i][k] = S(0);
      } else {
        x_motion(w.E[i], w.r[i], A[p], Ap[i]);
      }
      for (int k = 0; k < 6; ++k) A[i][k] = Ap[i][k] + s6[k] * acc[tp.vi[i]];
    }
    inertia_apply_ib(w.Ib[i], A[i], F[i]);
  }
  for (int i = n - 1; i >= 0; --i) {
    const int p = tp.parent[i];
    if (p >= 0) {
      S f[6];
      xt_force(w.E[i], w.r[i], F[i], f);
      for (int k = 0; k < 6; ++k) F[p][k] = F[p][k] + f[k];
    }
  }
  // reverse: force adjoints root -> leaves (F[p] += X^T F[i]); A is reused
  // for them
  S (&Fb)[kNL][6] = A;
  for (int i = 0; i < n; ++i) {
    const int p = tp.parent[i];
    if (tp.jtype[i] == SIM_JOINT_FREE) {
      for (int k = 0; k < 6; ++k) Fb[i][k] = wv[tp.vi[i] + k];
    } else {
      const bool pr = tp.jtype[i] == SIM_JOINT_PRISMATIC;
      S s6[6];
      scol(pr, w.ax[i], s6);
      for (int k = 0; k < 6; ++k) Fb[i][k] = s6[k] * wv[tp.vi[i]];
      if (p >= 0) {
        S y[6];
        x_motion(w.E[i], w.r[i], Fb[p], y);
        gq[tp.qi[i]] = gq[tp.qi[i]] + spair(pr, w.ax[i], F[i], y);
        for (int k = 0; k < 6; ++k) Fb[i][k] = Fb[i][k] + y[k];
      }
    }
  }
  // F = I A: A_bar = I F_bar (in place; F is no longer needed)
  S (&Ab)[kNL][6] = F;
  for (int i = 0; i < n; ++i) inertia_apply_ib(w.Ib[i], Fb[i], Ab[i]);
  // reverse of A = X A_parent + S acc, leaves -> root
  for (int i = n - 1; i >= 0; --i) {
    if (tp.jtype[i] == SIM_JOINT_FREE) continue;
    const int p = tp.parent[i];
    const bool pr = tp.jtype[i] == SIM_JOINT_PRISMATIC;
    gq[tp.qi[i]] = gq[tp.qi[i]] + spair(pr, w.ax[i], Ab[i], Ap[i]);
    if (p >= 0) {
      S f[6];
      xt_force(w.E[i], w.r[i], Ab[i], f);
      for (int k = 0; k < 6; ++k) Ab[p][k] = Ab[p][k] + f[k];
    }
  }
}

// One reversed projected Gauss-Seidel solve on the rows idx[0..m) of A
// (leading dimension r): from xb (adjoint of the result, [m], consumed) and
// the stored sweep vectors (stride ld), adds the adjoints of A, b (full
// index space) and of the bounds ([m]).  Row by row, last sweep first: the
// clamp sends x_bar_i to the active bound (a value exactly on a bound counts
// as inside) or to y_bar_i; then b_bar_i, A_bar_i. and x_bar_j (j != i)
// follow from y_i = -(b_i + sum_{j != i} A_ij x_j) / A_ii, and x_bar_i is
// reset (x_i was overwritten).
template <typename S>
ABA_HD void pgs_reverse(int m, const int* idx, int r, const S* A, const S* b, const S* lo, const S* hi, int niter,
                        const S* sweeps, int ld, S* xb, S* Ab, S* bb, S* lob, S* hib) {
  for (int it = niter - 1; it >= 0; --it) {
    const S* xs = sweeps + it * ld;
    const S* xe = sweeps + (it + 1) * ld;
    for (int i = m - 1; i >= 0; --i) {
      const int ri = idx[i];
      S d = S(0);
      for (int j = 0; j < m; ++j)
        if (j != i) d = fmadd(A[ri * r + idx[j]], j < i ? xe[j] : xs[j], d);
      const S y = -(b[ri] + d) / A[ri * r + ri];
      S yb = S(0);
      if (val(y) < val(lo[i])) lob[i] = lob[i] + xb[i];
      else if (val(y) > val(hi[i])) hib[i] = hib[i] + xb[i];
      else yb = xb[i];
      xb[i] = S(0);
      const S db = -yb / A[ri * r + ri];
      bb[ri] = bb[ri] + db;
      Ab[ri * r + ri] = fmadd(db, y, Ab[ri * r + ri]);
      for (int j = 0; j < m; ++j)
        if (j != i) {
          Ab[ri * r + idx[j]] = fmadd(db, j < i ? xe[j] : xs[j], Ab[ri * r + idx[j]]);
          xb[j] = fmadd(db, A[ri * r + idx[j]], xb[j]);
        }
    }
  }
}

// pgs_reverse on a staged copy (PgsStage): every statement runs in the
// order of pgs_reverse, so the result is bitwise the same.  A sweep's row
// values y_i depend only on the stored sweep vectors, not on the adjoints,
// so they are computed for all rows first (independent chains), then the
// adjoint rows run last to first with x_bar held in registers; rows and
// columns are unrolled over kNR and predicated on m.
template <typename S>
ABA_HD void pgs_reverse_staged(int m, const int* idx, int r, const S* A, const S* b, const S* lo, const S* hi,
                               int niter, const S* sweeps, int ld, S* xb, S* Ab, S* bb, S* lob, S* hib,
                               const PgsStage<S>& g) {
  // as in pgs_staged: rows at stride kNR, zero beyond m
  // (the kept rows' indices, 0 beyond m, address valid entries of A and
  // A_bar, so the copies read them with no condition and their loads issue
  // together)
  int ix[kNR];
#pragma unroll
  for (int i = 0; i < kNR; ++i) ix[i] = i < m ? idx[i] : 0;
#pragma unroll
  for (int i = 0; i < kNR; ++i) {
#pragma unroll
    for (int j = 0; j < kNR; ++j) {
      const bool in = i < m && j < m;
      const S aij = A[ix[i] * r + ix[j]], abij = Ab[ix[i] * r + ix[j]];
      g[kStA + i * kNR + j] = in ? aij : S(0);
      g[kStAb + i * kNR + j] = in ? abij : S(0);
    }
    g[kStB + i] = S(0);
    g[kStX + i] = S(0);
    g[kStXe + i] = S(0);
  }
  for (int i = 0; i < m; ++i) {
    const int ri = idx[i];
    g[kStB + i] = b[ri];
    g[kStBb + i] = bb[ri];
    g[kStLo + i] = lo[i];
    g[kStHi + i] = hi[i];
    g[kStLob + i] = lob[i];
    g[kStHib + i] = hib[i];
  }
  S xbr[kNR];
#pragma unroll
  for (int i = 0; i < kNR; ++i) xbr[i] = i < m ? xb[i] : S(0);
  // (a sweep row is read with the index clamped below m, so its loads carry
  // no condition and issue together; the staged entries past m stay zero)
#pragma unroll
  for (int j = 0; j < kNR; ++j) {
    const S v = sweeps[niter * ld + (j < m ? j : 0)];
    g[kStX + j] = j < m ? v : S(0);
  }
  for (int it = niter - 1; it >= 0; --it) {
    // x at the start (xs) and at the end (xe) of sweep it; xe is the
    // previous sweep's xs, already staged
#pragma unroll
    for (int j = 0; j < kNR; ++j) {
      const S v = sweeps[it * ld + (j < m ? j : 0)];
      g[kStXe + j] = g[kStX + j];
      g[kStX + j] = j < m ? v : S(0);
    }
    // (every row with no condition, so that all their loads issue
    // together: beyond m the staged block and vectors are zero, the terms
    // add nothing, and such a row's value, divided by one, is not used)
    S y[kNR];
#pragma unroll
    for (int i = 0; i < kNR; ++i) {
      S d = S(0);
#pragma unroll
      for (int j = 0; j < kNR; ++j)
        if (j != i) d = fmadd_pad(g[kStA + i * kNR + j], j < i ? g[kStXe + j] : g[kStX + j], d, i < m && j < m);
      const S aii = g[kStA + i * kNR + i];
      y[i] = -(g[kStB + i] + d) / (i < m ? aii : S(1));
    }
#pragma unroll
    for (int i = kNR - 1; i >= 0; --i) {
      if (i >= m) continue;
      S yb = S(0);
      if (val(y[i]) < val(g[kStLo + i])) g[kStLob + i] = g[kStLob + i] + xbr[i];
      else if (val(y[i]) > val(g[kStHi + i])) g[kStHib + i] = g[kStHib + i] + xbr[i];
      else yb = xbr[i];
      xbr[i] = S(0);
      const S db = -yb / g[kStA + i * kNR + i];
      g[kStBb + i] = g[kStBb + i] + db;
      g[kStAb + i * kNR + i] = fmadd(db, y[i], g[kStAb + i * kNR + i]);
#pragma unroll
      for (int j = 0; j < kNR; ++j)
        if (j != i) {  // beyond m: zero entries, nothing changes
          g[kStAb + i * kNR + j] = fmadd_pad(db, j < i ? g[kStXe + j] : g[kStX + j], g[kStAb + i * kNR + j], j < m);
          xbr[j] = fmadd_pad(db, g[kStA + i * kNR + j], xbr[j], j < m);
        }
    }
  }
  for (int i = 0; i < m; ++i) {
    const int ri = idx[i];
    for (int j = 0; j < m; ++j) Ab[ri * r + idx[j]] = g[kStAb + i * kNR + j];
    bb[ri] = g[kStBb + i];
    lob[i] = g[kStLob + i];
    hib[i] = g[kStHib + i];
  }
#pragma unroll
  for (int i = 0; i < kNR; ++i)
    if (i < m) xb[i] = xbr[i];
}

// Adjoint state of one reverse step with contact.
template <typename S>
struct Adj {
  S Jb[kNR][kNV], MJb[kNV][kNR], Ab[kNR * kNR], bb[kNR];
  S Ewb[kNL][9], owb[kNL][3];
};

// One reverse step: recomputes the step from (q, qd) under u (recording),
// then turns xbar = (q1_bar, qd1_bar) [nq + nv] into the adjoint of (q, qd)
// in place, writes ubar [nu] and adds the friction coefficient's adjoint to
// mub.
template <typename S, typename R>
ABA_HD void contact_step_vjp(const CTopo& tp, const Par<R>& P, const S* q, const S* qd, const S* u, R dt_, S mu,
                             S* xbar, S* ubar, S& mub, Work<S>& w, Rec<S>& rc, Adj<S>& ad, Art<S>& art,
                             PgsStage<S> stage = {nullptr, 0}) {
  const int n = tp.n, nq = tp.nq, nv = tp.nv;
  S q1[kNQ], qd1[kNV];
  contact_step(tp, P, q, qd, u, dt_, mu, q1, qd1, w, &rc, stage, &art);
  const S dt = S(dt_);
  S qb[kNQ], qdb[kNV], qd1b[kNV], qdmb[kNV];
#pragma unroll
  for (int k = 0; k < kNQ; ++k) qb[k] = S(0);
  for (int k = 0; k < nv; ++k) {
    qdb[k] = S(0);
    qd1b[k] = xbar[nq + k];
  }
  // ---- integrator: q1 from q and qd1
  for (int i = 0; i < n; ++i) {
    if (tp.jtype[i] == SIM_JOINT_FREE) {
      const int qi = tp.qi[i], vi = tp.vi[i];
      const S* qt = q + qi + 3;
      const S* v1 = qd1 + vi;
      const S* p1b = xbar + qi;
      const S* qt1b = xbar + qi + 3;
      S Rm[9];
      quat_R(qt, Rm);
      // p1 = p + dt R v1_lin
      for (int a = 0; a < 3; ++a) qb[qi + a] = qb[qi + a] + p1b[a];
      for (int b = 0; b < 3; ++b)
        qd1b[vi + 3 + b] = qd1b[vi + 3 + b] + dt * (Rm[b] * p1b[0] + Rm[3 + b] * p1b[1] + Rm[6 + b] * p1b[2]);
      S dtp[3] = {dt * p1b[0], dt * p1b[1], dt * p1b[2]}, gr[4];
      quat_rot_grad4(qt, dtp, v1 + 3, gr);
      for (int k = 0; k < 4; ++k) qb[qi + 3 + k] = qb[qi + 3 + k] + gr[k];
      // quat1 = rr / |rr|, rr = quat + h quat (x) (w1, 0)
      const S h = S(0.5) * dt;
      S dq[4], cr[3], rr[4];
      cross3(qt, v1, cr);
      for (int k = 0; k < 3; ++k) dq[k] = qt[3] * v1[k] + cr[k];
      dq[3] = -dot3(qt, v1);
      for (int k = 0; k < 4; ++k) rr[k] = qt[k] + h * dq[k];
      const S nrm = sq_root(rr[0] * rr[0] + rr[1] * rr[1] + rr[2] * rr[2] + rr[3] * rr[3]);
      S q1n[4], rb[4];
      for (int k = 0; k < 4; ++k) q1n[k] = rr[k] / nrm;
      const S dd = q1n[0] * qt1b[0] + q1n[1] * qt1b[1] + q1n[2] * qt1b[2] + q1n[3] * qt1b[3];
      for (int k = 0; k < 4; ++k) rb[k] = (qt1b[k] - q1n[k] * dd) / nrm;
      S t1[3], t2[3];
      cross3(v1, rb, t1);   // w1 x rb_v
      cross3(rb, qt, t2);   // rb_v x u
      for (int k = 0; k < 3; ++k) {
        qb[qi + 3 + k] = qb[qi + 3 + k] + rb[k] + h * (t1[k] - rb[3] * v1[k]);
        qd1b[vi + k] = qd1b[vi + k] + h * (qt[3] * rb[k] + t2[k] - rb[3] * qt[k]);
      }
      qb[qi + 6] = qb[qi + 6] + rb[3] + h * dot3(v1, rb);
    } else {
      qb[tp.qi[i]] = qb[tp.qi[i]] + xbar[tp.qi[i]];
      qd1b[tp.vi[i]] = qd1b[tp.vi[i]] + dt * xbar[tp.qi[i]];
    }
  }
  for (int k = 0; k < nv; ++k) qdmb[k] = qd1b[k];
  const int na = rc.na, r = rc.r;
  if (na > 0) {
    // ---- impulses: qd1 = qd_minus + MJ x
    S xb[kNR];
    S gv[kNV];
#pragma unroll
    for (int k = 0; k < kNV; ++k) gv[k] = k < nv ? qd1b[k] : S(0);
    for (int j = 0; j < r; ++j) {
      S s = S(0);
      const S xj = w.x[j];
#pragma unroll
      for (int k = 0; k < kNV; ++k) {
        s = fmadd_pad(w.MJ[k][j], gv[k], s, k < nv);  // gv zero beyond nv
        ad.MJb[k][j] = mul_pad(gv[k], xj, k < nv);
      }
      xb[j] = s;
    }
    // (all of it: the adjoint of A below reads past r * r, times zero)
#pragma unroll
    for (int k = 0; k < kNR * kNR; ++k) ad.Ab[k] = S(0);
    for (int i = 0; i < r; ++i) ad.bb[i] = S(0);
    // ---- second solve (all kept rows; tangent bounds +-mu lambda_n)
    const int nk = rc.nk, nkn = rc.nkn;
    S lo[kNR], hi[kNR], lob[kNR], hib[kNR], xkb[kNR];
    for (int i = 0; i < nk; ++i) {
      const int ri = rc.keep[i];
      if (ri % 3 == 0) {
        lo[i] = S(0);
        hi[i] = S(Big<typename RealOf<S>::type>::v);
      } else {
        lo[i] = -(mu * rc.lamn[ri / 3]);
        hi[i] = mu * rc.lamn[ri / 3];
      }
      lob[i] = hib[i] = S(0);
      xkb[i] = xb[ri];
    }
    if (stage.p)
      pgs_reverse_staged(nk, rc.keep, r, w.A, w.b, lo, hi, tp.niter, &rc.x2[0][0], kNR, xkb, ad.Ab, ad.bb, lob, hib,
                         stage);
    else
      pgs_reverse(nk, rc.keep, r, w.A, w.b, lo, hi, tp.niter, &rc.x2[0][0], kNR, xkb, ad.Ab, ad.bb, lob, hib);
    S lamb[kNC];
    for (int c = 0; c < na; ++c) lamb[c] = S(0);
    for (int i = 0; i < nk; ++i) {
      const int ri = rc.keep[i];
      if (ri % 3 != 0) {
        const S gb = hib[i] - lob[i];
        lamb[ri / 3] = lamb[ri / 3] + mu * gb;
        mub = mub + rc.lamn[ri / 3] * gb;
      }
    }
    // ---- first solve (kept normal rows, [0, inf))
    S xnb[kNC], lo1[kNC], hi1[kNC], lob1[kNC], hib1[kNC];
    for (int i = 0; i < nkn; ++i) {
      xnb[i] = lamb[rc.kn[i] / 3];
      lo1[i] = S(0);
      hi1[i] = S(Big<typename RealOf<S>::type>::v);
      lob1[i] = hib1[i] = S(0);
    }
    if (stage.p)
      pgs_reverse_staged(nkn, rc.kn, r, w.A, w.b, lo1, hi1, tp.niter, &rc.x1[0][0], kNC, xnb, ad.Ab, ad.bb, lob1,
                         hib1, stage);
    else
      pgs_reverse(nkn, rc.kn, r, w.A, w.b, lo1, hi1, tp.niter, &rc.x1[0][0], kNC, xnb, ad.Ab, ad.bb, lob1, hib1);
    // ---- A = J MJ, b = J qd_minus + (beta/dt) phi (normal rows)
    const S bdt = S(tp.beta) / dt;
    S phib[kNC];
    for (int c = 0; c < na; ++c) phib[c] = S(0);
    // (row i of A_bar, then column k of J, held in registers, zero beyond r;
    // the sums run over all kNR terms with no condition, a term beyond r
    // being zero times a cleared or finite entry, three columns of MJ (of
    // A_bar) per pass, so that a pass's loads issue together; each sum runs
    // in the same order.  Every index stays inside its array: kNV and r are
    // multiples of 3, and the rows of A_bar at stride r end before
    // kNR * kNR.)
    static_assert(kNV % 3 == 0, "column blocks of three");
    for (int i = 0; i < r; ++i) {
      S Abi[kNR];
#pragma unroll
      for (int j = 0; j < kNR; ++j) {
        const S v = ad.Ab[i * r + j];
        Abi[j] = j < r ? v : S(0);
      }
      const S bbi = ad.bb[i];
      for (int k0 = 0; k0 < nv; k0 += 3) {
#pragma unroll
        for (int kk = 0; kk < 3; ++kk) {
          const int k = k0 + kk;
          S s = mul_pad(bbi, rc.qdm[k], k < nv);
#pragma unroll
          for (int j = 0; j < kNR; ++j) s = fmadd_pad(Abi[j], w.MJ[k][j], s, j < r && k < nv);
          const S jik = w.J[i][k];
          if (k < nv) {
            ad.Jb[i][k] = s;
            qdmb[k] = fmadd(jik, bbi, qdmb[k]);
          }
        }
      }
      if (i % 3 == 0) phib[i / 3] = phib[i / 3] + bdt * bbi;
    }
    for (int k = 0; k < nv; ++k) {
      S Jk[kNR];
#pragma unroll
      for (int i = 0; i < kNR; ++i) {
        const S v = w.J[i][k];
        Jk[i] = i < r ? v : S(0);
      }
      for (int j0 = 0; j0 < r; j0 += 3) {
#pragma unroll
        for (int jj = 0; jj < 3; ++jj) {
          const int j = j0 + jj;
          S s = S(0);
#pragma unroll
          for (int i = 0; i < kNR; ++i) s = fmadd_pad(Jk[i], ad.Ab[i * r + j], s, i < r);
          ad.MJb[k][j] = ad.MJb[k][j] + s;
        }
      }
    }
    // ---- MJ = M^-1 J^T: W = M^-1 MJ_bar; J_bar += W^T; q_bar -= d/dq <W, M(q) MJ>
    // (the copies and sums run over all kNV / kNQ entries with no
    // condition, so that their loads issue together; the entries beyond nv
    // and nq are zero or never read)
    for (int j = 0; j < r; ++j) {
      S col[kNV], Wj[kNV], mj[kNV];
#pragma unroll
      for (int k = 0; k < kNV; ++k) {
        col[k] = ad.MJb[k][j];
        mj[k] = w.MJ[k][j];
        Wj[k] = S(0);
      }
      minv_apply(tp, art, col, Wj);
#pragma unroll
      for (int k = 0; k < kNV; ++k) ad.Jb[j][k] = add_pad(ad.Jb[j][k], Wj[k], k < nv);
      S gqj[kNQ];
#pragma unroll
      for (int k = 0; k < kNQ; ++k) gqj[k] = S(0);
      id_vjp_static(tp, art, mj, Wj, gqj);
#pragma unroll
      for (int k = 0; k < kNQ; ++k) qb[k] = sub_pad(qb[k], gqj[k], k < nq);
    }
    // ---- contact rows and gaps through the world poses
    for (int i = 0; i < n; ++i) {
      for (int k = 0; k < 9; ++k) ad.Ewb[i][k] = S(0);
      for (int k = 0; k < 3; ++k) ad.owb[i][k] = S(0);
    }
    const int dirs[3] = {1, 0, 2};
    for (int c = 0; c < na; ++c) {
      const int kc = rc.act[c], l = tp.clink[kc], sb = kParLink * n + kParSphere * kc;
      const S cc[3] = {S(P(sb)), S(P(sb + 1)), S(P(sb + 2))};
      const S rad = S(P(sb + 3));
      const S* pw = rc.pw[c];
      S pwb[3] = {S(0), S(0), S(0)};
      for (int j = l; j >= 0; j = tp.parent[j]) {
        S d[3];
        for (int k = 0; k < 3; ++k) d[k] = pw[k] - w.ow[j][k];
        S db[3] = {S(0), S(0), S(0)};
        if (tp.jtype[j] == SIM_JOINT_FREE) {
          for (int e = 0; e < 3; ++e) {
            const S Re[3] = {w.Ew[j][3 * e], w.Ew[j][3 * e + 1], w.Ew[j][3 * e + 2]};
            S ca[3], cl_[3];
            for (int dd = 0; dd < 3; ++dd) {
              ca[dirs[dd]] = ad.Jb[3 * c + dd][tp.vi[j] + e];
              cl_[dirs[dd]] = ad.Jb[3 * c + dd][tp.vi[j] + 3 + e];
            }
            // col_ang = Re x d, col_lin = Re
            S t1[3], t2[3];
            cross3(d, ca, t1);
            cross3(ca, Re, t2);
            for (int k = 0; k < 3; ++k) {
              ad.Ewb[j][3 * e + k] = ad.Ewb[j][3 * e + k] + t1[k] + cl_[k];
              db[k] = db[k] + t2[k];
            }
          }
        } else {
          S cb[3];
          for (int dd = 0; dd < 3; ++dd) cb[dirs[dd]] = ad.Jb[3 * c + dd][tp.vi[j]];
          S zb[3];
          if (tp.jtype[j] == SIM_JOINT_PRISMATIC) {
            for (int k = 0; k < 3; ++k) zb[k] = cb[k];
          } else {
            // col = z x d
            S z[3];
            for (int b = 0; b < 3; ++b)
              z[b] = w.Ew[j][b] * w.ax[j][0] + w.Ew[j][3 + b] * w.ax[j][1] + w.Ew[j][6 + b] * w.ax[j][2];
            cross3(d, cb, zb);
            cross3(cb, z, db);
          }
          // z = Ew^T a
          for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) ad.Ewb[j][3 * a + b] = ad.Ewb[j][3 * a + b] + w.ax[j][a] * zb[b];
        }
        for (int k = 0; k < 3; ++k) {
          pwb[k] = pwb[k] + db[k];
          ad.owb[j][k] = ad.owb[j][k] - db[k];
        }
      }
      // pw = ow_l + Ew_l^T cl; cl = cc - rad Ew_l[:, 1]; phi = ow_l[1] + (Ew_l^T cc)[1] - rad
      S clb[3];
      for (int b = 0; b < 3; ++b) {
        clb[b] = w.Ew[l][3 * b] * pwb[0] + w.Ew[l][3 * b + 1] * pwb[1] + w.Ew[l][3 * b + 2] * pwb[2];
        for (int a = 0; a < 3; ++a) ad.Ewb[l][3 * b + a] = ad.Ewb[l][3 * b + a] + rc.cl[c][b] * pwb[a];
      }
      for (int a = 0; a < 3; ++a) {
        ad.owb[l][a] = ad.owb[l][a] + pwb[a];
        ad.Ewb[l][3 * a + 1] = ad.Ewb[l][3 * a + 1] - rad * clb[a];
      }
      ad.owb[l][1] = ad.owb[l][1] + phib[c];
      for (int b = 0; b < 3; ++b) ad.Ewb[l][3 * b + 1] = ad.Ewb[l][3 * b + 1] + phib[c] * cc[b];
    }
    // world poses: Ew_i = E_i Ew_p, ow_i = ow_p + Ew_p^T r_i (root: Ew = E, ow = r)
    for (int i = n - 1; i >= 0; --i) {
      const int p = tp.parent[i];
      S Eb[9], rb[3];
      if (p >= 0) {
        for (int a = 0; a < 3; ++a)
          for (int k = 0; k < 3; ++k) {
            S s = S(0), t = S(0);
            for (int c2 = 0; c2 < 3; ++c2) {
              s = s + ad.Ewb[i][3 * a + c2] * w.Ew[p][3 * k + c2];
              t = t + w.E[i][3 * c2 + a] * ad.Ewb[i][3 * c2 + k];
            }
            Eb[3 * a + k] = s;
            ad.Ewb[p][3 * a + k] = ad.Ewb[p][3 * a + k] + t;
          }
        for (int k = 0; k < 3; ++k) {
          rb[k] = w.Ew[p][3 * k] * ad.owb[i][0] + w.Ew[p][3 * k + 1] * ad.owb[i][1] + w.Ew[p][3 * k + 2] * ad.owb[i][2];
          ad.owb[p][k] = ad.owb[p][k] + ad.owb[i][k];
          for (int a = 0; a < 3; ++a) ad.Ewb[p][3 * k + a] = ad.Ewb[p][3 * k + a] + w.r[i][k] * ad.owb[i][a];
        }
      } else {
        for (int k = 0; k < 9; ++k) Eb[k] = ad.Ewb[i][k];
        for (int k = 0; k < 3; ++k) rb[k] = ad.owb[i][k];
      }
      if (tp.jtype[i] == SIM_JOINT_FREE) {
        // E = R(quat)^T, r = p
        const int qi = tp.qi[i];
        for (int k = 0; k < 3; ++k) qb[qi + k] = qb[qi + k] + rb[k];
        // <Eb, R^T> = sum_ab Eb[a][b] R[b][a] = sum_b e_b^T R (Eb^T)_col...: per basis pair
        for (int a = 0; a < 3; ++a)
          for (int b = 0; b < 3; ++b) {
            const S eb = Eb[3 * a + b];
            S ea[3] = {S(0), S(0), S(0)}, ebv[3] = {S(0), S(0), S(0)}, gr[4];
            ea[a] = S(1);
            ebv[b] = eb;
            // Eb[a][b] R[b][a] = ebv^T R ea (ebv = eb e_b)
            quat_rot_grad4(q + qi + 3, ebv, ea, gr);
            for (int k = 0; k < 4; ++k) qb[qi + 3 + k] = qb[qi + 3 + k] + gr[k];
          }
      } else if (tp.jtype[i] == SIM_JOINT_PRISMATIC) {
        // r = r_T + q E^T a (E = E_T)
        S s = S(0);
        for (int k = 0; k < 3; ++k)
          s = s + rb[k] * (w.E[i][k] * w.ax[i][0] + w.E[i][3 + k] * w.ax[i][1] + w.E[i][6 + k] * w.ax[i][2]);
        qb[tp.qi[i]] = qb[tp.qi[i]] + s;
      } else {
        // dE/dq = -[a]x E
        const S* a = w.ax[i];
        const S K[9] = {S(0), -a[2], a[1], a[2], S(0), -a[0], -a[1], a[0], S(0)};
        S s = S(0);
        for (int r_ = 0; r_ < 3; ++r_)
          for (int c_ = 0; c_ < 3; ++c_) {
            const S dE = -(K[3 * r_] * w.E[i][c_] + K[3 * r_ + 1] * w.E[i][3 + c_] + K[3 * r_ + 2] * w.E[i][6 + c_]);
            s = s + Eb[3 * r_ + c_] * dE;
          }
        qb[tp.qi[i]] = qb[tp.qi[i]] + s;
      }
    }
  }
  // ---- the smooth step: qd_minus = qd + dt FD(q, qd, u)
  S qddb[kNV], taub[kNV];
  for (int k = 0; k < nv; ++k) {
    qdb[k] = qdb[k] + qdmb[k];
    qddb[k] = dt * qdmb[k];
  }
  minv_apply(tp, art, qddb, taub);
  for (int i = 0; i < n; ++i)
    if (tp.jtype[i] != SIM_JOINT_FREE) ubar[tp.ui[i]] = taub[tp.vi[i]];
  S gq[kNQ], gqd[kNV];
  for (int k = 0; k < nq; ++k) gq[k] = S(0);
  for (int k = 0; k < nv; ++k) gqd[k] = S(0);
  id_vjp(tp, P, w, q, qd, rc.qdd, true, taub, gq, gqd);
  // joint limits: the limit torque tau_l(q, qd) adds to the control, so its
  // slopes (-k, -d outside the range) carry tau_bar to q and qd
  if (tp.has_limits)
    for (int i = 0; i < n; ++i) {
      if (tp.jtype[i] == SIM_JOINT_FREE) continue;
      const double* L = tp.lim[i];
      const S qv = q[tp.qi[i]];
      if (val(qv) > val(S(L[1])) || val(qv) < val(S(L[0]))) {
        qb[tp.qi[i]] = qb[tp.qi[i]] - S(L[2]) * taub[tp.vi[i]];
        qdb[tp.vi[i]] = qdb[tp.vi[i]] - S(L[3]) * taub[tp.vi[i]];
      }
    }
  for (int k = 0; k < nq; ++k) xbar[k] = qb[k] - gq[k];
  for (int k = 0; k < nv; ++k) xbar[nq + k] = qdb[k] - gqd[k];
}

}  // namespace aba_contact
