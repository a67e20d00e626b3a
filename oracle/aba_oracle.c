/*
 * Plain FP64 CPU oracle: ABA forward dynamics, semi-implicit Euler, and the
 * reverse-time adjoint with checkpointing.  TEST INFRASTRUCTURE ONLY (see
 * oracle.h): never part of the product path.
 *
 * The forward pass (aba_fwd.inc) is instantiated twice: for double and for
 * double complex (complex-step derivative checks).  The reverse pass below
 * is real-only.  Every reverse statement is the adjoint of one forward
 * statement, applied in the exact reverse order of the forward pass
 * (Sec. 4.1, "Each operation in the forward simulation has its
 * corresponding adjoint operation in the backward pass"; Sec. 4.2, Eq.
 * intermediate: recompute Z^k = G(x^{k-1}), then the adjoints of F and G).
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

int orc_nq(const orc_model *m) {
  int s = 0;
  for (int i = 0; i < m->n; ++i) s += (m->jtype[i] == ORC_FREE) ? 7 : (m->jtype[i] == ORC_SPHERICAL) ? 4 : 1;
  return s;
}
int orc_nv(const orc_model *m) {
  int s = 0;
  for (int i = 0; i < m->n; ++i) s += (m->jtype[i] == ORC_FREE) ? 6 : (m->jtype[i] == ORC_SPHERICAL) ? 3 : 1;
  return s;
}
int orc_nu(const orc_model *m) {
  int s = 0;
  for (int i = 0; i < m->n; ++i) s += (m->jtype[i] == ORC_FREE) ? 0 : (m->jtype[i] == ORC_SPHERICAL) ? 3 : 1;
  return s;
}

#define CAT_(a, b) a##b
#define CAT(a, b) CAT_(a, b)

/* real instantiation */
#define S double
#define FN(name) CAT(name, _r)
#define SSIN sin
#define SCOS cos
#define SSQRT sqrt
#define SREAL(x) (x)
#define PGS_SOLVE(n, it, A, b, lo, hi, x0, x) orc_pgs_solve((n), (it), (A), (b), (lo), (hi), (x0), (x), NULL)
#include "aba_fwd.inc"
#include "contact.inc"
#undef PGS_SOLVE
#undef S
#undef FN
#undef SSIN
#undef SCOS
#undef SSQRT
#undef SREAL

/* complex instantiation (analytic continuation; no abs; the joint-limit
   switch decides on real parts) */
#define S double complex
#define FN(name) CAT(name, _c)
#define SSIN csin
#define SCOS ccos
#define SSQRT csqrt
#define SREAL(x) creal(x)
#define PGS_SOLVE(n, it, A, b, lo, hi, x0, x) orc_pgs_solve_c((n), (it), (A), (b), (lo), (hi), (x0), (x))
#include "aba_fwd.inc"
#include "contact.inc"
#undef PGS_SOLVE
#undef S
#undef FN
#undef SSIN
#undef SCOS
#undef SSQRT
#undef SREAL

typedef link_tape_r tape_t;

/* ---- exported forward entry points ------------------------------------ */

void orc_fd(const orc_model *m, const double *q, const double *qd,
            const double *tau, double *qdd) {
  fd_r(m, q, qd, tau, qdd);
}

void orc_fd_c(const orc_model *m, const void *q, const void *qd,
              const void *tau, void *qdd) {
  fd_c(m, (const double complex *)q, (const double complex *)qd,
       (const double complex *)tau, (double complex *)qdd);
}

void orc_step(const orc_model *m, const double *q, const double *qd,
              const double *tau, double dt, double *q1, double *qd1) {
  const int nv = orc_nv(m);
  double *qdd = (double *)malloc(sizeof(double) * (size_t)nv);
  fd_r(m, q, qd, tau, qdd);
  integrate_r(m, q, qd, qdd, dt, q1, qd1);
  free(qdd);
}

int orc_rollout(const orc_model *m, const double *q0, const double *qd0,
                const double *tau, double dt, int T, double *qT, double *qdT,
                double *traj) {
  if (T < 0) return -1;
  return rollout_r(m, q0, qd0, tau, dt, T, qT, qdT, traj);
}

int orc_rollout_c(const orc_model *m, const void *q0, const void *qd0,
                  const void *tau, double dt, int T, void *qT, void *qdT) {
  if (T < 0) return -1;
  return rollout_c(m, (const double complex *)q0, (const double complex *)qd0,
                   (const double complex *)tau, dt, T, (double complex *)qT,
                   (double complex *)qdT, NULL);
}

/* ---- reverse mode ----------------------------------------------------- */

typedef struct {
  double X[36], v[6], vJ[6], c[6], h[6];
  double IA[36], pA[6], U[18], D[9], Di[9], u[3], Ia[36], pa[6], ap[6], a[6], qdd[3];
  double S[18]; /* adjoint of the motion subspace (its nd columns) */
} link_bar;

/* y += A^T x */
static void tvec_add(const double *A, const double *x, double *y) {
  for (int i = 0; i < 6; ++i)
    for (int k = 0; k < 6; ++k) y[i] += A[6 * k + i] * x[k];
}
/* y += A x */
static void vec_add(const double *A, const double *x, double *y) {
  for (int i = 0; i < 6; ++i)
    for (int k = 0; k < 6; ++k) y[i] += A[6 * i + k] * x[k];
}
/* M += a b^T */
static void outer_add(const double *a, const double *b, double *M) {
  for (int i = 0; i < 6; ++i)
    for (int j = 0; j < 6; ++j) M[6 * i + j] += a[i] * b[j];
}

/* d R(quat) / d quat_k for R = (w^2 - v.v) I + 2 v v^T + 2 w [v]x. */
static void quat_R_grad(const double *qt, const double *Rbar, double *qtbar) {
  double x = qt[0], y = qt[1], z = qt[2], w = qt[3];
  double v[3] = {x, y, z};
  for (int k = 0; k < 4; ++k) {
    double dR[9];
    if (k < 3) {
      double e[3] = {0, 0, 0};
      e[k] = 1;
      double ex[9];
      skew3_r(e, ex);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          dR[3 * i + j] = (i == j ? -2.0 * v[k] : 0.0) +
                          2.0 * (e[i] * v[j] + v[i] * e[j]) + 2.0 * w * ex[3 * i + j];
    } else {
      double vx[9];
      skew3_r(v, vx);
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
          dR[3 * i + j] = (i == j ? 2.0 * w : 0.0) + 2.0 * vx[3 * i + j];
    }
    double s = 0;
    for (int e = 0; e < 9; ++e) s += Rbar[e] * dR[e];
    qtbar[k] += s;
  }
}

/* Adjoint of the spatial inertia of link i, Ibar (dense 6x6, every entry
 * taken as an independent variable), expressed in the ten inertial
 * parameters of the link (link frame): mass m, first moment h = m c, and
 * the rotational inertia about the link origin I_O = I_c - m [c]x^2, i.e.
 * I = [I_O, [h]x; [h]x^T, m 1].  Output order: m, h (3), I_O xx yy zz xy
 * xz yz, where an off-diagonal parameter stands for both of its entries.
 * ADDS into pbar[10]. */
static void inertia_params_add(const double *Ibar, double *pbar) {
  pbar[0] += Ibar[6 * 3 + 3] + Ibar[6 * 4 + 4] + Ibar[6 * 5 + 5];
  double P[9]; /* top-right block minus bottom-left block */
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) P[3 * r + c] = Ibar[6 * r + 3 + c] - Ibar[6 * (3 + r) + c];
  pbar[1] += P[3 * 2 + 1] - P[3 * 1 + 2];
  pbar[2] += P[3 * 0 + 2] - P[3 * 2 + 0];
  pbar[3] += P[3 * 1 + 0] - P[3 * 0 + 1];
  pbar[4] += Ibar[0];
  pbar[5] += Ibar[7];
  pbar[6] += Ibar[14];
  pbar[7] += Ibar[1] + Ibar[6];
  pbar[8] += Ibar[2] + Ibar[12];
  pbar[9] += Ibar[8] + Ibar[13];
}

/* Partial derivatives of the joint-limit torque (see limit_torque in
 * aba_fwd.inc) with respect to q and qd; returns whether a limit is
 * active. */
static int limit_slopes(const orc_model *m, int i, double q, double qd, double *dq, double *dqd) {
  (void)qd;
  *dq = 0;
  *dqd = 0;
  if (!m->limits || (m->jtype[i] != ORC_REVOLUTE && m->jtype[i] != ORC_PRISMATIC)) return 0;
  const double *L = m->limits + 4 * i;
  if (q > L[1] || q < L[0]) {
    *dq = -L[2];
    *dqd = -L[3];
    return 1;
  }
  return 0;
}

/* Adjoint of one 1-dof link's placement and axis, ADDED into fb[9], from
 * the link's dense transform adjoint Xbar and motion-subspace adjoint Sbar
 * at joint coordinate q (see orc_rollout_grad_params for the three
 * parameter directions).  X = XJ(q; a) XT(E_T, r_T), XT = plucker(E_T, r_T):
 *   r_T:  dXT/dr_k = [0 0; -E_T [e_k]x 0];
 *   E_T -> exp(-[phi]x) E_T:  dXT/dphi_k = plucker'(-[e_k]x E_T, r_T);
 *   a -> exp([w]x) a, da = e_k x a:
 *     revolute  EJ = I - sin q [a]x + (1 - cos q)[a]x^2, S = [a; 0],
 *       dEJ = -sin q [da]x + (1 - cos q)([da]x [a]x + [a]x [da]x);
 *     prismatic XJ = [I 0; -[q a]x I], S = [0; a], dXJ = [0 0; -q [da]x 0];
 *   and the axis output is w_bar x a, the gradient with respect to the axis
 *   vector along the unit sphere.  A spherical joint has no axis: its three
 *   axis entries stay zero, and its XJ is the rotation of its quaternion.
 * ql points to the link's joint coordinates. */
static void frame_params_add(const orc_model *m, int i, const double *ql, const double *Xbar, const double *Sbar,
                             double *fb) {
  const double *ax = m->axis + 3 * i, *ET = m->E_T + 9 * i, *rT = m->r_T + 3 * i;
  const int prism = m->jtype[i] == ORC_PRISMATIC, sph = m->jtype[i] == ORC_SPHERICAL;
  const double q = ql[0];
  double XJ[36], XT[36], zero3[3] = {0, 0, 0}, I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  if (sph) {
    double R[9], EJ[9];
    quat_R_r(ql, R);
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) EJ[3 * a + b] = R[3 * b + a];
    plucker_r(EJ, zero3, XJ);
  } else if (prism) {
    double ra[3] = {q * ax[0], q * ax[1], q * ax[2]};
    plucker_r(I3, ra, XJ);
  } else {
    double EJ[9];
    joint_rot_r(q, ax, EJ);
    plucker_r(EJ, zero3, XJ);
  }
  plucker_r(ET, rT, XT);
  for (int k = 0; k < 3; ++k) {
    double ek[3] = {0, 0, 0}, ekx[9], dXT[36], dX[36];
    ek[k] = 1;
    skew3_r(ek, ekx);
    /* r_T */
    for (int j = 0; j < 36; ++j) dXT[j] = 0;
    double Ee[9];
    mat3_mul_r(ET, ekx, Ee);
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) dXT[6 * (3 + r) + c] = -Ee[3 * r + c];
    mat6_mul_r(XJ, dXT, dX);
    double sr = 0;
    for (int j = 0; j < 36; ++j) sr += Xbar[j] * dX[j];
    fb[3 + k] += sr;
    /* E_T rotation: d(plucker(E, r)) = [dE 0; -dE [r]x dE] with dE = -[e_k]x E_T */
    double dE[9], rx[9], dErx[9];
    mat3_mul_r(ekx, ET, dE);
    for (int j = 0; j < 9; ++j) dE[j] = -dE[j];
    skew3_r(rT, rx);
    mat3_mul_r(dE, rx, dErx);
    for (int j = 0; j < 36; ++j) dXT[j] = 0;
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) {
        dXT[6 * r + c] = dE[3 * r + c];
        dXT[6 * (3 + r) + 3 + c] = dE[3 * r + c];
        dXT[6 * (3 + r) + c] = -dErx[3 * r + c];
      }
    mat6_mul_r(XJ, dXT, dX);
    double sp = 0;
    for (int j = 0; j < 36; ++j) sp += Xbar[j] * dX[j];
    fb[k] += sp;
  }
  if (sph) return;
  /* axis: w_bar_k = <Xbar, dXJ_k XT> + Sbar . dS_k */
  double wb[3];
  for (int k = 0; k < 3; ++k) {
    double da[3] = {0, 0, 0}, dax[9], dXJ[36], dX[36];
    /* da = e_k x a */
    da[(k + 1) % 3] = -ax[(k + 2) % 3];
    da[(k + 2) % 3] = ax[(k + 1) % 3];
    skew3_r(da, dax);
    for (int j = 0; j < 36; ++j) dXJ[j] = 0;
    if (prism) {
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) dXJ[6 * (3 + r) + c] = -q * dax[3 * r + c];
    } else {
      double axx[9], t1[9], t2[9], dEJ[9];
      skew3_r(ax, axx);
      mat3_mul_r(dax, axx, t1);
      mat3_mul_r(axx, dax, t2);
      for (int j = 0; j < 9; ++j) dEJ[j] = -sin(q) * dax[j] + (1.0 - cos(q)) * (t1[j] + t2[j]);
      plucker_r(dEJ, zero3, dXJ);
    }
    mat6_mul_r(dXJ, XT, dX);
    double sw = 0;
    for (int j = 0; j < 36; ++j) sw += Xbar[j] * dX[j];
    for (int j = 0; j < 3; ++j) sw += Sbar[prism ? 3 + j : j] * da[j];
    wb[k] = sw;
  }
  fb[6] += wb[1] * ax[2] - wb[2] * ax[1];
  fb[7] += wb[2] * ax[0] - wb[0] * ax[2];
  fb[8] += wb[0] * ax[1] - wb[1] * ax[0];
}

/* Reverse of aba_tape_r: ADD d<qdd_bar, qdd>/d(q, qd, tau), and, when
 * param_bar is not NULL, the adjoint of every link's inertial parameters
 * ([n][10], see inertia_params_add), when frame_bar is not NULL that of
 * every 1-dof link's placement and axis ([n][9], see frame_params_add). */
static int aba_vjp(const orc_model *m, const double *q, const double *qd,
                   const tape_t *L, const double *qdd_bar, double *q_bar,
                   double *qd_bar, double *tau_bar, double *param_bar, double *frame_bar) {
  const int n = m->n;
  int qi[n], vi[n], ui[n];
  layout_r(m, qi, vi, ui);
  link_bar *B = (link_bar *)calloc((size_t)n, sizeof(link_bar));
  if (!B) return -1;
  const double *g = m->gravity;
  const double a0[6] = {0, 0, 0, -g[0], -g[1], -g[2]};
  double E0bar[9] = {0};

  for (int i = 0; i < n; ++i)
    if (m->jtype[i] != ORC_FREE)
      for (int k = 0; k < ndof_r(m, i); ++k) B[i].qdd[k] = qdd_bar[vi[i] + k];

  /* reverse of pass 3, leaves -> root */
  for (int i = n - 1; i >= 0; --i) {
    const tape_t *l = &L[i];
    link_bar *b = &B[i];
    const int lam = m->parent[i];
    if (m->jtype[i] == ORC_FREE) {
      /* abase = ap + [0; E0 g];  a = ap */
      const double *ab = qdd_bar + vi[i];
      for (int k = 0; k < 6; ++k) b->ap[k] += ab[k] + b->a[k];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) E0bar[3 * r + c] += ab[3 + r] * g[c];
      /* ap = -IA^{-1} pA:  w = IA^{-T} ap_bar; pA_bar -= w; IA_bar -= w ap^T */
      double IAt[36], w[6];
      mat6_transpose_r(l->IA, IAt);
      solve6_r(IAt, b->ap, w);
      for (int k = 0; k < 6; ++k) b->pA[k] -= w[k];
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) b->IA[6 * r + c] -= w[r] * l->ap[c];
      continue;
    }
    const int nd = ndof_r(m, i);
    double Sv[18];
    motion_subspace_r(m, i, Sv);
    /* a = ap + S qdd */
    for (int k = 0; k < 6; ++k) b->ap[k] += b->a[k];
    for (int j = 0; j < nd; ++j)
      for (int r = 0; r < 6; ++r) {
        b->qdd[j] += Sv[6 * j + r] * b->a[r];
        b->S[6 * j + r] += b->a[r] * l->qdd[j];
      }
    /* qdd = D^-1 w, w = u - U^T ap */
    double w[3], wb[3];
    for (int j = 0; j < nd; ++j) {
      w[j] = l->u[j];
      for (int r = 0; r < 6; ++r) w[j] -= l->U[6 * j + r] * l->ap[r];
    }
    for (int k = 0; k < nd; ++k)
      for (int j = 0; j < nd; ++j) b->Di[3 * k + j] += b->qdd[k] * w[j];
    for (int j = 0; j < nd; ++j) {
      wb[j] = 0;
      for (int k = 0; k < nd; ++k) wb[j] += l->Di[3 * k + j] * b->qdd[k];
    }
    for (int j = 0; j < nd; ++j) {
      b->u[j] += wb[j];
      for (int r = 0; r < 6; ++r) {
        b->U[6 * j + r] -= l->ap[r] * wb[j];
        b->ap[r] -= l->U[6 * j + r] * wb[j];
      }
    }
    /* ap = X a_lam + c */
    const double *al = (lam < 0) ? a0 : L[lam].a;
    if (lam >= 0) tvec_add(l->X, b->ap, B[lam].a);
    outer_add(b->ap, al, b->X);
    for (int k = 0; k < 6; ++k) b->c[k] += b->ap[k];
  }

  /* reverse of pass 2, root -> leaves */
  for (int i = 0; i < n; ++i) {
    if (m->jtype[i] == ORC_FREE) continue;
    const tape_t *l = &L[i];
    link_bar *b = &B[i];
    const int lam = m->parent[i];
    const int nd = ndof_r(m, i);
    double Sv[18];
    motion_subspace_r(m, i, Sv);
    if (lam >= 0) {
      const link_bar *bl = &B[lam];
      /* pA_lam += X^T pa */
      vec_add(l->X, bl->pA, b->pa);
      outer_add(l->pa, bl->pA, b->X);
      /* IA_lam += X^T Ia X:  Ia_bar += X IAb X^T;
         X_bar += Ia X IAb^T + Ia^T X IAb */
      double T1[36], T2[36], Xt[36], IAbt[36], Iat[36];
      mat6_transpose_r(l->X, Xt);
      mat6_mul_r(l->X, bl->IA, T1);
      mat6_mul_r(T1, Xt, T2);
      for (int k = 0; k < 36; ++k) b->Ia[k] += T2[k];
      mat6_transpose_r(bl->IA, IAbt);
      mat6_transpose_r(l->Ia, Iat);
      mat6_mul_r(l->Ia, l->X, T1);
      mat6_mul_r(T1, IAbt, T2);
      for (int k = 0; k < 36; ++k) b->X[k] += T2[k];
      mat6_mul_r(Iat, l->X, T1);
      mat6_mul_r(T1, bl->IA, T2);
      for (int k = 0; k < 36; ++k) b->X[k] += T2[k];
      /* pa = pA + Ia c + U y, y = D^-1 u */
      for (int k = 0; k < 6; ++k) b->pA[k] += b->pa[k];
      outer_add(b->pa, l->c, b->Ia);
      tvec_add(l->Ia, b->pa, b->c);
      double y[3], yb[3];
      for (int k = 0; k < nd; ++k) {
        y[k] = 0;
        for (int j = 0; j < nd; ++j) y[k] += l->Di[3 * k + j] * l->u[j];
      }
      for (int k = 0; k < nd; ++k) {
        yb[k] = 0;
        for (int r = 0; r < 6; ++r) {
          yb[k] += l->U[6 * k + r] * b->pa[r];
          b->U[6 * k + r] += b->pa[r] * y[k];
        }
      }
      for (int k = 0; k < nd; ++k)
        for (int j = 0; j < nd; ++j) {
          b->Di[3 * k + j] += yb[k] * l->u[j];
          b->u[j] += l->Di[3 * k + j] * yb[k];
        }
      /* Ia = IA - U D^-1 U^T:  U_bar -= Ia_bar U D^-T + Ia_bar^T U D^-1,
         Di_bar -= U^T Ia_bar U */
      for (int k = 0; k < 36; ++k) b->IA[k] += b->Ia[k];
      for (int k = 0; k < nd; ++k)
        for (int r = 0; r < 6; ++r) {
          double s_ = 0;
          for (int c = 0; c < 6; ++c)
            for (int j = 0; j < nd; ++j)
              s_ += (b->Ia[6 * r + c] * l->Di[3 * k + j] + b->Ia[6 * c + r] * l->Di[3 * j + k]) * l->U[6 * j + c];
          b->U[6 * k + r] -= s_;
        }
      for (int j = 0; j < nd; ++j)
        for (int k = 0; k < nd; ++k) {
          double s_ = 0;
          for (int r = 0; r < 6; ++r)
            for (int c = 0; c < 6; ++c) s_ += l->U[6 * j + r] * b->Ia[6 * r + c] * l->U[6 * k + c];
          b->Di[3 * j + k] -= s_;
        }
    }
    /* Di = D^-1:  D_bar -= D^-T Di_bar D^-T */
    for (int j = 0; j < nd; ++j)
      for (int k = 0; k < nd; ++k) {
        double s_ = 0;
        for (int p = 0; p < nd; ++p)
          for (int r = 0; r < nd; ++r) s_ += l->Di[3 * p + j] * b->Di[3 * p + r] * l->Di[3 * k + r];
        b->D[3 * j + k] -= s_;
      }
    /* u = tau + tau_limit(q, qd) - S^T pA */
    for (int j = 0; j < nd; ++j) tau_bar[ui[i] + j] += b->u[j];
    if (nd == 1) {
      double dq, dqd;
      if (limit_slopes(m, i, q[qi[i]], qd[vi[i]], &dq, &dqd)) {
        q_bar[qi[i]] += dq * b->u[0];
        qd_bar[vi[i]] += dqd * b->u[0];
      }
    }
    for (int j = 0; j < nd; ++j)
      for (int r = 0; r < 6; ++r) {
        b->pA[r] -= Sv[6 * j + r] * b->u[j];
        b->S[6 * j + r] -= b->u[j] * l->pA[r];
      }
    /* D = S^T U */
    for (int j = 0; j < nd; ++j)
      for (int k = 0; k < nd; ++k)
        for (int r = 0; r < 6; ++r) {
          b->U[6 * k + r] += Sv[6 * j + r] * b->D[3 * j + k];
          b->S[6 * j + r] += b->D[3 * j + k] * l->U[6 * k + r];
        }
    /* U = IA S */
    for (int k = 0; k < nd; ++k)
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
          b->IA[6 * r + c] += b->U[6 * k + r] * Sv[6 * k + c];
          b->S[6 * k + c] += l->IA[6 * r + c] * b->U[6 * k + r];
        }
  }

  /* reverse of pass 1, leaves -> root */
  for (int i = n - 1; i >= 0; --i) {
    const tape_t *l = &L[i];
    link_bar *b = &B[i];
    const int lam = m->parent[i];
    /* pA(initial) = crf(v) h */
    double F[36], C[36];
    crf6_r(l->v, F);
    tvec_add(F, b->pA, b->h);
    crm6_r(b->pA, C);
    tvec_add(C, l->h, b->v);
    /* h = I v */
    tvec_add(l->Isp, b->h, b->v);
    /* the link's spatial inertia enters twice: IA = I + children's shares,
       and h = I v */
    if (param_bar) {
      double Ibar[36];
      for (int k = 0; k < 36; ++k) Ibar[k] = b->IA[k];
      outer_add(b->h, l->v, Ibar);
      inertia_params_add(Ibar, param_bar + 10 * i);
    }
    if (m->jtype[i] == ORC_FREE) {
      for (int k = 0; k < 6; ++k) qd_bar[vi[i] + k] += b->v[k];
      double Rbar[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Rbar[3 * r + c] = E0bar[3 * c + r];
      quat_R_grad(q + qi[i] + 3, Rbar, q_bar + qi[i] + 3);
      continue;
    }
    const double *ax = m->axis + 3 * i;
    /* c = crm(v) vJ */
    double CJ[36], CJt[36];
    crm6_r(l->vJ, CJ);
    mat6_transpose_r(CJ, CJt);
    for (int r = 0; r < 6; ++r)
      for (int k = 0; k < 6; ++k) b->v[r] -= CJt[6 * r + k] * b->c[k];
    crm6_r(l->v, C);
    tvec_add(C, b->c, b->vJ);
    /* v = X v_lam + vJ */
    if (lam >= 0) {
      tvec_add(l->X, b->v, B[lam].v);
      outer_add(b->v, L[lam].v, b->X);
    }
    for (int k = 0; k < 6; ++k) b->vJ[k] += b->v[k];
    /* vJ = S qd */
    const int nd = ndof_r(m, i);
    double Sv[18];
    motion_subspace_r(m, i, Sv);
    for (int k = 0; k < nd; ++k)
      for (int r = 0; r < 6; ++r) {
        qd_bar[vi[i] + k] += Sv[6 * k + r] * b->vJ[r];
        b->S[6 * k + r] += b->vJ[r] * qd[vi[i] + k];
      }
    /* X = XJ(q) XT.  Revolute: dX/dq = plucker(dEJ/dq, 0) XT with
       dEJ/dq = -cos q [a]x + sin q [a]x^2.  Prismatic: XJ = [I 0; -[q a]x I],
       dXJ/dq = [0 0; -[a]x 0].  Spherical: XJ = [E 0; 0 E], E = R(quat)^T,
       so XJ_bar = X_bar XT^T, E_bar = the sum of its diagonal blocks, and
       R_bar = E_bar^T goes to the quaternion. */
    if (m->jtype[i] == ORC_SPHERICAL) {
      double ET[9], rT[3], XT[36], XJb[36], Rbar[9];
      for (int k = 0; k < 9; ++k) ET[k] = m->E_T[9 * i + k];
      for (int k = 0; k < 3; ++k) rT[k] = m->r_T[3 * i + k];
      plucker_r(ET, rT, XT);
      for (int r = 0; r < 6; ++r)
        for (int c = 0; c < 6; ++c) {
          double s_ = 0;
          for (int k = 0; k < 6; ++k) s_ += b->X[6 * r + k] * XT[6 * c + k];
          XJb[6 * r + c] = s_;
        }
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Rbar[3 * c + r] = XJb[6 * r + c] + XJb[6 * (3 + r) + 3 + c];
      quat_R_grad(q + qi[i], Rbar, q_bar + qi[i]);
    } else {
      double axx[9], ax2[9], dE[9], zero3[3] = {0, 0, 0}, dXJ[36], XT[36], dX[36];
      double qq = q[qi[i]], s = sin(qq), c = cos(qq);
      skew3_r(ax, axx);
      if (m->jtype[i] == ORC_PRISMATIC) {
        for (int k = 0; k < 36; ++k) dXJ[k] = 0;
        for (int r = 0; r < 3; ++r)
          for (int cc = 0; cc < 3; ++cc) dXJ[6 * (3 + r) + cc] = -axx[3 * r + cc];
      } else {
        mat3_mul_r(axx, axx, ax2);
        for (int k = 0; k < 9; ++k) dE[k] = -c * axx[k] + s * ax2[k];
        plucker_r(dE, zero3, dXJ);
      }
      double ET[9], rT[3];
      for (int k = 0; k < 9; ++k) ET[k] = m->E_T[9 * i + k];
      for (int k = 0; k < 3; ++k) rT[k] = m->r_T[3 * i + k];
      plucker_r(ET, rT, XT);
      mat6_mul_r(dXJ, XT, dX);
      double sdot = 0;
      for (int k = 0; k < 36; ++k) sdot += b->X[k] * dX[k];
      q_bar[qi[i]] += sdot;
    }
    if (frame_bar) frame_params_add(m, i, q + qi[i], b->X, b->S, frame_bar + 9 * i);
  }
  free(B);
  return 0;
}

void orc_fd_vjp(const orc_model *m, const double *q, const double *qd,
                const double *tau, const double *qdd_bar, double *q_bar,
                double *qd_bar, double *tau_bar) {
  const int nv = orc_nv(m);
  tape_t *L = (tape_t *)malloc(sizeof(tape_t) * (size_t)m->n);
  double *qdd = (double *)malloc(sizeof(double) * (size_t)nv);
  aba_tape_r(m, q, qd, tau, L, qdd);
  aba_vjp(m, q, qd, L, qdd_bar, q_bar, qd_bar, tau_bar, NULL, NULL);
  free(qdd);
  free(L);
}

/* Adjoint of quat_step (orientation step by a body-frame angular velocity
 * w1): given the adjoint q1b of quat1, ADD into qtb (4) and w1b (3). */
static void quat_step_vjp(const double *qt, const double *w1, double dt, const double *q1b, double *qtb,
                          double *w1b) {
  double wq[4] = {w1[0], w1[1], w1[2], 0}, dq[4], qr[4], q1[4];
  quat_mul_r(qt, wq, dq);
  for (int k = 0; k < 4; ++k) qr[k] = qt[k] + 0.5 * dt * dq[k];
  const double nrm = sqrt(qr[0] * qr[0] + qr[1] * qr[1] + qr[2] * qr[2] + qr[3] * qr[3]);
  for (int k = 0; k < 4; ++k) q1[k] = qr[k] / nrm;
  /* quat1 = qr / |qr| */
  double dotq = 0, ob[4];
  for (int k = 0; k < 4; ++k) dotq += q1[k] * q1b[k];
  for (int k = 0; k < 4; ++k) ob[k] = (q1b[k] - q1[k] * dotq) / nrm;
  /* qr = qt + dt/2 * qt (x) (w1, 0):  o_v = qt_w w1 + qt_v x w1, o_w = -qt_v . w1 */
  const double h = 0.5 * dt;
  for (int k = 0; k < 4; ++k) qtb[k] += ob[k];
  const double cr[3] = {w1[1] * ob[2] - w1[2] * ob[1], w1[2] * ob[0] - w1[0] * ob[2],
                        w1[0] * ob[1] - w1[1] * ob[0]}; /* w1 x ob_v */
  for (int k = 0; k < 3; ++k) qtb[k] += h * (cr[k] - w1[k] * ob[3]);
  qtb[3] += h * (w1[0] * ob[0] + w1[1] * ob[1] + w1[2] * ob[2]);
  const double axo[3] = {qt[1] * ob[2] - qt[2] * ob[1], qt[2] * ob[0] - qt[0] * ob[2],
                         qt[0] * ob[1] - qt[1] * ob[0]}; /* qt_v x ob_v */
  for (int k = 0; k < 3; ++k) w1b[k] += h * (qt[3] * ob[k] - axo[k] - qt[k] * ob[3]);
}

/* Adjoint of one semi-implicit Euler step taken from x^t = (q, qd) with
 * forward intermediates L and accelerations qdd.  Input (q1bar, qd1bar) is
 * the adjoint of x^{t+1}; output (qbar, qdbar) is the adjoint of x^t and
 * taubar the adjoint of u^t (all overwritten). */
static int step_vjp(const orc_model *m, const double *q, const double *qd,
                    const double *qdd, const tape_t *L, double dt,
                    const double *q1bar, const double *qd1bar, double *qbar,
                    double *qdbar, double *taubar, double *qddbar, double *pbar, double *fbar) {
  const int n = m->n, nu = orc_nu(m);
  int qi[n], vi[n], ui[n];
  layout_r(m, qi, vi, ui);
  for (int k = 0; k < nu; ++k) taubar[k] = 0;
  for (int i = 0; i < n; ++i) {
    if (m->jtype[i] == ORC_FREE) {
      const double *p = q + qi[i], *qt = q + qi[i] + 3;
      (void)p;
      double v1[6];
      for (int k = 0; k < 6; ++k) v1[k] = qd[vi[i] + k] + dt * qdd[vi[i] + k];
      double R[9];
      quat_R_r(qt, R);
      double *qtb = qbar + qi[i] + 3;
      for (int k = 0; k < 4; ++k) qtb[k] = 0;
      double v1bar[6];
      for (int k = 0; k < 6; ++k) v1bar[k] = qd1bar[vi[i] + k];
      quat_step_vjp(qt, v1, dt, q1bar + qi[i] + 3, qtb, v1bar);
      /* p1 = p + dt R(qt) v1_lin */
      const double *p1b = q1bar + qi[i];
      for (int k = 0; k < 3; ++k) qbar[qi[i] + k] = p1b[k];
      double Rbar[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Rbar[3 * r + c] = dt * p1b[r] * v1[3 + c];
      quat_R_grad(qt, Rbar, qtb);
      for (int c = 0; c < 3; ++c)
        for (int r = 0; r < 3; ++r) v1bar[3 + c] += dt * R[3 * r + c] * p1b[r];
      /* v1 = v + dt qdd */
      for (int k = 0; k < 6; ++k) {
        qdbar[vi[i] + k] = v1bar[k];
        qddbar[vi[i] + k] = dt * v1bar[k];
      }
    } else if (m->jtype[i] == ORC_SPHERICAL) {
      /* w1 = w + dt wdot; quat1 = quat_step(quat, w1) */
      const double *qt = q + qi[i];
      double w1[3], w1bar[3];
      for (int k = 0; k < 3; ++k) {
        w1[k] = qd[vi[i] + k] + dt * qdd[vi[i] + k];
        w1bar[k] = qd1bar[vi[i] + k];
        qbar[qi[i] + k] = 0;
      }
      qbar[qi[i] + 3] = 0;
      quat_step_vjp(qt, w1, dt, q1bar + qi[i], qbar + qi[i], w1bar);
      for (int k = 0; k < 3; ++k) {
        qdbar[vi[i] + k] = w1bar[k];
        qddbar[vi[i] + k] = dt * w1bar[k];
      }
    } else {
      const double tot = qd1bar[vi[i]] + dt * q1bar[qi[i]];
      qddbar[vi[i]] = dt * tot;
      qbar[qi[i]] = q1bar[qi[i]];
      qdbar[vi[i]] = tot;
    }
  }
  return aba_vjp(m, q, qd, L, qddbar, qbar, qdbar, taubar, pbar, fbar);
}

static void tape_qdd(const orc_model *m, const tape_t *L, double *qdd) {
  const int n = m->n;
  int qi[n], vi[n], ui[n];
  layout_r(m, qi, vi, ui);
  for (int i = 0; i < n; ++i) {
    if (m->jtype[i] == ORC_FREE)
      for (int k = 0; k < 6; ++k) qdd[vi[i] + k] = L[i].abase[k];
    else
      for (int k = 0; k < ndof_r(m, i); ++k) qdd[vi[i] + k] = L[i].qdd[k];
  }
}

int orc_rollout_grad_params(const orc_model *m, const double *q0, const double *qd0,
                            const double *tau, double dt, int T, int K,
                            const double *gqT, const double *gqdT,
                            const double *gtraj, double *gq0, double *gqd0,
                            double *gtau, double *gparam, double *gframe, double *qT, double *qdT) {
  if (T < 0 || K < 0) return -1;
  if (gparam)
    for (int k = 0; k < 10 * m->n; ++k) gparam[k] = 0;
  if (gframe)
    for (int k = 0; k < 9 * m->n; ++k) gframe[k] = 0;
  const int n = m->n, nq = orc_nq(m), nv = orc_nv(m), nu = orc_nu(m);
  const int nx = nq + nv;
  const int ncp = (K >= 1) ? (T + K - 1) / K : 0;
  double *ck = NULL, *scratch = NULL, *states = NULL;
  tape_t *tapes = NULL;
  tape_t *tape = (tape_t *)malloc(sizeof(tape_t) * (size_t)n);
  double *work = (double *)malloc(sizeof(double) * (size_t)(4 * nx + 3 * nv));
  if (K >= 1) {
    ck = (double *)malloc(sizeof(double) * (size_t)(ncp > 0 ? ncp : 1) * nx);
    scratch = (double *)malloc(sizeof(double) * (size_t)K * nx);
  } else {
    states = (double *)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1) * nx);
    tapes = (tape_t *)malloc(sizeof(tape_t) * (size_t)(T > 0 ? T : 1) * n);
  }
  if (!tape || !work || (K >= 1 && (!ck || !scratch)) || (K == 0 && (!states || !tapes))) {
    free(tape); free(work); free(ck); free(scratch); free(states); free(tapes);
    return -1;
  }
  double *x = work, *x1 = x + nx, *xb = x1 + nx, *xb1 = xb + nx;
  double *qdd = xb1 + nx, *qddbar = qdd + nv, *spare = qddbar + nv;
  (void)spare;

  /* forward sweep: store x^t at every K-th step (or every intermediate) */
  memcpy(x, q0, sizeof(double) * nq);
  memcpy(x + nq, qd0, sizeof(double) * nv);
  for (int t = 0; t < T; ++t) {
    if (K >= 1 && t % K == 0) memcpy(ck + (size_t)(t / K) * nx, x, sizeof(double) * nx);
    tape_t *Lt = tape;
    if (K == 0) {
      memcpy(states + (size_t)t * nx, x, sizeof(double) * nx);
      Lt = tapes + (size_t)t * n;
    }
    aba_tape_r(m, x, x + nq, tau + (size_t)t * nu, Lt, qdd);
    integrate_r(m, x, x + nq, qdd, dt, x1, x1 + nq);
    memcpy(x, x1, sizeof(double) * nx);
  }
  if (qT) memcpy(qT, x, sizeof(double) * nq);
  if (qdT) memcpy(qdT, x + nq, sizeof(double) * nv);

  /* reverse sweep */
  memcpy(xb, gqT, sizeof(double) * nq);
  memcpy(xb + nq, gqdT, sizeof(double) * nv);
  if (gtraj && T > 0)
    for (int k = 0; k < nx; ++k) xb[k] += gtraj[(size_t)(T - 1) * nx + k];

  int rc = 0;
  if (K >= 1) {
    for (int s = ncp - 1; s >= 0 && rc == 0; --s) {
      const int t0 = s * K;
      const int t1 = (t0 + K < T) ? t0 + K : T;
      /* replay the segment from its checkpoint */
      memcpy(scratch, ck + (size_t)s * nx, sizeof(double) * nx);
      for (int j = 1; j < t1 - t0; ++j) {
        const double *xp = scratch + (size_t)(j - 1) * nx;
        double *xn = scratch + (size_t)j * nx;
        aba_tape_r(m, xp, xp + nq, tau + (size_t)(t0 + j - 1) * nu, tape, qdd);
        integrate_r(m, xp, xp + nq, qdd, dt, xn, xn + nq);
      }
      for (int t = t1 - 1; t >= t0 && rc == 0; --t) {
        const double *xt = scratch + (size_t)(t - t0) * nx;
        aba_tape_r(m, xt, xt + nq, tau + (size_t)t * nu, tape, qdd);
        rc = step_vjp(m, xt, xt + nq, qdd, tape, dt, xb, xb + nq, xb1, xb1 + nq,
                      gtau + (size_t)t * nu, qddbar, gparam, gframe);
        memcpy(xb, xb1, sizeof(double) * nx);
        if (gtraj && t >= 1)
          for (int k = 0; k < nx; ++k) xb[k] += gtraj[(size_t)(t - 1) * nx + k];
      }
    }
  } else {
    for (int t = T - 1; t >= 0 && rc == 0; --t) {
      const double *xt = states + (size_t)t * nx;
      const tape_t *Lt = tapes + (size_t)t * n;
      tape_qdd(m, Lt, qdd);
      rc = step_vjp(m, xt, xt + nq, qdd, Lt, dt, xb, xb + nq, xb1, xb1 + nq,
                    gtau + (size_t)t * nu, qddbar, gparam, gframe);
      memcpy(xb, xb1, sizeof(double) * nx);
      if (gtraj && t >= 1)
        for (int k = 0; k < nx; ++k) xb[k] += gtraj[(size_t)(t - 1) * nx + k];
    }
  }
  memcpy(gq0, xb, sizeof(double) * nq);
  memcpy(gqd0, xb + nq, sizeof(double) * nv);

  free(tape); free(work); free(ck); free(scratch); free(states); free(tapes);
  return rc;
}

int orc_rollout_grad(const orc_model *m, const double *q0, const double *qd0,
                     const double *tau, double dt, int T, int K,
                     const double *gqT, const double *gqdT,
                     const double *gtraj, double *gq0, double *gqd0,
                     double *gtau, double *qT, double *qdT) {
  return orc_rollout_grad_params(m, q0, qd0, tau, dt, T, K, gqT, gqdT, gtraj, gq0, gqd0, gtau, NULL,
                                 NULL, qT, qdT);
}

int orc_adjoint_along_params(const orc_model *m, const double *states, const double *tau,
                             double dt, int T, const double *gqT, const double *gqdT,
                             const double *gtraj, double *gq0, double *gqd0, double *gtau,
                             double *gparam, double *gframe) {
  if (T < 0) return -1;
  if (gparam)
    for (int k = 0; k < 10 * m->n; ++k) gparam[k] = 0;
  if (gframe)
    for (int k = 0; k < 9 * m->n; ++k) gframe[k] = 0;
  const int n = m->n, nq = orc_nq(m), nv = orc_nv(m), nu = orc_nu(m);
  const int nx = nq + nv;
  tape_t *tape = (tape_t *)malloc(sizeof(tape_t) * (size_t)n);
  double *work = (double *)malloc(sizeof(double) * (size_t)(2 * nx + 2 * nv));
  if (!tape || !work) { free(tape); free(work); return -1; }
  double *xb = work, *xb1 = xb + nx, *qdd = xb1 + nx, *qddbar = qdd + nv;
  memcpy(xb, gqT, sizeof(double) * nq);
  memcpy(xb + nq, gqdT, sizeof(double) * nv);
  if (gtraj && T > 0)
    for (int k = 0; k < nx; ++k) xb[k] += gtraj[(size_t)(T - 1) * nx + k];
  int rc = 0;
  /* the given states play the role of per-step checkpoints (Sec. 4.2) */
  for (int t = T - 1; t >= 0 && rc == 0; --t) {
    const double *xt = states + (size_t)t * nx;
    aba_tape_r(m, xt, xt + nq, tau + (size_t)t * nu, tape, qdd);
    rc = step_vjp(m, xt, xt + nq, qdd, tape, dt, xb, xb + nq, xb1, xb1 + nq,
                  gtau + (size_t)t * nu, qddbar, gparam, gframe);
    memcpy(xb, xb1, sizeof(double) * nx);
    if (gtraj && t >= 1)
      for (int k = 0; k < nx; ++k) xb[k] += gtraj[(size_t)(t - 1) * nx + k];
  }
  memcpy(gq0, xb, sizeof(double) * nq);
  memcpy(gqd0, xb + nq, sizeof(double) * nv);
  free(tape);
  free(work);
  return rc;
}

int orc_adjoint_along(const orc_model *m, const double *states, const double *tau,
                      double dt, int T, const double *gqT, const double *gqdT,
                      const double *gtraj, double *gq0, double *gqd0, double *gtau) {
  return orc_adjoint_along_params(m, states, tau, dt, T, gqT, gqdT, gtraj, gq0, gqd0, gtau, NULL, NULL);
}

/* ---- contact (contact.inc) --------------------------------------------- */

int orc_contact_assembly(const orc_model *m, const orc_contacts *C, const double *q, int *act, double *phi,
                         double *J, double *MJ) {
  return contact_assembly_r(m, C, q, act, phi, J, MJ);
}

int orc_step_contact(const orc_model *m, const orc_contacts *C, const double *q, const double *qd,
                     const double *tau, double dt, double *q1, double *qd1, double *lam) {
  return step_contact_r(m, C, q, qd, tau, dt, q1, qd1, lam);
}

int orc_step_contact_c(const orc_model *m, const orc_contacts *C, const void *q, const void *qd, const void *tau,
                       double dt, void *q1, void *qd1) {
  return step_contact_c(m, C, (const double complex *)q, (const double complex *)qd,
                        (const double complex *)tau, dt, (double complex *)q1, (double complex *)qd1, NULL);
}

int orc_rollout_contact(const orc_model *m, const orc_contacts *C, const double *q0, const double *qd0,
                        const double *tau, double dt, int T, double *qT, double *qdT, double *traj, int *n_contacts) {
  if (T < 0) return -1;
  const int nq = orc_nq(m), nv = orc_nv(m), nu = orc_nu(m);
  double *x = (double *)malloc(sizeof(double) * (size_t)(2 * (nq + nv)));
  if (!x) return -1;
  double *x1 = x + nq + nv;
  memcpy(x, q0, sizeof(double) * nq);
  memcpy(x + nq, qd0, sizeof(double) * nv);
  for (int t = 0; t < T; ++t) {
    const int na = step_contact_r(m, C, x, x + nq, tau + (size_t)t * nu, dt, x1, x1 + nq, NULL);
    if (n_contacts) n_contacts[t] = na;
    memcpy(x, x1, sizeof(double) * (nq + nv));
    if (traj) memcpy(traj + (size_t)t * (nq + nv), x, sizeof(double) * (nq + nv));
  }
  memcpy(qT, x, sizeof(double) * nq);
  memcpy(qdT, x + nq, sizeof(double) * nv);
  free(x);
  return 0;
}

/* Gradient of a loss on the final state through a rollout with contact:
 * the step map's exact derivative (complex step, h = 1e-30, one input
 * direction at a time, at the stored states) applied in reverse time
 * (Eq. adj_r).  Valid where no contact switches on or off and no solver
 * bound changes activity under an infinitesimal change, i.e. away from the
 * kinks of the piecewise-smooth step map. */
int orc_rollout_contact_grad(const orc_model *m, const orc_contacts *C, const double *q0, const double *qd0,
                             const double *tau, double dt, int T, const double *gqT, const double *gqdT,
                             double *gq0, double *gqd0, double *gtau, double *gmu) {
  if (T < 0) return -1;
  const int nq = orc_nq(m), nv = orc_nv(m), nu = orc_nu(m), nx = nq + nv;
  double *xs = (double *)malloc(sizeof(double) * (size_t)(T + 1) * nx);
  double complex *xc = (double complex *)malloc(sizeof(double complex) * (size_t)(nx + nu));
  double *xb = (double *)malloc(sizeof(double) * (size_t)(2 * nx));
  if (!xs || !xc || !xb) { free(xs); free(xc); free(xb); return -1; }
  memcpy(xs, q0, sizeof(double) * nq);
  memcpy(xs + nq, qd0, sizeof(double) * nv);
  for (int t = 0; t < T; ++t) {
    double *cur = xs + (size_t)t * nx, *nxt = cur + nx;
    step_contact_r(m, C, cur, cur + nq, tau + (size_t)t * nu, dt, nxt, nxt + nq, NULL);
  }
  double *xb1 = xb + nx;
  memcpy(xb, gqT, sizeof(double) * nq);
  memcpy(xb + nq, gqdT, sizeof(double) * nv);
  const double h = 1e-30;
  double complex *in = xc, *uc = xc + nx;
  double complex out1[nx];
  double mu_acc = 0;
  for (int t = T - 1; t >= 0; --t) {
    const double *cur = xs + (size_t)t * nx;
    for (int j = 0; j < nx + nu; ++j) {
      for (int k = 0; k < nx; ++k) in[k] = cur[k];
      for (int k = 0; k < nu; ++k) uc[k] = tau[(size_t)t * nu + k];
      if (j < nx) in[j] += I * h;
      else uc[j - nx] += I * h;
      step_contact_c(m, C, in, in + nq, uc, dt, out1, out1 + nq, NULL);
      double s = 0;
      for (int k = 0; k < nx; ++k) s += xb[k] * cimag(out1[k]) / h;
      if (j < nx) xb1[j] = s;
      else gtau[(size_t)t * nu + (j - nx)] = s;
    }
    if (gmu) {
      /* the friction coefficient's column of this step's Jacobian */
      for (int k = 0; k < nx; ++k) in[k] = cur[k];
      for (int k = 0; k < nu; ++k) uc[k] = tau[(size_t)t * nu + k];
      step_contact_mu_c(m, C, in, in + nq, uc, dt, C->mu + I * h, out1, out1 + nq, NULL);
      double s = 0;
      for (int k = 0; k < nx; ++k) s += xb[k] * cimag(out1[k]) / h;
      mu_acc += s;
    }
    memcpy(xb, xb1, sizeof(double) * nx);
  }
  if (gmu) *gmu = mu_acc;
  memcpy(gq0, xb, sizeof(double) * nq);
  memcpy(gqd0, xb + nq, sizeof(double) * nv);
  free(xs); free(xc); free(xb);
  return 0;
}
