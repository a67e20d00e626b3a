/*
 * Plain FP64 CPU oracle for articulated-body forward dynamics (ABA),
 * semi-implicit Euler time stepping and the reverse-time adjoint with
 * per-step checkpointing.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  It shares no code, header, table or helper with the GPU
 * library; the two meet only through plain arrays produced by the seeded
 * input generators.
 *
 * Everything is written with dense 6x6 matrices and plain loops, in the
 * order the method states it, so that it can be read against the paper:
 *   - state x = [q, qdot], control u per step           (Sec. 3, "Articulated
 *                                                         body dynamics")
 *   - ABA, three traversals root->leaf, leaf->root,
 *     root->leaf                                         (Sec. 3; Fig. 1;
 *                                                         Sec. 4.1, five modules)
 *   - adjoint recursion R^k through time                 (Sec. 3, Eq. adj_back;
 *                                                         Sec. 4.1, Eq. adj_r)
 *   - store the initial state of each step, recompute
 *     the step's intermediates during backpropagation    (Sec. 4.2,
 *                                                         Eq. intermediate)
 *   - checkpoint interval k                              (App. B)
 *
 * Conventions (the paper states none; see the readings listed in the design
 * notes): Featherstone Plucker transforms X = [E 0; -E[r]x E] from parent to
 * child coordinates, motion vectors [w; v], force vectors [n; f], revolute
 * joint about a unit axis a with E_J(q) = I - sin q [a]x + (1 - cos q)[a]x^2,
 * gravity entered as a fictitious base acceleration.
 *
 * Prismatic joint (type 2): the link slides by q along the unit axis a of
 * the joint frame, X_J(q) = [I 0; -[q a]x I], motion subspace S = [0; a].
 *
 * Spherical joint (type 3): a ball joint at the joint frame's origin.
 * q = quat[4] (x, y, z, w) of the link frame relative to the joint frame,
 * velocity = the link's angular velocity relative to its parent in link
 * coordinates (3), control = the joint torque in link coordinates (3);
 * X_J = [E 0; 0 E] with E = R(quat)^T, motion subspace S = [1; 0] (6x3).
 *
 * Free-floating root (joint type 1, only at link 0): q = (p_world[3],
 * quat[4] stored x,y,z,w), velocity = body-frame spatial velocity [w_b; v_b].
 * The root is unactuated; tau holds one entry per revolute or prismatic
 * joint.
 */
#ifndef ABA_ORACLE_H
#define ABA_ORACLE_H

#include <stddef.h>

#define ORC_REVOLUTE 0
#define ORC_FREE 1
#define ORC_PRISMATIC 2
#define ORC_SPHERICAL 3

typedef struct {
  int n;                 /* number of links */
  const int *parent;     /* parent[i] < i; -1 = attached to the fixed base
                            (or, for a free root, no parent)               */
  const int *jtype;      /* ORC_REVOLUTE, ORC_PRISMATIC, ORC_SPHERICAL, or
                            ORC_FREE (link 0 only)                         */
  const double *E_T;     /* 9n: fixed rotation parent->joint frame, rowmajor */
  const double *r_T;     /* 3n: joint origin in parent coordinates          */
  const double *axis;    /* 3n: joint axis in the link frame, unit length
                            (the Python wrapper normalises it)             */
  const double *mass;    /* n                                               */
  const double *com;     /* 3n: centre of mass in the link frame            */
  const double *Ic;      /* 6n: inertia about the COM: xx yy zz xy xz yz    */
  const double *gravity; /* 3                                               */
  const double *limits;  /* nullable [n][4]: joint limits lo, hi and the
                            stiffness k and damping d of the one-sided
                            spring-damper that acts outside [lo, hi]:
                            tau_l = -k (q - hi) - d qd above hi,
                            -k (q - lo) - d qd below lo, added to the
                            joint's control (1-dof joints only)           */
} orc_model;

#ifdef __cplusplus
extern "C" {
#endif

int orc_nq(const orc_model *m);
int orc_nv(const orc_model *m);
int orc_nu(const orc_model *m);

/* Forward dynamics qdd = FD(q, qd, tau).  For a free root the first six
 * entries of qdd are the body-frame spatial acceleration of the root. */
void orc_fd(const orc_model *m, const double *q, const double *qd,
            const double *tau, double *qdd);
/* Same, complex-valued (used for complex-step derivative checks). */
void orc_fd_c(const orc_model *m, const void *q, const void *qd,
              const void *tau, void *qdd);

/* Reverse mode of one forward-dynamics evaluation: given qdd_bar, ADD
 * d<qdd_bar, qdd>/d(q, qd, tau) into q_bar, qd_bar, tau_bar. */
void orc_fd_vjp(const orc_model *m, const double *q, const double *qd,
                const double *tau, const double *qdd_bar, double *q_bar,
                double *qd_bar, double *tau_bar);

/* One semi-implicit Euler step. */
void orc_step(const orc_model *m, const double *q, const double *qd,
              const double *tau, double dt, double *q1, double *qd1);

/* T-step rollout.  tau is [T][nu].  traj (nullable) is [T][nq + nv]:
 * traj[t] = (q^{t+1}, qd^{t+1}). */
int orc_rollout(const orc_model *m, const double *q0, const double *qd0,
                const double *tau, double dt, int T, double *qT, double *qdT,
                double *traj);
int orc_rollout_c(const orc_model *m, const void *q0, const void *qd0,
                  const void *tau, double dt, int T, void *qT, void *qdT);

/* Gradient of a loss L(x^T, traj) through a T-step rollout by the adjoint
 * method.  K >= 1: store the state every K steps and recompute during the
 * reverse sweep; K == 0: store every step's intermediates (no recompute).
 * gtraj may be NULL.  Outputs are overwritten.  qT/qdT (nullable) receive
 * the final state.  Returns 0 on success, -1 on allocation failure or bad
 * arguments. */
int orc_rollout_grad(const orc_model *m, const double *q0, const double *qd0,
                     const double *tau, double dt, int T, int K,
                     const double *gqT, const double *gqdT,
                     const double *gtraj, double *gq0, double *gqd0,
                     double *gtau, double *qT, double *qdT);

/* As orc_rollout_grad, and also gradients with respect to model
 * parameters, summed over all steps (each output nullable).  Sec. 4.1,
 * after Eq. adj_r: the gradient of any other parameter follows from the same
 * per-step adjoints as the control gradient; Sec. 6.3 (parameter
 * estimation).
 *   gparam [n][10]: every link's ten inertial parameters (m, h_x, h_y, h_z,
 *     I_xx, I_yy, I_zz, I_xy, I_xz, I_yz) with h = m c the first moment and
 *     I the rotational inertia about the link origin (I_c - m [c]x^2), all
 *     in the link frame; an off-diagonal parameter stands for both of its
 *     matrix entries.
 *   gframe [n][9]: every 1-dof link's placement and axis (zero for a free
 *     root): (phi_bar[3], r_T_bar[3], axis_bar[3]).  phi: rotation of the
 *     joint frame, E_T -> exp(-[phi]x) E_T, phi in joint-frame coordinates;
 *     r_T_bar: the gradient with respect to r_T (parent coordinates);
 *     axis_bar: the gradient with respect to the axis vector along the unit
 *     sphere (link coordinates, orthogonal to the axis): a change da
 *     orthogonal to the axis changes the loss by axis_bar . da. */
int orc_rollout_grad_params(const orc_model *m, const double *q0, const double *qd0,
                            const double *tau, double dt, int T, int K,
                            const double *gqT, const double *gqdT,
                            const double *gtraj, double *gq0, double *gqd0,
                            double *gtau, double *gparam, double *gframe, double *qT, double *qdT);

/* The reverse sweep alone, along a given trajectory: states is [T][nq + nv]
 * with row t = x^t (the initial state of step t), used as the per-step
 * checkpoints; seeds and outputs as orc_rollout_grad. */
int orc_adjoint_along(const orc_model *m, const double *states, const double *tau,
                      double dt, int T, const double *gqT, const double *gqdT,
                      const double *gtraj, double *gq0, double *gqd0, double *gtau);
int orc_adjoint_along_params(const orc_model *m, const double *states, const double *tau,
                             double dt, int T, const double *gqT, const double *gqdT,
                             const double *gtraj, double *gq0, double *gqd0, double *gtau,
                             double *gparam, double *gframe);

/* ---- contact resolution inside a step (contact.inc) -----------------
 * Contact spheres against the ground plane y = 0 (see contact.inc for the
 * model): link[k], centre[k][3] in link coordinates, radius[k]; box
 * friction coefficient mu; Baumgarte factor beta on the gap; PGS sweeps
 * niter for each of the two solves. */
typedef struct {
  int n;
  const int *link;
  const double *center;
  const double *radius;
  double mu, beta;
  int niter;
} orc_contacts;

/* Detection and assembly at q: active contacts act[], gaps phi[], J
 * ([3m][nv], rows normal e_y, tangents e_x, e_z per contact) and M^-1 J^T
 * ([nv][3m]); returns m.  Arrays sized for C->n contacts. */
int orc_contact_assembly(const orc_model *m, const orc_contacts *C, const double *q, int *act, double *phi,
                         double *J, double *MJ);
/* One step with contact resolution; returns the number of active contacts,
 * lam (nullable, [3 C->n]) their impulses.  _c: complex inputs. */
int orc_step_contact(const orc_model *m, const orc_contacts *C, const double *q, const double *qd,
                     const double *tau, double dt, double *q1, double *qd1, double *lam);
int orc_step_contact_c(const orc_model *m, const orc_contacts *C, const void *q, const void *qd, const void *tau,
                       double dt, void *q1, void *qd1);
/* Rollout with contact (traj, n_contacts nullable: [T][nq+nv], [T]). */
int orc_rollout_contact(const orc_model *m, const orc_contacts *C, const double *q0, const double *qd0,
                        const double *tau, double dt, int T, double *qT, double *qdT, double *traj, int *n_contacts);
/* Gradient of <gqT, qT> + <gqdT, qdT> through a rollout with contact (the
 * step map's exact derivative by complex step, in reverse time); gmu
 * (nullable) receives the derivative with respect to the friction
 * coefficient mu. */
int orc_rollout_contact_grad(const orc_model *m, const orc_contacts *C, const double *q0, const double *qd0,
                             const double *tau, double dt, int T, const double *gqT, const double *gqdT,
                             double *gq0, double *gqd0, double *gtau, double *gmu);

/* ---- contact solver (pgs_oracle.c) ---------------------------------
 * Projected Gauss-Seidel on the MLCP a = A x + b, lo <= x <= hi (Sec. 4.1,
 * Eq. mlcp; App. C), n rows, niter sweeps from x0; A is [n][n] row-major.
 * sweeps (nullable) [niter + 1][n] receives x at the start of every sweep
 * and the result.  orc_pgs_adjoint reverses the solve from those stored
 * vectors: given x_bar it returns A_bar [n][n], b_bar, lo_bar, hi_bar and
 * x0_bar [n] (overwritten).  orc_pgs_solve_c: the solve in complex
 * arithmetic (inputs and output double complex), for complex-step checks. */
void orc_pgs_solve(int n, int niter, const double *A, const double *b, const double *lo,
                   const double *hi, const double *x0, double *x, double *sweeps);
void orc_pgs_solve_c(int n, int niter, const void *A, const void *b, const void *lo,
                     const void *hi, const void *x0, void *x);
void orc_pgs_adjoint(int n, int niter, const double *A, const double *b, const double *lo,
                     const double *hi, const double *sweeps, const double *xbar, double *Abar,
                     double *bbar, double *lobar, double *hibar, double *x0bar);

#ifdef __cplusplus
}
#endif

#endif
