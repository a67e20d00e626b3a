/*
 * abadj -- batched differentiable articulated-body dynamics on AMD MI355X
 * (gfx950): forward dynamics by the Articulated Body Algorithm, semi-implicit
 * Euler time stepping, and the reverse-time adjoint that stores only each
 * step's initial state and recomputes the step's intermediates.
 *
 * Method references (Qiao, Liang, Koltun, Lin, "Efficient Differentiable
 * Simulation of Articulated Bodies", ICML 2021):
 *   - state x = [q, qdot], one control u per step      Sec. 3, "Articulated
 *                                                       body dynamics"
 *   - ABA, three tree traversals                        Sec. 3; Fig. 1;
 *                                                       Sec. 4.1 (modules)
 *   - adjoint recursion through time                    Sec. 3, Eq. adj_back;
 *                                                       Sec. 4.1, Eq. adj_r
 *   - checkpoint the initial state of each step,
 *     recompute intermediates in the backward pass      Sec. 4.2, Eq.
 *                                                       intermediate; Fig. 2
 *   - checkpoint interval K                             App. B
 *
 * Conventions
 *   - Links of a system are given in topological order (parent < child).
 *     parent = -1 attaches a link to the fixed base; a free-floating root
 *     (joint type SIM_JOINT_FREE) is allowed only at local index 0, with
 *     parent -1, and then every other link of that system has a parent.
 *   - Plucker transform parent -> link: X = [E 0; -E[r]x E] with
 *     revolute joint (motion subspace S = [a; 0]):
 *       E = E_J(q) E_T, E_J(q) = I - sin q [a]x + (1 - cos q)[a]x^2, r = r_T;
 *     prismatic joint (S = [0; a], translation by q a in link coordinates):
 *       E = E_T, r = r_T + q E_T^T a.
 *     Both are X = X_J(q) X_T with X_J(q) = exp(-q crm(S))   (Sec. 3; the
 *     joint models of Featherstone's spatial algebra, which Sec. 3 follows).
 *     Spherical (ball) joint (S = [1; 0], the link frame's three angular
 *     unit vectors): E = R(quat)^T E_T, r = r_T, with
 *     R(quat) = (w^2 - u.u) I + 2 u u^T + 2 w [u]x for quat = (u, w)
 *     (the quaternion operators of App. G).  It has no axis (its axis entry
 *     is not read) and no joint limits.
 *   - Revolute or prismatic joint: one q, one qdot, one control (torque or
 *     force).  Spherical joint: q = quat[4] stored x, y, z, w, qdot = the
 *     joint's angular velocity in link coordinates (3), three torques (link
 *     coordinates).  Free root:
 *     q = (p_world[3], quat[4] stored x, y, z, w), velocity = body-frame
 *     spatial velocity [w; v] (6 entries), unactuated.
 *   - Gravity enters as a fictitious base acceleration; for a free root the
 *     base acceleration reported is the true body-frame acceleration.
 *   - Semi-implicit Euler: qd1 = qd + dt qdd, q1 = q + dt qd1; free root:
 *     p1 = p + dt R(quat) v1_lin, quat1 = normalize(quat + dt/2 quat x (w1, 0));
 *     spherical joint: w1 = w + dt wdot, quat1 as for the free root.
 *   - Gradients with respect to a spherical joint's quaternion are the
 *     gradient along the unit sphere (orthogonal to the quaternion): the
 *     radial part depends only on how the step is continued off the sphere
 *     and is removed by the next step's normalisation anyway.
 *   - Batched vectors are system-concatenated in the order of the
 *     topology: q [sum nq], qd [sum nv], control rows [sum nu]; a control
 *     sequence is [T][sum nu], a trajectory [T][sum nq + sum nv] whose row t
 *     holds (q^{t+1}, qd^{t+1}) (all q first, then all qd).
 *
 * Memory and streams
 *   - Host pointers are marked "host"; all others are DEVICE pointers,
 *     owned by the caller, of the handle's dtype (float for SIM_F32,
 *     double for SIM_F64), contiguous.
 *   - The handle owns only its packed per-link constants (device memory
 *     allocated by sim_create, freed by sim_destroy).
 *   - sim_forward / sim_backward / sim_aba only enqueue work on `stream`
 *     (a hipStream_t; NULL = the default stream).  They never synchronise
 *     and never memset, so they may be captured into a HIP graph; they
 *     allocate nothing, except sim_backward's first call with a new binomial
 *     schedule (K < 0, below).  Scratch memory is the caller's workspace.
 *
 * Errors: every entry point returns SIM_OK (0) or a negative code; no C++
 * exception crosses the ABI.  sim_last_error() returns a thread-local
 * description of the last failure on the calling thread.
 */
#ifndef ABADJ_H
#define ABADJ_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SIM_OK 0
#define SIM_ERR_INVALID_ARG (-1)
#define SIM_ERR_INVALID_TOPOLOGY (-2)
#define SIM_ERR_WORKSPACE_TOO_SMALL (-3)
#define SIM_ERR_UNSUPPORTED_DTYPE (-4)
#define SIM_ERR_HIP (-5)

#define SIM_F32 0
#define SIM_F64 1

#define SIM_JOINT_REVOLUTE 0
#define SIM_JOINT_FREE 1
#define SIM_JOINT_PRISMATIC 2
#define SIM_JOINT_SPHERICAL 3

/* Largest number of links in one system (one wavefront of 64 lanes). */
#define SIM_MAX_LINKS 64

typedef struct sim_handle *sim_t;

/* Tree structure of a batch of independent systems (host arrays). */
typedef struct {
  int32_t n_sys;               /* number of systems, >= 1                 */
  const int32_t *link_offset;  /* [n_sys + 1], links of system s are
                                  link_offset[s] .. link_offset[s+1]-1    */
  const int32_t *parent;       /* [n_links] local parent index, -1 = base */
  const int32_t *jtype;        /* [n_links] SIM_JOINT_*                   */
} sim_topology;

/* Per-link model parameters (host arrays, double precision). */
typedef struct {
  const double *E_T;      /* [9 n_links] row-major rotation parent->joint   */
  const double *r_T;      /* [3 n_links] joint origin, parent coordinates   */
  const double *axis;     /* [3 n_links] unit joint axis, link coordinates  */
  const double *mass;     /* [n_links] > 0                                  */
  const double *com;      /* [3 n_links] centre of mass, link coordinates   */
  const double *Ic;       /* [6 n_links] inertia about the COM:
                             xx yy zz xy xz yz                              */
  const double *gravity;  /* [3] e.g. (0, -9.81, 0)                         */
  const double *limits;   /* nullable [4 n_links]: joint limits (lo, hi, k, d)
                             per link; outside [lo, hi] a one-sided spring
                             and damper adds tau_l = -k (q - hi) - d qd
                             (above hi) or -k (q - lo) - d qd (below lo) to
                             the joint's control; ignored for a free root.
                             Finite, lo <= hi, k >= 0, d >= 0; an unlimited
                             joint takes lo, hi = -+1e30 (or k = d = 0).
                             The paper names joint limits without a model
                             (Sec. 2); this is the model used.            */
} sim_params;

typedef struct {
  int32_t n_sys, n_links;
  int32_t nq, nv, nu;     /* totals over the batch                        */
  int32_t n_waves;        /* wavefronts per launch (one per workgroup)    */
  int32_t n_slots;        /* n_waves * 64 lane slots                      */
  int32_t max_depth;      /* deepest tree level (root = 0)                */
  int32_t has_free;       /* 1 if any system has a free-floating root      */
  int32_t dtype;
  int32_t frames_identity; /* 1 if, after the library rotates every link
                              frame so that its joint axis is z, every
                              parent->joint rotation is the identity (the
                              kernels then use a specialised variant)     */
  int32_t chain;          /* 1 if every system is a fixed-base serial chain
                              of revolute joints (parent of link i is link
                              i-1); the kernels then pass parent/child
                              quantities between neighbouring lanes'
                              registers                                   */
  int32_t has_prism;      /* 1 if any joint is prismatic (the kernels then
                              use their general variant)                  */
  int32_t adjoint_dtype;  /* arithmetic of sim_backward's recompute and
                              reverse passes: SIM_F64, or SIM_F32 (FP32
                              handles only; see sim_set_adjoint_dtype)    */
  int32_t has_ball;       /* 1 if any joint is spherical (the kernels then
                              use their general variant)                  */
} sim_info_t;

/* Build a handle: validates the topology and parameters, orders every
 * system breadth-first, packs systems into wavefronts (one lane per link),
 * and uploads the per-link constants in the requested dtype.  topo and
 * params are host memory, deep-copied; the caller may free them on return.
 * Errors: SIM_ERR_INVALID_ARG (null pointers, bad dtype value ->
 * SIM_ERR_UNSUPPORTED_DTYPE), SIM_ERR_INVALID_TOPOLOGY (parent >= own
 * index, free joint not at a root, more than SIM_MAX_LINKS links, non-unit
 * axis, non-positive mass, non-finite numbers), SIM_ERR_HIP (device
 * allocation or copy failed). */
int sim_create(const sim_topology *topo, const sim_params *params, int dtype, sim_t *out);

/* Release the handle and its device constants.  NULL is ignored. */
void sim_destroy(sim_t h);

int sim_get_info(sim_t h, sim_info_t *out);

/* Arithmetic of the backward pass (Sec. 3, Eq. adj_back; Sec. 4.1, Eq.
 * adj_r; Sec. 4.2).  An FP32 handle keeps its inputs, outputs, checkpoints
 * and forward rollout in FP32 (segment replays for K > 1 and binomial
 * advances also run the FP32 step, so they reproduce the forward's states
 * bit for bit).  With SIM_F64 (the default) each step's intermediates are
 * recomputed in FP64 from the exactly widened FP32 state and control, the
 * reverse sweeps through the adjoints of the integrator and the three ABA
 * passes run in FP64, and so does the adjoint state carried from step to
 * step; the outputs are rounded to FP32 once.  The result is the gradient
 * of the step map along the FP32 trajectory to FP64 round-off (store-all,
 * K == 0, reverses the FP32 intermediates it stored).  SIM_F32 runs the
 * whole backward pass in FP32: faster, but on long chains and chaotic
 * rollouts the reverse recursion loses digits (gradient errors of 1e-3 and
 * more).  FP64 handles accept SIM_F64 only.  Takes effect for later
 * sim_backward calls (and graphs captured after the change).  Errors:
 * SIM_ERR_INVALID_ARG (null handle), SIM_ERR_UNSUPPORTED_DTYPE. */
int sim_set_adjoint_dtype(sim_t h, int dtype);

/* Health of the results: *nonfinite_count receives the number of
 * non-finite numbers (NaN or infinity) that the kernels enqueued on this
 * handle wrote to their outputs (qT, qdT, traj, qdd, gq0, gqd0, gtau) since
 * the previous sim_status call, and the counter is reset.  A diverging
 * rollout propagates NaN to its final state, so a zero count after
 * sim_forward + sim_backward means every output is finite.  Synchronises
 * `stream` (the stream the kernels were enqueued on); not for use during
 * stream capture.  Kernels of one handle running concurrently on several
 * streams share the counter.  Counts above INT_MAX are reported as INT_MAX.
 * Errors: SIM_ERR_INVALID_ARG (null handle or pointer), SIM_ERR_HIP. */
int sim_status(sim_t h, void *stream, int *nonfinite_count);

/* Launch geometry of the handle's kernels (the autotuner's knobs; they
 * change no arithmetic, only how wavefronts are grouped into workgroups and
 * so where they run and how much LDS a workgroup takes).
 *   waves_per_block: 1, 2 or 4 wavefronts per workgroup in the forward,
 *     single-evaluation and non-pipelined adjoint kernels;
 *   pairs_per_block: 1 or 2 producer/consumer wavefront pairs per
 *     workgroup in the pipelined adjoint;
 *   pipelined: 1 = K == 1 adjoints use the pipelined kernel (one wavefront
 *     recomputes step t-1 while another reverses step t), 0 = one wavefront
 *     does both.
 * A choice whose LDS would exceed the device's per-workgroup limit is
 * reduced at launch.  Default (from occupancy): 4 waves per block;
 * pipelined with 2 pairs per block while the pipelined pairs fit one
 * wavefront per SIMD, otherwise not pipelined.  Not thread-safe against
 * concurrent launches on the same handle.  Errors: SIM_ERR_INVALID_ARG. */
typedef struct {
  int32_t waves_per_block;
  int32_t pairs_per_block;
  int32_t pipelined;
} sim_tiling_t;
int sim_get_tiling(sim_t h, sim_tiling_t *out);
int sim_set_tiling(sim_t h, const sim_tiling_t *tiling);

/* Autotuner: time every launch geometry on this device for a forward plus
 * backward rollout of T_probe steps with checkpoint interval K (a probe
 * rollout from the zero state with unit quaternions and zero torques; run
 * time does not depend on the values), then keep the fastest on the handle
 * (as sim_set_tiling would).  The forward and the one-wave adjoint share
 * waves_per_block, so whole pairs of choices are compared.  Store-all
 * probes (K == 0) are shortened to at most 2 GiB of workspace.  Allocates
 * and frees its own probe buffers, synchronises `stream` (a hipStream_t,
 * NULL = default), and must not be called during stream capture.
 * chosen (nullable) receives the winner, ms_per_step (nullable) its
 * forward+backward time per probe step.  Arithmetic is unaffected by the
 * choice.  Errors: SIM_ERR_INVALID_ARG (K < -4096, T_probe outside 1..100000),
 * SIM_ERR_HIP (probe allocation or launch failed; the tiling is left as it
 * was).
 * Choices are kept per process, keyed by what decides the run time: the
 * batch's packed structure (every lane's topology fields and joint types,
 * the wave depths), the kernel variant, the dtype and adjoint dtype, K,
 * T_probe and the device.  A later call with the same key (another handle
 * of the same structure, say) applies the kept choice without probing,
 * allocating or synchronising, and reports the ms_per_step measured then. */
int sim_autotune(sim_t h, int K, int T_probe, void *stream, sim_tiling_t *chosen, double *ms_per_step);

/* Forgets every choice sim_autotune kept (the next call probes again). */
void sim_autotune_cache_clear(void);

/* Bytes of workspace needed by sim_forward/sim_backward for T steps with a
 * checkpoint every K >= 1 steps (K > 1 adds a K-state replay buffer); for
 * K < 0, binomial checkpointing with s = -K snapshots (s + 1 state records:
 * the backward pass rebuilds every state from x^0 and the snapshots on the
 * schedule of sim_checkpoint_schedule, the memory floor of App. B's
 * trade-off); or,
 * for K == 0 (store-all), every step's initial state and all per-link
 * intermediates the reverse passes read (56 numbers per link and step;
 * three cheap by-products are rebuilt from them), so the backward pass
 * reruns none of the ABA sweeps.  Pure function of (h, T, K). */
int sim_workspace_bytes(sim_t h, int T, int K, size_t *bytes);

/* Binomial checkpointing schedule for reversing T steps with s snapshots
 * (the recursion of Griewank's "revolve": a segment of l steps is advanced
 * to a split point m, snapshotted there, its tail reversed with one
 * snapshot fewer and then its head with all of them; m is taken from the
 * binomial bound beta(s, t) = C(s + t, s) so that no step is advanced more
 * than the minimal number of times).  Pure host function, used by
 * sim_backward for K = -s and exposed for planning and testing.  actions
 * (nullable, capacity pairs) receives (op, arg) int32 pairs: op & 7 =
 * 0 RESTORE (slot op >> 3, time arg), 1 ADVANCE (arg steps), 2 TAKESHOT
 * (slot op >> 3), 3 ADJOINT (reverse step arg); slot 0 holds x^0.
 * *n_actions receives the count, *advanced (nullable) the number of plain
 * steps advanced (the recompute beyond one re-evaluation per step).
 * Errors: SIM_ERR_INVALID_ARG (T < 0, s outside 1..4096, capacity too
 * small). */
int sim_checkpoint_schedule(int T, int s, int32_t *actions, int capacity, int *n_actions,
                            long long *advanced);

/* Forward rollout of T steps of size dt (Sec. 3; Sec. 4.1 time
 * integration).  q0 [nq], qd0 [nv], tau [T][nu] -> qT [nq], qdT [nv];
 * traj (nullable) [T][nq + nv].  With a workspace, the initial state of
 * every K-th step (K >= 1) is stored there for sim_backward (Sec. 4.2;
 * App. B), or with K == 0 every step's state and intermediates (store-all,
 * the memory-hungry alternative the checkpointing replaces), or with K < 0
 * (binomial checkpointing) only x^0;
 * workspace == NULL runs the plain forward pass (nothing stored).
 * Errors: SIM_ERR_INVALID_ARG (T < 0, K < -4096, dt not finite or <= 0,
 * null required pointer), SIM_ERR_WORKSPACE_TOO_SMALL, SIM_ERR_HIP. */
int sim_forward(sim_t h, const void *q0, const void *qd0, const void *tau, double dt, int T, int K,
                void *qT, void *qdT, void *traj, void *workspace, size_t workspace_bytes,
                void *stream);

/* Adjoint (reverse-time) pass of the rollout last run by sim_forward on
 * this workspace with the same tau, dt, T and K (Sec. 3, Eq. adj_back;
 * Sec. 4.1, Eq. adj_r; Sec. 4.2).  Seeds: gqT [nq], gqdT [nv] = dL/dx^T;
 * gtraj (nullable) [T][nq + nv] = dL/dtraj.  Outputs (overwritten, not
 * accumulated): gq0 [nq], gqd0 [nv], gtau [T][nu].  Reads the checkpoints
 * in the workspace and, for K > 1, uses the rest of it as replay scratch.
 * For K < 0 it runs the binomial schedule of sim_checkpoint_schedule(T, -K)
 * with the workspace's snapshot slots; the schedule is built on the host on
 * the first call with a new (T, K), uploaded into device memory of the
 * handle (one allocation, an upload ordered on `stream`) and kept, one
 * buffer per (T, K), until sim_destroy, so that first call allocates and
 * must not be made during stream capture; later calls with that (T, K)
 * allocate nothing and may be captured.
 * For a free root, gq0's quaternion entries are the gradient with respect
 * to the raw components under the rotation formula
 * R = (w^2 - u.u) I + 2 u u^T + 2 w [u]x; only their component tangent to
 * the unit sphere is gauge-independent.
 * gparam (nullable) [n_links][10]: the gradient with respect to every
 * link's ten inertial parameters, summed over the rollout (Sec. 4.1, after
 * Eq. adj_r: other parameters follow from the same per-step adjoints as the
 * controls), per link in the caller's link order and link frame:
 * (m, h_x, h_y, h_z, I_xx, I_yy, I_zz, I_xy, I_xz, I_yz) with h = m c the
 * first moment and I = I_c - m [c]x^2 the rotational inertia about the link
 * origin; an off-diagonal parameter stands for both of its matrix entries.
 * gframe (nullable) [n_links][9]: the gradient with respect to every
 * revolute or prismatic link's joint placement X_T = (E_T, r_T) and joint
 * axis a, summed over the rollout, per link in the caller's link order
 * (zeros for a free root): (phi_bar[3], r_T_bar[3], axis_bar[3]).
 *   phi_bar: a rotation of the joint frame, E_T -> exp(-[phi]x) E_T with phi
 *     in joint-frame coordinates, changes the loss by phi_bar . phi;
 *   r_T_bar: the gradient with respect to r_T (parent coordinates);
 *   axis_bar: the gradient with respect to the axis vector along the unit
 *     sphere (link coordinates, orthogonal to a): a change da orthogonal
 *     to a changes the loss by axis_bar . da.
 * Either parameter output selects kernels that accumulate the model
 * parameters' adjoints; without them the adjoint runs without that work.
 * Errors as sim_forward. */
int sim_backward(sim_t h, const void *tau, double dt, int T, int K, const void *gqT,
                 const void *gqdT, const void *gtraj, void *gq0, void *gqd0, void *gtau,
                 void *gparam, void *gframe, void *workspace, size_t workspace_bytes,
                 void *stream);

/* sim_backward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and results, but the K > 1 replay buffer
 * lives in a static device array of the library (64 MiB, one per GPU, held
 * until the process ends) instead of the caller's workspace.  checkpoints
 * is the workspace of the matching sim_forward call; only its checkpoint
 * part is read (checkpoint_bytes at least sim_workspace_bytes for the same
 * T and K minus the replay buffer, i.e. the full size for K <= 1).  K >= 0
 * only (binomial schedules need a device copy of the schedule).  Every call
 * on one GPU shares that array: calls that overlap in time on one GPU (on
 * different streams, or from several threads) race and give wrong results;
 * serialise them.  Calls no allocating routine.  Errors: as sim_backward;
 * SIM_ERR_INVALID_ARG for K < 0; SIM_ERR_WORKSPACE_TOO_SMALL when the
 * replay buffer (K state records, see sim_workspace_bytes) exceeds 64 MiB or
 * checkpoint_bytes is too small; SIM_ERR_HIP if the array's device address
 * cannot be obtained. */
int sim_backward_noalloc(sim_t h, const void *tau, double dt, int T, int K, const void *gqT,
                         const void *gqdT, const void *gtraj, void *gq0, void *gqd0, void *gtau,
                         void *gparam, void *gframe, void *checkpoints, size_t checkpoint_bytes,
                         void *stream);

/* Forward-mode (tangent) rollout: the T-step rollout of sim_forward with
 * one input direction (dq0 [nq], dqd0 [nv], dtau [T][nu]) carried along,
 * giving the final state and its directional derivative
 * dqT, dqdT = d(q^T, qd^T)/d(q^0, qd^0, u) . (dq0, dqd0, dtau); traj and
 * dtraj (both given or both NULL) [T][nq + nv] receive every step's state
 * and tangent.  No workspace: forward mode needs no checkpoints.  With
 * T = 1 this is the one-step Jacobian-vector product ds'/da . da of the
 * sample enhancement in Sec. 5; sim_backward with T = 1 gives the
 * vector-Jacobian product used by the policy enhancement.  All arrays are
 * device memory of the handle's dtype.  Errors: SIM_ERR_INVALID_ARG (T < 0,
 * dt not finite or <= 0, null required pointer, only one of traj/dtraj),
 * SIM_ERR_HIP. */
int sim_forward_jvp(sim_t h, const void *q0, const void *qd0, const void *tau, const void *dq0,
                    const void *dqd0, const void *dtau, double dt, int T, void *qT, void *qdT,
                    void *dqT, void *dqdT, void *traj, void *dtraj, void *stream);

/* Forward dynamics of every system at one state (Sec. 3, ABA):
 * q [nq], qd [nv], tau [nu] -> qdd [nv] (a free root's 6 entries are its
 * true body-frame spatial acceleration).  Errors: SIM_ERR_INVALID_ARG,
 * SIM_ERR_HIP. */
int sim_aba(sim_t h, const void *q, const void *qd, const void *tau, void *qdd, void *stream);

/* Algorithmic floating-point operations per time step for the whole batch
 * (one add, subtract, multiply, divide, square root, sine or cosine = 1),
 * counted by running the per-link arithmetic once with an operation-
 * counting scalar type.  kind: 0 = one ABA evaluation, 1 = one forward
 * step (ABA + integration), 2 = one backward step (recompute + adjoint). */
int sim_flops(sim_t h, int kind, double *flops_per_step);

/* Thread-local description of the last error on this thread ("" if none). */
const char *sim_last_error(void);

/* ---- contact solver ------------------------------------------------------
 * Projected Gauss-Seidel (PGS) on a batch of independent mixed linear
 * complementarity problems, and its adjoint (Sec. 4.1 "Collision
 * resolution", Eq. mlcp; App. C).  Problem p: find x with
 *   a = A x + b,  lo <= x <= hi,
 *   a_i >= 0 where x_i = lo_i, a_i <= 0 where x_i = hi_i, a_i = 0 between
 * (lo = 0, hi = +inf gives 0 <= a perp x >= 0).  The solve runs exactly
 * niter sweeps from x0; a sweep sets the rows in order,
 *   y_i = -(b_i + sum_{j != i} A_ij x_j) / A_ii,  x_i = min(max(y_i, lo_i), hi_i)
 * (the bounds are fixed inputs and must be finite: an unbounded side takes
 * a large finite value such as +-FLT_MAX; A_ii must be nonzero).
 * Arrays are DEVICE pointers of the dtype (SIM_F32 or SIM_F64), caller-owned:
 * A [batch][n][n] row-major, b, lo, hi, x0, x [batch][n]; 1 <= n <=
 * SIM_PGS_MAX_ROWS.  Calls only enqueue work on `stream` (NULL = default):
 * no allocation, no synchronisation.  Errors: SIM_ERR_INVALID_ARG (sizes,
 * null arrays), SIM_ERR_UNSUPPORTED_DTYPE, SIM_ERR_WORKSPACE_TOO_SMALL,
 * SIM_ERR_HIP; sim_last_error() describes the failure. */
#define SIM_PGS_MAX_ROWS 16

/* Bytes of the workspace that keeps x at the start of every sweep (and the
 * result) for the adjoint: (niter + 1) * n * batch * sizeof(dtype), and for
 * n >= 13 another niter * n * batch elements after them, which
 * sim_pgs_adjoint uses as scratch (the sweep vectors stay as they are). */
int sim_pgs_workspace_bytes(int dtype, int batch, int n, int niter, size_t *bytes);

/* Solve.  workspace (nullable): when given (workspace_bytes at least
 * sim_pgs_workspace_bytes), the sweep vectors are stored there for
 * sim_pgs_adjoint. */
int sim_pgs_solve(int dtype, int batch, int n, int niter, const void *A, const void *b,
                  const void *lo, const void *hi, const void *x0, void *x, void *workspace,
                  size_t workspace_bytes, void *stream);

/* Adjoint of sim_pgs_solve, from the workspace of that solve (same A, b,
 * lo, hi, batch, n, niter): given xbar = dL/dx [batch][n], writes
 * Abar [batch][n][n], bbar, lobar, hibar and x0bar [batch][n] (overwritten).
 * The sweeps are reversed row by row: a clamped row sends its adjoint to
 * the active bound (a value exactly on a bound counts as inside), a free
 * row to b, A and the other rows' values it was computed from. */
int sim_pgs_adjoint(int dtype, int batch, int n, int niter, const void *A, const void *b,
                    const void *lo, const void *hi, const void *xbar, void *workspace,
                    size_t workspace_bytes, void *Abar, void *bbar, void *lobar, void *hibar,
                    void *x0bar, void *stream);

/* ---- contact inside the step ----------------------------------------------
 * Rollouts with collision detection and contact resolution between the
 * dynamics and the integrator (Sec. 4.1 "Collision resolution": detection,
 * then the MLCP of Eq. mlcp solved by projected Gauss-Seidel), and their
 * gradient, for a batch of systems that share one topology and one set of
 * contact spheres (per-system parameters).
 *
 * Contact model: spheres fixed in links against the ground plane y = 0; a
 * sphere with centre height below its radius (gap phi < 0) is active.  Per
 * active contact three rows (normal e_y, tangents e_x, e_z) of J, the world
 * velocity of the sphere's lowest point; A = J M^-1 J^T, b = J qd_minus +
 * (beta/dt) phi on the normal rows, qd_minus = qd + dt qdd.  niter PGS sweeps
 * from zero solve the normal rows with lambda_n >= 0, then niter sweeps solve
 * all rows with each tangent boxed by +-mu times that contact's first normal
 * impulse; rows with A_ii = 0 take no impulse.  qd1 = qd_minus +
 * M^-1 J^T lambda; positions move with qd1 (a free root: p1 = p + dt R v1_lin
 * and quat1 = normalize(quat + dt/2 quat (x) (w1, 0)); 1-dof joints:
 * q1 = q + dt qd1).
 *
 * Model (host memory, read during the call only): n links in topological
 * order, parent[0] = -1, 0 <= parent[i] < i; jtype SIM_JOINT_REVOLUTE or
 * SIM_JOINT_PRISMATIC, SIM_JOINT_FREE only for link 0; ncontacts spheres on
 * links contact_link[]; gravity (world); mu, beta >= 0; niter >= 0; joint
 * limits (nullable): the limit torque adds to the control of the step's
 * forward dynamics, with its slopes in the gradient.
 *
 * Per-system parameters (DEVICE, dtype, [nparams][batch], entry k of
 * system s at k * batch + s): per link i at 25 i: E_T (9, row-major, parent
 * -> joint frame), r_T (3, joint origin in the parent frame), axis (3, any
 * nonzero length: the joint moves along axis / |axis|), mass, com (3, link
 * frame), inertia about the com (xx, yy, zz, xy, xz, yz); then per sphere k
 * at 25 n + 4 k: centre (3, link frame), radius.
 *
 * States are DEVICE arrays of the dtype, entry-major: q [nq][batch], qd
 * [nv][batch], tau [T][nu][batch]; a free root's q is (p_world, quat x, y,
 * z, w), its qd the body-frame (w, v).  Calls only enqueue work on `stream`
 * (NULL = default): no allocation, no synchronisation.  Errors:
 * SIM_ERR_INVALID_ARG, SIM_ERR_INVALID_TOPOLOGY, SIM_ERR_UNSUPPORTED_DTYPE,
 * SIM_ERR_HIP; sim_last_error() describes the failure. */
#define SIM_CONTACT_MAX_LINKS 16
#define SIM_CONTACT_MAX_SPHERES 4

/* Launch geometry of the contact kernels.  Every system is one lane; this
 * chooses how many share a wavefront: rollout_systems_per_wave in {8, 4, 2}
 * (two wavefronts per workgroup in FP32, one in FP64; each system's
 * articulated quantities sit in LDS), grad_systems_per_wave in {16, 8, 4}
 * (one wavefront per workgroup), and where the gradient keeps each
 * system's Gauss-Seidel and articulated working copies: grad_lds = 1 in LDS
 * (at most 16 systems per CU at a time), 0 in private memory (every system
 * in flight at once; only with 16 systems per wavefront).  Fewer per
 * wavefront spread a small batch over more CUs.  Every geometry computes
 * the same results bit for bit; sim_contact_autotune picks the fastest for
 * a batch. */
typedef struct {
  int rollout_systems_per_wave;
  int grad_systems_per_wave;
  int grad_lds;
} sim_contact_tiling_t;

typedef struct {
  int n;
  const int *parent;
  const int *jtype;
  int ncontacts;
  const int *contact_link;
  double mu, beta;
  int niter;
  double gravity[3];
  const double *limits;               /* nullable [4 n]: joint limits (lo, hi, k, d) of the
                                         1-dof joints, shared by the batch, as in
                                         sim_params (ignored for the free root) */
  const sim_contact_tiling_t *tiling; /* nullable: 8 and 16 systems per wavefront, LDS */
} sim_contact_model;

/* Sizes of the model's state, control and parameter vectors (each output
 * nullable). */
int sim_contact_param_count(const sim_contact_model *m, int *nq, int *nv, int *nu, int *nparams);

/* Algorithmic floating-point operations of one step with contact at the
 * state (q, qd) under tau (HOST double arrays of one system; params [nparams]
 * in the order above): step_flops for the plain step, grad_flops for one
 * reverse step of sim_contact_rollout_grad (the step's recompute and its
 * reverse statements).  Counted on the host by running the step's
 * statements with a counting scalar that keeps its value, so detection,
 * dropped rows and clamps decide as on the device; every +, -, *, /, sqrt,
 * sin and cos counts 1. */
int sim_contact_flops(const sim_contact_model *m, const double *params, const double *q, const double *qd,
                      const double *tau, double dt, double *step_flops, double *grad_flops);

/* T steps with contact from (q0, qd0).  Writes qT, qdT; traj (nullable)
 * receives x_0 .. x_T as [T + 1][nq + nv][batch] (q then qd per state, the
 * input of sim_contact_rollout_grad); ncontacts (nullable, DEVICE int
 * [T][batch]) the active-contact count of every step. */
int sim_contact_rollout(const sim_contact_model *m, int dtype, int batch, const void *params, const void *q0,
                        const void *qd0, const void *tau, double dt, int T, void *traj, void *qT, void *qdT,
                        int *ncontacts, void *stream);

/* Gradient of L = <gqT, qT> + <gqdT, qdT> through the rollout whose states
 * traj [T + 1][nq + nv][batch] sim_contact_rollout wrote (same model,
 * params, tau, dt): the reverse recursion x_bar_t = (dx_{t+1}/dx_t)^T
 * x_bar_{t+1}, tau_bar_t = (dx_{t+1}/dtau_t)^T x_bar_{t+1} with each step's
 * exact Jacobian at the stored state (detection, row and clamp decisions as
 * taken).  Writes gq0 [nq][batch], gqd0 [nv][batch], gtau [T][nu][batch]
 * and, when gmu (DEVICE [batch]) is not NULL, dL/dmu of every system (the
 * friction coefficient as a model parameter, Sec. 4.1 "other parameters").
 * Each reverse step recomputes the step from its stored state and runs its
 * statements backwards (Sec. 4.1 "Collision resolution", App. C): the
 * integrator, the impulse, both Gauss-Seidel solves from their recorded
 * sweeps, A and b, M^-1 J^T, the contact geometry, the smooth ABA step.
 * At most 64 PGS sweeps (niter) are recorded. */
int sim_contact_rollout_grad(const sim_contact_model *m, int dtype, int batch, const void *params, const void *traj,
                             const void *tau, double dt, int T, const void *gqT, const void *gqdT, void *gq0,
                             void *gqd0, void *gtau, void *gmu, void *stream);

/* Launch-geometry autotuner for the contact kernels: times T_probe steps of
 * sim_contact_rollout from (q0, qd0) under tau (DEVICE [T_probe][nu][batch])
 * and their sim_contact_rollout_grad at every geometry of
 * sim_contact_tiling_t, on the caller's model, parameters and batch, and
 * writes the fastest of each to *chosen (m->tiling is ignored) and their
 * ms per probe step (nullable).  The probe should start from a state like
 * the ones the calls will see: a step in contact costs several times one in
 * free flight.  A set-up call, unlike the others: it
 * allocates its probe buffers with hipMalloc, frees them, and synchronises
 * `stream`.  Errors as for the rollout, SIM_ERR_HIP when the probe buffers
 * cannot be allocated. */
int sim_contact_autotune(const sim_contact_model *m, int dtype, int batch, const void *params, const void *q0,
                         const void *qd0, const void *tau, double dt, int T_probe, void *stream,
                         sim_contact_tiling_t *chosen, double *rollout_ms, double *grad_ms);

#ifdef __cplusplus
}
#endif

#endif
