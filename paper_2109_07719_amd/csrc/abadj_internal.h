// Internal launch interface between the host runtime and the kernels.
#pragma once

#include <string>

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace aba {

constexpr int kWave = 64;

// integer per-lane fields, stored [field][slot]
// CI_FIDX: index of a free root among the batch's free roots (-1 otherwise);
// CI_LINK: the link's index in the caller's batch-concatenated link order
enum CiField {
  CI_PARENT = 0, CI_DEPTH, CI_CFIRST, CI_CCOUNT, CI_JTYPE, CI_QIDX, CI_VIDX, CI_UIDX, CI_FIDX, CI_LINK, CI_COUNT
};
// floating per-lane fields, stored [field][slot]
enum CfField {
  CF_ET = 0,          // 9
  CF_RT = 9,          // 3
  CF_AX = 12,         // 3
  CF_M = 15,          // 1
  CF_MC = 16,         // 3
  CF_IB = 19,         // 6: xx yy zz xy xz yz
  CF_RL = 25,         // 9: rotation from the caller's link frame to the kernels' (joint axis = z)
  CF_LIM = 34,        // 4: joint limits lo, hi, stiffness k, damping d (read when has_limits)
  CF_COUNT = 38
};

template <typename S>
struct Packed {
  const int32_t* ci;     // [CI_COUNT][nslots]
  const S* cf;           // [CF_COUNT][nslots]
  const int32_t* wmaxd;  // [nwaves] deepest level present in each wave
  int nslots;
  int nwaves;
  int nfree;             // number of free-floating roots in the batch
  S g[3];                // gravity
  int nq, nv, nu;        // totals over the batch
  unsigned long long* status;  // device counter of non-finite numbers written to outputs
  int has_limits;        // some joint has limits (CF_LIM)
};

template <typename S>
struct FwdArgs {
  Packed<S> P;
  S dt;
  int T, K;
  const S* q0;
  const S* qd0;
  const S* tau;  // [T][nu]
  S* qT;
  S* qdT;
  S* traj;       // nullable [T][nq + nv]
  S* ck;         // nullable: K >= 1 checkpoints [ceil(T/K)][state width][nslots];
                 // K == 0 every step's state and intermediates
                 // [T][state width + kTapeFields][nslots]
};

template <typename S>
struct BwdArgs {
  Packed<S> P;
  S dt;
  int T, K;
  const S* tau;
  const S* gqT;
  const S* gqdT;
  const S* gtraj;  // nullable
  S* gq0;
  S* gqd0;
  S* gtau;
  S* ck;           // checkpoints (K < 0: x^0 and the snapshot slots, written here)
  S* scratch;      // K > 1: [K][state width][nslots]
  S* gparam;       // nullable: [n_links][10] inertial-parameter gradients
  S* gframe;       // nullable: [n_links][9] placement and axis gradients
  const int32_t* sched;  // K < 0: binomial checkpointing actions, (op, arg) pairs
  int nsched;
  int adj64;       // S = float only: recompute each step and run the reverse passes in FP64 (inputs,
                   // outputs, checkpoints and replays stay FP32)
};

// Actions of a binomial checkpointing schedule (K < 0, s = -K snapshots).
// op & 7 is the action, op >> 3 a snapshot slot (slot 0 holds x^0):
//   RESTORE slot, t : the current state becomes the snapshot (x^t)
//   ADVANCE n       : n plain steps from the current state
//   TAKESHOT slot   : store the current state in the slot
//   ADJOINT t       : reverse step t from the current state x^t
enum SchedOp { SCH_RESTORE = 0, SCH_ADVANCE = 1, SCH_TAKESHOT = 2, SCH_ADJOINT = 3 };

// forward-mode (tangent) rollout: values and one tangent direction
template <typename S>
struct JvpArgs {
  Packed<S> P;
  S dt;
  int T;
  const S* q0;
  const S* qd0;
  const S* tau;   // [T][nu]
  const S* dq0;   // tangents of the inputs (same layouts)
  const S* dqd0;
  const S* dtau;
  S* qT;
  S* qdT;
  S* dqT;         // tangents of the final state
  S* dqdT;
  S* traj;        // nullable [T][nq + nv]
  S* dtraj;       // nullable [T][nq + nv]
};

template <typename S>
struct AbaArgs {
  Packed<S> P;
  const S* q;
  const S* qd;
  const S* tau;
  S* qdd;
};

// A stored state record: two numbers per lane slot ([2][nslots]: q, qd of a
// revolute link; p.x, p.y of a free root) followed by the remaining eleven
// numbers of every free root ([11][nfree]).
__host__ __device__ inline size_t state_record(int nslots, int nfree) { return 2 * (size_t)nslots + 11 * (size_t)nfree; }
// per-lane intermediates stored per step in store-all mode (K == 0)
constexpr int tape_width() { return 56; }

// What the kernels may specialise on.  has_free: the batch contains
// free-floating roots; eti: every revolute joint frame is the identity after
// axis canonicalisation; chain: every system is a fixed-base serial chain
// (in every wave, a non-root link's parent is the previous lane).
struct Shape {
  bool has_free = false;
  bool eti = false;
  bool chain = false;
  bool has_prism = false;  // some joint is prismatic
  bool has_limits = false; // joint limits were given
  bool has_ball = false;   // some joint is spherical
};

// Launch geometry.  waves_per_block: wavefronts per workgroup in the
// single-wave kernels (each wavefront on its own systems); pairs_per_block:
// producer/consumer wavefront pairs per workgroup in the pipelined adjoint;
// pipelined: whether K == 1 uses the pipelined adjoint at all.  The host
// pads the wave count to a multiple of kMaxWavesPerBlock with empty
// wavefronts, so every choice divides it.
constexpr int kMaxWavesPerBlock = 4;
constexpr int kMaxPairsPerBlock = 2;
struct Tiling {
  int waves_per_block = 1;
  int pairs_per_block = 1;
  bool pipelined = true;
};

// Link-frame kinds of a kernel variant.  kFrIdentity: every E_T the
// identity after canonicalisation, every joint revolute; kFrGeneral: any
// E_T, every joint revolute; kFrGeneralJoints: any E_T, prismatic joints
// among the revolute ones (the joint type becomes a per-lane value) and
// joint limits; kFrBall: as kFrGeneralJoints, and ball joints.
enum : int { kFrIdentity = 0, kFrGeneral = 1, kFrGeneralJoints = 2, kFrBall = 3 };

// The library's error channel (sim_last_error; abadj_runtime.hip): sets the
// thread's message and returns code / clears it.
int report_error(int code, const std::string& msg);
void clear_error();

// Launchers: pick the kernel variant for the handle's shape and launch it on
// `stream` (abadj_kernels.hip; the adjoint in abadj_kernels_bwd.hip).  The serial-chain variants live in their own
// translation unit (abadj_kernels_chain.hip), reached through the *_chain
// launchers for frame kinds kFrIdentity and kFrGeneral.
template <typename S>
hipError_t launch_forward(const FwdArgs<S>& a, const Shape& sh, const Tiling& tl, hipStream_t st);
template <typename S>
hipError_t launch_backward(const BwdArgs<S>& a, const Shape& sh, const Tiling& tl, hipStream_t st);
template <typename S>
hipError_t launch_aba(const AbaArgs<S>& a, const Shape& sh, const Tiling& tl, hipStream_t st);
template <typename S>
hipError_t launch_forward_jvp(const JvpArgs<S>& a, const Shape& sh, const Tiling& tl, hipStream_t st);
// FP32 handles whose adjoint runs in FP64 (BwdArgs::adj64), non-chain
// variants (abadj_kernels_bwd64.hip)
hipError_t launch_backward_adj64(const BwdArgs<float>& a, const Shape& sh, const Tiling& tl, hipStream_t st);
template <typename S, int FR>
hipError_t launch_forward_chain(const FwdArgs<S>& a, const Tiling& tl, hipStream_t st);
template <typename S, int FR>
hipError_t launch_backward_chain(const BwdArgs<S>& a, const Tiling& tl, hipStream_t st);
template <typename S, int FR>
hipError_t launch_aba_chain(const AbaArgs<S>& a, const Tiling& tl, hipStream_t st);
template <typename S, int FR>
hipError_t launch_forward_jvp_chain(const JvpArgs<S>& a, const Tiling& tl, hipStream_t st);

}  // namespace aba
