// HIP kernels for gfx950: batched ABA forward dynamics + semi-implicit
// Euler (forward rollout with checkpoints) and the reverse-time adjoint
// (backward rollout with per-step recompute).  Included by the two kernel
// translation units (abadj_kernels.hip: trees and free roots;
// abadj_kernels_chain.hip: serial chains), which instantiate disjoint sets
// of variants.
//
// Layout on the GPU:
//   * one wavefront (64 lanes) per workgroup; several systems are packed
//     into a wave, one lane per link, links of a system contiguous in
//     breadth-first order (children of a link occupy consecutive lanes);
//   * each lane keeps its link's constants and its step intermediates in
//     VGPRs for the whole rollout; the time loop runs inside the kernel;
//   * the tree recursions of the three ABA passes (and of their adjoints)
//     are level-synchronous sweeps over tree depth; parent/child quantities
//     move through a per-wave LDS exchange buffer [field][lane];
//   * checkpoints are stored per lane slot, [checkpoint][field][slot], so
//     every store and reload is a coalesced 256-byte row per wave.
//
// Method: ABA (Sec. 3; Fig. 1), modules in the order of Sec. 4.1, adjoints
// in reverse order, intermediates recomputed from the stored initial state
// of each step (Sec. 4.2, Eq. intermediate), checkpoint interval K with
// segment replay (App. B).
#pragma once

#include "aba_lane.h"
#include "abadj_internal.h"
#include "dual.h"

namespace aba {

namespace {

constexpr int XB = 27;  // exchange-buffer fields per lane

// Synchronisation of the lanes of one wavefront around the LDS exchange
// buffer: the wave executes its LDS operations in order, so a compiler
// barrier with wavefront-scope release/acquire fences suffices (the same
// construction as HIP's __syncwarp).  Workgroup barriers stay free for the
// producer/consumer hand-off of the pipelined adjoint.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cross-lane moves for batches of serial chains, where the parent of every
// non-root link sits in the previous lane and its only child in the next:
// from_prev gives lane i the value of lane i-1 (DPP wave_shr:1), from_next
// that of lane i+1 (wave_shl:1); a lane without a source gets 0.  DPP reads
// the registers of the whole wavefront, so these run with every lane
// active (outside the per-depth branches).
constexpr int kDppWaveShl1 = 0x130;
constexpr int kDppWaveShr1 = 0x138;
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(x), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double x) {
  return __builtin_amdgcn_update_dpp(0.0, x, CTRL, 0xf, 0xf, true);
}
template <int CTRL, typename S>
__device__ __forceinline__ Dual<S> dpp_mov(const Dual<S>& x) {
  return Dual<S>(dpp_mov<CTRL>(x.v), dpp_mov<CTRL>(x.d));
}
template <int CTRL, typename S>
__device__ __forceinline__ V6<S> dpp6(const V6<S>& v) {
  return v6<S>(v3<S>(dpp_mov<CTRL>(v.a.x), dpp_mov<CTRL>(v.a.y), dpp_mov<CTRL>(v.a.z)),
               v3<S>(dpp_mov<CTRL>(v.l.x), dpp_mov<CTRL>(v.l.y), dpp_mov<CTRL>(v.l.z)));
}
template <int CTRL, typename S>
__device__ __forceinline__ SySp<S> dpp21(const SySp<S>& M) {
  SySp<S> R;
  R.A = sy3<S>(dpp_mov<CTRL>(M.A.xx), dpp_mov<CTRL>(M.A.yy), dpp_mov<CTRL>(M.A.zz), dpp_mov<CTRL>(M.A.xy),
               dpp_mov<CTRL>(M.A.xz), dpp_mov<CTRL>(M.A.yz));
#pragma unroll
  for (int k = 0; k < 9; ++k) R.B.m[k] = dpp_mov<CTRL>(M.B.m[k]);
  R.C = sy3<S>(dpp_mov<CTRL>(M.C.xx), dpp_mov<CTRL>(M.C.yy), dpp_mov<CTRL>(M.C.zz), dpp_mov<CTRL>(M.C.xy),
               dpp_mov<CTRL>(M.C.xz), dpp_mov<CTRL>(M.C.yz));
  return R;
}
template <typename S>
__device__ __forceinline__ V6<S> from_prev(const V6<S>& v) { return dpp6<kDppWaveShr1>(v); }
template <typename S>
__device__ __forceinline__ SySp<S> from_prev(const SySp<S>& M) { return dpp21<kDppWaveShr1>(M); }
template <typename S>
__device__ __forceinline__ V6<S> from_next(const V6<S>& v) { return dpp6<kDppWaveShl1>(v); }
template <typename S>
__device__ __forceinline__ SySp<S> from_next(const SySp<S>& M) { return dpp21<kDppWaveShl1>(M); }

__device__ __forceinline__ void sincos_(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ __forceinline__ void sincos_(double x, double* s, double* c) { sincos(x, s, c); }
template <typename S>
__device__ __forceinline__ void sincos_(const Dual<S>& x, Dual<S>* s, Dual<S>* c) {
  S sv, cv;
  sincos_(x.v, &sv, &cv);
  *s = Dual<S>(sv, cv * x.d);
  *c = Dual<S>(cv, -sv * x.d);
}

struct Lane {
  int lane, slot;
  int par, depth, cfirst, ccount, jtype, qidx, vidx, uidx, fidx, link;
  __device__ bool active() const { return jtype >= 0; }
  // revolute or prismatic (jtype 0 or 2; -1 marks an idle lane, 1 a free
  // root, 3 a ball joint)
  __device__ bool onedof() const { return (jtype & 1) == 0; }
  __device__ bool ball() const { return jtype == 3; }
};

// wb: the wave batch (64 lane slots) this wavefront works on
template <typename S>
__device__ __forceinline__ Lane load_lane(const Packed<S>& P, int wb) {
  Lane l;
  l.lane = threadIdx.x % kWave;
  l.slot = wb * kWave + l.lane;
  const int ns = P.nslots;
  const int32_t* ci = P.ci;
  l.par = ci[CI_PARENT * ns + l.slot];
  l.depth = ci[CI_DEPTH * ns + l.slot];
  l.cfirst = ci[CI_CFIRST * ns + l.slot];
  l.ccount = ci[CI_CCOUNT * ns + l.slot];
  l.jtype = ci[CI_JTYPE * ns + l.slot];
  l.qidx = ci[CI_QIDX * ns + l.slot];
  l.vidx = ci[CI_VIDX * ns + l.slot];
  l.uidx = ci[CI_UIDX * ns + l.slot];
  l.fidx = ci[CI_FIDX * ns + l.slot];
  l.link = ci[CI_LINK * ns + l.slot];
  return l;
}

// Per-link constants.  The host canonicalises every joint axis to e_z, so
// the motion subspace is a compile-time constant unless prismatic joints
// are present; with kFrIdentity so is E_T.  The build's no-signed-zeros /
// finite-math flags let the compiler fold the resulting structural zeros
// and ones through the generic spatial-algebra code.
template <typename S, int FR>
__device__ __forceinline__ LinkC<S> load_linkc(const Packed<S>& P, const Lane& l) {
  const int ns = P.nslots, slot = l.slot;
  const S* cf = P.cf;
  LinkC<S> L;
  if constexpr (FR == kFrIdentity) {
#pragma unroll
    for (int k = 0; k < 9; ++k) L.ET.m[k] = (k % 4 == 0) ? S(1) : S(0);
  } else {
#pragma unroll
    for (int k = 0; k < 9; ++k) L.ET.m[k] = cf[(CF_ET + k) * ns + slot];
  }
  L.rT = v3<S>(cf[(CF_RT + 0) * ns + slot], cf[(CF_RT + 1) * ns + slot], cf[(CF_RT + 2) * ns + slot]);
  if constexpr (FR >= kFrGeneralJoints) {
    L.prism = l.jtype == 2;
    const S ang = L.prism ? S(0) : S(1);
    L.sm = v6<S>(v3<S>(S(0), S(0), ang), v3<S>(S(0), S(0), S(1) - ang));
  } else {
    L.prism = false;
    L.sm = v6<S>(v3<S>(S(0), S(0), S(1)), zero3<S>());
  }
  L.m = cf[CF_M * ns + slot];
  L.mc = v3<S>(cf[(CF_MC + 0) * ns + slot], cf[(CF_MC + 1) * ns + slot], cf[(CF_MC + 2) * ns + slot]);
  L.Ib = sy3<S>(cf[(CF_IB + 0) * ns + slot], cf[(CF_IB + 1) * ns + slot], cf[(CF_IB + 2) * ns + slot],
                cf[(CF_IB + 3) * ns + slot], cf[(CF_IB + 4) * ns + slot], cf[(CF_IB + 5) * ns + slot]);
  return L;
}

// Joint transform of a 1-dof lane from its coordinate q (the tape keeps
// sin q, cos q of a revolute joint and q itself of a prismatic one).
template <typename S>
__device__ __forceinline__ void joint_transform(const LinkC<S>& L, S q, Tape<S>& t) {
  if (L.prism) {
    t.sq = q;
    t.cq = S(1);
  } else {
    sincos_(q, &t.sq, &t.cq);
  }
  joint_X(L, t);
}

// Dynamic LDS of a workgroup, sized by the launcher: one exchange buffer per
// wavefront (single-wave kernels), or per producer/consumer pair two
// exchange buffers and the double-buffered tape (pipelined adjoint).
extern __shared__ __align__(16) unsigned char abadj_lds[];
template <typename S>
__device__ __forceinline__ S* lds() {
  return reinterpret_cast<S*>(abadj_lds);
}
template <typename S>
__device__ __forceinline__ V3<S> gravity(const Packed<S>& P) {
  return v3<S>(P.g[0], P.g[1], P.g[2]);
}
// wave batch of a single-wave kernel's wavefront, and its place in the block
__device__ __forceinline__ int wave_in_block() { return threadIdx.x / kWave; }
__device__ __forceinline__ int wave_batch() { return blockIdx.x * (blockDim.x / kWave) + wave_in_block(); }

// ---- exchange buffer [field][lane]
template <typename S>
__device__ __forceinline__ void put6(S* xb, int f0, int lane, const V6<S>& v) {
  xb[(f0 + 0) * kWave + lane] = v.a.x;
  xb[(f0 + 1) * kWave + lane] = v.a.y;
  xb[(f0 + 2) * kWave + lane] = v.a.z;
  xb[(f0 + 3) * kWave + lane] = v.l.x;
  xb[(f0 + 4) * kWave + lane] = v.l.y;
  xb[(f0 + 5) * kWave + lane] = v.l.z;
}
template <typename S>
__device__ __forceinline__ V6<S> get6(const S* xb, int f0, int lane) {
  return v6<S>(v3<S>(xb[(f0 + 0) * kWave + lane], xb[(f0 + 1) * kWave + lane], xb[(f0 + 2) * kWave + lane]),
               v3<S>(xb[(f0 + 3) * kWave + lane], xb[(f0 + 4) * kWave + lane], xb[(f0 + 5) * kWave + lane]));
}
template <typename S>
__device__ __forceinline__ void put21(S* xb, int f0, int lane, const SySp<S>& M) {
  const S v[21] = {M.A.xx, M.A.yy, M.A.zz, M.A.xy, M.A.xz, M.A.yz, M.B.m[0], M.B.m[1], M.B.m[2], M.B.m[3], M.B.m[4],
                   M.B.m[5], M.B.m[6], M.B.m[7], M.B.m[8], M.C.xx, M.C.yy, M.C.zz, M.C.xy, M.C.xz, M.C.yz};
#pragma unroll
  for (int k = 0; k < 21; ++k) xb[(f0 + k) * kWave + lane] = v[k];
}
template <typename S>
__device__ __forceinline__ SySp<S> get21(const S* xb, int f0, int lane) {
  S v[21];
#pragma unroll
  for (int k = 0; k < 21; ++k) v[k] = xb[(f0 + k) * kWave + lane];
  SySp<S> M;
  M.A = sy3<S>(v[0], v[1], v[2], v[3], v[4], v[5]);
#pragma unroll
  for (int k = 0; k < 9; ++k) M.B.m[k] = v[6 + k];
  M.C = sy3<S>(v[15], v[16], v[17], v[18], v[19], v[20]);
  return M;
}

// per-lane state: 1-dof lanes use q[0], qd[0]; a free root uses
// q = (p, quat) and qd = body velocity [w; v]; a ball joint (only in the
// general variant, which has FREE set) q[0..3] = quat, qd[0..2] = w
template <typename S, bool FREE>
struct State {
  S q[FREE ? 7 : 1];
  S qd[FREE ? 6 : 1];
};

template <typename S, bool FREE>
__device__ __forceinline__ Q4<S> st_quat(const State<S, FREE>& s) {
  Q4<S> r;
  if constexpr (FREE) {
    r.x = s.q[3];
    r.y = s.q[4];
    r.z = s.q[5];
    r.w = s.q[6];
  } else {
    r.x = r.y = r.z = S(0);
    r.w = S(1);
  }
  return r;
}
template <typename S, bool FREE>
__device__ __forceinline__ Q4<S> st_ball_quat(const State<S, FREE>& s) {
  Q4<S> r;
  if constexpr (FREE) {
    r.x = s.q[0];
    r.y = s.q[1];
    r.z = s.q[2];
    r.w = s.q[3];
  } else {
    r.x = r.y = r.z = S(0);
    r.w = S(1);
  }
  return r;
}
template <typename S, bool FREE>
__device__ __forceinline__ V3<S> st_ball_w(const State<S, FREE>& s) {
  if constexpr (FREE) return v3<S>(s.qd[0], s.qd[1], s.qd[2]);
  return zero3<S>();
}
template <typename S, bool FREE>
__device__ __forceinline__ V6<S> st_vel6(const State<S, FREE>& s) {
  if constexpr (FREE) return v6<S>(v3<S>(s.qd[0], s.qd[1], s.qd[2]), v3<S>(s.qd[3], s.qd[4], s.qd[5]));
  return zero6<S>();
}

// Every member is assigned on every path (value selects, masked loads), so
// the compiler keeps the state in registers instead of selecting which
// member a load goes to.
template <typename S, bool FREE>
__device__ __forceinline__ void load_state(State<S, FREE>& s, const Lane& l, const S* q, const S* qd) {
  if constexpr (FREE) {
    const bool rev = l.onedof(), fr = l.jtype == 1, bl = l.ball();
#pragma unroll
    for (int k = 0; k < 7; ++k) s.q[k] = ((k == 0 && rev) || fr || (k < 4 && bl)) ? q[l.qidx + k] : s.q[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) s.qd[k] = ((k == 0 && rev) || fr || (k < 3 && bl)) ? qd[l.vidx + k] : s.qd[k];
  } else {
    if (l.onedof()) {
      s.q[0] = q[l.qidx];
      s.qd[0] = qd[l.vidx];
    }
  }
}
template <typename S, bool FREE>
__device__ __forceinline__ void store_state(const State<S, FREE>& s, const Lane& l, S* q, S* qd) {
  if (l.onedof()) {
    q[l.qidx] = s.q[0];
    qd[l.vidx] = s.qd[0];
  } else if constexpr (FREE) {
    if (l.jtype == 1) {
#pragma unroll
      for (int k = 0; k < 7; ++k) q[l.qidx + k] = s.q[k];
#pragma unroll
      for (int k = 0; k < 6; ++k) qd[l.vidx + k] = s.qd[k];
    } else if (l.ball()) {
#pragma unroll
      for (int k = 0; k < 4; ++k) q[l.qidx + k] = s.q[k];
#pragma unroll
      for (int k = 0; k < 3; ++k) qd[l.vidx + k] = s.qd[k];
    }
  }
}
// Non-finite outputs are counted with integer tests on the bit pattern.
// The device code is built with finite-math folding, under which the
// compiler may assume the exponent field is never all ones and remove even
// an integer test, so the bits first pass through a register move the
// compiler cannot see into.  Each kernel adds its count to the handle's
// counter once at the end.
__device__ __forceinline__ unsigned opaque_u32(unsigned u) {
  unsigned r;
  asm volatile("v_mov_b32 %0, %1" : "=v"(r) : "v"(u));
  return r;
}
__device__ __forceinline__ int nonfinite(float x) {
  return (opaque_u32(__float_as_uint(x)) & 0x7f800000u) == 0x7f800000u;
}
__device__ __forceinline__ int nonfinite(double x) {
  const unsigned hi = (unsigned)((unsigned long long)__double_as_longlong(x) >> 32);
  return (opaque_u32(hi) & 0x7ff00000u) == 0x7ff00000u;
}
template <typename S, bool FREE>
__device__ __forceinline__ int nonfinite_state(const State<S, FREE>& s, const Lane& l) {
  int n = 0;
  if (l.onedof()) {
    n = nonfinite(s.q[0]) + nonfinite(s.qd[0]);
  } else if constexpr (FREE) {
    if (l.jtype == 1) {
#pragma unroll
      for (int k = 0; k < 7; ++k) n += nonfinite(s.q[k]);
#pragma unroll
      for (int k = 0; k < 6; ++k) n += nonfinite(s.qd[k]);
    } else if (l.ball()) {
#pragma unroll
      for (int k = 0; k < 4; ++k) n += nonfinite(s.q[k]);
#pragma unroll
      for (int k = 0; k < 3; ++k) n += nonfinite(s.qd[k]);
    }
  }
  return n;
}
__device__ __forceinline__ void report_nonfinite(unsigned long long* status, int n) {
  if (n > 0) atomicAdd(status, (unsigned long long)n);
}

// stored state records (see state_record): [2][nslots] then [11][nfree]
// (nfree: free roots and ball joints, which keep q[0..6], qd[0..5] alike).
// The second row holds q[1] of such a lane or qd of a 1-dof link; it is
// chosen by value selects, not by selecting which member to address, so
// that the state stays in registers.
template <typename S, bool FREE>
__device__ __forceinline__ void put_slot(const State<S, FREE>& s, S* base, int nslots, int nfree, int slot,
                                         int fidx) {
  base[slot] = s.q[0];
  if constexpr (FREE) {
    const bool fr = fidx >= 0;
    base[nslots + slot] = fr ? s.q[1] : s.qd[0];
    if (fr) {
      S* ex = base + 2 * (size_t)nslots;
#pragma unroll
      for (int k = 0; k < 5; ++k) ex[(size_t)k * nfree + fidx] = s.q[2 + k];
#pragma unroll
      for (int k = 0; k < 6; ++k) ex[(size_t)(5 + k) * nfree + fidx] = s.qd[k];
    }
  } else {
    base[nslots + slot] = s.qd[0];
  }
}
template <typename S, bool FREE>
__device__ __forceinline__ void get_slot(State<S, FREE>& s, const S* base, int nslots, int nfree, int slot,
                                         int fidx) {
  s.q[0] = base[slot];
  const S second = base[nslots + slot];
  if constexpr (FREE) {
    const bool fr = fidx >= 0;
    s.q[1] = fr ? second : s.q[1];
    s.qd[0] = fr ? s.qd[0] : second;
    if (fr) {
      const S* ex = base + 2 * (size_t)nslots;
#pragma unroll
      for (int k = 0; k < 5; ++k) s.q[2 + k] = ex[(size_t)k * nfree + fidx];
#pragma unroll
      for (int k = 0; k < 6; ++k) s.qd[k] = ex[(size_t)(5 + k) * nfree + fidx];
    }
  } else {
    s.qd[0] = second;
  }
}

// Writes a link's inertial-parameter gradient, turned from the kernels'
// link frame back to the caller's: the kernels' parameters are
// mc' = Rl mc and Ib' = Rl Ib Rl^T, so mc_bar = Rl^T mc'_bar and, with the
// symmetric matrix G of the Ib adjoint (off-diagonals halved), G = Rl^T G' Rl.
// Returns the number of non-finite values written.
template <typename Sp, typename S>
__device__ __forceinline__ int store_param_bar(const ParamBar<S>& g, const Packed<Sp>& P, const Lane& l,
                                               Sp* out) {
  const int ns = P.nslots;
  M3<S> Rl;
#pragma unroll
  for (int k = 0; k < 9; ++k) Rl.m[k] = S(P.cf[(CF_RL + k) * ns + l.slot]);
  const V3<S> mc = mulT(Rl, g.mc);
  const Sy3<S> G = congT(Rl, sy3<S>(g.Ib.xx, g.Ib.yy, g.Ib.zz, S(0.5) * g.Ib.xy, S(0.5) * g.Ib.xz,
                                      S(0.5) * g.Ib.yz));
  const S v[10] = {g.m, mc.x, mc.y, mc.z, G.xx, G.yy, G.zz, S(2) * G.xy, S(2) * G.xz, S(2) * G.yz};
  Sp* o = out + (size_t)l.link * 10;
  int n = 0;
#pragma unroll
  for (int k = 0; k < 10; ++k) {
    o[k] = Sp(v[k]);
    n += nonfinite(o[k]);
  }
  return n;
}

// Writes a link's placement and axis gradient (phi_bar, r_T_bar, axis_bar)
// in the caller's frames from the accumulators in the kernels' joint frame
// (xi, w; frame_bar_add).  The kernels' X_T' = rot(Rl) X_T rot(Rp)^T, so a
// joint-frame perturbation xi of the caller's X_T is rot(Rl) xi here:
// xi = [Rl^T xi'_a; Rl^T xi'_l], phi_bar = xi_a and r_T_bar = E_T^T xi_l =
// Rp^T E_T'^T xi'_l.  The axis rotation adjoint is w = Rl^T (xi'_a + w'),
// and the gradient along the unit sphere is w x a = Rl^T ((xi'_a + w') x e_z).
// A ball joint has placement gradients only; a free root has none: zeros.
// Returns the number of non-finite values.
template <typename Sp, typename S>
__device__ __forceinline__ int store_frame_bar(const ParamBar<S>& g, const Packed<Sp>& P, const Lane& l,
                                               const LinkC<S>& L, Sp* out) {
  const int ns = P.nslots;
  S v[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) v[k] = S(0);
  if (l.onedof() || l.ball()) {
    M3<S> Rl, Rp;
#pragma unroll
    for (int k = 0; k < 9; ++k) Rl.m[k] = S(P.cf[(CF_RL + k) * ns + l.slot]);
    const int ps = l.slot - l.lane + l.par;
#pragma unroll
    for (int k = 0; k < 9; ++k) Rp.m[k] = (l.par >= 0) ? S(P.cf[(CF_RL + k) * ns + ps]) : ((k % 4 == 0) ? S(1) : S(0));
    const V3<S> phi = mulT(Rl, g.xi.a);
    const V3<S> rb = mulT(Rp, mulT(L.ET, g.xi.l));
    // a ball joint has no axis (and Rl = 1)
    const V3<S> w = l.ball() ? zero3<S>() : g.xi.a + g.w;
    const V3<S> ab = mulT(Rl, v3<S>(w.y, -w.x, S(0)));
    v[0] = phi.x; v[1] = phi.y; v[2] = phi.z;
    v[3] = rb.x; v[4] = rb.y; v[5] = rb.z;
    v[6] = ab.x; v[7] = ab.y; v[8] = ab.z;
  }
  Sp* o = out + (size_t)l.link * 9;
  int n = 0;
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    o[k] = Sp(v[k]);
    n += nonfinite(o[k]);
  }
  return n;
}

// Value part of a plain or dual scalar (branch decisions of the tangent
// rollout follow the value, as in the plain rollout).
__device__ __forceinline__ float val_(float x) { return x; }
__device__ __forceinline__ double val_(double x) { return x; }
template <typename S>
__device__ __forceinline__ S val_(const Dual<S>& x) {
  return x.v;
}

// The lane's slot index hidden from loop-invariant code motion: the limit
// constants are then re-read (from cache) where they are used instead of
// being hoisted out of the time loop into registers, which would cost the
// general-joints forward a wave of occupancy.  An empty asm statement on a
// register value, no memory access.
__device__ __forceinline__ int opaque_slot(const Lane& l) {
  int s = l.slot;
  asm volatile("" : "+v"(s));
  return s;
}

// A 1-dof lane's control with its joint-limit torque added: outside
// [lo, hi] a one-sided spring and damper, tau_l = -k (q - hi) - d qd above
// hi, -k (q - lo) - d qd below lo (the limits model of sim_params).  Only
// the general-joints variant carries it (handles with limits take that
// variant); the others compile it away.
template <int FR, typename S, typename T, bool FREE>
__device__ __forceinline__ V3<T> limit_tau(const Packed<S>& P, const Lane& l, const State<T, FREE>& st, V3<T> tau) {
  if constexpr (FR < kFrGeneralJoints) return tau;
  if (!P.has_limits || !l.onedof()) return tau;
  const int ns = P.nslots;
  const int slot = opaque_slot(l);
  const S lo = P.cf[(CF_LIM + 0) * ns + slot], hi = P.cf[(CF_LIM + 1) * ns + slot];
  const S k = P.cf[(CF_LIM + 2) * ns + slot], d = P.cf[(CF_LIM + 3) * ns + slot];
  const T q = st.q[0], qd = st.qd[0];
  if (val_(q) > hi) tau.x = tau.x - T(k) * (q - T(hi)) - T(d) * qd;
  else if (val_(q) < lo) tau.x = tau.x - T(k) * (q - T(lo)) - T(d) * qd;
  return tau;
}
// A lane's controls at one step (row: the step's [nu] controls): a 1-dof
// joint's torque in x, a ball joint's three torques (BALL: the general
// variant, the only one that takes ball joints).
template <bool BALL, typename S>
__device__ __forceinline__ V3<S> load_ctl(const S* row, const Lane& l) {
  V3<S> u = zero3<S>();
  if (l.onedof()) u.x = row[l.uidx];
  if constexpr (BALL) {
    if (l.ball()) u = v3<S>(row[l.uidx], row[l.uidx + 1], row[l.uidx + 2]);
  }
  return u;
}
template <typename R, typename S>
__device__ __forceinline__ V3<R> cvt3(const V3<S>& v) {
  return v3<R>(R(v.x), R(v.y), R(v.z));
}
// its partial derivatives with respect to q and qd (zero inside the range)
// (T: the adjoint's scalar type; the switch compares the same values as the
// forward's, widened exactly)
template <int FR, typename S, typename T, bool FREE>
__device__ __forceinline__ void limit_slopes(const Packed<S>& P, const Lane& l, const State<T, FREE>& st, T& dq,
                                             T& dqd) {
  dq = dqd = T(0);
  if constexpr (FR < kFrGeneralJoints) return;
  if (!P.has_limits || !l.onedof()) return;
  const int ns = P.nslots;
  const T q = st.q[0];
  const int slot = opaque_slot(l);
  if (q > T(P.cf[(CF_LIM + 1) * ns + slot]) || q < T(P.cf[(CF_LIM + 0) * ns + slot])) {
    dq = -T(P.cf[(CF_LIM + 2) * ns + slot]);
    dqd = -T(P.cf[(CF_LIM + 3) * ns + slot]);
  }
}

// Everything one ABA evaluation leaves in a lane.
template <typename S>
struct Step {
  Tape<S> t;
  V6<S> abase;  // free root: true body-frame acceleration; ball joint:
                // [joint acceleration; u = tau - pA_a]
};
template <typename R, typename S>
__device__ __forceinline__ Step<R> cvt_step(const Step<S>& o) {
  Step<R> w;
  w.t = widen<R>(o.t);
  w.abase = widen<R>(o.abase);
  return w;
}
// (also narrows the adjoint state back to the I/O type at the end)
template <typename R, typename S, bool FREE>
__device__ __forceinline__ State<R, FREE> cvt_state(const State<S, FREE>& x) {
  State<R, FREE> w;
#pragma unroll
  for (int k = 0; k < (FREE ? 7 : 1); ++k) w.q[k] = R(x.q[k]);
#pragma unroll
  for (int k = 0; k < (FREE ? 6 : 1); ++k) w.qd[k] = R(x.qd[k]);
  return w;
}

// Step intermediates handed to the reverse passes (store-all records in HBM
// and the pipelined adjoint's LDS tape), per lane slot, [field][stride]:
// sin q, cos q, v, I^A, p^A, 1/D, u, p^a, a', qdd, base acceleration.  E
// (from sin q, cos q), U (entries of I^A for a z-axis joint) and c (from v
// and qd) are rebuilt by the reader in a few operations, which also keeps
// their structural zeros visible to the compiler.
constexpr int kTapeFields = tape_width();

template <typename S>
__device__ __forceinline__ void put_tape(const Step<S>& o, S* base, int ns, int slot) {
  const Tape<S>& t = o.t;
  int f = 0;
  auto w = [&](S x) { base[(size_t)(f++) * ns + slot] = x; };
  auto w6 = [&](const V6<S>& v) { w(v.a.x); w(v.a.y); w(v.a.z); w(v.l.x); w(v.l.y); w(v.l.z); };
  w(t.sq); w(t.cq);
  w6(t.v);
  w(t.IA.A.xx); w(t.IA.A.yy); w(t.IA.A.zz); w(t.IA.A.xy); w(t.IA.A.xz); w(t.IA.A.yz);
#pragma unroll
  for (int k = 0; k < 9; ++k) w(t.IA.B.m[k]);
  w(t.IA.C.xx); w(t.IA.C.yy); w(t.IA.C.zz); w(t.IA.C.xy); w(t.IA.C.xz); w(t.IA.C.yz);
  w6(t.pA); w(t.Dinv); w(t.u); w6(t.pa); w6(t.ap); w(t.qdd); w6(o.abase);
}
template <typename S>
__device__ __forceinline__ void get_tape(Step<S>& o, const S* base, int ns, int slot, const LinkC<S>& L, S qd,
                                         bool rev) {
  Tape<S>& t = o.t;
  int f = 0;
  auto r = [&]() { return base[(size_t)(f++) * ns + slot]; };
  auto r6 = [&](V6<S>& v) { v.a.x = r(); v.a.y = r(); v.a.z = r(); v.l.x = r(); v.l.y = r(); v.l.z = r(); };
  t.sq = r(); t.cq = r();
  r6(t.v);
  t.IA.A.xx = r(); t.IA.A.yy = r(); t.IA.A.zz = r(); t.IA.A.xy = r(); t.IA.A.xz = r(); t.IA.A.yz = r();
#pragma unroll
  for (int k = 0; k < 9; ++k) t.IA.B.m[k] = r();
  t.IA.C.xx = r(); t.IA.C.yy = r(); t.IA.C.zz = r(); t.IA.C.xy = r(); t.IA.C.xz = r(); t.IA.C.yz = r();
  r6(t.pA); t.Dinv = r(); t.u = r(); r6(t.pa); r6(t.ap); t.qdd = r(); r6(o.abase);
  joint_X(L, t);
  t.U = mul(t.IA, L.sm);
  t.c = rev ? crm(t.v, qd * L.sm) : zero6<S>();
}

// The three ABA passes for a wave of serial chains with fixed bases (every
// active lane a 1-dof joint): parent/child quantities move between neighbouring
// lanes in registers.  A root never pushes to its parent, so the lane after
// a chain's leaf always hands the leaf zeros.
template <typename S>
__device__ __forceinline__ void aba_wave_chain(const V3<S>& g, const Lane& l, const LinkC<S>& L,
                                               const State<S, false>& st, S tau, int maxd, Step<S>& o) {
  Tape<S>& t = o.t;
  const bool act = l.active();
  const bool hp = l.par >= 0;
  joint_transform(L, st.q[0], t);
  // pass 1: velocities, root -> leaves
  t.v = zero6<S>();
  for (int d = 0; d <= maxd; ++d) {
    const V6<S> vp = from_prev(t.v);
    if (act && l.depth == d) t.v = p1_velocity(L, t, st.qd[0], hp ? vp : zero6<S>());
  }
  // pass 1: bias terms (parallel over links)
  if (act) p1_bias(L, t.v, st.qd[0], true, t.c, t.pA, t.IA);
  // pass 2: articulated inertias, leaves -> root
  SySp<S> IAu = zero_sysp<S>();
  V6<S> pAu = zero6<S>();
  for (int d = maxd; d >= 0; --d) {
    const SySp<S> cI = from_next(IAu);
    const V6<S> cp = from_next(pAu);
    if (act && l.depth == d) {
      t.IA = t.IA + cI;
      t.pA = t.pA + cp;
      p2_local(L, t, tau);
      if (hp) p2_push(L, t, IAu, pAu);
    }
  }
  // pass 3: accelerations, root -> leaves
  const V6<S> a0 = v6<S>(zero3<S>(), -g);
  V6<S> a = zero6<S>();
  for (int d = 0; d <= maxd; ++d) {
    const V6<S> ap = from_prev(a);
    if (act && l.depth == d) a = p3_accel(L, t, hp ? ap : a0);
  }
}

// One ABA evaluation for the whole wave (all three passes).  tau: the
// lane's controls (load_ctl).  BALL: the variant that also takes ball joints.
template <typename S, bool FREE, bool CHAIN, bool BALL = false>
__device__ __forceinline__ void aba_wave(const V3<S>& g, const Lane& l, const LinkC<S>& L,
                                         const State<S, FREE>& st, const V3<S>& tau, int maxd, S* xb,
                                         Step<S>& o) {
  if constexpr (CHAIN) {
    static_assert(!FREE, "the chain variant has fixed bases only");
    aba_wave_chain<S>(g, l, L, st, tau.x, maxd, o);
    return;
  }
  static_assert(!BALL || FREE, "ball joints run in the general (FREE) variant");
  Tape<S>& t = o.t;
  const bool act = l.active();
  const bool rev = l.onedof();
  const bool ball = BALL && l.ball();
  // pass 1: joint transforms (parallel over links)
  if (rev) joint_transform(L, st.q[0], t);
  if constexpr (BALL) {
    if (ball) t.E = ball_E(st_ball_quat(st), L.ET);
  }
  // pass 1: velocities, root -> leaves
  for (int d = 0; d <= maxd; ++d) {
    if (act && l.depth == d) {
      if (rev) {
        const V6<S> vp = (l.par >= 0) ? get6(xb, 0, l.par) : zero6<S>();
        t.v = p1_velocity(L, t, st.qd[0], vp);
      } else if (ball) {
        const V6<S> vp = (l.par >= 0) ? get6(xb, 0, l.par) : zero6<S>();
        t.v = xform(t.E, L.rT, vp) + v6<S>(st_ball_w(st), zero3<S>());
      } else {
        // free root: the ABA runs in the inertial frame that moves with the
        // root's current linear velocity (a Galilean shift, exact: joint
        // accelerations and the root's angular acceleration do not change,
        // its linear acceleration changes by w x v_lin, added back in pass 3).
        // A fast-moving base (a long free fall) otherwise puts large
        // cancelling terms into every link's bias force and acceleration.
        t.v = v6<S>(st_vel6(st).a, zero3<S>());
      }
      put6(xb, 0, l.lane, t.v);
    }
    wave_sync();
  }
  // pass 1: bias terms (parallel over links)
  if (act) p1_bias(L, t.v, st.qd[0], rev, t.c, t.pA, t.IA);
  if constexpr (BALL) {
    if (ball) t.c = crm(t.v, v6<S>(st_ball_w(st), zero3<S>()));
  }
  // pass 2: articulated inertias, leaves -> root
  for (int d = maxd; d >= 0; --d) {
    if (act && l.depth == d) {
      for (int k = 0; k < l.ccount; ++k) {
        t.IA = t.IA + get21(xb, 0, l.cfirst + k);
        t.pA = t.pA + get6(xb, 21, l.cfirst + k);
      }
      if (rev) {
        p2_local(L, t, tau.x);
        if (l.par >= 0) {
          SySp<S> IAu;
          V6<S> pAu;
          p2_push(L, t, IAu, pAu);
          put21(xb, 0, l.lane, IAu);
          put6(xb, 21, l.lane, pAu);
        }
      } else if (ball) {
        o.abase.l = ball_p2_local(t, tau);
        if (l.par >= 0) {
          SySp<S> IAu;
          V6<S> pAu;
          ball_p2_push(L, t, tau, IAu, pAu);
          put21(xb, 0, l.lane, IAu);
          put6(xb, 21, l.lane, pAu);
        }
      }
    }
    wave_sync();
  }
  // pass 3: accelerations, root -> leaves
  const V6<S> a0 = v6<S>(zero3<S>(), -g);
  for (int d = 0; d <= maxd; ++d) {
    if (act && l.depth == d) {
      if (rev) {
        const V6<S> ap = (l.par >= 0) ? get6(xb, 0, l.par) : a0;
        put6(xb, 0, l.lane, p3_accel(L, t, ap));
      } else if (ball) {
        const V6<S> ap = (l.par >= 0) ? get6(xb, 0, l.par) : a0;
        put6(xb, 0, l.lane, ball_p3(L, t, ap, o.abase.a));
      } else if constexpr (FREE) {
        root_accel(t.IA, t.pA, st_quat(st), g, t.ap, o.abase);
        const V6<S> v = st_vel6(st);
        o.abase.l = o.abase.l - cross(v.a, v.l);
        put6(xb, 0, l.lane, t.ap);
      }
    }
    wave_sync();
  }
}

template <typename S, bool FREE, bool BALL = false>
__device__ __forceinline__ void integrate_lane(State<S, FREE>& st, const Lane& l, const Step<S>& o, S dt) {
  if (l.onedof()) {
    integrate_joint(st.q[0], st.qd[0], o.t.qdd, dt);
  } else if (BALL && l.ball()) {
    if constexpr (FREE) {
      // w1 = w + dt wdot; quat1 = normalize(quat + dt/2 quat (x) (w1, 0))
      const V3<S> w1 = st_ball_w(st) + dt * o.abase.a;
      const Q4<S> q1 = quat_step(st_ball_quat(st), w1, dt);
      st.q[0] = q1.x; st.q[1] = q1.y; st.q[2] = q1.z; st.q[3] = q1.w;
      st.qd[0] = w1.x; st.qd[1] = w1.y; st.qd[2] = w1.z;
    }
  } else if constexpr (FREE) {
    if (l.jtype == 1) {
      V3<S> p = v3<S>(st.q[0], st.q[1], st.q[2]);
      Q4<S> qt = st_quat(st);
      V6<S> v = st_vel6(st);
      integrate_root(p, qt, v, o.abase, dt);
      st.q[0] = p.x; st.q[1] = p.y; st.q[2] = p.z;
      st.q[3] = qt.x; st.q[4] = qt.y; st.q[5] = qt.z; st.q[6] = qt.w;
      st.qd[0] = v.a.x; st.qd[1] = v.a.y; st.qd[2] = v.a.z;
      st.qd[3] = v.l.x; st.qd[4] = v.l.y; st.qd[5] = v.l.z;
    }
  }
}

// ------------------------------------------------------------------ kernels

template <typename S, bool FREE, int FR, bool CHAIN>
__global__ __launch_bounds__(kWave * kMaxWavesPerBlock) void k_aba(AbaArgs<S> A) {
  S* xb = CHAIN ? nullptr : lds<S>() + wave_in_block() * (XB * kWave);
  const int wb = wave_batch();
  const Lane l = load_lane(A.P, wb);
  const int maxd = A.P.wmaxd[wb];
  // every lane slot holds valid constants, so load them unconditionally
  // (keeps the compile-time axis and frame constants visible to folding)
  constexpr bool BALL = FREE && FR == kFrBall;
  const LinkC<S> L = load_linkc<S, FR>(A.P, l);
  State<S, FREE> st = {};
  V3<S> tau = zero3<S>();
  if (l.active()) {
    load_state(st, l, A.q, A.qd);
    tau = load_ctl<BALL>(A.tau, l);
  }
  Step<S> o;
  aba_wave<S, FREE, CHAIN, BALL>(gravity(A.P), l, L, st, limit_tau<FR>(A.P, l, st, tau), maxd, xb, o);
  int nonfin = 0;
  if (l.onedof()) {
    A.qdd[l.vidx] = o.t.qdd;
    nonfin = nonfinite(o.t.qdd);
  } else if (BALL && l.ball()) {
    const S a[3] = {o.abase.a.x, o.abase.a.y, o.abase.a.z};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      A.qdd[l.vidx + k] = a[k];
      nonfin += nonfinite(a[k]);
    }
  } else if constexpr (FREE) {
    if (l.jtype == 1) {
      const S a[6] = {o.abase.a.x, o.abase.a.y, o.abase.a.z, o.abase.l.x, o.abase.l.y, o.abase.l.z};
#pragma unroll
      for (int k = 0; k < 6; ++k) {
        A.qdd[l.vidx + k] = a[k];
        nonfin += nonfinite(a[k]);
      }
    }
  }
  report_nonfinite(A.P.status, nonfin);
}

// Forward rollout.  MODE 0: plain; 1: store the initial state of every
// K-th step; 2: store every step's initial state and intermediates
// (store-all).  With a trajectory buffer, also write x^{t+1} for every step.
template <typename S, bool FREE, int FR, bool CHAIN, int MODE>
__global__ __launch_bounds__(kWave * kMaxWavesPerBlock) void k_forward(FwdArgs<S> A) {
  S* xb = CHAIN ? nullptr : lds<S>() + wave_in_block() * (XB * kWave);
  const int wb = wave_batch();
  const Lane l = load_lane(A.P, wb);
  const int maxd = A.P.wmaxd[wb];
  const int ns = A.P.nslots;
  const int nu = A.P.nu;
  constexpr bool BALL = FREE && FR == kFrBall;
  const LinkC<S> L = load_linkc<S, FR>(A.P, l);
  State<S, FREE> st = {};
  if (l.active()) load_state(st, l, A.q0, A.qd0);
  V3<S> tau_next = (l.active() && A.T > 0) ? load_ctl<BALL>(A.tau, l) : zero3<S>();
  const size_t RW = state_record(ns, A.P.nfree);
  const int nf = A.P.nfree;
  int nonfin = 0;  // non-finite outputs
  for (int t = 0; t < A.T; ++t) {
    if constexpr (MODE == 1) {
      if (l.active() && (t % A.K) == 0) put_slot(st, A.ck + (size_t)(t / A.K) * RW, ns, nf, l.slot, l.fidx);
    }
    const V3<S> tau = tau_next;
    if (l.active() && t + 1 < A.T) tau_next = load_ctl<BALL>(A.tau + (size_t)(t + 1) * nu, l);
    Step<S> o;
    aba_wave<S, FREE, CHAIN, BALL>(gravity(A.P), l, L, st, limit_tau<FR>(A.P, l, st, tau), maxd, xb, o);
    if constexpr (MODE == 2) {
      if (l.active()) {
        S* row = A.ck + (size_t)t * (RW + (size_t)kTapeFields * ns);
        put_slot(st, row, ns, nf, l.slot, l.fidx);
        put_tape(o, row + RW, ns, l.slot);
      }
    }
    if (l.active()) integrate_lane<S, FREE, BALL>(st, l, o, A.dt);
    if (A.traj != nullptr) {
      if (l.active()) {
        S* row = A.traj + (size_t)t * (A.P.nq + A.P.nv);
        store_state(st, l, row, row + A.P.nq);
        nonfin += nonfinite_state(st, l);
      }
    }
  }
  if (l.active()) {
    store_state(st, l, A.qT, A.qdT);
    nonfin += nonfinite_state(st, l);
  }
  report_nonfinite(A.P.status, nonfin);
}

// One reverse step: recompute the ABA intermediates of step t from its
// initial state st, then run the adjoints of the integrator, pass 3, pass 2
// and pass 1, in the scalar type R (S, or FP64 for an FP32 forward: in FP32
// the reverse sweeps lose digits on long chains, and the rounding of FP32
// intermediates is amplified by the adjoints of chaotic rollouts).  xb1 holds the adjoint of x^{t+1} on entry and that of x^t on
// exit; tau_bar^t is written to gtau.
template <typename S, typename R, bool FREE, int FR, bool CHAIN, bool PARAMS>
__device__ __forceinline__ void bwd_reverse(const BwdArgs<S>& A, const Lane& l, const LinkC<R>& L, int maxd,
                                            R* xb, const State<R, FREE>& st, Step<R> o, int t,
                                            State<R, FREE>& xb1, int& nonfin, ParamBar<R>& pg) {
  constexpr bool BALL = FREE && FR == kFrBall;
  const bool act = l.active();
  const bool rev = l.onedof();
  const bool ball = BALL && l.ball();
  const V3<R> g = v3<R>(R(A.P.g[0]), R(A.P.g[1]), R(A.P.g[2]));
  const R dt = R(A.dt);
  Tape<R>& tp = o.t;
  // ball joint: what the stored tapes leave out (E from the quaternion,
  // c = v x [w; 0], the joint-space blocks from IA and u)
  Q4<R> bq = {R(0), R(0), R(0), R(1)};
  V3<R> bw = zero3<R>();
  Q4<R> bqb = {R(0), R(0), R(0), R(0)};
  V3<R> bwb = zero3<R>(), bqddb = zero3<R>(), bs = zero3<R>();
  BallBar<R> bb;
  ball_bar_zero(bb);
  if constexpr (BALL) {
    if (ball) {
      bq = st_ball_quat(st);
      bw = st_ball_w(st);
      tp.E = ball_E(bq, L.ET);
      tp.c = crm(tp.v, v6<R>(bw, zero3<R>()));
      tp.Ai = sy3_inv(tp.IA.A);
      tp.y = mul(tp.Ai, o.abase.l);
      tp.W = mul(sy_to_m3(tp.Ai), tp.IA.B);
      // integrator: w1 = w + dt wdot, quat1 = quat_step(quat, w1)
      const Q4<R> q1b = st_ball_quat(xb1);
      bwb = st_ball_w(xb1);
      bqb = quat_step_adj(bq, bw + dt * o.abase.a, dt, q1b, bwb);
      bqddb = dt * bwb;
    }
  }

  // adjoint of the integrator
  R acc_q = R(0), acc_qd = R(0), qddb = R(0);
  V6<R> qddb6 = zero6<R>();
  V3<R> pb = zero3<R>();
  Q4<R> quatb = {R(0), R(0), R(0), R(0)};
  V6<R> vb6 = zero6<R>();
  if (rev) {
    const R tot = xb1.qd[0] + dt * xb1.q[0];
    qddb = dt * tot;
    acc_q = xb1.q[0];
    acc_qd = tot;
  } else if constexpr (FREE) {
    if (l.jtype == 1) {
      pb = v3<R>(xb1.q[0], xb1.q[1], xb1.q[2]);
      quatb.x = xb1.q[3]; quatb.y = xb1.q[4]; quatb.z = xb1.q[5]; quatb.w = xb1.q[6];
      vb6 = st_vel6(xb1);
      const V6<R> v = st_vel6(st);
      qddb6 = integrate_root_adj(st_quat(st), v, o.abase, dt, pb, quatb, vb6);
      // the Galilean shift's term of the root acceleration, -w x v_lin
      vb6.a = vb6.a + cross(qddb6.l, v.l);
      vb6.l = vb6.l + cross(v.a, qddb6.l);
    }
  }
  Bar<R> b;
  bar_zero(b, PARAMS);
  // Each reverse sweep keeps only what a parent or child needs inside the
  // level loop; the statements that update a link's own accumulators run
  // once for all lanes outside it.
  // reverse of pass 3, leaves -> root
  SySp<R> IAb = zero_sysp<R>();
  V6<R> pAb = zero6<R>();
  V6<R> apb = zero6<R>();
  R g3 = R(0);
  if constexpr (CHAIN) {
    V6<R> up = zero6<R>();
    for (int d = maxd; d >= 0; --d) {
      const V6<R> ab = from_next(up);
      if (act && l.depth == d) {
        apb = r3_path(L, tp, ab, qddb, g3);
        if (l.par >= 0) up = xformT(tp.E, joint_r(L, tp), apb);
      }
    }
  } else {
    for (int d = maxd; d >= 0; --d) {
      if (act && l.depth == d) {
        V6<R> ab = zero6<R>();
        for (int k = 0; k < l.ccount; ++k) ab = ab + get6(xb, 0, l.cfirst + k);
        if (rev) {
          apb = r3_path(L, tp, ab, qddb, g3);
          if (l.par >= 0) put6(xb, 0, l.lane, xformT(tp.E, joint_r(L, tp), apb));
        } else if (ball) {
          apb = ball_r3_path(tp, ab, bqddb, bs);
          if (l.par >= 0) put6(xb, 0, l.lane, xformT(tp.E, L.rT, apb));
        } else if constexpr (FREE) {
          r3_root(tp.IA, tp.ap, st_quat(st), g, ab, qddb6, quatb, IAb, pAb);
        }
      }
      wave_sync();
    }
  }
  if (rev) r3_local(L, tp, b, apb, g3);
  if constexpr (BALL) {
    if (ball) ball_r3_local(tp, b, bb, apb, bs);
  }
  // reverse of pass 2, root -> leaves
  R taub = R(0);
  V3<R> btaub = zero3<R>();
  SySp<R> N = zero_sysp<R>();
  V6<R> pab = zero6<R>();
  if constexpr (CHAIN) {
    for (int d = 0; d <= maxd; ++d) {
      const SySp<R> IAbp = from_prev(IAb);
      const V6<R> pAbp = from_prev(pAb);
      if (act && l.depth == d) taub = r2_path(L, tp, b, l.par >= 0, IAbp, pAbp, N, pab, IAb, pAb);
    }
  } else {
    for (int d = 0; d <= maxd; ++d) {
      if (act && l.depth == d) {
        if (rev || ball) {
          const bool hp = l.par >= 0;
          const SySp<R> IAbp = hp ? get21(xb, 0, l.par) : zero_sysp<R>();
          const V6<R> pAbp = hp ? get6(xb, 21, l.par) : zero6<R>();
          if (rev) taub = r2_path(L, tp, b, hp, IAbp, pAbp, N, pab, IAb, pAb);
          else btaub = ball_r2_path(L, tp, bb, o.abase.l, hp, IAbp, pAbp, N, pab, IAb, pAb);
        }
        put21(xb, 0, l.lane, IAb);
        put6(xb, 21, l.lane, pAb);
      }
      wave_sync();
    }
  }
  if (rev && l.par >= 0) r2_local(L, tp, b, N, pab);
  if constexpr (BALL) {
    if (ball && l.par >= 0) ball_r2_local(tp, b, N, pab);
  }
  // inertial-parameter adjoint of this step: IAb and pAb are final here
  if constexpr (PARAMS) {
    if (A.gparam != nullptr && act) param_bar_add(pg, IAb, tp.v, pAb);
  }
  // reverse of pass 1, leaves -> root
  V6<R> own = act ? r1_own(L, tp.v, b, pAb, st.qd[0], rev) : zero6<R>();
  if constexpr (BALL) {
    if (ball) own = ball_r1_own(L, tp.v, b, pAb, bw);
  }
  V6<R> vbar = zero6<R>();
  if constexpr (CHAIN) {
    V6<R> up = zero6<R>();
    for (int d = maxd; d >= 0; --d) {
      const V6<R> vb = from_next(up);
      if (act && l.depth == d) {
        vbar = vb + own;
        if (l.par >= 0) up = xformT(tp.E, joint_r(L, tp), vbar);
      }
    }
  } else {
    for (int d = maxd; d >= 0; --d) {
      if (act && l.depth == d) {
        V6<R> vb = zero6<R>();
        for (int k = 0; k < l.ccount; ++k) vb = vb + get6(xb, 0, l.cfirst + k);
        vbar = vb + own;
        if (rev || ball) {
          if (l.par >= 0) put6(xb, 0, l.lane, xformT(tp.E, joint_r(L, tp), vbar));
        } else if constexpr (FREE) {
          // the ABA saw the root velocity [w; 0]
          vb6.a = vb6.a + vbar.a;
        }
      }
      wave_sync();
    }
  }
  if (rev) r1_local(L, tp, b, vbar, st.qd[0]);
  if constexpr (BALL) {
    if (ball) bwb = bwb + ball_r1_local(tp, b, vbar, bw);
  }
  // placement and axis adjoint of this step (every 1-dof link; a ball
  // link's placement)
  if constexpr (PARAMS) {
    if (A.gframe != nullptr && rev) {
      r2_sbar(tp, b);
      frame_bar_add(pg, L, tp, b);
    }
    if constexpr (BALL) {
      if (A.gframe != nullptr && ball) ball_frame_bar_add(pg, bq, b);
    }
  }
  // adjoint of the step's initial state; tau_bar (the joint-limit torque
  // adds its slopes times u_bar)
  if (rev) {
    R lq, lqd;
    limit_slopes<FR>(A.P, l, st, lq, lqd);
    xb1.q[0] = acc_q + b.q + lq * taub;
    xb1.qd[0] = acc_qd + b.qd + lqd * taub;
    const S taub_out = S(taub);
    A.gtau[(size_t)t * A.P.nu + l.uidx] = taub_out;
    nonfin += nonfinite(taub_out);
  } else if (ball) {
    if constexpr (BALL) {
      const Q4<R> qa = ball_quat_bar(bq, b.G.a);
      xb1.q[0] = bqb.x + qa.x; xb1.q[1] = bqb.y + qa.y; xb1.q[2] = bqb.z + qa.z; xb1.q[3] = bqb.w + qa.w;
      xb1.qd[0] = bwb.x; xb1.qd[1] = bwb.y; xb1.qd[2] = bwb.z;
      const S tb[3] = {S(btaub.x), S(btaub.y), S(btaub.z)};
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        A.gtau[(size_t)t * A.P.nu + l.uidx + k] = tb[k];
        nonfin += nonfinite(tb[k]);
      }
    }
  } else if constexpr (FREE) {
    if (l.jtype == 1) {
      xb1.q[0] = pb.x; xb1.q[1] = pb.y; xb1.q[2] = pb.z;
      xb1.q[3] = quatb.x; xb1.q[4] = quatb.y; xb1.q[5] = quatb.z; xb1.q[6] = quatb.w;
      xb1.qd[0] = vb6.a.x; xb1.qd[1] = vb6.a.y; xb1.qd[2] = vb6.a.z;
      xb1.qd[3] = vb6.l.x; xb1.qd[4] = vb6.l.y; xb1.qd[5] = vb6.l.z;
    }
  }
  if (act && A.gtraj != nullptr && t >= 1) {
    State<S, FREE> gt = {};
    const S* row = A.gtraj + (size_t)(t - 1) * (A.P.nq + A.P.nv);
    load_state(gt, l, row, row + A.P.nq);
#pragma unroll
    for (int k = 0; k < (FREE ? 7 : 1); ++k) xb1.q[k] += R(gt.q[k]);
#pragma unroll
    for (int k = 0; k < (FREE ? 6 : 1); ++k) xb1.qd[k] += R(gt.qd[k]);
  }
}

// One adjoint step from the stored state st (in the forward's type S): the
// step's intermediates are recomputed in R from the exactly widened state
// and control, then reversed in R.  With R = double for an FP32 forward the
// gradient is that of the step map at the FP32 trajectory's states to FP64
// round-off; only the outputs are rounded to FP32.  xb is sized for R.
template <typename S, typename R, bool FREE, int FR, bool CHAIN, bool PARAMS>
__device__ __forceinline__ void bwd_step(const BwdArgs<S>& A, const Lane& l, const LinkC<R>& LR, int maxd,
                                         S* xb, const State<S, FREE>& st, const V3<S>& tau, int t,
                                         State<R, FREE>& xb1, int& nonfin, ParamBar<R>& pg) {
  R* const xr = reinterpret_cast<R*>(xb);
  const State<R, FREE> sr = cvt_state<R>(st);
  Step<R> o;
  aba_wave<R, FREE, CHAIN, FREE && FR == kFrBall>(widen<R>(gravity(A.P)), l, LR, sr,
                                                          limit_tau<FR>(A.P, l, sr, cvt3<R>(tau)), maxd, xr, o);
  bwd_reverse<S, R, FREE, FR, CHAIN, PARAMS>(A, l, LR, maxd, xr, sr, o, t, xb1, nonfin, pg);
}

// Adjoint of x^T (plus the trajectory seed of the last step) in R.
template <typename S, typename R, bool FREE>
__device__ __forceinline__ State<R, FREE> seed_state(const BwdArgs<S>& A, const Lane& l) {
  State<S, FREE> x = {};
  if (l.active()) {
    load_state(x, l, A.gqT, A.gqdT);
    if (A.gtraj != nullptr && A.T > 0) {
      State<S, FREE> gt = {};
      const S* row = A.gtraj + (size_t)(A.T - 1) * (A.P.nq + A.P.nv);
      load_state(gt, l, row, row + A.P.nq);
#pragma unroll
      for (int k = 0; k < (FREE ? 7 : 1); ++k) x.q[k] += gt.q[k];
#pragma unroll
      for (int k = 0; k < (FREE ? 6 : 1); ++k) x.qd[k] += gt.qd[k];
    }
  }
  return cvt_state<R>(x);
}

// Writes the adjoints of x^0 and the model-parameter gradients; returns the
// number of non-finite values written.
template <typename S, typename R, bool FREE, bool PARAMS>
__device__ __forceinline__ int store_adjoint(const BwdArgs<S>& A, const Lane& l, const LinkC<S>& L,
                                             const State<R, FREE>& xb1, const ParamBar<R>& pg) {
  const State<S, FREE> x0 = cvt_state<S>(xb1);
  store_state(x0, l, A.gq0, A.gqd0);
  int n = nonfinite_state(x0, l);
  if constexpr (PARAMS) {
    if (A.gparam != nullptr) n += store_param_bar(pg, A.P, l, A.gparam);
    if (A.gframe != nullptr) n += store_frame_bar(pg, A.P, l, widen<R>(L), A.gframe);
  }
  return n;
}

// Backward (adjoint) rollout, reverse time.  K == 1 reloads every step's
// checkpoint; K > 1 replays each K-step segment from its checkpoint into
// the scratch buffer first.  The next state and control are fetched one
// step ahead.
// In FP32, fixed-base batches (trees, chains) run several wavefronts per
// SIMD, so the kernel is held to two waves per SIMD (at most 256 VGPRs; it
// needs a few more, which spill): otherwise the occupancy would halve.
// Free-root batches pack few lanes per system and run at most one
// wavefront per SIMD; FP64 would spill heavily under the limit.
// PARAMS: the variant that also accumulates model-parameter gradients.
// R: the scalar type of the reverse passes (see bwd_reverse); the exchange
// buffer is sized for it.
template <typename S, typename R, bool FREE, int FR, bool CHAIN, bool PARAMS>
__global__ __launch_bounds__(kWave * kMaxWavesPerBlock)
__attribute__((amdgpu_waves_per_eu((FREE || sizeof(R) > 4) ? 1 : 2))) void k_backward(BwdArgs<S> A) {
  S* xb = CHAIN ? nullptr : reinterpret_cast<S*>(lds<R>() + wave_in_block() * (XB * kWave));
  const int wb = wave_batch();
  const Lane l = load_lane(A.P, wb);
  const int maxd = A.P.wmaxd[wb];
  const int ns = A.P.nslots;
  const int nu = A.P.nu;
  constexpr bool BALL = FREE && FR == kFrBall;
  const bool act = l.active();
  const size_t RW = state_record(ns, A.P.nfree);
  const int nf = A.P.nfree;
  const LinkC<S> L = load_linkc<S, FR>(A.P, l);
  const LinkC<R> LR = widen<R>(L);
  int nonfin = 0;  // non-finite outputs
  ParamBar<R> pg;
  param_bar_zero(pg);
  State<R, FREE> xb1 = seed_state<S, R, FREE>(A, l);
  if (A.K == 0) {
    // store-all: read every step's intermediates instead of recomputing
    for (int t = A.T - 1; t >= 0; --t) {
      State<S, FREE> st = {};
      Step<S> o;
      if (act) {
        const S* row = A.ck + (size_t)t * (RW + (size_t)kTapeFields * ns);
        get_slot(st, row, ns, nf, l.slot, l.fidx);
        get_tape(o, row + RW, ns, l.slot, L, st.qd[0], l.onedof());
      }
      // the stored intermediates are the forward's (type S), widened
      bwd_reverse<S, R, FREE, FR, CHAIN, PARAMS>(A, l, LR, maxd, reinterpret_cast<R*>(xb), cvt_state<R>(st),
                                                 cvt_step<R>(o), t, xb1, nonfin, pg);
    }
  } else if (A.K == 1) {
    State<S, FREE> nxt = {};
    V3<S> tau_nxt = zero3<S>();
    if (A.T > 0 && act) {
      get_slot(nxt, A.ck + (size_t)(A.T - 1) * RW, ns, nf, l.slot, l.fidx);
      tau_nxt = load_ctl<BALL>(A.tau + (size_t)(A.T - 1) * nu, l);
    }
    for (int t = A.T - 1; t >= 0; --t) {
      const State<S, FREE> st = nxt;
      const V3<S> tau = tau_nxt;
      if (t > 0 && act) {
        get_slot(nxt, A.ck + (size_t)(t - 1) * RW, ns, nf, l.slot, l.fidx);
        tau_nxt = load_ctl<BALL>(A.tau + (size_t)(t - 1) * nu, l);
      }
      bwd_step<S, R, FREE, FR, CHAIN, PARAMS>(A, l, LR, maxd, xb, st, tau, t, xb1, nonfin, pg);
    }
  } else if (A.K < 0) {
    // binomial checkpointing: every wave runs the same host-built schedule
    // (uniform control flow; the actions are read through the scalar path)
    State<S, FREE> cur = {};
    int tc = 0;
    for (int i = 0; i < A.nsched; ++i) {
      const int op = A.sched[2 * i], arg = A.sched[2 * i + 1];
      const int what = op & 7, slot = op >> 3;
      if (what == SCH_RESTORE) {
        if (act) get_slot(cur, A.ck + (size_t)slot * RW, ns, nf, l.slot, l.fidx);
        tc = arg;
      } else if (what == SCH_ADVANCE) {
        for (int j = 0; j < arg; ++j, ++tc) {
          const V3<S> tau = act ? load_ctl<BALL>(A.tau + (size_t)tc * nu, l) : zero3<S>();
          Step<S> o;
          aba_wave<S, FREE, CHAIN, BALL>(gravity(A.P), l, L, cur, limit_tau<FR>(A.P, l, cur, tau), maxd, xb, o);
          if (act) integrate_lane<S, FREE, BALL>(cur, l, o, A.dt);
        }
      } else if (what == SCH_TAKESHOT) {
        if (act) put_slot(cur, A.ck + (size_t)slot * RW, ns, nf, l.slot, l.fidx);
      } else {
        const V3<S> tau = act ? load_ctl<BALL>(A.tau + (size_t)arg * nu, l) : zero3<S>();
        bwd_step<S, R, FREE, FR, CHAIN, PARAMS>(A, l, LR, maxd, xb, cur, tau, arg, xb1, nonfin, pg);
      }
    }
  } else {
    const int ncp = (A.T + A.K - 1) / A.K;
    for (int s = ncp - 1; s >= 0; --s) {
      const int t0 = s * A.K;
      const int t1 = min(t0 + A.K, A.T);
      // replay the segment from its checkpoint into the scratch buffer
      State<S, FREE> st = {};
      if (act) {
        get_slot(st, A.ck + (size_t)s * RW, ns, nf, l.slot, l.fidx);
        put_slot(st, A.scratch, ns, nf, l.slot, l.fidx);
      }
      V3<S> tau_nxt = (act && t1 - t0 > 1) ? load_ctl<BALL>(A.tau + (size_t)t0 * nu, l) : zero3<S>();
      for (int j = 1; j < t1 - t0; ++j) {
        const V3<S> tau = tau_nxt;
        if (act && j + 1 < t1 - t0) tau_nxt = load_ctl<BALL>(A.tau + (size_t)(t0 + j) * nu, l);
        Step<S> o;
        aba_wave<S, FREE, CHAIN, BALL>(gravity(A.P), l, L, st, limit_tau<FR>(A.P, l, st, tau), maxd, xb, o);
        if (act) {
          integrate_lane<S, FREE, BALL>(st, l, o, A.dt);
          put_slot(st, A.scratch + (size_t)j * RW, ns, nf, l.slot, l.fidx);
        }
      }
      State<S, FREE> nxt = {};
      if (act) get_slot(nxt, A.scratch + (size_t)(t1 - 1 - t0) * RW, ns, nf, l.slot, l.fidx);
      tau_nxt = act ? load_ctl<BALL>(A.tau + (size_t)(t1 - 1) * nu, l) : zero3<S>();
      for (int t = t1 - 1; t >= t0; --t) {
        const State<S, FREE> cur = nxt;
        const V3<S> tau = tau_nxt;
        if (t > t0 && act) {
          get_slot(nxt, A.scratch + (size_t)(t - 1 - t0) * RW, ns, nf, l.slot, l.fidx);
          tau_nxt = load_ctl<BALL>(A.tau + (size_t)(t - 1) * nu, l);
        }
        bwd_step<S, R, FREE, FR, CHAIN, PARAMS>(A, l, LR, maxd, xb, cur, tau, t, xb1, nonfin, pg);
      }
    }
  }
  if (act) nonfin += store_adjoint<S, R, FREE, PARAMS>(A, l, L, xb1, pg);
  report_nonfinite(A.P.status, nonfin);
}

// Pipelined adjoint for K == 1: two wavefronts per workgroup on the same
// systems.  Wave 0 (producer) reloads step t-1's checkpoint and recomputes
// its ABA intermediates while wave 1 (consumer) runs the reverse passes of
// step t; the intermediates move through a double-buffered LDS tape.  Phase
// k: the producer recomputes step T-1-k into buffer k%2 while the consumer
// reverses step T-k from buffer (k-1)%2; one workgroup barrier ends every
// phase (both waves execute exactly T+1 of them).
// LDS of one pair: the producer's and the consumer's exchange buffers, then
// the two tape buffers (all in the adjoint's type R: the producer
// recomputes in R).
template <typename S, typename R, bool FREE, int FR, bool CHAIN>
__host__ __device__ constexpr size_t pipe_lds_per_pair() {
  constexpr int TW = kTapeFields + (FREE ? 13 : 2);  // tape + state per lane
  return (size_t)((CHAIN ? 0 : 2 * XB) + 2 * TW) * kWave * sizeof(R);
}

template <typename S, typename R, bool FREE, int FR, bool CHAIN, bool PARAMS>
__global__ __launch_bounds__(2 * kWave * kMaxPairsPerBlock) void k_backward_pipe(BwdArgs<S> A) {
  constexpr int TW = kTapeFields + (FREE ? 13 : 2);
  const int pair = threadIdx.x / (2 * kWave);
  const int wid = (threadIdx.x / kWave) & 1;
  R* const base = reinterpret_cast<R*>(abadj_lds + pair * pipe_lds_per_pair<S, R, FREE, FR, CHAIN>());
  R* const xb = CHAIN ? nullptr : base + wid * (XB * kWave);
  // the two tape buffers: tape(k) = tbuf0 + (k & 1) * TW * kWave.  Offsets
  // from the LDS base (not a pointer picked from an array) keep the accesses
  // ds_* instructions rather than flat ones.
  R* const tbuf0 = base + (CHAIN ? 0 : 2 * XB * kWave);
  const int wb = blockIdx.x * (blockDim.x / (2 * kWave)) + pair;
  const Lane l = load_lane(A.P, wb);
  const int maxd = A.P.wmaxd[wb];
  const int ns = A.P.nslots;
  const int nu = A.P.nu;
  constexpr bool BALL = FREE && FR == kFrBall;
  const bool act = l.active();
  const size_t RW = state_record(ns, A.P.nfree);
  const int nf = A.P.nfree;
  const LinkC<S> L = load_linkc<S, FR>(A.P, l);
  const LinkC<R> LR = widen<R>(L);
  if (wid == 0) {
    State<S, FREE> nxt = {};
    V3<S> tau_nxt = zero3<S>();
    if (A.T > 0 && act) {
      get_slot(nxt, A.ck + (size_t)(A.T - 1) * RW, ns, nf, l.slot, l.fidx);
      tau_nxt = load_ctl<BALL>(A.tau + (size_t)(A.T - 1) * nu, l);
    }
    for (int k = 0; k <= A.T; ++k) {
      if (k < A.T) {
        const int t = A.T - 1 - k;
        const State<R, FREE> st = cvt_state<R>(nxt);
        const V3<R> tau = cvt3<R>(tau_nxt);
        if (t > 0 && act) {
          get_slot(nxt, A.ck + (size_t)(t - 1) * RW, ns, nf, l.slot, l.fidx);
          tau_nxt = load_ctl<BALL>(A.tau + (size_t)(t - 1) * nu, l);
        }
        Step<R> o;
        aba_wave<R, FREE, CHAIN, BALL>(widen<R>(gravity(A.P)), l, LR, st, limit_tau<FR>(A.P, l, st, tau), maxd, xb,
                                       o);
        R* tb = tbuf0 + (size_t)(k & 1) * (TW * kWave);
#pragma unroll
        for (int j = 0; j < (FREE ? 7 : 1); ++j) tb[(size_t)j * kWave + l.lane] = st.q[j];
#pragma unroll
        for (int j = 0; j < (FREE ? 6 : 1); ++j) tb[(size_t)((FREE ? 7 : 1) + j) * kWave + l.lane] = st.qd[j];
        put_tape(o, tb + (size_t)(FREE ? 13 : 2) * kWave, kWave, l.lane);
      }
      __syncthreads();
    }
  } else {
    int nonfin = 0;  // non-finite outputs
    ParamBar<R> pg;
    param_bar_zero(pg);
    State<R, FREE> xb1 = seed_state<S, R, FREE>(A, l);
    for (int k = 0; k <= A.T; ++k) {
      if (k >= 1) {
        const int t = A.T - k;
        const R* tb = tbuf0 + (size_t)((k - 1) & 1) * (TW * kWave);
        State<R, FREE> st;
#pragma unroll
        for (int j = 0; j < (FREE ? 7 : 1); ++j) st.q[j] = tb[(size_t)j * kWave + l.lane];
#pragma unroll
        for (int j = 0; j < (FREE ? 6 : 1); ++j) st.qd[j] = tb[(size_t)((FREE ? 7 : 1) + j) * kWave + l.lane];
        Step<R> o;
        get_tape(o, tb + (size_t)(FREE ? 13 : 2) * kWave, kWave, l.lane, LR, st.qd[0], l.onedof());
        bwd_reverse<S, R, FREE, FR, CHAIN, PARAMS>(A, l, LR, maxd, xb, st, o, t, xb1, nonfin, pg);
      }
      __syncthreads();
    }
    if (act) nonfin += store_adjoint<S, R, FREE, PARAMS>(A, l, L, xb1, pg);
    report_nonfinite(A.P.status, nonfin);
  }
}

// Forward-mode rollout: the same step as k_forward with every value carried
// as a dual number (value, derivative along the given input direction), so
// it returns x^T and d x^T = (dx^T/dx^0) dx^0 + sum_t (dx^T/du^t) du^t, and
// optionally both trajectories.  With T = 1 this is the one-step
// Jacobian-vector product behind the sample enhancement of Sec. 5.
template <typename S>
__device__ __forceinline__ LinkC<Dual<S>> dual_const(const LinkC<S>& L) {
  LinkC<Dual<S>> D;
#pragma unroll
  for (int k = 0; k < 9; ++k) D.ET.m[k] = Dual<S>(L.ET.m[k], S(0));
  D.rT = v3<Dual<S>>(Dual<S>(L.rT.x, S(0)), Dual<S>(L.rT.y, S(0)), Dual<S>(L.rT.z, S(0)));
  D.sm = v6<Dual<S>>(v3<Dual<S>>(Dual<S>(L.sm.a.x, S(0)), Dual<S>(L.sm.a.y, S(0)), Dual<S>(L.sm.a.z, S(0))),
                     v3<Dual<S>>(Dual<S>(L.sm.l.x, S(0)), Dual<S>(L.sm.l.y, S(0)), Dual<S>(L.sm.l.z, S(0))));
  D.prism = L.prism;
  D.m = Dual<S>(L.m, S(0));
  D.mc = v3<Dual<S>>(Dual<S>(L.mc.x, S(0)), Dual<S>(L.mc.y, S(0)), Dual<S>(L.mc.z, S(0)));
  D.Ib = sy3<Dual<S>>(Dual<S>(L.Ib.xx, S(0)), Dual<S>(L.Ib.yy, S(0)), Dual<S>(L.Ib.zz, S(0)),
                      Dual<S>(L.Ib.xy, S(0)), Dual<S>(L.Ib.xz, S(0)), Dual<S>(L.Ib.yz, S(0)));
  return D;
}

template <typename S, bool FREE>
__device__ __forceinline__ void split_state(const State<Dual<S>, FREE>& x, State<S, FREE>& v, State<S, FREE>& d) {
#pragma unroll
  for (int k = 0; k < (FREE ? 7 : 1); ++k) {
    v.q[k] = x.q[k].v;
    d.q[k] = x.q[k].d;
  }
#pragma unroll
  for (int k = 0; k < (FREE ? 6 : 1); ++k) {
    v.qd[k] = x.qd[k].v;
    d.qd[k] = x.qd[k].d;
  }
}

template <typename S, bool FREE, int FR, bool CHAIN>
__global__ __launch_bounds__(kWave * kMaxWavesPerBlock) void k_forward_jvp(JvpArgs<S> A) {
  using D = Dual<S>;
  D* xb = CHAIN ? nullptr : lds<D>() + wave_in_block() * (XB * kWave);
  const int wb = wave_batch();
  const Lane l = load_lane(A.P, wb);
  const int maxd = A.P.wmaxd[wb];
  const int nu = A.P.nu;
  const LinkC<D> L = dual_const(load_linkc<S, FR>(A.P, l));
  const V3<D> g = v3<D>(D(A.P.g[0], S(0)), D(A.P.g[1], S(0)), D(A.P.g[2], S(0)));
  const D dt = D(A.dt, S(0));
  State<S, FREE> sv = {}, sd = {};
  if (l.active()) {
    load_state(sv, l, A.q0, A.qd0);
    load_state(sd, l, A.dq0, A.dqd0);
  }
  State<D, FREE> st;
#pragma unroll
  for (int k = 0; k < (FREE ? 7 : 1); ++k) st.q[k] = D(sv.q[k], sd.q[k]);
#pragma unroll
  for (int k = 0; k < (FREE ? 6 : 1); ++k) st.qd[k] = D(sv.qd[k], sd.qd[k]);
  constexpr bool BALL = FREE && FR == kFrBall;
  int nonfin = 0;
  for (int t = 0; t < A.T; ++t) {
    V3<S> tv = zero3<S>(), td = zero3<S>();
    if (l.active()) {
      tv = load_ctl<BALL>(A.tau + (size_t)t * nu, l);
      td = load_ctl<BALL>(A.dtau + (size_t)t * nu, l);
    }
    const V3<D> tau = v3<D>(D(tv.x, td.x), D(tv.y, td.y), D(tv.z, td.z));
    Step<D> o;
    aba_wave<D, FREE, CHAIN, BALL>(g, l, L, st, limit_tau<FR>(A.P, l, st, tau), maxd, xb, o);
    if (l.active()) integrate_lane<D, FREE, BALL>(st, l, o, dt);
    if (A.traj != nullptr && l.active()) {
      split_state(st, sv, sd);
      S* row = A.traj + (size_t)t * (A.P.nq + A.P.nv);
      S* drow = A.dtraj + (size_t)t * (A.P.nq + A.P.nv);
      store_state(sv, l, row, row + A.P.nq);
      store_state(sd, l, drow, drow + A.P.nq);
      nonfin += nonfinite_state(sv, l) + nonfinite_state(sd, l);
    }
  }
  if (l.active()) {
    split_state(st, sv, sd);
    store_state(sv, l, A.qT, A.qdT);
    store_state(sd, l, A.dqT, A.dqdT);
    nonfin += nonfinite_state(sv, l) + nonfinite_state(sd, l);
  }
  report_nonfinite(A.P.status, nonfin);
}


// ------------------------------------------------------------ launchers
// Largest dynamic LDS one workgroup may take on the current device.
inline size_t lds_limit() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 64 * 1024;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    return 64 * 1024;
  return (size_t)v;
}

// waves per block of the single-wave kernels, reduced until the exchange
// buffers fit (the wave count is a multiple of every power of two up to
// kMaxWavesPerBlock)
template <typename S, bool C>
int single_wpb(const Tiling& tl, int nwaves, size_t& lds) {
  int w = tl.waves_per_block;
  if (w != 1 && w != 2 && w != 4) w = 1;
  const size_t per = C ? 0 : (size_t)XB * kWave * sizeof(S);
  while (w > 1 && (per * w > lds_limit() || nwaves % w != 0)) w /= 2;
  lds = per * w;
  return w;
}

// One kernel variant (FREE F, frame kind E, CHAIN C) of each entry.
template <typename S, bool F, int E, bool C>
hipError_t launch_aba_v(const AbaArgs<S>& a, const Tiling& tl, hipStream_t st) {
  if (a.P.nwaves == 0) return hipSuccess;
  size_t lds = 0;
  const int w = single_wpb<S, C>(tl, a.P.nwaves, lds);
  hipLaunchKernelGGL((k_aba<S, F, E, C>), dim3(a.P.nwaves / w), dim3(kWave * w), lds, st, a);
  return hipGetLastError();
}

template <typename S, bool F, int E, bool C>
hipError_t launch_forward_v(const FwdArgs<S>& a, const Tiling& tl, hipStream_t st) {
  if (a.P.nwaves == 0) return hipSuccess;
  const int mode = (a.ck == nullptr) ? 0 : (a.K == 0) ? 2 : 1;
  size_t lds = 0;
  const int w = single_wpb<S, C>(tl, a.P.nwaves, lds);
  const dim3 grid(a.P.nwaves / w), block(kWave * w);
  if (mode == 0) hipLaunchKernelGGL((k_forward<S, F, E, C, 0>), grid, block, lds, st, a);
  else if (mode == 1) hipLaunchKernelGGL((k_forward<S, F, E, C, 1>), grid, block, lds, st, a);
  else hipLaunchKernelGGL((k_forward<S, F, E, C, 2>), grid, block, lds, st, a);
  return hipGetLastError();
}

template <typename S, typename R, bool F, int E, bool C, bool PARAMS>
hipError_t launch_backward_p(const BwdArgs<S>& a, const Tiling& tl, hipStream_t st) {
  if (a.K == 1 && tl.pipelined) {
    const size_t per = pipe_lds_per_pair<S, R, F, E, C>();
    int p = tl.pairs_per_block == 2 ? 2 : 1;
    while (p > 1 && (per * p > lds_limit() || a.P.nwaves % p != 0)) p /= 2;
    hipLaunchKernelGGL((k_backward_pipe<S, R, F, E, C, PARAMS>), dim3(a.P.nwaves / p), dim3(2 * kWave * p),
                       per * p, st, a);
  } else {
    size_t lds = 0;
    const int w = single_wpb<R, C>(tl, a.P.nwaves, lds);
    hipLaunchKernelGGL((k_backward<S, R, F, E, C, PARAMS>), dim3(a.P.nwaves / w), dim3(kWave * w), lds, st, a);
  }
  return hipGetLastError();
}
// the kernels that accumulate model-parameter gradients only when asked for;
// R: the reverse passes' scalar type
template <typename S, typename R, bool F, int E, bool C>
hipError_t launch_backward_v(const BwdArgs<S>& a, const Tiling& tl, hipStream_t st) {
  if (a.P.nwaves == 0) return hipSuccess;
  if (a.gparam != nullptr || a.gframe != nullptr) return launch_backward_p<S, R, F, E, C, true>(a, tl, st);
  return launch_backward_p<S, R, F, E, C, false>(a, tl, st);
}

template <typename S, bool F, int E, bool C>
hipError_t launch_forward_jvp_v(const JvpArgs<S>& a, const Tiling& tl, hipStream_t st) {
  if (a.P.nwaves == 0) return hipSuccess;
  // the exchange buffers hold dual numbers
  size_t lds = 0;
  const int w = single_wpb<Dual<S>, C>(tl, a.P.nwaves, lds);
  hipLaunchKernelGGL((k_forward_jvp<S, F, E, C>), dim3(a.P.nwaves / w), dim3(kWave * w), lds, st, a);
  return hipGetLastError();
}

// Kernel variants: FREE (some system has a free-floating root), the
// link-frame kind FR (kFrIdentity: every joint frame the identity after
// canonicalisation; kFrGeneralJoints: prismatic joints or joint limits),
// CHAIN (every system is a fixed-base serial chain of revolute joints;
// register exchange between lanes).  Batches with prismatic joints or
// joint limits take the general variant (FREE, kFrGeneralJoints), which
// handles every 1-dof joint type, free roots and the limits; batches with
// ball joints the ball variant (FREE, kFrBall), which adds them (a variant
// of its own, so that the others keep their register budgets).
enum class Variant { kFree, kFreeEti, kTree, kTreeEti, kChain, kChainEti, kGeneral, kBall };

inline Variant variant(const Shape& sh) {
  if (sh.has_ball) return Variant::kBall;
  if (sh.has_prism || sh.has_limits) return Variant::kGeneral;
  if (sh.has_free) return sh.eti ? Variant::kFreeEti : Variant::kFree;
  if (sh.chain) return sh.eti ? Variant::kChainEti : Variant::kChain;
  return sh.eti ? Variant::kTreeEti : Variant::kTree;
}

}  // namespace

// One switch per entry: L<FREE, FR, CHAIN> is the per-variant launcher of
// the including translation unit (with scalar types TS...), LC<FR> the
// chain launcher of abadj_kernels_chain.hip.
#define ABADJ_DISPATCH(L, LC, ...)                                                 \
  switch (variant(sh)) {                                                          \
    case Variant::kFree: return L<__VA_ARGS__, true, kFrGeneral, false>(a, tl, st);     \
    case Variant::kFreeEti: return L<__VA_ARGS__, true, kFrIdentity, false>(a, tl, st); \
    case Variant::kTree: return L<__VA_ARGS__, false, kFrGeneral, false>(a, tl, st);    \
    case Variant::kTreeEti: return L<__VA_ARGS__, false, kFrIdentity, false>(a, tl, st); \
    case Variant::kChain: return LC<S, kFrGeneral>(a, tl, st);                    \
    case Variant::kChainEti: return LC<S, kFrIdentity>(a, tl, st);                \
    case Variant::kGeneral: return L<__VA_ARGS__, true, kFrGeneralJoints, false>(a, tl, st); \
    case Variant::kBall: return L<__VA_ARGS__, true, kFrBall, false>(a, tl, st);   \
  }                                                                               \
  return hipErrorInvalidValue;

}  // namespace aba
