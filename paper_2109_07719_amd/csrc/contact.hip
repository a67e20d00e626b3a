// Collision detection and contact resolution inside the time step
// (Sec. 4.1 "Collision resolution": detection and an MLCP solved by
// projected Gauss-Seidel between the dynamics and the integrator), batched
// over systems of one topology, and the gradient of a rollout through
// contact.
//
// Contact model: spheres fixed in links against the ground plane y = 0.
//   - a sphere is active when its centre is lower than its radius (gap
//     phi = centre_y - radius < 0);
//   - per active contact three rows (normal e_y, tangents e_x, e_z) of J,
//     the world velocity of the sphere's lowest point as a point of its
//     link;
//   - impulses lambda solve a = A lambda + b with A = J M^-1 J^T and
//     b = J qd_minus + (beta/dt) phi on the normal rows, qd_minus = qd +
//     dt qdd: first the normal rows alone with lambda_n >= 0, then all rows
//     with the tangents boxed by +-mu times those first normal impulses;
//     a row with A_ii = 0 (no joint moves the point along it) is left out;
//   - qd1 = qd_minus + M^-1 J^T lambda; the positions then move with qd1
//     (p1 = p + dt R v_lin1 and the normalised quaternion step for a free
//     root, q1 = q + dt qd1 for 1-dof joints).
//
// Design: the forward runs one lane per system, a few systems to a wave, and
// keeps the whole tree's articulated quantities in LDS (the gradient keeps
// them in private memory, see k_contact_adj).  J comes from the
// world poses and joint axes along the contact link's path to the root;
// each column of M^-1 J^T is the articulated-body response to a unit force
// at the contact point (passes 2 and 3 of the ABA with the factorisation
// of the step's own pass 2 reused, no velocity or gravity terms).  The
// gradient runs backwards in time, also one lane per system: each step is
// recomputed from the stored state, then its statements are reversed
// (contact_adjoint.h), and the adjoint of the state is carried to the
// previous step (Sec. 3, Eq. adj_back; Sec. 4.1, Eq. adj_r).
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <type_traits>

#include "../../include/abadj.h"
#include "abadj_internal.h"
#include "contact_adjoint.h"

namespace {

using namespace aba_contact;


// ---- operation count (host) --------------------------------------------------
// A counting scalar that carries its value, so that every data-dependent
// decision (detection, dropped rows, clamps) is taken as on the device:
// every +, -, *, /, sqrt, sin and cos counts 1.
thread_local long long g_cops = 0;
struct CD {
  double v = 0;
  CD() = default;
  template <typename T, typename = std::enable_if_t<std::is_arithmetic_v<T>>>
  CD(T x) : v(double(x)) {}
};
inline CD cd_(double x) { ++g_cops; return CD(x); }
inline CD operator+(CD a, CD b) { return cd_(a.v + b.v); }
inline CD operator-(CD a, CD b) { return cd_(a.v - b.v); }
inline CD operator*(CD a, CD b) { return cd_(a.v * b.v); }
inline CD operator/(CD a, CD b) { return cd_(a.v / b.v); }
inline CD operator-(CD a) { return CD(-a.v); }
inline CD& operator+=(CD& a, CD b) { a = a + b; return a; }
inline bool operator<(CD a, CD b) { return a.v < b.v; }
inline bool operator>(CD a, CD b) { return a.v > b.v; }
inline CD val(CD x) { return x; }
inline CD sq_root(CD x) { return cd_(std::sqrt(x.v)); }
inline void sin_cos(CD x, CD& s, CD& c) { s = cd_(std::sin(x.v)); c = cd_(std::cos(x.v)); }
// the terms of an unrolled sum past its true length are not counted
inline CD fmadd_pad(CD a, CD b, CD c, bool live) { return live ? a * b + c : c; }
inline CD mul_pad(CD a, CD b, bool live) { return live ? a * b : CD(0); }
inline CD add_pad(CD a, CD b, bool live) { return live ? a + b : a; }
inline CD sub_pad(CD a, CD b, bool live) { return live ? a - b : a; }

}  // namespace

namespace aba_contact {
template <>
struct Big<CD> { static constexpr double v = 1e300; };
template <>
struct RealOf<CD> { using type = CD; };
}  // namespace aba_contact

namespace {

// ---- kernels ---------------------------------------------------------------

constexpr int kWave = 64;

template <typename R>
struct RollArgs {
  CTopo tp;
  int B, T;
  R dt;
  const R* P;     // [np][B]
  const R* q0;    // [nq][B]
  const R* qd0;   // [nv][B]
  const R* tau;   // [T][nu][B]
  R* traj;        // nullable: [T + 1][nq + nv][B]
  R* qT;          // [nq][B]
  R* qdT;         // [nv][B]
  int* ncont;     // nullable: [T][B]
};

// Systems per workgroup of the rollout: each keeps its Work record in LDS
// (16 x 9.7 KB in FP32, 8 x 19.4 KB in FP64), so the step's many dependent
// accesses to the tree's articulated quantities see LDS rather than scratch
// latency.  A system is one lane; SPL systems share a wave (the workgroup's
// SPW / SPL waves spread over the CU's SIMDs).  Systems in one wave advance
// in lockstep and serialise wherever their contact sets differ, while a
// wave per system pays a full issue slot, and a full private-memory
// request, for one lane's work.  On the landing quadrupeds (4096 x 200
// steps) the rollout took 141, 134, 114, 110 and about 156 ms at 1, 2, 4, 8
// and 16 systems per wave, the FP64 reverse 4560 (scaled from 1000 steps),
// 2173, 1858 and 1578 ms at 1, 2, 4 and 8.  Fewer systems per wave spread a
// small batch over more CUs, so SPL is a launch choice (sim_contact_tiling_t,
// sim_contact_autotune): 8 (the default), 4 or 2 systems per wave, two waves
// per workgroup in FP32 and one in FP64, whose Work records are twice as
// large.
template <typename R>
constexpr int roll_spw(int spl) { return sizeof(R) == 4 ? 2 * spl : spl; }

template <typename R, int SPL>
__global__ __launch_bounds__(kWave * roll_spw<R>(SPL) / SPL) void k_contact_rollout(RollArgs<R> a) {
  constexpr int SPW = roll_spw<R>(SPL);
  static_assert(SPW * sizeof(Work<R>) <= 160 * 1024, "LDS budget");
  static_assert(SPW % SPL == 0 && SPL <= kWave, "whole waves");
  static_assert((sizeof(Work<R>) / sizeof(R)) % 2 == 1, "odd Work stride");
  __shared__ Work<R> wsh[SPW];
  const int ln = threadIdx.x % kWave;
  const int sw = (threadIdx.x / kWave) * SPL + ln;
  const int s = blockIdx.x * SPW + sw;
  if (ln >= SPL || s >= a.B) return;
  const CTopo& tp = a.tp;
  const size_t B = (size_t)a.B;
  const Par<R> P{a.P, B, s};
  const int nq = tp.nq, nv = tp.nv, nu = tp.nu, nx = nq + nv;
  R x[2][kNX], u[kNL];
  for (int k = 0; k < nq; ++k) x[0][k] = a.q0[k * B + s];
  for (int k = 0; k < nv; ++k) x[0][nq + k] = a.qd0[k * B + s];
  if (a.traj)
    for (int k = 0; k < nx; ++k) a.traj[k * B + s] = x[0][k];
  Work<R>& w = wsh[sw];
  int cur = 0;
  for (int t = 0; t < a.T; ++t) {
    for (int k = 0; k < nu; ++k) u[k] = a.tau[((size_t)t * nu + k) * B + s];
    const int na = contact_step(tp, P, x[cur], x[cur] + nq, u, a.dt, R(tp.mu), x[cur ^ 1], x[cur ^ 1] + nq, w);
    cur ^= 1;
    if (a.ncont) a.ncont[(size_t)t * B + s] = na;
    if (a.traj)
      for (int k = 0; k < nx; ++k) a.traj[((size_t)(t + 1) * nx + k) * B + s] = x[cur][k];
  }
  for (int k = 0; k < nq; ++k) a.qT[k * B + s] = x[cur][k];
  for (int k = 0; k < nv; ++k) a.qdT[k * B + s] = x[cur][nq + k];
}

template <typename R>
struct GradArgs {
  CTopo tp;
  int B, T;
  R dt;
  const R* P;     // [np][B]
  const R* traj;  // [T + 1][nq + nv][B] from the rollout
  const R* tau;   // [T][nu][B]
  const R* gqT;   // [nq][B]
  const R* gqdT;  // [nv][B]
  R* gq0;         // [nq][B]
  R* gqd0;        // [nv][B]
  R* gtau;        // [T][nu][B]
  R* gmu;         // nullable: [B]
};

// The rollout gradient by the step's reverse statements, backwards in time:
// per step, contact_step_vjp recomputes the step from the stored state and
// runs the adjoints of the integrator, the impulse update, both
// Gauss-Seidel solves (from their recorded sweep vectors), A and b, the
// unit-impulse responses, the contact geometry and the smooth ABA step.
// One lane per system; R is the arithmetic (FP64 for FP32 I/O: the
// recompute and the reverse sweeps start from the widened FP32 states, so
// the gradient is that of the step map along the FP32 trajectory).  Unlike
// the rollout, every record (Work, the sweep record, the adjoint arrays)
// stays in private memory: in FP64 the Work records alone would hold the LDS
// to 8 systems per CU, two rounds of 4096 systems, and having all systems in
// flight at once pays more than LDS latency.
// Measured on the landing quadrupeds (4096 x 200 steps, FP64 reverse): Work
// in LDS, 8 per wave, 1581 ms; private, 8 per wave 1353, 16 per wave 964,
// 32 per wave 993 ms.
// SPL is a launch choice here too (16, the default, 8 or 4 systems per wave,
// one wave per workgroup): a smaller batch reaches more CUs with fewer.
// LDS (the default): each system's Gauss-Seidel working copies (PgsStage,
// one LDS column per lane) and its copy of the articulated quantities with
// the solves' scratch (Art) sit in LDS, where the solves' and the
// responses' inner loops see LDS rather than private-memory latency; that
// holds a CU to 16 systems at a time (160 KiB).  Without it (the same
// copies in private memory) every system of a large batch is in flight at
// once; the autotuner picks.
template <typename S, typename R, int SPL, bool LDS>
__global__ __launch_bounds__(kWave) void k_contact_adj(GradArgs<S> a) {
  constexpr int SPW = SPL;
  static_assert(SPL <= kWave, "one wave per workgroup");
  __shared__ R stg[LDS ? kStage * SPW : 1];
  __shared__ Art<R> art_sh[LDS ? SPW : 1];
  const int ln = threadIdx.x % kWave;
  const int sw = (threadIdx.x / kWave) * SPL + ln;
  const int s = blockIdx.x * SPW + sw;
  if (ln >= SPL || s >= a.B) return;
  // without LDS the same staged statements run on private copies, so the
  // two placements compile to the same arithmetic (the same multiply-adds
  // fused) and give the same bits
  R stg_priv[LDS ? 1 : kStage];
  const PgsStage<R> stage{LDS ? stg + sw : stg_priv, LDS ? SPW : 1};
  Art<R> art_priv;
  Art<R>& art = LDS ? art_sh[sw] : art_priv;
  // read in place from the kernel arguments (a uniform scalar load per
  // topology entry; a local copy would live in scratch, one per lane); its
  // constants arrive rounded to S (constants_as_seen_by)
  const CTopo& tp = a.tp;
  const size_t B = (size_t)a.B;
  const Par<S> P{a.P, B, s};
  const int nq = tp.nq, nv = tp.nv, nu = tp.nu, nx = nq + nv;
  Rec<R> rc;
  Adj<R> ad;
  R xb[kNX], x[kNX], u[kNL], ub[kNL];
  for (int k = 0; k < nq; ++k) xb[k] = R(a.gqT[k * B + s]);
  for (int k = 0; k < nv; ++k) xb[nq + k] = R(a.gqdT[k * B + s]);
  R mub = R(0);
  Work<R> w;
  for (int t = a.T - 1; t >= 0; --t) {
    for (int k = 0; k < nx; ++k) x[k] = R(a.traj[((size_t)t * nx + k) * B + s]);
    for (int k = 0; k < nu; ++k) u[k] = R(a.tau[((size_t)t * nu + k) * B + s]);
    contact_step_vjp(tp, P, x, x + nq, u, a.dt, R(tp.mu), xb, ub, mub, w, rc, ad, art, stage);
    for (int k = 0; k < nu; ++k) a.gtau[((size_t)t * nu + k) * B + s] = S(ub[k]);
  }
  for (int k = 0; k < nq; ++k) a.gq0[k * B + s] = S(xb[k]);
  for (int k = 0; k < nv; ++k) a.gqd0[k * B + s] = S(xb[nq + k]);
  if (a.gmu) a.gmu[s] = S(mub);
}

int cfail(int code, const std::string& msg) { return aba::report_error(code, msg); }

// The launch geometry the model asks for (m->tiling, NULL = the defaults).
constexpr int kRollSplDefault = 8, kGradSplDefault = 16;
bool roll_spl_ok(int spl) { return spl == 8 || spl == 4 || spl == 2; }
bool grad_spl_ok(int spl) { return spl == 16 || spl == 8 || spl == 4; }

template <typename R>
hipError_t launch_rollout(const RollArgs<R>& a, int spl, hipStream_t st) {
  const int spw = roll_spw<R>(spl);
  const dim3 grid((a.B + spw - 1) / spw), block(kWave * (spw / spl));
  switch (spl) {
    case 8: hipLaunchKernelGGL((k_contact_rollout<R, 8>), grid, block, 0, st, a); break;
    case 4: hipLaunchKernelGGL((k_contact_rollout<R, 4>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((k_contact_rollout<R, 2>), grid, block, 0, st, a); break;
  }
  return hipGetLastError();
}
// The model's constants as a rollout in S saw them (rounded to S), for the
// reverse pass, which runs in FP64 for both dtypes.
template <typename S>
CTopo constants_as_seen_by(CTopo tp) {
  for (int k = 0; k < 3; ++k) tp.g[k] = double(S(tp.g[k]));
  tp.mu = double(S(tp.mu));
  tp.beta = double(S(tp.beta));
  for (int i = 0; i < kNL; ++i)
    for (int k = 0; k < 4; ++k) tp.lim[i][k] = double(S(tp.lim[i][k]));
  return tp;
}

template <typename S>
hipError_t launch_grad(const GradArgs<S>& a, int spl, bool lds, hipStream_t st) {
  // both dtypes reverse in FP64
  const dim3 grid((a.B + spl - 1) / spl), block(kWave);
  if (!lds) {
    hipLaunchKernelGGL((k_contact_adj<S, double, 16, false>), grid, block, 0, st, a);
    return hipGetLastError();
  }
  switch (spl) {
    case 16: hipLaunchKernelGGL((k_contact_adj<S, double, 16, true>), grid, block, 0, st, a); break;
    case 8: hipLaunchKernelGGL((k_contact_adj<S, double, 8, true>), grid, block, 0, st, a); break;
    default: hipLaunchKernelGGL((k_contact_adj<S, double, 4, true>), grid, block, 0, st, a); break;
  }
  return hipGetLastError();
}

int make_topo(const char* who, const sim_contact_model* m, CTopo* tp) {
  if (!m || !m->parent || !m->jtype || (m->ncontacts > 0 && !m->contact_link))
    return cfail(SIM_ERR_INVALID_ARG, std::string(who) + ": null model argument");
  if (m->n < 1 || m->n > kNL)
    return cfail(SIM_ERR_INVALID_TOPOLOGY, std::string(who) + ": need 1 <= n <= " + std::to_string(kNL));
  if (m->ncontacts < 0 || m->ncontacts > kNC)
    return cfail(SIM_ERR_INVALID_ARG, std::string(who) + ": need 0 <= ncontacts <= " + std::to_string(kNC));
  if (m->niter < 0 || !(m->mu >= 0) || !(m->beta >= 0))
    return cfail(SIM_ERR_INVALID_ARG, std::string(who) + ": need niter >= 0, mu >= 0, beta >= 0");
  if (m->tiling && (!roll_spl_ok(m->tiling->rollout_systems_per_wave) ||
                    !grad_spl_ok(m->tiling->grad_systems_per_wave) ||
                    (m->tiling->grad_lds != 0 && m->tiling->grad_lds != 1) ||
                    (m->tiling->grad_lds == 0 && m->tiling->grad_systems_per_wave != 16)))
    return cfail(SIM_ERR_INVALID_ARG, std::string(who) + ": tiling needs rollout_systems_per_wave in {8, 4, 2}, "
                                                         "grad_systems_per_wave in {16, 8, 4} and grad_lds 1, "
                                                         "or grad_systems_per_wave 16 with grad_lds 0");
  *tp = CTopo{};
  tp->n = m->n;
  tp->nc = m->ncontacts;
  tp->niter = m->niter;
  tp->mu = m->mu;
  tp->beta = m->beta;
  for (int k = 0; k < 3; ++k) tp->g[k] = m->gravity[k];
  int nq = 0, nv = 0, nu = 0;
  for (int i = 0; i < m->n; ++i) {
    const int p = m->parent[i], jt = m->jtype[i];
    if (i == 0 ? p != -1 : (p < 0 || p >= i))
      return cfail(SIM_ERR_INVALID_TOPOLOGY, std::string(who) + ": need parent[0] = -1 and 0 <= parent[i] < i");
    if (jt == SIM_JOINT_FREE ? i != 0 : (jt != SIM_JOINT_REVOLUTE && jt != SIM_JOINT_PRISMATIC))
      return cfail(SIM_ERR_INVALID_TOPOLOGY,
                   std::string(who) + ": joints must be revolute or prismatic, a free joint only at link 0");
    tp->parent[i] = p;
    tp->jtype[i] = jt;
    tp->qi[i] = nq;
    tp->vi[i] = nv;
    tp->ui[i] = nu;
    if (jt == SIM_JOINT_FREE) { nq += 7; nv += 6; }
    else { nq += 1; nv += 1; nu += 1; }
  }
  if (m->limits) {
    for (int i = 0; i < m->n; ++i) {
      if (m->jtype[i] == SIM_JOINT_FREE) continue;
      const double* L = m->limits + 4 * i;
      if (!(std::isfinite(L[0]) && std::isfinite(L[1]) && std::isfinite(L[2]) && std::isfinite(L[3])) ||
          !(L[0] <= L[1]) || !(L[2] >= 0) || !(L[3] >= 0))
        return cfail(SIM_ERR_INVALID_ARG, std::string(who) + ": joint limits need finite lo <= hi, k >= 0, d >= 0");
      for (int k = 0; k < 4; ++k) tp->lim[i][k] = L[k];
    }
    tp->has_limits = 1;
  }
  for (int k = 0; k < m->ncontacts; ++k) {
    if (m->contact_link[k] < 0 || m->contact_link[k] >= m->n)
      return cfail(SIM_ERR_INVALID_ARG, std::string(who) + ": contact_link out of range");
    tp->clink[k] = m->contact_link[k];
  }
  tp->nq = nq;
  tp->nv = nv;
  tp->nu = nu;
  tp->np = kParLink * m->n + kParSphere * m->ncontacts;
  return SIM_OK;
}

}  // namespace

extern "C" {

int sim_contact_param_count(const sim_contact_model* m, int* nq, int* nv, int* nu, int* nparams) {
  aba::clear_error();
  CTopo tp;
  const int rc = make_topo("sim_contact_param_count", m, &tp);
  if (rc) return rc;
  if (nq) *nq = tp.nq;
  if (nv) *nv = tp.nv;
  if (nu) *nu = tp.nu;
  if (nparams) *nparams = tp.np;
  return SIM_OK;
}

int sim_contact_flops(const sim_contact_model* m, const double* params, const double* q, const double* qd,
                      const double* tau, double dt, double* step_flops, double* grad_flops) {
  aba::clear_error();
  CTopo tp;
  const int rc = make_topo("sim_contact_flops", m, &tp);
  if (rc) return rc;
  if (!params || !q || !qd || (tp.nu > 0 && !tau) || !step_flops || !grad_flops)
    return cfail(SIM_ERR_INVALID_ARG, "sim_contact_flops: null argument");
  const Par<double> P{params, 1, 0};
  const int nx = tp.nq + tp.nv;
  {
    auto* w = new Work<CD>;
    CD x[kNX], x1[kNX], u[kNL];
    for (int k = 0; k < tp.nq; ++k) x[k] = CD(q[k]);
    for (int k = 0; k < tp.nv; ++k) x[tp.nq + k] = CD(qd[k]);
    for (int k = 0; k < tp.nu; ++k) u[k] = CD(tau[k]);
    g_cops = 0;
    contact_step(tp, P, x, x + tp.nq, u, dt, CD(tp.mu), x1, x1 + tp.nq, *w);
    *step_flops = (double)g_cops;
    delete w;
  }
  {
    // one reverse step: the recompute and the reverse statements
    auto* w = new Work<CD>;
    auto* rc = new Rec<CD>;
    auto* ad = new Adj<CD>;
    auto* art = new Art<CD>;
    CD x[kNX], xb[kNX], u[kNL], ub[kNL], mub(0.0);
    for (int k = 0; k < tp.nq; ++k) x[k] = CD(q[k]);
    for (int k = 0; k < tp.nv; ++k) x[tp.nq + k] = CD(qd[k]);
    for (int k = 0; k < tp.nu; ++k) u[k] = CD(tau[k]);
    for (int k = 0; k < nx; ++k) xb[k] = CD(1.0);
    g_cops = 0;
    contact_step_vjp(tp, P, x, x + tp.nq, u, dt, CD(tp.mu), xb, ub, mub, *w, *rc, *ad, *art);
    *grad_flops = (double)g_cops;
    delete w;
    delete rc;
    delete ad;
    delete art;
  }
  return SIM_OK;
}

int sim_contact_rollout(const sim_contact_model* m, int dtype, int batch, const void* params, const void* q0,
                        const void* qd0, const void* tau, double dt, int T, void* traj, void* qT, void* qdT,
                        int* ncontacts, void* stream) {
  aba::clear_error();
  CTopo tp;
  int rc = make_topo("sim_contact_rollout", m, &tp);
  if (rc) return rc;
  if (dtype != SIM_F32 && dtype != SIM_F64)
    return cfail(SIM_ERR_UNSUPPORTED_DTYPE, "sim_contact_rollout: dtype must be SIM_F32 or SIM_F64");
  if (batch < 0 || T < 0 || !(dt > 0))
    return cfail(SIM_ERR_INVALID_ARG, "sim_contact_rollout: need batch >= 0, T >= 0, dt > 0");
  if (batch == 0) return SIM_OK;
  if (!params || !q0 || !qd0 || !qT || !qdT || (T > 0 && tp.nu > 0 && !tau))
    return cfail(SIM_ERR_INVALID_ARG, "sim_contact_rollout: null array argument");
  const int spl = m->tiling ? m->tiling->rollout_systems_per_wave : kRollSplDefault;
  hipError_t e;
  if (dtype == SIM_F64) {
    RollArgs<double> a{tp, batch, T, dt, (const double*)params, (const double*)q0, (const double*)qd0,
                       (const double*)tau, (double*)traj, (double*)qT, (double*)qdT, ncontacts};
    e = launch_rollout(a, spl, (hipStream_t)stream);
  } else {
    RollArgs<float> a{tp, batch, T, (float)dt, (const float*)params, (const float*)q0, (const float*)qd0,
                      (const float*)tau, (float*)traj, (float*)qT, (float*)qdT, ncontacts};
    e = launch_rollout(a, spl, (hipStream_t)stream);
  }
  if (e != hipSuccess) return cfail(SIM_ERR_HIP, std::string("sim_contact_rollout: launch failed: ") + hipGetErrorString(e));
  return SIM_OK;
}

int sim_contact_rollout_grad(const sim_contact_model* m, int dtype, int batch, const void* params, const void* traj,
                             const void* tau, double dt, int T, const void* gqT, const void* gqdT, void* gq0,
                             void* gqd0, void* gtau, void* gmu, void* stream) {
  aba::clear_error();
  CTopo tp;
  int rc = make_topo("sim_contact_rollout_grad", m, &tp);
  if (rc) return rc;
  if (dtype != SIM_F32 && dtype != SIM_F64)
    return cfail(SIM_ERR_UNSUPPORTED_DTYPE, "sim_contact_rollout_grad: dtype must be SIM_F32 or SIM_F64");
  if (batch < 0 || T < 0 || !(dt > 0))
    return cfail(SIM_ERR_INVALID_ARG, "sim_contact_rollout_grad: need batch >= 0, T >= 0, dt > 0");
  if (m->niter > kSweepMax)
    return cfail(SIM_ERR_INVALID_ARG, "sim_contact_rollout_grad: at most " + std::to_string(kSweepMax) +
                                          " PGS sweeps (niter) are recorded for the adjoint");
  if (batch == 0) return SIM_OK;
  if (!params || !traj || !gqT || !gqdT || !gq0 || !gqd0 || (T > 0 && tp.nu > 0 && (!tau || !gtau)))
    return cfail(SIM_ERR_INVALID_ARG, "sim_contact_rollout_grad: null array argument");
  const int spl = m->tiling ? m->tiling->grad_systems_per_wave : kGradSplDefault;
  const bool lds = m->tiling ? m->tiling->grad_lds != 0 : true;
  hipError_t e;
  if (dtype == SIM_F64) {
    GradArgs<double> a{constants_as_seen_by<double>(tp), batch, T, dt, (const double*)params, (const double*)traj, (const double*)tau,
                       (const double*)gqT, (const double*)gqdT, (double*)gq0, (double*)gqd0, (double*)gtau,
                       (double*)gmu};
    e = launch_grad(a, spl, lds, (hipStream_t)stream);
  } else {
    GradArgs<float> a{constants_as_seen_by<float>(tp), batch, T, (float)dt, (const float*)params, (const float*)traj, (const float*)tau,
                      (const float*)gqT, (const float*)gqdT, (float*)gq0, (float*)gqd0, (float*)gtau,
                      (float*)gmu};
    e = launch_grad(a, spl, lds, (hipStream_t)stream);
  }
  if (e != hipSuccess)
    return cfail(SIM_ERR_HIP, std::string("sim_contact_rollout_grad: launch failed: ") + hipGetErrorString(e));
  return SIM_OK;
}

int sim_contact_autotune(const sim_contact_model* m, int dtype, int batch, const void* params, const void* q0,
                         const void* qd0, const void* tau, double dt, int T_probe, void* stream,
                         sim_contact_tiling_t* chosen, double* rollout_ms, double* grad_ms) {
  aba::clear_error();
  CTopo tp;
  int rc = make_topo("sim_contact_autotune", m, &tp);
  if (rc) return rc;
  if (dtype != SIM_F32 && dtype != SIM_F64)
    return cfail(SIM_ERR_UNSUPPORTED_DTYPE, "sim_contact_autotune: dtype must be SIM_F32 or SIM_F64");
  if (batch < 1 || T_probe < 1 || !(dt > 0))
    return cfail(SIM_ERR_INVALID_ARG, "sim_contact_autotune: need batch >= 1, T_probe >= 1, dt > 0");
  if (m->niter > kSweepMax)
    return cfail(SIM_ERR_INVALID_ARG, "sim_contact_autotune: at most " + std::to_string(kSweepMax) +
                                          " PGS sweeps (niter) are recorded for the adjoint");
  if (!params || !q0 || !qd0 || (tp.nu > 0 && !tau) || !chosen)
    return cfail(SIM_ERR_INVALID_ARG, "sim_contact_autotune: null argument");
  const hipStream_t st = (hipStream_t)stream;
  const size_t es = dtype == SIM_F64 ? sizeof(double) : sizeof(float);
  const size_t B = (size_t)batch, T = (size_t)T_probe, nq = tp.nq, nv = tp.nv, nu = tp.nu;
  // probe buffers: traj, qT, qdT, gq0, gqd0, gtau, and the zero seeds gqT, gqdT
  const size_t n_traj = (T + 1) * (nq + nv) * B, n_tau = T * nu * B;
  const size_t total = (n_traj + 2 * (nq + nv) * B + n_tau + (nq + nv) * B) * es;
  char* buf = nullptr;
  if (hipMalloc(&buf, total) != hipSuccess) return cfail(SIM_ERR_HIP, "sim_contact_autotune: probe allocation failed");
  char* p = buf;
  auto take = [&](size_t n) { char* r = p; p += n * es; return r; };
  void* traj = take(n_traj);
  void* qT = take(nq * B);
  void* qdT = take(nv * B);
  void* gq0 = take(nq * B);
  void* gqd0 = take(nv * B);
  void* gtau = take(n_tau);
  void* gqT = take(nq * B);
  void* gqdT = take(nv * B);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  sim_contact_model mm = *m;
  sim_contact_tiling_t t{kRollSplDefault, kGradSplDefault, 1};
  mm.tiling = &t;
  int best_r = kRollSplDefault, best_g = kGradSplDefault, best_l = 1;
  float ms_r = 0.f, ms_g = 0.f;
  rc = SIM_OK;
  do {
    if (hipMemsetAsync(gqT, 0, (nq + nv) * B * es, st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
      rc = cfail(SIM_ERR_HIP, "sim_contact_autotune: set-up failed");
      break;
    }
    // each geometry runs once untimed, then once between events
    auto timed = [&](auto&& run, float* ms) -> int {
      int r = run();
      if (r) return r;
      if (hipEventRecord(e0, st) != hipSuccess) return cfail(SIM_ERR_HIP, "sim_contact_autotune: event failed");
      r = run();
      if (r) return r;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
          hipEventElapsedTime(ms, e0, e1) != hipSuccess)
        return cfail(SIM_ERR_HIP, "sim_contact_autotune: timing failed");
      return SIM_OK;
    };
    const int rspl[3] = {8, 4, 2}, gspl[4] = {16, 8, 4, 16}, glds[4] = {1, 1, 1, 0};
    for (int k = 0; k < 3 && !rc; ++k) {
      t.rollout_systems_per_wave = rspl[k];
      float ms = 0.f;
      rc = timed([&] { return sim_contact_rollout(&mm, dtype, batch, params, q0, qd0, tau, dt, T_probe, traj, qT, qdT,
                                                  nullptr, stream); }, &ms);
      if (!rc && (k == 0 || ms < ms_r)) { ms_r = ms; best_r = rspl[k]; }
    }
    for (int k = 0; k < 4 && !rc; ++k) {
      t.grad_systems_per_wave = gspl[k];
      t.grad_lds = glds[k];
      float ms = 0.f;
      rc = timed([&] { return sim_contact_rollout_grad(&mm, dtype, batch, params, traj, tau, dt, T_probe, gqT, gqdT,
                                                       gq0, gqd0, gtau, nullptr, stream); }, &ms);
      if (!rc && (k == 0 || ms < ms_g)) { ms_g = ms; best_g = gspl[k]; best_l = glds[k]; }
    }
  } while (false);
  (void)hipStreamSynchronize(st);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  (void)hipFree(buf);
  if (rc) return rc;
  chosen->rollout_systems_per_wave = best_r;
  chosen->grad_systems_per_wave = best_g;
  chosen->grad_lds = best_l;
  if (rollout_ms) *rollout_ms = ms_r / T_probe;
  if (grad_ms) *grad_ms = ms_g / T_probe;
  return SIM_OK;
}

}  // extern "C"
