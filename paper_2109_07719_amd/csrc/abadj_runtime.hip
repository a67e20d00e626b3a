// Host runtime behind the C ABI of include/abadj.h: validation, breadth-first
// ordering, packing of systems into wavefronts (one lane per link), upload of
// the per-link constants, workspace sizing, kernel launches, error codes, and
// algorithmic operation counts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <tuple>
#include <type_traits>
#include <vector>

#include "../../include/abadj.h"
#include "aba_lane.h"
#include "abadj_internal.h"

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

}  // namespace

namespace aba {
// the library's one error channel (sim_last_error), for the other units
int report_error(int code, const std::string& msg) { return fail(code, msg); }
void clear_error() { g_err.clear(); }
}  // namespace aba

namespace {

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
constexpr int kMaxSnapshots = 4096;

}  // namespace

struct sim_handle {
  int dtype = SIM_F32;
  int n_sys = 0, n_links = 0, nq = 0, nv = 0, nu = 0;
  int nwaves = 0, nslots = 0, max_depth = 0, nfree = 0;
  bool has_free = false;
  bool eti = false;  // every joint frame is the identity after canonicalisation
  bool chain = false;  // every system is a fixed-base serial chain of revolute joints
  bool has_prism = false;  // some joint is prismatic
  bool has_limits = false;  // joint limits were given
  bool has_ball = false;  // some joint is spherical
  aba::Tiling tiling;  // launch geometry
  int adj_dtype = SIM_F64;  // arithmetic of the reverse passes (FP32 handles: SIM_F32 or SIM_F64)
  // binomial checkpointing schedules, one device copy per (T, s) used, kept
  // until sim_destroy (a captured graph may replay any of them)
  struct Sched {
    int T, s, n;
    std::vector<int32_t> host;  // source of the asynchronous upload, kept alive
    int32_t* dev;
  };
  std::vector<Sched> scheds;
  double g[3] = {0, 0, 0};
  int32_t* d_ci = nullptr;
  void* d_cf = nullptr;
  int32_t* d_wmaxd = nullptr;
  unsigned long long* d_status = nullptr;  // non-finite outputs written since the last sim_status
  // host-side structure summary for operation counting
  std::vector<int32_t> jtype, parent, nchild;
  // what decides the kernels' run time (the packed structure, the variant,
  // the dtype): the autotuner's cache key, with the adjoint dtype and K
  unsigned long long signature = 0;
};

namespace {

// Launch geometry before any tuning, from occupancy alone.  While the
// producer/consumer pairs of the pipelined adjoint fit one wavefront per
// SIMD, the adjoint is pipelined with two pairs per workgroup (a workgroup
// spreads its wavefronts over the CU's SIMDs, while separate one-pair
// workgroups on one CU may share SIMDs); beyond that the pipelining only
// oversubscribes the SIMDs and one wavefront per step is used.
aba::Tiling default_tiling(int nwaves) {
  aba::Tiling t;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0) cus = v;
  }
  const int simds = 4 * cus;
  t.waves_per_block = 4;
  t.pipelined = 2 * nwaves <= simds;
  t.pairs_per_block = 2;
  return t;
}

aba::Shape shape(const sim_handle* h) {
  aba::Shape sh;
  sh.has_free = h->has_free;
  sh.eti = h->eti;
  sh.chain = h->chain;
  sh.has_prism = h->has_prism;
  sh.has_limits = h->has_limits;
  sh.has_ball = h->has_ball;
  return sh;
}

template <typename S>
aba::Packed<S> packed(const sim_handle* h) {
  aba::Packed<S> P;
  P.ci = h->d_ci;
  P.cf = static_cast<const S*>(h->d_cf);
  P.wmaxd = h->d_wmaxd;
  P.status = h->d_status;
  P.nslots = h->nslots;
  P.nwaves = h->nwaves;
  P.nfree = h->nfree;
  for (int k = 0; k < 3; ++k) P.g[k] = static_cast<S>(h->g[k]);
  P.nq = h->nq;
  P.nv = h->nv;
  P.nu = h->nu;
  P.has_limits = h->has_limits ? 1 : 0;
  return P;
}

size_t elem(const sim_handle* h) { return h->dtype == SIM_F64 ? sizeof(double) : sizeof(float); }

size_t ckpt_bytes(const sim_handle* h, int T, int K) {
  const size_t rec = aba::state_record(h->nslots, h->nfree);
  if (K < 0) return align256((size_t)(1 - K) * rec * elem(h));  // x^0 and -K snapshots
  if (K == 0) return align256((size_t)T * (rec + (size_t)aba::tape_width() * h->nslots) * elem(h));
  const size_t ncp = (T > 0) ? (size_t)((T + K - 1) / K) : 0;
  return align256(ncp * rec * elem(h));
}
size_t scratch_bytes(const sim_handle* h, int K) {
  if (K <= 1) return 0;
  return align256((size_t)K * aba::state_record(h->nslots, h->nfree) * elem(h));
}

// ---- binomial checkpointing (App. B's trade-off taken to its limit: T
// steps reversed with s snapshots).  beta(s, t) = C(s + t, s) is the number
// of steps that s free snapshots can reverse when no step is advanced more
// than t times; a segment of l steps is split at m with
// l - beta(s - 1, t) <= m <= beta(s, t - 1) (t minimal with beta(s, t) >= l):
// advance m steps, snapshot, reverse the last l - m steps with s - 1 free
// snapshots, then the first m with s (the binomial recursion of Griewank's
// "revolve" checkpointing).
struct Schedule {
  std::vector<int32_t> a;  // (op, arg) pairs, see aba::SchedOp
  long long advanced = 0;  // plain steps advanced (the recompute count)
  int cur = 0;             // time of the state the schedule holds in registers
  int s_total = 0;
  void op(int what, int slot, int arg) {
    a.push_back(what + 8 * slot);
    a.push_back(arg);
  }
  void restore(int slot, int t) {
    if (cur != t) op(aba::SCH_RESTORE, slot, t);
    cur = t;
  }
};
double beta_(int s, int t) {
  double b = 1.0;  // C(s + t, s), saturating
  for (int k = 1; k <= s; ++k) {
    b = b * (double)(t + k) / (double)k;
    if (b > 1e18) return 1e18;
  }
  return b;
}
void revolve_(Schedule& S, int a, int l, int s, int slot_a) {
  while (l > 0) {
    if (l == 1) {
      S.restore(slot_a, a);
      S.op(aba::SCH_ADJOINT, 0, a);
      return;
    }
    if (s == 0) {
      for (int k = l - 1; k >= 0; --k) {
        S.restore(slot_a, a);
        if (k > 0) {
          S.op(aba::SCH_ADVANCE, 0, k);
          S.advanced += k;
          S.cur = a + k;
        }
        S.op(aba::SCH_ADJOINT, 0, a + k);
      }
      return;
    }
    int t = 1;
    while (beta_(s, t) < l) ++t;
    int m = l - (int)std::min<double>(beta_(s - 1, t), (double)l);
    m = std::max(1, std::min(m, l - 1));
    const int slot = S.s_total - s + 1;
    S.restore(slot_a, a);
    S.op(aba::SCH_ADVANCE, 0, m);
    S.advanced += m;
    S.cur = a + m;
    S.op(aba::SCH_TAKESHOT, slot, 0);
    revolve_(S, a + m, l - m, s - 1, slot);
    l = m;  // then the first m steps, with all s snapshots free again
  }
}
Schedule make_schedule(int T, int s) {
  Schedule S;
  S.s_total = s;
  S.cur = 0;  // the kernel starts from x^0 (slot 0) loaded explicitly
  S.op(aba::SCH_RESTORE, 0, 0);
  revolve_(S, 0, T, s, 0);
  return S;
}

// Rotation R with R a = e_z for a unit axis a (Rodrigues about a x e_z).
void axis_to_z(const double* a_in, double R[9]) {
  const double n = std::sqrt(a_in[0] * a_in[0] + a_in[1] * a_in[1] + a_in[2] * a_in[2]);
  const double a[3] = {a_in[0] / n, a_in[1] / n, a_in[2] / n};
  const double c = a[2];
  for (int k = 0; k < 9; ++k) R[k] = (k % 4 == 0) ? 1.0 : 0.0;
  if (c > 1.0 - 1e-15) return;
  if (c < -1.0 + 1e-15) {  // half turn about x
    R[4] = -1.0;
    R[8] = -1.0;
    return;
  }
  double k[3] = {a[1], -a[0], 0.0};  // a x e_z
  const double s = std::sqrt(k[0] * k[0] + k[1] * k[1]);
  k[0] /= s;
  k[1] /= s;
  const double K[9] = {0, -k[2], k[1], k[2], 0, -k[0], -k[1], k[0], 0};
  double K2[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) K2[3 * i + j] = K[3 * i] * K[j] + K[3 * i + 1] * K[3 + j] + K[3 * i + 2] * K[6 + j];
  for (int e = 0; e < 9; ++e) R[e] += s * K[e] + (1.0 - c) * K2[e];
}

void mat3_mul(const double* A, const double* B, double* C) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[j] + A[3 * i + 1] * B[3 + j] + A[3 * i + 2] * B[6 + j];
}
void mat3_mul_bt(const double* A, const double* B, double* C) {  // A B^T
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C[3 * i + j] = A[3 * i] * B[3 * j] + A[3 * i + 1] * B[3 * j + 1] + A[3 * i + 2] * B[3 * j + 2];
}

bool finite_all(const double* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

template <typename S>
int upload(sim_handle* h, const std::vector<int32_t>& ci, const std::vector<double>& cf,
           const std::vector<int32_t>& wmaxd) {
  std::vector<S> cfs(cf.size());
  for (size_t i = 0; i < cf.size(); ++i) cfs[i] = static_cast<S>(cf[i]);
  if (hipMalloc(&h->d_ci, ci.size() * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&h->d_cf, cfs.size() * sizeof(S)) != hipSuccess ||
      hipMalloc(&h->d_wmaxd, wmaxd.size() * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&h->d_status, sizeof(unsigned long long)) != hipSuccess)
    return fail(SIM_ERR_HIP, "sim_create: device allocation failed");
  const unsigned long long zero = 0;
  if (hipMemcpy(h->d_ci, ci.data(), ci.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_cf, cfs.data(), cfs.size() * sizeof(S), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_wmaxd, wmaxd.data(), wmaxd.size() * sizeof(int32_t), hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(h->d_status, &zero, sizeof(zero), hipMemcpyHostToDevice) != hipSuccess)
    return fail(SIM_ERR_HIP, "sim_create: upload failed");
  return SIM_OK;
}

void release(sim_handle* h) {
  if (!h) return;
  if (h->d_ci) (void)hipFree(h->d_ci);
  if (h->d_cf) (void)hipFree(h->d_cf);
  if (h->d_wmaxd) (void)hipFree(h->d_wmaxd);
  if (h->d_status) (void)hipFree(h->d_status);
  h->d_status = nullptr;
  for (auto& c : h->scheds)
    if (c.dev) (void)hipFree(c.dev);
  h->scheds.clear();
  h->d_ci = nullptr;
  h->d_cf = nullptr;
  h->d_wmaxd = nullptr;
}

}  // namespace

extern "C" {

const char* sim_last_error(void) { return g_err.c_str(); }

int sim_create(const sim_topology* topo, const sim_params* prm, int dtype, sim_t* out) {
  g_err.clear();
  if (!topo || !prm || !out) return fail(SIM_ERR_INVALID_ARG, "sim_create: null argument");
  *out = nullptr;
  if (dtype != SIM_F32 && dtype != SIM_F64) return fail(SIM_ERR_UNSUPPORTED_DTYPE, "sim_create: dtype must be SIM_F32 or SIM_F64");
  if (topo->n_sys < 1 || !topo->link_offset || !topo->parent || !topo->jtype)
    return fail(SIM_ERR_INVALID_ARG, "sim_create: empty batch or null topology array");
  if (!prm->E_T || !prm->r_T || !prm->axis || !prm->mass || !prm->com || !prm->Ic || !prm->gravity)
    return fail(SIM_ERR_INVALID_ARG, "sim_create: null parameter array");
  const int ns = topo->n_sys;
  const int32_t* off = topo->link_offset;
  if (off[0] != 0) return fail(SIM_ERR_INVALID_TOPOLOGY, "sim_create: link_offset[0] must be 0");
  for (int s = 0; s < ns; ++s) {
    const int n = off[s + 1] - off[s];
    if (n < 1 || n > SIM_MAX_LINKS)
      return fail(SIM_ERR_INVALID_TOPOLOGY, "sim_create: system " + std::to_string(s) + " has " +
                                                std::to_string(n) + " links (allowed 1.." +
                                                std::to_string(SIM_MAX_LINKS) + ")");
  }
  const int nl = off[ns];
  if (!finite_all(prm->E_T, 9 * (size_t)nl) || !finite_all(prm->r_T, 3 * (size_t)nl) ||
      !finite_all(prm->axis, 3 * (size_t)nl) || !finite_all(prm->mass, nl) || !finite_all(prm->com, 3 * (size_t)nl) ||
      !finite_all(prm->Ic, 6 * (size_t)nl) || !finite_all(prm->gravity, 3) ||
      (prm->limits && !finite_all(prm->limits, 4 * (size_t)nl)))
    return fail(SIM_ERR_INVALID_TOPOLOGY, "sim_create: non-finite parameter");
  if (prm->limits)
    for (int L = 0; L < nl; ++L) {
      const double* lm = prm->limits + 4 * (size_t)L;
      if (!(lm[0] <= lm[1]) || lm[2] < 0 || lm[3] < 0)
        return fail(SIM_ERR_INVALID_TOPOLOGY, "sim_create: joint limits need lo <= hi, k >= 0, d >= 0");
    }

  sim_handle* h = new (std::nothrow) sim_handle();
  if (!h) return fail(SIM_ERR_INVALID_ARG, "sim_create: out of host memory");
  h->dtype = dtype;
  h->n_sys = ns;
  h->n_links = nl;
  for (int k = 0; k < 3; ++k) h->g[k] = prm->gravity[k];
  h->jtype.assign(topo->jtype, topo->jtype + nl);
  h->parent.assign(topo->parent, topo->parent + nl);
  h->nchild.assign(nl, 0);

  // per system: validation, breadth-first order, depth, offsets
  std::vector<int> sys_q(ns + 1, 0), sys_v(ns + 1, 0), sys_u(ns + 1, 0), sys_depth(ns, 0);
  std::vector<int> loc_q(nl), loc_v(nl), loc_u(nl), depth(nl), bfs(nl), bfs_pos(nl);
  for (int s = 0; s < ns; ++s) {
    const int b = off[s], n = off[s + 1] - off[s];
    int q = 0, v = 0, u = 0;
    for (int i = 0; i < n; ++i) {
      const int p = topo->parent[b + i], jt = topo->jtype[b + i];
      if (p < -1 || p >= i) {
        delete h;
        return fail(SIM_ERR_INVALID_TOPOLOGY, "sim_create: system " + std::to_string(s) + " link " + std::to_string(i) +
                                                  ": parent must satisfy -1 <= parent < index");
      }
      if (jt != SIM_JOINT_REVOLUTE && jt != SIM_JOINT_FREE && jt != SIM_JOINT_PRISMATIC && jt != SIM_JOINT_SPHERICAL) {
        delete h;
        return fail(SIM_ERR_INVALID_TOPOLOGY, "sim_create: unknown joint type");
      }
      if (jt == SIM_JOINT_FREE && (i != 0 || p != -1)) {
        delete h;
        return fail(SIM_ERR_INVALID_TOPOLOGY, "sim_create: a free joint is allowed only at local index 0 with parent -1");
      }
      if (i > 0 && p == -1 && topo->jtype[b] == SIM_JOINT_FREE) {
        delete h;
        return fail(SIM_ERR_INVALID_TOPOLOGY, "sim_create: with a free root every other link needs a parent");
      }
      if (!(prm->mass[b + i] > 0)) {
        delete h;
        return fail(SIM_ERR_INVALID_TOPOLOGY, "sim_create: mass must be positive");
      }
      if (jt == SIM_JOINT_PRISMATIC) h->has_prism = true;
      if (jt == SIM_JOINT_SPHERICAL) h->has_ball = true;
      if (jt != SIM_JOINT_FREE && jt != SIM_JOINT_SPHERICAL) {
        const double* a = prm->axis + 3 * (size_t)(b + i);
        const double nrm = std::sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]);
        if (std::fabs(nrm - 1.0) > 1e-6) {
          delete h;
          return fail(SIM_ERR_INVALID_TOPOLOGY, "sim_create: joint axes must be unit vectors");
        }
      }
      depth[b + i] = (p < 0) ? 0 : depth[b + p] + 1;
      sys_depth[s] = std::max(sys_depth[s], depth[b + i]);
      if (p >= 0) h->nchild[b + p] += 1;
      loc_q[b + i] = q;
      loc_v[b + i] = v;
      loc_u[b + i] = (jt == SIM_JOINT_FREE) ? -1 : u;
      if (jt == SIM_JOINT_FREE) {
        q += 7;
        v += 6;
        h->has_free = true;
      } else if (jt == SIM_JOINT_SPHERICAL) {
        q += 4;
        v += 3;
        u += 3;
      } else {
        q += 1;
        v += 1;
        u += 1;
      }
    }
    sys_q[s + 1] = sys_q[s] + q;
    sys_v[s + 1] = sys_v[s] + v;
    sys_u[s + 1] = sys_u[s] + u;
    // breadth-first order: roots, then children of each dequeued link
    int w = 0;
    for (int i = 0; i < n; ++i)
      if (topo->parent[b + i] < 0) bfs[b + w++] = i;
    for (int r = 0; r < w; ++r) {
      const int cur = bfs[b + r];
      for (int i = cur + 1; i < n; ++i)
        if (topo->parent[b + i] == cur) bfs[b + w++] = i;
    }
    for (int k = 0; k < n; ++k) bfs_pos[b + bfs[b + k]] = k;
  }
  h->nq = sys_q[ns];
  h->nv = sys_v[ns];
  h->nu = sys_u[ns];

  // pack systems into wavefronts: group by tree depth (so a wave's
  // level-synchronous sweeps are not stretched by one deep system), largest
  // first, first fit
  std::vector<int> order(ns);
  for (int s = 0; s < ns; ++s) order[s] = s;
  std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
    if (sys_depth[a] != sys_depth[c]) return sys_depth[a] > sys_depth[c];
    return (off[a + 1] - off[a]) > (off[c + 1] - off[c]);
  });
  std::vector<int> wave_used, wave_depth, sys_wave(ns), sys_lane0(ns);
  int group_start = 0;
  for (int k = 0; k < ns; ++k) {
    const int s = order[k];
    const int n = off[s + 1] - off[s];
    if (k > 0 && sys_depth[s] != sys_depth[order[k - 1]]) group_start = (int)wave_used.size();
    int w = -1;
    for (int c = group_start; c < (int)wave_used.size(); ++c)
      if (wave_used[c] + n <= aba::kWave) {
        w = c;
        break;
      }
    if (w < 0) {
      w = (int)wave_used.size();
      wave_used.push_back(0);
      wave_depth.push_back(0);
    }
    sys_wave[s] = w;
    sys_lane0[s] = wave_used[w];
    wave_used[w] += n;
    wave_depth[w] = std::max(wave_depth[w], sys_depth[s]);
  }
  // pad with empty wavefronts so that every launch geometry divides the count
  while (wave_used.size() % aba::kMaxWavesPerBlock != 0) {
    wave_used.push_back(0);
    wave_depth.push_back(0);
  }
  h->nwaves = (int)wave_used.size();
  h->nslots = h->nwaves * aba::kWave;
  h->max_depth = 0;
  for (int d : wave_depth) h->max_depth = std::max(h->max_depth, d);

  const int NS = h->nslots;
  static const double I3[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
  std::vector<double> Rcan(9 * (size_t)nl);
  for (int L = 0; L < nl; ++L) {
    if (topo->jtype[L] != SIM_JOINT_FREE && topo->jtype[L] != SIM_JOINT_SPHERICAL)
      axis_to_z(prm->axis + 3 * (size_t)L, Rcan.data() + 9 * (size_t)L);
    else
      for (int k = 0; k < 9; ++k) Rcan[9 * (size_t)L + k] = I3[k];
  }
  bool eti = true;
  std::vector<int32_t> ci((size_t)aba::CI_COUNT * NS, 0);
  std::vector<double> cf((size_t)aba::CF_COUNT * NS, 0.0);
  for (int slot = 0; slot < NS; ++slot) ci[(size_t)aba::CI_JTYPE * NS + slot] = -1;
  for (int slot = 0; slot < NS; ++slot) ci[(size_t)aba::CI_PARENT * NS + slot] = -1;
  for (int slot = 0; slot < NS; ++slot) ci[(size_t)aba::CI_FIDX * NS + slot] = -1;
  for (int s = 0; s < ns; ++s) {
    const int b = off[s], n = off[s + 1] - off[s];
    const int base_slot = sys_wave[s] * aba::kWave + sys_lane0[s];
    for (int i = 0; i < n; ++i) {
      const int L = b + i;
      const int slot = base_slot + bfs_pos[L];
      const int lane = slot % aba::kWave;
      auto CI = [&](int f) -> int32_t& { return ci[(size_t)f * NS + slot]; };
      auto CF = [&](int f) -> double& { return cf[(size_t)f * NS + slot]; };
      const int p = topo->parent[L];
      CI(aba::CI_PARENT) = (p < 0) ? -1 : (lane - bfs_pos[L] + bfs_pos[b + p]);
      CI(aba::CI_DEPTH) = depth[L];
      int first = -1, cnt = 0;
      for (int j = i + 1; j < n; ++j)
        if (topo->parent[b + j] == i) {
          const int lj = lane - bfs_pos[L] + bfs_pos[b + j];
          if (first < 0 || lj < first) first = lj;
          ++cnt;
        }
      CI(aba::CI_CFIRST) = (cnt > 0) ? first : 0;
      CI(aba::CI_CCOUNT) = cnt;
      CI(aba::CI_JTYPE) = topo->jtype[L];
      CI(aba::CI_QIDX) = sys_q[s] + loc_q[L];
      CI(aba::CI_VIDX) = sys_v[s] + loc_v[L];
      CI(aba::CI_UIDX) = (loc_u[L] < 0) ? -1 : sys_u[s] + loc_u[L];
      // free roots and ball joints keep their state in the extended records
      if (topo->jtype[L] == SIM_JOINT_FREE || topo->jtype[L] == SIM_JOINT_SPHERICAL) CI(aba::CI_FIDX) = h->nfree++;
      CI(aba::CI_LINK) = L;
      // joint-axis canonicalisation: rotate the link frame by Rl so that its
      // axis becomes e_z (Rl = 1 for a free root or ball joint, which have
      // no axis; the parent frame was rotated by Rp):
      //   E_T' = Rl E_T Rp^T, r_T' = Rp r_T, c' = Rl c, Ic' = Rl Ic Rl^T.
      // Joint angles, velocities, torques and everything the caller sees are
      // unchanged.
      const double* Rl = Rcan.data() + 9 * (size_t)L;
      const double* Rp = (p < 0) ? I3 : Rcan.data() + 9 * (size_t)(b + p);
      double T1[9], ETn[9];
      mat3_mul(Rl, prm->E_T + 9 * (size_t)L, T1);
      mat3_mul_bt(T1, Rp, ETn);
      for (int k = 0; k < 9; ++k) CF(aba::CF_ET + k) = ETn[k];
      const double* rt = prm->r_T + 3 * (size_t)L;
      for (int k = 0; k < 3; ++k) CF(aba::CF_RT + k) = Rp[3 * k] * rt[0] + Rp[3 * k + 1] * rt[1] + Rp[3 * k + 2] * rt[2];
      CF(aba::CF_AX + 0) = 0.0;
      CF(aba::CF_AX + 1) = 0.0;
      CF(aba::CF_AX + 2) = 1.0;
      const double m = prm->mass[L];
      const double* c0 = prm->com + 3 * (size_t)L;
      const double c[3] = {Rl[0] * c0[0] + Rl[1] * c0[1] + Rl[2] * c0[2], Rl[3] * c0[0] + Rl[4] * c0[1] + Rl[5] * c0[2],
                           Rl[6] * c0[0] + Rl[7] * c0[1] + Rl[8] * c0[2]};
      const double* I0 = prm->Ic + 6 * (size_t)L;
      const double J[9] = {I0[0], I0[3], I0[4], I0[3], I0[1], I0[5], I0[4], I0[5], I0[2]};
      double T2[9], Jn[9];
      mat3_mul(Rl, J, T2);
      mat3_mul_bt(T2, Rl, Jn);
      const double I[6] = {Jn[0], Jn[4], Jn[8], Jn[1], Jn[2], Jn[5]};
      if (topo->jtype[L] != SIM_JOINT_FREE)
        for (int k = 0; k < 9; ++k) eti = eti && std::fabs(ETn[k] - I3[k]) < 1e-12;
      CF(aba::CF_M) = m;
      for (int k = 0; k < 3; ++k) CF(aba::CF_MC + k) = m * c[k];
      // inertia about the link origin: Ic - m [c]x^2 = Ic + m (|c|^2 1 - c c^T)
      CF(aba::CF_IB + 0) = I[0] + m * (c[1] * c[1] + c[2] * c[2]);
      CF(aba::CF_IB + 1) = I[1] + m * (c[0] * c[0] + c[2] * c[2]);
      CF(aba::CF_IB + 2) = I[2] + m * (c[0] * c[0] + c[1] * c[1]);
      CF(aba::CF_IB + 3) = I[3] - m * c[0] * c[1];
      CF(aba::CF_IB + 4) = I[4] - m * c[0] * c[2];
      CF(aba::CF_IB + 5) = I[5] - m * c[1] * c[2];
      for (int k = 0; k < 9; ++k) CF(aba::CF_RL + k) = Rl[k];
      const double* lm = prm->limits ? prm->limits + 4 * (size_t)L : nullptr;
      CF(aba::CF_LIM + 0) = lm ? lm[0] : -1e30;
      CF(aba::CF_LIM + 1) = lm ? lm[1] : 1e30;
      CF(aba::CF_LIM + 2) = lm ? lm[2] : 0.0;
      CF(aba::CF_LIM + 3) = lm ? lm[3] : 0.0;
    }
  }
  h->eti = eti;
  h->has_limits = prm->limits != nullptr;
  if (eti) {  // make the identity exact
    for (int slot = 0; slot < NS; ++slot)
      if (ci[(size_t)aba::CI_JTYPE * NS + slot] == SIM_JOINT_REVOLUTE ||
          ci[(size_t)aba::CI_JTYPE * NS + slot] == SIM_JOINT_PRISMATIC)
        for (int k = 0; k < 9; ++k) cf[(size_t)(aba::CF_ET + k) * NS + slot] = I3[k];
  }
  // children of a link are consecutive lanes in breadth-first order
  for (int slot = 0; slot < NS; ++slot) {
    const int cnt = ci[(size_t)aba::CI_CCOUNT * NS + slot];
    const int first = ci[(size_t)aba::CI_CFIRST * NS + slot];
    const int w = slot / aba::kWave;
    for (int k = 0; k < cnt; ++k) {
      const int cs = w * aba::kWave + first + k;
      if (ci[(size_t)aba::CI_PARENT * NS + cs] != slot % aba::kWave) {
        delete h;
        return fail(SIM_ERR_INVALID_TOPOLOGY, "sim_create: internal packing error (children not contiguous)");
      }
    }
  }
  // serial chains of revolute joints: if every non-root link's parent sits
  // in the previous lane, a lane's only possible child is the next lane, and
  // the kernels exchange parent/child quantities between neighbouring lanes'
  // registers
  bool chain = !h->has_free && !h->has_prism && !h->has_limits && !h->has_ball;
  for (int slot = 0; chain && slot < NS; ++slot) {
    const int p = ci[(size_t)aba::CI_PARENT * NS + slot];
    if (ci[(size_t)aba::CI_JTYPE * NS + slot] >= 0 && p >= 0 && p != slot % aba::kWave - 1) chain = false;
  }
  h->chain = chain;
  h->tiling = default_tiling(h->nwaves);
  std::vector<int32_t> wmaxd(wave_depth.begin(), wave_depth.end());
  {
    // FNV-1a over the structure: every packed integer field except the
    // caller's link numbering, the wave depths, the variant flags and the dtype
    unsigned long long x = 1469598103934665603ull;
    auto mix = [&](long long v) {
      for (int b = 0; b < 8; ++b) {
        x ^= (unsigned long long)((v >> (8 * b)) & 0xff);
        x *= 1099511628211ull;
      }
    };
    mix(dtype);
    mix(h->nwaves);
    mix(NS);
    mix(h->nfree);
    mix(h->has_free | h->eti << 1 | h->chain << 2 | h->has_prism << 3 | h->has_limits << 4 | h->has_ball << 5);
    for (int f = 0; f < aba::CI_COUNT; ++f)
      if (f != aba::CI_LINK)
        for (int slot = 0; slot < NS; ++slot) mix(ci[(size_t)f * NS + slot]);
    for (int32_t d : wmaxd) mix(d);
    h->signature = x;
  }
  const int rc = (dtype == SIM_F64) ? upload<double>(h, ci, cf, wmaxd) : upload<float>(h, ci, cf, wmaxd);
  if (rc != SIM_OK) {
    release(h);
    delete h;
    return rc;
  }
  *out = h;
  return SIM_OK;
}

void sim_destroy(sim_t h) {
  if (!h) return;
  release(h);
  delete h;
}

int sim_get_info(sim_t h, sim_info_t* o) {
  if (!h || !o) return fail(SIM_ERR_INVALID_ARG, "sim_get_info: null argument");
  o->n_sys = h->n_sys;
  o->n_links = h->n_links;
  o->nq = h->nq;
  o->nv = h->nv;
  o->nu = h->nu;
  o->n_waves = h->nwaves;
  o->n_slots = h->nslots;
  o->max_depth = h->max_depth;
  o->has_free = h->has_free ? 1 : 0;
  o->frames_identity = h->eti ? 1 : 0;
  o->chain = h->chain ? 1 : 0;
  o->has_prism = h->has_prism ? 1 : 0;
  o->dtype = h->dtype;
  o->adjoint_dtype = h->adj_dtype;
  o->has_ball = h->has_ball ? 1 : 0;
  return SIM_OK;
}

int sim_set_adjoint_dtype(sim_t h, int dtype) {
  g_err.clear();
  if (!h) return fail(SIM_ERR_INVALID_ARG, "sim_set_adjoint_dtype: null handle");
  if (dtype != SIM_F32 && dtype != SIM_F64)
    return fail(SIM_ERR_UNSUPPORTED_DTYPE, "sim_set_adjoint_dtype: dtype must be SIM_F32 or SIM_F64");
  if (h->dtype == SIM_F64 && dtype != SIM_F64)
    return fail(SIM_ERR_UNSUPPORTED_DTYPE, "sim_set_adjoint_dtype: an FP64 handle's adjoint runs in FP64");
  h->adj_dtype = dtype;
  return SIM_OK;
}

int sim_status(sim_t h, void* stream, int* nonfinite_count) {
  g_err.clear();
  if (!h || !nonfinite_count) return fail(SIM_ERR_INVALID_ARG, "sim_status: null argument");
  hipStream_t st = (hipStream_t)stream;
  unsigned long long v = 0;
  if (hipMemcpyAsync(&v, h->d_status, sizeof(v), hipMemcpyDeviceToHost, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess || hipMemsetAsync(h->d_status, 0, sizeof(v), st) != hipSuccess)
    return fail(SIM_ERR_HIP, "sim_status: could not read the counter");
  // a 64-bit device counter, reported saturated at INT_MAX
  *nonfinite_count = v > 2147483647ull ? 2147483647 : (int)v;
  return SIM_OK;
}

int sim_get_tiling(sim_t h, sim_tiling_t* t) {
  if (!h || !t) return fail(SIM_ERR_INVALID_ARG, "sim_get_tiling: null argument");
  t->waves_per_block = h->tiling.waves_per_block;
  t->pairs_per_block = h->tiling.pairs_per_block;
  t->pipelined = h->tiling.pipelined ? 1 : 0;
  return SIM_OK;
}

int sim_set_tiling(sim_t h, const sim_tiling_t* t) {
  if (!h || !t) return fail(SIM_ERR_INVALID_ARG, "sim_set_tiling: null argument");
  const int w = t->waves_per_block, p = t->pairs_per_block;
  if ((w != 1 && w != 2 && w != 4) || (p != 1 && p != 2) || (t->pipelined != 0 && t->pipelined != 1))
    return fail(SIM_ERR_INVALID_ARG,
                "sim_set_tiling: waves_per_block must be 1, 2 or 4, pairs_per_block 1 or 2, pipelined 0 or 1");
  h->tiling.waves_per_block = w;
  h->tiling.pairs_per_block = p;
  h->tiling.pipelined = t->pipelined != 0;
  return SIM_OK;
}

int sim_workspace_bytes(sim_t h, int T, int K, size_t* bytes) {
  if (!h || !bytes) return fail(SIM_ERR_INVALID_ARG, "sim_workspace_bytes: null argument");
  if (T < 0 || K < -kMaxSnapshots)
    return fail(SIM_ERR_INVALID_ARG, "sim_workspace_bytes: need T >= 0 and K >= -" + std::to_string(kMaxSnapshots));
  *bytes = ckpt_bytes(h, T, K) + scratch_bytes(h, K);
  return SIM_OK;
}

// The device copy of the binomial schedule for (T, s): built and uploaded
// the first time that pair is used (an allocation and an upload ordered on
// `stream`), then reused by later calls and graph captures of them.  Every
// pair keeps its own buffer until sim_destroy, so a schedule in use by an
// earlier launch or a captured graph is never overwritten.
static int ensure_schedule(sim_handle* h, int T, int s, hipStream_t stream, const int32_t** dev, int* n) {
  for (const auto& c : h->scheds)
    if (c.T == T && c.s == s) {
      *dev = c.dev;
      *n = c.n;
      return SIM_OK;
    }
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(stream, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(SIM_ERR_INVALID_ARG, "sim_backward: the first call with a new (T, K < 0) uploads its checkpointing "
                                     "schedule and cannot be captured; run it once outside the capture");
  Schedule S = make_schedule(T, s);
  sim_handle::Sched c;
  c.T = T;
  c.s = s;
  c.n = (int)(S.a.size() / 2);
  c.host = std::move(S.a);
  c.dev = nullptr;
  const size_t bytes = std::max<size_t>(c.host.size(), 2) * sizeof(int32_t);
  if (hipMalloc(&c.dev, bytes) != hipSuccess) return fail(SIM_ERR_HIP, "sim_backward: schedule allocation failed");
  if (!c.host.empty() &&
      hipMemcpyAsync(c.dev, c.host.data(), c.host.size() * sizeof(int32_t), hipMemcpyHostToDevice, stream) !=
          hipSuccess) {
    (void)hipFree(c.dev);
    return fail(SIM_ERR_HIP, "sim_backward: schedule upload failed");
  }
  h->scheds.push_back(std::move(c));
  *dev = h->scheds.back().dev;
  *n = h->scheds.back().n;
  return SIM_OK;
}

int sim_checkpoint_schedule(int T, int s, int32_t* actions, int capacity, int* n_actions, long long* advanced) {
  g_err.clear();
  if (T < 0 || s < 1 || s > kMaxSnapshots || !n_actions)
    return fail(SIM_ERR_INVALID_ARG, "sim_checkpoint_schedule: need T >= 0, 1 <= s <= " +
                                         std::to_string(kMaxSnapshots) + " and n_actions");
  const Schedule S = make_schedule(T, s);
  *n_actions = (int)(S.a.size() / 2);
  if (advanced) *advanced = S.advanced;
  if (actions) {
    if (capacity < *n_actions) return fail(SIM_ERR_INVALID_ARG, "sim_checkpoint_schedule: capacity too small");
    std::memcpy(actions, S.a.data(), S.a.size() * sizeof(int32_t));
  }
  return SIM_OK;
}

static int check_run(sim_t h, double dt, int T, int K, const char* who) {
  if (!h) return fail(SIM_ERR_INVALID_ARG, std::string(who) + ": null handle");
  if (T < 0) return fail(SIM_ERR_INVALID_ARG, std::string(who) + ": T must be >= 0");
  if (K < -kMaxSnapshots)
    return fail(SIM_ERR_INVALID_ARG, std::string(who) + ": K must be >= -" + std::to_string(kMaxSnapshots) +
                                         " (K < 0: binomial checkpointing with -K snapshots; 0: store-all)");
  if (!std::isfinite(dt) || !(dt > 0)) return fail(SIM_ERR_INVALID_ARG, std::string(who) + ": dt must be finite and > 0");
  return SIM_OK;
}

int sim_forward(sim_t h, const void* q0, const void* qd0, const void* tau, double dt, int T, int K, void* qT,
                void* qdT, void* traj, void* workspace, size_t workspace_bytes, void* stream) {
  g_err.clear();
  int rc = check_run(h, dt, T, K, "sim_forward");
  if (rc) return rc;
  if (!q0 || !qd0 || !qT || !qdT || (T > 0 && h->nu > 0 && !tau))
    return fail(SIM_ERR_INVALID_ARG, "sim_forward: null array argument");
  if (workspace) {
    size_t need = 0;
    sim_workspace_bytes(h, T, K, &need);
    if (workspace_bytes < need)
      return fail(SIM_ERR_WORKSPACE_TOO_SMALL, "sim_forward: workspace of " + std::to_string(workspace_bytes) +
                                                   " bytes, need " + std::to_string(need));
  }
  hipError_t e;
  if (h->dtype == SIM_F64) {
    aba::FwdArgs<double> a;
    a.P = packed<double>(h);
    a.dt = dt;
    a.T = T;
    a.K = (K < 0) ? std::max(T, 1) : K;  // K < 0: only x^0 is stored
    a.q0 = (const double*)q0;
    a.qd0 = (const double*)qd0;
    a.tau = (const double*)tau;
    a.qT = (double*)qT;
    a.qdT = (double*)qdT;
    a.traj = (double*)traj;
    a.ck = (double*)workspace;
    e = aba::launch_forward(a, shape(h), h->tiling, (hipStream_t)stream);
  } else {
    aba::FwdArgs<float> a;
    a.P = packed<float>(h);
    a.dt = (float)dt;
    a.T = T;
    a.K = (K < 0) ? std::max(T, 1) : K;  // K < 0: only x^0 is stored
    a.q0 = (const float*)q0;
    a.qd0 = (const float*)qd0;
    a.tau = (const float*)tau;
    a.qT = (float*)qT;
    a.qdT = (float*)qdT;
    a.traj = (float*)traj;
    a.ck = (float*)workspace;
    e = aba::launch_forward(a, shape(h), h->tiling, (hipStream_t)stream);
  }
  if (e != hipSuccess) return fail(SIM_ERR_HIP, std::string("sim_forward: launch failed: ") + hipGetErrorString(e));
  return SIM_OK;
}

}  // extern "C"

// The adjoint pass behind sim_backward and sim_backward_noalloc.  replay:
// nullptr = the K > 1 replay buffer follows the checkpoints in the
// workspace; otherwise the device buffer to use for it (the workspace then
// needs only the checkpoints).
static int backward_impl(const char* who, sim_t h, const void* tau, double dt, int T, int K, const void* gqT,
                         const void* gqdT, const void* gtraj, void* gq0, void* gqd0, void* gtau, void* gparam,
                         void* gframe, void* workspace, size_t workspace_bytes, void* replay, void* stream) {
  int rc = check_run(h, dt, T, K, who);
  if (rc) return rc;
  if (!gqT || !gqdT || !gq0 || !gqd0 || (T > 0 && h->nu > 0 && (!tau || !gtau)) || (T > 0 && !workspace))
    return fail(SIM_ERR_INVALID_ARG, std::string(who) + ": null array argument");
  const size_t ck = ckpt_bytes(h, T, K);
  size_t need = 0;
  sim_workspace_bytes(h, T, K, &need);
  if (replay) need = ck;
  if (T > 0 && workspace_bytes < need)
    return fail(SIM_ERR_WORKSPACE_TOO_SMALL, std::string(who) + ": workspace of " +
                                                 std::to_string(workspace_bytes) + " bytes, need " +
                                                 std::to_string(need));
  const int32_t* sched = nullptr;
  int nsched = 0;
  if (K < 0) {
    rc = ensure_schedule(h, T, -K, (hipStream_t)stream, &sched, &nsched);
    if (rc) return rc;
  }
  void* const rbuf = replay ? replay : (void*)((char*)workspace + ck);
  hipError_t e;
  if (h->dtype == SIM_F64) {
    aba::BwdArgs<double> a;
    a.P = packed<double>(h);
    a.dt = dt;
    a.T = T;
    a.K = K;
    a.tau = (const double*)tau;
    a.gqT = (const double*)gqT;
    a.gqdT = (const double*)gqdT;
    a.gtraj = (const double*)gtraj;
    a.gq0 = (double*)gq0;
    a.gqd0 = (double*)gqd0;
    a.gtau = (double*)gtau;
    a.ck = (double*)workspace;
    a.scratch = (K > 1) ? (double*)rbuf : nullptr;
    a.sched = sched;
    a.nsched = nsched;
    a.adj64 = 0;
    a.gparam = (double*)gparam;
    a.gframe = (double*)gframe;
    e = aba::launch_backward(a, shape(h), h->tiling, (hipStream_t)stream);
  } else {
    aba::BwdArgs<float> a;
    a.P = packed<float>(h);
    a.dt = (float)dt;
    a.T = T;
    a.K = K;
    a.tau = (const float*)tau;
    a.gqT = (const float*)gqT;
    a.gqdT = (const float*)gqdT;
    a.gtraj = (const float*)gtraj;
    a.gq0 = (float*)gq0;
    a.gqd0 = (float*)gqd0;
    a.gtau = (float*)gtau;
    a.ck = (float*)workspace;
    a.scratch = (K > 1) ? (float*)rbuf : nullptr;
    a.sched = sched;
    a.nsched = nsched;
    a.adj64 = h->adj_dtype == SIM_F64 ? 1 : 0;
    a.gparam = (float*)gparam;
    a.gframe = (float*)gframe;
    e = aba::launch_backward(a, shape(h), h->tiling, (hipStream_t)stream);
  }
  if (e != hipSuccess) return fail(SIM_ERR_HIP, std::string(who) + ": launch failed: " + hipGetErrorString(e));
  return SIM_OK;
}

// ---- the adjoint pass without allocation.  The K > 1 replay buffer lives
// in a file-scope device array, one copy per GPU, kept until the process
// ends.  In host code `scratch` only names the symbol: its device address
// on each GPU comes from hipGetSymbolAddress, taken once per device with
// that device current, and only that address is handed to kernels.
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
constexpr int kMaxDevices = 64;
}  // namespace
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this GPU's scratch array (looked up on first use).
static int noalloc_scratch(void** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(SIM_ERR_HIP, "sim_backward_noalloc: no current device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(SIM_ERR_HIP, std::string("sim_backward_noalloc: scratch address lookup failed: ") +
                                   hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return SIM_OK;
}

extern "C" {

int sim_backward(sim_t h, const void* tau, double dt, int T, int K, const void* gqT, const void* gqdT,
                 const void* gtraj, void* gq0, void* gqd0, void* gtau, void* gparam, void* gframe,
                 void* workspace, size_t workspace_bytes, void* stream) {
  g_err.clear();
  return backward_impl("sim_backward", h, tau, dt, T, K, gqT, gqdT, gtraj, gq0, gqd0, gtau, gparam, gframe,
                       workspace, workspace_bytes, nullptr, stream);
}

int sim_backward_noalloc(sim_t h, const void* tau, double dt, int T, int K, const void* gqT, const void* gqdT,
                         const void* gtraj, void* gq0, void* gqd0, void* gtau, void* gparam, void* gframe,
                         void* checkpoints, size_t checkpoint_bytes, void* stream) {
  g_err.clear();
  if (!h) return fail(SIM_ERR_INVALID_ARG, "sim_backward_noalloc: null handle");
  if (K < 0)
    return fail(SIM_ERR_INVALID_ARG, "sim_backward_noalloc: binomial checkpointing (K < 0) is not available "
                                     "without allocation; use K >= 0");
  const size_t rep = scratch_bytes(h, K);
  if (rep > kNoAllocScratchBytes)
    return fail(SIM_ERR_WORKSPACE_TOO_SMALL, "sim_backward_noalloc: the K = " + std::to_string(K) +
                                                 " replay buffer needs " + std::to_string(rep) +
                                                 " bytes, above the library's static scratch of " +
                                                 std::to_string(kNoAllocScratchBytes) + " bytes");
  void* buf = nullptr;
  const int rc = noalloc_scratch(&buf);
  if (rc) return rc;
  return backward_impl("sim_backward_noalloc", h, tau, dt, T, K, gqT, gqdT, gtraj, gq0, gqd0, gtau, gparam,
                       gframe, checkpoints, checkpoint_bytes, buf, stream);
}

int sim_forward_jvp(sim_t h, const void* q0, const void* qd0, const void* tau, const void* dq0, const void* dqd0,
                    const void* dtau, double dt, int T, void* qT, void* qdT, void* dqT, void* dqdT, void* traj,
                    void* dtraj, void* stream) {
  g_err.clear();
  int rc = check_run(h, dt, T, 1, "sim_forward_jvp");
  if (rc) return rc;
  if (!q0 || !qd0 || !dq0 || !dqd0 || !qT || !qdT || !dqT || !dqdT || (T > 0 && h->nu > 0 && (!tau || !dtau)))
    return fail(SIM_ERR_INVALID_ARG, "sim_forward_jvp: null array argument");
  if ((traj == nullptr) != (dtraj == nullptr))
    return fail(SIM_ERR_INVALID_ARG, "sim_forward_jvp: traj and dtraj must both be given or both be NULL");
  hipError_t e;
  auto fill = [&](auto& a, auto* tag) {
    using S = std::remove_pointer_t<decltype(tag)>;
    a.P = packed<S>(h);
    a.dt = (S)dt;
    a.T = T;
    a.q0 = (const S*)q0;
    a.qd0 = (const S*)qd0;
    a.tau = (const S*)tau;
    a.dq0 = (const S*)dq0;
    a.dqd0 = (const S*)dqd0;
    a.dtau = (const S*)dtau;
    a.qT = (S*)qT;
    a.qdT = (S*)qdT;
    a.dqT = (S*)dqT;
    a.dqdT = (S*)dqdT;
    a.traj = (S*)traj;
    a.dtraj = (S*)dtraj;
  };
  if (h->dtype == SIM_F64) {
    aba::JvpArgs<double> a;
    fill(a, (double*)nullptr);
    e = aba::launch_forward_jvp(a, shape(h), h->tiling, (hipStream_t)stream);
  } else {
    aba::JvpArgs<float> a;
    fill(a, (float*)nullptr);
    e = aba::launch_forward_jvp(a, shape(h), h->tiling, (hipStream_t)stream);
  }
  if (e != hipSuccess) return fail(SIM_ERR_HIP, std::string("sim_forward_jvp: launch failed: ") + hipGetErrorString(e));
  return SIM_OK;
}

int sim_aba(sim_t h, const void* q, const void* qd, const void* tau, void* qdd, void* stream) {
  g_err.clear();
  if (!h || !q || !qd || !qdd || (h->nu > 0 && !tau)) return fail(SIM_ERR_INVALID_ARG, "sim_aba: null argument");
  hipError_t e;
  if (h->dtype == SIM_F64) {
    aba::AbaArgs<double> a;
    a.P = packed<double>(h);
    a.q = (const double*)q;
    a.qd = (const double*)qd;
    a.tau = (const double*)tau;
    a.qdd = (double*)qdd;
    e = aba::launch_aba(a, shape(h), h->tiling, (hipStream_t)stream);
  } else {
    aba::AbaArgs<float> a;
    a.P = packed<float>(h);
    a.q = (const float*)q;
    a.qd = (const float*)qd;
    a.tau = (const float*)tau;
    a.qdd = (float*)qdd;
    e = aba::launch_aba(a, shape(h), h->tiling, (hipStream_t)stream);
  }
  if (e != hipSuccess) return fail(SIM_ERR_HIP, std::string("sim_aba: launch failed: ") + hipGetErrorString(e));
  return SIM_OK;
}

}  // extern "C"

namespace {
// The autotuner's choices, per process: (signature, adjoint dtype, K,
// T_probe, device) -> (tiling, ms per probe step).
struct TuneKey {
  unsigned long long sig;
  int adj, K, T, dev;
  bool operator<(const TuneKey& o) const {
    return std::tie(sig, adj, K, T, dev) < std::tie(o.sig, o.adj, o.K, o.T, o.dev);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, std::pair<aba::Tiling, double>> g_tune;
}  // namespace

extern "C" {

void sim_autotune_cache_clear(void) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  g_tune.clear();
}

int sim_autotune(sim_t h, int K, int T_probe, void* stream, sim_tiling_t* chosen, double* ms_per_step) {
  g_err.clear();
  if (!h) return fail(SIM_ERR_INVALID_ARG, "sim_autotune: null handle");
  if (K < -kMaxSnapshots || T_probe < 1 || T_probe > 100000)
    return fail(SIM_ERR_INVALID_ARG, "sim_autotune: need K >= -" + std::to_string(kMaxSnapshots) +
                                         " and 1 <= T_probe <= 100000");
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(SIM_ERR_HIP, "sim_autotune: no current device");
  const TuneKey key{h->signature, h->dtype == SIM_F32 ? h->adj_dtype : SIM_F64, K, T_probe, dev};
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    const auto it = g_tune.find(key);
    if (it != g_tune.end()) {
      h->tiling = it->second.first;
      if (chosen) {
        chosen->waves_per_block = h->tiling.waves_per_block;
        chosen->pairs_per_block = h->tiling.pairs_per_block;
        chosen->pipelined = h->tiling.pipelined ? 1 : 0;
      }
      if (ms_per_step) *ms_per_step = it->second.second;
      return SIM_OK;
    }
  }
  hipStream_t st = (hipStream_t)stream;
  const size_t es = elem(h);
  // store-all probes are capped at 2 GiB of workspace
  int T = T_probe;
  if (K == 0) {
    size_t per = 0;
    sim_workspace_bytes(h, 1, 0, &per);
    while (T > 8 && (size_t)T * per > (size_t(2) << 30)) T /= 2;
  }
  size_t ws_bytes = 0;
  sim_workspace_bytes(h, T, K, &ws_bytes);
  const size_t nq = h->nq, nv = h->nv, nu = h->nu;
  // probe rollout: zero state (unit quaternions on free roots), zero
  // torques, zero seeds; the kernels' run time does not depend on values
  std::vector<double> q0h(nq, 0.0);
  for (size_t L = 0, qi = 0; L < h->jtype.size(); ++L) {
    if (h->jtype[L] == SIM_JOINT_FREE) {
      q0h[qi + 6] = 1.0;
      qi += 7;
    } else if (h->jtype[L] == SIM_JOINT_SPHERICAL) {
      q0h[qi + 3] = 1.0;
      qi += 4;
    } else {
      qi += 1;
    }
  }
  std::vector<unsigned char> q0b(nq * es);
  for (size_t i = 0; i < nq; ++i) {
    if (es == sizeof(double)) {
      std::memcpy(q0b.data() + i * es, &q0h[i], es);
    } else {
      const float f = (float)q0h[i];
      std::memcpy(q0b.data() + i * es, &f, es);
    }
  }
  const size_t sizes[] = {nq, nv, nu * T, nq, nv, nq, nv, nq, nv, nu * T};
  void* buf[10] = {};
  void* ws = nullptr;
  hipEvent_t ev[2] = {nullptr, nullptr};
  const aba::Tiling saved = h->tiling;
  auto cleanup = [&]() {
    for (void* b : buf) if (b) (void)hipFree(b);
    if (ws) (void)hipFree(ws);
    for (hipEvent_t x : ev) if (x) (void)hipEventDestroy(x);
  };
  bool ok = hipEventCreate(&ev[0]) == hipSuccess && hipEventCreate(&ev[1]) == hipSuccess;
  for (int i = 0; ok && i < 10; ++i) ok = hipMalloc(&buf[i], std::max<size_t>(sizes[i], 1) * es) == hipSuccess;
  ok = ok && hipMalloc(&ws, std::max<size_t>(ws_bytes, 1)) == hipSuccess;
  for (int i = 0; ok && i < 10; ++i) ok = hipMemsetAsync(buf[i], 0, std::max<size_t>(sizes[i], 1) * es, st) == hipSuccess;
  ok = ok && (nq == 0 || hipMemcpyAsync(buf[0], q0b.data(), nq * es, hipMemcpyHostToDevice, st) == hipSuccess);
  ok = ok && hipStreamSynchronize(st) == hipSuccess;
  if (!ok) {
    cleanup();
    return fail(SIM_ERR_HIP, "sim_autotune: could not allocate or initialise the probe buffers");
  }
  void *q0 = buf[0], *qd0 = buf[1], *tau = buf[2], *qT = buf[3], *qdT = buf[4], *gqT = buf[5], *gqdT = buf[6],
       *gq0 = buf[7], *gqd0 = buf[8], *gtau = buf[9];
  const double dt = 1e-3;
  // best of three timed launches after one untimed
  auto timed = [&](auto&& launch, double& best) -> bool {
    if (launch() != SIM_OK) return false;
    best = 1e300;
    for (int r = 0; r < 3; ++r) {
      if (hipEventRecord(ev[0], st) != hipSuccess || launch() != SIM_OK || hipEventRecord(ev[1], st) != hipSuccess ||
          hipEventSynchronize(ev[1]) != hipSuccess)
        return false;
      float ms = 0;
      if (hipEventElapsedTime(&ms, ev[0], ev[1]) != hipSuccess) return false;
      best = std::min(best, (double)ms);
    }
    return true;
  };
  auto fwd = [&]() { return sim_forward(h, q0, qd0, tau, dt, T, K, qT, qdT, nullptr, ws, ws_bytes, stream); };
  auto bwd = [&]() {
    return sim_backward(h, tau, dt, T, K, gqT, gqdT, nullptr, gq0, gqd0, gtau, nullptr, nullptr, ws, ws_bytes,
                        stream);
  };
  const int wpbs[3] = {1, 2, 4};
  double F[3], Bnp[3], Bp[2] = {1e300, 1e300};
  ok = true;
  for (int i = 0; ok && i < 3; ++i) {
    h->tiling.waves_per_block = wpbs[i];
    h->tiling.pipelined = false;
    ok = timed(fwd, F[i]) && timed(bwd, Bnp[i]);
  }
  for (int p = 1; ok && K == 1 && p <= 2; ++p) {
    h->tiling.pipelined = true;
    h->tiling.pairs_per_block = p;
    ok = timed(bwd, Bp[p - 1]);
  }
  if (!ok) {
    h->tiling = saved;
    const std::string msg = g_err.empty() ? std::string("HIP call failed") : g_err;
    cleanup();
    return fail(SIM_ERR_HIP, "sim_autotune: probe failed: " + msg);
  }
  // forward and non-pipelined adjoint share waves_per_block
  double best = 1e300;
  aba::Tiling win;
  for (int i = 0; i < 3; ++i) {
    for (int c = 0; c < 3; ++c) {  // c = 0: one-wave adjoint; 1, 2: pipelined with c pairs
      const double b = (c == 0) ? Bnp[i] : Bp[c - 1];
      if (F[i] + b < best) {
        best = F[i] + b;
        win.waves_per_block = wpbs[i];
        win.pipelined = c > 0;
        win.pairs_per_block = c > 0 ? c : saved.pairs_per_block;
      }
    }
  }
  h->tiling = win;
  cleanup();
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[key] = {win, best / T};
  }
  if (chosen) {
    chosen->waves_per_block = win.waves_per_block;
    chosen->pairs_per_block = win.pairs_per_block;
    chosen->pipelined = win.pipelined ? 1 : 0;
  }
  if (ms_per_step) *ms_per_step = best / T;
  return SIM_OK;
}

}  // extern "C"

// ------------------------------------------------------------ operation counts
namespace {

thread_local long long g_ops = 0;

// Counting scalar with the constant folding the kernels' build flags allow
// (x*0 -> 0, x+0 -> x, x*1 -> x, x-0 -> x, 0-x -> -x): operations with a
// known zero or one operand are free, every other +, -, *, /, sqrt counts 1.
struct Op {
  int k = 2;  // 0: the constant 0, 1: the constant 1, 2: any other value
  Op() = default;
  Op(double x) : k(x == 0.0 ? 0 : (x == 1.0 ? 1 : 2)) {}
};
inline Op var_() {
  Op o;
  o.k = 2;
  return o;
}
inline Op operator+(Op a, Op b) {
  if (a.k == 0) return b;
  if (b.k == 0) return a;
  ++g_ops;
  return var_();
}
inline Op operator-(Op a, Op b) {
  if (b.k == 0) return a;
  if (a.k == 0) return var_();
  ++g_ops;
  return var_();
}
inline Op operator*(Op a, Op b) {
  if (a.k == 0 || b.k == 0) return Op(0.0);
  if (a.k == 1) return b;
  if (b.k == 1) return a;
  ++g_ops;
  return var_();
}
inline Op operator/(Op a, Op b) {
  if (a.k == 0) return Op(0.0);
  if (b.k == 1) return a;
  ++g_ops;
  return var_();
}
inline Op operator-(Op a) { return a.k == 0 ? a : var_(); }
inline Op sqrt(Op) {
  ++g_ops;
  return var_();
}

template <typename F>
long long count(F&& f) {
  g_ops = 0;
  f();
  return g_ops;
}

struct LinkOps {
  long long fd_rev, fd_rev_push, p1_root_rev_extra, child_fwd, integ_rev;
  long long fd_free, integ_free;
  long long bwd_rev, bwd_rev_push, child_bwd, integ_adj_rev;
  long long bwd_free;
  long long fd_ball, fd_ball_push, integ_ball, bwd_ball, bwd_ball_push;
};

// prism: count a prismatic joint's link instead of a revolute one
LinkOps link_ops(bool eti, bool prism) {
  using namespace aba;
  LinkOps o{};
  LinkC<Op> L{};
  L.prism = prism;  // canonicalised joint axis e_z: S = [e_z; 0] or [0; e_z]
  L.sm = prism ? v6<Op>(zero3<Op>(), v3<Op>(Op(0.0), Op(0.0), Op(1.0)))
               : v6<Op>(v3<Op>(Op(0.0), Op(0.0), Op(1.0)), zero3<Op>());
  if (eti)
    for (int k = 0; k < 9; ++k) L.ET.m[k] = Op((k % 4 == 0) ? 1.0 : 0.0);
  Tape<Op> t{};
  V6<Op> v{}, w{};
  SySp<Op> M{}, M2{};
  Q4<Op> qt{};
  V3<Op> g{};
  Bar<Op> b{};
  // one 1-dof ABA evaluation (sin and cos counted as one operation each)
  o.fd_rev = (prism ? 0 : 2) + count([&] {
               joint_X(L, t);
               t.v = p1_velocity(L, t, Op(), v);
               p1_bias(L, t.v, Op(), true, t.c, t.pA, t.IA);
               p2_local(L, t, Op());
               (void)p3_accel(L, t, v);
             });
  o.fd_rev_push = count([&] { p2_push(L, t, M, w); });
  o.child_fwd = 27;  // IA (21) and pA (6) of each child added to its parent
  o.integ_rev = count([&] {
    Op q, qd;
    integrate_joint(q, qd, Op(), Op());
  });
  o.fd_free = count([&] {
    p1_bias(L, v, Op(), false, t.c, t.pA, t.IA);
    root_accel(t.IA, t.pA, qt, g, t.ap, w);
  });
  o.integ_free = count([&] {
    V3<Op> p{};
    integrate_root(p, qt, v, w, Op());
  });
  o.integ_adj_rev = 3;  // qd_tot = qd_bar + dt q_bar; qdd_bar = dt qd_tot
  o.bwd_rev = count([&] {
    (void)r3_link(L, t, b, v, Op());
    (void)r2_link(L, t, b, false, M, v, M2, w);
    (void)r1_link(L, t, b, v, w, Op());
  });
  o.bwd_rev_push = count([&] {
                     (void)xformT(t.E, joint_r(L, t), v);         // a_bar to the parent
                     (void)r2_link(L, t, b, true, M, v, M2, w);  // parent share of pass 2
                   }) -
                   count([&] { (void)r2_link(L, t, b, false, M, v, M2, w); });
  o.child_bwd = 12;  // a_bar (6) and v_bar (6) of each child added to its parent
  o.bwd_free = count([&] {
    V3<Op> pb{};
    Q4<Op> qb{};
    V6<Op> vb{};
    (void)integrate_root_adj(qt, v, w, Op(), pb, qb, vb);
    r3_root(M, v, qt, g, v, w, qb, M2, w);
    (void)r1_root(L, v, w, w);
  });
  // ball joint: pass 1 (E from the quaternion), 2 and 3; the push to the
  // parent; the integrator; the reverse step (with the rebuild of E, c and
  // the joint-space blocks the stored tapes leave out)
  {
    V3<Op> w3{}, a3{};
    o.fd_ball = count([&] {
      ball_p1(L, t, qt, w3, v);
      p1_bias(L, t.v, Op(), false, t.c, t.pA, t.IA);
      t.c = crm(t.v, v6<Op>(w3, zero3<Op>()));
      (void)ball_p2_local(t, w3);
      (void)ball_p3(L, t, v, a3);
    });
    o.fd_ball_push = count([&] { ball_p2_push(L, t, w3, M, w); });
    o.integ_ball = 3 + count([&] {
                     V3<Op> w1 = w3 + Op() * a3;
                     (void)quat_step(qt, w1, Op());
                   });
    auto rebuild = [&] {
      t.E = ball_E(qt, L.ET);
      t.c = crm(t.v, v6<Op>(w3, zero3<Op>()));
      t.Ai = sy3_inv(t.IA.A);
      t.y = mul(t.Ai, a3);
      t.W = mul(sy_to_m3(t.Ai), t.IA.B);
    };
    o.bwd_ball = count([&] {
      rebuild();
      V3<Op> wb{}, s3{};
      (void)quat_step_adj(qt, w3 + Op() * a3, Op(), qt, wb);
      BallBar<Op> bb{};
      SySp<Op> N{};
      V6<Op> pab{};
      const V6<Op> apb = ball_r3_path(t, v, w3, s3);
      ball_r3_local(t, b, bb, apb, s3);
      (void)ball_r2_path(L, t, bb, a3, false, M, v, N, pab, M2, w);
      (void)ball_r1_own(L, t.v, b, w, w3);
      (void)ball_r1_local(t, b, v, w3);
      (void)ball_quat_bar(qt, b.G.a);
    });
    o.bwd_ball_push = count([&] {
                        BallBar<Op> bb{};
                        SySp<Op> N{};
                        V6<Op> pab{};
                        (void)xformT(t.E, L.rT, v);  // a_bar to the parent
                        (void)ball_r2_path(L, t, bb, a3, true, M, v, N, pab, M2, w);
                        ball_r2_local(t, b, N, pab);
                      }) -
                      count([&] {
                        BallBar<Op> bb{};
                        SySp<Op> N{};
                        V6<Op> pab{};
                        (void)ball_r2_path(L, t, bb, a3, false, M, v, N, pab, M2, w);
                      });
  }
  return o;
}

}  // namespace

extern "C" int sim_flops(sim_t h, int kind, double* flops) {
  if (!h || !flops) return fail(SIM_ERR_INVALID_ARG, "sim_flops: null argument");
  if (kind < 0 || kind > 2) return fail(SIM_ERR_INVALID_ARG, "sim_flops: kind must be 0, 1 or 2");
  const LinkOps orev = link_ops(h->eti, false), opri = link_ops(h->eti, true);
  double fd = 0, fwd = 0, bwd = 0;
  for (int i = 0; i < h->n_links; ++i) {
    const LinkOps& o = (h->jtype[i] == SIM_JOINT_PRISMATIC) ? opri : orev;
    if (h->jtype[i] == SIM_JOINT_FREE) {
      fd += (double)o.fd_free;
      fwd += (double)(o.fd_free + o.integ_free);
      bwd += (double)o.bwd_free;
    } else if (h->jtype[i] == SIM_JOINT_SPHERICAL) {
      const bool push = h->parent[i] >= 0;
      const double f = (double)(o.fd_ball + (push ? o.fd_ball_push : 0));
      fd += f;
      fwd += f + (double)o.integ_ball;
      bwd += (double)(o.bwd_ball + (push ? o.bwd_ball_push : 0));
    } else {
      const bool push = h->parent[i] >= 0;
      const double f = (double)(o.fd_rev + (push ? o.fd_rev_push : 0));
      fd += f;
      fwd += f + (double)o.integ_rev;
      bwd += (double)(o.integ_adj_rev + o.bwd_rev + (push ? o.bwd_rev_push : 0));
    }
    fd += (double)(o.child_fwd * h->nchild[i]);
    fwd += (double)(o.child_fwd * h->nchild[i]);
    bwd += (double)(o.child_bwd * h->nchild[i]);
  }
  // the backward step recomputes one forward dynamics evaluation
  bwd += fd;
  *flops = (kind == 0) ? fd : (kind == 1) ? fwd : bwd;
  return SIM_OK;
}
