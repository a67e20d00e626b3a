// Test-only host emulation of the GPU path's arithmetic.
//
// Calls the same per-link functions the kernels call (csrc/aba_lane.h),
// link by link in a sequential tree order instead of level-synchronous
// lanes, in double or float.  Lets the CPU test suite check the structured
// forward and adjoint statements against the oracle without a GPU.  Never
// loaded by the package.
#include <cmath>
#include <vector>

#include "../../paper_2109_07719_amd/csrc/aba_lane.h"

using namespace aba;

namespace {

template <typename S>
struct Sys {
  int n;
  const int* parent;
  const int* jtype;
  std::vector<LinkC<S>> L;
  S g[3];
  std::vector<int> qi, vi, ui;
};

template <typename S>
Sys<S> make_sys(int n, const int* parent, const int* jtype, const double* cf, const double* g) {
  Sys<S> s;
  s.n = n;
  s.parent = parent;
  s.jtype = jtype;
  s.L.resize(n);
  for (int i = 0; i < n; ++i) {
    const double* c = cf + 25 * (size_t)i;
    LinkC<S>& L = s.L[i];
    for (int k = 0; k < 9; ++k) L.ET.m[k] = (S)c[k];
    L.rT = v3<S>((S)c[9], (S)c[10], (S)c[11]);
    // c[12..14] is the canonicalised joint axis e_z: S = [a; 0] revolute,
    // [0; a] prismatic
    const V3<S> ax = v3<S>((S)c[12], (S)c[13], (S)c[14]);
    L.prism = jtype[i] == 2;
    L.sm = L.prism ? v6<S>(zero3<S>(), ax) : v6<S>(ax, zero3<S>());
    L.m = (S)c[15];
    L.mc = v3<S>((S)c[16], (S)c[17], (S)c[18]);
    L.Ib = sy3<S>((S)c[19], (S)c[20], (S)c[21], (S)c[22], (S)c[23], (S)c[24]);
  }
  for (int k = 0; k < 3; ++k) s.g[k] = (S)g[k];
  int q = 0, v = 0, u = 0;
  for (int i = 0; i < n; ++i) {
    s.qi.push_back(q);
    s.vi.push_back(v);
    s.ui.push_back(jtype[i] == 1 ? -1 : u);
    if (jtype[i] == 1) {
      q += 7;
      v += 6;
    } else if (jtype[i] == 3) {
      q += 4;
      v += 3;
      u += 3;
    } else {
      q += 1;
      v += 1;
      u += 1;
    }
  }
  return s;
}

template <typename S>
struct Out {
  std::vector<Tape<S>> t;
  std::vector<V3<S>> u3, qdd3;  // ball joints: tau - pA_a and the joint acceleration
  V6<S> abase;
};

template <typename S>
V3<S> vec3_of(const S* x) {
  return v3<S>(x[0], x[1], x[2]);
}
template <typename S>
Q4<S> quat4_of(const S* x) {
  return Q4<S>{x[0], x[1], x[2], x[3]};
}

template <typename S>
Q4<S> quat_of(const S* q) {
  return Q4<S>{q[3], q[4], q[5], q[6]};
}

template <typename S>
void fd_seq(const Sys<S>& s, const S* q, const S* qd, const S* tau, Out<S>& o, S* qdd) {
  const int n = s.n;
  o.t.assign(n, Tape<S>{});
  o.u3.assign(n, zero3<S>());
  o.qdd3.assign(n, zero3<S>());
  for (int i = 0; i < n; ++i) {
    Tape<S>& t = o.t[i];
    const LinkC<S>& L = s.L[i];
    if (s.jtype[i] == 3) {
      const V6<S> vp = s.parent[i] >= 0 ? o.t[s.parent[i]].v : zero6<S>();
      const V3<S> w = vec3_of(qd + s.vi[i]);
      ball_p1(L, t, quat4_of(q + s.qi[i]), w, vp);
      p1_bias(L, t.v, S(0), false, t.c, t.pA, t.IA);
      t.c = crm(t.v, v6<S>(w, zero3<S>()));
      continue;
    }
    if (s.jtype[i] != 1) {
      const S qq = q[s.qi[i]];
      t.sq = L.prism ? qq : (S)std::sin(qq);
      t.cq = L.prism ? S(1) : (S)std::cos(qq);
      joint_X(L, t);
      const V6<S> vp = s.parent[i] >= 0 ? o.t[s.parent[i]].v : zero6<S>();
      t.v = p1_velocity(L, t, qd[s.vi[i]], vp);
    } else {
      // free root: the kernels' Galilean shift (the ABA sees [w; 0])
      const S* v = qd + s.vi[i];
      t.v = v6<S>(v3<S>(v[0], v[1], v[2]), zero3<S>());
    }
    p1_bias(L, t.v, s.jtype[i] != 1 ? qd[s.vi[i]] : S(0), s.jtype[i] != 1, t.c, t.pA, t.IA);
  }
  for (int i = n - 1; i >= 0; --i) {
    Tape<S>& t = o.t[i];
    if (s.jtype[i] == 1) continue;
    if (s.jtype[i] == 3) {
      const V3<S> tau3 = vec3_of(tau + s.ui[i]);
      o.u3[i] = ball_p2_local(t, tau3);
      if (s.parent[i] >= 0) {
        SySp<S> IAu;
        V6<S> pAu;
        ball_p2_push(s.L[i], t, tau3, IAu, pAu);
        o.t[s.parent[i]].IA = o.t[s.parent[i]].IA + IAu;
        o.t[s.parent[i]].pA = o.t[s.parent[i]].pA + pAu;
      }
      continue;
    }
    p2_local(s.L[i], t, tau[s.ui[i]]);
    if (s.parent[i] >= 0) {
      SySp<S> IAu;
      V6<S> pAu;
      p2_push(s.L[i], t, IAu, pAu);
      o.t[s.parent[i]].IA = o.t[s.parent[i]].IA + IAu;
      o.t[s.parent[i]].pA = o.t[s.parent[i]].pA + pAu;
    }
  }
  const V6<S> a0 = v6<S>(zero3<S>(), v3<S>(-s.g[0], -s.g[1], -s.g[2]));
  std::vector<V6<S>> acc(n);
  for (int i = 0; i < n; ++i) {
    Tape<S>& t = o.t[i];
    if (s.jtype[i] == 3) {
      acc[i] = ball_p3(s.L[i], t, s.parent[i] >= 0 ? acc[s.parent[i]] : a0, o.qdd3[i]);
      qdd[s.vi[i]] = o.qdd3[i].x;
      qdd[s.vi[i] + 1] = o.qdd3[i].y;
      qdd[s.vi[i] + 2] = o.qdd3[i].z;
    } else if (s.jtype[i] != 1) {
      acc[i] = p3_accel(s.L[i], t, s.parent[i] >= 0 ? acc[s.parent[i]] : a0);
      qdd[s.vi[i]] = t.qdd;
    } else {
      root_accel(t.IA, t.pA, quat_of(q + s.qi[i]), v3<S>(s.g[0], s.g[1], s.g[2]), t.ap, o.abase);
      const S* v = qd + s.vi[i];
      o.abase.l = o.abase.l - cross(v3<S>(v[0], v[1], v[2]), v3<S>(v[3], v[4], v[5]));
      acc[i] = t.ap;
      const S a[6] = {o.abase.a.x, o.abase.a.y, o.abase.a.z, o.abase.l.x, o.abase.l.y, o.abase.l.z};
      for (int k = 0; k < 6; ++k) qdd[s.vi[i] + k] = a[k];
    }
  }
}

template <typename S>
void integrate_seq(const Sys<S>& s, S* q, S* qd, const S* qdd, const Out<S>& o, S dt) {
  for (int i = 0; i < s.n; ++i) {
    if (s.jtype[i] == 3) {
      S* w = qd + s.vi[i];
      for (int k = 0; k < 3; ++k) w[k] = w[k] + dt * qdd[s.vi[i] + k];
      const Q4<S> q1 = quat_step(quat4_of(q + s.qi[i]), vec3_of(w), dt);
      S* qq = q + s.qi[i];
      qq[0] = q1.x; qq[1] = q1.y; qq[2] = q1.z; qq[3] = q1.w;
    } else if (s.jtype[i] != 1) {
      integrate_joint(q[s.qi[i]], qd[s.vi[i]], qdd[s.vi[i]], dt);
    } else {
      S* qq = q + s.qi[i];
      S* v = qd + s.vi[i];
      V3<S> p = v3<S>(qq[0], qq[1], qq[2]);
      Q4<S> qt = quat_of(qq);
      V6<S> vv = v6<S>(v3<S>(v[0], v[1], v[2]), v3<S>(v[3], v[4], v[5]));
      integrate_root(p, qt, vv, o.abase, dt);
      qq[0] = p.x; qq[1] = p.y; qq[2] = p.z;
      qq[3] = qt.x; qq[4] = qt.y; qq[5] = qt.z; qq[6] = qt.w;
      v[0] = vv.a.x; v[1] = vv.a.y; v[2] = vv.a.z; v[3] = vv.l.x; v[4] = vv.l.y; v[5] = vv.l.z;
    }
  }
}

// one reverse step, mirrors the kernel's bwd_step (sequential tree order)
// pg (nullable): per-link parameter accumulators; the placement and axis
// part (frame_bar_add) is formed when it is given
template <typename S>
void bwd_seq(const Sys<S>& s, const S* q, const S* qd, const S* tau, S dt, S* qb, S* qdb, S* taub,
             std::vector<ParamBar<S>>* pg) {
  const int n = s.n;
  Out<S> o;
  std::vector<S> qdd(qdb ? 0 : 0);
  int nv = 0;
  for (int i = 0; i < n; ++i) nv += (s.jtype[i] == 1) ? 6 : (s.jtype[i] == 3) ? 3 : 1;
  qdd.assign(nv, S(0));
  fd_seq(s, q, qd, tau, o, qdd.data());
  std::vector<Bar<S>> b(n);
  for (auto& x : b) bar_zero(x, pg != nullptr);
  std::vector<S> acc_q(n), acc_qd(n), qddb(n);
  V6<S> qddb6 = zero6<S>(), vb6 = zero6<S>();
  V3<S> pb = zero3<S>();
  Q4<S> quatb{};
  int root = -1;
  std::vector<BallBar<S>> bb(n);
  for (auto& x : bb) ball_bar_zero(x);
  std::vector<V3<S>> qddb3(n, zero3<S>()), wb3(n, zero3<S>()), taub3(n, zero3<S>());
  std::vector<Q4<S>> qtb(n, Q4<S>{});
  for (int i = 0; i < n; ++i) {
    if (s.jtype[i] == 3) {
      // w1 = w + dt qdd; quat1 = quat_step(quat, w1)
      const V3<S> w1 = vec3_of(qd + s.vi[i]) + dt * o.qdd3[i];
      wb3[i] = vec3_of(qdb + s.vi[i]);
      qtb[i] = quat_step_adj(quat4_of(q + s.qi[i]), w1, dt, quat4_of(qb + s.qi[i]), wb3[i]);
      qddb3[i] = dt * wb3[i];
      continue;
    }
    if (s.jtype[i] != 1) {
      const S tot = qdb[s.vi[i]] + dt * qb[s.qi[i]];
      qddb[i] = dt * tot;
      acc_q[i] = qb[s.qi[i]];
      acc_qd[i] = tot;
    } else {
      root = i;
      const S* x = qb + s.qi[i];
      pb = v3<S>(x[0], x[1], x[2]);
      quatb = Q4<S>{x[3], x[4], x[5], x[6]};
      const S* y = qdb + s.vi[i];
      vb6 = v6<S>(v3<S>(y[0], y[1], y[2]), v3<S>(y[3], y[4], y[5]));
      const S* v = qd + s.vi[i];
      const V6<S> vv = v6<S>(v3<S>(v[0], v[1], v[2]), v3<S>(v[3], v[4], v[5]));
      qddb6 = integrate_root_adj(quat_of(q + s.qi[i]), vv, o.abase, dt, pb, quatb, vb6);
      vb6.a = vb6.a + cross(qddb6.l, vv.l);
      vb6.l = vb6.l + cross(vv.a, qddb6.l);
    }
  }
  std::vector<V6<S>> ab(n, zero6<S>()), vb(n, zero6<S>()), pAb(n, zero6<S>());
  std::vector<SySp<S>> IAb(n, zero_sysp<S>());
  const V3<S> g = v3<S>(s.g[0], s.g[1], s.g[2]);
  for (int i = n - 1; i >= 0; --i) {
    if (s.jtype[i] == 3) {
      V3<S> sv;
      const V6<S> apb = ball_r3_path(o.t[i], ab[i], qddb3[i], sv);
      ball_r3_local(o.t[i], b[i], bb[i], apb, sv);
      if (s.parent[i] >= 0) ab[s.parent[i]] = ab[s.parent[i]] + xformT(o.t[i].E, s.L[i].rT, apb);
    } else if (s.jtype[i] != 1) {
      const V6<S> apb = r3_link(s.L[i], o.t[i], b[i], ab[i], qddb[i]);
      if (s.parent[i] >= 0) ab[s.parent[i]] = ab[s.parent[i]] + xformT(o.t[i].E, joint_r(s.L[i], o.t[i]), apb);
    } else {
      r3_root(o.t[i].IA, o.t[i].ap, quat_of(q + s.qi[i]), g, ab[i], qddb6, quatb, IAb[i], pAb[i]);
    }
  }
  for (int i = 0; i < n; ++i) {
    if (s.jtype[i] == 1) continue;
    const int p = s.parent[i];
    const bool hp = p >= 0;
    if (s.jtype[i] == 3) {
      SySp<S> N;
      V6<S> pab;
      const V3<S> tb = ball_r2_path(s.L[i], o.t[i], bb[i], o.u3[i], hp, hp ? IAb[p] : zero_sysp<S>(),
                                    hp ? pAb[p] : zero6<S>(), N, pab, IAb[i], pAb[i]);
      if (hp) ball_r2_local(o.t[i], b[i], N, pab);
      taub[s.ui[i]] = tb.x;
      taub[s.ui[i] + 1] = tb.y;
      taub[s.ui[i] + 2] = tb.z;
      continue;
    }
    taub[s.ui[i]] = r2_link(s.L[i], o.t[i], b[i], hp, hp ? IAb[p] : zero_sysp<S>(), hp ? pAb[p] : zero6<S>(),
                            IAb[i], pAb[i]);
  }
  for (int i = n - 1; i >= 0; --i) {
    if (s.jtype[i] == 3) {
      const V3<S> w = vec3_of(qd + s.vi[i]);
      const V6<S> vbar = vb[i] + ball_r1_own(s.L[i], o.t[i].v, b[i], pAb[i], w);
      wb3[i] = wb3[i] + ball_r1_local(o.t[i], b[i], vbar, w);
      if (s.parent[i] >= 0) vb[s.parent[i]] = vb[s.parent[i]] + xformT(o.t[i].E, s.L[i].rT, vbar);
    } else if (s.jtype[i] != 1) {
      const V6<S> up = r1_link(s.L[i], o.t[i], b[i], vb[i], pAb[i], qd[s.vi[i]]);
      if (s.parent[i] >= 0) vb[s.parent[i]] = vb[s.parent[i]] + up;
    } else {
      vb6.a = vb6.a + r1_root(s.L[i], o.t[i].v, vb[i], pAb[i]).a;
    }
  }
  if (pg)
    for (int i = 0; i < n; ++i)
      if (s.jtype[i] == 3) {
        ball_frame_bar_add((*pg)[i], quat4_of(q + s.qi[i]), b[i]);
      } else if (s.jtype[i] != 1) {
        r2_sbar(o.t[i], b[i]);
        frame_bar_add((*pg)[i], s.L[i], o.t[i], b[i]);
      }
  for (int i = 0; i < n; ++i) {
    if (s.jtype[i] == 3) {
      const Q4<S> qa = ball_quat_bar(quat4_of(q + s.qi[i]), b[i].G.a);
      S* x = qb + s.qi[i];
      x[0] = qtb[i].x + qa.x; x[1] = qtb[i].y + qa.y; x[2] = qtb[i].z + qa.z; x[3] = qtb[i].w + qa.w;
      S* y = qdb + s.vi[i];
      y[0] = wb3[i].x; y[1] = wb3[i].y; y[2] = wb3[i].z;
      continue;
    }
    if (s.jtype[i] != 1) {
      qb[s.qi[i]] = acc_q[i] + b[i].q;
      qdb[s.vi[i]] = acc_qd[i] + b[i].qd;
    }
  }
  if (root >= 0) {
    S* x = qb + s.qi[root];
    x[0] = pb.x; x[1] = pb.y; x[2] = pb.z;
    x[3] = quatb.x; x[4] = quatb.y; x[5] = quatb.z; x[6] = quatb.w;
    S* y = qdb + s.vi[root];
    y[0] = vb6.a.x; y[1] = vb6.a.y; y[2] = vb6.a.z; y[3] = vb6.l.x; y[4] = vb6.l.y; y[5] = vb6.l.z;
  }
}

template <typename S>
void rollout_grad(int n, const int* parent, const int* jtype, const double* cf, const double* g, const S* q0,
                  const S* qd0, const S* tau, double dt_, int T, const S* gqT, const S* gqdT, S* gq0, S* gqd0,
                  S* gtau, S* qT, S* qdT, S* gframe) {
  Sys<S> s = make_sys<S>(n, parent, jtype, cf, g);
  const S dt = (S)dt_;
  int nq = 0, nv = 0, nu = 0;
  for (int i = 0; i < n; ++i) {
    nq += jtype[i] == 1 ? 7 : jtype[i] == 3 ? 4 : 1;
    nv += jtype[i] == 1 ? 6 : jtype[i] == 3 ? 3 : 1;
    nu += jtype[i] == 1 ? 0 : jtype[i] == 3 ? 3 : 1;
  }
  std::vector<S> xs((size_t)(T + 1) * (nq + nv));
  std::copy(q0, q0 + nq, xs.begin());
  std::copy(qd0, qd0 + nv, xs.begin() + nq);
  std::vector<S> qdd(nv);
  for (int t = 0; t < T; ++t) {
    S* cur = xs.data() + (size_t)t * (nq + nv);
    S* nxt = cur + (nq + nv);
    std::copy(cur, cur + nq + nv, nxt);
    Out<S> o;
    fd_seq(s, cur, cur + nq, tau + (size_t)t * nu, o, qdd.data());
    integrate_seq(s, nxt, nxt + nq, qdd.data(), o, dt);
  }
  const S* last = xs.data() + (size_t)T * (nq + nv);
  std::copy(last, last + nq, qT);
  std::copy(last + nq, last + nq + nv, qdT);
  std::vector<S> qb(gqT, gqT + nq), qdb(gqdT, gqdT + nv);
  std::vector<ParamBar<S>> pg(n);
  for (auto& x : pg) param_bar_zero(x);
  for (int t = T - 1; t >= 0; --t) {
    const S* cur = xs.data() + (size_t)t * (nq + nv);
    bwd_seq(s, cur, cur + nq, tau + (size_t)t * nu, dt, qb.data(), qdb.data(), gtau + (size_t)t * nu,
            gframe ? &pg : nullptr);
  }
  // placement and axis accumulators in the kernels' frames: xi (6), w (3)
  if (gframe)
    for (int i = 0; i < n; ++i) {
      const ParamBar<S>& x = pg[i];
      const S v[9] = {x.xi.a.x, x.xi.a.y, x.xi.a.z, x.xi.l.x, x.xi.l.y, x.xi.l.z, x.w.x, x.w.y, x.w.z};
      for (int k = 0; k < 9; ++k) gframe[9 * i + k] = v[k];
    }
  std::copy(qb.begin(), qb.end(), gq0);
  std::copy(qdb.begin(), qdb.end(), gqd0);
}

}  // namespace

extern "C" {

void emu_fd_d(int n, const int* parent, const int* jtype, const double* cf, const double* g, const double* q,
              const double* qd, const double* tau, double* qdd) {
  Sys<double> s = make_sys<double>(n, parent, jtype, cf, g);
  Out<double> o;
  fd_seq(s, q, qd, tau, o, qdd);
}
void emu_fd_f(int n, const int* parent, const int* jtype, const double* cf, const double* g, const float* q,
              const float* qd, const float* tau, float* qdd) {
  Sys<float> s = make_sys<float>(n, parent, jtype, cf, g);
  Out<float> o;
  fd_seq(s, q, qd, tau, o, qdd);
}
void emu_rollout_grad_d(int n, const int* parent, const int* jtype, const double* cf, const double* g,
                        const double* q0, const double* qd0, const double* tau, double dt, int T, const double* gqT,
                        const double* gqdT, double* gq0, double* gqd0, double* gtau, double* qT, double* qdT,
                        double* gframe) {
  rollout_grad<double>(n, parent, jtype, cf, g, q0, qd0, tau, dt, T, gqT, gqdT, gq0, gqd0, gtau, qT, qdT, gframe);
}
void emu_rollout_grad_f(int n, const int* parent, const int* jtype, const double* cf, const double* g,
                        const float* q0, const float* qd0, const float* tau, double dt, int T, const float* gqT,
                        const float* gqdT, float* gq0, float* gqd0, float* gtau, float* qT, float* qdT,
                        float* gframe) {
  rollout_grad<float>(n, parent, jtype, cf, g, q0, qd0, tau, dt, T, gqT, gqdT, gq0, gqd0, gtau, qT, qdT, gframe);
}
}
